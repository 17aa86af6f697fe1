"""MI355X-native replica-exchange grand-canonical (REGC) sampling and multistate
reweighting (arXiv:1908.11118).  The compute path is the HIP library
`libregc_hip.so` built from `csrc/`; `regc` is its thin ctypes binding and
`workloads` builds seeded synthetic inputs.  Submodules are imported on use."""
__all__ = ["regc", "workloads"]
