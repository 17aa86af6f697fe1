"""Thin ctypes binding of libregc_hip.so (include/regc.h).

Argument marshalling only: every step of sampling and reweighting runs in the HIP
library.  PyTorch, when present, only supplies the HIP stream the work is
enqueued on.  If the library has not been built the first call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libregc_hip.so")

OK, EINVAL, ENOMEM, EHIP, ECAPACITY, ESTATE, EUNSUPPORTED, ENOCONV = 0, -1, -2, -3, -4, -5, -6, -7
MODE_LJ, MODE_IDEAL = 0, 1
FP64, FP32PAIR = 0, 1
NSTAT = 10
STAT_NAMES = ["disp_att", "disp_acc", "ins_att", "ins_acc", "del_att", "del_acc",
              "cap_rej", "empty_rej", "wall_rej", "core_rej"]

# every symbol include/regc.h declares
EXPORTS = ["regc_default_opts", "regc_create", "regc_create_batch", "regc_get_layout", "regc_set_stream",
           "regc_run", "regc_sync", "regc_get_sweep", "regc_get_walkers", "regc_set_walkers", "regc_energies",
           "regc_sample_count", "regc_get_samples", "regc_samples_device", "regc_clear_samples",
           "regc_get_stats", "regc_get_pair_counts", "regc_get_histograms", "regc_get_trace", "regc_timing_enable", "regc_timing_get",
           "regc_checkpoint", "regc_restore", "regc_destroy", "regc_mbar_create", "regc_mbar_set_stream",
           "regc_mbar_set_samples", "regc_mbar_load_run", "regc_mbar_set_solver", "regc_mbar_solve", "regc_mbar_targets", "regc_mbar_targets_static",
           "regc_mbar_timing", "regc_mbar_destroy", "regc_mlp_param_count", "regc_mlp_create",
           "regc_mlp_set_stream", "regc_mlp_set_params", "regc_mlp_get_params", "regc_mlp_forward",
           "regc_mlp_loss_grads", "regc_mlp_train", "regc_mlp_timing", "regc_mlp_destroy",
           "regc_set_proposal", "regc_set_class_proposal", "regc_capture_voxels", "regc_get_proposal_stats", "regc_set_observables",
           "regc_observables_device", "regc_get_observables", "regc_mbar_set_observables", "regc_mbar_observables",
           "regc_track_minima", "regc_get_minima", "regc_aiat_phase", "regc_strerror", "regc_last_error",
           "regc_default_reweight_opts", "regc_reweight", "regc_mlp_step", "regc_proposal_eval",
           "regc_count_pairs", "regc_batch_means"]


class RegcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"regc error {code}: {msg}")
        self.code = code


_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u32p = C.POINTER(C.c_uint32)


class Potential(C.Structure):
    _fields_ = [("eps_gg", C.c_double), ("sig_gg", C.c_double), ("eps_gs", C.c_double),
                ("sig_gs", C.c_double), ("rcut", C.c_double), ("hc_frac", C.c_double),
                ("shifted", C.c_int), ("mode", C.c_int)]


class System(C.Structure):
    _fields_ = [("n_slab", C.c_int), ("slab_xyz", _dp), ("lx", C.c_double), ("ly", C.c_double),
                ("z_lo", C.c_double), ("z_hi", C.c_double), ("lambda1", C.c_double), ("n_max", C.c_int)]


class Grid(C.Structure):
    _fields_ = [("n_t", C.c_int), ("n_mu", C.c_int), ("t", _dp), ("mu", _dp)]


class ObsSpec(C.Structure):
    _fields_ = [("dz", C.c_double), ("layer_lo", C.c_double), ("layer_hi", C.c_double), ("dr", C.c_double),
                ("n_r", C.c_int)]


class ReweightOpts(C.Structure):
    _fields_ = [("n_batches", C.c_int), ("n_boot", C.c_int), ("record_size", C.c_int64),
                ("block_records", C.c_int64), ("seed", C.c_uint64), ("n_sites", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("precision", C.c_int), ("p_disp", C.c_double), ("p_ins", C.c_double),
                ("max_disp", C.c_double), ("trials_per_sweep", C.c_int), ("swap_every", C.c_int),
                ("sample_every", C.c_int), ("swap_scheme", C.c_int), ("sample_capacity", C.c_int64),
                ("trace_capacity", C.c_int64), ("walkers_per_block", C.c_int), ("sweeps_per_launch", C.c_int),
                ("slab_bins", C.c_int), ("split", C.c_int), ("cull", C.c_int),
                ("graph_intervals", C.c_int), ("schedule", C.c_int), ("x0", C.c_double), ("mc_cycles", C.c_int),
                ("md_steps", C.c_int), ("md_dt", C.c_double), ("md_tau", C.c_double), ("resync_every", C.c_int),
                ("batch_trials", C.c_int), ("slab_cell", C.c_double),
                ("persistent", C.c_int),
                ("balance", C.c_int)]


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.regc_default_opts.argtypes = [C.POINTER(Opts)]
        L.regc_default_opts.restype = None
        L.regc_create.argtypes = [C.POINTER(Potential), C.POINTER(System), C.POINTER(Grid), C.POINTER(Opts),
                                  C.POINTER(vp)]
        L.regc_create_batch.argtypes = [C.c_int, C.POINTER(Potential), C.POINTER(System), C.POINTER(Grid),
                                        C.POINTER(Opts), C.POINTER(vp)]
        L.regc_get_layout.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.regc_set_stream.argtypes = [vp, vp]
        L.regc_run.argtypes = [vp, C.c_int64]
        L.regc_sync.argtypes = [vp]
        L.regc_get_sweep.argtypes = [vp, _i64p]
        L.regc_get_walkers.argtypes = [vp, _i32p, _dp, _i32p, _dp]
        L.regc_set_walkers.argtypes = [vp, _i32p, _dp, _i32p]
        L.regc_energies.argtypes = [vp, _dp]
        L.regc_sample_count.argtypes = [vp, _i64p]
        L.regc_get_samples.argtypes = [vp, _dp, _i32p, _i32p, C.c_int64, _i64p]
        L.regc_samples_device.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), _i64p]
        L.regc_clear_samples.argtypes = [vp]
        L.regc_get_stats.argtypes = [vp, _i64p, _i64p, _i64p]
        L.regc_get_histograms.argtypes = [vp, _i64p]
        L.regc_get_pair_counts.argtypes = [vp, _i64p, _i64p]
        L.regc_count_pairs.argtypes = [vp, C.c_int]
        L.regc_get_trace.argtypes = [vp, _u32p, _i32p, C.c_int64, _i64p]
        L.regc_timing_enable.argtypes = [vp, C.c_int]
        L.regc_timing_get.argtypes = [vp, _dp, _i64p, _dp, _i64p]
        L.regc_checkpoint.argtypes = [vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]
        L.regc_restore.argtypes = [vp, vp, C.c_size_t]
        L.regc_destroy.argtypes = [vp]
        L.regc_destroy.restype = None
        L.regc_mbar_create.argtypes = [C.POINTER(Grid), C.c_double, C.c_int, C.POINTER(vp)]
        L.regc_mbar_set_stream.argtypes = [vp, vp]
        L.regc_mbar_set_samples.argtypes = [vp, C.c_int64, vp, vp, vp, C.c_int]
        L.regc_mbar_load_run.argtypes = [vp, vp, C.c_int, C.c_int64]
        L.regc_mbar_set_solver.argtypes = [vp, C.c_int, C.c_int]
        L.regc_mbar_solve.argtypes = [vp, C.c_double, C.c_int, _dp, C.POINTER(C.c_int), _dp]
        L.regc_mbar_targets.argtypes = [vp, C.POINTER(Grid), _dp, _dp, _dp, _dp, _dp, _i32p]
        L.regc_mbar_targets_static.argtypes = [vp, C.POINTER(Grid), _dp, _dp, _dp, _dp, _i32p]
        L.regc_batch_means.argtypes = [C.c_int64, vp, vp, C.c_int, C.c_int, C.c_int, _dp, _dp, vp]
        L.regc_mbar_timing.argtypes = [vp, _dp, _i64p]
        L.regc_default_reweight_opts.argtypes = [C.POINTER(ReweightOpts)]
        L.regc_default_reweight_opts.restype = None
        L.regc_reweight.argtypes = [vp, C.POINTER(Grid), C.c_double, C.c_int, C.POINTER(ReweightOpts)] + \
            [_dp] * 5 + [_i32p] + [_dp] * 5
        L.regc_mbar_destroy.argtypes = [vp]
        L.regc_mbar_destroy.restype = None
        _u16p = C.POINTER(C.c_uint16)
        L.regc_mlp_param_count.argtypes = [_i64p]
        L.regc_mlp_create.argtypes = [C.POINTER(C.c_float), C.POINTER(vp)]
        L.regc_mlp_set_stream.argtypes = [vp, vp]
        L.regc_mlp_set_params.argtypes = [vp, C.POINTER(C.c_float)]
        L.regc_mlp_get_params.argtypes = [vp, C.POINTER(C.c_float)]
        L.regc_mlp_forward.argtypes = [vp, C.c_int, C.c_int, _u16p, _i32p, _i32p, C.POINTER(C.c_float)]
        L.regc_mlp_loss_grads.argtypes = [vp, C.c_int, C.c_int, _u16p, _i32p, _i32p, _i32p, _dp,
                                          C.POINTER(C.c_float)]
        L.regc_mlp_train.argtypes = [vp, C.c_int64, C.c_int, vp, vp, C.c_int64, C.c_int, C.c_double,
                                     C.c_uint64, _dp]
        L.regc_mlp_step.argtypes = [vp, C.c_int, C.c_int, _u16p, _i32p, _i32p, _i32p, C.c_double, _dp,
                                    C.POINTER(C.c_float)]
        L.regc_proposal_eval.argtypes = [vp, C.c_int, C.c_int, _i32p, _dp, _i32p, C.POINTER(C.c_float), _dp, _dp]
        L.regc_mlp_timing.argtypes = [vp, _dp, _i64p]
        L.regc_mlp_destroy.argtypes = [vp]
        L.regc_mlp_destroy.restype = None
        L.regc_set_proposal.argtypes = [vp, vp, C.c_double]
        L.regc_set_class_proposal.argtypes = [vp, C.c_int, vp, C.c_double]
        L.regc_get_proposal_stats.argtypes = [vp, _i64p]
        L.regc_capture_voxels.argtypes = [vp, vp, vp]
        L.regc_set_observables.argtypes = [vp, C.POINTER(ObsSpec)]
        L.regc_track_minima.argtypes = [vp, C.c_int]
        L.regc_get_minima.argtypes = [vp, C.c_int, _dp, _dp]
        L.regc_aiat_phase.argtypes = [_dp, C.c_int, C.c_int, _dp, _i32p]
        L.regc_observables_device.argtypes = [vp, C.POINTER(vp), C.POINTER(C.c_int)]
        L.regc_get_observables.argtypes = [vp, _u32p, C.c_int64, _i64p]
        L.regc_mbar_set_observables.argtypes = [vp, vp, C.c_int, C.c_int]
        L.regc_mbar_observables.argtypes = [vp, C.POINTER(Grid), _dp, _dp]
        L.regc_strerror.argtypes = [C.c_int]
        L.regc_strerror.restype = C.c_char_p
        L.regc_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int, allow=()):
    if rc != OK and rc not in allow:
        raise RegcError(rc, lib().regc_last_error().decode())
    return rc


def _p(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _torch_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # torch absent: the null stream
        pass
    return None


def _grid(t, mu, keep):
    ta = np.ascontiguousarray(t, dtype=np.float64)
    ma = np.ascontiguousarray(mu, dtype=np.float64)
    keep.extend([ta, ma])
    return Grid(len(ta), len(ma), _p(ta, _dp), _p(ma, _dp))


class Regc:
    """A REGC simulation (one workload) or an uneven batch (a list of workloads
    sharing potential and schedule) advanced on the GPU."""

    def __init__(self, workloads, precision: int = FP64, sample_capacity: int = 0, trace_capacity: int = 0,
                 walkers_per_block: int = 0, sweeps_per_launch: int = 0, slab_bins: int = 0, split: int = 0,
                 cull: int = 0, graph_intervals: int = 0, resync_every: int = 0, batch_trials: int = 0, slab_cell: float = 0.0,
                 persistent: int = 0, balance: int = 0,
                 stream=None):
        wl = list(workloads) if isinstance(workloads, (list, tuple)) else [workloads]
        w0 = wl[0]
        self.workloads = wl
        self.precision = precision
        self._keep = []
        pot = Potential(w0.eps_gg, w0.sig_gg, w0.eps_gs, w0.sig_gs, w0.rc, w0.hc_frac, w0.shifted, w0.mode)
        systems = (System * len(wl))()
        grids = (Grid * len(wl))()
        for k, w in enumerate(wl):
            slab = np.ascontiguousarray(w.slab, dtype=np.float64).reshape(-1, 3)
            self._keep.append(slab)
            systems[k] = System(slab.shape[0], _p(slab, _dp), w.lx, w.ly, w.zlo, w.zhi, w.lambda1, w.n_max)
            grids[k] = _grid(w.t, w.mu, self._keep)
        o = Opts()
        lib().regc_default_opts(C.byref(o))
        o.seed, o.precision = w0.seed, precision
        o.p_disp, o.p_ins, o.max_disp = w0.p_disp, w0.p_ins, w0.max_disp
        o.trials_per_sweep, o.swap_every = w0.trials_per_sweep, w0.swap_every
        o.sample_every, o.swap_scheme = w0.sample_every, w0.swap_scheme
        o.sample_capacity, o.trace_capacity = sample_capacity, trace_capacity
        o.walkers_per_block, o.sweeps_per_launch, o.slab_bins = walkers_per_block, sweeps_per_launch, slab_bins
        o.split, o.cull, o.graph_intervals = split, cull, graph_intervals
        o.schedule = int(getattr(w0, "schedule", 0))
        o.x0 = float(getattr(w0, "x0", 0.99))
        o.mc_cycles = int(getattr(w0, "mc_cycles", 10))
        o.md_steps = int(getattr(w0, "md_steps", 0))
        o.md_dt = float(getattr(w0, "md_dt", 0.005))
        o.md_tau = float(getattr(w0, "md_tau", 0.1))
        o.resync_every = resync_every
        o.batch_trials = batch_trials
        o.slab_cell = slab_cell
        o.persistent = persistent
        o.balance = balance
        self.opts = o
        h = C.c_void_p()
        if len(wl) == 1:
            _check(lib().regc_create(C.byref(pot), systems, grids, C.byref(o), C.byref(h)))
        else:
            _check(lib().regc_create_batch(len(wl), C.byref(pot), systems, grids, C.byref(o), C.byref(h)))
        self.h = h
        nc = C.c_int()
        _check(lib().regc_get_layout(h, C.byref(nc), None, None))
        offs = (C.c_int * nc.value)()
        cnts = (C.c_int * nc.value)()
        _check(lib().regc_get_layout(h, None, offs, cnts))
        self.offsets, self.counts = list(offs), list(cnts)
        self.W = sum(self.counts)
        self.n_obs = 0
        self.n_max_all = max(w.n_max for w in wl)
        self.K_max = max(w.trials for w in wl)
        s = stream if stream is not None else _torch_stream()
        if s is not None:
            _check(lib().regc_set_stream(h, s))

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            lib().regc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- sampling ----------------------------------------------------------
    def run(self, n_sweeps: int):
        _check(lib().regc_run(self.h, int(n_sweeps)))

    def sync(self):
        _check(lib().regc_sync(self.h))

    @property
    def sweep(self) -> int:
        s = C.c_int64()
        _check(lib().regc_get_sweep(self.h, C.byref(s)))
        return s.value

    def walkers(self, xyz: bool = True):
        n = np.zeros(self.W, np.int32)
        e = np.zeros(self.W)
        lab = np.zeros(self.W, np.int32)
        x = np.zeros((self.W, self.n_max_all, 3)) if xyz else None
        _check(lib().regc_get_walkers(self.h, _p(n, _i32p), _p(e, _dp), _p(lab, _i32p), _p(x, _dp)))
        return {"n": n, "e": e, "label": lab, "xyz": x}

    def set_walkers(self, n, xyz, label=None):
        n = np.ascontiguousarray(n, dtype=np.int32)
        x = np.zeros((self.W, self.n_max_all, 3))
        for w in range(self.W):
            x[w, : n[w]] = np.asarray(xyz[w])[: n[w]]
        lab = None if label is None else np.ascontiguousarray(label, dtype=np.int32)
        _check(lib().regc_set_walkers(self.h, _p(n, _i32p), _p(x, _dp), _p(lab, _i32p)))

    def energies(self):
        e = np.zeros(self.W)
        _check(lib().regc_energies(self.h, _p(e, _dp)))
        return e

    def sample_count(self) -> int:
        c = C.c_int64()
        _check(lib().regc_sample_count(self.h, C.byref(c)))
        return c.value

    def samples(self):
        cnt = self.sample_count()
        e = np.zeros(cnt)
        n = np.zeros(cnt, np.int32)
        s = np.zeros(cnt, np.int32)
        got = C.c_int64()
        _check(lib().regc_get_samples(self.h, _p(e, _dp), _p(n, _i32p), _p(s, _i32p), cnt, C.byref(got)))
        return {"e": e[: got.value], "n": n[: got.value], "state": s[: got.value]}

    def clear_samples(self):
        _check(lib().regc_clear_samples(self.h))

    def stats(self):
        st = np.zeros((self.W, NSTAT), np.int64)
        att = np.zeros((4, self.W), np.int64)
        acc = np.zeros((4, self.W), np.int64)
        _check(lib().regc_get_stats(self.h, _p(st, _i64p), _p(att, _i64p), _p(acc, _i64p)))
        return {"stats": st, "swap_att": att, "swap_acc": acc}

    def count_pairs(self, on: bool = True):
        _check(lib().regc_count_pairs(self.h, int(on)))

    def pair_counts(self):
        a, b = C.c_int64(), C.c_int64()
        _check(lib().regc_get_pair_counts(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def histograms(self):
        h = np.zeros((self.W, self.n_max_all + 1), np.int64)
        _check(lib().regc_get_histograms(self.h, _p(h, _i64p)))
        return h

    def trace(self, cap_sweeps: int):
        words = (self.K_max + 31) // 32
        bits = np.zeros((cap_sweeps, self.W, words), np.uint32)
        nps = np.zeros((cap_sweeps, self.W), np.int32)
        got = C.c_int64()
        _check(lib().regc_get_trace(self.h, _p(bits, _u32p), _p(nps, _i32p), cap_sweeps, C.byref(got)))
        return bits[: got.value], nps[: got.value]

    def timing_enable(self, on: bool = True):
        _check(lib().regc_timing_enable(self.h, int(on)))

    def timing(self):
        a, b = C.c_double(), C.c_double()
        na, nb = C.c_int64(), C.c_int64()
        _check(lib().regc_timing_get(self.h, C.byref(a), C.byref(na), C.byref(b), C.byref(nb)))
        return {"ms_sweep": a.value, "n_sweep": na.value, "ms_swap": b.value, "n_swap": nb.value}

    def checkpoint(self) -> bytes:
        size = C.c_size_t()
        _check(lib().regc_checkpoint(self.h, None, 0, C.byref(size)))
        buf = C.create_string_buffer(size.value)
        _check(lib().regc_checkpoint(self.h, buf, size.value, C.byref(size)))
        return buf.raw

    def restore(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().regc_restore(self.h, buf, len(blob)))

    def set_proposal(self, mlp, alpha: float, cls: Optional[int] = None):
        """Learned insertion proposal from the network's current parameters with
        mixture weight alpha, for class `cls` of a batch or for every class (mlp None
        or alpha 0: the plain method)."""
        h = mlp.h if mlp is not None else None
        if cls is None:
            _check(lib().regc_set_proposal(self.h, h, float(alpha)))
        else:
            _check(lib().regc_set_class_proposal(self.h, int(cls), h, float(alpha)))

    def set_observables(self, dz: float, layer, dr: float, nr: int):
        """Record per-sample axial z-bin counts, layer pair counts by lateral distance
        and the layer population with every sample (None-like nr < 0 switches off)."""
        if nr < 0:
            _check(lib().regc_set_observables(self.h, None))
            self.n_obs = 0
            return
        spec = ObsSpec(float(dz), float(layer[0]), float(layer[1]), float(dr), int(nr))
        _check(lib().regc_set_observables(self.h, C.byref(spec)))
        p, k = C.c_void_p(), C.c_int()
        _check(lib().regc_observables_device(self.h, C.byref(p), C.byref(k)))
        self.n_obs = k.value

    def track_minima(self, on: bool = True):
        _check(lib().regc_track_minima(self.h, int(on)))

    def minima(self, cls: int = 0):
        """(e_min [n_max+1], xyz [n_max+1, n_max, 3]) of class cls."""
        nm = self.workloads[cls].n_max
        e = np.zeros(nm + 1)
        x = np.zeros((nm + 1, nm, 3))
        _check(lib().regc_get_minima(self.h, cls, _p(e, _dp), _p(x, _dp)))
        return e, x

    def observables(self):
        """Observable records [records * W, n_obs] (uint32), in the order of samples()."""
        recs = self.sample_count() // max(self.W, 1)
        out = np.zeros((max(recs, 1), self.W, self.n_obs), np.uint32)
        got = C.c_int64()
        _check(lib().regc_get_observables(self.h, _p(out, _u32p), recs, C.byref(got)))
        return out[: got.value].reshape(-1, self.n_obs)

    def capture_voxels(self, vox_dev_ptr: int, n_dev_ptr: int):
        """Voxel lists [W][n_max] (uint16) and N [W] of the walkers into device memory
        (asynchronous on the context's stream)."""
        _check(lib().regc_capture_voxels(self.h, C.c_void_p(vox_dev_ptr), C.c_void_p(n_dev_ptr)))

    def proposal_eval(self, n, xyz, skip, cls: int = 0):
        """The sampler's network on configurations: (logits [C, 4096], lse [C], lnp [C, 4096])."""
        n = np.ascontiguousarray(n, dtype=np.int32)
        nc = len(n)
        x = np.zeros((nc, self.n_max_all, 3))
        for k in range(nc):
            x[k, : n[k]] = np.asarray(xyz[k], dtype=np.float64).reshape(-1, 3)[: n[k]]
        sk = np.ascontiguousarray(skip, dtype=np.int32)
        lg = np.zeros((nc, 4096), np.float32)
        lse = np.zeros(nc)
        lnp = np.zeros((nc, 4096))
        _check(lib().regc_proposal_eval(self.h, cls, nc, _p(n, _i32p), _p(x, _dp), _p(sk, _i32p), _p(lg, _fp),
                                        _p(lse, _dp), _p(lnp, _dp)))
        return lg, lse, lnp

    def proposal_stats(self):
        """{'passes', 'cached', 'drawn', 'drawn_accepted'} of the learned proposal."""
        out = np.zeros(4, np.int64)
        _check(lib().regc_get_proposal_stats(self.h, _p(out, _i64p)))
        return dict(zip(("passes", "cached", "drawn", "drawn_accepted"), (int(x) for x in out)))


class Mbar:
    """Multistate reweighting on a T x mu grid (GPU)."""

    def __init__(self, t, mu, n_max: int, lambda1: float = 1.0, stream=None):
        self._keep = []
        g = _grid(t, mu, self._keep)
        self.t = np.asarray(t, dtype=np.float64)
        self.mu = np.asarray(mu, dtype=np.float64)
        self.n_max = n_max
        h = C.c_void_p()
        _check(lib().regc_mbar_create(C.byref(g), lambda1, n_max, C.byref(h)))
        self.h = h
        s = stream if stream is not None else _torch_stream()
        if s is not None:
            _check(lib().regc_mbar_set_stream(h, s))

    def close(self):
        if getattr(self, "h", None):
            lib().regc_mbar_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_samples(self, e, n, state):
        e = np.ascontiguousarray(e, dtype=np.float64)
        n = np.ascontiguousarray(n, dtype=np.int32)
        s = np.ascontiguousarray(state, dtype=np.int32)
        _check(lib().regc_mbar_set_samples(self.h, len(e), e.ctypes.data, n.ctypes.data, s.ctypes.data, 0))

    def set_samples_device(self, ns: int, e_ptr: int, n_ptr: int, s_ptr: int):
        _check(lib().regc_mbar_set_samples(self.h, int(ns), C.c_void_p(e_ptr), C.c_void_p(n_ptr),
                                           C.c_void_p(s_ptr), 1))

    def load_run(self, run: Regc, cls: int = 0, skip_records: int = 0):
        _check(lib().regc_mbar_load_run(self.h, run.h, cls, skip_records))

    def set_solver(self, method: int = 1, memory: int = 8):
        _check(lib().regc_mbar_set_solver(self.h, method, memory))

    def solve(self, tol: float = 1e-10, max_iter: int = 10000, allow_noconv: bool = False):
        f = np.zeros(len(self.t) * len(self.mu))
        it = C.c_int()
        d = C.c_double()
        rc = _check(lib().regc_mbar_solve(self.h, tol, max_iter, _p(f, _dp), C.byref(it), C.byref(d)),
                    allow=(ENOCONV,) if allow_noconv else ())
        return f, rc == OK, it.value, d.value

    def targets(self, t, mu):
        keep = []
        g = _grid(t, mu, keep)
        K = len(keep[0]) * len(keep[1])
        f, mn, me, me2 = np.zeros(K), np.zeros(K), np.zeros(K), np.zeros(K)
        pn = np.zeros((K, self.n_max + 1))
        ph = np.zeros(K, np.int32)
        _check(lib().regc_mbar_targets(self.h, C.byref(g), _p(f, _dp), _p(mn, _dp), _p(me, _dp), _p(me2, _dp),
                                       _p(pn, _dp), _p(ph, _i32p)))
        return {"f": f, "mean_n": mn, "mean_e": me, "mean_e2": me2, "p_n": pn, "phase": ph}

    def targets_static(self, t, mu):
        """regc_mbar_targets_static: the averages of targets() without p_n, with no
        allocation in the library."""
        keep = []
        g = _grid(t, mu, keep)
        K = len(keep[0]) * len(keep[1])
        f, mn, me, me2 = np.zeros(K), np.zeros(K), np.zeros(K), np.zeros(K)
        ph = np.zeros(K, np.int32)
        _check(lib().regc_mbar_targets_static(self.h, C.byref(g), _p(f, _dp), _p(mn, _dp), _p(me, _dp),
                                              _p(me2, _dp), _p(ph, _i32p)))
        return {"f": f, "mean_n": mn, "mean_e": me, "mean_e2": me2, "phase": ph}

    def reweight(self, t, mu, tol: float = 1e-10, max_iter: int = 10000, n_batches: int = 20, n_boot: int = 100,
                 record_size: int = 0, block_records: int = 0, seed: int = 1, n_sites: float = 0.0,
                 allow_noconv: bool = False):
        """Estimates with errors (regc_reweight): on the sampled grid f, direct mean N
        and its batch-means SE; on the target grid mean N, bootstrap SE, phase,
        coverage (n_sites > 0) and heat capacity with their SEs, p(N)."""
        keep = []
        g = _grid(t, mu, keep)
        K = len(keep[0]) * len(keep[1])
        S = len(self.t) * len(self.mu)
        o = ReweightOpts()
        lib().regc_default_reweight_opts(C.byref(o))
        o.n_batches, o.n_boot, o.record_size, o.block_records = n_batches, n_boot, record_size, block_records
        o.seed, o.n_sites = seed, n_sites
        out = {k: np.zeros(S) for k in ("f_states", "mean_state_n", "se_state_n")}
        for k in ("mean_n", "se_n", "coverage", "se_coverage", "heat_cap", "se_heat_cap"):
            out[k] = np.zeros(K)
        out["phase"] = np.zeros(K, np.int32)
        out["p_n"] = np.zeros((K, self.n_max + 1))
        cov = n_sites > 0
        rc = _check(lib().regc_reweight(
            self.h, C.byref(g), tol, max_iter, C.byref(o), _p(out["f_states"], _dp), _p(out["mean_state_n"], _dp),
            _p(out["se_state_n"], _dp), _p(out["mean_n"], _dp), _p(out["se_n"], _dp), _p(out["phase"], _i32p),
            _p(out["coverage"], _dp) if cov else None, _p(out["se_coverage"], _dp) if cov else None,
            _p(out["heat_cap"], _dp), _p(out["se_heat_cap"], _dp), _p(out["p_n"], _dp)),
            allow=(ENOCONV,) if allow_noconv else ())
        if not cov:
            del out["coverage"], out["se_coverage"]
        out["converged"] = rc == OK
        return out

    def set_observables(self, obs):
        """Per-sample observables [ns, n_obs] in the order of the samples (uint32)."""
        ob = np.ascontiguousarray(obs, dtype=np.uint32)
        _check(lib().regc_mbar_set_observables(self.h, ob.ctypes.data_as(C.c_void_p), ob.shape[1], 0))
        self.n_obs = ob.shape[1]

    def observables(self, t, mu, n_obs: int):
        """Reweighted observables: mean [nT, nMu, n_obs] and the average conditional on
        N, cond [nT, n_max+1, n_obs]."""
        keep = []
        g = _grid(t, mu, keep)
        mean = np.zeros((len(t), len(mu), n_obs))
        cond = np.zeros((len(t), self.n_max + 1, n_obs))
        _check(lib().regc_mbar_observables(self.h, C.byref(g), _p(mean, _dp), _p(cond, _dp)))
        return mean, cond

    def timing(self):
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().regc_mbar_timing(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value


_fp = C.POINTER(C.c_float)
_u16p = C.POINTER(C.c_uint16)


class Mlp:
    """The learned insertion proposal network on the GPU (training and evaluation)."""

    def __init__(self, params=None, stream=None):
        cnt = C.c_int64()
        _check(lib().regc_mlp_param_count(C.byref(cnt)))
        self.n_params = cnt.value
        flat = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        if flat is not None and flat.size != self.n_params:
            raise ValueError("parameter vector has the wrong length")
        h = C.c_void_p()
        _check(lib().regc_mlp_create(_p(flat, _fp), C.byref(h)))
        self.h = h
        s = stream if stream is not None else _torch_stream()
        if s is not None:
            _check(lib().regc_mlp_set_stream(h, s))

    def close(self):
        if getattr(self, "h", None):
            lib().regc_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        _check(lib().regc_mlp_get_params(self.h, _p(out, _fp)))
        return out

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        _check(lib().regc_mlp_set_params(self.h, _p(flat, _fp)))

    @staticmethod
    def _batch(vox, n, excl):
        vox = np.ascontiguousarray(vox, dtype=np.uint16)
        return vox, np.ascontiguousarray(n, dtype=np.int32), np.ascontiguousarray(excl, dtype=np.int32)

    def forward(self, vox, n, excl):
        vox, n, excl = self._batch(vox, n, excl)
        B, nmax = vox.shape
        out = np.zeros((B, 4096), np.float32)
        _check(lib().regc_mlp_forward(self.h, B, nmax, _p(vox, _u16p), _p(n, _i32p), _p(excl, _i32p), _p(out, _fp)))
        return out

    def loss_grads(self, vox, n, excl, target):
        vox, n, excl = self._batch(vox, n, excl)
        tgt = np.ascontiguousarray(target, dtype=np.int32)
        B, nmax = vox.shape
        loss = C.c_double()
        g = np.zeros(self.n_params, np.float32)
        _check(lib().regc_mlp_loss_grads(self.h, B, nmax, _p(vox, _u16p), _p(n, _i32p), _p(excl, _i32p),
                                         _p(tgt, _i32p), C.byref(loss), _p(g, _fp)))
        return loss.value, g

    def step(self, vox, n, excl, target, lr: float = 1e-3):
        """One Adam step on the batch; returns (loss, the gradient applied)."""
        vox, n, excl = self._batch(vox, n, excl)
        tgt = np.ascontiguousarray(target, dtype=np.int32)
        B, nmax = vox.shape
        loss = C.c_double()
        g = np.zeros(self.n_params, np.float32)
        _check(lib().regc_mlp_step(self.h, B, nmax, _p(vox, _u16p), _p(n, _i32p), _p(excl, _i32p), _p(tgt, _i32p),
                                   lr, C.byref(loss), _p(g, _fp)))
        return loss.value, g

    def train(self, n_examples: int, nmax: int, vox_dev_ptr: int, n_dev_ptr: int, steps: int, batch: int = 256,
              lr: float = 1e-3, seed: int = 1):
        loss = C.c_double()
        _check(lib().regc_mlp_train(self.h, n_examples, nmax, C.c_void_p(vox_dev_ptr), C.c_void_p(n_dev_ptr), steps,
                                    batch, lr, seed, C.byref(loss)))
        return loss.value

    def timing(self):
        ms = C.c_double()
        st = C.c_int64()
        _check(lib().regc_mlp_timing(self.h, C.byref(ms), C.byref(st)))
        return ms.value, st.value


def aiat_phase(e_min, mu):
    """aiAT@REGC phase map along mu from the lowest recorded energies per N."""
    e = np.ascontiguousarray(e_min, dtype=np.float64)
    m = np.ascontiguousarray(mu, dtype=np.float64)
    out = np.zeros(len(m), dtype=np.int32)
    _check(lib().regc_aiat_phase(_p(e, _dp), len(e) - 1, len(m), _p(m, _dp), _p(out, _i32p)))
    return out



def batch_means(state, n, n_states: int, n_batches: int = 20):
    """regc_batch_means: per-state mean N and batch-means SE.  state and n are numpy
    arrays, or int32 torch tensors on the GPU (read in place, on torch's stream)."""
    mean, se = np.zeros(n_states), np.zeros(n_states)
    if hasattr(state, "data_ptr"):
        assert state.dtype == n.dtype and str(state.dtype) == "torch.int32" and state.is_cuda and n.is_cuda
        assert state.is_contiguous() and n.is_contiguous() and state.numel() == n.numel()
        _check(lib().regc_batch_means(state.numel(), C.c_void_p(state.data_ptr()), C.c_void_p(n.data_ptr()),
                                      n_states, n_batches, 1, _p(mean, _dp), _p(se, _dp), _torch_stream()))
    else:
        s = np.ascontiguousarray(state, dtype=np.int32)
        v = np.ascontiguousarray(n, dtype=np.int32)
        assert s.shape == v.shape
        _check(lib().regc_batch_means(len(s), _p(s, _i32p), _p(v, _i32p), n_states, n_batches, 0, _p(mean, _dp),
                                      _p(se, _dp), _torch_stream()))
    return mean, se
