"""CPU oracle of the REGC method (arXiv:1908.11118) -- TEST INFRASTRUCTURE ONLY.

Plain FP64 C code (regc_oracle.c: Philox, LJ energies, the GC/displacement chain,
the replica-exchange step; mbar_oracle.c: the naive multistate reweighting) plus a
ctypes wrapper.  Only tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It never imports the HIP package and shares no code with it.

Any object with the attributes of a workload (slab, lx, ly, zlo, zhi, t, mu, n_max,
eps_gg, sig_gg, eps_gs, sig_gs, rc, shifted, mode, hc_frac, lambda1, seed, p_disp,
p_ins, max_disp, trials_per_sweep, swap_every, sample_every, swap_scheme, sites)
describes a problem.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_DIR, "liboracle.so")
_SOURCES = ["regc_oracle.c", "mbar_oracle.c"]
NSTAT = 10
STAT_NAMES = ["disp_att", "disp_acc", "ins_att", "ins_acc", "del_att", "del_acc",
              "cap_rej", "empty_rej", "wall_rej", "core_rej"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc: -O2, no FP contraction, no fast-math, OpenMP."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", _LIB_PATH] + [os.path.join(_DIR, s) for s in _SOURCES] + ["-lm"]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u32p = C.POINTER(C.c_uint32)


class _Config(C.Structure):
    _fields_ = [("eps_gg", C.c_double), ("sig_gg", C.c_double), ("eps_gs", C.c_double),
                ("sig_gs", C.c_double), ("rc", C.c_double), ("shifted", C.c_int), ("mode", C.c_int),
                ("hc_frac", C.c_double), ("n_slab", C.c_int), ("slab", _dp),
                ("lx", C.c_double), ("ly", C.c_double), ("zlo", C.c_double), ("zhi", C.c_double),
                ("n_sites", C.c_int), ("sites", _dp), ("lambda1", C.c_double), ("n_max", C.c_int),
                ("n_t", C.c_int), ("n_mu", C.c_int), ("t", _dp), ("mu", _dp),
                ("seed", C.c_uint64), ("p_disp", C.c_double), ("p_ins", C.c_double),
                ("max_disp", C.c_double), ("trials_per_sweep", C.c_int), ("swap_every", C.c_int),
                ("sample_every", C.c_int), ("swap_scheme", C.c_int), ("walker_offset", C.c_int),
                ("class_id", C.c_int), ("net", C.POINTER(C.c_float)), ("alpha", C.c_double),
                ("schedule", C.c_int), ("x0", C.c_double), ("mc_cycles", C.c_int),
                ("obs_dz", C.c_double), ("obs_layer_lo", C.c_double), ("obs_layer_hi", C.c_double),
                ("obs_dr", C.c_double), ("obs_nr", C.c_int), ("md_steps", C.c_int), ("md_dt", C.c_double),
                ("md_tau", C.c_double)]


class _Walkers(C.Structure):
    _fields_ = [("n", _i32p), ("e", _dp), ("label", _i32p), ("wos", _i32p), ("xyz", _dp),
                ("site", _i32p), ("stats", _i64p), ("swap_att", _i64p), ("swap_acc", _i64p),
                ("margin", C.POINTER(C.c_float)), ("obs", _dp), ("min_e", _dp), ("min_xyz", _dp),
                ("vel", _dp), ("tv", _dp)]


def _declare(L):
    L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.orc_lj.argtypes = [C.c_double] * 4 + [C.c_int]
    L.orc_lj.restype = C.c_double
    L.orc_state_lnz.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int]
    L.orc_state_lnz.restype = C.c_double
    L.orc_total_energy.argtypes = [C.POINTER(_Config), C.c_int, _dp]
    L.orc_total_energy.restype = C.c_double
    L.orc_run.argtypes = [C.POINTER(_Config), C.POINTER(_Walkers), _i64p, C.c_int64,
                          _dp, _i32p, _i32p, C.c_int64, _i64p, _u32p, _i32p, C.c_int]
    L.orc_run.restype = C.c_int
    L.orc_swap_step.argtypes = [C.POINTER(_Config), C.POINTER(_Walkers), C.c_int64]
    L.orc_swap_lnratio.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double,
                                   C.c_double, C.c_int, C.c_double, C.c_int]
    L.orc_swap_lnratio.restype = C.c_double
    L.orc_voxel_of.argtypes = [C.POINTER(_Config), _dp]
    L.orc_voxel_of.restype = C.c_int
    L.orc_net_logits.argtypes = [C.POINTER(_Config), _dp, C.c_int, C.c_int, C.POINTER(C.c_float)]
    L.orc_net_logits.restype = C.c_double
    L.orc_gumbel_argmax.argtypes = [C.POINTER(_Config), C.POINTER(C.c_float), C.c_uint32, C.c_uint32,
                                    C.c_uint32, _dp]
    L.orc_gumbel_argmax.restype = C.c_int
    L.orc_md_forces.argtypes = [C.POINTER(_Config), _dp, C.c_int, _dp]
    L.orc_md_forces.restype = C.c_double
    L.orc_aiat_phase.argtypes = [C.c_int, _dp, C.c_int, _dp, _i32p]
    L.orc_checkpoint_size.argtypes = [C.POINTER(_Config)]
    L.orc_checkpoint_size.restype = C.c_size_t
    L.orc_checkpoint.argtypes = [C.POINTER(_Config), C.POINTER(_Walkers), C.c_int64, C.c_void_p, C.c_size_t]
    L.orc_checkpoint.restype = C.c_int
    L.orc_restore.argtypes = [C.POINTER(_Config), C.POINTER(_Walkers), _i64p, C.c_void_p, C.c_size_t]
    L.orc_restore.restype = C.c_int
    L.orc_obs_count.argtypes = [C.POINTER(_Config)]
    L.orc_obs_count.restype = C.c_int
    L.orc_observables.argtypes = [C.POINTER(_Config), _dp, C.c_int, _dp]
    L.orc_mbar_observables.argtypes = [C.c_int, _dp, _dp, C.c_int64, _dp, _i32p, _dp, C.c_int, _dp, C.c_int,
                                       _dp, _dp, C.c_int]
    L.orc_mbar_solve.argtypes = [C.c_int, _dp, _dp, _i64p, C.c_int64, _dp, _i32p, C.c_double,
                                 C.c_int, _dp, _dp, C.POINTER(C.c_int), _dp, C.c_int]
    L.orc_mbar_solve.restype = C.c_int
    L.orc_mbar_iterate.argtypes = [C.c_int, _dp, _dp, _i64p, C.c_int64, _dp, _i32p, _dp, _dp,
                                   _dp, C.c_int]
    L.orc_mbar_targets.argtypes = [C.c_int, _dp, _dp, C.c_int64, _dp, _i32p, _dp, C.c_int, _dp,
                                   _dp, _dp, _dp, _dp, _i32p, C.c_int]
    L.orc_batch_means.argtypes = [C.c_int, C.c_int64, _i32p, _i32p, C.c_int, _dp, _dp]
    L.orc_boot_multiplicity.argtypes = [C.c_int64, C.c_int64, C.c_int, C.c_uint64, _i32p]
    L.orc_mbar_bootstrap.argtypes = [C.c_int, _dp, _dp, C.c_int64, _dp, _i32p, _i32p, C.c_int64, C.c_int64,
                                     C.c_int, C.c_uint64, _dp, C.c_double, C.c_int, C.c_int, _dp, _dp, C.c_int,
                                     _dp, _dp, _dp, _dp, C.c_int]
    L.orc_mbar_bootstrap.restype = C.c_int
    L.orc_heat_capacity_coverage.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp]


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def default_threads() -> int:
    """Host threads for the oracle: the CPUs this process may run on, capped by
    OMP_NUM_THREADS when that is set."""
    try:
        n = max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return n


# ----------------------------------------------------------------------------
def philox4x32_10(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, _u32p), _p(k, _u32p), _p(out, _u32p))
    return out


def lj(r2: float, eps: float = 1.0, sig: float = 1.0, rc: float = 2.5, shifted: int = 1) -> float:
    return lib().orc_lj(r2, eps, sig, rc, shifted)


def state_lnz(T: float, mu: float, lambda1: float = 1.0, mode: int = 0) -> float:
    return lib().orc_state_lnz(T, mu, lambda1, mode)


def state_arrays(w):
    """beta_s and lnz_s of every state s = l*n_mu + m."""
    t = np.asarray(w.t, dtype=np.float64)
    mu = np.asarray(w.mu, dtype=np.float64)
    beta = np.empty(len(t) * len(mu))
    lnz = np.empty_like(beta)
    for l, T in enumerate(t):
        for m, u in enumerate(mu):
            beta[l * len(mu) + m] = 1.0 / T
            lnz[l * len(mu) + m] = state_lnz(float(T), float(u), w.lambda1, w.mode)
    return beta, lnz


class Chain:
    """All walkers of one REGC simulation, advanced by the C oracle.

    net / alpha: the learned insertion proposal (FP32 parameter vector of the
    network, mixture weight of its branch); alpha = 0 or net = None is the plain
    method."""

    def __init__(self, w, n_threads: int | None = None, walker_offset: int = 0, class_id: int = 0,
                 net=None, alpha: float = 0.0, observables=None):
        self.w = w
        self.S = len(w.t) * len(w.mu)
        self.n_max = int(w.n_max)
        self.K = w.trials_per_sweep if w.trials_per_sweep > 0 else self.n_max + 1
        if getattr(w, "schedule", 0) == 1:
            self.K = 1 + int(getattr(w, "mc_cycles", 10)) * self.n_max     # trials per REGC step, at most
        self.n_threads = n_threads or default_threads()
        self._slab = np.ascontiguousarray(w.slab, dtype=np.float64).reshape(-1, 3)
        sites = getattr(w, "sites", None)
        self._sites = (np.ascontiguousarray(sites, dtype=np.float64).reshape(-1, 3)
                       if sites is not None else np.zeros((0, 3)))
        self._t = np.ascontiguousarray(w.t, dtype=np.float64)
        self._mu = np.ascontiguousarray(w.mu, dtype=np.float64)
        c = _Config()
        c.eps_gg, c.sig_gg, c.eps_gs, c.sig_gs, c.rc = w.eps_gg, w.sig_gg, w.eps_gs, w.sig_gs, w.rc
        c.shifted, c.mode, c.hc_frac = w.shifted, w.mode, w.hc_frac
        c.n_slab = self._slab.shape[0]
        c.slab = _p(self._slab, _dp)
        c.lx, c.ly, c.zlo, c.zhi = w.lx, w.ly, w.zlo, w.zhi
        c.n_sites = self._sites.shape[0]
        c.sites = _p(self._sites, _dp)
        c.lambda1, c.n_max = w.lambda1, w.n_max
        c.n_t, c.n_mu = len(self._t), len(self._mu)
        c.t, c.mu = _p(self._t, _dp), _p(self._mu, _dp)
        c.seed = w.seed
        c.p_disp, c.p_ins, c.max_disp = w.p_disp, w.p_ins, w.max_disp
        c.trials_per_sweep, c.swap_every = w.trials_per_sweep, w.swap_every
        c.sample_every, c.swap_scheme = w.sample_every, w.swap_scheme
        c.walker_offset, c.class_id = walker_offset, class_id
        self._net = None
        if net is not None:
            self._net = np.ascontiguousarray(net, dtype=np.float32).ravel()
            c.net = self._net.ctypes.data_as(C.POINTER(C.c_float))
        c.alpha = float(alpha)
        c.schedule = int(getattr(w, "schedule", 0))
        c.x0 = float(getattr(w, "x0", 0.99))
        c.mc_cycles = int(getattr(w, "mc_cycles", 10))
        c.md_steps = int(getattr(w, "md_steps", 0))
        c.md_dt = float(getattr(w, "md_dt", 0.005))
        c.md_tau = float(getattr(w, "md_tau", 0.1))
        if observables:
            c.obs_dz = float(observables["dz"])
            c.obs_layer_lo, c.obs_layer_hi = (float(v) for v in observables["layer"])
            c.obs_dr, c.obs_nr = float(observables["dr"]), int(observables["nr"])
        self.cfg = c
        self.n_obs = lib().orc_obs_count(C.byref(c))
        S = self.S
        # initial state: empty walkers, walker w holds state w
        self.n = np.zeros(S, dtype=np.int32)
        self.e = np.zeros(S, dtype=np.float64)
        self.label = np.arange(S, dtype=np.int32)
        self.wos = np.arange(S, dtype=np.int32)
        self.xyz = np.zeros((S, self.n_max, 3), dtype=np.float64)
        self.site = np.full((S, self.n_max), -1, dtype=np.int32)
        self.stats = np.zeros((S, NSTAT), dtype=np.int64)
        self.swap_att = np.zeros((4, S), dtype=np.int64)
        self.swap_acc = np.zeros((4, S), dtype=np.int64)
        self.sweep = np.zeros(1, dtype=np.int64)
        # lowest-energy recorded configuration per N
        self.min_e = np.full(self.n_max + 1, np.inf)
        self.min_xyz = np.zeros((self.n_max + 1, self.n_max, 3))
        # molecular dynamics: velocities and the temperature they belong to (0: none yet)
        self.vel = np.zeros((S, self.n_max, 3))
        self.tv = np.zeros(S)

    def _walkers(self):
        W = _Walkers()
        W.n, W.e = _p(self.n, _i32p), _p(self.e, _dp)
        W.label, W.wos = _p(self.label, _i32p), _p(self.wos, _i32p)
        W.xyz = _p(self.xyz, _dp)
        W.site = _p(self.site, _i32p) if self.w.mode == 2 else None
        W.stats = _p(self.stats, _i64p)
        W.swap_att, W.swap_acc = _p(self.swap_att, _i64p), _p(self.swap_acc, _i64p)
        W.min_e, W.min_xyz = _p(self.min_e, _dp), _p(self.min_xyz, _dp)
        W.vel, W.tv = _p(self.vel, _dp), _p(self.tv, _dp)
        return W

    def set_walkers(self, n, xyz, e=None, label=None):
        """Load explicit configurations (energies recomputed unless given)."""
        self.n[:] = n
        self.xyz[:] = 0.0
        for w in range(self.S):
            self.xyz[w, : n[w]] = xyz[w][: n[w]]
        if e is None:
            e = [self.energy(self.xyz[w, : n[w]]) for w in range(self.S)]
        self.e[:] = e
        if label is not None:
            self.label[:] = label
            self.wos[self.label] = np.arange(self.S, dtype=np.int32)

    def energy(self, xyz) -> float:
        x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        return lib().orc_total_energy(C.byref(self.cfg), x.shape[0], _p(x, _dp))

    def run(self, n_sweeps: int, trace: bool = False, margins: bool = False):
        """Advance n_sweeps sweeps.  Returns dict with samples (e, n, state) and,
        when trace is set, accept bits [n_sweeps, S, words] and N [n_sweeps, S];
        with margins, the learned proposal's per-trial decision margins
        [n_sweeps, S, K] (+inf where the network took no part)."""
        S = self.S
        every = self.w.sample_every
        s0 = int(self.sweep[0])
        n_samp = 0
        if every > 0:
            n_samp = ((s0 + n_sweeps) // every - s0 // every) * S
        se = np.zeros(max(n_samp, 1), dtype=np.float64)
        sn = np.zeros(max(n_samp, 1), dtype=np.int32)
        ss = np.zeros(max(n_samp, 1), dtype=np.int32)
        cnt = np.zeros(1, dtype=np.int64)
        words = (self.K + 31) // 32
        tb = np.zeros((n_sweeps, S, words), dtype=np.uint32) if trace else None
        tn = np.zeros((n_sweeps, S), dtype=np.int32) if trace else None
        W = self._walkers()
        ob = np.zeros((max(n_samp, 1), self.n_obs), dtype=np.float64) if self.n_obs else None
        if ob is not None:
            W.obs = _p(ob, _dp)
        mg = np.zeros((n_sweeps, S, self.K), dtype=np.float32) if margins else None
        if margins:
            W.margin = mg.ctypes.data_as(C.POINTER(C.c_float))
        rc = lib().orc_run(C.byref(self.cfg), C.byref(W), _p(self.sweep, _i64p), n_sweeps,
                           _p(se, _dp), _p(sn, _i32p), _p(ss, _i32p), n_samp, _p(cnt, _i64p),
                           _p(tb, _u32p), _p(tn, _i32p), self.n_threads)
        if rc != 0:
            raise RuntimeError(f"oracle run failed ({rc})")
        k = int(cnt[0])
        out = {"e": se[:k], "n": sn[:k], "state": ss[:k]}
        if trace:
            out["bits"], out["trace_n"] = tb, tn
        if margins:
            out["margin"] = mg
        if ob is not None:
            out["obs"] = ob[:k]
        return out

    def observables(self, xyz):
        """Observables (z-bin counts, layer pair counts by lateral distance, layer
        population) of one configuration."""
        x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        out = np.zeros(self.n_obs)
        lib().orc_observables(C.byref(self.cfg), _p(x, _dp), x.shape[0], _p(out, _dp))
        return out

    def md_forces(self, xyz):
        """(potential energy, forces [n, 3]) of a configuration."""
        x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        f = np.zeros_like(x)
        e = lib().orc_md_forces(C.byref(self.cfg), _p(x, _dp), x.shape[0], _p(f, _dp))
        return e, f

    def voxel_of(self, p) -> int:
        q = np.ascontiguousarray(p, dtype=np.float64).reshape(3)
        return lib().orc_voxel_of(C.byref(self.cfg), _p(q, _dp))

    def net_logits(self, xyz, skip: int = -1):
        """Network logits [4096] (FP32) for the occupancy of xyz without particle
        `skip`, and the FP64 log-normaliser."""
        if self._net is None:
            raise ValueError("no network attached")
        x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        out = np.zeros(4096, dtype=np.float32)
        lse = lib().orc_net_logits(C.byref(self.cfg), _p(x, _dp), x.shape[0], int(skip),
                                   out.ctypes.data_as(C.POINTER(C.c_float)))
        return out, lse

    def gumbel_argmax(self, logits, t: int, sweep: int, walker: int):
        lg = np.ascontiguousarray(logits, dtype=np.float32)
        gap = np.zeros(1)
        v = lib().orc_gumbel_argmax(C.byref(self.cfg), lg.ctypes.data_as(C.POINTER(C.c_float)), t, sweep,
                                    walker, _p(gap, _dp))
        return v, float(gap[0])

    def checkpoint(self) -> bytes:
        """The sampling state between sweeps (the HIP library's checkpoint layout)."""
        size = lib().orc_checkpoint_size(C.byref(self.cfg))
        buf = C.create_string_buffer(size)
        rc = lib().orc_checkpoint(C.byref(self.cfg), C.byref(self._walkers()), int(self.sweep[0]), buf, size)
        if rc != 0:
            raise RuntimeError(f"oracle checkpoint failed ({rc})")
        return buf.raw

    def restore(self, blob: bytes):
        """Continue from a checkpoint (the oracle's or the HIP library's)."""
        buf = C.create_string_buffer(bytes(blob), len(blob))
        rc = lib().orc_restore(C.byref(self.cfg), C.byref(self._walkers()), _p(self.sweep, _i64p), buf, len(blob))
        if rc != 0:
            raise ValueError("checkpoint does not match this oracle configuration")

    def swap_step(self, q: int):
        W = self._walkers()
        lib().orc_swap_step(C.byref(self.cfg), C.byref(W), q)


def swap_lnratio(beta_a, lnz_a, beta_b, lnz_b, e_i, n_i, e_j, n_j) -> float:
    return lib().orc_swap_lnratio(beta_a, lnz_a, beta_b, lnz_b, e_i, int(n_i), e_j, int(n_j))


# ----------------------------------------------------------------------------
def mbar_solve(beta, lnz, omega, e, n, tol=1e-10, max_iter=10000, f0=None, n_threads=None):
    """Naive self-consistent solution.  Returns (f, logd, converged, iters, delta)."""
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    lnz = np.ascontiguousarray(lnz, dtype=np.float64)
    omega = np.ascontiguousarray(omega, dtype=np.int64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.int32)
    S = len(beta)
    f = np.zeros(S) if f0 is None else np.array(f0, dtype=np.float64)
    logd = np.zeros(len(e))
    it = C.c_int(0)
    delta = np.zeros(1)
    rc = lib().orc_mbar_solve(S, _p(beta, _dp), _p(lnz, _dp), _p(omega, _i64p), len(e), _p(e, _dp),
                              _p(n, _i32p), tol, max_iter, _p(f, _dp), _p(logd, _dp), C.byref(it),
                              _p(delta, _dp), n_threads or default_threads())
    return f, logd, rc == 0, it.value, float(delta[0])


def mbar_iterate(beta, lnz, omega, e, n, f_in, n_threads=None):
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    lnz = np.ascontiguousarray(lnz, dtype=np.float64)
    omega = np.ascontiguousarray(omega, dtype=np.int64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.int32)
    f_in = np.ascontiguousarray(f_in, dtype=np.float64)
    f_out = np.zeros_like(f_in)
    logd = np.zeros(len(e))
    lib().orc_mbar_iterate(len(beta), _p(beta, _dp), _p(lnz, _dp), _p(omega, _i64p), len(e),
                           _p(e, _dp), _p(n, _i32p), _p(f_in, _dp), _p(f_out, _dp), _p(logd, _dp),
                           n_threads or default_threads())
    return f_out, logd


def mbar_targets(tbeta, tlnz, e, n, logd, n_max, n_threads=None):
    """Returns dict f, mean_n, mean_e, mean_e2, p_n [T, n_max+1], phase."""
    tbeta = np.ascontiguousarray(tbeta, dtype=np.float64)
    tlnz = np.ascontiguousarray(tlnz, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.int32)
    logd = np.ascontiguousarray(logd, dtype=np.float64)
    T = len(tbeta)
    f = np.zeros(T)
    mn, me, me2 = np.zeros(T), np.zeros(T), np.zeros(T)
    pn = np.zeros((T, n_max + 1))
    ph = np.zeros(T, dtype=np.int32)
    lib().orc_mbar_targets(T, _p(tbeta, _dp), _p(tlnz, _dp), len(e), _p(e, _dp), _p(n, _i32p),
                           _p(logd, _dp), n_max, _p(f, _dp), _p(mn, _dp), _p(me, _dp), _p(me2, _dp),
                           _p(pn, _dp), _p(ph, _i32p), n_threads or default_threads())
    return {"f": f, "mean_n": mn, "mean_e": me, "mean_e2": me2, "p_n": pn, "phase": ph}


def mbar_observables(tbeta, tlnz, e, n, logd, n_max, obs, n_threads=None):
    """Reweighted observables at T target states: mean [T, n_obs] and the average
    conditional on N, cond [T, n_max+1, n_obs] (0 where p(N) = 0)."""
    tbeta = np.ascontiguousarray(tbeta, dtype=np.float64)
    tlnz = np.ascontiguousarray(tlnz, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.int32)
    logd = np.ascontiguousarray(logd, dtype=np.float64)
    obs = np.ascontiguousarray(obs, dtype=np.float64)
    T, no = len(tbeta), obs.shape[1]
    mean = np.zeros((T, no))
    cond = np.zeros((T, n_max + 1, no))
    lib().orc_mbar_observables(T, _p(tbeta, _dp), _p(tlnz, _dp), len(e), _p(e, _dp), _p(n, _i32p), _p(logd, _dp),
                               n_max, _p(obs, _dp), no, _p(mean, _dp), _p(cond, _dp), n_threads or default_threads())
    return mean, cond


def aiat_phase(min_e, mu):
    """aiAT@REGC phase (the N of lowest E_min(N) - E_min(0) - N mu) at each mu."""
    me = np.ascontiguousarray(min_e, dtype=np.float64)
    m = np.ascontiguousarray(mu, dtype=np.float64)
    out = np.zeros(len(m), dtype=np.int32)
    lib().orc_aiat_phase(len(me) - 1, _p(me, _dp), len(m), _p(m, _dp), _p(out, _i32p))
    return out



def batch_means(n_states, state, n, n_batches=20):
    """Per sampled state: mean N and its batch-means standard error (NaN for a state
    with fewer samples than batches)."""
    st = np.ascontiguousarray(state, dtype=np.int32)
    nn = np.ascontiguousarray(n, dtype=np.int32)
    mean, se = np.zeros(n_states), np.zeros(n_states)
    lib().orc_batch_means(n_states, len(st), _p(st, _i32p), _p(nn, _i32p), n_batches, _p(mean, _dp), _p(se, _dp))
    return mean, se


def boot_multiplicity(records, block, replicate, seed):
    """How often each record occurs in moving-block bootstrap replicate `replicate`."""
    out = np.zeros(records, dtype=np.int32)
    lib().orc_boot_multiplicity(records, block, replicate, seed, _p(out, _i32p))
    return out


def mbar_bootstrap(beta, lnz, e, n, state, record_size, block, n_boot, seed, f_start, tbeta, tlnz, n_max,
                   tol=1e-10, max_iter=100000, n_threads=None):
    """Bootstrap standard errors of <N> and C at target states.  Returns (se_n, se_c,
    rep_n [n_boot, T], rep_c [n_boot, T], converged)."""
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    lnz = np.ascontiguousarray(lnz, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.int32)
    st = np.ascontiguousarray(state, dtype=np.int32)
    f0 = np.ascontiguousarray(f_start, dtype=np.float64)
    tbeta = np.ascontiguousarray(tbeta, dtype=np.float64)
    tlnz = np.ascontiguousarray(tlnz, dtype=np.float64)
    T = len(tbeta)
    se_n, se_c = np.zeros(T), np.zeros(T)
    rn, rcap = np.zeros((n_boot, T)), np.zeros((n_boot, T))
    rc = lib().orc_mbar_bootstrap(len(beta), _p(beta, _dp), _p(lnz, _dp), len(e), _p(e, _dp), _p(n, _i32p),
                                  _p(st, _i32p), record_size, block, n_boot, seed, _p(f0, _dp), tol, max_iter, T,
                                  _p(tbeta, _dp), _p(tlnz, _dp), n_max, _p(se_n, _dp), _p(se_c, _dp), _p(rn, _dp),
                                  _p(rcap, _dp), n_threads or default_threads())
    return se_n, se_c, rn, rcap, rc == 0


def heat_capacity_coverage(tbeta, mean_n, mean_e, mean_e2, n_sites):
    """C = beta^2 (<E^2> - <E>^2) and theta = <N> / n_sites at each target."""
    tbeta = np.ascontiguousarray(tbeta, dtype=np.float64)
    a, b, c = (np.ascontiguousarray(x, dtype=np.float64) for x in (mean_n, mean_e, mean_e2))
    hc, cov = np.zeros(len(tbeta)), np.zeros(len(tbeta))
    lib().orc_heat_capacity_coverage(len(tbeta), _p(tbeta, _dp), _p(a, _dp), _p(b, _dp), _p(c, _dp), float(n_sites),
                                     _p(hc, _dp), _p(cov, _dp))
    return hc, cov
