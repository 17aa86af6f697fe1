"""Seeded synthetic inputs for REGC runs: frozen LJ slabs, (T, mu) grids and the
five workload presets.

This module holds input construction only (geometry and parameter values); none of
the sampling or reweighting arithmetic lives here, so both the HIP library's tests
and the CPU oracle's tests may use it.

Geometry reading (the paper's own LJ system, Sec. III.A and the Appendix, is an
fcc(111) A18 slab with eV parameters; the workloads here are LJ reduced units):
a slab of `layers` square nets of n x n atoms with in-plane spacing s = L/n,
interlayer spacing s/sqrt(2), alternate layers shifted by (s/2, s/2) (fcc(100)
stacking), the top layer in the plane z = z_lo = 0.  Gas lives in
[0, Lx) x [0, Ly) x [z_lo, z_lo + H], periodic in x and y, hard walls in z.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


def linear_grid(lo: float, hi: float, n: int) -> np.ndarray:
    """n values from lo to hi, endpoints included (uniform spacing as in Sec. III.A)."""
    if n == 1:
        return np.array([lo], dtype=np.float64)
    return np.array([lo + (hi - lo) * k / (n - 1) for k in range(n)], dtype=np.float64)


def fcc100_slab(n: int, layers: int, box: float, rc: Optional[float] = None) -> np.ndarray:
    """Square-net fcc(100)-stacked slab, n x n atoms per layer, top layer at z = 0.

    Atoms deeper than rc below the top plane never interact with the gas (the gas
    is confined to z >= 0) and are dropped when rc is given.
    Returns float64 [n_atoms, 3] with x, y in [0, box).
    """
    s = box / n
    dz = s / math.sqrt(2.0)
    out = []
    for k in range(layers):
        off = 0.5 * s if (k % 2) else 0.0
        z = -k * dz
        if rc is not None and -z >= rc:
            continue
        for j in range(n):
            for i in range(n):
                out.append(((i * s + off) % box, (j * s + off) % box, z))
    return np.array(out, dtype=np.float64).reshape(-1, 3)


def hollow_sites(n: int, box: float, height: float, second_height: Optional[float] = None,
                 n_second: int = 0) -> np.ndarray:
    """Adsorption sites above a square net: the n*n four-fold hollow positions at
    `height`, plus optionally the first `n_second` top-site positions at
    `second_height` (used for small interacting lattice-gas systems)."""
    s = box / n
    out = [((i + 0.5) * s, (j + 0.5) * s, height) for j in range(n) for i in range(n)]
    if n_second:
        extra = [(i * s, j * s, second_height) for j in range(n) for i in range(n)]
        out.extend(extra[:n_second])
    return np.array(out, dtype=np.float64).reshape(-1, 3)


@dataclasses.dataclass
class Workload:
    """One REGC problem: potential, surface, box, state grid and schedule."""
    name: str
    slab: np.ndarray
    lx: float
    ly: float
    zlo: float
    zhi: float
    t: np.ndarray
    mu: np.ndarray
    n_max: int
    eps_gg: float = 1.0
    sig_gg: float = 1.0
    eps_gs: float = 1.0
    sig_gs: float = 1.0
    rc: float = 2.5
    shifted: int = 1
    mode: int = 0               # 0 LJ, 1 ideal gas, 2 site lattice (oracle only)
    hc_frac: float = 0.5
    lambda1: float = 1.0
    seed: int = 1
    p_disp: float = 0.5
    p_ins: float = 0.25
    max_disp: float = 0.2
    trials_per_sweep: int = 0   # 0: n_max + 1 (state-independent sweep length)
    swap_every: int = 10
    sample_every: int = 1
    swap_scheme: int = 0
    n_sweeps: int = 1000
    sites: Optional[np.ndarray] = None
    # schedule 0: K-trial sweeps of mixed moves (the unit of a run is the sweep);
    # schedule 1: the paper's REGC step (unit: the step): with probability x0 one
    # particle-exchange attempt per walker, else a replica-exchange step, then
    # mc_cycles cycles of N displacement attempts
    schedule: int = 0
    x0: float = 0.99
    mc_cycles: int = 10
    # schedule 1 with md_steps > 0: the canonical part is md_steps velocity-Verlet steps
    # of md_dt (unit mass) under the stochastic velocity-rescaling thermostat (time md_tau;
    # 0: none) instead of the MC cycles
    md_steps: int = 0
    md_dt: float = 0.005
    md_tau: float = 0.1

    @property
    def n_states(self) -> int:
        return len(self.t) * len(self.mu)

    @property
    def volume(self) -> float:
        return self.lx * self.ly * (self.zhi - self.zlo)

    @property
    def trials(self) -> int:
        """Trials per sweep (schedule 0), at most per REGC step (schedule 1)."""
        if self.schedule == 1:
            return 1 + self.mc_cycles * self.n_max
        return self.trials_per_sweep if self.trials_per_sweep > 0 else self.n_max + 1

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def config1(n_sweeps: int = 10_000) -> Workload:
    """Plain REGC in FP64: 4x4x2 = 32-atom slab, gas box 6x6x8, N <= 40,
    8 T in [0.5, 2] x 8 mu in [-8, -2] = 64 replicas, swaps every 10 sweeps, seed 1."""
    box = 6.0
    return Workload(name="c1-plain-fp64-64rep", slab=fcc100_slab(4, 2, box, rc=2.5),
                    lx=box, ly=box, zlo=0.0, zhi=8.0,
                    t=linear_grid(0.5, 2.0, 8), mu=linear_grid(-8.0, -2.0, 8),
                    n_max=40, n_sweeps=n_sweeps)


def config2(n_sweeps: int = 100_000) -> Workload:
    """FP32 pair terms, FP64 totals: 8x8x3 = 192-atom slab, box 12^3, N <= 200,
    32 x 32 = 1024 replicas, samples every 100 sweeps."""
    box = 12.0
    return Workload(name="c2-fp32-1024rep-192slab", slab=fcc100_slab(8, 3, box, rc=2.5),
                    lx=box, ly=box, zlo=0.0, zhi=12.0,
                    t=linear_grid(0.5, 2.0, 32), mu=linear_grid(-8.0, -2.0, 32),
                    n_max=200, sample_every=100, n_sweeps=n_sweeps)


def config3_classes(n_sweeps: int = 10_000) -> List[Workload]:
    """Uneven batch: four slab classes {6,8,10,12}^2 x 3 layers (L = 1.5 n, H = 12),
    N <= 500, each class a 32 x 32 (T, mu) grid: 4096 replicas in all."""
    out = []
    for n in (6, 8, 10, 12):
        box = 1.5 * n
        out.append(Workload(name=f"c3-class{n}x{n}", slab=fcc100_slab(n, 3, box, rc=2.5),
                            lx=box, ly=box, zlo=0.0, zhi=12.0,
                            t=linear_grid(0.5, 2.0, 32), mu=linear_grid(-8.0, -2.0, 32),
                            n_max=500, sample_every=100, n_sweeps=n_sweeps))
    return out


def ideal_gas(n_t: int = 2, n_mu: int = 2, n_max: int = 40, n_sweeps: int = 4000) -> Workload:
    """epsilon = 0: the chain must give a Poisson N of mean z V truncated at n_max."""
    box = 6.0
    return Workload(name="ideal", slab=np.zeros((0, 3)), lx=box, ly=box, zlo=0.0, zhi=8.0,
                    t=linear_grid(0.8, 1.6, n_t), mu=linear_grid(-7.0, -5.5, n_mu),
                    n_max=n_max, mode=1, eps_gg=0.0, eps_gs=0.0, n_sweeps=n_sweeps)


def small_lj(n_t: int = 2, n_mu: int = 2, n_max: int = 12, box: float = 6.0, height: float = 4.0,
             n_sweeps: int = 200, t=(0.9, 1.5), mu=(-6.0, -3.0), seed: int = 1) -> Workload:
    """A small LJ slab system for quick parity and statistics tests."""
    return Workload(name="small-lj", slab=fcc100_slab(4, 2, box, rc=2.5), lx=box, ly=box,
                    zlo=0.0, zhi=height, t=linear_grid(t[0], t[1], n_t),
                    mu=linear_grid(mu[0], mu[1], n_mu), n_max=n_max, n_sweeps=n_sweeps, seed=seed)


def paper_schedule(w: Workload, x0: float = 0.99, mc_cycles: int = 10, sample_every: int = 100) -> Workload:
    """The workload run with the paper's REGC step (Sec. II.A): sample_every counts
    REGC steps (the paper records after every 100 steps, Sec. III.A)."""
    return w.replace(schedule=1, x0=x0, mc_cycles=mc_cycles, sample_every=sample_every)


def paper_schedule_md(w: Workload, x0: float = 0.99, md_steps: int = 10, md_dt: float = 0.005,
                      md_tau: float = 0.1, sample_every: int = 100) -> Workload:
    """The paper's REGC step with molecular dynamics as the canonical part (REGCMD)."""
    return w.replace(schedule=1, x0=x0, md_steps=md_steps, md_dt=md_dt, md_tau=md_tau, sample_every=sample_every)


def random_configuration(rng: np.random.Generator, w: Workload, n: int, min_dist: float = 0.85,
                         max_tries: int = 20000) -> np.ndarray:
    """n gas positions in the gas region, no two gas atoms closer than min_dist and
    none closer than min_dist to a slab atom (minimum image in x, y)."""
    pts: list = []
    tries = 0
    while len(pts) < n and tries < max_tries:
        tries += 1
        p = np.array([rng.uniform(0, w.lx), rng.uniform(0, w.ly), rng.uniform(w.zlo, w.zhi)])
        ok = True
        for q in list(pts) + [a for a in w.slab]:
            d = p - q
            d[0] -= w.lx * round(d[0] / w.lx)
            d[1] -= w.ly * round(d[1] / w.ly)
            if d @ d < min_dist * min_dist:
                ok = False
                break
        if ok:
            pts.append(p)
    if len(pts) < n:
        raise RuntimeError("could not place the requested number of particles")
    return np.array(pts, dtype=np.float64).reshape(-1, 3)


# ---------------------------------------------------------------------------
# learned insertion proposal: network shape and seeded initial weights
MLP_GRID = 16
MLP_NV = MLP_GRID ** 3
MLP_HIDDEN = 128
MLP_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")
MLP_SHAPES = {"W1": (MLP_NV, MLP_HIDDEN), "b1": (MLP_HIDDEN,), "W2": (MLP_HIDDEN, MLP_HIDDEN),
              "b2": (MLP_HIDDEN,), "W3": (MLP_HIDDEN, MLP_HIDDEN), "b3": (MLP_HIDDEN,),
              "W4": (MLP_NV, MLP_HIDDEN), "b4": (MLP_NV,)}


def mlp_init(seed: int = 0, occupancy_scale: float = 20.0, out_scale: float = 0.1) -> dict:
    """Seeded float32 initial weights.  W1 is stored voxel-major ([4096][128]: the
    column of each input voxel is contiguous), W2/W3 as [out][in], W4 as [4096][128]
    (one row per output voxel).  Normal entries with std 1/sqrt(occupancy_scale)
    (W1), sqrt(2/128) (W2, W3) and out_scale/sqrt(128) (W4); zero biases."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.normal(0.0, 1.0 / math.sqrt(occupancy_scale), MLP_SHAPES["W1"]),
         "W2": rng.normal(0.0, math.sqrt(2.0 / MLP_HIDDEN), MLP_SHAPES["W2"]),
         "W3": rng.normal(0.0, math.sqrt(2.0 / MLP_HIDDEN), MLP_SHAPES["W3"]),
         "W4": rng.normal(0.0, out_scale / math.sqrt(MLP_HIDDEN), MLP_SHAPES["W4"])}
    for b in ("b1", "b2", "b3", "b4"):
        p[b] = np.zeros(MLP_SHAPES[b])
    return {k: np.asarray(v, dtype=np.float32) for k, v in p.items()}


def mlp_pack(p: dict) -> np.ndarray:
    """Parameters concatenated in MLP_ORDER as one float32 vector."""
    return np.concatenate([np.asarray(p[k], np.float32).ravel() for k in MLP_ORDER])


def mlp_unpack(flat) -> dict:
    out, o = {}, 0
    for k in MLP_ORDER:
        size = int(np.prod(MLP_SHAPES[k]))
        out[k] = np.asarray(flat[o:o + size], np.float32).reshape(MLP_SHAPES[k])
        o += size
    return out
