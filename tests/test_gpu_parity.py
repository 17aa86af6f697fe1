"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

FP64 mode: identical accept/reject sequences and integer N trajectories, running
energies within 1e-10 relative (different summation order only).  FP32 pair mode:
per-configuration energies within 1e-5 relative of the FP64 oracle, long-run <N>
within 3 standard errors.  Reweighting: free energies and reweighted averages
against the naive FP64 oracle."""
import math
import struct
import sys

import numpy as np
import pytest

import oracle
from paper_1908_11118_amd import regc
from paper_1908_11118_amd import workloads as W
from tests.stats_util import assert_within_3se, batch_means, per_state_series

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    torch.cuda.set_device(0)


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _first_divergence(bits_a, bits_b, n_a, n_b):
    d = np.argwhere(bits_a != bits_b)
    if len(d):
        s, w, word = d[0]
        x = int(bits_a[s, w, word] ^ bits_b[s, w, word])
        return f"sweep {s} walker {w} trial {32 * word + (x & -x).bit_length() - 1}"
    d = np.argwhere(n_a != n_b)
    if len(d):
        return f"N differs at sweep {d[0][0]} walker {d[0][1]}"
    return None


def _fp64_trajectory(w, sweeps, **kw):
    _say(f"[fp64 trajectory] {w.name} S={w.n_states} sweeps={sweeps} {kw}")
    ref = oracle.Chain(w)
    r = ref.run(sweeps, trace=True)
    with regc.Regc(w, precision=regc.FP64, trace_capacity=sweeps, sample_capacity=0, **kw) as g:
        g.run(sweeps)
        bits, nps = g.trace(sweeps)
        wk = g.walkers()
        smp = g.samples()
        st = g.stats()
        hist = g.histograms()
    where = _first_divergence(bits, r["bits"], nps, r["trace_n"])
    assert where is None, f"trajectory diverges: {where}"
    assert np.array_equal(wk["n"], ref.n)
    assert np.array_equal(wk["label"], ref.label)
    assert np.allclose(wk["e"], ref.e, rtol=1e-10, atol=1e-9)
    for k in range(ref.S):
        assert np.allclose(wk["xyz"][k, : ref.n[k]], ref.xyz[k, : ref.n[k]], rtol=0, atol=0)
    assert np.array_equal(st["stats"], ref.stats)
    assert np.array_equal(st["swap_att"], ref.swap_att)
    assert np.array_equal(st["swap_acc"], ref.swap_acc)
    assert np.array_equal(smp["n"], r["n"]) and np.array_equal(smp["state"], r["state"])
    assert np.allclose(smp["e"], r["e"], rtol=1e-10, atol=1e-9)
    if w.sample_every > 0:
        ref_hist = np.zeros_like(hist)
        np.add.at(ref_hist, (r["state"], r["n"]), 1)
        assert np.array_equal(hist, ref_hist)
    return ref, wk


def test_fp64_trajectories_config1():
    """64 replicas, 32-atom slab, N <= 40, 10^3 sweeps: bit-identical decisions."""
    _fp64_trajectory(W.config1(), 1000)


def test_fp64_trajectories_binned_slab_and_scheme1():
    """6x6x3 slab (binned columns), odd grid sizes, diagonal swap scheme."""
    w = W.config3_classes()[0].replace(t=W.linear_grid(0.6, 1.8, 4), mu=W.linear_grid(-6.0, -2.5, 4),
                                       n_max=60, swap_scheme=1, sample_every=3)
    _fp64_trajectory(w, 300)
    w2 = w.replace(t=W.linear_grid(0.6, 1.8, 3), mu=W.linear_grid(-6.0, -2.5, 5), swap_scheme=0, seed=7)
    _fp64_trajectory(w2, 200, slab_bins=-1)


def test_fp64_trajectories_irregular_slab_rectangular_box():
    """Binned slab columns on a rectangular box (14 x 8.5: 5 x 3 columns) with an
    irregular slab: random atoms, a dense cluster in one corner column (the other
    columns padded) and atoms within 0.05 of both periodic edges, so the column
    block's wrap in x and in y and the padding are all exercised."""
    rng = np.random.default_rng(11)
    lx, ly = 14.0, 8.5
    spread = np.column_stack([rng.uniform(0, lx, 40), rng.uniform(0, ly, 40), rng.uniform(-2.0, 0.0, 40)])
    corner = np.column_stack([rng.uniform(0, 2.0, 20), rng.uniform(0, 2.0, 20), rng.uniform(-2.0, 0.0, 20)])
    edges = np.array([[lx - 0.02, 0.3, -0.2], [0.01, ly - 0.05, -0.4], [lx - 0.01, ly - 0.01, -0.1],
                      [7.0, 0.0, -0.3], [0.0, 4.0, -0.6]])
    w = W.small_lj(n_t=3, n_mu=3, n_max=40).replace(
        name="irregular-slab", slab=np.vstack([spread, corner, edges]), lx=lx, ly=ly, zlo=0.9, zhi=6.0,
        t=W.linear_grid(0.8, 1.6, 3), mu=W.linear_grid(-4.0, -2.0, 3), sample_every=2)
    assert math.floor(lx / (w.rc + w.max_disp)) == 5 and math.floor(ly / (w.rc + w.max_disp)) == 3
    _, wk = _fp64_trajectory(w, 200)
    assert wk["n"].max() > 10


@pytest.mark.parametrize("wpb,spl,split,cull", [(1, 1, 1, 0), (4, 3, 1, 1), (8, 0, 1, 0), (1, 0, 2, 0), (1, 7, 2, 1),
                                             (1, 0, 4, 0), (1, 3, 4, 1)])
def test_fp64_invariant_to_launch_shape(wpb, spl, split, cull):
    """Walkers per block, sweeps per launch, waves per walker and the cull pass
    change nothing but summation order: trajectories stay identical."""
    w = W.small_lj(n_t=4, n_mu=4, n_max=20, n_sweeps=60)
    _fp64_trajectory(w, 60, walkers_per_block=wpb, sweeps_per_launch=spl, split=split, cull=cull)
    w2 = W.config3_classes()[0].replace(t=W.linear_grid(0.6, 1.8, 3), mu=W.linear_grid(-6.0, -2.5, 3), n_max=40)
    _fp64_trajectory(w2, 40, walkers_per_block=wpb, sweeps_per_launch=spl, split=split, cull=cull)


@pytest.mark.parametrize("batch,wpb,spl,split", [(1, 0, 0, 0), (2, 1, 3, 0), (2, 4, 0, 0), (4, 1, 7, 0),
                                                (4, 8, 0, 0), (4, 0, 0, 4), (4, 0, 3, 4), (2, 0, 0, 2)])
def test_fp64_batched_trials_keep_the_trajectories(batch, wpb, spl, split):
    """Trials decided in batches of 2 or 4 (corrected by the pair terms of the moves
    accepted earlier in the batch, a trial whose particle index or particle changed
    left to the next batch) give the sequential chain's accept bits, N, labels and
    counters: small N, N above a group's lanes, a binned slab, walkers per block; in
    one wave per walker, or (split equal to the batch) one wave per trial."""
    kw = dict(batch_trials=batch, walkers_per_block=wpb, sweeps_per_launch=spl, split=split)
    w = W.small_lj(n_t=4, n_mu=4, n_max=20, n_sweeps=60)
    _fp64_trajectory(w, 60, **kw)
    w2 = W.config2(60).replace(t=np.array([0.9, 1.6]), mu=np.array([-3.0, -2.0]), n_max=160, sample_every=5)
    _, wk = _fp64_trajectory(w2, 60, **kw)
    assert wk["n"].max() > 100
    # a dense, strongly interacting system: many accepted moves inside each batch
    w3 = W.small_lj(n_t=2, n_mu=2, n_max=40, t=(0.7, 1.2), mu=(-3.0, -1.5), height=5.0)
    _, wk3 = _fp64_trajectory(w3, 150, **kw)
    assert wk3["n"].max() > 25


def test_fp64_batched_trials_ideal_gas_and_caps():
    """The batched kernel where only prefactors decide (ideal gas: every index
    change after an accepted insertion or removal), at the cap N = n_max and with one
    trial per sweep."""
    _fp64_trajectory(W.ideal_gas(n_t=2, n_mu=3, n_max=30), 300, batch_trials=4)
    _fp64_trajectory(W.ideal_gas(n_t=2, n_mu=2, n_max=6).replace(mu=W.linear_grid(-3.0, -2.0, 2)), 200,
                     batch_trials=4)
    _fp64_trajectory(W.small_lj(n_t=2, n_mu=3, n_max=8).replace(trials_per_sweep=1), 200, batch_trials=4)
    _fp64_trajectory(W.small_lj(n_t=1, n_mu=1, n_max=1, n_sweeps=300).replace(swap_every=0), 300, batch_trials=2)
    # one wave per trial
    _fp64_trajectory(W.ideal_gas(n_t=2, n_mu=3, n_max=30), 300, batch_trials=4, split=4)
    _fp64_trajectory(W.ideal_gas(n_t=2, n_mu=2, n_max=6).replace(mu=W.linear_grid(-3.0, -2.0, 2)), 200,
                     batch_trials=4, split=4)
    _fp64_trajectory(W.small_lj(n_t=2, n_mu=3, n_max=8).replace(trials_per_sweep=1), 200, batch_trials=4, split=4)
    _fp64_trajectory(W.small_lj(n_t=1, n_mu=1, n_max=1, n_sweeps=300).replace(swap_every=0), 300, batch_trials=2,
                     split=2)


@pytest.mark.parametrize("split,cull,cell", [(1, 0, 0.0), (2, 0, 0.0), (1, 1, 0.0), (2, 1, 0.0), (4, 0, 0.0),
                                             (4, 1, 0.0), (1, 0, 1.25), (2, 0, 1.25)])
def test_fp64_dense_walkers(split, cull, cell):
    """N well above 64 (a wave's width), binned 8x8x3 slab (columns of the smallest
    width, or 1.25 times it: 3 x 3 columns): every wave of a split walker owns gas
    candidates."""
    w = W.config2(60).replace(t=np.array([0.9, 1.6]), mu=np.array([-3.0, -2.0]), n_max=160, sample_every=5)
    _, wk = _fp64_trajectory(w, 60, split=split, cull=cull, slab_cell=cell)
    assert wk["n"].max() > 100


@pytest.mark.parametrize("split", [1, 2, 4])
def test_fp64_walkers_above_two_wave_widths(split):
    """N above 128 up to the cap: with one wave per walker the gas loop runs more than
    one step of two candidates per lane; with two waves each wave takes its two blocks
    in one pass; with four, one block each."""
    w = W.config2(40).replace(t=np.array([0.8, 1.2]), mu=np.array([-2.0, -1.0]), n_max=210, sample_every=4)
    _, wk = _fp64_trajectory(w, 40, split=split)
    assert wk["n"].max() > 150


def test_fp64_pair_counters_agree_across_launch_shapes():
    """The candidate and in-cutoff pair counts behind the roofline figures are properties
    of the trajectory: with FP64 trajectories identical for every one-trial launch shape
    (one, two or four waves per walker, the cull pass), both counts must be too, and the
    ideal gas evaluates no pairs at all."""
    w = W.config2(40).replace(t=np.array([0.8, 1.2]), mu=np.array([-2.0, -1.0]), n_max=210, sample_every=4)
    counts = {}
    for kw in (dict(split=1), dict(split=2), dict(split=4), dict(split=1, cull=1), dict(split=2, cull=1)):
        _say(f"[pair counts] {kw}")
        with regc.Regc(w, precision=regc.FP64, sample_capacity=0, **kw) as g:
            g.run(30)
            counts[tuple(sorted(kw.items()))] = g.pair_counts()
            n_max_seen = int(g.walkers()["n"].max())
    assert n_max_seen > 130   # some walkers beyond two wave widths, some steps ragged
    vals = set(counts.values())
    assert len(vals) == 1, counts
    cand, useful = vals.pop()
    assert 0 < useful < cand
    with regc.Regc(W.ideal_gas(n_t=2, n_mu=3, n_max=30), precision=regc.FP64, sample_capacity=0) as g:
        g.run(50)
        assert g.pair_counts() == (0, 0)


def test_fp64_edge_cases():
    # N capped at 1, one state, no exchange, K = 1 trial per sweep
    _fp64_trajectory(W.small_lj(n_t=1, n_mu=1, n_max=1, n_sweeps=500).replace(swap_every=0), 500)
    _fp64_trajectory(W.small_lj(n_t=2, n_mu=3, n_max=8).replace(trials_per_sweep=1), 300)
    # no slab at all
    _fp64_trajectory(W.small_lj(n_t=2, n_mu=2, n_max=15).replace(slab=np.zeros((0, 3))), 150)
    # ideal gas mode, also with two waves per walker in the one-trial kernel
    _fp64_trajectory(W.ideal_gas(n_t=2, n_mu=3, n_max=30), 300)
    _fp64_trajectory(W.ideal_gas(n_t=2, n_mu=3, n_max=30), 300, split=2)
    _fp64_trajectory(W.ideal_gas(n_t=2, n_mu=3, n_max=30), 300, split=4)


def _batch_classes():
    """Three classes; a batch shares one schedule (that of its first class)."""
    c3 = W.config3_classes()
    out = [c3[1].replace(t=W.linear_grid(0.6, 1.8, 3), mu=W.linear_grid(-5.0, -2.5, 4), n_max=70),
           W.small_lj(n_t=2, n_mu=3, n_max=30),
           c3[0].replace(t=W.linear_grid(0.7, 1.5, 4), mu=W.linear_grid(-6.0, -3.0, 2), n_max=50)]
    return [w.replace(sample_every=3, swap_every=10) for w in out]


@pytest.mark.parametrize("graph", [0, 2])
def test_fp64_uneven_batch(graph, persistent=0, **kw):
    """Three classes of different slab, box, n_max and grid in the same launches:
    each class's trajectories equal a lone oracle simulation with the batch's
    Philox stream offsets; with graph replay of whole exchange intervals too."""
    classes = _batch_classes()
    sweeps = 63
    _say(f"[batch] {len(classes)} classes, graph={graph} persistent={persistent} {kw}")
    with regc.Regc(classes, precision=regc.FP64, trace_capacity=sweeps, graph_intervals=graph,
                   sample_capacity=0, persistent=persistent, **kw) as g:
        g.run(25)
        g.run(sweeps - 25)
        bits, nps = g.trace(sweeps)
        wk = g.walkers()
        st = g.stats()
        smp = g.samples()
        offs, cnts = g.offsets, g.counts
    W_all = sum(cnts)
    for c, w in enumerate(classes):
        ref = oracle.Chain(w, walker_offset=offs[c], class_id=c)
        r = ref.run(sweeps, trace=True)
        sl = slice(offs[c], offs[c] + cnts[c])
        words = r["bits"].shape[2]
        where = _first_divergence(bits[:, sl, :words], r["bits"], nps[:, sl], r["trace_n"])
        assert where is None, f"class {c}: {where}"
        assert np.array_equal(wk["n"][sl], ref.n) and np.array_equal(wk["label"][sl], ref.label)
        assert np.allclose(wk["e"][sl], ref.e, rtol=1e-10, atol=1e-9)
        assert np.array_equal(st["stats"][sl], ref.stats)
        assert np.array_equal(st["swap_acc"][:, sl], ref.swap_acc)
        rec_n = smp["n"].reshape(-1, W_all)[:, sl].ravel()
        assert np.array_equal(rec_n, r["n"])


@pytest.mark.parametrize("wpb,graph,persistent", [(2, 0, 0), (4, 2, 0), (2, 0, 1)])
def test_fp64_balanced_walker_order_keeps_the_trajectories(wpb, graph, persistent):
    """The walker order dealt by particle count before every launch (forced on; with
    four walkers per workgroup the 6-walker class keeps its order) changes only which
    wave runs which walker: every class still follows the oracle trial by trial, also
    under graph replay and inside persistent launches.  A walker left out or run twice
    in a launch would break its trajectory."""
    test_fp64_uneven_batch(graph, persistent=persistent, balance=1, walkers_per_block=wpb)


def test_fp64_balanced_walker_order_many_workgroups():
    """The walker order dealt over several workgroups per class: two classes of 64
    walkers (8 x 8 states) in workgroups of 8, walkers spread from empty to dense, so
    that the counting sort sees many particle counts and every workgroup receives one
    walker of each eighth of the ranks; each class still follows the oracle trial by
    trial."""
    c3 = W.config3_classes()
    classes = [c3[0].replace(t=W.linear_grid(0.6, 1.8, 8), mu=W.linear_grid(-6.0, -2.0, 8), n_max=60),
               W.small_lj(n_t=8, n_mu=8, n_max=30, mu=(-5.0, -2.0))]
    classes = [w.replace(sample_every=5, swap_every=10) for w in classes]
    sweeps = 40
    _say("[batch] 2 classes x 64 walkers, walker order forced on, 8 walkers per workgroup")
    with regc.Regc(classes, precision=regc.FP64, trace_capacity=sweeps, sample_capacity=0, balance=1,
                   walkers_per_block=8) as g:
        g.run(sweeps)
        bits, nps = g.trace(sweeps)
        wk = g.walkers()
        st = g.stats()
        offs, cnts = g.offsets, g.counts
    assert len(set(wk["n"].tolist())) > 10
    for c, w in enumerate(classes):
        ref = oracle.Chain(w, walker_offset=offs[c], class_id=c)
        r = ref.run(sweeps, trace=True)
        sl = slice(offs[c], offs[c] + cnts[c])
        words = r["bits"].shape[2]
        where = _first_divergence(bits[:, sl, :words], r["bits"], nps[:, sl], r["trace_n"])
        assert where is None, f"class {c}: {where}"
        assert np.array_equal(wk["n"][sl], ref.n) and np.array_equal(wk["label"][sl], ref.label)
        assert np.allclose(wk["e"][sl], ref.e, rtol=1e-10, atol=1e-9)
        assert np.array_equal(st["stats"][sl], ref.stats)


def test_checkpoint_restore_continues_identically():
    w = W.small_lj(n_t=2, n_mu=4, n_max=20)
    _say("[checkpoint] small_lj 2x4")
    with regc.Regc(w, sample_capacity=0) as a:
        a.run(50)
        blob = a.checkpoint()
        a.run(70)
        ref = a.walkers()
        ref_st = a.stats()
    with regc.Regc(w) as b:
        # corrupted buffers are rejected before anything changes: header of 40 bytes,
        # then N (int32 per walker), E (float64), labels (int32), walker of state (int32)
        nw = len(w.t) * len(w.mu)
        for off, value in ((40, w.n_max + 1), (40 + 12 * nw, struct.unpack_from("<i", blob, 40 + 12 * nw + 4)[0])):
            bad = bytearray(blob)
            struct.pack_into("<i", bad, off, value)
            with pytest.raises(regc.RegcError) as ei:
                b.restore(bytes(bad))
            assert ei.value.code == regc.EINVAL
            assert b.sweep == 0
        b.restore(blob)
        assert b.sweep == 50
        b.run(70)
        got = b.walkers()
        st = b.stats()
    for k in ("n", "label"):
        assert np.array_equal(got[k], ref[k])
    assert np.array_equal(got["e"], ref["e"])
    assert np.array_equal(got["xyz"], ref["xyz"])
    assert np.array_equal(st["stats"], ref_st["stats"])
    # the oracle restored from the GPU's blob continues along the same trajectory, and
    # the GPU restored from an oracle checkpoint along the oracle's
    orc = oracle.Chain(w)
    orc.restore(blob)
    assert int(orc.sweep[0]) == 50
    orc.run(70)
    assert np.array_equal(orc.n, got["n"]) and np.array_equal(orc.label, got["label"])
    assert np.allclose(orc.e, got["e"], rtol=1e-10, atol=1e-10)
    for wk in range(nw):
        assert np.allclose(orc.xyz[wk, : orc.n[wk]], got["xyz"][wk, : got["n"][wk]], rtol=0, atol=1e-12)
    assert np.array_equal(orc.stats, st["stats"])
    o2 = oracle.Chain(w)
    o2.run(30)
    oblob = o2.checkpoint()
    o2.run(40)
    with regc.Regc(w) as c:
        c.restore(oblob)
        assert c.sweep == 30
        c.run(40)
        g2 = c.walkers()
        st2 = c.stats()
    assert np.array_equal(g2["n"], o2.n) and np.array_equal(g2["label"], o2.label)
    assert np.allclose(g2["e"], o2.e, rtol=1e-10, atol=1e-10)
    assert np.array_equal(st2["stats"], o2.stats)


def test_autotune_picks_the_fastest_measured_shape():
    """The launch-shape autotuner measures every candidate (graph replay included)
    and returns the best of its own table; the shape it picks leaves FP64
    trajectories unchanged."""
    from paper_1908_11118_amd import autotune
    w = W.small_lj(n_t=4, n_mu=4, n_max=20)
    _say("[autotune] small_lj 4x4")
    res = autotune.autotune(w, precision=regc.FP64, warm_sweeps=50, measure_sweeps=20, cache_path=None)
    rates = [row["trials_per_s"] for row in res["table"]]
    assert len(rates) >= 8 and all(np.isfinite(r) and r > 0 for r in rates)
    assert res["trials_per_s"] == max(rates)
    assert res["options"] in [row["options"] for row in res["table"]]
    assert any(row["options"].get("graph_intervals", 0) > 0 for row in res["table"])
    _fp64_trajectory(w, 40, **res["options"])


def test_capacity_and_state_errors():
    w = W.small_lj(n_t=2, n_mu=2, n_max=10)
    with regc.Regc(w, sample_capacity=4 * 5) as g:
        g.run(5)
        with pytest.raises(regc.RegcError) as ei:
            g.run(1)
        assert ei.value.code == regc.ECAPACITY
        assert g.sweep == 5
        g.clear_samples()
        g.run(5)
        assert g.sample_count() == 20


# ---------------------------------------------------------------------------
# FP32 pair mode
# ---------------------------------------------------------------------------
def test_fp32_configuration_energies_config2_scale():
    """1024 replicas, 192-atom slab, N <= 200, the benchmark's launch shape: the
    oracle re-evaluates sampled walkers' configurations in FP64."""
    w = W.config2()
    _say("[fp32 energies] config2 1024 walkers, 1000 sweeps")
    with regc.Regc(w, precision=regc.FP32PAIR, sample_capacity=0) as g:
        g.run(1000)
        wk = g.walkers()
        e_re = g.energies()
    ch = oracle.Chain(w.replace(t=w.t[:1], mu=w.mu[:1]))
    rng = np.random.default_rng(0)
    idx = np.concatenate([np.argsort(wk["n"])[-16:], rng.choice(len(wk["n"]), 24, replace=False)])
    assert wk["n"].max() > 100
    for k in idx:
        ref = ch.energy(wk["xyz"][k, : wk["n"][k]])
        tol = 1e-5 * max(1.0, abs(ref))
        assert abs(e_re[k] - ref) <= tol, (k, e_re[k], ref)
        assert abs(wk["e"][k] - ref) <= tol, (k, wk["e"][k], ref)


def test_fp32_configuration_energies_config3_batch():
    """4096 replicas in four slab classes (N <= 500) in the benchmark's launch shape
    (graph-replayed exchange intervals): after 600 sweeps the running and recomputed
    energies of sampled walkers of every class agree with the oracle's FP64 energy of
    the same configuration to 1e-5 relative."""
    classes = W.config3_classes()
    _say("[fp32 energies] config3 4096 walkers, 600 sweeps")
    with regc.Regc(classes, precision=regc.FP32PAIR, sample_capacity=0, graph_intervals=10) as g:
        g.run(600)
        wk = g.walkers()
        e_re = g.energies()
        offs, cnts = g.offsets, g.counts
    rng = np.random.default_rng(1)
    assert wk["n"].max() > 400
    for c, w in enumerate(classes):
        ch = oracle.Chain(w.replace(t=w.t[:1], mu=w.mu[:1]))
        n_c = wk["n"][offs[c]:offs[c] + cnts[c]]
        idx = offs[c] + np.concatenate([np.argsort(n_c)[-4:], rng.choice(cnts[c], 6, replace=False)])
        for k in idx:
            ref = ch.energy(wk["xyz"][k, : wk["n"][k]])
            tol = 1e-5 * max(1.0, abs(ref))
            assert abs(e_re[k] - ref) <= tol, (c, k, e_re[k], ref)
            assert abs(wk["e"][k] - ref) <= tol, (c, k, wk["e"][k], ref)


def test_fp32_long_run_mean_n_within_3se():
    w = W.small_lj(n_t=2, n_mu=3, n_max=24, t=(0.9, 1.4), mu=(-5.0, -3.0)).replace(sample_every=2)
    sweeps, burn = 16000, 1000
    _say(f"[fp32 statistics] small_lj 2x3, {sweeps} sweeps")
    ref = oracle.Chain(w)
    ref.run(burn)
    r = ref.run(sweeps)
    with regc.Regc(w, precision=regc.FP32PAIR, sample_capacity=(burn + sweeps) * 6) as g:
        g.run(burn)
        g.clear_samples()
        g.run(sweeps)
        s = g.samples()
    n_ref, _ = per_state_series(r, ref.S)
    n_gpu, _ = per_state_series(s, ref.S)
    z = []
    for k in range(ref.S):
        m1, se1 = batch_means(n_ref[:, k])
        m2, se2 = batch_means(n_gpu[:, k])
        z.append((m2 - m1) / math.sqrt(se1 ** 2 + se2 ** 2 + 1e-12))
    z = np.array(z)
    assert np.all(np.abs(z) < 3.0), z


# ---------------------------------------------------------------------------
# Reweighting
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("t_mu,sweeps", [((2, 2), 40), ((1, 3), 60), ((2, 1), 30)])
def test_mbar_few_states_short_runs(t_mu, sweeps):
    """Anderson-accelerated solve on grids of 2-4 states and a few hundred correlated
    samples (where more history than free components would make the least squares
    ill-posed): converges to the naive oracle's free energies."""
    w = W.small_lj(n_t=t_mu[0], n_mu=t_mu[1], n_max=12, n_sweeps=sweeps)
    _say(f"[mbar small] {t_mu} {sweeps} sweeps")
    ref = oracle.Chain(w)
    r = ref.run(sweeps)
    beta, lnz = oracle.state_arrays(w)
    omega = np.bincount(r["state"], minlength=len(beta))
    f_ref, _, ok, _, _ = oracle.mbar_solve(beta, lnz, omega, r["e"], r["n"], tol=1e-11, max_iter=20000)
    mb = regc.Mbar(w.t, w.mu, w.n_max)
    mb.set_samples(r["e"], r["n"], r["state"])
    f_gpu, conv, _, _ = mb.solve(tol=1e-10, max_iter=5000)
    mb.close()
    assert ok and conv and np.all(np.isfinite(f_gpu))
    assert np.max(np.abs(f_gpu - f_ref)) < 1e-7, (f_gpu, f_ref)


@pytest.mark.parametrize("method", [1, 0])
def test_mbar_matches_oracle(method):
    """GPU reweighting (factorised over temperatures, plain or Anderson-accelerated
    fixed point) against the naive FP64 oracle on the same config-1 samples."""
    w = W.config1(400)
    _say(f"[mbar] config1 400 sweeps, solver {method}")
    with regc.Regc(w, precision=regc.FP64, sample_capacity=400 * 64) as g:
        g.run(400)
        s = g.samples()
        mb = regc.Mbar(w.t, w.mu, w.n_max)
        mb.set_solver(method, 8)
        mb.load_run(g, 0, skip_records=40)
    keep = slice(40 * 64, None)
    e, n, st = s["e"][keep], s["n"][keep], s["state"][keep]
    beta, lnz = oracle.state_arrays(w)
    omega = np.bincount(st, minlength=len(beta))
    f_ref, logd, ok, it, _ = oracle.mbar_solve(beta, lnz, omega, e, n, tol=1e-11, max_iter=20000)
    f_gpu, conv, it_gpu, d = mb.solve(tol=1e-11, max_iter=20000)
    assert ok and conv
    assert np.max(np.abs(f_gpu - f_ref)) < 1e-7, np.max(np.abs(f_gpu - f_ref))
    tt, tm = W.linear_grid(0.5, 2.0, 11), W.linear_grid(-8.0, -2.0, 13)
    got = mb.targets(tt, tm)
    TB = np.repeat(1.0 / tt, len(tm))
    TZ = np.array([oracle.state_lnz(a, b) for a in tt for b in tm])
    ref = oracle.mbar_targets(TB, TZ, e, n, logd, w.n_max)
    assert np.allclose(got["mean_n"], ref["mean_n"], rtol=1e-7, atol=1e-7)
    assert np.allclose(got["mean_e"], ref["mean_e"], rtol=1e-7, atol=1e-6)
    assert np.allclose(got["mean_e2"], ref["mean_e2"], rtol=1e-7, atol=1e-5)
    assert np.allclose(got["p_n"], ref["p_n"], atol=1e-8)
    assert np.allclose(got["f"] - got["f"][0], ref["f"] - ref["f"][0], atol=1e-7)
    # phase map: identical wherever the top two probabilities are distinguishable
    srt = np.sort(ref["p_n"], axis=1)
    clear = srt[:, -1] - srt[:, -2] > 1e-9
    assert np.array_equal(got["phase"][clear], ref["phase"][clear])
    mb.close()


def test_mbar_failed_reload_leaves_no_samples():
    """A rejected sample set replaces the handle's earlier samples by none: the
    solve then refuses (ESTATE) instead of running on half-replaced buffers, and a
    valid reload gives the earlier solution again."""
    w = W.small_lj(n_t=2, n_mu=2, n_max=10)
    rng = np.random.default_rng(3)
    ns = 400
    e = rng.normal(size=ns)
    n = rng.integers(0, w.n_max + 1, ns)
    st = rng.integers(0, 4, ns)
    _say("[mbar] failed reload")
    mb = regc.Mbar(w.t, w.mu, w.n_max)
    mb.set_samples(e, n, st)
    f1, conv, _, _ = mb.solve(tol=1e-10)
    assert conv
    bad = st[:100].copy()
    bad[-1] = 4                                   # outside the 2 x 2 grid
    with pytest.raises(regc.RegcError) as ei:
        mb.set_samples(e[:100], n[:100], bad)
    assert ei.value.code == regc.EINVAL
    with pytest.raises(regc.RegcError) as ei:
        mb.solve(tol=1e-10)
    assert ei.value.code == regc.ESTATE
    mb.set_samples(e, n, st)
    f2, conv, _, _ = mb.solve(tol=1e-10)
    assert conv and np.allclose(f1, f2, atol=1e-12)
    mb.close()


def test_mbar_ideal_gas_iid_samples():
    """GPU reweighting of i.i.d. truncated-Poisson samples against the oracle on the
    same samples, with an unsampled state and an empty N segment."""
    rng = np.random.default_rng(4)
    t, mu, V, n_max = np.array([1.0, 1.2, 1.5]), np.array([-4.6, -4.0, -3.4, -3.0]), 288.0, 45
    es, ns, ss = [], [], []
    for l, T in enumerate(t):
        for m, u in enumerate(mu):
            if (l, m) == (1, 2):
                continue           # an unsampled state
            zv = math.exp(u / T) * T ** 1.5 * V
            k = np.arange(n_max + 1)
            lp = k * math.log(zv) - np.array([math.lgamma(i + 1) for i in k])
            p = np.exp(lp - lp.max())
            p /= p.sum()
            x = rng.choice(n_max + 1, 3000, p=p)
            ns.append(x)
            es.append(rng.normal(-0.3, 0.1, len(x)) * x)
            ss.append(np.full(len(x), l * len(mu) + m))
    e, n, st = np.concatenate(es), np.concatenate(ns).astype(np.int32), np.concatenate(ss).astype(np.int32)
    beta = np.repeat(1 / t, len(mu))
    lnz = np.array([oracle.state_lnz(T, u) for T in t for u in mu])
    omega = np.bincount(st, minlength=len(beta))
    f_ref, logd, ok, _, _ = oracle.mbar_solve(beta, lnz, omega, e, n, tol=1e-11)
    mb = regc.Mbar(t, mu, n_max)
    mb.set_samples(e, n, st)
    f_gpu, conv, _, _ = mb.solve(tol=1e-11)
    assert ok and conv and np.max(np.abs(f_gpu - f_ref)) < 1e-8
    got = mb.targets(t, mu)
    ref = oracle.mbar_targets(beta, lnz, e, n, logd, n_max)
    assert np.allclose(got["mean_n"], ref["mean_n"], rtol=1e-9, atol=1e-9)
    assert np.allclose(got["f"], ref["f"] - ref["f"][0] + got["f"][0], atol=1e-8)
    mb.close()


# ---------------------------------------------------------------------------
# The paper's REGC step (x0 coin, one particle-exchange attempt, MC cycles)
# ---------------------------------------------------------------------------
def test_fp64_trajectories_paper_schedule_config1():
    """64 replicas, x0 = 0.99, 10 MC cycles of N displacements per step, samples every
    10 steps: identical decisions, exchanges, samples."""
    w = W.paper_schedule(W.config1(), x0=0.99, mc_cycles=10, sample_every=10)
    _fp64_trajectory(w, 300)


@pytest.mark.parametrize("wpb,spl", [(1, 0), (4, 7)])
def test_fp64_paper_schedule_variants(wpb, spl):
    """Frequent exchange steps, few cycles, a binned slab, launch shapes."""
    w = W.paper_schedule(W.config3_classes()[0].replace(t=W.linear_grid(0.6, 1.8, 4), mu=W.linear_grid(-6.0, -2.5, 4),
                                                       n_max=60), x0=0.7, mc_cycles=2, sample_every=3)
    _fp64_trajectory(w, 200, walkers_per_block=wpb, sweeps_per_launch=spl)
    _fp64_trajectory(W.paper_schedule(W.ideal_gas(n_t=2, n_mu=3, n_max=30), x0=0.8, mc_cycles=1, sample_every=1), 400,
                     walkers_per_block=wpb, sweeps_per_launch=spl)


def test_paper_schedule_rejects_unsupported():
    w = W.paper_schedule(W.small_lj())
    with pytest.raises(regc.RegcError):
        regc.Regc([w, w.replace(seed=2)], precision=regc.FP64)
    with pytest.raises(regc.RegcError):
        regc.Regc(w, precision=regc.FP64, graph_intervals=2)
    net = regc.Mlp(W.mlp_pack(W.mlp_init(0)))
    with regc.Regc(w, precision=regc.FP64) as g:
        with pytest.raises(regc.RegcError):
            g.set_proposal(net, 0.5)
    net.close()


# ---------------------------------------------------------------------------
# Structural observables with the samples, and their reweighting
# ---------------------------------------------------------------------------
OBS = dict(dz=0.12, layer=(0.6, 1.6), dr=0.1, nr=28)


def test_fp64_observables_match_the_oracle():
    """Per-sample axial counts and layer pair counts: bit-exact against the oracle
    along identical FP64 trajectories (samples every sweep and every 3 sweeps)."""
    for w, sweeps in ((W.config1(), 120), (W.small_lj(n_t=2, n_mu=3, n_max=16, mu=(-4.0, -2.0)).replace(
            sample_every=3), 150)):
        _say(f"[observables] {w.name} sweeps={sweeps}")
        ref = oracle.Chain(w, observables=OBS)
        r = ref.run(sweeps)
        with regc.Regc(w, precision=regc.FP64, sample_capacity=(sweeps // w.sample_every + 1) * w.n_states) as g:
            g.set_observables(OBS["dz"], OBS["layer"], OBS["dr"], OBS["nr"])
            g.run(sweeps)
            smp = g.samples()
            ob = g.observables()
        assert np.array_equal(smp["n"], r["n"])
        assert ob.shape == r["obs"].shape
        assert np.array_equal(ob.astype(np.float64), r["obs"])
        assert r["obs"][:, -1].max() > 0          # the layer is populated


def test_mbar_observables_match_the_oracle():
    w = W.small_lj(n_t=2, n_mu=3, n_max=16, mu=(-4.5, -2.5)).replace(sample_every=1)
    ref = oracle.Chain(w, observables=OBS)
    ref.run(300)
    out = ref.run(3000)
    beta, lnz = oracle.state_arrays(w)
    omega = np.bincount(out["state"], minlength=w.n_states)
    f, logd, ok, _, _ = oracle.mbar_solve(beta, lnz, omega, out["e"], out["n"], tol=1e-12)
    assert ok
    tt, tm = np.array([0.95, 1.2, 1.45]), np.array([-4.2, -3.1])
    tb = np.repeat(1.0 / tt, len(tm))
    tz = np.array([oracle.state_lnz(T, m) for T in tt for m in tm])
    mean_ref, cond_ref = oracle.mbar_observables(tb, tz, out["e"], out["n"], logd, w.n_max, out["obs"])
    mb = regc.Mbar(w.t, w.mu, w.n_max)
    mb.set_samples(out["e"], out["n"], out["state"])
    mb.solve(tol=1e-12, max_iter=20000)
    mb.set_observables(out["obs"].astype(np.uint32))
    mean, cond = mb.observables(tt, tm, out["obs"].shape[1])
    mb.close()
    scale = np.abs(mean_ref).max()
    assert np.abs(mean.reshape(-1, mean.shape[-1]) - mean_ref).max() <= 1e-8 * scale
    # the conditional average depends on T only; the oracle repeats it for every mu
    cref = cond_ref.reshape(len(tt), len(tm), w.n_max + 1, -1)[:, 0]
    assert np.abs(cond - cref).max() <= 1e-8 * max(1.0, np.abs(cref).max())


def test_mbar_load_run_carries_the_observables():
    w = W.small_lj(n_t=2, n_mu=2, n_max=12).replace(sample_every=2)
    with regc.Regc(w, precision=regc.FP64, sample_capacity=400 * w.n_states) as g:
        g.set_observables(OBS["dz"], OBS["layer"], OBS["dr"], OBS["nr"])
        g.run(600)
        smp = g.samples()
        ob = g.observables()
        a = regc.Mbar(w.t, w.mu, w.n_max)
        a.load_run(g, 0, 20)
        a.solve(tol=1e-11, max_iter=20000)
        m1, c1 = a.observables(w.t, w.mu, g.n_obs)
    b = regc.Mbar(w.t, w.mu, w.n_max)
    skip = 20 * w.n_states
    b.set_samples(smp["e"][skip:], smp["n"][skip:], smp["state"][skip:])
    b.solve(tol=1e-11, max_iter=20000)
    b.set_observables(ob[skip:])
    m2, c2 = b.observables(w.t, w.mu, ob.shape[1])
    a.close()
    b.close()
    assert np.allclose(m1, m2, rtol=1e-12, atol=1e-12) and np.allclose(c1, c2, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# aiAT@REGC: lowest recorded energy and configuration per N
# ---------------------------------------------------------------------------
def test_fp64_minima_and_aiat_map_match_the_oracle():
    w = W.config1()
    sweeps = 200
    _say("[minima] config1")
    ref = oracle.Chain(w)
    ref.run(sweeps)
    with regc.Regc(w, precision=regc.FP64, sample_capacity=(sweeps + 1) * w.n_states) as g:
        g.track_minima(True)
        g.run(sweeps)
        e_min, xyz = g.minima(0)
    seen = np.isfinite(ref.min_e)
    assert np.array_equal(np.isfinite(e_min), seen)
    assert np.allclose(e_min[seen], ref.min_e[seen], rtol=1e-10, atol=1e-9)
    for N in np.nonzero(seen)[0]:
        assert np.array_equal(xyz[N, :N], ref.min_xyz[N, :N]), N
    mu = np.linspace(-9.0, -1.0, 161)
    assert np.array_equal(regc.aiat_phase(e_min, mu), oracle.aiat_phase(ref.min_e, mu))


@pytest.mark.parametrize("persist,split,wpb", [(1, 0, 0), (4, 2, 0), (3, 1, 4), (2, 1, 1)])
def test_fp64_persistent_launch_keeps_the_trajectories(persist, split, wpb):
    """Whole exchange intervals in one cooperative launch, the exchange steps inside
    it between grid barriers: accept bits, N, labels, samples and exchange counters
    equal the oracle's -- one class (two or one waves per walker, a partly filled
    workgroup of four walkers), an odd grid with the diagonal scheme, and the uneven
    batch of three classes (runs that do not start on an interval boundary)."""
    w = W.small_lj(n_t=4, n_mu=4, n_max=20, n_sweeps=60)
    _fp64_trajectory(w, 60, persistent=persist, split=split, walkers_per_block=wpb)
    w3 = W.config3_classes()[0].replace(t=W.linear_grid(0.6, 1.8, 3), mu=W.linear_grid(-6.0, -2.5, 5),
                                        n_max=60, swap_scheme=1, sample_every=3)
    _fp64_trajectory(w3, 100, persistent=persist, split=split, walkers_per_block=wpb)
    test_fp64_uneven_batch(0, persistent=persist, split=split, walkers_per_block=wpb)


def test_persistent_launch_option_errors():
    w = W.small_lj(n_t=2, n_mu=2, n_max=10)
    for bad in (dict(persistent=2, graph_intervals=2), dict(persistent=2, cull=1), dict(persistent=2, batch_trials=4),
                dict(persistent=2, split=4), dict(persistent=-1), dict(balance=2), dict(balance=-2)):
        with pytest.raises(regc.RegcError) as ei:
            regc.Regc(w, **bad)
        assert ei.value.code == regc.EINVAL, bad


def test_fp64_minima_per_class_of_a_batch():
    classes = _batch_classes()
    sweeps = 45
    with regc.Regc(classes, precision=regc.FP64, sample_capacity=(sweeps // 3 + 1) * sum(
            w.n_states for w in classes)) as g:
        g.track_minima(True)
        g.run(sweeps)
        mins = [g.minima(c) for c in range(len(classes))]
        offs = g.offsets
    for c, w in enumerate(classes):
        ref = oracle.Chain(w, walker_offset=offs[c], class_id=c)
        ref.run(sweeps)
        e_min, xyz = mins[c]
        seen = np.isfinite(ref.min_e)
        assert np.array_equal(np.isfinite(e_min), seen), c
        assert np.allclose(e_min[seen], ref.min_e[seen], rtol=1e-10, atol=1e-9), c
        for N in np.nonzero(seen)[0]:
            assert np.array_equal(xyz[N, :N], ref.min_xyz[N, :N]), (c, N)


# ---------------------------------------------------------------------------
# Molecular dynamics as the canonical part of the REGC step
# ---------------------------------------------------------------------------
def _md_trajectory(w, steps, atol=1e-9):
    _say(f"[md] {w.name} steps={steps}")
    ref = oracle.Chain(w)
    r = ref.run(steps, trace=True)
    with regc.Regc(w, precision=regc.FP64, trace_capacity=steps,
                   sample_capacity=(steps // max(w.sample_every, 1) + 1) * w.n_states) as g:
        g.run(steps)
        bits, nps = g.trace(steps)
        wk = g.walkers()
        st = g.stats()
        smp = g.samples()
    assert _first_divergence(bits, r["bits"], nps, r["trace_n"]) is None
    assert np.array_equal(wk["n"], ref.n) and np.array_equal(wk["label"], ref.label)
    assert np.array_equal(st["stats"], ref.stats) and np.array_equal(st["swap_acc"], ref.swap_acc)
    for k in range(ref.S):
        assert np.allclose(wk["xyz"][k, : ref.n[k]], ref.xyz[k, : ref.n[k]], rtol=0, atol=atol), k
    assert np.allclose(wk["e"], ref.e, rtol=1e-9, atol=1e-9)
    assert np.array_equal(smp["n"], r["n"])
    assert np.allclose(smp["e"], r["e"], rtol=1e-9, atol=1e-9)
    return ref


def test_fp64_md_trajectories_config1():
    """64 replicas, x0 = 0.9, 10 velocity-Verlet steps with the thermostat per REGC
    step: identical exchange decisions and N, positions within 1e-9 after 300 MD steps."""
    ref = _md_trajectory(W.paper_schedule_md(W.config1(), x0=0.9, md_steps=10, sample_every=5), 30)
    assert ref.n.sum() > 0


def test_fp64_md_variants():
    # no thermostat (NVE between exchange attempts), a binned slab, frequent exchanges
    w = W.paper_schedule_md(W.config3_classes()[0].replace(t=W.linear_grid(0.6, 1.8, 3),
                                                          mu=W.linear_grid(-4.0, -2.5, 3), n_max=60),
                            x0=0.7, md_steps=4, md_dt=0.004, md_tau=0.0, sample_every=2)
    _md_trajectory(w, 40)
    _md_trajectory(W.paper_schedule_md(W.ideal_gas(n_t=2, n_mu=2, n_max=30), x0=0.8, md_steps=3, sample_every=1), 60)


def test_fp32_md_lj_mean_n_matches_the_monte_carlo_oracle():
    w = W.small_lj(n_t=2, n_mu=2, n_max=14, mu=(-4.5, -3.0)).replace(sample_every=1)
    ref = oracle.Chain(w)
    ref.run(1000)
    r = ref.run(20000)
    wm = W.paper_schedule_md(w, x0=0.7, md_steps=5, md_dt=0.005, md_tau=0.05, sample_every=1)
    steps = 30000
    with regc.Regc(wm, precision=regc.FP32PAIR, sample_capacity=steps * w.n_states) as g:
        g.run(2000)
        g.clear_samples()
        g.run(steps)
        smp = g.samples()
    na, _ = per_state_series(r, w.n_states)
    nb, _ = per_state_series(smp, w.n_states)
    z = []
    for s in range(w.n_states):
        ma, sa = batch_means(na[:, s])
        mb, sb = batch_means(nb[:, s])
        z.append((ma - mb) / math.hypot(sa, sb))
    assert_within_3se(z, "FP32 MD against the Monte Carlo oracle")
