"""What the trained proposal network gains over the method without it, on the
64-replica system of the learned-proposal workload (4x4x2 slab, box 6x6x8, N <= 40):
a network trained on the GPU from plain runs' configurations lowers the held-out
cross-entropy of a left-out particle's voxel below the uniform proposal's ln 4096,
and from one equilibrated state the same number of sweeps accepts more insertions
with it (alpha = 0.9) than with uniform insertion (alpha = 0), while an untrained
random network, whose proposal ignores the occupancy, does not."""
import sys

import numpy as np
import pytest

from paper_1908_11118_amd import proposal as P
from paper_1908_11118_amd import regc
from paper_1908_11118_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _insertions(w, blob, net, alpha, sweeps):
    """Insertion attempts and acceptances (skipped attempts at the cap excluded) over
    `sweeps` sweeps from the checkpoint."""
    with regc.Regc(w.replace(sample_every=0, seed=3), precision=regc.FP32PAIR, sample_capacity=0) as g:
        g.restore(blob)
        if net is not None:
            g.set_proposal(net, alpha)
        st0 = g.stats()["stats"].copy()
        g.run(sweeps)
        st = g.stats()["stats"] - st0
    att = int(st[:, 2].sum() - st[:, 6].sum())
    return att, int(st[:, 3].sum())


def test_trained_network_accepts_more_insertions_than_uniform_insertion():
    w = W.config1()
    _say("[gain] capturing 2 x 10000 sweeps of plain runs")
    vox, n = P.capture_dataset(w, seeds=(1, 2), burnin=2000, sweeps=10000)
    _say(f"[gain] training on {int(vox.shape[0])} configurations")
    net = P.train(vox, n, steps=20000, batch=256, lr=1e-3)
    del vox, n
    # held-out cross-entropy: configurations of a third seed
    vt, nt = P.capture_dataset(w, seeds=(7,), burnin=1000, sweeps=100)
    vh = vt.cpu().numpy().view(np.uint16)
    nh = nt.cpu().numpy()
    rng = np.random.default_rng(5)
    sel = rng.choice(np.nonzero(nh > 0)[0], 4096, replace=False)
    excl = rng.integers(0, nh[sel]).astype(np.int32)
    loss, _ = net.loss_grads(vh[sel], nh[sel], excl, vh[sel, excl].astype(np.int32))
    _say(f"[gain] held-out loss {loss:.4f} against ln 4096 = {np.log(4096.0):.4f}")
    assert loss < np.log(4096.0) - 0.1

    blob = P.equilibrated_state(w, seed=3, burnin=2000)
    sweeps = 3000
    a0, k0 = _insertions(w, blob, None, 0.0, sweeps)
    a1, k1 = _insertions(w, blob, net, 0.9, sweeps)
    rnd = regc.Mlp(W.mlp_pack(W.mlp_init(11, out_scale=3.0)))
    a2, k2 = _insertions(w, blob, rnd, 0.9, sweeps)
    p0, p1, p2 = k0 / a0, k1 / a1, k2 / a2
    se = lambda p, a: np.sqrt(p * (1 - p) / a)
    z_gain = (p1 - p0) / np.hypot(se(p1, a1), se(p0, a0))
    _say(f"[gain] insertion acceptance: uniform {p0:.4f} ({a0}), trained {p1:.4f} ({a1}), random {p2:.4f} ({a2}); "
         f"z = {z_gain:.1f}")
    # binomial SEs understate the spread of correlated chains, hence the wide margin
    assert z_gain > 6.0
    assert p2 < p1
    for m in (net, rnd):
        m.close()
