"""GPU parity of the learned-proposal network: bfloat16-MFMA forward and
cross-entropy gradients against the oracle's bfloat16-emulating path (same
rounding points) and against FP64; Adam steps and training on the device."""
import sys

import numpy as np
import pytest

from oracle import mlp_oracle as M
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


def _batch(rng, B=64, nmax=40):
    n = rng.integers(1, nmax + 1, B)
    # particles cluster in a few layers near the surface, as adsorbed gas does
    vox = np.zeros((B, nmax), np.uint16)
    for b in range(B):
        iz = rng.integers(0, 3, nmax)
        vox[b] = (iz * 256 + rng.integers(0, 256, nmax)).astype(np.uint16)
    excl = np.array([rng.integers(0, k) for k in n], np.int32)
    target = np.array([vox[b, excl[b]] for b in range(B)], np.int32)
    return vox, n.astype(np.int32), excl, target


def _params(seed):
    p = W.mlp_init(seed, out_scale=1.0)
    rng = np.random.default_rng(seed + 100)
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = rng.normal(0, 0.1, p[k].shape).astype(np.float32)
    return p


def test_forward_matches_bf16_oracle():
    _say("[mlp] forward")
    rng = np.random.default_rng(0)
    p = _params(1)
    vox, n, excl, _ = _batch(rng)
    net = regc.Mlp(W.mlp_pack(p))
    got = net.forward(vox, n, excl)
    ref = M.forward(p, vox, n, excl, "bf16")["logits"]
    ref64 = M.forward({k: v.astype(np.float64) for k, v in p.items()}, vox, n, excl, "fp64")["logits"]
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-3 * scale, np.abs(got - ref).max() / scale
    assert np.abs(got - ref64).max() <= 3e-2 * scale
    net.close()


def test_gradients_match_bf16_oracle():
    _say("[mlp] gradients")
    rng = np.random.default_rng(2)
    p = _params(3)
    vox, n, excl, target = _batch(rng, B=128)
    net = regc.Mlp(W.mlp_pack(p))
    loss, g = net.loss_grads(vox, n, excl, target)
    gd = W.mlp_unpack(g)
    lref, gref = M.loss_and_grads(p, vox, n, excl, target, "bf16")
    l64, g64 = M.loss_and_grads({k: v.astype(np.float64) for k, v in p.items()}, vox, n, excl, target, "fp64")
    assert abs(loss - lref) <= 1e-4 * max(1.0, abs(lref))
    for k in W.MLP_ORDER:
        scale = np.abs(gref[k]).max()
        err = np.abs(gd[k] - gref[k]).max() / scale
        assert err <= 1e-3, (k, err)
        err64 = np.abs(gd[k] - g64[k]).max() / np.abs(g64[k]).max()
        assert err64 <= 5e-2, (k, err64)
    net.close()


def test_training_lowers_the_loss():
    import torch
    _say("[mlp] training")
    rng = np.random.default_rng(4)
    nmax, ns = 24, 4096
    # a data set with structure: particles sit on a few preferred voxels
    prefer = rng.choice(4096, 32, replace=False)
    vox = prefer[rng.integers(0, 32, (ns, nmax))].astype(np.int16)
    n = rng.integers(2, nmax + 1, ns).astype(np.int32)
    vdev = torch.from_numpy(vox).cuda()
    ndev = torch.from_numpy(n).cuda()
    net = regc.Mlp(W.mlp_pack(W.mlp_init(5)))
    p0 = net.params()
    # one step: the first Adam step moves every parameter by lr * sign(g) (up to eps)
    net.train(ns, nmax, vdev.data_ptr(), ndev.data_ptr(), steps=1, batch=256, lr=1e-3, seed=9)
    p1 = net.params()
    step = np.abs(p1 - p0)
    moved = step[step > 0]
    assert moved.size > 0 and np.all(moved <= 1e-3 * (1 + 1e-5))
    assert np.median(moved) > 0.9e-3
    first = net.train(ns, nmax, vdev.data_ptr(), ndev.data_ptr(), steps=1, batch=256, lr=1e-3, seed=10)
    last = net.train(ns, nmax, vdev.data_ptr(), ndev.data_ptr(), steps=300, batch=256, lr=1e-3, seed=11)
    assert last < first - 2.0, (first, last)
    assert last < np.log(4096) - 3.0
    ms, steps = net.timing()
    _say(f"[mlp] {steps} steps in {ms:.1f} ms")
    net.close()


def test_training_rejects_a_bad_set():
    """A device training set with an N above nmax or a voxel index of 4096 or more
    among an example's first N entries is refused before any step; entries past N
    are not looked at."""
    import torch
    _say("[mlp] training set checks")
    rng = np.random.default_rng(6)
    nmax, ns = 8, 256
    vox = rng.integers(0, 4096, (ns, nmax)).astype(np.int16)
    n = np.full(ns, 4, dtype=np.int32)
    vox[5, 6] = 5000                       # past N = 4: ignored
    net = regc.Mlp(W.mlp_pack(W.mlp_init(5)))
    p0 = net.params()
    for bad_vox, bad_n in ((True, False), (False, True)):
        v, m = vox.copy(), n.copy()
        if bad_vox:
            v[100, 2] = 5000
        if bad_n:
            m[7] = nmax + 1
        vdev, ndev = torch.from_numpy(v).cuda(), torch.from_numpy(m).cuda()
        with pytest.raises(regc.RegcError) as ei:
            net.train(ns, nmax, vdev.data_ptr(), ndev.data_ptr(), steps=1, batch=64, lr=1e-3, seed=1)
        assert ei.value.code == regc.EINVAL
        assert np.array_equal(net.params(), p0)
    vdev, ndev = torch.from_numpy(vox).cuda(), torch.from_numpy(n).cuda()
    net.train(ns, nmax, vdev.data_ptr(), ndev.data_ptr(), steps=1, batch=64, lr=1e-3, seed=1)
    assert not np.array_equal(net.params(), p0)
    net.close()
