"""GPU parity of the soft-mask adjoint: dL/dp against the oracle's FP64 reference
gradient (itself pinned by closed forms and finite differences), plus the
single-voxel closed form, autograd wiring and GPU finite differences."""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_02894_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_02894_amd import shape3d

    shape3d.load()
    return shape3d


def gpu(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check_grad(S, p, sp, gout, name):
    say("%s shape=%s gout=%s" % (name, p.shape, np.round(gout, 3)))
    pt = gpu(p)
    feats, saved = S.soft_forward(pt, sp)
    ref = O.shape3d(p, sp)
    np.testing.assert_allclose(feats, ref["features"], rtol=1e-9)
    got = S.soft_backward(pt, saved, gout).cpu().numpy().astype(np.float64)
    exp = O.soft_grad(p, sp, gout)
    scale = np.abs(exp).max()
    assert scale > 0
    # float32 output of FP64 arithmetic: relative 1e-6 of the largest entry
    np.testing.assert_allclose(got, exp, rtol=2e-6, atol=2e-6 * scale, err_msg=name)
    assert np.array_equal(got != 0, exp != 0) or np.abs(got[(got != 0) != (exp != 0)]).max() < 1e-6 * scale
    return got, exp


def test_single_soft_voxel_closed_form(S):
    p = np.zeros((3, 3, 3), np.float32)
    p[1, 1, 1] = 1.0
    got, _ = check_grad(S, p, (1, 1, 1), [1, 0, 0, 0, 0, 0], "single voxel dV")
    assert got[1, 1, 1] == pytest.approx(0.5, rel=1e-6)
    assert got[2, 1, 1] == pytest.approx(1 / 12, rel=1e-6)
    got, _ = check_grad(S, p, (1, 1, 1), [0, 1, 0, 0, 0, 0], "single voxel dA")
    assert got[1, 1, 1] == pytest.approx(2 * math.sqrt(3), rel=1e-6)
    assert got[1, 0, 1] == pytest.approx(1 / math.sqrt(3), rel=1e-6)
    # anisotropic spacing: the diameter has a unique maximising pair
    check_grad(S, p, (1.3, 0.8, 1.05), [0.7, 1.3, 0.9, 0.4, 0.5, 0.6], "single voxel all features")


@pytest.mark.parametrize("seed", range(3))
def test_soft_grad_vs_oracle(S, seed):
    g = np.random.default_rng(seed)
    p, _ = synth.differentiable_small(seed, shape=(24, 26, 37))
    sp = tuple(float(x) for x in g.uniform(0.6, 1.4, size=3))
    gout = g.uniform(-1, 1, size=6)
    check_grad(S, p, sp, gout, "soft %d" % seed)


def test_soft_grad_32cube_loss(S):
    # the differentiable workload's gradient-check instance: L = area + 0.1 volume + diameter
    p, sp = synth.differentiable_small(0, shape=(32, 32, 32))
    check_grad(S, p, sp, [0.1, 1.0, 1.0, 0.0, 0.0, 0.0], "32^3 L")


def test_autograd_function(S):
    import torch

    p, sp = synth.differentiable_small(1, shape=(20, 22, 24))
    say("autograd")
    pt = gpu(p).requires_grad_(True)
    f = S.shape_features(pt, sp)
    w = torch.tensor([0.1, 1.0, 1.0, 0.3, 0.2, 0.1], dtype=torch.float64, device=pt.device)
    (f * w).sum().backward()
    exp = O.soft_grad(p, sp, w.cpu().numpy())
    np.testing.assert_allclose(pt.grad.cpu().numpy(), exp, rtol=2e-6, atol=2e-6 * np.abs(exp).max())


def fd_check(S, p, sp, gout, name, seed=3, n=40, need=25):
    """Central finite differences of L = gout . F on the GPU forward pass
    against the GPU backward pass, at voxels away from the isolevel; a voxel
    whose perturbation changes a maximising pair (a kink of L) is skipped."""
    say("GPU finite differences: " + name)
    pt = gpu(p)
    f0, saved = S.soft_forward(pt, sp)
    grad = S.soft_backward(pt, saved, gout).cpu().numpy()
    h = 2.0 ** -13
    cand = np.argwhere((p > 0.05) & (p < 0.95) & (np.abs(p - 0.5) > 4 * h))
    rng = np.random.default_rng(seed)
    checked = 0
    for idx in map(tuple, cand[rng.choice(len(cand), size=min(n, len(cand)), replace=False)]):
        pp, pm = p.copy(), p.copy()
        pp[idx] += np.float32(h)
        pm[idx] -= np.float32(h)
        fp, sp_ = S.soft_forward(gpu(pp), sp)
        fm, sm_ = S.soft_forward(gpu(pm), sp)
        same = all(np.array_equal(np.ctypeslib.as_array(x.pair_ids), np.ctypeslib.as_array(saved.pair_ids))
                   for x in (sp_, sm_))
        if not same:
            continue
        fd = (np.dot(gout, fp) - np.dot(gout, fm)) / (2 * h)
        assert grad[idx] == pytest.approx(fd, rel=5e-4, abs=5e-5), (name, idx)
        checked += 1
    assert checked >= need, (name, checked)


def test_gpu_finite_differences(S):
    p, sp = synth.differentiable_small(2, shape=(20, 20, 20))
    fd_check(S, p, sp, np.array([0.1, 1.0, 1.0, 0.5, 0.7, 0.3]), "20^3, all six features")


def test_gpu_finite_differences_32cube(S):
    # the differentiable workload's gradient-check instance: 32^3, L = area + 0.1 volume + diameter
    p, sp = synth.differentiable_small(0, shape=(32, 32, 32))
    fd_check(S, p, sp, np.array([0.1, 1.0, 1.0, 0.0, 0.0, 0.0]), "32^3, L = area + 0.1 volume + diameter",
             n=60, need=40)


def test_differentiable_full_size(S):
    # the differentiable workload at full size: 256^3 soft mask, L = area + 0.1 volume + diameter
    say("differentiable 256^3: generate")
    p, sp = synth.differentiable_roi(0)
    gout = [0.1, 1.0, 1.0, 0.0, 0.0, 0.0]
    check_grad(S, p, sp, gout, "differentiable 256^3")
