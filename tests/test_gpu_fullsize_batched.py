"""Full-size parity of the batched workloads, in the configuration bench.py
times (graph replay, default pair-pass setting): every ROI of the 4096-ROI
uint8 batch against the single-ROI entry point (bit for bit), a sample of
ROIs against the oracle, and the 256-ROI batched soft forward and backward
against single-ROI calls and, on its smallest ROIs, against the oracle's FP64
features and gradient."""
import os
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


def check_features(got, exp, name):
    np.testing.assert_allclose(got[:2], exp[:2], rtol=1e-9, err_msg=name)   # volume, area
    np.testing.assert_allclose(got[2:], exp[2:], rtol=1e-6, err_msg=name)   # diameters


def test_batched_4096_rois_full_size(S):
    import torch

    say("batched 4096 ROIs: generate")
    buf, offs, shapes, sps = synth.batched_rois_torch(4096, 0)
    table = S.roi_table(offs, shapes, sps)
    say("batched 4096 ROIs: record + replay")
    out, status = S.batched(buf, table, graph=True)
    out2, _ = S.batched(buf, table, graph=True)
    assert np.array_equal(out, out2)
    assert np.all(status == 0)
    say("batched 4096 ROIs: single-ROI calls")
    V = np.zeros(len(offs), np.int64)
    for r in range(len(offs)):
        n = int(np.prod(shapes[r]))
        f, st, _ = S.features(buf[int(offs[r]):int(offs[r]) + n].view(shapes[r]), sps[r], stats=True)
        assert np.array_equal(f, out2[r]), r
        V[r] = st["V"]
    # oracle on a sample spanning the vertex counts (up to 60k vertices)
    order = np.argsort(V)
    small = order[V[order] <= 60000]
    picks = small[np.linspace(0, len(small) - 1, 8).astype(int)]
    host = buf.cpu().numpy()
    for r in picks:
        n = int(np.prod(shapes[r]))
        m = host[int(offs[r]):int(offs[r]) + n].reshape(shapes[r])
        say("batched 4096 ROIs: oracle on ROI %d (V=%d)" % (r, V[r]))
        exp = O.shape3d(m, sps[r])
        check_features(out2[r], exp["features"], "ROI %d" % r)
    del torch


def test_batched_soft_256_rois_full_size(S):
    import torch

    say("batched soft 256 ROIs: generate")
    workers = max(1, min(16, os.cpu_count() or 1))
    buf, offs, shapes, sps = synth.soft_batch(256, 0, workers=workers)
    base = torch.from_numpy(buf).cuda()
    table = S.roi_table(offs, shapes, sps)
    say("batched soft 256 ROIs: forward (record + replay) and backward")
    out, saved = S.batched_soft_forward(base, table, graph=True)
    out2, saved2 = S.batched_soft_forward(base, table, graph=True)
    assert np.array_equal(out, out2)
    gout = np.ones((len(offs), 6))
    grad = S.batched_soft_backward(base, table, saved2, gout).cpu().numpy()
    sizes = np.array([int(np.prod(s)) for s in shapes])
    order = np.argsort(sizes)
    # single-ROI calls on a sample: identical features and gradients
    for r in order[np.linspace(0, len(order) - 1, 6).astype(int)]:
        n = sizes[r]
        p = buf[offs[r]:offs[r] + n].reshape(shapes[r])
        pt = torch.from_numpy(np.ascontiguousarray(p)).cuda()
        say("batched soft: single-ROI calls on ROI %d %s" % (r, shapes[r]))
        f1, s1 = S.soft_forward(pt, sps[r])
        assert np.array_equal(f1, out2[r]), r
        g1 = S.soft_backward(pt, s1, gout[r]).cpu().numpy()
        assert np.array_equal(g1.reshape(-1), grad[offs[r]:offs[r] + n]), r
    # oracle features and FP64 gradient on the two smallest ROIs
    for r in order[:2]:
        n = sizes[r]
        p = buf[offs[r]:offs[r] + n].reshape(shapes[r])
        say("batched soft: oracle on ROI %d %s" % (r, shapes[r]))
        exp = O.shape3d(p, sps[r])
        check_features(out2[r], exp["features"], "soft ROI %d" % r)
        eg = O.soft_grad(p, sps[r], gout[r])
        got = grad[offs[r]:offs[r] + n].reshape(shapes[r]).astype(np.float64)
        np.testing.assert_allclose(got, eg, rtol=2e-6, atol=2e-6 * np.abs(eg).max(), err_msg="soft ROI %d" % r)
