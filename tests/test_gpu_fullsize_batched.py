"""Full-size parity of the batched workloads, in the configuration bench.py
times (graph replay, default pair-pass setting), against the oracle on every
ROI:

* the 4,096-ROI uint8 batch: V and T equal; area and volume within relative
  1e-9; the in-plane diameters and their maximising pairs equal to the
  oracle's; the 3D diameter and its pair equal to the oracle's all-pairs
  maximum (ROIs of up to 20,000 vertices) or to the exact maximum over the
  extreme points of the oracle's vertex set (larger ROIs; the farthest pair
  of a point set lies on its convex hull);
* the 256-ROI float32 soft batch: the same for the forward features, and the
  batched backward's dL/dp against the oracle's FP64 gradient on 32 ROIs
  spread over the size range.

The oracle runs in a pool of worker processes (tests/oracle_pool.py)."""
import os
import sys

import numpy as np
import pytest

from paper_2510_02894_amd import synth
from tests import oracle_pool

pytestmark = pytest.mark.gpu

BRUTE_MAX = 20000


def say(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def pool_workers():
    return max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def S():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_02894_amd import shape3d

    shape3d.load()
    return shape3d


def check_roi(r, got, st, status, ref):
    name = "ROI %d" % r
    assert st["V"] == ref["V"], name
    assert st["T"] == ref["T"], name
    if ref["V"] == 0:
        assert status == 1, name
        np.testing.assert_array_equal(got, np.zeros(6), err_msg=name)
        return
    assert status == 0, name
    np.testing.assert_allclose(got[0], abs(ref["signed_volume"]), rtol=1e-9, atol=0, err_msg=name)
    np.testing.assert_allclose(got[1], ref["area"], rtol=1e-9, atol=0, err_msg=name)
    np.testing.assert_array_equal(got[2:], np.sqrt(ref["d2"]), err_msg=name)
    np.testing.assert_array_equal(st["pair_ids"], ref["pair_ids"], err_msg=name)


def test_batched_4096_rois_full_size(S):
    say("batched 4096 ROIs: generate")
    buf, offs, shapes, sps = synth.batched_rois_torch(4096, 0)
    table = S.roi_table(offs, shapes, sps)
    say("batched 4096 ROIs: record + replay")
    out, status = S.batched(buf, table, graph=True)
    out2, status2 = S.batched(buf, table, graph=True)
    assert np.array_equal(out, out2) and np.array_equal(status, status2)
    say("batched 4096 ROIs: per-ROI statistics")
    out3, status3, stats = S.batched(buf, table, stats=True)
    assert np.array_equal(out3, out2) and np.array_equal(status3, status2)
    host = buf.cpu().numpy()
    say("batched 4096 ROIs: oracle on every ROI (%d workers)" % pool_workers())
    ref = oracle_pool.run(host, offs, shapes, sps, brute_max=BRUTE_MAX, workers=pool_workers())
    n3 = sum(1 for x in ref if x["method3d"] == "extreme points")
    say("batched 4096 ROIs: compare (%d ROIs with the 3D diameter from extreme points)" % n3)
    for r in range(len(offs)):
        check_roi(r, out2[r], stats[r], status2[r], ref[r])


def test_batched_soft_256_rois_full_size(S):
    import torch

    say("batched soft 256 ROIs: generate")
    buf, offs, shapes, sps = synth.soft_batch(256, 0, workers=pool_workers())
    base = torch.from_numpy(buf).cuda()
    table = S.roi_table(offs, shapes, sps)
    say("batched soft 256 ROIs: forward (record + replay) and backward")
    out, saved = S.batched_soft_forward(base, table, graph=True)
    out2, saved2 = S.batched_soft_forward(base, table, graph=True)
    assert np.array_equal(out, out2)
    gout = np.ones((len(offs), 6))
    grad = S.batched_soft_backward(base, table, saved2, gout).cpu().numpy()
    say("batched soft 256 ROIs: per-ROI statistics")
    out3, status3, stats = S.batched(base, table, stats=True)
    assert np.array_equal(out3, out2)
    sizes = np.array([int(np.prod(s)) for s in shapes])
    order = np.argsort(sizes)
    sample = set(int(r) for r in order[np.linspace(0, len(order) - 1, 32).astype(int)])
    gjobs = {}
    for r in sample:
        pid = np.array([[saved2[r].pair_ids[f][0], saved2[r].pair_ids[f][1]] for f in range(4)], dtype=np.int64)
        gjobs[r] = (gout[r], pid)
    say("batched soft 256 ROIs: oracle on every ROI, gradients on %d (%d workers)" % (len(sample), pool_workers()))
    ref = oracle_pool.run(buf, offs, shapes, sps, brute_max=BRUTE_MAX, workers=pool_workers(), grad=gjobs)
    for r in range(len(offs)):
        assert saved2[r].n_vertices == stats[r]["V"] and saved2[r].status == status3[r], r
        np.testing.assert_array_equal(gjobs[r][1] if r in gjobs else stats[r]["pair_ids"], stats[r]["pair_ids"])
        check_roi(r, out2[r], stats[r], status3[r], ref[r])
    for r in sorted(sample):
        n = sizes[r]
        eg = ref[r]["grad"]
        got = grad[offs[r]:offs[r] + n].reshape(shapes[r]).astype(np.float64)
        np.testing.assert_allclose(got, eg, rtol=2e-6, atol=2e-6 * np.abs(eg).max(), err_msg="soft ROI %d" % r)
