"""GPU parity of the pruned 3D diameter pass: with pruning forced on, every
result (features and maximising pairs) equals the all-pairs pass and the
oracle, on tie-rich shapes (boxes, single voxels), a sphere (the least
prunable shape), random masks, ellipsoid unions and batches, including a
batch with more than 2^16 plane buckets, where whole buckets are pruned too.
The single-ROI cases switch the small-ROI path off, so that they run the
general pipeline that prunes."""
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
    before = shape3d.get_prune()
    shape3d.set_small_path(False)
    yield shape3d
    shape3d.set_small_path(True)
    shape3d.set_prune(before)


def sphere(n, r):
    c = (n - 1) / 2.0
    z, y, x = np.mgrid[:n, :n, :n]
    return (((z - c) ** 2 + (y - c) ** 2 + (x - c) ** 2) <= r * r).astype(np.uint8)


def cases():
    g = np.random.default_rng(17)
    out = [("voxel", synth.box_mask((3, 4, 5), (1, 1, 1), (1, 1, 1)), (1.0, 1.0, 1.0)),
           ("box 6x9x7", synth.box_mask((8, 11, 9), (1, 1, 1), (6, 9, 7)), (1.0, 1.0, 1.0)),
           ("box 30x20x25 aniso", synth.box_mask((32, 22, 27), (1, 1, 1), (30, 20, 25)), (1.25, 0.7, 0.7)),
           ("sphere r=20", sphere(44, 20), (1.0, 1.0, 1.0)),
           ("random 30^3", synth.random_mask((30, 31, 29), 0.3, g), (0.9, 1.0, 1.1)),
           ("ellipsoid 64^3", synth.single_roi(6)[0], (1.0, 1.0, 1.0)),
           ("soft 32^3", synth.differentiable_small(3)[0], (1.0, 1.0, 1.0))]
    return out


def test_pruned_equals_all_pairs_and_oracle(S):
    import torch

    for name, m, sp in cases():
        vol = torch.from_numpy(m).cuda()
        say("prune %s" % name)
        S.set_prune(0)
        f0, st0, rc0 = S.features(vol, sp, stats=True)
        S.set_prune(2)
        f2, st2, rc2 = S.features(vol, sp, stats=True)
        assert rc0 == rc2
        np.testing.assert_array_equal(f2, f0, err_msg=name)
        np.testing.assert_array_equal(st2["pair_ids"], st0["pair_ids"], err_msg=name)
        ref = O.shape3d(m, sp)
        np.testing.assert_array_equal(f2[2:], ref["features"][2:], err_msg=name)
        np.testing.assert_array_equal(st2["pair_ids"], ref["pair_ids"], err_msg=name)


def test_pruned_batch(S):
    import torch

    buf, offs, shapes, sps = synth.batched_rois(60, seed=9, lmin=6, lmax=60)
    base = torch.from_numpy(buf).cuda()
    table = S.roi_table(offs, shapes, sps)
    say("pruned batch of 60 ROIs")
    S.set_prune(0)
    o0, s0 = S.batched(base, table)
    S.set_prune(2)
    o2, s2 = S.batched(base, table)
    o2g, s2g = S.batched(base, table, graph=True)
    o2r, s2r = S.batched(base, table, graph=True)
    np.testing.assert_array_equal(o2, o0)
    np.testing.assert_array_equal(s2, s0)
    np.testing.assert_array_equal(o2g, o0)
    np.testing.assert_array_equal(o2r, o0)
    for r in range(0, len(offs), 7):
        m = buf[offs[r]:offs[r] + int(np.prod(shapes[r]))].reshape(shapes[r])
        ref = O.shape3d(m, sps[r])
        np.testing.assert_array_equal(o2[r, 2:], ref["features"][2:])


def test_pruned_buckets(S):
    """More than 2^16 plane buckets: buckets whose box cannot hold their
    family's planar diameter are dropped before the pair pass."""
    buf, offs, shapes, sps = synth.batched_rois_torch(400, 11, lmin=40.0, lmax=64.0)
    assert sum(2 * (d[0] + d[1] + d[2]) + 3 for d in shapes) >= 1 << 16
    table = S.roi_table(offs, shapes, sps)
    say("bucket pruning: 400 ROIs")
    S.set_prune(0)
    o0, s0, st0 = S.batched(buf, table, stats=True)
    S.set_prune(2)
    o2, s2, st2 = S.batched(buf, table, stats=True)
    o2g, _ = S.batched(buf, table, graph=True)
    o2r, _ = S.batched(buf, table, graph=True)
    np.testing.assert_array_equal(o2, o0)
    np.testing.assert_array_equal(s2, s0)
    np.testing.assert_array_equal(o2g, o0)
    np.testing.assert_array_equal(o2r, o0)
    for r in range(len(offs)):
        np.testing.assert_array_equal(st2[r]["pair_ids"], st0[r]["pair_ids"], err_msg="ROI %d" % r)
        # the in-plane pair count covers the dropped buckets' pairs too
        assert st2[r]["pairs_2d"] == st0[r]["pairs_2d"], r
    host = buf.cpu().numpy()
    for r in range(0, len(offs), 50):
        m = host[offs[r]:offs[r] + int(np.prod(shapes[r]))].reshape(shapes[r])
        ref = O.shape3d(m, sps[r])
        np.testing.assert_array_equal(o2[r, 2:], ref["features"][2:])
        np.testing.assert_array_equal(st2[r]["pair_ids"], ref["pair_ids"])
