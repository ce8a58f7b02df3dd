"""GPU parity of the pruned 3D diameter pass: with pruning forced on, every
result (features and maximising pairs) equals the all-pairs pass and the
oracle, on tie-rich shapes (boxes, single voxels), a sphere (the least
prunable shape), random masks, ellipsoid unions and batches."""
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
    yield shape3d
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
