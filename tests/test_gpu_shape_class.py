"""GPU parity of the whole Shape class (shape3d_class, and the batched calls
with SHAPE3D_SHAPE_CLASS) against the oracle's shape_class.

Bar, per member:
  * the six paper features: as in test_gpu_parity (area and volume within
    relative 1e-9, diameters equal to the oracle's exact FP64 maxima), and
    bit-identical to the plain six-feature call;
  * VoxelVolume: relative 1e-12 (an integer count times the spacing product,
    rounded in a different order on each side);
  * SurfaceVolumeRatio, Sphericity, Compactness1/2, SphericalDisproportion:
    relative 1e-9 (closed forms of volume and area);
  * the axis lengths: relative 1e-9, plus an absolute 1e-6 of the major axis:
    the GPU sums the moments exactly in integers and the oracle in two FP64
    passes, and both eigen-solvers are backward stable (errors of order
    eps * the largest eigenvalue), which 4 sqrt(lambda) magnifies for a
    vanishing eigenvalue (a flat region) to about 4 sqrt(eps lambda_max);
  * Elongation and Flatness: relative 1e-9 plus absolute 1e-6, for the same
    reason.
"""
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


def gpu(vol):
    import torch

    return torch.from_numpy(np.ascontiguousarray(vol)).cuda()


def check_class(got, ref, name):
    """got: float64[17] from the library; ref: the oracle's shape_class dict."""
    e = ref["features"]
    np.testing.assert_allclose(got[:2], e[:2], rtol=1e-9, atol=0, err_msg=name)
    np.testing.assert_array_equal(got[2:6], e[2:6], err_msg=name)
    np.testing.assert_allclose(got[6], e[6], rtol=1e-12, atol=0, err_msg=name)
    np.testing.assert_allclose(got[7:12], e[7:12], rtol=1e-9, atol=0, err_msg=name)
    major = max(abs(e[12]), abs(got[12]))
    np.testing.assert_allclose(got[12:15], e[12:15], rtol=1e-9, atol=1e-6 * major, err_msg=name)
    np.testing.assert_allclose(got[15:17], e[15:17], rtol=1e-9, atol=1e-6, err_msg=name)


def compare(S, vol, sp, name):
    say("%s shape=%s dtype=%s spacing=%s" % (name, vol.shape, vol.dtype, tuple(sp)))
    ref = O.shape_class(vol, sp)
    t = gpu(vol)
    f, st, rc = S.shape_class(t, sp, stats=True)
    assert rc == ref["status"], name
    assert st["V"] == ref["V"] and st["T"] == ref["T"], name
    np.testing.assert_array_equal(st["pair_ids"], ref["pair_ids"], err_msg=name)
    check_class(f, ref, name)
    # the six features do not depend on whether the moments are summed
    np.testing.assert_array_equal(f[:6], S.features(t, sp), err_msg=name)
    return f, ref


def test_single_voxel_and_empty(S):
    m = np.zeros((5, 6, 7), np.uint8)
    m[2, 3, 4] = 1
    f, _ = compare(S, m, (1.25, 0.7, 0.7), "single voxel")
    # one voxel: every eigenvalue 0, so the axes, Elongation and Flatness are 0
    np.testing.assert_array_equal(f[12:], np.zeros(5))
    assert abs(f[6] - 1.25 * 0.7 * 0.7) <= 1e-15
    say("empty")
    f, st, rc = S.shape_class(gpu(np.zeros((4, 5, 6), np.uint8)), (1, 1, 1), stats=True)
    assert rc == S.EMPTY
    np.testing.assert_array_equal(f, np.zeros(17))


def test_boxes_and_flat_regions(S):
    g = np.random.default_rng(11)
    for i in range(5):
        shape = tuple(int(x) for x in g.integers(6, 30, size=3))
        size = [int(g.integers(1, s - 1)) for s in shape]
        lo = [int(g.integers(0, s - z + 1)) for s, z in zip(shape, size)]
        sp = tuple(float(x) for x in g.uniform(0.4, 2.0, size=3))
        compare(S, synth.box_mask(shape, lo, size), sp, "box %d" % i)
    # a single plane and a single line: vanishing eigenvalues
    m = np.zeros((7, 20, 30), np.uint8)
    m[3, 2:15, 4:25] = 1
    compare(S, m, (1.0, 0.8, 1.3), "plane")
    m = np.zeros((9, 9, 40), np.uint8)
    m[4, 4, 3:37] = 1
    compare(S, m, (1.0, 1.0, 0.5), "line")


def test_random_and_ellipsoids(S):
    g = np.random.default_rng(12)
    for i, shape in enumerate([(3, 3, 3), (23, 2, 47), (4, 40, 130), (33, 34, 35), (17, 64, 100)]):
        m = synth.random_mask(shape, float(g.uniform(0.1, 0.8)), g)
        sp = tuple(float(x) for x in g.uniform(0.5, 1.5, size=3))
        compare(S, m, sp, "random %d" % i)
    m, sp = synth.single_roi(0)
    compare(S, m, sp, "single ROI 64^3")
    m, _ = synth.single_roi(3, shape=(45, 301, 70))
    compare(S, m, (1.25, 0.7, 0.7), "ellipsoid over many bricks")


def test_soft_masks(S):
    p, sp = synth.differentiable_small(0)
    compare(S, p, sp, "soft 32^3")
    p = synth.soft_roi((30, 41, 52), synth.rng(9, 0), 4, 3.0, 9.0, 1.5)
    compare(S, p, (2.0, 0.8, 0.8), "soft anisotropic")


def test_batched_shape_class(S):
    """The batched call with SHAPE3D_SHAPE_CLASS: every ROI against the
    oracle and bit-identical to the single-ROI call; the six-feature batch is
    unchanged by the flag."""
    import torch

    buf, offs, shapes, sps = synth.batched_rois(48, 7, lmin=4.0, lmax=40.0)
    base = torch.from_numpy(buf).cuda()
    table = S.roi_table(offs, shapes, sps)
    say("batched shape class: 48 ROIs")
    out, status, stats = S.batched(base, table, stats=True, shape_class=True)
    out6, status6 = S.batched(base, table)
    np.testing.assert_array_equal(status, status6)
    np.testing.assert_array_equal(out[:, :6], out6)
    outg, _ = S.batched(base, table, graph=True, shape_class=True)
    outg2, _ = S.batched(base, table, graph=True, shape_class=True)
    np.testing.assert_array_equal(outg, out)
    np.testing.assert_array_equal(outg2, out)
    for r in range(len(offs)):
        n = int(np.prod(shapes[r]))
        m = buf[offs[r]:offs[r] + n].reshape(shapes[r])
        ref = O.shape_class(m, sps[r])
        assert status[r] == ref["status"], r
        assert stats[r]["V"] == ref["V"] and stats[r]["T"] == ref["T"], r
        np.testing.assert_array_equal(stats[r]["pair_ids"], ref["pair_ids"], err_msg="ROI %d" % r)
        check_class(out[r], ref, "ROI %d" % r)
        one = S.shape_class(base[int(offs[r]):int(offs[r]) + n].view(shapes[r]), sps[r])
        np.testing.assert_array_equal(one, out[r], err_msg="ROI %d" % r)


def test_batched_dev_shape_class_with_labels(S):
    """shape3d_batched_dev with SHAPE3D_SHAPE_CLASS on a label map: each label's
    crop (strided view of the map) against the oracle on the extracted mask."""
    import torch

    g = np.random.default_rng(13)
    lab = np.zeros((30, 40, 50), np.uint8)
    boxes = []
    for k in range(1, 5):
        lo = [int(g.integers(0, 20)), int(g.integers(0, 28)), int(g.integers(0, 36))]
        size = [int(g.integers(3, 10)), int(g.integers(3, 12)), int(g.integers(3, 14))]
        part = synth.random_mask(size, 0.7, g).astype(bool)
        sub = lab[lo[0]:lo[0] + size[0], lo[1]:lo[1] + size[1], lo[2]:lo[2] + size[2]]
        sub[part & (sub == 0)] = k
        boxes.append((k, lo, size))
    base = torch.from_numpy(lab.reshape(-1).copy()).cuda()
    d1, d2 = lab.shape[1], lab.shape[2]
    offs = [lo[0] * d1 * d2 + lo[1] * d2 + lo[2] for _, lo, _ in boxes]
    shapes = [tuple(size) for _, _, size in boxes]
    sps = [(1.0, 0.9, 1.1)] * len(boxes)
    table = S.roi_table_ex(offs, shapes, sps, strides=[(d1 * d2, d2)] * len(boxes), labels=[k for k, _, _ in boxes])
    tdev = S.table_to_device(table)
    say("batched_dev shape class: label crops")
    out, status = S.batched_dev(base, tdev, len(boxes), (10, 12, 14), shape_class=True)
    out = out.cpu().numpy()
    status = status.cpu().numpy()
    for r, (k, lo, size) in enumerate(boxes):
        crop = lab[lo[0]:lo[0] + size[0], lo[1]:lo[1] + size[1], lo[2]:lo[2] + size[2]]
        m = (crop == k).astype(np.uint8)
        ref = O.shape_class(m, sps[r])
        assert status[r] == ref["status"], r
        check_class(out[r], ref, "label %d" % k)


def test_large_roi_shape_class_full_size(S):
    """The benchmark's large ROI (300 x 512 x 512): the moment members against
    the oracle's (the six features are covered by test_gpu_fullsize)."""
    say("large ROI shape class: generate")
    mask, sp = synth.large_roi(0)
    t = gpu(mask)
    say("large ROI shape class: GPU")
    f = S.shape_class(t, sp)
    np.testing.assert_array_equal(f[:6], S.features(t, sp))
    say("large ROI shape class: oracle moments")
    n, _, cov = O.moments(mask, sp)
    base = dict(features=f[:6].copy(), status=0, V=0, T=0, pair_ids=None, signed_volume=0.0)
    ref = O.shape_class(mask, sp, base=base)
    assert ref["n_inside"] == n == int(mask.astype(bool).sum())
    check_class(f, ref, "large ROI")
