"""GPU parity: the HIP library against the CPU FP64 oracle, on the same seeded inputs.

Bar: vertex and triangle counts and vertex sets bit-exact; area and volume
within relative 1e-9; diameters within relative 1e-6 (the refinement makes
them exact FP64 maxima, so they are also compared for equality with the
oracle's, as are the maximising pairs).
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_02894_amd import synth

pytestmark = pytest.mark.gpu

RTOL_AV = 1e-9
RTOL_D = 1e-6


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


def compare(S, vol, sp, name, exact_pairs=True):
    say("%s shape=%s dtype=%s spacing=%s" % (name, vol.shape, vol.dtype, tuple(sp)))
    ref = O.shape3d(vol, sp)
    f, st, rc = S.features(gpu(vol), sp, stats=True)
    assert rc == ref["status"], name
    assert st["V"] == ref["V"], name
    assert st["T"] == ref["T"], name
    rf = ref["features"]
    np.testing.assert_allclose(f[:2], rf[:2], rtol=RTOL_AV, atol=0, err_msg=name)
    np.testing.assert_allclose(f[2:], rf[2:], rtol=RTOL_D, atol=0, err_msg=name)
    if exact_pairs:
        np.testing.assert_array_equal(f[2:], rf[2:], err_msg=name)
        np.testing.assert_array_equal(st["pair_ids"], ref["pair_ids"], err_msg=name)
    return f, st, ref


def test_single_voxel(S):
    for sp in [(1.0, 1.0, 1.0), (1.25, 0.7, 0.7), (0.3, 2.0, 1.1)]:
        m = np.zeros((5, 6, 7), np.uint8)
        m[2, 3, 4] = 1
        f, st, ref = compare(S, m, sp, "single voxel")
    m = np.ones((1, 1, 1), np.uint8)
    f, _, _ = compare(S, m, (1, 1, 1), "1x1x1")
    np.testing.assert_allclose(f, [1 / 6, np.sqrt(3), 1, 1, 1, 1], rtol=1e-15)


def test_empty_mask(S):
    say("empty")
    f, st, rc = S.features(gpu(np.zeros((9, 10, 11), np.uint8)), (1, 1, 1), stats=True)
    assert rc == S.EMPTY and st["V"] == 0
    np.testing.assert_array_equal(f, np.zeros(6))


def test_boxes(S):
    g = np.random.default_rng(4)
    for i in range(6):
        a = [int(x) for x in g.integers(1, 9, size=3)]
        shape = tuple(a[k] + int(g.integers(0, 40)) for k in range(3))
        lo = [int(g.integers(0, shape[k] - a[k] + 1)) for k in range(3)]
        sp = tuple(float(x) for x in g.uniform(0.5, 1.5, size=3))
        compare(S, synth.box_mask(shape, lo, a), sp, "box %d" % i)


@pytest.mark.parametrize("shape", [(3, 3, 3), (5, 7, 33), (9, 31, 32), (12, 17, 65), (20, 21, 22), (4, 40, 130),
                                   (23, 2, 47)])
def test_random_masks(S, shape):
    g = np.random.default_rng(sum(shape))
    for dens in (0.15, 0.5, 0.85):
        sp = tuple(float(x) for x in g.uniform(0.4, 1.6, size=3))
        compare(S, synth.random_mask(shape, dens, g), sp, "random %s %.2f" % (shape, dens))


def test_labels_any_nonzero(S):
    g = np.random.default_rng(9)
    m = (g.integers(0, 4, size=(14, 15, 48)) * 60).astype(np.uint8)  # labels 0, 60, 120, 180
    compare(S, m, (1.0, 0.8, 1.2), "labels")


def test_ellipsoid_single_roi(S):
    m, sp = synth.single_roi(0)
    compare(S, m, sp, "single ROI 64^3")
    m, sp = synth.single_roi(3)
    compare(S, m, (1.25, 0.7, 0.7), "single ROI 64^3 anisotropic")


def test_many_bricks_ragged(S):
    # several bricks along every direction, dims with ragged tails
    g = synth.rng(77, 0)
    params = synth.ellipsoid_params(g, 6, 6.0, 20.0, 10.0, 60.0)
    m = synth.ellipsoid_union((45, 301, 70), params).astype(np.uint8)
    compare(S, m, (1.1, 0.9, 0.6), "ellipsoids 45x301x70")


def test_vertex_set(S):
    g = np.random.default_rng(12)
    for shape in [(6, 9, 40), (17, 33, 64)]:
        m = synth.random_mask(shape, 0.4, g)
        sp = (0.9, 1.1, 0.7)
        say("vertex set %s" % (shape,))
        ids, pos, _ = O.vertices(m, sp)
        gid, gpos = S.vertices(gpu(m), sp)
        gid = gid.cpu().numpy()
        gpos = gpos.cpu().numpy()
        o = np.argsort(gid)
        np.testing.assert_array_equal(gid[o], ids)
        np.testing.assert_array_equal(gpos[o], pos)


def test_soft_masks(S):
    for seed in range(3):
        p, _ = synth.differentiable_small(seed, shape=(24, 26, 37))
        sp = (1.0, 0.9, 1.2)
        compare(S, p, sp, "soft %d" % seed)
    g = np.random.default_rng(5)
    p = g.random((11, 13, 50)).astype(np.float32)
    compare(S, p, (0.7, 1.0, 1.3), "soft uniform noise")


def test_soft_binary_values_equal_binary(S):
    g = np.random.default_rng(6)
    m = synth.random_mask((10, 12, 40), 0.5, g)
    sp = (1.2, 0.8, 1.0)
    say("soft {0,1} vs binary")
    fb = S.features(gpu(m), sp)
    fs = S.features(gpu(m.astype(np.float32)), sp)
    np.testing.assert_array_equal(fb[2:], fs[2:])
    np.testing.assert_allclose(fb[:2], fs[:2], rtol=1e-12)


def test_deterministic(S):
    m, sp = synth.single_roi(1)
    say("determinism")
    a = S.features(gpu(m), sp, stats=True)
    b = S.features(gpu(m), sp, stats=True)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1]["pair_ids"], b[1]["pair_ids"])


def test_plain_entry_point(S):
    m, sp = synth.single_roi(2)
    say("shape3d() entry point")
    f, rc = S.shape3d_u8(gpu(m), sp)
    ref = O.shape3d(m, sp)
    np.testing.assert_allclose(f, ref["features"], rtol=RTOL_AV)


def test_errors(S):
    import torch

    say("error paths")
    t = torch.zeros((4, 4, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(S.Shape3DError) as e:
        S.features(t, (1.0, -1.0, 1.0))
    assert e.value.status == S.EINVAL
    with pytest.raises(S.Shape3DError) as e:
        S.features(t, (1.0, float("nan"), 1.0))
    assert e.value.status == S.EINVAL
    # dims larger than the allocation are refused before any kernel runs: a
    # raw 100-byte hipMalloc (the runtime that libshape3d.so uses) is exactly
    # the allocation the range check sees
    import ctypes

    lib = S.load()
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    dims = (ctypes.c_int64 * 3)(64, 64, 64)
    sp = (ctypes.c_double * 3)(1, 1, 1)
    out = (ctypes.c_double * 6)(*([7.0] * 6))
    p = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(p), 100) == 0
    try:
        assert lib.shape3d(p, dims, sp, out) == S.EINVAL
        assert list(out) == [7.0] * 6  # outputs untouched on failure
        small = (ctypes.c_int64 * 3)(4, 5, 5)  # exactly 100 voxels: accepted
        assert lib.shape3d(p, small, sp, out) in (S.OK, S.EMPTY)
    finally:
        hip.hipFree(p)
    # the binding checks a batch table against the tensor before the call
    t = torch.zeros(100, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        S.batched(t, S.roi_table([0], [(5, 5, 5)], [(1, 1, 1)]))
