"""The entry point that allocates nothing (shape3d_noalloc, static device
scratch) against the existing entry point shape3d_ex, through the C ABI: two
calls in a row, the second on a smaller input, then its limits."""
import ctypes
import sys

import numpy as np
import pytest

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


def via_ex(S, m, sp):
    import torch

    lib = S.load()
    vol = torch.from_numpy(m).cuda()
    dims, spc = S._dims_spacing(m.shape, sp)
    out = (ctypes.c_double * 6)()
    st = S.Stats()
    rc = lib.shape3d_ex(ctypes.c_void_p(vol.data_ptr()), S.U8 if m.dtype == np.uint8 else S.F32, dims, spc, out,
                        ctypes.byref(st), 0, S._stream())
    return np.array(out[:]), rc


def via_noalloc(S, m, sp):
    import torch

    lib = S.load()
    vol = torch.from_numpy(m).cuda()
    dims, spc = S._dims_spacing(m.shape, sp)
    out = torch.full((6,), -1.0, dtype=torch.float64, device="cuda")
    status = torch.full((1,), -100, dtype=torch.int32, device="cuda")
    rc = lib.shape3d_noalloc(ctypes.c_void_p(vol.data_ptr()), S.U8 if m.dtype == np.uint8 else S.F32, dims, spc,
                             ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(status.data_ptr()), S._stream())
    torch.cuda.synchronize()
    return out.cpu().numpy(), int(status.item()), rc


def test_noalloc_matches_shape3d_ex(S):
    g = np.random.default_rng(8)
    inputs = [("64^3 ellipsoid", synth.single_roi(7)[0], (1.25, 0.7, 0.7)),
              ("20x24x28 random", synth.random_mask((20, 24, 28), 0.3, g), (1.0, 1.0, 1.0)),
              ("soft 32^3", synth.differentiable_small(4)[0], (0.8, 0.8, 2.0)),
              ("5x3x4 box", synth.box_mask((5, 3, 4), (1, 1, 1), (3, 1, 2)), (1.0, 1.0, 1.0))]
    for name, m, sp in inputs:  # each input is smaller than the one before
        say("noalloc vs shape3d_ex: %s" % name)
        f_ex, rc_ex = via_ex(S, m, sp)
        f_na, st_na, rc_na = via_noalloc(S, m, sp)
        assert rc_na == S.OK and rc_ex in (S.OK, S.EMPTY)
        assert st_na == rc_ex, name
        np.testing.assert_allclose(f_na[:2], f_ex[:2], rtol=1e-12, atol=0, err_msg=name)
        np.testing.assert_array_equal(f_na[2:], f_ex[2:], err_msg=name)


def test_noalloc_limits(S):
    import torch

    lib = S.load()
    # beyond the voxel limit: refused on the host, nothing enqueued
    big = torch.zeros((257, 256, 256), dtype=torch.uint8, device="cuda")
    dims, spc = S._dims_spacing(big.shape, (1, 1, 1))
    out = torch.full((6,), -1.0, dtype=torch.float64, device="cuda")
    status = torch.full((1,), -100, dtype=torch.int32, device="cuda")
    say("noalloc: over the voxel limit")
    rc = lib.shape3d_noalloc(ctypes.c_void_p(big.data_ptr()), S.U8, dims, spc, ctypes.c_void_p(out.data_ptr()),
                             ctypes.c_void_p(status.data_ptr()), S._stream())
    torch.cuda.synchronize()
    assert rc == S.ECAPACITY and int(status.item()) == -100
    # within the voxel limit but with more vertices than the scratch holds:
    # status ECAPACITY on the device, out untouched
    say("noalloc: mesh beyond the scratch")
    g = np.random.default_rng(3)
    m = synth.random_mask((64, 128, 128), 0.5, g)
    f, st, rc = via_noalloc(S, m, (1, 1, 1))
    assert rc == S.OK and st == S.ECAPACITY and (f == -1.0).all()
    # and the next call is unaffected
    m2, sp2 = synth.single_roi(8)
    f_ex, rc_ex = via_ex(S, m2, sp2)
    f_na, st_na, rc_na = via_noalloc(S, m2, sp2)
    assert rc_na == S.OK and st_na == rc_ex
    np.testing.assert_array_equal(f_na[2:], f_ex[2:])
