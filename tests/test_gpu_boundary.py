"""GPU parity of the caller-workspace, device-output entry points:
shape3d_ex_async (one ROI) and shape3d_batched_dev (a ROI table in device
memory, with strided crops and label selection), against the oracle and
against the host-output calls, including capacity errors and rejected table
entries."""
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


def expect(out, status, ref, what):
    assert status == ref["status"], what
    np.testing.assert_allclose(out[:2], ref["features"][:2], rtol=1e-9, atol=0, err_msg=what)
    np.testing.assert_array_equal(out[2:], ref["features"][2:], err_msg=what)


def single_cases():
    g = np.random.default_rng(41)
    cases = [("ellipsoid 64^3", synth.single_roi(3)[0], (1.0, 1.0, 1.0)),
             ("random 9x23x40", synth.random_mask((9, 23, 40), 0.4, g), (0.7, 1.1, 0.9)),
             ("box", synth.box_mask((7, 9, 8), (1, 2, 1), (4, 5, 6)), (1.25, 0.7, 0.7)),
             ("single voxel", synth.box_mask((3, 3, 3), (1, 1, 1), (1, 1, 1)), (1.0, 2.0, 0.5)),
             ("soft 32^3", synth.differentiable_small(2)[0], (1.0, 1.0, 1.0))]
    return cases


def test_async_matches_oracle(S):
    import torch

    for name, m, sp in single_cases():
        ref = O.shape3d(m, sp)
        dt = S.U8 if m.dtype == np.uint8 else S.F32
        say("async %s V=%d" % (name, ref["V"]))
        ws = torch.empty(S.workspace_size(m.shape, dt, ref["V"]), dtype=torch.uint8, device="cuda")
        out, st = S.features_async(torch.from_numpy(m).cuda(), sp, ws)
        torch.cuda.synchronize()
        expect(out.cpu().numpy(), int(st.item()), ref, name)
        # the same workspace again: nothing carried over from the last call
        out2, st2 = S.features_async(torch.from_numpy(m).cuda(), sp, ws)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out2.cpu().numpy(), out.cpu().numpy())


def test_async_empty_and_capacity(S):
    import torch

    m = np.zeros((5, 6, 7), np.uint8)
    ws = torch.empty(S.workspace_size(m.shape, S.U8, 0), dtype=torch.uint8, device="cuda")
    out, st = S.features_async(torch.from_numpy(m).cuda(), (1, 1, 1), ws)
    torch.cuda.synchronize()
    assert int(st.item()) == S.EMPTY and not out.any()
    # a workspace for half the vertices: status ECAPACITY on the device, out untouched
    m, sp = synth.single_roi(4)
    ref = O.shape3d(m, sp)
    say("capacity: V=%d, workspace for %d" % (ref["V"], ref["V"] // 2))
    ws = torch.empty(S.workspace_size(m.shape, S.U8, ref["V"] // 2), dtype=torch.uint8, device="cuda")
    out, st = S.features_async(torch.from_numpy(m).cuda(), sp, ws)
    torch.cuda.synchronize()
    assert int(st.item()) == S.ECAPACITY and not out.any()
    # the worst-case size always fits
    ws = torch.empty(S.workspace_size(m.shape, S.U8), dtype=torch.uint8, device="cuda")
    out, st = S.features_async(torch.from_numpy(m).cuda(), sp, ws)
    torch.cuda.synchronize()
    expect(out.cpu().numpy(), int(st.item()), ref, "worst-case workspace")
    # a workspace too small for even the fixed buffers is an argument error
    with pytest.raises(S.Shape3DError) as e:
        S.features_async(torch.from_numpy(m).cuda(), sp, torch.empty(4096, dtype=torch.uint8, device="cuda"))
    assert e.value.status == S.ECAPACITY


def label_volume(seed=7, shape=(60, 70, 80)):
    """A label map: three ellipsoids labelled 1, 2, 3 (later labels win)."""
    g = synth.rng(99, seed)
    vol = np.zeros(shape, np.uint8)
    for lab in (1, 2, 3):
        p = synth.ellipsoid_params(g, 1, 5, 14, 16, min(shape) - 16)
        vol[synth.ellipsoid_union(shape, p)] = lab
    return vol


def crops_of(vol):
    """Bounding-box crops of each label: (offset, dims, strides, label)."""
    D = vol.shape
    rows = []
    for lab in (1, 2, 3):
        idx = np.argwhere(vol == lab)
        if len(idx) == 0:
            continue
        lo, hi = idx.min(0), idx.max(0) + 1
        off = (lo[0] * D[1] + lo[1]) * D[2] + lo[2]
        rows.append((int(off), tuple(int(x) for x in hi - lo), (D[1] * D[2], D[2]), lab, lo, hi))
    return rows


def test_batched_dev_matches_host_batched(S):
    import torch

    buf, offs, shapes, sps = synth.batched_rois(40, seed=3, lmin=6, lmax=40)
    base = torch.from_numpy(buf).cuda()
    out_h, st_h = S.batched(base, S.roi_table(offs, shapes, sps))
    tab = S.table_to_device(S.roi_table_ex(offs, shapes, sps))
    md = tuple(int(max(s[k] for s in shapes)) for k in range(3))
    say("batched_dev eager, 40 ROIs, max dims %s" % (md,))
    out, st = S.batched_dev(base, tab, len(offs), md)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(st.cpu().numpy(), st_h)
    np.testing.assert_array_equal(out.cpu().numpy(), out_h)
    say("batched_dev with a workspace")
    vtot = sum(O.count_vertices(buf[o:o + int(np.prod(s))].reshape(s)) for o, s in zip(offs, shapes))
    ws = torch.empty(S.batched_workspace_size(len(offs), md, S.U8, vtot), dtype=torch.uint8, device="cuda")
    out, st = S.batched_dev(base, tab, len(offs), md, workspace=ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(st.cpu().numpy(), st_h)
    np.testing.assert_array_equal(out.cpu().numpy(), out_h)


def test_batched_dev_crops_and_labels(S):
    import torch

    vol = label_volume()
    rows = crops_of(vol)
    sp = [(1.25, 0.7, 0.8), (1.0, 1.0, 1.0), (0.5, 0.9, 1.5)][:len(rows)]
    offs = [r[0] for r in rows]
    dims = [r[1] for r in rows]
    strides = [r[2] for r in rows]
    labels = [r[3] for r in rows]
    # plus: label 0 over the whole volume (nonzero = inside), dense
    offs.append(0)
    dims.append(vol.shape)
    strides.append((0, 0))
    labels.append(0)
    sp.append((1.0, 1.0, 1.0))
    tab = S.table_to_device(S.roi_table_ex(offs, dims, sp, strides, labels))
    base = torch.from_numpy(vol.reshape(-1)).cuda()
    say("crops of %d labels + the whole label map" % len(rows))
    out, st = S.batched_dev(base, tab, len(offs), vol.shape)
    torch.cuda.synchronize()
    out, st = out.cpu().numpy(), st.cpu().numpy()
    for r, row in enumerate(rows):
        lo, hi = row[4], row[5]
        crop = vol[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        ref = O.shape3d((crop == row[3]).astype(np.uint8), sp[r])
        expect(out[r], int(st[r]), ref, "label %d" % row[3])
    ref = O.shape3d((vol != 0).astype(np.uint8), sp[-1])
    expect(out[-1], int(st[-1]), ref, "nonzero")
    # graph replay, then the same graph on new table contents: the entries
    # rotated by one (the same meshes, so the recorded capacity holds)
    out_g, st_g = S.batched_dev(base, tab, len(offs), vol.shape, graph=True)
    out_g2, st_g2 = S.batched_dev(base, tab, len(offs), vol.shape, graph=True, out=out_g, status=st_g)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out_g2.cpu().numpy(), out)
    k = len(offs)
    rot = lambda xs: [xs[(i + 1) % k] for i in range(k)]
    tab2 = S.table_to_device(S.roi_table_ex(rot(offs), rot(dims), rot(sp), rot(strides), rot(labels)))
    tab.copy_(tab2)
    out_g3, st_g3 = S.batched_dev(base, tab, len(offs), vol.shape, graph=True, out=out_g, status=st_g)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out_g3.cpu().numpy(), np.array(rot(list(out))))
    np.testing.assert_array_equal(st_g3.cpu().numpy(), np.array(rot(list(st))))


def test_batched_dev_rejects_bad_entries(S):
    import ctypes

    import torch

    m, sp = synth.single_roi(5, shape=(20, 24, 28))
    n = m.size
    host = np.ascontiguousarray(np.concatenate([m.reshape(-1), m.reshape(-1)]))
    # a raw allocation of exactly 2 n bytes (the runtime libshape3d.so uses),
    # so that the table check sees the true end of the data
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    base = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(base), 2 * n) == 0
    try:
        assert hip.hipMemcpy(base, host.ctypes.data, 2 * n, 1) == 0  # host to device
        hip.hipDeviceSynchronize()
        ref = O.shape3d(m, sp)
        offs = [0, n, n + 1, 0, 0, 0, 0]
        dims = [m.shape, m.shape, m.shape, (20, 24, 29), m.shape, m.shape, m.shape]
        strides = [(0, 0), (0, 0), (0, 0), (0, 0), (24 * 28, 27), (0, 0), (0, 0)]
        labels = [0, 0, 0, 0, 0, 300, 0]
        sps = [sp] * 7
        sps[6] = (1.0, -1.0, 1.0)
        tab = S.table_to_device(S.roi_table_ex(offs, dims, sps, strides, labels))
        out = torch.zeros((7, 6), dtype=torch.float64, device="cuda")
        st = torch.full((7,), -100, dtype=torch.int32, device="cuda")
        md = (ctypes.c_int64 * 3)(20, 24, 28)
        say("rejected table entries")
        rc = S.load().shape3d_batched_dev(base, S.U8, ctypes.c_void_p(tab.data_ptr()), 7, md,
                                          ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.data_ptr()), None, 0,
                                          0, S._stream())
        assert rc == S.OK
        torch.cuda.synchronize()
        out, st = out.cpu().numpy(), st.cpu().numpy()
        # 0, 1: valid; 2: one element past the allocation; 3: dims above max_dims;
        # 4: row stride below dims[2]; 5: label out of range; 6: negative spacing
        expect(out[0], int(st[0]), ref, "first")
        expect(out[1], int(st[1]), ref, "second")
        assert list(st[2:]) == [S.EINVAL] * 5
        assert not out[2:].any()
    finally:
        hip.hipFree(base)
    # float32 tables take no label
    p = torch.from_numpy(synth.differentiable_small(1)[0]).cuda()
    tab = S.table_to_device(S.roi_table_ex([0, 0], [p.shape, p.shape], [(1, 1, 1)] * 2, None, [0, 1]))
    out, st = S.batched_dev(p.reshape(-1), tab, 2, p.shape)
    torch.cuda.synchronize()
    ref = O.shape3d(p.cpu().numpy(), (1, 1, 1))
    expect(out[0].cpu().numpy(), int(st[0].item()), ref, "soft")
    assert int(st[1].item()) == S.EINVAL
