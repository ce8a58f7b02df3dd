"""CPU-side checks of the C ABI: the library loads and exports what the header declares."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shape3d.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(shape3d[a-z_0-9]*)\s*\(", text, flags=re.M)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("shape3d", "shape3d_ex", "shape3d_vertices", "shape3d_batched", "shape3d_soft_forward",
              "shape3d_soft_backward", "shape3d_batched_soft_forward", "shape3d_batched_soft_backward",
              "shape3d_get_tuning", "shape3d_set_tuning", "shape3d_autotune", "shape3d_last_error", "shape3d_release",
              "shape3d_version", "shape3d_workspace_size", "shape3d_workspace_size_v", "shape3d_batched_workspace_size",
              "shape3d_ex_async", "shape3d_batched_dev", "shape3d_noalloc", "shape3d_class", "shape3d_batched_ex",
              "shape3d_label_rois", "shape3d_host_stream"):
        assert n in names


def test_header_constants_match_binding():
    """Flag and size constants of the header equal the binding's copies."""
    from paper_2510_02894_amd import shape3d as S

    text = open(HEADER).read()
    defs = dict(re.findall(r"^#define (SHAPE3D_[A-Z0-9_]+) \(?(-?[0-9]+)\)?\s*(?:/\*.*)?$", text, flags=re.M))
    assert int(defs["SHAPE3D_N_CLASS"]) == S.N_CLASS == len(S.SHAPE_FEATURES) == 17
    assert int(defs["SHAPE3D_SHAPE_CLASS"]) == S.SHAPE_CLASS
    assert int(defs["SHAPE3D_BATCH_GRAPH"]) == S.BATCH_GRAPH
    assert int(defs["SHAPE3D_U8"]) == S.U8 and int(defs["SHAPE3D_F32"]) == S.F32
    for name, val in (("OK", S.OK), ("EMPTY", S.EMPTY), ("EINVAL", S.EINVAL), ("ENODEV", S.ENODEV),
                      ("EHIP", S.EHIP), ("ECAPACITY", S.ECAPACITY), ("ENOMEM", S.ENOMEM), ("EINTERNAL", S.EINTERNAL)):
        assert int(defs["SHAPE3D_" + name]) == val, name


def test_library_exports_every_declared_symbol():
    from paper_2510_02894_amd import shape3d as S

    if not os.path.exists(S.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(S.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", S.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (shape3d[a-z_0-9]*)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_version_and_no_device_error():
    from paper_2510_02894_amd import shape3d as S

    if not os.path.exists(S.LIB_PATH):
        pytest.skip("library not built")
    lib = S.load()
    assert lib.shape3d_version() >= 100
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    dims = (ctypes.c_int64 * 3)(4, 4, 4)
    sp = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    out = (ctypes.c_double * 6)()
    # no device: the call must fail loudly, never compute on the CPU
    rc = lib.shape3d(ctypes.c_void_p(0x1000), dims, sp, out)
    assert rc in (S.ENODEV, S.EINVAL)
    rc = lib.shape3d(None, dims, sp, out)
    assert rc == S.EINVAL


def test_cpu_tensor_is_rejected():
    import torch

    from paper_2510_02894_amd import shape3d as S

    if not os.path.exists(S.LIB_PATH):
        pytest.skip("library not built")
    with pytest.raises(TypeError):
        S.features(torch.zeros((4, 4, 4), dtype=torch.uint8), (1, 1, 1))


def test_binding_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C sizes and field offsets."""
    from paper_2510_02894_amd import shape3d as S

    structs = {"shape3d_stats": S.Stats, "shape3d_soft_saved": S.SoftSaved, "shape3d_roi": S.Roi,
               "shape3d_tuning": S.Tuning, "shape3d_roi_ex": S.RoiEx}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "shape3d.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_tuning_setting_is_validated_without_a_device():
    from paper_2510_02894_amd import shape3d as S

    if not os.path.exists(S.LIB_PATH):
        pytest.skip("library not built")
    before = S.get_tuning()
    assert before == (8, 1024, 0, 1)
    for bad in [(3, 256, 0, 0), (8, 100, 0, 0), (8, 2048, 0, 0), (8, 256, -1, 0), (8, 256, 65, 0), (16, 256, 0, 0),
                (2, 256, 0, 1), (8, 256, 0, 2)]:
        with pytest.raises(S.Shape3DError) as ei:
            S.set_tuning(*bad)
        assert ei.value.status == S.EINVAL
        assert S.get_tuning() == before
    for kernel, tiles in ((0, (2, 4, 8)), (1, (4, 8))):
        for it in tiles:
            for jc in (64, 128, 256, 512, 1024):
                S.set_tuning(it, jc, 2, kernel)
                assert S.get_tuning() == (it, jc, 2, kernel)
    S.set_tuning(*before)


def test_workspace_size_arithmetic_without_a_device():
    """Workspace sizes are host arithmetic: positive, growing with the vertex
    bound, the worst case above any bound, and refused where the mesh could
    exceed the kernels' 32-bit row indices."""
    from paper_2510_02894_amd import shape3d as S

    if not os.path.exists(S.LIB_PATH):
        pytest.skip("library not built")
    sizes = [S.workspace_size((64, 64, 64), S.U8, v) for v in (0, 100, 10_000, 100_000)]
    assert all(b > 0 for b in sizes) and sizes == sorted(sizes) and sizes[0] < sizes[-1]
    worst = S.workspace_size((64, 64, 64), S.U8)
    assert worst >= S.workspace_size((64, 64, 64), S.U8, 3 * 65 ** 3)
    assert S.workspace_size((64, 64, 64), S.F32, 10_000) > S.workspace_size((64, 64, 64), S.U8, 10_000)
    # 1e6 x 1e3 x 32767: every edge crossing gives ~1e14 rows, far past 2^31
    with pytest.raises(S.Shape3DError) as e:
        S.workspace_size((1_000_000, 1000, 32767))
    assert e.value.status == S.ECAPACITY
    # a vertex bound near 2^31 is refused as well
    with pytest.raises(S.Shape3DError) as e:
        S.workspace_size((64, 64, 64), S.U8, 1 << 31)
    assert e.value.status == S.ECAPACITY
    for bad in [(0, 4, 4), (4, 4, 40000)]:
        with pytest.raises(S.Shape3DError) as e:
            S.workspace_size(bad)
        assert e.value.status == S.EINVAL
    with pytest.raises(S.Shape3DError) as e:
        S.workspace_size((4, 4, 4), 7)
    assert e.value.status == S.EINVAL
    b1 = S.batched_workspace_size(1, (64, 64, 64), S.U8, 10_000)
    b4 = S.batched_workspace_size(4, (64, 64, 64), S.U8, 10_000)
    assert b4 > b1 > 0


def test_batch_extent_check_in_binding():
    """The binding refuses a dense ROI table that reaches past the base tensor
    (pure host arithmetic, checked before any library call)."""
    from paper_2510_02894_amd import shape3d as S

    t = S.roi_table([0, 64], [(4, 4, 4), (4, 4, 4)], [(1, 1, 1)] * 2)
    S._check_extents(t, 128)
    with pytest.raises(ValueError):
        S._check_extents(t, 127)
    with pytest.raises(ValueError):
        S._check_extents(S.roi_table([-1], [(1, 1, 1)], [(1, 1, 1)]), 10)


def test_uncovered_ranges_of_a_packed_buffer():
    """The batched soft backward zeroes only the elements outside every ROI:
    the ranges come from the table (overlaps, gaps, a tail, back-to-back ROIs)."""
    from paper_2510_02894_amd import shape3d as S

    t = S.roi_table([3, 20, 10], [(1, 2, 3), (2, 2, 2), (1, 1, 5)], [(1, 1, 1)] * 3)
    assert S._uncovered(t, 40) == [(0, 3), (9, 10), (15, 20), (28, 40)]
    t = S.roi_table([0, 6], [(1, 2, 3), (1, 1, 4)], [(1, 1, 1)] * 2)
    assert S._uncovered(t, 10) == []
    t = S.roi_table([0, 2], [(1, 1, 5), (1, 1, 2)], [(1, 1, 1)] * 2)  # the second inside the first
    assert S._uncovered(t, 8) == [(5, 8)]
