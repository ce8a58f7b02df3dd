"""Python binding of ``libshape3d.so`` (see ``include/shape3d.h``).

Argument marshalling only: every step of the computation runs in the HIP
library.  Volumes are CUDA/HIP torch tensors (``torch.uint8`` binary masks or
``torch.float32`` soft masks, C-contiguous, shape (d0, d1, d2)); the work runs
on the current torch stream.  There is no CPU path: a missing library or a CPU
tensor raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshape3d.so")

OK, EMPTY, EINVAL, ENODEV, EHIP, ECAPACITY, ENOMEM, EINTERNAL = 0, 1, -1, -2, -3, -4, -5, -6
U8, F32 = 0, 1
FEATURES = (
    "MeshVolume",
    "SurfaceArea",
    "Maximum3DDiameter",
    "Maximum2DDiameterSlice",
    "Maximum2DDiameterColumn",
    "Maximum2DDiameterRow",
)
# The whole Shape class (shape3d_class): the six features, then the members
# that follow from the mesh volume, surface area, inside-voxel count and the
# principal axes of the inside voxels.
SHAPE_FEATURES = FEATURES + (
    "VoxelVolume",
    "SurfaceVolumeRatio",
    "Sphericity",
    "Compactness1",
    "Compactness2",
    "SphericalDisproportion",
    "MajorAxisLength",
    "MinorAxisLength",
    "LeastAxisLength",
    "Elongation",
    "Flatness",
)
N_CLASS = len(SHAPE_FEATURES)
PHASES = ("mesh_pass", "mesh_rows", "buckets", "pair_maxima", "refine", "finalize", "total")


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_vertices", ctypes.c_int64),
        ("n_triangles", ctypes.c_int64),
        ("pair_ids", (ctypes.c_int64 * 2) * 4),
        ("pairs_3d", ctypes.c_int64),
        ("pairs_2d", ctypes.c_int64),
        ("candidates", ctypes.c_int64 * 4),
        ("ms", ctypes.c_float * 8),
    ]

    def as_dict(self):
        return dict(
            V=int(self.n_vertices),
            T=int(self.n_triangles),
            pair_ids=np.array([[self.pair_ids[f][0], self.pair_ids[f][1]] for f in range(4)], dtype=np.int64),
            pairs_3d=int(self.pairs_3d),
            pairs_2d=int(self.pairs_2d),
            candidates=[int(x) for x in self.candidates],
            ms={PHASES[k]: float(self.ms[k]) for k in range(len(PHASES))},
        )


class SoftSaved(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int64 * 3),
        ("spacing", ctypes.c_double * 3),
        ("features", ctypes.c_double * 6),
        ("signed_volume", ctypes.c_double),
        ("pair_ids", (ctypes.c_int64 * 2) * 4),
        ("n_vertices", ctypes.c_int64),
        ("status", ctypes.c_int),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [("itile_blocks", ctypes.c_int32), ("jchunk_blocks", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("prune", ctypes.c_int32), ("small_path", ctypes.c_int32)]

    def as_tuple(self):
        return (self.itile_blocks, self.jchunk_blocks, self.blocks_per_cu, self.kernel)


class Roi(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("dims", ctypes.c_int64 * 3), ("spacing", ctypes.c_double * 3)]


class RoiEx(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("dims", ctypes.c_int64 * 3), ("spacing", ctypes.c_double * 3),
                ("strides", ctypes.c_int64 * 2), ("label", ctypes.c_int32), ("reserved", ctypes.c_int32)]


BATCH_GRAPH = 1
SHAPE_CLASS = 2


class Shape3DError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("shape3d failed with status %d: %s" % (status, message))
        self.status = status


_lib = None


def load():
    """Load ``libshape3d.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libshape3d.so is not built; run `python -m paper_2510_02894_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        i64p = ctypes.POINTER(ctypes.c_int64)
        f64p = ctypes.POINTER(ctypes.c_double)
        lib.shape3d.argtypes = [ctypes.c_void_p, i64p, f64p, f64p]
        lib.shape3d.restype = ctypes.c_int
        lib.shape3d_ex.argtypes = [ctypes.c_void_p, ctypes.c_int, i64p, f64p, f64p, ctypes.POINTER(Stats),
                                   ctypes.c_int, ctypes.c_void_p]
        lib.shape3d_ex.restype = ctypes.c_int
        lib.shape3d_vertices.argtypes = [ctypes.c_void_p, ctypes.c_int, i64p, f64p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int64, i64p, ctypes.c_void_p]
        lib.shape3d_vertices.restype = ctypes.c_int
        lib.shape3d_soft_forward.argtypes = [ctypes.c_void_p, i64p, f64p, f64p, ctypes.POINTER(SoftSaved),
                                             ctypes.c_void_p]
        lib.shape3d_soft_forward.restype = ctypes.c_int
        lib.shape3d_soft_backward.argtypes = [ctypes.c_void_p, ctypes.POINTER(SoftSaved), f64p, ctypes.c_void_p,
                                              ctypes.c_void_p]
        lib.shape3d_soft_backward.restype = ctypes.c_int
        lib.shape3d_batched.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Roi), ctypes.c_int64,
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                        ctypes.c_void_p]
        lib.shape3d_batched.restype = ctypes.c_int
        lib.shape3d_batched_ex.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Roi), ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(Stats), ctypes.c_int, ctypes.c_void_p]
        lib.shape3d_batched_ex.restype = ctypes.c_int
        lib.shape3d_class.argtypes = [ctypes.c_void_p, ctypes.c_int, i64p, f64p, f64p, ctypes.POINTER(Stats),
                                      ctypes.c_void_p]
        lib.shape3d_class.restype = ctypes.c_int
        lib.shape3d_batched_soft_forward.argtypes = [ctypes.c_void_p, ctypes.POINTER(Roi), ctypes.c_int64, f64p,
                                                     ctypes.POINTER(SoftSaved), ctypes.c_int, ctypes.c_void_p]
        lib.shape3d_batched_soft_forward.restype = ctypes.c_int
        lib.shape3d_batched_soft_backward.argtypes = [ctypes.c_void_p, ctypes.POINTER(Roi), ctypes.c_int64,
                                                      ctypes.POINTER(SoftSaved), f64p, ctypes.c_void_p,
                                                      ctypes.c_void_p]
        lib.shape3d_batched_soft_backward.restype = ctypes.c_int
        lib.shape3d_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
        lib.shape3d_get_tuning.restype = ctypes.c_int
        lib.shape3d_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
        lib.shape3d_set_tuning.restype = ctypes.c_int
        lib.shape3d_autotune.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Roi), ctypes.c_int64,
                                         ctypes.c_int, ctypes.c_char_p, ctypes.POINTER(Tuning),
                                         ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
        lib.shape3d_autotune.restype = ctypes.c_int
        sizep = ctypes.POINTER(ctypes.c_size_t)
        lib.shape3d_workspace_size.argtypes = [i64p, ctypes.c_int, sizep]
        lib.shape3d_workspace_size.restype = ctypes.c_int
        lib.shape3d_workspace_size_v.argtypes = [i64p, ctypes.c_int, ctypes.c_int64, sizep]
        lib.shape3d_workspace_size_v.restype = ctypes.c_int
        lib.shape3d_batched_workspace_size.argtypes = [ctypes.c_int64, i64p, ctypes.c_int, ctypes.c_int64, sizep]
        lib.shape3d_batched_workspace_size.restype = ctypes.c_int
        lib.shape3d_ex_async.argtypes = [ctypes.c_void_p, ctypes.c_int, i64p, f64p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        lib.shape3d_ex_async.restype = ctypes.c_int
        lib.shape3d_batched_dev.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, i64p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                            ctypes.c_int, ctypes.c_void_p]
        lib.shape3d_batched_dev.restype = ctypes.c_int
        lib.shape3d_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int, i64p, f64p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]
        lib.shape3d_noalloc.restype = ctypes.c_int
        lib.shape3d_label_rois.argtypes = [ctypes.c_void_p, i64p, f64p, ctypes.c_int32, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.shape3d_label_rois.restype = ctypes.c_int
        lib.shape3d_host_stream.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, i64p, f64p,
                                            ctypes.c_int64, f64p, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                            ctypes.c_void_p]
        lib.shape3d_host_stream.restype = ctypes.c_int
        lib.shape3d_last_error.argtypes = []
        lib.shape3d_last_error.restype = ctypes.c_char_p
        lib.shape3d_release.argtypes = []
        lib.shape3d_release.restype = ctypes.c_int
        lib.shape3d_version.argtypes = []
        lib.shape3d_version.restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(status: int, allow_empty: bool = True) -> int:
    if status < 0 or (status == EMPTY and not allow_empty):
        msg = load().shape3d_last_error().decode(errors="replace")
        raise Shape3DError(status, msg)
    return status


def _dims_spacing(shape, spacing):
    dims = (ctypes.c_int64 * 3)(*[int(x) for x in shape])
    sp = (ctypes.c_double * 3)(*[float(x) for x in spacing])
    return dims, sp


def _volume(vol):
    import torch

    if not isinstance(vol, torch.Tensor) or not vol.is_cuda:
        raise TypeError("volume must be a GPU torch tensor")
    if vol.dim() != 3:
        raise ValueError("volume must be 3-D")
    if vol.dtype == torch.uint8:
        dt = U8
    elif vol.dtype == torch.float32:
        dt = F32
    else:
        raise TypeError("volume dtype must be uint8 or float32")
    if not vol.is_contiguous():
        raise ValueError("volume must be C-contiguous")
    return dt


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def features(vol, spacing: Sequence[float] = (1.0, 1.0, 1.0), stats: bool = False, timing: bool = False):
    """The six features (float64 numpy array, order of ``FEATURES``); with
    ``stats=True`` returns ``(features, stats_dict, status)``."""
    lib = load()
    dt = _volume(vol)
    dims, sp = _dims_spacing(vol.shape, spacing)
    out = (ctypes.c_double * 6)()
    st = Stats()
    rc = lib.shape3d_ex(ctypes.c_void_p(vol.data_ptr()), dt, dims, sp, out, ctypes.byref(st), 1 if timing else 0,
                        _stream())
    _check(rc)
    f = np.array(out[:], dtype=np.float64)
    if stats:
        d = st.as_dict()
        if rc == EMPTY:
            d["pair_ids"][:] = -1
        return f, d, rc
    return f


def shape_class(vol, spacing: Sequence[float] = (1.0, 1.0, 1.0), stats: bool = False):
    """The whole Shape class (float64 numpy array [17], order of
    ``SHAPE_FEATURES``); with ``stats=True`` returns ``(features, stats_dict, status)``."""
    lib = load()
    dt = _volume(vol)
    dims, sp = _dims_spacing(vol.shape, spacing)
    out = (ctypes.c_double * N_CLASS)()
    st = Stats()
    rc = lib.shape3d_class(ctypes.c_void_p(vol.data_ptr()), dt, dims, sp, out, ctypes.byref(st), _stream())
    _check(rc)
    f = np.array(out[:], dtype=np.float64)
    if stats:
        d = st.as_dict()
        if rc == EMPTY:
            d["pair_ids"][:] = -1
        return f, d, rc
    return f


def features_dict(vol, spacing=(1.0, 1.0, 1.0)):
    return dict(zip(FEATURES, features(vol, spacing).tolist()))


def shape3d_u8(mask, spacing=(1.0, 1.0, 1.0)):
    """The plain synchronous entry point ``shape3d`` (binary mask, null stream)."""
    lib = load()
    if _volume(mask) != U8:
        raise TypeError("shape3d takes a uint8 mask")
    dims, sp = _dims_spacing(mask.shape, spacing)
    out = (ctypes.c_double * 6)()
    rc = lib.shape3d(ctypes.c_void_p(mask.data_ptr()), dims, sp, out)
    _check(rc)
    return np.array(out[:], dtype=np.float64), rc


def vertices(vol, spacing=(1.0, 1.0, 1.0), with_pos: bool = True):
    """(canonical ids int64 tensor [V], positions float64 tensor [V, 3] or None)."""
    import torch

    lib = load()
    dt = _volume(vol)
    dims, sp = _dims_spacing(vol.shape, spacing)
    n = ctypes.c_int64(0)
    rc = lib.shape3d_vertices(ctypes.c_void_p(vol.data_ptr()), dt, dims, sp, None, None, 0, ctypes.byref(n),
                              _stream())
    if rc not in (OK, EMPTY, ECAPACITY):
        _check(rc)
    V = int(n.value)
    ids = torch.empty(max(V, 1), dtype=torch.int64, device=vol.device)
    pos = torch.empty((max(V, 1), 3), dtype=torch.float64, device=vol.device) if with_pos else None
    if V > 0:
        rc = lib.shape3d_vertices(ctypes.c_void_p(vol.data_ptr()), dt, dims, sp, ctypes.c_void_p(ids.data_ptr()),
                                  ctypes.c_void_p(pos.data_ptr()) if pos is not None else None, V, ctypes.byref(n),
                                  _stream())
        _check(rc)
    return ids[:V], (pos[:V] if pos is not None else None)


def roi_table(offsets, shapes, spacings):
    """ctypes array of ROI descriptors (element offsets, (d0, d1, d2), spacing)."""
    n = len(offsets)
    tab = (Roi * n)()
    for r in range(n):
        tab[r].offset = int(offsets[r])
        for k in range(3):
            tab[r].dims[k] = int(shapes[r][k])
            tab[r].spacing[k] = float(spacings[r][k])
    return tab


def _check_extents(table, numel: int):
    """Every ROI of a dense table lies inside a base tensor of numel elements."""
    for r in range(len(table)):
        d = [int(table[r].dims[k]) for k in range(3)]
        if min(d) < 1 or int(table[r].offset) < 0 or int(table[r].offset) + d[0] * d[1] * d[2] > numel:
            raise ValueError("ROI %d (offset %d, dims %s) does not fit in a base of %d elements"
                             % (r, int(table[r].offset), d, numel))


def workspace_size(shape, dtype: int = U8, max_vertices: int = -1) -> int:
    """Bytes of a caller workspace for one ROI of this shape (see shape3d_workspace_size_v)."""
    n = ctypes.c_size_t(0)
    dims = (ctypes.c_int64 * 3)(*[int(x) for x in shape])
    _check(load().shape3d_workspace_size_v(dims, int(dtype), int(max_vertices), ctypes.byref(n)))
    return int(n.value)


def batched_workspace_size(n_rois: int, max_dims, dtype: int = U8, max_vertices: int = -1) -> int:
    n = ctypes.c_size_t(0)
    md = (ctypes.c_int64 * 3)(*[int(x) for x in max_dims])
    _check(load().shape3d_batched_workspace_size(int(n_rois), md, int(dtype), int(max_vertices), ctypes.byref(n)))
    return int(n.value)


def _workspace(ws):
    import torch

    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or not ws.is_contiguous():
        raise TypeError("workspace must be a contiguous GPU tensor")
    if ws.data_ptr() % 256:
        raise ValueError("workspace must be 256-byte aligned")
    return ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()


def features_async(vol, spacing, workspace):
    """shape3d_ex_async: (out float64 tensor [6], status int32 tensor [1]), both
    on the GPU and written on the current stream (nothing is read back)."""
    import torch

    lib = load()
    dt = _volume(vol)
    dims, sp = _dims_spacing(vol.shape, spacing)
    out = torch.zeros(6, dtype=torch.float64, device=vol.device)
    status = torch.full((1,), -100, dtype=torch.int32, device=vol.device)
    wp, wb = _workspace(workspace)
    _check(lib.shape3d_ex_async(ctypes.c_void_p(vol.data_ptr()), dt, dims, sp, ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(status.data_ptr()), wp, wb, _stream()))
    return out, status


def features_noalloc(vol, spacing, out=None, status=None):
    """shape3d_noalloc (no allocation inside the library; the caller provides
    out float64 [6] and status int32 [1] on the GPU, created here if None)."""
    import torch

    lib = load()
    dt = _volume(vol)
    dims, sp = _dims_spacing(vol.shape, spacing)
    if out is None:
        out = torch.zeros(6, dtype=torch.float64, device=vol.device)
    if status is None:
        status = torch.full((1,), -100, dtype=torch.int32, device=vol.device)
    _check(lib.shape3d_noalloc(ctypes.c_void_p(vol.data_ptr()), dt, dims, sp, ctypes.c_void_p(out.data_ptr()),
                               ctypes.c_void_p(status.data_ptr()), _stream()))
    return out, status


def roi_table_ex(offsets, shapes, spacings, strides=None, labels=None):
    """ctypes array of shape3d_roi_ex descriptors (strides 0 = dense, label 0 = nonzero)."""
    n = len(offsets)
    tab = (RoiEx * n)()
    for r in range(n):
        tab[r].offset = int(offsets[r])
        for k in range(3):
            tab[r].dims[k] = int(shapes[r][k])
            tab[r].spacing[k] = float(spacings[r][k])
        if strides is not None:
            tab[r].strides[0] = int(strides[r][0])
            tab[r].strides[1] = int(strides[r][1])
        tab[r].label = int(labels[r]) if labels is not None else 0
    return tab


def table_to_device(table, device="cuda"):
    """The bytes of a ctypes ROI table as a GPU uint8 tensor."""
    import torch

    raw = np.frombuffer(bytes(table), dtype=np.uint8).copy()
    return torch.from_numpy(raw).to(device)


def batched_dev(base, table_dev, n_rois: int, max_dims, workspace=None, graph: bool = False, out=None, status=None,
                shape_class: bool = False):
    """shape3d_batched_dev: features of n_rois ROIs described by the
    shape3d_roi_ex table held in the GPU tensor ``table_dev``; returns
    (out float64 tensor [n, 6] or [n, 17] with ``shape_class``, status int32
    tensor [n]) on the GPU."""
    import torch

    lib = load()
    if not isinstance(base, torch.Tensor) or not base.is_cuda or not base.is_contiguous():
        raise TypeError("base must be a contiguous GPU tensor")
    dt = U8 if base.dtype == torch.uint8 else (F32 if base.dtype == torch.float32 else None)
    if dt is None:
        raise TypeError("base dtype must be uint8 or float32")
    if table_dev.numel() * table_dev.element_size() < n_rois * ctypes.sizeof(RoiEx):
        raise ValueError("table_dev holds fewer than n_rois descriptors")
    nf = N_CLASS if shape_class else 6
    if out is None:
        out = torch.zeros((n_rois, nf), dtype=torch.float64, device=base.device)
    elif out.numel() < n_rois * nf or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of n_rois x %d" % nf)
    if status is None:
        status = torch.full((n_rois,), -100, dtype=torch.int32, device=base.device)
    md = (ctypes.c_int64 * 3)(*[int(x) for x in max_dims])
    wp, wb = (None, 0) if workspace is None else _workspace(workspace)
    _check(lib.shape3d_batched_dev(ctypes.c_void_p(base.data_ptr()), dt, ctypes.c_void_p(table_dev.data_ptr()),
                                   int(n_rois), md, ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(status.data_ptr()), wp, wb,
                                   (BATCH_GRAPH if graph else 0) | (SHAPE_CLASS if shape_class else 0), _stream()))
    return out, status


def host_stream(vols, spacings, shape_class: bool = False):
    """shape3d_host_stream: features of volumes held in HOST memory (numpy
    arrays or CPU torch tensors, pinned or not, all uint8 or all float32,
    C-contiguous), each copied to the GPU while the previous one is computed.
    Returns (out float64[n, 6] or [n, 17], status int32[n]) as numpy arrays."""
    import torch

    lib = load()
    n = len(vols)
    if n < 1 or len(spacings) != n:
        raise ValueError("need one spacing per volume")
    ptrs = (ctypes.c_void_p * n)()
    dims = (ctypes.c_int64 * (3 * n))()
    sp = (ctypes.c_double * (3 * n))()
    dt = None
    for i, v in enumerate(vols):
        if isinstance(v, torch.Tensor):
            if v.is_cuda or not v.is_contiguous() or v.dim() != 3:
                raise ValueError("host volumes must be 3-D contiguous CPU tensors")
            d = U8 if v.dtype == torch.uint8 else (F32 if v.dtype == torch.float32 else None)
            ptrs[i] = v.data_ptr()
        else:
            v = np.asarray(v)
            if v.ndim != 3 or not v.flags["C_CONTIGUOUS"]:
                raise ValueError("host volumes must be 3-D C-contiguous arrays")
            d = U8 if v.dtype == np.uint8 else (F32 if v.dtype == np.float32 else None)
            ptrs[i] = v.ctypes.data
        if d is None or (dt is not None and d != dt):
            raise TypeError("volumes must all be uint8 or all float32")
        dt = d
        for k in range(3):
            dims[3 * i + k] = int(v.shape[k])
            sp[3 * i + k] = float(spacings[i][k])
    nf = N_CLASS if shape_class else 6
    out = np.zeros((n, nf))
    status = np.zeros(n, dtype=np.int32)
    _check(lib.shape3d_host_stream(ptrs, dt, dims, sp, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   status.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                   SHAPE_CLASS if shape_class else 0, _stream()))
    return out, status


def label_rois(labels, spacing=(1.0, 1.0, 1.0), max_label: int = 255, counts: bool = True):
    """shape3d_label_rois: the device ROI table of labels 1..max_label of the
    C-contiguous uint8 GPU label map ``labels`` (each entry crops the map to
    the label's box and selects the label).  Returns (table uint8 GPU tensor
    of max_label descriptors, voxel counts int64 GPU tensor or None, largest
    crop dims int64 GPU tensor [3]); nothing is read back to the host."""
    import torch

    lib = load()
    if _volume(labels) != U8:
        raise TypeError("labels must be a uint8 tensor")
    dims, sp = _dims_spacing(labels.shape, spacing)
    table = torch.empty(int(max_label) * ctypes.sizeof(RoiEx), dtype=torch.uint8, device=labels.device)
    cnt = torch.empty(int(max_label), dtype=torch.int64, device=labels.device) if counts else None
    maxd = torch.empty(3, dtype=torch.int64, device=labels.device)
    _check(lib.shape3d_label_rois(ctypes.c_void_p(labels.data_ptr()), dims, sp, int(max_label),
                                  ctypes.c_void_p(table.data_ptr()),
                                  ctypes.c_void_p(cnt.data_ptr()) if cnt is not None else None,
                                  ctypes.c_void_p(maxd.data_ptr()), _stream()))
    return table, cnt, maxd


def label_features(labels, spacing=(1.0, 1.0, 1.0), max_label: int = 255, shape_class: bool = False,
                   graph: bool = False):
    """Features of every label 1..max_label of a GPU label map, each in its
    own bounding box: shape3d_label_rois, then shape3d_batched_dev on the
    map.  The batch is sized by the largest crop, read back once; the
    features and statuses stay on the GPU (out [max_label, 6 or 17], status
    [max_label]; a label with no voxel has status EMPTY)."""
    table, _, maxd = label_rois(labels, spacing, max_label, counts=False)
    md = [int(x) for x in maxd.cpu().tolist()]
    base = labels.view(-1)
    return batched_dev(base, table, int(max_label), md, graph=graph, shape_class=shape_class)


def batched(base, table, graph: bool = False, stats: bool = False, shape_class: bool = False):
    """Features of a batch of ROIs packed in the 1-D GPU tensor ``base``
    (uint8 or float32); ``table`` from ``roi_table``.  Returns
    (features float64[n, 6], status int32[n]), with ``shape_class`` the whole
    Shape class (float64[n, 17]), and with ``stats`` also a list of per-ROI
    statistics dicts (V, T, pair_ids, ...)."""
    import torch

    lib = load()
    if not isinstance(base, torch.Tensor) or not base.is_cuda or not base.is_contiguous():
        raise TypeError("base must be a contiguous GPU tensor")
    if base.dtype == torch.uint8:
        dt = U8
    elif base.dtype == torch.float32:
        dt = F32
    else:
        raise TypeError("base dtype must be uint8 or float32")
    n = len(table)
    _check_extents(table, base.numel())
    out = np.zeros((n, N_CLASS if shape_class else 6), dtype=np.float64)
    status = np.zeros(n, dtype=np.int32)
    flags = (BATCH_GRAPH if graph else 0) | (SHAPE_CLASS if shape_class else 0)
    if not stats and not shape_class:
        rc = lib.shape3d_batched(ctypes.c_void_p(base.data_ptr()), dt, table, n,
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 status.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), flags, _stream())
        _check(rc)
        return out, status
    st = (Stats * n)() if stats else None
    rc = lib.shape3d_batched_ex(ctypes.c_void_p(base.data_ptr()), dt, table, n,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                status.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), st, flags, _stream())
    _check(rc)
    if not stats:
        return out, status
    dicts = []
    for r in range(n):
        d = st[r].as_dict()
        if status[r] == EMPTY:
            d["pair_ids"][:] = -1
        dicts.append(d)
    return out, status, dicts


def soft_forward(p, spacing=(1.0, 1.0, 1.0)):
    """Features of a float32 soft mask and the context its backward pass needs."""
    lib = load()
    if _volume(p) != F32:
        raise TypeError("soft masks are float32")
    dims, sp = _dims_spacing(p.shape, spacing)
    out = (ctypes.c_double * 6)()
    saved = SoftSaved()
    _check(lib.shape3d_soft_forward(ctypes.c_void_p(p.data_ptr()), dims, sp, out, ctypes.byref(saved), _stream()))
    return np.array(out[:], dtype=np.float64), saved


def soft_backward(p, saved: SoftSaved, grad_out):
    """dL/dp (float32 tensor like p) for L = sum_f grad_out[f] * F_f."""
    import torch

    lib = load()
    if _volume(p) != F32:
        raise TypeError("soft masks are float32")
    g = (ctypes.c_double * 6)(*[float(x) for x in np.asarray(grad_out, dtype=np.float64).reshape(6)])
    grad = torch.empty_like(p)
    _check(lib.shape3d_soft_backward(ctypes.c_void_p(p.data_ptr()), ctypes.byref(saved), g,
                                     ctypes.c_void_p(grad.data_ptr()), _stream()))
    return grad


def _uncovered(table, numel: int):
    """The element ranges [a, b) of a packed buffer of numel elements that no
    ROI of the table covers."""
    spans = sorted((int(r.offset), int(r.offset) + int(r.dims[0]) * int(r.dims[1]) * int(r.dims[2])) for r in table)
    out, pos = [], 0
    for a, b in spans:
        if a > pos:
            out.append((pos, min(a, numel)))
        pos = max(pos, b)
    if pos < numel:
        out.append((pos, numel))
    return [(a, b) for a, b in out if b > a]


def _soft_base(base):
    import torch

    if not isinstance(base, torch.Tensor) or not base.is_cuda or not base.is_contiguous():
        raise TypeError("base must be a contiguous GPU tensor")
    if base.dtype != torch.float32:
        raise TypeError("soft masks are float32")


def batched_soft_forward(base, table, graph: bool = False):
    """Features of a batch of float32 soft masks packed in ``base`` and the
    per-ROI contexts of the backward pass: (features float64[n, 6], saved)."""
    lib = load()
    _soft_base(base)
    n = len(table)
    out = np.zeros((n, 6), dtype=np.float64)
    saved = (SoftSaved * n)()
    _check(lib.shape3d_batched_soft_forward(ctypes.c_void_p(base.data_ptr()), table, n,
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), saved,
                                            BATCH_GRAPH if graph else 0, _stream()))
    return out, saved


def batched_soft_backward(base, table, saved, grad_out, grad=None):
    """dL/dbase (float32 tensor like base; 0 outside the ROIs unless ``grad``
    is given) for L = sum_r sum_f grad_out[r, f] * F_f(ROI r)."""
    import torch

    lib = load()
    _soft_base(base)
    n = len(table)
    g = np.ascontiguousarray(np.asarray(grad_out, dtype=np.float64).reshape(n, 6))
    if grad is None:
        # every element of every ROI is written by the call: only the elements
        # outside all ROIs need their zeros
        grad = torch.empty_like(base)
        for a, b in _uncovered(table, base.numel()):
            grad[a:b].zero_()
    _check(lib.shape3d_batched_soft_backward(ctypes.c_void_p(base.data_ptr()), table, n, saved,
                                             g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             ctypes.c_void_p(grad.data_ptr()), _stream()))
    return grad


def _autograd_function():
    import torch

    class Shape3DFunction(torch.autograd.Function):
        """features = Shape3DFunction.apply(p, spacing): float64 tensor [6] on p's
        device; differentiable with respect to the float32 soft mask p."""

        @staticmethod
        def forward(ctx, p, spacing):
            p = p.contiguous()
            feats, saved = soft_forward(p, spacing)
            ctx.save_for_backward(p)
            ctx.saved = saved
            return torch.tensor(feats, dtype=torch.float64, device=p.device)

        @staticmethod
        def backward(ctx, grad_out):
            (p,) = ctx.saved_tensors
            g = grad_out.detach().to("cpu", torch.float64).numpy()
            return soft_backward(p, ctx.saved, g), None

    return Shape3DFunction


def _batched_autograd_function():
    import torch

    class BatchedShape3DFunction(torch.autograd.Function):
        """features = BatchedShape3DFunction.apply(base, table, graph): float64
        tensor [n, 6]; differentiable with respect to the packed float32 soft
        masks ``base``."""

        @staticmethod
        def forward(ctx, base, table, graph):
            feats, saved = batched_soft_forward(base, table, graph)
            ctx.save_for_backward(base)
            ctx.table = table
            ctx.saved = saved
            return torch.from_numpy(feats).to(base.device)

        @staticmethod
        def backward(ctx, grad_out):
            (base,) = ctx.saved_tensors
            g = grad_out.detach().to("cpu", torch.float64).numpy()
            return batched_soft_backward(base, ctx.table, ctx.saved, g), None, None

    return BatchedShape3DFunction


_FN = None
_BFN = None


def batched_shape_features(base, table, graph: bool = False):
    """Differentiable features [n, 6] of packed float32 soft masks (see
    BatchedShape3DFunction)."""
    global _BFN
    if _BFN is None:
        _BFN = _batched_autograd_function()
    return _BFN.apply(base, table, graph)


def shape_features(p, spacing=(1.0, 1.0, 1.0)):
    """Differentiable features of a soft mask (see Shape3DFunction)."""
    global _FN
    if _FN is None:
        _FN = _autograd_function()
    return _FN.apply(p, tuple(float(x) for x in spacing))


def get_tuning():
    """Current pair-pass setting (itile_blocks, jchunk_blocks, blocks_per_cu, kernel)."""
    t = Tuning()
    _check(load().shape3d_get_tuning(ctypes.byref(t)))
    return t.as_tuple()


def get_prune() -> int:
    """3D pruning mode: 0 never, 1 for large ROIs (default), 2 always."""
    t = Tuning()
    _check(load().shape3d_get_tuning(ctypes.byref(t)))
    return int(t.prune)


def set_tuning(itile_blocks: int, jchunk_blocks: int, blocks_per_cu: int = 0, kernel: int = 0, prune=None):
    """Replace the pair-pass setting; ``prune`` None keeps the current choice."""
    t = Tuning()
    _check(load().shape3d_get_tuning(ctypes.byref(t)))
    t = Tuning(int(itile_blocks), int(jchunk_blocks), int(blocks_per_cu), int(kernel),
               int(t.prune if prune is None else prune), int(t.small_path))
    _check(load().shape3d_set_tuning(ctypes.byref(t)))


def set_prune(mode: int):
    """3D pruning mode: 0 never, 1 for large ROIs (default), 2 always."""
    t = Tuning()
    _check(load().shape3d_get_tuning(ctypes.byref(t)))
    t.prune = int(mode)
    _check(load().shape3d_set_tuning(ctypes.byref(t)))


def get_small_path() -> bool:
    """Whether small single ROIs take the exact all-pairs kernel (default True)."""
    t = Tuning()
    _check(load().shape3d_get_tuning(ctypes.byref(t)))
    return bool(t.small_path)


def set_small_path(on: bool):
    """Switch the small single-ROI path on or off (results are identical)."""
    t = Tuning()
    _check(load().shape3d_get_tuning(ctypes.byref(t)))
    t.small_path = 1 if on else 0
    _check(load().shape3d_set_tuning(ctypes.byref(t)))


def autotune(base, table, reps: int = 2, cache_path=None):
    """Choose the pair-pass setting for this batch (see shape3d_autotune):
    returns ((itile, jchunk, blocks_per_cu, kernel), pair-pass ms)."""
    import torch

    lib = load()
    if not isinstance(base, torch.Tensor) or not base.is_cuda or not base.is_contiguous():
        raise TypeError("base must be a contiguous GPU tensor")
    dt = U8 if base.dtype == torch.uint8 else (F32 if base.dtype == torch.float32 else None)
    if dt is None:
        raise TypeError("base dtype must be uint8 or float32")
    t = Tuning()
    ms = ctypes.c_double(0.0)
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(lib.shape3d_autotune(ctypes.c_void_p(base.data_ptr()), dt, table, len(table), int(reps), path,
                                ctypes.byref(t), ctypes.byref(ms), _stream()))
    return t.as_tuple(), float(ms.value)


def release():
    return load().shape3d_release()


def version() -> int:
    return load().shape3d_version()
