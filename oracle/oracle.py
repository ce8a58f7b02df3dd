"""Python access to the CPU FP64 oracle (``shape3d_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check in
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``.  The product
library never imports this module.  It builds ``liboracle.so`` with gcc when it
is missing (``build()`` also rebuilds it on request).

Every function takes numpy arrays on the host.  The volume is C-contiguous with
shape (d0, d1, d2); ``spacing`` is in the same axis order.  ``uint8`` volumes
are binary masks (nonzero = inside); ``float32`` volumes are soft masks
(inside iff p > 0.5, vertices interpolated at the 0.5 level).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "shape3d_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EMPTY, EINVAL, ECAPACITY, ENOMEM, EINTERNAL = 0, 1, -1, -4, -5, -6
FEATURES = (
    "MeshVolume",
    "SurfaceArea",
    "Maximum3DDiameter",
    "Maximum2DDiameterSlice",
    "Maximum2DDiameterColumn",
    "Maximum2DDiameterRow",
)

# The whole Shape class: the six features above, then the members that are
# closed forms of the mesh volume V, surface area A and inside-voxel count,
# and the principal-axis members (eigenvalues of the inside voxels'
# coordinate covariance).
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

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = [
            "gcc", "-O2", "-std=c11", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
            "-fPIC", "-shared", "-o", tmp, _SRC, "-lm",
        ]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        f64p = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        lib.oracle_count_vertices.argtypes = [vp, ctypes.c_int, i64p, f64p, i64p]
        lib.oracle_vertices.argtypes = [vp, ctypes.c_int, i64p, f64p, ctypes.c_int64, i64p, f64p, f64p, i64p]
        lib.oracle_mesh.argtypes = [vp, ctypes.c_int, i64p, f64p, f64p, f64p, f64p, i64p, ctypes.c_int64, i64p]
        lib.oracle_diameters.argtypes = [i64p, f64p, ctypes.c_int64, i64p, f64p, i64p]
        lib.oracle_diameters_which.argtypes = [i64p, f64p, ctypes.c_int64, i64p, ctypes.c_int, f64p, i64p]
        lib.oracle_shape3d.argtypes = [vp, ctypes.c_int, i64p, f64p, f64p, i64p, i64p, f64p]
        lib.oracle_soft_grad.argtypes = [vp, i64p, f64p, f64p, i64p, f64p]
        lib.oracle_cube_triangles.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        lib.oracle_moments.argtypes = [vp, ctypes.c_int, i64p, f64p, i64p, f64p, f64p]
        lib.oracle_max_pair_rows.argtypes = [f64p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, f64p,
                                             ctypes.POINTER(ctypes.c_int)]
        _lib = lib
    return _lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _vol(vol: np.ndarray):
    vol = np.ascontiguousarray(vol)
    if vol.ndim != 3:
        raise ValueError("volume must be 3-D")
    if vol.dtype == np.uint8:
        return vol, 0
    if vol.dtype == np.float32:
        return vol, 1
    raise TypeError("volume must be uint8 or float32")


def _dims_sp(vol: np.ndarray, spacing):
    dims = np.array(vol.shape, dtype=np.int64)
    sp = np.ascontiguousarray(np.asarray(spacing, dtype=np.float64).reshape(3))
    return dims, sp


def _check(st: int, what: str):
    if st not in (OK, EMPTY):
        raise RuntimeError("oracle %s failed with status %d" % (what, st))


def count_vertices(vol: np.ndarray, spacing=(1.0, 1.0, 1.0)) -> int:
    lib = _load()
    vol, dt = _vol(vol)
    dims, sp = _dims_sp(vol, spacing)
    n = np.zeros(1, dtype=np.int64)
    _check(lib.oracle_count_vertices(vol.ctypes.data, dt, _p(dims, ctypes.c_int64), _p(sp, ctypes.c_double),
                                     _p(n, ctypes.c_int64)), "count_vertices")
    return int(n[0])


def vertices(vol: np.ndarray, spacing=(1.0, 1.0, 1.0)):
    """(ids int64[V] ascending, pos float64[V,3], t float64[V])."""
    lib = _load()
    vol, dt = _vol(vol)
    dims, sp = _dims_sp(vol, spacing)
    n = count_vertices(vol, spacing)
    ids = np.zeros(max(n, 1), dtype=np.int64)
    pos = np.zeros((max(n, 1), 3), dtype=np.float64)
    t = np.zeros(max(n, 1), dtype=np.float64)
    n2 = np.zeros(1, dtype=np.int64)
    _check(lib.oracle_vertices(vol.ctypes.data, dt, _p(dims, ctypes.c_int64), _p(sp, ctypes.c_double), n,
                               _p(ids, ctypes.c_int64), _p(pos, ctypes.c_double), _p(t, ctypes.c_double),
                               _p(n2, ctypes.c_int64)), "vertices")
    return ids[:n], pos[:n], t[:n]


def mesh(vol: np.ndarray, spacing=(1.0, 1.0, 1.0), origin=None, triangles: bool = False):
    """(area, signed_volume, n_triangles, tri_ids int64[T,3] or None)."""
    lib = _load()
    vol, dt = _vol(vol)
    dims, sp = _dims_sp(vol, spacing)
    if origin is None:
        origin = 0.5 * dims.astype(np.float64) * sp
    org = np.ascontiguousarray(np.asarray(origin, dtype=np.float64).reshape(3))
    area = np.zeros(1)
    sv = np.zeros(1)
    nt = np.zeros(1, dtype=np.int64)
    null = ctypes.POINTER(ctypes.c_int64)()
    _check(lib.oracle_mesh(vol.ctypes.data, dt, _p(dims, ctypes.c_int64), _p(sp, ctypes.c_double),
                           _p(org, ctypes.c_double), _p(area, ctypes.c_double), _p(sv, ctypes.c_double),
                           _p(nt, ctypes.c_int64), 0, null), "mesh")
    tris = None
    if triangles:
        T = int(nt[0])
        tris = np.zeros((max(T, 1), 3), dtype=np.int64)
        _check(lib.oracle_mesh(vol.ctypes.data, dt, _p(dims, ctypes.c_int64), _p(sp, ctypes.c_double),
                               _p(org, ctypes.c_double), _p(area, ctypes.c_double), _p(sv, ctypes.c_double),
                               _p(nt, ctypes.c_int64), T, _p(tris, ctypes.c_int64)), "mesh")
        tris = tris[:T]
    return float(area[0]), float(sv[0]), int(nt[0]), tris


def diameters(ids: np.ndarray, pos: np.ndarray, dims, which: int = 15):
    """(d2[4] = squared {3D, slice, column, row}, pair_idx int64[4,2] into the vertex list).

    ``which`` selects features by bit (bit 0: 3D, bit 1 + k: planes of axis k)."""
    lib = _load()
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    dims = np.ascontiguousarray(np.asarray(dims, dtype=np.int64).reshape(3))
    d2 = np.zeros(4)
    pidx = np.zeros(8, dtype=np.int64)
    _check(lib.oracle_diameters_which(_p(ids, ctypes.c_int64), _p(pos, ctypes.c_double), len(ids),
                                      _p(dims, ctypes.c_int64), int(which), _p(d2, ctypes.c_double),
                                      _p(pidx, ctypes.c_int64)), "diameters")
    return d2, pidx.reshape(4, 2)


def shape3d(vol: np.ndarray, spacing=(1.0, 1.0, 1.0)):
    """dict(features=float64[6], status, V, T, pair_ids=int64[4,2], signed_volume)."""
    lib = _load()
    vol, dt = _vol(vol)
    dims, sp = _dims_sp(vol, spacing)
    out = np.zeros(6)
    counts = np.zeros(2, dtype=np.int64)
    pairs = np.zeros(8, dtype=np.int64)
    sv = np.zeros(1)
    st = lib.oracle_shape3d(vol.ctypes.data, dt, _p(dims, ctypes.c_int64), _p(sp, ctypes.c_double),
                            _p(out, ctypes.c_double), _p(counts, ctypes.c_int64), _p(pairs, ctypes.c_int64),
                            _p(sv, ctypes.c_double))
    _check(st, "shape3d")
    return dict(features=out, status=int(st), V=int(counts[0]), T=int(counts[1]),
                pair_ids=pairs.reshape(4, 2), signed_volume=float(sv[0]))


def moments(vol: np.ndarray, spacing=(1.0, 1.0, 1.0)):
    """(inside-voxel count, mean float64[3], population covariance float64[3,3]) of
    the physical coordinates index * spacing of the voxels inside the region."""
    lib = _load()
    vol, dt = _vol(vol)
    dims, sp = _dims_sp(vol, spacing)
    n = np.zeros(1, dtype=np.int64)
    mean = np.zeros(3)
    cov = np.zeros(9)
    _check(lib.oracle_moments(vol.ctypes.data, dt, _p(dims, ctypes.c_int64), _p(sp, ctypes.c_double),
                              _p(n, ctypes.c_int64), _p(mean, ctypes.c_double), _p(cov, ctypes.c_double)),
           "moments")
    return int(n[0]), mean, cov.reshape(3, 3)


def shape_class(vol: np.ndarray, spacing=(1.0, 1.0, 1.0), base=None):
    """dict(features=float64[17] in the order of SHAPE_FEATURES, eigenvalues
    float64[3] ascending, n_inside, status, and the entries of ``shape3d``).

    The extra members are the Shape class's definitions, written out:
      VoxelVolume            = n_inside * s0 * s1 * s2
      SurfaceVolumeRatio     = A / V
      Sphericity             = (36 pi V^2)^(1/3) / A
      Compactness1           = V / (sqrt(pi) * A^(3/2))
      Compactness2           = 36 pi V^2 / A^3
      SphericalDisproportion = A / (36 pi V^2)^(1/3)
      Major/Minor/LeastAxisLength = 4 sqrt(lambda), lambda the largest, middle
                               and smallest eigenvalue of the covariance
      Elongation             = sqrt(lambda_minor / lambda_major)
      Flatness               = sqrt(lambda_least / lambda_major)
    with V = MeshVolume and A = SurfaceArea.  Readings: an empty region gives
    all zeros; negative eigenvalues (rounding of a singular covariance) count
    as 0; Elongation and Flatness are 0 when lambda_major is 0 (one voxel).
    ``base`` may pass an earlier ``shape3d`` result for the same input."""
    r = dict(base) if base is not None else shape3d(vol, spacing)
    n, _, cov = moments(vol, spacing)
    f = np.zeros(len(SHAPE_FEATURES))
    f[:6] = r["features"]
    lam = np.zeros(3)
    if r["status"] == OK:
        sp = np.asarray(spacing, dtype=np.float64).reshape(3)
        V, A = f[0], f[1]
        lam = np.maximum(np.linalg.eigvalsh(cov), 0.0)  # ascending
        f[6] = n * sp[0] * sp[1] * sp[2]
        f[7] = A / V
        f[8] = (36.0 * np.pi * V * V) ** (1.0 / 3.0) / A
        f[9] = V / (np.sqrt(np.pi) * A ** 1.5)
        f[10] = 36.0 * np.pi * V * V / A ** 3
        f[11] = A / (36.0 * np.pi * V * V) ** (1.0 / 3.0)
        f[12], f[13], f[14] = 4.0 * np.sqrt(lam[2]), 4.0 * np.sqrt(lam[1]), 4.0 * np.sqrt(lam[0])
        f[15] = np.sqrt(lam[1] / lam[2]) if lam[2] > 0 else 0.0
        f[16] = np.sqrt(lam[0] / lam[2]) if lam[2] > 0 else 0.0
    r.update(features=f, eigenvalues=lam, n_inside=n, covariance=cov)
    return r


def soft_grad(p: np.ndarray, spacing, grad_out, pair_ids: Optional[np.ndarray] = None) -> np.ndarray:
    """dL/dp (float64, shape of p) for L = sum_f grad_out[f] * F_f."""
    lib = _load()
    p = np.ascontiguousarray(p, dtype=np.float32)
    dims, sp = _dims_sp(p, spacing)
    g = np.ascontiguousarray(np.asarray(grad_out, dtype=np.float64).reshape(6))
    out = np.zeros(p.shape, dtype=np.float64)
    pp = ctypes.POINTER(ctypes.c_int64)()
    if pair_ids is not None:
        pair_ids = np.ascontiguousarray(np.asarray(pair_ids, dtype=np.int64).reshape(8))
        pp = _p(pair_ids, ctypes.c_int64)
    _check(lib.oracle_soft_grad(p.ctypes.data, _p(dims, ctypes.c_int64), _p(sp, ctypes.c_double),
                                _p(g, ctypes.c_double), pp, _p(out, ctypes.c_double)), "soft_grad")
    return out


def cube_triangles(case: int):
    """Triangles (cube-edge triples) the oracle traces for one of the 256 cases."""
    lib = _load()
    buf = (ctypes.c_int * 48)()
    n = ctypes.c_int(0)
    _check(lib.oracle_cube_triangles(int(case), buf, ctypes.byref(n)), "cube_triangles")
    return [tuple(buf[3 * i:3 * i + 3]) for i in range(n.value)]


def max_pair_rows(pos: np.ndarray, i0: int, i1: int):
    """(max squared distance over i in [i0, i1), j > i; OpenMP threads used)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    best = np.zeros(1)
    th = ctypes.c_int(0)
    _check(lib.oracle_max_pair_rows(_p(pos, ctypes.c_double), len(pos), int(i0), int(i1),
                                    _p(best, ctypes.c_double), ctypes.byref(th)), "max_pair_rows")
    return float(best[0]), th.value


def decode_ids(ids: np.ndarray, dims):
    """Canonical ids -> (u int64[V,3] edge start voxel, a int64[V] edge axis)."""
    d = np.asarray(dims, dtype=np.int64)
    ids = np.asarray(ids, dtype=np.int64)
    a = ids % 3
    lin = ids // 3
    u2 = lin % (d[2] + 2) - 1
    lin = lin // (d[2] + 2)
    u1 = lin % (d[1] + 2) - 1
    u0 = lin // (d[1] + 2) - 1
    return np.stack([u0, u1, u2], axis=1), a


def label_rois(labels: np.ndarray, max_label: int, spacing=(1.0, 1.0, 1.0)):
    """Input preprocessing of a uint8 label map (the paper's open problem of
    staging inputs, Sec. 3 discussion; Table 2 transfer column), by its plain
    definition: for each label l in 1..max_label, the smallest box holding
    every voxel equal to l, that box's first voxel as a flat offset into the
    map, and the number of such voxels.

    Returns a list of dicts {label, count, lo (3,), dims (3,), offset,
    strides (2,), spacing}; a label with no voxel gets count 0, a 1x1x1 box at
    the origin and offset 0.  ``crop(labels, entry)`` gives the entry's mask.
    """
    lab = np.ascontiguousarray(labels)
    if lab.dtype != np.uint8 or lab.ndim != 3:
        raise ValueError("labels must be a 3-D uint8 array")
    d = lab.shape
    out = []
    for l in range(1, int(max_label) + 1):
        idx = np.nonzero(lab == l)
        n = int(idx[0].size)
        if n == 0:
            lo = np.zeros(3, np.int64)
            dims = np.ones(3, np.int64)
        else:
            lo = np.array([int(a.min()) for a in idx], np.int64)
            hi = np.array([int(a.max()) for a in idx], np.int64)
            dims = hi - lo + 1
        out.append(dict(label=l, count=n, lo=lo, dims=dims,
                        offset=int(lo[0] * d[1] * d[2] + lo[1] * d[2] + lo[2]),
                        strides=(d[1] * d[2], d[2]), spacing=tuple(float(s) for s in spacing)))
    return out


def crop(labels: np.ndarray, entry) -> np.ndarray:
    """The binary mask (uint8) of ``entry``'s label inside ``entry``'s box."""
    lo, dims = entry["lo"], entry["dims"]
    sub = labels[lo[0]:lo[0] + dims[0], lo[1]:lo[1] + dims[1], lo[2]:lo[2] + dims[2]]
    return (sub == entry["label"]).astype(np.uint8)
