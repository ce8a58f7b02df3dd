"""Seeded synthetic inputs (region-of-interest masks and soft masks).

This module only draws random shapes; it holds none of the shape-feature
arithmetic.  Tests, the benchmark and the oracle checks all take their inputs
from here, so the GPU path and the oracle always see the same arrays.

Shapes are built in index space (voxel centres at integer coordinates, axis 0
slowest).  Every generator takes an explicit ``numpy.random.Generator``; use
``rng(config, roi)`` for the fixed workload seeds.

The paper measured on kidney-tumour CT segmentations; these generators are
synthetic stand-ins with the same size range (tens of kilobytes to tens of
megabytes of mask, a few thousand to about a million mesh vertices).
"""
from __future__ import annotations

import numpy as np


def rng(config: int, roi: int = 0) -> np.random.Generator:
    """Generator for workload ``config`` and region ``roi``."""
    return np.random.default_rng(np.random.SeedSequence([2510, 2894, int(config), int(roi)]))


def _rotation(g: np.random.Generator) -> np.ndarray:
    """Uniformly random rotation matrix (QR of a Gaussian matrix, sign-fixed)."""
    q, r = np.linalg.qr(g.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def ellipsoid_params(g: np.random.Generator, n: int, semi_lo, semi_hi, centre_lo, centre_hi):
    """n ellipsoids: (centre[3], semi-axes[3], rotation[3,3]) each."""
    out = []
    for _ in range(n):
        semi = g.uniform(semi_lo, semi_hi, size=3)
        centre = g.uniform(centre_lo, centre_hi, size=3)
        out.append((centre, semi, _rotation(g)))
    return out


def _ellipsoid_field(shape, centre, semi, rot, margin=0.0):
    """Bounding-box slices and the normalised radius sum((R^T (x - c) / a)^2) on them."""
    reach = float(np.max(semi)) + margin + 1.0
    lo = [max(0, int(np.floor(centre[k] - reach))) for k in range(3)]
    hi = [min(shape[k], int(np.ceil(centre[k] + reach)) + 1) for k in range(3)]
    if any(h <= l for l, h in zip(lo, hi)):
        return None, None
    zz, yy, xx = np.meshgrid(*[np.arange(lo[k], hi[k], dtype=np.float64) - centre[k] for k in range(3)],
                             indexing="ij")
    pts = np.stack([zz, yy, xx], axis=-1)
    q = pts @ rot  # rows are (x - c)^T R  ->  R^T (x - c)
    rr = np.sum((q / semi) ** 2, axis=-1)
    sl = tuple(slice(lo[k], hi[k]) for k in range(3))
    return sl, rr


def ellipsoid_union(shape, params) -> np.ndarray:
    """Boolean union of ellipsoids evaluated at voxel centres."""
    out = np.zeros(shape, dtype=bool)
    for centre, semi, rot in params:
        sl, rr = _ellipsoid_field(shape, centre, semi, rot)
        if sl is not None:
            out[sl] |= rr <= 1.0
    return out


def random_mask(shape, density: float, g: np.random.Generator) -> np.ndarray:
    """I.i.d. Bernoulli mask (uint8 0/1)."""
    return (g.random(shape) < density).astype(np.uint8)


def box_mask(shape, lo, size) -> np.ndarray:
    m = np.zeros(shape, dtype=np.uint8)
    m[lo[0]:lo[0] + size[0], lo[1]:lo[1] + size[1], lo[2]:lo[2] + size[2]] = 1
    return m


def single_roi(seed: int = 0, shape=(64, 64, 64)):
    """One ellipsoid, semi-axes U[8, 24] voxels, random orientation, centre U[24, 40]^3.

    Returns (uint8 mask, spacing) with spacing (1, 1, 1) mm.
    """
    g = rng(1, seed)
    params = ellipsoid_params(g, 1, 8.0, 24.0, 24.0, 40.0)
    return ellipsoid_union(shape, params).astype(np.uint8), (1.0, 1.0, 1.0)


def large_roi(seed: int = 0, shape=(300, 512, 512), n_ellipsoids: int = 20, sigma: float = 3.0):
    """Union of 20 ellipsoids (semi-axes U[20, 90] voxels, centres uniform over
    the array), Gaussian-smoothed indicator (sigma 3) thresholded at 0.5.

    The array is (300, 512, 512) in (axis0, axis1, axis2) order, i.e. 300 slices
    of 512 x 512; spacing (1.25, 0.7, 0.7) mm in the same order.
    """
    from scipy.ndimage import gaussian_filter

    g = rng(2, seed)
    params = ellipsoid_params(g, n_ellipsoids, 20.0, 90.0, 0.0, 1.0)
    params = [(c * np.asarray(shape, dtype=np.float64), s, r) for c, s, r in params]
    ind = ellipsoid_union(shape, params).astype(np.float32)
    sm = gaussian_filter(ind, sigma=sigma, mode="constant", truncate=4.0)
    return (sm > 0.5).astype(np.uint8), (1.25, 0.7, 0.7)


def signed_distance(inside: np.ndarray, spacing=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Signed distance (negative inside) between voxel centres and the boundary,
    from two Euclidean distance transforms, shifted by half a voxel."""
    from scipy.ndimage import distance_transform_edt

    out_d = distance_transform_edt(~inside, sampling=spacing)
    in_d = distance_transform_edt(inside, sampling=spacing)
    return np.where(inside, -(in_d - 0.5), out_d - 0.5)


def soft_roi(shape, g: np.random.Generator, n_ellipsoids: int = 8, semi_lo: float = 16.0,
             semi_hi: float = 64.0, tau: float = 1.0) -> np.ndarray:
    """float32 probability mask p = sigmoid(-sd / tau) of an ellipsoid union."""
    shape = tuple(int(s) for s in shape)
    lo = np.minimum(np.asarray(shape) * 0.25, np.asarray(shape) / 2.0)
    hi = np.asarray(shape) - lo
    params = ellipsoid_params(g, n_ellipsoids, semi_lo, semi_hi, lo, hi)
    inside = ellipsoid_union(shape, params)
    sd = signed_distance(inside)
    return (1.0 / (1.0 + np.exp(sd / tau))).astype(np.float32)


def soft_batch_params(n: int, seed: int = 0, lmin: float = 48.0, lmax: float = 160.0):
    """Per-ROI parameters of the batched soft workload: cubic edge L log-uniform
    in [lmin, lmax], tau U[0.5, 2] voxels, 8 ellipsoids with semi-axes
    U[L/16, L/4] and centres uniform in the middle half of the box (the 256^3
    differentiable workload scaled to L)."""
    out = []
    for r in range(n):
        g = rng(5, seed * 1000003 + r)
        L = int(round(float(np.exp(g.uniform(np.log(lmin), np.log(lmax))))))
        tau = float(g.uniform(0.5, 2.0))
        out.append((L, tau, int(g.integers(0, 2 ** 63 - 1))))
    return out


def _soft_batch_member(args):
    L, tau, sub = args
    g = np.random.default_rng(sub)
    return soft_roi((L, L, L), g, 8, L / 16.0, L / 4.0, tau)


SOFT_BATCH_SPACING = (2.0, 0.8, 0.8)


def soft_batch(n: int, seed: int = 0, lmin: float = 48.0, lmax: float = 160.0, workers: int = 1):
    """Packed float32 soft masks of the batched soft workload: (buffer,
    offsets, shapes, spacings); spacing (2.0, 0.8, 0.8) mm in array order for
    every ROI.  ``workers`` > 1 generates in a process pool."""
    params = soft_batch_params(n, seed, lmin, lmax)
    if workers > 1:
        import multiprocessing as mp

        with mp.get_context("fork").Pool(workers) as pool:
            vols = pool.map(_soft_batch_member, params, chunksize=1)
    else:
        vols = [_soft_batch_member(p) for p in params]
    sizes = [v.size for v in vols]
    offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    buf = np.concatenate([v.reshape(-1) for v in vols]).astype(np.float32)
    return buf, offsets, [v.shape for v in vols], [SOFT_BATCH_SPACING] * n


def differentiable_roi(seed: int = 0, shape=(256, 256, 256)):
    """Soft mask of an 8-ellipsoid union, semi-axes U[16, 64], tau = 1 voxel; spacing (1, 1, 1)."""
    return soft_roi(shape, rng(4, seed), 8, 16.0, 64.0, 1.0), (1.0, 1.0, 1.0)


def differentiable_small(seed: int = 0, shape=(32, 32, 32)):
    """Small instance of the differentiable workload (semi-axes U[3, 8])."""
    return soft_roi(shape, rng(4, 1000 + seed), 8, 3.0, 8.0, 1.0), (1.0, 1.0, 1.0)


def batched_params(n: int, seed: int = 0, lmin: float = 8.0, lmax: float = 128.0):
    """Per-ROI parameters of the batched workload: edge L log-uniform in
    [lmin, lmax], per-axis aspect log-uniform in [0.5, 2] (dims clipped to
    [4, 256]), spacing U[0.5, 1.5] mm per axis, 1-6 ellipsoids with centres
    uniform in the box and semi-axes U[0.15, 0.45] times the box."""
    out = []
    for r in range(n):
        g = rng(3, seed * 1000003 + r)
        L = float(np.exp(g.uniform(np.log(lmin), np.log(lmax))))
        aspect = np.exp(g.uniform(np.log(0.5), np.log(2.0), size=3))
        dims = tuple(int(np.clip(round(L * a), 4, 256)) for a in aspect)
        spacing = tuple(float(x) for x in g.uniform(0.5, 1.5, size=3))
        k = int(g.integers(1, 7))
        ell = []
        for _ in range(k):
            centre = g.uniform(0.0, 1.0, size=3) * (np.asarray(dims) - 1)
            semi = g.uniform(0.15, 0.45, size=3) * np.asarray(dims)
            ell.append((centre, semi, _rotation(g)))
        out.append((dims, spacing, ell))
    return out


def batched_rois(n: int, seed: int = 0, lmin: float = 8.0, lmax: float = 128.0):
    """Packed uint8 masks of the batched workload: (buffer, offsets, shapes,
    spacings), ROI r occupying buffer[offsets[r]:offsets[r] + prod(shapes[r])]."""
    params = batched_params(n, seed, lmin, lmax)
    sizes = [int(np.prod(d)) for d, _, _ in params]
    offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    buf = np.zeros(int(sum(sizes)), dtype=np.uint8)
    for (dims, _, ell), off, sz in zip(params, offsets, sizes):
        buf[off:off + sz] = ellipsoid_union(dims, ell).reshape(-1)
    return buf, offsets, [p[0] for p in params], [p[1] for p in params]


def batched_rois_torch(n: int, seed: int = 0, lmin: float = 8.0, lmax: float = 128.0, device="cuda:0"):
    """As batched_rois, evaluated with torch on ``device`` (the parameters are
    the same draws; the packed buffer is a uint8 tensor on the device)."""
    import torch

    params = batched_params(n, seed, lmin, lmax)
    sizes = [int(np.prod(d)) for d, _, _ in params]
    offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    buf = torch.zeros(int(sum(sizes)), dtype=torch.uint8, device=device)
    for (dims, _, ell), off, sz in zip(params, offsets, sizes):
        view = buf[int(off):int(off) + sz].view(dims)
        for centre, semi, rot in ell:
            reach = float(np.max(semi)) + 1.0
            lo = [max(0, int(np.floor(centre[k] - reach))) for k in range(3)]
            hi = [min(dims[k], int(np.ceil(centre[k] + reach)) + 1) for k in range(3)]
            if any(h <= l for l, h in zip(lo, hi)):
                continue
            axes = [torch.arange(lo[k], hi[k], dtype=torch.float64, device=device) - float(centre[k])
                    for k in range(3)]
            zz, yy, xx = torch.meshgrid(*axes, indexing="ij")
            pts = torch.stack([zz, yy, xx], dim=-1)
            q = pts @ torch.as_tensor(rot, dtype=torch.float64, device=device)
            rr = torch.sum((q / torch.as_tensor(semi, dtype=torch.float64, device=device)) ** 2, dim=-1)
            sub = view[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
            sub |= (rr <= 1.0).to(torch.uint8)
    return buf, offsets, [p[0] for p in params], [p[1] for p in params]


def label_map(seed: int = 0, shape=(96, 128, 128), n_labels: int = 6, semi_lo: float = 3.0, semi_hi: float = 24.0,
              noise: float = 0.0):
    """A uint8 label map: label l = 1..n_labels painted as one rotated
    ellipsoid each (later labels over earlier ones), semi-axes U[semi_lo,
    semi_hi] voxels, centres uniform over the array (so some touch the
    border), plus i.i.d. voxels of random labels 1..n_labels with probability
    ``noise`` (stray voxels stretch a label's box).  A stand-in for organ and
    tumour label maps (labels 1 and 2 in the paper's kidney data)."""
    g = rng(6, seed)
    lab = np.zeros(shape, dtype=np.uint8)
    params = ellipsoid_params(g, n_labels, semi_lo, semi_hi, 0.0, 1.0)
    for l, (c, s, r) in enumerate(params, start=1):
        c = c * np.asarray(shape, dtype=np.float64)
        sl, rr = _ellipsoid_field(shape, c, s, r)
        if sl is not None:
            lab[sl][rr <= 1.0] = l
    if noise > 0.0:
        hit = g.random(shape) < noise
        lab[hit] = g.integers(1, n_labels + 1, size=int(hit.sum()), dtype=np.uint8)
    return lab
