"""Brute-force helpers for pinning the oracle on small inputs.

These recompute the vertex set and the diameters straight from their
definitions with numpy, independently of the C oracle: a vertex for every pair
of 6-neighbour voxels (with the one-voxel zero pad) whose inside test differs,
and maxima over all vertex pairs.
"""
import numpy as np


def inside(vol):
    return (vol != 0) if vol.dtype == np.uint8 else (vol > np.float32(0.5))


def vertex_set(vol, spacing):
    """ids (ascending) and positions from neighbour label changes (np.diff)."""
    ins = np.pad(inside(vol), 1)
    pval = np.pad(vol.astype(np.float64), 1) if vol.dtype == np.float32 else None
    d = np.array(vol.shape, dtype=np.int64)
    recs = []
    for a in range(3):
        ch = np.diff(ins.astype(np.int8), axis=a) != 0
        idx = np.argwhere(ch)  # padded coordinates of the lower end point
        u = idx - 1            # array coordinates, in [-1, d-1] along a
        if pval is not None:
            hi = idx.copy()
            hi[:, a] += 1
            pa = pval[tuple(idx.T)]
            pb = pval[tuple(hi.T)]
            t = (0.5 - pa) / (pb - pa)
        else:
            t = np.full(len(u), 0.5)
        lin = ((u[:, 0] + 1) * (d[1] + 2) + (u[:, 1] + 1)) * (d[2] + 2) + (u[:, 2] + 1)
        ids = 3 * lin + a
        pos = u.astype(np.float64)
        pos[:, a] += t
        pos = pos * np.asarray(spacing, dtype=np.float64)
        key = 2 * u
        key[:, a] += 1
        recs.append((ids, pos, key))
    ids = np.concatenate([r[0] for r in recs])
    pos = np.concatenate([r[1] for r in recs])
    key = np.concatenate([r[2] for r in recs])
    o = np.argsort(ids, kind="stable")
    return ids[o], pos[o], key[o]


def max_d2(pos, groups=None):
    """Maximum squared pairwise distance (over pairs in the same group if given)."""
    if len(pos) < 2:
        return 0.0
    diff = pos[:, None, :] - pos[None, :, :]
    d2 = np.sum(diff * diff, axis=-1)
    if groups is not None:
        d2 = np.where(groups[:, None] == groups[None, :], d2, -1.0)
    np.fill_diagonal(d2, -1.0)
    return max(float(d2.max()), 0.0)


def diameters(vol, spacing):
    """(3D, slice, column, row) maximum distances by brute force."""
    ids, pos, key = vertex_set(vol, spacing)
    out = [np.sqrt(max_d2(pos))]
    for k in range(3):
        out.append(np.sqrt(max_d2(pos, key[:, k])))
    return np.array(out), len(ids)


def max_pair(ids, pos, groups=None):
    """(max d2, (id_lo, id_hi)): the largest squared distance over vertex pairs
    (in the same group if given) and, among the pairs that reach it exactly,
    the lexicographically smallest pair of canonical ids; (0.0, (-1, -1)) when
    no pair exists.  Squared distances are evaluated as (dx*dx + dy*dy) + dz*dz
    in FP64, so equal distances compare equal."""
    ids = np.asarray(ids, dtype=np.int64)
    pos = np.asarray(pos, dtype=np.float64)
    n = len(ids)
    if n < 2:
        return 0.0, (-1, -1)
    dx = pos[:, None, 0] - pos[None, :, 0]
    dy = pos[:, None, 1] - pos[None, :, 1]
    dz = pos[:, None, 2] - pos[None, :, 2]
    d2 = (dx * dx + dy * dy) + dz * dz
    valid = ~np.eye(n, dtype=bool)
    if groups is not None:
        groups = np.asarray(groups)
        valid &= groups[:, None] == groups[None, :]
    if not valid.any():
        return 0.0, (-1, -1)
    m = float(d2[valid].max())
    ii, jj = np.nonzero(valid & (d2 == m))
    lo = np.minimum(ids[ii], ids[jj])
    hi = np.maximum(ids[ii], ids[jj])
    k = np.lexsort((hi, lo))[0]
    return m, (int(lo[k]), int(hi[k]))


def max_pairs(vol, spacing):
    """[(d2, (id_lo, id_hi))] for the 3D, slice, column and row diameters."""
    ids, pos, key = vertex_set(vol, spacing)
    out = [max_pair(ids, pos)]
    for k in range(3):
        out.append(max_pair(ids, pos, key[:, k]))
    return out


def max_pair_chunked(ids, pos, chunk=1024):
    """As max_pair (no groups), in row chunks so that large point sets fit in
    memory: (max d2, (id_lo, id_hi)) with the lexicographically smallest pair
    of canonical ids among the pairs at the maximum."""
    ids = np.asarray(ids, dtype=np.int64)
    pos = np.asarray(pos, dtype=np.float64)
    n = len(ids)
    if n < 2:
        return 0.0, (-1, -1)
    best = -1.0
    pair = (-1, -1)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        dx = pos[s:e, None, 0] - pos[None, :, 0]
        dy = pos[s:e, None, 1] - pos[None, :, 1]
        dz = pos[s:e, None, 2] - pos[None, :, 2]
        d2 = (dx * dx + dy * dy) + dz * dz
        d2[np.arange(e - s), np.arange(s, e)] = -1.0
        m = float(d2.max())
        if m < best:
            continue
        ii, jj = np.nonzero(d2 == m)
        lo = np.minimum(ids[s + ii], ids[jj])
        hi = np.maximum(ids[s + ii], ids[jj])
        k = np.lexsort((hi, lo))[0]
        cand = (int(lo[k]), int(hi[k]))
        if m > best or cand < pair:
            best, pair = m, cand
    return best, pair


def hull_max_pair(ids, pos):
    """The exact maximum squared distance and its smallest-id pair, searched
    over the extreme points only: a farthest pair of a point set consists of
    two extreme points of its convex hull (|x - q|^2 is strictly convex along
    a segment, so a point that is a proper convex combination of others is
    strictly closer to q than one of them).  Candidates are qhull's vertices
    together with the points it reports as coplanar with a facet, so that an
    extreme point that the hull merged into a facet within rounding is kept."""
    from scipy.spatial import ConvexHull

    h = ConvexHull(pos)
    cand = [h.vertices]
    if len(h.coplanar):
        cand.append(h.coplanar[:, 0])
    c = np.unique(np.concatenate(cand))
    return max_pair_chunked(np.asarray(ids)[c], np.asarray(pos)[c])
