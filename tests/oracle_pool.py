"""The oracle on many ROIs at once, in worker processes (test infrastructure).

The full-size batched parity tests compare every ROI of a batch with the
oracle.  The ROIs are independent, so a pool of spawned workers (one oracle
thread each) runs them side by side.  The packed volumes reach the workers as
a read-only memory map of a file the caller writes; no worker touches the GPU.

Per ROI, a worker returns the vertex count, the triangle count, area and
signed volume, the three in-plane diameters with their canonical id pairs,
and the 3D diameter with its pair: from the oracle's all-pairs maximum when
the ROI has at most `brute_max` vertices, else from the extreme points of the
oracle's vertex set (brute.hull_max_pair), which is exact at any size.
Optionally it also returns the oracle's FP64 soft gradient for given pairs.
"""
import os

import numpy as np


def _init():
    os.environ["OMP_NUM_THREADS"] = "1"


def roi_job(job):
    """job: dict(path, dtype, offset, shape, spacing, brute_max, grad_out, pair_ids)."""
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from oracle import oracle as O
    from tests import brute

    dt = np.dtype(job["dtype"])
    n = int(np.prod(job["shape"]))
    mm = np.memmap(job["path"], dtype=dt, mode="r")
    vol = np.array(mm[job["offset"]:job["offset"] + n]).reshape(job["shape"])
    del mm
    sp = job["spacing"]
    ids, pos, _ = O.vertices(vol, sp)
    area, sv, nt, _ = O.mesh(vol, sp)
    r = dict(V=len(ids), T=nt, area=area, signed_volume=sv)
    if len(ids) == 0:
        r.update(d2=np.zeros(4), pair_ids=-np.ones((4, 2), dtype=np.int64), method3d="empty")
        return r
    d2, pidx = O.diameters(ids, pos, vol.shape, which=14)
    pair_ids = np.where(pidx >= 0, ids[np.maximum(pidx, 0)], -1)
    if len(ids) <= job["brute_max"]:
        d3, p3 = O.diameters(ids, pos, vol.shape, which=1)
        d2[0] = d3[0]
        pair_ids[0] = ids[p3[0]] if p3[0, 0] >= 0 else (-1, -1)
        r["method3d"] = "oracle all pairs"
    else:
        m, pr = brute.hull_max_pair(ids, pos)
        d2[0] = m
        pair_ids[0] = pr
        r["method3d"] = "extreme points"
    r.update(d2=d2, pair_ids=np.sort(pair_ids, axis=1))
    if job.get("grad_out") is not None:
        r["grad"] = O.soft_grad(vol, sp, job["grad_out"], pair_ids=job["pair_ids"])
    return r


def run(host: np.ndarray, offsets, shapes, spacings, brute_max: int = 20000, workers: int = 16, grad=None,
        tmpdir=None):
    """Oracle results for every ROI of a packed host buffer.  grad: optional
    {roi: (grad_out[6], pair_ids[4, 2])} for which the soft gradient is also
    returned."""
    import multiprocessing as mp
    import tempfile

    d = tempfile.mkdtemp(dir=tmpdir)
    path = os.path.join(d, "rois.bin")
    try:
        np.ascontiguousarray(host).tofile(path)
        jobs = []
        for r in range(len(offsets)):
            g = (grad or {}).get(r)
            jobs.append(dict(path=path, dtype=host.dtype.str, offset=int(offsets[r]),
                             shape=tuple(int(x) for x in shapes[r]), spacing=tuple(float(x) for x in spacings[r]),
                             brute_max=int(brute_max), grad_out=None if g is None else np.asarray(g[0], float),
                             pair_ids=None if g is None else np.asarray(g[1], np.int64)))
        # largest first, so that the pool's tail is short
        order = sorted(range(len(jobs)), key=lambda r: -int(np.prod(jobs[r]["shape"])))
        with mp.get_context("spawn").Pool(max(1, workers), initializer=_init) as pool:
            res = pool.map(roi_job, [jobs[r] for r in order], chunksize=1)
        out = [None] * len(jobs)
        for r, x in zip(order, res):
            out[r] = x
        return out
    finally:
        try:
            os.remove(path)
        except OSError:
            pass
        os.rmdir(d)
