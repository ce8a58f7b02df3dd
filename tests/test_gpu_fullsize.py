"""Parity at the benchmark's full size (large ROI, 300 x 512 x 512 uint8), in the
launch configuration bench.py times.

The oracle finishes the vertex set, the mesh and the in-plane diameters at
this size; for the 3D diameter it would need 5e11 pair evaluations, so the
check uses a property that holds at any size: the farthest pair of a point set
is a pair of vertices of its convex hull, so the exact maximum over the hull
vertices of the oracle's positions is the exact diameter.
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


def hull_diameter2(pos):
    from scipy.spatial import ConvexHull

    hv = np.unique(ConvexHull(pos).vertices)
    P = pos[hv]
    best = 0.0
    for s in range(0, len(P), 2048):
        d = P[s:s + 2048, None, :] - P[None, :, :]
        best = max(best, float(np.max(np.sum(d * d, axis=-1))))
    return best, len(hv)


def test_large_roi_full_size():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_02894_amd import shape3d as S

    say("large ROI: generate")
    mask, sp = synth.large_roi(0)
    vol = torch.from_numpy(mask).cuda()
    say("large ROI: GPU features")
    f, st, rc = S.features(vol, sp, stats=True, timing=True)
    say("large ROI: GPU vertices")
    gid, gpos = S.vertices(vol, sp)
    gid = gid.cpu().numpy()
    gpos = gpos.cpu().numpy()
    say("large ROI: oracle vertices and mesh")
    ids, pos, _ = O.vertices(mask, sp)
    assert st["V"] == len(ids)
    o = np.argsort(gid)
    np.testing.assert_array_equal(gid[o], ids)
    np.testing.assert_array_equal(gpos[o], pos)
    area, sv, nt, _ = O.mesh(mask, sp)
    assert st["T"] == nt
    assert f[0] == pytest.approx(abs(sv), rel=1e-9)
    assert f[1] == pytest.approx(area, rel=1e-9)
    say("large ROI: oracle in-plane diameters")
    d2, pidx = O.diameters(ids, pos, mask.shape, which=14)
    np.testing.assert_array_equal(f[3:], np.sqrt(d2[1:]))
    np.testing.assert_array_equal(st["pair_ids"][1:], ids[pidx[1:]])
    say("large ROI: 3D diameter via the convex hull")
    best, nh = hull_diameter2(pos)
    assert f[2] == pytest.approx(np.sqrt(best), rel=1e-12)
    # the reported pair realises the diameter exactly
    i, j = st["pair_ids"][0]
    pi, pj = pos[np.searchsorted(ids, i)], pos[np.searchsorted(ids, j)]
    dd = pi - pj
    assert np.sqrt((dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]) == f[2]
