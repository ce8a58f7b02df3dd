"""GPU parity of the small-plane-bucket kernel.  A batch with more than 2^16
plane buckets sends the buckets of at most 16 blocks of 32 rows to their own
kernel under the split-f16 pair pass; the FP32 pass and single-ROI calls keep
every bucket in the work list.  All of them must give identical features and
pairs, and a sample of ROIs must match the oracle."""
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
    yield shape3d
    shape3d.set_tuning(8, 1024, 0, 1)


def test_small_bucket_kernel_matches_work_list(S):
    import torch

    say("small buckets: generate 400 ROIs")
    buf, offs, shapes, sps = synth.batched_rois_torch(400, 11, lmin=40.0, lmax=64.0)
    # plane buckets of the batch: 2 d_k + 1 per axis and ROI
    n_buckets = sum(2 * (d[0] + d[1] + d[2]) + 3 for d in shapes)
    assert n_buckets >= 1 << 16
    table = S.roi_table(offs, shapes, sps)
    ref = None
    for it, jc, kern in [(8, 512, 1), (4, 64, 1), (8, 128, 0), (4, 256, 0)]:
        say("small buckets: tiling %d x %d kernel %d" % (it, jc, kern))
        S.set_tuning(it, jc, 0, kern)
        out, status = S.batched(buf, table)
        assert np.all(status == 0)
        if ref is None:
            ref = out
        assert np.array_equal(out, ref), (it, jc, kern)
    S.set_tuning(8, 1024, 0, 1)
    out, _ = S.batched(buf, table, graph=True)
    assert np.array_equal(out, ref)
    host = buf.cpu().numpy()
    sizes = [int(np.prod(s)) for s in shapes]
    for r in (0, 57, 199, 398):
        say("small buckets: single-ROI call on ROI %d %s" % (r, shapes[r]))
        f = S.features(buf[int(offs[r]):int(offs[r]) + sizes[r]].view(shapes[r]), sps[r])
        assert np.array_equal(f, ref[r]), r
    for r in (3, 250):
        say("small buckets: oracle on ROI %d %s" % (r, shapes[r]))
        m = host[int(offs[r]):int(offs[r]) + sizes[r]].reshape(shapes[r])
        exp = O.shape3d(m, sps[r])["features"]
        np.testing.assert_allclose(ref[r][:2], exp[:2], rtol=1e-9)
        np.testing.assert_allclose(ref[r][2:], exp[2:], rtol=1e-6)
