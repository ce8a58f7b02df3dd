"""GPU parity of the batched entry point: every ROI of a packed batch against
the oracle, against the single-ROI entry point, and through hipGraph replay."""
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


def pack(masks, align_pad):
    """Packs masks back to back with `align_pad` filler elements before each."""
    offs, parts, pos = [], [], 0
    for m in masks:
        pos += align_pad
        parts.append(np.zeros(align_pad, dtype=m.dtype))
        offs.append(pos)
        parts.append(m.reshape(-1))
        pos += m.size
    return np.concatenate(parts), offs


def check_batch(S, masks, spacings, name, align_pad=0, graph=False):
    import torch

    buf, offs = pack(masks, align_pad)
    table = S.roi_table(offs, [m.shape for m in masks], spacings)
    say("%s: %d ROIs, pad %d, graph %s" % (name, len(masks), align_pad, graph))
    out, status = S.batched(torch.from_numpy(buf).cuda(), table, graph=graph)
    for r, (m, sp) in enumerate(zip(masks, spacings)):
        ref = O.shape3d(m, sp)
        assert status[r] == ref["status"], (name, r)
        np.testing.assert_allclose(out[r, :2], ref["features"][:2], rtol=1e-9, atol=0, err_msg="%s %d" % (name, r))
        np.testing.assert_array_equal(out[r, 2:], ref["features"][2:], err_msg="%s %d" % (name, r))
    return out, status, buf, table


def test_batch_small_rois(S):
    buf, offs, shapes, sps = synth.batched_rois(48, seed=1, lmin=4, lmax=28)
    masks = [buf[o:o + int(np.prod(s))].reshape(s) for o, s in zip(offs, shapes)]
    check_batch(S, masks, sps, "small ROIs")


def test_batch_unaligned_offsets_and_empty(S):
    g = np.random.default_rng(3)
    masks, sps = [], []
    for i in range(20):
        shape = tuple(int(x) for x in g.integers(1, 40, size=3))
        m = synth.random_mask(shape, float(g.uniform(0.05, 0.9)), g)
        if i % 7 == 3:
            m[:] = 0  # empty ROI
        masks.append(m)
        sps.append(tuple(float(x) for x in g.uniform(0.5, 1.5, size=3)))
    check_batch(S, masks, sps, "unaligned", align_pad=3)


def test_batch_soft(S):
    masks, sps = [], []
    for i in range(6):
        p, _ = synth.differentiable_small(i, shape=(12 + i, 20, 17 + 3 * i))
        masks.append(p)
        sps.append((1.0, 0.8 + 0.1 * i, 1.2))
    check_batch(S, masks, sps, "soft", align_pad=1)


def test_batch_matches_single_roi_calls(S):
    import torch

    buf, offs, shapes, sps = synth.batched_rois(24, seed=2, lmin=6, lmax=40)
    table = S.roi_table(offs, shapes, sps)
    say("batched vs single calls")
    out, status = S.batched(torch.from_numpy(buf).cuda(), table)
    for r in range(len(offs)):
        m = buf[offs[r]:offs[r] + int(np.prod(shapes[r]))].reshape(shapes[r])
        f = S.features(torch.from_numpy(m).cuda(), sps[r])
        np.testing.assert_array_equal(out[r], f)


def test_graph_replay_and_capacity_fallback(S):
    import torch

    S.release()  # fresh workspace: the first call sizes the buffers
    g = np.random.default_rng(5)
    shapes = [(20, 24, 30), (16, 16, 16), (30, 10, 12)]
    sps = [(1.0, 0.9, 1.1), (0.7, 0.7, 1.3), (1.2, 1.0, 0.8)]
    sparse = [synth.box_mask(s, (2, 2, 2), (4, 4, 4)) for s in shapes]
    buf, offs = pack(sparse, 0)
    table = S.roi_table(offs, shapes, sps)
    dev = torch.from_numpy(buf).cuda()
    say("graph capture")
    a, _ = S.batched(dev, table, graph=True)
    say("graph replay")
    b, _ = S.batched(dev, table, graph=True)
    np.testing.assert_array_equal(a, b)
    # same layout, far more vertices than the recorded buffers hold
    dense = [synth.random_mask(s, 0.5, g) for s in shapes]
    dev.copy_(torch.from_numpy(pack(dense, 0)[0]).cuda())
    say("graph replay on larger meshes")
    c, st = S.batched(dev, table, graph=True)
    for r, (m, sp) in enumerate(zip(dense, sps)):
        ref = O.shape3d(m, sp)
        np.testing.assert_allclose(c[r, :2], ref["features"][:2], rtol=1e-9)
        np.testing.assert_array_equal(c[r, 2:], ref["features"][2:])
    say("graph replay after re-recording")
    d, _ = S.batched(dev, table, graph=True)
    np.testing.assert_array_equal(c, d)
