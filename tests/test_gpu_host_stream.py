"""GPU tests of shape3d_host_stream: volumes that start in host memory, each
copied to the device while the previous one is computed.

Bar: every volume's features and status are bit-identical to the same
volume's shape3d_ex call on a device copy (which the parity tests hold to the
oracle), and the small volumes also meet the oracle bar directly (area and
volume relative 1e-9, diameters equal).  Cases: pageable numpy volumes of
mixed sizes (ragged, empty, larger than one 32 MiB staging chunk), pinned
torch volumes, float32 soft masks, the Shape class, one volume, and argument
errors.
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


@pytest.fixture(scope="module")
def S():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_02894_amd import shape3d

    shape3d.load()
    return shape3d


def on_device(S, vols, sps, shape_class=False):
    import torch

    outs, sts = [], []
    for v, sp in zip(vols, sps):
        t = torch.from_numpy(np.ascontiguousarray(np.asarray(v))).cuda()
        if shape_class:
            f, st, rc = S.shape_class(t, sp, stats=True)
        else:
            f, st, rc = S.features(t, sp, stats=True)
        outs.append(f)
        sts.append(rc)
    return np.array(outs), np.array(sts)


def small_volumes(seed, n, dtype=np.uint8):
    g = np.random.default_rng(seed)
    vols, sps = [], []
    for i in range(n):
        shape = tuple(int(x) for x in g.integers(3, 48, size=3))
        if dtype == np.uint8:
            v = synth.random_mask(shape, float(g.uniform(0.05, 0.6)), g)
        else:
            v = synth.soft_roi(shape, g, 3, 2.0, 10.0, 1.0)
        vols.append(np.ascontiguousarray(v))
        sps.append(tuple(float(x) for x in g.uniform(0.5, 1.5, size=3)))
    return vols, sps


def test_pageable_mixed_sizes(S):
    vols, sps = small_volumes(1, 9)
    vols.insert(3, np.zeros((5, 6, 7), np.uint8))  # empty
    sps.insert(3, (1.0, 1.0, 1.0))
    mask, sp = synth.large_roi(0)  # 78.6 MB: three staging chunks
    vols.insert(6, mask)
    sps.insert(6, sp)
    say("host stream: %d pageable volumes" % len(vols))
    out, status = S.host_stream(vols, sps)
    ref, rst = on_device(S, vols, sps)
    np.testing.assert_array_equal(status, rst)
    np.testing.assert_array_equal(out, ref)
    assert status[3] == S.EMPTY
    for i, (v, s) in enumerate(zip(vols, sps)):
        if v.size > 200000:
            continue
        r = O.shape3d(v, s)
        assert status[i] == r["status"], i
        np.testing.assert_allclose(out[i, :2], r["features"][:2], rtol=1e-9, atol=0)
        np.testing.assert_array_equal(out[i, 2:], r["features"][2:])


def test_pinned_and_soft(S):
    import torch

    vols, sps = small_volumes(2, 6, np.float32)
    pinned = [torch.from_numpy(v).pin_memory() for v in vols]
    say("host stream: pinned float32 volumes")
    out, status = S.host_stream(pinned, sps)
    ref, rst = on_device(S, vols, sps)
    np.testing.assert_array_equal(status, rst)
    np.testing.assert_array_equal(out, ref)
    say("host stream: the same volumes pageable")
    out2, status2 = S.host_stream(vols, sps)
    np.testing.assert_array_equal(out2, out)
    np.testing.assert_array_equal(status2, status)


def test_shape_class_and_single(S):
    vols, sps = small_volumes(3, 5)
    say("host stream: Shape class")
    out, status = S.host_stream(vols, sps, shape_class=True)
    ref, rst = on_device(S, vols, sps, shape_class=True)
    np.testing.assert_array_equal(status, rst)
    np.testing.assert_array_equal(out, ref)
    say("host stream: one volume")
    out1, st1 = S.host_stream(vols[:1], sps[:1])
    np.testing.assert_array_equal(out1[0], out[0, :6])


def test_errors(S):
    vols, sps = small_volumes(4, 2)
    with pytest.raises(TypeError):
        S.host_stream([vols[0], vols[1].astype(np.float32)], sps)
    with pytest.raises(ValueError):
        S.host_stream(vols, sps[:1])
    with pytest.raises(S.Shape3DError):
        S.host_stream(vols, [sps[0], (1.0, -1.0, 1.0)])
