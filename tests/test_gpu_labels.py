"""GPU parity of the label preprocessing (shape3d_label_rois) and of the
features of every label computed from its table (shape3d_batched_dev).

Bar: the table (offset, dims, spacing, strides, label), the voxel counts and
the largest crop are bit-exact against the oracle's label_rois; the features
of each label's crop meet the single-ROI bar against the oracle run on the
oracle's crop (area and volume relative 1e-9, diameters and their pairs
equal).  Cases: ragged map sizes (not multiples of 16 bytes), maps whose
first byte is not 16-byte aligned, tiny maps, labels above max_label
(ignored), absent labels (1-voxel crop, status EMPTY), stray voxels that
stretch a box, labels touching the map's border, and a full-size
300 x 512 x 512 map.
"""
import ctypes
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


def dev_map(lab, shift=0):
    """The label map on the GPU, starting `shift` bytes into its allocation."""
    import torch

    n = lab.size
    raw = torch.zeros(n + shift + 64, dtype=torch.uint8, device="cuda")
    raw[shift:shift + n] = torch.from_numpy(lab.reshape(-1)).cuda()
    return raw[shift:shift + n].view(lab.shape)


def table_entries(S, table, n):
    raw = table.cpu().numpy().tobytes()
    return (S.RoiEx * n).from_buffer_copy(raw[:n * ctypes.sizeof(S.RoiEx)])


def check_table(S, lab, max_label, sp, shift=0):
    t = dev_map(lab, shift)
    table, cnt, maxd = S.label_rois(t, sp, max_label)
    ents = table_entries(S, table, max_label)
    ref = O.label_rois(lab, max_label, sp)
    cnt = cnt.cpu().numpy()
    md = np.ones(3, np.int64)
    for i, e in enumerate(ref):
        g = ents[i]
        name = "label %d" % e["label"]
        assert g.label == e["label"] and g.reserved == 0, name
        assert g.offset == e["offset"], name
        assert list(g.dims) == [int(v) for v in e["dims"]], name
        assert tuple(g.spacing) == e["spacing"], name
        assert tuple(g.strides) == e["strides"], name
        assert cnt[i] == e["count"], name
        if e["count"]:
            md = np.maximum(md, e["dims"])
    np.testing.assert_array_equal(maxd.cpu().numpy(), md)
    return t, table, ref


def check_features(S, t, table, ref, shape_class=False):
    import torch

    max_label = len(ref)
    md = [int(x) for x in np.max([e["dims"] for e in ref], axis=0)]
    out, status = S.batched_dev(t.view(-1), table, max_label, md, shape_class=shape_class)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    status = status.cpu().numpy()
    for i, e in enumerate(ref):
        name = "label %d" % e["label"]
        if e["count"] == 0:
            assert status[i] == S.EMPTY, name
            np.testing.assert_array_equal(out[i], 0.0, err_msg=name)
            continue
        m = O.crop(t.cpu().numpy(), e)
        r = O.shape_class(m, e["spacing"]) if shape_class else O.shape3d(m, e["spacing"])
        assert status[i] == r["status"], name
        f = r["features"]
        np.testing.assert_allclose(out[i, :2], f[:2], rtol=1e-9, atol=0, err_msg=name)
        np.testing.assert_array_equal(out[i, 2:6], f[2:6], err_msg=name)
        if shape_class:
            np.testing.assert_allclose(out[i, 6:12], f[6:12], rtol=1e-9, atol=0, err_msg=name)
            major = max(abs(f[12]), abs(out[i, 12]))
            np.testing.assert_allclose(out[i, 12:15], f[12:15], rtol=1e-9, atol=1e-6 * major, err_msg=name)
            np.testing.assert_allclose(out[i, 15:17], f[15:17], rtol=1e-9, atol=1e-6, err_msg=name)


@pytest.mark.parametrize("shift", [0, 3, 13])
def test_label_table_ragged_and_misaligned(S, shift):
    g = np.random.default_rng(40 + shift)
    for trial in range(3):
        shape = tuple(int(x) for x in g.integers(5, 70, size=3))
        lab = synth.label_map(10 * shift + trial, shape=shape, n_labels=6, semi_lo=2.0, semi_hi=20.0, noise=2e-4)
        lab[g.random(shape) < 1e-3] = 250  # above max_label: ignored
        say("label table shape=%s shift=%d" % (shape, shift))
        t, table, ref = check_table(S, lab, 8, (1.0, 0.8, 1.3), shift)
        check_features(S, t, table, ref)


def test_tiny_maps(S):
    g = np.random.default_rng(7)
    for shape in [(1, 1, 1), (1, 1, 17), (2, 3, 5), (3, 1, 33), (4, 4, 4)]:
        lab = g.integers(0, 4, size=shape).astype(np.uint8)
        say("tiny label map %s" % (shape,))
        for shift in (0, 7):
            t, table, ref = check_table(S, lab, 3, (0.5, 1.0, 2.0), shift)
            check_features(S, t, table, ref)


def test_runs_across_rows(S):
    """Rows narrower than a 16-byte chunk, and full chunks of one label that
    cross a row boundary (no single-run shortcut may be taken there)."""
    lab = np.zeros((6, 7, 9), np.uint8)
    lab[1:5, 2:6, :] = 2
    lab[2, 3, 4] = 1
    lab[5, 6, 8] = 1
    say("runs across rows")
    t, table, ref = check_table(S, lab, 2, (1.0, 1.0, 1.0), 0)
    check_features(S, t, table, ref)
    lab = np.full((3, 2, 20), 5, np.uint8)
    lab[0, 0, :3] = 0
    t, table, ref = check_table(S, lab, 5, (1.0, 1.0, 1.0), 5)
    check_features(S, t, table, ref)


def test_label_shape_class_and_binding(S):
    import torch

    lab = synth.label_map(3, shape=(64, 90, 110), n_labels=5)
    say("label_features shape class")
    t = dev_map(lab)
    out, status = S.label_features(t, (1.25, 0.7, 0.7), 6, shape_class=True)
    table, _, _ = S.label_rois(t, (1.25, 0.7, 0.7), 6)
    ref = O.label_rois(lab, 6, (1.25, 0.7, 0.7))
    out2, status2 = S.batched_dev(t.view(-1), table, 6, lab.shape, shape_class=True)
    torch.cuda.synchronize()
    # sizing the batch by the map's dims instead of the largest crop changes nothing
    np.testing.assert_array_equal(out.cpu().numpy(), out2.cpu().numpy())
    np.testing.assert_array_equal(status.cpu().numpy(), status2.cpu().numpy())
    check_features(S, t, table, ref, shape_class=True)


def test_errors(S):
    import torch

    lab = torch.zeros((4, 4, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(S.Shape3DError):
        S.label_rois(lab, (1, 1, 1), 0)
    with pytest.raises(S.Shape3DError):
        S.label_rois(lab, (1, 1, 1), 256)
    with pytest.raises(TypeError):
        S.label_rois(lab.float(), (1, 1, 1), 3)


def test_label_table_full_size(S):
    lab = synth.label_map(9, shape=(300, 512, 512), n_labels=12, semi_lo=10.0, semi_hi=90.0, noise=1e-7)
    say("label table 300x512x512")
    t, table, ref = check_table(S, lab, 16, (1.25, 0.7, 0.7), 0)
    say("label features: the smaller labels")
    small = [e for e in ref if 0 < e["count"] < 200000]
    assert small
    import torch

    md = [int(x) for x in np.max([e["dims"] for e in ref], axis=0)]
    out, status = S.batched_dev(t.view(-1), table, len(ref), md)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    for e in small:
        i = e["label"] - 1
        r = O.shape3d(O.crop(lab, e), e["spacing"])
        np.testing.assert_allclose(out[i, :2], r["features"][:2], rtol=1e-9, atol=0)
        np.testing.assert_array_equal(out[i, 2:6], r["features"][2:6])
