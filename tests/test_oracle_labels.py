"""Pins of the oracle's label preprocessing (oracle.label_rois / crop): the
bounding box and voxel count of each label of a uint8 label map, and the flat
offset of the box's first voxel.

* planted boxes: disjoint solid boxes with known corners and sizes give
  exactly those boxes and counts (the product of the sizes);
* brute force: on tiny maps, pure-Python loops over every voxel;
* properties on random label maps: the crop holds every voxel of its label
  (count equality), each of its six faces holds at least one (minimality),
  and the flat offset addresses the box's first voxel.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_02894_amd import synth


def brute_boxes(lab, max_label):
    d0, d1, d2 = lab.shape
    res = {}
    for z, y, x in itertools.product(range(d0), range(d1), range(d2)):
        l = int(lab[z, y, x])
        if l == 0 or l > max_label:
            continue
        if l not in res:
            res[l] = [[z, y, x], [z, y, x], 0]
        lo, hi, _ = res[l]
        for k, v in enumerate((z, y, x)):
            lo[k] = min(lo[k], v)
            hi[k] = max(hi[k], v)
        res[l][2] += 1
    return res


def test_planted_boxes():
    g = np.random.default_rng(5)
    for trial in range(6):
        shape = tuple(int(x) for x in g.integers(8, 40, size=3))
        lab = np.zeros(shape, np.uint8)
        # disjoint boxes: one slab of axis 0 each
        n = int(g.integers(1, 5))
        cuts = np.sort(g.choice(np.arange(1, shape[0]), size=min(n, shape[0] - 1), replace=False))
        edges = [0] + list(cuts) + [shape[0]]
        labels = g.choice(np.arange(1, 256), size=len(edges) - 1, replace=False)
        want = {}
        for i, l in enumerate(labels):
            z0, z1 = edges[i], edges[i + 1]
            lo = [int(z0), int(g.integers(0, shape[1])), int(g.integers(0, shape[2]))]
            size = [int(g.integers(1, z1 - z0 + 1)), int(g.integers(1, shape[1] - lo[1] + 1)),
                     int(g.integers(1, shape[2] - lo[2] + 1))]
            lo[0] = int(g.integers(z0, z1 - size[0] + 1))
            lab[lo[0]:lo[0] + size[0], lo[1]:lo[1] + size[1], lo[2]:lo[2] + size[2]] = l
            want[int(l)] = (lo, size)
        ents = O.label_rois(lab, 255, (1.0, 2.0, 3.0))
        assert len(ents) == 255
        for e in ents:
            l = e["label"]
            if l in want:
                lo, size = want[l]
                assert list(e["lo"]) == lo and list(e["dims"]) == size
                assert e["count"] == size[0] * size[1] * size[2]
                assert e["offset"] == lo[0] * shape[1] * shape[2] + lo[1] * shape[2] + lo[2]
            else:
                assert e["count"] == 0 and list(e["dims"]) == [1, 1, 1] and e["offset"] == 0
            assert e["strides"] == (shape[1] * shape[2], shape[2])
            assert e["spacing"] == (1.0, 2.0, 3.0)


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_tiny(seed):
    g = np.random.default_rng(100 + seed)
    shape = tuple(int(x) for x in g.integers(1, 7, size=3))
    lab = g.integers(0, 6, size=shape).astype(np.uint8)
    lab[g.random(shape) < 0.5] = 0
    max_label = 4  # labels 5 are ignored
    ref = brute_boxes(lab, max_label)
    for e in O.label_rois(lab, max_label):
        l = e["label"]
        if l in ref:
            lo, hi, n = ref[l]
            assert list(e["lo"]) == lo
            assert list(e["dims"]) == [h - a + 1 for a, h in zip(lo, hi)]
            assert e["count"] == n
        else:
            assert e["count"] == 0


def test_properties_random_maps():
    for seed in range(3):
        lab = synth.label_map(seed, shape=(40, 50, 60), n_labels=7, semi_lo=2.0, semi_hi=12.0, noise=1e-4)
        for e in O.label_rois(lab, 9):
            l = e["label"]
            total = int((lab == l).sum())
            assert e["count"] == total
            if total == 0:
                continue
            c = O.crop(lab, e)
            assert int(c.sum()) == total  # the box holds every voxel of l
            for k in range(3):  # and is the smallest such box
                assert c.take(0, axis=k).any() and c.take(c.shape[k] - 1, axis=k).any()
            z, y, x = (int(v) for v in e["lo"])
            assert e["offset"] == np.ravel_multi_index((z, y, x), lab.shape)
