"""CPU checks of the test helpers used by the full-size batched parity tests:
the extreme-point search for the farthest pair and the oracle worker pool."""
import numpy as np

from oracle import oracle as O
from paper_2510_02894_amd import synth
from tests import brute, oracle_pool


def test_chunked_and_hull_max_pair_match_brute_force():
    g = np.random.default_rng(5)
    for n in (7, 50, 700):
        pos = g.normal(size=(n, 3))
        ids = np.sort(g.choice(10 * n, size=n, replace=False)).astype(np.int64)
        ref = brute.max_pair(ids, pos)
        assert brute.max_pair_chunked(ids, pos, chunk=64) == ref
        assert brute.hull_max_pair(ids, pos) == ref
    # a lattice: many pairs tie at the maximum, the smallest ids must win
    u = np.stack(np.meshgrid(*[np.arange(4.0)] * 3, indexing="ij"), -1).reshape(-1, 3) * 0.5
    ids = np.arange(len(u), dtype=np.int64) * 3 + 1
    ref = brute.max_pair(ids, u)
    assert brute.max_pair_chunked(ids, u, chunk=5) == ref
    assert brute.hull_max_pair(ids, u) == ref


def test_hull_max_pair_on_mesh_vertices():
    m, sp = synth.single_roi(2, shape=(30, 30, 30))
    ids, pos, _ = O.vertices(m, sp)
    assert brute.hull_max_pair(ids, pos) == brute.max_pair_chunked(ids, pos)


def test_oracle_pool_matches_oracle():
    buf, offs, shapes, sps = synth.batched_rois(6, 3, lmin=4.0, lmax=16.0)
    res = oracle_pool.run(buf, offs, shapes, sps, brute_max=60, workers=2)
    for r in range(len(offs)):
        n = int(np.prod(shapes[r]))
        m = buf[offs[r]:offs[r] + n].reshape(shapes[r])
        ref = O.shape3d(m, sps[r])
        assert res[r]["V"] == ref["V"] and res[r]["T"] == ref["T"]
        np.testing.assert_array_equal(np.sqrt(res[r]["d2"]), ref["features"][2:])
        np.testing.assert_array_equal(res[r]["pair_ids"], ref["pair_ids"])
        assert abs(abs(res[r]["signed_volume"]) - ref["features"][0]) <= 1e-12 * ref["features"][0]
        assert abs(res[r]["area"] - ref["features"][1]) <= 1e-12 * ref["features"][1]
    assert {x["method3d"] for x in res} >= {"extreme points"}
