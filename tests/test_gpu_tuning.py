"""GPU checks of the pair-pass tiles and their autotuner: every tiling gives
bit-identical results (single ROI with plane buckets, a mixed batch, graph
replay after a change of tiles), and the autotuner picks a valid tiling and
reuses its cache."""
import sys

import numpy as np
import pytest

from paper_2510_02894_amd import synth

pytestmark = pytest.mark.gpu

TILINGS = [(it, jc, 0) for it in (2, 4, 8) for jc in (64, 128, 256, 512, 1024)] + \
    [(it, jc, 1) for it in (4, 8) for jc in (64, 128, 256, 512, 1024)]


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
    # single-ROI calls run the general pipeline (the one the tiles belong to)
    shape3d.set_small_path(False)
    yield shape3d
    shape3d.set_small_path(True)
    shape3d.set_tuning(8, 1024, 0, 1)


def test_every_tiling_gives_identical_results_single_roi(S):
    import torch

    m = synth.ellipsoid_union((70, 90, 110), synth.ellipsoid_params(synth.rng(9, 0), 4, 10.0, 40.0, 20.0, 60.0))
    vol = torch.from_numpy(m.astype(np.uint8)).cuda()
    sp = (1.1, 0.8, 0.9)
    ref = None
    for it, jc, kern in TILINGS:
        say("single ROI tiling %d x %d kernel %d" % (it, jc, kern))
        S.set_tuning(it, jc, 0, kern)
        f, st, _ = S.features(vol, sp, stats=True)
        got = (f.tolist(), st["pair_ids"].tolist(), st["V"], st["T"])
        if ref is None:
            ref = got
        assert got == ref, (it, jc, kern)
    S.set_tuning(8, 1024, 0, 1)


def test_every_tiling_gives_identical_results_batched_and_graph(S):
    import torch

    buf, offs, shapes, sps = synth.batched_rois(40, 7, lmin=8.0, lmax=48.0)
    base = torch.from_numpy(buf).cuda()
    table = S.roi_table(offs, shapes, sps)
    S.set_tuning(8, 1024, 0, 1)
    ref, _ = S.batched(base, table)
    for it, jc, kern in TILINGS:
        for bpc in (0, 1):
            say("batch tiling %d x %d, %d blocks/CU, kernel %d" % (it, jc, bpc, kern))
            S.set_tuning(it, jc, bpc, kern)
            out, _ = S.batched(base, table, graph=True)   # records a graph with these tiles
            assert np.array_equal(out, ref), (it, jc, bpc, kern)
            out, _ = S.batched(base, table, graph=True)   # replays it
            assert np.array_equal(out, ref), (it, jc, bpc, kern)
    S.set_tuning(8, 1024, 0, 1)


def test_autotune_and_cache(S, tmp_path):
    import torch

    buf, offs, shapes, sps = synth.batched_rois(24, 3, lmin=8.0, lmax=40.0)
    base = torch.from_numpy(buf).cuda()
    table = S.roi_table(offs, shapes, sps)
    ref, _ = S.batched(base, table)
    cache = tmp_path / "tiles.txt"
    say("autotune")
    best, ms = S.autotune(base, table, reps=1, cache_path=str(cache))
    assert (best[0], best[1], best[3]) in TILINGS and best[2] == 0 and ms > 0
    assert S.get_tuning() == best
    lines = cache.read_text().split("\n")
    assert len([l for l in lines if l.strip()]) == 1
    key, kern, it, jc, bpc, ms_file = lines[0].split()
    assert (int(it), int(jc), int(bpc), int(kern)) == best and key.startswith("u8:n")
    # a cache hit takes the stored tiles without timing
    S.set_tuning(2, 64, 0)
    best2, ms2 = S.autotune(base, table, reps=1, cache_path=str(cache))
    assert best2 == best and ms2 == pytest.approx(float(ms_file))
    assert len([l for l in cache.read_text().split("\n") if l.strip()]) == 1
    out, _ = S.batched(base, table, graph=True)
    assert np.array_equal(out, ref)
    S.set_tuning(8, 1024, 0, 1)
