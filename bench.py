#!/usr/bin/env python3
"""Benchmark of the shape-feature path on one MI355X.

Workload (one step = one full call of the library: marching-cubes mesh pass,
plane buckets, all-pairs 3D and in-plane maxima, exact refinement, results on
the host): the large single ROI, a uint8 mask of 300 x 512 x 512 voxels
(axis 0 = slices) with spacing (1.25, 0.7, 0.7) mm, the union of 20 seeded
ellipsoids (semi-axes 20-90 voxels) thresholded after Gaussian smoothing
(sigma 3).  Four copies of the mask rotate through the steps so the 256 MB
Infinity Cache does not hold the input.

Prints one JSON line.  value = 3D diameter vertex pairs V(V-1)/2 per second of
whole-call time with every vertex pair evaluated (the pair pass's pruning
switched off); roofline of that call's dominant kernel (the MFMA pair pass),
8 algorithmic flops per vertex pair (3D and in-plane) over its time from HIP
events recorded around it inside the library, against the peak of the
contraction's dtype.  `effective` gives the library's default call on the same
masks, which skips pair tiles that cannot hold the diameter (identical
results), as V(V-1)/2 per second.  cpu_baseline = the FP64 oracle timed on a
bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3   # MI355X dense FP32 matrix peak
PEAK_F16_MFMA_TFLOPS = 2500.0   # MI355X dense FP16 matrix peak
PEAK_HBM_GBS = 8000.0           # MI355X HBM3E
# Algorithmic work of the all-pairs maximum: 8 flops per vertex pair (3 sub,
# 3 mul, 2 add of |x_i - x_j|^2; the compare is not counted).
ALG_FLOPS_PER_PAIR = 8
# Flops the matrix cores execute per vertex pair (the Gram form, padding and
# split terms included): kernel 0 v_mfma_f32_16x16x4_f32, 2048 flops per 256
# pairs; kernel 1 v_mfma_f32_32x32x16_f16 (split f16), 32768 per 1024 pairs.
MFMA_FLOPS_PER_PAIR = {0: 8, 1: 32}
PEAK_TFLOPS = {0: PEAK_FP32_MFMA_TFLOPS, 1: PEAK_F16_MFMA_TFLOPS}
DTYPE_LABEL = {0: "fp32 MFMA filter + fp64 exact maxima; int64/fp64 area and volume",
               1: "split-f16 MFMA filter + fp64 exact maxima; int64/fp64 area and volume"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(files=None):
    """Hash of the kernel sources (all of csrc, or the given files plus the shared headers)."""
    from paper_2510_02894_amd.profiling import source_hash as h

    return h(files)


def measured_traffic(kernel: str, tiles=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current sources of that kernel (and, for the pair pass,
    with the same tiles)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel)
    from paper_2510_02894_amd.profiling import KERNEL_SOURCES

    if not k or k.get("source_hash") != source_hash(KERNEL_SOURCES.get(kernel)):
        return None
    if tiles is not None and list(rec.get("tiles", [])) != list(tiles):
        return None
    return k.get("hbm_bytes_per_launch")


def cpu_baseline(mask, spacing, target_s):
    from oracle import oracle as O

    t0 = time.perf_counter()
    ids, pos, _ = O.vertices(mask, spacing)
    t_vert = time.perf_counter() - t0
    V = len(ids)
    # calibrate on 1,024 rows (after a warm-up call that starts the OpenMP
    # threads), then size the sample to about target_s seconds
    O.max_pair_rows(pos, 0, 16)
    rows = min(V, 1024)
    t0 = time.perf_counter()
    O.max_pair_rows(pos, 0, rows)
    dt = time.perf_counter() - t0
    rate_rows = rows / max(dt, 1e-6)
    nrows = int(min(V, max(rows, rate_rows * target_s)))
    t0 = time.perf_counter()
    _, threads = O.max_pair_rows(pos, 0, nrows)
    dt = time.perf_counter() - t0
    pairs = sum(V - 1 - i for i in range(0, nrows)) if nrows < 10000 else nrows * (V - 1) - nrows * (nrows - 1) // 2
    return dict(
        value=pairs / dt,
        unit="pairs/s",
        cores=int(threads),
        kind="oracle",
        sample="rows 0..%d of the FP64 all-pairs maximum over the %d mesh vertices of the same mask "
               "(%.3g of %.3g pairs, %.1f s; vertex extraction %.1f s)" % (
                   nrows, V, float(pairs), V * (V - 1) / 2.0, dt, t_vert),
    )


def bench_single_roi(args, S):
    """Latency of the plain entry point on the single-ROI workload (64^3 uint8,
    one ellipsoid with semi-axes 8-24 voxels): host-to-host, synchronous."""
    import torch

    from paper_2510_02894_amd import synth

    mask, sp = synth.single_roi(0)
    vol = torch.from_numpy(mask).cuda()
    for _ in range(5):
        S.shape3d_u8(vol, sp)
    torch.cuda.synchronize()
    lat = []
    for _ in range(max(20, 5 * args.steps)):
        t0 = time.perf_counter()
        S.shape3d_u8(vol, sp)
        lat.append(1e6 * (time.perf_counter() - t0))
    # the same calls through the general pipeline (small-mesh path off)
    S.set_small_path(False)
    for _ in range(5):
        S.shape3d_u8(vol, sp)
    lat_general = []
    for _ in range(max(20, 5 * args.steps)):
        t0 = time.perf_counter()
        S.shape3d_u8(vol, sp)
        lat_general.append(1e6 * (time.perf_counter() - t0))
    S.set_small_path(True)
    _, st, _ = S.features(vol, sp, stats=True, timing=True)
    rec = {
        "workload": "single ROI: uint8 64^3, one ellipsoid (semi-axes 8-24 voxels), spacing (1,1,1) mm",
        "vertices": st["V"],
        "calls": len(lat),
        "latency_us_median": float(np.median(lat)),
        "latency_us_p10": float(np.percentile(lat, 10)),
        "latency_us_p90": float(np.percentile(lat, 90)),
        "latency_us_median_general_pipeline": float(np.median(lat_general)),
        "device_phases_ms_general_pipeline": st["ms"],
    }
    log("single ROI: median %.1f us host-to-host (general pipeline %.1f us)" % (
        rec["latency_us_median"], rec["latency_us_median_general_pipeline"]))
    return rec


def bench_batched(args, S):
    """ROIs/s of the batched workload (4096 uint8 ROIs, edges log-uniform 8-128
    voxels) replayed as one hipGraph, beside a loop of single-ROI calls."""
    import torch

    from paper_2510_02894_amd import synth

    t0 = time.perf_counter()
    buf, offs, shapes, sps = synth.batched_rois_torch(args.batch_rois, 0)
    torch.cuda.synchronize()
    log("batched: generated %d ROIs (%.2f GB) in %.1f s" % (len(offs), buf.numel() / 1e9, time.perf_counter() - t0))
    table = S.roi_table(offs, shapes, sps)

    def timed_graph():
        out, status = S.batched(buf, table, graph=True)   # eager run + graph recording
        for _ in range(max(1, args.warmup)):
            S.batched(buf, table, graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out2, _ = S.batched(buf, table, graph=True)
        torch.cuda.synchronize()
        return out, status, out2, 1e3 * (time.perf_counter() - t0) / args.steps

    default_tiles = S.get_tuning()
    out, status, out2, ms_default = timed_graph()
    tiles = default_tiles
    if not args.no_autotune:
        tiles, _ = S.autotune(buf, table, reps=2)
        out, status, out2, ms_graph = timed_graph()
        log("batched: autotuned tiles %s (default %s: %.2f ms)" % (tiles, default_tiles, ms_default))
    else:
        ms_graph = ms_default
    t0 = time.perf_counter()
    for _ in range(max(1, args.steps // 2)):
        S.batched(buf, table, graph=False)
    torch.cuda.synchronize()
    ms_eager = 1e3 * (time.perf_counter() - t0) / max(1, args.steps // 2)
    rec = {
        "workload": "%d uint8 ROIs, edges log-uniform 8-128 voxels, aspect 0.5-2, 1-6 ellipsoids, spacing "
                    "U[0.5,1.5] mm" % len(offs),
        "voxels": int(buf.numel()),
        "ms_per_batch_graph": ms_graph,
        "ms_per_batch_eager": ms_eager,
        "rois_per_s": len(offs) / (ms_graph * 1e-3),
        "tiles": list(tiles),
        "ms_per_batch_default_tiles": ms_default,
        "empty_rois": int(np.sum(status == 1)),
    }
    if not args.skip_sequential:
        # sequential single-ROI calls on the same inputs (one pass)
        seq = np.zeros_like(out)
        pairs = 0
        t0 = time.perf_counter()
        for r in range(len(offs)):
            n = int(np.prod(shapes[r]))
            seq[r], st, _ = S.features(buf[int(offs[r]):int(offs[r]) + n].view(shapes[r]), sps[r], stats=True)
            pairs += st["V"] * (st["V"] - 1) // 2
        torch.cuda.synchronize()
        ms_seq = 1e3 * (time.perf_counter() - t0)
        rec.update({
            "pairs_3d": pairs,
            "pairs_3d_per_s": pairs / (ms_graph * 1e-3),
            "sequential_single_roi_ms": ms_seq,
            "sequential_rois_per_s": len(offs) / (ms_seq * 1e-3),
            "speedup_vs_sequential": ms_seq / ms_graph,
            "identical_to_single_roi_calls": bool(np.array_equal(out2, seq)),
        })
        log("batched: graph %.2f ms, eager %.2f ms, sequential %.1f ms, %.3g 3D pairs" % (
            ms_graph, ms_eager, ms_seq, pairs))
    else:
        log("batched: graph %.2f ms, eager %.2f ms" % (ms_graph, ms_eager))
    return rec


def bench_differentiable(args, S):
    """Forward vs forward+backward on the 256^3 soft mask (L = area + 0.1 volume + diameter)."""
    import torch

    from paper_2510_02894_amd import synth

    t0 = time.perf_counter()
    p, sp = synth.differentiable_roi(0)
    log("differentiable: generated %s in %.1f s" % (p.shape, time.perf_counter() - t0))
    pt = torch.from_numpy(p).cuda()
    gout = [0.1, 1.0, 1.0, 0.0, 0.0, 0.0]
    if not args.no_autotune:
        S.autotune(pt.view(-1), S.roi_table([0], [p.shape], [sp]), reps=2)
    for _ in range(max(1, args.warmup)):
        f, saved = S.soft_forward(pt, sp)
        S.soft_backward(pt, saved, gout)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S.features(pt, sp)
    torch.cuda.synchronize()
    ms_fwd = 1e3 * (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        f, saved = S.soft_forward(pt, sp)
        g = S.soft_backward(pt, saved, gout)
    torch.cuda.synchronize()
    ms_fb = 1e3 * (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g = S.soft_backward(pt, saved, gout)
    torch.cuda.synchronize()
    ms_b = 1e3 * (time.perf_counter() - t0) / args.steps
    _, st, _ = S.features(pt, sp, stats=True, timing=True)
    rec = {
        "workload": "float32 soft mask 256^3, 8-ellipsoid union, tau 1 voxel; L = area + 0.1 volume + diameter",
        "vertices": st["V"],
        "fwd_ms": ms_fwd,
        "fwd_bwd_ms": ms_fb,
        "bwd_ms": ms_b,
        "ratio": ms_fb / ms_fwd,
        "tiles": list(S.get_tuning()),
        "fwd_phases_ms": st["ms"],
    }
    log("differentiable: fwd %.2f ms, fwd+bwd %.2f ms" % (ms_fwd, ms_fb))
    return rec


def bench_batched_soft(args, S):
    """Batched soft masks (256 float32 ROIs, cubic edges log-uniform 48-160,
    tau U[0.5, 2], spacing (2.0, 0.8, 0.8) mm): batched forward alone vs
    forward + backward of all six features (grad_out = 1)."""
    import torch

    from paper_2510_02894_amd import synth

    t0 = time.perf_counter()
    workers = max(1, min(16, os.cpu_count() or 1))
    buf, offs, shapes, sps = synth.soft_batch(args.soft_rois, 0, workers=workers)
    base = torch.from_numpy(buf).cuda()
    del buf
    torch.cuda.synchronize()
    log("batched soft: generated %d ROIs (%.2f GB) in %.1f s" % (len(offs), base.numel() * 4 / 1e9,
                                                                time.perf_counter() - t0))
    table = S.roi_table(offs, shapes, sps)
    if not args.no_autotune:
        S.autotune(base, table, reps=2)
    gout = np.ones((len(offs), 6))
    grad = torch.empty_like(base)
    for _ in range(max(1, args.warmup)):
        f, saved = S.batched_soft_forward(base, table, graph=True)
        S.batched_soft_backward(base, table, saved, gout, grad=grad)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S.batched(base, table, graph=True)
    torch.cuda.synchronize()
    ms_fwd = 1e3 * (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        f, saved = S.batched_soft_forward(base, table, graph=True)
        S.batched_soft_backward(base, table, saved, gout, grad=grad)
    torch.cuda.synchronize()
    ms_fb = 1e3 * (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S.batched_soft_backward(base, table, saved, gout, grad=grad)
    torch.cuda.synchronize()
    ms_b = 1e3 * (time.perf_counter() - t0) / args.steps
    V = int(sum(s.n_vertices for s in saved))
    rec = {
        "workload": "%d float32 soft ROIs, cubic edges log-uniform 48-160 voxels, 8-ellipsoid unions, tau U[0.5,2], "
                    "spacing (2.0,0.8,0.8) mm; gradients of all six features" % len(offs),
        "voxels": int(base.numel()),
        "vertices": V,
        "fwd_ms": ms_fwd,
        "fwd_bwd_ms": ms_fb,
        "bwd_ms": ms_b,
        "ratio": ms_fb / ms_fwd,
        "bwd_hbm_gbs": 3 * 4 * base.numel() / (ms_b * 1e-3) / 1e9,
        "tiles": list(S.get_tuning()),
    }
    log("batched soft: fwd %.2f ms, fwd+bwd %.2f ms, bwd %.2f ms" % (ms_fwd, ms_fb, ms_b))
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--copies", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-differentiable", action="store_true")
    ap.add_argument("--batch-rois", type=int, default=4096)
    ap.add_argument("--skip-batched-soft", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default pair-pass tiles")
    ap.add_argument("--skip-single", action="store_true")
    ap.add_argument("--soft-rois", type=int, default=256)
    ap.add_argument("--skip-large", action="store_true",
                    help="only the batched / differentiable sections (for profiling them)")
    ap.add_argument("--skip-sequential", action="store_true",
                    help="batched section without the loop of single-ROI calls")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device-to-device copy (known bytes) to scale HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2510_02894_amd import shape3d as S
    from paper_2510_02894_amd import synth

    S.load()
    if args.copy_calibration:
        nbytes = 256 << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 device copies of %d bytes" % nbytes)
        del src, dst
    if args.skip_large:
        rec = {"single_roi": None if args.skip_single else bench_single_roi(args, S),
               "batched": None if args.skip_batched else bench_batched(args, S),
               "differentiable": None if args.skip_differentiable else bench_differentiable(args, S),
               "batched_soft": None if args.skip_batched_soft else bench_batched_soft(args, S)}
        print(json.dumps(rec), flush=True)
        return
    t0 = time.perf_counter()
    mask, spacing = synth.large_roi(0)
    log("generated mask %s in %.1f s (%d voxels inside)" % (mask.shape, time.perf_counter() - t0,
                                                          int(mask.sum())))
    dev = torch.device("cuda:0")
    vols = [torch.from_numpy(mask).to(dev) for _ in range(max(1, args.copies))]
    torch.cuda.synchronize()

    # pair-pass tiles: tuned separately for the default call (pruned 3D
    # pairs) and for the call that evaluates every pair
    prune_default = S.get_prune()
    table1 = S.roi_table([0], [mask.shape], [spacing])
    tiles = tiles_eff = S.get_tuning()
    if not args.no_autotune:
        tiles_eff, _ = S.autotune(vols[0].view(-1), table1, reps=2)
        S.set_prune(0)
        try:
            tiles, _ = S.autotune(vols[0].view(-1), table1, reps=2)
        finally:
            S.set_prune(prune_default)
        log("large ROI: autotuned pair-pass tiles %s (default call), %s (every pair)" % (tiles_eff, tiles))

    def step(i):
        return S.features(vols[i % len(vols)], spacing, stats=True, timing=True)

    def timed(label):
        for i in range(args.warmup):
            f, st, rc = step(i)
            log("%s warmup %d: %.3f ms total, V=%d" % (label, i, st["ms"]["total"], st["V"]))
        torch.cuda.synchronize()
        phases = []
        t0 = time.perf_counter()
        for i in range(args.steps):
            f, st, rc = step(i)
            phases.append(st["ms"])
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.steps
        avg = {k: float(np.mean([p[k] for p in phases])) for k in phases[0]}
        log("%s: %.3f ms per call; phases (ms): %s" % (label, ms, ", ".join("%s %.4f" % kv for kv in avg.items())))
        return f, st, ms, avg, phases

    # the library's default call (exact; the 3D pair tiles that cannot hold
    # the diameter are skipped), then every vertex pair evaluated
    S.set_tuning(*tiles_eff)
    f_eff, st_eff, ms_eff, avg_eff, _ = timed("default call")
    S.set_prune(0)
    S.set_tuning(*tiles)
    try:
        f, st, ms_per_step, avg, phases = timed("all pairs")
    finally:
        S.set_prune(prune_default)
    assert np.array_equal(f, f_eff) and np.array_equal(st["pair_ids"], st_eff["pair_ids"]), \
        "pruned and all-pairs calls differ"
    V = st["V"]
    pairs3 = V * (V - 1) // 2
    pairs2 = st["pairs_2d"]

    t_pair = avg["pair_maxima"] * 1e-3
    kern = int(tiles[3])
    achieved = ALG_FLOPS_PER_PAIR * (pairs3 + pairs2) / t_pair / 1e12
    traffic = measured_traffic("k_pair_maxima_h" if kern == 1 else "k_pair_maxima", tiles)
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[kern], "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS[kern], "traffic": traffic,
                "kernel": "split-f16 v_mfma_f32_32x32x16_f16" if kern == 1 else "fp32 v_mfma_f32_16x16x4_f32",
                "work": "%d algorithmic flops per vertex pair x (V(V-1)/2 + in-plane pairs) = %.4g flops per launch"
                        % (ALG_FLOPS_PER_PAIR, ALG_FLOPS_PER_PAIR * float(pairs3 + pairs2)),
                "kernel_ms": avg["pair_maxima"]}
    # share of the matrix pipe's peak that the kernel's executed MFMA flops reach
    # (dense Gram operands, split terms and padding included): not a roofline
    mfma_occupancy = MFMA_FLOPS_PER_PAIR[kern] * (pairs3 + pairs2) / t_pair / 1e12 / PEAK_TFLOPS[kern]
    effective = {
        "what": "the library's default call on the same masks: exact pruned 3D pairs (tiles whose bounding-box "
                "distance bound is below a vertex-pair distance are skipped); identical results",
        "effective_pairs_per_s": pairs3 / (ms_eff * 1e-3),
        "ms_per_step": ms_eff,
        "phases_ms": avg_eff,
        "speedup_vs_all_pairs": ms_per_step / ms_eff,
        "tiles": list(tiles_eff),
    }
    N = int(np.prod(mask.shape))
    t_mesh = (avg["mesh_pass"] + avg["mesh_rows"]) * 1e-3
    tc, te = measured_traffic("k_mesh_pass"), measured_traffic("k_mesh_rows")
    mesh_traffic = tc + te if tc is not None and te is not None else None
    mesh_bytes = N * 1 + 24 * V
    mesh = {"bound": "hbm", "achieved": mesh_bytes / t_mesh / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": mesh_bytes / t_mesh / 1e9 / PEAK_HBM_GBS, "traffic": mesh_traffic}

    single = None if args.skip_single else bench_single_roi(args, S)
    batched = None if args.skip_batched else bench_batched(args, S)
    differentiable = None if args.skip_differentiable else bench_differentiable(args, S)
    batched_soft = None if args.skip_batched_soft else bench_batched_soft(args, S)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a bounded sample (about %.0f s)" % args.cpu_seconds)
        cpu = cpu_baseline(mask, spacing, args.cpu_seconds)

    rec = {
        "metric": "diameter vertex-pairs/s",
        "value": pairs3 / (ms_per_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_LABEL[kern],
        "data": "synthetic",
        "config": {
            "workload": "large ROI: uint8 mask 300x512x512 (axis0 = slices), spacing (1.25,0.7,0.7) mm, "
                        "union of 20 ellipsoids, Gaussian-smoothed (sigma 3) and thresholded",
            "voxels": N,
            "inside_voxels": int(mask.sum()),
            "vertices": V,
            "triangles": st["T"],
            "pairs_3d": pairs3,
            "pairs_in_plane": pairs2,
        },
        "roofline": roofline,
        "mfma_pipe_occupancy": mfma_occupancy,
        "effective": effective,
        "cpu_baseline": cpu,
        "tiles": list(tiles),
        "phases_ms": avg,
        "step_ms_median": float(np.median([p["total"] for p in phases])),
        "step_ms_p10": float(np.percentile([p["total"] for p in phases], 10)),
        "step_ms_p90": float(np.percentile([p["total"] for p in phases], 90)),
        "mesh_roofline": mesh,
        "single_roi": single,
        "batched": batched,
        "differentiable": differentiable,
        "batched_soft": batched_soft,
        "features": [float(x) for x in f],
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
