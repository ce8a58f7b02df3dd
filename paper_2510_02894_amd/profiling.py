"""Summaries of rocprofv3 runs of the benchmark (CSV output), for the
measurement records kept with the repository.

    python -m paper_2510_02894_amd.profiling trace DIR --title T --command C [--out FILE]
    python -m paper_2510_02894_amd.profiling counters DIR [DIR ...] --title T --command C [--out FILE]
    python -m paper_2510_02894_amd.profiling traffic FETCH_DIR WRITE_DIR --workload W --tiles 8 1024 0 1
                                              --command-fetch C1 --command-write C2 [--out profiles/traffic.json]

DIR is a rocprofv3 output directory written with ``--output-format csv``
(``run_kernel_trace.csv`` for ``--kernel-trace``, ``run_counter_collection.csv``
for ``--pmc``).  Dispatches are grouped into library calls by the first kernel
of each call (k_head_clear for the general pipeline, k_small_head for the
small-mesh path); a call that runs the pruning pass (k_prune_box) is a
call with pruning, one without it a call that evaluates every pair.  This
module reads only the profiler's text output; it runs nothing on the GPU.
"""
from __future__ import annotations

import argparse
import csv
import glob
import gzip
import hashlib
import json
import os
import re
import sys
from collections import OrderedDict, defaultdict

CALL_HEADS = ("k_head_clear", "k_small_head")
# call classes
ALL_PAIRS = "general pipeline, every pair"
PRUNED = "general pipeline with the pruning pass"
SMALL = "single ROI, small-mesh path"
COPY_BYTES = 256 << 20  # the benchmark's calibration copy (--copy-calibration)


def short_name(name: str) -> str:
    """Kernel name without its argument list and return type."""
    depth = 0
    for i in range(len(name) - 1, -1, -1):
        if name[i] == ")":
            depth += 1
        elif name[i] == "(":
            depth -= 1
            if depth == 0:
                name = name[:i]
                break
    name = name.replace("void ", "").replace("(anonymous namespace)::", "")
    return name.strip()


def base_name(name: str) -> str:
    """Short name without namespace and template arguments (k_mesh_pass<0> -> k_mesh_pass)."""
    n = short_name(name)
    n = re.sub(r"<.*>$", "", n)
    return n.split("::")[-1]


def _open(d: str, suffix: str):
    """The first *suffix (or *suffix.gz) file under d, opened as text."""
    for suf in (suffix, suffix + ".gz"):
        hits = sorted(glob.glob(os.path.join(d, "**", "*" + suf), recursive=True))
        if hits:
            return gzip.open(hits[0], "rt") if suf.endswith(".gz") else open(hits[0])
    raise FileNotFoundError("no *%s under %s" % (suffix, d))


def read_trace(d: str):
    """Kernel dispatches in start order: dicts with name, ns, vgpr, lds, scratch, grid, wg."""
    rows = []
    with _open(d, "kernel_trace.csv") as fh:
        for r in csv.DictReader(fh):
            rows.append(dict(name=short_name(r["Kernel_Name"]), start=int(r["Start_Timestamp"]),
                             ns=int(r["End_Timestamp"]) - int(r["Start_Timestamp"]),
                             vgpr=int(r.get("VGPR_Count", 0) or 0), lds=int(r.get("LDS_Block_Size", 0) or 0),
                             scratch=int(r.get("Scratch_Size", 0) or 0),
                             grid=int(r.get("Grid_Size_X", 0) or 0), wg=int(r.get("Workgroup_Size_X", 0) or 0)))
    rows.sort(key=lambda x: x["start"])
    return rows


def read_counters(d: str):
    """Counter values per dispatch in dispatch order: list of (name, {counter: value}, workgroups)."""
    per = OrderedDict()
    with _open(d, "counter_collection.csv") as fh:
        for r in csv.DictReader(fh):
            key = int(r["Dispatch_Id"])
            ent = per.setdefault(key, [short_name(r["Kernel_Name"]), {}, int(r.get("Start_Timestamp", 0) or 0),
                                       int(r.get("Grid_Size", 0) or 0) // max(int(r.get("Workgroup_Size", 1) or 1), 1)])
            ent[1][r["Counter_Name"]] = ent[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    out = sorted(per.values(), key=lambda e: e[2])
    return [(n, c, wgs) for n, c, _, wgs in out]


def _disp_rois(disp):
    return [w if n.endswith("k_mesh_totals") else 0 for n, _, w in disp]


def split_calls(names, rois=None):
    """Indices of the dispatches grouped by library call, with a call class;
    dispatches before the first call are dropped.  rois[i]: for a dispatch of
    k_mesh_totals (one workgroup per ROI), the call's ROI count."""
    calls, cur = [], None
    for i, n in enumerate(names):
        b = n.split("::")[-1]
        if b in CALL_HEADS:
            cur = [b, []]
            calls.append(cur)
        if cur is not None:
            cur[1].append(i)
    out = []
    for head, idx in calls:
        if head == "k_small_head":
            out.append((SMALL, idx))
            continue
        bases = {names[i].split("::")[-1].split("<")[0] for i in idx}
        n_rois = max([rois[i] for i in idx if rois and rois[i]] or [1])
        kind = "batch of %d ROIs" % n_rois if n_rois > 1 else "single ROI"
        out.append(("%s, %s" % (kind, PRUNED if "k_prune_box" in bases else ALL_PAIRS), idx))
    return out


def _rois(rows):
    return [r["grid"] // max(r["wg"], 1) if r["name"].endswith("k_mesh_totals") else 0 for r in rows]


def _classes(groups):
    return sorted(groups, key=lambda c: (c.startswith("batch"), c == SMALL, c))


def trace_tables(rows):
    """Markdown tables of kernel time per call class."""
    names = [r["name"] for r in rows]
    groups = defaultdict(list)
    for cls, idx in split_calls(names, _rois(rows)):
        groups[cls].append(idx)
    lines = []
    for cls in _classes(groups):
        calls = groups[cls]
        agg = OrderedDict()
        for idx in calls:
            for i in idx:
                r = rows[i]
                a = agg.setdefault(r["name"], dict(n=0, ns=0, vgpr=r["vgpr"], lds=r["lds"], scratch=r["scratch"],
                                                   grid=r["grid"], wg=r["wg"]))
                a["n"] += 1
                a["ns"] += r["ns"]
        total = sum(a["ns"] for a in agg.values())
        lines.append("### %s calls (%d calls; kernel time per call %.1f us)" % (cls, len(calls), total / 1e3 / len(calls)))
        lines.append("")
        lines.append("| kernel | launches | avg us | us per call | % | workgroups | wg size | VGPR | LDS B | scratch B |")
        lines.append("|---|---|---|---|---|---|---|---|---|---|")
        for n, a in sorted(agg.items(), key=lambda kv: -kv[1]["ns"]):
            if a["ns"] < 0.002 * total:
                continue
            lines.append("| %s | %d | %.2f | %.2f | %.1f | %d | %d | %d | %d | %d |" % (
                n, a["n"], a["ns"] / 1e3 / a["n"], a["ns"] / 1e3 / len(calls), 100.0 * a["ns"] / total,
                a["grid"] // max(a["wg"], 1), a["wg"], a["vgpr"], a["lds"], a["scratch"]))
        lines.append("")
    return lines


def counter_tables(dirs):
    """Per-kernel counter sums per dispatch (averaged over dispatches) per call class."""
    merged = defaultdict(lambda: defaultdict(list))  # (cls, kernel) -> counter -> values per dispatch
    counters = []
    for d in dirs:
        disp = read_counters(d)
        names = [n for n, _, _ in disp]
        for cls, idx in split_calls(names, _disp_rois(disp)):
            for i in idx:
                n, c, _ = disp[i]
                for k, v in c.items():
                    if k not in counters:
                        counters.append(k)
                    merged[(cls, n)][k].append(v)
    lines = []
    keys = sorted(merged, key=lambda k: (k[0], k[1]))
    for cls in _classes({k[0] for k in keys}):
        ks = [k for k in keys if k[0] == cls]
        lines.append("### %s calls: counters per dispatch (mean over dispatches)" % cls)
        lines.append("")
        lines.append("| kernel | " + " | ".join(counters) + " |")
        lines.append("|---|" + "---|" * len(counters))
        for k in ks:
            vals = merged[k]
            cells = []
            for c in counters:
                v = vals.get(c)
                cells.append("%.4g" % (sum(v) / len(v)) if v else "")
            lines.append("| %s | %s |" % (k[1], " | ".join(cells)))
        lines.append("")
    return lines, merged


def copy_scale(d: str, counter: str):
    """Counter KiB of the calibration copy (a plain device copy of COPY_BYTES)."""
    disp = read_counters(d)
    vals = [c[counter] for n, c, _ in disp if counter in c and ("copy" in n.lower()) and c[counter] > 0]
    if not vals:
        return None
    v = max(vals)  # the 256 MiB copies are the largest copy dispatches
    return COPY_BYTES / (v * 1024.0), v


def source_hash(files=None) -> str:
    """Hash of the kernel sources (all of csrc, or the given files plus the shared headers), as bench.py computes it."""
    shared = ["mc_table.h", "s3d_device.h", "s3d_internal.h", "s3d_launch.h"]
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    names = sorted(os.listdir(csrc)) if files is None else sorted(set(files) | set(shared))
    h = hashlib.sha256()
    for n in names:
        if n.endswith((".hip", ".h")):
            with open(os.path.join(csrc, n), "rb") as fh:
                h.update(n.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "k_pair_maxima_h": ["pairs.hip"], "k_pair_maxima": ["pairs.hip"],
    "k_brick_scatter": ["pairs.hip"], "k_brick_hist": ["pairs.hip"],
    "k_mesh_pass": ["mesh.hip"], "k_mesh_rows": ["mesh.hip"],
}


def traffic(fetch_dir, write_dir, cls="single ROI, " + ALL_PAIRS):
    """HBM bytes per launch of the profiled kernels of `cls` calls, scaled by the calibration copy."""
    sf = copy_scale(fetch_dir, "FETCH_SIZE")
    sw = copy_scale(write_dir, "WRITE_SIZE")
    if sf is None or sw is None:
        raise RuntimeError("no calibration copy in the counter runs (run the benchmark with --copy-calibration)")
    res = {}
    for d, counter, scale in ((fetch_dir, "FETCH_SIZE", sf[0]), (write_dir, "WRITE_SIZE", sw[0])):
        disp = read_counters(d)
        names = [n for n, _, _ in disp]
        per = defaultdict(list)
        for c, idx in split_calls(names, _disp_rois(disp)):
            if c != cls:
                continue
            for i in idx:
                per[base_name(disp[i][0])].append(disp[i][1].get(counter, 0.0) * 1024.0 * scale)
        for k, v in per.items():
            res.setdefault(k, {})[counter] = sum(v) / len(v)
    return res, sf, sw


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--out")
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--title", required=True)
    c.add_argument("--command", action="append", required=True)
    c.add_argument("--out")
    f = sub.add_parser("traffic")
    f.add_argument("fetch_dir")
    f.add_argument("write_dir")
    f.add_argument("--workload", required=True)
    f.add_argument("--tiles", type=int, nargs=4, required=True)
    f.add_argument("--command-fetch", required=True)
    f.add_argument("--command-write", required=True)
    f.add_argument("--out")
    f.add_argument("--md")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        lines = ["# " + a.title, "", "Kernel trace, command:", "", "    " + a.command, ""]
        lines += trace_tables(read_trace(a.dir))
        text = "\n".join(lines) + "\n"
    elif a.cmd == "counters":
        lines = ["# " + a.title, "", "Counter runs (one rocprofv3 --pmc pass each), commands:", ""]
        lines += ["    " + x for x in a.command] + [""]
        tab, _ = counter_tables(a.dirs)
        lines += tab
        text = "\n".join(lines) + "\n"
    else:
        res, sf, sw = traffic(a.fetch_dir, a.write_dir)
        rec = OrderedDict(
            source_hash=source_hash(), workload=a.workload, tiles=a.tiles, scale_fetch=sf[0], scale_write=sw[0],
            calibration="device copy of %d bytes: FETCH_SIZE %.1f KiB, WRITE_SIZE %.1f KiB" % (COPY_BYTES, sf[1], sw[1]),
            commands=OrderedDict(fetch=a.command_fetch, write=a.command_write), kernels=OrderedDict())
        for k in sorted(res):
            if k not in KERNEL_SOURCES:
                continue
            fb, wb = res[k].get("FETCH_SIZE", 0.0), res[k].get("WRITE_SIZE", 0.0)
            rec["kernels"][k] = OrderedDict(fetch_bytes=fb, write_bytes=wb, hbm_bytes_per_launch=fb + wb,
                                            source_hash=source_hash(KERNEL_SOURCES[k]))
        text = json.dumps(rec, indent=1) + "\n"
        if a.md:
            lines = ["", "## HBM traffic per launch (all-pairs calls)", "",
                     "Scaled by the calibration copy: " + rec["calibration"] +
                     " -> fetch x%.3f, write x%.3f." % (sf[0], sw[0]), "", "    " + a.command_fetch,
                     "    " + a.command_write, "", "| kernel | fetch MB | write MB | total MB |", "|---|---|---|---|"]
            for k in sorted(res, key=lambda k: -(res[k].get("FETCH_SIZE", 0) + res[k].get("WRITE_SIZE", 0))):
                fb, wb = res[k].get("FETCH_SIZE", 0.0), res[k].get("WRITE_SIZE", 0.0)
                if fb + wb < 1e6:
                    continue
                lines.append("| %s | %.1f | %.1f | %.1f |" % (k, fb / 1e6, wb / 1e6, (fb + wb) / 1e6))
            with open(a.md, "a") as fh:
                fh.write("\n".join(lines) + "\n")
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    else:
        sys.stdout.write(text)


if __name__ == "__main__":
    main()
