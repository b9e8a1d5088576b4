#!/usr/bin/env python3
"""SlimSell BFS benchmark on one MI355X.

Workload: R-MAT scale 22, edge factor 16 (a, b, c = .57, .19, .19), seed 1,
symmetrised with self-loops and duplicates dropped; C = 64, sigma = n (full
sort), sel-max semiring, SlimWork on, SlimChunk on; 64 roots drawn uniformly
from the nonzero-degree vertices (seed 1002).  One step = one BFS from each of
the 64 roots.  The graph is built and uploaded before the timed region.

Printed (one JSON line): whole-job GTEPS over the timed steps, the Graph500
harmonic mean of per-root GTEPS, the roofline of the level kernel (algorithmic
bytes per launch from the fused per-level counters over its event-timed mean
duration), the split-length sweep, an Erdos-Renyi graph of the same size, and
the oracle's CPU rate on a bounded sample of roots.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, public spec
C = 64

# Bytes each processed row moves in the level post-processing and the
# gathered-vector element size (see the byte model in the design notes).
ROW_BYTES = {"tropical": 8, "real": 14, "boolean": 7, "selmax": 16}
GATHER_BYTES = {"tropical": 4, "real": 4, "boolean": 1, "selmax": 4}


PROFILE_DIR = os.path.join(ROOT, "profiles")
# profile summaries by kernel: (file base name, substrings that together name
# the kernel in the rocprofv3 trace (every launch form of it), workload text)
PROFILES = {
    "level_kernel<selmax>": ("level_kernel_selmax_rmat_s22", ("ss::level_kernel", "<ss::SelMax"),
                             "R-MAT s22, 64 roots, sel-max, sigma = n"),
    "level_kernel<batch>": ("level_kernel_batch_rmat_s21", ("ss::level_kernel", "<ss::Batch"),
                            "R-MAT s21, 64 roots in one boolean SpMM, sigma = n"),
    "level_kernel<dp>": ("level_kernel_dp_rmat_s22", ("ss::level_kernel", "<ss::Dp"),
                         "R-MAT s22, DP transformation after tropical BFS, 16 roots"),
    "push_kernels<selmax>": ("push_kernels_selmax_rmat_s22", ("push_",),
                             "R-MAT s22, sel-max, forced push schedule, 16 roots"),
}
KERNEL_SOURCES = ["paper_2010_09913_amd/csrc/kernels.hip", "paper_2010_09913_amd/csrc/device.h",
                  "paper_2010_09913_amd/csrc/internal.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from its committed counter summary,
    or None when there is none or the kernel sources changed since."""
    base = PROFILES.get(kernel, (None,))[0]
    if base is None:
        return None
    try:
        with open(os.path.join(PROFILE_DIR, base + ".json")) as f:
            prof = json.load(f)
    except (OSError, ValueError):
        return None
    if prof.get("source_hash") != kernel_source_hash() or prof.get("kernel") != kernel:
        return None
    return prof.get("traffic_bytes_per_launch")


def named(name: str, parts) -> bool:
    """Whether a kernel name contains every one of the given substrings."""
    return all(p in name for p in parts)


def _csv_rows(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _find(d, suffix):
    for name in sorted(os.listdir(d)):
        if name.endswith(suffix):
            return os.path.join(d, name)
    raise FileNotFoundError(f"no *{suffix} in {d}")


def profile_summary(args) -> int:
    """Summarise rocprofv3 output for one kernel (kernel trace, FETCH_SIZE and
    WRITE_SIZE of the same command, and the same counters of a 1 GiB device
    copy that calibrates them) into profiles/<kernel file>.{md,json}."""
    kernel = args.kernel
    base, match, workload = PROFILES[kernel]
    stats = _csv_rows(_find(args.trace, "_kernel_stats.csv"))
    rows = [r for r in stats if named(r["Name"], match)]
    calls = sum(int(r["Calls"]) for r in rows)
    total_ns = sum(float(r["TotalDurationNs"]) for r in rows)

    def per_dispatch(d, counter, name_part):
        rr = [r for r in _csv_rows(_find(d, "_counter_collection.csv"))
              if named(r["Kernel_Name"], name_part) and r["Counter_Name"] == counter]
        return sum(float(r["Counter_Value"]) for r in rr) / len(rr), len(rr)

    prof = {"kernel": kernel, "workload": workload, "source_hash": kernel_source_hash(),
            "calls": calls, "avg_duration_ns": total_ns / max(calls, 1),
            "instances": [r["Name"][:90] for r in rows]}
    if args.fetch and args.write and args.copy_fetch and args.copy_write:
        fetch_kib, n_f = per_dispatch(args.fetch, "FETCH_SIZE", match)
        write_kib, n_w = per_dispatch(args.write, "WRITE_SIZE", match)
        copy_f, _ = per_dispatch(args.copy_fetch, "FETCH_SIZE", ("copyBuffer",))
        copy_w, _ = per_dispatch(args.copy_write, "WRITE_SIZE", ("copyBuffer",))
        gib_kib = float(1 << 20)                  # the copy reads and writes 1 GiB
        f_scale, w_scale = gib_kib / copy_f, gib_kib / copy_w
        prof.update(fetch_kib_per_dispatch=fetch_kib, write_kib_per_dispatch=write_kib,
                    dispatches_counted=[n_f, n_w], copy_fetch_kib=copy_f, copy_write_kib=copy_w,
                    fetch_scale=f_scale, write_scale=w_scale,
                    traffic_bytes_per_launch=(fetch_kib * f_scale + write_kib * w_scale) * 1024.0)
    os.makedirs(args.out_dir, exist_ok=True)
    with open(os.path.join(args.out_dir, base + ".json"), "w") as f:
        json.dump(prof, f, indent=1)
    top = sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:8]
    cmds = [c for c in (args.cmd_trace, args.cmd_fetch, args.cmd_write, args.cmd_copy_fetch,
                        args.cmd_copy_write) if c]
    lines = [f"# {kernel} on {workload}", "",
             "Commands (run from the repository root, `cd /tmp && export TMPDIR=/tmp` first):", ""]
    lines += [f"    {c}" for c in cmds]
    lines += ["", "Kernel trace (`--kernel-trace --stats`), top kernels by total time:", "",
              "| Kernel | Calls | Average ns | Min ns | Max ns | % |", "|---|---|---|---|---|---|"]
    for r in top:
        lines.append(f"| `{r['Name'][:70]}` | {r['Calls']} | {float(r['AverageNs']):.0f} | "
                     f"{r['MinNs']} | {r['MaxNs']} | {float(r['Percentage']):.1f} |")
    lines += ["", f"{kernel}: {calls} calls, average {prof['avg_duration_ns']:.0f} ns "
              f"(all instances whose name contains {' and '.join('`' + m + '`' for m in match)})."]
    if "traffic_bytes_per_launch" in prof:
        lines += ["", "HBM counters per dispatch (KiB), and the copy probe (1 GiB read + 1 GiB "
                  "written per dispatch) that calibrates them:", "",
                  "| | FETCH_SIZE | WRITE_SIZE |", "|---|---|---|",
                  f"| {kernel}, per dispatch | {prof['fetch_kib_per_dispatch']:.0f} | "
                  f"{prof['write_kib_per_dispatch']:.0f} |",
                  f"| copy probe, per dispatch | {prof['copy_fetch_kib']:.0f} | "
                  f"{prof['copy_write_kib']:.0f} |",
                  f"| scale (1 GiB / copy reading) | {prof['fetch_scale']:.3f} | "
                  f"{prof['write_scale']:.3f} |", "",
                  f"Traffic per launch: {prof['traffic_bytes_per_launch'] / 1e6:.1f} MB "
                  f"(scaled fetch + write)."]
    if args.pmc:
        lines += pmc_summary(args, match, prof)
        with open(os.path.join(args.out_dir, base + ".json"), "w") as f:
            json.dump(prof, f, indent=1)
    lines += ["", f"Kernel sources hash {prof['source_hash']}.", ""]
    with open(os.path.join(args.out_dir, base + ".md"), "w") as f:
        f.write("\n".join(lines))
    print(json.dumps(prof))
    return 0


def pmc_summary(args, match: str, prof: dict) -> list:
    """Stall and cache counters of the kernel (one rocprofv3 --pmc pass per
    directory), per dispatch, for all dispatches and for the long ones (the
    levels that sweep most of the layout), with the ratios that explain where
    the time goes."""
    per = {}
    for d in args.pmc:
        for r in _csv_rows(_find(d, "_counter_collection.csv")):
            if not named(r["Kernel_Name"], match):
                continue
            key = (d, int(r["Dispatch_Id"]))
            e = per.setdefault(key, {"_ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
            e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    groups = {"all dispatches": list(per.values()),
              "dispatches over 100 us": [e for e in per.values() if e["_ns"] > 100e3]}

    def ratio(es, a, b):
        num = sum(e.get(a, 0.0) for e in es)
        den = sum(e.get(b, 0.0) for e in es)
        return num / den if den else None

    out = {}
    lines = ["", "Stall and cache counters (`--pmc`, one pass per command):", ""]
    lines += [f"    {c}" for c in args.cmd_pmc]
    lines += ["", "| Ratio | " + " | ".join(groups) + " |", "|---|" + "---|" * len(groups)]
    rows = [("wave cycles waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES)", "SQ_WAIT_ANY", "SQ_WAVE_CYCLES"),
            ("cycles waiting on an instruction (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES)",
             "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES"),
            ("L2 hit rate (TCC_HIT / (TCC_HIT + TCC_MISS))", "TCC_HIT_sum", None),
            ("L1 to L2 read latency, cycles (TCP_TCC_READ_REQ_LATENCY / TCP_TCC_READ_REQ)",
             "TCP_TCC_READ_REQ_LATENCY_sum", "TCP_TCC_READ_REQ_sum"),
            ("L2 to memory read latency, cycles (TCC_EA0_RDREQ_LEVEL / TCC_EA0_RDREQ)",
             "TCC_EA0_RDREQ_LEVEL_sum", "TCC_EA0_RDREQ_sum"),
            ("L2 memory-read credit stalls per read request", "TCC_EA0_RDREQ_DRAM_CREDIT_STALL_sum",
             "TCC_EA0_RDREQ_sum")]
    for label, a, b in rows:
        vals = []
        for g, es in groups.items():
            if b is None:
                hit = sum(e.get("TCC_HIT_sum", 0.0) for e in es)
                miss = sum(e.get("TCC_MISS_sum", 0.0) for e in es)
                v = hit / (hit + miss) if hit + miss else None
            else:
                v = ratio(es, a, b)
            vals.append(v)
            out.setdefault(g, {})[label] = v
        lines.append(f"| {label} | " + " | ".join("n/a" if v is None else f"{v:.3f}" for v in vals)
                     + " |")
    lines += ["", "Dispatches: " + ", ".join(f"{g} {len(es)}" for g, es in groups.items()) + "."]
    prof["pmc"] = out
    return lines


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def nonempty_chunks(deg: np.ndarray, chunks: int) -> int:
    """Chunks with at least one edge under a full sort (the ones the level
    kernel visits and tests): rows sorted by decreasing degree."""
    return int((np.count_nonzero(deg) + C - 1) // C)


def work_units(deg: np.ndarray, split: int) -> int:
    """Work units of a level under a full sort (chunk lengths are the
    degrees of every 64th row in decreasing order) for SlimChunk split
    length `split`, without packing: one per non-empty chunk, or one per
    piece of a chunk longer than `split`."""
    d = np.sort(np.asarray(deg, np.int64))[::-1]
    cl = d[::C]
    cl = cl[cl > 0]
    if split <= 0:
        return int(len(cl))
    return int(np.where(cl > split, (cl + split - 1) // split, 1).sum())


# Bytes a level reads per work unit besides its chunk: the 16-byte unit
# descriptor and the chunk's one-byte "all rows final" flag (a unit whose
# chunk is final is skipped after these; the rows of every processed chunk
# are counted in ROW_BYTES).
UNIT_BYTES = 17


def algorithmic_bytes(levels: dict, r: int, iters: int, semi: str, n: int,
                      units: int) -> float:
    """Bytes the method must move for all levels of root r."""
    cells = levels["active_cells"][r][:iters].astype(np.float64)
    chunks = levels["active_chunks"][r][:iters].astype(np.float64)
    per_level = (4.0 * cells + ROW_BYTES[semi] * C * chunks + 8.0 * chunks
                 + UNIT_BYTES * units + GATHER_BYTES[semi] * n)
    return float(per_level.sum())


def run_workload(ss, G, roots, semi, split, steps, warmup, deg_t, count_pass=True,
                 schedule=0, persistent=False):
    import torch
    # warm-up (also fixes the per-root component sizes)
    res = None
    for _ in range(warmup):
        res = G.bfs(roots, semi, split_len=split, schedule=schedule, persistent=persistent)
    torch.cuda.synchronize()
    if res is None:
        res = G.bfs(roots, semi, split_len=split, schedule=schedule, persistent=persistent)
        torch.cuda.synchronize()
    reached = (res.dist >= 0)
    m_cc = ((reached.to(torch.int64) * deg_t[None, :]).sum(dim=1) // 2).cpu().numpy()
    out = dict(m_cc=m_cc)
    if count_pass:
        cres = G.bfs(roots, semi, split_len=split, level_cap=64)
        out["levels"] = cres.levels
        out["iterations"] = cres.iterations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    r = None
    for _ in range(steps):
        r = G.bfs(roots, semi, split_len=split, timing="bfs", schedule=schedule,
                  persistent=persistent)
        runs.append(r.runs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the outputs of the last timed step, checked against the oracle later
    out.update(wall=wall, runs=runs, result=r)
    # one more step, untimed, with events around every level launch (the
    # per-launch kernel time of the roofline)
    r = G.bfs(roots, semi, split_len=split, timing=True, schedule=schedule,
              persistent=persistent)
    torch.cuda.synchronize()
    out["kernel_runs"] = r.runs
    return out


def summarise(out, roots, semi, n, units, steps):
    m_cc = out["m_cc"].astype(np.float64)
    bfs_ms = np.stack([r["bfs_ms"] for r in out["runs"]])        # [steps, roots]
    kern_ms = out["kernel_runs"]["kernel_ms"]                      # [roots], one step
    launches = out["kernel_runs"]["launches"]
    teps = m_cc[None, :] / (bfs_ms * 1e-3)
    hmean = teps.size / np.sum(1.0 / teps) / 1e9
    whole = m_cc.sum() * steps / out["wall"] / 1e9
    s = dict(gteps_wall=whole, gteps_hmean=hmean, ms_per_step=out["wall"] * 1e3 / steps,
             mean_bfs_ms=float(bfs_ms.mean()), level_launches=int(launches.sum()),
             mean_launch_ms=float(kern_ms.sum() / launches.sum()))
    if "levels" in out:
        iters = out["iterations"]
        per_root = np.array([algorithmic_bytes(out["levels"], i, int(iters[i]), semi, n, units)
                             for i in range(len(roots))])
        bytes_per_step = per_root.sum()
        kernel_s = kern_ms.sum() / 1e3
        achieved = bytes_per_step / kernel_s / 1e9
        s.update(bytes_per_launch=float(bytes_per_step / launches.sum()),
                 achieved_gbs=achieved, frac=achieved / HBM_PEAK_GBS,
                 cells_per_bfs=float(np.mean([out["levels"]["active_cells"][i][:iters[i]].sum()
                                              for i in range(len(roots))])))
    return s


def same_outputs(a, b) -> bool:
    """Whether two BFS results of the same roots agree element by element
    (distances, parents, iteration counts), compared on the device."""
    import torch
    ok = torch.equal(a.dist, b.dist) and np.array_equal(a.iterations, b.iterations)
    if a.parent is not None or b.parent is not None:
        ok = ok and a.parent is not None and b.parent is not None and \
            torch.equal(a.parent, b.parent)
    return bool(ok)


def _events_ms(torch, fn, reps=3):
    """Median wall time of fn() on the current stream, by torch events."""
    out = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b))
    return float(np.median(out))


def storage_report(ss, e, sigmas) -> dict:
    """Words (4 B) of each representation of Table "sizes", from the built
    SlimSell layout (E directed entries, P padding cells, n_c chunks):
    SlimSell col + cs + cl = E + P + 2 n_c; Sell-C-sigma pads val as well as col,
    2(E + P) + 2 n_c; CSR val + col + row = 2E + n; AL = E + n."""
    out = {}
    for sg in sigmas:
        L = ss.layout_build(e.src, e.dst, e.n, sigma=sg, arrays=False)
        E, P, nc, n = L.entries, L.cells - L.entries, L.n_chunks, e.n
        slim, sell = E + P + 2 * nc, 2 * (E + P) + 2 * nc
        out["n" if sg == 0 else str(sg)] = {
            "padding": int(P), "slimsell": int(slim), "sell_c_sigma": int(sell),
            "csr": int(2 * E + n), "al": int(E + n),
            "slimsell_vs_sell": round(slim / sell, 4), "slimsell_vs_al": round(slim / (E + n), 4)}
    return out


def bench_sell(ss, e, roots, torch) -> dict:
    """Speedup of SlimSell over Sell-C-sigma (val streamed beside col), per
    semiring, for a small and a large sorting scope (Table "slimsell")."""
    out = {}
    for sg in (1, 1 << 18):
        G = ss.Graph.from_edgelist(e, sigma=sg)
        row = {}
        for semi in ("boolean", "real", "tropical", "selmax"):
            t = {}
            for sell in (False, True):
                G.bfs(roots, semi, sell=sell)
                tot = 0.0
                for _ in range(2):
                    r = G.bfs(roots, semi, sell=sell, timing="bfs")
                    tot += float(r.runs["bfs_ms"].sum())
                torch.cuda.synchronize()
                t[sell] = tot / (2 * len(roots))
            row[semi] = {"slimsell_ms": round(t[False], 4), "sell_ms": round(t[True], 4),
                         "speedup": round(t[True] / t[False], 3)}
            log(f"sell sigma={sg} {semi}: {row[semi]}")
        G.close()
        out[f"sigma_{sg}"] = row
    return out


def bench_scale20(ss, graphgen, torch) -> dict:
    """R-MAT scale 20, sigma = 2^14, 16 roots one at a time: GTEPS per
    semiring, and the per-level shape of sel-max with and without SlimWork
    (active cells and time per level, one root)."""
    e = graphgen.rmat(20, 16, seed=1)
    roots = graphgen.pick_roots(e, 16, seed=1001)
    G = ss.Graph.from_edgelist(e, sigma=1 << 14)
    deg = torch.from_numpy(G.degrees().astype(np.int64)).cuda()
    out = {}
    for semi in ("tropical", "real", "boolean", "selmax"):
        G.bfs(roots, semi)
        r = G.bfs(roots, semi, timing="bfs")
        torch.cuda.synchronize()
        m_cc = ((r.dist >= 0).to(torch.int64) * deg[None, :]).sum(dim=1).cpu().numpy() / 2
        teps = m_cc / (r.runs["bfs_ms"] * 1e-3)
        out[semi] = {"gteps_hmean": round(float(len(teps) / np.sum(1.0 / teps) / 1e9), 3),
                     "mean_bfs_ms": round(float(np.mean(r.runs["bfs_ms"])), 4)}
        log(f"scale 20 {semi}: {out[semi]}")
    shape = {}
    for sw in (0, 1, 2):
        G.bfs(roots[:1], "selmax", slimwork=sw)
        r = G.bfs(roots[:1], "selmax", slimwork=sw, level_cap=32, timing=True)
        it = int(r.iterations[0])
        shape[f"slimwork_{sw}"] = {
            "active_cells": r.levels["active_cells"][0][:it].tolist(),
            "level_ms": [round(float(x), 4) for x in r.levels["ms"][0][:it]],
            "bfs_ms": round(float(r.runs["bfs_ms"][0]), 4)}
    out["selmax_levels_root0"] = shape
    G.close()
    return out


def dp_bytes(runs, n_pad: int, nonempty: int, reached) -> np.ndarray:
    """Algorithmic bytes of the DP transformation's sweep per root: col cells
    streamed (4 B), per processed row its degree read and its best-v write
    (8 B), cs + cl per processed chunk (8 B), the live test (row distance,
    4 B) over every non-empty chunk, one read of the codes (n/4 B) and one v
    read per reached vertex (4 B)."""
    return (4.0 * runs["dp_cells"] + 8.0 * C * runs["dp_chunks"] + 8.0 * runs["dp_chunks"]
            + 4.0 * C * nonempty + n_pad / 4.0 + 4.0 * np.asarray(reached, np.float64))


def bench_dp(G, roots, torch, nonempty: int) -> dict:
    """Mean BFS time per root without and with parents: sel-max yields them from
    the product, the other semirings by the DP transformation after the BFS
    (the paper's "No-DP" vs "DP"); and the roofline of the DP sweep kernel
    (tropical distances, event-timed sweep, counted cells)."""
    out = {}
    for semi in ("tropical", "real", "boolean", "selmax"):
        row = {}
        for dp in (False, True):
            kw = dict(dp=dp, want_parent=dp, want_real=False)
            G.bfs(roots, semi, **kw)
            tot = 0.0
            for _ in range(2):
                r = G.bfs(roots, semi, timing="bfs", **kw)
                tot += float(r.runs["bfs_ms"].sum())
            torch.cuda.synchronize()
            row["dp_ms" if dp else "no_dp_ms"] = round(tot / (2 * len(roots)), 4)
        out[semi] = row
        log(f"dp {semi}: {row}")
    r = G.bfs(roots, "tropical", dp=True, want_parent=True, timing=True, level_cap=1)
    torch.cuda.synchronize()
    reached = (r.dist >= 0).sum(dim=1).cpu().numpy()
    n_pad = (G.n + C - 1) // C * C
    b = dp_bytes(r.runs, n_pad, nonempty, reached)
    ms = r.runs["dp_ms"].astype(np.float64)
    achieved = float(b.sum() / (ms.sum() * 1e-3) / 1e9)
    out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "traffic": measured_traffic("level_kernel<dp>"),
                       "kernel": "level_kernel<dp>", "bytes_per_launch": round(float(b.mean())),
                       "mean_launch_ms": round(float(ms.mean()), 5),
                       "cells_per_launch": round(float(r.runs["dp_cells"].mean()))}
    log(f"dp roofline: {out['roofline']}")
    return out


def batched_bytes(levels: dict, iters: int, n_pad: int, units: int, pairs: int) -> float:
    """Algorithmic bytes of one batched BFS (64-bit masks): per level the col
    cells streamed (4 B), per processed row its visited mask read and its new
    frontier mask written (16 B), cs + cl per processed chunk (8 B), each work
    unit's descriptor and chunk flag (UNIT_BYTES), one read of the gathered
    masks (8 B per row) and a visited-mask write per row that gained bits
    (8 B); plus one 2-byte level record per (vertex, root) reached."""
    cells = levels["active_cells"][:iters].astype(np.float64)
    chunks = levels["active_chunks"][:iters].astype(np.float64)
    disc = levels["discovered"][:iters].astype(np.float64)
    per_level = (4.0 * cells + 16.0 * C * chunks + 8.0 * chunks + UNIT_BYTES * units
                 + 8.0 * n_pad + 8.0 * disc)
    return float(per_level.sum() + 2.0 * pairs)


def bench_batched(ss, graphgen, torch, checks: dict) -> dict:
    """64 roots in one boolean SpMM vs 64 plain runs (R-MAT s21), and 256
    Erdos-Renyi graphs (n log-uniform in [2^10, 2^18], mean degree 8-64) in one
    union solved by one level loop.  Host copies of the outputs (all 64 slots
    of s21, two slots of every ER graph) go to `checks` for the oracle."""
    e = graphgen.rmat(21, 16, seed=1)
    roots = graphgen.pick_roots(e, 64, seed=1004)
    G = ss.Graph.from_edgelist(e, sigma=0)
    deg = torch.from_numpy(G.degrees().astype(np.int64)).cuda()
    G.bfs_batch(roots[None, :])
    t_batch = _events_ms(torch, lambda: G.bfs_batch(roots[None, :]))
    dist, _, _, _ = G.bfs_batch(roots[None, :])
    d = dist.view(64, -1)
    m_cc = float(((d >= 0).to(torch.int64) * deg[None, :]).sum() // 2)
    checks["batched_rmat_s21"] = [(e, roots, d.cpu().numpy())]
    # roofline of the batched level kernel: per-level counters and events
    _, it_b, lv, rs = G.bfs_batch(roots[None, :], level_cap=64, timing=True)
    torch.cuda.synchronize()
    pairs = int((d >= 0).sum().item()) - 64
    deg_h = G.degrees()
    units_b = work_units(deg_h, G.get_tune()["split_len"])
    n_pad_b = (G.n + C - 1) // C * C
    bb = batched_bytes(lv, it_b, n_pad_b, units_b, pairs)
    launches = int(rs["launches"])
    kms = float(rs["kernel_ms"])
    achieved_b = bb / (kms * 1e-3) / 1e9
    roof_b = {"bound": "hbm", "achieved": round(achieved_b, 1), "peak": HBM_PEAK_GBS,
              "unit": "GB/s", "frac": round(achieved_b / HBM_PEAK_GBS, 4),
              "traffic": measured_traffic("level_kernel<batch>"), "kernel": "level_kernel<batch>",
              "bytes_per_launch": round(bb / launches), "mean_launch_ms": round(kms / launches, 5),
              "levels": int(it_b), "launches": launches}
    log(f"batched roofline: {roof_b}")
    G.bfs(roots, "selmax")
    t_plain = _events_ms(torch, lambda: G.bfs(roots, "selmax"), reps=2)
    G.bfs(roots, "boolean")
    t_bool = _events_ms(torch, lambda: G.bfs(roots, "boolean"), reps=2)
    G.close()
    log(f"batched s21: {t_batch:.2f} ms vs 64 sel-max {t_plain:.2f} ms, boolean {t_bool:.2f} ms")
    out = {"rmat_s21_64_roots": {
        "batched_ms": round(t_batch, 3), "plain_selmax_ms": round(t_plain, 3),
        "plain_boolean_ms": round(t_bool, 3), "gteps_batched": round(m_cc / t_batch / 1e6, 3),
        "gteps_plain_selmax": round(m_cc / t_plain / 1e6, 3),
        "speedup_vs_selmax": round(t_plain / t_batch, 2), "roofline": roof_b}}
    t = time.perf_counter()
    graphs = graphgen.er_set(256, seed=3)
    Gm = ss.Graph.from_many(graphs)
    build = time.perf_counter() - t
    R = np.full((256, 64), -1, np.int32)
    for i, g in enumerate(graphs):
        rr = graphgen.pick_roots(g, 64, seed=5000 + i)
        R[i, :len(rr)] = rr
    Gm.bfs_batch(R)
    t_many = _events_ms(torch, lambda: Gm.bfs_batch(R))
    Gm.bfs_batch(R, persistent=True)
    t_many_p = _events_ms(torch, lambda: Gm.bfs_batch(R, persistent=True))
    t = time.perf_counter()
    at = Gm.autotune(R, batched=True, repeats=1, force=True)
    tune_s = time.perf_counter() - t
    Gm.bfs_batch(R)
    t_many_t = _events_ms(torch, lambda: Gm.bfs_batch(R))
    Gm.bfs_batch(R, persistent=True)
    t_many_tp = _events_ms(torch, lambda: Gm.bfs_batch(R, persistent=True))
    dist, iters, _, _ = Gm.bfs_batch(R)
    ns, off = Gm.parts()
    degm = torch.from_numpy(Gm.degrees().astype(np.int64)).cuda()
    edges = 0.0
    dd = dist
    sample = []
    for i in range(256):
        blk = dd[64 * off[i]: 64 * (off[i] + ns[i])].view(64, int(ns[i]))
        edges += float(((blk >= 0).to(torch.int64) * degm[off[i]:off[i] + ns[i]][None, :]).sum() // 2)
        used = int((R[i] >= 0).sum())
        slots = sorted({0, used - 1})
        sample.append((graphs[i], R[i][slots], blk[slots].cpu().numpy()))
    checks["batched_er_256"] = sample
    Gm.close()
    log(f"256 ER graphs: {t_many:.2f} ms (persistent {t_many_p:.2f}, autotuned {t_many_t:.2f} / "
        f"{t_many_tp:.2f}), {iters} levels, build {build:.1f}s")
    forms = {"launch_per_level": t_many, "persistent": t_many_p,
             "autotuned_launch_per_level": t_many_t, "autotuned_persistent": t_many_tp}
    out["er_256_graphs"] = {"vertices": int(ns.sum()), "roots": int((R >= 0).sum()),
                            "levels": int(iters), "tune": at["best"], "tune_s": round(tune_s, 1),
                            "build_s": round(build, 1),
                            "ms": {k: round(v, 3) for k, v in forms.items()},
                            "gteps": {k: round(edges / v / 1e6, 3) for k, v in forms.items()},
                            "fastest_form": min(forms, key=forms.get)}
    return out


def bench_learned(ss, graphgen, torch) -> dict:
    """Learned per-level schedule vs the fixed heuristic vs each forced variant,
    total BFS time over the roots (R-MAT s24; 4096^2 grid with 5% of edges
    removed).  The model was trained on timings of the scale-12..22 graphs."""
    from paper_2010_09913_amd import scheduler
    path = scheduler.DEFAULT_MODEL
    if not os.path.exists(path):
        return {"skipped": "no trained model at " + os.path.relpath(path, ROOT)}
    ss.sched_load(np.load(path))
    out = {"model": os.path.relpath(path, ROOT)}
    cases = [("rmat_s24", lambda: graphgen.rmat(24, 16, seed=1), 8, 1005, None),
             ("grid_4096_cut5", lambda: graphgen.grid(4096, 4096, 0.05, seed=5), 4, 1005, 1)]
    for name, make, nroots, seed, slow_roots in cases:
        e = make()
        roots = graphgen.pick_roots(e, nroots, seed=seed)
        G = ss.Graph.from_edgelist(e, sigma=0)
        res = {}
        first = None  # outputs of the first root under the first mode
        agree = True
        for mode in ["learned", "heuristic", "pull", "pull-split256", "pull-split1024", "push",
                     "learned+persistent", "heuristic+persistent", "push+persistent"]:
            sched, pers = mode.split("+")[0], mode.endswith("+persistent")
            rr = roots
            if slow_roots and mode.startswith("pull"):
                rr = roots[:slow_roots]   # pull-only on the grid is O(levels x n): few roots
            x0 = G.bfs([int(rr[0])], "selmax", schedule=sched, persistent=pers)
            if first is None:
                first = x0
            else:
                agree = agree and same_outputs(first, x0)
            tot = 0.0
            for r in rr:
                x = G.bfs([int(r)], "selmax", schedule=sched, timing="bfs", persistent=pers)
                tot += float(x.runs["bfs_ms"][0])
            res[mode] = round(tot / len(rr), 3)
            log(f"{name} {mode}: {tot / len(rr):.2f} ms per BFS")
        G.close()
        res["forms_agree"] = bool(agree)
        res["learned_vs_heuristic"] = round(res["heuristic"] / res["learned"], 3)
        res["best_forced"] = min(("pull", "pull-split256", "pull-split1024", "push"),
                                 key=lambda m: res[m])
        out[name] = {"ms_per_bfs": res, "roots": int(len(roots))}
    ss.sched_clear()
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--roots", type=int, default=64)
    ap.add_argument("--split", type=int, default=-1, help="SlimChunk split length (-1 = default)")
    ap.add_argument("--semiring", default="selmax",
                    choices=["tropical", "real", "boolean", "selmax"])
    ap.add_argument("--cpu-roots", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the split sweep and ER graph")
    ap.add_argument("--only-timed", action="store_true",
                    help="warm-up and timed steps only (for profiler runs)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched SpMM comparison")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates the HBM byte counters)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-schedule comparison (R-MAT s24, 4096^2 grid)")
    ap.add_argument("--profile-summary", action="store_true",
                    help="summarise rocprofv3 output into profiles/ (no GPU needed)")
    ap.add_argument("--kernel", default="level_kernel<selmax>", choices=sorted(PROFILES),
                    help="kernel --profile-summary summarises")
    ap.add_argument("--only", choices=["batched", "dp", "push"],
                    help="run one form alone, warm-up and timed steps only (for profiler "
                         "runs): batched = 64 roots of R-MAT s21 in one SpMM; dp = tropical "
                         "BFS with parents by the DP transformation, 16 roots of R-MAT s22; "
                         "push = sel-max with the forced push schedule, 16 roots of R-MAT s22")
    for name in ("trace", "fetch", "write", "copy-fetch", "copy-write"):
        ap.add_argument("--" + name, help="rocprofv3 output directory")
        ap.add_argument("--cmd-" + name, default="", help="the command that produced it")
    ap.add_argument("--pmc", action="append", default=[],
                    help="rocprofv3 --pmc output directory of stall/cache counters (repeatable)")
    ap.add_argument("--cmd-pmc", action="append", default=[], help="the commands that produced them")
    ap.add_argument("--out-dir", default=os.path.join(ROOT, "profiles"),
                    help="where --profile-summary writes")
    args = ap.parse_args()
    if args.profile_summary:
        return profile_summary(args)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import torch

    import graphgen
    import paper_2010_09913_amd as ss

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": src.numel() * 4,
                          "copy_probe_bytes_written": dst.numel() * 4, "launches": 4}))
        return 0
    semi = args.semiring
    if args.only:
        return run_only(args, ss, graphgen, torch)

    t = time.perf_counter()
    e = graphgen.rmat(args.scale, 16, seed=1)
    roots = graphgen.pick_roots(e, args.roots, seed=1002)
    log(f"generated {e.name}: {e.m} tuples in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    G = ss.Graph.from_edgelist(e, sigma=0)
    build_s = time.perf_counter() - t
    info = G.info()
    deg = G.degrees()
    deg_t = torch.from_numpy(deg.astype(np.int64)).cuda()
    log(f"built SlimSell layout in {build_s:.1f}s: {info}")
    nonempty = nonempty_chunks(deg, info["chunks"])

    def units_of(split):
        return work_units(deg, G.get_tune()["split_len"] if split == -1 else split)

    out = run_workload(ss, G, roots, semi, args.split, args.steps, args.warmup, deg_t,
                       count_pass=not args.only_timed)
    s = summarise(out, roots, semi, e.n, units_of(args.split), args.steps)
    log(f"main: {s}")

    result = {
        "metric": "GTEPS (whole job) and % of HBM peak, SlimSell BFS, R-MAT s22",
        "value": round(s["gteps_wall"], 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(s["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded R-MAT generator)",
        "config": {
            "workload": f"R-MAT scale {args.scale} ef16 (.57/.19/.19) seed 1, {semi} semiring, "
                        f"C=64, sigma=n, SlimWork on, SlimChunk split "
                        f"{'default' if args.split == -1 else args.split}, "
                        f"{len(roots)} roots (seed 1002), one BFS per root per step",
            "n": e.n, "undirected_edges": int(info["entries"] // 2),
            "cells": int(info["cells"]), "padding": int(info["padding"]),
            "max_degree": int(info["max_cl"]), "roots": int(len(roots)),
            "parallelism": "single GPU",
        },
        "gteps_hmean": round(s["gteps_hmean"], 4),
        "mean_bfs_ms": round(s["mean_bfs_ms"], 4),
        "build_s": round(build_s, 2),
    }
    if "achieved_gbs" in s:
        result["roofline"] = {
            "bound": "hbm", "achieved": round(s["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(s["frac"], 4),
            "traffic": measured_traffic(f"level_kernel<{semi}>"),
            "kernel": f"level_kernel<{semi}>",
            "bytes_per_launch": round(s["bytes_per_launch"]),
            "mean_launch_ms": round(s["mean_launch_ms"], 5),
        }

    if not args.only_timed and not args.no_extra:
        # the same workload with the direction-aware schedules and the autotuner
        forms = {}
        for sched, pers in (("none", True), ("heuristic", False), ("heuristic", True),
                            ("learned", False), ("learned", True)):
            if sched == "learned":
                from paper_2010_09913_amd import scheduler
                if not os.path.exists(scheduler.DEFAULT_MODEL):
                    continue
                ss.sched_load(np.load(scheduler.DEFAULT_MODEL))
            o2 = run_workload(ss, G, roots, semi, args.split, max(1, args.steps // 2), 1, deg_t,
                              count_pass=False, schedule=sched, persistent=pers)
            s2 = summarise(o2, roots, semi, e.n, units_of(args.split), max(1, args.steps // 2))
            name = ("pull" if sched == "none" else sched + "_schedule") + (
                "_persistent" if pers else "")
            forms[name] = {"gteps": round(s2["gteps_wall"], 4),
                           "gteps_hmean": round(s2["gteps_hmean"], 4),
                           "mean_bfs_ms": round(s2["mean_bfs_ms"], 4),
                           "same_outputs": same_outputs(out["result"], o2["result"])}
            log(f"{name}: {s2}")
        ss.sched_clear()
        default_tune = G.get_tune()
        t = time.perf_counter()
        at = G.autotune(roots[:8], semi, repeats=2, force=True)
        tune_s = time.perf_counter() - t
        o2 = run_workload(ss, G, roots, semi, -1, max(1, args.steps // 2), 1, deg_t)
        s2 = summarise(o2, roots, semi, e.n, units_of(-1), max(1, args.steps // 2))
        forms["autotuned"] = {"gteps": round(s2["gteps_wall"], 4),
                              "frac": round(s2.get("frac", 0.0), 4), "tune": at["best"],
                              "configs_timed": at["evaluated"], "tune_s": round(tune_s, 1)}
        log(f"autotuned {at}: {s2}")
        G.set_tune(**default_tune)
        result["forms"] = forms
        sweep = {}
        for split in (0, 256, 1024, 4096):
            o2 = run_workload(ss, G, roots, semi, split, max(1, args.steps // 2), 1, deg_t)
            s2 = summarise(o2, roots, semi, e.n, units_of(split), max(1, args.steps // 2))
            sweep[str(split)] = {"gteps": round(s2["gteps_wall"], 4),
                                 "frac": round(s2.get("frac", 0.0), 4)}
            log(f"split {split}: {s2}")
        result["split_sweep"] = sweep
        result["dp"] = bench_dp(G, roots[:16], torch, nonempty)
        G.close()
        result["slimsell_vs_sell"] = bench_sell(ss, e, roots[:8], torch)
        result["storage_words"] = {"rmat_s22": storage_report(ss, e, (1, 64, 2048, 1 << 14, 0))}
        # Erdos-Renyi graph of the same size (mean degree 32)
        er = graphgen.er(1 << args.scale, 16 << args.scale, seed=2)
        er_roots = graphgen.pick_roots(er, args.roots, seed=1003)
        Ge = ss.Graph.from_edgelist(er, sigma=0)
        deg_e = torch.from_numpy(Ge.degrees().astype(np.int64)).cuda()
        sp = Ge.get_tune()["split_len"] if args.split == -1 else args.split
        ne = work_units(Ge.degrees(), sp)
        oe = run_workload(ss, Ge, er_roots, semi, args.split, max(1, args.steps // 2), 1, deg_e)
        se = summarise(oe, er_roots, semi, er.n, ne, max(1, args.steps // 2))
        log(f"er: {se}")
        result["storage_words"]["er_2^22"] = storage_report(ss, er, (1, 2048, 0))
        result["er_2^22_deg32"] = {"gteps": round(se["gteps_wall"], 4),
                                   "gteps_hmean": round(se["gteps_hmean"], 4),
                                   "frac": round(se.get("frac", 0.0), 4)}
        Ge.close()

    if not args.only_timed and not args.no_extra:
        result["rmat_s20_sigma2^14"] = bench_scale20(ss, graphgen, torch)
    checks = {"headline": [(e, roots, out["result"])]}
    if not args.only_timed and not args.no_batch:
        result["batched"] = bench_batched(ss, graphgen, torch, checks)
    if not args.only_timed and not args.no_learned:
        result["learned_schedule"] = bench_learned(ss, graphgen, torch)

    if not args.no_cpu and not args.only_timed:
        cpu_leg(args, e, roots, result, checks)
    print(json.dumps(result), flush=True)
    return 0


def run_only(args, ss, graphgen, torch) -> int:
    """One form alone (warm-up, then the timed steps), for profiler runs."""
    if args.only == "batched":
        e = graphgen.rmat(21, 16, seed=1)
        roots = graphgen.pick_roots(e, 64, seed=1004)
        G = ss.Graph.from_edgelist(e, sigma=0)
        step = lambda: G.bfs_batch(roots[None, :])  # noqa: E731
    else:
        e = graphgen.rmat(args.scale, 16, seed=1)
        roots = graphgen.pick_roots(e, 16, seed=1002)
        G = ss.Graph.from_edgelist(e, sigma=0)
        if args.only == "dp":
            step = lambda: G.bfs(roots, "tropical", dp=True)  # noqa: E731
        else:
            step = lambda: G.bfs(roots, "selmax", schedule="push")  # noqa: E731
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / max(args.steps, 1)
    G.close()
    print(json.dumps({"only": args.only, "steps": args.steps, "ms_per_step": round(ms, 4)}),
          flush=True)
    return 0


def _check_roots(oracle, g, roots, dist, parent, iterations, pool):
    """Roots whose distances (and parents, iteration counts where given)
    differ from the oracle's queue BFS and max-ID parent pass."""
    def one(i):
        r = int(roots[i])
        d = oracle.bfs(g, r)
        ok = np.array_equal(dist[i], d)
        if parent is not None:
            ok = ok and np.array_equal(parent[i], oracle.parents_max(g, r, d))
        if iterations is not None:
            ok = ok and int(iterations[i]) == int(d.max()) + 1
        return ok
    return [int(roots[i]) for i, ok in enumerate(pool.map(one, range(len(roots)))) if not ok]


def cpu_leg(args, e, roots, result, checks) -> None:
    """The CPU leg: the oracle timed on a bounded sample of the headline
    workload (cpu_baseline, one thread; cpu_baseline_all_cores), then every
    timed output kept in `checks` compared element by element with it
    (validated): all headline roots, all 64 batched slots of R-MAT s21 and
    two slots of each of the 256 Erdos-Renyi graphs."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    t = time.perf_counter()
    g = oracle.csr_from_edgelist(e)
    log(f"oracle CSR in {time.perf_counter() - t:.1f}s")
    sample = roots[: args.cpu_roots]
    rates = []
    t_all = time.perf_counter()
    for r in sample:
        t = time.perf_counter()
        d = oracle.bfs(g, int(r))
        oracle.parents_max(g, int(r), d)
        dt = time.perf_counter() - t
        rates.append(oracle.component_edges(g, d) / dt)
    cpu_s = time.perf_counter() - t_all
    rates = np.array(rates)
    result["cpu_baseline"] = {
        "value": round(float(len(rates) / np.sum(1.0 / rates) / 1e9), 5),
        "unit": "GTEPS", "cores": 1, "kind": "oracle",
        "sample": f"{len(sample)} of the {len(roots)} roots: FIFO-queue BFS + max-ID parent "
                  f"pass (the sel-max outputs), 1 thread, {cpu_s:.1f}s total",
    }
    # the level-synchronous OpenMP oracle on all host threads (distances)
    rates = []
    t_all = time.perf_counter()
    for r in sample:
        t = time.perf_counter()
        d = oracle.bfs_omp(g, int(r))
        dt = time.perf_counter() - t
        rates.append(oracle.component_edges(g, d) / dt)
    rates = np.array(rates)
    result["cpu_baseline_all_cores"] = {
        "value": round(float(len(rates) / np.sum(1.0 / rates) / 1e9), 5),
        "unit": "GTEPS", "cores": oracle.threads(), "kind": "oracle",
        "cpu": cpu_model(),
        "sample": f"the same {len(sample)} roots: level-synchronous top-down OpenMP BFS "
                  f"(distances), {time.perf_counter() - t_all:.1f}s total",
    }
    # validation of the timed outputs (the oracle calls release the GIL, so a
    # thread pool runs them in parallel)
    t = time.perf_counter()
    report, bad = {}, []
    with ThreadPoolExecutor(max_workers=16) as pool:
        for (ee, rr, res) in checks.get("headline", []):
            par = res.parent.cpu().numpy() if res.parent is not None else None
            wrong = _check_roots(oracle, g, rr, res.dist.cpu().numpy(), par, res.iterations, pool)
            report["headline_roots"] = int(len(rr))
            bad += [("headline", r) for r in wrong]
        del g
        for (ee, rr, dist) in checks.get("batched_rmat_s21", []):
            gb = oracle.csr_from_edgelist(ee)
            wrong = _check_roots(oracle, gb, rr, dist, None, None, pool)
            report["batched_rmat_s21_slots"] = int(len(rr))
            bad += [("batched_rmat_s21", r) for r in wrong]
            del gb
        n_er = 0
        for (ee, rr, dist) in checks.get("batched_er_256", []):
            gi = oracle.csr_from_edgelist(ee)
            wrong = _check_roots(oracle, gi, rr, dist, None, None, pool)
            n_er += len(rr)
            bad += [("batched_er_256", ee.name, r) for r in wrong]
        if n_er:
            report["batched_er_256_slots"] = n_er
    forms_ok = all(f.get("same_outputs", True) for f in result.get("forms", {}).values())
    for case in result.get("learned_schedule", {}).values():
        if isinstance(case, dict) and "ms_per_bfs" in case:
            forms_ok = forms_ok and case["ms_per_bfs"].get("forms_agree", True)
    report["other_forms_equal_to_checked_outputs"] = bool(forms_ok)
    report["mismatches"] = [list(map(str, b)) for b in bad[:16]]
    report["seconds"] = round(time.perf_counter() - t, 1)
    result["validated"] = not bad and forms_ok
    result["validation"] = report
    log(f"validation: {report}")


if __name__ == "__main__":
    sys.exit(main())
