"""Benchmark: A-sources matched per second on the 10M x 10M full-sky cross-match.

One step = one hlc_xmatch call (keygen, both radix sorts, layouts, B ranges,
filter, certification, output packing, count read-back) on FP64 inputs
already resident in HBM. The headline value uses the FP32+recheck filter;
the plain FP64 filter is timed beside it. Also measured (the "forms" field):
the batched form on 10,000 cone jobs against one plain FP64 call per job,
the emulated HEALPix + quad-direction partition (completeness loss against
the exact pair set, and time), the streaming form on 400M x 100M held in
pinned host memory (PCIe-inclusive) and the 20M x 20M precision stress at
r = 0.5, 1 and 5 arcsec. Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms xmatch,batch,quad,stream,stress]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per launch of the match (filter) kernel: the working
# layout of every A source and every B entry (halo copies included) read
# once, which is what the method must move:
#   FP64 form: 28 B per entry (x, y, z f64 + u32 index).
#   FP32 form: 16 B per entry (x, y, z f32 + u32 index), plus 32 B per
#              candidate inside the certified band (its FP64 re-read).
# What the kernel actually moves (its 32-B in-place A records, one cache
# line each, and its staged candidates) is the measured `traffic`.
MATCH_BYTES = {
    "fp64": lambda na, nbh, nband: 28 * (na + nbh),
    "fp32": lambda na, nbh, nband: 16 * (na + nbh) + 32 * nband,
}
# Whole-call canonical bytes: FP64 (ra, dec) of every source read once and
# every pair written once.
CALL_BYTES = lambda na, nb, npairs: 16 * (na + nb) + 16 * npairs
# VALU issue cycles per second of the whole chip (256 CUs x 4 SIMDs x 2.4 GHz)
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9

# HBM traffic of the filter kernel, measured with rocprofv3 counters
# (FETCH_SIZE and WRITE_SIZE passes, scaled by a 1 GiB copy) and recorded
# with a hash of the kernel sources it was measured on; reported only while
# the sources are unchanged.
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "hbm_traffic_k_filter_fullsky_10Mx10M_2arcsec.md")
KERNEL_SOURCES = ["match.hip", "hlc_device.hpp", "hlc_kernels.hpp"]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2301_07331_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """Bytes per launch from the committed record, or None if the kernel sources changed since."""
    try:
        text = open(TRAFFIC_RECORD).read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines() if line.startswith(("traffic_bytes", "source_sha256")))
    if fields.get("source_sha256", "").strip() != kernel_sources_sha256():
        return None
    return float(fields["traffic_bytes"])


def traffic_from_pmc(fetch_dir, write_dir, kernel="k_filter<true>"):
    """HBM bytes per launch of `kernel` from two rocprofv3 --pmc runs of
    `bench.py --copy-calibration` (FETCH_SIZE, WRITE_SIZE in KiB per
    dispatch), each scaled so that the 1 GiB device copy reads / writes 1 GiB."""
    import csv

    def per_kernel(d, counter):
        rows = [r for r in csv.DictReader(open(os.path.join(d, "p_counter_collection.csv")))
                if r["Counter_Name"] == counter]
        target = [float(r["Counter_Value"]) for r in rows if kernel in r["Kernel_Name"]]
        copies = [float(r["Counter_Value"]) for r in rows
                  if "hlc" not in r["Kernel_Name"] and ("copy" in r["Kernel_Name"].lower()
                                                        or "elementwise" in r["Kernel_Name"].lower())]
        return sum(target) / len(target), max(copies)

    f_k, f_copy = per_kernel(fetch_dir, "FETCH_SIZE")
    w_k, w_copy = per_kernel(write_dir, "WRITE_SIZE")
    gib_kib = float(1 << 20)
    fetch = f_k * (gib_kib / f_copy) * 1024.0
    write = w_k * (gib_kib / w_copy) * 1024.0
    return {"fetch_bytes": fetch, "write_bytes": write, "traffic_bytes": fetch + write,
            "fetch_scale": gib_kib / f_copy, "write_scale": gib_kib / w_copy,
            "source_sha256": kernel_sources_sha256()}


def _csvs(d, suffix):
    import glob
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def short_kernel(name):
    """'void hlc::(anonymous namespace)::k_filter<true>(hlc::MatchArgs, ...)' -> 'k_filter<true>'."""
    import re
    head = name.split("(hlc::")[0].split("(unsigned")[0].split("(double")[0].split("(float")[0]
    head = re.sub(r"^void ", "", head)
    head = head.split("::")[-1] if "<" not in head else re.sub(r"^.*::(?=[^:<]*<)", "", head)
    return head.strip()


def pmc_summary(ktrace_dir, pmc_dirs):
    """Per-kernel table from one rocprofv3 --kernel-trace --stats run and
    several --pmc runs of the same command with --copy-calibration: average
    duration, HBM bytes fetched and written per dispatch (FETCH_SIZE and
    WRITE_SIZE in KiB, each scaled by what it reads for the 1 GiB device
    copy), achieved GB/s of that traffic, and per-wave instruction counts,
    wait and LDS-conflict figures where the passes hold them. Markdown."""
    import csv
    from collections import defaultdict
    dur, calls = {}, {}
    for f in _csvs(ktrace_dir, "kernel_stats.csv"):
        for r in csv.DictReader(open(f)):
            if "hlc" not in r["Name"]:
                continue
            dur[short_kernel(r["Name"])] = float(r["AverageNs"]) * 1e-3
            calls[short_kernel(r["Name"])] = int(r["Calls"])
    vals = defaultdict(lambda: defaultdict(list))  # kernel -> counter -> per-dispatch values
    copy = defaultdict(list)
    for d in pmc_dirs:
        for f in _csvs(d, "counter_collection.csv"):
            for r in csv.DictReader(open(f)):
                k = r["Kernel_Name"]
                v = float(r["Counter_Value"])
                c = r["Counter_Name"]
                if "hlc" not in k and ("copy" in k.lower() or "elementwise" in k.lower()):
                    copy[c].append(v)
                elif "hlc" in k:
                    vals[short_kernel(k)][c].append(v)
    gib_kib = float(1 << 20)
    scale = {c: gib_kib / max(copy[c]) for c in ("FETCH_SIZE", "WRITE_SIZE") if copy.get(c)}
    mean = lambda x: sum(x) / len(x) if x else None
    rows = []
    for k in sorted(set(vals) | set(dur), key=lambda k: -(dur.get(k) or 0)):
        c = vals[k]
        f = mean(c.get("FETCH_SIZE", []))
        w = mean(c.get("WRITE_SIZE", []))
        fb = f * scale["FETCH_SIZE"] * 1024 if f is not None and "FETCH_SIZE" in scale else None
        wb = w * scale["WRITE_SIZE"] * 1024 if w is not None and "WRITE_SIZE" in scale else None
        t = dur.get(k)
        waves = mean(c.get("SQ_WAVES", []))
        per_wave = lambda n: (mean(c[n]) / waves) if waves and c.get(n) else None
        wait = (mean(c["SQ_WAIT_ANY"]) / mean(c["SQ_WAVE_CYCLES"])
                if c.get("SQ_WAIT_ANY") and c.get("SQ_WAVE_CYCLES") and mean(c["SQ_WAVE_CYCLES"]) else None)
        # share of the chip's VALU issue capacity over the kernel's duration:
        # 4 cycles per wave64 VALU instruction, 1024 SIMDs at 2.4 GHz
        valu_busy = (4.0 * mean(c["SQ_INSTS_VALU"]) / (t * 1e-6 * VALU_ISSUE_PER_S)
                     if c.get("SQ_INSTS_VALU") and t else None)
        gbs = ((fb or 0) + (wb or 0)) / (t * 1e-6) / 1e9 if t and (fb is not None or wb is not None) else None
        rows.append((k, calls.get(k), t, fb, wb, gbs, waves, per_wave("SQ_INSTS_VALU"), per_wave("SQ_INSTS_VMEM_RD"),
                     per_wave("SQ_INSTS_VMEM_WR"), per_wave("SQ_INSTS_LDS"), mean(c.get("SQ_LDS_BANK_CONFLICT", [])),
                     wait, valu_busy))
    fmt = lambda x, p="{:.3g}": "-" if x is None else p.format(x)
    out = ["| kernel | calls | avg us | fetched B | written B | GB/s (fetch+write) | frac of 8 TB/s | waves | VALU/wave "
           "| VMEM rd/wave | VMEM wr/wave | LDS/wave | LDS bank-conflict cycles | wait/wave-cycles | VALU issue share |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for (k, nc, t, fb, wb, gbs, waves, valu, vr, vw, lds, bc, wait, vb) in rows:
        out.append(f"| {k} | {fmt(nc, '{:d}')} | {fmt(t, '{:.1f}')} | {fmt(fb)} | {fmt(wb)} | {fmt(gbs, '{:.0f}')} | "
                   f"{fmt(gbs / HBM_PEAK_GBS if gbs else None, '{:.3f}')} | {fmt(waves, '{:.0f}')} | {fmt(valu, '{:.0f}')} | "
                   f"{fmt(vr, '{:.1f}')} | {fmt(vw, '{:.1f}')} | {fmt(lds, '{:.1f}')} | {fmt(bc, '{:.3g}')} | "
                   f"{fmt(wait, '{:.2f}')} | {fmt(vb, '{:.2f}')} |")
    out.append("")
    out.append(f"copy scaling: " + ", ".join(f"{c} x{v:.4f}" for c, v in scale.items()))
    return "\n".join(out)


def call_timeline(ktrace_dir, call, first="k_extent_sample", with_kernel=None):
    """The kernels of one call, in start order, from a rocprofv3
    --kernel-trace -f csv folder: queue, start and end (us from the call's
    first kernel) and duration. A call starts at each launch of `first` (the
    footprint sample of a single call; k_zero_u64 for the batched form);
    with `with_kernel` only the calls that launch a kernel of that name
    count. `call` indexes those calls from 0 (negative: from the last).
    Markdown."""
    import csv
    rows = []
    for f in _csvs(ktrace_dir, "kernel_trace.csv"):
        for r in csv.DictReader(open(f)):
            if "hlc" in r["Kernel_Name"]:
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r.get("Queue_Id", ""),
                             short_kernel(r["Kernel_Name"])))
    rows.sort()
    starts = [i for i, r in enumerate(rows) if r[3] == first] + [len(rows)]
    calls = [rows[a:b] for a, b in zip(starts[:-1], starts[1:])]
    if with_kernel:
        calls = [c for c in calls if any(r[3] == with_kernel for r in c)]
    if not -len(calls) <= call < len(calls):
        raise SystemExit(f"the trace holds {len(calls)} such calls")
    sel = calls[call]
    t0 = sel[0][0]
    out = ["| queue | start us | end us | us | kernel |", "|---|---|---|---|---|"]
    for (a, b, q, k) in sel:
        out.append(f"| {q} | {(a - t0) / 1e3:.1f} | {(b - t0) / 1e3:.1f} | {(b - a) / 1e3:.1f} | {k} |")
    return "\n".join(out)


def warm_up(call, calls, seconds=0.3):
    """Untimed calls: at least `calls` of them and at least `seconds` of them,
    so the GPU has left its idle clocks before the timed region."""
    import torch
    t0 = time.perf_counter()
    k = 0
    while k < calls or time.perf_counter() - t0 < seconds:
        call()
        k += 1
    torch.cuda.synchronize()


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--n", type=int, default=10_000_000, help="sources per catalogue")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-reps", type=int, default=3)
    p.add_argument("--precisions", default="fp32,fp64")
    p.add_argument("--zone-height", type=float, default=0.0, help="arcsec; 0 = automatic")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run a plain device copy of known size (for HBM counter scaling)")
    p.add_argument("--forms", default="xmatch,batch,quad,stream,stress",
                   help="xmatch (the headline, always run), batch (10,000 jobs), quad (paper-scheme "
                        "emulation), stream (400M x 100M from pinned host memory) and stress (20M x 20M "
                        "precision stress at r = 0.5, 1, 5 arcsec)")
    p.add_argument("--no-single-thread", action="store_true",
                   help="skip the single-thread oracle timings of the patch and full-sky workloads")
    p.add_argument("--pmc-summary", nargs="+", metavar="DIR",
                   help="print a per-kernel counter table from a rocprofv3 --kernel-trace --stats folder "
                        "followed by one or more --pmc folders, and exit")
    p.add_argument("--timeline", nargs="+", metavar="ARG",
                   help="KTRACE_DIR CALL [FIRST_KERNEL [WITH_KERNEL]]: print the kernels of one call (numbered "
                        "from 0, negative from the last; calls start at FIRST_KERNEL, default k_extent_sample, and "
                        "count only if they launch WITH_KERNEL) from a rocprofv3 --kernel-trace -f csv folder, "
                        "and exit")
    p.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                   help="print the filter kernel's HBM traffic from two rocprofv3 --pmc output folders and exit")
    return p.parse_args()


def bench_batch(hlc, torch, dev, steps, warmup):
    """The batched form on 10,000 cone jobs, FP32 and FP64, against one plain
    FP64 hlc_xmatch call per job (the same jobs, the same pair set)."""
    import numpy as np
    import synth
    t0 = time.time()
    b = synth.batch_jobs()
    jobs = [(int(b.a_off[j]), int(b.na[j]), int(b.b_off[j]), int(b.nb[j]), float(b.r_arcsec[j]))
            for j in range(b.njobs)]
    print(f"[bench] generated {b.njobs} jobs ({len(b.a_ra)} + {len(b.b_ra)} sources) in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    a_ra, a_dec, b_ra, b_dec = (torch.from_numpy(x).to(dev) for x in (b.a_ra, b.a_dec, b.b_ra, b.b_dec))
    cap = len(b.a_ra) // 2 + 1024
    out = torch.empty((cap, 2), dtype=torch.int32, device=dev)
    sep = torch.empty(cap, dtype=torch.float64, device=dev)
    cnt = torch.empty(len(jobs), dtype=torch.int64, device=dev)
    res = {}
    table = hlc.job_table(jobs)  # built once, as a caller repeating the batch would
    for name, prec in (("fp32", hlc.HLC_FP32_RECHECK), ("fp64", hlc.HLC_FP64)):
        for _ in range(max(1, warmup)):  # the first call tunes the zone-height factor
            st, n = hlc.hlc_xmatch_batch(table, a_ra, a_dec, b_ra, b_dec, out, sep, cnt, precision=prec)
            if st != hlc.HLC_OK:
                raise hlc.HLCError(st, "batch warmup")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st, n = hlc.hlc_xmatch_batch(table, a_ra, a_dec, b_ra, b_dec, out, sep, cnt, precision=prec)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        s_ = hlc.last_stats()
        res[name] = {"ms_per_call": ms, "a_sources_per_s": len(b.a_ra) / (ms * 1e-3), "pairs": int(n),
                     "tuned": {"zone_height_factor": s_["zone_height_arcsec"], "batch_tile": int(s_["batch_tile"]),
                               "batch_blocks_per_cu": int(s_["batch_blocks_per_cu"])}}
        print(f"[bench] batch {name}: {ms:.3f} ms/call, {n} pairs, tuned {res[name]['tuned']}", file=sys.stderr,
              flush=True)
        # the same call at the untuned defaults (factor 1, 1024-source tiles, 4 blocks per CU)
        dflt = {"zone_height_factor": 1.0, "batch_tile": 1024, "batch_blocks_per_cu": 4}
        for _ in range(max(1, warmup)):
            hlc.hlc_xmatch_batch(table, a_ra, a_dec, b_ra, b_dec, out, sep, cnt, precision=prec, tuning=dflt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st, nd = hlc.hlc_xmatch_batch(table, a_ra, a_dec, b_ra, b_dec, out, sep, cnt, precision=prec,
                                          tuning=dflt)
        torch.cuda.synchronize()
        msd = (time.perf_counter() - t0) / steps * 1e3
        if st != hlc.HLC_OK or nd != n:
            raise RuntimeError(f"batch {name} at the default configuration: status {st}, {nd} pairs vs {n}")
        res[name]["default_ms_per_call"] = msd
        print(f"[bench] batch {name} default configuration: {msd:.3f} ms/call", file=sys.stderr, flush=True)
    # plain FP64: one call per job
    jout = torch.empty((max(int(b.na.max()), 1024), 2), dtype=torch.int32, device=dev)
    jsep = torch.empty(jout.shape[0], dtype=torch.float64, device=dev)
    total = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (ao, na, bo, nb, r) in jobs:
        if na == 0 or nb == 0:
            continue
        st, n = hlc.hlc_xmatch(a_ra[ao:ao + na], a_dec[ao:ao + na], b_ra[bo:bo + nb], b_dec[bo:bo + nb], r,
                               jout, jsep, precision=hlc.HLC_FP64)
        if st == hlc.HLC_E_OVERFLOW:
            jout = torch.empty((n + 1024, 2), dtype=torch.int32, device=dev)
            jsep = torch.empty(n + 1024, dtype=torch.float64, device=dev)
            st, n = hlc.hlc_xmatch(a_ra[ao:ao + na], a_dec[ao:ao + na], b_ra[bo:bo + nb], b_dec[bo:bo + nb], r,
                                   jout, jsep, precision=hlc.HLC_FP64)
        if st != hlc.HLC_OK:
            raise hlc.HLCError(st, "per-job call")
        total += n
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    res["per_job_fp64"] = {"ms_per_call": ms, "a_sources_per_s": len(b.a_ra) / (ms * 1e-3), "pairs": int(total)}
    print(f"[bench] per-job FP64 loop: {ms:.1f} ms, {total} pairs", file=sys.stderr, flush=True)
    if not (res["fp32"]["pairs"] == res["fp64"]["pairs"] == total):
        raise RuntimeError(f"batched and per-job pair counts differ: {res}")
    res["workload"] = f"{b.njobs} cone jobs, {len(b.a_ra)} A + {len(b.b_ra)} B sources, r 0.5-3 arcsec"
    return res


def bench_stream(hlc, torch):
    """The streaming form on the 400M x 100M workload held in pinned host
    memory: wall time of one call including every host <-> device copy
    (PCIe-inclusive), with a sink that only counts the pairs it is handed."""
    import synth
    t0 = time.time()
    c = synth.large_pair()
    print(f"[bench] generated {c.name} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    def pinned(x):
        t = torch.empty(len(x), dtype=torch.float64, pin_memory=True)
        t.numpy()[:] = x
        return t

    arrs = [pinned(x) for x in (c.a_ra, c.a_dec, c.b_ra, c.b_dec)]
    na, nb, r, name_w = c.na, c.nb, c.r_arcsec, c.name
    del c
    res = {}
    for name, prec in (("fp32", hlc.HLC_FP32_RECHECK), ("fp64", hlc.HLC_FP64)):
        got = [0]

        def sink(p, s_, k):
            got[0] += k
            return 0

        secs = []
        for _ in range(2):  # the first call also sizes the library's streaming buffers
            got[0] = 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, n = hlc.hlc_xmatch_stream(*arrs, r, sink, precision=prec, ring_pairs=1 << 26)
            torch.cuda.synchronize()
            secs.append(time.perf_counter() - t0)
            if st != hlc.HLC_OK or got[0] != n:
                raise hlc.HLCError(st, "stream")
        sec = secs[-1]
        h2d = 16 * (na + nb)
        d2h = 16 * n
        res[name] = {"seconds": sec, "first_call_seconds": secs[0], "a_sources_per_s_pcie_inclusive": na / sec,
                     "pairs": int(n),
                     "h2d_bytes": h2d, "d2h_bytes": d2h, "link_gbs": (h2d + d2h) / sec / 1e9}
        print(f"[bench] stream {name}: {sec:.2f} s, {n} pairs", file=sys.stderr, flush=True)
    res["workload"] = f"{name_w}: {na} A x {nb} B in pinned host memory, r={r} arcsec"
    res["transfer_model"] = hlc.transfer_model()
    return res


def bench_stress(hlc, torch, dev, steps, warmup):
    """The precision-stress workload at full size (20M x 20M, 10,000 clumps,
    counterparts on [0.99 r, 1.01 r]) for r = 0.5, 1, 5 arcsec: FP32 + FP64
    recheck against plain FP64, the plain call's geometry."""
    import synth
    res = {}
    for r in (0.5, 1.0, 5.0):
        t0 = time.time()
        c = synth.stress_pair(r)
        print(f"[bench] generated {c.name} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
        arrs = [torch.from_numpy(x).to(dev) for x in (c.a_ra, c.a_dec, c.b_ra, c.b_dec)]
        out = sep = None
        cap = 0
        row = {}
        for name, prec in (("fp32", hlc.HLC_FP32_RECHECK), ("fp64", hlc.HLC_FP64)):
            for k in range(max(1, warmup) + 1):
                st, n = hlc.hlc_xmatch(*arrs, r, out, sep, precision=prec, capacity=cap)
                if st == hlc.HLC_E_OVERFLOW or (st == hlc.HLC_OK and cap == 0 and n > 0):
                    cap = n + 1024
                    out = torch.empty((cap, 2), dtype=torch.int32, device=dev)
                    sep = torch.empty(cap, dtype=torch.float64, device=dev)
                elif st != hlc.HLC_OK:
                    raise hlc.HLCError(st, f"stress r={r}")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(max(1, min(steps, 5))):
                st, n = hlc.hlc_xmatch(*arrs, r, out, sep, precision=prec, capacity=cap)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / max(1, min(steps, 5)) * 1e3
            if st != hlc.HLC_OK:
                raise hlc.HLCError(st, f"stress r={r}")
            s = hlc.last_stats()
            row[name] = {"ms_per_call": ms, "a_sources_per_s": c.na / (ms * 1e-3), "pairs": int(n),
                         "candidates": int(s["n_candidates"]), "band": int(s["n_band"])}
            print(f"[bench] stress r={r} {name}: {ms:.2f} ms, {n} pairs, {s['n_candidates']} candidates",
                  file=sys.stderr, flush=True)
        if row["fp32"]["pairs"] != row["fp64"]["pairs"]:
            raise RuntimeError(f"stress r={r}: FP32 and FP64 forms disagree on the pair count")
        res[f"r{r:g}"] = row
        del arrs, out, sep
        torch.cuda.empty_cache()
    res["workload"] = "stress 20000000x20000000, 10000 clumps (sigma 30 arcsec), counterparts on [0.99 r, 1.01 r]"
    return res


def bench_quad(hlc, torch, a_ra, a_dec, b_ra, b_dec, r, out, sep, exact_pairs):
    """The paper's HEALPix + quad-direction partition, emulated on the same
    workload: pairs it finds (a subset of the exact set), the loss, and time."""
    res = {}
    for order in (10, 12, 13):
        hlc.hlc_xmatch_quad(a_ra, a_dec, b_ra, b_dec, r, order, out, sep)  # warm the workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, n = hlc.hlc_xmatch_quad(a_ra, a_dec, b_ra, b_dec, r, order, out, sep)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        if st != hlc.HLC_OK:
            raise hlc.HLCError(st, f"quad order {order}")
        res[f"order{order}"] = {"ms": ms, "pairs": int(n), "lost": int(exact_pairs - n),
                                "loss_frac": (exact_pairs - n) / exact_pairs}
        print(f"[bench] quad order {order}: {ms:.2f} ms, {n} pairs ({exact_pairs - n} lost)", file=sys.stderr,
              flush=True)
    return res


def main():
    args = parse()
    if args.pmc_summary:
        print(pmc_summary(args.pmc_summary[0], args.pmc_summary[1:]))
        return
    if args.timeline:
        print(call_timeline(args.timeline[0], int(args.timeline[1]), *args.timeline[2:4]))
        return
    if args.traffic_from:
        print(json.dumps(traffic_from_pmc(*args.traffic_from)))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the cross-match "
              "is built and measured on a single MI355X.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2301_07331_amd as hlc
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    hlc.load()
    dev = torch.device("cuda:0")
    t0 = time.time()
    cat = synth.fullsky_pair(args.n)
    gen_s = time.time() - t0
    print(f"[bench] generated {cat.name} in {gen_s:.1f}s", file=sys.stderr, flush=True)
    a_ra, a_dec, b_ra, b_dec = (torch.from_numpy(x).to(dev) for x in (cat.a_ra, cat.a_dec, cat.b_ra, cat.b_dec))
    na, nb, r = cat.na, cat.nb, cat.r_arcsec
    cap = int(0.5 * na) + 1024
    out = torch.empty((cap, 2), dtype=torch.int32, device=dev)
    sep = torch.empty(cap, dtype=torch.float64, device=dev)
    tuning = {"zone_height_arcsec": args.zone_height} if args.zone_height > 0 else None

    if args.copy_calibration:
        # a plain copy kernel of known size: 1 GiB read, 1 GiB written
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    results = {}
    for name in args.precisions.split(","):
        prec = hlc.HLC_FP32_RECHECK if name == "fp32" else hlc.HLC_FP64
        def one():
            st, _ = hlc.hlc_xmatch(a_ra, a_dec, b_ra, b_dec, r, out, sep, precision=prec, tuning=tuning)
            if st != hlc.HLC_OK:
                raise hlc.HLCError(st, "warmup")
        warm_up(one, args.warmup)
        # timed steps: the filter kernel alone is timed by two HIP events on
        # its stream (HLC_TIME_FILTER); the per-stage events of HLC_PROFILE
        # are taken in separate calls after the timed region
        filt = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            st, n = hlc.hlc_xmatch(a_ra, a_dec, b_ra, b_dec, r, out, sep, precision=prec,
                                   flags=hlc.HLC_TIME_FILTER, tuning=tuning)
            if st != hlc.HLC_OK:
                raise hlc.HLCError(st, "timed step")
            filt.append(hlc.last_stats()["t_match_ms"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = wall / args.steps * 1e3
        stats = []
        for _ in range(3):
            st, n = hlc.hlc_xmatch(a_ra, a_dec, b_ra, b_dec, r, out, sep, precision=prec,
                                   flags=hlc.HLC_PROFILE, tuning=tuning)
            if st != hlc.HLC_OK:
                raise hlc.HLCError(st, "profiled step")
            stats.append(hlc.last_stats())
        s0 = stats[-1]
        stage = {k: statistics.median(s[k] for s in stats)
                 for k in ("t_keygen_ms", "t_sort_ms", "t_layout_ms", "t_ranges_ms", "t_match_ms",
                           "t_certify_ms", "t_total_ms")}
        # the filter's time in the timed steps (HIP events on its stream)
        stage["t_match_ms"] = statistics.mean(filt)
        mb = MATCH_BYTES[name](na, s0["nb_halo"], s0["n_band"])
        results[name] = dict(ms_per_step=ms, n_pairs=int(n), stage_ms=stage, nb_halo=int(s0["nb_halo"]),
                             n_candidates=int(s0["n_candidates"]), n_band=int(s0["n_band"]),
                             n_ties=int(s0["n_ties"]), zone_height_arcsec=s0["zone_height_arcsec"],
                             n_zones=int(s0["n_zones"]), match_bytes=int(mb),
                             match_gbs=mb / (stage["t_match_ms"] * 1e-3) / 1e9 if stage["t_match_ms"] > 0 else None)
        print(f"[bench] {name}: {ms:.3f} ms/step, {n} pairs, stages {stage}", file=sys.stderr, flush=True)

    if len(results) == 2 and results["fp32"]["n_pairs"] != results["fp64"]["n_pairs"]:
        raise RuntimeError("FP32 and FP64 forms disagree on the pair count")

    head = results.get("fp32") or next(iter(results.values()))
    head_name = "fp32" if "fp32" in results else next(iter(results))
    value = na / (head["ms_per_step"] * 1e-3)
    # dominant kernel of the headline form: the filter kernel (one launch per
    # step, timed by HIP events on the call's stream)
    t_match = head["stage_ms"]["t_match_ms"]
    achieved = head["match_bytes"] / (t_match * 1e-3) / 1e9 if t_match > 0 else None
    roofline = {
        "kernel": f"k_filter<{'FP32' if head_name == 'fp32' else 'FP64'}>",
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
        "traffic": recorded_traffic() if head_name == "fp32" else None,
    }

    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    extra = {}
    if "quad" in forms:
        extra["quad_direction"] = bench_quad(hlc, torch, a_ra, a_dec, b_ra, b_dec, r, out, sep, head["n_pairs"])
    if "batch" in forms or "stream" in forms or "stress" in forms:
        del a_ra, a_dec, b_ra, b_dec, out, sep
        torch.cuda.empty_cache()
    if "stress" in forms:
        extra["stress"] = bench_stress(hlc, torch, dev, args.steps, args.warmup)
    if "batch" in forms:
        extra["batch"] = bench_batch(hlc, torch, dev, args.steps, args.warmup)
    if "stream" in forms:
        extra["stream"] = bench_stream(hlc, torch)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = len(os.sched_getaffinity(0))
        times = []
        npairs = None
        for _ in range(args.cpu_reps):
            res = oracle.xmatch(cat.a_ra, cat.a_dec, cat.b_ra, cat.b_dec, r, nthreads=threads, sort=False)
            times.append(res.seconds)
            npairs = len(res)
        t = statistics.median(times)
        cpu = {"value": na / t, "unit": "A-sources/s", "cores": threads, "kind": "oracle",
               "sample": f"whole workload ({na}x{nb}, r={r}\"), median of {args.cpu_reps} runs, "
                         f"{t:.2f} s each, unsorted output",
               "pairs": npairs, "cpu_model": cpu_model()}
        if npairs != head["n_pairs"]:
            raise RuntimeError(f"oracle found {npairs} pairs, GPU {head['n_pairs']}")
        if not args.no_single_thread:
            one = {}
            patch = synth.patch_pair()
            for label, c in (("patch_100k", patch), ("fullsky", cat)):
                reps = 3 if c.na <= 1_000_000 else 1
                ts = [oracle.xmatch(c.a_ra, c.a_dec, c.b_ra, c.b_dec, c.r_arcsec, nthreads=1, sort=False).seconds
                      for _ in range(reps)]
                ts1 = statistics.median(ts)
                one[label] = {"seconds": ts1, "a_sources_per_s": c.na / ts1, "na": c.na, "nb": c.nb,
                              "runs": reps}
                print(f"[bench] oracle single thread {label}: {ts1:.2f} s", file=sys.stderr, flush=True)
            cpu["single_thread"] = one

    line = {
        "metric": "A-sources matched/s at 10Mx10M, r=2\" (FP32+recheck vs FP64); % HBM roofline",
        "value": value,
        "unit": "A-sources/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 in, f32 filter + f64 certify" if head_name == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"fullsky {na}x{nb}, r=2 arcsec, band+caps+seam mix, 40% counterparts",
                   "na": na, "nb": nb, "r_arcsec": r, "precision": head_name},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": {k: {"ms_per_step": v["ms_per_step"], "a_sources_per_s": na / (v["ms_per_step"] * 1e-3),
                      "stage_ms": v["stage_ms"], "match_gbs": v["match_gbs"],
                      "match_frac_hbm": (v["match_gbs"] / HBM_PEAK_GBS) if v["match_gbs"] else None,
                      "call_frac_hbm": CALL_BYTES(na, nb, v["n_pairs"]) / (v["stage_ms"]["t_total_ms"] * 1e-3)
                      / 1e9 / HBM_PEAK_GBS,
                      "pairs": v["n_pairs"], "nb_halo": v["nb_halo"], "candidates": v["n_candidates"],
                      "band": v["n_band"], "ties": v["n_ties"], "zone_height_arcsec": v["zone_height_arcsec"],
                      "zones": v["n_zones"]}
                  for k, v in results.items()},
    }
    line["forms"].update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
