#!/usr/bin/env python3
"""Throughput of the P-MPSM equi-join on one MI355X.

One step = one complete mpsm_join call (every phase: S run sort, R range
partitioning and partition sort, start search, merge join, result) over the
benchmark workload, with the inputs already resident in HBM.  The headline
workload is the largest single-GPU one: |R| = 2^28 log-normal keys with
duplicates joined with |S| = 2^30 (1..16 copies of every distinct key).

Prints one JSON line.  Fields beyond the common contract:
  roofline      the dominant kernel's achieved algorithmic HBM bandwidth
                against the MI355X peak, timed with HIP events recorded
                between the kernels of the timed steps on the join's stream;
  path_roofline the same for the whole step (algorithmic bytes of the path);
  steps_ms      per-step device time of every launch step, averaged;
  cpu_baseline  the CPU oracle on a bounded sample of the same workload:
                its join over key-range slices on all host threads (up to
                16), and single-threaded, with the host's CPU model, cores
                and RAM;
  other_workloads  the same figures for the other single-join workloads
                (plain and learned).
"""
import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "join throughput (M tuples/s of |R|+|S|) + % HBM roofline; learned vs plain"

# algorithmic HBM bytes of each launch step, per tuple of the relation it reads
# S's histogram pass is folded into its scatter on large inputs (the step
# then only redoes runs whose bucket regions overflowed): no bytes of its own
STEP_BYTES = {
    # S's and R's second-level histograms are folded into their scatters
    # (large inputs): the steps remain as the exact redo of overflowing
    # segments, with nothing to do when every bucket fit its region
    "s_histogram": ("S", 0), "s_scatter": ("S", 32), "s_bucket_sort": ("S", 32),
    "r1_histogram": ("R", 16), "r1_scatter": ("R", 32), "r2_histogram": ("R", 0), "r2_scatter": ("R", 32),
    "r_bucket_sort": ("R", 32), "join": ("RS", 16),
}
KERNEL_OF_STEP = {
    "s_histogram": "k_bucket_hist", "s_scatter": "k_bucket_scatter", "s_bucket_sort": "k_bucket_sort",
    "r1_histogram": "k_bucket_hist", "r1_scatter": "k_bucket_scatter", "r2_histogram": "k_bucket_hist",
    "r2_scatter": "k_bucket_scatter", "r_bucket_sort": "k_bucket_sort", "join": "k_join",
}


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    from paper_1207_0145_amd import build as hipbuild
    for f in (*hipbuild.HEADERS, "mpsm.hip"):
        with open(os.path.join(ROOT, "paper_1207_0145_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(step: str, workload: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_digest") != kernel_source_digest():
        return None
    return t.get("steps", {}).get(step, {}).get("hbm_bytes_per_launch")


WORKLOAD_KEYS = {
    "fk_uniform": "R keys a 64-bit bijective mix of a permutation, S uniform foreign keys",
    "fk_small": "R keys a permutation of [0, 2^20), S uniform foreign keys",
    "skewed": "R keys from 64 Gaussian blobs, S Zipf(1.0) foreign keys",
    "lognormal": "R keys floor(exp(2Z) 2^28) with duplicates, S 1..16 copies of every distinct R key",
}

# launch steps -> (kernel name prefix, occurrence of that kernel inside one join)
STEP_DISPATCH = {
    # S and R's second level: the scatter into regions, then the histogram
    # and the redo scatter for segments whose regions overflowed (launched
    # always, most often with nothing to do); R's first level: histogram and
    # staged scatter
    "s_histogram": ("k_bucket_hist", 0),
    "s_scatter": [("void k_bucket_scatter<true>", 0), ("k_redo_scatter", 0)],
    "r1_histogram": ("k_bucket_hist", 1), "r1_scatter": ("void k_bucket_scatter<false>", 0),
    "r2_histogram": ("k_bucket_hist", 2),
    "r2_scatter": [("void k_bucket_scatter<true>", 1), ("k_redo_scatter", 1)],
    # the sorts: the two-per-CU kernel, then the one-per-CU kernel over the larger buckets
    "s_bucket_sort": [("void k_bucket_sort_cs<1024, 4", 0), ("void k_bucket_sort_cs<1024, 8", 0)],
    "r_bucket_sort": [("void k_bucket_sort_cs<1024, 4", 1), ("void k_bucket_sort_cs<1024, 8", 1)],
    "search": ("k_search", 0), "join": ("void k_join<0", 0),
}


def _read_csv(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _per_join(rows, name_key, start_key):
    """Split dispatch rows (in dispatch order) into joins at k_init_result."""
    rows = sorted(rows, key=lambda r: int(r["Dispatch_Id"]))
    joins, cur = [], None
    for r in rows:
        if r[name_key].startswith("k_init_result"):
            cur = []
            joins.append(cur)
        if cur is not None:
            cur.append(r)
    return joins


def _nth(join, prefix, k):
    hits = [r for r in join if r["Kernel_Name"].startswith(prefix)]
    return hits[k] if k < len(hits) else None


def step_times(names, evsets, steps):
    """Average device time of every launch step from the join's markers.
    R's partitioning and sort may run on a second stream beside S's bucket
    sort, starting once S's scatter is done: R's first step then counts from
    s_scatter, and the partition step from the later of the two phases'
    ends."""
    ix = {n: i for i, n in enumerate(names)}

    def el(a, b):
        return sum(e.elapsed(ix[a], ix[b]) for e in evsets) / steps

    out = {names[i]: el(names[i - 1], names[i]) for i in range(1, len(names))}
    overlapped = el("s_oversize_sort", "r1_splitters") < 0
    if overlapped:
        out["r1_splitters"] = el("s_scatter", "r1_splitters")
        last = "r_oversize_sort" if el("s_oversize_sort", "r_oversize_sort") > 0 else "s_oversize_sort"
        out["partitions"] = el(last, "partitions")
    return out, overlapped


def summarize_profiles(kt_csv, fetch_csv, write_csv, workload, nR, nS, command):
    """HBM bytes and durations per launch step from a rocprofv3 kernel trace
    and two counter runs (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), scaled
    by what the counters read for a 1 GiB device copy in the same runs."""
    kt = _per_join(_read_csv(kt_csv), "Kernel_Name", "Start_Timestamp")
    cal = {}
    for label, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _read_csv(path)
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"] or "copy" in r["Kernel_Name"].lower()]
        big = max(copies, key=lambda r: float(r["Counter_Value"]))
        cal[label] = {"copy_kib": float(big["Counter_Value"]), "factor": (1 << 30) / (1024.0 * float(big["Counter_Value"]))}
        cal[label]["joins"] = _per_join(rows, "Kernel_Name", "Start_Timestamp")
    steps = {}
    for step, spec in STEP_DISPATCH.items():
        picks = spec if isinstance(spec, list) else [spec]   # a step may span several dispatches
        durs = []
        for j in kt:
            rows = [_nth(j, prefix, k) for prefix, k in picks]
            if all(r is not None for r in rows):
                durs.append(sum((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in rows))
        fs = [_nth(cal["fetch"]["joins"][0], prefix, k) for prefix, k in picks]
        ws = [_nth(cal["write"]["joins"][0], prefix, k) for prefix, k in picks]
        if not durs or any(r is None for r in fs + ws):
            continue
        fb = sum(float(f["Counter_Value"]) for f in fs) * 1024 * cal["fetch"]["factor"]
        wb = sum(float(w["Counter_Value"]) for w in ws) * 1024 * cal["write"]["factor"]
        rel, per = STEP_BYTES.get(step, ("RS", 0))
        alg = per * {"S": nS, "R": nR, "RS": nR + nS}[rel]
        f = fs[0]
        steps[step] = {"kernel": " + ".join(r["Kernel_Name"].split("(")[0][:60] for r in fs),
                       "avg_launch_ms": round(sum(durs) / len(durs), 4),
                       "launches": len(durs), "fetch_bytes": round(fb), "write_bytes": round(wb),
                       "hbm_bytes_per_launch": round(fb + wb), "algorithmic_bytes": alg or None,
                       "traffic_over_algorithmic": round((fb + wb) / alg, 3) if alg else None}
    return {"workload": workload, "nR": nR, "nS": nS, "kernel_source_digest": kernel_source_digest(),
            "calibration": {k: {"copy_counter_kib": v["copy_kib"], "bytes_per_counter_byte": round(v["factor"], 4)}
                            for k, v in cal.items()},
            "command": command, "steps": steps}


WORKLOAD_TITLE = {
    "fk_uniform": "|R| = 2^26, |S| = 2^28, uniform foreign keys",
    "fk_small": "|R| = 2^20, |S| = 2^22, uniform foreign keys",
    "skewed": "|R| = 2^26 clustered keys, |S| = 2^28 Zipf(1.0) foreign keys",
    "lognormal": "|R| = 2^28 log-normal keys with duplicates, |S| = 2^30, 1..16 copies per distinct key",
}


def profile_markdown(t, kt_csv, workload):
    """Text summary of a profile: the per-kernel statistics of the kernel
    trace, the per-step durations and HBM bytes of `t` (summarize_profiles),
    and the dispatch sequence of the last join of the trace."""
    stats_csv = kt_csv.replace("kernel_trace", "kernel_stats")
    out = [f"# P-MPSM join on {workload} ({WORKLOAD_TITLE.get(workload, '')}), MI355X", "",
           "Plain join (sampled splitters, index start search).  R's partitioning and sort run on a second "
           "stream beside S's bucket sort (from the end of S's scatter on): their durations are durations in "
           "that shared setting.", "",
           f"Kernel source digest: {t['kernel_source_digest']}.  Commands (run from /tmp, TMPDIR=/tmp):", "",
           "```", t.get("command", ""), "```", ""]
    if os.path.exists(stats_csv):
        out += ["| kernel | calls | avg (us) | total (ms) |", "|---|---|---|---|"]
        for r in _read_csv(stats_csv)[:18]:
            name = r["Name"].split("(")[0].replace("void ", "")
            out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                       f"{float(r['TotalDurationNs']) / 1e6:.2f} |")
        out.append("")
    cal = t["calibration"]
    out += [f"Per launch step: HBM bytes from FETCH_SIZE x {cal['fetch']['bytes_per_counter_byte']} and "
            f"WRITE_SIZE x {cal['write']['bytes_per_counter_byte']} (the factors that make the counters read "
            "1 GiB for the 1 GiB device copy in the same runs).", "",
            "| step | kernel | avg launch (ms) | HBM read (GB) | HBM write (GB) | algorithmic (GB) | "
            "traffic / algorithmic | achieved alg. GB/s |", "|---|---|---|---|---|---|---|---|"]
    for step, v in t["steps"].items():
        alg = v["algorithmic_bytes"]
        out.append(f"| {step} | `{v['kernel']}` | {v['avg_launch_ms']:.3f} | {v['fetch_bytes'] / 1e9:.2f} | "
                   f"{v['write_bytes'] / 1e9:.2f} | {alg / 1e9 if alg else 0:.2f} | "
                   f"{v['traffic_over_algorithmic'] or '-'} | "
                   f"{alg / (v['avg_launch_ms'] * 1e-3) / 1e9 if alg else 0:.0f} |")
    joins = _per_join(_read_csv(kt_csv), "Kernel_Name", "Start_Timestamp")
    if joins:
        j = sorted(joins[-1], key=lambda r: int(r["Start_Timestamp"]))
        t0 = int(j[0]["Start_Timestamp"])
        out += ["", "Dispatches of the last join of the trace (start and duration in ms; queue 1 is the "
                "join's stream, queue 2 the second stream):", "", "| start | duration | queue | kernel |",
                "|---|---|---|---|"]
        for r in j:
            if "copyBuffer" in r["Kernel_Name"]:
                continue
            out.append(f"| {(int(r['Start_Timestamp']) - t0) / 1e6:.3f} | "
                       f"{(int(r['End_Timestamp']) - int(r['Start_Timestamp'])) / 1e6:.3f} | "
                       f"{r.get('Queue_Id', '')} | `{r['Kernel_Name'].split('(')[0].replace('void ', '')}` |")
    if t.get("sq"):
        out += ["", "Wave-level instruction counts (SQ counters, one more run of the same command with "
                "`--pmc " + " ".join(SQ_COUNTERS) + "`), per tuple of the step's relation "
                "(S for S's steps, R for R's, both for the join):", "",
                "| step | VALU | LDS | SALU | VMEM | SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES |", "|---|---|---|---|---|---|"]
        for step, v in t["sq"].items():
            pt = v["per_tuple"]
            out.append(f"| {step} | {pt['valu']} | {pt['lds']} | {pt['salu']} | {pt['vmem']} | "
                       f"{v['wait_inst_any_over_wave_cycles']} |")
    return "\n".join(out) + "\n"


SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_INSTS_VMEM", "SQ_WAVE_CYCLES",
               "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY")


# calls of `--workload hostruns --steps 1 --warmup 1`, in order: each form is
# run twice (the warm-up, then the timed call)
HOSTRUNS_CALLS = ["device-resident S", "chunk 2^28", "chunk 2^26", "chunk 2^24", "spilled runs rejoined",
                  "chunk 2^24, runs not kept"]


def summarize_host_trace(kt_csv, mc_csv, command):
    """Markdown summary of a rocprofv3 kernel and memory-copy trace of the
    hostruns experiment: per timed call its span, its copies in and out of
    device memory (by the copy engines, or by the runtime's copy kernels)
    and its own kernels."""
    ev = []
    for r in _read_csv(kt_csv):
        ev.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), "kernel", r["Kernel_Name"].split("(")[0]))
    for r in _read_csv(mc_csv):
        ev.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), "copy", r["Direction"]))
    ev.sort()
    starts = [i for i, e in enumerate(ev) if e[2] == "kernel" and e[3].startswith("k_init_result")]
    if len(starts) != 2 * len(HOSTRUNS_CALLS):
        raise SystemExit(f"expected {2 * len(HOSTRUNS_CALLS)} joins in the trace, found {len(starts)}")
    out = ["# Join with S in pinned host memory (hostruns: |R| = 2^26, |S| = 2^28 uniform foreign keys), MI355X", "",
           "Kernel and memory-copy trace of the timed call of each form (the second of its two calls).  Copies in "
           "and out are the host link's; the runtime moves some of them with copy kernels (`copyBuffer`), listed "
           "with the copies.  Copies under 0.05 ms (the read-back of the result) are left out; the device-resident "
           "form copies nothing else.  Kernel durations are summed over both streams, and a kernel's duration "
           "includes the time it waits for compute units that copy kernels hold.", "",
           "Command (run from /tmp, TMPDIR=/tmp):", "", "```", command, "```", "",
           "| form | call span ms | copies in: n, total ms, each min-max ms | copies out: n, total ms, each min-max ms "
           "| join kernels ms (sum of durations) | three longest kernels, ms |", "|---|---|---|---|---|---|"]
    for c, name in enumerate(HOSTRUNS_CALLS):
        a = starts[2 * c + 1]
        b = starts[2 * c + 2] if 2 * c + 2 < len(starts) else len(ev)
        call = ev[a:b]
        t0 = call[0][0]
        t1 = max(e[1] for e in call)
        ins, outs, kern = [], [], {}
        for t, u, kind, nm in call:
            ms = (u - t) / 1e6
            if kind == "copy" or "copyBuffer" in nm:
                if ms >= 0.05:
                    (ins if "HOST_TO_DEVICE" in nm else outs).append(ms)
            else:
                kern[nm] = kern.get(nm, 0.0) + ms

        def cell(x):
            return f"{len(x)}, {sum(x):.1f}, {min(x):.2f}-{max(x):.2f}" if x else "0"

        top = sorted(kern.items(), key=lambda kv: -kv[1])[:3]
        out.append(f"| {name} | {(t1 - t0) / 1e6:.2f} | {cell(ins)} | {cell(outs)} | {sum(kern.values()):.2f} | "
                   + "; ".join(f"`{k.replace('void ', '')[:40]}` {v:.2f}" for k, v in top) + " |")
    return "\n".join(out) + "\n"


def summarize_sq(sq_csv, nR, nS):
    """Per launch step of the first join in a counter run of SQ_COUNTERS:
    every counter summed over the step's dispatches, and the wave-level
    instruction counts per tuple of the step's relation."""
    rows = _read_csv(sq_csv)
    by_disp = {}
    for r in rows:
        d = by_disp.setdefault(r["Dispatch_Id"], {"Dispatch_Id": r["Dispatch_Id"], "Kernel_Name": r["Kernel_Name"],
                                                  "Start_Timestamp": r.get("Start_Timestamp", "0")})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    joins = _per_join(list(by_disp.values()), "Kernel_Name", "Start_Timestamp")
    if not joins:
        return {}
    out = {}
    for step, spec in STEP_DISPATCH.items():
        picks = spec if isinstance(spec, list) else [spec]
        ds = [_nth(joins[0], prefix, k) for prefix, k in picks]
        if any(d is None for d in ds):
            continue
        tot = {c: sum(d.get(c, 0.0) for d in ds) for c in SQ_COUNTERS}
        rel = STEP_BYTES.get(step, ("RS", 0))[0]
        n = {"S": nS, "R": nR, "RS": nR + nS}[rel]
        out[step] = {"counters": {c: int(v) for c, v in tot.items()},
                     "per_tuple": {"tuples": n, "valu": round(tot["SQ_INSTS_VALU"] / n, 2),
                                   "lds": round(tot["SQ_INSTS_LDS"] / n, 2),
                                   "salu": round(tot["SQ_INSTS_SALU"] / n, 2),
                                   "vmem": round(tot["SQ_INSTS_VMEM"] / n, 3)},
                     "wait_inst_any_over_wave_cycles": round(tot["SQ_WAIT_INST_ANY"] / tot["SQ_WAVE_CYCLES"], 3)
                     if tot["SQ_WAVE_CYCLES"] else None}
    return out


def copy_bandwidth(torch, dev, nbytes=1 << 30, reps=5):
    """Read+write bandwidth of a plain device-to-device copy (the runtime's
    copy kernel) on this GPU: the practical ceiling next to the 8 TB/s peak."""
    x = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(reps):
        y.copy_(x)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del x, y
    return 2 * nbytes / (ms * 1e-3) / 1e9


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info():
    """CPU model, logical cores and RAM of this host (lscpu, /proc/meminfo)."""
    import subprocess
    info = {"cores": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() == "Model name":
                info["cpu_model"] = v.strip()
            elif k.strip() == "Socket(s)":
                info["sockets"] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/meminfo") as f:
            kb = int(f.readline().split()[1])
        info["ram_gib"] = round(kb / 2**20, 1)
    except (OSError, ValueError, IndexError):
        pass
    return info


def cpu_baseline(workload: str, shift: int, threads: int):
    """The CPU oracle on the same workload recipe at 1/2^shift of its size:
    its sort-merge join with one thread, and the same join split into
    key-range slices that `threads` threads join side by side."""
    import numpy as np
    import oracle
    import workloads
    w = workloads.make(workload, scale_shift=shift)
    n = len(w.R) + len(w.S)
    t0 = time.perf_counter()
    r1 = oracle.join(w.R, w.S)
    dt1 = time.perf_counter() - t0
    smp = np.sort(w.R[np.random.default_rng(0).integers(0, len(w.R), 1 << 14), 0])
    nsl = 4 * threads
    bounds = np.unique(smp[(np.arange(1, nsl) * len(smp)) // nsl])
    t0 = time.perf_counter()
    rt = oracle.join_sliced(w.R, w.S, bounds, threads=threads)
    dtt = time.perf_counter() - t0
    assert (rt.count, rt.checksum) == (r1.count, r1.checksum)
    sample = (f"{workload} at 1/{1 << shift} scale (|R|={len(w.R)}, |S|={len(w.S)}, same recipe): "
              f"{dtt:.1f} s for the oracle's sort-merge join over {len(bounds) + 1} key-range slices "
              f"on {threads} threads; {dt1:.1f} s on one thread (count {r1.count})")
    return {"value": round(n / dtt / 1e6, 3), "unit": "M tuples/s", "cores": threads, "kind": "oracle",
            "sample": sample, "single_thread": {"value": round(n / dt1 / 1e6, 3), "cores": 1, "seconds": round(dt1, 2)},
            "host": host_info()}


def variant_stats(mpsm, torch, R, S, cfg, dev):
    """One extra call with statistics (synchronising; outside the timed steps)."""
    ws = mpsm.alloc_workspace(R.shape[0], S.shape[0], cfg, dev)
    st = mpsm.MpsmStats()
    out = torch.zeros(2, dtype=torch.int64, device=dev)
    mpsm.join_into(R, S, out, ws, cfg, stats=st)
    d = {name: getattr(st, name) for name, _ in st._fields_}
    del ws
    return {k: (round(v, 5) if isinstance(v, float) else v) for k, v in d.items()}


def run_variant(mpsm, torch, R, S, out, cfg, args, names, nR, nS, label, steps):
    """Time `steps` calls of another configuration, same inputs."""
    dev = R.device
    ws = mpsm.alloc_workspace(nR, nS, cfg, dev)
    for _ in range(args.warmup):
        mpsm.join_into(R, S, out, ws, cfg)
    evsets = [mpsm.EventSet(len(names)) for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for k in range(steps):
        mpsm.join_events_into(R, S, out, ws, evsets[k], cfg)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    steps_ms, _ = step_times(names, evsets, steps)
    for e in evsets:
        e.close()
    count, checksum = [v & 0xFFFFFFFFFFFFFFFF for v in out.cpu().tolist()]
    del ws
    log(f"{label}: {ms:.3f} ms/step")
    return {"ms_per_step": round(ms, 4), "value": round((nR + nS) / (ms * 1e-3) / 1e6, 2),
            "result": {"count": count, "checksum": f"{checksum:#018x}"},
            "steps_ms": {k: round(v, 4) for k, v in steps_ms.items() if v > 0.0005},
            "stats": variant_stats(mpsm, torch, R, S, cfg, dev)}


def batch_bench(args):
    """The 256-join batch: one graph-captured launch sequence per step, the
    autotuned tuning, per-join latency percentiles from the GPU wall clock,
    and the same joins run one mpsm_join call at a time for comparison."""
    import numpy as np
    import torch
    import paper_1207_0145_amd as mpsm
    import workloads
    log("generating batch (256 joins)")
    ws = workloads.make("batch")
    joins = [(torch.from_numpy(w.R.view(np.int64)).cuda(), torch.from_numpy(w.S.view(np.int64)).cuda()) for w in ws]
    nR = sum(len(w.R) for w in ws)
    nS = sum(len(w.S) for w in ws)
    del ws
    cache = os.path.join(tempfile.gettempdir(), "mpsm_batch_autotune.txt") if args.autotune_cache is None \
        else args.autotune_cache
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)

    def timed(waves):
        """Autotuned batch with the given waves (0: automatic): ms per graph
        replay and per-join completion times of the last replay."""
        b = mpsm.Batch(joins, mpsm.config(waves=waves))
        tun = b.autotune(cache)
        log(f"waves {waves}: tuning {tun}")
        for _ in range(args.warmup):
            b.run(use_graph=True)
        torch.cuda.synchronize()
        t0.record()
        for _ in range(args.steps):
            b.run(use_graph=True)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / args.steps
        tm = b.times.cpu().numpy().view(np.uint64).astype(np.float64) / mpsm.clock_hz() * 1e6   # us
        return b, tun, ms, tm[:, 2] - tm[:, 0], tm[:, 2] - tm[:, 1]

    def pct(x):
        return {"p50": round(float(np.percentile(x, 50)), 1), "p99": round(float(np.percentile(x, 99)), 1)}

    b1, tun1, ms1, total1, _ = timed(1)
    b1.close()
    b, tun, ms, total_us, work_us = timed(0)
    log(f"one wave {ms1:.3f} ms, waves {ms:.3f} ms")
    res = b.results()
    # the same joins, one call each, on one stream
    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    wsz = max(mpsm.workspace_bytes(R.shape[0], S.shape[0]) for R, S in joins)
    wbuf = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    for R, S in joins[:8]:
        mpsm.join_into(R, S, out, wbuf)
    torch.cuda.synchronize()
    t0.record()
    for R, S in joins:
        mpsm.join_into(R, S, out, wbuf)
    t1.record()
    torch.cuda.synchronize()
    seq_ms = t0.elapsed_time(t1)
    path_bytes = 48 * nS + 64 * nR
    line = {
        "metric": METRIC, "value": round((nR + nS) / (ms * 1e-3) / 1e6, 2), "unit": "M tuples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"batch: 256 joins, |R_b| log-uniform in [2^12, 2^22], |S_b| = k_b |R_b| (k_b in 1..8), "
                               f"half uniform, half Zipf(0.5..1.2) foreign keys; sum |R| = {nR}, sum |S| = {nS}",
                   "launch": "one hipGraph replay per step (mpsm_join_batch over device descriptors, joins "
                             "taken in 4 waves by size)", "tuning": tun},
        "path_roofline": {"algorithmic_bytes": path_bytes, "achieved": round(path_bytes / (ms * 1e-3) / 1e9, 1),
                          "unit": "GB/s", "frac": round(path_bytes / (ms * 1e-3) / 8e12, 4)},
        "per_join_us": {"done_since_batch_start": pct(total_us), "done_since_first_item": pct(work_us)},
        "one_wave": {"ms_per_step": round(ms1, 4), "tuning": tun1,
                     "per_join_us": {"done_since_batch_start": pct(total1)}},
        "one_call_per_join": {"ms": round(seq_ms, 3), "value": round((nR + nS) / (seq_ms * 1e-3) / 1e6, 2)},
        "result": {"pairs": int(sum(c for c, _ in res))},
    }
    print(json.dumps(line), flush=True)


def unit_costs(mpsm, ws, nR, nS, cfg):
    """Section 4.3 cost |R_u| log2 |R_u| + Q |R_u| + |S_u| of every join unit
    of the last join run in workspace ws (R partitions joined together and
    their S slices in all Q runs): (max, mean) over the units."""
    import math
    import numpy as np
    lay = mpsm.layout(nR, nS, cfg)

    def part(off, nbytes):
        return ws[off:off + nbytes].cpu().numpy()

    P = int(part(lay["off_partitions"], 4).view(np.uint32)[0])
    Q = lay["runs"]
    plen = part(lay["off_part_len"], 4 * P).view(np.uint32).astype(np.int64)
    span = part(lay["off_join_span"], P)
    o = part(lay["off_offsets"], 4 * (P + 1) * Q).view(np.uint32).reshape(P + 1, Q).astype(np.int64)
    costs = []
    for p in np.nonzero(span)[0]:
        r = int(plen[p:p + span[p]].sum())
        sl = int(np.maximum(o[p + span[p]] - o[p], 0).sum())
        costs.append(r * math.log2(max(r, 1)) + Q * r + sl)
    return max(costs), sum(costs) / len(costs)


def time_join(mpsm, torch, R, S, cfg, args, steps):
    """ms per call (steps timed calls after the warm-up) and the result."""
    ws = mpsm.alloc_workspace(R.shape[0], S.shape[0], cfg, R.device)
    out = torch.zeros(2, dtype=torch.int64, device=R.device)
    for _ in range(args.warmup):
        mpsm.join_into(R, S, out, ws, cfg)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(steps):
        mpsm.join_into(R, S, out, ws, cfg)
    t1.record()
    torch.cuda.synchronize()
    c, k = [v & 0xFFFFFFFFFFFFFFFF for v in out.cpu().tolist()]
    return t0.elapsed_time(t1) / steps, (c, f"{k:#018x}"), ws


def experiment_bench(args):
    """The paper's other experiments on one GPU, one JSON line each:
      negcorr  (Section 5.6) |R| = 2^24, |S| = 2^26 negatively correlated
               80:20 keys; sampled, learned and cost-balanced splitters: time
               and the largest / mean Section 4.3 cost of the join units;
      roles    (Section 5.4) |R| = 2^24 uniform foreign keys, |S| = m |R| for
               m = 1, 4, 8, 16; R private (as given) against S private;
      locskew  (Section 5.5) |R| = 2^24, |S| = 2^26 uniform foreign keys, S
               unordered against S ordered small to large in one cluster per
               S run;
      hostruns (Section 3.1) |R| = 2^26, |S| = 2^28 uniform foreign keys with
               S and its sorted runs in pinned host memory, for several
               chunk sizes (the share of S on the device at a time), against
               the join with S in device memory and the time S takes over
               the host link in and out; and the join phase alone, a new R
               joined with the runs left in host memory;
      hostruns_large  the same forms with |S| = 2^31 (32 GiB of S in host
               memory) and a device workspace of a few GiB."""
    import numpy as np
    import torch
    import paper_1207_0145_amd as mpsm
    import workloads
    dev = torch.device("cuda", 0)

    def to_dev(a):
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(dev)

    steps = args.steps
    base = {"metric": METRIC, "unit": "M tuples/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
            "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "u64", "data": "synthetic"}
    if args.workload == "negcorr":
        w = workloads.negcorr(1 << 24, 1 << 26, seed=0x1207014500000701)
        R, S = to_dev(w.R), to_dev(w.S)
        forms = {"sampled": mpsm.config(), "learned": mpsm.config(splitter=mpsm.SPLIT_LEARNED,
                                                                  search=mpsm.SEARCH_LEARNED),
                 "cost": mpsm.config(splitter=mpsm.SPLIT_COST)}
        res = {}
        for name, cfg in forms.items():
            ms, r, ws = time_join(mpsm, torch, R, S, cfg, args, steps)
            mx, mean = unit_costs(mpsm, ws, R.shape[0], S.shape[0], cfg)
            res[name] = {"ms_per_step": round(ms, 4), "value": round((R.shape[0] + S.shape[0]) / (ms * 1e-3) / 1e6, 2),
                         "result": r, "unit_cost_max": round(mx), "unit_cost_mean": round(mean),
                         "unit_cost_max_over_mean": round(mx / mean, 3)}
            log(f"negcorr {name}: {ms:.3f} ms, unit cost max/mean {mx / mean:.3f}")
            del ws
        line = {**base, "value": res["sampled"]["value"], "ms_per_step": res["sampled"]["ms_per_step"],
                "config": {"workload": f"negcorr: |R|=2^24, |S|=2^26, 80% of R keys in the top 20% and 80% of S "
                                       f"keys in the bottom 20% of [0, {w.meta['domain']})"}, "forms": res}
    elif args.workload == "roles":
        res = {}
        for m in (1, 4, 8, 16):
            w = workloads.fk_uniform(1 << 24, m << 24, seed=0x1207014500000800 + m, spread=True)
            R, S = to_dev(w.R), to_dev(w.S)
            del w
            row = {}
            for name, role in (("R_private", mpsm.ROLE_AS_GIVEN), ("S_private", mpsm.ROLE_SWAP)):
                ms, r, ws = time_join(mpsm, torch, R, S, mpsm.config(role=role), args, steps)
                del ws
                row[name] = {"ms_per_step": round(ms, 4), "result": r}
                log(f"roles m={m} {name}: {ms:.3f} ms")
            res[f"m{m}"] = row
            del R, S
            torch.cuda.empty_cache()
        line = {**base, "value": round((5 << 24) / (res["m4"]["R_private"]["ms_per_step"] * 1e-3) / 1e6, 2),
                "ms_per_step": res["m4"]["R_private"]["ms_per_step"],
                "config": {"workload": "roles: |R|=2^24 uniform foreign keys, |S| = m |R|; value at m = 4, R private"},
                "multiplicities": res}
    elif args.workload == "hostruns":
        w = workloads.make("fk_uniform")
        nR, nS = len(w.R), len(w.S)
        R = to_dev(w.R)
        Sh = torch.empty((nS, 2), dtype=torch.int64, pin_memory=True)
        Sh.copy_(torch.from_numpy(w.S.view(np.int64)))
        del w
        runs = torch.empty((nS, 2), dtype=torch.int64, pin_memory=True)
        out = torch.zeros(2, dtype=torch.int64, device=dev)
        # copy rates of the host link (pinned memory, one copy of S each way)
        Sd = Sh.to(dev)
        rates = {}
        for name, dst, src in (("h2d", Sd, Sh), ("d2h", runs, Sd)):
            dst.copy_(src, non_blocking=True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(3):
                dst.copy_(src, non_blocking=True)
            torch.cuda.synchronize()
            rates[name + "_GBps"] = round(3 * nS * 16 / (time.perf_counter() - t) / 1e9, 1)
        log(f"host link: {rates}")
        ms_dev, r_dev, ws = time_join(mpsm, torch, R, Sd, mpsm.config(), args, steps)
        del ws, Sd
        torch.cuda.empty_cache()
        log(f"hostruns device-resident S: {ms_dev:.3f} ms")
        res = {"device_resident": {"ms_per_step": round(ms_dev, 4), "result": r_dev}}
        for lg in (28, 26, 24):
            nbytes = mpsm.join_host_runs_workspace_bytes(nR, nS, 1 << lg)
            ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            for _ in range(args.warmup):
                mpsm.join_host_runs_into(R, Sh, runs, out, ws, 1 << lg)
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t0.record()
            for _ in range(steps):
                mpsm.join_host_runs_into(R, Sh, runs, out, ws, 1 << lg)
            t1.record()
            torch.cuda.synchronize()
            ms = t0.elapsed_time(t1) / steps
            c, k = [v & 0xFFFFFFFFFFFFFFFF for v in out.cpu().tolist()]
            res[f"chunk_2^{lg}"] = {"ms_per_step": round(ms, 4), "value": round((nR + nS) / (ms * 1e-3) / 1e6, 2),
                                    "result": (c, f"{k:#018x}"), "workspace_GiB": round(nbytes / 2**30, 3)}
            log(f"hostruns chunk 2^{lg}: {ms:.3f} ms, workspace {nbytes / 2**30:.2f} GiB")
            del ws
            torch.cuda.empty_cache()
        # the join phase alone over the runs the last call left in host memory:
        # S's runs read back over the link, in key order
        nbytes = mpsm.join_spilled_runs_workspace_bytes(nR, nS)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        for _ in range(args.warmup):
            mpsm.join_spilled_runs_into(R, runs, out, ws)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record()
        for _ in range(steps):
            mpsm.join_spilled_runs_into(R, runs, out, ws)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / steps
        c, k = [v & 0xFFFFFFFFFFFFFFFF for v in out.cpu().tolist()]
        res["spilled_runs_rejoined"] = {"ms_per_step": round(ms, 4), "value": round((nR + nS) / (ms * 1e-3) / 1e6, 2),
                                        "result": (c, f"{k:#018x}"), "workspace_GiB": round(nbytes / 2**30, 3),
                                        "link_floor_ms": round(nS * 16 / rates["h2d_GBps"] / 1e6, 2)}
        log(f"hostruns spilled runs rejoined: {ms:.3f} ms, workspace {nbytes / 2**30:.2f} GiB")
        del ws
        # runs not kept: S crosses the link once
        nbytes = mpsm.join_host_runs_workspace_bytes(nR, nS, 1 << 24)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        for _ in range(args.warmup):
            mpsm.join_host_runs_into(R, Sh, None, out, ws, 1 << 24)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record()
        for _ in range(steps):
            mpsm.join_host_runs_into(R, Sh, None, out, ws, 1 << 24)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / steps
        c, k = [v & 0xFFFFFFFFFFFFFFFF for v in out.cpu().tolist()]
        res["chunk_2^24_runs_not_kept"] = {"ms_per_step": round(ms, 4), "value": round((nR + nS) / (ms * 1e-3) / 1e6, 2),
                                           "result": (c, f"{k:#018x}"),
                                           "link_floor_ms": round(nS * 16 / rates["h2d_GBps"] / 1e6, 2)}
        log(f"hostruns chunk 2^24, runs not kept: {ms:.3f} ms")
        del ws
        # the least the host link allows, one way after the other: S in and its runs out
        floor_ms = nS * 16 * (1 / rates["h2d_GBps"] + 1 / rates["d2h_GBps"]) / 1e6
        line = {**base, "value": res["chunk_2^26"]["value"], "ms_per_step": res["chunk_2^26"]["ms_per_step"],
                "config": {"workload": "hostruns: |R|=2^26, |S|=2^28 uniform foreign keys; S and its sorted runs "
                                       "in pinned host memory, value at a chunk of 2^26 tuples"},
                "host_link_inclusive": True,   # these rates include S's copies over the host link
                "chunks": res, "host_link": rates, "host_link_floor_ms": round(floor_ms, 2)}
    elif args.workload == "hostruns_large":
        # S of 2^31 tuples (32 GiB) in pinned host memory against a device
        # workspace of a few GiB: the join's device footprint follows the chunk
        nR, nS, chunk = 1 << 26, 1 << 31, 1 << 24
        log("generating |R| = 2^26, |S| = 2^31 uniform foreign keys")
        w = workloads.fk_uniform(nR, nS, seed=0x1207014500000b01, spread=True)
        R = to_dev(w.R)
        Sh = torch.empty((nS, 2), dtype=torch.int64, pin_memory=True)
        Sh.copy_(torch.from_numpy(w.S.view(np.int64)))
        del w
        runs = torch.empty((nS, 2), dtype=torch.int64, pin_memory=True)
        out = torch.zeros(2, dtype=torch.int64, device=dev)
        res = {}

        def timed(name, nbytes, call):
            ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            for _ in range(args.warmup):
                call(ws)
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t0.record()
            for _ in range(steps):
                call(ws)
            t1.record()
            torch.cuda.synchronize()
            ms = t0.elapsed_time(t1) / steps
            c, k = [v & 0xFFFFFFFFFFFFFFFF for v in out.cpu().tolist()]
            res[name] = {"ms_per_step": round(ms, 3), "value": round((nR + nS) / (ms * 1e-3) / 1e6, 2),
                         "count": c, "count_is_nS": c == nS, "checksum": f"{k:#018x}",
                         "workspace_GiB": round(nbytes / 2**30, 3)}
            log(f"hostruns_large {name}: {ms:.1f} ms, workspace {nbytes / 2**30:.2f} GiB, count {c}")
            del ws

        hb = mpsm.join_host_runs_workspace_bytes(nR, nS, chunk)
        timed("runs_kept", hb, lambda ws: mpsm.join_host_runs_into(R, Sh, runs, out, ws, chunk))
        timed("spilled_runs_rejoined", mpsm.join_spilled_runs_workspace_bytes(nR, nS),
              lambda ws: mpsm.join_spilled_runs_into(R, runs, out, ws))
        timed("runs_not_kept", hb, lambda ws: mpsm.join_host_runs_into(R, Sh, None, out, ws, chunk))
        line = {**base, "value": res["runs_kept"]["value"], "ms_per_step": res["runs_kept"]["ms_per_step"],
                "config": {"workload": "hostruns_large: |R|=2^26, |S|=2^31 uniform foreign keys; S (32 GiB) and "
                                       "its sorted runs in pinned host memory, chunks of 2^24 tuples"},
                "host_link_inclusive": True, "forms": res,
                "device_resident_workspace_GiB": round(mpsm.workspace_bytes(nR, nS) / 2**30, 1)}
    else:   # locskew
        w = workloads.fk_uniform(1 << 24, 1 << 26, seed=0x1207014500000901, spread=True)
        runs = mpsm.layout(len(w.R), len(w.S))["runs"]
        res = {}
        for name, ww in (("unordered", w), ("clustered", workloads.location_skew(w, runs, seed=3))):
            R, S = to_dev(ww.R), to_dev(ww.S)
            ms, r, ws = time_join(mpsm, torch, R, S, mpsm.config(), args, steps)
            del ws
            res[name] = {"ms_per_step": round(ms, 4), "result": r}
            log(f"locskew {name}: {ms:.3f} ms")
        line = {**base, "value": round(((1 << 24) + (1 << 26)) / (res["unordered"]["ms_per_step"] * 1e-3) / 1e6, 2),
                "ms_per_step": res["unordered"]["ms_per_step"],
                "config": {"workload": f"locskew: |R|=2^24, |S|=2^26 uniform foreign keys; S unordered or ordered "
                                       f"small to large in {runs} clusters (one per S run)"}, "orders": res}
    print(json.dumps(line), flush=True)


def measure(args, workload, steps, learned=True):
    """Plain (and learned) form of one single-join workload: timed steps,
    per-step device times, the dominant step's roofline and the whole
    path's."""
    import numpy as np
    import torch
    import paper_1207_0145_amd as mpsm
    import workloads

    log(f"generating {workload}")
    w = workloads.make(workload)
    nR, nS = len(w.R), len(w.S)
    dev = torch.device("cuda", 0)
    R = torch.from_numpy(w.R.view(np.int64)).to(dev)
    S = torch.from_numpy(w.S.view(np.int64)).to(dev)
    del w
    search = {"index": mpsm.SEARCH_INDEX, "binary": mpsm.SEARCH_BINARY, "interp": mpsm.SEARCH_INTERP}[args.search]
    cfg = mpsm.config(search=search)
    cfg_learned = mpsm.config(splitter=mpsm.SPLIT_LEARNED, search=mpsm.SEARCH_LEARNED)
    lay = mpsm.layout(nR, nS, cfg)
    ws = mpsm.alloc_workspace(nR, nS, cfg, dev)
    out = torch.zeros(2, dtype=torch.int64, device=dev)
    names = mpsm.marker_names()
    log(f"{workload}: |R|={nR} |S|={nS} workspace={ws.numel() / 2**30:.2f} GiB runs={lay['runs']} "
        f"R levels={lay['levels']}")
    if args.calibrate_copy:
        x = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        log("copy calibration: 1073741824 bytes read and written once")
        del x, y
    for i in range(args.warmup):
        mpsm.join_into(R, S, out, ws, cfg)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    evsets = [mpsm.EventSet(len(names)) for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for k in range(steps):
        mpsm.join_events_into(R, S, out, ws, evsets[k], cfg)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    log(f"{workload}: timed {steps} steps: {ms:.3f} ms/step")
    count, checksum = [v & 0xFFFFFFFFFFFFFFFF for v in out.cpu().tolist()]
    steps_ms, overlapped = step_times(names, evsets, steps)
    for e in evsets:
        e.close()

    def step_bytes(step):
        rel, b = STEP_BYTES[step]
        return b * {"S": nS, "R": nR, "RS": nR + nS}[rel]

    dom = max((s for s in STEP_BYTES if steps_ms.get(s, 0) > 0), key=lambda s: steps_ms[s])
    achieved = step_bytes(dom) / (steps_ms[dom] * 1e-3) / 1e9
    path_bytes = 48 * nS + 64 * nR
    path_gbs = path_bytes / (ms * 1e-3) / 1e9
    res = {
        "nR": nR, "nS": nS, "ms_per_step": round(ms, 4), "value": round((nR + nS) / (ms * 1e-3) / 1e6, 2),
        "variant": "plain (sampled splitters, " + args.search + " start search)",
        "runs": lay["runs"], "run_len": lay["run_len"], "r_levels": lay["levels"],
        "result": {"count": count, "checksum": f"{checksum:#018x}"},
        "roofline": {"bound": "hbm", "kernel": KERNEL_OF_STEP[dom], "step": dom,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom, workload), "algorithmic_bytes": step_bytes(dom),
                     "avg_launch_ms": round(steps_ms[dom], 4),
                     # the kernel's launch time includes sharing the GPU with
                     # R's phase when that runs on the second stream (beside
                     # S's steps after the scatter)
                     "concurrent_with": "R partitioning and sort (second stream)"
                     if overlapped and dom in ("s_bucket_sort", "s_oversize_sort") else None},
        "path_roofline": {"algorithmic_bytes": path_bytes, "achieved": round(path_gbs, 1), "unit": "GB/s",
                          "frac": round(path_gbs / HBM_PEAK_GBS, 4)},
        "steps_ms": {k: round(v, 4) for k, v in steps_ms.items()},
    }
    if learned:
        res["learned"] = run_variant(mpsm, torch, R, S, out, cfg_learned, args, names, nR, nS,
                                     f"{workload} learned", steps)
        res["learned_over_plain_speedup"] = round(ms / res["learned"]["ms_per_step"], 4)
        res["plain_stats"] = variant_stats(mpsm, torch, R, S, cfg, dev)
    del ws, R, S
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lognormal",
                    choices=["fk_uniform", "fk_small", "skewed", "lognormal", "batch", "negcorr", "roles",
                             "locskew", "hostruns", "hostruns_large"])
    ap.add_argument("--extra", default="fk_uniform,skewed",
                    help="comma-separated single-join workloads reported beside the headline ('' for none)")
    ap.add_argument("--autotune-cache", default=None, help="batch workload: autotuner cache file")
    ap.add_argument("--cpu-sample-shift", type=int, default=4)
    ap.add_argument("--cpu-threads", type=int, default=0, help="threads of the CPU baseline (0: all cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-CDF variant")
    ap.add_argument("--search", default="index", choices=["index", "binary", "interp"])
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--summarize-profiles", nargs=3, metavar=("KERNEL_TRACE_CSV", "FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_<workload>.json from rocprofv3 output (no GPU needed)")
    ap.add_argument("--profile-command", default="", help="command line recorded in the summary")
    ap.add_argument("--summarize-sq", default=None, metavar="SQ_CSV",
                    help="with --summarize-profiles: also the SQ counter run's per-step instruction counts")
    ap.add_argument("--summarize-host-trace", nargs=2, metavar=("KERNEL_TRACE_CSV", "MEMORY_COPY_TRACE_CSV"),
                    help="write profiles/hostruns_fk_uniform.md from a trace of --workload hostruns")
    args = ap.parse_args()
    if args.summarize_host_trace:
        md = summarize_host_trace(*args.summarize_host_trace, args.profile_command)
        with open(os.path.join(ROOT, "profiles", "hostruns_fk_uniform.md"), "w") as f:
            f.write(md)
        print(md)
        return
    if args.summarize_profiles:
        sizes = {"fk_uniform": (1 << 26, 1 << 28), "skewed": (1 << 26, 1 << 28), "fk_small": (1 << 20, 1 << 22),
                 "lognormal": (1 << 28, 1 << 30)}
        nR, nS = sizes[args.workload]
        t = summarize_profiles(*args.summarize_profiles, args.workload, nR, nS, args.profile_command)
        if args.summarize_sq:
            t["sq"] = summarize_sq(args.summarize_sq, nR, nS)
        out = os.path.join(ROOT, "profiles", f"traffic_{args.workload}.json")
        with open(out, "w") as f:
            json.dump(t, f, indent=1)
        with open(os.path.join(ROOT, "profiles", f"pmpsm_join_{args.workload}.md"), "w") as f:
            f.write(profile_markdown(t, args.summarize_profiles[0], args.workload))
        print(json.dumps(t, indent=1))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        batch_bench(args)
        return
    if args.workload in ("negcorr", "roles", "locskew", "hostruns", "hostruns_large"):
        experiment_bench(args)
        return
    import torch
    main_res = measure(args, args.workload, args.steps, learned=not args.no_learned)
    copy_gbs = copy_bandwidth(torch, torch.device("cuda", 0))
    log(f"device copy: {copy_gbs:.0f} GB/s")
    m = main_res
    m["roofline"]["frac_of_measured_copy"] = round(m["roofline"]["achieved"] / copy_gbs, 4)
    m["path_roofline"]["frac_of_measured_copy"] = round(m["path_roofline"]["achieved"] / copy_gbs, 4)
    line = {
        "metric": METRIC, "value": m["value"], "unit": "M tuples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: |R|=2^{m['nR'].bit_length() - 1}, |S|=2^{m['nS'].bit_length() - 1}, "
                               f"{WORKLOAD_KEYS[args.workload]}, 16-byte tuples (u64 key, u64 payload)",
                   "nR": m["nR"], "nS": m["nS"], "variant": m["variant"], "runs": m["runs"], "run_len": m["run_len"],
                   "r_levels": m["r_levels"]},
        "result": m["result"], "roofline": m["roofline"], "path_roofline": m["path_roofline"],
        "measured_copy_GBps": round(copy_gbs, 1), "steps_ms": m["steps_ms"],
    }
    for k in ("learned", "learned_over_plain_speedup", "plain_stats"):
        if k in m:
            line[k] = m[k]
    extras = {}
    for wl in [x for x in args.extra.split(",") if x and x != args.workload]:
        e = measure(args, wl, max(5, args.steps // 2), learned=not args.no_learned)
        e.pop("plain_stats", None)
        if "learned" in e:
            e["learned"].pop("stats", None)
            e["learned"].pop("steps_ms", None)
        extras[wl] = e
    if extras:
        line["other_workloads"] = extras
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        log(f"cpu baseline (oracle, 1 and {threads} threads, 1/{1 << args.cpu_sample_shift} scale)")
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_sample_shift, threads)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
