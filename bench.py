#!/usr/bin/env python3
"""CPMA benchmark on one MI355X.

Headline (printed as one JSON line): batch-update throughput of uniform 40-bit
keys on a CPMA of 1e8 keys, batches of 1e7 -- the paper's microbenchmark
(Section "Evaluation on microbenchmarks": 100 M start, batches of uniform
keys), with every insert batch followed by a delete batch of as many present
keys so that the set stays at 1e8 keys whatever the step count.  A step is one
insert batch and one delete batch (each: sort, locate, merge, density count,
redistribute, resize) over keys already resident in HBM; the value counts the
keys of both batches.

Beside it: per-batch-size insert / delete throughput and p50 / p99 latency
(1e1 .. 1e6, each insert followed by a delete of present keys), a batched
range_map of Zipf(1.2) lengths against one launch per query, bytes per key,
per-phase device time from HIP events recorded inside the library, the roofline
of the dominant kernel, and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "insert keys/s at batch 1e3–1e7; range_map keys/s (%HBM peak); p99 latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# ---- HBM traffic of the main merge kernel from rocprofv3 counter runs ------------
MERGE_KERNEL = "k_merge_wave<unsigned int>"
MERGE_SOURCES = ["common.hpp", "leaf.hpp", "update.hpp", "merge_wave.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_merge_wave_traffic_update_pairs1e7_n1e8.md")
VALU_FILE = os.path.join(ROOT, "profiles", "k_merge_wave_valu_update_pairs1e7_n1e8.md")
# VALU reference rate: 256 CUs x 4 SIMDs, one wave64 VALU instruction per SIMD
# every 4 cycles (16 lanes), 2.4 GHz peak engine clock.  Not a ceiling: gfx950
# issues some wave64 VALU instructions in fewer cycles.
VALU_PEAK_INSTS_PER_S = 256 * 4 * 2.4e9 / 4


SCAN_KERNEL = "k_rm_interior<true>"
SCAN_SOURCES = ["common.hpp", "scan_lane.hpp", "query.hpp"]
# after the timed steps the headline run takes PHASE_STEPS more steps (every
# phase timed); each step merges twice (its insert and its delete batch)
PHASE_STEPS = 3
MERGES_PER_STEP = 2
TAIL_MERGES = MERGES_PER_STEP * PHASE_STEPS
SCAN_VALU_FILE = os.path.join(ROOT, "profiles", "k_rm_interior_valu_gate_n1e9.md")


def run_key(args, kind="steps"):
    """What a counter summary must have been taken on to be reported beside this
    run: the kernel's sources and the run's shape."""
    if kind == "gate":
        return {"source": merge_source_hash(SCAN_SOURCES), "serve_n": str(int(args.serve_n))}
    return {"source": merge_source_hash(), "steps": str(args.steps), "warmup": str(args.warmup),
            "n0": str(int(args.n)), "batch": str(int(args.batch))}


def key_lines(key):
    return [f"{k}={v}" for k, v in key.items()]


def read_summary(path, key):
    """The key=value block of a committed counter summary, or None when it is
    missing or was taken on other sources or another run shape."""
    try:
        with open(path) as fh:
            kv = dict(l.strip().split("=", 1) for l in fh if "=" in l and not l.startswith("|"))
    except OSError:
        return None
    if any(kv.get(k) != v for k, v in key.items()):
        return None
    return kv


def merge_source_hash(sources=None):
    """Hash of the sources that define a kernel (default: the main merge kernel):
    counters taken on another version of it are not reported."""
    import hashlib
    h = hashlib.sha256()
    for f in (sources or MERGE_SOURCES):
        with open(os.path.join(ROOT, "paper_2305_05055_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_rows(path):
    import csv
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("cpma_dev::", "")
            rows.append((int(r["Dispatch_Id"]), name, r["Counter_Name"], float(r["Counter_Value"])))
    rows.sort()
    return rows


def pmc_summary(fetch_csv, write_csv, steps, cmd_fetch, cmd_write, key):
    """Traffic per timed launch of the merge kernel: FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch), each scaled by what the counter reads for the 1 GiB
    calibration copy (the largest copy dispatch of the run)."""
    out = {}
    for tag, path, ctr in (("read", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = [r for r in pmc_rows(path) if r[2] == ctr]
        copy = max(v for _, n, _, v in rows if n == "__amd_rocclr_copyBuffer")
        factor = float(1 << 30) / (copy * 1024.0)
        merge = [v for _, n, _, v in rows if n == MERGE_KERNEL]
        timed = merge[-(MERGES_PER_STEP * steps + TAIL_MERGES):-TAIL_MERGES]
        out[tag] = {"copy_kib": copy, "factor": factor,
                    "kib_per_launch": sum(timed) / len(timed),
                    "bytes_per_launch": sum(timed) / len(timed) * 1024.0 * factor,
                    "launches": len(timed)}
    total = out["read"]["bytes_per_launch"] + out["write"]["bytes_per_launch"]
    lines = [
        f"# {MERGE_KERNEL}: HBM traffic per launch, insert + delete batch pairs of 1e7 on 1e8 keys", "",
        "Two counter runs of the headline steps (each run in /tmp after "
        "`cd /tmp && export TMPDIR=/tmp`):", "", "```", cmd_fetch, cmd_write, "```", "",
        "The first dispatch of each run is a 1 GiB device-to-device copy "
        "(`--calibrate-copy`); the counter's reading for it gives the scale factor "
        "(bytes actually moved / counter bytes).", "",
        "| counter | calibration copy (KiB) | factor | per timed launch (KiB) | per launch (bytes, scaled) |",
        "|---|---|---|---|---|"]
    for tag, ctr in (("read", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        o = out[tag]
        lines.append(f"| {ctr} | {o['copy_kib']:.1f} | {o['factor']:.4f} | {o['kib_per_launch']:.1f} | "
                     f"{o['bytes_per_launch']:.4e} |")
    lines += ["", f"Timed launches averaged: {out['read']['launches']}.", "",
              "Machine-readable (read by bench.py, which reports the figure only for a run of the "
              "same shape on the same kernel sources; `source` is the hash of the kernel's sources "
              "when the counters were taken):", "", "```",
              f"traffic_bytes_per_launch={total:.6e}"] + key_lines(key) + ["```", ""]
    return "\n".join(lines)


def valu_summary(csv_path, kernel, pick, title, what, cmd, key):
    """VALU (and LDS, SALU) instructions and waves per launch of `kernel` from one
    rocprofv3 --pmc run; pick(list) selects the launches to average."""
    ctrs = ("SQ_INSTS_VALU", "SQ_WAVES", "SQ_INSTS_LDS", "SQ_INSTS_SALU")
    rows = pmc_rows(csv_path)
    avg = {}
    for ctr in ctrs:
        timed = pick([v for _, n, c, v in rows if n == kernel and c == ctr])
        avg[ctr] = sum(timed) / len(timed)
        nl = len(timed)
    lines = [
        f"# {kernel}: instructions per launch, {title}", "",
        f"One counter run of {what} (run in /tmp after "
        "`cd /tmp && export TMPDIR=/tmp`):", "", "```", cmd, "```", "",
        "Counts are chip totals per dispatch (SQ_WAVES equals the launched waves).  bench.py "
        "divides the per-launch count by the launch time it measures and by a reference rate of "
        "one wave64 VALU instruction per SIMD every 4 cycles at 2.4 GHz (256 CUs x 4 SIMDs x "
        "2.4 GHz / 4 = 6.1e11 wave instructions/s).  The ratio is a reference, not a ceiling: "
        "gfx950 issues some wave64 VALU instructions in fewer cycles, and the merge kernel "
        "measures above 1.", "",
        "| counter | per timed launch |", "|---|---|"]
    for ctr in ctrs:
        lines.append(f"| {ctr} | {avg[ctr]:.4e} |")
    lines += ["", f"Launches averaged: {nl}.", "",
              "Machine-readable (read by bench.py, which reports the figure only for a run of the "
              "same shape on the same kernel sources; `source` is the hash of the kernel's sources "
              "when the counters were taken):", "", "```",
              f"valu_insts_per_launch={avg['SQ_INSTS_VALU']:.6e}", f"waves_per_launch={avg['SQ_WAVES']:.6e}"]
    lines += key_lines(key) + ["```", ""]
    return "\n".join(lines)


def kernel_valu(path, key):
    """VALU instructions per launch from a committed counter summary, or None."""
    kv = read_summary(path, key)
    return float(kv["valu_insts_per_launch"]) if kv else None


def merge_traffic(key):
    """HBM bytes per merge launch from the committed counter summary, or None."""
    kv = read_summary(TRAFFIC_FILE, key)
    return float(kv["traffic_bytes_per_launch"]) if kv else None


PROF_DIR = "/tmp/cpma_prof"
STEPS_TRACE_FILE = os.path.join(ROOT, "profiles", "update_pairs1e7_n1e8_kernel_trace.md")
GATE_TRACE_FILE = os.path.join(ROOT, "profiles", "range_gate_n1e9_kernel_trace.md")


def trace_rows(path):
    """(dispatch id, kernel name, duration ns) of every row of a rocprofv3
    kernel_trace.csv, in dispatch order."""
    import csv
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("cpma_dev::", "")
            rows.append((int(r["Dispatch_Id"]), name, int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    rows.sort()
    return rows


def trace_table(rows):
    per = {}
    for _, name, ns in rows:
        c, t = per.get(name, (0, 0))
        per[name] = (c + 1, t + ns)
    total = sum(t for _, t in per.values())
    lines = ["| kernel | calls | total ms | avg us | share |", "|---|---|---|---|---|"]
    for name, (c, t) in sorted(per.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| `{name}` | {c} | {t * 1e-6:.3f} | {t * 1e-3 / c:.1f} | {100.0 * t / total:.1f}% |")
    return lines, total


# diagnostic runs summarised whole: flag, summary file, title, what the run does
WHOLE_RUN_TRACES = {
    "range": ("--range-only", "range_map_zipf1e6_n1e8_kernel_trace.md",
              "range_map: 1e6 Zipf(1.2) exact-count queries on a 1e8-key CPMA",
              "The run builds the 1e8-key set and times the batched range_map on the default layout (3 passes "
              "after a warm-up), runs the autotuner (its trial builds on a sample included), times the autotuned "
              "layout, then 2000 single-query launches against one batched launch of the same 2000, 64 short "
              "queries eager and from a HIP graph, and 6 contains calls of 1e6 keys.  Every kernel of the run."),
    "sweep": ("--sweep-only", "small_batches_sweep_n1e8_kernel_trace.md",
              "insert and delete batches of 10 to 1e6 keys on a 1e8-key CPMA",
              "The run builds the 1e8-key set, then for each batch size alternates an insert of fresh keys "
              "and a delete of present keys (30 / 30 / 20 / 10 / 5 / 3 of each at 10 / 100 / 1e3 / 1e4 / 1e5 "
              "/ 1e6 keys; up to 4096 keys the one-workgroup preparation k_small_prep, above it the sorted "
              "pipeline).  Every kernel of the run."),
    "fg": ("--fg-only", "fgraph_rmat24_er_kernel_trace.md",
           "F-Graph on a symmetric R-MAT graph (scale 24) and an Erdos-Renyi graph (1e7 vertices, p = 5e-6)",
           "Each graph is built from device-generated edges, then BFS from vertex 0, 10 PageRank iterations, "
           "the vertex offsets, connected components and single-source betweenness, each timed after a "
           "warm-up; on the R-MAT graph also edge-insert batches of 1e5, 1e6 and 1e7.  Every kernel of the run "
           "(torch's generator kernels included)."),
}


# the kernels that open an update batch: validation alone, with the first LSD
# digit's counts, or with the MSD split's bucket counts
VALIDATION_KERNELS = ("k_validate", "k_validate_hist", "k_validate_msd")
# the fills before it
CLEAR_KERNELS = ("k_fill", "k_clear2")


def trace_summary(kind, csv_path, args):
    """Markdown summary of a rocprofv3 --kernel-trace run.  steps: the kernels of
    the timed headline steps (every update batch opens with its validation
    kernel, after the fills that clear its counters and flags; the timed
    batches are the 2K before the last PHASE_STEPS steps' 2 * PHASE_STEPS); gate: every launch from the first range_map kernel
    on (one warm-up and three timed passes of the cold range gate)."""
    rows = trace_rows(csv_path)
    shape = f"--steps {args.steps} --warmup {args.warmup}"
    if kind == "steps":
        cmd = ("rocprofv3 --kernel-trace --stats --output-format csv -d " + PROF_DIR + "/tr_steps -o run -- "
               f"python3 /root/repo/bench.py --only-steps --no-cpu-baseline {shape}")
        starts = [i for i, r in enumerate(rows) if r[1] in VALIDATION_KERNELS]
        nb = MERGES_PER_STEP * args.steps
        first, last = starts[-(nb + TAIL_MERGES)], starts[-TAIL_MERGES]
        # each batch's validation follows the fills that clear its counters
        # and flags
        while rows[first - 1][1].startswith(CLEAR_KERNELS):
            first -= 1
        while rows[last - 1][1].startswith(CLEAR_KERNELS):
            last -= 1
        sel = rows[first:last]
        title = "insert + delete batch pairs of 1e7 uniform 40-bit keys on a 1e8-key CPMA"
        what = (f"The run builds the 1e8-key set, takes {args.warmup} warm-up and {args.steps} timed steps "
                f"(each an insert batch of 1e7 fresh keys and a delete batch of 1e7 present keys), then "
                f"{PHASE_STEPS} more steps with every phase timed.  The table covers the {nb} batches of the "
                "timed steps: from the first launch of the first timed batch to the last launch before the "
                "first of the phase-timed batches.")
        out = STEPS_TRACE_FILE
    elif kind in WHOLE_RUN_TRACES:
        flag, fname, title, what = WHOLE_RUN_TRACES[kind]
        cmd = ("rocprofv3 --kernel-trace --stats --output-format csv -d " + PROF_DIR + f"/tr_{kind} -o run -- "
               f"python3 /root/repo/bench.py {flag}")
        sel = rows
        out = os.path.join(ROOT, "profiles", fname)
    else:
        cmd = ("rocprofv3 --kernel-trace --stats --output-format csv -d " + PROF_DIR + "/tr_gate -o run -- "
               "python3 /root/repo/bench.py --gate-only")
        first = next(i for i, r in enumerate(rows) if r[1].startswith("k_rm_"))
        sel = rows[first:]
        title = "range_map on cold data, 1e9 keys"
        what = ("The run builds a set of 1e9 uniform 40-bit keys and runs the cold range gate: 1e3 queries "
                "of about 1e6 keys at random starts plus one query over the whole key space, one warm-up "
                "pass and three timed passes.  The table covers every launch from the first range_map "
                "kernel on.")
        out = GATE_TRACE_FILE
    table, total = trace_table(sel)
    lines = [f"# Kernel trace: {title}", "", "Command (run in /tmp after "
             "`cd /tmp && export TMPDIR=/tmp`):", "", "```", cmd, "```", "", what, "",
             f"Launches: {len(sel)}; kernel time: {total * 1e-6:.3f} ms.", ""] + table + [""]
    text = "\n".join(lines)
    with open(out, "w") as fh:
        fh.write(text)
    print(text)


def host_info():
    """The host CPU the oracle ran on: model name and usable cores."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def zipf_section(cp, torch, c, seed, sizes=(10 ** 5, 10 ** 6, 10 ** 7), reps=3):
    """Skewed batches on the uniform set c: inserts of k Zipf(0.99) 34-bit keys
    (Section "Evaluation on microbenchmarks", setup), each followed by a delete
    batch of k keys from the same distribution (mostly present, repeats
    included), as the paper's Zipf insert / delete table."""
    out = {"keys": "Zipf(0.99) over 34-bit keys, unscrambled (popular keys are small)",
           "paper_context": "paper, 64-core Xeon, inserts/s (deletes/s): 1e5 7.2e7 (8.7e7), "
                            "1e6 1.7e8 (2.2e8), 1e7 3.1e8 (4.6e8)"}
    off = 0
    for k in sizes:
        ins = [to_dev(synth.zipf_keys(k, seed, offset=off + 2 * i * k)) for i in range(reps)]
        dls = [to_dev(synth.zipf_keys(k, seed, offset=off + (2 * i + 1) * k)) for i in range(reps)]
        off += 2 * reps * k
        torch.cuda.synchronize()
        ti, td, added, removed = [], [], 0, 0
        for i in range(reps):
            t0 = time.perf_counter()
            added += c.insert_batch(ins[i])
            t1 = time.perf_counter()
            removed += c.delete_batch(dls[i])
            t2 = time.perf_counter()
            ti.append(t1 - t0)
            td.append(t2 - t1)
        out[f"{k:.0e}"] = {"insert_keys_s": k / float(np.mean(ti)), "delete_keys_s": k / float(np.mean(td)),
                           "distinct_added_per_batch": added / reps, "removed_per_batch": removed / reps,
                           "insert_p50_ms": float(np.percentile(ti, 50) * 1e3), "reps": reps}
    log(f"zipf: {out}")
    return out


def growth_section(cp, torch, base_dev, seed, factors=(1.1, 1.2, 1.5, 2.0), batches=10, k=10 ** 7):
    """The growing-factor sweep of the paper's appendix: for each factor, the
    set of 1e8 uniform keys takes 1e8 more in batches of 1e7; total insert time,
    bytes per key after each batch (average and worst) and a full-range scan
    after each batch (average)."""
    out = {"setup": "build 1e8 uniform 40-bit keys, insert 10 batches of 1e7 fresh keys; "
                    "after each batch: bytes/key and one full-range range_map"}
    full_lo = to_dev(np.array([0], np.uint64))
    full_hi = to_dev(np.array([(1 << 64) - 1], np.uint64))
    bs = [to_dev(synth.uniform_keys(k, seed, offset=i * k)) for i in range(batches)]
    for g in factors:
        cfg = cp.default_config()
        cfg.grow = g
        cfg.build_density = 0.0
        c = cp.CPMA(base_dev, config=cfg)
        c.range_map(full_lo, full_hi)
        torch.cuda.synchronize()
        t_ins, sizes, scans, grows = 0.0, [], [], 0
        L_prev = c.geometry()[0]
        for b in bs:
            t0 = time.perf_counter()
            c.insert_batch(b)
            t_ins += time.perf_counter() - t0
            L = c.geometry()[0]
            grows += L > L_prev
            L_prev = L
            sizes.append(c.bytes() / c.size())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.range_map(full_lo, full_hi)
            torch.cuda.synchronize()
            scans.append(time.perf_counter() - t0)
        out[str(g)] = {"insert_keys_s": batches * k / t_ins, "bytes_per_key_avg": float(np.mean(sizes)),
                       "bytes_per_key_max": float(np.max(sizes)), "full_scan_ms_avg": float(np.mean(scans)) * 1e3,
                       "grows": int(grows)}
        c.close()
        torch.cuda.empty_cache()
    best_ins = max(out[str(g)]["insert_keys_s"] for g in factors)
    for g in factors:
        out[str(g)]["insert_ratio_from_best"] = out[str(g)]["insert_keys_s"] / best_ins
    log(f"growth: {out}")
    return out


def pma_section(cp, torch, base_dev, seed, k=10 ** 7, warm=2, steps=5, q=100_000):
    """The paper's compression ablation: the same 1e8 uniform 40-bit keys as the
    CPMA and as the uncompressed PMA (raw 8-byte keys per leaf, same leaves,
    bounds and batch algorithm).  For each: bytes per key, insert + delete
    steps of 1e7-key batches (as the headline), batched range_map of q Zipf(1.2)
    exact-count queries on 1..1e6 keys, and one scan of the whole set."""
    keys_sorted = torch.unique(base_dev).cpu().numpy().view(np.uint64)
    lens = synth.zipf_lengths(q, seed, alpha=1.2, lmax=10 ** 6)
    lo, hi = synth.range_queries_by_count(keys_sorted, lens, seed + 1)
    first_del = to_dev(keys_sorted[synth.sample_indices(len(keys_sorted), k, seed + 2)])
    del keys_sorted
    dlo, dhi = to_dev(lo), to_dev(hi)
    ins = [to_dev(synth.uniform_keys(k, seed + 3, offset=(i + 50) * k)) for i in range(warm + steps)]
    full_lo = to_dev(np.array([0], np.uint64))
    full_hi = to_dev(np.array([(1 << 64) - 1], np.uint64))
    out = {"n0": int(base_dev.numel()), "batch": k, "steps": steps, "queries": q,
           "paper_context": "paper, 64 cores: the CPMA beats the PMA on batch inserts from 16 cores up "
                            "(memory bandwidth) and on the largest range queries (1.3x); the PMA wins small "
                            "ranges (no decoding)"}
    for name, unc in (("cpma", False), ("pma", True)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = cp.CPMA(base_dev, uncompressed=unc)
        torch.cuda.synchronize()
        r = {"build_s": time.perf_counter() - t0, "bytes_per_key": c.bytes() / c.size(),
             "leaves": c.geometry()[0]}
        for i in range(warm):
            c.insert_batch(ins[i])
            c.delete_batch(first_del if i == 0 else ins[i - 1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(warm, warm + steps):
            c.insert_batch(ins[i])
            c.delete_batch(ins[i - 1])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        r["update_keys_s"] = 2 * k * steps / dt
        r["ms_per_step"] = dt / steps * 1e3
        tr = time_range(torch, c, dlo, dhi)
        r["range_keys_s"] = tr["keys_per_s"]
        r["range_scan_alg_GBps"] = tr["scan_alg_GBps"]
        c.range_map(full_lo, full_hi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            c.range_map(full_lo, full_hi)
        torch.cuda.synchronize()
        r["full_scan_ms"] = (time.perf_counter() - t0) / 5 * 1e3
        r["full_scan_keys_s"] = c.size() / (r["full_scan_ms"] * 1e-3)
        r["bytes_after"] = c.bytes()
        out[name] = r
        c.close()
        torch.cuda.empty_cache()
    out["pma_over_cpma"] = {key: out["pma"][key] / out["cpma"][key]
                            for key in ("bytes_per_key", "update_keys_s", "range_keys_s", "full_scan_keys_s")}
    log(f"pma vs cpma: {out}")
    return out


def kv_section(cp, torch, base_dev, seed, k=10 ** 7, warm=2, steps=5, q=100_000, fg_scale=24, leaf_bytes=0):
    """The key-value CPMA: the 1e8 uniform 40-bit keys with random 8-byte values.
    Bytes per key; steps of an upsert of 1e7 fresh key-value pairs and a delete
    of 1e7 present keys (as the headline); the same upsert on present keys
    (value overwrites); get of 1e6 keys; range_map_values of q Zipf(1.2)
    exact-count queries.  Then a weighted F-Graph: the R-MAT graph of the
    F-Graph section with random edge weights, and every vertex's weighted
    degree (one range_map_values query per vertex)."""
    n0 = int(base_dev.numel())
    vals = synth.uniform_keys_torch(n0, seed, "cuda", bits=64)
    keys_sorted = torch.unique(base_dev).cpu().numpy().view(np.uint64)
    lens = synth.zipf_lengths(q, seed + 1, alpha=1.2, lmax=10 ** 6)
    lo, hi = synth.range_queries_by_count(keys_sorted, lens, seed + 2)
    first_del = to_dev(keys_sorted[synth.sample_indices(len(keys_sorted), k, seed + 3)])
    probe = to_dev(np.concatenate([keys_sorted[synth.sample_indices(len(keys_sorted), 500000, seed + 4)],
                                   synth.uniform_keys(500000, seed + 5)]))
    over = to_dev(keys_sorted[synth.sample_indices(len(keys_sorted), k, seed + 6)])
    del keys_sorted
    dlo, dhi = to_dev(lo), to_dev(hi)
    ins = [to_dev(synth.uniform_keys(k, seed + 7, offset=(i + 90) * k)) for i in range(warm + steps)]
    ivals = synth.uniform_keys_torch(k, seed + 8, "cuda", bits=64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c = cp.CPMA(base_dev, values=vals, leaf_bytes=leaf_bytes)
    torch.cuda.synchronize()
    out = {"n0": n0, "batch": k, "steps": steps, "build_s": time.perf_counter() - t0,
           "bytes_per_key": c.bytes() / c.size(), "leaf_bytes": c.geometry()[1], "leaves": c.geometry()[0],
           "layout": "keys delta-coded as in the CPMA, 8-byte values at each leaf's end"}
    for i in range(warm):
        c.insert_kv(ins[i], ivals)
        c.delete_batch(first_del if i == 0 else ins[i - 1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(warm, warm + steps):
        c.insert_kv(ins[i], ivals)
        c.delete_batch(ins[i - 1])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["upsert_delete_keys_s"] = 2 * k * steps / dt
    out["ms_per_step"] = dt / steps * 1e3
    c.insert_kv(over, ivals)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        c.insert_kv(over, ivals)
    torch.cuda.synchronize()
    out["overwrite_1e7_present_keys_s"] = 3 * k / (time.perf_counter() - t0)
    c.get(probe)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        c.get(probe)
    torch.cuda.synchronize()
    out["get_1e6_per_s"] = 5 * probe.numel() / (time.perf_counter() - t0)
    c.range_map_values(dlo, dhi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        s_, n_ = c.range_map_values(dlo, dhi)
    torch.cuda.synchronize()
    dtq = (time.perf_counter() - t0) / 3
    out["range_values_keys_s"] = int(n_.sum().item()) / dtq
    out["range_values_queries"] = q
    c.close()
    del vals, ivals, ins, first_del, probe, over, dlo, dhi
    torch.cuda.empty_cache()
    if fg_scale > 0:
        nv = 1 << fg_scale
        src, dst = synth.rmat_edges_torch(nv * 8, seed + 10, scale=fg_scale, device="cuda")
        ekeys = synth.edge_keys_torch(src, dst)
        del src, dst
        w = synth.uniform_keys_torch(int(ekeys.numel()), seed + 11, "cuda", bits=20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = cp.CPMA(ekeys, values=w, leaf_bytes=min(leaf_bytes or 1024, 1024))
        torch.cuda.synchronize()
        wg = {"scale": fg_scale, "edges": g.size(), "build_s": time.perf_counter() - t0,
              "bytes_per_edge": g.bytes() / g.size()}
        del ekeys, w
        vlo = torch.arange(nv, device="cuda", dtype=torch.int64) << 32
        vhi = vlo + (1 << 32)
        g.range_map_values(vlo, vhi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.range_map_values(vlo, vhi)
        torch.cuda.synchronize()
        wg["weighted_degrees_ms"] = (time.perf_counter() - t0) * 1e3
        g.bfs(nv, 0, symmetric=True, device=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.bfs(nv, 0, symmetric=True, device=True)
        torch.cuda.synchronize()
        wg["bfs_ms"] = (time.perf_counter() - t0) * 1e3
        out["weighted_fgraph"] = wg
        g.close()
        torch.cuda.empty_cache()
    log(f"key-value: {out}")
    return out


def rebuild_section(cp, torch, base_dev, seed, fracs=(0.1, 1.0)):
    """Both branches of a large insert batch on the 1e8-key set, at k = n / 10
    and k = n: the full rebuild (every leaf merged, then everything spread at
    build density) and the counted batch path (count, redistribute, grow).
    Each insert is timed once after a warm-up of the same size, on a fresh
    set."""
    n = int(base_dev.numel())
    out = {}
    for f in fracs:
        k = int(f * n)
        bs = [to_dev(synth.uniform_keys(k, seed, offset=i * k)) for i in range(2)]
        row = {}
        for tag, rf in (("rebuild", f * 0.5), ("batch_path", 1e9)):
            cfg = cp.default_config()
            cfg.rebuild_frac = rf
            c = cp.CPMA(base_dev, config=cfg)
            c.insert_batch(bs[0])           # warm-up: sizes the scratch
            c.delete_batch(bs[0])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.insert_batch(bs[1])
            torch.cuda.synchronize()
            row[tag + "_insert_ms"] = (time.perf_counter() - t0) * 1e3
            t0 = time.perf_counter()
            c.delete_batch(bs[1])
            torch.cuda.synchronize()
            row[tag + "_delete_ms"] = (time.perf_counter() - t0) * 1e3
            c.close()
            torch.cuda.empty_cache()
        out[f"k_over_n_{f:g}"] = row
        del bs
    log(f"rebuild vs batch path: {out}")
    return out


def graph_kernels(g, torch, nv):
    """The vertex offset array, connected components and single-source
    betweenness from vertex 0 (outputs in HBM), each timed once after a warm-up."""
    out = {}
    for name, fn in (("offsets_ms", lambda: g.offsets(nv, device=True)),
                     ("cc_ms", lambda: g.cc(nv, device=True)),
                     ("bc_ms", lambda: g.bc(nv, 0, device=True))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t0) * 1e3
        if name == "cc_ms":
            lab = r
            out["components"] = int((lab == torch.arange(nv, device=lab.device, dtype=lab.dtype)).sum().item())
    return out


def er_section(cp, torch, seed, n=10 ** 7, p=5e-6):
    """The paper's synthetic graph: Erdos-Renyi with n = 1e7 vertices and edge
    probability 5e-6 (n^2 p ordered pairs drawn uniformly, self-loops dropped,
    symmetrised), stored as one CPMA; BFS, 10 PageRank iterations, CC, BC."""
    m = int(n * n * p)
    s, d = synth.er_edges_torch(m, seed, n, device="cuda")
    keys = synth.edge_keys_torch(s, d)
    del s, d
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = cp.CPMA(keys)
    torch.cuda.synchronize()
    out = {"vertices": n, "edge_prob": p, "edges": g.size(), "build_s": time.perf_counter() - t0,
           "bytes_per_edge": g.bytes() / g.size(), "gbytes": g.bytes() / 1e9}
    del keys
    torch.cuda.empty_cache()
    g.bfs(n, 0, symmetric=True, device=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.bfs(n, 0, symmetric=True, device=True)
    torch.cuda.synchronize()
    out["bfs_ms"] = (time.perf_counter() - t0) * 1e3
    g.pagerank(n, iters=1, device=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.pagerank(n, iters=10, device=True)
    torch.cuda.synchronize()
    out["pagerank_10_iters_ms"] = (time.perf_counter() - t0) * 1e3
    out.update(graph_kernels(g, torch, n))
    log(f"er graph: {out}")
    g.close()
    return out


def fgraph_section(cp, torch, scale, seed):
    """F-Graph: symmetric R-MAT graph with 2^scale vertices from 2^(scale+3) samples."""
    nv = 1 << scale
    src, dst = synth.rmat_edges_torch(1 << (scale + 3), seed, scale=scale, device="cuda")
    keys = synth.edge_keys_torch(src, dst)
    del src, dst
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = cp.CPMA(keys)
    torch.cuda.synchronize()
    out = {"scale": scale, "vertices": nv, "edges": g.size(), "build_s": time.perf_counter() - t0,
           "bytes_per_edge": g.bytes() / g.size()}
    del keys
    # outputs stay in HBM while timed (a host copy of 2^24 levels would add a
    # 64 MB PCIe transfer to an algorithm that runs in memory)
    g.bfs(nv, 0, symmetric=True, device=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lv = g.bfs(nv, 0, symmetric=True, device=True)
    torch.cuda.synchronize()
    out["bfs_ms"] = (time.perf_counter() - t0) * 1e3
    lv = lv.cpu().numpy().view(np.uint32)
    reach = lv[lv != 0xFFFFFFFF]
    out["bfs_levels"] = int(reach.max()) + 1
    out["bfs_reached"] = int(len(reach))
    g.pagerank(nv, iters=1, device=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.pagerank(nv, iters=10, device=True)
    torch.cuda.synchronize()
    out["pagerank_10_iters_ms"] = (time.perf_counter() - t0) * 1e3
    out.update(graph_kernels(g, torch, nv))
    ins = {}
    for k in (10 ** 5, 10 ** 6, 10 ** 7):
        s2, d2 = synth.rmat_edges_torch(k // 2, seed + k, scale=scale, device="cuda")
        b = synth.edge_keys_torch(s2, d2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.insert_batch(b)
        ins[f"{k:.0e}"] = len(b) / (time.perf_counter() - t0)
    out["edge_insert_keys_s"] = ins
    log(f"fgraph: {out}")
    g.close()
    return out


def time_range(torch, c, dlo, dhi, reps=3):
    """Batched range_map on device queries: wall time per pass and the scan
    kernel's algorithmic bytes and device time from the library's HIP events."""
    c.range_map(dlo, dhi)
    torch.cuda.synchronize()
    c.stats_select(["range_scan"])
    t0 = time.perf_counter()
    for _ in range(reps):
        s_, n_ = c.range_map(dlo, dhi)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    st = c.stats()
    c.stats_enable(False)
    keys = int(n_.sum().item())
    sc_launch, sc_ms, sc_bytes = st["range_scan"]
    out = {"keys_per_pass": keys, "keys_per_s": keys / dt, "ms_per_pass": dt * 1e3,
           "scan_kernel_ms": sc_ms / max(1, sc_launch), "scan_alg_bytes": sc_bytes / max(1, sc_launch)}
    out["scan_alg_GBps"] = out["scan_alg_bytes"] / (out["scan_kernel_ms"] * 1e-3) / 1e9
    out["frac_hbm_alg"] = out["scan_alg_GBps"] / HBM_PEAK_GBS
    return out


def redist_section(cp, torch, seed, n=10 ** 7, batches=8, k=20000):
    """Window redistribution: a set of n uniform 40-bit keys, then insert batches
    whose k keys all fall in one narrow key range (2^28 of the 2^40 key space, a
    different range per batch), so that a few leaves overflow and windows of many
    leaves are rebuilt without growing the set.  REDIST phase time and
    algorithmic bytes (every window leaf read and rewritten) from the library's
    HIP events."""
    c = cp.CPMA(to_dev(synth.uniform_keys(n, seed)))
    starts = synth.uniform_keys(batches + 1, seed + 1, bits=40)
    bs = [to_dev(int(x0) + synth.uniform_keys(k, seed + 2 + i, bits=28)) for i, x0 in enumerate(starts)]
    c.insert_batch(bs[0])  # warm-up
    torch.cuda.synchronize()
    L0 = c.geometry()[0]
    c.stats_select(["redist"])
    t0 = time.perf_counter()
    for b in bs[1:]:
        c.insert_batch(b)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = c.stats()
    c.stats_enable(False)
    launches, ms, alg = st["redist"]
    out = {"n": n, "batches": batches, "batch_keys": k, "key_range_bits": 28,
           "leaves_before": L0, "leaves_after": c.geometry()[0],
           "insert_keys_s": batches * k / dt, "redist_rounds": launches,
           "redist_ms_per_batch": ms / batches,
           "redist_alg_GBps": (alg / (ms * 1e-3) / 1e9) if ms > 0 else None}
    out["redist_frac_hbm_alg"] = out["redist_alg_GBps"] / HBM_PEAK_GBS if out["redist_alg_GBps"] else None
    log(f"redistribution: {out}")
    c.close()
    return out


def range_cpu_baseline(keys_sorted, lo, hi, target_keys=6e9):
    """The oracle's lower_bound + sum on a prefix of the same queries holding
    about target_keys keys, on one host core and on every usable core."""
    import oracle
    lens_est = np.searchsorted(keys_sorted, hi) - np.searchsorted(keys_sorted, lo)
    m = int(np.searchsorted(np.cumsum(lens_est), target_keys)) + 1
    m = min(m, len(lo))
    keys = int(lens_est[:m].sum())
    out = {"queries": m, "keys": keys, "kind": "oracle", "unit": "keys/s",
           "sample": f"the first {m} of the Zipf(1.2) queries ({keys:.3e} keys): lower_bound + sum"}
    threads = len(os.sched_getaffinity(0))
    for tag, th in (("one_core", 0), ("all_cores", threads)):
        t0 = time.perf_counter()
        oracle.range_map(keys_sorted, lo[:m], hi[:m], threads=th)
        dt = time.perf_counter() - t0
        out[tag] = {"value": keys / dt, "cores": max(1, th), "s": dt}
    out["host"] = host_info()
    log(f"range cpu baseline: {out}")
    return out


def range_section(cp, torch, c, base_dev, q, seed, with_cpu=False):
    """Batched range_map on the 1e8-key set: q queries whose lengths (in keys)
    are Zipf(1.2) on 1..1e6, each covering exactly its length of the sorted set;
    on the default layout and on the autotuned one; against one launch per query."""
    keys_sorted = torch.unique(base_dev).cpu().numpy().view(np.uint64)
    lens = synth.zipf_lengths(q, seed, alpha=1.2, lmax=10 ** 6)
    lo, hi = synth.range_queries_by_count(keys_sorted, lens, seed + 1)
    # membership: 1e6 keys, half drawn from the set and half fresh
    probe = np.concatenate([keys_sorted[synth.sample_indices(len(keys_sorted), 500000, seed + 2)],
                            synth.uniform_keys(500000, seed + 3)])
    cpu = range_cpu_baseline(keys_sorted, lo, hi) if with_cpu else None
    del keys_sorted
    dlo, dhi = to_dev(lo), to_dev(hi)
    out = {"queries": q, "lengths": "Zipf(1.2) on 1..1e6 keys, exact counts",
           "default": time_range(torch, c, dlo, dhi), "cpu_baseline": cpu}
    dprobe = to_dev(probe)
    c.contains(dprobe)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        hit = c.contains(dprobe)
    torch.cuda.synchronize()
    out["contains_1e6_per_s"] = 5 * len(probe) / (time.perf_counter() - t0)
    out["contains_hits"] = int(hit.sum().item())
    cfg, rep = cp.autotune(base_dev, insert_weight=0.0, range_keys=int(lens.mean()), queries=100_000)
    out["autotune"] = rep
    tuned = cp.CPMA(base_dev, config=cfg)
    torch.cuda.synchronize()
    res = time_range(torch, tuned, dlo, dhi)
    res["leaf_bytes"], res["range_chunk"] = int(cfg.leaf_bytes), int(cfg.range_chunk)
    out["autotuned"] = res
    # one launch per query on a prefix of the same queries
    m = min(2000, q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(m):
        tuned.range_map(dlo[i:i + 1], dhi[i:i + 1])
    torch.cuda.synchronize()
    per_q = (time.perf_counter() - t0) / m
    one = [tuned.range_map(dlo[i:i + 1], dhi[i:i + 1]) for i in range(m)]  # untimed: their results
    one_s = torch.cat([x[0] for x in one])
    one_n = torch.cat([x[1] for x in one])
    del one
    t0 = time.perf_counter()
    bs, bn = tuned.range_map(dlo[:m], dhi[:m])
    torch.cuda.synchronize()
    out["one_launch_per_query_s_per_query"] = per_q
    out["batched_speedup_on_prefix"] = (per_q * m) / (time.perf_counter() - t0)
    # the two forms must give identical results
    out["batched_equals_one_per_query"] = bool(torch.equal(bs, one_s) and torch.equal(bn, one_n))
    out["batched_speedup_extrapolated"] = (per_q * q) / (res["ms_per_pass"] * 1e-3)
    # a small batch (64 of the queries of at most 8 keys, so launches rather
    # than scanning set the time) back to back: eager calls against replays of
    # the same call captured once in a HIP graph
    short = torch.from_numpy(np.flatnonzero(lens <= 8)[:64]).cuda()
    slo, shi = dlo[short].clone(), dhi[short].clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        tuned.range_map(slo, shi)  # sizes the scratch buffers before capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        tuned.range_map(slo, shi)
    reps = 500
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        tuned.range_map(slo, shi)
    torch.cuda.synchronize()
    out["small_batch_64_eager_us"] = (time.perf_counter() - t0) / reps * 1e6
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    out["small_batch_64_graph_us"] = (time.perf_counter() - t0) / reps * 1e6
    del graph
    tuned.close()
    log(f"range_map: default {out['default']['keys_per_s']:.3e} keys/s, autotuned (S={res['leaf_bytes']}, "
        f"chunk={res['range_chunk']}) {res['keys_per_s']:.3e} keys/s, scan {res['scan_alg_GBps']:.0f} GB/s alg; "
        f"64 short queries {out['small_batch_64_eager_us']:.1f} us eager, {out['small_batch_64_graph_us']:.1f} us "
        f"from a HIP graph; contains {out['contains_1e6_per_s']:.3e} keys/s")
    return out


def gate_section(cp, torch, c, n0, seed, gate_key):
    """range_map on cold data: 1e3 queries of about 1e6 keys at random starts
    (width = 1e6 * floor(2^40 / n0)) plus one query over the whole key space, on
    a set far larger than the 256 MB last-level cache."""
    width = np.uint64(10 ** 6 * ((1 << 40) // n0))
    lo = synth.uniform_keys(1000, seed)
    hi = lo + width
    lo = np.concatenate([lo, np.array([0], np.uint64)])
    hi = np.concatenate([hi, np.array([(1 << 64) - 1], np.uint64)])
    res = time_range(torch, c, to_dev(lo), to_dev(hi))
    res["n0"] = c.size()
    res["queries"] = "1e3 of ~1e6 keys + 1 full range"
    # what bounds the scan instead of HBM: VALU issue (counted instructions per
    # launch over the launch time, against the issue peak)
    valu = kernel_valu(SCAN_VALU_FILE, gate_key)
    res["valu_issue_frac"] = valu / (res["scan_kernel_ms"] * 1e-3) / VALU_PEAK_INSTS_PER_S if valu else None
    log(f"range gate: {res['keys_per_s']:.3e} keys/s, scan {res['scan_alg_GBps']:.0f} GB/s "
        f"({100 * res['frac_hbm_alg']:.1f}% of HBM peak)")
    return res


def serving_section(cp, torch, c, base, nreq, seed):
    """Open-loop Poisson stream of mixed requests against the resident set c
    (built from the keys `base`)."""
    n0 = len(base)
    width = (1 << 40) // n0

    def requests(count, s0):
        kinds = synth.uniform_float(count, s0)
        lens = synth.zipf_lengths(count, s0 + 1, alpha=1.2, lmax=10 ** 5)
        sizes = synth.log_uniform_sizes(count, s0 + 2)
        los = synth.uniform_keys(count, s0 + 3)
        out = []
        for i in range(count):
            if kinds[i] < 0.70:
                lo = los[i:i + 1]
                out.append(cp.ServedRequest(cp.REQ_RANGE, lo, lo + np.uint64(int(lens[i]) * width)))
            elif kinds[i] < 0.95:
                out.append(cp.ServedRequest(cp.REQ_INSERT, synth.uniform_keys(int(sizes[i]), s0 + 4, offset=10 ** 7 * i)))
            else:
                idx = synth.sample_indices(len(base), int(sizes[i]), s0 + 5 + i)
                out.append(cp.ServedRequest(cp.REQ_DELETE, base[idx]))
        return out

    def run(reqs, slots, rate=None):
        srv = cp.Server(c, max_slots=slots)
        t0 = cp.clock_ns()
        if rate is None:
            for r in reqs:
                srv.submit(r)
        else:
            gaps = -np.log(1.0 - synth.uniform_float(len(reqs), seed + 77)) / rate
            arrive = t0 + np.cumsum(gaps) * 1e9
            for r, ta in zip(reqs, arrive):
                while cp.clock_ns() < ta:
                    pass
                srv.submit(r)
        steps = srv.stop()
        t1 = max(r.req.t_done_ns for r in reqs)
        lat = np.array([(r.req.t_done_ns - r.t_submit_ns) * 1e-6 for r in reqs])
        wait = np.array([(r.req.t_admit_ns - r.t_submit_ns) * 1e-6 for r in reqs])
        ends = {}
        for r in reqs:
            ends[r.req.step] = max(ends.get(r.req.step, 0), r.req.t_done_ns)
        early = sum(1 for r in reqs if r.req.step > 0 and r.req.t_admit_ns < ends[r.req.step - 1])
        return {"ops_s": len(reqs) / ((t1 - t0) * 1e-9), "steps": steps,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "admit_wait_p50_ms": float(np.percentile(wait, 50)),
                "admitted_while_previous_step_ran": early}

    out = {"n0": c.size(), "requests": nreq, "mix": "70% range (Zipf(1.2) 1..1e5), 25% insert, 5% delete "
           "(log-uniform 10..1e6 keys)"}
    sat = run(requests(nreq, seed + 100), 4096)
    sat256 = run(requests(nreq, seed + 150), 256)
    fifo = run(requests(nreq // 4, seed + 200), 1)
    out["saturation_batched"] = sat
    out["saturation_batched_256_slots"] = sat256
    out["saturation_one_request_per_step"] = fifo
    for frac in (0.5, 0.8):
        out[f"poisson_{frac}"] = run(requests(nreq // 2, seed + int(300 + 100 * frac)), 4096,
                                     rate=frac * sat["ops_s"])
    log(f"serving: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=9)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=float, default=1e8)
    ap.add_argument("--batch", type=float, default=1e7)
    ap.add_argument("--sweep", default="1e1,1e2,1e3,1e4,1e5,1e6")
    ap.add_argument("--queries", type=float, default=1e6)
    ap.add_argument("--leaf-bytes", type=int, default=0)
    ap.add_argument("--cpu-batches", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-steps", action="store_true", help="skip every side measurement")
    ap.add_argument("--fg-scale", type=int, default=24, help="R-MAT scale of the F-Graph section (0: skip)")
    ap.add_argument("--serve-n", type=float, default=1e9,
                    help="keys of the resident set for the cold range gate and serving (0: skip both)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device to device (reference dispatch for HBM byte counters)")
    ap.add_argument("--fg-only", action="store_true", help="run only the F-Graph section (diagnostics)")
    ap.add_argument("--gate-only", action="store_true", help="run only the cold range gate (diagnostics)")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving loop (diagnostics)")
    ap.add_argument("--pma-only", action="store_true",
                    help="run only the comparison with the uncompressed PMA (diagnostics)")
    ap.add_argument("--kv-only", action="store_true", help="run only the key-value section (diagnostics)")
    ap.add_argument("--range-only", action="store_true", help="run only the batched range_map section (diagnostics)")
    ap.add_argument("--sweep-only", action="store_true", help="run only the batch-size sweep (diagnostics)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the merge kernel's traffic summary from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--valu-summary", metavar="CSV",
                    help="write the merge kernel's instruction summary from one rocprofv3 --pmc run and exit")
    ap.add_argument("--scan-valu-summary", metavar="CSV",
                    help="write the range scan kernel's instruction summary from a --pmc run of --gate-only")
    ap.add_argument("--trace-summary", nargs=2, metavar=("KIND", "CSV"),
                    help="KIND steps, gate, range, sweep or fg: write the kernel time summary of a rocprofv3 "
                         "--kernel-trace run of the headline steps, --gate-only, --range-only, --sweep-only or "
                         "--fg-only, and exit")
    args = ap.parse_args()

    shape = f"--steps {args.steps} --warmup {args.warmup}"
    if args.trace_summary:
        trace_summary(args.trace_summary[0], args.trace_summary[1], args)
        return
    if args.valu_summary or args.scan_valu_summary:
        ctr = "rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES SQ_INSTS_LDS SQ_INSTS_SALU --output-format csv "
        if args.valu_summary:
            cmd = (ctr + "-d " + PROF_DIR + "/pmc_valu -o run -- python3 /root/repo/bench.py --only-steps "
                   f"--no-cpu-baseline {shape}")
            m = MERGES_PER_STEP * args.steps
            text = valu_summary(args.valu_summary, MERGE_KERNEL, lambda v: v[-(m + TAIL_MERGES):-TAIL_MERGES],
                                "insert + delete batch pairs of 1e7 on 1e8 keys",
                                "the headline steps (the merges of the timed steps' inserts and deletes)", cmd,
                                run_key(args))
            path = VALU_FILE
        else:
            cmd = ctr + "-d " + PROF_DIR + "/pmc_scan -o run -- python3 /root/repo/bench.py --gate-only"
            text = valu_summary(args.scan_valu_summary, SCAN_KERNEL, lambda v: v[-3:],
                                "the cold range gate on 1e9 keys", "the cold range gate (its last three "
                                "timed passes)", cmd, run_key(args, "gate"))
            path = SCAN_VALU_FILE
        with open(path, "w") as fh:
            fh.write(text)
        print(text)
        return
    if args.pmc_summary:
        base = "rocprofv3 --pmc {c} --output-format csv -d " + PROF_DIR + "/pmc_{t} -o run -- " \
               f"python3 /root/repo/bench.py --only-steps --no-cpu-baseline --calibrate-copy {shape}"
        text = pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.steps,
                           base.format(c="FETCH_SIZE", t="fetch"), base.format(c="WRITE_SIZE", t="write"),
                           run_key(args))
        with open(TRAFFIC_FILE, "w") as fh:
            fh.write(text)
        print(text)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the CPMA hot path here runs on a single "
              "MI355X (multi-GPU sharding by key range is a design note, not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2305_05055_amd as cp

    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {src.numel() * 8} bytes read and written")
        del src, dst
    n0 = int(args.n)
    k = int(args.batch)
    seed = synth.SEED_BASE + 2
    if args.fg_only:
        print(json.dumps({"rmat": fgraph_section(cp, torch, args.fg_scale, seed + 60),
                          "er": er_section(cp, torch, seed + 65)}), flush=True)
        return
    if args.gate_only:
        big_d = synth.uniform_keys_torch(int(args.serve_n), seed + 70, "cuda")
        big = cp.CPMA(big_d)
        del big_d
        torch.cuda.empty_cache()
        print(json.dumps(gate_section(cp, torch, big, int(args.serve_n), seed + 80, run_key(args, "gate"))),
              flush=True)
        return
    if args.serve_only:
        big_d = synth.uniform_keys_torch(int(args.serve_n), seed + 70, "cuda")
        big = cp.CPMA(big_d)
        big_host = big_d.cpu().numpy().view(np.uint64)
        del big_d
        torch.cuda.empty_cache()
        print(json.dumps(serving_section(cp, torch, big, big_host, args.serve_requests, seed + 90)), flush=True)
        return

    if args.kv_only:
        print(json.dumps(kv_section(cp, torch, synth.uniform_keys_torch(n0, seed, "cuda"), seed + 49,
                                    fg_scale=args.fg_scale, leaf_bytes=args.leaf_bytes)), flush=True)
        return
    if args.pma_only:
        print(json.dumps(pma_section(cp, torch, synth.uniform_keys_torch(n0, seed, "cuda"), seed + 48)), flush=True)
        return

    # ---- base set: exactly n0 distinct uniform 40-bit keys -----------------------
    t = time.time()
    base = synth.uniform_keys(n0, seed)
    c = cp.CPMA(to_dev(base), leaf_bytes=args.leaf_bytes)
    extra = []
    off = n0
    while c.size() < n0:
        need = n0 - c.size()
        more = synth.uniform_keys(need, seed, offset=off)
        off += need
        c.insert_batch(to_dev(more))
        extra.append(more)
    base_all = np.concatenate([base] + extra) if extra else base
    base_dev = to_dev(base_all) if not args.only_steps else None
    torch.cuda.synchronize()
    L, S = c.geometry()
    log(f"built n={c.size()} L={L} S={S} bytes/key={c.bytes() / c.size():.3f} in {time.time() - t:.1f}s")
    result_extra = {"bytes_per_key_at_n0": c.bytes() / c.size(), "leaves_at_n0": L, "leaf_bytes": S}

    if args.range_only:
        print(json.dumps(range_section(cp, torch, c, base_dev if base_dev is not None else to_dev(base_all),
                                       int(args.queries), seed + 10)), flush=True)
        return
    # ---- batched range_map (Zipf(1.2) lengths 1..1e6) vs one launch per query -----
    if not args.only_steps and not args.sweep_only and args.queries > 0:
        result_extra["range_map"] = range_section(cp, torch, c, base_dev, int(args.queries), seed + 10,
                                                  with_cpu=not args.no_cpu_baseline)
    base_dev = None
    torch.cuda.empty_cache()

    # ---- batch-size sweep: insert k fresh keys, then delete k present keys --------
    per_batch = {}
    if not args.only_steps or args.sweep_only:
        sizes = [int(float(x)) for x in args.sweep.split(",") if x]
        reps = {10: 30, 100: 30, 1000: 20, 10000: 10, 100000: 5, 1000000: 3}
        total_del = sum(s * reps.get(s, 3) for s in sizes)
        del_idx = synth.sample_indices(len(base_all), total_del, seed + 20)
        dpos = 0
        gen_off = 10 ** 11
        for s in sizes:
            r = reps.get(s, 3)
            ins_b = [to_dev(synth.uniform_keys(s, seed + 30, offset=gen_off + i * s)) for i in range(r)]
            gen_off += r * s
            del_b = [to_dev(base_all[del_idx[dpos + i * s: dpos + (i + 1) * s]]) for i in range(r)]
            dpos += r * s
            torch.cuda.synchronize()
            ti, td = [], []
            for i in range(r):
                t0 = time.perf_counter()
                c.insert_batch(ins_b[i])
                ti.append(time.perf_counter() - t0)
                t0 = time.perf_counter()
                c.delete_batch(del_b[i])
                td.append(time.perf_counter() - t0)
            ti, td = np.array(ti), np.array(td)
            per_batch[f"{s:.0e}"] = {
                "insert_keys_s": s / ti.mean(), "delete_keys_s": s / td.mean(),
                "insert_p50_ms": float(np.percentile(ti, 50) * 1e3),
                "insert_p99_ms": float(np.percentile(ti, 99) * 1e3),
                "delete_p50_ms": float(np.percentile(td, 50) * 1e3),
                "delete_p99_ms": float(np.percentile(td, 99) * 1e3), "reps": r}
            log(f"k={s:.0e}: insert {s / ti.mean():.3e}/s delete {s / td.mean():.3e}/s "
                f"p99 {np.percentile(ti, 99) * 1e3:.2f} ms")
        result_extra["per_batch"] = per_batch
        if args.sweep_only:
            print(json.dumps(per_batch), flush=True)
            return

    # ---- headline: W warm-up + K timed steps, each an insert batch of k fresh
    # keys and a delete batch of k present keys (the previous step's insert
    # batch; the first step deletes k keys sampled from the base set), so the
    # set stays at n0 .. n0 + k keys ------------------------------------------
    nb = args.warmup + args.steps
    n_phase_steps = PHASE_STEPS
    ins = [to_dev(synth.uniform_keys(k, seed + 40, offset=i * k)) for i in range(nb + n_phase_steps)]
    first_del = to_dev(base_all[synth.sample_indices(len(base_all), k, seed + 50)])

    def dels(i):
        return first_del if i == 0 else ins[i - 1]

    torch.cuda.synchronize()
    n_seen = [c.size()]
    for i in range(args.warmup):
        c.insert_batch(ins[i])
        n_seen.append(c.size())
        c.delete_batch(dels(i))
        n_seen.append(c.size())
    torch.cuda.synchronize()
    # the timed steps record HIP events around the merge kernel only (each event
    # record idles the GPU for a few microseconds); every phase is timed on
    # separate steps afterwards
    c.stats_select(["merge"])
    lat, lat_i, lat_d = [], [], []
    added = removed = 0
    t0 = time.perf_counter()
    for i in range(args.warmup, nb):
        ts = time.perf_counter()
        added += c.insert_batch(ins[i])
        tm = time.perf_counter()
        n_seen.append(c.size())
        removed += c.delete_batch(dels(i))
        te = time.perf_counter()
        n_seen.append(c.size())
        lat.append(te - ts)
        lat_i.append(tm - ts)
        lat_d.append(te - tm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = c.stats()
    c.stats_enable(False)
    n_after = c.size()
    dt = t1 - t0
    value = args.steps * 2 * k / dt
    log(f"headline: {value:.3e} keys/s (inserted + deleted), {dt / args.steps * 1e3:.2f} ms/step, "
        f"insert {k / np.mean(lat_i):.3e}/s, delete {k / np.mean(lat_d):.3e}/s, n={n_after}")
    c.stats_enable(True)
    for i in range(nb, nb + n_phase_steps):
        c.insert_batch(ins[i])
        c.delete_batch(dels(i))
    stp = c.stats()
    c.stats_enable(False)
    phases = {name: {"launches": v[0], "ms": v[1], "alg_bytes": v[2]} for name, v in stp.items()}
    phases["steps"] = n_phase_steps

    # roofline of the dominant single kernel of the step (the merge)
    mg_l, mg_ms, mg_b = st["merge"]
    dominant = max(("merge", "sort", "locate", "count", "redist"), key=lambda p: stp[p][1])
    roof = None
    key = run_key(args)
    if mg_l > 0 and mg_ms > 0:
        ach = (mg_b / mg_l) / ((mg_ms / mg_l) * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": MERGE_KERNEL if S <= 1024 else "k_merge_lane",
                "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": merge_traffic(key),
                "alg_bytes_per_launch": mg_b / mg_l, "avg_launch_ms": mg_ms / mg_l,
                "launches": mg_l, "dominant_phase": dominant}
        # what bounds it instead: VALU issue (counted instructions per launch over
        # the launch time, against the issue peak)
        valu = kernel_valu(VALU_FILE, key)
        roof["valu_issue_frac"] = (valu / ((mg_ms / mg_l) * 1e-3) / VALU_PEAK_INSTS_PER_S) if valu else None
    result_extra["steps_detail"] = {
        "insert_keys_s": k / float(np.mean(lat_i)), "delete_keys_s": k / float(np.mean(lat_d)),
        "insert_p50_ms": float(np.percentile(lat_i, 50) * 1e3), "insert_p99_ms": float(np.percentile(lat_i, 99) * 1e3),
        "delete_p50_ms": float(np.percentile(lat_d, 50) * 1e3), "delete_p99_ms": float(np.percentile(lat_d, 99) * 1e3),
        "keys_added": added, "keys_removed": removed,
        "paper_context": "paper, 64-core Xeon, batch 1e7: 2.4e8 inserts/s and 4.7e8 deletes/s (uniform keys)"}
    n_seen.append(n_after)
    result_extra["bytes_per_key_final"] = c.bytes() / c.size()
    result_extra["bytes_held_per_key_final"] = c.bytes_held() / c.size()
    del ins, first_del
    if not args.only_steps:
        result_extra["zipf"] = zipf_section(cp, torch, c, seed + 45)
    c.trim()
    result_extra["bytes_held_per_key_after_trim"] = c.bytes_held() / c.size()

    c.close()
    torch.cuda.empty_cache()
    if not args.only_steps:
        bd = to_dev(base_all)
        result_extra["rebuild"] = rebuild_section(cp, torch, bd, seed + 46)
        result_extra["growth"] = growth_section(cp, torch, bd, seed + 47)
        result_extra["pma_vs_cpma"] = pma_section(cp, torch, bd, seed + 48)
        result_extra["key_value"] = kv_section(cp, torch, bd, seed + 49, fg_scale=args.fg_scale)
        del bd
        torch.cuda.empty_cache()
    if not args.only_steps:
        result_extra["redistribution"] = redist_section(cp, torch, seed + 50)
        torch.cuda.empty_cache()
    if not args.only_steps and args.fg_scale > 0:
        result_extra["fgraph"] = fgraph_section(cp, torch, args.fg_scale, seed + 60)
        torch.cuda.empty_cache()
        result_extra["er_graph"] = er_section(cp, torch, seed + 65)
        torch.cuda.empty_cache()
    if not args.only_steps and args.serve_n > 0:
        # one resident set of serve_n keys: the cold range gate, then the serving loop
        n_big = int(args.serve_n)
        big_d = synth.uniform_keys_torch(n_big, seed + 70, "cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        big = cp.CPMA(big_d)
        torch.cuda.synchronize()
        log(f"built {big.size()} keys in {time.perf_counter() - t0:.1f}s, {big.bytes() / big.size():.3f} B/key")
        big_host = big_d.cpu().numpy().view(np.uint64)
        del big_d
        torch.cuda.empty_cache()
        result_extra["range_gate"] = gate_section(cp, torch, big, n_big, seed + 80, run_key(args, "gate"))
        result_extra["serving"] = serving_section(cp, torch, big, big_host, args.serve_requests, seed + 90)
        big.close()
        del big_host

    # ---- CPU baseline: the oracle taking the same kind of steps -----------------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("cpu baseline: oracle set of n0 keys ...")
        S_host = oracle.build_set(base_all)
        nbat = args.cpu_batches
        prev = base_all[synth.sample_indices(len(base_all), k, seed + 50)]
        t0 = time.perf_counter()
        for i in range(nbat):
            b = synth.uniform_keys(k, seed + 40, offset=i * k)
            S_host, _ = oracle.insert(S_host, b)
            S_host, _ = oracle.delete(S_host, prev)
            prev = b
        tc = time.perf_counter() - t0
        cpu = {"value": nbat * 2 * k / tc, "unit": "keys/s", "cores": 1, "kind": "oracle",
               "sample": f"{nbat} steps of the same workload (insert {k:.0e} uniform 40-bit keys into the "
                         f"{n0:.0e}-key set, then delete {k:.0e} present keys; sorted-vector set_union / "
                         f"set_difference, single thread), {tc:.1f} s",
               "host": host_info()}
        log(f"cpu baseline {cpu['value']:.3e} keys/s")

    out = {
        "metric": METRIC, "value": value, "unit": "keys/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "plain CPMA at scale: 1e8 uniform 40-bit keys; each step inserts a batch of 1e7 "
                               "fresh uniform keys and deletes a batch of 1e7 present keys",
                   "value_counts": "keys of the insert and the delete batch", "n0": n0, "batch": k,
                   "n_range": [int(min(n_seen)), int(max(n_seen))], "leaf_bytes": S, "key_bits": 40},
        "roofline": roof, "cpu_baseline": cpu,
        "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
        "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
        "latency_of": "one step (insert batch + delete batch)",
        "phases": phases,
    }
    out.update(result_extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
