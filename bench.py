"""Benchmark: GCUPS of Smith-Waterman database search on one MI355X.

Default workload (the headline; synthetic stand-in for the Environmental NR search of
Section 5.1): 6,000,000 database sequences (log-normal lengths, median 200, sigma 0.8,
clipped to 10..8000; about 1.65e9 residues at Robinson-Robinson frequencies) searched
with six synthetic queries of lengths 144, 375, 729, 1000, 2005 and 5478; BLOSUM62, gap
open 10, gap extend 2.  One step is one search of every query against the whole
database (all stages of the path: query profiles, packed-int16 inter-task kernel,
intra-task kernel for routed sequences, saturation recompute, scores in the caller's
order in HBM).  GCUPS = sum(|Q|) * |D| / t (Section 5.2, Eq. 4), |D| the unpadded
residue count.

Other workloads (``--workload``): ``plain`` (2,000 sequences, one query of 144),
``long_mix`` (10,000 sequences, 1% of them 10,000..35,000 long; queries 5478 and
35000), ``batched`` (200,000 sequences, 64 queries of lengths 50..5000 in one captured
HIP graph; BLOSUM62/BLOSUM50 x gaps 10/2 and 11/1).  Serving is measured by
``--workload served`` (open-loop Poisson arrivals at 2, 8 and 32 queries/s against
a resident 4.35e6-sequence database through the continuous-batching server; p50/p99
latency).

Prints one JSON line with a roofline object for the dominant kernel (timed with HIP
events on the stream that launches it) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic operations per DP cell (Section 2, Eqs. 1-3): H-Goe, E-Ge and max, F-Ge and
# max, H(diag)+SM, three maxima for H, running maximum.
OPS_PER_CELL = 10
# VALU peaks of MI355X: 256 CUs x 64 lanes x 2.4 GHz, x2 for packed int16 halves.
PEAK_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12
PEAK_INT16_TOPS = 2 * PEAK_INT32_TOPS
KERNEL_SRC = os.path.join(ROOT, "paper_1702_07195_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "inter16_full_scale_traffic.json")
TRAFFIC_FILE_Q2 = os.path.join(ROOT, "profiles", "inter16q2_batched_traffic.json")
TRAFFIC_FILE_INTRA = os.path.join(ROOT, "profiles", "intra32_long_mix_traffic.json")
_SECTION = b"// ------------------------------------------------------------------------ "


def kernel_hash(section: str = "inter") -> str:
    """Hash of the source a kernel is built from: for k_inter16 ("inter") the shared
    helpers, profile and packing kernels and k_inter16 (everything before the intra-task
    section); for k_inter16q2 ("inter_q2") those plus its own section; for k_intra32
    ("intra") those plus the intra-task section."""
    with open(KERNEL_SRC, "rb") as f:
        src = f.read()
    cut = src.find(_SECTION + b"intra-task")
    head = src[:cut if cut >= 0 else len(src)]
    if section == "inter":
        return hashlib.sha256(head).hexdigest()[:16]
    if section == "intra":
        end = src.find(_SECTION, cut + len(_SECTION)) if cut >= 0 else -1
        body = src[cut:end if end >= 0 else len(src)] if cut >= 0 else b""
        return hashlib.sha256(head + body).hexdigest()[:16]
    q2 = src.find(_SECTION + b"inter-task, two queries")
    return hashlib.sha256(head + (src[q2:] if q2 >= 0 else b"")).hexdigest()[:16]


def load_counters(path: str = TRAFFIC_FILE, section: str = "inter"):
    """Per-launch figures from committed PMC runs (HBM bytes, VALU instructions), if they
    were taken on the current kernel source; else None."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash(section):
        return None
    return t


def load_traffic(path: str = TRAFFIC_FILE, section: str = "inter"):
    """HBM bytes per launch from committed PMC runs, if taken on the current kernel."""
    t = load_counters(path, section)
    return t.get("bytes_per_launch") if t else None


def valu_issue(counters, avg_s: float):
    """VALU issue utilisation of a launch: wave instructions x 64 lanes over the lane
    slots of the chip (256 CUs x 64 lanes x 2.4 GHz) in the launch's average time."""
    if not counters or not counters.get("sq_insts_valu_per_launch") or avg_s <= 0:
        return None
    lanes = counters["sq_insts_valu_per_launch"] * 64
    return round(lanes / (PEAK_INT32_TOPS * 1e12 * avg_s), 3)


def cpu_baseline(db, queries, sm, go, ge, gpu_scores, budget_cells: float):
    """Time the oracle on a length-stratified sample of sequences (all queries) and check
    the sampled GPU scores against it bit for bit."""
    import oracle

    lengths = db.lengths
    order = np.argsort(lengths, kind="stable")
    per_seq = float(sum(len(q) for q in queries)) * float(max(lengths.mean(), 1.0))
    n = int(max(16, min(len(order), budget_cells / max(per_seq, 1.0))))
    idx = order[np.linspace(0, len(order) - 1, n).astype(np.int64)]
    # the host share of one GPU is 16 cores, whatever the machine reports
    threads = max(1, min(os.cpu_count() or 1, 16))
    # a database smaller than the budget is searched several times (the first pass checked)
    pass_cells = float(sum(len(q) for q in queries)) * float(lengths[idx].sum())
    reps = int(min(200, max(1, budget_cells // max(pass_cells, 1.0))))
    cells = 0
    t0 = time.perf_counter()
    exact = True
    for r in range(reps):
        for q, g in zip(queries, gpu_scores):
            want = oracle.search(q, db.residues, db.offsets, sm, go, ge, index=idx,
                                 threads=threads)
            if r == 0:
                exact &= bool(np.array_equal(want, g[idx]))
            cells += len(q) * int(lengths[idx].sum())
    dt = time.perf_counter() - t0
    # one host thread on a sixteenth of the sample (every sixteenth sampled sequence)
    idx1 = idx[::16] if len(idx) >= 16 else idx
    cells1 = 0
    t1 = time.perf_counter()
    for r in range(reps):
        for q, g in zip(queries, gpu_scores):
            want = oracle.search(q, db.residues, db.offsets, sm, go, ge, index=idx1, threads=1)
            if r == 0:
                exact &= bool(np.array_equal(want, g[idx1]))
            cells1 += len(q) * int(lengths[idx1].sum())
    dt1 = time.perf_counter() - t1
    return {"value": round(cells / dt / 1e9, 3), "unit": "GCUPS", "cores": threads,
            "kind": "oracle", "machine_cores": os.cpu_count(), "cpu_model": cpu_model(),
            "cores_note": "all cores of this GPU's host share (16 threads, or every core "
                          "if the machine has fewer)",
            "sample": f"{n} database sequences (stratified by length) x {len(queries)} "
                      f"queries{f', searched {reps} times' if reps > 1 else ''}, "
                      f"{cells:.3e} cells, {dt:.1f} s",
            "single_core": {"value": round(cells1 / dt1 / 1e9, 3), "unit": "GCUPS",
                            "sample": f"{len(idx1)} of those sequences, {cells1:.3e} cells, "
                                      f"{dt1:.1f} s"}}, exact


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


INT16_NOTE = ("achieved counts the recurrence's 10 int16 operations per cell; clamping E "
              "and F at zero removes the maximum with 0, so a packed cell pair issues 9 "
              "arithmetic instructions (plus one byte permute in k_inter16), and frac can "
              "reach 1 before the VALU is fully busy")


def roofline(kernel: str, cells_per_launch: float, launches: int, total_ms: float,
             int16: bool, traffic=None):
    avg_s = total_ms / max(launches, 1) / 1e3
    if avg_s <= 0:
        return None
    achieved = OPS_PER_CELL * cells_per_launch / avg_s / 1e12
    peak = PEAK_INT16_TOPS if int16 else PEAK_INT32_TOPS
    out = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 2),
           "unit": "Tops/s (int16)" if int16 else "Tops/s (int32)",
           "frac": round(achieved / peak, 3), "traffic": traffic, "kernel": kernel,
           "avg_launch_ms": round(avg_s * 1e3, 3), "launches": launches}
    if int16:
        out["note"] = INT16_NOTE
    return out


def base_result(args, value, elapsed, dtype, config):
    return {
        "metric": "GCUPS per query length (1 GPU, bit-exact)",
        "value": round(value, 1),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": config,
    }


def run_searches(args, w, db, queries):
    """Time `steps` passes of single-query searches (device-resident outputs)."""
    import torch
    from paper_1702_07195_amd import swmi, synth

    sm, go, ge = w.matrix_values, w.gap_open, w.gap_extend
    D = int(db.offsets[-1])
    h = swmi.sw_db_load(db.residues, db.offsets, len(synth.ALPHABET))
    dev = torch.device("cuda:0")
    outs = [torch.zeros(db.n_seqs, dtype=torch.int32, device=dev) for _ in queries]
    stream = torch.cuda.current_stream()

    def step():
        for k, q in enumerate(queries):
            h.search_async(q, sm, go, ge, outs[k], stream)

    if args.copy_mib > 0:
        n = args.copy_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    h.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timing = {k: h.timing_read(k) for k in (swmi.SW_KERNEL_INTER16, swmi.SW_KERNEL_INTRA_LONG,
                                             swmi.SW_KERNEL_RECOMPUTE)}
    h.timing_enable(False)
    # each query alone (synchronised before and after): one warm-up run, then the median
    # of seven
    per_query = {}
    for k, q in enumerate(queries):
        h.search_async(q, sm, go, ge, outs[k], stream)
        torch.cuda.synchronize()
        ts = []
        for _ in range(7):
            torch.cuda.synchronize()
            t = time.perf_counter()
            h.search_async(q, sm, go, ge, outs[k], stream)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        per_query[str(len(q))] = round(len(q) * D / float(np.median(ts)) / 1e9, 1)
    # per-launch algorithmic cells of each kernel, query by query (same plans as timed)
    stats = []
    for k, q in enumerate(queries):
        h.search_async(q, sm, go, ge, outs[k], stream)
        stats.append(h.stats())
    torch.cuda.synchronize()
    # host-inclusive rate: the blocking call, scores copied to host memory
    t = time.perf_counter()
    for q in queries:
        h.search(q, sm, go, ge)
    host_s = time.perf_counter() - t
    host_inclusive = round(sum(len(q) for q in queries) * D / host_s / 1e9, 1)
    scores = [o.cpu().numpy() for o in outs]
    # sorting stage: the 100 best hits of the last query, checked against a host sort
    h.topk(outs[-1], 100)
    torch.cuda.synchronize()
    t = time.perf_counter()
    idx, sc = h.topk(outs[-1], 100)
    topk_ms = (time.perf_counter() - t) * 1e3
    order = np.lexsort((np.arange(db.n_seqs), -scores[-1].astype(np.int64)))[:len(idx)]
    topk = {"k": 100, "ms": round(topk_ms, 3),
            "exact": bool(np.array_equal(idx, order) and np.array_equal(sc, scores[-1][order]))}
    latency = None
    if args.workload == "plain":
        latency = longest_pair_bound(args, db, queries, sm, go, ge, elapsed)
    h.free()
    return elapsed, timing, per_query, scores, topk, stats, host_inclusive, latency


def longest_pair_bound(args, db, queries, sm, go, ge, elapsed):
    """A search cannot end before its longest pair is swept: with the query in one band,
    that pair alone takes (n + 63) anti-diagonal steps of a lane-to-lane dependency chain.
    Measured by searching a database of that one sequence."""
    import torch
    from paper_1702_07195_amd import swmi, synth

    k = int(np.argmax(db.lengths))
    one = synth.db_from_seqs([db.seq(k)])
    h1 = swmi.sw_db_load(one.residues, one.offsets, len(synth.ALPHABET))
    out = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()
    for q in queries:
        h1.search_async(q, sm, go, ge, out, stream)
    torch.cuda.synchronize()
    reps = 20
    t = time.perf_counter()
    for _ in range(reps):
        for q in queries:
            h1.search_async(q, sm, go, ge, out, stream)
    torch.cuda.synchronize()
    pair_ms = (time.perf_counter() - t) / reps * 1e3
    st = h1.stats()
    h1.free()
    n = int(db.lengths[k])
    search_ms = elapsed / args.steps * 1e3
    return {"longest_sequence": n, "anti_diagonal_steps": n + 63,
            "rows_per_lane": st["intra_rows"],
            "longest_pair_alone_ms": round(pair_ms, 3),
            "step_us": round(pair_ms * 1e3 / (n + 63), 4),
            "search_ms": round(search_ms, 3),
            "frac": round(pair_ms / search_ms, 3),
            "note": "latency bound: the search takes frac of its time at the bound set by "
                    "its longest pair's dependency chain"}


def intra_roofline(stats, launches, total_ms, counters=None):
    """Roofline of the main intra-task launch from its own algorithmic cells: int32 cells
    at the int32 peak and packed-int16 (two pairs per wave) cells at the int16 peak; frac
    is the time that work needs at those peaks over the measured launch time.  HBM
    traffic and VALU issue come from committed PMC runs of the same kernel source."""
    if launches <= 0 or total_ms <= 0:
        return None
    c32 = sum(st["cells_intra32"] for st in stats)
    c16 = sum(st["cells_intra16"] for st in stats)
    per = len(stats)  # launches per step (one per query)
    avg_s = total_ms / launches / 1e3
    c32l, c16l = c32 / per, c16 / per
    t_peak = OPS_PER_CELL * (c32l / (PEAK_INT32_TOPS * 1e12) + c16l / (PEAK_INT16_TOPS * 1e12))
    achieved = OPS_PER_CELL * (c32l + c16l) / avg_s / 1e12
    peak = OPS_PER_CELL * (c32l + c16l) / t_peak / 1e12
    return {"bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 2),
            "unit": "Tops/s (int32, with packed-int16 cells at twice the rate)",
            "frac": round(t_peak / avg_s, 3),
            "traffic": counters.get("bytes_per_launch") if counters else None,
            "valu_issue": valu_issue(counters, avg_s),
            "kernel": "k_intra32 (main intra-task launch)",
            "avg_launch_ms": round(avg_s * 1e3, 3), "launches": launches,
            "cells_int32_per_launch": int(c32l), "cells_int16_per_launch": int(c16l),
            "note": "cells are the launch's own (query rows x residues of its pairs); the "
                    "critical-pair launch and the inter-task kernel run beside it"}


def bench_search(args, w, label):
    from paper_1702_07195_amd import swmi

    db = w.make_db()
    queries = w.make_queries()
    D = int(db.offsets[-1])
    elapsed, timing, per_query, scores, topk, stats, host_inc, latency = \
        run_searches(args, w, db, queries)
    cells_per_step = sum(len(q) for q in queries) * D
    gcups = cells_per_step * args.steps / elapsed / 1e9
    n16, ms16 = timing[swmi.SW_KERNEL_INTER16]
    nlo, mslo = timing[swmi.SW_KERNEL_INTRA_LONG]
    # the dominant kernel is the one with more device time, priced at its own cells
    if ms16 >= mslo:
        cells16 = sum(st["cells_inter16"] for st in stats) / len(stats)
        counters = load_counters() if label == "full-scale plain search" else None
        roof = roofline("k_inter16", cells16, n16, ms16, True,
                        counters.get("bytes_per_launch") if counters else None)
        if roof is not None:
            roof["valu_issue"] = valu_issue(counters, roof["avg_launch_ms"] / 1e3)
    else:
        counters = (load_counters(TRAFFIC_FILE_INTRA, "intra")
                    if label == "long-sequence mix" else None)
        roof = intra_roofline(stats, nlo, mslo, counters)
    config = {"workload": label, "db_seqs": db.n_seqs, "db_residues": D,
              "query_lengths": [len(q) for q in queries], "matrix": w.matrix,
              "gap_open": w.gap_open, "gap_extend": w.gap_extend}
    result = base_result(args, gcups, elapsed, "i16+i32", config)
    result["per_query_gcups"] = per_query
    result["host_inclusive_gcups"] = host_inc
    result["search_stats"] = stats
    if latency is not None:
        result["latency_bound"] = latency
    result["topk"] = topk
    result["roofline"] = roof
    result["kernel_ms_per_step"] = {
        "k_inter16": round(ms16 / args.steps, 3),
        "k_intra32_long": round(mslo / args.steps, 3),
        "k_intra32_recompute": round(timing[swmi.SW_KERNEL_RECOMPUTE][1] / args.steps, 3)}
    if not args.no_cpu:
        base, exact = cpu_baseline(db, queries, w.matrix_values, w.gap_open, w.gap_extend,
                                   scores, args.cpu_cells)
        result["cpu_baseline"] = base
        result["bit_exact_sample"] = exact
    return result


def bench_batched(args):
    """64 queries in captured HIP graphs, with the autotuned strip height, waves per CU and
    bin width (tuned first on BLOSUM62 10/2, outside the timed region)."""
    import torch
    from paper_1702_07195_amd import autotune, swmi, synth

    w = synth.BATCHED
    db = w.make_db()
    qs = synth.batched_queries(64)
    D = int(db.offsets[-1])
    cells = sum(len(q) for q in qs) * D
    h = swmi.sw_db_load(db.residues, db.offsets, len(synth.ALPHABET))
    out = torch.zeros((len(qs), db.n_seqs), dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()
    if args.copy_mib > 0:  # a copy of known size, to scale profiler byte counters
        src = torch.ones(args.copy_mib << 20, dtype=torch.uint8, device="cuda:0")
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        del src
    if args.no_tune:
        best, timings = autotune.Config(), {}
    else:
        best, timings = autotune.tune(h, D, qs, synth.BLOSUM62, 10, 2, out,
                                      use_cache=not args.no_tune_cache,
                                      log=lambda m: print(m, file=sys.stderr, flush=True))
    variants = {}
    total_t = 0.0
    graph_scores = None
    for mat in ("BLOSUM62", "BLOSUM50"):
        for go, ge in ((10, 2), (11, 1)):
            sm = synth.MATRICES[mat]
            plans = autotune.BinnedPlans(h, qs, sm, go, ge, out, best)
            try:
                for _ in range(args.warmup):
                    plans.launch(stream)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    plans.launch(stream)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if mat == "BLOSUM62" and (go, ge) == (10, 2):
                    plans.gather()
                    graph_scores = out.cpu().numpy()
            finally:
                plans.free()
            variants[f"{mat} {go}/{ge}"] = round(cells * args.steps / dt / 1e9, 1)
            total_t += dt
    # kernel timing and reference scores from an eager batched search of the same queries
    sm = synth.BLOSUM62
    h.timing_enable(True)
    scores_host = h.search_batch(qs, sm, 10, 2)
    n16, ms16 = h.timing_read(swmi.SW_KERNEL_INTER16)
    h.timing_enable(False)
    gcups = 4 * cells * args.steps / total_t / 1e9
    config = {"workload": "batched (64 queries, hipGraph replay)", "db_seqs": db.n_seqs,
              "db_residues": D, "n_queries": len(qs), "query_lengths": "U{50..5000}",
              "matrices": ["BLOSUM62", "BLOSUM50"], "gaps": ["10/2", "11/1"],
              "autotuned": best.as_dict()}
    result = base_result(args, gcups, total_t / 4, "i16+i32", config)
    result["per_variant_gcups"] = variants
    result["autotune_ms"] = timings
    # (a batch runs two queries per lane in k_inter16q2 unless SW_KNOB_QUERY_PAIRS is 0;
    # the algorithmic work per cell is the same 10 int16 operations)
    q2 = bool(swmi.get_knob(swmi.SW_KNOB_QUERY_PAIRS))
    kname = "k_inter16q2" if q2 else "k_inter16"
    counters = load_counters(TRAFFIC_FILE_Q2, "inter_q2") if q2 else None
    result["roofline"] = roofline(f"{kname} (eager batch, default configuration)", cells,
                                  n16, ms16, True,
                                  counters.get("bytes_per_launch") if counters else None)
    if result["roofline"] is not None:
        # frac counts the recurrence's 10 operations per cell and can exceed the share of
        # issue slots the kernel fills; this is that share, from the committed counters
        result["roofline"]["valu_issue"] = valu_issue(
            counters, result["roofline"]["avg_launch_ms"] / 1e3)
    result["graph_equals_eager"] = bool(np.array_equal(graph_scores, scores_host))
    if not args.no_cpu:
        base, exact = cpu_baseline(db, qs[:8], sm, 10, 2, list(scores_host[:8]),
                                   args.cpu_cells)
        result["cpu_baseline"] = base
        result["bit_exact_sample"] = exact
    h.free()
    return result


def bench_served(args):
    """Open-loop Poisson arrivals against the resident database through the
    continuous-batching server; p50/p99 latency and achieved GCUPS per rate."""
    import threading
    from paper_1702_07195_amd import swmi, synth

    w = synth.SERVED if args.seqs is None else synth.scaled(synth.SERVED, args.seqs)
    db = w.make_db()
    D = int(db.offsets[-1])
    sm, go, ge = w.matrix_values, w.gap_open, w.gap_extend
    h = swmi.sw_db_load(db.residues, db.offsets, len(synth.ALPHABET))
    rates = [float(r) for r in args.rates.split(",")]
    counts = [int(x) for x in str(args.requests).split(",")]
    counts = counts + [counts[-1]] * (len(rates) - len(counts))
    per_rate = {}
    check = None
    for ri, rate in enumerate(rates):
        n = counts[ri]
        queries = synth.served_queries(n, seed=1702_1004 + ri)
        arrivals = synth.poisson_arrivals(n, rate, seed=1702_2004 + ri)
        results = [None] * n
        with swmi.SwServer(h, sm, go, ge, slots=args.slots, max_batch=args.max_batch,
                           mem_budget_bytes=int(args.mem_budget_gib * (1 << 30))) as sv:
            # warm the slots (workspaces) before timing
            for t in [sv.submit(queries[0]) for _ in range(args.slots)]:
                sv.wait(t)
            c_warm = sv.counters()
            tickets = [None] * n
            t0 = time.perf_counter()

            def submitter():
                for k in range(n):
                    delay = t0 + arrivals[k] - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                    tickets[k] = sv.submit(queries[k])

            th = threading.Thread(target=submitter)
            th.start()
            th.join()
            for k in range(n):
                results[k] = sv.wait(tickets[k])
            t_end = time.perf_counter()
            c0 = sv.counters()
        lat = np.array([r[1] for r in results])
        cells = sum(len(q) for q in queries) * D
        achieved = cells / (t_end - t0) / 1e9
        # submission to completion of the first and last request: the served window
        per_rate[f"{rate:g}"] = {
            "requests": n, "p50_ms": round(float(np.percentile(lat, 50)), 2),
            "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "mean_queue_ms": round(float(np.mean([r[2] for r in results])), 2),
            "achieved_gcups": round(achieved, 1),
            "offered_gcups": round(rate * float(np.mean([len(q) for q in queries])) * D / 1e9, 1),
            # served roofline: the window's algorithmic int16 operations over the peak
            "roofline_frac": round(achieved * OPS_PER_CELL / 1e3 / PEAK_INT16_TOPS, 3),
            "server": {k: c0[k] - (c_warm[k] if k in ("launches", "records", "paired",
                                                      "exact_runs") else 0)
                       for k in c0}}
        if check is None:
            # the same queries searched alone must give the same scores as in the mix
            check = all(np.array_equal(h.search(queries[k], sm, go, ge), results[k][0])
                        for k in range(min(4, n)))
    mid = per_rate[f"{rates[len(rates) // 2]:g}"]
    config = {"workload": "served (open-loop Poisson arrivals, continuous batching)",
              "db_seqs": db.n_seqs, "db_residues": D, "query_lengths": "log-normal median 350",
              "rates_per_s": rates, "slots": args.slots, "max_batch": args.max_batch,
              "matrix": w.matrix, "gap_open": go, "gap_extend": ge}
    result = base_result(args, mid["achieved_gcups"], 0.0, "i16+i32", config)
    result["steps"] = sum(counts[:len(rates)])
    result["ms_per_step"] = mid["p50_ms"]
    result["serving"] = per_rate
    result["alone_equals_mix"] = bool(check)
    result["note"] = ("continuous batching in sessions: one persistent launch serves every "
                      "query admitted while it runs; a query arriving while others are on "
                      "the device is published as a record whose work items queue right "
                      "behind theirs (at most `slots` records in flight, the rest wait on the "
                      "host, where two of similar length can share a record's lanes); "
                      "server.launches counts session launches, server.max_in_flight the "
                      "most records on the device at once")
    # served roofline at the middle rate: its achieved int16 operations over the peak
    result["roofline"] = {"bound": "alu",
                          "achieved": round(mid["achieved_gcups"] * OPS_PER_CELL / 1e3, 2),
                          "peak": round(PEAK_INT16_TOPS, 2), "unit": "Tops/s (int16)",
                          "frac": mid["roofline_frac"], "traffic": None,
                          "kernel": "k_serve (session launch)",
                          "note": "whole served window, arrival gaps included"}
    h.free()
    return result


def calibrate():
    """Sustained cell rates of the three integer tiers, without memory traffic."""
    import ctypes

    import torch  # noqa: F401  (one HIP runtime per process: torch's)

    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1702_07195_amd", "libswmi_calib.so"))
    f = lib.swcal_cellmix
    f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    f.restype = ctypes.c_int
    out = {}
    for kind, name in ((0, "int16x2 packed"), (1, "int32"), (2, "int8x4 SWAR")):
        rows = {}
        for waves in (4, 8, 12, 16):
            ms, cells = ctypes.c_double(), ctypes.c_double()
            rc = f(kind, waves, 4096 if kind != 2 else 1024, ctypes.byref(ms), ctypes.byref(cells))
            if rc != 0:
                raise RuntimeError(f"swcal_cellmix({kind}, {waves}) returned {rc}")
            rows[str(waves)] = round(cells.value / ms.value / 1e6, 1)
        out[name] = {"gcups_equiv_by_waves_per_cu": rows, "best": max(rows.values())}
    return {"calibration": "register-only DP cell mix, 16 rows x 2 chains per lane",
            "unit": "GCUPS-equivalent", "tiers": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # default: 3 timed steps, 100 for the plain search, whose step (one search of about
    # 0.3 ms) is otherwise dominated by the first launch's start from an idle device
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="full",
                    choices=["full", "plain", "long_mix", "batched", "served"])
    ap.add_argument("--rates", default="2,8,32", help="served: arrival rates per second")
    ap.add_argument("--requests", default="48,96,192",
                    help="served: requests per rate (one value, or one per rate)")
    ap.add_argument("--slots", type=int, default=2, help="served: records on the device at once (session mode) or stream slots (batch mode)")
    ap.add_argument("--max-batch", type=int, default=8, help="served: queries per launch")
    ap.add_argument("--mem-budget-gib", type=float, default=64.0,
                    help="served: device memory budget of the batches in flight")
    ap.add_argument("--seqs", type=int, default=None, help="override database size (testing)")
    ap.add_argument("--cpu-cells", type=float, default=2.5e10,
                    help="oracle sample size in cells (about 10-30 s on the host)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched: skip the autotuner (automatic strip height and grid)")
    ap.add_argument("--no-tune-cache", action="store_true",
                    help="batched: re-run the autotuner instead of reading its cache")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (calibrates the "
                         "HBM byte counters of a profiler run)")
    ap.add_argument("--calibrate", action="store_true",
                    help="time register-only copies of the DP cell at int16 x 2, int32 and "
                         "SWAR int8 x 4 (libswmi_calib.so) and exit")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 100 if args.workload == "plain" else 3
    if args.calibrate:
        print(json.dumps(calibrate()), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); "
              "across GPUs the database would be sharded by sequence groups, each GPU "
              "searching its shard and the scores gathered", file=sys.stderr)
        sys.exit(2)

    from paper_1702_07195_amd import synth

    if args.workload == "batched":
        result = bench_batched(args)
    elif args.workload == "served":
        result = bench_served(args)
    else:
        w, label = {"full": (synth.FULL_SCALE, "full-scale plain search"),
                    "plain": (synth.PLAIN, "plain search"),
                    "long_mix": (synth.LONG_MIX, "long-sequence mix")}[args.workload]
        if args.seqs is not None:
            w = synth.scaled(w, args.seqs)
        result = bench_search(args, w, label)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
