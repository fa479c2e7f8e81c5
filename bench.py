"""Benchmark: GCUPS of the full-scale plain database search on one MI355X.

Workload (synthetic stand-in for the paper's Environmental NR search, Section 5.1):
6,000,000 database sequences (log-normal lengths, median 200, sigma 0.8, clipped to
10..8000; about 1.65e9 residues at Robinson-Robinson frequencies) searched with six
synthetic queries of lengths 144, 375, 729, 1000, 2005 and 5478; BLOSUM62, gap open 10,
gap extend 2.  One step is one search of every query against the whole database (all
stages of the path: query profiles, packed-int16 inter-task kernel, saturation recompute,
scores in the caller's order in HBM).  GCUPS = sum(|Q|) * |D| / t (Section 5.2, Eq. 4),
with |D| the unpadded residue count.

Prints one JSON line.  Extra fields: per-query-length GCUPS, a roofline object for the
inter-task kernel (timed with HIP events on its own stream) and the CPU oracle timed on
a bounded sample of the same workload.
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

# int16 algorithmic operations per DP cell (Section 2, Eqs. 1-3): H-Goe, E-Ge and max,
# F-Ge and max, H(diag)+SM, three maxima for H, running maximum.
OPS_PER_CELL = 10
# Packed-int16 VALU peak of MI355X: 256 CUs x 64 lanes x 2 halves x 2.4 GHz.
PEAK_INT16_TOPS = 256 * 64 * 2 * 2.4e9 / 1e12
KERNEL_SRC = os.path.join(ROOT, "paper_1702_07195_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "inter16_full_scale_traffic.json")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(per_launch_cells: float):
    """HBM bytes per launch from committed PMC runs, if taken on the current kernel."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(db, queries, sm, go, ge, gpu_scores, budget_cells: float):
    """Time the oracle on a stratified sample of sequences (all queries), and check the
    sampled GPU scores against it bit for bit."""
    import oracle
    from paper_1702_07195_amd import synth  # noqa: F401

    lengths = db.lengths
    order = np.argsort(lengths, kind="stable")
    per_seq = float(sum(len(q) for q in queries)) * float(lengths.mean())
    n = int(max(64, min(len(order), budget_cells / max(per_seq, 1.0))))
    idx = order[np.linspace(0, len(order) - 1, n).astype(np.int64)]
    threads = os.cpu_count() or 1
    cells = 0
    t0 = time.perf_counter()
    exact = True
    for q, g in zip(queries, gpu_scores):
        want = oracle.search(q, db.residues, db.offsets, sm, go, ge, index=idx, threads=threads)
        exact &= bool(np.array_equal(want, g[idx]))
        cells += len(q) * int(lengths[idx].sum())
    dt = time.perf_counter() - t0
    return {"value": cells / dt / 1e9, "unit": "GCUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n} database sequences (stratified by length) x all {len(queries)} "
                      f"queries, {cells:.3e} cells, {dt:.1f} s"}, exact


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seqs", type=int, default=None, help="override database size (testing)")
    ap.add_argument("--cpu-cells", type=float, default=1.2e10,
                    help="oracle sample size in cells (about 10-30 s on the host)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (calibrates the "
                         "HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the database would be sharded across GPUs as described in DESIGN.md",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1702_07195_amd import swmi, synth

    w = synth.FULL_SCALE if args.seqs is None else synth.scaled(synth.FULL_SCALE, args.seqs)
    db = w.make_db()
    queries = w.make_queries()
    sm, go, ge = w.matrix_values, w.gap_open, w.gap_extend
    D = int(db.offsets[-1])
    h = swmi.sw_db_load(db.residues, db.offsets, len(synth.ALPHABET))
    dev = torch.device("cuda:0")
    outs = [torch.zeros(db.n_seqs, dtype=torch.int32, device=dev) for _ in queries]
    stream = torch.cuda.current_stream()

    def step(per_query=None):
        for k, q in enumerate(queries):
            if per_query is not None:
                torch.cuda.synchronize()
                t = time.perf_counter()
            h.search_async(q, sm, go, ge, outs[k], stream)
            if per_query is not None:
                torch.cuda.synchronize()
                per_query[k] += time.perf_counter() - t

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
    launches, kernel_ms = h.timing_read()
    h.timing_enable(False)

    # per-query-length GCUPS (separate pass, each query synchronised on its own)
    per_q = [0.0] * len(queries)
    step(per_q)
    per_query = {str(len(q)): round(len(q) * D / per_q[k] / 1e9, 1)
                 for k, q in enumerate(queries)}

    cells_per_step = sum(len(q) for q in queries) * D
    gcups = cells_per_step * args.steps / elapsed / 1e9
    cells_per_launch = cells_per_step / len(queries)
    avg_launch_s = kernel_ms / max(launches, 1) / 1e3
    achieved = OPS_PER_CELL * cells_per_launch / avg_launch_s / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(PEAK_INT16_TOPS, 2),
                "unit": "Tops/s (int16)", "frac": round(achieved / PEAK_INT16_TOPS, 3),
                "traffic": load_traffic(cells_per_launch),
                "kernel": "k_inter16", "avg_launch_ms": round(avg_launch_s * 1e3, 3),
                "launches": launches}

    result = {
        "metric": "GCUPS per query length (1 GPU, bit-exact)",
        "value": round(gcups, 1),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i16",
        "data": "synthetic",
        "config": {"workload": "full-scale plain search", "db_seqs": db.n_seqs,
                   "db_residues": D, "query_lengths": [len(q) for q in queries],
                   "matrix": w.matrix, "gap_open": go, "gap_extend": ge},
        "per_query_gcups": per_query,
        "roofline": roofline,
    }
    if not args.no_cpu:
        gpu_scores = [o.cpu().numpy() for o in outs]
        base, exact = cpu_baseline(db, queries, sm, go, ge, gpu_scores, args.cpu_cells)
        result["cpu_baseline"] = base
        result["bit_exact_sample"] = exact
    h.free()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
