"""Autotuner for batched searches: strip height, persistent waves per CU and bin width.

A candidate configuration is timed on the real workload: the queries are sorted by
length and cut into bins of ``bin_width`` queries, each bin is captured as a HIP-graph
plan (``sw_plan_create``) with the candidate's strip height and waves per CU, and the
plans are replayed back to back.  The fastest candidate is kept in a JSON cache keyed by
a signature of the workload (database size and residue count, query count and length
histogram), so later runs with the same shape skip the search.  Scores do not depend on
the configuration (every candidate is a different schedule of the same exact DP).

Cache file: ``$SWMI_AUTOTUNE_CACHE`` or ``~/.cache/swmi_autotune.json``.
"""
from __future__ import annotations

import dataclasses
import json
import os
import time

import numpy as np

from . import swmi

STRIP_HEIGHTS = (16, 24, 28, 32, 40)  # 28: query-pair searches only
WAVES_PER_CU = (0, 8, 12, 16)      # 0 = occupancy limit of the kernel
BIN_WIDTHS = (0, 32, 16)           # 0 = the whole batch in one launch


@dataclasses.dataclass(frozen=True)
class Config:
    strip_rows: int = 0
    waves_per_cu: int = 0
    bin_width: int = 0

    def as_dict(self):
        return dataclasses.asdict(self)


def cache_path() -> str:
    return os.environ.get("SWMI_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache",
                                       "swmi_autotune.json"))


def signature(db: "swmi.SwDb", residues: int, queries) -> str:
    lens = np.array([len(q) for q in queries], dtype=np.int64)
    hist = np.histogram(lens, bins=[0, 128, 256, 512, 1024, 2048, 4096, 8192, 1 << 30])[0]
    return (f"n{db.n_seqs}-r{int(residues) >> 20}M-q{len(lens)}-"
            + "-".join(str(int(x)) for x in hist))


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(cache: dict):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def bins(queries, width: int):
    """Indices of the queries, sorted by length (longest first), cut into bins."""
    order = sorted(range(len(queries)), key=lambda k: -len(queries[k]))
    if width <= 0 or width >= len(order):
        return [order]
    return [order[i:i + width] for i in range(0, len(order), width)]


class BinnedPlans:
    """One captured plan per bin; ``out`` rows follow the caller's query order."""

    def __init__(self, db, queries, matrix, gap_open, gap_extend, out, config: Config):
        import torch
        self.plans = []
        self.bins = bins(queries, config.bin_width)
        old = {k: swmi.get_knob(k) for k in (swmi.SW_KNOB_STRIP_ROWS, swmi.SW_KNOB_GRID_WAVES)}
        try:
            swmi.set_knob(swmi.SW_KNOB_STRIP_ROWS, config.strip_rows)
            swmi.set_knob(swmi.SW_KNOB_GRID_WAVES, config.waves_per_cu)
            self.bufs = []
            for b in self.bins:
                buf = torch.empty((len(b), db.n_seqs), dtype=torch.int32, device=out.device)
                self.plans.append(db.plan([queries[k] for k in b], matrix, gap_open,
                                          gap_extend, buf))
                self.bufs.append(buf)
        finally:
            for k, v in old.items():
                swmi.set_knob(k, v)
        self.out = out

    def launch(self, stream=None):
        for p in self.plans:
            p.launch(stream)

    def gather(self):
        """Copy the bins' scores into ``out`` (caller's query order)."""
        import torch
        for b, buf in zip(self.bins, self.bufs):
            self.out[torch.tensor(b, device=self.out.device)] = buf

    def free(self):
        for p in self.plans:
            p.free()
        self.plans = []


def default_candidates():
    """Strip heights x bin widths at the occupancy limit, plus lower wave counts for the
    usual best strip height."""
    return ([Config(t, 0, b) for b in (0, 16) for t in STRIP_HEIGHTS] +
            [Config(24, w, 0) for w in WAVES_PER_CU if w != 0])


def time_config(db, queries, matrix, gap_open, gap_extend, out, config: Config,
                reps: int = 1) -> float:
    import torch
    plans = BinnedPlans(db, queries, matrix, gap_open, gap_extend, out, config)
    try:
        stream = torch.cuda.current_stream()
        plans.launch(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plans.launch(stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps
    finally:
        plans.free()


def tune(db, residues: int, queries, matrix, gap_open, gap_extend, out, use_cache=True,
         candidates=None, log=None) -> tuple:
    """Best Config for this workload (from the cache, or timed), and the timings."""
    key = signature(db, residues, queries)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return Config(**cache[key]["config"]), cache[key].get("timings", {})
    if candidates is None:
        candidates = default_candidates()
    timings = {}
    best, best_t = None, float("inf")
    for c in candidates:
        t = time_config(db, queries, matrix, gap_open, gap_extend, out, c)
        timings[json.dumps(c.as_dict(), sort_keys=True)] = round(t * 1e3, 3)
        if log:
            log(f"autotune {c}: {t * 1e3:.2f} ms")
        if t < best_t:
            best, best_t = c, t
    if use_cache:
        cache[key] = {"config": best.as_dict(), "timings": timings}
        _save_cache(cache)
    return best, timings
