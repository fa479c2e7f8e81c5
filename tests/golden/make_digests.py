"""Write oracle score digests for the full-size workloads (test infrastructure).

The oracle (plain int32 Gotoh, paper Section 2, Eqs. 1-3) scores every query of a
workload against every database sequence; this script stores, per slice of the score
vector in the caller's order, the SHA-256 of the int32 little-endian scores, their sum,
their maximum and a coarse histogram.  A GPU test recomputes the same figures from the
library's scores, so parity at full size covers every sequence, not a sample, and a
mismatch is localised to a slice and a score range.

Only ``oracle`` (the scores) and ``synth`` (the seeded inputs) are used.  The output is
``tests/golden/digests.txt``, one line per slice; slices already in the file are
skipped, so an interrupted run resumes where it stopped.

    python tests/golden/make_digests.py [--only long_mix,full_scale,batched] [--threads N]
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1702_07195_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "digests.txt")

# Histogram bin edges of a slice's scores (the last bin is open-ended).
HIST_EDGES = (0, 1, 20, 40, 80, 160, 320, 640, 1280, 32767)

# Slice length (sequences) per workload: a full-scale slice of the 5478-residue query
# is about 4e11 cells, a few minutes of the oracle on a handful of host cores.
SLICE = {"full_scale": 250_000, "long_mix": 10_000, "batched": 200_000}

# Matrix and gap settings per workload (the batched workload is checked under two of
# its four settings).
SETTINGS = {
    "long_mix": [("BLOSUM62", 10, 2)],
    "full_scale": [("BLOSUM62", 10, 2)],
    "batched": [("BLOSUM62", 10, 2), ("BLOSUM50", 11, 1)],
}

WORKLOADS = {"long_mix": synth.LONG_MIX, "full_scale": synth.FULL_SCALE,
             "batched": synth.BATCHED}


def queries_of(name: str) -> list:
    if name == "batched":
        return synth.batched_queries(64)
    return WORKLOADS[name].make_queries()


def slice_record(scores: np.ndarray) -> tuple:
    """(sha256 hex, sum, max, histogram string) of one slice of int32 scores."""
    s = np.ascontiguousarray(scores, dtype="<i4")
    digest = hashlib.sha256(s.tobytes()).hexdigest()
    hist = np.histogram(s, bins=list(HIST_EDGES) + [1 << 31])[0]
    return digest, int(s.sum(dtype=np.int64)), int(s.max()) if len(s) else 0, \
        ",".join(str(int(c)) for c in hist)


def key(fields) -> tuple:
    return tuple(fields[:8])


def read_done(path: str = OUT) -> set:
    done = set()
    if os.path.exists(path):
        with open(path) as f:
            for line in f:
                if line.strip() and not line.startswith("#"):
                    done.add(key(line.split()))
    return done


def parse(path: str = OUT) -> list:
    """Every slice line as a dict (used by the GPU digest test)."""
    out = []
    if not os.path.exists(path):
        return out
    with open(path) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            w = line.split()
            out.append(dict(workload=w[0], matrix=w[1], gap_open=int(w[2]),
                            gap_extend=int(w[3]), query=int(w[4]), qlen=int(w[5]),
                            begin=int(w[6]), end=int(w[7]), sha256=w[8], sum=int(w[9]),
                            max=int(w[10]), hist=w[11]))
    return out


HEADER = """\
# Oracle score digests of the full-size workloads, written by tests/golden/make_digests.py
# (oracle + seeded synthetic inputs only; paper Section 2, Eqs. 1-3).
# Fields: workload matrix gap_open gap_extend query_index query_len begin end
#         sha256(int32 LE scores[begin:end], caller order) sum max histogram
# Histogram bins: [0,1) [1,20) [20,40) [40,80) [80,160) [160,320) [320,640) [640,1280)
#                 [1280,32767) [32767,inf)
"""


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="long_mix,full_scale,batched")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    done = read_done()
    if not os.path.exists(OUT):
        with open(OUT, "w") as f:
            f.write(HEADER)
    for name in args.only.split(","):
        w = WORKLOADS[name]
        t0 = time.time()
        db = w.make_db()
        qs = queries_of(name)
        print(f"{name}: {db.n_seqs} sequences, {int(db.offsets[-1])} residues, "
              f"{len(qs)} queries ({time.time() - t0:.0f} s to generate)", flush=True)
        step = SLICE[name]
        for mat, go, ge in SETTINGS[name]:
            sm = synth.MATRICES[mat]
            for qi, q in enumerate(qs):
                for b in range(0, db.n_seqs, step):
                    e = min(db.n_seqs, b + step)
                    k = (name, mat, str(go), str(ge), str(qi), str(len(q)), str(b), str(e))
                    if k in done:
                        continue
                    t1 = time.time()
                    idx = np.arange(b, e, dtype=np.int64)
                    scores = oracle.search(q, db.residues, db.offsets, sm, go, ge,
                                           index=idx, threads=args.threads)
                    digest, total, mx, hist = slice_record(scores)
                    line = " ".join(k) + f" {digest} {total} {mx} {hist}\n"
                    with open(OUT, "a") as f:
                        f.write(line)
                    cells = len(q) * int(db.offsets[e] - db.offsets[b])
                    dt = time.time() - t1
                    print(f"{name} {mat} {go}/{ge} q{qi} m={len(q)} [{b},{e}) "
                          f"{dt:.0f} s {cells / dt / 1e9:.2f} GCUPS", flush=True)
        del db


if __name__ == "__main__":
    main()
