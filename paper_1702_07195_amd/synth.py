"""Seeded synthetic inputs for protein database search.

This module only *generates inputs*: residue codes, sequence lengths, substitution
matrices and the workload recipes.  It contains none of the alignment arithmetic, so
both the GPU path and the CPU oracle can draw from it without sharing any method code.

The paper evaluates on the Environmental NR database (release 2016_11) and twenty
Swiss-Prot queries (Section 5.1).  Neither is available here, so every workload is a
synthetic stand-in with the shape of those inputs:

* residues are i.i.d. over the 20 standard amino acids at the background
  frequencies of Robinson & Robinson, PNAS 88:8880 (1991), Table 1;
* sequence lengths follow ``clip(rint(exp(ln(median) + sigma * N(0, 1))), lo, hi)``;
* substitution scores come from BLOSUM62 / BLOSUM50 (Henikoff & Henikoff, PNAS
  89:10915, 1992), the matrix family used in Section 5.1, transcribed from the
  published tables in the usual 24-letter order ``ARNDCQEGHILKMFPSTWYVBZX*``.

All randomness comes from numpy's PCG64 with explicit seeds.
"""
from __future__ import annotations

import dataclasses
from typing import Iterator

import numpy as np

# --------------------------------------------------------------------------- alphabet
ALPHABET = "ARNDCQEGHILKMFPSTWYVBZX*"
N_STANDARD = 20  # codes 0..19 are the standard amino acids; 20..23 are B, Z, X, *
CODE = {c: i for i, c in enumerate(ALPHABET)}

# Robinson & Robinson (1991) background frequencies, in ALPHABET order (first 20).
RR_FREQS = np.array([
    0.07805, 0.05129, 0.04487, 0.05364, 0.01925, 0.04264, 0.06295, 0.07377,
    0.02199, 0.05142, 0.09019, 0.05744, 0.02243, 0.03856, 0.05203, 0.07120,
    0.05841, 0.01330, 0.03216, 0.06441,
], dtype=np.float64)

# --------------------------------------------------------------------------- matrices
_BLOSUM62_ROWS = """
 4 -1 -2 -2  0 -1 -1  0 -2 -1 -1 -1 -1 -2 -1  1  0 -3 -2  0 -2 -1  0 -4
-1  5  0 -2 -3  1  0 -2  0 -3 -2  2 -1 -3 -2 -1 -1 -3 -2 -3 -1  0 -1 -4
-2  0  6  1 -3  0  0  0  1 -3 -3  0 -2 -3 -2  1  0 -4 -2 -3  3  0 -1 -4
-2 -2  1  6 -3  0  2 -1 -1 -3 -4 -1 -3 -3 -1  0 -1 -4 -3 -3  4  1 -1 -4
 0 -3 -3 -3  9 -3 -4 -3 -3 -1 -1 -3 -1 -2 -3 -1 -1 -2 -2 -1 -3 -3 -2 -4
-1  1  0  0 -3  5  2 -2  0 -3 -2  1  0 -3 -1  0 -1 -2 -1 -2  0  3 -1 -4
-1  0  0  2 -4  2  5 -2  0 -3 -3  1 -2 -3 -1  0 -1 -3 -2 -2  1  4 -1 -4
 0 -2  0 -1 -3 -2 -2  6 -2 -4 -4 -2 -3 -3 -2  0 -2 -2 -3 -3 -1 -2 -1 -4
-2  0  1 -1 -3  0  0 -2  8 -3 -3 -1 -2 -1 -2 -1 -2 -2  2 -3  0  0 -1 -4
-1 -3 -3 -3 -1 -3 -3 -4 -3  4  2 -3  1  0 -3 -2 -1 -3 -1  3 -3 -3 -1 -4
-1 -2 -3 -4 -1 -2 -3 -4 -3  2  4 -2  2  0 -3 -2 -1 -2 -1  1 -4 -3 -1 -4
-1  2  0 -1 -3  1  1 -2 -1 -3 -2  5 -1 -3 -1  0 -1 -3 -2 -2  0  1 -1 -4
-1 -1 -2 -3 -1  0 -2 -3 -2  1  2 -1  5  0 -2 -1 -1 -1 -1  1 -3 -1 -1 -4
-2 -3 -3 -3 -2 -3 -3 -3 -1  0  0 -3  0  6 -4 -2 -2  1  3 -1 -3 -3 -1 -4
-1 -2 -2 -1 -3 -1 -1 -2 -2 -3 -3 -1 -2 -4  7 -1 -1 -4 -3 -2 -2 -1 -2 -4
 1 -1  1  0 -1  0  0  0 -1 -2 -2  0 -1 -2 -1  4  1 -3 -2 -2  0  0  0 -4
 0 -1  0 -1 -1 -1 -1 -2 -2 -1 -1 -1 -1 -2 -1  1  5 -2 -2  0 -1 -1  0 -4
-3 -3 -4 -4 -2 -2 -3 -2 -2 -3 -2 -3 -1  1 -4 -3 -2 11  2 -3 -4 -3 -2 -4
-2 -2 -2 -3 -2 -1 -2 -3  2 -1 -1 -2 -1  3 -3 -2 -2  2  7 -1 -3 -2 -1 -4
 0 -3 -3 -3 -1 -2 -2 -3 -3  3  1 -2  1 -1 -2 -2  0 -3 -1  4 -3 -2 -1 -4
-2 -1  3  4 -3  0  1 -1  0 -3 -4  0 -3 -3 -2  0 -1 -4 -3 -3  4  1 -1 -4
-1  0  0  1 -3  3  4 -2  0 -3 -3  1 -1 -3 -1  0 -1 -3 -2 -2  1  4 -1 -4
 0 -1 -1 -1 -2 -1 -1 -1 -1 -1 -1 -1 -1 -1 -2  0  0 -2 -1 -1 -1 -1 -1 -4
-4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4  1
"""

_BLOSUM50_ROWS = """
 5 -2 -1 -2 -1 -1 -1  0 -2 -1 -2 -1 -1 -3 -1  1  0 -3 -2  0 -2 -1 -1 -5
-2  7 -1 -2 -4  1  0 -3  0 -4 -3  3 -2 -3 -3 -1 -1 -3 -1 -3 -1  0 -1 -5
-1 -1  7  2 -2  0  0  0  1 -3 -4  0 -2 -4 -2  1  0 -4 -2 -3  4  0 -1 -5
-2 -2  2  8 -4  0  2 -1 -1 -4 -4 -1 -4 -5 -1  0 -1 -5 -3 -4  5  1 -1 -5
-1 -4 -2 -4 13 -3 -3 -3 -3 -2 -2 -3 -2 -2 -4 -1 -1 -5 -3 -1 -3 -3 -2 -5
-1  1  0  0 -3  7  2 -2  1 -3 -2  2  0 -4 -1  0 -1 -1 -1 -3  0  4 -1 -5
-1  0  0  2 -3  2  6 -3  0 -4 -3  1 -2 -3 -1 -1 -1 -3 -2 -3  1  5 -1 -5
 0 -3  0 -1 -3 -2 -3  8 -2 -4 -4 -2 -3 -4 -2  0 -2 -3 -3 -4 -1 -2 -2 -5
-2  0  1 -1 -3  1  0 -2 10 -4 -3  0 -1 -1 -2 -1 -2 -3  2 -4  0  0 -1 -5
-1 -4 -3 -4 -2 -3 -4 -4 -4  5  2 -3  2  0 -3 -3 -1 -3 -1  4 -4 -3 -1 -5
-2 -3 -4 -4 -2 -2 -3 -4 -3  2  5 -3  3  1 -4 -3 -1 -2 -1  1 -4 -3 -1 -5
-1  3  0 -1 -3  2  1 -2  0 -3 -3  6 -2 -4 -1  0 -1 -3 -2 -3  0  1 -1 -5
-1 -2 -2 -4 -2  0 -2 -3 -1  2  3 -2  7  0 -3 -2 -1 -1  0  1 -3 -1 -1 -5
-3 -3 -4 -5 -2 -4 -3 -4 -1  0  1 -4  0  8 -4 -3 -2  1  4 -1 -4 -4 -2 -5
-1 -3 -2 -1 -4 -1 -1 -2 -2 -3 -4 -1 -3 -4 10 -1 -1 -4 -3 -3 -2 -1 -2 -5
 1 -1  1  0 -1  0 -1  0 -1 -3 -3  0 -2 -3 -1  5  2 -4 -2 -2  0  0 -1 -5
 0 -1  0 -1 -1 -1 -1 -2 -2 -1 -1 -1 -1 -2 -1  2  5 -3 -2  0  0 -1  0 -5
-3 -3 -4 -5 -5 -1 -3 -3 -3 -3 -2 -3 -1  1 -4 -4 -3 15  2 -3 -5 -2 -3 -5
-2 -1 -2 -3 -3 -1 -2 -3  2 -1 -1 -2  0  4 -3 -2 -2  2  8 -1 -3 -2 -1 -5
 0 -3 -3 -4 -1 -3 -3 -4 -4  4  1 -3  1 -1 -3 -2  0 -3 -1  5 -4 -3 -1 -5
-2 -1  4  5 -3  0  1 -1  0 -4 -4  0 -3 -4 -2  0  0 -5 -3 -4  5  2 -1 -5
-1  0  0  1 -3  4  5 -2  0 -3 -3  1 -1 -4 -1  0 -1 -2 -2 -3  2  5 -1 -5
-1 -1 -1 -1 -2 -1 -1 -2 -1 -1 -1 -1 -1 -2 -2 -1  0 -3 -1 -1 -1 -1 -1 -5
-5 -5 -5 -5 -5 -5 -5 -5 -5 -5 -5 -5 -5 -5 -5 -5 -5 -5 -5 -5 -5 -5 -5  1
"""


def _parse(rows: str) -> np.ndarray:
    m = np.array([[int(x) for x in line.split()] for line in rows.strip().splitlines()],
                 dtype=np.int32)
    assert m.shape == (len(ALPHABET), len(ALPHABET))
    return m


BLOSUM62 = _parse(_BLOSUM62_ROWS)
BLOSUM50 = _parse(_BLOSUM50_ROWS)
MATRICES = {"BLOSUM62": BLOSUM62, "BLOSUM50": BLOSUM50}


def encode(text: str) -> np.ndarray:
    """Letters of ALPHABET -> uint8 codes."""
    return np.array([CODE[c] for c in text], dtype=np.uint8)


def decode(codes) -> str:
    return "".join(ALPHABET[int(c)] for c in codes)


# --------------------------------------------------------------------------- sampling
def _residue_lut(freqs: np.ndarray) -> np.ndarray:
    """2^16-entry table that maps a uniform uint16 to a residue code.

    Quantising the CDF to 1/65536 keeps every frequency within 1.6e-5 of its target.
    """
    cdf = np.cumsum(freqs / freqs.sum())
    mids = (np.arange(65536, dtype=np.float64) + 0.5) / 65536.0
    return np.minimum(np.searchsorted(cdf, mids, side="right"), len(freqs) - 1).astype(np.uint8)


_RR_LUT = _residue_lut(RR_FREQS)


def residues(rng: np.random.Generator, count: int, chunk: int = 1 << 27) -> np.ndarray:
    """``count`` i.i.d. residue codes (0..19) at the Robinson-Robinson frequencies."""
    out = np.empty(int(count), dtype=np.uint8)
    for s in range(0, int(count), chunk):
        e = min(int(count), s + chunk)
        out[s:e] = _RR_LUT[rng.integers(0, 65536, size=e - s, dtype=np.uint16)]
    return out


def lognormal_lengths(rng: np.random.Generator, count: int, median: float, sigma: float,
                      lo: int, hi: int) -> np.ndarray:
    """``clip(rint(exp(ln(median) + sigma * z)), lo, hi)`` with z ~ N(0, 1), as int64."""
    z = rng.standard_normal(int(count))
    return np.clip(np.rint(np.exp(np.log(median) + sigma * z)), lo, hi).astype(np.int64)


@dataclasses.dataclass
class SeqDB:
    """A database in the C-ABI's input form: concatenated codes plus n+1 offsets."""
    residues: np.ndarray  # uint8[offsets[-1]]
    offsets: np.ndarray   # int64[n_seqs + 1]

    @property
    def n_seqs(self) -> int:
        return len(self.offsets) - 1

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def seq(self, k: int) -> np.ndarray:
        return self.residues[self.offsets[k]:self.offsets[k + 1]]


def db_from_lengths(rng: np.random.Generator, lengths: np.ndarray) -> SeqDB:
    offsets = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    return SeqDB(residues(rng, int(offsets[-1])), offsets)


def db_from_seqs(seqs) -> SeqDB:
    lengths = np.array([len(s) for s in seqs], dtype=np.int64)
    offsets = np.zeros(len(seqs) + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    res = np.concatenate([np.asarray(s, dtype=np.uint8) for s in seqs]) if len(seqs) else \
        np.zeros(0, dtype=np.uint8)
    return SeqDB(res.astype(np.uint8), offsets)


def random_matrix(rng: np.random.Generator, alphabet: int, lo: int = -10, hi: int = 10,
                  symmetric: bool = False) -> np.ndarray:
    m = rng.integers(lo, hi + 1, size=(alphabet, alphabet)).astype(np.int32)
    if symmetric:
        m = np.triu(m) + np.triu(m, 1).T
    return np.ascontiguousarray(m, dtype=np.int32)


# --------------------------------------------------------------------------- workloads
@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload recipe (all sizes, laws and seeds)."""
    name: str
    n_seqs: int
    median: float
    sigma: float
    lo: int
    hi: int
    query_lengths: tuple
    matrix: str = "BLOSUM62"
    gap_open: int = 10
    gap_extend: int = 2
    db_seed: int = 0
    query_seed: int = 0
    # long-sequence mix: fraction of sequences drawn uniformly from [long_lo, long_hi]
    long_frac: float = 0.0
    long_lo: int = 0
    long_hi: int = 0

    def make_db(self) -> SeqDB:
        rng = np.random.Generator(np.random.PCG64(self.db_seed))
        lengths = lognormal_lengths(rng, self.n_seqs, self.median, self.sigma, self.lo, self.hi)
        if self.long_frac > 0:
            n_long = int(round(self.long_frac * self.n_seqs))
            idx = rng.permutation(self.n_seqs)[:n_long]
            lengths[idx] = rng.integers(self.long_lo, self.long_hi + 1, size=n_long)
        return db_from_lengths(rng, lengths)

    def make_queries(self) -> list:
        rng = np.random.Generator(np.random.PCG64(self.query_seed))
        return [residues(rng, m) for m in self.query_lengths]

    @property
    def matrix_values(self) -> np.ndarray:
        return MATRICES[self.matrix]


# Section 5.1 uses BLOSUM62 with gap penalties 10 (open) and 2 (extend).
PLAIN = Workload("plain", n_seqs=2000, median=250, sigma=0.7, lo=20, hi=2000,
                 query_lengths=(144,), db_seed=1702_0001, query_seed=1702_1001)

# Query lengths of the paper's twenty-query set span 144..5478 (Section 5.1).
FULL_SCALE = Workload("full_scale", n_seqs=6_000_000, median=200, sigma=0.8, lo=10,
                      hi=8000, query_lengths=(144, 375, 729, 1000, 2005, 5478),
                      db_seed=1702_0002, query_seed=1702_1002)

BATCHED = Workload("batched", n_seqs=200_000, median=200, sigma=0.8, lo=10, hi=8000,
                   query_lengths=(), db_seed=1702_0003, query_seed=1702_1003)

LONG_MIX = Workload("long_mix", n_seqs=10_000, median=300, sigma=0.8, lo=10, hi=8000,
                    query_lengths=(5478, 35000), db_seed=1702_0005, query_seed=1702_1005,
                    long_frac=0.01, long_lo=10_000, long_hi=35_000)

SERVED = Workload("served", n_seqs=4_350_000, median=200, sigma=0.8, lo=10, hi=8000,
                  query_lengths=(), db_seed=1702_0004, query_seed=1702_1004)


def batched_queries(n: int = 64, lo: int = 50, hi: int = 5000, seed: int = 1702_1003) -> list:
    rng = np.random.Generator(np.random.PCG64(seed))
    lens = rng.integers(lo, hi + 1, size=n)
    return [residues(rng, int(m)) for m in lens]


def served_queries(n: int, seed: int = 1702_1004, median: float = 350, sigma: float = 0.8,
                   lo: int = 30, hi: int = 5000) -> list:
    rng = np.random.Generator(np.random.PCG64(seed))
    lens = lognormal_lengths(rng, n, median, sigma, lo, hi)
    return [residues(rng, int(m)) for m in lens]


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Open-loop arrival times (seconds from start) of n requests at ``rate`` per second."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def scaled(w: Workload, n_seqs: int, name: str | None = None) -> Workload:
    """The same length law and seeds at a smaller sequence count (for tests)."""
    return dataclasses.replace(w, n_seqs=n_seqs, name=name or f"{w.name}_{n_seqs}")


def iter_chunks(n: int, size: int) -> Iterator[tuple]:
    for s in range(0, n, size):
        yield s, min(n, s + size)
