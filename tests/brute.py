"""Independent references used to pin the oracle (pure Python, tiny inputs only).

None of these evaluates the Gotoh recurrences of the oracle.  Each one computes the
local alignment score from a different, textbook definition:

* ``enumerate_best``: the definition itself.  Every alignment between every pair of
  substrings is enumerated (matches, gaps in either sequence, gaps in both sequences
  next to each other) and scored as the sum of substitution scores minus, for each
  maximal run of k gap symbols, ``gap_open + k * gap_extend`` (paper, Section 2: Goe is
  open + extend, Ge is extend).  The empty alignment scores 0.
* ``linear_gap_sw``: Smith & Waterman's 1981 single-matrix recurrence with a linear
  gap cost of ``g`` per gap symbol, which the affine model reduces to when the open
  penalty is 0.
* ``kadane_diagonals``: the best ungapped local alignment, i.e. the maximum subarray
  (Kadane) of substitution scores along every diagonal.
* ``longest_common_substring``.
"""
from __future__ import annotations


def enumerate_best(q, d, sm, gap_open: int, gap_extend: int) -> int:
    q = [int(x) for x in q]
    d = [int(x) for x in d]
    m, n = len(q), len(d)
    best = 0

    # Depth-first walk over alignment columns, starting from every (i0, j0) and
    # recording the running score after every column (an alignment may end anywhere).
    # `last` is the kind of the previous column: 'M' (pair), 'I' (query residue
    # against a gap) or 'D' (database residue against a gap).
    def walk(i, j, last, s):
        nonlocal best
        if s > best:
            best = s
        if i < m and j < n:
            walk(i + 1, j + 1, "M", s + sm[q[i]][d[j]])
        if i < m:
            walk(i + 1, j, "I", s - (gap_extend if last == "I" else gap_open + gap_extend))
        if j < n:
            walk(i, j + 1, "D", s - (gap_extend if last == "D" else gap_open + gap_extend))

    for i0 in range(m + 1):
        for j0 in range(n + 1):
            walk(i0, j0, None, 0)
    return best


def linear_gap_sw(q, d, sm, g: int) -> int:
    m, n = len(q), len(d)
    H = [[0] * (n + 1) for _ in range(m + 1)]
    best = 0
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            H[i][j] = max(0,
                          H[i - 1][j - 1] + sm[int(q[i - 1])][int(d[j - 1])],
                          H[i][j - 1] - g,
                          H[i - 1][j] - g)
            best = max(best, H[i][j])
    return best


def kadane_diagonals(q, d, sm) -> int:
    m, n = len(q), len(d)
    best = 0
    for off in range(-(m - 1), n):
        run = 0
        for i in range(m):
            j = i + off
            if 0 <= j < n:
                run = max(0, run + sm[int(q[i])][int(d[j])])
                best = max(best, run)
    return best


def longest_common_substring(a, b) -> int:
    a = [int(x) for x in a]
    b = [int(x) for x in b]
    best = 0
    for i in range(len(a)):
        for j in range(len(b)):
            k = 0
            while i + k < len(a) and j + k < len(b) and a[i + k] == b[j + k]:
                k += 1
            best = max(best, k)
    return best
