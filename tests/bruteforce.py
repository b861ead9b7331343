"""Independent checks used to pin the CPU oracle (test helpers only).

Nothing here evaluates the paper's recurrence (Eq. 1).  Each function
reaches the same quantity by another route:

* ``enumerate_h``: exhaustive enumeration of every alignment path (match,
  insertion, deletion moves; each gap run of k bases costs
  gap_open + k*gap_extend) from every start cell; H(i, j) is the best score
  of any path whose last consumed target/query bases are (i, j), floored
  at 0.  Exponential -- tiny inputs only.
* ``kadane_table``: the ungapped case; Kadane's maximum-subarray running
  value along every diagonal.
* ``linear_sw_table``: the classic single-matrix Smith-Waterman with a
  linear gap penalty (Smith & Waterman 1981), which Eq. 1 reduces to when
  gap_open is 0.
* ``common_suffix_table``: longest common substring by direct comparison
  (the case where any mismatch or gap is prohibitively costly).
* ``first_max``: the end-position convention (highest value, then smallest
  target row, then smallest query column).
"""
from __future__ import annotations

import sys

NEG = None


def _s(tb, qb, a, b):
    # N (unknown base) scores the mismatch against every base, N included
    return a if tb == qb and tb != "N" else b


def enumerate_h(q, t, scoring, band=None):
    """H table (list of rows over t, columns over q) by exhaustive search.
    With band=w, only paths whose every cell (last consumed target base,
    last consumed query base) satisfies |i - j| <= w are counted."""
    a, b, o, e = scoring
    m, n = len(q), len(t)
    H = [[0] * m for _ in range(n)]
    sys.setrecursionlimit(10000)

    def dfs(i, j, last, score, used_t, used_q):
        # (i, j): next target / query base to consume
        if used_t and used_q:
            ti, qj = i - 1, j - 1
            if band is not None and abs(ti - qj) > band:
                return
            if score > H[ti][qj]:
                H[ti][qj] = score
        if i < n and j < m:
            dfs(i + 1, j + 1, "M", score + _s(t[i], q[j], a, b), True, True)
        if i < n:   # consume a target base against a gap
            dfs(i + 1, j, "D", score - (e if last == "D" else o + e), True, used_q)
        if j < m:   # consume a query base against a gap
            dfs(i, j + 1, "I", score - (e if last == "I" else o + e), used_t, True)

    for i0 in range(n):
        for j0 in range(m):
            dfs(i0, j0, "", 0, False, False)
    return H


def kadane_table(q, t, scoring):
    """Ungapped: best sum of a run of S along the diagonal ending at (i, j)."""
    a, b = scoring[0], scoring[1]
    m, n = len(q), len(t)
    H = [[0] * m for _ in range(n)]
    for d in range(-(m - 1), n):          # diagonal i - j = d
        run = 0
        i, j = max(d, 0), max(-d, 0)
        while i < n and j < m:
            run = max(0, run + _s(t[i], q[j], a, b))
            H[i][j] = run
            i += 1
            j += 1
    return H


def linear_sw_table(q, t, match, mismatch, gap):
    """Textbook Smith-Waterman, linear gap penalty ``gap`` per base."""
    m, n = len(q), len(t)
    H = [[0] * m for _ in range(n)]
    for i in range(n):
        for j in range(m):
            diag = (H[i - 1][j - 1] if i and j else 0) + _s(t[i], q[j], match, mismatch)
            up = (H[i - 1][j] if i else 0) - gap
            left = (H[i][j - 1] if j else 0) - gap
            H[i][j] = max(0, diag, up, left)
    return H


def common_suffix_table(q, t):
    """Length of the longest common suffix of t[..i] and q[..j], by direct
    comparison backwards from (i, j)."""
    m, n = len(q), len(t)
    L = [[0] * m for _ in range(n)]
    for i in range(n):
        for j in range(m):
            k = 0
            while i - k >= 0 and j - k >= 0 and t[i - k] == q[j - k]:
                k += 1
            L[i][j] = k
    return L


def first_max(H):
    """(score, q_end, t_end) under the end-position convention."""
    best, bi, bj = 0, -1, -1
    for i, row in enumerate(H):
        for j, v in enumerate(row):
            if v > best:
                best, bi, bj = v, i, j
    return best, bj, bi


def enumerate_starts(q, t, scoring, q_end, t_end):
    """Every (t_start, q_start) of an alignment path whose first and last
    moves align a base pair, whose last aligned pair is (t_end, q_end), with
    the best score such paths reach; returns (best score, set of starts).
    Exhaustive search over paths (same move costs as enumerate_h)."""
    a, b, o, e = scoring
    m, n = len(q), len(t)
    best = [None]
    starts = set()
    sys.setrecursionlimit(10000)

    def dfs(i, j, last, score, i0, j0):
        # (i, j): next target / query base to consume
        if last == "M" and i - 1 == t_end and j - 1 == q_end:
            if best[0] is None or score > best[0]:
                best[0] = score
                starts.clear()
            if score == best[0]:
                starts.add((i0, j0))
        if i > t_end + 1 or j > q_end + 1:
            return
        if i < n and j < m:
            dfs(i + 1, j + 1, "M", score + _s(t[i], q[j], a, b), i0, j0)
        if i < n and last != "":
            dfs(i + 1, j, "D", score - (e if last == "D" else o + e), i0, j0)
        if j < m and last != "":
            dfs(i, j + 1, "I", score - (e if last == "I" else o + e), i0, j0)

    for i0 in range(t_end + 1):
        for j0 in range(q_end + 1):
            dfs(i0, j0, "", 0, i0, j0)
    return best[0], starts
