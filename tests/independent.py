"""Independent checks that pin the oracle to something other than itself.

None of these functions shares code or method with ``oracle/sw_oracle.c``:

* ``brute_force`` enumerates every alignment path explicitly (no dynamic
  programming) for tiny sequences;
* ``ungapped`` scores every diagonal segment from prefix sums (the no-gap
  special case, i.e. a maximum-subarray problem per diagonal);
* ``linear_gap`` is the textbook single-matrix Smith-Waterman for gap cost
  g per residue, with the start found by a backward global
  (Needleman-Wunsch-style) alignment anchored at the end;
* ``anchored_affine_score`` is a global Gotoh alignment that must begin and end
  with aligned residue pairs (used to check that reported coordinates delimit
  an optimal alignment).

The tie rule is the project's reading of a point the paper leaves open: end =
lexicographically smallest (query, reference) end among optimal alignments;
start = lexicographically largest start among optimal alignments with that end.
"""
from __future__ import annotations

import sys

import numpy as np

NONE = (0, -1, -1, -1, -1)


def _pick(records):
    """records: iterable of (score, (i_s, j_s), (i_e, j_e))."""
    records = list(records)
    S = max([r[0] for r in records] + [0])
    if S <= 0:
        return NONE
    end = min(r[2] for r in records if r[0] == S)
    start = max(r[1] for r in records if r[0] == S and r[2] == end)
    return (S, start[0], end[0], start[1], end[1])


def brute_force(q, r, B, go, ge):
    """Every local alignment as an explicit path: it starts and ends with an
    aligned pair; steps are M (both advance), D (query only), I (reference
    only); a gap run pays go for its first residue and ge for each further one;
    a D run may be followed directly by an I run and vice versa."""
    m, n = len(q), len(r)
    recs = []
    sys.setrecursionlimit(10000)

    def walk(i, j, score, kind, start):
        if kind == "M":
            recs.append((score, start, (i, j)))
        if i + 1 < m and j + 1 < n:
            walk(i + 1, j + 1, score + int(B[q[i + 1]][r[j + 1]]), "M", start)
        if i + 1 < m:
            walk(i + 1, j, score - (ge if kind == "D" else go), "D", start)
        if j + 1 < n:
            walk(i, j + 1, score - (ge if kind == "I" else go), "I", start)

    for i0 in range(m):
        for j0 in range(n):
            walk(i0, j0, int(B[q[i0]][r[j0]]), "M", (i0, j0))
    return _pick(recs)


def ungapped(q, r, B):
    """Best diagonal segment (gaps forbidden).  Prefix sums per diagonal; for
    each end cell, the best segment is the prefix sum minus the minimum earlier
    prefix (ties resolved by the same rule as everywhere)."""
    m, n = len(q), len(r)
    recs = []
    for d in range(-(m - 1), n):
        cells = [(i, i + d) for i in range(max(0, -d), min(m, n - d))]
        vals = [int(B[q[i]][r[j]]) for i, j in cells]
        pref = np.concatenate([[0], np.cumsum(vals)]) if vals else np.zeros(1)
        for e in range(len(cells)):
            for s in range(e + 1):
                recs.append((int(pref[e + 1] - pref[s]), cells[s], cells[e]))
    return _pick(recs)


def linear_gap(q, r, B, g):
    """Textbook single-matrix SW with linear gaps (cost g per gap residue)."""
    m, n = len(q), len(r)
    H = np.zeros((m + 1, n + 1), dtype=np.int64)
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            H[i, j] = max(0, H[i - 1, j - 1] + int(B[q[i - 1]][r[j - 1]]),
                          H[i - 1, j] - g, H[i, j - 1] - g)
    S = int(H.max())
    if S == 0:
        return NONE
    ie, je = [(i - 1, j - 1) for i in range(1, m + 1) for j in range(1, n + 1) if H[i, j] == S][0]
    # V[i][j]: best global alignment of q[i..ie] x r[j..je] whose last column
    # is the aligned pair (ie, je); G = alignments that also begin with (i, j).
    NEG = -(1 << 40)
    V = np.full((ie + 2, je + 2), NEG, dtype=np.int64)
    best_start = None
    for i in range(ie, -1, -1):
        for j in range(je, -1, -1):
            if i == ie and j == je:
                V[i, j] = int(B[q[i]][r[j]])
                G = V[i, j]
            else:
                diag = V[i + 1, j + 1]
                G = int(B[q[i]][r[j]]) + diag if diag > NEG // 2 else NEG
                V[i, j] = max(G, V[i + 1, j] - g, V[i, j + 1] - g)
            if G == S and (best_start is None or (i, j) > best_start):
                best_start = (i, j)
    return (S, best_start[0], ie, best_start[1], je)


def anchored_affine_score(q, r, B, go, ge):
    """Best global Gotoh alignment of q and r that begins with the aligned pair
    (0, 0) and ends with the aligned pair (m-1, n-1)."""
    m, n = len(q), len(r)
    NEG = -(1 << 40)
    M = np.full((m, n), NEG, dtype=np.int64)   # ends with aligned pair (i, j)
    X = np.full((m, n), NEG, dtype=np.int64)   # ends with query residue i in a gap
    Y = np.full((m, n), NEG, dtype=np.int64)   # ends with reference residue j in a gap
    for i in range(m):
        for j in range(n):
            s = int(B[q[i]][r[j]])
            if i == 0 and j == 0:
                M[i, j] = s
            elif i > 0 and j > 0:
                M[i, j] = s + max(M[i - 1, j - 1], X[i - 1, j - 1], Y[i - 1, j - 1])
            if i > 0:
                X[i, j] = max(M[i - 1, j] - go, X[i - 1, j] - ge, Y[i - 1, j] - go)
            if j > 0:
                Y[i, j] = max(M[i, j - 1] - go, Y[i, j - 1] - ge, X[i, j - 1] - go)
    return int(M[m - 1, n - 1])
