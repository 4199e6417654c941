"""Pins of the identity / coverage oracle against facts that do not depend on
it: exhaustive enumeration of every global alignment on tiny inputs, the
closed forms of self-alignment and of the gapless case, agreement with the
Smith-Waterman oracle's score on the box it reports, and the integer keep
rule.  A planted mistake in a copy of the oracle must fail one of them."""
import shutil

import numpy as np
import pytest

import oracle
from oracle import IdentityLib


def enumerate_alignments(n_q, n_r):
    """Every global alignment as a list of moves: 'M' (a pair), 'D' (a query
    residue against a gap), 'I' (a reference residue against a gap)."""
    out = []

    def rec(i, j, path):
        if i == n_q and j == n_r:
            out.append(list(path))
            return
        if i < n_q and j < n_r:
            path.append("M"); rec(i + 1, j + 1, path); path.pop()
        if i < n_q:
            path.append("D"); rec(i + 1, j, path); path.pop()
        if j < n_r:
            path.append("I"); rec(i, j + 1, path); path.pop()
    rec(0, 0, [])
    return out


def brute_box(q, r, B, go, ge):
    best = None
    for path in enumerate_alignments(len(q), len(r)):
        i = j = 0
        s = m = 0
        prev = None
        for mv in path:
            if mv == "M":
                s += int(B[q[i], r[j]])
                m += int(q[i] == r[j])
                i += 1
                j += 1
            else:
                s -= ge if mv == prev else go
                if mv == "D":
                    i += 1
                else:
                    j += 1
            prev = mv
        key = (s, m, -len(path))
        if best is None or key > best:
            best = key
    return best[0], best[1], -best[2]


@pytest.fixture(scope="module")
def B():
    return oracle.default().scores


def battery(I, B):
    rng = np.random.default_rng(17)
    for t in range(160):
        alpha = [2, 3, 20][t % 3]
        m, n = (int(x) for x in rng.integers(1, 6, 2))
        q = rng.integers(0, alpha, m).astype(np.int8)
        r = rng.integers(0, alpha, n).astype(np.int8)
        go, ge = [(11, 1), (2, 1), (1, 0), (3, 3), (5, 2)][t % 5]
        if I.box(q, r, B, go, ge) != brute_box(q, r, B, go, ge):
            return "brute m=%d n=%d go=%d ge=%d" % (m, n, go, ge)
    for t in range(30):
        L = int(rng.integers(1, 60))
        s = rng.integers(0, 20, L).astype(np.int8)
        if I.box(s, s, B) != (int(sum(int(B[c, c]) for c in s)), L, L):
            return "self"
        r = rng.integers(0, 20, L).astype(np.int8)
        big = 10 ** 6
        exp = (int(sum(int(B[a, b]) for a, b in zip(s, r))), int((s == r).sum()), L)
        if I.box(s, r, B, big, big) != exp:
            return "gapless"
    O = oracle.default()
    for t in range(40):  # the SW box of a homolog pair scores S globally
        m = int(rng.integers(8, 40))
        q = rng.integers(0, 20, m).astype(np.int8)
        cut = int(rng.integers(1, m))
        r = np.concatenate([rng.integers(0, 20, 3), q[:cut], rng.integers(0, 20, int(rng.integers(1, 5))),
                            q[cut:], rng.integers(0, 20, 2)]).astype(np.int8)
        go, ge = [(11, 1), (4, 1), (6, 2)][t % 3]
        S, qs, qe, rs, re = O.align(q, r, go, ge)
        if S == 0:
            continue
        s, mt, c = I.box(q[qs:qe + 1], r[rs:re + 1], B, go, ge)
        if s != S or not (max(qe - qs + 1, re - rs + 1) <= c <= (qe - qs + 1) + (re - rs + 1)) or mt > c:
            return "box score"
    # keep rule, integer thresholds, both coverages
    codes = np.array([0, 1, 2, 3, 4, 5, 0, 1, 2, 3, 9, 9, 9, 9, 9], dtype=np.int8)
    offs = np.array([0, 6, 10, 15], dtype=np.int64)
    pairs = np.array([[0, 1], [1, 0], [0, 2]], dtype=np.int32)
    aligned = np.array([[21, 0, 3, 0, 3], [21, 0, 3, 0, 3], [0, -1, -1, -1, -1]], dtype=np.int32)
    rec = I.batch(codes, offs, pairs, aligned, B, 11, 1, 300, 700)
    # box 4x4 identical: 4 matches in 4 columns; coverage 4/6 of seq 0 < 0.7, 4/4 of seq 1
    S = int(sum(int(B[c, c]) for c in range(4)))
    if rec[0].tolist() != [S, 4, 4, 0] or rec[1].tolist() != [S, 4, 4, 0] or rec[2].tolist() != [0, 0, 0, 0]:
        return "keep rule %r" % rec.tolist()
    rec = I.batch(codes, offs, pairs[:1], aligned[:1], B, 11, 1, 300, 666)
    if rec[0, 3] != 1:
        return "keep at the threshold"
    rec = I.batch(codes, offs, pairs[:1], aligned[:1], B, 11, 1, 1000, 600)
    if rec[0, 3] != 1:
        return "identity 1.0 kept at 1000"
    return None


@pytest.fixture(scope="module")
def I():
    return oracle.identity_lib()


def test_battery_passes(I, B):
    assert battery(I, B) is None


def test_brute_force_counts():
    # Delannoy numbers: the enumerator visits every alignment
    assert [len(enumerate_alignments(k, k)) for k in range(1, 5)] == [3, 13, 63, 321]


PLANTS = [
    # a mismatch counted as a match
    ("triple d = add(Hp[j], scores[24 * a + b], a == b ? 1 : 0, 1);",
     "triple d = add(Hp[j], scores[24 * a + b], 1, 1);"),
    # fewer matches preferred
    ("if (a.m != b.m) return a.m > b.m;", "if (a.m != b.m) return a.m < b.m;"),
    # more columns preferred
    ("return a.c < b.c;", "return a.c > b.c;"),
    # gap extension without a column
    ("E = best2(add(E, -(int64_t)ge, 0, 1), add(Hc[j], -(int64_t)go, 0, 1));",
     "E = best2(add(E, -(int64_t)ge, 0, 0), add(Hc[j], -(int64_t)go, 0, 1));"),
    # vertical gap opened at the extension cost
    ("add(Hp[j + 1], -(int64_t)go, 0, 1));", "add(Hp[j + 1], -(int64_t)ge, 0, 1));"),
    # coverage of the reference measured against the query length
    ("(1000 * (int64_t)(a[4] - a[3] + 1) >= (int64_t)cov_permille * n);",
     "(1000 * (int64_t)(a[4] - a[3] + 1) >= (int64_t)cov_permille * m);"),
]


@pytest.mark.parametrize("k", range(len(PLANTS)))
def test_pins_catch_planted_mistake(k, tmp_path, B):
    if not shutil.which("gcc"):
        pytest.skip("gcc missing")
    old, new = PLANTS[k]
    src = open(oracle.IDENTITY_SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / "planted.c"
    path.write_text(src.replace(old, new))
    lib = str(tmp_path / "libplanted.so")
    oracle.compile_oracle(str(path), lib)
    assert battery(IdentityLib(lib), B) is not None, "pins missed: %r -> %r" % (old, new)
