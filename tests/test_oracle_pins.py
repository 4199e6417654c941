"""Pins for the CPU oracle (no GPU).  Each check comes from outside the oracle:
brute-force enumeration, closed forms, invariants and textbook special cases
(see tests/independent.py).  The last test plants plausible mistakes in copies
of the oracle's C source and requires the pins to catch every one of them."""
import os
import shutil
import tempfile

import numpy as np
import pytest

import oracle
from oracle import OracleLib
from tests import independent as I

GAPS = [(11, 1), (2, 1), (1, 0), (3, 3), (5, 2), (1, 1)]
STD20 = "ARNDCQEGHILKMFPSTWYV"


@pytest.fixture(scope="module")
def O():
    return oracle.default()


# ---------------------------------------------------------------- matrix table

def test_matrix_table_properties(O):
    B = O.scores.astype(int)
    L = O.letters
    assert L == "ARNDCQEGHILKMFPSTWYVBZX*"
    assert (B == B.T).all()
    assert B.min() == -4 and B.max() == 11
    diag = {"A": 4, "R": 5, "N": 6, "D": 6, "C": 9, "Q": 5, "E": 5, "G": 6, "H": 8, "I": 4,
            "L": 4, "K": 5, "M": 5, "F": 6, "P": 7, "S": 4, "T": 5, "W": 11, "Y": 7, "V": 4}
    for a, v in diag.items():
        assert B[L.index(a), L.index(a)] == v, a
    std = [L.index(a) for a in STD20]
    off = max(B[i, j] for i in std for j in std if i != j)
    assert off == 3 and off < min(B[i, i] for i in std)
    star = L.index("*")
    assert all(B[star, j] == -4 for j in range(23)) and B[star, star] == 1


def test_encoder_rejects_unknown_letters(O):
    assert list(O.encode(b"ARN*")) == [0, 1, 2, 23]
    for bad in (b"AJ", b"a", b"U", b"-"):
        with pytest.raises(ValueError):
            O.encode(bad)


# ---------------------------------------------------------------- brute force

def _tiny_cases(seed, count, max_len=6):
    rng = np.random.default_rng(seed)
    for t in range(count):
        m, n = (int(x) for x in rng.integers(1, max_len + 1, 2))
        k = int(rng.choice([1, 2, 3, 20, 24]))
        letters = rng.choice(24 if k == 24 else 20, k, replace=False)
        q = rng.choice(letters, m).astype(np.int8)
        r = rng.choice(letters, n).astype(np.int8)
        if t % 7 == 0:  # repeats
            r = np.concatenate([q, q])[:n].astype(np.int8)
        if t % 5 == 1:  # a gap of 2-3 residues between two strong matches
            hi = rng.choice([4, 17, 18], 2)          # C, W, Y
            ins = rng.integers(0, 20, int(rng.integers(2, 4))).astype(np.int8)
            q = np.array([hi[0], hi[1]], np.int8)
            r = np.concatenate([[hi[0]], ins, [hi[1]]]).astype(np.int8)
            if t % 2:
                q, r = r, q
        yield q, r, GAPS[t % len(GAPS)]


def test_brute_force_tiny(O):
    B = O.scores
    n = 0
    for q, r, (go, ge) in _tiny_cases(1, 600):
        assert O.align(q, r, go, ge) == I.brute_force(q, r, B, go, ge), (q, r, go, ge)
        n += 1
    assert n == 600


def test_brute_force_ties_single_letter(O):
    # one-letter sequences: every diagonal segment ties; the rule decides
    B = O.scores
    for a in range(24):
        for m in range(1, 6):
            for n in range(1, 6):
                q = np.full(m, a, np.int8)
                r = np.full(n, a, np.int8)
                for go, ge in GAPS[:3]:
                    assert O.align(q, r, go, ge) == I.brute_force(q, r, B, go, ge)


# ---------------------------------------------------------------- closed form

def test_self_alignment_closed_form(O):
    rng = np.random.default_rng(2)
    B = O.scores.astype(int)
    std = np.array([O.letters.index(a) for a in STD20], dtype=np.int8)
    for t in range(200):
        n = int(rng.integers(1, 400))
        s = rng.choice(std, n).astype(np.int8)
        for go, ge in [(11, 1), (2, 1), (5, 2)]:
            S = int(sum(B[c, c] for c in s))
            assert O.align(s, s, go, ge) == (S, 0, n - 1, 0, n - 1)
    s = O.encode(STD20)
    assert O.align(s, s)[0] == 116


# ---------------------------------------------------------------- symmetry

def _n_optimal(O, q, r, go, ge):
    """(number of cells with H = S, number of reversed-prefix cells with H' = S)."""
    S, qs, qe, rs, re = O.align(q, r, go, ge)
    if S == 0:
        return 0, 0
    ends = int((O.fill_H(q, r, go, ge) == S).sum())
    starts = int((O.fill_H(q[:qe + 1][::-1].copy(), r[:re + 1][::-1].copy(), go, ge) == S).sum())
    return ends, starts


def test_swap_symmetry(O):
    rng = np.random.default_rng(3)
    B = O.scores
    exact = 0
    for t in range(150):
        m, n = (int(x) for x in rng.integers(1, 60, 2))
        k = int(rng.choice([2, 4, 20]))
        letters = rng.choice(20, k, replace=False)
        q = rng.choice(letters, m).astype(np.int8)
        r = rng.choice(letters, n).astype(np.int8)
        if t % 3 == 0:
            r = q.copy()
            r[rng.integers(0, m, max(1, m // 4))] = rng.choice(letters)
        go, ge = GAPS[t % 3]
        a = O.align(q, r, go, ge)
        b = O.align(r, q, go, ge)
        assert a[0] == b[0]
        if a[0] == 0:
            assert a == b == I.NONE
            continue
        if _n_optimal(O, q, r, go, ge) == (1, 1) and _n_optimal(O, r, q, go, ge) == (1, 1):
            assert (a[1], a[2], a[3], a[4]) == (b[3], b[4], b[1], b[2])
            exact += 1
        # the swapped report must delimit an optimal alignment of (q, r)
        qs, qe, rs, re = b[3], b[4], b[1], b[2]
        assert I.anchored_affine_score(q[qs:qe + 1], r[rs:re + 1], B, go, ge) == a[0]
    assert exact > 20


# ---------------------------------------------------------------- special cases

def test_ungapped_special_case(O):
    rng = np.random.default_rng(4)
    for t in range(60):
        m, n = (int(x) for x in rng.integers(1, 50, 2))
        q = rng.integers(0, 24, m).astype(np.int8)
        r = rng.integers(0, 24, n).astype(np.int8)
        if t % 4 == 0:
            r = np.concatenate([q[::2], q])[:n].astype(np.int8)
        assert O.align(q, r, 10 ** 6, 10 ** 6) == I.ungapped(q, r, O.scores)


def test_linear_gap_special_case(O):
    rng = np.random.default_rng(5)
    for t in range(60):
        m, n = (int(x) for x in rng.integers(1, 45, 2))
        letters = rng.choice(20, int(rng.choice([3, 20])), replace=False)
        q = rng.choice(letters, m).astype(np.int8)
        r = rng.choice(letters, n).astype(np.int8)
        g = int(rng.integers(1, 8))
        assert O.align(q, r, g, g) == I.linear_gap(q, r, O.scores, g)


# ---------------------------------------------------------------- bounds

def test_bounds_and_monotonicity(O):
    rng = np.random.default_rng(6)
    B = O.scores.astype(int)
    for t in range(100):
        m, n = (int(x) for x in rng.integers(1, 120, 2))
        q = rng.integers(0, 20, m).astype(np.int8)
        r = rng.integers(0, 20, n).astype(np.int8)
        S = O.align(q, r)[0]
        assert max(0, B[np.ix_(q, r)].max()) <= S <= 11 * min(m, n)
        x = rng.integers(0, 20, int(rng.integers(1, 20))).astype(np.int8)
        assert O.align(np.concatenate([q, x]), r)[0] >= S
        assert O.align(q, np.concatenate([x, r]))[0] >= S


def test_empty_and_invalid(O):
    assert O.align(b"", b"ACD") == I.NONE
    assert O.align(b"ACD", b"") == I.NONE
    assert O.align(b"W", b"W") == (11, 0, 0, 0, 0)
    assert O.align(b"*", b"W") == I.NONE
    for go, ge in [(0, 0), (2, 3), (-1, 0), (1, -1)]:
        with pytest.raises(ValueError):
            O.align(b"AC", b"AC", go, ge)


def test_batch_matches_single(O):
    rng = np.random.default_rng(7)
    L = rng.integers(0, 80, 40)
    offs = np.concatenate([[0], np.cumsum(L)])
    codes = rng.integers(0, 24, int(offs[-1])).astype(np.int8)
    pairs = rng.integers(0, 40, (200, 2)).astype(np.int32)
    pairs[0] = [-1, 3]
    pairs[1] = [3, 40]
    out = O.batch(codes, offs, pairs, 11, 1, threads=4)
    assert tuple(out[0]) == (-1, -1, -1, -1, -1) and tuple(out[1]) == (-1, -1, -1, -1, -1)
    for k in range(2, 200):
        a, b = pairs[k]
        assert tuple(out[k]) == O.align(codes[offs[a]:offs[a + 1]], codes[offs[b]:offs[b + 1]])


# ---------------------------------------------------------------- golden regression

def test_golden_cases(O):
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_cases.tsv")
    n = 0
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            q, r, go, ge, *exp = line.rstrip("\n").split("\t")
            assert O.align(q.encode(), r.encode(), int(go), int(ge)) == tuple(int(x) for x in exp)
            n += 1
    assert n >= 50


# ---------------------------------------------------------------- planted mistakes

MUTATIONS = [
    ("e = imax(e - ge, left - go);", "e = imax(e - go, left - go);"),
    ("e = imax(e - ge, left - go);", "e = imax(e - ge, left - ge);"),
    ("int32_t f = imax(Frow[j] - ge, up - go);", "int32_t f = imax(Frow[j] - go, up - go);"),
    ("int32_t f = imax(Frow[j] - ge, up - go);", "int32_t f = imax(Frow[j] - ge, up - ge);"),
    ("            h = imax(h, f);\n", "            (void)f;\n"),
    ("            h = imax(h, e);\n", "            (void)e;\n"),
    ("            h = imax(h, 0);\n", "            (void)0;\n"),
    ("if (h > best) {", "if (h >= best && h > 0) {"),
    ("            diag = up;\n", "            diag = left;\n"),
    ("out->q_start = ie - a;", "out->q_start = ie - b;"),
    ("out->r_start = je - b;", "out->r_start = je - b + 1;"),
    ("out->q_end = ie;", "out->q_end = je;"),
    ("r + je, -1, je + 1, mx", "r + je, -1, je, mx"),
    ("q + ie, -1, ie + 1, r", "q + ie, -1, ie, r"),
    ("left = h;\n            if", "left = up;\n            if"),
]


def _battery(O):
    """A short run of the pins above; False as soon as one fails."""
    B = O.scores
    try:
        for q, r, (go, ge) in _tiny_cases(11, 120, max_len=5):
            if O.align(q, r, go, ge) != I.brute_force(q, r, B, go, ge):
                return False
        rng = np.random.default_rng(12)
        for t in range(15):
            m, n = (int(x) for x in rng.integers(1, 30, 2))
            q = rng.integers(0, 20, m).astype(np.int8)
            r = rng.integers(0, 20, n).astype(np.int8)
            if O.align(q, r, 10 ** 6, 10 ** 6) != I.ungapped(q, r, B):
                return False
            if O.align(q, q, 11, 1) != (int(sum(int(B[c, c]) for c in q)), 0, m - 1, 0, m - 1):
                return False
            if O.align(q, r)[0] != O.align(r, q)[0]:
                return False
        for t in range(20):  # homolog with a planted indel: reported box must be optimal
            m = int(rng.integers(6, 25))
            q = rng.integers(0, 20, m).astype(np.int8)
            cut = int(rng.integers(1, m))
            r = np.concatenate([q[:cut], rng.integers(0, 20, int(rng.integers(2, 6))), q[cut:]]).astype(np.int8)
            if t % 2:
                q, r = r, q
            go, ge = [(2, 1), (5, 2), (11, 1)][t % 3]
            S, qs, qe, rs, re = O.align(q, r, go, ge)
            if S < I.anchored_affine_score(q, r, B, go, ge):
                return False
            if S and I.anchored_affine_score(q[qs:qe + 1], r[rs:re + 1], B, go, ge) != S:
                return False
    except ValueError:
        return False
    return True


def test_pins_pass_on_the_real_oracle(O):
    assert _battery(O)


@pytest.mark.parametrize("k", range(len(MUTATIONS)))
def test_pins_catch_planted_mistake(k, tmp_path):
    old, new = MUTATIONS[k]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = str(tmp_path / "libmutant.so")
    oracle.compile_oracle(str(path), lib)
    assert not _battery(OracleLib(lib)), "pins missed: %r -> %r" % (old, new)
