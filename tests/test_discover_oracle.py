"""Pins of the candidate-discovery oracle against facts that do not depend on
it: brute-force set intersection on tiny inputs, closed forms for periodic
and repeat-free sequences, the symmetry of the overlap product, and the two
pair filters of a self search (each unordered pair kept exactly once).  A
planted mistake in a copy of the oracle must fail at least one of them."""
import shutil

import numpy as np
import pytest

import oracle
from oracle import DiscoverLib

LETTERS = "ARNDCQEGHILKMFPSTWYV"


def pack(seqs):
    asc = np.frombuffer("".join(seqs).encode(), dtype=np.uint8).copy()
    offs = np.zeros(len(seqs) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(s) for s in seqs])
    return asc, offs


def codes(D, seqs):
    asc, offs = pack(seqs)
    return oracle.default().encode(asc.tobytes()) if len(asc) else np.zeros(0, np.int8), offs


def run(D, qs, rs, k, t, mode=0):
    qc, qo = codes(D, qs)
    rc, ro = codes(D, rs)
    q, r, c = D.discover_codes(qc, qo, rc, ro, k, t, mode)
    return {(int(a), int(b)): int(x) for a, b, x in zip(q, r, c)}, (q, r)


def brute(qs, rs, k, t, mode=0):
    """Per pair: the size of the intersection of the two k-mer sets."""
    def kset(s):
        return {s[p:p + k] for p in range(len(s) - k + 1)}
    out = {}
    for i, a in enumerate(qs):
        for j, b in enumerate(rs):
            if mode == 1 and not i < j:
                continue
            if mode == 2 and (i == j or (i > j and i % 2 != j % 2) or (i < j and i % 2 == j % 2)):
                continue
            c = len(kset(a) & kset(b))
            if c >= t and c > 0:
                out[(i, j)] = c
    return out


def rand_set(rng, n, alpha, lmax):
    return ["".join(rng.choice(list(alpha), size=int(rng.integers(0, lmax + 1)))) for _ in range(n)]


def check_brute(D):
    rng = np.random.default_rng(7)
    for alpha, lmax in (("AC", 12), ("ACD", 14), (LETTERS, 30), ("W", 9)):
        for k in (1, 2, 3, 6):
            for t in (1, 2, 3):
                qs = rand_set(rng, 6, alpha, lmax)
                rs = rand_set(rng, 5, alpha, lmax)
                got, (q, r) = run(D, qs, rs, k, t)
                if got != brute(qs, rs, k, t):
                    return "brute k=%d t=%d alpha=%s" % (k, t, alpha)
                if list(zip(q, r)) != sorted(zip(q, r)):
                    return "order"
                for mode in (1, 2):
                    got, _ = run(D, qs, qs, k, t, mode)
                    if got != brute(qs, qs, k, t, mode):
                        return "brute mode=%d k=%d t=%d" % (mode, k, t)
    return None


def check_closed_forms(D):
    # a repeat-free sequence of length L has L-k+1 distinct k-mers (0 if L < k)
    for L in range(0, 21):
        for k in (1, 3, 6):
            s = LETTERS[:L]
            got, _ = run(D, [s], [s], k, 1)
            exp = max(L - k + 1, 0)
            if got.get((0, 0), 0) != exp:
                return "repeat-free L=%d k=%d" % (L, k)
    # period p of distinct letters: min(p, L-k+1) distinct k-mers; two shifts
    # of one periodic string share all of them once both are long enough
    for p in (1, 2, 5, 7):
        for k in (1, 2, 6):
            unit = LETTERS[3:3 + p]
            a = (unit * 10)[:k + p + 4]
            b = (unit * 12)[2:2 + k + p + 1]
            got, _ = run(D, [a], [a, b], k, 1)
            if got.get((0, 0)) != p or got.get((0, 1)) != p:
                return "periodic p=%d k=%d" % (p, k)
    # a homopolymer shares one k-mer with itself whatever its length (>= k)
    got, _ = run(D, ["W" * 40], ["W" * 6, "W" * 5], 6, 1)
    if got != {(0, 0): 1}:
        return "homopolymer"
    return None


def check_symmetry(D):
    rng = np.random.default_rng(11)
    qs = rand_set(rng, 30, "ACDE", 40)
    rs = rand_set(rng, 25, "ACDE", 40)
    for k, t in ((3, 2), (4, 1), (6, 2)):
        a, _ = run(D, qs, rs, k, t)
        b, _ = run(D, rs, qs, k, t)
        if a != {(j, i): c for (i, j), c in b.items()}:
            return "symmetry k=%d" % k
    return None


def check_self_filters(D):
    rng = np.random.default_rng(5)
    s = rand_set(rng, 40, "ACD", 30)
    full, _ = run(D, s, s, 3, 2, 0)
    upper, _ = run(D, s, s, 3, 2, 1)
    parity, _ = run(D, s, s, 3, 2, 2)
    off = {p: c for p, c in full.items() if p[0] != p[1]}
    unordered = {tuple(sorted(p)) for p in off}
    for kept in (upper, parity):
        if any(p[0] == p[1] for p in kept):
            return "diagonal kept"
        if {tuple(sorted(p)) for p in kept} != unordered or len(kept) != len(unordered):
            return "filter does not keep each unordered pair once"
        if any(full[p] != c for p, c in kept.items()):
            return "filter changed a count"
    if any(i > j for i, j in upper):
        return "upper filter"
    return None


def battery(D):
    for f in (check_brute, check_closed_forms, check_symmetry, check_self_filters):
        bad = f(D)
        if bad:
            return bad
    return None


@pytest.fixture(scope="module")
def D():
    return oracle.discover_lib()


def test_brute_force_tiny(D):
    assert check_brute(D) is None


def test_closed_forms(D):
    assert check_closed_forms(D) is None


def test_symmetry(D):
    assert check_symmetry(D) is None


def test_self_filters(D):
    assert check_self_filters(D) is None


def test_distinct_counts_are_the_diagonal(D):
    rng = np.random.default_rng(3)
    s = rand_set(rng, 50, "ACDEF", 60)
    asc, offs = pack(s)
    dk = oracle.distinct_kmers(asc, offs, 4)
    full, _ = run(D, s, s, 4, 1)
    assert all(full.get((i, i), 0) == dk[i] for i in range(len(s)))
    assert all(c <= min(dk[i], dk[j]) for (i, j), c in full.items())


def test_empty_and_invalid(D):
    got, _ = run(D, [], ["ACDEFG"], 3, 1)
    assert got == {}
    got, _ = run(D, ["", "AC"], ["ACDEFG", ""], 3, 1)
    assert got == {}
    with pytest.raises(ValueError):
        oracle.discover(*pack(["ACDJ"]), *pack(["ACD"]), k=2, min_shared=1)


PLANTS = [
    # keep repeated k-mers of a sequence (rows of A are not sets)
    ("if (t == first || A->cols[t] != A->cols[u - 1]) A->cols[u++] = A->cols[t];",
     "A->cols[u++] = A->cols[t];"),
    # lose the last window of every sequence
    ("for (int64_t p = 0; p + k <= L; ++p) {", "for (int64_t p = 0; p + k < L; ++p) {"),
    # strict threshold
    ("if (acc[r] >= min_shared && keep_pair(q, r, mode)) {",
     "if (acc[r] > min_shared && keep_pair(q, r, mode)) {"),
    # parity rule below the diagonal inverted
    ("if (q > r) return (q & 1) == (r & 1);", "if (q > r) return (q & 1) != (r & 1);"),
    # triangle taken on the wrong side
    ("if (mode == 1) return q < r;", "if (mode == 1) return q > r;"),
    # k-mer code that forgets the first residue's position
    ("x = x * KMER_ALPHABET + c;", "x = x + c;"),
]


def test_pins_pass_on_the_real_oracle(D):
    assert battery(D) is None


@pytest.mark.parametrize("k", range(len(PLANTS)))
def test_pins_catch_planted_mistake(k, tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc missing")
    old, new = PLANTS[k]
    src = open(oracle.DISCOVER_SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / "planted.c"
    path.write_text(src.replace(old, new))
    lib = str(tmp_path / "libplanted.so")
    oracle.compile_oracle(str(path), lib)
    assert battery(DiscoverLib(lib)) is not None, "pins missed: %r -> %r" % (old, new)
