"""Writes oracle_cases.tsv: seeded adversarial pairs with the oracle's results.

Calls only the oracle package.  The stored values are a regression record of
the oracle (each case is also re-derived by the pins in test_oracle_pins.py
where an independent check applies) and fixtures for the GPU parity tests.
Columns: query, reference, gap_open, gap_extend, score, q_start, q_end,
r_start, r_end.
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import oracle  # noqa: E402

LET = "ARNDCQEGHILKMFPSTWYVBZX*"


def cases():
    rng = np.random.default_rng(20230303)
    out = []
    for t in range(80):
        kind = t % 8
        m, n = (int(x) for x in rng.integers(1, 40, 2))
        if kind == 0:      # single letter runs
            a = LET[int(rng.integers(0, 24))]
            q, r = a * m, a * n
        elif kind == 1:    # two-letter low complexity
            ab = rng.choice(list(LET[:20]), 2, replace=False)
            q = "".join(rng.choice(ab, m)); r = "".join(rng.choice(ab, n))
        elif kind == 2:    # tandem repeats
            u = "".join(rng.choice(list(LET[:20]), int(rng.integers(1, 5))))
            q = (u * 40)[:m]; r = (u * 40)[int(rng.integers(0, 3)):][:n]
        elif kind == 3:    # lengths 1-3
            q = "".join(rng.choice(list(LET), int(rng.integers(1, 4))))
            r = "".join(rng.choice(list(LET), int(rng.integers(1, 4))))
        elif kind == 4:    # rare symbols B Z X *
            q = "".join(rng.choice(list("BZX*AC"), m)); r = "".join(rng.choice(list("BZX*AC"), n))
        elif kind == 5:    # homolog with an indel
            q = "".join(rng.choice(list(LET[:20]), m))
            cut = int(rng.integers(0, m))
            r = q[:cut] + "".join(rng.choice(list(LET[:20]), int(rng.integers(1, 6)))) + q[cut:]
        elif kind == 6:    # self
            q = "".join(rng.choice(list(LET[:20]), m)); r = q
        else:              # random
            q = "".join(rng.choice(list(LET[:20]), m)); r = "".join(rng.choice(list(LET[:20]), n))
        go, ge = [(11, 1), (2, 1), (1, 0), (3, 3), (11, 2)][t % 5]
        out.append((q, r, go, ge))
    return out


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_cases.tsv")
    with open(path, "w") as f:
        f.write("# query\treference\tgap_open\tgap_extend\tscore\tq_start\tq_end\tr_start\tr_end\n")
        f.write("# written by make_golden.py from the CPU oracle\n")
        for q, r, go, ge in cases():
            res = oracle.align(q.encode(), r.encode(), go, ge)
            f.write("\t".join([q, r, str(go), str(ge)] + [str(x) for x in res]) + "\n")


if __name__ == "__main__":
    main()
