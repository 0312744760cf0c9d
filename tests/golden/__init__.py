"""Stored expected values.  Every file here is either a value printed in the
paper (with its citation) or the output of a committed script in this folder
that calls only the oracle."""
import numpy as np


def load_single(path):
    """Parse single_permanents.txt: blocks of
    ``case n seed``, ``perm re im``, then n rows of 2n numbers (re im ...)."""
    cases = []
    with open(path) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    i = 0
    while i < len(lines):
        head = lines[i].split()
        assert head[0] == "case"
        n, seed = int(head[1]), int(head[2])
        pr = lines[i + 1].split()
        assert pr[0] == "perm"
        perm = complex(float(pr[1]), float(pr[2]))
        rows = []
        for r in range(n):
            v = np.array([float(x) for x in lines[i + 2 + r].split()])
            rows.append(v[0::2] + 1j * v[1::2])
        cases.append({"n": n, "seed": seed, "perm": perm, "A": np.array(rows)})
        i += 2 + n
    return cases
