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


def load_repeated(path):
    """Parse repeated_permanents.txt: the unitary block, then per pattern its
    index, S, T and the value as (re_hi, re_lo, im_hi, im_lo)."""
    with open(path) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    head = lines[0].split()
    assert head[0] == "unitary"
    m = int(head[1])
    rows = []
    for r in range(m):
        v = np.array([float(x) for x in lines[1 + r].split()])
        rows.append(v[0::2] + 1j * v[1::2])
    U = np.array(rows)
    cases = []
    i = 1 + m
    while i < len(lines):
        idx = int(lines[i].split()[1])
        S = np.array([int(x) for x in lines[i + 1].split()[1:]], dtype=np.int32)
        T = np.array([int(x) for x in lines[i + 2].split()[1:]], dtype=np.int32)
        q = [float(x) for x in lines[i + 3].split()[1:]]
        cases.append({"index": idx, "S": S, "T": T, "perm": complex(q[0] + q[1], q[2] + q[3])})
        i += 4
    return U, cases
