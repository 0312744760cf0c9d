"""Stored expected values.  Every file here is either a value printed in the
paper (with its citation) or the output of a committed script in this folder
that calls only the oracle."""
import numpy as np


def load_single_set(n):
    """Stored values for n x n collision-free blocks (make_golden.py): a list
    of {n, seed, perm, A}, the blocks read from single_n<n>_blocks.npy."""
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    txt = os.path.join(here, f"single_n{n}.txt")
    npy = os.path.join(here, f"single_n{n}_blocks.npy")
    blocks = np.load(npy, allow_pickle=False)
    cases = []
    with open(txt) as f:
        for ln in f:
            if not ln.strip() or ln.startswith("#"):
                continue
            head = ln.split()
            assert head[0] == "case" and int(head[1]) == n
            k = len(cases)
            cases.append({"n": n, "seed": int(head[2]), "perm": complex(float(head[3]), float(head[4])),
                          "A": blocks[k]})
    assert blocks.shape == (len(cases), n, n)
    return cases


SINGLE_SIZES = (24, 28, 30, 32)


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


def load_minors(n):
    """Stored permanents of minors of the seed-0 block (make_golden_minors.py):
    (A, [(i, j, value), ...]) with A from single_n<n>_blocks.npy."""
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    A = np.load(os.path.join(here, f"single_n{n}_blocks.npy"), allow_pickle=False)[0]
    out = []
    with open(os.path.join(here, f"minors_n{n}.txt")) as f:
        for ln in f:
            if not ln.strip() or ln.startswith("#"):
                continue
            head = ln.split()
            assert head[0] == "minor" and int(head[1]) == n and int(head[2]) == 0
            out.append((int(head[3]), int(head[4]), complex(float(head[5]), float(head[6]))))
    return A, out


MINOR_SIZES = (30, 32)
