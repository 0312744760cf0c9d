"""Write stored oracle values for sampled derivative entries at full size.

For the seed-0 block A of make_golden.py (single_n<n>_blocks.npy), the
derivative of perm(A) with respect to A_ij is the permanent of the minor with
row i and column j removed (every multiplicity is 1).  This calls only the
oracle (x87 extended-precision Ryser) on those (n-1) x (n-1) minors.

usage: python tests/golden/make_golden_minors.py [n ...]    (default: 30 32)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle     # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def entries(n: int):
    # corners, the middle and off-diagonal spreads of rows and columns
    return [(0, 0), (n // 4, 2 * n // 3), (n // 2, 3), (2 * n // 3, n - 1), (n - 1, n // 3), (n - 1, n - 1)]


def write_size(n: int, count: int) -> None:
    A = np.load(os.path.join(HERE, f"single_n{n}_blocks.npy"), allow_pickle=False)[0]
    out = os.path.join(HERE, f"minors_n{n}.txt")
    lines = [f"# oracle (Ryser, 80-bit long double) permanents of the minors of the seed-0 block\n",
             f"# of single_n{n}_blocks.npy: d perm / d A_ij = perm(A without row i and column j)\n",
             "# written by tests/golden/make_golden_minors.py\n"]
    for (i, j) in entries(n)[:count]:
        minor = np.delete(np.delete(A, i, axis=0), j, axis=1)
        t = time.time()
        re, im = oracle.perm_ryser_ld(minor)
        print(f"n={n} ({i},{j}) {time.time() - t:.1f}s on {oracle.num_threads()} threads", flush=True)
        lines.append(f"minor {n} 0 {i} {j} {float(re)!r} {float(im)!r}\n")
    with open(out + ".tmp", "w") as f:
        f.writelines(lines)
    os.replace(out + ".tmp", out)


def main():
    sizes = [int(a) for a in sys.argv[1:]] or [30, 32]
    for n in sizes:
        write_size(n, 6 if n <= 30 else 4)


if __name__ == "__main__":
    main()
