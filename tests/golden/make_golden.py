"""Write stored oracle values for full-size single permanents.

Calls only the oracle (x87 extended-precision Ryser) on the seeded workload:
the leading n x n block of a Haar unitary on m = 2 n^2 modes, seeds 0..15.
The blocks themselves are stored beside the values (``single_n<n>_blocks.npy``,
complex128, shape (16, n, n)), so a check elsewhere does not depend on the
LAPACK build that produced the QR factorisation on another host.

usage: python tests/golden/make_golden.py [n ...]     (default: 24 28 30 32)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle     # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SEEDS = range(16)


def write_size(n: int) -> None:
    txt = os.path.join(HERE, f"single_n{n}.txt")
    npy = os.path.join(HERE, f"single_n{n}_blocks.npy")
    blocks = np.stack([workloads.collision_free_block(n, s) for s in SEEDS])
    lines = [f"# oracle (Ryser, 80-bit long double) permanents of the leading {n} x {n} block\n",
             f"# of haar({2 * n * n}, seed); blocks in single_n{n}_blocks.npy (same order)\n",
             "# written by tests/golden/make_golden.py\n"]
    for k, seed in enumerate(SEEDS):
        t = time.time()
        re, im = oracle.perm_ryser_ld(blocks[k])
        print(f"n={n} seed={seed} {time.time() - t:.1f}s on {oracle.num_threads()} threads", flush=True)
        lines.append(f"case {n} {seed} {float(re)!r} {float(im)!r}\n")
    with open(npy + ".tmp", "wb") as f:
        np.save(f, blocks, allow_pickle=False)
    with open(txt + ".tmp", "w") as f:
        f.writelines(lines)
    os.replace(npy + ".tmp", npy)
    os.replace(txt + ".tmp", txt)


def main():
    sizes = [int(a) for a in sys.argv[1:]] or [24, 28, 30, 32]
    for n in sizes:
        write_size(n)


if __name__ == "__main__":
    main()
