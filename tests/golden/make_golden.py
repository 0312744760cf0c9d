"""Write stored oracle values for full-size single permanents.

Calls only the oracle (x87 extended-precision Ryser) on the seeded workload:
the leading n x n block of a Haar unitary on m = 2 n^2 modes.  The block
itself is stored beside the value, so a check elsewhere does not depend on the
LAPACK build that produced the QR factorisation.

usage: python tests/golden/make_golden.py [out_path]
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle     # noqa: E402
import workloads  # noqa: E402

CASES = [(24, s) for s in range(4)] + [(28, 0), (28, 1), (30, 0), (30, 1), (32, 0)]


def main():
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(__file__), "single_permanents.txt")
    with open(out + ".tmp", "w") as f:
        f.write("# oracle (Ryser, 80-bit long double) permanents of collision-free blocks\n")
        f.write("# written by tests/golden/make_golden.py\n")
        for n, seed in CASES:
            A = workloads.collision_free_block(n, seed)
            t = time.time()
            re, im = oracle.perm_ryser_ld(A)
            print(f"n={n} seed={seed} {time.time() - t:.1f}s", flush=True)
            f.write(f"case {n} {seed}\n")
            f.write(f"perm {float(re)!r} {float(im)!r}\n")
            for r in range(n):
                f.write(" ".join(f"{float(x.real)!r} {float(x.imag)!r}" for x in A[r]) + "\n")
            f.flush()
    os.replace(out + ".tmp", out)


if __name__ == "__main__":
    main()
