"""Write stored oracle values for the 40-photon repeated-row workload.

The 256 (S, T) pairs are bounded compositions (sum 40, at most 4 per mode, 20
modes) drawn by the seeded generator; the interferometer is the 20-mode Haar
unitary of seed 0.  At 40 photons the alternating Ryser sum cancels beyond
what an 80-bit mantissa holds, so the values are computed with the oracle's
quad-precision multiplicity formula, on the side with fewer digit vectors
(perm(A^T) = perm(A)).  Ten patterns are stored with the unitary itself:
the three with the fewest digit vectors, and seven more chosen to span the
cost range up to the most expensive of the 256 (6e8 digit vectors) in both
column classes (at most 16 and 17 to 20 distinct power modes).

usage: python tests/golden/make_golden_repeated.py [out_path]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle     # noqa: E402
import workloads  # noqa: E402

# pattern indices into repeated_patterns(256, seed=1): cheapest three, then
# quantiles of the cost for 13..16 and 17..20 distinct power modes
PATTERNS = [46, 78, 235, 107, 246, 61, 222, 156, 124, 242]


def main():
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(__file__), "repeated_permanents.txt")
    pats = workloads.repeated_patterns(count=256, seed=1)
    cost = [min(int(np.prod(S[S > 0] + 1)), int(np.prod(T[T > 0] + 1))) for S, T in pats]
    order = PATTERNS
    U = workloads.haar(20, 0)
    with open(out + ".tmp", "w") as f:
        f.write("# oracle (multiplicity Ryser, IEEE quad precision) permanents, 40 photons in 20 modes\n")
        f.write("# written by tests/golden/make_golden_repeated.py\n")
        f.write("unitary 20\n")
        for r in range(20):
            f.write(" ".join(f"{float(x.real)!r} {float(x.imag)!r}" for x in U[r]) + "\n")
        for idx in order:
            S, T = pats[idx]
            t = time.time()
            cs = int(np.prod(S[S > 0] + 1))
            ct = int(np.prod(T[T > 0] + 1))
            if ct < cs:
                _, parts = oracle.perm_mult_quad(np.ascontiguousarray(U.T), T, S)
            else:
                _, parts = oracle.perm_mult_quad(U, S, T)
            print(f"pattern {idx} cost {cost[idx]} {time.time() - t:.1f}s", flush=True)
            f.write(f"pattern {int(idx)}\n")
            f.write("S " + " ".join(str(int(v)) for v in S) + "\n")
            f.write("T " + " ".join(str(int(v)) for v in T) + "\n")
            f.write("perm " + " ".join(repr(float(v)) for v in parts) + "\n")
            f.flush()
    os.replace(out + ".tmp", out)


if __name__ == "__main__":
    main()
