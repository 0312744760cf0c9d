"""Parity of the HIP forward sweep (through the C ABI) against the oracle."""
import math
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def tol_for(n):
    return 1e-10 if n <= 20 else 1e-8


@pytest.fixture(scope="module")
def eng():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_04006_amd as pq
    return pq.Engine(0)


def dev(U):
    return torch.from_numpy(np.ascontiguousarray(U, dtype=np.complex128)).cuda()


def run(eng, U, S, T):
    p, a = eng.perm(dev(U), list(S), list(T))
    torch.cuda.synchronize()
    return complex(p.item()), complex(a.item())


def test_single_n12_haar_block(eng):
    U = workloads.haar(24, 0)[:12, :12]
    ones = [1] * 12
    p, a = run(eng, U, ones, ones)
    ref = oracle.perm_ryser(U)
    print("n=12 rel err", rel(p, ref))
    assert rel(p, ref) < 1e-10
    assert a == p


@pytest.mark.parametrize("n", list(range(1, 21)))
def test_unit_multiplicity_sizes(eng, n):
    # spans lanes-only (n <= 7), partial lanes and several time digits
    U = workloads.gaussian_matrix(n, seed=1000 + n)
    ones = [1] * n
    p, _ = run(eng, U, ones, ones)
    ref = oracle.perm_ryser(U)
    assert rel(p, ref) < 1e-10, (n, p, ref)


@pytest.mark.parametrize("seed", range(16))
def test_repeated_rows_and_columns(eng, seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(2, 9))
    n = int(rng.integers(1, 13))
    U = workloads.haar(m, 50 + seed)
    S = workloads.random_occupations(rng, m, n, cap=5)
    T = workloads.random_occupations(rng, m, n, cap=5)
    p, a = run(eng, U, S, T)
    ref = oracle.perm_mult(U, S, T)
    if abs(ref) < 1e-13:
        assert abs(p) < 1e-12
    else:
        assert rel(p, ref) < 1e-10, (S, T, p, ref)
        assert rel(a, ref * oracle.normaliser(S, T)) < 1e-10


def test_fixed_row_with_multiplicity(eng):
    # every row repeated: the fixed group itself has radix mu_f > 1
    U = workloads.haar(5, 3)
    S = [2, 2, 2, 1, 3]
    T = [3, 2, 2, 2, 1]
    p, _ = run(eng, U, S, T)
    assert rel(p, oracle.perm_mult(U, S, T)) < 1e-10
    S = [2, 2, 2, 2, 2]
    T = [2, 2, 2, 2, 2]
    p, _ = run(eng, U, S, T)
    assert rel(p, oracle.perm_mult(U, S, T)) < 1e-10


def test_special_cases(eng):
    U = workloads.haar(4, 1)
    assert run(eng, U, [1, 0, 0, 0], [1, 1, 0, 0]) == (0j, 0j)
    assert run(eng, U, [0, 0, 0, 0], [0, 0, 0, 0]) == (1 + 0j, 1 + 0j)
    p, a = run(eng, U, [0, 0, 3, 0], [0, 3, 0, 0])
    assert rel(p, 6 * U[1, 2] ** 3) < 1e-14
    assert rel(a, U[1, 2] ** 3) < 1e-14
    # identity: perm(I_{S,S}) = prod s!
    p, a = run(eng, np.eye(4), [3, 0, 2, 1], [3, 0, 2, 1])
    assert p == 12 and abs(a - 1) < 1e-15


def test_identity_and_ones_matrices(eng):
    for n in (6, 13, 18):
        p, _ = run(eng, np.ones((n, n)), [1] * n, [1] * n)
        assert rel(p, math.factorial(n)) < 1e-12
        p, _ = run(eng, np.eye(n), [1] * n, [1] * n)
        assert rel(p, 1.0) < 1e-14


def test_completeness_four_photons_eight_modes(eng):
    U = workloads.haar(8, 1)
    S = [1, 1, 1, 1, 0, 0, 0, 0]
    total = 0.0
    outs = workloads.fock_outputs(8, 4, at_most=True)
    assert len(outs) == 495
    Ud = dev(U)
    for T in outs:
        _, a = eng.perm(Ud, S, list(T))
        total += abs(complex(a.item())) ** 2
    assert abs(total - 1.0) < 1e-12


def test_paper_example_circuit(eng):
    U = oracle.mesh_unitary([(np.pi / 3, 0.0), (np.pi / 4, 0.0), (np.pi / 5, 0.0), (np.pi / 6, 0.0)],
                            [(1, 2), (2, 3), (0, 1), (3, 4)], 5)
    S = [1, 2, 0, 2, 1]
    total = 0.0
    for T in workloads.fock_outputs(5, 6):
        _, a = run(eng, U, S, T)
        ref = oracle.amplitude(U, S, T)
        assert abs(a - ref) < 1e-13
        total += abs(a) ** 2
    assert abs(total - 1.0) < 1e-12


def test_determinism(eng):
    U = workloads.collision_free_block(20, 7)
    ones = [1] * 20
    a = run(eng, U, ones, ones)
    b = run(eng, U, ones, ones)
    assert a == b


def test_submatrix_of_large_unitary_via_ldu(eng):
    # U resident as the full m x m interferometer, occupations select the block
    n, m = 14, 2 * 14 * 14
    Ufull = workloads.haar(m, 4)
    S = [1] * n + [0] * (m - n)
    p, _ = run(eng, Ufull, S, S)
    assert rel(p, oracle.perm_ryser(Ufull[:n, :n])) < 1e-10
    # non-trivial row/column selections and orientation
    S = [0] * m
    T = [0] * m
    for j in (3, 17, 100, 391):
        S[j] = 2
    for i in (0, 5, 250, 391):
        T[i] = 2
    p, _ = run(eng, Ufull, S, T)
    assert rel(p, oracle.perm_mult(Ufull, S, T)) < 1e-10


@pytest.mark.parametrize("seed", [0, 1])
def test_collision_free_n24(eng, seed):
    U = workloads.collision_free_block(24, seed)
    p, _ = run(eng, U, [1] * 24, [1] * 24)
    ref = oracle.perm_ryser(U)
    print("n=24 rel err", rel(p, ref))
    assert rel(p, ref) < 1e-8


@pytest.mark.parametrize("n", [24, 28, 30, 32])
def test_golden_full_size_single(eng, n):
    # all 16 seeds of each headline size against the oracle's stored values
    from tests.golden import load_single_set
    cases = load_single_set(n)
    assert len(cases) == 16
    worst = 0.0
    for c in cases:
        p, _ = run(eng, c["A"], [1] * n, [1] * n)
        err = rel(p, c["perm"])
        worst = max(worst, err)
        assert err < 1e-8, (n, c["seed"], err)
    print(f"n={n}: 16 seeds, worst rel err {worst:.2e}")


def test_invariances_full_size(eng):
    # properties that hold at any size: row/column permutation and diagonal scaling
    n = 28
    A = workloads.collision_free_block(n, 5)
    ones = [1] * n
    p, _ = run(eng, A, ones, ones)
    rng = np.random.default_rng(11)
    pr, pc = rng.permutation(n), rng.permutation(n)
    q, _ = run(eng, A[pr][:, pc], ones, ones)
    assert rel(q, p) < 1e-11
    d = np.exp(1j * rng.uniform(0, 2 * np.pi, n)) * rng.uniform(0.5, 2.0, n)
    s, _ = run(eng, d[:, None] * A, ones, ones)
    assert rel(s, np.prod(d) * p) < 1e-11
