"""Pins for the oracle: values and identities fixed by the paper and by the
mathematics, chosen so that a dropped term, a wrong sign or index, or a
transposed operand in any oracle routine fails at least one of them."""
import itertools as it
import math
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def subfactorial(n):
    # !n = n! sum_{k=0}^n (-1)^k / k!  (exact, integer recurrence)
    d = [1, 0]
    for k in range(2, n + 1):
        d.append((k - 1) * (d[-1] + d[-2]))
    return d[n]


# --------------------------------------------------------------- definition
@pytest.mark.parametrize("n", range(0, 9))
def test_bruteforce_identity_and_ones(n):
    assert oracle.perm_bruteforce(np.eye(n)) == 1.0
    assert oracle.perm_bruteforce(np.ones((n, n))) == math.factorial(n)
    assert oracle.perm_bruteforce(np.ones((n, n)) - np.eye(n)) == subfactorial(n)


def test_bruteforce_small_closed_forms():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    (p, q), (r, s) = a[0, :2], a[1, :2]
    assert rel(oracle.perm_bruteforce(a[:2, :2]), p * s + q * r) < 1e-15
    # 3x3: expansion along the first row with 2x2 permanent minors
    e = (a[0, 0] * (a[1, 1] * a[2, 2] + a[1, 2] * a[2, 1])
         + a[0, 1] * (a[1, 0] * a[2, 2] + a[1, 2] * a[2, 0])
         + a[0, 2] * (a[1, 0] * a[2, 1] + a[1, 1] * a[2, 0]))
    assert rel(oracle.perm_bruteforce(a), e) < 1e-15
    # a permanent is not a determinant: the signed version differs
    assert abs(oracle.perm_bruteforce(a) - np.linalg.det(a)) > 1e-3


# ------------------------------------------------------------------- Ryser
@pytest.mark.parametrize("n", range(1, 9))
def test_ryser_matches_definition(n):
    a = workloads.gaussian_matrix(n, seed=100 + n)
    assert rel(oracle.perm_ryser(a), oracle.perm_bruteforce(a)) < 1e-14


@pytest.mark.parametrize("n", range(1, 21))
def test_ryser_integer_matrices(n):
    pj = oracle.perm_ryser(np.ones((n, n)))
    pd = oracle.perm_ryser(np.ones((n, n)) - np.eye(n))
    if n <= 12:   # every partial sum is an integer below 2^64: exact
        assert pj == math.factorial(n)
        assert pd == subfactorial(n)
    else:
        # Ryser cancels terms up to k^n (|X| = k) down to n!: rounding error is
        # bounded by (n + 2) eps_ld sum_k C(n,k) k^n, with eps_ld = 2^-64
        bound = (n + 2) * 2.0 ** -64 * float(sum(math.comb(n, k) * k ** n for k in range(n + 1)))
        assert abs(pj - math.factorial(n)) <= bound
        assert abs(pd - subfactorial(n)) <= bound
        assert bound / math.factorial(n) < 1e-7      # the bound itself is tight enough to pin
    assert oracle.perm_ryser(np.eye(n)) == 1.0


@pytest.mark.parametrize("n", [12, 15])
def test_ryser_invariances(n):
    rng = np.random.default_rng(n)
    a = workloads.gaussian_matrix(n, seed=n)
    p = oracle.perm_ryser(a)
    pr, pc = rng.permutation(n), rng.permutation(n)
    assert rel(oracle.perm_ryser(a[pr][:, pc]), p) < 1e-13
    assert rel(oracle.perm_ryser(a.T), p) < 1e-13
    dr = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    dc = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    scaled = dr[:, None] * a * dc[None, :]
    assert rel(oracle.perm_ryser(scaled), np.prod(dr) * np.prod(dc) * p) < 1e-12


def test_ryser_laplace_expansion():
    n = 13
    a = workloads.gaussian_matrix(n, seed=7)
    full = oracle.perm_ryser(a)
    lap = 0j
    for j in range(n):
        minor = np.delete(np.delete(a, 0, axis=0), j, axis=1)
        lap += a[0, j] * oracle.perm_ryser(minor)
    assert rel(lap, full) < 1e-13


def test_ryser_haar_block_rows_are_not_swapped():
    # a non-symmetric block: using a row where a column belongs would change
    # the value (the check is only that the value equals the brute force)
    u = workloads.collision_free_block(7, seed=3)
    assert rel(oracle.perm_ryser(u), oracle.perm_bruteforce(u)) < 1e-13


# ------------------------------------------------------ repeated rows/cols
def _random_pattern(rng, m, n):
    S = workloads.random_occupations(rng, m, n)
    T = workloads.random_occupations(rng, m, n)
    return S, T


@pytest.mark.parametrize("seed", range(12))
def test_mult_matches_expanded_definition(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(2, 6))
    n = int(rng.integers(0, 8))
    U = workloads.haar(m, seed)
    S, T = _random_pattern(rng, m, n)
    ref = oracle.perm_bruteforce(oracle.expand(U, S, T))
    assert rel(oracle.perm_mult(U, S, T), ref) < 1e-13 or abs(ref) < 1e-14


def test_mult_transpose_symmetry():
    rng = np.random.default_rng(5)
    U = workloads.haar(6, 5)
    for _ in range(10):
        S, T = _random_pattern(rng, 6, 7)
        a = oracle.perm_mult(U, S, T)
        b = oracle.perm_mult(np.ascontiguousarray(U.T), T, S)
        assert rel(a, b) < 1e-13


def test_mult_identity_gives_factorials():
    for S in ([3, 0, 2, 1], [1, 1, 1, 1], [4, 0, 0, 0], [0, 2, 2, 0]):
        S = np.array(S, dtype=np.int32)
        want = float(np.prod([math.factorial(s) for s in S]))
        assert oracle.perm_mult(np.eye(4), S, S) == want
    # different supports on the identity: zero
    assert oracle.perm_mult(np.eye(3), [1, 1, 0], [0, 1, 1]) == 0


def test_mult_equals_binary_ryser_for_unit_multiplicities():
    U = workloads.haar(14, 2)
    S = np.ones(14, dtype=np.int32)
    assert rel(oracle.perm_mult(U, S, S), oracle.perm_ryser(U)) < 1e-13


def test_mult_special_cases():
    U = workloads.haar(4, 0)
    assert oracle.perm_mult(U, [1, 0, 0, 0], [1, 1, 0, 0]) == 0          # photon number differs
    assert oracle.perm_mult(U, [0, 0, 0, 0], [0, 0, 0, 0]) == 1          # vacuum
    assert oracle.perm_mult(U, [0, 0, 2, 0], [0, 2, 0, 0]) == pytest.approx(2 * U[1, 2] ** 2, rel=1e-15)


# ------------------------------------------------- two-mode beamsplitter
@pytest.mark.parametrize("theta,phi", [(0.3, 0.0), (np.pi / 5, 1.1), (2.2, -0.7)])
def test_two_mode_expansion(theta, phi):
    B = oracle.beamsplitter(theta, phi)
    assert np.allclose(B @ B.conj().T, np.eye(2), atol=1e-15)
    for n in range(4):
        for m in range(4):
            for p in range(n + m + 1):
                q = n + m - p
                want = oracle.two_mode_amplitude(theta, phi, n, m, p, q)
                got = oracle.amplitude(B, [n, m], [p, q])
                assert abs(got - want) < 1e-13, (n, m, p, q)


def test_hong_ou_mandel_dip():
    B = oracle.beamsplitter(np.pi / 4, 0.0)
    assert abs(oracle.amplitude(B, [1, 1], [1, 1])) < 1e-15
    assert oracle.probability(B, [1, 1], [2, 0]) == pytest.approx(0.5, abs=1e-15)


# ---------------------------------------------------------- completeness
def test_completeness_four_photons_eight_modes():
    U = workloads.haar(8, 1)
    S = np.array([1, 1, 1, 1, 0, 0, 0, 0], dtype=np.int32)
    outs = workloads.fock_outputs(8, 4, at_most=True)
    assert len(outs) == 495
    probs = np.array([oracle.probability(U, S, T) for T in outs])
    nonzero = [T for T in outs if T.sum() == 4]
    assert len(nonzero) == 330
    assert np.all(probs[[T.sum() < 4 for T in outs]] == 0)
    assert abs(probs.sum() - 1.0) < 1e-13


def _paper_circuit(phi=0.0):
    # Boson Sampling example: input (1,2,0,2,1) through beamsplitters
    # theta = pi/3 on (1,2), pi/4 on (2,3), pi/5 on (0,1), pi/6 on (3,4)
    return oracle.mesh_unitary([(np.pi / 3, phi), (np.pi / 4, phi), (np.pi / 5, phi), (np.pi / 6, phi)],
                               [(1, 2), (2, 3), (0, 1), (3, 4)], 5)


@pytest.mark.parametrize("phi", [0.0, np.pi / 4])
def test_paper_sampling_example(phi):
    U = _paper_circuit(phi)
    S = np.array([1, 2, 0, 2, 1], dtype=np.int32)
    outs = workloads.fock_outputs(5, 6)
    assert len(outs) == 210
    probs = {tuple(T): oracle.probability(U, S, T) for T in outs}
    assert abs(sum(probs.values()) - 1.0) < 1e-13
    # the printed samples must be possible outcomes
    for sample in [(0, 1, 2, 1, 2), (2, 0, 3, 0, 1)]:
        assert probs[sample] > 1e-6
    # a photon entering mode 4 meets only the (3,4) cell, so it leaves in
    # mode 3 or 4: all six photons in mode 0 is impossible
    assert probs[(6, 0, 0, 0, 0)] < 1e-30


# -------------------------------------------------------------- gradients
def test_gradient_finite_differences():
    rng = np.random.default_rng(3)
    U = workloads.haar(5, 3)
    S = np.array([2, 1, 0, 1, 1], dtype=np.int32)
    T = np.array([1, 0, 3, 1, 0], dtype=np.int32)
    g = oracle.perm_grad(U, S, T)
    h = 1e-6
    for (i, j) in [(0, 0), (2, 1), (3, 4), (2, 3), (1, 1)]:
        E = np.zeros_like(U)
        E[i, j] = h
        fd = (oracle.perm_mult(U + E, S, T) - oracle.perm_mult(U - E, S, T)) / (2 * h)
        assert abs(fd - g[i, j]) < 1e-8, (i, j)
        # holomorphic: an imaginary step gives i times the same derivative
        fdi = (oracle.perm_mult(U + 1j * E, S, T) - oracle.perm_mult(U - 1j * E, S, T)) / (2 * h)
        assert abs(fdi - 1j * g[i, j]) < 1e-8


def test_gradient_euler_identities():
    U = workloads.haar(6, 4)
    S = np.array([1, 2, 0, 1, 0, 2], dtype=np.int32)
    T = np.array([0, 1, 3, 0, 2, 0], dtype=np.int32)
    g = oracle.perm_grad(U, S, T)
    p = oracle.perm_mult(U, S, T)
    for i in range(6):
        assert abs(np.sum(U[i, :] * g[i, :]) - T[i] * p) < 1e-13
    for j in range(6):
        assert abs(np.sum(U[:, j] * g[:, j]) - S[j] * p) < 1e-13


def test_gradient_unit_multiplicity_is_minor():
    A = workloads.gaussian_matrix(6, seed=9)
    ones = np.ones(6, dtype=np.int32)
    g = oracle.perm_grad(A, ones, ones)
    for i, j in [(0, 0), (2, 5), (5, 1)]:
        minor = np.delete(np.delete(A, i, axis=0), j, axis=1)
        assert abs(g[i, j] - oracle.perm_bruteforce(minor)) < 1e-13


# -------------------------------------------------------- chain-rule rows
def test_extend_row_is_laplace_expansion():
    U = workloads.haar(9, 6)
    rows = [3, 3, 7]
    cols = [2, 0, 5, 1]
    out = oracle.extend_row(U, rows, cols)
    S = np.zeros(9, dtype=np.int32)
    S[cols] = 1
    for l in range(9):
        T = np.bincount(rows + [l], minlength=9).astype(np.int32)
        assert abs(out[l] - oracle.perm_mult(U, S, T)) < 1e-14


def test_chain_rule_marginals_sum_to_one():
    # sum over the next mode of the chain-rule weights, normalised by
    # (k-1)!-free counting, reproduces the marginal: for k = 1 the weights are
    # |U[l, c0]|^2 and sum to 1 for a unitary
    U = workloads.haar(6, 8)
    w = oracle.chain_rule_distribution(U, [4, 1, 2], [])
    assert abs(w.sum() - 1.0) < 1e-14


# ------------------------------------------------------------------ mesh
def test_mesh_is_unitary_and_cells_compose():
    ang = workloads.mesh_angles(0)
    U = oracle.mesh_unitary(ang, workloads.MESH_CELLS, workloads.MESH_MODES)
    assert len(workloads.MESH_CELLS) == 66 and ang.shape == (66, 2)
    assert np.allclose(U @ U.conj().T, np.eye(12), atol=1e-13)
    one = oracle.mesh_unitary([(0.4, 1.3)], [(0, 1)], 2)
    assert np.allclose(one, oracle.beamsplitter(0.4, 1.3))


@pytest.mark.parametrize("n", [24, 28, 30, 32])
def test_golden_values_present_and_pinned(n):
    """Stored oracle values for the full-size single permanents (16 seeds per
    size) were written by tests/golden/make_golden.py, which calls only the
    oracle.  Check that every stored block is the workload's (the leading
    n x n block of haar(2 n^2, seed), to rounding of the QR on this host), and
    that each value has the scale |perm| ~ sqrt(n!) m^(-n/2) of such blocks
    within a few orders of magnitude."""
    from tests.golden import load_single_set
    cases = load_single_set(n)
    assert [c["seed"] for c in cases] == list(range(16))
    m = 2 * n * n
    scale = math.sqrt(math.factorial(n)) * m ** (-n / 2)
    for c in cases:
        assert 1e-4 < abs(c["perm"]) / scale < 1e4
    for c in cases[:2]:
        A = workloads.collision_free_block(n, c["seed"])
        assert np.max(np.abs(A - c["A"])) < 1e-12


def test_golden_value_recomputes_at_n24():
    # the stored n = 24 values are the oracle's, not a later edit
    from tests.golden import load_single_set
    for c in load_single_set(24)[:3]:
        re, im = oracle.perm_ryser_ld(c["A"])
        assert complex(float(re), float(im)) == c["perm"]


def test_mesh_jacobian_matches_finite_differences():
    cells = [(0, 1), (1, 2), (0, 1), (2, 3), (1, 2)]
    rng = np.random.default_rng(4)
    ang = rng.uniform(0, 2 * np.pi, size=(len(cells), 2))
    J = oracle.mesh_jacobian(ang, cells, 4)
    h = 1e-6
    for q in range(len(cells)):
        for k in range(2):
            a1 = ang.copy(); a1[q, k] += h
            a0 = ang.copy(); a0[q, k] -= h
            fd = (oracle.mesh_unitary(a1, cells, 4) - oracle.mesh_unitary(a0, cells, 4)) / (2 * h)
            assert np.max(np.abs(fd - J[q, k])) < 1e-8


def test_mesh_loss_gradient_matches_finite_differences():
    cells = [(0, 1), (1, 2), (2, 3), (0, 1), (1, 2)]
    rng = np.random.default_rng(5)
    ang = rng.uniform(0, 2 * np.pi, size=(len(cells), 2))
    S = np.array([1, 1, 0, 0], np.int32)
    pats = [np.array(t, np.int32) for t in ([1, 0, 1, 0], [0, 1, 0, 1], [1, 1, 0, 0], [0, 0, 1, 1])]
    g = oracle.mesh_loss_grad(ang, cells, 4, S, pats)
    h = 1e-6

    def L(a):
        return oracle.mesh_loss(oracle.mesh_unitary(a, cells, 4), S, pats)
    for q in range(len(cells)):
        for k in range(2):
            a1 = ang.copy(); a1[q, k] += h
            a0 = ang.copy(); a0[q, k] -= h
            assert abs((L(a1) - L(a0)) / (2 * h) - g[q, k]) < 1e-6 * max(1.0, abs(g[q, k]))


def test_quad_precision_multiplicity_formula():
    rng = np.random.default_rng(21)
    for _ in range(6):
        U = workloads.haar(5, int(rng.integers(0, 1000)))
        S = workloads.random_occupations(rng, 5, 6, cap=3)
        T = workloads.random_occupations(rng, 5, 6, cap=3)
        q, _ = oracle.perm_mult_quad(U, S, T)
        ref = oracle.perm_bruteforce(oracle.expand(U, S, T))
        assert abs(q - ref) <= 1e-14 * max(1.0, abs(ref))
    # integer pins: perm(J_n) = n! and the identity with repeats
    n = 14
    q, parts = oracle.perm_mult_quad(np.ones((1, 1)), [n], [n])
    assert q == math.factorial(n)
    q, _ = oracle.perm_mult_quad(np.eye(4), [3, 0, 2, 1], [3, 0, 2, 1])
    assert q == 12


def test_golden_repeated_values_present():
    path = os.path.join(GOLDEN, "repeated_permanents.txt")
    if not os.path.exists(path):
        pytest.skip("golden file not generated")
    from tests.golden import load_repeated
    U, cases = load_repeated(path)
    assert U.shape == (20, 20) and np.max(np.abs(U @ U.conj().T - np.eye(20))) < 1e-13
    for c in cases:
        assert c["S"].sum() == 40 and c["T"].sum() == 40 and c["S"].max() <= 4 and c["T"].max() <= 4


def test_chain_rule_sampler_reproduces_born_rule():
    # averaged over every order of the input modes, the probability that the
    # chain rule draws the multiset T (summed over draw sequences) is the
    # Born-rule probability |perm(U_{T,S})|^2 / (prod S! prod T!)
    import itertools as it
    m, inputs = 4, [0, 2, 3]
    U = workloads.haar(m, 11)
    S = np.zeros(m, np.int32)
    S[inputs] = 1
    n = len(inputs)
    prob = {}
    orders = list(it.permutations(inputs))
    for order in orders:
        def walk(rows, p):
            k = len(rows) + 1
            if k > n:
                T = tuple(np.bincount(rows, minlength=m))
                prob[T] = prob.get(T, 0.0) + p / len(orders)
                return
            w = oracle.chain_rule_distribution(U, order, rows)
            w = w / w.sum()
            for l in range(m):
                if w[l] > 0:
                    walk(rows + [l], p * w[l])
        walk([], 1.0)
    for T in workloads.fock_outputs(m, n):
        want = oracle.probability(U, S, T)
        assert abs(prob.get(tuple(int(v) for v in T), 0.0) - want) < 1e-12, T
    assert abs(sum(prob.values()) - 1.0) < 1e-12


@pytest.mark.parametrize("inputs", [[0, 0, 1], [2, 2, 2], [0, 1, 1, 3]])
def test_chain_rule_reproduces_born_rule_with_repeated_inputs(inputs):
    # random Fock inputs put several photons in one mode: the column list then
    # repeats that mode, and the exhaustive walk over input orders and draws
    # must still give |perm(U_{T,S})|^2 / (prod S! prod T!) for every T
    m = 4
    U = workloads.haar(m, 5)
    n = len(inputs)
    S = np.bincount(inputs, minlength=m).astype(np.int32)
    prob = {}
    orders = list(it.permutations(inputs))
    for order in orders:
        def walk(rows, p):
            if len(rows) == n:
                T = tuple(np.bincount(rows, minlength=m))
                prob[T] = prob.get(T, 0.0) + p / len(orders)
                return
            w = oracle.chain_rule_distribution(U, order, rows)
            w = w / w.sum()
            for l in range(m):
                if w[l] > 0:
                    walk(rows + [l], p * w[l])
        walk([], 1.0)
    for T in workloads.fock_outputs(m, n):
        assert abs(prob.get(tuple(int(v) for v in T), 0.0) - oracle.probability(U, S, T)) < 1e-12, T


def test_chain_rule_sample_inverts_the_cdf():
    U = workloads.haar(5, 2)
    order = [3, 0, 1]
    rows, margins = oracle.chain_rule_sample(U, order, [0.0, 0.5, 0.999999])
    w0 = oracle.chain_rule_distribution(U, order, [])
    assert rows[0] == int(np.argmax(w0 > 0))          # u = 0 picks the first mode with weight
    assert len(rows) == 3 and all(0 <= r < 5 for r in rows) and len(margins) == 3


def test_chain_rule_sample_interior_uniforms_closed_form():
    # Two photons, weights written out by hand (not through the oracle's
    # permanent): step 1 draws l with weight |U[l, c1]|^2 (a 1 x 1 permanent),
    # step 2 with weight |U[r1, c1] U[l, c2] + U[r1, c2] U[l, c1]|^2 (the
    # 2 x 2 permanent ad + bc).  For uniforms strictly inside every CDF
    # interval the draw must be that interval's mode: an off-by-one in the
    # inversion, a reversed cumulative order or a swapped column fails here.
    m = 5
    U = workloads.haar(m, 12)
    for order in ([3, 0], [1, 4], [2, 2]):        # the last one repeats an input mode
        c1, c2 = order
        w1 = np.abs(U[:, c1]) ** 2
        cdf1 = np.cumsum(w1) / w1.sum()
        lo1 = np.concatenate([[0.0], cdf1[:-1]])
        for i in range(m):
            if w1[i] < 1e-12:
                continue
            for frac in (0.25, 0.5, 0.75):
                u1 = lo1[i] + frac * (cdf1[i] - lo1[i])
                w2 = np.abs(U[i, c1] * U[:, c2] + U[i, c2] * U[:, c1]) ** 2
                cdf2 = np.cumsum(w2) / w2.sum()
                lo2 = np.concatenate([[0.0], cdf2[:-1]])
                for j in range(m):
                    if w2[j] < 1e-12:
                        continue
                    u2 = lo2[j] + 0.5 * (cdf2[j] - lo2[j])
                    rows, margins = oracle.chain_rule_sample(U, order, [u1, u2])
                    assert rows == [i, j], (order, i, j, rows)
                    assert min(margins) > 0.0


# ------------------------------------------------------------------ losses
def _detected(m, n):
    for k in range(n + 1):
        for T in workloads.fock_outputs(m, k):
            yield T


def test_lossy_distribution_is_normalised_and_binomial_for_uniform_loss():
    # uniform transmissivity: every photon survives independently, so the
    # detected photon number is Binomial(n, eta)
    m, eta = 4, 0.7
    U = workloads.haar(m, 31)
    S = np.array([1, 1, 0, 1], np.int32)
    n = 3
    by_k = np.zeros(n + 1)
    for T in _detected(m, n):
        by_k[int(T.sum())] += oracle.lossy_probability(U, [eta] * m, S, T)
    for k in range(n + 1):
        assert abs(by_k[k] - math.comb(n, k) * eta ** k * (1 - eta) ** (n - k)) < 1e-12
    assert abs(by_k.sum() - 1.0) < 1e-12


def test_lossy_mean_occupation():
    # <n_i> = eta_i sum_j |U_ij|^2 s_j for Fock inputs through a linear
    # interferometer followed by loss on mode i
    m = 4
    U = workloads.haar(m, 32)
    eta = [0.9, 0.5, 0.25, 1.0]
    S = np.array([2, 0, 1, 1], np.int32)
    mean = np.zeros(m)
    for T in _detected(m, 4):
        mean += T * oracle.lossy_probability(U, eta, S, T)
    want = np.array(eta) * (np.abs(U) ** 2 @ S)
    assert np.max(np.abs(mean - want)) < 1e-12


def test_no_loss_reduces_to_ideal_and_dilation_is_unitary():
    m = 3
    U = workloads.haar(m, 33)
    S = np.array([1, 2, 0], np.int32)
    for T in workloads.fock_outputs(m, 3):
        assert abs(oracle.lossy_probability(U, [1.0] * m, S, T) - oracle.probability(U, S, T)) < 1e-14
    Ud = oracle.loss_dilation(U, [0.3, 0.6, 0.9])
    assert np.max(np.abs(Ud @ Ud.conj().T - np.eye(6))) < 1e-14


def test_general_lossy_form_mean_occupation():
    # A = V diag(sqrt(eta)) W: mean detected occupation <n_j> = sum_i |A_ji|^2 s_i
    # for Fock inputs through any passive linear network (first moment only
    # depends on |A|^2), here with the two unitaries on either side of the loss
    m = 4
    V, W = workloads.haar(m, 34), workloads.haar(m, 35)
    eta = [0.9, 0.35, 0.6, 1.0]
    S = np.array([1, 2, 0, 1], np.int32)
    A = np.zeros((m, m), complex)
    for j in range(m):
        for i in range(m):
            A[j, i] = sum(V[j, k] * math.sqrt(eta[k]) * W[k, i] for k in range(m))
    mean = np.zeros(m)
    for T in _detected(m, 4):
        mean += T * oracle.lossy_probability(W, eta, S, T, V=V)
    assert np.max(np.abs(mean - (np.abs(A) ** 2) @ S)) < 1e-12


def test_uniform_loss_commutes_with_the_interferometer():
    # equal transmissivity on every mode commutes with any unitary: loss
    # between W and V gives the same detection statistics as loss after V W
    m, eta = 3, 0.55
    V, W = workloads.haar(m, 36), workloads.haar(m, 37)
    S = np.array([2, 0, 1], np.int32)
    for T in _detected(m, 3):
        a = oracle.lossy_probability(W, [eta] * m, S, T, V=V)
        b = oracle.lossy_probability(V @ W, [eta] * m, S, T)
        assert abs(a - b) < 1e-14


def test_general_dilation_blocks_and_special_cases():
    m = 3
    V, W = workloads.haar(m, 38), workloads.haar(m, 39)
    eta = [0.2, 0.7, 1.0]
    Ud = oracle.loss_dilation_vw(V, eta, W)
    assert np.max(np.abs(Ud @ Ud.conj().T - np.eye(2 * m))) < 1e-14
    # the system block is the lossy transfer matrix, element by element
    for j in range(m):
        for i in range(m):
            a = sum(V[j, k] * math.sqrt(eta[k]) * W[k, i] for k in range(m))
            assert abs(Ud[j, i] - a) < 1e-15
    # no unitary after the loss: the dilation of loss after W
    assert np.max(np.abs(oracle.loss_dilation_vw(np.eye(m), eta, W) - oracle.loss_dilation(W, eta))) < 1e-15
    # total loss: nothing reaches the detectors
    S = np.array([1, 1, 0], np.int32)
    assert abs(oracle.lossy_probability(W, [0.0] * m, S, np.zeros(m, np.int32), V=V) - 1.0) < 1e-14


# -------------------------------------------------------------- loop hafnian
def involutions(n):
    # number of single-pair matchings of n vertices: T(n) = T(n-1) + (n-1) T(n-2)
    t = [1, 1]
    for k in range(2, n + 1):
        t.append(t[-1] + (k - 1) * t[-2])
    return t[n]


def odd_double_factorial(n):
    # (n - 1)!! perfect matchings of n (even) vertices
    return math.prod(range(n - 1, 0, -2)) if n % 2 == 0 else 0


@pytest.mark.parametrize("n", range(0, 11))
def test_lhaf_bruteforce_counts_matchings(n):
    J = [[1] * n for _ in range(n)]
    assert oracle.lhaf_bruteforce(J, loops=False) == odd_double_factorial(n)
    assert oracle.lhaf_bruteforce(J) == involutions(n)


def test_lhaf_bruteforce_small_closed_forms():
    rng = np.random.default_rng(3)
    a = rng.integers(-9, 10, (4, 4)).tolist()
    assert oracle.lhaf_bruteforce([]) == 1
    assert oracle.lhaf_bruteforce([[a[0][0]]]) == a[0][0]
    assert oracle.lhaf_bruteforce([r[:2] for r in a[:2]]) == a[0][1] + a[0][0] * a[1][1]
    three = [r[:3] for r in a[:3]]
    assert oracle.lhaf_bruteforce(three) == (a[0][0] * a[1][1] * a[2][2] + a[0][0] * a[1][2]
                                              + a[1][1] * a[0][2] + a[2][2] * a[0][1])
    assert oracle.lhaf_bruteforce(three, loops=False) == 0
    assert oracle.lhaf_bruteforce(a, loops=False) == a[0][1] * a[2][3] + a[0][2] * a[1][3] + a[0][3] * a[1][2]


@pytest.mark.parametrize("k", range(1, 6))
def test_haf_complete_bipartite_is_factorial(k):
    # perfect matchings of K_{k,k}: k!
    n = 2 * k
    B = [[1 if (i < k) != (j < k) else 0 for j in range(n)] for i in range(n)]
    assert oracle.lhaf_bruteforce(B, loops=False) == math.factorial(k)


@pytest.mark.parametrize("seed", range(24))
def test_lhaf_rep_matches_bruteforce_on_expanded_matrix(seed):
    # upper triangle only: a non-symmetric A would expose a transposed read
    rng = np.random.default_rng(seed)
    d = int(rng.integers(1, 6))
    reps = rng.integers(0, 4, d)
    while reps.sum() > 10:
        reps[int(rng.integers(0, d))] = 0
    A = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    g = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    B = oracle.expand_lhaf(A, g, reps)
    for gamma, loops in ((g, True), (None, False)):
        want = complex(oracle.lhaf_bruteforce(B, loops=loops))
        got = oracle.lhaf_rep(A, gamma, reps)
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (reps, loops)


@pytest.mark.parametrize("seed", range(6))
def test_haf_rep_block_matrix_is_repeated_permanent(seed):
    # haf([[0, B], [B^T, 0]]) with repetitions (t, s) pairs row copies with
    # column copies only: perm(B_{t,s}) (ties the hafnian table to Ryser)
    rng = np.random.default_rng(100 + seed)
    k = int(rng.integers(2, 9))
    B = workloads.gaussian_matrix(k, seed)
    t = rng.integers(0, 4, k)
    s = np.zeros(k, np.int64)
    for _ in range(int(t.sum())):
        s[int(rng.integers(0, k))] += 1
    while np.prod(t + 1) * np.prod(s + 1) > (1 << 22):
        t[int(np.argmax(t))] -= 1
        s[int(np.argmax(s))] -= 1
    M = np.zeros((2 * k, 2 * k), np.complex128)
    M[:k, k:] = B
    M[k:, :k] = B.T
    got = oracle.lhaf_rep(M, None, np.concatenate([t, s]))
    want = oracle.perm_mult(B, s, t)
    assert rel(got, want) <= 1e-13
    # loops of weight zero change nothing
    assert rel(oracle.lhaf_rep(M, np.zeros(2 * k), np.concatenate([t, s])), want) <= 1e-13


@pytest.mark.parametrize("reps", [[3], [2, 2], [1, 2, 3], [5, 0, 4], [2] * 6, [10, 10, 10], [1] * 12])
def test_lhaf_rep_constant_matrix_hermite_form(reps):
    # A = a J, gamma = g 1: every matching of N vertices with j pairs counts
    # a^j g^(N-2j); there are N! / (j! (N-2j)! 2^j) of them
    a, g = 0.75 - 0.5j, 0.5 + 0.25j
    d = len(reps)
    N = sum(reps)
    want = sum(math.factorial(N) / (math.factorial(j) * math.factorial(N - 2 * j) * 2 ** j) * a ** j * g ** (N - 2 * j)
               for j in range(N // 2 + 1))
    got = oracle.lhaf_rep(np.full((d, d), a), np.full(d, g), reps)
    assert rel(got, want) <= 1e-14
    want_haf = (math.factorial(N) / (math.factorial(N // 2) * 2 ** (N // 2)) * a ** (N // 2)) if N % 2 == 0 else 0
    assert abs(oracle.lhaf_rep(np.full((d, d), a), None, reps) - want_haf) <= 1e-14 * max(1, abs(want_haf))


@pytest.mark.parametrize("seed", range(4))
def test_lhaf_rep_diagonal_scaling_and_mode_permutation(seed):
    rng = np.random.default_rng(200 + seed)
    d = 6
    A = workloads.symmetric_gaussian(d, seed)
    g = workloads.loop_vector(d, seed)
    reps = rng.integers(0, 4, d)
    base = oracle.lhaf_rep(A, g, reps)
    D = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    scaled = oracle.lhaf_rep(D[:, None] * A * D[None, :], D * g, reps)
    assert rel(scaled, np.prod(D ** reps) * base) <= 1e-13
    p = rng.permutation(d)
    assert rel(oracle.lhaf_rep(A[np.ix_(p, p)], g[p], reps[p]), base) <= 1e-13


def test_lhaf_rep_loops_only_and_no_loops():
    rng = np.random.default_rng(7)
    d = 5
    g = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    reps = np.array([2, 0, 3, 1, 1])
    assert rel(oracle.lhaf_rep(np.zeros((d, d)), g, reps), np.prod(g ** reps)) <= 1e-15
    A = workloads.gbs_matrix(d, 1)
    assert oracle.lhaf_rep(A, np.zeros(d), reps) == oracle.lhaf_rep(A, None, reps)
    assert oracle.lhaf_rep(A, None, [1, 0, 0, 0, 0]) == 0
    assert oracle.lhaf_rep(A, g, [0] * d) == 1


def squeezed_shells(r, nmax):
    # total photon number of independent squeezed vacua: mode i holds 2k
    # photons with probability (2k)! / (2^k k!)^2 tanh^(2k) r_i / cosh r_i; a
    # passive interferometer keeps the total
    dist = np.zeros(nmax + 1)
    dist[0] = 1.0
    for ri in r:
        single = np.zeros(nmax + 1)
        for k in range(nmax // 2 + 1):
            single[2 * k] = math.factorial(2 * k) / (2 ** k * math.factorial(k)) ** 2 * np.tanh(ri) ** (2 * k) / np.cosh(ri)
        dist = np.convolve(dist, single)[:nmax + 1]
    return dist


def test_gbs_photon_shells_match_squeezed_statistics():
    # squeezed vacua through a Haar interferometer: p(t) = |haf(B_t)|^2 /
    # (prod t! prod cosh r) with B = U diag(tanh r) U^T (Gaussian Boson
    # Sampling appendix, pure state, no displacement); every output with two
    # photons in one mode needs the pair weight B_ii between its copies
    import itertools
    d = 3
    r = np.array([0.5, 0.3, 0.4])
    U = workloads.haar(d, 3)
    B = (U * np.tanh(r)) @ U.T
    want = squeezed_shells(r, 12)
    for N in range(0, 13):
        shell = 0.0
        for t in itertools.product(range(N + 1), repeat=d):
            if sum(t) == N:
                h = oracle.lhaf_rep(B, None, list(t))
                shell += abs(h) ** 2 / (math.prod(math.factorial(x) for x in t) * np.prod(np.cosh(r)))
        assert abs(shell - want[N]) <= 1e-15 + 1e-13 * want[N], N
