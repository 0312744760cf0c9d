"""Parity of the adjoint Gray-code sweep (pq_perm_grad) against the oracle's
gradient t_i s_j perm(U_{T-e_i, S-e_j})."""
import numpy as np
import pytest

import oracle
import workloads
from tests.tolerance import assert_entries_close, floor_of, vjp_floor

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def eng():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_04006_amd as pq
    return pq.Engine(0)


def dev(U):
    return torch.from_numpy(np.ascontiguousarray(U, dtype=np.complex128)).cuda()


def oracle_vjp(U, Ss, Ts, g):
    """oracle.perm_vjp on each pattern's own modes (the oracle's gradient takes
    at most 128 modes; perm(U_{T,S}) only reads the rows of T and columns of S)."""
    m = U.shape[0]
    if m <= 128:
        return oracle.perm_vjp(U, Ss, Ts, g)
    dU = np.zeros((m, m), dtype=np.complex128)
    for S, T, gp in zip(Ss, Ts, g):
        modes = np.union1d(np.flatnonzero(S), np.flatnonzero(T))
        sub = oracle.perm_vjp(U[np.ix_(modes, modes)], [np.asarray(S)[modes]], [np.asarray(T)[modes]], [gp])
        dU[np.ix_(modes, modes)] += sub
    return dU


def check(eng, U, Ss, Ts, g, tol=1e-10):
    # every entry by its own relative error; an absolute floor only below the
    # rounding scale of that entry's Gray-code sum (tests/tolerance.py)
    dU, perm = eng.perm_grad(dev(U), Ss, Ts, torch.from_numpy(np.asarray(g, dtype=np.complex128)))
    dU = dU.cpu().numpy()
    perm = perm.cpu().numpy()
    ref = oracle_vjp(U, Ss, Ts, g)
    assert_entries_close(dU, ref, tol, vjp_floor(U, Ss, Ts, g), "dU")
    for p, (S, T) in enumerate(zip(Ss, Ts)):
        r = oracle.perm_mult(U, S, T)
        assert_entries_close(perm[p], r, tol, floor_of(U, S, T), f"perm[{p}]")
    return dU


@pytest.mark.parametrize("seed", range(6))
def test_random_patterns_with_repeats(eng, seed):
    rng = np.random.default_rng(seed)
    m = 7
    U = workloads.haar(m, 40 + seed)
    Ss, Ts, g = [], [], []
    for p in range(12):
        n = int(rng.integers(1, 9))
        Ss.append(workloads.random_occupations(rng, m, n, cap=3))
        Ts.append(workloads.random_occupations(rng, m, n, cap=3))
        g.append(complex(rng.standard_normal(), rng.standard_normal()))
    check(eng, U, Ss, Ts, g)


def test_unit_multiplicity_larger(eng):
    # n = 12 collision-free: 6 lane digits, 5 time digits, several adjoint chunks
    m = 24
    U = workloads.haar(m, 8)
    rng = np.random.default_rng(8)
    Ss, Ts, g = [], [], []
    for p in range(3):
        S = np.zeros(m, np.int32)
        T = np.zeros(m, np.int32)
        S[rng.choice(m, 12, replace=False)] = 1
        T[rng.choice(m, 12, replace=False)] = 1
        Ss.append(S)
        Ts.append(T)
        g.append(complex(rng.standard_normal(), rng.standard_normal()))
    check(eng, U, Ss, Ts, g)


def test_mesh_shaped_patterns(eng):
    # 12-mode mesh, 8 photons in modes 0..7, collision-free outputs
    U = oracle.mesh_unitary(workloads.mesh_angles(0), workloads.MESH_CELLS, workloads.MESH_MODES)
    pats = workloads.mesh_patterns(count=48, seed=1)
    S = np.zeros(12, np.int32)
    S[:8] = 1
    rng = np.random.default_rng(2)
    g = [complex(rng.standard_normal(), rng.standard_normal()) for _ in range(48)]
    check(eng, U, [S] * 48, list(pats), g)


def test_euler_identity_single_pattern(eng):
    U = workloads.haar(6, 4)
    S = np.array([1, 2, 0, 1, 0, 2], np.int32)
    T = np.array([0, 1, 3, 0, 2, 0], np.int32)
    dU, perm = eng.perm_grad(dev(U), [S], [T], torch.ones(1, dtype=torch.complex128))
    d = np.conj(dU.cpu().numpy())           # d perm / dU
    p = complex(perm.cpu().numpy()[0])
    for i in range(6):
        assert abs(np.sum(U[i, :] * d[i, :]) - T[i] * p) < 1e-12
    for j in range(6):
        assert abs(np.sum(U[:, j] * d[:, j]) - S[j] * p) < 1e-12


def test_trivial_patterns_have_zero_gradient(eng):
    U = workloads.haar(4, 1)
    dU, perm = eng.perm_grad(dev(U), [[1, 0, 0, 0], [0, 0, 0, 0]], [[1, 1, 0, 0], [0, 0, 0, 0]],
                             torch.ones(2, dtype=torch.complex128))
    assert np.all(dU.cpu().numpy() == 0)
    assert np.array_equal(perm.cpu().numpy(), np.array([0, 1], dtype=np.complex128))


def _wide_patterns(m, ns, seed):
    rng = np.random.default_rng(seed)
    Ss, Ts = [], []
    for n in ns:
        S = np.zeros(m, np.int32)
        T = np.zeros(m, np.int32)
        S[rng.choice(m, n, replace=False)] = 1
        T[rng.choice(m, n, replace=False)] = 1
        Ss.append(S)
        Ts.append(T)
    g = [complex(rng.standard_normal(), rng.standard_normal()) for _ in ns]
    return Ss, Ts, g


@pytest.mark.parametrize("ns", [(13,), (16, 14), (17, 8, 3), (20,)])
def test_wide_collision_free_patterns(eng, ns):
    # 13..20 distinct columns: the long-walk reverse sweep (four lanes per
    # term), mixed with small patterns that take the chunked reverse sweep
    n = max(ns)
    m = 2 * n * n
    U = workloads.haar(m, 300 + n)
    Ss, Ts, g = _wide_patterns(m, ns, n)
    check(eng, U, Ss, Ts, g, tol=1e-10)


def _laplace_check(U, S, T, d, p, tol):
    # collision-free: sum_j U_ij d perm/dU_ij = perm for every row i of the
    # pattern, and the same down every column (Laplace expansion)
    rows = np.flatnonzero(T)
    cols = np.flatnonzero(S)
    worst = 0.0
    for i in rows:
        terms = U[i, cols] * d[i, cols]
        worst = max(worst, abs(np.sum(terms) - p) / np.sum(np.abs(terms)))
    for j in cols:
        terms = U[rows, j] * d[rows, j]
        worst = max(worst, abs(np.sum(terms) - p) / np.sum(np.abs(terms)))
    assert worst < tol, worst
    return worst


@pytest.mark.parametrize("n", [22, 24, 27])
def test_wide_gradient_sampled_entries(eng, n):
    # 6, 6 and 7 columns per lane; oracle minors on sampled entries
    m = 2 * n * n
    U = workloads.haar(m, n)
    Ss, Ts, _ = _wide_patterns(m, (n,), 5)
    S, T = Ss[0], Ts[0]
    dU, perm = eng.perm_grad(dev(U), [S], [T], torch.ones(1, dtype=torch.complex128))
    d = np.conj(dU.cpu().numpy())
    p = complex(perm.cpu().numpy()[0])
    ref_p = oracle.perm_mult(U, S, T)
    assert abs(p - ref_p) < 1e-8 * abs(ref_p)
    _laplace_check(U, S, T, d, p, 1e-9)
    rows = np.flatnonzero(T)
    cols = np.flatnonzero(S)
    for (a, b) in [(0, 0), (5, n - 7), (n - 1, 11), (12, n - 1)]:
        i, j = rows[a], cols[b]
        S1, T1 = S.copy(), T.copy()
        S1[j] -= 1
        T1[i] -= 1
        want = oracle.perm_mult(U, S1, T1)
        assert abs(d[i, j] - want) < 1e-8 * abs(want), (a, b)
    # entries outside the pattern's support are zero
    mask = np.ones((m, m), bool)
    mask[np.ix_(rows, cols)] = False
    assert np.all(dU.cpu().numpy()[mask] == 0)


def test_wide_gradient_full_size_n30(eng):
    # n = 30 (32 padded columns, 8 per lane): the forward value of the same
    # sweep against the forward kernel, and the Laplace expansion along every
    # row and column of the pattern
    n, m = 30, 1800
    U = workloads.haar(m, 30)
    S = np.zeros(m, np.int32)
    T = np.zeros(m, np.int32)
    S[:n] = 1
    T[:n] = 1
    dU, perm = eng.perm_grad(dev(U), [S], [T], torch.ones(1, dtype=torch.complex128))
    d = np.conj(dU.cpu().numpy())
    p = complex(perm.cpu().numpy()[0])
    pf, _ = eng.perm(dev(U), S, T)
    pf = complex(pf.cpu().numpy())
    assert abs(p - pf) < 1e-10 * abs(pf)
    worst = _laplace_check(U, S, T, d, p, 1e-9)
    print(f"n=30 gradient: Laplace identity worst relative residual {worst:.2e}")


def test_wide_gradient_is_deterministic(eng):
    n, m = 20, 800
    U = workloads.haar(m, 31)
    Ss, Ts, g = _wide_patterns(m, (n, 18), 7)
    gt = torch.from_numpy(np.asarray(g, dtype=np.complex128))
    a, _ = eng.perm_grad(dev(U), Ss, Ts, gt)
    b, _ = eng.perm_grad(dev(U), Ss, Ts, gt)
    assert torch.equal(a, b)


def test_wide_pattern_with_repeats_is_rejected(eng):
    # more than 24 distinct columns is supported for collision-free patterns only
    import paper_2403_04006_amd as pq
    m = 60
    U = workloads.haar(m, 2)
    S = np.zeros(m, np.int32)
    T = np.zeros(m, np.int32)
    S[:26] = 1
    T[:24] = 1
    T[30] = 2
    with pytest.raises(pq.PqError):
        eng.perm_grad(dev(U), [S], [T], torch.ones(1, dtype=torch.complex128))


def test_repeated_patterns_are_swept_once_and_summed(eng):
    # the same pattern three times (with other patterns between its copies):
    # identical patterns are swept once, their cotangents summed in pattern
    # order, and every copy's forward value is written
    m = 9
    U = workloads.haar(m, 77)
    rng = np.random.default_rng(77)
    base = [(workloads.random_occupations(rng, m, n, cap=2), workloads.random_occupations(rng, m, n, cap=2))
            for n in (5, 6, 4)]
    order = [0, 1, 0, 2, 1, 0]
    Ss = [base[i][0] for i in order]
    Ts = [base[i][1] for i in order]
    g = [complex(rng.standard_normal(), rng.standard_normal()) for _ in order]
    check(eng, U, Ss, Ts, g)
    _, perm = eng.perm_grad(dev(U), Ss, Ts, torch.from_numpy(np.asarray(g, dtype=np.complex128)))
    perm = perm.cpu().numpy()
    assert perm[0] == perm[2] == perm[5] and perm[1] == perm[4]


_VARIANT_REF = {}


@pytest.mark.parametrize("digits,swizzle", [(1, 0), (1, 1), (2, 0), (2, 1), (3, 0), (3, 1)])
@pytest.mark.parametrize("n", [16, 21])
def test_wide_walk_variants_against_oracle(eng, n, digits, swizzle):
    # every form of the long-walk reverse sweep (register flip digits 1..3,
    # quad exchanges by DPP or ds_swizzle) against the oracle's minors, entry
    # by entry; n = 21 pads 3 of its 24 columns
    m = 2 * n * n
    U = workloads.haar(m, 500 + n)
    Ss, Ts, g = _wide_patterns(m, (n,), 600 + n)
    if n not in _VARIANT_REF:
        _VARIANT_REF[n] = oracle_vjp(U, Ss, Ts, g), oracle.perm_mult(U, Ss[0], Ts[0])
    ref, ref_p = _VARIANT_REF[n]
    eng.walk_variant(digits, bool(swizzle))
    try:
        dU, perm = eng.perm_grad(dev(U), Ss, Ts, torch.from_numpy(np.asarray(g, dtype=np.complex128)))
    finally:
        eng.walk_variant(3, False)
    tol = 1e-10 if n <= 20 else 1e-8
    assert_entries_close(dU.cpu().numpy(), ref, tol, vjp_floor(U, Ss, Ts, g), "dU")
    assert_entries_close(perm.cpu().numpy()[0], ref_p, tol, floor_of(U, Ss[0], Ts[0]), "perm")


@pytest.mark.parametrize("digits,swizzle", [(1, 0), (2, 1), (3, 0)])
def test_wide_walk_variants_n30_laplace(eng, digits, swizzle):
    # n = 30 (8 columns per lane, 2 padded): the forward value of the same
    # sweep against the forward kernel, and the Laplace expansion along every
    # row and column, for three forms of the walk
    n, m = 30, 1800
    U = workloads.haar(m, 30)
    S = np.zeros(m, np.int32)
    T = np.zeros(m, np.int32)
    S[:n] = 1
    T[:n] = 1
    eng.walk_variant(digits, bool(swizzle))
    try:
        dU, perm = eng.perm_grad(dev(U), [S], [T], torch.ones(1, dtype=torch.complex128))
    finally:
        eng.walk_variant(3, False)
    d = np.conj(dU.cpu().numpy())
    p = complex(perm.cpu().numpy()[0])
    pf, _ = eng.perm(dev(U), S, T)
    pf = complex(pf.cpu().numpy())
    assert abs(p - pf) < 1e-10 * abs(pf)
    _laplace_check(U, S, T, d, p, 1e-9)


def test_walk_variant_rejects_out_of_range(eng):
    import paper_2403_04006_amd as pq
    for digits, sw in ((0, 0), (4, 0), (1, 2)):
        with pytest.raises(pq.PqError):
            eng.walk_variant(digits, sw)
    eng.walk_variant(3, False)


@pytest.mark.parametrize("n", [30, 32])
def test_wide_gradient_full_size_against_stored_minors(eng, n):
    # the reverse walk's derivative entries at full size against the oracle's
    # permanents of the corresponding minors (tests/golden/make_golden_minors.py),
    # each entry by its own relative error, 1e-8 for n <= 32
    from tests.golden import load_minors
    A, minors = load_minors(n)
    S = np.ones(n, np.int32)
    dU, perm = eng.perm_grad(dev(A), [S], [S], torch.ones(1, dtype=torch.complex128))
    d = np.conj(dU.cpu().numpy())
    for i, j, want in minors:
        err = abs(d[i, j] - want) / abs(want)
        print(f"n={n} d perm / d A[{i},{j}]: rel err {err:.2e}", flush=True)
        assert err < 1e-8, (i, j, d[i, j], want)
