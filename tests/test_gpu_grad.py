"""Parity of the adjoint Gray-code sweep (pq_perm_grad) against the oracle's
gradient t_i s_j perm(U_{T-e_i, S-e_j})."""
import numpy as np
import pytest

import oracle
import workloads

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


def check(eng, U, Ss, Ts, g, tol=1e-10):
    dU, perm = eng.perm_grad(dev(U), Ss, Ts, torch.from_numpy(np.asarray(g, dtype=np.complex128)))
    dU = dU.cpu().numpy()
    perm = perm.cpu().numpy()
    ref = oracle.perm_vjp(U, Ss, Ts, g)
    scale = max(1e-300, np.max(np.abs(ref)))
    err = np.max(np.abs(dU - ref)) / scale
    for p, (S, T) in enumerate(zip(Ss, Ts)):
        r = oracle.perm_mult(U, S, T)
        assert abs(perm[p] - r) <= tol * max(abs(r), 1e-300) or abs(r) < 1e-14
    assert err < tol, err
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
