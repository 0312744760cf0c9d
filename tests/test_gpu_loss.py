"""Lossy interferometers: the loss dilations (loss after U, and the general
A = V diag(sqrt(eta)) W) against the oracle's beamsplitter construction, and
lossy sampling / all-outputs against the oracle's lossy detection
probabilities."""
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


def test_dilation_matches_oracle(eng):
    U = workloads.haar(7, 40)
    eta = [0.95, 0.5, 1.0, 0.0, 0.3, 0.8, 0.65]
    Ud = eng.loss_dilation(dev(U), eta).cpu().numpy()
    want = oracle.loss_dilation(U, eta)
    assert np.max(np.abs(Ud - want)) < 1e-15
    assert np.max(np.abs(Ud @ Ud.conj().T - np.eye(14))) < 1e-14


def test_lossy_all_outputs_marginal(eng):
    # every output of the dilation, summed over the environment modes, is the
    # lossy detection probability of each system pattern
    import paper_2403_04006_amd as pq
    m = 4
    U = workloads.haar(m, 41)
    eta = [0.9, 0.6, 0.75, 0.4]
    S = [1, 0, 2, 1]
    n = sum(S)
    Ud = eng.loss_dilation(dev(U), eta)
    _, amp = eng.perm_all_outputs(Ud, S + [0] * m)
    p = np.abs(amp.cpu().numpy()) ** 2
    det = {}
    for r in range(pq.fock_count(2 * m, n)):
        T2 = pq.fock_unrank(2 * m, n, r)
        key = tuple(T2[:m])
        det[key] = det.get(key, 0.0) + p[r]
    for k in range(n + 1):
        for T in workloads.fock_outputs(m, k):
            want = oracle.lossy_probability(U, eta, np.array(S, np.int32), T)
            assert abs(det.get(tuple(int(v) for v in T), 0.0) - want) < 1e-13
    assert abs(sum(det.values()) - 1.0) < 1e-13


def test_lossy_samples_follow_the_lossy_distribution(eng):
    m, inputs = 4, [0, 1, 3]
    U = workloads.haar(m, 42)
    eta = [0.9, 0.5, 0.7, 0.8]
    rng = np.random.default_rng(6)
    N = 60000
    order = np.stack([rng.permutation(inputs) for _ in range(N)]).astype(np.int32)
    u = rng.random((N, 3))
    out = eng.sample_chain_lossy(dev(U), eta, torch.from_numpy(order), torch.from_numpy(u)).cpu().numpy()
    S = np.zeros(m, np.int32)
    S[inputs] = 1
    counts = {}
    for row in out:
        T = tuple(np.bincount(row[row >= 0], minlength=m))
        counts[T] = counts.get(T, 0) + 1
    chi2, cells = 0.0, 0
    for k in range(4):
        for T in workloads.fock_outputs(m, k):
            e = N * oracle.lossy_probability(U, eta, S, T)
            o = counts.get(tuple(int(v) for v in T), 0)
            if e > 0:
                chi2 += (o - e) ** 2 / e
                cells += 1
    # 34 outputs with up to 3 photons in 4 modes: P(chi2 > 80) < 1e-5 at 33 dof
    print(f"lossy chi^2 over {cells} outputs: {chi2:.1f}")
    assert chi2 < 80


@pytest.mark.parametrize("m", [1, 5, 16, 37])
def test_general_dilation_matches_oracle(eng, m):
    # 16 x 16 tiles of the V D W product: one tile, several, and a ragged tail
    V, W = workloads.haar(m, 50 + m), workloads.haar(m, 60 + m)
    eta = list(np.random.default_rng(m).random(m))
    eta[0] = 0.0
    if m > 2:
        eta[-1] = 1.0
    Ud = eng.loss_dilation_vw(dev(V), eta, dev(W)).cpu().numpy()
    want = oracle.loss_dilation_vw(V, eta, W)
    # each entry of V D W is a length-m complex dot product of unit-bounded
    # terms: |error| <= 4 m eps
    assert np.max(np.abs(Ud - want)) < 4 * m * 2.3e-16
    assert np.max(np.abs(Ud @ Ud.conj().T - np.eye(2 * m))) < 1e-13
    # with V = I it is the dilation of loss after W
    I = dev(np.eye(m))
    got = eng.loss_dilation_vw(I, eta, dev(W)).cpu().numpy()
    assert np.max(np.abs(got - eng.loss_dilation(dev(W), eta).cpu().numpy())) < 1e-15


def test_general_lossy_all_outputs_marginal(eng):
    import paper_2403_04006_amd as pq
    m = 4
    V, W = workloads.haar(m, 43), workloads.haar(m, 44)
    eta = [0.9, 0.3, 0.75, 0.5]
    S = [2, 0, 1, 1]
    n = sum(S)
    Ud = eng.loss_dilation_vw(dev(V), eta, dev(W))
    _, amp = eng.perm_all_outputs(Ud, S + [0] * m)
    p = np.abs(amp.cpu().numpy()) ** 2
    det = {}
    for r in range(pq.fock_count(2 * m, n)):
        T2 = pq.fock_unrank(2 * m, n, r)
        key = tuple(T2[:m])
        det[key] = det.get(key, 0.0) + p[r]
    for k in range(n + 1):
        for T in workloads.fock_outputs(m, k):
            want = oracle.lossy_probability(W, eta, np.array(S, np.int32), T, V=V)
            assert abs(det.get(tuple(int(v) for v in T), 0.0) - want) < 1e-13


def test_loss_argument_errors(eng):
    import paper_2403_04006_amd as pq
    U = dev(workloads.haar(3, 0))
    with pytest.raises(pq.PqError):
        eng.loss_dilation(U, [0.5, 1.2, 0.5])
    with pytest.raises(ValueError):
        eng.loss_dilation(U, [0.5, 0.5])
    with pytest.raises(pq.PqError):
        eng.loss_dilation_vw(U, [0.5, -0.1, 0.5], U)
    with pytest.raises(ValueError):
        eng.loss_dilation_vw(U, [0.5, 0.5, 0.5], dev(workloads.haar(4, 0)))
