"""Chain-rule boson sampling on the device (pq_sample_chain): replay against
the oracle's sampler on the same orders and uniforms, and the Born-rule
distribution of the samples."""
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


def replay(eng, U, inputs, samples, seed, check=None):
    rng = np.random.default_rng(seed)
    n = len(inputs)
    order = np.stack([rng.permutation(inputs) for _ in range(samples)]).astype(np.int32)
    u = rng.random((samples, n))
    out = eng.sample_chain(dev(U), torch.from_numpy(order), torch.from_numpy(u)).cpu().numpy()
    assert out.shape == (samples, n)
    agree, near = 0, 0
    for s in range(samples if check is None else check):
        rows, margins = oracle.chain_rule_sample(U, list(order[s]), u[s])
        for k in range(n):
            if out[s, k] != rows[k]:
                # only a decision within rounding of a cumulative-weight
                # boundary may differ; the draws that follow then diverge
                assert margins[k] < 1e-9, (s, k, margins[k])
                near += 1
                break
        else:
            agree += 1
    return out, agree, near


@pytest.mark.parametrize("n,m", [(3, 5), (6, 16), (11, 24), (17, 40)])
def test_replay_matches_oracle(eng, n, m):
    # 2..17 photons: lane digits only, lane + wavefront digits, and time digits
    U = workloads.haar(m, 100 + n)
    _, agree, near = replay(eng, U, list(range(n)), samples=40, seed=n)
    assert agree + near == 40 and agree >= 39


def test_replay_sampling_shape_full_size(eng):
    # 20 photons in 400 modes (input modes 0..19), three full samples
    U = workloads.haar(400, 0)
    _, agree, near = replay(eng, U, list(range(20)), samples=64, seed=7, check=3)
    assert agree == 3


def test_samples_follow_born_rule(eng):
    # 3 photons in 5 modes: 60000 samples (random input orders and uniforms)
    # against |perm(U_{T,S})|^2 / prod T! over all 35 output multisets
    m, inputs = 5, [0, 1, 2]
    U = workloads.haar(m, 21)
    rng = np.random.default_rng(4)
    N = 60000
    order = np.stack([rng.permutation(inputs) for _ in range(N)]).astype(np.int32)
    u = rng.random((N, 3))
    out = eng.sample_chain(dev(U), torch.from_numpy(order), torch.from_numpy(u)).cpu().numpy()
    S = np.zeros(m, np.int32)
    S[inputs] = 1
    counts = {}
    for row in out:
        T = tuple(np.bincount(row, minlength=m))
        counts[T] = counts.get(T, 0) + 1
    chi2 = 0.0
    outs = workloads.fock_outputs(m, 3)
    for T in outs:
        p = oracle.probability(U, S, T)
        e = N * p
        o = counts.get(tuple(int(v) for v in T), 0)
        if e > 0:
            chi2 += (o - e) ** 2 / e
        else:
            assert o == 0
    # 34 degrees of freedom: P(chi2 > 80) < 1e-5
    print(f"Born-rule chi^2 over 35 outputs: {chi2:.1f}")
    assert chi2 < 80


def test_sampling_is_deterministic(eng):
    U = dev(workloads.haar(30, 3))
    rng = np.random.default_rng(9)
    order = torch.from_numpy(np.stack([rng.permutation(12) for _ in range(50)]).astype(np.int32))
    u = torch.from_numpy(rng.random((50, 12)))
    a = eng.sample_chain(U, order, u)
    b = eng.sample_chain(U, order, u)
    assert torch.equal(a, b)


def test_argument_errors(eng):
    import paper_2403_04006_amd as pq
    U = dev(workloads.haar(4, 0))
    with pytest.raises(pq.PqError):
        eng.sample_chain(U, torch.zeros((2, 5), dtype=torch.int32), torch.zeros((2, 5)))   # n > m
    with pytest.raises(ValueError):
        eng.sample_chain(U, torch.zeros((2, 3), dtype=torch.int32), torch.zeros((2, 4)))


def fock_input(rng, m, n):
    # random Fock input: n photons thrown uniformly into m modes (repeats allowed)
    return [int(x) for x in np.repeat(np.arange(m), workloads.random_occupations(rng, m, n))]


@pytest.mark.parametrize("n,m", [(4, 8), (9, 18), (14, 28)])
def test_replay_repeated_input_modes(eng, n, m):
    # random Fock inputs with photons = modes / 2 (the shape of the paper's
    # boson-sampling benchmark), so input modes repeat in the column lists
    rng = np.random.default_rng(500 + n)
    inputs = fock_input(rng, m, n)
    assert len(set(inputs)) < n
    U = workloads.haar(m, 600 + n)
    _, agree, near = replay(eng, U, inputs, samples=24, seed=n)
    assert agree + near == 24 and agree >= 23


def test_replay_random_fock_input_full_size(eng):
    # 20 photons in 40 modes from a random Fock input (repeated modes)
    rng = np.random.default_rng(40)
    inputs = fock_input(rng, 40, 20)
    assert len(set(inputs)) < 20
    U = workloads.haar(40, 1)
    _, agree, near = replay(eng, U, inputs, samples=64, seed=41, check=3)
    assert agree == 3


def test_samples_follow_born_rule_repeated_inputs(eng):
    # input (2, 1, 0, 0): 60000 samples against |perm(U_{T,S})|^2/(prod S! prod T!)
    m, inputs = 4, [0, 0, 1]
    U = workloads.haar(m, 22)
    rng = np.random.default_rng(5)
    N = 60000
    order = np.stack([rng.permutation(inputs) for _ in range(N)]).astype(np.int32)
    u = rng.random((N, 3))
    out = eng.sample_chain(dev(U), torch.from_numpy(order), torch.from_numpy(u)).cpu().numpy()
    S = np.bincount(inputs, minlength=m).astype(np.int32)
    counts = {}
    for row in out:
        T = tuple(np.bincount(row, minlength=m))
        counts[T] = counts.get(T, 0) + 1
    chi2 = 0.0
    outs = workloads.fock_outputs(m, 3)
    for T in outs:
        e = N * oracle.probability(U, S, T)
        o = counts.get(tuple(int(v) for v in T), 0)
        if e > 0:
            chi2 += (o - e) ** 2 / e
        else:
            assert o == 0
    # 19 degrees of freedom: P(chi2 > 60) < 1e-5
    print(f"Born-rule chi^2 over 20 outputs (repeated input): {chi2:.1f}")
    assert chi2 < 60


def test_out_of_range_input_mode_is_reported(eng):
    # the kernel range-checks every input mode: a bad sample reads nothing
    # through it and is written as -1, the call reports PQ_EINVAL, and the
    # other samples are drawn as usual
    import paper_2403_04006_amd as pq
    m, n = 6, 3
    U = dev(workloads.haar(m, 3))
    rng = np.random.default_rng(2)
    order = np.stack([rng.permutation(n) for _ in range(4)]).astype(np.int32)
    u = rng.random((4, n))
    good = eng.sample_chain(U, torch.from_numpy(order), torch.from_numpy(u)).cpu().numpy()
    for bad in (m, -1, 1 << 20):
        o2 = order.copy()
        o2[2, 1] = bad
        o2_t = torch.from_numpy(o2).cuda()
        u_t = torch.from_numpy(u).cuda()
        out = torch.full((4, n), 7, dtype=torch.int32, device="cuda")
        st = eng._lib.pq_sample_chain(eng._ctx, U.data_ptr(), m, m, n, 4, o2_t.data_ptr(), u_t.data_ptr(),
                                      out.data_ptr(), pq._stream_handle(U.device))
        assert st == pq._lib.PQ_EINVAL, st
        assert "outside" in eng._lib.pq_last_error(eng._ctx).decode()
        got = out.cpu().numpy()
        assert (got[2] == -1).all()
        assert np.array_equal(np.delete(got, 2, axis=0), np.delete(good, 2, axis=0))
    # the ctx recovers: the next valid call succeeds
    again = eng.sample_chain(U, torch.from_numpy(order), torch.from_numpy(u)).cpu().numpy()
    assert np.array_equal(again, good)
