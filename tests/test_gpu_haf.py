"""Loop hafnian (pq_lhaf) on the GPU against the oracle: random repetition
patterns at sizes the oracle's occupation table finishes in seconds, the
paper's (2, ..., 2) repetitions up to 28 vertices, and at 40 vertices (the
benchmark size) identities that hold at any size: the block-matrix hafnian
equals a repeated permanent (oracle Ryser), the constant-matrix Hermite form,
diagonal scaling and mode permutation."""
import math

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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda()


def tol(N):
    # relative error bound of the FP64 sum (see the design notes): 1e-10 up
    # to 20 vertices, 1e-8 up to 40
    return 1e-10 if N <= 20 else 1e-8


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def gpu_lhaf(eng, A, g, reps):
    out = eng.lhaf(dev(A), None if g is None else dev(g), list(reps))
    torch.cuda.synchronize()
    return complex(out.cpu().numpy()[0])


@pytest.mark.parametrize("seed", range(16))
def test_lhaf_random_patterns_match_oracle(eng, seed):
    rng = np.random.default_rng(500 + seed)
    d = int(rng.integers(1, 13))
    reps = rng.integers(0, 4, d)
    while np.prod(reps + 1) > (1 << 21) or reps.sum() > 24:
        reps[int(np.argmax(reps))] -= 1
    A = workloads.symmetric_gaussian(d, seed) if seed % 2 else workloads.gbs_matrix(d, seed)
    g = workloads.loop_vector(d, seed)
    N = int(reps.sum())
    for gamma in (g, None):
        want = oracle.lhaf_rep(A, gamma, reps)
        got = gpu_lhaf(eng, A, gamma, reps)
        if gamma is None and N % 2:
            assert got == 0
            continue
        assert rel(got, want) <= tol(N), (seed, list(reps), gamma is None)


@pytest.mark.parametrize("d", [4, 8, 11, 12, 14])
def test_repetitions_two_match_oracle(eng, d):
    # the paper's (2, ..., 2) repetitions; d = 14 spans many wavefronts, inner
    # blocks and reflected segments
    A = workloads.gbs_matrix(d, d)
    g = workloads.loop_vector(d, d)
    reps = [2] * d
    for gamma in (g, None):
        want = oracle.lhaf_rep(A, gamma, reps)
        got = gpu_lhaf(eng, A, gamma, reps)
        assert rel(got, want) <= tol(2 * d), (d, gamma is None)


@pytest.mark.parametrize("n", [1, 7, 12, 16, 20])
def test_unit_repetitions_match_oracle(eng, n):
    A = workloads.symmetric_gaussian(n, 40 + n)
    g = workloads.loop_vector(n, 40 + n)
    want = oracle.lhaf_rep(A, g, [1] * n)
    assert rel(gpu_lhaf(eng, A, g, [1] * n), want) <= tol(n)


def test_reads_upper_triangle_and_leading_dimension(eng):
    # a non-symmetric matrix inside a wider buffer: the definition reads the
    # pairs i <= k only
    rng = np.random.default_rng(3)
    d, D = 7, 11
    big = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    g = workloads.loop_vector(d, 3)
    reps = [2, 0, 1, 3, 1, 2, 1]
    want = oracle.lhaf_rep(big[:d, :d], g, reps)
    out = eng.lhaf(dev(big)[:d, :d], dev(g), reps)
    torch.cuda.synchronize()
    assert rel(complex(out.cpu().numpy()[0]), want) <= 1e-10


def test_block_matrix_is_repeated_permanent_at_40_vertices(eng):
    # haf([[0, B], [B^T, 0]]) with repetitions (2, ..., 2): perm(B_{t,s}), t =
    # s = (2, ..., 2) on a 10 x 10 block, by the oracle's Ryser sum and by the
    # permanent engine
    B = workloads.collision_free_block(10, 5) * 3.0
    M = np.zeros((20, 20), np.complex128)
    M[:10, 10:] = B
    M[10:, :10] = B.T
    s = np.full(10, 2, np.int32)
    want = oracle.perm_mult(B, s, s)
    got = gpu_lhaf(eng, M, None, [2] * 20)
    assert rel(got, want) <= tol(40)
    # zero loops take the loop path and change nothing
    assert rel(gpu_lhaf(eng, M, np.zeros(20), [2] * 20), want) <= tol(40)
    p, _ = eng.perm(dev(B), s, s)
    torch.cuda.synchronize()
    assert rel(got, complex(p.cpu().item())) <= tol(40)


def test_constant_matrix_hermite_form_at_40_vertices(eng):
    a, gv = 0.05 - 0.02j, 0.3 + 0.1j
    d = 20
    N = 2 * d
    want = sum(math.factorial(N) / (math.factorial(j) * math.factorial(N - 2 * j) * 2 ** j) * a ** j * gv ** (N - 2 * j)
               for j in range(N // 2 + 1))
    got = gpu_lhaf(eng, np.full((d, d), a), np.full(d, gv), [2] * d)
    assert rel(got, want) <= tol(N)
    want_haf = math.factorial(N) / (math.factorial(N // 2) * 2 ** (N // 2)) * a ** (N // 2)
    assert rel(gpu_lhaf(eng, np.full((d, d), a), None, [2] * d), want_haf) <= tol(N)


@pytest.mark.parametrize("d", [16, 20])
def test_scaling_and_permutation_at_full_size(eng, d):
    rng = np.random.default_rng(d)
    A = workloads.gbs_matrix(d, 7)
    g = workloads.loop_vector(d, 7)
    reps = np.full(d, 2)
    base = gpu_lhaf(eng, A, g, reps)
    D = np.exp(1j * rng.uniform(0, 2 * np.pi, d)) * rng.uniform(0.8, 1.25, d)
    scaled = gpu_lhaf(eng, D[:, None] * A * D[None, :], D * g, reps)
    assert rel(scaled, np.prod(D ** reps) * base) <= tol(2 * d)
    p = rng.permutation(d)
    assert rel(gpu_lhaf(eng, A[np.ix_(p, p)], g[p], reps[p]), base) <= tol(2 * d)


def test_special_cases(eng):
    A = workloads.gbs_matrix(5, 1)
    g = workloads.loop_vector(5, 1)
    assert gpu_lhaf(eng, A, g, [0] * 5) == 1
    assert gpu_lhaf(eng, A, None, [0, 1, 0, 2, 0]) == 0
    assert rel(gpu_lhaf(eng, A, g, [0, 0, 1, 0, 0]), g[2]) <= 1e-15
    assert rel(gpu_lhaf(eng, A, None, [0, 0, 0, 2, 0]), A[3, 3]) <= 1e-15
    assert rel(gpu_lhaf(eng, A, g, [1, 1, 0, 0, 0]), A[0, 1] + g[0] * g[1]) <= 1e-15


def test_deterministic(eng):
    A = workloads.gbs_matrix(16, 2)
    g = workloads.loop_vector(16, 2)
    a = eng.lhaf(dev(A), dev(g), [2] * 16)
    b = eng.lhaf(dev(A), dev(g), [2] * 16)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_argument_errors(eng):
    import paper_2403_04006_amd as pq
    A = dev(workloads.gbs_matrix(4, 0))
    with pytest.raises(pq.PqError):
        eng.lhaf(A, None, [1, -1, 0, 0])
    with pytest.raises(pq.PqError):
        eng.lhaf(A, None, [30, 30, 4, 2])          # N > 64
    with pytest.raises(pq.PqError):
        eng.lhaf(A, None, [2 ** 31 - 1, 1, 0, 0])  # no overflow in the vertex count
    big = dev(workloads.gbs_matrix(50, 0))
    with pytest.raises(pq.PqError):
        eng.lhaf(big, None, [1] * 50)              # more than 48 occupied modes
    with pytest.raises(pq.PqError):
        eng.lhaf(big, None, [1] * 42 + [0] * 8)    # 34 Gray-walked modes (N even)
    with pytest.raises(ValueError):
        eng.lhaf(A, None, [1, 1])


def test_gbs_photon_shells_match_squeezed_statistics(eng):
    # squeezed vacua through a Haar interferometer: p(t) = |haf(B_t)|^2 /
    # (prod t! prod cosh r), B = U diag(tanh r) U^T; a passive interferometer
    # keeps the total photon number, so each shell sum equals the convolution
    # of the single-mode squeezed distributions
    import itertools
    d = 4
    r = np.array([0.5, 0.3, 0.4, 0.6])
    U = workloads.haar(d, 4)
    B = (U * np.tanh(r)) @ U.T
    Bd = dev(B)
    nmax = 14
    want = np.zeros(nmax + 1)
    want[0] = 1.0
    for ri in r:
        single = np.zeros(nmax + 1)
        for k in range(nmax // 2 + 1):
            single[2 * k] = math.factorial(2 * k) / (2 ** k * math.factorial(k)) ** 2 * np.tanh(ri) ** (2 * k) / np.cosh(ri)
        want = np.convolve(want, single)[:nmax + 1]
    for N in range(0, nmax + 1, 2):
        pats = [t for t in itertools.product(range(N + 1), repeat=d) if sum(t) == N]
        outs = eng.lhaf_many(Bd, None, np.array(pats)).cpu().numpy()
        fact = np.array([math.prod(math.factorial(x) for x in t) for t in pats], dtype=np.float64)
        shell = float(np.sum(np.abs(outs) ** 2 / fact)) / float(np.prod(np.cosh(r)))
        assert abs(shell - want[N]) <= 1e-15 + 1e-12 * want[N], (N, shell, want[N])


def test_many_patterns_match_single_calls_and_oracle(eng):
    # uneven batch: trivial, odd, zero and (2, ..., 2) patterns, loops on
    # and off; every value equals its single call (up to the order of the
    # chunk sums) and, where small, the oracle
    rng = np.random.default_rng(77)
    d = 14
    A = workloads.gbs_matrix(d, 8)
    g = workloads.loop_vector(d, 8)
    pats = [np.zeros(d, np.int64), np.eye(d, dtype=np.int64)[3], np.full(d, 2)]
    for _ in range(37):
        v = rng.integers(0, 3, d)
        v[rng.random(d) < 0.4] = 0
        pats.append(v)
    pats = np.array(pats)
    for gamma in (g, None):
        many = eng.lhaf_many(dev(A), None if gamma is None else dev(gamma), pats).cpu().numpy()
        for q, v in enumerate(pats):
            single = gpu_lhaf(eng, A, gamma, v)
            N = int(v.sum())
            if gamma is None and N % 2:
                assert many[q] == 0 and single == 0
                continue
            assert rel(many[q], single) <= 1e-12, (q, list(v))
            if np.prod(v + 1) <= (1 << 16):
                assert rel(many[q], oracle.lhaf_rep(A, gamma, v)) <= tol(N), (q, list(v))


def test_many_argument_errors(eng):
    import paper_2403_04006_amd as pq
    A = dev(workloads.gbs_matrix(4, 0))
    assert eng.lhaf_many(A, None, np.zeros((0, 4), np.int32)).numel() == 0
    with pytest.raises(pq.PqError):
        eng.lhaf_many(A, None, np.array([[1, 1, 0, 0], [1, -1, 0, 0]]))
    with pytest.raises(ValueError):
        eng.lhaf_many(A, None, np.array([1, 1, 0, 0]))


def sum_condition(a, gv, reps, loops):
    # sum |w P| / |sum w P| of the vertex-sign sum on a constant matrix (the
    # cancellation the FP64 sum goes through; used for the error bound only)
    import itertools
    from math import comb
    d, N = len(reps), sum(reps)
    f = min((i for i in range(d) if reps[i] > 0), key=lambda i: reps[i])
    J = N // 2
    absum, tot = 0.0, 0j
    for digs in itertools.product(*[range(reps[i] if i == f else reps[i] + 1) if reps[i] else range(1)
                                    for i in range(d)]):
        S = sum(reps[i] - 2 * digs[i] for i in range(d) if reps[i])
        w = 1.0
        for i in range(d):
            if reps[i]:
                w *= (-1) ** digs[i] * comb(reps[i] - 1 if i == f else reps[i], digs[i])
        x, l = a * S * S / 2, gv * S
        if loops:
            P = sum(x ** j * l ** (N - 2 * j) / (math.factorial(j) * math.factorial(N - 2 * j)) for j in range(J + 1))
        else:
            P = x ** J / math.factorial(J)
        absum += abs(w * P)
        tot += w * P
    return absum / abs(tot)


@pytest.mark.parametrize("reps", [[32, 32], [1, 63], [20, 0, 44], [64], [8, 8, 8, 8]])
def test_largest_vertex_count(eng, reps):
    # N up to 64 (the limit) on few modes: radix-33, -45 and -64 digits, the
    # power x^32 (squarings only); constant matrix against the Hermite form.
    # The alternating sum cancels strongly here (condition ~1e11 at N = 64),
    # so the bound is the FP64 rounding of the sum times its condition.
    a, gv = 0.02 + 0.01j, 0.15 - 0.05j
    d = len(reps)
    N = sum(reps)
    want = sum(math.factorial(N) / (math.factorial(j) * math.factorial(N - 2 * j) * 2 ** j) * a ** j * gv ** (N - 2 * j)
               for j in range(N // 2 + 1))
    got = gpu_lhaf(eng, np.full((d, d), a), np.full(d, gv), reps)
    assert rel(got, want) <= 64 * 2.0 ** -52 * sum_condition(a, gv, reps, True)
    want_haf = math.factorial(N) / (math.factorial(N // 2) * 2 ** (N // 2)) * a ** (N // 2)
    got_haf = gpu_lhaf(eng, np.full((d, d), a), None, reps)
    assert rel(got_haf, want_haf) <= 64 * 2.0 ** -52 * sum_condition(a, gv, reps, False)


@pytest.mark.parametrize("N", range(1, 34))
def test_constant_matrix_every_vertex_count(eng, N):
    # every grouping of the loop polynomial's floor(N/2) Hermite factors (four
    # at a time, then a pair and a single) and both parities of N, on a
    # constant matrix against the closed form (matchings of the complete
    # graph); the bound is the larger of the size tolerance and the FP64
    # rounding of the vertex-sign sum times its condition
    a, gv = 0.04 - 0.03j, 0.2 + 0.15j
    reps = [N // 3, N // 3, N - 2 * (N // 3)]
    want = sum(math.factorial(N) / (math.factorial(j) * math.factorial(N - 2 * j) * 2 ** j) * a ** j * gv ** (N - 2 * j)
               for j in range(N // 2 + 1))
    got = gpu_lhaf(eng, np.full((3, 3), a), np.full(3, gv), reps)
    bound = max(tol(N), 64 * 2.0 ** -52 * sum_condition(a, gv, reps, True))
    assert rel(got, want) <= bound, (N, rel(got, want), bound)


def lane_plan(reps):
    """Lane states, time states and inner block of pq_lhaf's plan (the
    planner's digit rules restated for choosing test cases)."""
    r = [x for x in reps if x > 0]
    f = int(np.argmin(r))
    rho = [x if i == f else x + 1 for i, x in enumerate(r)]
    order = sorted(range(len(r)), key=lambda i: (rho[i] != 1, -rho[i]))
    lane, prod, big = set(), 1, 0
    for i in order:
        if rho[i] == 1:
            lane.add(i)
        elif big < 6 and prod * rho[i] <= 64:
            lane.add(i)
            prod *= rho[i]
            big += 1
    rest = [i for i in range(len(r)) if i not in lane]
    reg = next((i for want in (3, 2) for i in rest if rho[i] == want), None)
    time = [rho[i] for i in rest if i != reg]
    ts, M = 1, 1
    for x in time:
        ts *= x
    for x in time:
        if M * x > 2048:
            break
        M *= x
    return prod, ts, M


@pytest.mark.parametrize("reps", [[2] * 14, [4, 4] + [2] * 10, [5, 5] + [1] * 16, [3, 3, 2] + [1] * 16])
def test_lane_packing_matches_unpacked_and_oracle(eng, reps):
    # between 33 and 63 lane states the idle lanes run a second Gray segment
    # of the same parity: 54, 50, 36 and 48 lane states, several segments of
    # each parity, full groups and leftover segments; the packed sweep
    # against the oracle, and against the unpacked one (the same terms added
    # in another order: they differ by the rounding of a sum that cancels to
    # about 1e-3 of its terms here, a few 1e-12 relative)
    L, ts, M = lane_plan(reps)
    assert 32 < L < 64 and ts // M >= 4, (L, ts, M)
    d = len(reps)
    A = workloads.gbs_matrix(d, d + 3)
    g = workloads.loop_vector(d, d + 3)
    N = sum(reps)
    try:
        for gamma in (g, None):
            eng.lhaf_pack("always")
            packed = gpu_lhaf(eng, A, gamma, reps)
            eng.lhaf_pack("never")
            plain = gpu_lhaf(eng, A, gamma, reps)
            assert rel(packed, plain) <= 1e-10, (reps, gamma is None)
            assert rel(packed, oracle.lhaf_rep(A, gamma, reps)) <= tol(N), (reps, gamma is None)
    finally:
        eng.lhaf_pack("auto")


def test_lane_packing_rejects_unknown_modes(eng):
    from paper_2403_04006_amd import _lib
    assert eng._lib.pq_lhaf_pack(eng._ctx, 3) == _lib.PQ_EINVAL
    assert eng._lib.pq_lhaf_pack(eng._ctx, -1) == _lib.PQ_EINVAL
    with pytest.raises(KeyError):
        eng.lhaf_pack("sometimes")
    eng.lhaf_pack("auto")
