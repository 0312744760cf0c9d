"""Every output amplitude of one input pattern (pq_perm_all_outputs) against
the oracle's amplitude of each output, and completeness of the output
distribution, in both of its forms (the sweep, and the contraction on matrix
products), and the two forms against each other at the benchmark size."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def engine():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_04006_amd as pq
    return pq.Engine(0)


@pytest.fixture(params=["never", "always"])
def eng(engine, request):
    # each test in the sweep form and in the contraction form
    engine.all_outputs_gemm(request.param)
    yield engine
    engine.all_outputs_gemm("auto")


def dev(U):
    return torch.from_numpy(np.ascontiguousarray(U, dtype=np.complex128)).cuda()


@pytest.mark.parametrize("S,seed", [
    ([2, 0, 1, 1, 0, 1], 0),          # repeated input mode (fixed group has occupation 1)
    ([0, 3, 0, 2, 0, 0], 1),          # all inputs repeated
    ([1, 1, 1, 1, 1, 0], 2),          # collision-free
])
def test_all_outputs_match_oracle(eng, S, seed):
    m = len(S)
    n = sum(S)
    U = workloads.haar(m, 70 + seed)
    perm, amp = eng.perm_all_outputs(dev(U), S)
    perm = perm.cpu().numpy()
    amp = amp.cpu().numpy()
    outs = workloads.fock_outputs(m, n)
    assert perm.shape == (len(outs),)
    for k, T in enumerate(outs):
        rp = oracle.perm_mult(U, np.array(S, np.int32), T)
        ra = oracle.amplitude(U, np.array(S, np.int32), T)
        assert abs(perm[k] - rp) <= 1e-10 * max(abs(rp), 1e-300) or abs(rp) < 1e-15, (k, T)
        assert abs(amp[k] - ra) <= 1e-12, (k, T)
    assert abs(np.sum(np.abs(amp) ** 2) - 1.0) < 1e-12


def test_completeness_four_photons_in_eight_modes(eng):
    # the 330 outputs with exactly 4 photons (input modes 0-3)
    U = workloads.haar(8, 1)
    S = [1, 1, 1, 1, 0, 0, 0, 0]
    _, amp = eng.perm_all_outputs(dev(U), S)
    amp = amp.cpu().numpy()
    assert amp.shape == (330,)
    assert abs(np.sum(np.abs(amp) ** 2) - 1.0) < 1e-12
    outs = workloads.fock_outputs(8, 4)
    for k in range(0, 330, 37):
        assert abs(amp[k] - oracle.amplitude(U, np.array(S, np.int32), outs[k])) < 1e-13


def test_completeness_with_repeats_larger(eng):
    # 7 photons, repeated inputs, 10 modes: 11440 outputs
    U = workloads.haar(10, 5)
    S = [2, 0, 1, 0, 3, 0, 0, 1, 0, 0]
    _, amp = eng.perm_all_outputs(dev(U), S)
    amp = amp.cpu().numpy()
    assert amp.shape == (11440,)
    assert abs(np.sum(np.abs(amp) ** 2) - 1.0) < 1e-12


def test_mesh_sized_all_outputs(eng):
    # 8 photons in the 12-mode mesh: all 75582 outputs, sampled against the oracle
    import paper_2403_04006_amd as pq
    U = oracle.mesh_unitary(workloads.mesh_angles(0), workloads.MESH_CELLS, workloads.MESH_MODES)
    S = [1] * 8 + [0] * 4
    perm, amp = eng.perm_all_outputs(dev(U), S)
    amp = amp.cpu().numpy()
    perm = perm.cpu().numpy()
    assert amp.shape == (75582,)
    assert abs(np.sum(np.abs(amp) ** 2) - 1.0) < 1e-11
    rng = np.random.default_rng(3)
    for r in rng.choice(75582, 24, replace=False):
        T = np.array(pq.fock_unrank(12, 8, int(r)), np.int32)
        rp = oracle.perm_mult(U, np.array(S, np.int32), T)
        assert abs(perm[r] - rp) <= 1e-10 * max(abs(rp), 1e-300) or abs(rp) < 1e-15


def test_vacuum_and_single_photon(eng):
    U = workloads.haar(5, 9)
    perm, amp = eng.perm_all_outputs(dev(U), [0, 0, 0, 0, 0])
    assert perm.cpu().numpy().tolist() == [1.0 + 0j] and amp.cpu().numpy().tolist() == [1.0 + 0j]
    perm, _ = eng.perm_all_outputs(dev(U), [0, 0, 1, 0, 0])
    # n = 1: outputs e_4, e_3, ..., e_0 in that order
    assert np.max(np.abs(perm.cpu().numpy() - U[::-1, 2])) < 1e-15


def test_argument_errors(eng):
    import paper_2403_04006_amd as pq
    U = dev(workloads.haar(4, 0))
    with pytest.raises(pq.PqError):
        eng.perm_all_outputs(U, [1, -1, 0, 0])
    with pytest.raises(ValueError):
        eng.perm_all_outputs(U, [1, 0, 0])
    big = dev(workloads.haar(40, 0))
    with pytest.raises(pq.PqError):
        eng.perm_all_outputs(big, [1] * 20 + [0] * 20)    # C(59, 20) outputs


def compositions_array(m, n):
    """Every occupation vector with n photons on m modes, in ascending
    lexicographic order (the output order), as rows of an array."""
    from functools import lru_cache

    @lru_cache(maxsize=None)
    def rec(q, k):
        if q == 1:
            return np.array([[k]], np.uint8)
        parts = []
        for v in range(k + 1):
            sub = rec(q - 1, k - v)
            parts.append(np.hstack([np.full((len(sub), 1), v, np.uint8), sub]))
        return np.vstack(parts)

    return rec(m, n)


def test_compositions_array_is_the_output_order():
    # against the enumeration the other tests use, where that one is small
    for m, n in ((4, 3), (5, 4), (3, 6)):
        want = np.array(workloads.fock_outputs(m, n))
        assert np.array_equal(compositions_array(m, n), want)


def test_forms_agree_at_benchmark_size(engine):
    # 10 photons in 16 modes (3,268,760 outputs, 512 terms): the contraction
    # against the sweep on every output, each within 1e-10 of its own size or
    # the rounding floor of its Gray-code sum, and a sample against the oracle
    from tests.tolerance import FLOOR_C, EPS
    import paper_2403_04006_amd as pq
    m, n = 16, 10
    U = workloads.haar(m, 1)
    S = [1] * n + [0] * (m - n)
    out = {}
    for form in ("never", "always"):
        engine.all_outputs_gemm(form)
        perm, amp = engine.perm_all_outputs(dev(U), S)
        out[form] = (perm.cpu().numpy(), amp.cpu().numpy())
    engine.all_outputs_gemm("auto")
    p_sweep, a_sweep = out["never"]
    p_gemm, a_gemm = out["always"]
    assert p_gemm.shape == (3268760,)
    # every output's term scale: prod over input columns j of
    # sqrt(sum_i t_i |U_ij|^2), the occupation vectors in output order
    T = compositions_array(m, n).astype(np.float64)
    assert T.shape == (3268760, m)
    col = T @ (np.abs(U[:, :n]) ** 2)
    scale = np.prod(np.sqrt(col), axis=1)
    floor = FLOOR_C * (n + 1) * EPS * scale
    err = np.abs(p_gemm - p_sweep)
    assert np.all(err <= np.maximum(1e-10 * np.abs(p_sweep), floor)), float(np.max(err / np.maximum(1e-10 * np.abs(p_sweep), floor)))
    assert abs(np.sum(np.abs(a_gemm) ** 2) - 1.0) < 1e-11
    rng = np.random.default_rng(5)
    for r in rng.choice(3268760, 16, replace=False):
        Tr = np.array(pq.fock_unrank(m, n, int(r)), np.int32)
        rp = oracle.perm_mult(U, np.array(S, np.int32), Tr)
        assert abs(p_gemm[r] - rp) <= max(1e-10 * abs(rp), floor[r]), (int(r), p_gemm[r], rp)


def test_form_mode_rejects_unknown_modes(engine):
    from paper_2403_04006_amd import _lib
    assert engine._lib.pq_all_outputs_gemm(engine._ctx, 3) == _lib.PQ_EINVAL
    with pytest.raises(KeyError):
        engine.all_outputs_gemm("sometimes")
    engine.all_outputs_gemm("auto")
