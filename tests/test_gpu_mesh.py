"""Differentiable circuit path on the GPU: beamsplitter mesh, permanents of
many patterns, the sampling loss, and gradients to the mesh angles, against
the oracle and central finite differences."""
import math

import numpy as np
import pytest

import oracle
from tests.tolerance import assert_entries_close
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ag():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_04006_amd.autograd as ag
    return ag


CELLS = workloads.MESH_CELLS
M = workloads.MESH_MODES


def test_mesh_forward_matches_oracle(ag):
    ang = workloads.mesh_angles(0)
    U = ag.mesh_unitary(torch.from_numpy(ang).cuda(), CELLS, M).cpu().numpy()
    ref = oracle.mesh_unitary(ang, CELLS, M)
    assert np.max(np.abs(U - ref)) < 1e-13
    assert np.max(np.abs(U @ U.conj().T - np.eye(M))) < 1e-13


def test_mesh_vjp_matches_oracle_jacobian(ag):
    ang = workloads.mesh_angles(3)
    rng = np.random.default_rng(1)
    gU = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    a = torch.from_numpy(ang).cuda().requires_grad_(True)
    U = ag.mesh_unitary(a, CELLS, M)
    U.backward(torch.from_numpy(gU).cuda())
    got = a.grad.cpu().numpy()
    J = oracle.mesh_jacobian(ang, CELLS, M)
    want = np.real(np.einsum("ab,qkab->qk", np.conj(gU), J))
    assert np.max(np.abs(got - want)) < 1e-11 * max(1.0, np.max(np.abs(want)))


def test_loss_and_its_gradient(ag):
    rng = np.random.default_rng(2)
    perm = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    ln = rng.uniform(0, 3, 300)
    p = torch.from_numpy(perm).cuda().requires_grad_(True)
    loss = ag.neg_log_prob(p, torch.from_numpy(ln).cuda())
    want = -np.mean(np.log(np.abs(perm) ** 2) - ln)
    assert abs(loss.item() - want) < 1e-14 * max(1.0, abs(want))
    loss.backward()
    assert np.max(np.abs(p.grad.cpu().numpy() - (-2.0 / 300) / np.conj(perm))) < 1e-14


def test_permamp_gradcheck_small(ag):
    U0 = workloads.haar(4, 3)
    S = [np.array([1, 2, 0, 1], np.int32), np.array([1, 1, 1, 0], np.int32)]
    T = [np.array([2, 0, 1, 1], np.int32), np.array([0, 1, 1, 1], np.int32)]
    U = torch.from_numpy(U0).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda X: ag.perm_amp(X, S, T), (U,), eps=1e-6, atol=1e-8, rtol=1e-6)


def _c5_inputs(npat):
    ang = workloads.mesh_angles(0)
    S = np.zeros(M, np.int32)
    S[:8] = 1
    pats = list(workloads.mesh_patterns(count=npat, seed=1))
    return ang, S, pats


def test_mesh_training_step_vs_oracle(ag):
    ang, S, pats = _c5_inputs(256)
    a = torch.from_numpy(ang).cuda().requires_grad_(True)
    loss = ag.mesh_loss(a, CELLS, M, S, pats)
    loss.backward()
    got_l = loss.item()
    got_g = a.grad.cpu().numpy()
    U = oracle.mesh_unitary(ang, CELLS, M)
    want_l = oracle.mesh_loss(U, S, pats)
    want_g = oracle.mesh_loss_grad(ang, CELLS, M, S, pats)
    assert abs(got_l - want_l) < 1e-12 * abs(want_l)
    # every angle's derivative is a sum over the patterns: each is compared
    # by its own relative error, with a floor of the same 1e-10 times the
    # sum of the patterns' contributions' magnitudes (where they cancel; 1.3
    # to 250 times the derivative here), and for the 8 derivatives that are
    # exactly 0 (cells whose action reaches only the columns of the empty
    # input modes 8..11, which no permanent reads) the rounding of the mesh
    # itself, 1e-14 of the largest
    J = oracle.mesh_jacobian(ang, CELLS, M)
    scale = np.zeros_like(want_g)
    for T in pats:
        p = oracle.perm_mult(U, S, T)
        scale += np.abs(np.real(np.einsum("ab,qkab->qk", oracle.perm_grad(U, S, T), J) / p))
    scale *= 2.0 / len(pats)
    floor = 1e-10 * scale + 1e-14 * np.max(np.abs(want_g))
    err = assert_entries_close(got_g, want_g, 1e-10, floor, "mesh gradient")
    print(f"mesh gradient vs oracle: max rel err {err:.2e}")


def test_mesh_training_step_vs_finite_differences(ag):
    # the full 4096-pattern workload; central differences, h = 1e-6, all 132 angles
    import paper_2403_04006_amd as pq
    ang, S, T_list = _c5_inputs(4096)
    pats = pq.PatternSet([S] * len(T_list), T_list, M)
    a = torch.from_numpy(ang).cuda().requires_grad_(True)
    loss = ag.mesh_loss(a, CELLS, M, pats)
    loss.backward()
    g = a.grad.cpu().numpy()
    h = 1e-6
    worst = 0.0
    with torch.no_grad():
        for q in range(ang.shape[0]):
            for k in range(2):
                a1 = ang.copy(); a1[q, k] += h
                a0 = ang.copy(); a0[q, k] -= h
                l1 = ag.mesh_loss(torch.from_numpy(a1).cuda(), CELLS, M, pats).item()
                l0 = ag.mesh_loss(torch.from_numpy(a0).cuda(), CELLS, M, pats).item()
                fd = (l1 - l0) / (2 * h)
                worst = max(worst, abs(fd - g[q, k]) / max(1.0, abs(g[q, k])))
    print(f"mesh gradient vs central differences: worst scaled err {worst:.2e}")
    assert worst < 1e-6
