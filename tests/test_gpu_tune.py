"""Chunk-size autotuning of the many-pattern path (pq_autotune_enable /
pq_autotune_last): tuned plans give the untuned outputs (up to the order of
the partial sums) and the oracle's, the kept policy is never slower than the
default one it was timed against, and a job list of the same shape reuses the
recorded policy without timing again."""
import numpy as np
import pytest

import oracle
import workloads
from tests.tolerance import assert_entries_close, extend_floor

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.fixture(scope="module")
def engines():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_04006_amd as pq
    tuned, plain = pq.Engine(0), pq.Engine(0)
    tuned.autotune(True)
    return tuned, plain


def dev(U):
    return torch.from_numpy(np.ascontiguousarray(U, dtype=np.complex128)).cuda()


def extend_jobs(samples, seed, photons=12, modes=60):
    # Clifford-Clifford-shaped EXTEND_ROW jobs: k - 1 drawn rows, first k
    # ordered input columns, k = 2..photons
    cols, rows = workloads.sampling_jobs(samples=samples, photons=photons, modes=modes, seed=seed)
    jobs, off = [], 0
    for s in range(samples):
        for k in range(2, photons + 1):
            rc = np.bincount(rows[s, :k - 1], minlength=modes)
            cc = np.bincount(cols[s, :k], minlength=modes)
            jobs.append({"op": 1, "rows": [(i, int(c)) for i, c in enumerate(rc) if c],
                         "cols": [(i, int(c)) for i, c in enumerate(cc) if c], "out": off})
            off += modes
    return jobs, off, cols, rows


def test_tuned_plan_matches_default_and_oracle(engines):
    tuned, plain = engines
    modes = 60
    U = workloads.haar(modes, 21)
    jobs, n_out, cols, rows = extend_jobs(40, 1)
    got, _ = tuned.perm_many(dev(U), jobs, n_out=n_out, with_amp=False)
    info = tuned.autotune_last()
    ref, _ = plain.perm_many(dev(U), jobs, n_out=n_out, with_amp=False)
    torch.cuda.synchronize()
    got, ref = got.cpu().numpy(), ref.cpu().numpy()
    assert info["candidates"] == 14
    assert 0 < info["best_ms"] <= info["default_ms"]
    assert (info["waves_per_cu"], info["chunks_per_wave"], info["min_chunk"]) in {
        (64, 8, 256), (16, 4, 64), (4, 2, 64), (8, 1, 64), (8, 2, 64), (8, 4, 64), (16, 2, 64), (16, 8, 64), (32, 4, 64),
        (32, 8, 64), (8, 2, 256), (16, 4, 256), (32, 8, 32), (64, 8, 32)}
    # tuned and default plans differ only in the order of the partial sums
    assert_entries_close(got, ref, 1e-12, np.concatenate([extend_floor(U, j) for j in jobs]), "tuned vs default")
    # a few extend-row outputs against the oracle's Laplace expansion
    for s, k in ((0, 12), (7, 9), (39, 12)):
        want = oracle.extend_row(U, list(rows[s, :k - 1]), list(cols[s, :k]))
        j = s * 11 + (k - 2)
        blk = got[j * modes:(j + 1) * modes]
        assert_entries_close(blk, want, 1e-10, extend_floor(U, jobs[j]), f"job {j}")
    # a repeated call reuses the kept plan
    again, _ = tuned.perm_many(dev(U), jobs, n_out=n_out, with_amp=False)
    torch.cuda.synchronize()
    assert np.array_equal(again.cpu().numpy(), got)


def test_same_shape_reuses_recorded_policy(engines):
    tuned, plain = engines
    modes = 60
    U = workloads.haar(modes, 22)
    jobs, n_out, _, _ = extend_jobs(40, 2)     # other draws, same shapes
    first = tuned.autotune_last()
    got, _ = tuned.perm_many(dev(U), jobs, n_out=n_out, with_amp=False)
    info = tuned.autotune_last()
    ref, _ = plain.perm_many(dev(U), jobs, n_out=n_out, with_amp=False)
    torch.cuda.synchronize()
    assert info["candidates"] == 0
    assert (info["waves_per_cu"], info["chunks_per_wave"], info["min_chunk"]) == (
        first["waves_per_cu"], first["chunks_per_wave"], first["min_chunk"])
    got, ref = got.cpu().numpy(), ref.cpu().numpy()
    assert_entries_close(got, ref, 1e-12, np.concatenate([extend_floor(U, j) for j in jobs]), "reused policy")


def test_tuning_repeated_permanents(engines):
    # uneven PERM jobs with repeated rows and columns
    tuned, plain = engines
    rng = np.random.default_rng(5)
    m = 12
    U = workloads.haar(m, 23)
    jobs, refs = [], []
    for k in range(48):
        n = int(rng.integers(6, 19))
        S = workloads.random_occupations(rng, m, n, cap=3)
        T = workloads.random_occupations(rng, m, n, cap=3)
        jobs.append({"op": 0, "rows": [(i, int(c)) for i, c in enumerate(T) if c],
                     "cols": [(i, int(c)) for i, c in enumerate(S) if c]})
        if k < 6:
            refs.append((k, oracle.perm_mult(U, S, T)))
    got, _ = tuned.perm_many(dev(U), jobs)
    info = tuned.autotune_last()
    ref, _ = plain.perm_many(dev(U), jobs)
    torch.cuda.synchronize()
    got, ref = got.cpu().numpy(), ref.cpu().numpy()
    assert info["candidates"] == 14 and info["best_ms"] <= info["default_ms"]
    for k in range(len(jobs)):
        assert rel(got[k], ref[k]) <= 1e-12
    for k, want in refs:
        assert rel(got[k], want) <= 1e-10


def test_graph_replays_match_direct_launches():
    # captured launch sequence replayed with the program's own GPU work and
    # synchronizations in between; every replay equals the direct launches
    # bit for bit (same plan, same kernels)
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_04006_amd as pq
    graph, plain = pq.Engine(0), pq.Engine(0)
    graph.graphs(True)
    modes = 60
    U = dev(workloads.haar(modes, 24))
    jobs, n_out, _, _ = extend_jobs(30, 3)
    ref, _ = plain.perm_many(U, jobs, n_out=n_out, with_amp=False)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    out = torch.empty(n_out, dtype=torch.complex128, device="cuda")
    x = torch.randn(256, 256, dtype=torch.float64, device="cuda")
    for rep in range(4):
        out.fill_(-1.0)
        torch.cuda.synchronize()
        graph.perm_many(U, jobs, n_out=n_out, with_amp=False, out=(out, None))
        y = x @ x                                   # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), rep
        assert torch.isfinite(y).all()
    # other output buffers: a second captured graph, same values
    out2 = torch.empty(n_out, dtype=torch.complex128, device="cuda")
    graph.perm_many(U, jobs, n_out=n_out, with_amp=False, out=(out2, None))
    torch.cuda.synchronize()
    assert np.array_equal(out2.cpu().numpy(), ref)
    graph.close()
    plain.close()


def test_no_decision_reads_as_zero():
    # a ctx that has tuned nothing reports no policy
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_04006_amd as pq
    fresh = pq.Engine(0)
    try:
        info = fresh.autotune_last()
    finally:
        fresh.close()
    assert (info["waves_per_cu"], info["chunks_per_wave"], info["min_chunk"]) == (0, 0, 0)
    assert info["best_ms"] == 0.0 and info["default_ms"] == 0.0 and info["candidates"] == 0


def test_perm_launch_shape_is_tuned_per_shape(engines):
    # pq_perm under the autotuner: 2, 1 and 4 rounds of the resident
    # wavefronts are timed once per plan shape (n and multiplicity class);
    # the kept shape sums the same terms in another partition
    tuned, plain = engines
    n = 24
    ones = [1] * n
    A = workloads.collision_free_block(n, 11)
    got, _ = tuned.perm(dev(A), ones, ones)
    info = tuned.autotune_last()
    ref, _ = plain.perm(dev(A), ones, ones)
    torch.cuda.synchronize()
    assert info["candidates"] == 3 and 0 < info["best_ms"] <= info["default_ms"]
    assert info["waves_per_cu"] > 0 and info["chunks_per_wave"] == 1 and info["min_chunk"] == 32
    assert rel(complex(got.item()), complex(ref.item())) <= 1e-12
    want = oracle.perm_ryser(A)
    assert rel(complex(got.item()), want) <= 1e-8
    # another matrix of the same shape reuses the decision
    B = workloads.collision_free_block(n, 12)
    got2, _ = tuned.perm(dev(B), ones, ones)
    info2 = tuned.autotune_last()
    torch.cuda.synchronize()
    assert info2["candidates"] == 0 and info2["waves_per_cu"] == info["waves_per_cu"]
    assert rel(complex(got2.item()), oracle.perm_ryser(B)) <= 1e-8
    # a shape with repeated rows and columns gets a decision of its own
    V = workloads.haar(8, 13)
    S = [2, 0, 3, 1, 0, 2, 1, 1]
    T = [1, 2, 1, 1, 2, 0, 2, 1]
    got3, _ = tuned.perm(dev(V), S, T)
    info3 = tuned.autotune_last()
    torch.cuda.synchronize()
    assert info3["candidates"] == 3
    assert rel(complex(got3.item()), oracle.perm_mult(V, S, T)) <= 1e-10


def test_noalloc_follows_the_recorded_launch_shape(engines):
    # after tuning, pq_perm and pq_perm_noalloc on that ctx run the same
    # launch shape, so they give the same bits
    import ctypes
    tuned, _ = engines
    n = 22
    ones = (ctypes.c_int32 * n)(*([1] * n))
    U = dev(workloads.collision_free_block(n, 14))
    a, _ = tuned.perm(U, [1] * n, [1] * n)
    lib = tuned._lib
    out = torch.empty(2, dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    st = lib.pq_perm_noalloc(tuned._ctx, U.data_ptr(), U.stride(0), n, ones, ones, out.data_ptr(), None,
                             torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == 0
    assert complex(out[0].item()) == complex(a.item())
