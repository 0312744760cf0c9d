"""Runtime services of the C ABI on the device: fault injection (the status
propagates and the ctx stays usable), cancellation of the work queue,
autotuning decisions persisted to a file, and the device's reported peak."""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_04006_amd as pq_
    return pq_


def dev(U):
    return torch.from_numpy(np.ascontiguousarray(U, dtype=np.complex128)).cuda()


def perm_job(S, T, out):
    return {"op": 0, "rows": [(i, int(c)) for i, c in enumerate(T) if c],
            "cols": [(i, int(c)) for i, c in enumerate(S) if c], "out": out}


def test_injected_faults_propagate_and_the_ctx_recovers(pq):
    eng = pq.Engine(0)
    U = workloads.haar(8, 3)
    S = [1, 1, 0, 2, 0, 1, 0, 0]
    T = [0, 1, 1, 1, 1, 0, 1, 0]
    ref = oracle.perm_mult(U, S, T)
    eng.fault_inject(pq._lib.PQ_FAULT_LAUNCH)
    with pytest.raises(pq.PqError) as ei:
        eng.perm(dev(U), S, T)
    assert ei.value.status == pq._lib.PQ_EDEVICE and "injected" in str(ei.value)
    eng.fault_inject(pq._lib.PQ_FAULT_NONE)
    p, _ = eng.perm(dev(U), S, T)
    assert abs(complex(p.item()) - ref) <= 1e-12 * abs(ref)
    # an allocation failure while planning a new job list, then the same list again
    rng = np.random.default_rng(5)
    jobs = [perm_job(workloads.random_occupations(rng, 8, 6, cap=2), workloads.random_occupations(rng, 8, 6, cap=2), k)
            for k in range(10)]
    eng.fault_inject(pq._lib.PQ_FAULT_ALLOC)
    with pytest.raises(pq.PqError) as ei:
        eng.perm_many(dev(U), jobs)
    assert ei.value.status == pq._lib.PQ_ENOMEM and "injected" in str(ei.value)
    eng.fault_inject(pq._lib.PQ_FAULT_NONE)
    out, _ = eng.perm_many(dev(U), jobs)
    out = out.cpu().numpy()
    for k, j in enumerate(jobs):
        S_ = np.zeros(8, np.int32)
        T_ = np.zeros(8, np.int32)
        for i, c in j["cols"]:
            S_[i] = c
        for i, c in j["rows"]:
            T_[i] = c
        r = oracle.perm_mult(U, S_, T_)
        assert abs(out[k] - r) <= 1e-12 * max(1.0, abs(r))
    with pytest.raises(pq.PqError):
        eng.fault_inject(7)
    eng.close()


def test_cancel_stops_the_queue_and_refuses_work_until_cleared(pq):
    eng = pq.Engine(0)
    U = dev(workloads.haar(20, 0))
    pats = workloads.repeated_patterns(count=64, seed=1)
    jobs = pq.JobSet([perm_job(S, T, k) for k, (S, T) in enumerate(pats)], 20)
    full, _ = eng.perm_many(U, jobs, with_amp=False)
    torch.cuda.synchronize()
    # time of the uncancelled queue (about 25 ms of sweeps)
    out = torch.full((64,), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    eng.perm_batched(U, jobs, with_amp=False, out=(out, None))
    torch.cuda.synchronize()
    assert torch.equal(out, full)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    eng.perm_batched(U, jobs, with_amp=False, out=(out, None))
    e1.record()
    torch.cuda.synchronize()
    t_full = e0.elapsed_time(e1)
    # the same batch, cancelled right after it is enqueued
    out.fill_(complex(np.nan, np.nan))
    e0.record()
    eng.perm_batched(U, jobs, with_amp=False, out=(out, None))
    eng.cancel(True)
    e1.record()
    torch.cuda.synchronize()
    t_cut = e0.elapsed_time(e1)
    print(f"queue: {t_full:.2f} ms, cancelled: {t_cut:.2f} ms", flush=True)
    got = out.cpu().numpy()
    done = ~np.isnan(got)
    assert np.array_equal(got[done], full.cpu().numpy()[done])     # finished jobs are exact
    assert t_cut < 0.8 * t_full
    with pytest.raises(pq.PqError) as ei:
        eng.perm_batched(U, jobs, with_amp=False, out=(out, None))
    assert ei.value.status == pq._lib.PQ_ECANCELLED
    with pytest.raises(pq.PqError) as ei:
        eng.perm(U, [1] + [0] * 19, [1] + [0] * 19)
    assert ei.value.status == pq._lib.PQ_ECANCELLED
    eng.cancel(False)
    eng.perm_batched(U, jobs, with_amp=False, out=(out, None))
    torch.cuda.synchronize()
    assert torch.equal(out, full)
    eng.close()


def test_autotune_decisions_persist_in_the_cache_file(pq, tmp_path, monkeypatch):
    path = tmp_path / "tune.jsonl"
    monkeypatch.setenv("PQ_AUTOTUNE_CACHE", str(path))
    monkeypatch.setenv("PQ_AUTOTUNE", "1")
    U = dev(workloads.haar(60, 21))
    cols, rows = workloads.sampling_jobs(samples=12, photons=10, modes=60, seed=8)
    jobs, off = [], 0
    for s in range(12):
        for k in range(2, 11):
            rc = np.bincount(rows[s, :k - 1], minlength=60)
            cc = np.bincount(cols[s, :k], minlength=60)
            jobs.append({"op": 1, "rows": [(i, int(c)) for i, c in enumerate(rc) if c],
                         "cols": [(i, int(c)) for i, c in enumerate(cc) if c], "out": off})
            off += 60
    first = pq.Engine(0)
    a, _ = first.perm_many(U, jobs, n_out=off, with_amp=False)
    info = first.autotune_last()
    first.close()
    assert info["candidates"] == 14
    lines = path.read_text().strip().splitlines()
    assert len(lines) == 1 and '"kind": "many"' in lines[0] and '"device": "gfx' in lines[0]
    # a new ctx (as a new process would) reads the decision: no timing runs
    second = pq.Engine(0)
    b, _ = second.perm_many(U, jobs, n_out=off, with_amp=False)
    info2 = second.autotune_last()
    second.close()
    assert info2["candidates"] == 0
    assert [info2["waves_per_cu"], info2["chunks_per_wave"], info2["min_chunk"]] == \
        [info["waves_per_cu"], info["chunks_per_wave"], info["min_chunk"]]
    assert torch.equal(a, b)
    # pq_perm's launch-shape decisions go to the same file (kind "perm")
    Ub = dev(workloads.collision_free_block(20, 5))
    ones = [1] * 20
    third = pq.Engine(0)
    p3, _ = third.perm(Ub, ones, ones)
    info3 = third.autotune_last()
    third.close()
    assert info3["candidates"] == 3
    lines = path.read_text().strip().splitlines()
    assert len(lines) == 2 and '"kind": "perm"' in lines[1]
    fourth = pq.Engine(0)
    p4, _ = fourth.perm(Ub, ones, ones)
    info4 = fourth.autotune_last()
    fourth.close()
    assert info4["candidates"] == 0 and info4["waves_per_cu"] == info3["waves_per_cu"]
    assert torch.equal(p3, p4)


def test_device_peak_matches_the_runtime_properties(pq):
    # the CU count and peak clock of torch's view of the same device, and the
    # FP64 vector peak as CUs x clock x 128 flops
    eng = pq.Engine(0)
    d = eng.device_peak()
    props = torch.cuda.get_device_properties(0)
    assert d["cus"] == props.multi_processor_count
    assert 500.0 <= d["clock_mhz"] <= 5000.0
    assert d["fp64_vector_peak_tflops"] == pytest.approx(d["cus"] * d["clock_mhz"] * 1e6 * 128 / 1e12)
    eng.close()
