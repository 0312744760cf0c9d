"""The allocation-free entry point (pq_perm_noalloc) against pq_perm, called
through the C ABI: two calls in a row, the second on a smaller input, each
equal to pq_perm's value (same kernels, same launch geometry) and to the
oracle's; a permanent too large for the static scratch is refused."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run(lib, ctx, fn, U, S, T):
    m = U.shape[0]
    perm = torch.full((1,), complex(7.0, 7.0), dtype=torch.complex128, device="cuda")
    amp = torch.full((1,), complex(7.0, 7.0), dtype=torch.complex128, device="cuda")
    Sa = (ctypes.c_int32 * m)(*[int(v) for v in S])
    Ta = (ctypes.c_int32 * m)(*[int(v) for v in T])
    st = getattr(lib, fn)(ctx, U.data_ptr(), U.stride(0), m, Sa, Ta, perm.data_ptr(), amp.data_ptr(),
                          torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return st, complex(perm.cpu()[0]), complex(amp.cpu()[0])


def test_noalloc_matches_pq_perm_on_two_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_04006_amd as pq
    lib = pq._lib.load()
    ctx = ctypes.c_void_p()
    assert lib.pq_create(ctypes.byref(ctx), 0) == 0
    try:
        # first call: n = 24 collision-free block (binary walk)
        A = workloads.collision_free_block(24, 3)
        U1 = torch.from_numpy(A).cuda()
        ones = [1] * 24
        print("noalloc: call 1, n=24 collision-free", flush=True)
        st, p1, a1 = _run(lib, ctx, "pq_perm_noalloc", U1, ones, ones)
        assert st == 0, lib.pq_last_error(ctx).decode()
        st, q1, b1 = _run(lib, ctx, "pq_perm", U1, ones, ones)
        assert st == 0
        assert p1 == q1 and a1 == b1
        ref1 = oracle.perm_ryser(A)
        assert abs(p1 - ref1) <= 1e-8 * abs(ref1)
        # second call, smaller and with repeated rows and columns (mixed radices)
        V = workloads.haar(7, 8)
        S = [2, 0, 1, 3, 0, 1, 1]
        T = [1, 2, 2, 0, 1, 1, 1]
        U2 = torch.from_numpy(V).cuda()
        print("noalloc: call 2, 8 photons with repeats in 7 modes", flush=True)
        st, p2, a2 = _run(lib, ctx, "pq_perm_noalloc", U2, S, T)
        assert st == 0, lib.pq_last_error(ctx).decode()
        st, q2, b2 = _run(lib, ctx, "pq_perm", U2, S, T)
        assert st == 0
        assert p2 == q2 and a2 == b2
        ref2 = oracle.perm_mult(V, S, T)
        assert abs(p2 - ref2) <= 1e-10 * abs(ref2)
        assert abs(a2 - oracle.amplitude(V, S, T)) <= 1e-10 * abs(ref2)
        # trivial problems write without scratch
        st, p3, a3 = _run(lib, ctx, "pq_perm_noalloc", U2, [1, 0, 0, 0, 0, 0, 0], [0] * 7)
        assert st == 0 and p3 == 0 and a3 == 0
    finally:
        lib.pq_destroy(ctx)


def test_noalloc_refuses_a_permanent_beyond_its_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_04006_amd as pq
    lib = pq._lib.load()
    ctx = ctypes.c_void_p()
    assert lib.pq_create(ctypes.byref(ctx), 0) == 0
    try:
        # 40 photons, 28 distinct rows (six of them three times), 40 columns:
        # 4096-state step tables plus the compact matrices exceed the buffer
        T = [3] * 6 + [1] * 22 + [0] * 12
        S = [1] * 40
        info = pq.plan_describe(S, T)
        assert info["inner_states"] == 4096 and not info["binary"]
        U = torch.from_numpy(workloads.haar(40, 2)).cuda()
        print("noalloc: oversized plan (refused on the host)", flush=True)
        st, p, a = _run(lib, ctx, "pq_perm_noalloc", U, S, T)
        assert st == pq._lib.PQ_ERANGE
        assert "scratch" in lib.pq_last_error(ctx).decode()
        assert p == complex(7.0, 7.0) and a == complex(7.0, 7.0)
    finally:
        lib.pq_destroy(ctx)
