"""CPU tests of the product's host side: the C ABI loads and exports every
declared symbol, planning invariants, the Gray code, and argument errors.
No GPU work is launched here."""
import ctypes
import itertools
import math
import os
import re

import numpy as np
import pytest

import paper_2403_04006_amd as pq
import workloads
from paper_2403_04006_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if not f.endswith(".h"):
            continue
        src = open(os.path.join(inc, f)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(pq_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert {"pq_create", "pq_destroy", "pq_perm", "pq_perm_batched", "pq_perm_grad"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name
    assert lib.pq_version().startswith(b"pq ")


def test_status_strings():
    lib = _lib.load()
    for s in range(6):
        assert lib.pq_strerror(s)
    assert lib.pq_strerror(99) == b"unknown status"


def test_null_arguments_are_rejected_without_a_device():
    lib = _lib.load()
    assert lib.pq_create(None, 0) == _lib.PQ_EINVAL
    assert lib.pq_perm(None, None, 0, 0, None, None, None, None, None) == _lib.PQ_EINVAL
    assert lib.pq_perm_batched(None, None, 0, 0, None, 0, None, None, None) == _lib.PQ_EINVAL
    assert lib.pq_perm_grad(None, None, 0, 0, 0, None, None, None, None, None, 0, None) == _lib.PQ_EINVAL
    assert lib.pq_autotune_enable(None, 1) == _lib.PQ_EINVAL
    pol = (ctypes.c_int32 * 3)()
    d1, d2, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    assert lib.pq_autotune_last(None, pol, ctypes.byref(d1), ctypes.byref(d2), ctypes.byref(c)) == _lib.PQ_EINVAL
    assert lib.pq_lhaf(None, None, 0, 0, None, None, None, None) == _lib.PQ_EINVAL
    assert lib.pq_lhaf_many(None, None, 0, 0, None, None, 0, None, None) == _lib.PQ_EINVAL
    assert lib.pq_graph_enable(None, 1) == _lib.PQ_EINVAL
    assert lib.pq_walk_variant(None, 1, 0) == _lib.PQ_EINVAL
    assert lib.pq_queue_mode(None, 0) == _lib.PQ_EINVAL
    assert lib.pq_lhaf_pack(None, 1) == _lib.PQ_EINVAL
    assert lib.pq_all_outputs_gemm(None, 1) == _lib.PQ_EINVAL
    assert lib.pq_device_peak(None, None, None, None) == _lib.PQ_EINVAL
    lib.pq_destroy(None)
    assert lib.pq_last_error(None) == b""


# ------------------------------------------------------------- Gray code
@pytest.mark.parametrize("radix", [[2, 2, 2, 2], [3, 2, 4], [5, 1, 3, 2], [4, 4, 3], [2, 5, 2, 3, 2]])
def test_gray_code_walks_every_state_once_with_unit_steps(radix):
    total = int(np.prod(radix))
    seen = set()
    prev = None
    for r in range(total):
        g = pq.gray_unrank(radix, r)
        assert all(0 <= g[k] < radix[k] for k in range(len(radix)))
        seen.add(tuple(g))
        if prev is None:
            assert g == [0] * len(radix)
        else:
            diff = [k for k in range(len(radix)) if g[k] != prev[k]]
            assert len(diff) == 1 and abs(g[diff[0]] - prev[diff[0]]) == 1
        prev = g
    assert len(seen) == total


def test_gray_code_binary_matches_reflected_binary():
    for r in range(256):
        g = pq.gray_unrank([2] * 8, r)
        assert sum(b << k for k, b in enumerate(g)) == r ^ (r >> 1)


def test_gray_code_rejects_out_of_range():
    with pytest.raises(pq.PqError):
        pq.gray_unrank([2, 3], 6)


def test_gray_code_reflection_of_low_digits():
    # within a run of the high digits, the low digits go forward when the high
    # Gray digits sum to an even number and backward otherwise
    radix = [3, 4, 2, 3]
    low = 12
    for hi in range(6):
        states = [tuple(pq.gray_unrank(radix, hi * low + p)[:2]) for p in range(low)]
        high = pq.gray_unrank(radix, hi * low)[2:]
        fwd = [tuple(pq.gray_unrank(radix[:2], q)) for q in range(low)]
        want = fwd if sum(high) % 2 == 0 else fwd[::-1]
        assert states == want


# --------------------------------------------------------------- planning
def brute_terms(mults):
    f = int(np.argmin(mults))
    return math.prod((m if k == f else m + 1) for k, m in enumerate(mults))


@pytest.mark.parametrize("seed", range(40))
def test_plan_invariants(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 12))
    n = int(rng.integers(1, 30))
    S = np.bincount(rng.integers(0, m, n), minlength=m)
    T = np.bincount(rng.integers(0, m, n), minlength=m)
    info = pq.plan_describe(list(S), list(T))
    assert info["status"] == 0 and info["trivial"] == 0 and info["n"] == n
    ts, tt = brute_terms(S[S > 0]), brute_terms(T[T > 0])
    assert info["terms"] == min(ts, tt)
    assert info["transposed"] == (1 if ts < tt else 0)
    it, pw = (S, T) if info["transposed"] else (T, S)
    assert info["rows"] == int((it > 0).sum()) and info["cols"] == int((pw > 0).sum())
    assert 1 <= info["lane_states"] <= 64
    assert info["lane_states"] * info["time_states"] == info["terms"]
    assert info["inner_states"] <= 4096
    assert info["binary"] == int(it.max() == 1 and pw.max() == 1)
    lg = sum(math.lgamma(int(v) + 1) for v in list(S) + list(T))
    assert info["log2_norm"] == pytest.approx(-0.5 * lg / math.log(2), abs=1e-12)


def test_plan_unit_multiplicity_uses_all_lanes():
    info = pq.plan_describe([1] * 30, [1] * 30)
    assert info["binary"] == 1 and info["terms"] == 2 ** 29
    assert info["lane_states"] == 64 and info["time_states"] == 2 ** 23


def test_plan_special_cases_and_errors():
    assert pq.plan_describe([1, 0], [0, 2])["trivial"] == 1
    assert pq.plan_describe([0, 0], [0, 0])["trivial"] == 2
    assert pq.plan_describe([-1, 1], [0, 0])["status"] == _lib.PQ_EINVAL
    assert pq.plan_describe([49], [49])["status"] == _lib.PQ_ERANGE
    # 40 distinct rows/cols, all ones: 2^39 terms is allowed
    assert pq.plan_describe([1] * 40, [1] * 40)["status"] == 0
    # terms reaching 2^62 are rejected: 47 ones and... (48 photons all
    # multiplicity 1 give 2^47, fine)
    assert pq.plan_describe([1] * 48, [1] * 48)["terms"] == 2 ** 47


def test_plan_repeated_workload_sizes():
    import workloads
    pats = workloads.repeated_patterns(count=16, seed=1)
    for S, T in pats:
        info = pq.plan_describe(list(S), list(T))
        assert info["status"] == 0 and info["n"] == 40
        assert info["terms"] == min(brute_terms(S[S > 0]), brute_terms(T[T > 0]))


def test_job_marshalling_matches_struct_layout():
    # the binding fills struct pq_job column-wise from numpy; read it back
    # through the ctypes definition of the struct
    jobs = [{"op": 0, "rows": [(1, 2), (3, 1)], "cols": [(0, 1), (2, 2)]},
            {"op": 1, "rows": [(4, 1)], "cols": [(1, 1), (5, 1)], "out": 10},
            {"op": 0, "rows": [], "cols": []}]
    ptr, keep, total = pq.Engine._job_array(jobs, 8)
    assert ctypes.sizeof(_lib.pq_job) == 56
    want = [(0, [1, 3], [2, 1], [0, 2], [1, 2], 0), (1, [4], [1], [1, 5], [1, 1], 10), (0, [], [], [], [], 18)]
    for k, (op, ri, rm, ci, cm, out) in enumerate(want):
        j = ptr[k]
        assert j.op == op and j.nr == len(ri) and j.nc == len(ci) and j.out_offset == out
        assert [j.row_idx[i] for i in range(j.nr)] == ri
        assert [j.row_mult[i] for i in range(j.nr)] == rm
        assert [j.col_idx[i] for i in range(j.nc)] == ci
        assert [j.col_mult[i] for i in range(j.nc)] == cm
    assert total == 19
    js = pq.JobSet(jobs, 8)
    assert js.njobs == 3 and js.n_out == 19


@pytest.mark.parametrize("m,n", [(1, 0), (1, 5), (3, 0), (4, 3), (5, 4), (6, 6)])
def test_fock_order_matches_enumeration(m, n):
    # output order of pq_perm_all_outputs: ascending lexicographic in
    # (T_0, ..., T_{m-1}), the order of the plain enumeration in workloads
    outs = workloads.fock_outputs(m, n)
    assert pq.fock_count(m, n) == math.comb(n + m - 1, n) == len(outs)
    for r, T in enumerate(outs):
        assert pq.fock_unrank(m, n, r) == [int(v) for v in T]


def test_fock_count_and_unrank_errors():
    assert pq.fock_count(0, 3) == -1
    assert pq.fock_count(3, -1) == -1
    assert pq.fock_count(200, 100) == -1          # above 2^62
    with pytest.raises(pq.PqError):
        pq.fock_unrank(4, 3, pq.fock_count(4, 3))
    with pytest.raises(pq.PqError):
        pq.fock_unrank(4, 3, -1)


def test_binding_constants_match_header():
    text = open(os.path.join(ROOT, "include", "pq.h")).read()
    defs = {k: v.split("/*")[0].strip() for k, v in re.findall(r"#define\s+(PQ_\w+)\s+(.+)", text)}
    assert int(defs["PQ_MAX_N"]) == _lib.PQ_MAX_N
    assert int(defs["PQ_GRAD_MAX_DIM"]) == _lib.PQ_GRAD_MAX_DIM
    assert defs["PQ_ALL_MAX_OUTPUTS"] == "(1ll << 31)" and _lib.PQ_ALL_MAX_OUTPUTS == 1 << 31
