"""MI355X permanent engine: Fock amplitudes perm(U_{T,S}) / sqrt(prod S! prod T!)
of linear-optical interferometers, computed by hand-written HIP kernels
(libpq.so) behind a C ABI.  This package only marshals arguments: tensors are
torch complex128 on the GPU, occupations are integer sequences on the host,
and every computation runs in the library's kernels on the caller's current
torch stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
from typing import Sequence

import torch

from . import _lib
from ._lib import PqError, pq_job, pq_plan_info, PQ_OP_PERM, PQ_OP_EXTEND_ROW, PQ_MAX_N  # noqa: F401

__all__ = [
    "Engine", "engine", "perm", "plan_describe", "gray_unrank", "fock_count", "fock_unrank", "PqError",
    "PatternSet", "JobSet", "PQ_OP_PERM", "PQ_OP_EXTEND_ROW",
]


def _check(status: int, ctx=None):
    if status != _lib.PQ_OK:
        lib = _lib.load()
        detail = lib.pq_last_error(ctx).decode() if ctx else lib.pq_strerror(status).decode()
        raise PqError(status, detail)


def _stream_handle(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _as_matrix(U: torch.Tensor) -> tuple:
    if not isinstance(U, torch.Tensor) or U.dtype != torch.complex128 or U.dim() != 2:
        raise TypeError("U must be a 2-D torch.complex128 tensor")
    if not U.is_cuda:
        raise TypeError("U must live on the GPU")
    if U.shape[0] != U.shape[1]:
        raise ValueError("U must be square")
    if U.stride(1) != 1:
        U = U.contiguous()
    return U, U.stride(0)



# numpy layout of struct pq_job (include/pq.h): three int32, four pointers at
# 8-byte alignment, one int64
_JOB_DTYPE = np.dtype({
    "names": ["op", "nr", "nc", "row_idx", "row_mult", "col_idx", "col_mult", "out_offset"],
    "formats": ["<i4", "<i4", "<i4", "<u8", "<u8", "<u8", "<u8", "<i8"],
    "offsets": [0, 4, 8, 16, 24, 32, 40, 48],
    "itemsize": 56,
})

class Engine:
    """One libpq context on one GPU (not thread-safe; one stream at a time)."""

    def __init__(self, device: int | torch.device | None = None):
        lib = _lib.load()
        if device is None:
            device = torch.cuda.current_device()
        self.device = torch.device("cuda", device if isinstance(device, int) else device.index or 0)
        ctx = ctypes.c_void_p()
        _check(lib.pq_create(ctypes.byref(ctx), self.device.index))
        self._ctx = ctx
        self._lib = lib

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.pq_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_peak(self) -> dict:
        """Compute units, peak clock and the FP64 vector peak they imply, as
        the HIP runtime reports the device (pq_device_peak)."""
        cus, khz, tf = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(self._lib.pq_device_peak(self._ctx, ctypes.byref(cus), ctypes.byref(khz), ctypes.byref(tf)),
               self._ctx)
        return {"cus": cus.value, "clock_mhz": khz.value / 1e3, "fp64_vector_peak_tflops": tf.value}

    # ----------------------------------------------------------- pq_perm
    def perm(self, U: torch.Tensor, S: Sequence[int], T: Sequence[int], *,
             out_perm: torch.Tensor | None = None, out_amp: torch.Tensor | None = None):
        """perm(U_{T,S}) and the amplitude, as 0-d complex128 device tensors."""
        U, ldu = _as_matrix(U)
        m = U.shape[0]
        if len(S) != m or len(T) != m:
            raise ValueError("S and T need one entry per mode")
        if out_perm is None:
            out_perm = torch.empty((), dtype=torch.complex128, device=U.device)
        if out_amp is None:
            out_amp = torch.empty((), dtype=torch.complex128, device=U.device)
        st = self._lib.pq_perm(self._ctx, U.data_ptr(), ldu, m, _lib.i32_array(S), _lib.i32_array(T),
                               out_perm.data_ptr(), out_amp.data_ptr(), _stream_handle(U.device))
        _check(st, self._ctx)
        return out_perm, out_amp

    # ------------------------------------------------------------ timing
    def profile(self, on: bool = True):
        """Bracket every sweep launch with HIP events (pq_profile_enable)."""
        _check(self._lib.pq_profile_enable(self._ctx, 1 if on else 0), self._ctx)

    def profile_read(self):
        """(launches, total sweep milliseconds) since the last read."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(self._lib.pq_profile_read(self._ctx, ctypes.byref(n), ctypes.byref(ms)), self._ctx)
        return n.value, ms.value

    # ------------------------------------------------- batched job lists
    @staticmethod
    def _job_array(jobs: Sequence[dict], m: int):
        """pq_job array for `jobs` (argument marshalling): the index and
        multiplicity lists of every job live in one int32 buffer and the
        structs are filled column-wise; returns (pointer, keep-alive, n_out)."""
        n = len(jobs)
        ops = np.empty(max(1, n), np.int32)
        nrs = np.zeros(max(1, n), np.int32)
        ncs = np.zeros(max(1, n), np.int32)
        outs = np.zeros(max(1, n), np.int64)
        flat: list = []
        total = 0
        for k, j in enumerate(jobs):
            op = int(j.get("op", PQ_OP_PERM))
            rows = j["rows"]
            cols = j["cols"]
            ops[k] = op
            nrs[k] = len(rows)
            ncs[k] = len(cols)
            flat.extend(int(r) for r, _ in rows)
            flat.extend(int(c) for _, c in rows)
            flat.extend(int(r) for r, _ in cols)
            flat.extend(int(c) for _, c in cols)
            off = int(j.get("out", total))
            outs[k] = off
            total = max(total, off + (m if op == PQ_OP_EXTEND_ROW else 1))
        buf = np.asarray(flat if flat else [0], dtype=np.int32)
        arr = np.zeros(max(1, n), dtype=_JOB_DTYPE)
        if n:
            start = np.zeros(n, np.int64)
            start[1:] = np.cumsum(2 * (nrs[:n].astype(np.int64) + ncs[:n]))[:-1]
            base = buf.ctypes.data
            arr["op"][:n] = ops[:n]
            arr["nr"][:n] = nrs[:n]
            arr["nc"][:n] = ncs[:n]
            arr["row_idx"][:n] = base + 4 * start
            arr["row_mult"][:n] = base + 4 * (start + nrs[:n])
            arr["col_idx"][:n] = base + 4 * (start + 2 * nrs[:n])
            arr["col_mult"][:n] = base + 4 * (start + 2 * nrs[:n] + ncs[:n])
            arr["out_offset"][:n] = outs[:n]
        ptr = ctypes.cast(arr.ctypes.data, ctypes.POINTER(pq_job))
        return ptr, (buf, arr), total

    def _run_jobs(self, fn, U, jobs, n_out, with_amp, out=None):
        U, ldu = _as_matrix(U)
        m = U.shape[0]
        if isinstance(jobs, JobSet):
            if jobs.m != m:
                raise ValueError("job set built for another mode count")
            arr, keep, total = jobs.jobs, None, jobs.n_out
            jobs = range(jobs.njobs)
        else:
            arr, keep, total = self._job_array(jobs, m)
        n_out = total if n_out is None else n_out
        if out is not None:
            # caller-owned outputs (stable pointers, e.g. for graph replays)
            perm, amp = out
            for t in (perm, amp):
                if t is not None and (t.dtype != torch.complex128 or t.device != U.device
                                      or not t.is_contiguous() or t.numel() < max(1, n_out)):
                    raise ValueError("out tensors must be contiguous complex128 on U's device, n_out long")
        else:
            perm = torch.zeros(max(1, n_out), dtype=torch.complex128, device=U.device)
            amp = torch.zeros(max(1, n_out), dtype=torch.complex128, device=U.device) if with_amp else None
        st = fn(self._ctx, U.data_ptr(), ldu, m, arr, len(jobs), perm.data_ptr(),
                amp.data_ptr() if amp is not None else None, _stream_handle(U.device))
        _check(st, self._ctx)
        return perm[:n_out], (amp[:n_out] if amp is not None else None)

    def perm_patterns(self, U: torch.Tensor, pats: "PatternSet", with_amp: bool = False):
        """perm(U_{T_p,S_p}) for a prepared PatternSet (pq_perm_many); returns
        (perm, amp or None), one entry per pattern."""
        U, ldu = _as_matrix(U)
        if U.shape[0] != pats.m:
            raise ValueError("pattern set built for another mode count")
        perm = torch.empty(max(1, pats.batch), dtype=torch.complex128, device=U.device)
        amp = torch.empty_like(perm) if with_amp else None
        st = self._lib.pq_perm_many(self._ctx, U.data_ptr(), ldu, pats.m, pats.jobs, pats.batch, perm.data_ptr(),
                                    amp.data_ptr() if amp is not None else None, _stream_handle(U.device))
        _check(st, self._ctx)
        return perm[:pats.batch], (amp[:pats.batch] if amp is not None else None)

    def grad_patterns(self, U: torch.Tensor, pats: "PatternSet", gperm: torch.Tensor, want_perm: bool = False):
        """dU = sum_p gperm[p] conj(d perm_p / dU) for a prepared PatternSet
        (pq_perm_grad); returns (dU, perm or None)."""
        U, ldu = _as_matrix(U)
        gperm = gperm.to(dtype=torch.complex128, device=U.device).contiguous()
        dU = torch.empty((pats.m, pats.m), dtype=torch.complex128, device=U.device)
        perm = torch.empty(max(1, pats.batch), dtype=torch.complex128, device=U.device) if want_perm else None
        st = self._lib.pq_perm_grad(self._ctx, U.data_ptr(), ldu, pats.m, pats.batch, pats.S_flat, pats.T_flat,
                                    gperm.data_ptr(), perm.data_ptr() if perm is not None else None,
                                    dU.data_ptr(), pats.m, _stream_handle(U.device))
        _check(st, self._ctx)
        return dU, (perm[:pats.batch] if perm is not None else None)

    def perm_all_outputs(self, U: torch.Tensor, S: Sequence[int], with_amp: bool = True):
        """perm(U_{T,S}) (and amplitudes) for every output pattern T with sum T =
        sum S, in the order of fock_unrank (pq_perm_all_outputs)."""
        U, ldu = _as_matrix(U)
        m = U.shape[0]
        if len(S) != m:
            raise ValueError("S needs one entry per mode")
        count = fock_count(m, int(sum(int(v) for v in S)))
        if count < 0 or count > _lib.PQ_ALL_MAX_OUTPUTS:
            raise PqError(_lib.PQ_ERANGE, f"more than {_lib.PQ_ALL_MAX_OUTPUTS} output patterns")
        perm = torch.empty(max(1, count), dtype=torch.complex128, device=U.device)
        amp = torch.empty_like(perm) if with_amp else None
        st = self._lib.pq_perm_all_outputs(self._ctx, U.data_ptr(), ldu, m, _lib.i32_array(S), perm.data_ptr(),
                                           amp.data_ptr() if amp is not None else None, _stream_handle(U.device))
        _check(st, self._ctx)
        return perm[:count], (amp[:count] if amp is not None else None)

    def sample_chain(self, U: torch.Tensor, order: torch.Tensor, uniforms: torch.Tensor) -> torch.Tensor:
        """Chain-rule boson samples (pq_sample_chain): order (samples, n) int32
        input modes and uniforms (samples, n) float64 on U's device; returns the
        drawn output modes (samples, n) int32 in draw order."""
        U, ldu = _as_matrix(U)
        m = U.shape[0]
        order = order.to(device=U.device, dtype=torch.int32).contiguous()
        uniforms = uniforms.to(device=U.device, dtype=torch.float64).contiguous()
        if order.dim() != 2 or uniforms.shape != order.shape:
            raise ValueError("order and uniforms need the same (samples, n) shape")
        samples, n = order.shape
        out = torch.empty((samples, n), dtype=torch.int32, device=U.device)
        st = self._lib.pq_sample_chain(self._ctx, U.data_ptr(), ldu, m, n, samples, order.data_ptr(),
                                       uniforms.data_ptr(), out.data_ptr(), _stream_handle(U.device))
        _check(st, self._ctx)
        return out

    def loss_dilation(self, U: torch.Tensor, eta: Sequence[float]) -> torch.Tensor:
        """2m x 2m unitary dilation of U followed by per-mode losses with
        transmissivities eta (pq_loss_dilation)."""
        U, ldu = _as_matrix(U)
        m = U.shape[0]
        if len(eta) != m:
            raise ValueError("eta needs one entry per mode")
        Ud = torch.empty((2 * m, 2 * m), dtype=torch.complex128, device=U.device)
        arr = (ctypes.c_double * m)(*[float(x) for x in eta])
        st = self._lib.pq_loss_dilation(self._ctx, U.data_ptr(), ldu, m, arr, Ud.data_ptr(), 2 * m,
                                        _stream_handle(U.device))
        _check(st, self._ctx)
        return Ud

    def cancel(self, on: bool = True):
        """Request (or clear) cancellation of this ctx's work (pq_cancel)."""
        _check(self._lib.pq_cancel(self._ctx, 1 if on else 0), self._ctx)

    def fault_inject(self, what: int):
        """Make every allocation (PQ_FAULT_ALLOC) or launch check
        (PQ_FAULT_LAUNCH) of this ctx fail; PQ_FAULT_NONE restores it."""
        _check(self._lib.pq_fault_inject(self._ctx, int(what)), self._ctx)

    def loss_dilation_vw(self, V: torch.Tensor, eta: Sequence[float], W: torch.Tensor) -> torch.Tensor:
        """2m x 2m unitary dilation of the lossy interferometer
        A = V diag(sqrt(eta)) W (pq_loss_dilation_vw)."""
        V, ldv = _as_matrix(V)
        W, ldw = _as_matrix(W)
        m = V.shape[0]
        if W.shape[0] != m or len(eta) != m:
            raise ValueError("V, W and eta must have the same mode count")
        Ud = torch.empty((2 * m, 2 * m), dtype=torch.complex128, device=V.device)
        arr = (ctypes.c_double * m)(*[float(x) for x in eta])
        st = self._lib.pq_loss_dilation_vw(self._ctx, V.data_ptr(), ldv, arr, W.data_ptr(), ldw, m, Ud.data_ptr(),
                                           2 * m, _stream_handle(V.device))
        _check(st, self._ctx)
        return Ud

    def autotune(self, on: bool = True):
        """Chunk-size autotuning of perm_many (pq_autotune_enable)."""
        _check(self._lib.pq_autotune_enable(self._ctx, 1 if on else 0), self._ctx)

    def graphs(self, on: bool = True):
        """Replay perm_many launch sequences as captured HIP graphs
        (pq_graph_enable)."""
        _check(self._lib.pq_graph_enable(self._ctx, 1 if on else 0), self._ctx)

    def queue_mode(self, mode: str = "auto"):
        """Which column classes perm_batched runs as work queues: "auto",
        "always" or "never" (pq_queue_mode)."""
        code = {"auto": 0, "always": 1, "never": 2}[mode]
        _check(self._lib.pq_queue_mode(self._ctx, code), self._ctx)

    def all_outputs_gemm(self, mode: str = "auto"):
        """Which form perm_all_outputs takes: "auto", "always" (the
        contraction on rocBLAS zgemm whenever its tables fit) or "never" (the
        sweep) (pq_all_outputs_gemm)."""
        code = {"auto": 0, "always": 1, "never": 2}[mode]
        _check(self._lib.pq_all_outputs_gemm(self._ctx, code), self._ctx)

    def lhaf_pack(self, mode: str = "auto"):
        """When the loop hafnian sweep fills idle lanes across Gray segments:
        "auto", "always" or "never" (pq_lhaf_pack)."""
        code = {"auto": 0, "always": 1, "never": 2}[mode]
        _check(self._lib.pq_lhaf_pack(self._ctx, code), self._ctx)

    def walk_variant(self, register_digits: int, swizzle: bool = False):
        """Form of the reverse sweep for wide collision-free patterns
        (pq_walk_variant)."""
        _check(self._lib.pq_walk_variant(self._ctx, int(register_digits), int(swizzle)), self._ctx)

    def autotune_last(self) -> dict:
        """The last autotuning decision (pq_autotune_last)."""
        pol = (ctypes.c_int32 * 3)()
        best, default = ctypes.c_double(), ctypes.c_double()
        cand = ctypes.c_int32()
        _check(self._lib.pq_autotune_last(self._ctx, pol, ctypes.byref(best), ctypes.byref(default),
                                          ctypes.byref(cand)), self._ctx)
        return {"waves_per_cu": pol[0], "chunks_per_wave": pol[1], "min_chunk": pol[2],
                "best_ms": best.value, "default_ms": default.value, "candidates": cand.value}

    def lhaf(self, A: torch.Tensor, gamma: torch.Tensor | None, reps: Sequence[int]) -> torch.Tensor:
        """Loop hafnian of filldiag(A_r, gamma_r) with mode i repeated reps[i]
        times (pq_lhaf); gamma None gives the hafnian.  Returns a 1-element
        complex128 tensor on A's device."""
        A, lda = _as_matrix(A)
        d = A.shape[0]
        r = np.ascontiguousarray(np.asarray(reps, dtype=np.int32))
        if r.shape != (d,):
            raise ValueError("reps needs one entry per mode")
        g_ptr = None
        if gamma is not None:
            if gamma.dtype != torch.complex128 or gamma.device != A.device or tuple(gamma.shape) != (d,):
                raise ValueError("gamma must be a complex128 vector of length d on A's device")
            gamma = gamma.contiguous()
            g_ptr = gamma.data_ptr()
        out = torch.empty(1, dtype=torch.complex128, device=A.device)
        st = self._lib.pq_lhaf(self._ctx, A.data_ptr(), lda, d, g_ptr,
                               r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), out.data_ptr(),
                               _stream_handle(A.device))
        _check(st, self._ctx)
        return out

    def lhaf_many(self, A: torch.Tensor, gamma: torch.Tensor | None, reps) -> torch.Tensor:
        """Loop hafnians of filldiag(A_r, gamma_r) for every repetition vector
        in `reps` (npat x d), in one submission (pq_lhaf_many); gamma None
        gives hafnians.  Returns an (npat,) complex128 tensor on A's device."""
        A, lda = _as_matrix(A)
        d = A.shape[0]
        r = np.ascontiguousarray(np.asarray(reps, dtype=np.int32))
        if r.ndim != 2 or r.shape[1] != d:
            raise ValueError("reps must be npat x d")
        g_ptr = None
        if gamma is not None:
            if gamma.dtype != torch.complex128 or gamma.device != A.device or tuple(gamma.shape) != (d,):
                raise ValueError("gamma must be a complex128 vector of length d on A's device")
            gamma = gamma.contiguous()
            g_ptr = gamma.data_ptr()
        npat = r.shape[0]
        out = torch.empty(max(1, npat), dtype=torch.complex128, device=A.device)
        st = self._lib.pq_lhaf_many(self._ctx, A.data_ptr(), lda, d, g_ptr,
                                    r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), npat, out.data_ptr(),
                                    _stream_handle(A.device))
        _check(st, self._ctx)
        return out[:npat]

    def sample_chain_lossy(self, U: torch.Tensor, eta: Sequence[float], order: torch.Tensor,
                           uniforms: torch.Tensor) -> torch.Tensor:
        """Chain-rule samples through U followed by per-mode losses: the draws
        on the loss dilation, with lost photons (modes >= m) reported as -1."""
        m = U.shape[0]
        out = self.sample_chain(self.loss_dilation(U, eta), order, uniforms)
        return torch.where(out >= m, torch.full_like(out, -1), out)

    def perm_many(self, U: torch.Tensor, jobs: Sequence[dict], n_out: int | None = None, with_amp: bool = True,
                  out: tuple | None = None):
        """Jobs {op, rows: [(mode, mult)], cols: [(mode, mult)], out} through the
        statically scheduled many-pattern path (pq_perm_many).  PERM jobs write
        perm(U_{T,S}) (and the amplitude) at `out`; EXTEND_ROW jobs write
        perm(U_{T+e_l,S}) for l = 0..m-1 at out..out+m-1.  Returns (perm, amp).
        `out` = (perm, amp or None): caller-owned output tensors."""
        return self._run_jobs(self._lib.pq_perm_many, U, jobs, n_out, with_amp, out)

    def perm_batched(self, U: torch.Tensor, jobs: Sequence[dict], n_out: int | None = None,
                     with_amp: bool = True, out: tuple | None = None):
        """The same jobs through pq_perm_batched (the boundary's batched call:
        a persistent work queue replayed from a captured HIP graph; pass fixed
        output tensors in `out` to replay one graph)."""
        return self._run_jobs(self._lib.pq_perm_batched, U, jobs, n_out, with_amp, out)

    # -------------------------------------------------------- pq_perm_grad
    def perm_grad(self, U: torch.Tensor, S_list, T_list, gperm: torch.Tensor, want_perm: bool = True):
        """dU = sum_p gperm[p] conj(d perm_p / dU); returns (dU, perm or None)."""
        U, ldu = _as_matrix(U)
        m = U.shape[0]
        batch = len(S_list)
        flatS = [int(v) for s in S_list for v in s]
        flatT = [int(v) for t in T_list for v in t]
        if len(flatS) != batch * m or len(flatT) != batch * m:
            raise ValueError("patterns need one entry per mode")
        gperm = gperm.to(dtype=torch.complex128, device=U.device).contiguous()
        dU = torch.empty((m, m), dtype=torch.complex128, device=U.device)
        perm = torch.empty(max(1, batch), dtype=torch.complex128, device=U.device) if want_perm else None
        st = self._lib.pq_perm_grad(self._ctx, U.data_ptr(), ldu, m, batch, _lib.i32_array(flatS),
                                    _lib.i32_array(flatT), gperm.data_ptr(),
                                    perm.data_ptr() if perm is not None else None,
                                    dU.data_ptr(), m, _stream_handle(U.device))
        _check(st, self._ctx)
        return dU, (perm[:batch] if perm is not None else None)


class JobSet:
    """A job list (dicts as for Engine.perm_many) marshalled once for repeated
    pq_perm_many / pq_perm_batched calls on interferometers with m modes."""

    def __init__(self, jobs: Sequence[dict], m: int):
        self.m = int(m)
        self.njobs = len(jobs)
        self.jobs, self._keep, self.n_out = Engine._job_array(jobs, self.m)


class PatternSet:
    """Input/output occupation patterns on m modes, marshalled once for
    repeated pq_perm_many / pq_perm_grad calls (e.g. every step of a training
    loop)."""

    def __init__(self, S_list, T_list, m: int):
        if len(S_list) != len(T_list):
            raise ValueError("S_list and T_list differ in length")
        self.m = int(m)
        self.batch = len(S_list)
        flatS, flatT = [], []
        jobs = []
        for p, (S, T) in enumerate(zip(S_list, T_list)):
            S = [int(v) for v in S]
            T = [int(v) for v in T]
            if len(S) != m or len(T) != m:
                raise ValueError("patterns need one entry per mode")
            flatS += S
            flatT += T
            jobs.append({"op": PQ_OP_PERM, "rows": [(i, c) for i, c in enumerate(T) if c > 0],
                         "cols": [(i, c) for i, c in enumerate(S) if c > 0], "out": p})
        self.S_flat = _lib.i32_array(flatS)
        self.T_flat = _lib.i32_array(flatT)
        self.jobs, self._keep, _ = Engine._job_array(jobs, m)


_engines: dict = {}


def engine(device: int | None = None) -> Engine:
    """Per-device default Engine."""
    if device is None:
        device = torch.cuda.current_device()
    if device not in _engines:
        _engines[device] = Engine(device)
    return _engines[device]


def perm(U: torch.Tensor, S: Sequence[int], T: Sequence[int]):
    """(perm, amp) of U_{T,S} on U's device (see Engine.perm)."""
    return engine(U.device.index).perm(U, S, T)


def plan_describe(S: Sequence[int], T: Sequence[int]) -> dict:
    """GPU-free planning summary of one permanent (pq_plan_describe)."""
    lib = _lib.load()
    info = pq_plan_info()
    m = len(S)
    lib.pq_plan_describe(m, _lib.i32_array(S), _lib.i32_array(T), ctypes.byref(info))
    return {name: getattr(info, name) for name, _ in pq_plan_info._fields_}


def fock_count(m: int, n: int) -> int:
    """Output patterns of n photons on m modes, C(n+m-1, n) (-1 on overflow)."""
    return int(_lib.load().pq_fock_count(int(m), int(n)))


def fock_unrank(m: int, n: int, rank: int) -> list:
    """Occupation vector of `rank` in the output order of perm_all_outputs
    (ascending lexicographic in (T_0, ..., T_{m-1}))."""
    out = (ctypes.c_int32 * max(1, m))()
    _check(_lib.load().pq_fock_unrank(int(m), int(n), int(rank), out))
    return [out[i] for i in range(m)]


def gray_unrank(radix: Sequence[int], rank: int) -> list:
    """Gray digits (least significant first) of `rank` in the reflected
    mixed-radix code with the given radices (pq_gray_unrank)."""
    lib = _lib.load()
    d = len(radix)
    out = (ctypes.c_int32 * max(1, d))()
    _check(lib.pq_gray_unrank(d, _lib.i32_array(radix), int(rank), out))
    return [out[k] for k in range(d)]
