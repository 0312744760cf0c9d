"""Oracle: slow, obviously-correct CPU reference for the permanent engine.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product library
never does, and this package imports nothing from the product.

What it computes (each function cites the passage it follows):

* ``perm_bruteforce(A)``   -- Eq. per_def: sum over permutations (n <= 10).
* ``perm_ryser(A)``        -- Ryser's inclusion-exclusion formula (the formula
                             the Boson Sampling benchmark section contrasts
                             with BB/FG), x87 extended precision.
* ``perm_mult(U, S, T)``   -- perm(U_{T,S}) with rows = output modes repeated
                             t_i times and columns = input modes repeated s_j
                             times (Eq. BS_prob), by Ryser's formula grouped
                             over equal columns.
* ``amplitude(U, S, T)``   -- perm(U_{T,S}) / sqrt(prod S! prod T!) (Eq. BS_prob).
* ``perm_grad(U, S, T)``   -- d perm / d U_ij = t_i s_j perm(U_{T-e_i, S-e_j}).
* ``extend_row(U, rows, cols)`` -- the Laplace expansion along a new last row
                             used by chain-rule boson sampling (Clifford &
                             Clifford's algorithm A, named in the Boson
                             Sampling benchmark section).
* ``chain_rule_sample(U, order, uniforms)`` -- one chain-rule draw sequence
                             with given input order and uniforms (CDF
                             inversion over the extend-row weights).
* ``loss_dilation(U, eta)``, ``lossy_probability(U, eta, S, T)`` -- per-mode
                             pure-loss channels after U as beamsplitters to
                             environment modes (Boson Sampling section), and
                             the detection probability of T marginalised over
                             the environment.
* ``loss_dilation_vw(V, eta, W)`` -- the general lossy interferometer
                             A = V diag(sqrt(eta)) W of the same section.
* ``beamsplitter(theta, phi)``, ``mesh_unitary(angles)`` -- the beamsplitter
                             matrix of the "Beamsplitter gate" section and a
                             rectangular mesh of such cells.
* ``lhaf_bruteforce(B)``  -- Eq. loop_hafnian (Eq. haf_def with loops off):
                             the sum over single-pair matchings of an
                             explicit matrix, lowest vertex matched first.
* ``lhaf_rep(A, gamma, reps)`` -- the loop hafnian of filldiag(A_r, gamma_r),
                             mode i repeated r_i times (the GBS detection
                             probability's matrix function), x87 extended
                             precision; gamma None gives the hafnian.
* ``two_mode_amplitude``   -- the two-mode Fock expansion of the beamsplitter
                             ("States and their evolution"), with the ket
                             normalisation the printed coefficient omits.

Readings of the paper taken here are listed in the design notes.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC_PATH = os.path.join(_HERE, "oracle.c")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall",
                        _SRC_PATH, "-o", tmp, "-lquadmath"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


@lru_cache(maxsize=1)
def _lib():
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    dptr = ctypes.POINTER(ctypes.c_double)
    ldptr = ctypes.POINTER(ctypes.c_longdouble)
    iptr = ctypes.POINTER(ctypes.c_int32)
    lib.orc_perm_bruteforce.argtypes = [dptr, ctypes.c_int, ctypes.c_int64, ldptr]
    lib.orc_perm_ryser.argtypes = [dptr, ctypes.c_int, ctypes.c_int64, ldptr]
    lib.orc_perm_ryser_mult.argtypes = [dptr, ctypes.c_int64, ctypes.c_int, iptr, iptr, ldptr]
    lib.orc_perm_grad.argtypes = [dptr, ctypes.c_int64, ctypes.c_int, iptr, iptr, ldptr]
    lib.orc_perm_ryser_mult_q.argtypes = [dptr, ctypes.c_int64, ctypes.c_int, iptr, iptr, dptr]
    lib.orc_lhaf_rep.argtypes = [dptr, ctypes.c_int64, ctypes.c_int, dptr, iptr, ldptr]
    for f in ("orc_perm_bruteforce", "orc_perm_ryser", "orc_perm_ryser_mult", "orc_perm_grad",
              "orc_perm_ryser_mult_q", "orc_lhaf_rep"):
        getattr(lib, f).restype = ctypes.c_int
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_long_double_mantissa_bits.restype = ctypes.c_int
    if lib.orc_long_double_mantissa_bits() != 64:
        raise RuntimeError("oracle requires 80-bit long double")
    return lib


def _cplx(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    if a.ndim != 2:
        raise ValueError("expected a matrix")
    return a


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _occ(v, m: int) -> np.ndarray:
    v = np.ascontiguousarray(np.asarray(v, dtype=np.int32))
    if v.shape != (m,):
        raise ValueError("occupation vector must have length m")
    return v


def num_threads() -> int:
    return int(_lib().orc_num_threads())


def perm_bruteforce_ld(A) -> tuple:
    A = _cplx(A)
    n = A.shape[0]
    if A.shape != (n, n) or n > 10:
        raise ValueError("square matrix with n <= 10 expected")
    out = (ctypes.c_longdouble * 2)()
    st = _lib().orc_perm_bruteforce(_dp(A), n, n, out)
    if st:
        raise RuntimeError(f"oracle error {st}")
    return out[0], out[1]


def perm_bruteforce(A) -> complex:
    """Eq. per_def: per(A) = sum_sigma prod_i A[sigma(i), i]."""
    re, im = perm_bruteforce_ld(A)
    return complex(float(re), float(im))


def perm_ryser_ld(A) -> tuple:
    A = _cplx(A)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("square matrix expected")
    out = (ctypes.c_longdouble * 2)()
    st = _lib().orc_perm_ryser(_dp(A), n, n, out)
    if st:
        raise RuntimeError(f"oracle error {st}")
    return out[0], out[1]


def perm_ryser(A) -> complex:
    """Ryser: per(A) = (-1)^n sum_X (-1)^{|X|} prod_i sum_{j in X} a_ij."""
    re, im = perm_ryser_ld(A)
    return complex(float(re), float(im))


def perm_mult_ld(U, S, T) -> tuple:
    U = _cplx(U)
    m = U.shape[0]
    if U.shape != (m, m):
        raise ValueError("U must be square")
    S, T = _occ(S, m), _occ(T, m)
    out = (ctypes.c_longdouble * 2)()
    ip = ctypes.POINTER(ctypes.c_int32)
    st = _lib().orc_perm_ryser_mult(_dp(U), m, m, S.ctypes.data_as(ip), T.ctypes.data_as(ip), out)
    if st:
        raise RuntimeError(f"oracle error {st}")
    return out[0], out[1]


def perm_mult(U, S, T) -> complex:
    """perm(U_{T,S}): rows = output modes (t_i copies), cols = input modes (s_j copies)."""
    re, im = perm_mult_ld(U, S, T)
    return complex(float(re), float(im))


def perm_mult_quad(U, S, T) -> tuple:
    """perm(U_{T,S}) by the multiplicity formula in IEEE quad precision;
    returns (value as complex, (re_hi, re_lo, im_hi, im_lo))."""
    U = _cplx(U)
    m = U.shape[0]
    S, T = _occ(S, m), _occ(T, m)
    out = (ctypes.c_double * 4)()
    ip = ctypes.POINTER(ctypes.c_int32)
    st = _lib().orc_perm_ryser_mult_q(_dp(U), m, m, S.ctypes.data_as(ip), T.ctypes.data_as(ip), out)
    if st:
        raise RuntimeError(f"oracle error {st}")
    return complex(out[0] + out[1], out[2] + out[3]), tuple(out)


def perm_mult_cheaper_side(U, S, T) -> complex:
    """perm(U_{T,S}) evaluated over whichever side has fewer Ryser digit
    vectors, using perm(A^T) = perm(A) (rows and columns swap roles)."""
    S = np.asarray(S, dtype=np.int64)
    T = np.asarray(T, dtype=np.int64)
    cost_s = int(np.prod(S[S > 0] + 1))
    cost_t = int(np.prod(T[T > 0] + 1))
    if cost_t < cost_s:
        return perm_mult(np.ascontiguousarray(np.asarray(U).T), T, S)
    return perm_mult(U, S, T)


def normaliser(S, T) -> float:
    """1 / sqrt(prod S! prod T!) (Eq. BS_prob)."""
    lg = sum(math.lgamma(int(s) + 1) for s in S) + sum(math.lgamma(int(t) + 1) for t in T)
    return math.exp(-0.5 * lg)


def amplitude(U, S, T) -> complex:
    """<T| U |S> = perm(U_{T,S}) / sqrt(prod S! prod T!)."""
    return perm_mult(U, S, T) * normaliser(S, T)


def probability(U, S, T) -> float:
    """p(S -> T) = |perm(U_{T,S})|^2 / (prod S! prod T!)  (Eq. BS_prob)."""
    return abs(amplitude(U, S, T)) ** 2


def expand(U, S, T) -> np.ndarray:
    """The n x n matrix U_{T,S}: row i of U repeated t_i times (outputs),
    column j repeated s_j times (inputs)."""
    U = np.asarray(U)
    rows = [i for i, t in enumerate(T) for _ in range(int(t))]
    cols = [j for j, s in enumerate(S) for _ in range(int(s))]
    return np.ascontiguousarray(U[np.ix_(rows, cols)])


def perm_grad_ld(U, S, T) -> np.ndarray:
    U = _cplx(U)
    m = U.shape[0]
    S, T = _occ(S, m), _occ(T, m)
    out = (ctypes.c_longdouble * (2 * m * m))()
    ip = ctypes.POINTER(ctypes.c_int32)
    st = _lib().orc_perm_grad(_dp(U), m, m, S.ctypes.data_as(ip), T.ctypes.data_as(ip), out)
    if st:
        raise RuntimeError(f"oracle error {st}")
    return np.array(out[:], dtype=np.longdouble).reshape(m, m, 2)


def perm_grad(U, S, T) -> np.ndarray:
    """d perm(U_{T,S}) / d U_ij = t_i s_j perm(U_{T-e_i, S-e_j}) (complex128 m x m)."""
    g = perm_grad_ld(U, S, T).astype(np.float64)
    return g[..., 0] + 1j * g[..., 1]


def perm_vjp(U, S_list, T_list, gperm) -> np.ndarray:
    """Torch convention: dU = sum_p gperm_p * conj(d perm_p / d U)."""
    U = np.asarray(U)
    dU = np.zeros(U.shape, dtype=np.complex128)
    for S, T, g in zip(S_list, T_list, gperm):
        dU += g * np.conj(perm_grad(U, S, T))
    return dU


def extend_row(U, rows, cols) -> np.ndarray:
    """Laplace expansion along a new last row (chain-rule boson sampling).

    rows: the k-1 output modes drawn so far (a multiset), cols: the k input
    modes in order.  L_j = perm(U[rows; cols minus col j]); returns
    out[l] = sum_j U[l, cols[j]] L_j = perm(U_{rows + l, cols}) for every mode l.
    """
    U = np.asarray(U, dtype=np.complex128)
    m = U.shape[0]
    rows = list(rows)
    cols = list(cols)
    k = len(cols)
    if len(rows) != k - 1:
        raise ValueError("need k-1 rows for k columns")
    T = np.bincount(np.asarray(rows, dtype=np.int64), minlength=m).astype(np.int32) if rows else np.zeros(m, np.int32)
    L = np.zeros(k, dtype=np.complex128)
    for j in range(k):
        S = np.zeros(m, dtype=np.int32)
        for q, c in enumerate(cols):
            if q != j:
                S[c] += 1
        L[j] = perm_mult(U, S, T)
    return U[:, cols] @ L


def beamsplitter(theta: float, phi: float) -> np.ndarray:
    """2x2 mode matrix of the paper's beamsplitter: [[t, -r*], [r, t]] with
    t = cos(theta), r = e^{i phi} sin(theta) ("Beamsplitter gate"); row index
    = output mode, column index = input mode."""
    t = math.cos(theta)
    r = complex(math.cos(phi), math.sin(phi)) * math.sin(theta)
    return np.array([[t, -r.conjugate()], [r, t]], dtype=np.complex128)


def mesh_unitary(angles, cells, modes: int) -> np.ndarray:
    """Product of beamsplitter cells, the first cell acting first:
    U = B_last ... B_2 B_1, each B acting on its mode pair (k, k+1)."""
    U = np.eye(modes, dtype=np.complex128)
    for (theta, phi), (a, b) in zip(np.asarray(angles, dtype=np.float64), cells):
        B = np.eye(modes, dtype=np.complex128)
        B[np.ix_([a, b], [a, b])] = beamsplitter(theta, phi)
        U = B @ U
    return U


def two_mode_amplitude(theta: float, phi: float, n: int, m: int, p: int, q: int) -> complex:
    """<p, q| B(theta, phi) |n, m> from the two-mode Fock expansion
    sum_k sum_l C(n,k) C(m,l) t^{n+m-k-l} (-r*)^l r^k |n-k+l, m+k-l>,
    where the coefficient multiplies creation-operator monomials; the ket
    |p, q> carries 1/sqrt(p! q!) and |n, m> carries 1/sqrt(n! m!), hence the
    factor sqrt(p! q! / (n! m!))."""
    if p + q != n + m:
        return 0j
    t = math.cos(theta)
    r = complex(math.cos(phi), math.sin(phi)) * math.sin(theta)
    s = 0j
    for k in range(n + 1):
        for l in range(m + 1):
            if n - k + l == p and m + k - l == q:
                s += math.comb(n, k) * math.comb(m, l) * t ** (n + m - k - l) * (-r.conjugate()) ** l * r ** k
    return s * math.sqrt(math.factorial(p) * math.factorial(q) / (math.factorial(n) * math.factorial(m)))


def mesh_loss(U, S, patterns) -> float:
    """-mean over patterns of log(|perm(U_{T,S})|^2 / prod T!)."""
    vals = []
    for T in patterns:
        p = perm_mult(U, S, T)
        vals.append(math.log(abs(p) ** 2) - sum(math.lgamma(int(t) + 1) for t in T))
    return -float(np.mean(vals))


def chain_rule_distribution(U, inputs_order, rows_so_far) -> np.ndarray:
    """Unnormalised weights |perm(U_{rows+l, cols[:k]})|^2 over modes l for the
    next draw of chain-rule sampling (k = len(rows_so_far) + 1)."""
    k = len(rows_so_far) + 1
    out = extend_row(U, rows_so_far, list(inputs_order[:k]))
    return np.abs(out) ** 2


def chain_rule_sample(U, order, uniforms):
    """One chain-rule sample (Clifford & Clifford's algorithm A, named in the
    Boson Sampling benchmark section): with the input modes in the given order,
    draw r_k for k = 1..n by inverting the cumulative weights
    |perm(U_{rows + l, order[:k]})|^2 over l (summed in mode order) at
    u_k * total: r_k is the first l whose cumulative weight exceeds it.
    Returns (rows, margins): margins[k] is the distance of u_k * total from the
    nearest cumulative weight, relative to the total (decisions closer than
    rounding to a boundary may legitimately differ between implementations)."""
    rows, margins = [], []
    for k in range(1, len(order) + 1):
        w = chain_rule_distribution(U, order, rows)
        cdf = np.cumsum(w)
        target = float(uniforms[k - 1]) * cdf[-1]
        r = int(np.searchsorted(cdf, target, side="right"))
        r = min(r, len(w) - 1)
        rows.append(r)
        margins.append(float(np.min(np.abs(cdf - target))) / cdf[-1])
    return rows, margins


def loss_dilation(U, eta) -> np.ndarray:
    """2m-mode unitary of U followed, on every output mode i, by a beamsplitter
    with transmissivity eta_i to an environment mode m + i (Boson Sampling
    section: t = sqrt(eta), r = sqrt(1 - eta)).  Built as the product of the
    beamsplitter layer and U acting on the system modes:
        [[t, -r], [r, t]]  on (i, m + i),   then  U (+) I  before it."""
    U = np.asarray(U, dtype=np.complex128)
    m = U.shape[0]
    big = np.eye(2 * m, dtype=np.complex128)
    big[:m, :m] = U
    layer = np.eye(2 * m, dtype=np.complex128)
    for i in range(m):
        t, r = math.sqrt(eta[i]), math.sqrt(1.0 - eta[i])
        layer[i, i], layer[i, m + i] = t, -r
        layer[m + i, i], layer[m + i, m + i] = r, t
    return layer @ big


def loss_dilation_vw(V, eta, W) -> np.ndarray:
    """2m-mode unitary of the general lossy interferometer A = V diag(sqrt(eta)) W
    (the singular value form of the Boson Sampling section): W on the system
    modes, then the pure-loss beamsplitter layer of loss_dilation, then V on
    the system modes, multiplied out as matrices in that order."""
    V = np.asarray(V, dtype=np.complex128)
    W = np.asarray(W, dtype=np.complex128)
    m = V.shape[0]
    left = np.eye(2 * m, dtype=np.complex128)
    left[:m, :m] = V
    return left @ loss_dilation(W, eta)


def lossy_probability(U, eta, S, T, V=None) -> float:
    """Probability of detecting T (sum T <= sum S) on the system modes after
    U, the losses and (if given) V: the sum over environment patterns E of the
    ideal probability of (T, E) on the dilation, inputs in the system modes."""
    m = len(S)
    n = int(np.sum(S))
    k = n - int(np.sum(T))
    if k < 0:
        return 0.0
    Ud = loss_dilation(U, eta) if V is None else loss_dilation_vw(V, eta, U)
    S2 = np.concatenate([np.asarray(S, np.int32), np.zeros(m, np.int32)])
    total = 0.0
    for E in _compositions(m, k):
        T2 = np.concatenate([np.asarray(T, np.int32), np.asarray(E, np.int32)])
        total += probability(Ud, S2, T2)
    return total


def _compositions(m: int, k: int):
    if m == 1:
        yield [k]
        return
    for v in range(k + 1):
        for rest in _compositions(m - 1, k - v):
            yield [v] + rest


def beamsplitter_derivatives(theta: float, phi: float) -> tuple:
    """d/dtheta and d/dphi of the beamsplitter matrix [[t, -r*], [r, t]],
    t = cos(theta), r = e^{i phi} sin(theta), differentiated entry by entry."""
    c, s = math.cos(theta), math.sin(theta)
    e = complex(math.cos(phi), math.sin(phi))
    d_theta = np.array([[-s, -e.conjugate() * c], [e * c, -s]], dtype=np.complex128)
    d_phi = np.array([[0.0, 1j * e.conjugate() * s], [1j * e * s, 0.0]], dtype=np.complex128)
    return d_theta, d_phi


def mesh_jacobian(angles, cells, modes: int) -> np.ndarray:
    """dU/dtheta_q and dU/dphi_q of U = B_N ... B_1 by the product rule:
    dU/dx_q = (B_N ... B_{q+1}) (dB_q/dx) (B_{q-1} ... B_1).
    Returns an array of shape (N, 2, modes, modes)."""
    angles = np.asarray(angles, dtype=np.float64)
    N = len(cells)
    emb = []
    for (theta, phi), (a, b) in zip(angles, cells):
        B = np.eye(modes, dtype=np.complex128)
        B[np.ix_([a, b], [a, b])] = beamsplitter(theta, phi)
        emb.append(B)
    prefix = [np.eye(modes, dtype=np.complex128)]
    for q in range(N):
        prefix.append(emb[q] @ prefix[-1])          # prefix[q] = B_{q-1} ... B_1
    J = np.zeros((N, 2, modes, modes), dtype=np.complex128)
    suffix = np.eye(modes, dtype=np.complex128)      # B_N ... B_{q+1}
    for q in range(N - 1, -1, -1):
        (theta, phi), (a, b) = angles[q], cells[q]
        for k, d in enumerate(beamsplitter_derivatives(theta, phi)):
            D = np.zeros((modes, modes), dtype=np.complex128)
            D[np.ix_([a, b], [a, b])] = d
            J[q, k] = suffix @ D @ prefix[q]
        suffix = suffix @ emb[q]
    return J


def mesh_loss_grad(angles, cells, modes: int, S, patterns) -> np.ndarray:
    """d/d(theta_q, phi_q) of L = -(1/N) sum_p log(|perm(U_{T_p,S})|^2 / prod T_p!):
    dL/dx = -(2/N) sum_p Re( sum_ab d perm_p/dU_ab dU_ab/dx / perm_p )."""
    U = mesh_unitary(angles, cells, modes)
    J = mesh_jacobian(angles, cells, modes)
    total = np.zeros(J.shape[:2])
    for T in patterns:
        p = perm_mult(U, S, T)
        G = perm_grad(U, S, T)
        dp = np.einsum("ab,qkab->qk", G, J)
        total += np.real(dp / p)
    return -2.0 * total / len(patterns)


# ------------------------------------------------------------ loop hafnians
def lhaf_bruteforce(B, loops: bool = True):
    """Eq. loop_hafnian (Eq. haf_def when ``loops`` is False): the sum over
    every single-pair matching of the vertices 0..N-1 of the product of its
    edge weights B[i][j] (i < j) and loop weights B[i][i].  Each matching is
    listed once by matching the lowest remaining vertex first (the ordering
    condition under Eq. haf_def).  Works on any element type (Python ints
    give exact integers); N <= 12."""
    B = [list(row) for row in B]
    n = len(B)
    if any(len(row) != n for row in B) or n > 12:
        raise ValueError("square matrix with N <= 12 expected")

    def rec(rem):
        if not rem:
            return 1
        v, rest = rem[0], rem[1:]
        total = B[v][v] * rec(rest) if loops else 0
        for k, u in enumerate(rest):
            total = total + B[v][u] * rec(rest[:k] + rest[k + 1:])
        return total

    return rec(tuple(range(n)))


def expand_lhaf(A, gamma, reps) -> np.ndarray:
    """filldiag(A_r, gamma_r): mode i repeated r_i times; the diagonal holds
    gamma (zeros when gamma is None)."""
    A = _cplx(A)
    reps = [int(v) for v in reps]
    idx = [i for i, r in enumerate(reps) for _ in range(r)]
    B = A[np.ix_(idx, idx)].copy()
    np.fill_diagonal(B, 0.0 if gamma is None else np.asarray(gamma, np.complex128)[idx])
    return B


def lhaf_rep_ld(A, gamma, reps) -> tuple:
    A = _cplx(A)
    d = A.shape[0]
    if A.shape != (d, d):
        raise ValueError("square matrix expected")
    r = _occ(reps, d)
    g = None
    if gamma is not None:
        g = np.ascontiguousarray(np.asarray(gamma, dtype=np.complex128))
        if g.shape != (d,):
            raise ValueError("gamma must have length d")
    out = (ctypes.c_longdouble * 2)()
    st = _lib().orc_lhaf_rep(_dp(A), d, d, _dp(g) if g is not None else None,
                             r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), out)
    if st:
        raise RuntimeError(f"oracle error {st}")
    return out[0], out[1]


def lhaf_rep(A, gamma, reps) -> complex:
    """Loop hafnian of filldiag(A_r, gamma_r) (Eq. loop_hafnian; Appendix,
    GBS detection probability); gamma None: the hafnian (Eq. haf_def).  Reads
    the upper triangle of A."""
    re, im = lhaf_rep_ld(A, gamma, reps)
    return complex(float(re), float(im))

