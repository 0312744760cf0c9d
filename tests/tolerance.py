"""Per-entry comparison with an absolute floor set by the sum's own scale.

A Glynn-type sum adds N = 2^(n-1) (or N mixed-radix) terms w prod_j c_j^k_j
whose magnitudes are far larger than the result: over the digit vectors the
column sum c_j = sum_i delta_i B_ij has mean square sum_i mu_i |B_ij|^2 (each
delta_i is a sum of mu_i independent signs), so the root-mean-square term is

    scale(U, S, T) = prod_j ( sum_i t_i |U_ij|^2 )^(s_j / 2).

Rounding leaves an error of order n * eps * scale whatever the value, so an
entry whose reference lies below that is compared in absolute terms against
the floor C * n * eps * scale; every other entry by its own relative error.
"""
import numpy as np

EPS = float(np.finfo(np.float64).eps)
FLOOR_C = 16.0


def term_scale(U, S, T) -> float:
    U = np.asarray(U)
    S = np.asarray(S)
    T = np.asarray(T)
    rows = np.flatnonzero(T > 0)
    cols = np.flatnonzero(S > 0)
    sub = np.abs(U[np.ix_(rows, cols)]) ** 2
    col = (sub * T[rows][:, None]).sum(axis=0)            # sum_i t_i |U_ij|^2 per column j
    return float(np.prod(col ** (S[cols] / 2.0)))


def floor_of(U, S, T) -> float:
    n = int(np.sum(S))
    return FLOOR_C * (n + 1) * EPS * term_scale(U, S, T)


def vjp_floor(U, Ss, Ts, g) -> np.ndarray:
    """Entrywise floor for dU = sum_p g_p conj(d perm_p / dU): the entry (a, b)
    of pattern p is t_a s_b perm(U_{T-e_a, S-e_b}), whose sum has its own scale."""
    U = np.asarray(U)
    m = U.shape[0]
    F = np.zeros((m, m))
    for S, T, gp in zip(Ss, Ts, g):
        S = np.asarray(S, dtype=np.int64)
        T = np.asarray(T, dtype=np.int64)
        for a in np.flatnonzero(T):
            for b in np.flatnonzero(S):
                S2, T2 = S.copy(), T.copy()
                S2[b] -= 1
                T2[a] -= 1
                F[a, b] += abs(gp) * T[a] * S[b] * floor_of(U, S2, T2)
    return F


def assert_entries_close(got, ref, rel, floor, what=""):
    """|got - ref| <= max(rel * |ref|, floor) for every entry (floor scalar or
    array); the message names the worst entry."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    err = np.abs(got - ref)
    allow = np.maximum(rel * np.abs(ref), floor)
    bad = err > allow
    if np.any(bad):
        ratio = np.where(allow > 0, err / np.where(allow > 0, allow, 1.0), np.inf)
        k = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
        raise AssertionError(f"{what} entry {k}: got {got[k]!r}, ref {ref[k]!r}, err {err[k]:.3e} > "
                             f"allowed {allow[k]:.3e} ({int(bad.sum())} of {bad.size} entries)")
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(np.abs(ref) > 0, err / np.abs(ref), 0.0)
    return float(np.max(r)) if r.size else 0.0


def extend_floor(U, job) -> np.ndarray:
    """Per-mode floor of an EXTEND_ROW job's outputs out[l] = perm(U_{T+e_l, S})
    (job in the binding's dict form: rows / cols as (mode, multiplicity))."""
    U = np.asarray(U)
    m = U.shape[0]
    S = np.zeros(m, np.int64)
    T = np.zeros(m, np.int64)
    for i, c in job["cols"]:
        S[i] += c
    for i, c in job["rows"]:
        T[i] += c
    F = np.zeros(m)
    for l in range(m):
        T[l] += 1
        F[l] = floor_of(U, S, T)
        T[l] -= 1
    return F
