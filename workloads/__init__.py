"""Seeded synthetic inputs for the permanent engine.

This module is shared by the product's tests and benchmark and by the oracle's
tests.  It holds random draws and index bookkeeping only -- no permanent,
amplitude or gradient arithmetic -- so that neither side can borrow the other's
method through it.

Workload recipes (all seeded, all synthetic):

* ``haar(m, seed)``: Haar-random m x m unitary from the QR factorisation of a
  complex Gaussian matrix with the phases of diag(R) divided out (the paper's
  benchmarks use Haar-random interferometers; its plug-in example draws one
  with scipy's unitary group sampler).
* single permanents: the leading n x n block of ``haar(2 n^2, seed)``
  (collision-free regime d >> n^2 of the Boson Sampling section).
* repeated rows/columns: occupations drawn uniformly from
  {v in {0..cap}^modes : sum v = photons}, independently for input and output.
* boson sampling: a 400-mode Haar interferometer with photons in modes 0..19.
* differentiation: a 12-mode rectangular beamsplitter mesh with angles uniform
  in [0, 2 pi) and collision-free 8-photon output patterns drawn with
  replacement.
* loop hafnians: the symmetric matrix U diag(tanh r) U^T of d single-mode
  squeezers (r = arcsinh 1, the paper's GBS benchmark squeezing) followed by a
  Haar interferometer U, with a seeded complex loop vector for displacement;
  repetitions (2, ..., 2) as in the paper's hafnian benchmarks.
"""
from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np

__all__ = [
    "haar", "gaussian_matrix", "collision_free_block", "bounded_compositions",
    "repeated_patterns", "fock_outputs", "sampling_jobs", "mesh_angles",
    "mesh_patterns", "random_occupations", "MESH_MODES", "MESH_CELLS",
    "gbs_matrix", "loop_vector", "symmetric_gaussian",
]


def haar(m: int, seed: int) -> np.ndarray:
    """Haar-random m x m unitary (complex128, C-contiguous)."""
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return np.ascontiguousarray(q * (d / np.abs(d))[None, :])


def gaussian_matrix(n: int, seed: int, scale: float | None = None) -> np.ndarray:
    """n x n complex Gaussian matrix with entries ~ CN(0, scale^2) (default 1/n)."""
    rng = np.random.default_rng(seed)
    s = (1.0 / np.sqrt(n)) if scale is None else scale
    z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * (s / np.sqrt(2.0))
    return np.ascontiguousarray(z)


def gbs_matrix(d: int, seed: int, r: float = float(np.arcsinh(1.0))) -> np.ndarray:
    """Symmetric d x d matrix U diag(tanh r) U^T with U = haar(d, seed)."""
    U = haar(d, seed)
    return np.ascontiguousarray((U * np.tanh(r)) @ U.T)


def loop_vector(d: int, seed: int, scale: float = 0.5) -> np.ndarray:
    """Complex loop weights ~ CN(0, scale^2), seeded apart from the matrix."""
    rng = np.random.default_rng(10_000 + seed)
    z = (rng.standard_normal(d) + 1j * rng.standard_normal(d)) * (scale / np.sqrt(2.0))
    return np.ascontiguousarray(z)


def symmetric_gaussian(d: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """(Z + Z^T) / 2 with Z ~ CN(0, scale^2) entries."""
    z = gaussian_matrix(d, seed, scale)
    return np.ascontiguousarray((z + z.T) / 2.0)


def collision_free_block(n: int, seed: int) -> np.ndarray:
    """Leading n x n block of a Haar unitary on m = 2 n^2 modes."""
    return np.ascontiguousarray(haar(2 * n * n, seed)[:n, :n])


@lru_cache(maxsize=None)
def _composition_counts(parts: int, total: int, cap: int) -> tuple:
    # counts[p][s] = number of v in {0..cap}^p with sum s (exact Python ints)
    counts = [[0] * (total + 1) for _ in range(parts + 1)]
    counts[0][0] = 1
    for p in range(1, parts + 1):
        for s in range(total + 1):
            counts[p][s] = sum(counts[p - 1][s - v] for v in range(0, min(cap, s) + 1))
    return tuple(tuple(row) for row in counts)


def bounded_compositions(rng: np.random.Generator, parts: int, total: int, cap: int) -> np.ndarray:
    """One vector drawn uniformly from {v in {0..cap}^parts : sum v = total}."""
    counts = _composition_counts(parts, total, cap)
    if counts[parts][total] == 0:
        raise ValueError("no composition with these bounds")
    u = int(rng.integers(0, counts[parts][total]))
    out = np.zeros(parts, dtype=np.int32)
    s = total
    for p in range(parts, 0, -1):
        for v in range(0, min(cap, s) + 1):
            c = counts[p - 1][s - v]
            if u < c:
                out[parts - p] = v
                s -= v
                break
            u -= c
    return out


def repeated_patterns(count: int = 256, seed: int = 1, modes: int = 20,
                      photons: int = 40, cap: int = 4) -> list:
    """``count`` independent (S, T) pairs of bounded compositions."""
    rng = np.random.default_rng(seed)
    pats = []
    for _ in range(count):
        s = bounded_compositions(rng, modes, photons, cap)
        t = bounded_compositions(rng, modes, photons, cap)
        pats.append((s, t))
    return pats


def random_occupations(rng: np.random.Generator, modes: int, photons: int, cap: int | None = None) -> np.ndarray:
    """Occupation vector with ``photons`` photons thrown uniformly into modes
    (optionally capped per mode by redrawing)."""
    while True:
        v = np.bincount(rng.integers(0, modes, size=photons), minlength=modes).astype(np.int32)
        if cap is None or v.max(initial=0) <= cap:
            return v


def fock_outputs(modes: int, photons: int, at_most: bool = False) -> list:
    """All occupation vectors on ``modes`` modes with exactly ``photons`` photons
    (or with at most ``photons`` when ``at_most``), in lexicographic order."""
    out = []
    top = photons
    for v in itertools.product(range(top + 1), repeat=modes):
        s = sum(v)
        if s == photons or (at_most and s <= photons):
            out.append(np.array(v, dtype=np.int32))
    return out


def sampling_jobs(samples: int = 1000, photons: int = 20, modes: int = 400, seed: int = 0):
    """Synthetic row/column sequences with the shape of a Clifford-Clifford run.

    For every sample: a random order of the input modes 0..photons-1 and a
    sequence of ``photons - 1`` output modes drawn uniformly (with replacement).
    Step k (k = 2..photons) of a sample uses the first k-1 drawn rows and the
    first k ordered input columns.  Returns (cols[samples, photons],
    rows[samples, photons - 1]) as int32 arrays.
    """
    rng = np.random.default_rng(seed)
    cols = np.stack([rng.permutation(photons) for _ in range(samples)]).astype(np.int32)
    rows = rng.integers(0, modes, size=(samples, photons - 1)).astype(np.int32)
    return cols, rows


MESH_MODES = 12
# rectangular (Clements) layout: 12 columns alternating pairs (0,1),(2,3),...
# and (1,2),(3,4),...; 6*6 + 6*5 = 66 cells, two angles (theta, phi) each.
MESH_CELLS = tuple(
    (k, k + 1)
    for col in range(MESH_MODES)
    for k in range(col % 2, MESH_MODES - 1, 2)
)


def mesh_angles(seed: int = 0) -> np.ndarray:
    """(66, 2) array of (theta, phi), uniform in [0, 2 pi)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0 * np.pi, size=(len(MESH_CELLS), 2))


def mesh_patterns(count: int = 4096, seed: int = 1, modes: int = MESH_MODES, photons: int = 8) -> np.ndarray:
    """``count`` collision-free output patterns (0/1 vectors with ``photons``
    ones), each an independent uniform draw of a ``photons``-subset of the
    modes (so patterns may repeat)."""
    rng = np.random.default_rng(seed)
    out = np.zeros((count, modes), dtype=np.int32)
    for p in range(count):
        out[p, rng.choice(modes, size=photons, replace=False)] = 1
    return out
