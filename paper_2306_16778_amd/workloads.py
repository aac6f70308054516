"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and assembles Hermitian test matrices
A = U diag(lambda) U^H with a prescribed spectrum; it contains none of the
method's arithmetic (no Taylor polynomial, roots, residues or solves), so the
oracle and the GPU path can both be fed from it.

The paper's experiments use real symmetric matrices with a random spectrum in
a fixed interval and finite-difference Laplacians (Sec. 5.1-5.4).  The
workloads below keep those spectra (uniform in an interval, or the 1D
Laplacian-like -(pi k/(n+1))^2 * scale) on complex Hermitian matrices with
Haar-like random eigenvectors.  All arrays are numpy complex128; matrices are
returned C-contiguous with A[i, j] the (i, j) entry.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BASE_SEED = 20230629


def rng_for(config: int, index: int = 0) -> np.random.Generator:
    return np.random.default_rng([BASE_SEED, config, index])


def complex_gaussian(rng: np.random.Generator, *shape) -> np.ndarray:
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def random_unitary(rng: np.random.Generator, n: int) -> np.ndarray:
    """Q of the QR factorization of a complex Gaussian matrix, phases fixed so diag(R) > 0."""
    G = complex_gaussian(rng, n, n)
    Q, R = np.linalg.qr(G)
    ph = np.diag(R) / np.abs(np.diag(R))
    return Q * ph[None, :]


def householder_unitary_apply(rng: np.random.Generator, n: int, M: np.ndarray, reflections: int = 3) -> np.ndarray:
    """Return U M U^H for U = D H_1 ... H_r (random Householder reflections H and
    random phase diagonal D).  O(r n^2) instead of a QR: used where thousands
    of large matrices are needed."""
    vs = [complex_gaussian(rng, n) for _ in range(reflections)]
    phase = np.exp(2j * np.pi * rng.random(n))
    X = M.astype(np.complex128, copy=True)
    for v in reversed(vs):
        v = v / np.linalg.norm(v)
        # H = I - 2 v v^H ; X <- H X H^H
        X = X - 2.0 * np.outer(v, v.conj() @ X)
        X = X - 2.0 * np.outer(X @ v, v.conj())
    X = phase[:, None] * X * phase.conj()[None, :]
    return X


def hermitian_with_known_eigenbasis(rng: np.random.Generator, lam: np.ndarray, reflections: int = 3):
    """(A, U) with A = U diag(lam) U^H and U = D H_1 ... H_r returned densely.

    Same construction as ``householder_unitary_apply`` (random Householder
    reflections and a random phase diagonal), O(r n^2), so that the largest
    orders the library accepts come with their eigenvectors without an O(n^3)
    eigensolver or QR.  A is symmetrised like ``hermitian_with_spectrum``."""
    n = lam.shape[0]
    vs = [complex_gaussian(rng, n) for _ in range(reflections)]
    vs = [v / np.linalg.norm(v) for v in vs]
    phase = np.exp(2j * np.pi * rng.random(n))
    A = np.diag(lam.astype(np.complex128))
    U = np.eye(n, dtype=np.complex128)
    for v in reversed(vs):
        # H = I - 2 v v^H ; A <- H A H^H ; U <- H U
        A -= 2.0 * np.outer(v, v.conj() @ A)
        A -= 2.0 * np.outer(A @ v, v.conj())
        U -= 2.0 * np.outer(v, v.conj() @ U)
    A *= phase[:, None]
    A *= phase.conj()[None, :]
    U *= phase[:, None]
    A = 0.5 * (A + A.conj().T)
    return A, U


def hermitian_with_spectrum(rng: np.random.Generator, lam: np.ndarray, cheap: bool = False) -> np.ndarray:
    n = lam.shape[0]
    if cheap:
        A = householder_unitary_apply(rng, n, np.diag(lam.astype(np.complex128)))
    else:
        U = random_unitary(rng, n)
        A = (U * lam[None, :]) @ U.conj().T
    return 0.5 * (A + A.conj().T)


@dataclass
class Problem:
    """One exp(tA)V instance.  V is None for V = I (the full matrix R_d(tA))."""

    A: np.ndarray
    V: np.ndarray | None
    t: float
    degree: int
    lam: np.ndarray | None = None
    name: str = ""


def config1_plain_cpu_sized(n: int = 64) -> Problem:
    """Dense Hermitian A, n = 64, spectrum uniform in [-10, 0]; t = 1; degree 16; V = I."""
    rng = rng_for(1)
    lam = rng.uniform(-10.0, 0.0, n)
    return Problem(hermitian_with_spectrum(rng, lam), None, 1.0, 16, lam, f"herm_n{n}_d16_VI")


def config2_fp64_at_scale(n: int = 2048, m: int = 16) -> Problem:
    """Dense Hermitian A, n = 2048, spectrum uniform in [-100, 0]; V n x 16 Gaussian; t = 1; degree 24."""
    rng = rng_for(2)
    lam = rng.uniform(-100.0, 0.0, n)
    A = hermitian_with_spectrum(rng, lam)
    V = complex_gaussian(rng, n, m)
    return Problem(A, V, 1.0, 24, lam, f"herm_n{n}_m{m}_d24")


def laplacian_like_spectrum(n: int, scale: float = 4e3) -> np.ndarray:
    """lambda_k = -scale (pi k/(n+1))^2, k = 1..n (1D Laplacian-like spectrum)."""
    k = np.arange(1, n + 1, dtype=np.float64)
    return -scale * (np.pi * k / (n + 1)) ** 2


def config3_precision(n: int = 4096, with_eigenvectors: bool = False):
    """Dense Hermitian A, n = 4096, 1D-Laplacian-like spectrum scaled by 4e3; V = I; degree 32.

    with_eigenvectors: also return the unitary U with A = U diag(lambda) U^H (before the
    final symmetrisation), as (problem, U)."""
    rng = rng_for(3)
    lam = laplacian_like_spectrum(n)
    U = random_unitary(rng, n)
    A = (U * lam[None, :]) @ U.conj().T
    prob = Problem(0.5 * (A + A.conj().T), None, 1.0, 32, lam, f"lap_n{n}_d32_VI")
    return (prob, U) if with_eigenvectors else prob


def config4_batch(count: int = 512, n_lo: int = 32, n_hi: int = 512, m: int = 4):
    """count independent Hermitian matrices, n log-uniform in [n_lo, n_hi], spectrum uniform in
    [-50, 0], V n x m Gaussian, t uniform in [0.1, 1], degree 16."""
    rng = rng_for(4)
    ns = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), count))).astype(int)
    out = []
    for i, n in enumerate(ns):
        r = rng_for(4, i + 1)
        lam = r.uniform(-50.0, 0.0, n)
        A = hermitian_with_spectrum(r, lam)
        V = complex_gaussian(r, n, m)
        t = float(r.uniform(0.1, 1.0))
        out.append(Problem(A, V, t, 16, lam, f"batch{i}_n{n}"))
    return out


@dataclass
class Request:
    arrival_s: float
    matrix_id: int
    n: int
    t: float
    v: np.ndarray
    reuse: bool


def config5_requests(count: int, qps: float, n_lo: int = 64, n_hi: int = 4096, reuse_frac: float = 0.2):
    """Poisson arrivals at ``qps``; n log-uniform in [n_lo, n_hi]; single Gaussian vector per request;
    t uniform in [0.1, 1]; a fraction ``reuse_frac`` reuses an earlier matrix with a new t.

    Returns (requests, matrix_spec) where matrix_spec[id] = (n, seed index) and the
    matrix itself is built lazily by ``config5_matrix`` (spectrum uniform in [-200, 0],
    cheap Householder eigenvectors)."""
    rng = rng_for(5)
    gaps = rng.exponential(1.0 / qps, count)
    arrivals = np.cumsum(gaps)
    reqs = []
    specs = []
    for i in range(count):
        reuse = bool(specs) and rng.random() < reuse_frac
        if reuse:
            mid = int(rng.integers(0, len(specs)))
        else:
            n = int(np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
            specs.append((n, len(specs)))
            mid = len(specs) - 1
        n = specs[mid][0]
        t = float(rng.uniform(0.1, 1.0))
        v = complex_gaussian(rng, n, 1)
        reqs.append(Request(float(arrivals[i]), mid, n, t, v, reuse))
    return reqs, specs


def config5_matrix(spec) -> np.ndarray:
    n, idx = spec
    r = rng_for(5, idx + 1)
    lam = r.uniform(-200.0, 0.0, n)
    return hermitian_with_spectrum(r, lam, cheap=True)


def config5_eigenpairs(spec):
    """(lambda, U) of the config-5 matrix of ``spec``: the spectrum and the unitary
    U = D H_1 H_2 H_3 it is built from (same seeded draws as ``config5_matrix``),
    so that results can be checked without an eigensolver at any order."""
    n, idx = spec
    r = rng_for(5, idx + 1)
    lam = r.uniform(-200.0, 0.0, n)
    vs = [complex_gaussian(r, n) for _ in range(3)]
    phase = np.exp(2j * np.pi * r.random(n))
    U = np.eye(n, dtype=np.complex128)
    for v in reversed(vs):
        v = v / np.linalg.norm(v)
        U -= 2.0 * np.outer(v, v.conj() @ U)
    U *= phase[:, None]
    return lam, U


def config5_matrix_device(spec, device="cuda"):
    """The config-5 matrix of ``spec`` assembled on the GPU with torch, from the same
    seeded draws as ``config5_matrix`` (spectrum uniform in [-200, 0], three
    Householder reflections and a phase diagonal), in two device passes: with the
    reflections in compact WY form H_1 H_2 H_3 = I - V T V^H (T from the 3 x 3 inner
    products, LAPACK's forward accumulation), U diag(lam) U^H is diag(lam) plus a
    rank-6 product P Q^H whose factors take O(n) host work.  Rounding differs from
    the CPU assembly and the result is Hermitian to rounding (the library reads
    one triangle), so checks must copy these bytes back rather than rebuild them."""
    import torch

    n, idx = spec
    r = rng_for(5, idx + 1)
    lam = r.uniform(-200.0, 0.0, n)
    vs = [complex_gaussian(r, n) for _ in range(3)]
    phase = np.exp(2j * np.pi * r.random(n))
    V = np.stack([v / np.linalg.norm(v) for v in vs], axis=1)
    G = V.conj().T @ V
    T = np.zeros((3, 3), dtype=np.complex128)
    for j in range(3):  # tau = 2 for unit reflectors
        T[:j, j] = -2.0 * (T[:j, :j] @ G[:j, j])
        T[j, j] = 2.0
    LV = lam[:, None] * V
    M = T @ (V.conj().T @ LV) @ T.conj().T
    # U L U^H = L - V T (LV)^H - (LV) T^H V^H + V M V^H = L + P Q^H, then D (.) D^H
    P = phase[:, None] * np.concatenate([V, LV], axis=1)
    Q = phase[:, None] * np.concatenate([V @ M.conj().T - LV @ T.conj().T, -(V @ T)], axis=1)
    host = torch.from_numpy(np.concatenate([P, np.ascontiguousarray(Q.conj().T).T, lam[:, None] + 0j], axis=1))
    draws = host.pin_memory().to(device, non_blocking=True) if str(device).startswith("cuda") else host
    Pd, Qhd = draws[:, :6], draws[:, 6:12].T
    A = Pd @ Qhd.contiguous()
    A.diagonal().add_(draws[:, 12])
    return A


# --------------------------------------------------------------------------
# banded workloads: the finite-difference Laplacians of Sec. 5 (B = 1D, C = 2D)
# and random Hermitian band matrices, in lower band storage (kd + 1, n):
# AB[i - j, j] = A[i, j] for j <= i <= j + kd
# --------------------------------------------------------------------------

def laplacian_1d_band(n: int):
    """(AB, kd) of the 1D Dirichlet finite-difference Laplacian on n interior
    points of [0, 1]: (u_{i-1} - 2 u_i + u_{i+1}) / h^2, h = 1 / (n + 1)."""
    h2 = float(n + 1) ** 2
    AB = np.zeros((2, n), dtype=np.complex128)
    AB[0, :] = -2.0 * h2
    AB[1, : n - 1] = h2
    return AB, 1


def laplacian_2d_band(s: int):
    """(AB, kd) of the 2D five-point Dirichlet Laplacian on an s x s grid of the
    unit square, unknowns numbered row by row (n = s^2, kd = s), h = 1 / (s + 1)."""
    n = s * s
    h2 = float(s + 1) ** 2
    AB = np.zeros((s + 1, n), dtype=np.complex128)
    AB[0, :] = -4.0 * h2
    for j in range(n):
        if (j + 1) % s != 0:  # east neighbour in the same grid row
            AB[1, j] = h2
        if j + s < n:  # north neighbour
            AB[s, j] = h2
    return AB, s


def random_hermitian_band(rng: np.random.Generator, n: int, kd: int, spread: float = 10.0, real: bool = False):
    """Random Hermitian band matrix with spectrum in roughly [-(R + spread), 0]:
    Gaussian entries in the band, each diagonal entry set to minus its row's
    off-diagonal absolute sum (Gershgorin) minus uniform(0, spread)."""
    AB = np.zeros((kd + 1, n), dtype=np.complex128)
    kw = min(kd, n - 1)  # diagonals that exist
    for k in range(1, kw + 1):
        g = rng.standard_normal(n - k) if real else complex_gaussian(rng, n - k)
        AB[k, : n - k] = g
    rad = np.zeros(n)
    for k in range(1, kw + 1):
        rad[: n - k] += np.abs(AB[k, : n - k])  # A[j + k, j] in column j ...
        rad[k:] += np.abs(AB[k, : n - k])  # ... and its conjugate in row j
    AB[0, :] = -rad - rng.uniform(0.0, spread, n)
    return AB, kd
