"""Pins for the band side of the oracle and for the degree choice (CPU only).

``matrix.band_to_dense`` writes out the Hermitian matrix a band storage holds, and
``matrix.expm_R_band`` applies the dense definition to it.  They are pinned to
what does not use their code: the band read off a dense matrix through numpy's
diagonals, the closed-form eigenpairs of the finite-difference Laplacians of
Sec. 5 (sine eigenvectors; the 2D spectrum is the sum of two 1D spectra), and
R_d of those spectra by Horner.  ``scalar.choose_degree`` is pinned to what
Sec. 4 states about the bound of Prop. prop:digit and Fig. fig:maple.
"""

import math

import numpy as np
import pytest

from oracle import matrix, scalar
from paper_2306_16778_amd import workloads as wl


def _band_from_dense(H, kd, upper=False):
    """Band storage of H (declared width kd) through numpy diagonals, a route
    independent of band_to_dense."""
    n = H.shape[0]
    AB = np.zeros((kd + 1, n), dtype=np.complex128)
    for k in range(min(kd, n - 1) + 1):
        if upper:
            AB[kd - k, k:] = np.diagonal(H, k)
        else:
            AB[k, : n - k] = np.diagonal(H, -k)
    return AB


@pytest.mark.parametrize("n,kd", [(1, 0), (6, 0), (7, 1), (9, 3), (12, 11), (5, 7)])
def test_band_round_trip(n, kd):
    """A Hermitian matrix restricted to its band, stored (lower or upper) and written
    out again, is the same matrix; the imaginary part of the stored diagonal is
    never read."""
    rng = np.random.default_rng(100 + n + kd)
    G = wl.complex_gaussian(rng, n, n)
    H = G + G.conj().T
    i, j = np.indices((n, n))
    H[np.abs(i - j) > kd] = 0
    for upper in (False, True):
        AB = _band_from_dense(H, kd, upper)
        AB[kd if upper else 0, :] += 1j * rng.standard_normal(n)
        assert np.array_equal(matrix.band_to_dense(AB, kd, upper), H)


def _laplacian_1d_eig(n):
    h = 1.0 / (n + 1)
    k = np.arange(1, n + 1)
    lam = -4.0 / h ** 2 * np.sin(k * np.pi * h / 2) ** 2
    U = math.sqrt(2.0 * h) * np.sin(np.outer(k, k) * np.pi * h)
    return lam, U


def test_laplacian_1d_closed_form():
    """Delta^1 (Sec. 5): eigenvalues -(4/h^2) sin^2(k pi h / 2) with eigenvectors
    sqrt(2h) sin(i k pi h); R_d(tB)v from them matches the band oracle."""
    n = 40
    AB, kd = wl.laplacian_1d_band(n)
    lam, U = _laplacian_1d_eig(n)
    A = matrix.band_to_dense(AB, kd)
    assert np.allclose(A @ U, U * lam, rtol=0, atol=1e-9 * np.abs(lam).max())
    rng = np.random.default_rng(7)
    v = wl.complex_gaussian(rng, n, 2)
    t = 0.5 / (n + 1) ** 2 * 40  # spectrum of tB in about [-80, 0]
    want = U @ (scalar.R_direct(t * lam, 16)[:, None] * (U.T @ v))
    assert matrix.rel_fro(matrix.expm_R_band(AB, kd, v, t, 16), want) < 1e-13


def test_laplacian_2d_closed_form():
    """Delta^2 on an s x s grid (Sec. 5): the Kronecker sum of two Delta^1, so its
    eigenpairs are (lam_i + lam_j, u_i (x) u_j); the band oracle agrees."""
    s = 7
    AB, kd = wl.laplacian_2d_band(s)
    assert kd == s
    lam1, U1 = _laplacian_1d_eig(s)
    lam = (lam1[:, None] + lam1[None, :]).ravel()
    U = np.kron(U1, U1)
    A = matrix.band_to_dense(AB, kd)
    assert np.allclose(A @ U, U * lam, rtol=0, atol=1e-9 * np.abs(lam).max())
    rng = np.random.default_rng(8)
    v = wl.complex_gaussian(rng, s * s, 1)
    t = 1.0 / (s + 1) ** 2 * 10
    want = U @ (scalar.R_direct(t * lam, 16)[:, None] * (U.T @ v))
    assert matrix.rel_fro(matrix.expm_R_band(AB, kd, v, t, 16), want) < 1e-13


@pytest.mark.parametrize("s,dim", [(1, 1), (2, 1), (33, 1), (1, 2), (3, 2), (9, 2)])
def test_laplacian_sine_transform_route(s, dim):
    """The closed-form route through the sine transform (any order) equals the
    band oracle's dense route on the same Laplacian."""
    AB, kd = wl.laplacian_1d_band(s) if dim == 1 else wl.laplacian_2d_band(s)
    n = AB.shape[1]
    rng = np.random.default_rng(10 + s)
    v = wl.complex_gaussian(rng, n, 3)
    t = 20.0 / (s + 1) ** 2
    want = matrix.expm_R_band(AB, kd, v, t, 16)
    assert matrix.rel_fro(matrix.expm_R_laplacian(s, dim, v, t, 16), want) < 1e-13


def test_random_band_is_hermitian_with_nonpositive_spectrum():
    """The random band workload: Hermitian, spectrum within [-(R + spread), 0]
    (Gershgorin), for complex and real entries."""
    rng = np.random.default_rng(9)
    for real in (False, True):
        AB, kd = wl.random_hermitian_band(rng, 50, 5, spread=10.0, real=real)
        A = matrix.band_to_dense(AB, kd)
        assert np.array_equal(A, A.conj().T)
        w = np.linalg.eigvalsh(A)
        assert w.max() <= 0.0
        if real:
            assert np.all(A.imag == 0)


def test_shifted_band_oracle():
    """expm_R_band with a shift c is e^c R_d(tA - cI)V (Remark rem:shift): for a
    diagonal band (kd = 0) this is the scalar formula entry by entry."""
    lam = np.array([2.0, 0.5, -1.0, 3.0])
    AB = lam[None, :].astype(np.complex128)
    v = np.ones((4, 1), dtype=np.complex128)
    t, c = 0.7, 3.0
    want = np.exp(c) / np.array([sum((-(t * x - c)) ** k / math.factorial(k) for k in range(17)) for x in lam])
    assert np.allclose(matrix.expm_R_band(AB, 0, v, t, 16, c=c)[:, 0], want, rtol=1e-14, atol=0)


def test_choose_degree_closed_form_when_rounding_is_negligible():
    """With 34 digits M_2 is negligible, so the chosen degree is the smallest even d
    with 2^-d <= tol (Prop. pro:err)."""
    for tol in (1e-4, 1e-7, 1e-10, 1e-15):
        d, b, ok = scalar.choose_degree(tol, 34)
        want = next(e for e in range(2, 66, 2) if 2.0 ** -e <= tol)
        assert ok and d == want and b <= tol


def test_choose_degree_fp64_matches_the_paper():
    """Sec. 4, after Prop. prop:digit: in 16 digits the bound guarantees an error of
    order 1e-8 around d = 30 and nothing much smaller; so 1e-7 is met by some
    d <= 30, and 1e-10 by none (the best degree is in [26, 34], bound of order 1e-8)."""
    d, b, ok = scalar.choose_degree(1e-7, 16)
    assert ok and d <= 30
    d, b, ok = scalar.choose_degree(1e-10, 16)
    assert not ok and 26 <= d <= 34 and 1e-9 < b < 1e-7


def test_choose_degree_grows_with_the_digits():
    """Fig. fig:maple: the more significant digits, the later the error turns up,
    so the best degree grows with D."""
    best = [scalar.choose_degree(0.0, D)[0] for D in (7, 10, 16, 20, 24)]
    assert all(a < b for a, b in zip(best, best[1:])), best
