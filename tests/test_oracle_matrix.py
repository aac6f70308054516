"""Pins for the matrix oracle (paper Sec. 3): CPU only.

The oracle computes R_d(tA)V by eigendecomposition.  These tests pin it to
things that do not use its code path: the invariances of the Remark after
eq. equ:ExpoMatRat, the error theorem of Sec. 3, the exact partial-fraction
sum and product form at 50 digits on tiny matrices, and the matrix polynomial
exp_d(-tA) inverted by a linear solve.
"""

import math

import numpy as np
import pytest

from oracle import matrix, scalar
from paper_2306_16778_amd import workloads as wl


def _herm(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    lam = rng.uniform(lo, hi, n)
    return wl.hermitian_with_spectrum(rng, lam), lam, rng


def test_zero_matrix_gives_identity():
    """R_d(0) = I (Remark after eq. equ:ExpoMatRat)."""
    for d in (2, 16, 32):
        Y = matrix.expm_R(np.zeros((7, 7), complex), None, 1.0, d)
        assert np.array_equal(Y, np.eye(7))
        assert np.allclose(matrix.expm_exact(np.zeros((5, 5), complex), None, 1.0), np.eye(5))


def test_diagonal_gives_diagonal():
    """Diagonal D -> diagonal R_d(D) with entries R_d(D_ii) (Remark after eq. equ:ExpoMatRat)."""
    D = np.diag(np.array([-7.0, -0.3, 0.0, -20.0, -1.5]) + 0j)
    for t in (1.0, 0.37):
        Y = matrix.expm_R(D, None, t, 16)
        assert np.max(np.abs(Y - np.diag(np.diag(Y)))) == 0
        # exp_d written as the plain power sum of Sec. 2 (not the oracle's Horner form)
        want = 1.0 / np.array([sum((-t * x) ** k / math.factorial(k) for k in range(17))
                               for x in D.diagonal().real])
        assert np.allclose(np.diag(Y), want, rtol=1e-15, atol=0)


def test_similarity_invariance():
    """R_d(P A P^{-1}) = P R_d(A) P^{-1} (Remark after eq. equ:ExpoMatRat), with P unitary."""
    rng = np.random.default_rng(3)
    lam = rng.uniform(-30, 0, 40)
    U = wl.random_unitary(rng, 40)
    A = (U * lam) @ U.conj().T
    A = 0.5 * (A + A.conj().T)
    Y = matrix.expm_R(A, None, 0.8, 24)
    want = (U * (1.0 / scalar.exp_d(-0.8 * lam, 24))) @ U.conj().T
    assert matrix.rel_fro(Y, want) < 1e-13


def test_hpd_output_and_error_theorem():
    """Spec(tA) <= 0: R_d(tA) is Hermitian with eigenvalues in (0, 1]; R_d(tA) - exp(tA) >= 0 with
    2-norm <= 2^-d (Prop. pro:err), and <= R_d(-rho) - e^-rho when d > 2 rho (Theorem of Sec. 3)."""
    A, lam, _ = _herm(50, -25, 0, 11)
    for d in (8, 16, 24):
        R = matrix.expm_R(A, None, 1.0, d)
        E = matrix.expm_exact(A, None, 1.0)
        assert np.allclose(R, R.conj().T, atol=1e-14)
        ev = np.linalg.eigvalsh(R)
        assert ev.min() > 0 and ev.max() <= 1 + 1e-14
        diff = np.linalg.eigvalsh(R - E)
        assert diff.min() > -1e-15
        assert diff.max() <= scalar.M1(d)
    # theorem: small spectrum, d > 2 rho
    A, lam, _ = _herm(30, -3, 0, 12)
    rho = np.max(np.abs(lam))
    d = 8
    assert d > 2 * rho
    R = matrix.expm_R(A, None, 1.0, d)
    E = matrix.expm_exact(A, None, 1.0)
    eps = scalar.R_direct(-rho, d) - np.exp(-rho)
    assert np.linalg.norm(R - E, 2) <= eps * (1 + 1e-10)


def test_exp_oracle_group_property():
    """exp(A) exp(-A) = I, checked on the exact-exponential oracle."""
    A, _, _ = _herm(30, -4, 2, 13)
    E1 = matrix.expm_exact(A, None, 1.0)
    E2 = matrix.expm_exact(A, None, -1.0)
    assert np.allclose(E1 @ E2, np.eye(30), atol=1e-12)


@pytest.mark.parametrize("d", [2, 4, 8, 16])
def test_brute_force_tiny(d):
    """Tiny n: sum_k a_k (tA + theta_k I)^{-1} V (eq. equ:expAx) and d! prod_k (tA+theta_k I)^{-1} V
    at 50 digits both match the eigendecomposition oracle."""
    rng = np.random.default_rng(100 + d)
    n = 5
    lam = rng.uniform(-6, 0, n)
    A = wl.hermitian_with_spectrum(rng, lam)
    V = wl.complex_gaussian(rng, n, 2)
    t = 0.7
    Y = matrix.expm_R(A, V, t, d)
    Yp = matrix.expm_R_pfd_mp(A, V, t, d)
    Yq = matrix.expm_R_product_mp(A, V, t, d)
    assert matrix.rel_fro(Yp, Yq) < 1e-14
    assert matrix.rel_fro(Y, Yp) < 1e-14
    Yi = matrix.expm_R(A, None, t, d)
    Ypi = matrix.expm_R_pfd_mp(A, None, t, d)
    assert matrix.rel_fro(Yi, Ypi) < 1e-14


def test_polynomial_route():
    """exp_d(-tA)^{-1} by matrix Horner and a solve (no eigenvectors, roots or residues)."""
    A, _, rng = _herm(40, -2.5, 0, 21)
    V = wl.complex_gaussian(rng, 40, 3)
    for d in (6, 16):
        Y = matrix.expm_R(A, V, 1.0, d)
        Z = matrix.expm_R_polysolve(A, V, 1.0, d)
        assert matrix.rel_fro(Y, Z) < 1e-12
        assert matrix.rel_fro(matrix.expm_R(A, None, 1.0, d), matrix.expm_R_polysolve(A, None, 1.0, d)) < 1e-12


def test_block_and_identity_consistent():
    """R_d(tA)V equals R_d(tA) @ V."""
    A, _, rng = _herm(33, -40, 0, 31)
    V = wl.complex_gaussian(rng, 33, 4)
    Y = matrix.expm_R(A, V, 0.5, 16)
    Z = matrix.expm_R(A, None, 0.5, 16) @ V
    assert matrix.rel_fro(Y, Z) < 1e-13


def test_lower_triangle_only():
    """The operand is the Hermitian matrix defined by the lower triangle of A."""
    A, _, rng = _herm(20, -10, 0, 41)
    B = A.copy()
    B[np.triu_indices(20, 1)] = 1e3 * wl.complex_gaussian(rng, 190)
    B[np.diag_indices(20)] += 5j
    assert np.array_equal(matrix.expm_R(A, None, 1.0, 16), matrix.expm_R(B, None, 1.0, 16))


def test_approximation_error_is_tiny_but_nonzero():
    """The parity target is R_d, not exp: at d = 16, spectrum in [-10, 0], the two differ by ~1e-6
    (bounded by the maximum of err_16, Prop. pro:wxcv1)."""
    P = wl.config1_plain_cpu_sized()
    R = matrix.expm_R(P.A, None, 1.0, 16)
    E = matrix.expm_exact(P.A, None, 1.0)
    gap = np.linalg.norm(R - E, 2)
    assert 1e-8 < gap <= max(scalar.err_shape(16, np.linspace(-10, 0, 401)))


def test_shifted_oracle_pins():
    """Shifting method (Remark rem:shift): e^c R_d(tA - cI).
    - c = 0 is R_d(tA) itself;
    - a diagonal matrix maps entry-wise to e^c / exp_d(-(t D_ii - c)), written here as
      the plain power sum of Sec. 2;
    - for a positive spectrum with c = largest eigenvalue of tA, the relative 2-norm
      error against exp(tA) is at most max_{x <= 0} |R_d(x) - e^x| <= 2^-d (Prop. pro:err),
      while the unshifted R_d(tA) is far off there."""
    A, lam, _ = _herm(30, -20, 0, 21)
    assert matrix.rel_fro(matrix.expm_R_shifted(A, None, 0.7, 16, 0.0), matrix.expm_R(A, None, 0.7, 16)) == 0.0
    D = np.diag(np.array([3.0, 0.5, -2.0, 10.0]) + 0j)
    c = 10.0
    Y = matrix.expm_R_shifted(D, None, 1.0, 16, c)
    want = np.array([math.exp(c) / sum((-(x - c)) ** k / math.factorial(k) for k in range(17))
                     for x in D.diagonal().real])
    assert np.max(np.abs(Y - np.diag(np.diag(Y)))) == 0
    assert np.allclose(np.diag(Y).real, want, rtol=1e-14, atol=0)
    P, lamp, _ = _herm(40, 0, 30, 22)
    for d in (16, 24):
        c = float(lamp.max())
        Ys = matrix.expm_R_shifted(P, None, 1.0, d, c)
        E = matrix.expm_exact(P, None, 1.0)
        rel2 = np.linalg.norm(Ys - E, 2) / np.linalg.norm(E, 2)
        assert rel2 <= 2.0 ** -d
        # the maximum lies in [-(d+2), -d/2] (Prop. pro:wxcv1); grid step 0.01
        assert rel2 <= max(scalar.err_shape(d, np.arange(-(d + 2), -d / 2, 0.01))) * (1 + 1e-6)
        R0 = matrix.expm_R(P, None, 1.0, d)
        assert np.linalg.norm(R0 - E, 2) / np.linalg.norm(E, 2) > 1e-3


def test_pfd_amplification_pins():
    """The residue-weighted amplification factor of the oracle (the factor by which
    rounding of the shifted solves reaches the pole sum, Prop. prop:digit):
    * degree 2, closed form: theta = -1 +- i, a = +-i, R_2(x) = 1/(1 - x + x^2/2),
      so for one eigenvalue x the factor is (2/sqrt((x-1)^2 + 1)) / R_2(x)
      = sqrt((1 - x)^2 + 1);
    * it never goes below 1 (triangle inequality) and is unitarily invariant;
    * a result small against V (a spectrum far below 0) makes it large."""
    for x in (0.0, -0.5, -3.0, -12.0):
        A = np.array([[x]], dtype=np.complex128)
        got = matrix.pfd_amplification(A, np.ones((1, 1)), 1.0, 2)
        assert abs(got - math.sqrt((1.0 - x) ** 2 + 1.0)) < 1e-14 * got
    rng = np.random.default_rng(11)
    lam = rng.uniform(-40.0, 0.0, 30)
    D = np.diag(lam).astype(np.complex128)
    V = wl.complex_gaussian(rng, 30, 2)
    U = wl.random_unitary(rng, 30)
    a0 = matrix.pfd_amplification(D, V, 0.7, 16)
    a1 = matrix.pfd_amplification(U @ D @ U.conj().T, U @ V, 0.7, 16)
    assert a0 >= 1.0 and abs(a0 - a1) < 1e-10 * a0
    far = matrix.pfd_amplification(D - 100 * np.eye(30), V, 0.7, 16)
    assert far > 100 * a0
    # brute force at n = 4: exact inverses at 50 digits (no eigendecomposition)
    import mpmath
    B = wl.hermitian_with_spectrum(rng, rng.uniform(-15.0, 0.0, 4))
    W = wl.complex_gaussian(rng, 4, 2)
    th, a = scalar.pfd_full_mp(16)
    with mpmath.workdps(50):
        tB = matrix._mp_matrix(B) * mpmath.mpf(0.9)
        Wm = matrix._mp_matrix(W)
        num = sum(abs(ak) * mpmath.mnorm(matrix._solve_cols(tB + tk * mpmath.eye(4), Wm), "f")
                  for tk, ak in zip(th, a))
    ref = float(num) / np.linalg.norm(matrix.expm_R_pfd_mp(B, W, 0.9, 16))
    assert abs(matrix.pfd_amplification(B, W, 0.9, 16) - ref) < 1e-12 * ref
