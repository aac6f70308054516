"""Matrix side of the method (paper Sec. 3, eqs. equ:ExpoMatRat and equ:expAx).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The library approximates exp(tA)V for Hermitian A by R_d(tA)V, where
R_d(z) = 1/exp_d(-z).  The method reaches R_d(tA)V exactly up to rounding, and
that result has a plain definition as a matrix function of a Hermitian matrix
(the paper extends any scalar approximation to diagonalizable matrices through
the eigendecomposition, Sec. 1):

    R_d(tA) V = U diag(1/exp_d(-t w_i)) U^H V,     A = U diag(w) U^H.

``expm_R`` writes that definition out; it never uses the partial fractions, so
the partial-fraction path is checked against an independent computation.
``expm_exact`` is the same with e^{t w_i}: it measures the approximation error,
it is not the parity target.

Conventions shared with the library's statement of the problem (not its code):
* A is given by its lower triangle (the strictly upper part is ignored and the
  imaginary part of the diagonal is dropped), so the operand is Hermitian by
  construction;
* V = None means V = I (the full matrix R_d(tA));
* arrays are numpy complex128; shapes (n, n) and (n, m).

The remaining functions are other routes to R_d(tA)V used only to pin this
oracle: exact partial-fraction sum and product form at 50 digits (n <= 8), and
matrix polynomial evaluation followed by a linear solve.
"""

from __future__ import annotations

import mpmath
import numpy as np

from . import scalar


def hermitian_from_lower(A: np.ndarray) -> np.ndarray:
    """The Hermitian matrix whose lower triangle is that of A (diagonal made real)."""
    A = np.asarray(A, dtype=np.complex128)
    L = np.tril(A, -1)
    return L + L.conj().T + np.diag(A.diagonal().real).astype(np.complex128)


def _eig(A: np.ndarray):
    # LAPACK zheevd through numpy, reading the lower triangle only.
    w, U = np.linalg.eigh(np.asarray(A, dtype=np.complex128), UPLO="L")
    return w, U


def _apply_spectral(U, f, V):
    """U diag(f) U^H V, with V = None meaning the identity."""
    if V is None:
        return (U * f[None, :]) @ U.conj().T
    V = np.asarray(V, dtype=np.complex128)
    return U @ (f[:, None] * (U.conj().T @ V))


def expm_R(A, V, t: float, d: int, eig=None):
    """R_d(tA) V by eigendecomposition (the oracle's definition of the result).

    r_i = 1/exp_d(-t w_i) is evaluated directly by Horner (Sec. 2.2).  For
    t w_i <= 0 every term is positive; eigenvalues with t w_i > 0 lie outside
    the domain the paper's bounds cover (Sec. 3, Theorem) but are still mapped.
    ``eig`` may pass a precomputed (w, U) of the same A.
    """
    scalar.check_degree(d)
    w, U = eig if eig is not None else _eig(A)
    r = scalar.R_direct(t * w, d)
    return _apply_spectral(U, r, V)


def expm_R_shifted(A, V, t: float, d: int, c: float, eig=None):
    """e^c R_d(tA - cI) V, the shifting method of Remark rem:shift, by
    eigendecomposition: r_i = e^c / exp_d(-(t w_i - c)) by Horner.  With c at or
    above the largest eigenvalue of tA every argument is <= 0, where the error
    bounds of Sec. 2.3 hold, and the relative error against exp(tA) is at most
    e^{c - alpha} max_{x <= 0} |R_d(x) - e^x| (alpha the largest eigenvalue)."""
    scalar.check_degree(d)
    w, U = eig if eig is not None else _eig(A)
    r = np.exp(c) * scalar.R_direct(t * w - c, d)
    return _apply_spectral(U, r, V)


def expm_exact(A, V, t: float, eig=None):
    """exp(tA) V = U diag(e^{t w_i}) U^H V (reported beside parity, never gated)."""
    w, U = eig if eig is not None else _eig(A)
    return _apply_spectral(U, np.exp(t * w), V)


def pfd_amplification(A, V, t: float, d: int, eig=None) -> float:
    """sum_k |a_k| ||(tA + theta_k I)^{-1} V||_F / ||R_d(tA) V||_F over all d poles.

    The rounding of each shifted solve (relative size u) enters the pole sum
    weighted by its residue, as in the scalar bound of Prop. prop:digit
    (sum_k |a_k| times the digit error); relative to the result this factor
    multiplies u.  So about u times this factor is the accuracy any FP64
    evaluation of the partial fractions can reach.  It is >= 1 (triangle
    inequality).  Frobenius norms are unitarily invariant, so with A = U
    diag(w) U^H only U^H V is needed.
    """
    w, U = eig if eig is not None else _eig(A)
    theta, a = scalar.pfd_all(d)
    W = U.conj().T if V is None else U.conj().T @ np.asarray(V, dtype=np.complex128)
    x = t * w
    num = sum(abs(ak) * np.linalg.norm(W / (x + th)[:, None]) for th, ak in zip(theta, a))
    den = np.linalg.norm(W * scalar.R_direct(x, d)[:, None])
    return float(num / den)


def band_to_dense(AB, kd: int, upper: bool = False) -> np.ndarray:
    """The Hermitian matrix stored in band form (the Laplacians of Sec. 5 and any
    Hermitian matrix with kd sub- and superdiagonals), written out by plain loops.

    Storage (LAPACK's band layout, column j of AB holding column j of A):
    lower: AB[i - j, j] = A[i, j] for j <= i <= min(n - 1, j + kd);
    upper: AB[kd + i - j, j] = A[i, j] for max(0, j - kd) <= i <= j.
    The other triangle follows by conjugation and the diagonal's imaginary part is
    dropped, as for the dense operand.
    """
    AB = np.asarray(AB, dtype=np.complex128)
    n = AB.shape[1]
    T = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        if upper:
            for i in range(max(0, j - kd), j + 1):
                T[j, i] = np.conj(AB[kd + i - j, j])  # the lower triangle's (j, i)
        else:
            for i in range(j, min(n, j + kd + 1)):
                T[i, j] = AB[i - j, j]
    return hermitian_from_lower(T)


def expm_R_band(AB, kd: int, V, t: float, d: int, c: float = 0.0, upper: bool = False):
    """R_d(tA)V (or e^c R_d(tA - cI)V with the shift) for A in band storage: the
    dense definition applied to the matrix the band stores."""
    A = band_to_dense(AB, kd, upper)
    return expm_R_shifted(A, V, t, d, c) if c else expm_R(A, V, t, d)


def expm_R_laplacian(s: int, dim: int, V, t: float, d: int):
    """R_d(tL)V for the Dirichlet finite-difference Laplacian L of Sec. 5 on s
    points per axis (dim = 1: B, order s; dim = 2: C, order s^2, unknowns numbered
    row by row), through its eigendecomposition in closed form: the orthonormal
    sine transform (DST-I) diagonalizes L with eigenvalues -(4/h^2) sin^2(k pi h/2)
    per axis, h = 1/(s+1), summed over the axes in 2D.  The transform is a library
    FFT, so any order the product path takes is within reach."""
    from scipy import fft

    h = 1.0 / (s + 1)
    lam1 = -4.0 / h ** 2 * np.sin(np.arange(1, s + 1) * np.pi * h / 2) ** 2
    V = np.asarray(V, dtype=np.complex128)
    m = V.shape[1]
    if dim == 1:
        W = fft.dst(V, type=1, norm="ortho", axis=0)
        return fft.dst(scalar.R_direct(t * lam1, d)[:, None] * W, type=1, norm="ortho", axis=0)
    lam = lam1[:, None] + lam1[None, :]  # (grid row, grid column)
    G = V.reshape(s, s, m)  # unknown i*s + j at grid row i, column j
    W = fft.dstn(G, type=1, norm="ortho", axes=(0, 1))
    return fft.dstn(scalar.R_direct(t * lam, d)[:, :, None] * W, type=1, norm="ortho", axes=(0, 1)).reshape(s * s, m)


def rel_fro(X, Y) -> float:
    """||X - Y||_F / ||Y||_F."""
    X = np.asarray(X)
    Y = np.asarray(Y)
    return float(np.linalg.norm(X - Y) / np.linalg.norm(Y))


# --------------------------------------------------------------------------
# routes used only to pin the oracle
# --------------------------------------------------------------------------

def _mp_matrix(M):
    return mpmath.matrix([[mpmath.mpc(complex(x)) for x in row] for row in np.asarray(M)])


def _solve_cols(M, B):
    """M^{-1} B column by column (mpmath's LU solve takes one right-hand side)."""
    out = mpmath.zeros(B.rows, B.cols)
    for j in range(B.cols):
        x = mpmath.lu_solve(M, B.column(j))
        for i in range(B.rows):
            out[i, j] = x[i]
    return out


def _to_numpy(M) -> np.ndarray:
    return np.array([[complex(M[i, j]) for j in range(M.cols)] for i in range(M.rows)], dtype=np.complex128)


def expm_R_pfd_mp(A, V, t: float, d: int, dps: int = 50):
    """sum_k a_k (tA + theta_k I)^{-1} V over all d poles at ``dps`` digits (eq. equ:ExpoMatRat / equ:expAx).

    Exact inversion by mpmath LU; for tiny n only (n <= 8).
    """
    Ah = hermitian_from_lower(A)
    n = Ah.shape[0]
    theta, a = scalar.pfd_full_mp(d)
    with mpmath.workdps(dps):
        tA = _mp_matrix(Ah) * mpmath.mpf(t)
        Vm = mpmath.eye(n) if V is None else _mp_matrix(V)
        S = mpmath.zeros(n, Vm.cols)
        for th, ak in zip(theta, a):
            S += ak * _solve_cols(tA + th * mpmath.eye(n), Vm)
        return _to_numpy(S)


def expm_R_product_mp(A, V, t: float, d: int, dps: int = 50):
    """d! prod_k (tA + theta_k I)^{-1} V at ``dps`` digits.

    exp_d(-z) = (1/d!) prod_k (z + theta_k) for even d, so R_d(z) = d!/prod_k (z + theta_k):
    this route uses the roots but no residue, hence no cancellation between residues.
    """
    Ah = hermitian_from_lower(A)
    n = Ah.shape[0]
    theta, _ = scalar.pfd_full_mp(d)
    with mpmath.workdps(dps):
        tA = _mp_matrix(Ah) * mpmath.mpf(t)
        Y = mpmath.eye(n) if V is None else _mp_matrix(V)
        for th in theta:
            Y = _solve_cols(tA + th * mpmath.eye(n), Y)
        return _to_numpy(Y * mpmath.factorial(d))


def expm_R_polysolve(A, V, t: float, d: int):
    """exp_d(-tA)^{-1} V: matrix Horner in FP64, then one LU solve.

    Uses neither eigenvectors, roots nor residues.  Accuracy degrades with
    cond(exp_d(-tA)) = exp_d(t rho) for tA <= 0, so pins use small t rho.
    """
    Ah = hermitian_from_lower(A)
    n = Ah.shape[0]
    Z = -t * Ah
    I = np.eye(n, dtype=np.complex128)
    S = I.copy()
    for k in range(d, 0, -1):
        S = I + (S @ Z) / k
    rhs = I if V is None else np.asarray(V, dtype=np.complex128)
    return np.linalg.solve(S, rhs)
