"""Scalar side of the method (paper Sec. 2, Sec. 4 and Remark rem:two_time_real_part).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation follows the paper, with one rename: the paper's truncation order ``n``
is called ``d`` here (the degree), because ``n`` is the matrix size elsewhere.

* exp_d(z) = sum_{k=0}^{d} z^k / k!                         (Sec. 2, first display)
* theta_k  = the d roots of exp_d                            (Sec. 2.1)
* R_d(z)   = 1 / exp_d(-z)                                   (Sec. 2.2)
* R_d(z)   = sum_k a_k / (z + theta_k)                       (Prop. pro:dec, eq. yoyo)
* a_k      = -d! / prod_{j != k} (theta_k - theta_j)         (eq. yoyo2)
* a_k      = -1 / exp_d'(theta_k) = d! / theta_k^d           (eq. yoyo234)
* |R_d(x) - e^x| <= M_1(d) = 2^{-d} for x <= 0               (Prop. pro:err)
* rounding bound M_2(d, D)                                   (Prop. prop:digit)

Extended precision comes from mpmath; FP64 values are produced only by rounding
the extended values (the paper's "exact first 16 digits" reading of eq. yoyo2).
"""

from __future__ import annotations

import math
from functools import lru_cache

import mpmath
import numpy as np

# Lower bound on the distance between two roots of exp_d, for every d >= 2
# (eq. eq:ecart).  The paper prints it to five digits.
GAMMA = 0.29044

_DPS = 60  # working decimal digits for the extended-precision routines


def check_degree(d: int) -> None:
    """The paper assumes d even from Sec. 2.2 on (R_d then has no real pole)."""
    if not isinstance(d, (int, np.integer)) or d < 2 or d % 2:
        raise ValueError(f"degree must be an even integer >= 2, got {d!r}")


# --------------------------------------------------------------------------
# exp_d and R_d evaluated directly (no roots, no residues)
# --------------------------------------------------------------------------

def exp_d(z, d: int):
    """Truncated Taylor series exp_d(z) = sum_{k<=d} z^k/k! (Sec. 2).

    Horner form: s = 1; for k = d..1: s = 1 + s*z/k.  Works for Python/numpy
    floats and complexes and for mpmath numbers alike.
    """
    s = 1
    for k in range(d, 0, -1):
        s = 1 + s * z / k
    return s


def R_direct(x, d: int):
    """R_d(x) = 1/exp_d(-x) (Sec. 2.2), evaluated directly by Horner.

    For x <= 0 every term of exp_d(-x) is positive, so in FP64 the relative
    error is a few d ulps.  This is the value the matrix oracle maps the
    eigenvalues through; it never touches the partial fractions.
    """
    return 1.0 / exp_d(-x, d)


# --------------------------------------------------------------------------
# roots and residues at extended precision
# --------------------------------------------------------------------------

@lru_cache(maxsize=None)
def roots_mp(d: int, dps: int = _DPS):
    """The d roots theta_k of exp_d at ``dps`` digits (Sec. 2.1).

    mpmath.polyroots (Durand-Kerner) on the coefficients 1/k!, highest degree
    first, with extra working precision; returned as a tuple of mpc.
    """
    check_degree(d)
    with mpmath.workdps(dps):
        coeffs = [mpmath.mpf(1) / mpmath.factorial(k) for k in range(d, -1, -1)]
        r = mpmath.polyroots(coeffs, maxsteps=400, extraprec=4 * dps)
        return tuple(mpmath.mpc(z) for z in r)


def residues_yoyo2_mp(theta, d: int, dps: int = _DPS):
    """a_k = -d! / prod_{j != k} (theta_k - theta_j)  (eq. yoyo2)."""
    with mpmath.workdps(dps):
        out = []
        for k, tk in enumerate(theta):
            p = mpmath.mpc(1)
            for j, tj in enumerate(theta):
                if j != k:
                    p *= tk - tj
            out.append(-mpmath.factorial(d) / p)
        return tuple(out)


def residues_power_mp(theta, d: int, dps: int = _DPS):
    """a_k = d! / theta_k^d  (second form of eq. yoyo234)."""
    with mpmath.workdps(dps):
        return tuple(mpmath.factorial(d) / t ** d for t in theta)


def residues_derivative_mp(theta, d: int, dps: int = _DPS):
    """a_k = -1 / exp_d'(theta_k) = -1 / exp_{d-1}(theta_k)  (first form of eq. yoyo234)."""
    with mpmath.workdps(dps):
        return tuple(-1 / exp_d(t, d - 1) for t in theta)


@lru_cache(maxsize=None)
def pfd_full_mp(d: int, dps: int = _DPS):
    """All d (theta_k, a_k) at extended precision, residues by eq. yoyo2."""
    th = roots_mp(d, dps)
    return th, residues_yoyo2_mp(th, d, dps)


# --------------------------------------------------------------------------
# FP64 constants: one representative per conjugate pair
# --------------------------------------------------------------------------

def pfd_pairs(d: int):
    """FP64 poles/residues, one per conjugate pair (Remark rem:two_time_real_part).

    For even d the roots come in d/2 conjugate pairs, none real (Sec. 2.1), and
    so do the residues.  We keep the member with Im theta > 0 and order the
    pairs by ascending Re theta (ties: ascending Im theta).  Values are the
    extended-precision ones rounded to FP64.

    Returns (theta, a), two complex128 arrays of length d/2.
    """
    th, a = pfd_full_mp(d)
    rows = [(complex(t), complex(r)) for t, r in zip(th, a) if mpmath.im(t) > 0]
    rows.sort(key=lambda p: (p[0].real, p[0].imag))
    if len(rows) != d // 2:
        raise RuntimeError("roots did not split into conjugate pairs")
    theta = np.array([p[0] for p in rows], dtype=np.complex128)
    a = np.array([p[1] for p in rows], dtype=np.complex128)
    return theta, a


def pfd_all(d: int):
    """FP64 poles/residues for all d roots (each pair plus its conjugate)."""
    theta, a = pfd_pairs(d)
    return np.concatenate([theta, theta.conj()]), np.concatenate([a, a.conj()])


# --------------------------------------------------------------------------
# partial-fraction evaluation (scalar)
# --------------------------------------------------------------------------

def pfd_eval(x, theta, a):
    """sum_k a_k/(x + theta_k) over the given poles (eq. yoyo), FP64 complex.

    ``theta`` and ``a`` must list every pole (use ``pfd_all``).  ``x`` may be an
    array; the sum runs in the order given.
    """
    x = np.asarray(x, dtype=np.complex128)
    s = np.zeros_like(x)
    for t, r in zip(theta, a):
        s = s + r / (x + t)
    return s


def pfd_eval_pairs(x, theta, a):
    """For real x: sum over pairs of 2 Re(a_k/(x + theta_k)) (Remark rem:two_time_real_part)."""
    x = np.asarray(x, dtype=np.float64)
    s = np.zeros_like(x)
    for t, r in zip(theta, a):
        s = s + 2.0 * (r / (x + t)).real
    return s


# --------------------------------------------------------------------------
# bounds printed in the paper
# --------------------------------------------------------------------------

def M1(d: int) -> float:
    """Uniform error bound |R_d(x) - e^x| <= 2^{-d} on x <= 0 (Prop. pro:err)."""
    return 2.0 ** (-d)


def M2(d: int, D: int, abs_residue_sum: float) -> float:
    """Rounding bound of Prop. prop:digit with D significant digits.

    M_2 = (C_1(D) + C_2(d, D)) * sum_k |a~_k|, valid when gamma > d 10^{1-D}
    (eq. eq:condDn).
    """
    eps = 10.0 ** (1 - D)
    if not GAMMA > d * eps:
        raise ValueError("condition eq:condDn fails")
    c1 = 2 * eps / (GAMMA * (1 - eps))
    c2 = 4 * d * eps / (GAMMA * (GAMMA - d * eps))
    return (c1 + c2) * abs_residue_sum


def choose_degree(tol: float, D: int, d_max: int = 64):
    """Degree adapted to the arithmetic (Sec. 4: the precision must be adapted to
    the degree, Fig. fig:maple; the bound of Prop. prop:digit).

    With D significant digits the evaluated partial fractions differ from e^x on
    x <= 0 by at most M_1(d) + M_2(d, D): Prop. pro:err bounds R_d - e^x, Prop.
    prop:digit bounds the rounded sum against R_d, and the two add.  M_1 falls
    with d and M_2 grows with sum_k |a_k|, so the total has a smallest value.

    Returns (d, bound, guaranteed): the smallest even d in [2, d_max] whose total
    bound is at most tol (guaranteed True); when no degree meets tol, the even
    degree with the smallest total bound (guaranteed False).
    """
    best = None
    for d in range(2, d_max + 1, 2):
        _, a = pfd_all(d)
        b = M1(d) + M2(d, D, float(np.sum(np.abs(a))))
        if b <= tol:
            return d, b, True
        if best is None or b < best[1]:
            best = (d, b)
    return best[0], best[1], False


def err_shape(d: int, x):
    """err_d(x) = R_d(x) - e^x on x <= 0 (Prop. pro:wxcv1), at extended precision."""
    # near 0 the difference is O(x^{d+2}) (eq. equ:pade), hence the generous precision
    with mpmath.workdps(160):
        return [float(1 / exp_d(-mpmath.mpf(float(xi)), d) - mpmath.exp(mpmath.mpf(float(xi))))
                for xi in np.atleast_1d(x)]


def taylor_of_R_mp(d: int, order: int):
    """Taylor coefficients c_j of R_d(z) at 0, j = 0..order, from the power series of 1/exp_d(-z).

    Pure power-series division (no roots): used to pin eq. equ:pade and the
    lambda_{d,d+1}, lambda_{d,d+2} values of Sec. 2.2.
    """
    with mpmath.workdps(_DPS):
        q = [mpmath.mpf(-1) ** k / mpmath.factorial(k) if k <= d else mpmath.mpf(0) for k in range(order + 1)]
        c = [mpmath.mpf(0)] * (order + 1)
        for j in range(order + 1):
            s = mpmath.mpf(1) if j == 0 else mpmath.mpf(0)
            for i in range(1, j + 1):
                s -= q[i] * c[j - i]
            c[j] = s / q[0]
        return c


def factorial(k: int) -> int:
    return math.factorial(k)
