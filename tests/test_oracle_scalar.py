"""Pins for the scalar oracle (paper Sec. 2 and Sec. 4): CPU only.

Each test checks the oracle against something other than itself: a closed
form, an identity that follows from a definition in the paper, a number the
paper prints (tests/golden/paper_facts.json), or a bound the paper proves.
"""

import json
import math
import os

import mpmath
import numpy as np
import pytest

from oracle import scalar

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))
DEGREES = [2, 4, 8, 16, 24, 32]


def test_degree2_closed_form():
    """exp_2(z) = 1 + z + z^2/2 has roots -1 +- i; eq. yoyo2 gives a = +-i (golden)."""
    g = GOLDEN["degree2_closed_form"]
    th, a = scalar.pfd_pairs(2)
    assert th.shape == (1,)
    assert abs(th[0] - complex(*g["theta"][0])) < 1e-15
    assert abs(a[0] - complex(*g["a"][0])) < 1e-15
    # R_2(z) = 2/(z^2 - 2z + 2) = 1/(1 - z + z^2/2) at a few points
    for z in [-3.0, -0.5, 0.0, 1.7j, -2 + 0.5j]:
        direct = 1.0 / (1 - z + z * z / 2)
        thf, af = scalar.pfd_all(2)
        assert abs(scalar.pfd_eval(z, thf, af) - direct) < 1e-15


@pytest.mark.parametrize("d", DEGREES)
def test_roots_reconstruct_polynomial(d):
    """prod_k (z - theta_k) / d! must have the coefficients 1/k! of exp_d (Sec. 2)."""
    th = scalar.roots_mp(d)
    assert len(th) == d
    with mpmath.workdps(60):
        poly = [mpmath.mpc(1)]  # coefficients, lowest degree first
        for t in th:
            nxt = [mpmath.mpc(0)] * (len(poly) + 1)
            for i, c in enumerate(poly):
                nxt[i] -= t * c
                nxt[i + 1] += c
            poly = nxt
        for k in range(d + 1):
            want = mpmath.mpf(1) / mpmath.factorial(k)
            got = poly[k] / mpmath.factorial(d)
            assert abs(got - want) <= mpmath.mpf(10) ** -40 * max(1, abs(want) * mpmath.factorial(d))


@pytest.mark.parametrize("d", DEGREES)
def test_root_facts(d):
    """Sec. 2.1: d/2 conjugate pairs, none real; 1 <= |theta| <= d (eq. equ:racn);
    no root strictly inside y^2 = 4(x+1); distinct roots at least gamma apart (eq. eq:ecart);
    |Im theta| >= gamma/2 (proof of Prop. prop:digit)."""
    th = [complex(t) for t in scalar.roots_mp(d)]
    gamma = GOLDEN["gamma"]["value"]
    for t in th:
        assert abs(t.imag) > 0.1
        assert 1.0 <= abs(t) <= d
        assert not (t.imag ** 2 < 4 * (t.real + 1))
        assert abs(t.imag) >= gamma / 2
        assert min(abs(t - s.conjugate()) for s in th) < 1e-30 + 1e-12  # conjugate present
    gaps = [abs(x - y) for i, x in enumerate(th) for y in th[i + 1:]]
    assert min(gaps) >= gamma
    thp, _ = scalar.pfd_pairs(d)
    assert len(thp) == d // 2 and np.all(thp.imag > 0)
    assert np.all(np.diff(thp.real) >= 0)


@pytest.mark.parametrize("d", DEGREES)
def test_residue_formulas_agree_extended(d):
    """eq. yoyo2 and both forms of eq. yoyo234 are equal in exact arithmetic."""
    th = scalar.roots_mp(d)
    a2 = scalar.residues_yoyo2_mp(th, d)
    ap = scalar.residues_power_mp(th, d)
    ad = scalar.residues_derivative_mp(th, d)
    for x, y, z in zip(a2, ap, ad):
        assert abs(x - y) <= 1e-45 * abs(x)
        assert abs(x - z) <= 1e-45 * abs(x)


@pytest.mark.parametrize("d", DEGREES)
def test_moment_identities(d):
    """Expansions of sum_k a_k/(z+theta_k) at 0 and at infinity.

    At 0 (eq. equ:pade): coefficient of z^j is 1/j! for j <= d, so
    sum_k a_k theta_k^{-(j+1)} = (-1)^j / j!;  lambda_{d,d+1} = 0 and
    lambda_{d,d+2} = -2(d+1) (Sec. 2.2, golden) fix the next two.
    At infinity R_d(z) ~ d!/z^d (exp_d(-z) has leading term z^d/d!, d even):
    sum_k a_k theta_k^j = 0 for j <= d-2 and sum_k a_k theta_k^{d-1} = -d!.
    """
    th, a = scalar.pfd_full_mp(d)
    with mpmath.workdps(60):
        tol = mpmath.mpf(10) ** -40
        for j in range(d + 1):
            s = sum(ak * tk ** (-(j + 1)) for tk, ak in zip(th, a))
            assert abs(s - mpmath.mpf(-1) ** j / mpmath.factorial(j)) < tol
        s1 = sum(ak * tk ** (-(d + 2)) for tk, ak in zip(th, a))
        assert abs(s1 * mpmath.factorial(d + 1) - GOLDEN["lambda_d_dplus1"]["value"]) < tol
        s2 = sum(ak * tk ** (-(d + 3)) for tk, ak in zip(th, a))
        # coefficient of z^{d+2} is (-1)^{d+2} s2 = lambda/(d+2)!
        assert abs(s2 * mpmath.factorial(d + 2) - (-2 * (d + 1))) < tol * mpmath.factorial(d + 2)
        for j in range(d - 1):
            assert abs(sum(ak * tk ** j for tk, ak in zip(th, a))) < tol * mpmath.factorial(d)
        assert abs(sum(ak * tk ** (d - 1) for tk, ak in zip(th, a)) + mpmath.factorial(d)) < tol * mpmath.factorial(d)


@pytest.mark.parametrize("d", [2, 8, 16, 32])
def test_taylor_of_R_power_series(d):
    """Power-series division alone reproduces eq. equ:pade and the printed lambda values."""
    c = scalar.taylor_of_R_mp(d, d + 2)
    with mpmath.workdps(60):
        for j in range(d + 1):
            assert abs(c[j] - mpmath.mpf(1) / mpmath.factorial(j)) < mpmath.mpf(10) ** -50
        assert abs(c[d + 1] * mpmath.factorial(d + 1)) < mpmath.mpf(10) ** -40
        assert abs(c[d + 2] * mpmath.factorial(d + 2) + 2 * (d + 1)) < mpmath.mpf(10) ** -40


@pytest.mark.parametrize("d", [4, 16, 24, 32])
def test_pfd_equals_direct(d):
    """Prop. pro:dec at extended precision, and Prop. prop:digit's bound M_2 for FP64 constants."""
    th, a = scalar.pfd_full_mp(d)
    with mpmath.workdps(60):
        for x in [-100, -37.5, -10, -1, -0.01, 0, 0.5, 3]:
            x = mpmath.mpf(x)
            s = sum(ak / (x + tk) for tk, ak in zip(th, a))
            assert abs(s - 1 / scalar.exp_d(-x, d)) < mpmath.mpf(10) ** -40
        # complex z away from the poles
        z = mpmath.mpc(-3, 2)
        s = sum(ak / (z + tk) for tk, ak in zip(th, a))
        assert abs(s - 1 / scalar.exp_d(-z, d)) < mpmath.mpf(10) ** -40
    thf, af = scalar.pfd_all(d)
    x = np.linspace(-100, 0, 4001)
    e3 = np.max(np.abs(scalar.pfd_eval(x, thf, af) - scalar.R_direct(x, d)))
    assert e3 <= scalar.M2(d, 16, float(np.sum(np.abs(af))))


@pytest.mark.parametrize("d", [2, 16, 32])
def test_pair_halving(d):
    """Remark rem:two_time_real_part: for real x the full sum equals sum over pairs of 2 Re."""
    thp, ap = scalar.pfd_pairs(d)
    thf, af = scalar.pfd_all(d)
    x = np.linspace(-60, 0, 301)
    full = scalar.pfd_eval(x, thf, af)
    half = scalar.pfd_eval_pairs(x, thp, ap)
    assert np.max(np.abs(full.imag)) < 1e-10
    assert np.max(np.abs(full.real - half)) < 1e-10


@pytest.mark.parametrize("d", [4, 8, 16, 24, 32])
def test_error_shape(d):
    """Prop. pro:err and Prop. pro:wxcv1: 0 < R_d(x) - e^x <= 2^-d on x < 0, one maximum at
    xi_d with d/2 <= -xi_d <= d+2 (eq. ineq:loc)."""
    xs = np.linspace(-3 * d - 10, -1e-3, 2000)
    err = np.array(scalar.err_shape(d, xs))
    assert np.all(err > 0)
    assert np.max(err) <= scalar.M1(d)
    i = int(np.argmax(err))
    xi = xs[i]
    assert d / 2 <= -xi <= d + 2
    # unimodal: increasing left of the max, decreasing right of it
    assert np.all(np.diff(err[: i + 1]) > -1e-300)
    assert np.all(np.diff(err[i:]) < 1e-300)


def test_paper_fp64_behaviour():
    """Sec. 4 (Fig. fig:ineg_triang, Prop. prop:digit): in FP64 the total error e_1 over [-100, 0]
    is smallest near d = 34; at d = 30 the bound is of order 1e-8 and the error of order 1e-10;
    eq. yoyo2 residues beat both forms of eq. yoyo234."""
    x = np.linspace(-100, 0, 2001)
    with mpmath.workdps(40):
        ex = np.array([float(mpmath.exp(xi)) for xi in x])
    e1 = {}
    for d in range(20, 46, 2):
        thf, af = scalar.pfd_all(d)
        e1[d] = np.max(np.abs(ex - scalar.pfd_eval(x, thf, af).real))
    best = min(e1, key=e1.get)
    g = GOLDEN["e1_min_degree_fp64"]
    assert abs(best - g["value"]) <= g["tolerance"]
    thf, af = scalar.pfd_all(30)
    m2 = scalar.M2(30, 16, float(np.sum(np.abs(af))))
    assert 1e-9 < m2 < 1e-7
    assert 1e-11 < e1[30] < 1e-9
    # residue formulas compared in FP64 (right panel of Fig. fig:ineg_triang), d = 32
    d = 32
    th = scalar.roots_mp(d)
    thc = np.array([complex(t) for t in th])
    rd = scalar.R_direct(x, d)
    errs = []
    for fn in (scalar.residues_yoyo2_mp, scalar.residues_power_mp, scalar.residues_derivative_mp):
        # the formula evaluated in FP64 from FP64 roots
        if fn is scalar.residues_yoyo2_mp:
            a = np.array([-math.factorial(d) / np.prod([tk - tj for j, tj in enumerate(thc) if j != k])
                          for k, tk in enumerate(thc)])
        elif fn is scalar.residues_power_mp:
            a = np.array([math.factorial(d) / tk ** d for tk in thc])
        else:
            a = np.array([-1.0 / scalar.exp_d(tk, d - 1) for tk in thc])
        errs.append(np.max(np.abs(scalar.pfd_eval(x, thc, a) - rd)))
    assert errs[0] <= errs[1] <= errs[2]


def test_condition_condDn():
    """Text after Prop. prop:digit: eq. eq:condDn holds with D = 16 even for d about 1e10."""
    g = GOLDEN["condDn_holds_1e10"]
    assert scalar.GAMMA > g["d"] * 10.0 ** (1 - g["D"])
    with pytest.raises(ValueError):
        scalar.M2(10 ** 16, 16, 1.0)


def test_degree_validation():
    for bad in [0, 1, 3, 17, -2]:
        with pytest.raises(ValueError):
            scalar.check_degree(bad)
