"""GPU parity of the banded route (expm_pfd_band_*, through the C ABI) with the
oracle's R_d(tA)V of the matrix the band stores (Sec. 5's finite-difference
Laplacians and random Hermitian band matrices).

Tolerance, derived from the arithmetic: the FP64 gate of the dense path, 1e-12
relative, raised where the arithmetic cannot reach it.  Each pole's banded LU with
partial pivoting is backward stable, so its solution X_k carries an error of about
u kappa_k ||X_k|| (kappa_k the condition number of tA + theta_k I, which the
Laplacians' spectra reaching -4/h^2 make large), and the residue sum weighs these
by |a_k| (Prop. prop:digit): the gate is 8u sum_k |a_k| kappa_k ||X_k|| / ||Y||
where that exceeds 1e-12.  Sizes span both kernel families (one wave per pole up
to kd = 3, a workgroup per pole from kd = 4), ragged orders (n below kd + 1,
n = 1) and right-hand-side blocks (m = 1, 16, 17, 40, 64).
"""

import sys

import numpy as np
import pytest

from oracle import matrix, scalar

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def _announce(msg):
    print(f"[case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ep():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_16778_amd import expm_pfd
    expm_pfd.load_library()
    return expm_pfd


def _dev(x):
    import torch
    return torch.from_numpy(np.asfortranarray(x)).to("cuda")


def _amplification(w, W, t, d, c=0.0):
    """sum_k |e^c a_k| kappa_k ||(tw - c + theta_k)^{-1} W|| / ||e^c R_d(tw - c) W|| for
    the spectrum w and W = U^H V (all d poles), with kappa_k = max |tw - c + theta_k|
    / min |tw - c + theta_k|, the condition number of the normal matrix tA - cI +
    theta_k I."""
    theta, a = scalar.pfd_all(d)
    x = t * w - c
    num = 0.0
    for th, ak in zip(theta, a):
        z = np.abs(x + th)
        num += abs(ak) * (z.max() / z.min()) * np.linalg.norm(W / (x + th)[:, None])
    return float(num / np.linalg.norm(W * scalar.R_direct(x, d)[:, None]))


def _gate(A, V, t, d, c=0.0):
    w, U = np.linalg.eigh(A)
    return max(1e-12, 8 * U64 * _amplification(w, U.conj().T @ V, t, d, c))


def _random_case(n, kd, m, tscale, seed, real=False):
    """Random Hermitian band matrix, t chosen so that the spectrum of tA lies in
    about [-40 tscale, 0]."""
    from paper_2306_16778_amd import workloads as wl
    rng = np.random.default_rng(seed)
    AB, _ = wl.random_hermitian_band(rng, n, kd, spread=10.0, real=real)
    V = wl.complex_gaussian(rng, n, m)
    if real:
        V = V.real.astype(np.complex128)
    t = 40.0 * tscale / max(1.0, float(np.max(np.abs(AB[0].real))) * 2)
    return AB, V, t


CASES = [  # (n, kd, m)
    (1, 0, 1), (9, 0, 3), (1, 1, 1), (2, 1, 1), (300, 1, 16), (257, 1, 64),
    (3, 2, 17), (129, 2, 40), (2, 3, 1), (200, 3, 16),
    (4, 4, 2), (150, 4, 17), (257, 5, 1), (100, 7, 16), (64, 16, 40), (300, 16, 1),
    (1, 31, 1), (20, 31, 17), (250, 31, 64), (40, 63, 1), (64, 63, 16), (400, 63, 17),
]


@pytest.mark.parametrize("n,kd,m", CASES)
def test_band_parity_random(ep, n, kd, m):
    AB, V, t = _random_case(n, kd, m, 1.0, 7 * n + kd + m)
    _announce(f"band n={n} kd={kd} m={m} t={t:.3g}")
    plan = ep.expm_pfd_band_plan(n, kd, 16, m)
    X = ep.expm_pfd_band_apply(plan, t, _dev(AB), _dev(V)).cpu().numpy()
    A = matrix.band_to_dense(AB, kd)
    err = matrix.rel_fro(X, matrix.expm_R(A, V, t, 16))
    assert err <= _gate(A, V, t, 16), err


def _to_upper(AB, kd):
    """The same Hermitian matrix in upper band storage."""
    n = AB.shape[1]
    UB = np.zeros_like(AB)
    UB[kd] = AB[0]
    for k in range(1, kd + 1):
        UB[kd - k, k:] = np.conj(AB[k, : n - k])
    return UB


@pytest.mark.parametrize("n,kd", [(120, 2), (130, 9)])
def test_band_upper_storage_gives_the_same_bits(ep, n, kd):
    """The upper band storage of the same matrix gives identical results (the
    kernels read the same values either way)."""
    AB, V, t = _random_case(n, kd, 3, 0.7, 31 + kd)
    _announce(f"band uplo n={n} kd={kd}")
    lo = ep.expm_pfd_band_apply(ep.expm_pfd_band_plan(n, kd, 16, 3), t, _dev(AB), _dev(V)).cpu().numpy()
    up = ep.expm_pfd_band_apply(ep.expm_pfd_band_plan(n, kd, 16, 3, uplo="U"), t, _dev(_to_upper(AB, kd)),
                                _dev(V)).cpu().numpy()
    assert np.array_equal(lo, up)


@pytest.mark.parametrize("n,kd", [(150, 1), (150, 12)])
def test_band_real_data(ep, n, kd):
    """Real symmetric band matrix and real V with real_data: one solve per pole
    pair and 2 Re of the pair sum (Remark rem:two_time_real_part); a real result
    within the gate."""
    AB, V, t = _random_case(n, kd, 3, 1.0, 41 + kd, real=True)
    _announce(f"band real n={n} kd={kd}")
    X = ep.expm_pfd_band_apply(ep.expm_pfd_band_plan(n, kd, 16, 3, real_data=True), t, _dev(AB),
                               _dev(V)).cpu().numpy()
    assert np.all(X.imag == 0)
    A = matrix.band_to_dense(AB, kd)
    assert matrix.rel_fro(X, matrix.expm_R(A, V, t, 16)) <= _gate(A, V, t, 16)


@pytest.mark.parametrize("kd,d", [(2, 16), (6, 16), (6, 32), (1, 64)])
def test_band_shift_and_degree(ep, kd, d):
    """Spectrum with a positive part and the shift in units of A (c = t shift) against
    e^c R_d(tA - cI)V (Remark rem:shift), at degrees 16, 32 and 64."""
    from paper_2306_16778_amd import workloads as wl
    rng = np.random.default_rng(50 + kd + d)
    n = 120
    AB, _ = wl.random_hermitian_band(rng, n, kd, spread=5.0)
    top = 2.0 * kd + 5.0  # Gershgorin: the spectrum lies in [-top - ..., 0]; move it up by top
    AB[0] += top
    V = wl.complex_gaussian(rng, n, 2)
    t = 0.6
    _announce(f"band shift kd={kd} d={d}")
    plan = ep.expm_pfd_band_plan(n, kd, d, 2, shift=top + 1.0, shift_scale_t=True)
    X = ep.expm_pfd_band_apply(plan, t, _dev(AB), _dev(V)).cpu().numpy()
    A = matrix.band_to_dense(AB, kd)
    c = t * (top + 1.0)
    err = matrix.rel_fro(X, matrix.expm_R_shifted(A, V, t, d, c))
    assert err <= _gate(A, V, t, d, c), err


def _laplacian_gate(s, dim, v, t, d):
    """The FP64 gate for the Laplacian, its spectrum and U^H v from the sine transform."""
    from scipy import fft
    h = 1.0 / (s + 1)
    lam1 = -4.0 / h ** 2 * np.sin(np.arange(1, s + 1) * np.pi * h / 2) ** 2
    if dim == 1:
        return max(1e-12, 8 * U64 * _amplification(lam1, fft.dst(v, type=1, norm="ortho", axis=0), t, d))
    lam = (lam1[:, None] + lam1[None, :]).ravel()
    W = fft.dstn(v.reshape(s, s, -1), type=1, norm="ortho", axes=(0, 1)).reshape(s * s, -1)
    return max(1e-12, 8 * U64 * _amplification(lam, W, t, d))


@pytest.mark.parametrize("s,dim,t,d", [
    (1000, 1, 1.0, 16), (1000, 1, 1.0, 32), (1000, 1, 1e-5, 16),
    (32, 2, 1.0, 16), (32, 2, 1.0, 32), (32, 2, 1e-3, 16), (63, 2, 1e-3, 32),
])
def test_laplacian_paper_workloads(ep, s, dim, t, d):
    """exp(B)v and exp(C)v of Sec. 5.4 at the paper's orders (about 10^3; the 2D
    grid of 63 x 63 is the widest band the route takes), v random of norm 1,
    against the oracle's closed form through the sine transform.  The absolute
    error is also checked: the paper reports absolute errors for these matrices,
    and R_d(tB)v is far smaller than v at t = 1."""
    from paper_2306_16778_amd import workloads as wl
    AB, kd = wl.laplacian_1d_band(s) if dim == 1 else wl.laplacian_2d_band(s)
    n = AB.shape[1]
    rng = np.random.default_rng(60 + s + dim)
    v = wl.complex_gaussian(rng, n, 1)
    v /= np.linalg.norm(v)
    _announce(f"laplacian dim={dim} s={s} t={t} d={d}")
    X = ep.expm_pfd_band_apply(ep.expm_pfd_band_plan(n, kd, d, 1), t, _dev(AB), _dev(v)).cpu().numpy()
    Y = matrix.expm_R_laplacian(s, dim, v, t, d)
    assert matrix.rel_fro(X, Y) <= _laplacian_gate(s, dim, v, t, d)
    assert np.linalg.norm(X - Y) <= 1e-10


def test_laplacian_1d_large(ep):
    """The 1D Laplacian at 2 x 10^5 unknowns, two columns, t with the spectrum of tB
    in [-400, 0] (the oracle's sine-transform route reaches any order)."""
    from paper_2306_16778_amd import workloads as wl
    s = 200_000
    AB, kd = wl.laplacian_1d_band(s)
    rng = np.random.default_rng(70)
    V = wl.complex_gaussian(rng, s, 2)
    t = 100.0 / (s + 1) ** 2
    _announce(f"laplacian 1D s={s}")
    X = ep.expm_pfd_band_apply(ep.expm_pfd_band_plan(s, kd, 16, 2), t, _dev(AB), _dev(V)).cpu().numpy()
    Y = matrix.expm_R_laplacian(s, 1, V, t, 16)
    assert matrix.rel_fro(X, Y) <= _laplacian_gate(s, 1, V, t, 16)


def test_band_plan_reuse_and_errors(ep):
    """One plan serves several t, right-hand-side counts and matrices of its shape
    (each call matching a fresh plan's bits); bad arguments are rejected."""
    import torch
    n, kd = 90, 6
    AB, V, t = _random_case(n, kd, 20, 1.0, 80)
    plan = ep.expm_pfd_band_plan(n, kd, 16, 20)
    _announce("band plan reuse")
    for tt, mm in ((t, 20), (0.5 * t, 3), (t, 1)):
        X = ep.expm_pfd_band_apply(plan, tt, _dev(AB), _dev(V[:, :mm])).cpu().numpy()
        X1 = ep.expm_pfd_band_apply(ep.expm_pfd_band_plan(n, kd, 16, mm), tt, _dev(AB),
                                    _dev(V[:, :mm])).cpu().numpy()
        assert np.array_equal(X, X1)
    Vd = _dev(V)
    with pytest.raises(ep.ExpmPfdError) as e:  # more columns than the plan's m_max
        ep.expm_pfd_band_apply(ep.expm_pfd_band_plan(n, kd, 16, 4), t, _dev(AB), Vd)
    assert e.value.code == -2
    with pytest.raises(ep.ExpmPfdError) as e:
        ep.expm_pfd_band_apply(plan, float("inf"), _dev(AB), Vd)
    assert e.value.code == -7
    with pytest.raises(ep.ExpmPfdError) as e:  # band storage with too few rows for kd
        ep.expm_pfd_band_apply(plan, t, _dev(AB[:kd]), Vd)
    assert e.value.code == -4
    torch.cuda.synchronize()
