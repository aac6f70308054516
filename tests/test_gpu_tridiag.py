"""GPU parity of the tridiagonal route (A = Q T Q^H once, then R_d(tA)V for several
t by tridiagonal solves, through the C ABI) against the oracle's R_d(tA)V, with the
same tolerances as the FP64 path (1e-12, raised to 8u times the residue
amplification factor where that is larger: Prop. prop:digit), and the spectrum of
the computed T against the spectrum A is built with."""

import sys

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import matrix
from paper_2306_16778_amd import workloads as wl

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


def _gate(err, A, V, t, d, eig=None):
    return err <= max(1e-12, 8 * U64 * matrix.pfd_amplification(A, V, t, d, eig=eig))


CASES = [
    # n, spectrum, m, degree, t values
    (1, (-5.0, 0.0), 1, 16, (1.0, 0.3)),
    (2, (-10.0, 0.0), 2, 16, (1.0,)),
    (3, (-30.0, 0.0), 1, 8, (0.5, 1.0)),
    (64, (-10.0, 0.0), 4, 16, (1.0, 0.25)),
    (130, (-100.0, 0.0), 16, 24, (1.0, 0.6, 0.1)),
    (257, (-50.0, 0.0), 5, 16, (0.9,)),
    (700, (-200.0, 0.0), 1, 16, (1.0, 0.45, 0.1)),
]


@pytest.mark.parametrize("n,spec,m,d,ts", CASES)
def test_tridiag_parity_several_t(ep, n, spec, m, d, ts):
    import torch
    rng = np.random.default_rng([20230629, 81, n])
    lam = rng.uniform(*spec, n)
    A = wl.hermitian_with_spectrum(rng, lam)
    V = wl.complex_gaussian(rng, n, m)
    _announce(f"tridiag n={n} m={m} d={d} t={ts}")
    tri = ep.expm_pfd_tridiag_plan(n, d, m)
    ep.expm_pfd_tridiag_factor(tri, _dev(A))
    dd, ee = ep.expm_pfd_tridiag_diagonals(tri)
    mu = sl.eigvalsh_tridiagonal(dd, ee) if n > 1 else dd
    assert np.max(np.abs(np.sort(mu) - np.sort(lam))) < 1e-12 * np.max(np.abs(lam))
    eig = np.linalg.eigh(A)
    Vd = _dev(V)
    for t in ts:
        X = ep.expm_pfd_tridiag_apply(tri, t, Vd)
        torch.cuda.synchronize()
        err = matrix.rel_fro(X.cpu().numpy(), matrix.expm_R(A, V, t, d, eig=eig))
        print(f"  t={t}: rel_fro={err:.3e}", file=sys.stderr, flush=True)
        assert _gate(err, A, V, t, d, eig), err


def test_tridiag_large_order_known_eigenpairs(ep):
    """n = 4500 (reflector rows of up to 72 KB held in LDS by the fused reduction
    step): A of the serving workload's construction (spectrum U[-200, 0], unitary
    from three Householder reflections and a phase diagonal), checked against the
    oracle given those eigenpairs, with the spectrum of the computed T."""
    import torch
    spec = (4500, 7)
    n = spec[0]
    lam, U = wl.config5_eigenpairs(spec)
    A = wl.config5_matrix(spec)
    V = wl.complex_gaussian(np.random.default_rng(85), n, 2)
    _announce(f"tridiag n={n} m=2 d=16 (known eigenpairs)")
    tri = ep.expm_pfd_tridiag_plan(n, 16, 2)
    ep.expm_pfd_tridiag_factor(tri, _dev(A))
    dd, ee = ep.expm_pfd_tridiag_diagonals(tri)
    mu = sl.eigvalsh_tridiagonal(dd, ee)
    assert np.max(np.abs(np.sort(mu) - np.sort(lam))) < 1e-12 * np.max(np.abs(lam))
    Vd = _dev(V)
    for t in (1.0, 0.2):
        X = ep.expm_pfd_tridiag_apply(tri, t, Vd)
        torch.cuda.synchronize()
        err = matrix.rel_fro(X.cpu().numpy(), matrix.expm_R(A, V, t, 16, eig=(lam, U)))
        print(f"  t={t}: rel_fro={err:.3e}", file=sys.stderr, flush=True)
        assert _gate(err, A, V, t, 16, (lam, U)), err


def test_tridiag_config2_shape_and_reuse(ep):
    """The benchmarked shape (n = 2048, spectrum U[-100, 0], V 2048 x 16, degree 24):
    one reduction, then t = 1 (the LU path's workload) and two more t, each against
    the oracle; the t = 1 result also against the LU path's FP64 result."""
    import torch
    prob = wl.config2_fp64_at_scale()
    n, m = prob.V.shape
    _announce(f"tridiag config 2 n={n} m={m}")
    Ad, Vd = _dev(prob.A), _dev(prob.V)
    tri = ep.expm_pfd_tridiag_plan(n, 24, m)
    ep.expm_pfd_tridiag_factor(tri, Ad)
    eig = np.linalg.eigh(prob.A)
    for t in (1.0, 0.5, 0.05):
        X = ep.expm_pfd_tridiag_apply(tri, t, Vd)
        torch.cuda.synchronize()
        err = matrix.rel_fro(X.cpu().numpy(), matrix.expm_R(prob.A, prob.V, t, 24, eig=eig))
        print(f"  t={t}: rel_fro={err:.3e}", file=sys.stderr, flush=True)
        assert _gate(err, prob.A, prob.V, t, 24, eig), err
        if t == 1.0:
            plan = ep.expm_pfd_plan(n, 24, 1.0, m, "fp64")
            Y = ep.expm_pfd_apply(plan, Ad, Vd)
            torch.cuda.synchronize()
            assert matrix.rel_fro(X.cpu().numpy(), Y.cpu().numpy()) < 2e-12


def test_tridiag_options_and_errors(ep):
    """Shift in units of A (problem shifted by t c) against the oracle's shifted
    result; the upper triangle gives the same bits as the lower one (the other set
    to NaN); argument errors."""
    import torch
    rng = np.random.default_rng(83)
    n, m, c = 120, 3, 12.0
    A = wl.hermitian_with_spectrum(rng, rng.uniform(0.0, 12.0, n))
    V = wl.complex_gaussian(rng, n, m)
    _announce("tridiag shift and uplo")
    tri = ep.expm_pfd_tridiag_plan(n, 16, m, shift=c, shift_scale_t=True)
    ep.expm_pfd_tridiag_factor(tri, _dev(A))
    for t in (1.0, 0.3):
        X = ep.expm_pfd_tridiag_apply(tri, t, _dev(V))
        torch.cuda.synchronize()
        assert matrix.rel_fro(X.cpu().numpy(), matrix.expm_R_shifted(A, V, t, 16, t * c)) < 1e-12
    Alo, Aup = A.copy(), A.copy()
    Alo[np.triu_indices(n, 1)] = np.nan
    Aup[np.tril_indices(n, -1)] = np.nan
    res = []
    for uplo, M in (("L", Alo), ("U", Aup)):
        tr = ep.expm_pfd_tridiag_plan(n, 16, m, uplo=uplo)
        ep.expm_pfd_tridiag_factor(tr, _dev(M))
        res.append(ep.expm_pfd_tridiag_apply(tr, 0.7, _dev(V)).cpu().numpy())
    assert np.array_equal(res[0], res[1]) and np.all(np.isfinite(res[0]))
    fresh = ep.expm_pfd_tridiag_plan(n, 16, m)
    with pytest.raises(ep.ExpmPfdError) as e:  # not factored yet
        ep.expm_pfd_tridiag_apply(fresh, 1.0, _dev(V))
    assert e.value.code == -7
    with pytest.raises(ep.ExpmPfdError) as e:  # more columns than the plan takes
        ep.expm_pfd_tridiag_apply(tri, 1.0, _dev(wl.complex_gaussian(rng, n, 4)))
    assert e.value.code == -2
