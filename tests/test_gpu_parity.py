"""GPU parity: the HIP path (through the C ABI) against the oracle, element by element.

Tolerances are relative Frobenius errors against R_d(tA)V computed by the oracle
(eigendecomposition, FP64):
  FP64 path  1e-12 (degree <= 24, spectra in [-100, 0]; rounding of the shifted
             solves is amplified by sum_k |a_k| relative to |R_d(tA)V|, which grows
             with the degree: about 1e-11 is reached at degree 32);
  mixed path 1e-10 (FP32 factorization recovered by FP64 refinement).
Every case prints its name before it touches the GPU.
"""

import sys

import numpy as np
import pytest

from oracle import matrix, scalar
from paper_2306_16778_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOLMX = 1e-10


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


def _run(ep, A, V, t, d, precision="fp64", m_max=None, shift=0.0, real_data=False):
    import torch
    n = A.shape[0]
    mm = 0 if V is None else (V.shape[1] if m_max is None else m_max)
    plan = ep.expm_pfd_plan(n, d, t, mm, precision, shift=shift, real_data=real_data)
    X = ep.expm_pfd_apply(plan, _dev(A), None if V is None else _dev(V))
    torch.cuda.synchronize()
    ep.expm_pfd_plan_check(plan)  # every one-launch sweep kept its dependency order
    return X.cpu().numpy()


def _problem(n, lo, hi, m, seed, t=1.0):
    rng = np.random.default_rng(seed)
    lam = rng.uniform(lo, hi, n)
    A = wl.hermitian_with_spectrum(rng, lam)
    V = None if m is None else wl.complex_gaussian(rng, n, m)
    return A, V, t


CASES = [
    # n, spectrum, m (None: V = I), degree, t
    (1, (-5, 0), 1, 16, 1.0),
    (1, (-5, 0), None, 2, 1.0),
    (5, (-10, 0), 3, 2, 0.5),
    (33, (-50, 0), 4, 16, 0.3),
    (64, (-10, 0), None, 16, 1.0),
    (65, (-100, 0), 16, 24, 1.0),
    (100, (-100, 0), 1, 16, 0.7),
    (130, (-20, 0), None, 8, 1.0),
    (200, (-100, 0), 16, 24, 1.0),
    (257, (-100, 0), 5, 16, 1.0),
    (300, (-40, 0), None, 16, 0.9),
    (150, (-100, 0), 40, 16, 1.0),   # three 16-column chains per pole block
    (128, (-60, 0), 64, 16, 0.8),    # four chains: widest one-launch sweep
    (96, (-30, 0), 65, 16, 1.0),     # 80-column blocks: sweeps by block products
]


@pytest.mark.parametrize("n,spec,m,d,t", CASES)
def test_fp64_parity_small(ep, n, spec, m, d, t):
    A, V, _ = _problem(n, spec[0], spec[1], m, 1000 + n + d)
    _announce(f"fp64 n={n} m={m} d={d} t={t}")
    X = _run(ep, A, V, t, d)
    Y = matrix.expm_R(A, V, t, d)
    assert matrix.rel_fro(X, Y) < TOL64


@pytest.mark.parametrize("n,spec,m,d,t", CASES)
def test_mixed_parity_small(ep, n, spec, m, d, t):
    A, V, _ = _problem(n, spec[0], spec[1], m, 2000 + n + d)
    _announce(f"mixed n={n} m={m} d={d} t={t}")
    X = _run(ep, A, V, t, d, "mixed")
    Y = matrix.expm_R(A, V, t, d)
    assert matrix.rel_fro(X, Y) < TOLMX


def test_config1_full_exponential(ep):
    """n = 64, V = I, degree 16, spectrum in [-10, 0]."""
    P = wl.config1_plain_cpu_sized()
    _announce("config1 fp64 n=64 V=I d=16")
    X = _run(ep, P.A, None, P.t, P.degree)
    Y = matrix.expm_R(P.A, None, P.t, P.degree)
    assert matrix.rel_fro(X, Y) < TOL64
    assert np.array_equal(X, X.conj().T)  # Hermitian by construction (Y + Y^H form)
    E = matrix.expm_exact(P.A, None, P.t)
    assert matrix.rel_fro(X, E) < 1e-4  # approximation error of R_16, reported not gated


@pytest.mark.parametrize("n", [1100, 1500])
def test_fp64_multi_panel_sizes(ep, n):
    """npad > 1024 switches the register panel to 2 rows per thread."""
    A, V, t = _problem(n, -100, 0, 16, 77 + n)
    _announce(f"fp64 n={n} m=16 d=24")
    X = _run(ep, A, V, t, 24)
    Y = matrix.expm_R(A, V, t, 24)
    assert matrix.rel_fro(X, Y) < TOL64
    _announce(f"mixed n={n} m=16 d=24")
    Xm = _run(ep, A, V, t, 24, "mixed")
    assert matrix.rel_fro(Xm, Y) < TOLMX


def test_diagonal_and_zero(ep):
    """Diagonal A gives diagonal R_d(tA) (Remark after eq. equ:ExpoMatRat); A = 0 gives V."""
    n = 70
    lam = -np.linspace(0, 30, n)
    D = np.diag(lam).astype(np.complex128)
    _announce("diagonal n=70 V=I d=16")
    X = _run(ep, D, None, 1.0, 16)
    want = 1.0 / scalar.exp_d(-lam, 16)
    assert np.max(np.abs(X - np.diag(np.diag(X)))) < 1e-14
    # absolute error, as bounded by Prop. prop:digit (entries range down to 1e-11 here)
    assert np.max(np.abs(np.diag(X).real - want)) < 1e-13
    V = wl.complex_gaussian(np.random.default_rng(5), n, 3)
    _announce("zero matrix n=70 m=3 d=16")
    Z = _run(ep, np.zeros((n, n), np.complex128), V, 1.0, 16)
    assert matrix.rel_fro(Z, V) < 1e-13


@pytest.mark.parametrize("n", [700, 2048])
@pytest.mark.parametrize("kind", ["ties", "far"])
def test_pivoting_ties_and_far_pivots(ep, n, kind):
    """Two matrices that drive the pivot search of the register panel.
    ties: A = -(100/n) 1 1^H (spectrum {-100, 0}); below the diagonal every column
      holds equal magnitudes at every elimination step, so every wave resolves
      exact ties (largest |Re|+|Im|, then the lowest position).
    far: A of 2 x 2 blocks [[-1, -50], [-50, -2500]] on rows (i, i + n/2)
      (spectrum {-2501, 0}); each column of the first half takes its pivot from
      the row n/2 below, so at n = 2048 rows move between blocks of the register
      panel at every column of the first half.
    Both paths against the oracle (a LAPACK pole sum in FP64 reaches 5e-14 and
    4e-15 on them)."""
    rng = np.random.default_rng(31 + n)
    if kind == "ties":
        A = np.full((n, n), -100.0 / n, np.complex128)
    else:
        A = np.zeros((n, n), np.complex128)
        h = n // 2
        i = np.arange(h)
        A[i, i] = -1.0
        A[i + h, i + h] = -2500.0
        A[i, i + h] = -50.0
        A[i + h, i] = -50.0
    V = wl.complex_gaussian(rng, n, 4)
    Y = matrix.expm_R(A, V, 1.0, 16)
    _announce(f"pivot {kind} fp64 n={n} m=4 d=16")
    X = _run(ep, A, V, 1.0, 16)
    assert matrix.rel_fro(X, Y) < TOL64
    _announce(f"pivot {kind} mixed n={n} m=4 d=16")
    Xm = _run(ep, A, V, 1.0, 16, "mixed")
    assert matrix.rel_fro(Xm, Y) < TOLMX


def test_lower_triangle_only(ep):
    A, V, t = _problem(90, -60, 0, 2, 9)
    B = A.copy()
    B[np.triu_indices(90, 1)] = 7.0 + 3.0j
    B[np.diag_indices(90)] += 2j
    _announce("upper garbage n=90 m=2 d=16")
    X1 = _run(ep, A, V, t, 16)
    X2 = _run(ep, B, V, t, 16)
    assert np.array_equal(X1, X2)


def test_deterministic(ep):
    A, V, t = _problem(180, -100, 0, 16, 10)
    _announce("determinism n=180 m=16 d=24")
    X1 = _run(ep, A, V, t, 24)
    X2 = _run(ep, A, V, t, 24)
    assert np.array_equal(X1, X2)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_plan_reuse_identical(ep, precision):
    """One plan applied three times: every one-launch sweep starts from the
    previous launch's counters and flags and gives the same bits."""
    import torch
    A, V, t = _problem(320, -100, 0, 7, 31)
    _announce(f"plan reuse {precision} n=320 m=7 d=16")
    plan = ep.expm_pfd_plan(320, 16, t, 7, precision)
    Ad, Vd = _dev(A), _dev(V)
    outs = []
    for _ in range(3):
        X = ep.expm_pfd_apply(plan, Ad, Vd)
        torch.cuda.synchronize()
        outs.append(X.cpu().numpy())
    ep.expm_pfd_plan_check(plan)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    Y = matrix.expm_R(A, V, t, 16)
    assert matrix.rel_fro(outs[0], Y) < (TOL64 if precision == "fp64" else TOLMX)


def test_config2_full_size_fp64_and_mixed(ep):
    """n = 2048, V 2048 x 16, degree 24, spectrum in [-100, 0]: the benchmarked launch configuration."""
    P = wl.config2_fp64_at_scale()
    Y = matrix.expm_R(P.A, P.V, P.t, P.degree)
    _announce("config2 fp64 n=2048 m=16 d=24")
    X = _run(ep, P.A, P.V, P.t, P.degree)
    assert matrix.rel_fro(X, Y) < TOL64
    _announce("config2 mixed n=2048 m=16 d=24")
    Xm = _run(ep, P.A, P.V, P.t, P.degree, "mixed")
    assert matrix.rel_fro(Xm, Y) < TOLMX


def test_config3_precision_study(ep):
    """n = 4096, V = I, degree 32, Laplacian-like spectrum down to -3.9e4 (kappa of
    the shifted matrices up to ~4e3).  The mixed path (FP32 LU, two FP64-residual
    refinement sweeps, a last sweep with a double-double residual) is gated at 1e-10.
    The FP64 path's error is reported, not gated: plain FP64 LU plus FP64
    accumulation of residues summing to 2.7e4 in magnitude reaches about 1.6e-10
    here, so only a loose sanity bound is asserted for it."""
    P = wl.config3_precision()
    Y = matrix.expm_R(P.A, None, P.t, P.degree)
    _announce("config3 mixed n=4096 V=I d=32")
    Xm = _run(ep, P.A, None, P.t, P.degree, "mixed")
    em = matrix.rel_fro(Xm, Y)
    assert np.array_equal(Xm, Xm.conj().T)
    _announce("config3 fp64 n=4096 V=I d=32")
    X = _run(ep, P.A, None, P.t, P.degree)
    e64 = matrix.rel_fro(X, Y)
    print(f"[config3] rel err mixed {em:.3e} fp64 {e64:.3e}", file=sys.stderr, flush=True)
    assert em < TOLMX
    assert e64 < 1e-8


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("mixed", TOLMX)])
def test_shifted_positive_spectrum(ep, precision, tol):
    """Shifting method (Remark rem:shift): spectrum in [0, 30], c = 30, so the library
    computes e^30 R_16(tA - 30 I) V; parity against the oracle's e^c R_d(tA - cI) V,
    and the relative error against exp(tA)V stays within the negative-spectrum bound."""
    A, V, t = _problem(300, 0.0, 30.0, 8, 4242)
    c = 30.0
    _announce(f"shift {precision} n=300 m=8 d=16 c={c}")
    X = _run(ep, A, V, t, 16, precision, shift=c)
    Y = matrix.expm_R_shifted(A, V, t, 16, c)
    assert matrix.rel_fro(X, Y) < tol
    E = matrix.expm_exact(A, V, t)
    assert matrix.rel_fro(X, E) < 1e-5
    # V = I with a negative shift (c below the spectrum is allowed; bounds then weaker)
    B, _, _ = _problem(100, -10.0, 0.0, None, 4243)
    _announce(f"shift {precision} n=100 V=I d=16 c=-2")
    XB = _run(ep, B, None, 1.0, 16, precision, shift=-2.0)
    assert matrix.rel_fro(XB, matrix.expm_R_shifted(B, None, 1.0, 16, -2.0)) < tol


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("mixed", TOLMX)])
def test_real_symmetric_fast_path(ep, precision, tol):
    """Real symmetric A and real V (Remark rem:two_time_real_part): with real_data the
    conjugate pole's solution is taken as the conjugate of the primal one, so only one
    pole per pair is solved.  Parity against the oracle; the imaginary parts of the
    inputs are not read in that mode."""
    rng = np.random.default_rng(77)
    n, m = 260, 5
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = rng.uniform(-80.0, 0.0, n)
    A = ((Q * lam) @ Q.T).astype(np.complex128)
    A = 0.5 * (A + A.T)
    V = rng.standard_normal((n, m)).astype(np.complex128)
    Y = matrix.expm_R(A, V, 1.0, 24)
    _announce(f"real fast path {precision} n={n} m={m} d=24")
    X = _run(ep, A, V, 1.0, 24, precision, real_data=True)
    assert matrix.rel_fro(X, Y) < tol
    # imaginary parts are ignored in this mode
    Aj = A + 1j * rng.standard_normal((n, n))
    Vj = V + 1j * rng.standard_normal((n, m))
    _announce(f"real fast path {precision} ignores imaginary parts")
    Xj = _run(ep, Aj, Vj, 1.0, 24, precision, real_data=True)
    assert np.array_equal(X, Xj)
    # the general path on the same data agrees to the tolerance
    X2 = _run(ep, A, V, 1.0, 24, precision)
    assert matrix.rel_fro(X2, Y) < tol


def test_apply_argument_errors(ep):
    """Apply-time argument checks of the C ABI (synchronous, before any launch):
    leading dimensions below n, m above the plan's m_max, V = I on a plan sized for
    thin V, a missing A or X; the plan stays usable afterwards."""
    import ctypes
    import torch
    lib = ep.load_library()
    n, m = 70, 4
    A, V, t = _problem(n, -20, 0, m, 606)
    Ad, Vd = _dev(A), _dev(V)
    X = torch.empty((m, n), dtype=torch.complex128, device="cuda").t()
    plan = ep.expm_pfd_plan(n, 16, t, m, "fp64")
    h, s = plan.handle, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    pa, pv, px = Ad.data_ptr(), Vd.data_ptr(), X.data_ptr()
    _announce("apply argument errors n=70 m=4")
    assert lib.expm_pfd_apply(h, pa, n - 1, pv, n, m, px, n, s) == -4      # lda < n
    assert lib.expm_pfd_apply(h, pa, n, pv, n - 1, m, px, n, s) == -4      # ldv < n
    assert lib.expm_pfd_apply(h, pa, n, pv, n, m, px, n - 1, s) == -4      # ldx < n
    assert lib.expm_pfd_apply(h, pa, n, pv, n, m + 1, px, n, s) == -2      # m > m_max
    assert lib.expm_pfd_apply(h, pa, n, pv, n, 0, px, n, s) == -2          # m < 1
    assert lib.expm_pfd_apply(h, pa, n, None, n, n, px, n, s) == -2        # V = I on a thin plan
    assert lib.expm_pfd_apply(h, None, n, pv, n, m, px, n, s) == -3        # A missing
    assert lib.expm_pfd_apply(h, pa, n, pv, n, m, None, n, s) == -3        # X missing
    assert lib.expm_pfd_apply(None, pa, n, pv, n, m, px, n, s) == -3       # no plan
    assert lib.expm_pfd_apply(h, pa, n, pv, n, m, px, n, s) == 0
    torch.cuda.synchronize()
    ep.expm_pfd_plan_check(plan)
    assert matrix.rel_fro(X.cpu().numpy(), matrix.expm_R(A, V, t, 16)) < TOL64
