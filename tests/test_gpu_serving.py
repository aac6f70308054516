"""GPU tests of the queued serving path: results of Poisson-arrival traces with
matrix reuse match the oracle, and each equals the same request evaluated alone
within the stated tolerance (a request may be evaluated in a group of a larger
padded order, which changes the summation order of its refinement products)."""

import sys

import numpy as np
import pytest

from oracle import matrix

pytestmark = pytest.mark.gpu


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


U64 = 2.0 ** -53


def _within(err, tol, A, v, t, eig=None):
    """err <= tol, where the FP64 gate (tol = 1e-12) is raised to 8 u times the
    oracle's residue amplification factor when that is larger: rounding of the
    shifted solves reaches the pole sum weighted by |a_k| (Prop. prop:digit), so a
    result ||R_d(tA)v|| much smaller than ||v|| (spectra far below 0) cannot be
    reached to 1e-12 relative by any FP64 evaluation of the partial fractions
    (LAPACK's FP64 solves summed the same way measure 2.0e-12 on one such request
    of the serving trace, amplification 1.0e4)."""
    if err <= tol:
        return True
    return tol == 1e-12 and err <= 8 * U64 * matrix.pfd_amplification(A, v, t, 16, eig=eig)


def _oracle(kept, specs, tol, eigh_max=1024):
    """Every kept (request, v, t, X) against the oracle's R_d(tA)v.  Orders up to
    eigh_max: eigendecomposition of the very bytes the queue factored (the device
    assembly, rebuilt on the device and copied back).  Larger orders: the eigenpairs
    the matrix is built from, which differ from the device bytes by the assembly's
    rounding (the result moves by about 1e-13 relative, up to 2e-12 measured).
    Returns the largest error."""
    from paper_2306_16778_amd import workloads as wl
    src, worst = {}, 0.0
    for r, v, t, X in kept:
        if r.matrix_id not in src:
            if r.n <= eigh_max:
                src[r.matrix_id] = (wl.config5_matrix_device(specs[r.matrix_id]).cpu().numpy(), None)
            else:
                src[r.matrix_id] = (None, wl.config5_eigenpairs(specs[r.matrix_id]))
        A, eig = src[r.matrix_id]
        err = matrix.rel_fro(X, matrix.expm_R(A, v, t, 16, eig=eig))
        assert _within(err, tol, A, v, t, eig), (r.n, err)
        worst = max(worst, err)
    return worst


def _alone(ep, kept, specs, precision, tol, count):
    """The first `count` kept requests through single-problem plans on the same device
    matrix: within the tolerance of the queue's result (same bits unless padded up)."""
    import torch
    from paper_2306_16778_amd import workloads as wl
    same = 0
    for r, v, t, X in kept[:count]:
        A = wl.config5_matrix_device(specs[r.matrix_id])
        plan = ep.expm_pfd_plan(r.n, 16, t, 1, precision)
        X1 = ep.expm_pfd_apply(plan, A, _dev(v))
        torch.cuda.synchronize()
        x1 = X1.cpu().numpy()
        assert matrix.rel_fro(X, x1) < tol
        same += int(np.array_equal(X, x1))
    return same


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_serving_trace_matches_oracle_and_alone(ep, precision, tol):
    from paper_2306_16778_amd import serving
    from paper_2306_16778_amd import workloads as wl

    _announce(f"serving {precision} 64 requests n in [64, 700]")
    reqs, specs = wl.config5_requests(64, 2000.0, 64, 700)
    stats, kept, _, _ = serving.replay(64, 2000.0, precision, budget_bytes=16 << 30, keep=lambda r: True,
                                       reqs=reqs, specs=specs)
    assert stats["completed"] == 64 and stats["submitted"] == 64 and stats["failed"] == 0
    assert stats["groups"] < 64  # requests were grouped
    assert stats["padded_up"] > 0  # some across padded orders
    assert any(r.reuse for r, *_ in kept)
    _oracle(kept, specs, tol)
    _alone(ep, kept, specs, precision, tol, 8)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_serving_full_order_range(ep, precision, tol):
    """Requests over the serving workload's whole order range, n log-uniform in
    [64, 4096], overlapping on the device (arrivals at 400/s).  The oracle uses the
    eigenpairs the matrices are built from (spectrum and Householder eigenvectors
    regenerated from the same seeds), so orders up to 4096 need no eigensolver;
    the matrices the queue factors are the device-assembled copies, which differ
    from U diag(lam) U^H only by rounding (about 1e-13 relative in the result)."""
    from paper_2306_16778_amd import serving
    from paper_2306_16778_amd import workloads as wl

    _announce(f"serving {precision} 40 requests n in [64, 4096]")
    reqs, specs = wl.config5_requests(40, 400.0, 64, 4096)
    stats, kept, _, _ = serving.replay(40, 400.0, precision, budget_bytes=32 << 30, keep=lambda r: True,
                                       reqs=reqs, specs=specs)
    assert stats["completed"] == 40 and stats["failed"] == 0
    assert max(r.n for r, *_ in kept) > 2048
    _oracle(kept, specs, tol)
    big = sorted(kept, key=lambda k: -k[0].n)[:2]
    _alone(ep, big, specs, precision, tol, 2)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_more_matrices_than_the_budget_holds(ep, precision, tol):
    """A budget that holds the workspace of one group and about three registered
    matrices serves a trace of 48 requests over 40 distinct matrices: the replay
    unregisters matrices least recently used (their memory returns to the budget
    once their requests are done) and registers them again when a later request
    reuses one.  Every request completes and matches the oracle."""
    from paper_2306_16778_amd import serving
    from paper_2306_16778_amd import workloads as wl

    reqs, specs = wl.config5_requests(48, 300.0, 200, 320)
    assert len(specs) > 30
    one = ep.expm_pfd_workspace_bytes(320, 16, 16, precision)
    mat = 320 * 320 * 16
    budget = 4 * one + 8 * mat
    _announce(f"serving {precision}: 48 requests, {len(specs)} matrices, budget {budget / 1e6:.0f} MB")
    stats, kept, _, _ = serving.replay(48, 300.0, precision, budget_bytes=budget, resident_bytes=3 * mat,
                                       max_group=4, lookahead=2, keep=lambda r: True, reqs=reqs, specs=specs)
    assert stats["completed"] == 48 and stats["failed"] == 0
    assert stats["peak_bytes"] <= budget
    assert stats["registered"] == 0  # everything released by the end (the replay unregisters; destroy frees)
    _oracle(kept, specs, tol)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_submit_with_matrix_in_place_and_unregister(ep, precision, tol):
    """Requests may pass their matrix with the submission (read in place) instead of
    a registered id; a registered matrix released while its requests are pending
    still serves them, and its id is rejected afterwards."""
    import torch
    from paper_2306_16778_amd import workloads as wl

    rng = np.random.default_rng(61)
    n = 180
    A = wl.hermitian_with_spectrum(rng, rng.uniform(-150.0, 0.0, n))
    B = wl.hermitian_with_spectrum(rng, rng.uniform(-90.0, 0.0, 97))
    vs = [wl.complex_gaussian(rng, n, 2) for _ in range(3)]
    q = ep.expm_pfd_queue_create(4 << 30, 16, precision)
    _announce(f"queue in-place matrix {precision}")
    Ad = _dev(A)
    outs = [ep.expm_pfd_submit(q, Ad, 0.3 * (k + 1), _dev(v)) for k, v in enumerate(vs)]
    mid = ep.expm_pfd_register_matrix(q, _dev(B))
    w = wl.complex_gaussian(rng, 97, 1)
    tk, XB = ep.expm_pfd_submit(q, mid, 0.7, _dev(w))
    ep.expm_pfd_unregister_matrix(q, mid)  # pending request still served
    with pytest.raises(ep.ExpmPfdError) as e:
        ep.expm_pfd_submit(q, mid, 0.7, _dev(w))
    assert e.value.code == -10
    with pytest.raises(ep.ExpmPfdError) as e:
        ep.expm_pfd_unregister_matrix(q, mid)
    assert e.value.code == -10
    assert ep.expm_pfd_wait(q, tk) == 0
    ep.expm_pfd_queue_drain(q)
    for k, ((_, X), v) in enumerate(zip(outs, vs)):
        assert matrix.rel_fro(X.cpu().numpy(), matrix.expm_R(A, v, 0.3 * (k + 1), 16)) < tol
    assert matrix.rel_fro(XB.cpu().numpy(), matrix.expm_R(B, w, 0.7, 16)) < tol
    st = ep.expm_pfd_queue_stats_get(q)
    assert st["completed"] == 4 and st["failed"] == 0 and st["registered"] == 0
    ep.expm_pfd_queue_destroy(q)
    torch.cuda.synchronize()


def test_queue_fp64_fallback(ep):
    """A mixed-precision queue whose refinement tolerance cannot be met (1e-300)
    solves every request again on the FP64 path: status 1 on each ticket, results
    within the FP64 gate, and the fallbacks counted in the statistics."""
    from paper_2306_16778_amd import workloads as wl

    rng = np.random.default_rng(62)
    n = 140
    A = wl.hermitian_with_spectrum(rng, rng.uniform(-200.0, 0.0, n))
    q = ep.expm_pfd_queue_create(4 << 30, 16, "mixed", ir_tol=1e-300)
    mid = ep.expm_pfd_register_matrix(q, _dev(A))
    vs = [wl.complex_gaussian(rng, n, 1) for _ in range(5)]
    _announce("queue FP64 fallback")
    outs = [ep.expm_pfd_submit(q, mid, 0.2 * (k + 1), _dev(v)) for k, v in enumerate(vs)]
    for tk, _ in outs:
        assert ep.expm_pfd_wait(q, tk) == 1
    for k, ((tk, X), v) in enumerate(zip(outs, vs)):
        assert ep.expm_pfd_poll(q, tk) == (True, 1)
        t = 0.2 * (k + 1)
        assert _within(matrix.rel_fro(X.cpu().numpy(), matrix.expm_R(A, v, t, 16)), 1e-12, A, v, t)
    st = ep.expm_pfd_queue_stats_get(q)
    assert st["fallbacks"] == 5 and st["completed"] == 5 and st["failed"] == 0
    ep.expm_pfd_queue_destroy(q)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_queue_shift_and_real_data(ep, precision, tol):
    """Queue options: the shifting method (spectrum in [0, 15]; c = 15 in units of A
    with shift_scale_t, so each request is shifted by t c, for t in [0.1, 1]) against
    the oracle's e^{tc} R_d(tA - tcI)v, and the real-data mode on a real symmetric
    matrix and real vectors against R_d(tA)v."""
    from paper_2306_16778_amd import workloads as wl

    rng = np.random.default_rng(57)
    n, c = 150, 15.0
    A = wl.hermitian_with_spectrum(rng, rng.uniform(0.0, 15.0, n))
    q = ep.expm_pfd_queue_create(4 << 30, 16, precision, shift=c, shift_scale_t=True)
    mid = ep.expm_pfd_register_matrix(q, _dev(A))
    vs = [wl.complex_gaussian(rng, n, 1) for _ in range(4)]
    _announce(f"queue shift {precision} n={n} c={c} (units of A)")
    ts = [1.0, 0.55, 0.3, 0.1]
    outs = [ep.expm_pfd_submit(q, mid, t, _dev(v)) for t, v in zip(ts, vs)]
    ep.expm_pfd_queue_drain(q)
    for t, (_, X), v in zip(ts, outs, vs):
        Y = matrix.expm_R_shifted(A, v, t, 16, t * c)
        assert matrix.rel_fro(X.cpu().numpy(), Y) < tol
    ep.expm_pfd_queue_destroy(q)

    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    B = (Q * rng.uniform(-80.0, 0.0, n)) @ Q.T
    B = (0.5 * (B + B.T)).astype(np.complex128)
    q = ep.expm_pfd_queue_create(4 << 30, 16, precision, real_data=True)
    mid = ep.expm_pfd_register_matrix(q, _dev(B))
    ws = [rng.standard_normal((n, 1)).astype(np.complex128) for _ in range(3)]
    _announce(f"queue real data {precision} n={n}")
    outs = [ep.expm_pfd_submit(q, mid, 0.4 * (k + 1), _dev(w)) for k, w in enumerate(ws)]
    ep.expm_pfd_queue_drain(q)
    for k, ((_, X), w) in enumerate(zip(outs, ws)):
        assert matrix.rel_fro(X.cpu().numpy(), matrix.expm_R(B, w, 0.4 * (k + 1), 16)) < tol
    ep.expm_pfd_queue_destroy(q)

    # uplo: a queue reading the upper triangle gives the same bits as one reading the
    # lower triangle, with the unread triangle set to NaN
    Blo, Bup = B.copy(), B.copy()
    Blo[np.triu_indices(n, 1)] = np.nan
    Bup[np.tril_indices(n, -1)] = np.nan
    res = []
    _announce(f"queue uplo {precision} n={n}")
    for uplo, M in (("L", Blo), ("U", Bup)):
        q = ep.expm_pfd_queue_create(4 << 30, 16, precision, uplo=uplo)
        mid = ep.expm_pfd_register_matrix(q, _dev(M))
        _, X = ep.expm_pfd_submit(q, mid, 0.5, _dev(ws[0]))
        ep.expm_pfd_queue_drain(q)
        res.append(X.cpu().numpy())
        ep.expm_pfd_queue_destroy(q)
    assert np.array_equal(res[0], res[1])
    assert matrix.rel_fro(res[0], matrix.expm_R(B, ws[0], 0.5, 16)) < tol


def test_queue_tridiagonal_reuse(ep):
    """A mixed-precision queue with a reuse threshold of 3: the request that brings a
    registered matrix to 3 uses asks for its reduction to tridiagonal form, and it
    and every later request of that matrix are served by tridiagonal solves (FP64
    throughout: the FP64 gate); requests before it may have gone the LU route
    (mixed tolerance). A matrix below the threshold and a matrix read in place keep
    the LU route. Then an FP64 queue with threshold 1 and the shift in units of A:
    every request of the matrix on the tridiagonal route, against the oracle's
    e^{tc} R_d(tA - tcI)v."""
    import torch
    from paper_2306_16778_amd import workloads as wl

    rng = np.random.default_rng(63)
    n, nb = 300, 97
    A = wl.hermitian_with_spectrum(rng, rng.uniform(-150.0, 0.0, n))
    B = wl.hermitian_with_spectrum(rng, rng.uniform(-90.0, 0.0, nb))
    q = ep.expm_pfd_queue_create(4 << 30, 16, "mixed", tridiag_reuse=3)
    mid = ep.expm_pfd_register_matrix(q, _dev(A))
    bid = ep.expm_pfd_register_matrix(q, _dev(B))
    _announce(f"queue tridiagonal reuse n={n}")
    cols = [1, 3, 16, 2, 1, 5, 16, 1, 4, 2]
    ts = [0.1 * (k + 1) for k in range(len(cols))]
    vs = [wl.complex_gaussian(rng, n, m) for m in cols]
    outs = [ep.expm_pfd_submit(q, mid, t, _dev(v)) for t, v in zip(ts, vs)]
    ws = [wl.complex_gaussian(rng, nb, 2) for _ in range(2)]
    bouts = [ep.expm_pfd_submit(q, bid, 0.5 + 0.2 * k, _dev(w)) for k, w in enumerate(ws)]
    _, Xin = ep.expm_pfd_submit(q, _dev(B), 0.9, _dev(ws[0]))
    ep.expm_pfd_queue_drain(q)
    for k, (t, (tk, X), v) in enumerate(zip(ts, outs, vs)):
        assert ep.expm_pfd_poll(q, tk) == (True, 0)
        err = matrix.rel_fro(X.cpu().numpy(), matrix.expm_R(A, v, t, 16))
        assert err < 1e-10 if k < 2 else _within(err, 1e-12, A, v, t), (k, err)
    for k, ((_, X), w) in enumerate(zip(bouts, ws)):
        assert matrix.rel_fro(X.cpu().numpy(), matrix.expm_R(B, w, 0.5 + 0.2 * k, 16)) < 1e-10
    assert matrix.rel_fro(Xin.cpu().numpy(), matrix.expm_R(B, ws[0], 0.9, 16)) < 1e-10
    st = ep.expm_pfd_queue_stats_get(q)
    assert st["reductions"] == 1 and 8 <= st["tridiag_requests"] <= 10, st
    assert st["completed"] == 13 and st["failed"] == 0
    # the registered bytes hold both matrices and the tridiagonal plan
    assert st["registered"] == 2 and st["registered_bytes"] > (n * n + nb * nb) * 16
    ep.expm_pfd_unregister_matrix(q, mid)
    st = ep.expm_pfd_queue_stats_get(q)
    assert st["registered"] == 1 and st["registered_bytes"] == nb * nb * 16
    ep.expm_pfd_queue_destroy(q)

    c = 15.0
    C = wl.hermitian_with_spectrum(rng, rng.uniform(0.0, c, n))
    q = ep.expm_pfd_queue_create(4 << 30, 16, "fp64", tridiag_reuse=1, shift=c, shift_scale_t=True)
    mid = ep.expm_pfd_register_matrix(q, _dev(C))
    _announce(f"queue tridiagonal reuse with shift n={n} c={c} (units of A)")
    ts = [1.0, 0.4, 0.15]
    vs = [wl.complex_gaussian(rng, n, 2) for _ in ts]
    outs = [ep.expm_pfd_submit(q, mid, t, _dev(v)) for t, v in zip(ts, vs)]
    ep.expm_pfd_queue_drain(q)
    for t, (_, X), v in zip(ts, outs, vs):
        Y = matrix.expm_R_shifted(C, v, t, 16, t * c)
        assert matrix.rel_fro(X.cpu().numpy(), Y) < 1e-12
    st = ep.expm_pfd_queue_stats_get(q)
    assert st["reductions"] == 1 and st["tridiag_requests"] == 3
    ep.expm_pfd_queue_destroy(q)
    torch.cuda.synchronize()


def test_budget_admission(ep):
    """A budget too small for one workspace rejects the request; a budget for one
    group at a time still completes every request (they queue, never run out of
    memory); a registration that cannot fit is rejected."""
    import torch
    from paper_2306_16778_amd import workloads as wl

    n = 256
    A = wl.config5_matrix_device((n, 3))
    V = torch.randn(n, 1, dtype=torch.complex128, device="cuda")
    one = ep.expm_pfd_workspace_bytes(n, 16, 16, "fp64")
    q = ep.expm_pfd_queue_create(n * n * 16 + one // 2, 16, "fp64")
    mid = ep.expm_pfd_register_matrix(q, A)
    with pytest.raises(ep.ExpmPfdError) as e:
        ep.expm_pfd_submit(q, mid, 0.5, V)
    assert e.value.code == -9
    with pytest.raises(ep.ExpmPfdError) as e:  # larger than the whole budget
        ep.expm_pfd_register_matrix(q, torch.zeros((1024, 1024), dtype=torch.complex128, device="cuda"))
    assert e.value.code == -9
    ep.expm_pfd_queue_destroy(q)
    _announce("budget for about one workspace, 10 requests")
    q = ep.expm_pfd_queue_create(n * n * 16 + int(1.5 * one), 16, "fp64")
    mid = ep.expm_pfd_register_matrix(q, A)
    outs = [ep.expm_pfd_submit(q, mid, 0.1 * (k + 1), V) for k in range(10)]
    ep.expm_pfd_queue_drain(q)
    st = ep.expm_pfd_queue_stats_get(q)
    assert st["completed"] == 10 and st["failed"] == 0
    assert st["peak_bytes"] <= n * n * 16 + int(1.5 * one)
    Ah = A.cpu().numpy()
    for k, (tk, X) in enumerate(outs):
        Y = matrix.expm_R(Ah, V.cpu().numpy(), 0.1 * (k + 1), 16)
        assert matrix.rel_fro(X.cpu().numpy(), Y) < 1e-12
    ep.expm_pfd_queue_destroy(q)


def test_queue_errors_and_poll(ep):
    """Queue error paths and completion polling: an unknown matrix id or ticket is
    rejected (EXPM_PFD_ERR_TICKET) without disturbing the queue, a request with more
    than 16 columns is rejected, and polling reports each accepted request done
    exactly when its result is final."""
    import torch
    from paper_2306_16778_amd import workloads as wl

    n = 96
    A = wl.config5_matrix_device((n, 11))
    q = ep.expm_pfd_queue_create(2 << 30, 16, "fp64")
    mid = ep.expm_pfd_register_matrix(q, A)
    V = torch.randn(n, 1, dtype=torch.complex128, device="cuda")
    _announce("queue error paths n=96")
    with pytest.raises(ep.ExpmPfdError) as e:
        ep.expm_pfd_submit(q, mid + 7, 0.5, V)
    assert e.value.code == -10
    with pytest.raises(ep.ExpmPfdError) as e:
        ep.expm_pfd_poll(q, 123456789)
    assert e.value.code == -10
    with pytest.raises(ep.ExpmPfdError) as e:
        ep.expm_pfd_wait(q, 987654321)
    assert e.value.code == -10
    with pytest.raises(ep.ExpmPfdError):
        ep.expm_pfd_submit(q, mid, 0.5, torch.randn(n, 17, dtype=torch.complex128, device="cuda"))
    tickets = [ep.expm_pfd_submit(q, mid, 0.2 * (k + 1), V) for k in range(4)]
    for k, (tk, X) in enumerate(tickets):
        assert ep.expm_pfd_wait(q, tk) == 0
        assert ep.expm_pfd_poll(q, tk) == (True, 0)
        Y = matrix.expm_R(A.cpu().numpy(), V.cpu().numpy(), 0.2 * (k + 1), 16)
        assert matrix.rel_fro(X.cpu().numpy(), Y) < 1e-12
    st = ep.expm_pfd_queue_stats_get(q)
    assert st["completed"] == 4 and st["submitted"] == 4 and st["failed"] == 0
    ep.expm_pfd_queue_destroy(q)
