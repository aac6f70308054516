"""GPU tests of the queued serving path: results of a Poisson-arrival trace with
matrix reuse match the oracle, and each equals the same request evaluated alone."""

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


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_serving_trace_matches_oracle_and_alone(ep, precision, tol):
    import torch
    from paper_2306_16778_amd import serving

    _announce(f"serving {precision} 48 requests n in [64, 700]")
    stats, kept, _ = serving.replay(48, qps=2000.0, precision=precision, degree=16, n_lo=64, n_hi=700,
                                    budget_bytes=16 << 30, keep=lambda r: True)
    assert stats["completed"] == 48 and stats["submitted"] == 48
    assert stats["groups"] < 48  # requests were grouped
    assert any(r.reuse for r, *_ in kept)
    for r, A, v, t, X in kept:
        Y = matrix.expm_R(A, v, t, 16)
        assert matrix.rel_fro(X, Y) < tol
    # alone: the same request through a single-problem plan gives the same bits
    for r, A, v, t, X in kept[:6]:
        n = A.shape[0]
        plan = ep.expm_pfd_plan(n, 16, t, 1, precision)
        X1 = ep.expm_pfd_apply(plan, torch.from_numpy(np.asfortranarray(A)).cuda(),
                               torch.from_numpy(np.asfortranarray(v)).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(X1.cpu().numpy(), X)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_serving_full_order_range(ep, precision, tol):
    """Requests over the serving workload's whole order range, n log-uniform in
    [64, 4096], overlapping on the device (arrivals at 400/s).  The oracle uses the
    eigenpairs the matrices are built from (spectrum and Householder eigenvectors
    regenerated from the same seeds), so orders up to 4096 need no eigensolver;
    the matrices the queue factors are the device-assembled copies, which differ
    from U diag(lam) U^H only by rounding (about 1e-13 relative in the result)."""
    import torch
    from paper_2306_16778_amd import serving
    from paper_2306_16778_amd import workloads as wl

    _announce(f"serving {precision} 40 requests n in [64, 4096]")
    stats, kept, _ = serving.replay(40, qps=400.0, precision=precision, degree=16, n_lo=64, n_hi=4096,
                                    budget_bytes=32 << 30, keep=lambda r: True)
    assert stats["completed"] == 40
    assert max(r.n for r, *_ in kept) > 2048
    eig = {}
    for r, A, v, t, X in kept:
        if r.matrix_id not in eig:
            rng = wl.rng_for(5, r.matrix_id + 1)
            lam = rng.uniform(-200.0, 0.0, r.n)
            _, U = wl.hermitian_with_known_eigenbasis(rng, lam)
            eig[r.matrix_id] = (lam, U)
        Y = matrix.expm_R(A, v, t, 16, eig=eig[r.matrix_id])
        err = matrix.rel_fro(X, Y)
        assert err < tol, (r.n, err)
    # alone: the two largest requests through single-problem plans give the same bits
    for r, A, v, t, X in sorted(kept, key=lambda k: -k[0].n)[:2]:
        plan = ep.expm_pfd_plan(r.n, 16, t, 1, precision)
        X1 = ep.expm_pfd_apply(plan, torch.from_numpy(np.asfortranarray(A)).cuda(),
                               torch.from_numpy(np.asfortranarray(v)).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(X1.cpu().numpy(), X)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_queue_shift_and_real_data(ep, precision, tol):
    """Queue options: the shifting method (spectrum in [0, 15], c = 15) against the
    oracle's e^c R_d(tA - cI)v, and the real-data mode on a real symmetric matrix and
    real vectors against R_d(tA)v."""
    import torch
    from paper_2306_16778_amd import workloads as wl

    rng = np.random.default_rng(57)
    n, c = 150, 15.0
    A = wl.hermitian_with_spectrum(rng, rng.uniform(0.0, 15.0, n))
    q = ep.expm_pfd_queue_create(4 << 30, 16, precision, shift=c)
    mid = ep.expm_pfd_register_matrix(q, torch.from_numpy(np.asfortranarray(A)).cuda())
    vs = [wl.complex_gaussian(rng, n, 1) for _ in range(3)]
    _announce(f"queue shift {precision} n={n} c={c}")
    ts = [1.0, 0.95, 0.9]  # c near the top of the spectrum of tA (Remark rem:shift)
    outs = [ep.expm_pfd_submit(q, mid, t, torch.from_numpy(np.asfortranarray(v)).cuda()) for t, v in zip(ts, vs)]
    ep.expm_pfd_queue_drain(q)
    for t, (_, X), v in zip(ts, outs, vs):
        Y = matrix.expm_R_shifted(A, v, t, 16, c)
        assert matrix.rel_fro(X.cpu().numpy(), Y) < tol
    ep.expm_pfd_queue_destroy(q)

    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    B = (Q * rng.uniform(-80.0, 0.0, n)) @ Q.T
    B = (0.5 * (B + B.T)).astype(np.complex128)
    q = ep.expm_pfd_queue_create(4 << 30, 16, precision, real_data=True)
    mid = ep.expm_pfd_register_matrix(q, torch.from_numpy(np.asfortranarray(B)).cuda())
    ws = [rng.standard_normal((n, 1)).astype(np.complex128) for _ in range(3)]
    _announce(f"queue real data {precision} n={n}")
    outs = [ep.expm_pfd_submit(q, mid, 0.4 * (k + 1), torch.from_numpy(np.asfortranarray(w)).cuda())
            for k, w in enumerate(ws)]
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
        mid = ep.expm_pfd_register_matrix(q, torch.from_numpy(np.asfortranarray(M)).cuda())
        _, X = ep.expm_pfd_submit(q, mid, 0.5, torch.from_numpy(np.asfortranarray(ws[0])).cuda())
        ep.expm_pfd_queue_drain(q)
        res.append(X.cpu().numpy())
        ep.expm_pfd_queue_destroy(q)
    assert np.array_equal(res[0], res[1])
    assert matrix.rel_fro(res[0], matrix.expm_R(B, ws[0], 0.5, 16)) < tol


def test_budget_admission(ep):
    """A budget too small for one workspace rejects the request; a budget for one
    group at a time still completes every request (they queue, never run out of memory)."""
    import torch
    from paper_2306_16778_amd import workloads as wl

    n = 256
    A = wl.config5_matrix_device((n, 3))
    V = torch.randn(n, 1, dtype=torch.complex128, device="cuda")
    one = ep.expm_pfd_workspace_bytes(n, 16, 16, "fp64")
    q = ep.expm_pfd_queue_create(n * n * 16 + one // 2, 16, "fp64")
    mid = ep.expm_pfd_register_matrix(q, A)
    with pytest.raises(ep.ExpmPfdError):
        ep.expm_pfd_submit(q, mid, 0.5, V)
    ep.expm_pfd_queue_destroy(q)
    _announce("budget for about one workspace, 10 requests")
    q = ep.expm_pfd_queue_create(n * n * 16 + int(1.5 * one), 16, "fp64")
    mid = ep.expm_pfd_register_matrix(q, A)
    outs = [ep.expm_pfd_submit(q, mid, 0.1 * (k + 1), V) for k in range(10)]
    ep.expm_pfd_queue_drain(q)
    st = ep.expm_pfd_queue_stats_get(q)
    assert st["completed"] == 10
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
        ep.expm_pfd_wait(q, tk)
        assert ep.expm_pfd_poll(q, tk)
        Y = matrix.expm_R(A.cpu().numpy(), V.cpu().numpy(), 0.2 * (k + 1), 16)
        assert matrix.rel_fro(X.cpu().numpy(), Y) < 1e-12
    st = ep.expm_pfd_queue_stats_get(q)
    assert st["completed"] == 4 and st["submitted"] == 4
    ep.expm_pfd_queue_destroy(q)
