"""GPU tests of graph replay, reusable batch plans and the autotuner.

Every variant must give the same bits as the direct launches: a captured graph
replays the same kernels with the descriptors uploaded ahead of it, and every
LU tile shape and batch schedule runs the same per-element arithmetic.  Graph
replays are interleaved with other device work and synchronizations, and each
replay is checked against the direct result for its own inputs.
"""

import sys

import numpy as np
import pytest

from oracle import matrix
from paper_2306_16778_amd import workloads as wl

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


def _problem(rng, n, m, lo=-60.0):
    A = wl.hermitian_with_spectrum(rng, rng.uniform(lo, 0.0, n))
    V = None if m is None else wl.complex_gaussian(rng, n, m)
    return A, V


def _apply(ep, plan, A, V):
    import torch
    X = ep.expm_pfd_apply(plan, _dev(A), None if V is None else _dev(V))
    torch.cuda.synchronize()
    return X.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("m", [4, None])
def test_graph_replay_matches_direct(ep, precision, m):
    import torch
    n, d, t = 200, 16, 0.7
    rng = np.random.default_rng(301)
    probs = [_problem(rng, n, m) for _ in range(3)]
    mm = 0 if m is None else m
    _announce(f"graph replay {precision} n={n} m={m}")
    direct = ep.expm_pfd_plan(n, d, t, mm, precision)
    graphed = ep.expm_pfd_plan(n, d, t, mm, precision, graph=True)
    want = [_apply(ep, direct, A, V) for A, V in probs]
    tol = 1e-12 if precision == "fp64" else 1e-10
    assert matrix.rel_fro(want[0], matrix.expm_R(probs[0][0], probs[0][1], t, d)) < tol
    # replays of one graph on changing inputs, with other device work in between
    for rep in range(5):
        k = rep % len(probs)
        A, V = probs[k]
        junk = torch.randn(1 << 20, device="cuda")
        junk.mul_(2.0).add_(1.0)
        got = _apply(ep, graphed, A, V)
        assert np.array_equal(got, want[k]), (rep, k)
    ep.expm_pfd_plan_check(graphed)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_lu_tiles_give_identical_bits(ep, precision):
    n, d, t, m = 300, 16, 1.0, 4
    rng = np.random.default_rng(302)
    A, V = _problem(rng, n, m)
    outs = []
    for tile in ep.LU_TILES:
        _announce(f"lu tile {tile} {precision} n={n}")
        plan = ep.expm_pfd_plan(n, d, t, m, precision, lu_tile=tile)
        outs.append(_apply(ep, plan, A, V))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    tol = 1e-12 if precision == "fp64" else 1e-10
    assert matrix.rel_fro(outs[0], matrix.expm_R(A, V, t, d)) < tol
    _announce(f"autotuned plan {precision} n={n}")
    tuned = ep.expm_pfd_plan(n, d, t, m, precision, autotune=True)
    assert np.array_equal(_apply(ep, tuned, A, V), outs[0])


def _batch(seed):
    rng = np.random.default_rng(seed)
    sizes = [40, 64, 70, 100, 130, 200, 257, 90, 120, 33]
    ms = [4, 4, 1, None, 4, 2, 4, 16, None, 3]
    probs = []
    for n, m in zip(sizes, ms):
        A, V = _problem(rng, n, m, -50.0)
        probs.append((A, V, float(rng.uniform(0.1, 1.0))))
    return probs


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("graph,autotune", [(False, False), (True, False), (True, True)])
def test_batch_plan_reuse(ep, precision, graph, autotune):
    """A batch plan applied to two input sets in turn (twice each) gives, every
    time, the bits of the one-shot batched entry point and of each problem alone."""
    import torch
    sets = [_batch(310), _batch(311)]
    n = [A.shape[0] for A, _, _ in sets[0]]
    m = [0 if V is None else V.shape[1] for _, V, _ in sets[0]]
    _announce(f"batch plan {precision} graph={graph} autotune={autotune}")
    bp = ep.expm_pfd_batch_plan(n, m, 16, precision, graph=graph, autotune=autotune)
    want = []
    for probs in sets:
        Xs = ep.expm_pfd_apply_batched([_dev(A) for A, _, _ in probs],
                                       [None if V is None else _dev(V) for _, V, _ in probs],
                                       [t for _, _, t in probs], 16, precision)
        torch.cuda.synchronize()
        want.append([X.cpu().numpy() for X in Xs])
    for rep in range(4):
        k = rep % 2
        probs = sets[k]
        Xs = ep.expm_pfd_batch_apply(bp, [_dev(A) for A, _, _ in probs],
                                     [None if V is None else _dev(V) for _, V, _ in probs],
                                     [t for _, _, t in probs])
        torch.cuda.synchronize()
        for i, X in enumerate(Xs):
            assert np.array_equal(X.cpu().numpy(), want[k][i]), (rep, i)
    ep.expm_pfd_batch_check(bp)
    info = ep.expm_pfd_batch_info(bp)
    assert info["schedule"] in (1, 2, 4)
    assert info["groups"] >= 2
    # parity of one set against the oracle
    tol = 1e-12 if precision == "fp64" else 1e-10
    for (A, V, t), X in zip(sets[1], want[1]):
        assert matrix.rel_fro(X, matrix.expm_R(A, V, t, 16)) < tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_plans_on_two_streams(ep, precision):
    """Two plans applied at the same time on two streams (each plan owns its
    workspace and sweep control line, so only concurrent applies of one plan race)
    give the same bits as the same applies one after another."""
    import torch
    rng = np.random.default_rng(404)
    probs = []
    for n, m in [(300, 16), (260, 4)]:
        lam = rng.uniform(-80.0, 0.0, n)
        A = wl.hermitian_with_spectrum(rng, lam)
        V = wl.complex_gaussian(rng, n, m)
        probs.append((_dev(A), _dev(V), n, m))
    plans = [ep.expm_pfd_plan(n, 24, 0.7, m, precision) for _, _, n, m in probs]
    _announce(f"two plans, sequential {precision}")
    ref = []
    for pl, (Ad, Vd, _, _) in zip(plans, probs):
        ref.append(ep.expm_pfd_apply(pl, Ad, Vd).clone())
    torch.cuda.synchronize()
    _announce(f"two plans, two streams {precision}")
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    outs = [None, None]
    for rep in range(3):
        for i, (pl, (Ad, Vd, _, _)) in enumerate(zip(plans, probs)):
            with torch.cuda.stream(streams[i]):
                outs[i] = ep.expm_pfd_apply(pl, Ad, Vd, stream=streams[i])
        torch.cuda.synchronize()
        for pl in plans:
            ep.expm_pfd_plan_check(pl)
        for a, b in zip(outs, ref):
            assert torch.equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_caller_stream_capture(ep, precision):
    """A caller captures expm_pfd_apply on its own stream into its own graph (the
    apply path makes no allocation, copy, fill or synchronisation, and the one-launch
    sweeps re-arm their control line on the device).  Each replay, with eager work of
    the same plan and a fill of the output between replays, gives the bits of a
    direct apply."""
    import torch
    rng = np.random.default_rng(505)
    n, m = 200, 8
    A = wl.hermitian_with_spectrum(rng, rng.uniform(-60.0, 0.0, n))
    V = wl.complex_gaussian(rng, n, m)
    Ad, Vd = _dev(A), _dev(V)
    plan = ep.expm_pfd_plan(n, 16, 0.6, m, precision)
    X0 = ep.expm_pfd_apply(plan, Ad, Vd).clone()
    torch.cuda.synchronize()
    Xg = torch.empty((m, n), dtype=torch.complex128, device="cuda").t()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    _announce(f"caller capture {precision} n={n} m={m}")
    with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
        ep.expm_pfd_apply(plan, Ad, Vd, X=Xg, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    for _ in range(3):
        Xg.zero_()
        Xe = ep.expm_pfd_apply(plan, Ad, Vd)
        g.replay()
        torch.cuda.synchronize()
        ep.expm_pfd_plan_check(plan)
        assert torch.equal(Xg, X0) and torch.equal(Xe, X0)
    assert matrix.rel_fro(Xg.cpu().numpy(), matrix.expm_R(A, V, 0.6, 16)) < (1e-12 if precision == "fp64" else 1e-10)
