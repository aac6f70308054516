"""Host-side logic on the CPU: the seeded input generators, the bench's bookkeeping
and its command-line contract.  No GPU and no HIP call is needed."""

import json
import os
import subprocess
import sys

import numpy as np

from paper_2306_16778_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_generators_are_deterministic():
    a = wl.config1_plain_cpu_sized()
    b = wl.config1_plain_cpu_sized()
    assert np.array_equal(a.A, b.A) and a.degree == 16 and a.V is None
    r1, s1 = wl.config5_requests(40, qps=50.0)
    r2, s2 = wl.config5_requests(40, qps=50.0)
    assert s1 == s2
    assert all(x.arrival_s == y.arrival_s and np.array_equal(x.v, y.v) for x, y in zip(r1, r2))


def test_hermitian_with_prescribed_spectrum():
    rng = np.random.default_rng(3)
    lam = rng.uniform(-50.0, 0.0, 40)
    for cheap in (False, True):
        A = wl.hermitian_with_spectrum(np.random.default_rng(4), lam, cheap=cheap)
        assert np.array_equal(A, A.conj().T)
        w = np.linalg.eigvalsh(A)
        assert np.allclose(np.sort(w), np.sort(lam), atol=1e-11)


def test_laplacian_like_spectrum():
    lam = wl.laplacian_like_spectrum(4096)
    assert lam.shape == (4096,) and np.all(np.diff(lam) < 0) and np.all(lam < 0)
    assert abs(lam[0] + 4e3 * (np.pi / 4097) ** 2) < 1e-15
    assert 3.9e4 < -lam[-1] < 4.0e4


def test_batch_and_request_shapes():
    probs = wl.config4_batch(24)
    for p in probs:
        n = p.A.shape[0]
        assert 32 <= n <= 512 and p.V.shape == (n, 4) and 0.1 <= p.t <= 1.0 and p.degree == 16
    reqs, specs = wl.config5_requests(400, qps=100.0)
    arr = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(arr) > 0)
    # Poisson arrivals at 100/s: 400 requests in about 4 s
    assert 3.0 < arr[-1] < 5.0
    reuse = np.mean([r.reuse for r in reqs])
    assert 0.12 < reuse < 0.28
    for r in reqs:
        assert 64 <= r.n <= 4096 and r.v.shape == (r.n, 1) and specs[r.matrix_id][0] == r.n


def test_serving_matrix_has_its_drawn_spectrum():
    """The serving workload's cheap unitary (Householder reflections and phases)
    keeps the spectrum drawn from the matrix's own seed."""
    spec = (48, 3)
    A = wl.config5_matrix(spec)
    r = wl.rng_for(5, spec[1] + 1)
    lam = r.uniform(-200.0, 0.0, spec[0])
    assert np.allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(lam), atol=1e-10)


def test_known_eigenbasis_generator():
    """The generator used where the oracle is given the eigenpairs: U is unitary,
    A = U diag(lam) U^H, and it draws what the serving workload's matrix draws from
    the same seed (the same reflections and phases)."""
    spec = (90, 7)
    r = wl.rng_for(5, spec[1] + 1)
    lam = r.uniform(-200.0, 0.0, spec[0])
    A, U = wl.hermitian_with_known_eigenbasis(r, lam)
    n = spec[0]
    assert np.array_equal(A, A.conj().T)
    assert np.max(np.abs(U.conj().T @ U - np.eye(n))) < 1e-14
    assert np.max(np.abs((U * lam) @ U.conj().T - A)) < 200 * 1e-14
    assert np.max(np.abs(A - wl.config5_matrix(spec))) < 200 * 1e-14


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_bench_bookkeeping():
    sys.path.insert(0, ROOT)
    import bench

    # LAPACK counts: d/2 factorizations of (8/3) n^3 and d solves of 8 n^2 m
    assert bench.algorithmic_flops(2048, 16, 24) == 12 * (8.0 / 3.0) * 2048 ** 3 + 24 * 8.0 * 2048 ** 2 * 16
    # the counters' traffic is reported only for the kernel sources they were taken on
    saved = dict(bench.TRAFFIC["mixed"])
    try:
        bench.TRAFFIC["mixed"]["sources_sha256"] = "0" * 64
        assert bench.measured_traffic("mixed") is None
    finally:
        bench.TRAFFIC["mixed"].update(saved)
    assert bench.measured_traffic("fp64") is None
    json.dumps({"x": bench.PEAK})


def test_stage_rates():
    """Per-stage rates of the bench line: flops and bytes over the summed launch times,
    matrix-core fraction for the products, HBM fraction (8 TB/s) for the rest, and
    the HBM fraction of every stage, latency-bound ones included."""
    sys.path.insert(0, ROOT)
    import bench

    b = {"lu_trail": {"launches": 15, "ms": 2.0, "flops": 2.0e11, "bytes": 4.0e9},
         "solve_gemm": {"launches": 6, "ms": 1.0, "flops": 1.0e9, "bytes": 4.0e9},
         "panel": {"launches": 0, "ms": 0.0, "flops": 0.0, "bytes": 0.0}}
    r = bench.stage_rates(b, "mixed")
    assert set(r) == {"lu_trail", "solve_gemm"}
    assert r["lu_trail"]["tflops"] == 100.0 and r["lu_trail"]["bound"] == "mfma"
    assert r["lu_trail"]["frac"] == round(100.0 / 157.3, 3)
    assert r["solve_gemm"]["gb_per_s"] == 4000.0 and r["solve_gemm"]["frac"] == 0.5
    assert bench.stage_rates(b, "fp64")["lu_trail"]["frac"] == round(100.0 / 78.6, 3)
    b["panel"] = {"launches": 4, "ms": 1.0, "flops": 1.0e9, "bytes": 1.0e8}
    assert bench.stage_rates(b, "mixed")["panel"] == {"tflops": 1.0, "gb_per_s": 100.0, "bound": "latency",
                                                      "frac": None, "hbm_frac": 0.0125}
    assert r["solve_gemm"]["hbm_frac"] == 0.5


def test_serving_eigenpairs_rebuild_the_matrix():
    """The eigenpairs the serving checks use are those the serving matrix is built
    from: U unitary and U diag(lam) U^H equal to the host-assembled matrix."""
    from paper_2306_16778_amd import workloads as wl

    spec = (150, 4)
    lam, U = wl.config5_eigenpairs(spec)
    assert np.allclose(U.conj().T @ U, np.eye(150), atol=1e-13)
    A = wl.config5_matrix(spec)
    assert np.abs((U * lam) @ U.conj().T - A).max() < 1e-12 * np.abs(A).max()
