"""The C-ABI library loads and exports what include/expm_pfd.h declares; host-side
logic (constants, argument validation, workspace sizing) checked without a GPU."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import scalar

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "expm_pfd.h")


def _lib():
    from paper_2306_16778_amd import expm_pfd
    return expm_pfd, expm_pfd.load_library()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(expm_pfd_\w+)\s*\(", text, re.M)))


def test_header_declares_expected_entry_points():
    names = declared_symbols()
    for n in ("expm_pfd_plan", "expm_pfd_apply", "expm_pfd_apply_batched", "expm_pfd_constants",
              "expm_pfd_destroy", "expm_pfd_strerror", "expm_pfd_workspace_bytes"):
        assert n in names


def test_binding_limits_match_header():
    from paper_2306_16778_amd import expm_pfd
    text = open(HEADER).read()
    assert int(re.search(r"#define EXPM_PFD_MAX_N\s+(\d+)", text).group(1)) == expm_pfd.MAX_N
    assert int(re.search(r"#define EXPM_PFD_MAX_DEGREE\s+(\d+)", text).group(1)) == expm_pfd.MAX_DEGREE


def test_library_exports_every_declared_symbol():
    mod, lib = _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", mod.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (expm_pfd_\w+)", out))
    for name in declared_symbols():
        assert name in exported, name
        assert hasattr(lib, name)
    assert set(mod.EXPORTED) == set(declared_symbols())


@pytest.mark.parametrize("d", [2, 4, 8, 16, 24, 32, 36, 48, 64])
def test_constants_match_oracle(d):
    """Library poles/residues (binary128 Aberth + eq. yoyo2) vs the oracle's mpmath values: <= 2 ulp."""
    mod, _ = _lib()
    th, a = mod.expm_pfd_constants(d)
    ot, oa = scalar.pfd_pairs(d)
    for x, y in ((th, ot), (a, oa)):
        for part in ("real", "imag"):
            xv, yv = getattr(x, part), getattr(y, part)
            ulps = np.abs(xv - yv) / np.spacing(np.abs(yv))
            assert np.max(ulps) <= 2


def test_argument_validation_without_device():
    mod, lib = _lib()
    h = ctypes.c_void_p()
    o = mod._Opts()
    for deg in (0, 1, 3, 17, 66):
        assert lib.expm_pfd_plan(ctypes.byref(h), 10, deg, 1.0, 0, ctypes.byref(o)) == -1
    assert lib.expm_pfd_plan(ctypes.byref(h), 0, 16, 1.0, 0, ctypes.byref(o)) == -2
    assert lib.expm_pfd_plan(ctypes.byref(h), 9000, 16, 1.0, 0, ctypes.byref(o)) == -2
    assert lib.expm_pfd_plan(ctypes.byref(h), 10, 16, float("nan"), 0, ctypes.byref(o)) == -7
    o.precision = 7
    assert lib.expm_pfd_plan(ctypes.byref(h), 10, 16, 1.0, 0, ctypes.byref(o)) == -7
    o.precision = 0
    o.shift = 800.0  # e^c overflows
    assert lib.expm_pfd_plan(ctypes.byref(h), 10, 16, 1.0, 0, ctypes.byref(o)) == -7
    o.shift = float("nan")
    assert lib.expm_pfd_plan(ctypes.byref(h), 10, 16, 1.0, 0, ctypes.byref(o)) == -7
    o.shift = 0.0
    assert lib.expm_pfd_plan(None, 10, 16, 1.0, 0, None) == -3
    assert lib.expm_pfd_apply(None, None, 1, None, 1, 1, None, 1, None) == -3
    assert lib.expm_pfd_destroy(None) == -3
    th = np.zeros(4)
    assert lib.expm_pfd_constants(5, th.ctypes.data, th.ctypes.data) == -1
    assert lib.expm_pfd_constants(4, None, th.ctypes.data) == -3
    for code in range(-12, 1):
        assert isinstance(mod.expm_pfd_strerror(code), str)


def test_workspace_bytes():
    mod, _ = _lib()
    n, d = 2048, 24
    b64 = mod.expm_pfd_workspace_bytes(n, d, 16, "fp64")
    bmx = mod.expm_pfd_workspace_bytes(n, d, 16, "mixed")
    # 12 shifted matrices dominate: 12 * 2048^2 * 16 bytes (FP64) or 8 bytes (FP32)
    assert 12 * n * n * 16 <= b64 < 12 * n * n * 16 * 1.1
    assert 12 * n * n * 8 + n * n * 16 <= bmx < b64


def test_batch_and_option_validation_without_device():
    """Batch plans and the speed options reject bad arguments before any device work."""
    mod, lib = _lib()
    h = ctypes.c_void_p()
    o = mod._Opts()
    n = np.array([64, 100, 33], dtype=np.int64)
    m = np.array([4, 0, 1], dtype=np.int64)
    assert lib.expm_pfd_batch_plan(None, 3, n.ctypes.data, m.ctypes.data, 16, None) == -3
    assert lib.expm_pfd_batch_plan(ctypes.byref(h), 0, n.ctypes.data, m.ctypes.data, 16, None) == -2
    assert lib.expm_pfd_batch_plan(ctypes.byref(h), 3, None, m.ctypes.data, 16, None) == -3
    assert lib.expm_pfd_batch_plan(ctypes.byref(h), 3, n.ctypes.data, m.ctypes.data, 15, None) == -1
    bad_m = np.array([4, 101, 1], dtype=np.int64)  # more columns than rows
    assert lib.expm_pfd_batch_plan(ctypes.byref(h), 3, n.ctypes.data, bad_m.ctypes.data, 16, None) == -2
    bad_n = np.array([64, 0, 33], dtype=np.int64)
    assert lib.expm_pfd_batch_plan(ctypes.byref(h), 3, bad_n.ctypes.data, m.ctypes.data, 16, None) == -2
    for tile in (-1, 4):
        o.lu_tile = tile
        assert lib.expm_pfd_plan(ctypes.byref(h), 10, 16, 1.0, 0, ctypes.byref(o)) == -7
        assert lib.expm_pfd_batch_plan(ctypes.byref(h), 3, n.ctypes.data, m.ctypes.data, 16, ctypes.byref(o)) == -7
    o.lu_tile = 0
    assert lib.expm_pfd_batch_apply(None, None, None, None, None, None, None, None, None, None) == -3
    o.uplo = 2
    assert lib.expm_pfd_plan(ctypes.byref(h), 10, 16, 1.0, 0, ctypes.byref(o)) == -7
    o.uplo = 0
    assert lib.expm_pfd_batch_check(None) == -3
    assert lib.expm_pfd_batch_destroy(None) == -3
    assert lib.expm_pfd_batch_info(None, None, None, None) == -3
    # option names of the binding map onto the C struct
    assert mod._opts("mixed", 0, graph=True, autotune=True, lu_tile="64x128").lu_tile == 3
    assert ctypes.sizeof(mod._Opts) == 56


def _c_layout(struct, fields, tmp_path):
    """sizeof and offsetof of a struct of include/expm_pfd.h, from the C compiler."""
    src = tmp_path / "layout.c"
    body = "".join(f'  printf("{f} %zu\\n", offsetof({struct}, {f}));\n' for f in fields)
    src.write_text(f'#include <stddef.h>\n#include <stdio.h>\n#include "expm_pfd.h"\n'
                   f'int main(void) {{\n  printf("sizeof %zu\\n", sizeof({struct}));\n{body}  return 0;\n}}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return {k: int(v) for k, v in (line.split() for line in out.splitlines())}


@pytest.mark.parametrize("cname,pyname", [("expm_pfd_opts", "_Opts"), ("expm_pfd_queue_stats", "_QueueStats")])
def test_binding_structs_match_the_c_layout(cname, pyname, tmp_path):
    """The ctypes mirrors of the option and statistics structs have the C layout."""
    mod, _ = _lib()
    cls = getattr(mod, pyname)
    names = [f for f, _ in cls._fields_]
    lay = _c_layout(cname, names, tmp_path)
    assert lay["sizeof"] == ctypes.sizeof(cls)
    for f in names:
        assert lay[f] == getattr(cls, f).offset, f


def test_noalloc_rejects_before_device_work():
    """The no-allocation entry point checks its arguments and its fixed scratch
    limit on the host, before it looks the scratch array up on a device."""
    mod, lib = _lib()
    o = mod._Opts()
    p = ctypes.c_void_p(1 << 20)  # never dereferenced: every call below is rejected first
    assert lib.expm_pfd_apply_noalloc(64, 16, 1.0, None, 64, None, 64, 64, p, 64, None, None, None) == -3
    assert lib.expm_pfd_apply_noalloc(64, 15, 1.0, p, 64, None, 64, 64, p, 64, None, None, None) == -1
    assert lib.expm_pfd_apply_noalloc(64, 16, 1.0, p, 63, None, 64, 64, p, 64, None, None, None) == -4
    assert lib.expm_pfd_apply_noalloc(64, 16, 1.0, p, 64, None, 64, 63, p, 64, None, None, None) == -2
    assert lib.expm_pfd_apply_noalloc(64, 16, 1.0, p, 64, p, 64, 65, p, 64, None, None, None) == -2
    assert lib.expm_pfd_apply_noalloc(64, 16, float("inf"), p, 64, p, 64, 4, p, 64, None, None, None) == -7
    # workspace beyond EXPM_PFD_NOALLOC_BYTES: FP64 thin blocks fit up to n = 896 at degree 16
    # (12 shifted matrices of 960^2 x 16 bytes alone exceed 128 MiB at degree 24)
    assert lib.expm_pfd_apply_noalloc(960, 16, 1.0, p, 960, p, 960, 4, p, 960, ctypes.byref(o), None, None) == -12
    assert lib.expm_pfd_apply_noalloc(4096, 16, 1.0, p, 4096, None, 4096, 4096, p, 4096, None, None, None) == -12
    o.precision = 1
    assert lib.expm_pfd_apply_noalloc(1152, 16, 1.0, p, 1152, p, 1152, 16, p, 1152, ctypes.byref(o), None,
                                      None) == -12
    text = open(HEADER).read()
    size = re.search(r"#define EXPM_PFD_NOALLOC_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert int(size.group(1)) << int(size.group(2)) == mod.NOALLOC_BYTES


def test_tridiag_validation_without_device():
    """The tridiagonal route's plan rejects bad arguments before any device work."""
    mod, lib = _lib()
    h = ctypes.c_void_p()
    assert lib.expm_pfd_tridiag_plan(None, 10, 16, 1, None) == -3
    assert lib.expm_pfd_tridiag_plan(ctypes.byref(h), 10, 15, 1, None) == -1
    assert lib.expm_pfd_tridiag_plan(ctypes.byref(h), 0, 16, 1, None) == -2
    assert lib.expm_pfd_tridiag_plan(ctypes.byref(h), 10, 16, 0, None) == -2
    assert lib.expm_pfd_tridiag_plan(ctypes.byref(h), 10, 16, 11, None) == -2
    assert lib.expm_pfd_tridiag_plan(ctypes.byref(h), 100, 16, 65, None) == -2
    assert lib.expm_pfd_tridiag_apply(None, 1.0, None, 1, 1, None, 1, None) == -3
    assert lib.expm_pfd_tridiag_factor(None, None, 1, None) == -3
    assert lib.expm_pfd_tridiag_destroy(None) == -3
    # the queue's reuse threshold: not negative, and not with real_data (the
    # tridiagonal route reads imaginary parts)
    o = mod._Opts()
    o.tridiag_reuse = -1
    assert lib.expm_pfd_queue_create(ctypes.byref(h), 1 << 30, 16, ctypes.byref(o), 8, 1) == -7
    o.tridiag_reuse, o.real_data = 2, 1
    assert lib.expm_pfd_queue_create(ctypes.byref(h), 1 << 30, 16, ctypes.byref(o), 8, 1) == -7


def test_band_validation_without_device():
    """The banded route's plan rejects bad arguments before any device work."""
    mod, lib = _lib()
    h = ctypes.c_void_p()
    assert lib.expm_pfd_band_plan(None, 10, 1, 16, 1, None) == -3
    assert lib.expm_pfd_band_plan(ctypes.byref(h), 10, 1, 15, 1, None) == -1
    assert lib.expm_pfd_band_plan(ctypes.byref(h), 0, 1, 16, 1, None) == -2
    assert lib.expm_pfd_band_plan(ctypes.byref(h), 10, -1, 16, 1, None) == -2
    assert lib.expm_pfd_band_plan(ctypes.byref(h), 10, 64, 16, 1, None) == -2  # kd above EXPM_PFD_BAND_MAX_KD
    assert lib.expm_pfd_band_plan(ctypes.byref(h), 10, 1, 16, 65, None) == -2
    assert lib.expm_pfd_band_plan(ctypes.byref(h), (1 << 24) + 1, 1, 16, 1, None) == -2
    o = mod._Opts()
    o.uplo = 3
    assert lib.expm_pfd_band_plan(ctypes.byref(h), 10, 1, 16, 1, ctypes.byref(o)) == -7
    assert lib.expm_pfd_band_apply(None, 1.0, None, 2, None, 10, 1, None, 10, None) == -3
    assert lib.expm_pfd_band_destroy(None) == -3
    text = open(HEADER).read()
    assert int(re.search(r"#define EXPM_PFD_BAND_MAX_KD\s+(\d+)", text).group(1)) == 63


@pytest.mark.parametrize("digits", [7, 16, 24, 34])
def test_choose_degree_matches_oracle(digits):
    """expm_pfd_choose_degree (host, from the library's binary128 residues) picks the
    oracle's degree for tolerances away from the thresholds, with the same flag and
    bound to a few ulps of the residue sums."""
    from oracle import scalar
    mod, lib = _lib()
    d = ctypes.c_int()
    b = ctypes.c_double()
    for tol in (1e-3, 1e-5, 3e-7, 3e-9, 1e-11, 1e-14, 0.0):
        rc = lib.expm_pfd_choose_degree(tol, digits, ctypes.byref(d), ctypes.byref(b))
        want_d, want_b, ok = scalar.choose_degree(tol, digits)
        assert (rc, d.value) == (0 if ok else 1, want_d), (digits, tol)
        assert abs(b.value - want_b) <= 1e-9 * want_b
    assert lib.expm_pfd_choose_degree(1e-8, 3, ctypes.byref(d), None) == -7
    assert lib.expm_pfd_choose_degree(float("nan"), 16, ctypes.byref(d), None) == -7
    assert lib.expm_pfd_choose_degree(1e-8, 16, None, None) == -3

