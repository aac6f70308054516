"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case patches one plausible mistake into the oracle (a dropped term, a wrong
sign, a wrong index, a transposed operand) and checks that a pin from
test_oracle_scalar / test_oracle_matrix fails.  Nothing here touches the GPU.
"""

import numpy as np
import pytest

from oracle import matrix, scalar
import tests.test_oracle_matrix as pins_m
import tests.test_oracle_scalar as pins_s


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_dropped_taylor_term_is_caught(monkeypatch):
    orig = scalar.exp_d

    def exp_d_short(z, d):  # drops the z^d/d! term
        return orig(z, d - 1)

    monkeypatch.setattr(scalar, "exp_d", exp_d_short)
    _fails(pins_m.test_brute_force_tiny, 8)


def test_wrong_horner_index_is_caught(monkeypatch):
    def exp_d_bad(z, d):
        s = 1
        for k in range(d, 0, -1):
            s = 1 + s * z / (k + 1)
        return s

    monkeypatch.setattr(scalar, "exp_d", exp_d_bad)
    _fails(pins_m.test_diagonal_gives_diagonal)


def test_transposed_eigenvectors_are_caught(monkeypatch):
    def apply_T(U, f, V):  # U^T instead of U^H
        if V is None:
            return (U * f[None, :]) @ U.T
        return U @ (f[:, None] * (U.T @ np.asarray(V, dtype=np.complex128)))

    monkeypatch.setattr(matrix, "_apply_spectral", apply_T)
    _fails(pins_m.test_polynomial_route)


def test_flipped_residue_sign_is_caught(monkeypatch):
    th, a = scalar.pfd_full_mp(16)
    bad = (th, tuple([-a[0]] + list(a[1:])))
    monkeypatch.setattr(scalar, "pfd_full_mp", lambda d, dps=60: bad)
    _fails(pins_s.test_moment_identities, 16)


def test_sign_of_shift_is_caught(monkeypatch):
    """(tA - theta I) instead of (tA + theta I) in the 50-digit route."""
    th, a = scalar.pfd_full_mp(8)
    monkeypatch.setattr(scalar, "pfd_full_mp", lambda d, dps=60: (tuple(-t for t in th), a))
    _fails(pins_m.test_brute_force_tiny, 8)


def test_wrong_pair_member_is_caught(monkeypatch):
    """Keeping Im theta > 0 poles but the residues of the conjugate member."""
    orig = scalar.pfd_pairs

    def pairs_bad(d):
        t, r = orig(d)
        return t, r.conj()

    monkeypatch.setattr(scalar, "pfd_pairs", pairs_bad)
    _fails(pins_s.test_degree2_closed_form)


def test_amplification_without_residue_weights_is_caught(monkeypatch):
    """The amplification factor with every |a_k| taken as 1 (residues dropped)."""
    orig = scalar.pfd_all

    def unit_residues(d):
        t, r = orig(d)
        return t, np.ones_like(r)

    monkeypatch.setattr(scalar, "pfd_all", unit_residues)
    _fails(pins_m.test_pfd_amplification_pins)
