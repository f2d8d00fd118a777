"""Host half of qaa_spectrum (no GPU): the levels and residual norms it
reports for a Lanczos tridiagonal matrix, against scipy's tridiagonal
eigensolver (LAPACK) and the definition of the Ritz residual."""
import numpy as np
import pytest
from scipy.linalg import eigh_tridiagonal

import paper_1103_1399_amd as qaa


def _random_tridiag(m, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=m) * 3.0, np.abs(rng.normal(size=m)) + 0.1


@pytest.mark.parametrize("m,k,seed", [(1, 1, 0), (2, 2, 1), (30, 3, 2), (200, 5, 3), (1000, 2, 4)])
def test_levels_and_bounds_match_lapack(m, k, seed):
    a, b = _random_tridiag(m, seed)
    ev, bd = qaa.qaa_debug_tridiag_levels(a, b, k)
    w, y = eigh_tridiagonal(a, b[:m - 1]) if m > 1 else (a.copy(), np.ones((1, 1)))
    kk = min(k, m)
    scale = max(np.abs(a) + 2 * b)
    assert np.allclose(ev[:kk], w[:kk], atol=1e-12 * scale, rtol=0)
    # residual norm of the Ritz pair: |beta_m| |last component of the unit eigenvector|
    ref = np.abs(b[m - 1]) * np.abs(y[m - 1, :kk])
    assert np.allclose(bd[:kk], ref, rtol=1e-6, atol=1e-14 * scale)
    assert np.all(np.isnan(ev[kk:])) and np.all(np.isnan(bd[kk:]))


def test_closed_krylov_space_uses_the_leading_block():
    """A negligible beta ends the matrix: the levels are those of the
    leading block, with zero-size residuals."""
    a, b = _random_tridiag(40, 5)
    b[11] = 1e-300
    ev, bd = qaa.qaa_debug_tridiag_levels(a, b, 3)
    w = eigh_tridiagonal(a[:12], b[:11], eigvals_only=True)
    assert np.allclose(ev, w[:3], atol=1e-12, rtol=0)
    assert np.all(bd < 1e-250)


def test_repeated_levels_are_merged():
    """Two decoupled copies of one block (as a degenerate level reached
    twice): each level is reported once."""
    a0, b0 = _random_tridiag(10, 6)
    a = np.concatenate([a0, a0])
    b = np.concatenate([b0[:9], [1e-9], b0[:9], [0.5]])
    ev, _ = qaa.qaa_debug_tridiag_levels(a, b, 4)
    w = eigh_tridiagonal(a0, b0[:9], eigvals_only=True)
    assert np.allclose(ev, w[:4], atol=1e-8, rtol=0)


def test_bad_arguments_are_rejected():
    with pytest.raises(qaa.QaaError):
        qaa.qaa_debug_tridiag_levels(np.zeros(0), np.zeros(0), 1)
    with pytest.raises(ValueError):
        qaa.qaa_debug_tridiag_levels(np.zeros(3), np.zeros(2), 1)
