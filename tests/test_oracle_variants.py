"""CPU pins of the oracle's eigensolver variants (paper §1: truncated top-r
projection; §5: one block Krylov iteration): closed-form truncation errors
on prescribed spectra, the truncation bound, exactness when the block holds
an invariant subspace with the positive eigenvectors, the Rayleigh-Ritz
monotonicity of the Ritz values, and Thm `bound` with the exact tail."""
import numpy as np
import pytest

import oracle
from workloads import random_spectrum_matrix, rng_for


def _cone(n, npos, seed):
    return random_spectrum_matrix(n, npos, rng_for(95, seed), pos=(0.5, 5.0), neg=(-5.0, -0.1))


@pytest.mark.parametrize("r", [0, 2, 5, 8, 12])
def test_truncation_closed_form(r):
    c = _cone(30, 8, r)
    Pi_r, lam = oracle.truncated_projection(c.X, r)
    Pi, _ = oracle.project(c.X)
    pos = np.sort(c.lam[c.lam > 0])[::-1]
    missing = pos[r:] if r < pos.size else np.zeros(0)
    err = np.linalg.norm(Pi - Pi_r)
    assert err == pytest.approx(np.sqrt(np.sum(missing ** 2)), abs=1e-10)
    # the bound stated for exact leading pairs: (n - r) max(lam_r, 0)^2
    lam_r = lam[r - 1] if r > 0 else lam[0]
    assert err <= np.sqrt(30 - r) * max(lam_r, 0.0) + 1e-12 or r == 0
    if r >= 8:
        assert np.abs(Pi_r - Pi).max() <= 1e-12


def test_block_krylov_exact_on_invariant_block():
    c = _cone(40, 6, 1)
    idx = np.argsort(c.lam)[::-1][:9]          # the 6 positive and 3 more eigenvectors
    X0 = c.Q[:, idx] @ np.linalg.qr(rng_for(95, 2).standard_normal((9, 9)))[0]
    Pi_k, theta, _ = oracle.block_krylov_projection(c.X, X0)
    Pi, _ = oracle.project(c.X)
    assert np.abs(Pi_k - Pi).max() <= 1e-10
    assert np.allclose(np.sort(theta)[::-1], np.sort(c.lam[idx])[::-1], atol=1e-10)


def test_block_krylov_ritz_values_increase_and_bound_holds():
    c = _cone(60, 5, 3)
    X0 = rng_for(95, 4).standard_normal((60, 8))
    # Ritz values of span(X0) alone
    Q0, _ = np.linalg.qr(X0)
    th0 = np.sort(np.linalg.eigvalsh(Q0.T @ oracle.symmetrize_lower(c.X) @ Q0))[::-1]
    Pi1, th1, Y1 = oracle.block_krylov_projection(c.X, X0, steps=1)
    Pi2, th2, Y2 = oracle.block_krylov_projection(c.X, X0, steps=2)
    lam = np.sort(c.lam)[::-1]
    assert np.all(th1 >= th0 - 1e-12) and np.all(th2 >= th1 - 1e-12)
    assert np.all(th2 <= lam[:8] + 1e-12)               # interlacing with the spectrum
    Pi, _ = oracle.project(c.X)
    A = oracle.symmetrize_lower(c.X)
    for Pik, th, Y in ((Pi1, th1, Y1), (Pi2, th2, Y2)):
        pos = th > 0
        Vt, Lt = Y[:, pos], th[pos]
        R = A @ Vt - Vt * Lt
        lhs = np.linalg.norm(Pik - Pi) ** 2
        rhs = 2 * np.linalg.norm(R) ** 2 + oracle.tail_exact(c.X, Vt) ** 2
        assert lhs <= rhs * (1 + 1e-10) + 1e-20
    assert np.linalg.norm(Pi2 - Pi) <= np.linalg.norm(Pi1 - Pi) * (1 + 1e-9)
