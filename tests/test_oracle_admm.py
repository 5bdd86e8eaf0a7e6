"""CPU pins of the ADMM oracle (paper §2 Alg. 1, §6.2 infeasibility tests):
closed-form SDP optima (minimum eigenvalue under a trace constraint; the
max-cut relaxation of the complete graph, N^2/4; the Lovász theta numbers of
C_5, K_N and the empty graph: sqrt 5, 1, N), the KKT conditions of the
returned point checked with LAPACK, the two infeasibility certificates, and
planted mistakes that the pins catch."""
import math

import numpy as np
import pytest

from oracle import admm as oadmm
from workloads import (complete_graph, cycle_graph, dual_infeasible, maxcut, primal_infeasible,
                       theta, trace_min)


def _solve(sdp, **kw):
    kw.setdefault("max_iter", 20000)
    return oadmm.admm(sdp.C, sdp.dense_constraints(), sdp.b, **kw)


def _kkt(sdp, res, tol):
    """Primal feasibility, dual slack S = C + sum_i y_i A_i psd, <S, Y> = 0."""
    A = sdp.dense_constraints()
    Y = res.Y
    assert np.linalg.eigvalsh(Y).min() >= -tol
    for Ai, bi in zip(A, sdp.b):
        assert abs(np.sum(Ai * Y) - bi) <= tol
    S = sdp.C + sum(yi * Ai for yi, Ai in zip(res.y, A))
    assert np.linalg.eigvalsh(S).min() >= -tol * max(1.0, np.abs(S).max())
    assert abs(np.sum(S * Y)) <= tol * max(1.0, np.abs(S).max())
    # the multiplier of the PSD block is -S at a solution
    assert np.abs(res.W + S).max() <= tol * max(1.0, np.abs(S).max())


def test_svec_is_an_isometry():
    rng = np.random.default_rng(5)
    for n in (1, 2, 5):
        X = rng.standard_normal((n, n)); X = X + X.T
        Y = rng.standard_normal((n, n)); Y = Y + Y.T
        assert oadmm.svec(X) @ oadmm.svec(Y) == pytest.approx(np.sum(X * Y))
        assert np.allclose(oadmm.smat(oadmm.svec(Y), n), Y)


@pytest.mark.parametrize("n", [6, 12])
def test_trace_min_is_smallest_eigenvalue(n):
    sdp = trace_min(n)
    res = _solve(sdp)
    lam, U = np.linalg.eigh(sdp.C)
    assert res.status == "solved"
    assert res.obj == pytest.approx(lam[0], abs=1e-5)
    v = U[:, 0]
    assert np.abs(res.Y - np.outer(v, v)).max() <= 1e-4
    _kkt(sdp, res, 1e-5)


@pytest.mark.parametrize("n", [4, 9])
def test_maxcut_complete_graph(n):
    # -<L, Y>/4 = -(n tr Y - 1^T Y 1)/4 >= -n^2/4, equality at 1^T Y 1 = 0
    sdp = maxcut(n, edges=complete_graph(n), weights=False)
    res = _solve(sdp)
    assert res.status == "solved"
    assert res.obj == pytest.approx(-n * n / 4.0, abs=1e-5)
    _kkt(sdp, res, 1e-5)


@pytest.mark.parametrize("edges,n,value", [
    (cycle_graph(5), 5, math.sqrt(5.0)),       # Lovasz: theta(C_5) = sqrt 5
    (complete_graph(6), 6, 1.0),              # theta(K_n) = 1
    ([], 7, 7.0),                             # theta of the empty graph = n
])
def test_theta_closed_forms(edges, n, value):
    sdp = theta(n, edges=edges)
    res = _solve(sdp)
    assert res.status == "solved"
    assert -res.obj == pytest.approx(value, abs=1e-5)
    _kkt(sdp, res, 1e-5)


def test_random_maxcut_kkt():
    sdp = maxcut(14, prob=0.4)
    res = _solve(sdp)
    assert res.status == "solved"
    _kkt(sdp, res, 1e-5)


def test_primal_infeasibility_certificate():
    res = _solve(primal_infeasible(8), max_iter=5000)
    assert res.status == "primal_infeasible"


def test_dual_infeasibility_certificate():
    res = _solve(dual_infeasible(8), max_iter=5000)
    assert res.status == "dual_infeasible"


def _pins_pass(sdp, res, value):
    if res.status != "solved" or abs(-res.obj - value) > 1e-4:
        return False
    try:
        _kkt(sdp, res, 1e-5)
    except AssertionError:
        return False
    return True


def test_pins_catch_planted_mistakes():
    """Plausible slips in the loop (a projection that forgets the cone or
    scales it, a wrong sign in the dual update) fail the closed-form value
    of theta(C_5) or the KKT conditions."""
    sdp = theta(5, edges=cycle_graph(5))
    assert _pins_pass(sdp, _solve(sdp), math.sqrt(5.0))

    def no_clip(V):
        return 0.5 * (V + V.T)   # "projection" that forgets the cone

    def half_clip(V):
        lam, U = np.linalg.eigh(0.5 * (V + V.T))
        return (U * np.maximum(lam, 0) * 0.5) @ U.T   # scaled wrongly

    for proj in (no_clip, half_clip):
        assert not _pins_pass(sdp, _solve(sdp, max_iter=3000, proj=proj), math.sqrt(5.0))
    # dual update with the wrong sign (the oracle run with rho < 0 flips it)
    assert not _pins_pass(sdp, _solve(sdp, max_iter=3000, rho=-0.1), math.sqrt(5.0))
