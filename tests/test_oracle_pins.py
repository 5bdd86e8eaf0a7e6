"""Pins of the oracle against facts other than the oracle itself.

Each test checks the oracle (FP64 Jacobi + clip, paper §1 eq. `projection`)
against a closed form, an invariant of the projection onto a closed convex
cone, LAPACK, or brute force on tiny inputs.  Together they are chosen so
that a dropped clip, a wrong sign, a transposed eigenvector matrix, a wrong
index or a missing symmetrization fails at least one of them
(test_oracle_mutations.py plants such mistakes and checks that they do).
"""
import math

import numpy as np
import pytest

import oracle
from workloads import (batched_cones, haar_orthogonal, from_spectrum,
                       random_spectrum_matrix, rng_for, single_cone)


def _rng(i):
    return np.random.default_rng(1000 + i)


def _sym(n, rng, scale=1.0):
    A = rng.standard_normal((n, n)) * scale
    return np.asfortranarray(A + A.T)


# ------------------------------------------------------------- closed forms --
def _pi_2x2(a, b, c):
    """Closed-form projection of [[a,b],[b,c]] (independent of the oracle)."""
    h = 0.5 * (a + c)
    r = math.hypot(0.5 * (a - c), b)
    lp, lm = h + r, h - r
    if lm >= 0:
        return np.array([[a, b], [b, c]]), (lm, lp)
    if lp <= 0:
        return np.zeros((2, 2)), (lm, lp)
    v = np.array([b, lp - a])
    if np.linalg.norm(v) < 1e-300 or abs(b) < 1e-300:
        v = np.array([lp - c, b])
    if np.linalg.norm(v) < 1e-300:
        v = np.array([1.0, 0.0]) if a >= c else np.array([0.0, 1.0])
    v = v / np.linalg.norm(v)
    return lp * np.outer(v, v), (lm, lp)


@pytest.mark.parametrize("seed", range(40))
def test_2x2_closed_form(seed):
    rng = _rng(seed)
    a, b, c = rng.uniform(-3, 3, 3)
    if seed % 5 == 0:
        b = 0.0
    X = np.array([[a, b], [b, c]], order="F")
    Pi, lam = oracle.project(X)
    Pc, (lm, lp) = _pi_2x2(a, b, c)
    assert np.allclose(lam, [lm, lp], atol=1e-14 * (1 + abs(lp) + abs(lm)))
    assert np.abs(Pi - Pc).max() <= 1e-13 * (1 + np.abs(X).max())


def test_2x2_worked_values():
    # [[1,2],[2,1]]: eigenvalues 3 and -1, eigenvector (1,1)/sqrt2 for 3.
    Pi, lam = oracle.project(np.array([[1.0, 2.0], [2.0, 1.0]], order="F"))
    assert np.allclose(lam, [-1.0, 3.0], atol=1e-15)
    assert np.allclose(Pi, 1.5 * np.ones((2, 2)), atol=1e-15)
    # [[0,1],[1,0]]: eigenvalues +-1, projection 0.5 * ones
    Pi, lam = oracle.project(np.array([[0.0, 1.0], [1.0, 0.0]], order="F"))
    assert np.allclose(Pi, 0.5 * np.ones((2, 2)), atol=1e-15)


def _eig3_trig(A):
    """Eigenvalues of a symmetric 3x3 by the trigonometric solution of the
    characteristic cubic (Smith 1961), ascending."""
    p1 = A[0, 1] ** 2 + A[0, 2] ** 2 + A[1, 2] ** 2
    q = np.trace(A) / 3.0
    if p1 == 0.0:
        return np.sort(np.diag(A))
    p2 = (A[0, 0] - q) ** 2 + (A[1, 1] - q) ** 2 + (A[2, 2] - q) ** 2 + 2 * p1
    p = math.sqrt(p2 / 6.0)
    B = (A - q * np.eye(3)) / p
    r = np.linalg.det(B) / 2.0
    r = min(1.0, max(-1.0, r))
    phi = math.acos(r) / 3.0
    e1 = q + 2 * p * math.cos(phi)
    e3 = q + 2 * p * math.cos(phi + 2 * math.pi / 3)
    e2 = 3 * q - e1 - e3
    return np.sort([e1, e2, e3])


@pytest.mark.parametrize("seed", range(25))
def test_3x3_trigonometric_eigenvalues(seed):
    X = _sym(3, _rng(100 + seed))
    lam, V = oracle.eigh(X)
    ref = _eig3_trig(np.asarray(X))
    assert np.abs(lam - ref).max() <= 1e-12 * (1 + np.abs(ref).max())
    # and the projection's squared distance equals the clipped eigenvalue mass
    Pi, _ = oracle.project(X)
    neg = ref[ref < 0]
    assert abs(np.linalg.norm(X - Pi) ** 2 - np.sum(neg ** 2)) <= 1e-11 * (1 + np.sum(ref ** 2))


@pytest.mark.parametrize("d", [
    [3.0, -1.0, 0.0, 2.0, -5.0],
    [1.0, 1.0, 1.0],
    [-1.0, -2.0, -3.0, -4.0],
    [0.0, 0.0, 0.0],
    [7.0],
    [-7.0],
    [2.0, -2.0, 2.0, -2.0, 2.0, -2.0],
])
def test_diagonal_inputs(d):
    d = np.array(d)
    X = np.asfortranarray(np.diag(d))
    Pi, lam = oracle.project(X)
    assert np.array_equal(Pi, np.diag(np.maximum(d, 0)))
    assert np.array_equal(lam, np.sort(d))


def test_empty_and_scalar():
    Pi, lam = oracle.project(np.zeros((0, 0)))
    assert Pi.shape == (0, 0) and lam.shape == (0,)
    for x in (-2.5, 0.0, 3.25):
        Pi, _ = oracle.project(np.array([[x]]))
        assert Pi[0, 0] == max(x, 0.0)


def test_psd_and_nsd_inputs():
    rng = _rng(7)
    for n in (5, 17, 40):
        Q = haar_orthogonal(n, rng)
        lam = rng.uniform(0.1, 4.0, n)
        X = from_spectrum(Q, lam)
        Pi, _ = oracle.project(X)
        assert np.abs(Pi - X).max() <= 1e-12 * np.abs(X).max()
        Pi, _ = oracle.project(-X)
        assert np.abs(Pi).max() <= 1e-12 * np.abs(X).max()


# ------------------------------------------------------ construction closed --
def test_construction_closed_form_config1():
    cone, _ = single_cone()
    Pi, lam = oracle.project(cone.X)
    exact = cone.sandwich(np.maximum(cone.lam, 0))
    assert np.allclose(lam, np.sort(cone.lam), atol=1e-12 * np.abs(cone.lam).max())
    assert oracle.rel_error(Pi, exact) <= 1e-13


def test_construction_closed_form_repeated_eigenvalues():
    # Pi is unique even when eigenvalues repeat (projection onto a closed
    # convex set); individual eigenvectors are not.
    rng = _rng(8)
    n = 30
    Q = haar_orthogonal(n, rng)
    lam = np.array([2.0] * 6 + [0.0] * 4 + [-1.0] * 20)
    X = from_spectrum(Q, lam)
    Pi, _ = oracle.project(X)
    assert oracle.rel_error(Pi, from_spectrum(Q, np.maximum(lam, 0))) <= 1e-13


def test_construction_closed_form_batched_cones():
    cones = batched_cones(count=6, n_min=16, n_max=80)
    for c in cones:
        Pi, _ = oracle.project(c.X)
        assert oracle.rel_error(Pi, c.sandwich(np.maximum(c.lam, 0))) <= 1e-12


# -------------------------------------------------------------- invariants --
@pytest.mark.parametrize("n", [4, 9, 33, 64])
def test_moreau_decomposition(n):
    """X = Pi(X) - Pi(-X) and <Pi(X), Pi(X) - X> = 0 (projection onto a
    self-dual cone), with Pi(X) psd and Pi(X) - X psd."""
    X = _sym(n, _rng(n))
    P, _ = oracle.project(X)
    M, _ = oracle.project(-X)
    scale = np.abs(X).max()
    assert np.abs(P - M - X).max() <= 1e-12 * scale * n
    assert abs(np.sum(P * (P - X))) <= 1e-12 * np.linalg.norm(X) ** 2
    assert np.linalg.eigvalsh(P).min() >= -1e-12 * scale * n
    assert np.linalg.eigvalsh(P - X).min() >= -1e-12 * scale * n


@pytest.mark.parametrize("n", [5, 20, 50])
def test_idempotence_and_distance(n):
    rng = _rng(200 + n)
    c = random_spectrum_matrix(n, max(1, n // 4), rng)
    P, _ = oracle.project(c.X)
    P2, _ = oracle.project(P)
    assert np.abs(P2 - P).max() <= 1e-12 * np.abs(P).max() * n
    neg = c.lam[c.lam < 0]
    assert abs(np.linalg.norm(c.X - P) ** 2 - np.sum(neg ** 2)) <= 1e-11 * np.sum(c.lam ** 2)


def test_nonexpansive_and_homogeneous():
    rng = _rng(300)
    for trial in range(6):
        n = 12 + 5 * trial
        X = _sym(n, rng)
        Y = X + 0.3 * _sym(n, rng)
        PX, _ = oracle.project(X)
        PY, _ = oracle.project(Y)
        assert np.linalg.norm(PX - PY) <= np.linalg.norm(X - Y) * (1 + 1e-12)
        t = rng.uniform(0.1, 7.0)
        PtX, _ = oracle.project(t * X)
        assert np.abs(PtX - t * PX).max() <= 1e-12 * t * np.abs(X).max() * n


def test_orthogonal_equivariance():
    rng = _rng(400)
    n = 25
    X = _sym(n, rng)
    U = haar_orthogonal(n, rng)
    PX, _ = oracle.project(X)
    PU, _ = oracle.project(U @ X @ U.T)
    assert np.abs(PU - U @ PX @ U.T).max() <= 1e-12 * np.abs(X).max() * n


@pytest.mark.parametrize("n", [2, 7, 31, 100])
def test_agrees_with_lapack(n):
    X = _sym(n, _rng(500 + n))
    Pi, lam = oracle.project(X)
    w, Q = np.linalg.eigh(X)
    ref = (Q * np.maximum(w, 0)) @ Q.T
    scale = np.linalg.norm(X, 2)
    assert np.abs(lam - w).max() <= 10 * n * np.finfo(float).eps * scale
    assert np.abs(Pi - ref).max() <= 10 * n * np.finfo(float).eps * scale


def test_jacobi_internals():
    rng = _rng(600)
    c = random_spectrum_matrix(60, 7, rng)
    lam, V, sweeps = oracle.eigh(c.X, return_sweeps=True)
    n = 60
    eps = np.finfo(float).eps
    assert np.abs(V.T @ V - np.eye(n)).max() <= 20 * n * eps
    assert np.abs((V * lam) @ V.T - c.X).max() <= 20 * n * eps * np.abs(c.lam).max()
    assert np.all(np.diff(lam) >= 0)
    assert np.abs(lam - np.sort(c.lam)).max() <= 20 * n * eps * np.abs(c.lam).max()
    assert 1 <= sweeps <= 20


def test_reads_lower_triangle_only():
    rng = _rng(700)
    X = _sym(12, rng)
    Y = X.copy(order="F")
    Y[np.triu_indices(12, 1)] = 1e6 * rng.standard_normal(66)
    P1, _ = oracle.project(X)
    P2, _ = oracle.project(Y)
    assert np.array_equal(P1, P2)


def test_rejects_nonfinite():
    X = np.eye(4, order="F")
    X[2, 1] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.project(X)


# ------------------------------------------------------------ brute force --
def _brute_force_projection(X, rng):
    """min_L ||X - L L^T||_F over lower-triangular L: coarse random search
    plus Nelder-Mead refinement (scipy), best of several starts."""
    from scipy.optimize import minimize
    n = X.shape[0]
    idx = np.tril_indices(n)

    def f(z):
        L = np.zeros((n, n))
        L[idx] = z
        return np.sum((X - L @ L.T) ** 2)

    k = len(idx[0])
    s = math.sqrt(max(np.abs(X).max(), 1e-3))
    best = None
    cand = [rng.uniform(-2 * s, 2 * s, k) for _ in range(400)]
    cand.sort(key=f)
    for z0 in cand[:6] + [np.zeros(k) + 1e-3]:
        r = minimize(f, z0, method="Nelder-Mead",
                     options=dict(xatol=1e-12, fatol=1e-22, maxiter=40000, maxfev=40000))
        r = minimize(f, r.x, method="BFGS", options=dict(gtol=1e-13))
        if best is None or r.fun < best.fun:
            best = r
    L = np.zeros((n, n))
    L[idx] = best.x
    return L @ L.T


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_tiny(seed):
    rng = _rng(800 + seed)
    n = 2 if seed < 3 else 3
    X = _sym(n, rng)
    Pi, _ = oracle.project(X)
    Pb = _brute_force_projection(np.asarray(X), rng)
    # the brute-force minimiser reaches the same unique minimum
    assert np.linalg.norm(X - Pb) >= np.linalg.norm(X - Pi) - 1e-9
    assert np.abs(Pb - Pi).max() <= 1e-5 * (1 + np.abs(X).max())


def test_kkt_characterisation_on_grid():
    """Y = Pi(X) iff Y psd, Y - X psd and <Y, Y - X> = 0.  On a grid of 2x2
    inputs, the oracle's output satisfies all three, and perturbing it in any
    of several directions breaks at least one."""
    vals = np.linspace(-2, 2, 7)
    for a in vals:
        for b in vals:
            for c in vals:
                X = np.array([[a, b], [b, c]], order="F")
                Y, _ = oracle.project(X)
                e1 = np.linalg.eigvalsh(Y).min()
                e2 = np.linalg.eigvalsh(Y - X).min()
                assert e1 >= -1e-13 and e2 >= -1e-13
                assert abs(np.sum(Y * (Y - X))) <= 1e-13 * (1 + np.sum(X * X))


# ------------------------------------------------ Thm `bound` as inequality --
def _rayleigh_ritz(X, S):
    Q, _ = np.linalg.qr(S)
    H = Q.T @ X @ Q
    th, W = np.linalg.eigh(0.5 * (H + H.T))
    return th, Q @ W


@pytest.mark.parametrize("seed", range(8))
def test_theorem_bound_holds_for_ritz_pairs(seed):
    """§5.2 Thm `bound`: for positive Ritz pairs (Vt, Lt) with Lt = Vt^T X Vt,
    ||Vt Lt Vt^T - Pi(X)||_F^2 <= 2||R||_F^2 + ||Pi(Vt_perp^T X Vt_perp)||_F^2.
    The trial subspace is a perturbed copy of the positive eigenspace, so the
    Ritz pairs are inexact; the check exercises tail_exact too."""
    rng = _rng(900 + seed)
    n, p = 40, 6
    c = random_spectrum_matrix(n, p, rng, pos=(0.5, 4.0), neg=(-4.0, -0.05))
    pos_vecs = c.Q[:, c.lam > 0]
    S = pos_vecs + (0.05 + 0.1 * seed) * rng.standard_normal((n, p + 3))[:, :p]
    S = np.hstack([S, rng.standard_normal((n, 3))])
    th, Y = _rayleigh_ritz(c.X, S)
    keep = th > 0
    Vt, Lt = Y[:, keep], th[keep]
    R = c.X @ Vt - Vt * Lt
    Pi, _ = oracle.project(c.X)
    lhs = np.linalg.norm((Vt * Lt) @ Vt.T - Pi) ** 2
    rhs = 2 * np.linalg.norm(R) ** 2 + oracle.tail_exact(c.X, Vt) ** 2
    assert lhs <= rhs * (1 + 1e-10) + 1e-24


def test_tail_exact_special_cases():
    rng = _rng(950)
    c = random_spectrum_matrix(30, 5, rng)
    Pi, _ = oracle.project(c.X)
    # empty Vt: the tail is the whole projection
    assert abs(oracle.tail_exact(c.X, np.zeros((30, 0))) - np.linalg.norm(Pi)) <= 1e-12 * np.linalg.norm(Pi)
    # exact positive eigenvectors: nothing positive left
    assert oracle.tail_exact(c.X, c.Q[:, c.lam > 0]) <= 1e-12 * np.linalg.norm(Pi)
    # only some of them: the tail is the norm of the missing positive part
    pos = np.flatnonzero(c.lam > 0)
    Vt = c.Q[:, pos[:2]]
    miss = c.lam[pos[2:]]
    assert abs(oracle.tail_exact(c.X, Vt) - np.sqrt(np.sum(miss ** 2))) <= 1e-11 * np.linalg.norm(Pi)


@pytest.mark.parametrize("n,m", [(12, 3), (40, 7), (33, 0)])
def test_complement_spectrum_closed_form(n, m):
    # X = Q diag(lam) Q^T and Vt = m columns of Q: the compression to the
    # complement has exactly the other prescribed eigenvalues
    rng = _rng(960 + n)
    c = random_spectrum_matrix(n, max(1, n // 4), rng, pos=(0.5, 3.0), neg=(-4.0, -0.01))
    idx = rng.permutation(n)
    Vt = c.Q[:, idx[:m]]
    mu = oracle.complement_spectrum(c.X, Vt)
    rest = np.sort(c.lam[idx[m:]])
    assert mu.shape == (n - m,)
    assert np.abs(mu - rest).max() <= 1e-12 * np.abs(c.lam).max() * n


def test_complement_spectrum_interlaces():
    # Cauchy interlacing for an arbitrary orthonormal Vt (n x m):
    # lam_k(X) <= mu_k <= lam_{k+m}(X), all ascending
    rng = _rng(970)
    n, m = 25, 4
    X = _sym(n, rng)
    Vt, _ = np.linalg.qr(rng.standard_normal((n, m)))
    mu = oracle.complement_spectrum(X, Vt)
    lam = np.linalg.eigvalsh(X)
    tol = 1e-12 * np.abs(lam).max() * n
    assert np.all(lam[: n - m] <= mu + tol)
    assert np.all(mu <= lam[m:] + tol)
    # the tail term is the norm of the compression's positive part
    pos = mu[mu > 0]
    assert abs(oracle.tail_exact(X, Vt) - np.sqrt(np.sum(pos ** 2))) <= tol * n


def test_complement_spectrum_catches_planted_mistakes():
    # the closed-form pin above fails for plausible slips in the shift trick
    rng = _rng(980)
    c = random_spectrum_matrix(15, 4, rng, pos=(0.5, 3.0), neg=(-4.0, -0.1))
    Vt = c.Q[:, :3]
    rest = np.sort(c.lam[3:])
    X = oracle.symmetrize_lower(c.X)
    n = 15

    def variant(shift_sign, drop_first):
        s = shift_sign * (2.0 * np.linalg.norm(X) + 1.0)
        P = np.eye(n) - Vt @ Vt.T
        lam = np.linalg.eigvalsh(P @ X @ P - s * (Vt @ Vt.T))
        return lam[3:] if drop_first else lam[:-3]

    assert np.abs(variant(+1, True) - rest).max() < 1e-10          # the oracle's form
    assert np.abs(variant(-1, True) - rest).max() > 1e-3           # wrong shift sign
    assert np.abs(variant(+1, False) - rest).max() > 1e-3          # wrong end dropped


def test_bound_counterexample_needs_positive_ritz_vectors():
    # The theorem is stated for positive Ritz pairs: with X = diag(1,-1) and
    # Vt = I (a negative Ritz pair kept), R = 0 and the tail is 0, yet the
    # error is 1.  This is why only theta > 0 pairs enter Vt.
    X = np.diag([1.0, -1.0])
    Pi, _ = oracle.project(X)
    Vt = np.eye(2)
    err = np.linalg.norm(Vt @ np.diag([1.0, -1.0]) @ Vt.T - Pi)
    assert err == pytest.approx(1.0)
    assert oracle.tail_exact(X, Vt) == 0.0


def test_golden_regression():
    """The oracle still reproduces its own stored outputs (regression only;
    the file is written by tests/golden/make_golden.py from oracle/)."""
    import json
    import os
    from workloads import batched_cones
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_small.json")
    data = json.load(open(path))
    cone, _ = single_cone()
    mats = {"single_cone_n50": cone.X}
    for i, c in enumerate(batched_cones(count=3, n_min=16, n_max=48)):
        mats[f"batched_cone_{i}_n{c.n}"] = c.X
    for case in data["cases"]:
        Pi, lam = oracle.project(mats[case["name"]])
        assert np.abs(lam - np.array(case["lam"])).max() <= 1e-12 * (1 + np.abs(lam).max())
        assert abs(np.linalg.norm(Pi) - case["pi_fro"]) <= 1e-12 * (1 + case["pi_fro"])
