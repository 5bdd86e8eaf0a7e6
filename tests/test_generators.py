"""Seeded input generators: spectra exactly as prescribed, orthogonal bases,
reproducibility, exact perturbation norms.  (No oracle involved.)"""
import numpy as np

from workloads import (HouseholderBasis, batched_cones, haar_orthogonal,
                       large_cone, poisson_arrivals, rng_for, serving_sessions,
                       single_cone, sym_perturbation, warm_sequence)


def test_haar_orthogonal_and_reproducible():
    Q1 = haar_orthogonal(40, rng_for(9, 0))
    Q2 = haar_orthogonal(40, rng_for(9, 0))
    assert np.array_equal(Q1, Q2)
    assert np.abs(Q1.T @ Q1 - np.eye(40)).max() < 1e-13


def test_single_cone_spectrum():
    cone, V0 = single_cone()
    assert cone.X.shape == (50, 50) and V0.shape == (50, 8)
    assert cone.n_pos == 5
    assert np.all((cone.lam[cone.lam > 0] >= 1) & (cone.lam[cone.lam > 0] <= 10))
    assert np.all((cone.lam[cone.lam < 0] >= -10) & (cone.lam[cone.lam < 0] <= -0.1))
    w = np.linalg.eigvalsh(cone.X)
    assert np.abs(w - np.sort(cone.lam)).max() < 50 * 1e-15 * 10 * 10
    assert np.array_equal(cone.X, cone.X.T)


def test_warm_sequence_perturbation_norms():
    seq = warm_sequence(n=60, n_pos=4, steps=6)
    c0 = next(seq)
    X_prev = c0.X
    for k, X in enumerate(seq):
        E = X - X_prev
        assert np.array_equal(E, E.T)
        want = 1e-3 * 0.98 ** k * np.linalg.norm(X_prev)
        assert abs(np.linalg.norm(E) - want) <= 1e-12 * want
        X_prev = X


def test_large_cone_small_instance():
    X, lam, basis = large_cone(n=120, n_pos=4, n_reflectors=8)
    w = np.linalg.eigvalsh(X)
    assert np.abs(w - np.sort(lam)).max() <= 1e-12 * np.abs(lam).max()
    assert np.count_nonzero(lam > 0) == 4
    assert np.all(lam[lam > 0] >= 1.0) and np.all(lam[lam > 0] <= 100.0)
    assert np.all(lam[lam < 0] <= -1e-3) and np.all(lam[lam < 0] >= -100.0)


def test_householder_basis_is_orthogonal():
    rng = rng_for(99, 0)
    b = HouseholderBasis(rng.standard_normal((30, 5)))
    Q = b.sandwich(np.ones(30))
    assert np.abs(Q - np.eye(30)).max() < 1e-13


def test_batched_and_sessions():
    cones = batched_cones(count=20, n_min=16, n_max=40)
    for c in cones:
        assert 16 <= c.n <= 40
        assert c.n_pos == max(1, int(round(0.1 * c.n)))
    ss = serving_sessions(count=10, n_max=128)
    for s in ss:
        assert 32 <= s.n <= 128 and 1 <= s.n_pos <= s.n
        mags = np.abs(s.cone.lam)
        assert mags.min() >= 1e-3 and mags.max() <= 1e2
    t, sid = poisson_arrivals(2000.0, 0.5, 64)
    assert np.all(np.diff(t) > 0) and t[-1] < 0.5
    assert abs(t.size - 1000) < 200 and sid.max() < 64


def test_sym_perturbation_exact_norm():
    E = sym_perturbation(33, 0.125, rng_for(7, 1))
    assert abs(np.linalg.norm(E) - 0.125) < 1e-15
    assert np.array_equal(E, E.T)
