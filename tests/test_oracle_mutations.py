"""Planted mistakes, on the CPU: each plausible slip in a projection routine
(a dropped clip, a wrong sign, a transposed eigenvector matrix, a shifted
index, a wrong power, a wrong threshold, the wrong triangle) must fail at
least one of the pins the oracle passes.  This shows the pins are able to
catch such a mistake in the oracle itself.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import random_spectrum_matrix, single_cone


def _pin_failures(project_fn):
    """Run a compact set of the pins on project_fn(X) -> Pi; return names of
    the pins it fails."""
    fails = []
    rng = np.random.default_rng(4242)
    # 2x2 closed form
    a, b, c = 1.0, 2.0, 1.0
    if not np.allclose(project_fn(np.array([[a, b], [b, c]], order="F")), 1.5 * np.ones((2, 2)), atol=1e-12):
        fails.append("2x2")
    # diagonal input with small positive, zero and negative entries
    d = np.array([0.3, -0.2, 0.0, 0.05, 2.0, -1.5])
    if not np.array_equal(project_fn(np.asfortranarray(np.diag(d))), np.diag(np.maximum(d, 0))):
        fails.append("diagonal")
    # construction closed form
    cone, _ = single_cone()
    exact = cone.sandwich(np.maximum(cone.lam, 0))
    if oracle.rel_error(project_fn(cone.X), exact) > 1e-10:
        fails.append("construction")
    # Moreau + psd-ness
    A = rng.standard_normal((9, 9))
    X = np.asfortranarray(A + A.T)
    P, M = project_fn(X), project_fn(-X)
    if np.abs(P - M - X).max() > 1e-10 or abs(np.sum(P * (P - X))) > 1e-10 * np.sum(X * X):
        fails.append("moreau")
    if np.linalg.eigvalsh(0.5 * (P + P.T)).min() < -1e-10:
        fails.append("psd")
    # distance identity on a prescribed spectrum
    c2 = random_spectrum_matrix(20, 4, rng)
    neg = c2.lam[c2.lam < 0]
    if abs(np.linalg.norm(c2.X - project_fn(c2.X)) ** 2 - np.sum(neg ** 2)) > 1e-9 * np.sum(c2.lam ** 2):
        fails.append("distance")
    # lower triangle only
    Y = X.copy(order="F")
    Y[np.triu_indices(9, 1)] = 7.0
    if not np.allclose(project_fn(Y), P, atol=1e-12):
        fails.append("lower")
    return fails


def _from_eigh(transform):
    def fn(X):
        Xs = np.asfortranarray(X)
        lam, V = oracle.eigh(Xs)
        return transform(np.asarray(Xs), lam, V)
    return fn


def test_oracle_passes_the_compact_suite():
    assert _pin_failures(lambda X: oracle.project(X)[0]) == []


MUTANTS = {
    "no_clip": lambda X, l, V: (V * l) @ V.T,
    "wrong_sign": lambda X, l, V: (V * np.minimum(l, 0)) @ V.T,
    "negated_result": lambda X, l, V: -(V * np.minimum(l, 0)) @ V.T,
    "transposed_V": lambda X, l, V: (V.T * np.maximum(l, 0)) @ V,
    "shifted_index": lambda X, l, V: (V * np.roll(np.maximum(l, 0), 1)) @ V.T,
    "squared_values": lambda X, l, V: (V * np.maximum(l, 0) ** 2) @ V.T,
    "wrong_threshold": lambda X, l, V: (V * np.where(l > 0.5, l, 0)) @ V.T,
    "upper_triangle": lambda X, l, V: oracle.project(np.asfortranarray(X.T))[0],
    "half_factor": lambda X, l, V: 0.5 * (V * np.maximum(l, 0)) @ V.T,
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    fails = _pin_failures(_from_eigh(MUTANTS[name]))
    assert fails, f"mutant {name} passed every pin"
