"""Seeded synthetic workloads with prescribed spectra.

The paper measures on SDPLIB problems inside an ADMM solver (§6.1, Table 1),
which are not available here.  These generators stand in for them: dense
symmetric matrices X = Q diag(lam) Q^T with a prescribed inertia (few positive
eigenvalues, as in Table 1's "rank" column) and ADMM-like warm-start
sequences X_{k+1} = X_k + E_k of slowly drifting matrices (§5.1: warm starting
across ADMM iterations).

Seeds: every stream is PCG64 seeded with SeedSequence([1912, 2767, config, stream]).
Nothing here computes a projection or an eigendecomposition.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Iterator, List, Optional

import numpy as np

__all__ = [
    "rng_for", "haar_orthogonal", "from_spectrum", "sym_perturbation",
    "cold_block", "Cone", "HouseholderBasis",
    "single_cone", "warm_sequence", "large_cone", "large_cone_sequence",
    "batched_cones", "serving_sessions", "poisson_arrivals", "SessionSpec",
    "session_sequence", "gapped_sessions",
    "random_spectrum_matrix",
]


def rng_for(config_id: int, stream_id: int = 0) -> np.random.Generator:
    """PCG64 stream for (config, stream)."""
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([1912, 2767, int(config_id), int(stream_id)])))


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal Q: QR of an N(0,1) matrix, columns signed by
    sign(diag R) (sign(0) taken as +1)."""
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return np.asfortranarray(Q * d)


def from_spectrum(Q: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """X = Q diag(lam) Q^T, exactly symmetrized, Fortran order."""
    X = (Q * lam) @ Q.T
    return np.asfortranarray(0.5 * (X + X.T))


def sym_perturbation(n: int, fro: float, rng: np.random.Generator) -> np.ndarray:
    """Symmetric Gaussian E = G + G^T rescaled to ||E||_F = fro."""
    G = rng.standard_normal((n, n))
    E = G + G.T
    nrm = np.linalg.norm(E)
    if nrm > 0:
        E *= fro / nrm
    return np.asfortranarray(E)


def cold_block(n: int, m: int, rng: np.random.Generator) -> np.ndarray:
    """N(0,1) n x m start block for a cold LOBPCG start."""
    return np.asfortranarray(rng.standard_normal((n, m)))


@dataclass
class Cone:
    """One symmetric matrix with a known spectrum: X = Q diag(lam) Q^T."""
    X: np.ndarray
    lam: np.ndarray
    Q: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def n_pos(self) -> int:
        return int(np.count_nonzero(self.lam > 0))

    def sandwich(self, d: np.ndarray) -> np.ndarray:
        """Q diag(d) Q^T in this cone's basis."""
        return from_spectrum(self.Q, d)


@dataclass
class HouseholderBasis:
    """Q = H_1 H_2 ... H_k with H_i = I - 2 v_i v_i^T / (v_i^T v_i)."""
    vs: np.ndarray  # n x k, column i is v_i

    def sandwich(self, d: np.ndarray) -> np.ndarray:
        """Q diag(d) Q^T formed by applying the reflectors on both sides, O(k n^2)."""
        X = np.diag(np.asarray(d, dtype=np.float64))
        # Q D Q^T = H_1 (H_2 (... (H_k D H_k) ...) H_2) H_1
        for i in range(self.vs.shape[1] - 1, -1, -1):
            v = self.vs[:, i]
            beta = 2.0 / float(v @ v)
            w = X @ v                      # X symmetric: X v = (v^T X)^T
            X -= beta * np.outer(v, w)     # H X
            w2 = X @ v
            X -= beta * np.outer(w2, v)    # (H X) H
        return np.asfortranarray(0.5 * (X + X.T))


def _permuted(rng, parts: List[np.ndarray]) -> np.ndarray:
    lam = np.concatenate(parts)
    return lam[rng.permutation(lam.size)]


def random_spectrum_matrix(n: int, n_pos: int, rng: np.random.Generator,
                           pos=(1.0, 10.0), neg=(-10.0, -0.1)) -> Cone:
    """Haar basis with n_pos eigenvalues U[pos] and n - n_pos eigenvalues U[neg]."""
    Q = haar_orthogonal(n, rng)
    lam = _permuted(rng, [rng.uniform(pos[0], pos[1], n_pos),
                          rng.uniform(neg[0], neg[1], n - n_pos)])
    return Cone(from_spectrum(Q, lam), lam, Q)


# ---------------------------------------------------------------- config 1 --
def single_cone(n: int = 50, n_pos: int = 5, block: int = 8, stream: int = 0):
    """Plain single cone: n=50, 5 eigenvalues U[1,10], 45 U[-10,-0.1], Haar
    basis; plus an N(0,1) n x 8 cold-start block.  Returns (Cone, V0)."""
    rng = rng_for(1, stream)
    cone = random_spectrum_matrix(n, n_pos, rng, pos=(1.0, 10.0), neg=(-10.0, -0.1))
    V0 = cold_block(n, block, rng)
    return cone, V0


# ---------------------------------------------------------------- config 2 --
def warm_sequence(n: int = 1000, n_pos: int = 20, steps: int = 200,
                  rel: float = 1e-3, decay: float = 0.98, stream: int = 0
                  ) -> Iterator[np.ndarray]:
    """ADMM-like sequence X_0..X_{steps-1}: X_0 = Q diag(lam) Q^T with n_pos
    eigenvalues U[0.5,5] and the rest U[-5,-0.01]; X_{k+1} = X_k + E_k with
    ||E_k||_F = rel * decay^k * ||X_k||_F.  Yields X_k (Fortran order).
    The first item yielded is the Cone of X_0 (for its exact spectrum)."""
    rng = rng_for(2, stream)
    Q = haar_orthogonal(n, rng)
    lam = _permuted(rng, [rng.uniform(0.5, 5.0, n_pos),
                          rng.uniform(-5.0, -0.01, n - n_pos)])
    X = from_spectrum(Q, lam)
    yield Cone(X.copy(order="F"), lam, Q)
    for k in range(1, steps):
        E = sym_perturbation(n, rel * decay ** (k - 1) * np.linalg.norm(X), rng)
        X = np.asfortranarray(X + E)
        yield X


# ---------------------------------------------------------------- config 3 --
def large_cone(n: int = 4000, n_pos: int = 40, n_reflectors: int = 64,
               stream: int = 0):
    """n=4000, Q = product of 64 seeded Householder reflectors, 40 eigenvalues
    10^U[0,2] and 3960 eigenvalues -10^U[-3,2], randomly permuted.
    Returns (X, lam, basis)."""
    rng = rng_for(3, stream)
    vs = np.asfortranarray(rng.standard_normal((n, n_reflectors)))
    lam = _permuted(rng, [10.0 ** rng.uniform(0.0, 2.0, n_pos),
                          -(10.0 ** rng.uniform(-3.0, 2.0, n - n_pos))])
    basis = HouseholderBasis(vs)
    X = basis.sandwich(lam)
    return X, lam, basis


def large_cone_sequence(n: int = 4000, n_pos: int = 40, steps: int = 50,
                        rel: float = 1e-4, n_reflectors: int = 64,
                        stream: int = 0, cumulative: bool = True) -> Iterator[np.ndarray]:
    """Warm-start sequence on the large cone.  cumulative: X_{k+1} = X_k + E_k
    with ||E_k||_F = rel * ||X_k||_F (a random walk); otherwise
    X_k = X_0 + E_k with ||E_k||_F = rel * ||X_0||_F (independent
    perturbations of the same matrix).  First item: (X_0, lam, basis)."""
    X0, lam, basis = large_cone(n, n_pos, n_reflectors, stream)
    yield (X0, lam, basis)
    rng = rng_for(3, 1000 + stream)
    X = X0
    nrm0 = np.linalg.norm(X0)
    for _ in range(1, steps):
        if cumulative:
            X = np.asfortranarray(X + sym_perturbation(n, rel * np.linalg.norm(X), rng))
        else:
            X = np.asfortranarray(X0 + sym_perturbation(n, rel * nrm0, rng))
        yield X


# ---------------------------------------------------------------- config 4 --
def batched_cones(count: int = 512, n_min: int = 16, n_max: int = 256,
                  frac_pos: float = 0.1, stream: int = 0) -> List[Cone]:
    """Independent cones with n_i ~ U{n_min..n_max}, p_i = max(1, round(0.1 n_i))
    eigenvalues U[0.1,10], the rest U[-10,-0.1], Haar bases."""
    rng = rng_for(4, stream)
    ns = rng.integers(n_min, n_max + 1, size=count)
    cones = []
    for n in ns:
        n = int(n)
        p = max(1, int(round(frac_pos * n)))
        cones.append(random_spectrum_matrix(n, p, rng, pos=(0.1, 10.0), neg=(-10.0, -0.1)))
    return cones


# ---------------------------------------------------------------- config 5 --
@dataclass
class SessionSpec:
    sid: int
    n: int
    n_pos: int
    cone: Cone = field(repr=False)


def serving_sessions(count: int = 64, n_min: int = 32, n_max: int = 2048,
                     stream: int = 0, build: bool = True) -> List[SessionSpec]:
    """Sessions with n_s = round(exp U[ln n_min, ln n_max]), positive fraction
    f ~ U[0.01, 0.20], p = max(1, round(f n)), magnitudes 10^U[-3,2] with p
    positive signs, Haar basis."""
    rng = rng_for(5, stream)
    out = []
    for s in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        f = rng.uniform(0.01, 0.20)
        p = max(1, int(round(f * n)))
        mag = 10.0 ** rng.uniform(-3.0, 2.0, n)
        sign = np.concatenate([np.ones(p), -np.ones(n - p)])
        lam = (mag * sign)[rng.permutation(n)]
        cone = Cone(None, lam, None)
        if build:
            Q = haar_orthogonal(n, rng)
            cone = Cone(from_spectrum(Q, lam), lam, Q)
        out.append(SessionSpec(s, n, p, cone))
    return out


def gapped_sessions(count: int = 6, n_min: int = 150, n_max: int = 500, frac_pos: float = 0.05,
                    stream: int = 0) -> List[SessionSpec]:
    """Sessions whose spectra keep a gap under the 1e-3 ||X||_F perturbations
    of session_sequence: p = max(1, round(frac_pos n)) eigenvalues U[1, 10],
    the rest U[-10, -0.1], Haar basis, n log-uniform in [n_min, n_max]."""
    rng = rng_for(5, 50_000 + stream)
    out = []
    for s in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        p = max(1, int(round(frac_pos * n)))
        cone = random_spectrum_matrix(n, p, rng, pos=(1.0, 10.0), neg=(-10.0, -0.1))
        out.append(SessionSpec(s, n, p, cone))
    return out


def poisson_arrivals(rate: float, duration: float, n_sessions: int,
                     stream: int = 0):
    """Poisson arrival times (exponential gaps, mean 1/rate) over [0, duration),
    each tagged with a uniformly random session id.  Returns (t, sid)."""
    rng = rng_for(5, 10_000 + stream)
    n_est = int(rate * duration * 1.2 + 100)
    gaps = rng.exponential(1.0 / rate, size=n_est)
    t = np.cumsum(gaps)
    while t[-1] < duration:
        more = rng.exponential(1.0 / rate, size=n_est)
        t = np.concatenate([t, t[-1] + np.cumsum(more)])
    t = t[t < duration]
    sid = rng.integers(0, n_sessions, size=t.size)
    return t, sid


def session_sequence(spec: SessionSpec, steps: int, rel: float = 1e-3,
                     stream: int = 0) -> Iterator[np.ndarray]:
    """The matrices one serving session submits: X_0 = its cone, then
    X_{k+1} = X_k + E_k with ||E_k||_F = rel * ||X_k||_F."""
    rng = rng_for(5, 20_000 + 1000 * stream + spec.sid)
    X = spec.cone.X
    yield X
    for _ in range(1, steps):
        X = np.asfortranarray(X + sym_perturbation(spec.n, rel * np.linalg.norm(X), rng))
        yield X
