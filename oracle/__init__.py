"""Oracle for the PSD-cone projection -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU
library and the product path never calls it.

What it computes (paper §1, definition of the projection, eq.
`eigendecomposition` and eq. `projection`): for a symmetric X with full
eigendecomposition X = Q diag(lam) Q^T,

    Pi(X) = argmin_{Y psd} ||X - Y||_F = Q diag(max(lam, 0)) Q^T .

The projection onto the closed convex PSD cone is unique, so the oracle is
that definition written out: an FP64 cyclic Jacobi eigendecomposition in
plain C (``jacobi.c``) followed by clipping.  Every function here takes plain
numpy float64 arrays; the lower triangle of X is what is read.

Pins (checked in ``tests/test_oracle_pins.py`` against things other than the
oracle itself): 2x2 and 3x3 closed forms, diagonal inputs, prescribed-spectrum
construction, the Moreau decomposition X = Pi(X) - Pi(-X) with
<Pi(X), Pi(X) - X> = 0, PSD-ness, idempotence, ||X - Pi(X)||_F^2 = sum of the
squared negative eigenvalues, nonexpansiveness, positive homogeneity,
orthogonal equivariance, LAPACK agreement, and brute-force minimisation on
tiny inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi.c")
_LIB = os.path.join(_HERE, "liboracle_jacobi.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``jacobi.c`` with gcc (-O2, OpenMP) into ``liboracle_jacobi.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
             "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_eigh.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, dp,
                                    ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        lib.oracle_eigh.restype = ctypes.c_int
        lib.oracle_project.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp,
                                       ctypes.c_int, dp]
        lib.oracle_project.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_fortran(X) -> np.ndarray:
    X = np.asarray(X, dtype=np.float64)
    if X.ndim != 2 or X.shape[0] != X.shape[1]:
        raise ValueError("X must be a square matrix")
    return np.asfortranarray(X)


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().oracle_num_threads())


class OracleError(RuntimeError):
    pass


def eigh(X, return_sweeps: bool = False):
    """Full eigendecomposition by cyclic Jacobi (lower triangle of X read).

    Returns (lam ascending, V) with X = V diag(lam) V^T.
    """
    X = _as_fortran(X)
    n = X.shape[0]
    lam = np.empty(n)
    V = np.empty((n, n), order="F")
    sweeps = ctypes.c_int(0)
    rc = _load().oracle_eigh(n, _ptr(X), max(n, 1), _ptr(lam), _ptr(V),
                             max(n, 1), ctypes.byref(sweeps))
    if rc != 0:
        raise OracleError(f"oracle_eigh failed with code {rc}")
    if return_sweeps:
        return lam, V, sweeps.value
    return lam, V


def project(X):
    """Exact PSD projection Pi(X) = V diag(max(lam,0)) V^T and all eigenvalues.

    Paper §1, eq. `projection` (left equality).  Returns (Pi, lam ascending).
    """
    X = _as_fortran(X)
    n = X.shape[0]
    Pi = np.empty((n, n), order="F")
    lam = np.empty(n)
    rc = _load().oracle_project(n, _ptr(X), max(n, 1), _ptr(Pi), max(n, 1),
                                _ptr(lam))
    if rc != 0:
        raise OracleError(f"oracle_project failed with code {rc}")
    return Pi, lam


def symmetrize_lower(X) -> np.ndarray:
    """The symmetric matrix whose lower triangle is that of X (the matrix
    every entry point of the library and the oracle actually projects)."""
    X = np.asarray(X, dtype=np.float64)
    L = np.tril(X)
    return L + np.tril(X, -1).T


def true_error(Pi_hat, Pi) -> float:
    """||Pi_hat - Pi||_F (Frobenius), the quantity Thm `bound` bounds (§5.2)."""
    return float(np.linalg.norm(np.asarray(Pi_hat) - np.asarray(Pi)))


def rel_error(Pi_hat, Pi, X=None) -> float:
    """Relative Frobenius error ||Pi_hat - Pi||_F / ||Pi||_F.

    When Pi = 0 the normaliser is ||X||_F (X given) so that an all-zero
    projection is still measured on the scale of its input.
    """
    d = true_error(Pi_hat, Pi)
    nrm = float(np.linalg.norm(Pi))
    if nrm == 0.0:
        nrm = float(np.linalg.norm(X)) if X is not None else 1.0
        if nrm == 0.0:
            return d
    return d / nrm


def tail_exact(X, Vt) -> float:
    """||Pi(Vt_perp^T X Vt_perp)||_F, the last term of Thm `bound` (§5.2).

    P = I - Vt Vt^T is the orthogonal projector onto the complement of the
    orthonormal columns Vt; P X P has spectrum eig(Vt_perp^T X Vt_perp) plus
    zeros, so ||Pi(P X P)||_F equals the theorem's term without forming
    Vt_perp.
    """
    X = symmetrize_lower(X)
    Vt = np.asarray(Vt, dtype=np.float64)
    n = X.shape[0]
    P = np.eye(n) - Vt @ Vt.T
    M = P @ X @ P
    M = 0.5 * (M + M.T)
    lam, _ = eigh(M)
    pos = lam[lam > 0]
    return float(np.sqrt(np.sum(pos * pos)))


def complement_spectrum(X, Vt) -> np.ndarray:
    """Eigenvalues (ascending) of Vt_perp^T X Vt_perp, the matrix whose
    positive part is the last term of Thm `bound` (§5.2), for orthonormal
    columns Vt (n x m).

    With P = I - Vt Vt^T and s = 2 ||X||_F + 1, the matrix P X P - s Vt Vt^T
    has spectrum eig(Vt_perp^T X Vt_perp) plus m copies of -s (range(Vt) is
    invariant with eigenvalue -s, its complement carries the compression),
    and -s lies below every eigenvalue of the compression; the m smallest
    eigenvalues are dropped.
    """
    X = symmetrize_lower(X)
    Vt = np.asarray(Vt, dtype=np.float64).reshape(X.shape[0], -1)
    n, m = X.shape[0], Vt.shape[1]
    s = 2.0 * float(np.linalg.norm(X)) + 1.0
    P = np.eye(n) - Vt @ Vt.T
    M = P @ X @ P - s * (Vt @ Vt.T)
    M = 0.5 * (M + M.T)
    lam, _ = eigh(M)
    return lam[m:]


def truncated_projection(X, r: int):
    """sum_{i <= r} max(lam_i, 0) v_i v_i^T over the r largest eigenpairs of
    X: the truncated projection the paper's §1 describes for solvers that
    compute a fixed number of leading eigenpairs.  Returns (Pi_r, lam
    descending)."""
    lam, V = eigh(X)
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    r = max(0, min(int(r), lam.size))
    w = np.maximum(lam[:r], 0.0)
    Pi = (V[:, :r] * w) @ V[:, :r].T
    return 0.5 * (Pi + Pi.T), lam


def block_krylov_projection(X, X0, steps: int = 1):
    """Rayleigh-Ritz on the block Krylov space span(X^k, A X^k) (paper §5,
    block Lanczos), restarted `steps` times from X^0 (n x m) keeping the m
    largest Ritz pairs, then the projection from the positive Ritz pairs:
    returns (Pi~, theta descending, Ritz vectors).  The orthonormal basis
    comes from a QR factorisation and the small eigenproblem from
    numpy.linalg.eigh (library primitives)."""
    A = symmetrize_lower(X)
    Xk = np.asarray(X0, dtype=np.float64)
    m = Xk.shape[1]
    theta = np.zeros(0)
    Y = Xk
    for _ in range(max(1, int(steps))):
        S, _ = np.linalg.qr(np.concatenate([Xk, A @ Xk], axis=1))
        H = S.T @ A @ S
        th, W = np.linalg.eigh(0.5 * (H + H.T))
        order = np.argsort(th)[::-1][:m]
        theta, Y = th[order], S @ W[:, order]
        Xk = Y
    pos = theta > 0
    Pi = (Y[:, pos] * theta[pos]) @ Y[:, pos].T
    return 0.5 * (Pi + Pi.T), theta, Y


__all__ = ["build", "eigh", "project", "true_error", "rel_error", "tail_exact",
           "complement_spectrum", "truncated_projection", "block_krylov_projection",
           "symmetrize_lower", "num_threads", "OracleError"]
