"""Approximate ADMM (paper §2, Alg. 1) for standard-form SDPs -- TEST
INFRASTRUCTURE ONLY.

Only ``tests/`` and ``bench.py``'s ``cpu_baseline`` leg may import this
module; it shares no code with the GPU library.

Problem (paper §2, problem (P)) for a semidefinite program in standard form

    minimize <C, Y>  subject to  <A_i, Y> = b_i (i = 1..p),  Y psd :

x = svec(Y) (the symmetric vectorisation with sqrt(2) off the diagonal, so
that x^T y = <X, Y>_F), P = 0, q = svec(C), and the constraint map
A x = (<A_i, Y>)_i stacked over x itself, with the cone C = {b} x svec(S_+).

Each iteration follows Alg. 1 in its order and notation: the linear system
of its first line is formed as the (d + m) x (d + m) matrix
[[P + sigma I, rho A^T], [rho A, -rho I]] and solved exactly (a dense LU,
refactored never: the matrix does not change), then the relaxed x update,
the projection onto C (the {b} part is b itself; the PSD part is the exact
projection of ``oracle.project`` or any supplied projector) and the dual
update.  Termination uses the primal and dual residuals of (P); the
infeasibility tests are those of §6.2 on the successive differences
dx = x^{k+1} - x^k and dy = y^{k+1} - y^k.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg

from . import project as _exact_project


def svec(Y: np.ndarray) -> np.ndarray:
    """Lower triangle of symmetric Y, column by column, off-diagonal entries
    times sqrt(2): svec(X)^T svec(Y) = <X, Y>_F."""
    Y = np.asarray(Y, dtype=np.float64)
    n = Y.shape[0]
    out = []
    for j in range(n):
        out.append(Y[j, j])
        for i in range(j + 1, n):
            out.append(math.sqrt(2.0) * Y[i, j])
    return np.array(out)


def smat(x: np.ndarray, n: int) -> np.ndarray:
    """Inverse of svec."""
    Y = np.zeros((n, n))
    k = 0
    for j in range(n):
        Y[j, j] = x[k]
        k += 1
        for i in range(j + 1, n):
            Y[i, j] = Y[j, i] = x[k] / math.sqrt(2.0)
            k += 1
    return Y


@dataclass
class AdmmResult:
    status: str                 # "solved", "max_iter", "primal_infeasible", "dual_infeasible"
    iters: int
    Y: np.ndarray               # primal matrix smat(x)
    y: np.ndarray               # multiplier of the equality block (length p)
    W: np.ndarray               # multiplier of the PSD block (matrix)
    obj: float                  # <C, Y>
    r_prim: float
    r_dual: float
    history: List[tuple] = field(default_factory=list)


def admm(C, A_list, b, rho=0.1, sigma=1e-6, alpha=1.6, max_iter=5000, eps_abs=1e-7,
         eps_rel=1e-7, eps_inf=1e-6, check_every=1, proj: Optional[Callable] = None,
         record: int = 0, Y0=None) -> AdmmResult:
    """Alg. 1 on min <C, Y> s.t. <A_i, Y> = b_i, Y psd.

    proj(V) -> Pi_{S+}(V) for a symmetric matrix V (default: the exact
    oracle projection).  record > 0 keeps (Y, y, W) of the first `record`
    iterations in ``history`` for iterate-by-iterate comparisons."""
    C = np.asarray(C, dtype=np.float64)
    n = C.shape[0]
    p = len(A_list)
    b = np.asarray(b, dtype=np.float64).reshape(p)
    proj = proj or (lambda V: _exact_project(np.asfortranarray(V))[0])
    d = n * (n + 1) // 2
    Aeq = np.array([svec(Ai) for Ai in A_list]).reshape(p, d)
    A = np.vstack([Aeq, np.eye(d)])            # m x d, m = p + d
    m = p + d
    q = svec(C)
    K = np.block([[sigma * np.eye(d), rho * A.T],
                  [rho * A, -rho * np.eye(m)]])
    lu = scipy.linalg.lu_factor(K)

    def proj_C(v):
        z = np.empty(m)
        z[:p] = b                               # the translated zero cone {b}
        z[p:] = svec(proj(smat(v[p:], n)))      # the PSD cone
        return z

    x = svec(Y0) if Y0 is not None else np.zeros(d)
    z = proj_C(A @ x)
    y = np.zeros(m)
    hist = []
    status, k = "max_iter", 0
    r_prim = r_dual = math.inf
    for k in range(1, max_iter + 1):
        rhs = np.concatenate([sigma * x - q + rho * A.T @ (z - y / rho), np.zeros(m)])
        sol = scipy.linalg.lu_solve(lu, rhs)
        xt, zt = sol[:d], sol[d:]
        x_new = alpha * xt + (1 - alpha) * x
        z_new = proj_C(alpha * zt + (1 - alpha) * z + y / rho)
        y_new = y + rho * (alpha * zt + (1 - alpha) * z - z_new)
        dx, dy = x_new - x, y_new - y
        x, z, y = x_new, z_new, y_new
        if record and k <= record:
            hist.append((smat(x, n), y[:p].copy(), smat(y[p:], n)))
        if k % check_every:
            continue
        Ax = A @ x
        Aty = A.T @ y
        r_prim = float(np.linalg.norm(Ax - z))
        r_dual = float(np.linalg.norm(q + Aty))
        if (r_prim <= eps_abs + eps_rel * max(np.linalg.norm(Ax), np.linalg.norm(z)) and
                r_dual <= eps_abs + eps_rel * max(np.linalg.norm(q), np.linalg.norm(Aty))):
            status = "solved"
            break
        inf = infeasibility(dx, dy, A, q, b, n, p, eps_inf)
        if inf:
            status = inf
            break
    return AdmmResult(status, k, smat(x, n), y[:p].copy(), smat(y[p:], n), float(q @ x),
                      r_prim, r_dual, hist)


def infeasibility(dx, dy, A, q, b, n, p, eps):
    """The approximate certificates of §6.2 on the successive differences.

    Dual infeasibility (the objective is unbounded below): xb = dx/||dx||
    with A_eq xb ~ 0, xb in the recession cone svec(S_+) (distance below
    eps), and q^T xb < -eps.  Primal infeasibility: yb = dy/||dy|| with
    A^T yb ~ 0 and support function sigma_C(yb) = b^T yb_eq + sup_{Z psd}
    <Yb_psd, Z> < 0, i.e. Yb_psd negative semidefinite (distance to S_- below
    eps) and b^T yb_eq < -eps."""
    ndx, ndy = float(np.linalg.norm(dx)), float(np.linalg.norm(dy))
    if ndx > 0:
        xb = dx / ndx
        Xb = smat(xb, n)
        dist_psd = float(np.linalg.norm(Xb - _exact_project(np.asfortranarray(Xb))[0]))
        if (np.linalg.norm(A[:p] @ xb) <= eps and dist_psd <= eps and q @ xb <= -eps):
            return "dual_infeasible"
    if ndy > 0:
        yb = dy / ndy
        Wb = smat(yb[p:], n)
        dist_nsd = float(np.linalg.norm(_exact_project(np.asfortranarray(Wb))[0]))
        if (np.linalg.norm(A.T @ yb) <= eps and dist_nsd <= eps and b @ yb[:p] <= -eps):
            return "primal_infeasible"
    return None


__all__ = ["svec", "smat", "admm", "infeasibility", "AdmmResult"]
