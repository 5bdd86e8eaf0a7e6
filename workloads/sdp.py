"""Seeded synthetic semidefinite programs in standard form

    minimize <C, Y>  subject to  <A_i, Y> = b_i,  Y psd,

standing in for the SDPLIB problems of the paper's §6.1 (max-cut relaxations
`maxG*`/`mcp*` and Lovász theta problems `theta*`), which are not available
here, plus two infeasible instances for §6.2.  Every constraint matrix A_i is
given by its entries in the lower triangle, (con, row, col, val) with
row >= col meaning A_con holds val at (row, col) and (col, row); the supports
of different constraints are disjoint.  Nothing here solves anything.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Tuple

import numpy as np

from .generators import rng_for

__all__ = ["Sdp", "maxcut", "theta", "trace_min", "primal_infeasible", "dual_infeasible",
           "random_graph", "cycle_graph", "complete_graph"]


@dataclass
class Sdp:
    C: np.ndarray      # n x n symmetric cost
    con: np.ndarray    # int32 constraint index of each entry (sorted ascending)
    row: np.ndarray    # int32, row >= col
    col: np.ndarray    # int32
    val: np.ndarray    # float64
    b: np.ndarray      # float64, one per constraint
    name: str = ""

    @property
    def n(self) -> int:
        return self.C.shape[0]

    @property
    def p(self) -> int:
        return int(self.b.size)

    def dense_constraints(self) -> List[np.ndarray]:
        """The A_i as dense symmetric matrices (small problems only)."""
        out = [np.zeros((self.n, self.n)) for _ in range(self.p)]
        for c, r, k, v in zip(self.con, self.row, self.col, self.val):
            out[c][r, k] = v
            out[c][k, r] = v
        return out


def _entries(items: List[Tuple[int, int, int, float]]):
    items = sorted(items, key=lambda t: (t[0], t[2], t[1]))
    con = np.array([t[0] for t in items], dtype=np.int32)
    row = np.array([t[1] for t in items], dtype=np.int32)
    col = np.array([t[2] for t in items], dtype=np.int32)
    val = np.array([t[3] for t in items], dtype=np.float64)
    return con, row, col, val


def random_graph(n: int, prob: float, rng) -> List[Tuple[int, int]]:
    """Erdos-Renyi edges (i > j) with probability prob."""
    U = rng.random((n, n))
    return [(i, j) for i in range(n) for j in range(i) if U[i, j] < prob]


def cycle_graph(n: int) -> List[Tuple[int, int]]:
    return [((i + 1) % n, i) if (i + 1) % n > i else (i, (i + 1) % n) for i in range(n)]


def complete_graph(n: int) -> List[Tuple[int, int]]:
    return [(i, j) for i in range(n) for j in range(i)]


def maxcut(n: int = 200, prob: float = 0.1, weights: bool = True, stream: int = 0,
           edges=None) -> Sdp:
    """Max-cut relaxation (SDPLIB maxG/mcp family): minimize -<L, Y>/4 with
    L the weighted graph Laplacian, subject to diag(Y) = 1."""
    rng = rng_for(6, stream)
    E = edges if edges is not None else random_graph(n, prob, rng)
    L = np.zeros((n, n))
    for (i, j) in E:
        w = rng.uniform(0.5, 1.5) if weights else 1.0
        L[i, j] -= w
        L[j, i] -= w
        L[i, i] += w
        L[j, j] += w
    C = np.asfortranarray(-0.25 * L)
    con, row, col, val = _entries([(i, i, i, 1.0) for i in range(n)])
    return Sdp(C, con, row, col, val, np.ones(n), name=f"maxcut{n}")


def theta(n: int = 100, prob: float = 0.2, stream: int = 0, edges=None) -> Sdp:
    """Lovasz theta (SDPLIB theta family): minimize -<J, Y> subject to
    tr(Y) = 1 and Y_ij = 0 on the edges of the graph."""
    rng = rng_for(7, stream)
    E = edges if edges is not None else random_graph(n, prob, rng)
    items = [(0, i, i, 1.0) for i in range(n)]
    for e, (i, j) in enumerate(sorted(E)):
        items.append((1 + e, max(i, j), min(i, j), 0.5))
    con, row, col, val = _entries(items)
    b = np.zeros(1 + len(E))
    b[0] = 1.0
    return Sdp(np.asfortranarray(-np.ones((n, n))), con, row, col, val, b, name=f"theta{n}")


def trace_min(n: int = 30, stream: int = 0) -> Sdp:
    """minimize <C, Y> subject to tr(Y) = 1 with a seeded symmetric C."""
    rng = rng_for(8, stream)
    G = rng.standard_normal((n, n))
    C = np.asfortranarray(0.5 * (G + G.T))
    con, row, col, val = _entries([(0, i, i, 1.0) for i in range(n)])
    return Sdp(C, con, row, col, val, np.ones(1), name=f"tracemin{n}")


def primal_infeasible(n: int = 12, stream: int = 0) -> Sdp:
    """tr(Y) = -1 with Y psd has no solution."""
    rng = rng_for(9, stream)
    G = rng.standard_normal((n, n))
    con, row, col, val = _entries([(0, i, i, 1.0) for i in range(n)])
    return Sdp(np.asfortranarray(0.5 * (G + G.T)), con, row, col, val, -np.ones(1),
               name=f"pinf{n}")


def dual_infeasible(n: int = 12, stream: int = 0) -> Sdp:
    """minimize -tr(Y) subject to Y_21 = 0: unbounded below (Y = t e_3 e_3^T)."""
    con, row, col, val = _entries([(0, 1, 0, 0.5)])
    return Sdp(np.asfortranarray(-np.eye(n)), con, row, col, val, np.zeros(1), name=f"dinf{n}")
