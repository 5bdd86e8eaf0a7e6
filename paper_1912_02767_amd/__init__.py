"""Warm-started approximate PSD-cone projection on AMD MI355X (gfx950).

Python binding over the C-ABI of ``include/psdp.h`` (``libpsdp.so``).  This
module only marshals arguments: every step of the projection runs in the HIP
kernels of the library.  PyTorch provides device memory and the stream.

    proj = Projector()
    res = proj.project(X)                  # X: (n, n) float64 CUDA tensor
    res.Pi, res.V, res.lam, res.info

A ``Session`` keeps the Ritz block of one matrix sequence on the device so
that the next projection is warm-started from it (paper §5.1: LOBPCG allows
warm starting; §6: the side is chosen from the previous iterate's inertia).
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

from . import _abi
from ._abi import (PREC_BF16, PREC_FP32, PREC_FP64, PSDP_ERR_CAPACITY,
                   PSDP_ERR_HIP, PSDP_ERR_INVALID_ARG, PSDP_ERR_NUMERICAL,
                   PSDP_ERR_OUT_OF_MEMORY, PSDP_FELL_BACK_FULL_EIG, PSDP_PENDING,
                   PSDP_NOT_CONVERGED, PSDP_OK, SIDE_AUTO, SIDE_FULL, SIDE_NEG,
                   SIDE_POS, LibraryMissing, load, status_str)

__all__ = ["Projector", "Session", "Server", "Result", "ServedResult", "PsdpError", "load",
           "status_str", "fortran", "PREC", "SIDE", "LibraryMissing", "transfer_stats"]

PREC = {"fp64": PREC_FP64, "fp32": PREC_FP32, "bf16": PREC_BF16}
SIDE = {"auto": SIDE_AUTO, "pos": SIDE_POS, "neg": SIDE_NEG, "full": SIDE_FULL}
METHOD = {"lobpcg": _abi.METHOD_LOBPCG, "block_krylov": _abi.METHOD_BLOCK_KRYLOV,
          "top_r": _abi.METHOD_TOP_R, "chebyshev": _abi.METHOD_CHEBYSHEV}


class PsdpError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {status_str(code)} ({code})")
        self.code = code


def _torch():
    import torch
    return torch


def fortran(t):
    """A column-major (Fortran-ordered) view of a 2-D tensor, copying only
    when the tensor is not already column-major."""
    if t.dim() != 2:
        raise ValueError("expected a matrix")
    if t.stride(0) == 1 and t.stride(1) >= max(1, t.shape[0]):
        return t
    return t.t().contiguous().t()


def _empty_f(rows, cols, device, dtype=None):
    torch = _torch()
    dtype = dtype or torch.float64
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


@dataclass
class Result:
    Pi: object          # (n, n) float64, column-major
    V: object           # (n, m_out) Ritz vectors of the approximated side
    lam: object         # (m_out,) Ritz values of the approximated side's matrix
    info: dict
    status: int


def _opts(lib, side="pos", prec="fp64", tol=0.0, max_iter=300, refine=True,
          ladder=True, seed=None, side_threshold=1.0 / 3.0, expand_cols=0,
          pos_hint=-1, fallback_full=False, block_guard=4, bound_rel_max=0.0,
          certify=True, certify_delta=0.0, warm_side="auto", method="lobpcg", method_param=0):
    o = _abi.Options()
    lib.psdp_default_options(ctypes.byref(o))
    o.side = SIDE[side] if isinstance(side, str) else int(side)
    o.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.refine_fp64 = 1 if refine else 0
    o.ladder = 1 if ladder else 0
    if seed is not None:
        o.seed = int(seed) & ((1 << 64) - 1)
    o.side_threshold = float(side_threshold)
    o.expand_cols = int(expand_cols)
    o.pos_hint = int(pos_hint)
    o.fallback_full = 1 if fallback_full else 0
    o.block_guard = int(block_guard)
    o.bound_rel_max = float(bound_rel_max)
    o.certify = 1 if certify else 0
    o.certify_delta = float(certify_delta)
    o.warm_side = SIDE[warm_side] if isinstance(warm_side, str) else int(warm_side)
    o.method = METHOD[method] if isinstance(method, str) else int(method)
    o.method_param = int(method_param)
    return o


class Projector:
    """A library handle bound to one device; calls enqueue on torch's
    current stream of that device."""

    def __init__(self, device: int = 0):
        self.lib = load()
        torch = _torch()
        if not torch.cuda.is_available():
            raise PsdpError(PSDP_ERR_HIP, "Projector: no GPU visible")
        self.device = int(device)
        self._h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        rc = self.lib.psdp_create(ctypes.byref(self._h), self.device, ctypes.c_void_p(stream))
        if rc != PSDP_OK:
            raise PsdpError(rc, "psdp_create")

    # ------------------------------------------------------------ plumbing
    def _sync_stream(self):
        torch = _torch()
        s = torch.cuda.current_stream(self.device).cuda_stream
        self.lib.psdp_set_stream(self._h, ctypes.c_void_p(s))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.lib.psdp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_matrix(self, X):
        torch = _torch()
        if X.dtype != torch.float64 or X.device.type != "cuda":
            raise TypeError("X must be a float64 CUDA tensor")
        if X.dim() != 2 or X.shape[0] != X.shape[1] or X.shape[0] < 1:
            raise ValueError("X must be a non-empty square matrix")
        return fortran(X)

    # ------------------------------------------------------------ calls
    def project(self, X, V=None, m_cap: Optional[int] = None, side="pos", prec="fp64",
                tol: float = 0.0, max_iter: int = 300, refine: bool = True, ladder: bool = True,
                seed=None, pos_hint: int = -1, expand_cols: int = 0, fallback_full: bool = False,
                side_threshold: float = 1.0 / 3.0, block_guard: int = 4, V_buf=None,
                Pi_out=None, lam_buf=None, raise_on_error: bool = True,
                bound_rel_max: float = 0.0, certify: bool = True, certify_delta: float = 0.0,
                warm_side="auto", method="lobpcg", method_param: int = 0) -> Result:
        """Pi(X) with LOBPCG on one spectral side (psdp_project).

        V: optional warm start (n x k).  V_buf: optional column-major
        (n x m_cap) device buffer reused in place (no copy of the block)."""
        torch = _torch()
        Xf = self._check_matrix(X)
        n = Xf.shape[0]
        self._sync_stream()
        if V_buf is None:
            k = 0 if V is None else V.shape[1]
            cap = int(m_cap or max(k, 64))
            cap = max(cap, k, 1)
            V_buf = _empty_f(n, cap, Xf.device)
            if k:
                V_buf[:, :k].copy_(V)
        else:
            k = 0 if V is None else int(V)
            cap = V_buf.shape[1]
            if V_buf.stride(0) != 1:
                raise ValueError("V_buf must be column-major")
        if lam_buf is None or lam_buf.numel() < cap:
            lam_buf = torch.empty(cap, dtype=torch.float64, device=Xf.device)
        Pi = Pi_out if Pi_out is not None else _empty_f(n, n, Xf.device)
        m_io = ctypes.c_int(k)
        opt = _opts(self.lib, side, prec, tol, max_iter, refine, ladder, seed, side_threshold,
                    expand_cols, pos_hint, fallback_full, block_guard, bound_rel_max, certify,
                    certify_delta, warm_side, method, method_param)
        info = _abi.Info()
        rc = self.lib.psdp_project(self._h, n, ctypes.c_void_p(Xf.data_ptr()), Xf.stride(1),
                                   ctypes.c_void_p(V_buf.data_ptr()), V_buf.stride(1), cap,
                                   ctypes.byref(m_io), ctypes.c_void_p(lam_buf.data_ptr()),
                                   ctypes.c_void_p(Pi.data_ptr()), Pi.stride(1),
                                   ctypes.byref(opt), ctypes.byref(info))
        if rc < 0 and raise_on_error:
            raise PsdpError(rc, "psdp_project")
        mo = m_io.value
        return Result(Pi, V_buf[:, :mo], lam_buf[:mo], info.as_dict(), rc)

    def full_eig(self, X, Pi_out=None, lam_out=None):
        """Exact Pi(X) via the FP64 full eigendecomposition (psdp_full_eig_project)."""
        torch = _torch()
        Xf = self._check_matrix(X)
        n = Xf.shape[0]
        self._sync_stream()
        Pi = Pi_out if Pi_out is not None else _empty_f(n, n, Xf.device)
        lam = lam_out if lam_out is not None else torch.empty(n, dtype=torch.float64, device=Xf.device)
        rc = self.lib.psdp_full_eig_project(self._h, n, ctypes.c_void_p(Xf.data_ptr()), Xf.stride(1),
                                            ctypes.c_void_p(lam.data_ptr()),
                                            ctypes.c_void_p(Pi.data_ptr()), Pi.stride(1))
        if rc < 0:
            raise PsdpError(rc, "psdp_full_eig_project")
        return Pi, lam

    def project_batched(self, Xs: Sequence, m_caps=None, Vs=None, prec="fp32", tol: float = 0.0,
                        max_iter: int = 300, seed=None, side="pos", variant: int = -1,
                        graph: bool = True, V_bufs=None, Pi_outs=None,
                        expand_cols: int = 0, fallback_full: bool = False) -> List[Result]:
        """Many uneven cones (n <= 256) in one persistent launch
        (psdp_project_batched).  m_caps[i] bounds cone i's block (at most 32)
        and is its cold-start width; Vs[i] (n x k, or None) warm-starts it."""
        torch = _torch()
        count = len(Xs)
        Xf = [self._check_matrix(x) for x in Xs]
        ns = [x.shape[0] for x in Xf]
        for x in Xf:
            if x.stride(1) != x.shape[0]:
                raise ValueError("batched cones need leading dimension n")
        self._sync_stream()
        caps = list(m_caps) if m_caps is not None else [min(32, max(1, n)) for n in ns]
        if V_bufs is None:
            V_bufs = [_empty_f(n, c, x.device) for n, c, x in zip(ns, caps, Xf)]
        m_in = [0] * count
        if Vs is not None:
            for i, v in enumerate(Vs):
                if v is not None and v.shape[1] > 0:
                    if V_bufs[i].data_ptr() != v.data_ptr():
                        V_bufs[i][:, :v.shape[1]].copy_(v)
                    m_in[i] = v.shape[1]
        lams = [torch.empty(c, dtype=torch.float64, device=x.device) for c, x in zip(caps, Xf)]
        Pis = Pi_outs if Pi_outs is not None else [_empty_f(n, n, x.device) for n, x in zip(ns, Xf)]
        IA = ctypes.c_int * count
        PA = ctypes.c_void_p * count
        n_arr = IA(*ns)
        cap_arr = IA(*caps)
        mio = IA(*m_in)
        X_arr = PA(*[x.data_ptr() for x in Xf])
        V_arr = PA(*[v.data_ptr() for v in V_bufs])
        L_arr = PA(*[l.data_ptr() for l in lams])
        P_arr = PA(*[p.data_ptr() for p in Pis])
        opt = _opts(self.lib, side, prec, tol, max_iter, True, True, seed, expand_cols=expand_cols,
                    fallback_full=fallback_full)
        opt.batch_variant = int(variant)
        opt.batch_graph = 1 if graph else 0
        infos = (_abi.Info * max(count, 1))()
        rc = self.lib.psdp_project_batched(self._h, count, n_arr, X_arr, V_arr, cap_arr, mio,
                                           L_arr, P_arr, ctypes.byref(opt), infos)
        if rc < 0 and rc != PSDP_ERR_NUMERICAL:
            raise PsdpError(rc, "psdp_project_batched")
        out = []
        for i in range(count):
            mo = mio[i]
            out.append(Result(Pis[i], V_bufs[i][:, :mo], lams[i][:mo], infos[i].as_dict(),
                              infos[i].status))
        return out

    def block_product(self, X, S, prec="fp64", Y_out=None):
        """Y = sym(X) S with the product kernel alone (psdp_block_product)."""
        torch = _torch()
        Xf = self._check_matrix(X)
        n = Xf.shape[0]
        Sf = fortran(S)
        k = Sf.shape[1]
        self._sync_stream()
        Y = Y_out if Y_out is not None else _empty_f(n, k, Xf.device)
        rc = self.lib.psdp_block_product(self._h, n, ctypes.c_void_p(Xf.data_ptr()), Xf.stride(1),
                                         ctypes.c_void_p(Sf.data_ptr()), Sf.stride(1), k,
                                         PREC[prec] if isinstance(prec, str) else int(prec),
                                         ctypes.c_void_p(Y.data_ptr()), Y.stride(1))
        if rc < 0:
            raise PsdpError(rc, "psdp_block_product")
        return Y

    def certify_tail(self, X, V, delta: float):
        """(certified, delta_eff, eta) of the tail certificate alone
        (psdp_certify_tail): every eigenvalue of V_perp^T sym(X) V_perp is
        below delta_eff when certified."""
        Xf = self._check_matrix(X)
        n = Xf.shape[0]
        self._sync_stream()
        m = 0 if V is None else V.shape[1]
        Vf = fortran(V) if m else None
        ok = ctypes.c_int(0)
        de, eta = ctypes.c_double(), ctypes.c_double()
        rc = self.lib.psdp_certify_tail(self._h, n, ctypes.c_void_p(Xf.data_ptr()), Xf.stride(1),
                                        ctypes.c_void_p(Vf.data_ptr() if m else 0),
                                        Vf.stride(1) if m else n, m, float(delta),
                                        ctypes.byref(ok), ctypes.byref(de), ctypes.byref(eta))
        if rc < 0:
            raise PsdpError(rc, "psdp_certify_tail")
        return bool(ok.value), de.value, eta.value

    def admm_solve(self, sdp, exact: bool = False, **opts):
        """Approximate ADMM (psdp_admm_solve) on a standard-form SDP given as
        host arrays: sdp.C (n x n), sdp.con/row/col/val (constraint entries,
        lower triangle), sdp.b.  Keyword options are the fields of
        psdp_admm_options.  Returns (Y, y, W, info)."""
        import numpy as np
        torch = _torch()
        self._sync_stream()
        dev = torch.device("cuda", self.device)
        n = int(sdp.C.shape[0])
        C = torch.from_numpy(np.asfortranarray(sdp.C, dtype=np.float64)).to(dev)
        con = np.ascontiguousarray(sdp.con, dtype=np.int32)
        row = np.ascontiguousarray(sdp.row, dtype=np.int32)
        col = np.ascontiguousarray(sdp.col, dtype=np.int32)
        val = np.ascontiguousarray(sdp.val, dtype=np.float64)
        b = np.ascontiguousarray(sdp.b, dtype=np.float64)
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        pr = _abi.Sdp(n, int(b.size), ctypes.c_void_p(C.data_ptr()), C.stride(1), int(val.size),
                      con.ctypes.data_as(ip), row.ctypes.data_as(ip), col.ctypes.data_as(ip),
                      val.ctypes.data_as(dp), b.ctypes.data_as(dp))
        o = _abi.AdmmOptions()
        self.lib.psdp_admm_default_options(ctypes.byref(o))
        o.exact = 1 if exact else 0
        for k, v in opts.items():
            if k == "prec" and isinstance(v, str):
                v = PREC[v]
            if k == "method" and isinstance(v, str):
                v = METHOD[v]
            setattr(o, k, v)
        Y = _empty_f(n, n, dev)
        W = _empty_f(n, n, dev)
        y = torch.empty(max(int(b.size), 1), dtype=torch.float64, device=dev)
        info = _abi.AdmmInfo()
        rc = self.lib.psdp_admm_solve(self._h, ctypes.byref(pr), ctypes.byref(o),
                                      ctypes.c_void_p(Y.data_ptr()), Y.stride(1),
                                      ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(W.data_ptr()),
                                      W.stride(1), ctypes.byref(info))
        if rc < 0:
            raise PsdpError(rc, "psdp_admm_solve")
        return Y, y[:int(b.size)], W, info.as_dict()

    # ------------------------------------------------------------ profiling
    def profile_enable(self, on: bool = True):
        self.lib.psdp_profile_enable(self._h, 1 if on else 0)

    def profile_filter(self, families: str = ""):
        """Time only these comma-separated kernel families ("" = all)."""
        self.lib.psdp_profile_filter(self._h, families.encode())

    def full_eig_batched(self, Xs: Sequence, m_caps=None, V_bufs=None, Pi_outs=None):
        """Exact projections of many small cones (n <= 256) in zero-padded
        buckets (psdp_full_eig_project_batched).  With m_caps, also the
        leading eigenpairs (positive + guard columns) per cone."""
        torch = _torch()
        count = len(Xs)
        Xf = [self._check_matrix(x) for x in Xs]
        ns = [x.shape[0] for x in Xf]
        for x in Xf:
            if x.stride(1) != x.shape[0]:
                raise ValueError("batched cones need leading dimension n")
        self._sync_stream()
        Pis = Pi_outs if Pi_outs is not None else [_empty_f(n, n, x.device) for n, x in zip(ns, Xf)]
        IA = ctypes.c_int * max(count, 1)
        PA = ctypes.c_void_p * max(count, 1)
        infos = (_abi.Info * max(count, 1))()
        lams = None
        if m_caps is not None:
            if V_bufs is None:
                V_bufs = [_empty_f(n, c, x.device) for n, c, x in zip(ns, m_caps, Xf)]
            lams = [torch.empty(c, dtype=torch.float64, device=x.device) for c, x in zip(m_caps, Xf)]
            mio = IA(*([0] * count))
            rc = self.lib.psdp_full_eig_project_batched(
                self._h, count, IA(*ns), PA(*[x.data_ptr() for x in Xf]),
                PA(*[v.data_ptr() for v in V_bufs]), IA(*m_caps), mio,
                PA(*[l.data_ptr() for l in lams]), PA(*[p.data_ptr() for p in Pis]), infos)
        else:
            mio = IA(*([0] * count))
            rc = self.lib.psdp_full_eig_project_batched(
                self._h, count, IA(*ns), PA(*[x.data_ptr() for x in Xf]), None, None, None, None,
                PA(*[p.data_ptr() for p in Pis]), infos)
        if rc < 0 and rc != PSDP_ERR_NUMERICAL:
            raise PsdpError(rc, "psdp_full_eig_project_batched")
        out = []
        for i in range(count):
            mo = mio[i] if m_caps is not None else 0
            V = V_bufs[i][:, :mo] if m_caps is not None else None
            lam = lams[i][:mo] if lams is not None else None
            out.append(Result(Pis[i], V, lam, infos[i].as_dict(), infos[i].status))
        return out

    def batched_tuning(self):
        """(launch shape, kernel ms) of the last project_batched call."""
        v = ctypes.c_int(-1)
        ms = ctypes.c_double(0.0)
        self.lib.psdp_batched_tuning(self._h, ctypes.byref(v), ctypes.byref(ms))
        return v.value, ms.value

    def profile_get(self, family: str):
        n = ctypes.c_long()
        ms, by, fl = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self.lib.psdp_profile_get(self._h, family.encode(), ctypes.byref(n), ctypes.byref(ms),
                                  ctypes.byref(by), ctypes.byref(fl))
        return {"launches": n.value, "ms": ms.value, "bytes": by.value, "flops": fl.value}


class Session:
    """Warm-start memory of one matrix sequence (one PSD variable of an ADMM
    solve): the Ritz block stays on the device between calls (paper §5.1:
    LOBPCG allows warm starting).  The side is chosen by the library's AUTO
    rule (paper §6) from the previous call's inertia estimate; this class
    only carries the library's own outputs (info.pos_est, info.block_side)
    into the next call."""

    def __init__(self, projector: Projector, n: int, m_cap: int = 64, prec="fp64",
                 tol: float = 0.0, side="auto", pos_hint: int = -1, **kw):
        torch = _torch()
        self.p = projector
        self.n = n
        self.m_cap = m_cap
        self.prec = prec
        self.tol = tol
        self.side_mode = side
        self.kw = kw
        self.V_buf = _empty_f(n, m_cap, torch.device("cuda", projector.device))
        self.lam_buf = torch.empty(m_cap, dtype=torch.float64, device=self.V_buf.device)
        self.m = 0
        self.block_side = SIDE_AUTO
        self.pos_hint = pos_hint
        self.calls = 0

    def project(self, X, Pi_out=None) -> Result:
        res = self.p.project(X, V=self.m, side=self.side_mode, prec=self.prec, tol=self.tol,
                             pos_hint=self.pos_hint, V_buf=self.V_buf, lam_buf=self.lam_buf,
                             Pi_out=Pi_out, warm_side=self.block_side, **self.kw)
        info = res.info
        if res.status >= 0:
            self.m = info["m_out"]
            self.block_side = info["block_side"]
            self.pos_hint = info["pos_est"]
        self.calls += 1
        return res


def transfer_stats(reset: bool = False) -> dict:
    """Device-to-host copies made by the library (psdp_transfer_stats)."""
    lib = load()
    c, b, m = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong()
    lib.psdp_transfer_stats(ctypes.byref(c), ctypes.byref(b), ctypes.byref(m), 1 if reset else 0)
    return {"copies": c.value, "bytes": b.value, "max_bytes": m.value}


@dataclass
class ServedResult:
    Pi: object          # (n, n) float64 projection written by the server
    info: dict
    status: int
    session: int
    lane: int           # 0 single-cone worker, 1 batching lane
    batch_size: int
    queue_ms: float
    latency_ms: float


class Server:
    """Request loop over many sessions (psdp_server_*): device-resident
    warm-start blocks, admission by device-memory footprint, worker streams
    and a batching lane for small requests (continuous batching)."""

    def __init__(self, device: int = 0, slots: int = 4, hbm_budget: int = 0,
                 batch_lane: bool = True, small_n: int = 256, max_batch: int = 512,
                 prec="fp32", tol: float = 0.0, max_iter: int = 300, seed=None,
                 block_guard: int = 4, method="lobpcg"):
        self.lib = load()
        torch = _torch()
        if not torch.cuda.is_available():
            raise PsdpError(PSDP_ERR_HIP, "Server: no GPU visible")
        self.device = int(device)
        cfg = _abi.ServerConfig()
        self.lib.psdp_server_default_config(ctypes.byref(cfg))
        cfg.slots = int(slots)
        cfg.hbm_budget = int(hbm_budget)
        cfg.batch_lane = 1 if batch_lane else 0
        cfg.small_n = int(small_n)
        cfg.max_batch = int(max_batch)
        cfg.opt = _opts(self.lib, "auto", prec, tol, max_iter, True, True, seed,
                        block_guard=block_guard, method=method)
        self._s = ctypes.c_void_p()
        rc = self.lib.psdp_server_create(ctypes.byref(self._s), self.device, ctypes.byref(cfg))
        if rc != 0:
            raise PsdpError(rc, "psdp_server_create")
        self._live = {}     # ticket -> (X, Pi) kept alive until the result is read
        self._n = {}

    def open_session(self, n: int, m_cap: int = 48, pos_hint: int = -1) -> int:
        sid = ctypes.c_int()
        rc = self.lib.psdp_server_open_session(self._s, int(n), int(m_cap), int(pos_hint),
                                               ctypes.byref(sid))
        if rc != 0:
            raise PsdpError(rc, "psdp_server_open_session")
        self._n[sid.value] = int(n)
        return sid.value

    def close_session(self, sid: int) -> int:
        return self.lib.psdp_server_close_session(self._s, int(sid))

    def submit(self, sid: int, X, Pi_out=None) -> int:
        torch = _torch()
        n = self._n[sid]
        Xf = fortran(X)
        if Xf.shape != (n, n) or Xf.dtype != torch.float64 or Xf.stride(1) != n:
            raise ValueError("X must be a float64 (n, n) matrix with leading dimension n")
        Pi = Pi_out if Pi_out is not None else _empty_f(n, n, Xf.device)
        t = ctypes.c_longlong()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        rc = self.lib.psdp_server_submit(self._s, int(sid), ctypes.c_void_p(Xf.data_ptr()),
                                         ctypes.c_void_p(Pi.data_ptr()), ctypes.c_void_p(stream),
                                         ctypes.byref(t))
        if rc != 0:
            raise PsdpError(rc, "psdp_server_submit")
        self._live[t.value] = (Xf, Pi)
        return t.value

    def wait(self, ticket: int, timeout_ms: float = -1.0) -> Optional[ServedResult]:
        r = _abi.ServerResult()
        rc = self.lib.psdp_server_wait(self._s, int(ticket), float(timeout_ms), ctypes.byref(r))
        if rc == PSDP_PENDING:
            return None
        if rc != 0:
            raise PsdpError(rc, "psdp_server_wait")
        _, Pi = self._live.pop(ticket)
        return ServedResult(Pi, r.info.as_dict(), r.info.status, r.session, r.lane, r.batch_size,
                            r.queue_ms, r.latency_ms)

    def drain(self):
        self.lib.psdp_server_drain(self._s)

    def session_block(self, sid: int):
        """(V, lam) copies of a session's warm-start block."""
        torch = _torch()
        n = self._n[sid]
        m = ctypes.c_int()
        rc = self.lib.psdp_server_session_block(self._s, int(sid), None, n, None, ctypes.byref(m))
        if rc != 0:
            raise PsdpError(rc, "psdp_server_session_block")
        V = _empty_f(n, max(m.value, 1), torch.device("cuda", self.device))
        lam = torch.empty(max(m.value, 1), dtype=torch.float64, device=V.device)
        rc = self.lib.psdp_server_session_block(self._s, int(sid), ctypes.c_void_p(V.data_ptr()), n,
                                                ctypes.c_void_p(lam.data_ptr()), ctypes.byref(m))
        if rc != 0:
            raise PsdpError(rc, "psdp_server_session_block")
        return V[:, :m.value], lam[:m.value]

    def stats(self) -> dict:
        st = _abi.ServerStats()
        self.lib.psdp_server_stats_get(self._s, ctypes.byref(st))
        return st.as_dict()

    def stats_reset(self):
        self.lib.psdp_server_stats_reset(self._s)

    def close(self):
        if self._s:
            self.lib.psdp_server_destroy(self._s)
            self._s = ctypes.c_void_p()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
