#!/usr/bin/env python3
"""Benchmark: warm-started PSD projections/s on one MI355X, against the on-GPU
full eigendecomposition path at relative Frobenius error <= 1e-6.

Default workload (one step = one warm-started projection of the next matrix):
  n1000_warm_seq  n = 1000, X_0 = Q diag(lam) Q^T with 20 eigenvalues in
                  [0.5, 5] and 980 in [-5, -0.01], X_{k+1} = X_k + E_k with
                  ||E_k||_F = 1e-3 * 0.98^k * ||X_k||_F, 200 matrices, block 24,
                  tolerance 1e-8, FP64 products.
  --workload n4000_mixed: n = 4000, Householder basis, 40 positive
                  eigenvalues, 50 warm-started steps at 1e-4 ||X||_F,
                  FP32 (or --prec bf16) products, FP64 ortho/RR/refinement.

Prints ONE JSON line (rank 0).  Inputs are generated on the host (seeded) and
uploaded before the timed region.  The cpu_baseline leg times the FP64 Jacobi
oracle on a bounded sample of the same matrices.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAKS = {  # MI355X published dense peaks
    "fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "hbm": 8.0e12,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(workload, steps_total):
    from workloads import large_cone_sequence, warm_sequence
    if workload == "n1000_warm_seq":
        seq = warm_sequence(n=1000, n_pos=20, steps=steps_total)
        c0 = next(seq)
        return 1000, 20, [c0.X] + list(seq), {"Pi0": c0.sandwich(np.maximum(c0.lam, 0))}
    seq = large_cone_sequence(n=4000, n_pos=40, steps=steps_total)
    X0, lam, basis = next(seq)
    mats = [X0]
    for X in seq:
        mats.append(X)
    return 4000, 40, mats, {"Pi0": basis.sandwich(np.maximum(lam, 0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="n1000_warm_seq",
                    choices=["n1000_warm_seq", "n4000_mixed"])
    ap.add_argument("--prec", default=None, choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--full-eig-samples", type=int, default=None)
    ap.add_argument("--oracle-samples", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build measures one GPU only (the projection of one cone "
              "runs on one device); --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1912_02767_amd as psdp

    wl = args.workload
    big = wl == "n4000_mixed"
    total = 50 if big else 200
    warm = max(0, args.warmup)
    steps = args.steps if args.steps is not None else total - warm
    steps = max(1, min(steps, total - warm))
    prec = args.prec or ("fp32" if big else "fp64")
    t_gen = time.time()
    n, p, mats, extra = make_inputs(wl, warm + steps)
    log(f"generated {len(mats)} matrices n={n} in {time.time() - t_gen:.1f}s")
    dev = torch.device("cuda", 0)
    Xs = [torch.from_numpy(np.asfortranarray(X)).to(dev) for X in mats]
    torch.cuda.synchronize()
    nrm_pi0 = float(np.linalg.norm(extra["Pi0"]))
    if big:
        tol = 1e-7 * nrm_pi0 / math.sqrt(2 * p)   # sqrt(2 m~) tol <= 1e-7 ||Pi||
        m_cap, block = 56, 48
    else:
        tol, m_cap, block = 1e-8, 24, 24

    proj = psdp.Projector(0)
    sess = psdp.Session(proj, n, m_cap=m_cap, tol=tol, side="pos", pos_hint=p, prec=prec,
                        block_guard=block - p)
    Pis = [psdp._empty_f(n, n, dev) for _ in range(2)]

    # ---- warmup (untimed): the first matrices of the sequence
    for k in range(warm):
        sess.project(Xs[k], Pi_out=Pis[k % 2])
    torch.cuda.synchronize()

    # ---- timed region: K warm-started projections
    proj.profile_enable(True)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    infos = []
    keep = {}
    sample_at = {warm, warm + steps // 2, warm + steps - 1}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        k = warm + i
        ev[i][0].record(stream)
        res = sess.project(Xs[k], Pi_out=Pis[i % 2])
        ev[i][1].record(stream)
        infos.append(res.info)
        if k in sample_at:
            keep[k] = res.Pi.clone()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])  # ms
    fams = {f: proj.profile_get(f) for f in
            ["product", "gram", "tsmm", "chol", "rr", "rebuild", "ingest"]}
    proj.profile_enable(False)
    value = steps / wall
    iters = np.array([inf["iters"] for inf in infos])
    statuses = [inf["status"] for inf in infos]

    # ---- on-GPU full eigendecomposition on the same matrices
    n_fe = args.full_eig_samples if args.full_eig_samples is not None else (3 if big else 10)
    fe_idx = [warm + int(i * max(1, steps - 1) / max(1, n_fe - 1)) for i in range(n_fe)] if n_fe else []
    fe_idx = sorted(set(min(k, warm + steps - 1) for k in fe_idx) | set(keep))
    fe_Pi = {}
    proj.full_eig(Xs[fe_idx[0]])  # warm the solver
    torch.cuda.synchronize()
    t_fe = 0.0
    for k in fe_idx:
        torch.cuda.synchronize()
        t = time.perf_counter()
        Pi_f, _ = proj.full_eig(Xs[k])
        torch.cuda.synchronize()
        t_fe += time.perf_counter() - t
        if k in keep:
            fe_Pi[k] = Pi_f.clone()
    fe_rate = len(fe_idx) / t_fe
    rel_vs_fe = {k: float(torch.linalg.norm(keep[k] - fe_Pi[k]) / torch.linalg.norm(fe_Pi[k]))
                 for k in keep}

    # ---- dominant kernel roofline (algorithmic bytes/flops / measured time)
    dom = max(fams, key=lambda f: fams[f]["ms"])
    fd = fams[dom]
    avg_ms = fd["ms"] / max(1, fd["launches"])
    flops_l = fd["flops"] / max(1, fd["launches"])
    bytes_l = fd["bytes"] / max(1, fd["launches"])
    if dom == "product":
        pk = PEAKS[prec]
        ridge = pk / PEAKS["hbm"]
        ai = flops_l / max(bytes_l, 1.0)
        if ai >= ridge:
            roof = {"bound": "mfma", "achieved": flops_l / (avg_ms * 1e-3) / 1e12, "peak": pk / 1e12,
                    "unit": "TFLOP/s"}
        else:
            roof = {"bound": "hbm", "achieved": bytes_l / (avg_ms * 1e-3) / 1e9,
                    "peak": PEAKS["hbm"] / 1e9, "unit": "GB/s"}
    elif dom in ("gram", "tsmm", "rebuild", "ingest"):
        roof = {"bound": "hbm", "achieved": bytes_l / (avg_ms * 1e-3) / 1e9,
                "peak": PEAKS["hbm"] / 1e9, "unit": "GB/s"}
    else:  # one-workgroup FP64 small-matrix kernels: plain vector ALU
        roof = {"bound": "alu", "achieved": flops_l / (avg_ms * 1e-3) / 1e12,
                "peak": PEAKS["fp64"] / 1e12, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = dom
    roof["avg_launch_ms"] = avg_ms

    # ---- CPU oracle on a bounded sample of the same matrices
    cpu = None
    rel_oracle = {}
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        n_or = args.oracle_samples if args.oracle_samples is not None else (0 if big else 3)
        ks = sorted(keep)[:n_or] if n_or else []
        if ks:
            t = time.perf_counter()
            for k in ks:
                Pi_ref, _ = oracle.project(mats[k])
                rel_oracle[k] = oracle.rel_error(keep[k].cpu().numpy(), Pi_ref)
            dt = time.perf_counter() - t
            cpu = {"value": len(ks) / dt, "unit": "projections/s", "cores": oracle.num_threads(),
                   "kind": "oracle",
                   "sample": f"{len(ks)} of the timed matrices (steps {ks}), FP64 cyclic Jacobi + clip"}
        else:
            # n = 4000: one Jacobi sweep on X_0 scaled by the sweep count the
            # same family needs at n = 1000 is not an oracle run; time the
            # oracle on the step-0 matrix's leading 1000 x 1000 block instead
            sub = np.asfortranarray(mats[0][:1000, :1000])
            t = time.perf_counter()
            oracle.project(sub)
            dt = time.perf_counter() - t
            scale = (n / 1000.0) ** 3
            cpu = {"value": 1.0 / (dt * scale), "unit": "projections/s", "cores": oracle.num_threads(),
                   "kind": "oracle",
                   "sample": "oracle on the leading 1000x1000 block of X_0, time scaled by (4000/1000)^3"}
    # step 0 exact (construction closed form) when the timed region covers it
    out = {
        "metric": "warm-started PSD projections/s vs full-eig at rel err <=1e-6; p50/p99 latency",
        "value": value,
        "unit": "projections/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": 1e3 * wall / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic (seeded prescribed-spectrum matrices; SDPLIB is not available)",
        "config": {"workload": wl, "n": n, "n_pos": p, "block": block, "tol": tol,
                   "matrices": len(mats), "products": prec,
                   "ortho_rr_refine": "fp64"},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "iters_mean": float(iters.mean()),
        "iters_max": int(iters.max()),
        "status_ok": int(sum(1 for s_ in statuses if s_ == 0)),
        "full_eig": {"value": fe_rate, "unit": "projections/s", "method": "rocsolver_dsyevd",
                     "samples": len(fe_idx)},
        "speedup_vs_full_eig": value / fe_rate,
        "rel_err_vs_full_eig_max": max(rel_vs_fe.values()) if rel_vs_fe else None,
        "rel_err_vs_oracle_max": max(rel_oracle.values()) if rel_oracle else None,
        "err_bound_rel_max": max(inf["err_bound"] / max(inf["pi_fro"], 1e-300) for inf in infos),
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels": {f: {"launches": v["launches"], "ms": round(v["ms"], 3),
                        "gflop": round(v["flops"] / 1e9, 3), "gbyte": round(v["bytes"] / 1e9, 3)}
                    for f, v in fams.items()},
    }
    print(json.dumps(out), flush=True)
    proj.close()


if __name__ == "__main__":
    main()
