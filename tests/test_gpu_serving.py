"""GPU tests of the serving loop (psdp_server_*): results in the concurrent
mix equal the results of each session run alone, every result matches the
oracle (relative Frobenius error <= 1e-6), admission by memory footprint
limits concurrency, and a session's warm-start block stays on the device."""
import time

import numpy as np
import pytest

import oracle
from workloads import gapped_sessions, serving_sessions, session_sequence

pytestmark = pytest.mark.gpu

REL = 1e-6


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _specs(count=6, n_max=600, stream=1):
    return serving_sessions(count=count, n_min=32, n_max=n_max, stream=stream)


def _requests(specs, steps):
    """Interleaved (session index, matrix) list: round-robin over sessions."""
    seqs = [list(session_sequence(sp, steps, stream=3)) for sp in specs]
    out = []
    for k in range(steps):
        for i, sq in enumerate(seqs):
            out.append((i, sq[k]))
    return out


def _serve(psdp, torch, specs, reqs, **kw):
    from gpu_util import to_dev
    srv = psdp.Server(0, **kw)
    sids = [srv.open_session(sp.n, m_cap=48, pos_hint=-1) for sp in specs]
    Xd = [to_dev(X) for _, X in reqs]
    torch.cuda.synchronize()
    tickets = [srv.submit(sids[i], x) for (i, _), x in zip(reqs, Xd)]
    results = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    blocks = [srv.session_block(s) for s in sids]
    srv.close()
    return results, stats, blocks


def _alone(psdp, torch, specs, reqs, **kw):
    out = [None] * len(reqs)
    for i in range(len(specs)):
        idx = [j for j, (s, _) in enumerate(reqs) if s == i]
        res, _, _ = _serve(psdp, torch, [specs[i]], [(0, reqs[j][1]) for j in idx], **kw)
        for j, r in zip(idx, res):
            out[j] = r
    return out


def test_mix_equals_alone_and_oracle(gpu):
    torch = gpu
    import paper_1912_02767_amd as psdp
    from gpu_util import to_host
    specs = _specs()
    reqs = _requests(specs, steps=3)
    mix, stats, _ = _serve(psdp, torch, specs, reqs, slots=4)
    alone = _alone(psdp, torch, specs, reqs, slots=4)
    print("stats", stats)
    assert stats["completed"] == len(reqs)
    assert stats["max_active"] >= 2, "requests of different sessions did not overlap"
    for (i, X), a, b in zip(reqs, mix, alone):
        assert a.status >= 0 and b.status >= 0, (a.info, b.info)
        Pa, Pb = to_host(a.Pi), to_host(b.Pi)
        Pi_ref, _ = oracle.project(X)
        ra = oracle.rel_error(Pa, Pi_ref, X)
        rb = oracle.rel_error(Pb, Pi_ref, X)
        assert ra <= REL and rb <= REL, (specs[i].n, ra, rb, a.info)
        assert np.linalg.norm(Pa - Pb) <= 2 * REL * max(np.linalg.norm(Pi_ref), 1e-300)


def test_batching_lane_gathers_small_requests(gpu):
    torch = gpu
    import paper_1912_02767_amd as psdp
    from gpu_util import to_host
    specs = _specs(count=10, n_max=200, stream=2)
    reqs = _requests(specs, steps=4)
    res, stats, _ = _serve(psdp, torch, specs, reqs, slots=2)
    print("stats", stats, "lanes", [r.lane for r in res], "sizes", [r.batch_size for r in res])
    # after the first (full-eig) request every small session is batch-eligible
    assert stats["batched_launches"] >= 1
    assert max(r.batch_size for r in res if r.lane == 1) >= 2
    for (i, X), r in zip(reqs, res):
        Pi_ref, _ = oracle.project(X)
        assert oracle.rel_error(to_host(r.Pi), Pi_ref, X) <= REL, r.info


def test_admission_by_memory_budget(gpu):
    torch = gpu
    import ctypes
    import paper_1912_02767_amd as psdp
    from gpu_util import to_host
    specs = serving_sessions(count=3, n_min=400, n_max=500, stream=4)
    reqs = _requests(specs, steps=2)
    # the server's estimate of the largest request: workspace + full-eig scratch
    nmax = max(sp.n for sp in specs)
    L = (nmax + 63) // 64 * 64
    b = ctypes.c_size_t()
    assert psdp.load().psdp_workspace_bytes(nmax, 48, 1, ctypes.byref(b)) == 0
    budget = int(1.05 * (b.value + 24 * L * L))  # room for one request at a time
    res, stats, _ = _serve(psdp, torch, specs, reqs, slots=4, batch_lane=False, hbm_budget=budget)
    print("stats", stats)
    assert stats["completed"] == len(reqs)
    assert stats["hbm_peak"] <= budget
    assert stats["max_active"] == 1
    for (i, X), r in zip(reqs, res):
        Pi_ref, _ = oracle.project(X)
        assert oracle.rel_error(to_host(r.Pi), Pi_ref, X) <= REL


def test_session_block_is_resident_and_ordered(gpu):
    torch = gpu
    import paper_1912_02767_amd as psdp
    from gpu_util import to_dev, to_host
    sp = _specs(count=1, n_max=300, stream=5)[0]
    seq = list(session_sequence(sp, 4, stream=5))
    srv = psdp.Server(0, slots=3)
    sid = srv.open_session(sp.n, m_cap=48, pos_hint=sp.n_pos)
    Xd = [to_dev(X) for X in seq]
    torch.cuda.synchronize()
    tickets, t_before, t_after = [], [], []
    for x in Xd:
        t_before.append(time.perf_counter())
        tickets.append(srv.submit(sid, x))
        t_after.append(time.perf_counter())
    res = [srv.wait(t) for t in tickets]
    V, lam = srv.session_block(sid)
    assert all(r.status >= 0 for r in res)
    # one session runs one request at a time, in submission order: request
    # k + 1 starts only after request k completed.  The server stamps a
    # submission inside [t_before, t_after], so start(k + 1) <= t_after(k + 1)
    # + queue(k + 1) and done(k) >= t_before(k) + latency(k).
    for k in range(len(res) - 1):
        start_next = 1e3 * t_after[k + 1] + res[k + 1].queue_ms
        done_prev = 1e3 * t_before[k] + res[k].latency_ms
        assert start_next + 0.5 >= done_prev, (k, start_next - done_prev)
    Vh = to_host(V)
    assert Vh.shape[1] >= 1
    assert np.abs(Vh.T @ Vh - np.eye(Vh.shape[1])).max() <= 1e-10
    Xl = seq[-1]
    Pi_ref, lam_ref = oracle.project(Xl)
    assert oracle.rel_error(to_host(res[-1].Pi), Pi_ref, Xl) <= REL
    assert res[-1].info["n_pos"] == int((lam_ref > 0).sum()) or res[-1].info["side_used"] == 3
    assert srv.close_session(sid) == 0
    srv.close()


def test_invalid_requests(gpu):
    torch = gpu
    import paper_1912_02767_amd as psdp
    srv = psdp.Server(0, slots=1)
    with pytest.raises(KeyError):
        srv.submit(999, torch.zeros(4, 4, dtype=torch.float64, device="cuda"))
    with pytest.raises(psdp.PsdpError):
        srv.open_session(10, m_cap=100)
    srv.close()


@pytest.mark.parametrize("method", ["lobpcg", "chebyshev"])
def test_mix_serves_warm_requests_with_the_block_solver(gpu, method):
    """Sessions whose spectra keep a gap: after each session's first request
    (no inertia estimate yet: the exact path) the warm-started requests are
    served by the block eigensolver on the positive side, in the mix as
    alone, and match the oracle and their stand-alone results (both
    eigensolvers)."""
    torch = gpu
    import paper_1912_02767_amd as psdp
    from gpu_util import to_host
    specs = gapped_sessions(count=5, stream=1)
    reqs = _requests(specs, steps=4)
    mix, stats, _ = _serve(psdp, torch, specs, reqs, slots=4, batch_lane=False, method=method)
    alone = _alone(psdp, torch, specs, reqs, slots=4, batch_lane=False, method=method)
    sides = [r.info["side_used"] for r in mix]
    print("stats", stats, "sides", sides)
    block = [k for k, s in enumerate(sides) if s == 1]
    assert len(block) >= len(specs), sides
    for k in block:
        assert mix[k].status == 0 and mix[k].info["certified"] == 1, mix[k].info
    for (i, X), a, b in zip(reqs, mix, alone):
        Pa, Pb = to_host(a.Pi), to_host(b.Pi)
        Pi_ref, _ = oracle.project(X)
        assert oracle.rel_error(Pa, Pi_ref, X) <= REL, (specs[i].n, a.info)
        assert np.linalg.norm(Pa - Pb) <= 2 * REL * max(np.linalg.norm(Pi_ref), 1e-300)


def test_session_blocks_never_copied_to_host(gpu):
    """While the server works, every device-to-host copy the library makes is
    smaller than the smallest session block (n x m doubles): the warm-start
    blocks stay in device memory between requests."""
    torch = gpu
    import paper_1912_02767_amd as psdp
    specs = gapped_sessions(count=4, n_min=200, n_max=400, stream=2)
    reqs = _requests(specs, steps=4)
    psdp.transfer_stats(reset=True)
    res, stats, blocks = _serve(psdp, torch, specs, reqs, slots=3)
    t = psdp.transfer_stats()
    smallest_block = min(8 * sp.n * max(1, V.shape[1]) for sp, (V, _) in zip(specs, blocks))
    print("transfers", t, "smallest block bytes", smallest_block)
    assert all(r.status >= 0 for r in res)
    assert t["copies"] > 0
    assert t["max_bytes"] < smallest_block
