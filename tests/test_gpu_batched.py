"""GPU parity of the batched persistent engine (many uneven cones in one
launch, paper §6.1 block-diagonal SDPs) against the oracle, through the
C-ABI (psdp_project_batched).

Bar: relative Frobenius error <= 1e-6 per cone on the FP64-refined path, and
the reported bound at least the true error (Thm `bound`, paper §5.2)."""
import math

import numpy as np
import pytest

import oracle
from workloads import batched_cones, random_spectrum_matrix, rng_for, sym_perturbation

pytestmark = pytest.mark.gpu

REL = 1e-6


@pytest.fixture(scope="module")
def proj():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from gpu_util import projector
    p = projector()
    yield p
    p.close()


def _caps(cones):
    # block: positive count + max(4, ceil(0.2 p)), at most 32
    out = []
    for c in cones:
        p = int((c.lam > 0).sum())
        out.append(min(32, c.X.shape[0], p + max(4, math.ceil(0.2 * p))))
    return out


def _check_cone(res, Xh, rel=REL):
    from gpu_util import to_host
    Pi_ref, _ = oracle.project(Xh)
    Pi = to_host(res.Pi)
    r = oracle.rel_error(Pi, Pi_ref, Xh)
    err = oracle.true_error(Pi, Pi_ref)
    assert r <= rel, (Xh.shape[0], r, res.info)
    slack = 10 * Xh.shape[0] * np.finfo(float).eps * np.linalg.norm(Xh)
    assert res.info["err_bound"] + slack >= err, (err, res.info)
    assert np.array_equal(Pi, Pi.T)
    return r


def _upload(cones):
    from gpu_util import to_dev
    return [to_dev(c.X) for c in cones]


def test_batch_matches_oracle_fp32(proj):
    cones = batched_cones(count=24, stream=1)
    caps = _caps(cones)
    res = proj.project_batched(_upload(cones), m_caps=caps, prec="fp32")
    worst = 0.0
    for c, r, cap in zip(cones, res, caps):
        assert r.status == 0, r.info
        assert r.info["n_pos"] == int((c.lam > 0).sum())
        assert r.info["m_out"] <= cap
        worst = max(worst, _check_cone(r, c.X))
    print(f"worst rel {worst:.2e}")


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_every_launch_shape(proj, variant):
    cones = batched_cones(count=10, n_min=16, n_max=256, stream=2)
    caps = _caps(cones)
    res = proj.project_batched(_upload(cones), m_caps=caps, prec="fp32", variant=variant)
    for c, r in zip(cones, res):
        assert r.status == 0, r.info
        _check_cone(r, c.X)


def test_fp64_products(proj):
    cones = batched_cones(count=8, stream=3)
    res = proj.project_batched(_upload(cones), m_caps=_caps(cones), prec="fp64")
    for c, r in zip(cones, res):
        assert r.status == 0 and r.info["prec_final"] == 0
        _check_cone(r, c.X)


def test_graph_replay_equals_eager(proj):
    import torch
    cones = batched_cones(count=12, stream=4)
    caps = _caps(cones)
    Xd = _upload(cones)
    eager = proj.project_batched(Xd, m_caps=caps, prec="fp32", variant=0, graph=False)
    ref = [r.Pi.clone() for r in eager]
    for rep in range(3):
        # eager work of the program between replays
        junk = torch.randn(512, 512, device="cuda", dtype=torch.float64)
        (junk @ junk).sum().item()
        torch.cuda.synchronize()
        got = proj.project_batched(Xd, m_caps=caps, prec="fp32", variant=0, graph=True)
        for a, b in zip(ref, got):
            assert torch.equal(a, b.Pi), f"replay {rep} differs"


def test_batched_equals_single(proj):
    from gpu_util import to_host
    cones = batched_cones(count=6, stream=5)
    caps = _caps(cones)
    Xd = _upload(cones)
    bat = proj.project_batched(Xd, m_caps=caps, prec="fp32")
    for c, x, r, cap in zip(cones, Xd, bat, caps):
        p = int((c.lam > 0).sum())
        s = proj.project(x, m_cap=cap, side="pos", pos_hint=p, prec="fp32")
        assert s.status == 0
        a, b = to_host(r.Pi), to_host(s.Pi)
        assert np.linalg.norm(a - b) <= 2 * REL * np.linalg.norm(b)


def test_warm_start_sequence(proj):
    from gpu_util import to_dev
    cones = batched_cones(count=8, stream=6)
    caps = _caps(cones)
    res = proj.project_batched(_upload(cones), m_caps=caps, prec="fp32")
    it_cold = [r.info["iters"] for r in res]
    Vs = [r.V.clone() for r in res]
    rng = rng_for(4, 99)
    X2 = [np.asfortranarray(c.X + sym_perturbation(c.X.shape[0], 1e-4 * np.linalg.norm(c.X), rng))
          for c in cones]
    res2 = proj.project_batched([to_dev(x) for x in X2], m_caps=caps, Vs=Vs, prec="fp32")
    for x, r in zip(X2, res2):
        assert r.status == 0
        _check_cone(r, x)
    it_warm = [r.info["iters"] for r in res2]
    print("cold", it_cold, "warm", it_warm)
    assert sum(it_warm) < sum(it_cold)


def test_negative_side(proj):
    from gpu_util import to_dev
    cones = [random_spectrum_matrix(n, n - max(1, n // 10), rng_for(40, n), pos=(0.1, 10.0),
                                    neg=(-10.0, -0.1)) for n in (20, 75, 140)]
    caps = [min(32, max(1, n // 10) + 4) for n in (20, 75, 140)]
    res = proj.project_batched([to_dev(c.X) for c in cones], m_caps=caps, prec="fp32", side="neg")
    for c, r in zip(cones, res):
        assert r.status == 0 and r.info["side_used"] == 2
        _check_cone(r, c.X)


def test_ragged_edges(proj):
    from gpu_util import to_dev
    ns = [1, 2, 3, 15, 16, 17, 63, 64, 65, 255, 256]
    cones = [random_spectrum_matrix(n, max(1, n // 10), rng_for(41, n)) for n in ns]
    caps = [min(32, n, max(1, n // 10) + 4) for n in ns]
    res = proj.project_batched([to_dev(c.X) for c in cones], m_caps=caps, prec="fp32")
    for c, r in zip(cones, res):
        assert r.status in (0, 1), r.info
        _check_cone(r, c.X)


def test_nonfinite_cone_isolated(proj):
    import torch
    from gpu_util import to_dev
    cones = batched_cones(count=4, stream=7)
    Xd = _upload(cones)
    Xd[1][3, 2] = float("nan")
    res = proj.project_batched(Xd, m_caps=_caps(cones), prec="fp32")
    assert res[1].status == -4
    for i in (0, 2, 3):
        assert res[i].status == 0
        _check_cone(res[i], cones[i].X)


def test_invalid_arguments(proj):
    import paper_1912_02767_amd as psdp
    from gpu_util import to_dev
    x = to_dev(random_spectrum_matrix(300, 5, rng_for(42, 0)).X)
    with pytest.raises(psdp.PsdpError):
        proj.project_batched([x], m_caps=[8])
    assert proj.project_batched([], m_caps=[]) == []


def test_full_size_batch_sampled(proj):
    """The 512-cone workload in the launch configuration the benchmark
    times; a sample of cones is checked against the oracle, every cone
    against its own bound and the statuses."""
    from gpu_util import to_host
    cones = batched_cones(count=512, stream=0)
    caps = _caps(cones)
    res = proj.project_batched(_upload(cones), m_caps=caps, prec="fp32")
    assert all(r.status == 0 for r in res), [r.info for r in res if r.status != 0][:3]
    rel_bound = max(r.info["err_bound"] / r.info["pi_fro"] for r in res)
    assert rel_bound <= 1e-6
    order = np.argsort([c.X.shape[0] for c in cones])
    sample = list(order[:4]) + list(order[-6:]) + list(order[250:254])
    for i in sample:
        _check_cone(res[i], cones[i].X)


def test_full_eig_batched_matches_oracle(proj):
    """Exact batched path: zero-padded buckets of order round_up(n, 32)."""
    from gpu_util import to_dev, to_host
    ns = [1, 5, 31, 32, 33, 64, 100, 200, 255, 256]
    cones = [random_spectrum_matrix(n, max(1, n // 7), rng_for(43, n)) for n in ns]
    caps = [min(48, n) for n in ns]
    res = proj.full_eig_batched([to_dev(c.X) for c in cones], m_caps=caps)
    for c, r, cap in zip(cones, res, caps):
        Pi_ref, lam_ref = oracle.project(c.X)
        assert r.status == 0
        assert oracle.rel_error(to_host(r.Pi), Pi_ref, c.X) <= 1e-12
        p = int((lam_ref > 0).sum())
        assert r.info["n_pos"] == p
        k = r.info["m_out"]
        assert k == min(cap, c.X.shape[0], p + max(4, math.ceil(0.2 * p)))
        # leading eigenpairs, largest first, in the cone's own coordinates
        lam = to_host(r.lam)
        assert np.allclose(lam, np.sort(lam_ref)[::-1][:k], atol=1e-10 * np.abs(lam_ref).max())
        V = to_host(r.V)
        assert np.abs(V.T @ V - np.eye(k)).max() <= 1e-10
    # projection only
    res2 = proj.full_eig_batched([to_dev(c.X) for c in cones])
    for a, b in zip(res, res2):
        assert np.array_equal(to_host(a.Pi), to_host(b.Pi))


def test_fallback_to_exact_path(proj):
    """A cone whose positive eigenvalues crowd against zero does not converge
    within a few iterations; with fallback_full the call returns it exact."""
    from gpu_util import to_dev, to_host
    rng = rng_for(44, 0)
    from workloads import from_spectrum, haar_orthogonal
    n = 120
    lam = np.concatenate([10.0 ** rng.uniform(-3, 2, 12), -(10.0 ** rng.uniform(-3, 2, n - 12))])
    lam[:3] = [1e-5, 2e-5, 3e-5]
    X = from_spectrum(haar_orthogonal(n, rng), lam)
    good = batched_cones(count=3, stream=8)
    Xs = [X] + [c.X for c in good]
    caps = [20] + _caps(good)
    res = proj.project_batched([to_dev(x) for x in Xs], m_caps=caps, prec="fp32", max_iter=15,
                               fallback_full=True)
    assert res[0].status == 2 and res[0].info["side_used"] == 3
    for x, r in zip(Xs, res):
        Pi_ref, _ = oracle.project(x)
        assert oracle.rel_error(to_host(r.Pi), Pi_ref, x) <= REL, r.info
