"""GPU parity: the HIP path against the oracle, through the C-ABI.

Tolerances: FP64 products give the projection to ~1e-12 relative; the
spec bar is 1e-6 relative Frobenius error, and the reported bound must
be at least the true error (Thm `bound`, paper §5.2)."""
import numpy as np
import pytest

import oracle
from workloads import (batched_cones, haar_orthogonal, from_spectrum,
                       random_spectrum_matrix, rng_for, single_cone, warm_sequence)

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


def _check(res, Xh, rel=REL, bound=True):
    from gpu_util import to_host
    Pi_ref, lam = oracle.project(Xh)
    Pi = to_host(res.Pi)
    r = oracle.rel_error(Pi, Pi_ref, Xh)
    err = oracle.true_error(Pi, Pi_ref)
    print(f"status={res.status} iters={res.info['iters']} m={res.info['m_out']} "
          f"npos={res.info['n_pos']} rel={r:.2e} err={err:.2e} bound={res.info['err_bound']:.2e}")
    assert r <= rel, (r, res.info)
    if bound:
        # Thm `bound` holds in exact arithmetic for the computed Ritz pairs;
        # the rebuild and the oracle each add rounding of order n u ||X||_F
        slack = 10 * Xh.shape[0] * np.finfo(float).eps * np.linalg.norm(Xh)
        assert res.info["err_bound"] + slack >= err, (err, res.info)
    return r, err, lam


def test_config1_single_cone_fp64(proj):
    from gpu_util import to_dev
    cone, V0 = single_cone()
    res = proj.project(to_dev(cone.X), V=to_dev(V0), m_cap=16, side="pos", tol=1e-10)
    assert res.status == 0
    r, err, lam = _check(res, cone.X)
    assert res.info["n_pos"] == 5
    # Ritz values of the positive pairs are the positive eigenvalues
    lam_gpu = np.sort(res.lam.cpu().numpy()[:5])
    assert np.abs(lam_gpu - np.sort(cone.lam[cone.lam > 0])).max() <= 1e-9


def test_full_eig_matches_oracle(proj):
    from gpu_util import to_dev, to_host
    cone, _ = single_cone()
    Pi, lam = proj.full_eig(to_dev(cone.X))
    Pi_ref, lam_ref = oracle.project(cone.X)
    assert oracle.rel_error(to_host(Pi), Pi_ref) <= 1e-12
    assert np.abs(to_host(lam) - lam_ref).max() <= 1e-12 * np.abs(lam_ref).max()


@pytest.mark.parametrize("n,npos", [(16, 2), (33, 3), (64, 6), (130, 9), (257, 12)])
def test_sizes_ragged(proj, n, npos):
    from gpu_util import to_dev
    c = random_spectrum_matrix(n, npos, rng_for(50, n))
    res = proj.project(to_dev(c.X), m_cap=32, side="pos", tol=1e-10, pos_hint=npos)
    assert res.status == 0
    _check(res, c.X)


def test_negative_side_moreau(proj):
    from gpu_util import to_dev
    # mostly positive spectrum: approximate the negative part of X
    c = random_spectrum_matrix(80, 74, rng_for(51, 0), pos=(0.5, 5.0), neg=(-5.0, -0.5))
    res = proj.project(to_dev(c.X), m_cap=24, side="neg", tol=1e-10, pos_hint=74)
    assert res.status == 0
    assert res.info["side_used"] == 2
    assert res.info["n_pos"] == 6
    _check(res, c.X)


def test_expansion_from_too_small_block(proj):
    from gpu_util import to_dev
    cone, V0 = single_cone()
    res = proj.project(to_dev(cone.X), V=to_dev(V0[:, :2]), m_cap=16, side="pos", tol=1e-10)
    assert res.status == 0
    assert res.info["expansions"] >= 1
    assert res.info["n_pos"] == 5
    _check(res, cone.X)


def test_warm_sequence_small(proj):
    import paper_1912_02767_amd as psdp
    from gpu_util import to_dev
    seq = warm_sequence(n=200, n_pos=6, steps=6)
    c0 = next(seq)
    sess = psdp.Session(proj, 200, m_cap=24, tol=1e-9, side="pos", pos_hint=6)
    iters = []
    for k, X in enumerate([c0.X] + list(seq)):
        res = sess.project(to_dev(X))
        assert res.status == 0
        iters.append(res.info["iters"])
        _check(res, X)
    print("iters", iters)
    assert max(iters[1:]) <= iters[0]


def test_nonfinite_input_rejected(proj):
    from gpu_util import to_dev
    import paper_1912_02767_amd as psdp
    X = np.eye(20)
    X[5, 3] = np.nan
    with pytest.raises(psdp.PsdpError) as e:
        proj.project(to_dev(X), m_cap=8, side="pos")
    assert e.value.code == psdp.PSDP_ERR_NUMERICAL


@pytest.mark.parametrize("method", ["lobpcg", "chebyshev"])
def test_trivial_inputs(proj, method):
    from gpu_util import to_dev, to_host
    # PSD input: Pi = X on the negative side (nothing negative to find)
    rng = rng_for(52, 0)
    Q = haar_orthogonal(40, rng)
    X = from_spectrum(Q, rng.uniform(0.5, 2.0, 40))
    res = proj.project(to_dev(X), m_cap=8, side="neg", tol=1e-10, method=method)
    assert np.abs(to_host(res.Pi) - X).max() <= 1e-9
    # NSD input: Pi = 0 on the positive side
    res = proj.project(to_dev(-X), m_cap=8, side="pos", tol=1e-10, method=method)
    assert np.abs(to_host(res.Pi)).max() <= 1e-9
    # n = 1
    res = proj.project(to_dev(np.array([[2.5]])), m_cap=1, side="pos", tol=1e-12, method=method)
    assert abs(to_host(res.Pi)[0, 0] - 2.5) <= 1e-12
    # zero matrix
    res = proj.project(to_dev(np.zeros((20, 20))), m_cap=4, side="pos", method=method,
                       raise_on_error=False)
    assert res.status >= 0 and np.abs(to_host(res.Pi)).max() == 0.0


@pytest.mark.parametrize("n,npos,m_cap", [(120, 10, 24), (300, 20, 26), (300, 22, 27), (400, 40, 48)])
def test_rr_methods_agree(n, npos, m_cap):
    """The Jacobi Rayleigh-Ritz (kept as a cross-check), the first
    tridiagonal design and the column-parallel one give the same projection
    to the parity bar (block 26 keeps trial bases within the 256-thread
    variant's 80, block 27 crosses to the 512-thread one; n = 400 with block
    48 reaches trial bases of 144)."""
    import os
    import torch
    import paper_1912_02767_amd as psdp
    from gpu_util import to_dev, to_host
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = random_spectrum_matrix(n, npos, rng_for(53, n))
    outs = []
    for method in ("1", "2", "0"):
        os.environ["PSDP_RR_METHOD"] = method
        p = psdp.Projector(0)
        res = p.project(to_dev(c.X), m_cap=m_cap, side="pos", tol=1e-10, pos_hint=npos,
                        block_guard=m_cap - npos)
        assert res.status == 0
        outs.append(to_host(res.Pi))
        _check(res, c.X)
        p.close()
    os.environ.pop("PSDP_RR_METHOD", None)
    assert np.abs(outs[0] - outs[1]).max() <= 1e-8
    assert np.abs(outs[0] - outs[2]).max() <= 1e-8


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_precision_ladder_warm(proj, prec):
    """Warm-started projection with low-precision products (paper §6.2
    mixed precision): the ladder (BF16 -> FP32 -> FP64) ends in FP64 at the
    1e-6 bar, and starting from BF16 costs at most a few more iterations than
    starting from FP32 (the FP32 copy of A is rebuilt at the switch)."""
    from gpu_util import to_dev
    from workloads import large_cone_sequence
    seq = large_cone_sequence(n=640, n_pos=12, steps=2, cumulative=False)
    X0, lam, basis = next(seq)
    X1 = next(seq)
    lam0 = np.sort(lam)[::-1]
    tol = 1e-7 * float(np.linalg.norm(np.maximum(lam0, 0))) / np.sqrt(32)
    r0 = proj.project(to_dev(X0), m_cap=20, side="pos", prec="fp64", tol=tol, pos_hint=12)
    assert r0.status == 0
    iters = {}
    for p in ("fp32", prec):
        res = proj.project(to_dev(X1), V=r0.V[:, :r0.info["m_out"]].clone(), m_cap=20, side="pos",
                           prec=p, tol=tol, pos_hint=12)
        assert res.status == 0 and res.info["prec_final"] == 0, res.info
        _check(res, X1)
        iters[p] = res.info["iters"]
    print("iters", iters)
    assert iters[prec] <= iters["fp32"] + 10


@pytest.mark.parametrize("max_iter", [1, 2, 3, 5])
def test_iteration_cap_with_queued_iteration(proj, max_iter):
    """One iteration is queued ahead of the state readback; the cap still
    holds exactly, and a repeat from the same warm start gives the same
    bytes (a dropped speculative iteration leaves no trace)."""
    from gpu_util import to_dev, to_host
    X = random_spectrum_matrix(300, 30, rng_for(41, 300)).X
    V0 = rng_for(41, 1).standard_normal((300, 36))
    Xd = to_dev(X)
    r1, r2 = (proj.project(Xd, V=to_dev(V0), m_cap=40, side="pos", tol=1e-14,
                           max_iter=max_iter, raise_on_error=False) for _ in range(2))
    assert r1.info["iters"] <= max_iter, r1.info
    assert r1.info["iters"] == r2.info["iters"]
    P1, P2 = to_host(r1.Pi), to_host(r2.Pi)
    assert np.isfinite(P1).all()
    assert np.array_equal(P1, P2)


def test_repeat_is_bitwise_identical(proj):
    """The pipelined loop is deterministic: the same warm-started call twice
    gives the same projection bytes."""
    from gpu_util import to_dev, to_host
    X = random_spectrum_matrix(500, 40, rng_for(42, 500)).X
    V0 = rng_for(42, 1).standard_normal((500, 46))
    Xd = to_dev(X)
    res = [proj.project(Xd, V=to_dev(V0), m_cap=48, side="pos", tol=1e-10)
           for _ in range(2)]
    assert res[0].info["iters"] == res[1].info["iters"]
    assert np.array_equal(to_host(res[0].Pi), to_host(res[1].Pi))
    _check(res[0], X)


def test_profile_filter_times_only_named_families(proj):
    from gpu_util import to_dev
    X = to_dev(random_spectrum_matrix(300, 20, rng_for(43, 300)).X)
    proj.profile_filter("rr")
    proj.profile_enable(True)
    proj.project(X, m_cap=32, side="pos", tol=1e-10)
    rr, gram = proj.profile_get("rr"), proj.profile_get("gram")
    proj.profile_enable(False)
    proj.profile_filter("")
    assert rr["launches"] > 0 and rr["ms"] > 0
    assert gram["launches"] == 0
    proj.profile_enable(True)
    proj.project(X, m_cap=32, side="pos", tol=1e-10)
    gram = proj.profile_get("gram")
    proj.profile_enable(False)
    assert gram["launches"] > 0


def test_product_tallies_split_by_precision(proj):
    """Block-product launches are also tallied per product precision; the
    split never exceeds the family total."""
    from gpu_util import to_dev
    X = to_dev(random_spectrum_matrix(600, 20, rng_for(44, 600)).X)
    proj.profile_enable(True)
    proj.project(X, m_cap=32, side="pos", prec="fp32", tol=1e-9)
    tot = proj.profile_get("product")
    parts = {p: proj.profile_get("product_" + p) for p in ("fp64", "fp32", "bf16")}
    proj.profile_enable(False)
    assert parts["fp32"]["launches"] > 0 and parts["fp32"]["flops"] > 0
    assert sum(v["launches"] for v in parts.values()) <= tot["launches"]
    assert sum(v["ms"] for v in parts.values()) <= tot["ms"] * (1 + 1e-9)


@pytest.mark.parametrize("limit,fell_back", [(0.0, False), (1.0, False), (1e-30, True)])
def test_bound_target_fallback(proj, limit, fell_back):
    """With fallback_full, a converged result whose a-posteriori bound is above
    bound_rel_max * ||Pi||_F takes the exact path; 0 disables the check."""
    from gpu_util import to_dev
    c = random_spectrum_matrix(200, 10, rng_for(45, 200))
    res = proj.project(to_dev(c.X), m_cap=24, side="pos", tol=1e-10, fallback_full=True,
                       bound_rel_max=limit, raise_on_error=False)
    if fell_back:
        assert res.status == 2 and res.info["side_used"] == 3, res.info  # fell back; full side
        assert res.info["n_pos_full"] == 10
        _check(res, c.X, rel=1e-12, bound=False)
    else:
        assert res.status == 0 and res.info["side_used"] == 1, res.info
        assert res.info["err_bound"] <= 1.0 * res.info["pi_fro"]
        _check(res, c.X)


def test_library_auto_side_choices(proj):
    """The library's AUTO rule (paper §6): the positive side when fewer than
    n/3 eigenvalues are estimated positive, the negative side when fewer
    than n/3 are negative, the exact path for a half/half inertia or when
    there is no estimate."""
    from gpu_util import to_dev
    mostly_pos = random_spectrum_matrix(240, 230, rng_for(46, 0), pos=(0.5, 5.0), neg=(-5.0, -0.5))
    res = proj.project(to_dev(mostly_pos.X), m_cap=24, side="auto", tol=1e-10, pos_hint=230)
    assert res.info["side_used"] == 2 and res.status == 0, res.info
    assert res.info["pos_est"] == 230 and res.info["block_side"] == 2
    _check(res, mostly_pos.X)
    mostly_neg = random_spectrum_matrix(240, 10, rng_for(46, 1))
    res = proj.project(to_dev(mostly_neg.X), m_cap=24, side="auto", tol=1e-10, pos_hint=10)
    assert res.info["side_used"] == 1 and res.status == 0, res.info
    assert res.info["pos_est"] == 10 and res.info["block_side"] == 1
    half = random_spectrum_matrix(240, 120, rng_for(46, 2))
    res = proj.project(to_dev(half.X), m_cap=24, side="auto", tol=1e-10, pos_hint=120,
                       raise_on_error=False)
    assert res.info["side_used"] == 3 and res.status == 2, res.info
    assert res.info["pos_est"] == 120 and res.info["block_side"] == 1
    _check(res, half.X, rel=1e-12, bound=False)
    res = proj.project(to_dev(mostly_neg.X), m_cap=24, side="auto", tol=1e-10, pos_hint=-1,
                       raise_on_error=False)
    assert res.info["side_used"] == 3 and res.info["pos_est"] == 10


def test_session_carries_library_side(proj):
    """A Session with side AUTO and no estimate: the first call takes the
    exact path, which returns the leading eigenpairs and the inertia; the
    next calls run the block solver on the positive side warm-started from
    that block.  A warm block of the other side is not used."""
    import paper_1912_02767_amd as psdp
    from gpu_util import to_dev
    seq = warm_sequence(n=300, n_pos=8, steps=4)
    c0 = next(seq)
    sess = psdp.Session(proj, 300, m_cap=24, tol=1e-9, side="auto", pos_hint=-1)
    sides = []
    for X in [c0.X] + list(seq):
        res = sess.project(to_dev(X))
        sides.append(res.info["side_used"])
        _check(res, X, bound=res.info["side_used"] != 3)
    assert sides[0] == 3 and all(s == 1 for s in sides[1:]), sides
    # a negative-side block offered to a positive-side call is dropped
    X = to_dev(c0.X)
    r = proj.project(X, V=sess.V_buf[:, :sess.m].clone(), m_cap=24, side="pos", tol=1e-9,
                     pos_hint=8, warm_side="neg")
    assert r.status == 0
    _check(r, c0.X)


@pytest.mark.parametrize("steps", [1, 2])
def test_block_krylov_variant_matches_oracle(proj, steps):
    """PSDP_METHOD_BLOCK_KRYLOV (paper §5: Rayleigh-Ritz on span(X, AX), a
    single block Lanczos iteration from the warm start) gives the oracle's
    projection from the same subspace; its reported bound covers the error."""
    from gpu_util import to_dev, to_host
    c = random_spectrum_matrix(300, 10, rng_for(47, steps))
    X0 = rng_for(47, 10 + steps).standard_normal((300, 16))
    res = proj.project(to_dev(c.X), V=to_dev(X0), m_cap=16, side="pos", tol=1e-14,
                       method="block_krylov", method_param=steps, raise_on_error=False)
    assert res.status in (0, 1), res.info
    Pi_k, theta, _ = oracle.block_krylov_projection(c.X, X0, steps=steps)
    Pi = to_host(res.Pi)
    lam = np.sort(res.lam.cpu().numpy())[::-1]
    print(steps, res.status, res.info["iters"], np.abs(Pi - Pi_k).max(), lam[:4], theta[:4])
    assert np.abs(lam - theta).max() <= 1e-9 * np.abs(theta).max()
    assert oracle.rel_error(Pi, Pi_k) <= 1e-9
    Pi_ref, _ = oracle.project(c.X)
    err = oracle.true_error(Pi, Pi_ref)
    assert res.info["err_bound"] >= err


@pytest.mark.parametrize("r", [6, 16])
def test_top_r_variant_matches_truncated_oracle(proj, r):
    """PSDP_METHOD_TOP_R (paper §1: the truncated projection over the r
    largest eigenpairs): the oracle's truncation, the truncation bound above
    the true error, and a certificate only when no positive eigenvalue is
    left out."""
    from gpu_util import to_dev, to_host
    c = random_spectrum_matrix(300, 12, rng_for(48, r), pos=(1.0, 10.0), neg=(-10.0, -0.1))
    res = proj.project(to_dev(c.X), m_cap=32, side="pos", tol=1e-10, method="top_r",
                       method_param=r, raise_on_error=False)
    assert res.status == 0, res.info
    Pi_r, lam = oracle.truncated_projection(c.X, r)
    Pi = to_host(res.Pi)
    Pi_ref, _ = oracle.project(c.X)
    print(r, res.info["m_out"], res.info["certified"], oracle.rel_error(Pi, Pi_r),
          res.info["trunc_bound"], oracle.true_error(Pi, Pi_ref))
    assert res.info["m_out"] == r
    assert oracle.rel_error(Pi, Pi_r) <= 1e-8
    assert res.info["trunc_bound"] + 1e-9 >= oracle.true_error(Pi, Pi_ref)
    if r >= 12:
        assert res.info["certified"] == 1 and oracle.rel_error(Pi, Pi_ref) <= 1e-8
    else:
        assert res.info["certified"] == 0 and np.isinf(res.info["err_bound"])


def _iid_like(n, npos, key):
    """Spectrum of the n = 4000 mixed-precision workload at a smaller order:
    npos eigenvalues 10^U[0, 2], the rest -10^U[-3, 2]."""
    rng = rng_for(49, key)
    lam = np.concatenate([10 ** rng.uniform(0, 2, npos), -10 ** rng.uniform(-3, 2, n - npos)])
    Q = haar_orthogonal(n, rng)
    return from_spectrum(Q, lam), lam


@pytest.mark.parametrize("n,npos,side", [(640, 7, "pos"), (300, 290, "neg"), (40, 3, "pos"),
                                         (130, 3, "pos")])
def test_chebyshev_variant_matches_oracle(proj, n, npos, side):
    """PSDP_METHOD_CHEBYSHEV (polynomial subspace extraction, paper §1): from
    a cold start the filtered passes reach the oracle's projection with the
    same certified bound; the Lanczos lower end is below the spectrum."""
    from gpu_util import to_dev
    X, lam = _iid_like(n, npos, n + npos)
    res = proj.project(to_dev(X), m_cap=24, side=side, method="chebyshev", raise_on_error=False)
    print(n, side, res.status, res.info["iters"], res.info["products"], res.info["spec_lower"],
          lam.min(), -lam.max())
    assert res.status == 0, res.info
    assert res.info["certified"] == 1
    assert res.info["products"] > 0
    low = lam.min() if side == "pos" else -lam.max()
    assert res.info["spec_lower"] <= low + 1e-9 * abs(low)
    _check(res, X)


def test_chebyshev_warm_sequence_and_expansion(proj):
    """Warm-started passes over a perturbed sequence, and a start block
    narrower than the positive part (the block is expanded)."""
    from gpu_util import to_dev, to_host
    c = random_spectrum_matrix(500, 12, rng_for(49, 7), pos=(1.0, 100.0), neg=(-100.0, -0.1))
    X = c.X
    r0 = proj.project(to_dev(X), m_cap=32, side="pos", pos_hint=4, method="chebyshev",
                      raise_on_error=False)
    assert r0.status == 0 and r0.info["expansions"] >= 1, r0.info
    _check(r0, X)
    rng = rng_for(49, 99)
    V, k = r0.V, r0.info["m_out"]
    for step in range(3):
        E = rng.standard_normal((500, 500))
        E = E + E.T
        Xs = X + E * (1e-4 * np.linalg.norm(X) / np.linalg.norm(E))
        r = proj.project(to_dev(Xs), V=V[:, :k].clone(), m_cap=32, side="pos",
                         method="chebyshev", raise_on_error=False)
        assert r.status == 0, r.info
        assert r.info["iters"] <= r0.info["iters"] + 1
        _check(r, Xs)
        V, k = r.V, r.info["m_out"]


def test_chebyshev_zero_cluster_is_honest(proj):
    """Eigenvalues clustered at zero and perturbed across it (the spectrum
    of the n = 4000 chain at n = 500): a positive eigenvalue in the cluster
    can stay outside the block, which the certificate then reports, and the
    residuals converge slowly; every result is within 1e-6 of the oracle or
    not PSDP_OK, and every finite bound covers the true error."""
    from gpu_util import to_dev, to_host
    X, lam = _iid_like(500, 12, 8)
    rng = rng_for(49, 98)
    V, k = None, 0
    for step in range(4):
        E = rng.standard_normal((500, 500))
        E = E + E.T
        X = X + E * (1e-4 * np.linalg.norm(X) / np.linalg.norm(E))
        r = proj.project(to_dev(X), V=None if V is None else V[:, :k].clone(), m_cap=32,
                         side="pos", pos_hint=12, method="chebyshev", max_iter=12,
                         raise_on_error=False)
        Pi_ref, _ = oracle.project(X)
        err = oracle.true_error(to_host(r.Pi), Pi_ref)
        rel = oracle.rel_error(to_host(r.Pi), Pi_ref, X)
        print(step, r.status, r.info["iters"], r.info["n_pos"], r.info["certified"], rel,
              r.info["err_bound"])
        if r.status == 0:
            assert rel <= REL
        if np.isfinite(r.info["err_bound"]):
            assert r.info["err_bound"] * (1 + 1e-6) + 1e-9 >= err
        V, k = r.V, r.info["m_out"]


def test_method_arguments_validated(proj):
    """An unknown method or a negative method_param is rejected before any
    launch; LOBPCG reports no Chebyshev figures."""
    from gpu_util import to_dev
    c = random_spectrum_matrix(64, 4, rng_for(50, 1))
    X = to_dev(c.X)
    for kw in ({"method": 4}, {"method": "chebyshev", "method_param": -1}):
        r = proj.project(X, m_cap=16, side="pos", raise_on_error=False, **kw)
        assert r.status == -1, (kw, r.info)
    r = proj.project(X, m_cap=16, side="pos", raise_on_error=False)
    assert r.status == 0 and r.info["products"] == 0 and np.isnan(r.info["spec_lower"])
    r = proj.project(X, m_cap=16, side="pos", method="chebyshev", method_param=6,
                     raise_on_error=False)
    assert r.status == 0 and r.info["products"] > 0
    _check(r, c.X)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_chebyshev_low_precision_passes(proj, prec):
    """With FP32 (or BF16) products requested, the filter's early passes run
    on the low-precision copy of A while the residuals are far above its
    rounding floor, the later ones in FP64: the result still meets 1e-6 with
    a certified bound."""
    from gpu_util import to_dev
    X, lam = _iid_like(900, 9, 51)
    res = proj.project(to_dev(X), m_cap=24, side="pos", prec=prec, method="chebyshev",
                       raise_on_error=False)
    assert res.status == 0 and res.info["certified"] == 1, res.info
    _check(res, X)
