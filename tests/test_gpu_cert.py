"""GPU: the tail certificate of the a-posteriori bound (paper §5.2, Thm
`bound`, the term ||Pi(Vt_perp^T A Vt_perp)||_F) through the C-ABI.

psdp_certify_tail proves that every eigenvalue of Vt_perp^T A Vt_perp lies
below delta_eff; the oracle gives that spectrum exactly
(oracle.complement_spectrum), so each case checks the certificate against
it: certified when the largest complement eigenvalue is clearly below delta,
refused when it is clearly above.  psdp_project then uses the certificate
by default: a result reported PSDP_OK must meet the accuracy it claims, on
a sequence whose positive eigenvalues leave the block (the n = 4000 random
walk's spectrum recipe at n = 1000)."""
import math

import numpy as np
import pytest

import oracle
from workloads import (from_spectrum, haar_orthogonal, large_cone_sequence, rng_for,
                       single_cone)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def proj():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from gpu_util import projector
    p = projector()
    yield p
    p.close()


def _matrix(n, m, top, rest_max, seed):
    """X = Q diag(lam) Q^T with m eigenvalues `top` (the block) and the others
    spread in [-5, rest_max] with rest_max the largest; returns X, V = the
    block's eigenvectors."""
    rng = rng_for(91, seed)
    Q = haar_orthogonal(n, rng)
    rest = -rng.uniform(0.01, 5.0, n - m)
    rest[0] = rest_max
    lam = np.concatenate([np.full(m, top) + rng.uniform(0, 1, m), rest])
    return from_spectrum(Q, lam), np.asfortranarray(Q[:, :m])


@pytest.mark.parametrize("n,m", [(64, 5), (130, 9), (700, 20), (1000, 48), (257, 0)])
@pytest.mark.parametrize("rest_max", [-1e-3, 4e-7, 5e-5])
def test_certify_tail_against_complement_spectrum(proj, n, m, rest_max):
    from gpu_util import to_dev
    X, V = _matrix(n, m, 2.0, rest_max, n + m)
    delta = 1e-6
    ok, delta_eff, eta = proj.certify_tail(to_dev(X), to_dev(V) if m else None, delta)
    mu = oracle.complement_spectrum(X, V)
    lam_max = mu.max()
    print(f"n={n} m={m} lam_max={lam_max:.3e} certified={ok} delta_eff={delta_eff:.3e} eta={eta:.3e}")
    assert delta_eff >= delta and eta < 0.1 * delta
    if ok:
        assert lam_max < delta_eff  # what the certificate states
    if lam_max < 0.5 * delta:
        assert ok  # clearly below: the margin eta is far smaller than delta
    if lam_max > 2.0 * delta_eff:
        assert not ok


def test_certify_tail_random_block(proj):
    # Vt not an invariant subspace: the compression's spectrum interlaces
    from gpu_util import to_dev
    n, m = 300, 12
    rng = rng_for(92, 0)
    Q = haar_orthogonal(n, rng)
    lam = np.concatenate([rng.uniform(1, 4, 6), -rng.uniform(0.2, 3.0, n - 6)])
    X = from_spectrum(Q, lam)
    # the block holds the positive eigenvectors plus random directions
    Z = rng.standard_normal((n, m - 6))
    Vb, _ = np.linalg.qr(np.concatenate([Q[:, :6], Z], axis=1))
    V = np.asfortranarray(Vb)
    mu = oracle.complement_spectrum(X, V)
    ok, de, eta = proj.certify_tail(to_dev(X), to_dev(V), 1e-6)
    assert mu.max() < -0.1 and ok
    # leave one positive eigenvector out: its direction stays in the complement
    V2 = np.asfortranarray(np.linalg.qr(np.concatenate([Q[:, :5], Z], axis=1))[0])
    mu2 = oracle.complement_spectrum(X, V2)
    ok2, _, _ = proj.certify_tail(to_dev(X), to_dev(V2), 1e-6)
    assert mu2.max() > 0.5 and not ok2


def test_project_default_is_certified(proj):
    from gpu_util import to_dev, to_host
    cone, V0 = single_cone()
    res = proj.project(to_dev(cone.X), V=to_dev(V0), m_cap=16, side="pos", tol=1e-10)
    assert res.status == 0
    info = res.info
    assert info["certified"] == 1 and info["cert_delta"] > 0
    n, npos = cone.X.shape[0], info["n_pos"]
    assert info["tail_est"] == pytest.approx(math.sqrt(n - npos) * info["cert_delta"])
    Pi_ref, _ = oracle.project(cone.X)
    err = oracle.true_error(to_host(res.Pi), Pi_ref)
    assert info["err_bound"] >= err


def test_certificate_off_gives_estimate(proj):
    from gpu_util import to_dev
    cone, V0 = single_cone()
    res = proj.project(to_dev(cone.X), V=to_dev(V0), m_cap=16, side="pos", tol=1e-10,
                       certify=False)
    assert res.status == 0
    assert res.info["certified"] == 0 and math.isnan(res.info["cert_delta"])


def _chain(n, npos, steps):
    seq = large_cone_sequence(n=n, n_pos=npos, steps=steps, cumulative=True)
    X0, lam, _ = next(seq)
    return [X0] + list(seq), lam


@pytest.mark.parametrize("fallback", [False, True])
def test_chain_ok_means_accurate(proj, fallback):
    """n = 1000 with the large cone's recipe (1% positive in [1, 100], the
    rest -10^U[-3, 2], Householder basis) and the random walk
    X_{k+1} = X_k + E_k, ||E_k|| = 1e-4 ||X_k||_F: from step 2 on, positive
    eigenvalues of order 1e-5 .. 1e-3 appear next to the cluster at zero and
    outside a 14-column block (their share of ||Pi||_F is ~1e-5 at step 2).
    Every step that returns PSDP_OK must be within 1e-6 of the oracle with a
    bound at least the true error; without fallback the later steps must
    not be PSDP_OK; with fallback every step is within 1e-6."""
    from gpu_util import to_dev, to_host
    import paper_1912_02767_amd as psdp
    n, npos, steps = 1000, 10, 9
    mats, lam0 = _chain(n, npos, steps)
    nrm_pi0 = float(np.linalg.norm(np.maximum(lam0, 0)))
    tol = 5e-7 * nrm_pi0 / math.sqrt(2 * npos)
    sess = psdp.Session(proj, n, m_cap=14, tol=tol, side="pos", pos_hint=npos, prec="fp64",
                        block_guard=4, fallback_full=fallback)
    statuses = []
    for k, X in enumerate(mats):
        res = sess.project(to_dev(X))
        Pi_ref, lam = oracle.project(X)
        Pi = to_host(res.Pi)
        rel = oracle.rel_error(Pi, Pi_ref, X)
        err = oracle.true_error(Pi, Pi_ref)
        info = res.info
        npos_true = int((lam > 0).sum())
        print(f"step {k}: status={res.status} side={info['side_used']} npos={info['n_pos']} "
              f"true_npos={npos_true} certified={info['certified']} rel={rel:.2e} "
              f"bound={info['err_bound']:.2e} err={err:.2e}", flush=True)
        statuses.append(res.status)
        slack = 10 * n * np.finfo(float).eps * np.linalg.norm(X)
        if res.status in (psdp.PSDP_OK, psdp.PSDP_FELL_BACK_FULL_EIG):
            assert rel <= 1e-6, (k, rel, info)
        if res.status == psdp.PSDP_OK:
            assert info["certified"] == 1
            assert info["err_bound"] + slack >= err, (k, err, info)
        else:
            assert res.status in (psdp.PSDP_NOT_CONVERGED, psdp.PSDP_FELL_BACK_FULL_EIG), res.status
            if res.status == psdp.PSDP_NOT_CONVERGED:
                assert info["err_bound"] + slack >= err
    assert statuses[0] == psdp.PSDP_OK
    if not fallback:
        # positive eigenvalues outside the block from step 2 on (largest
        # missing share ~1e-5 of ||Pi||): no such step may be reported OK
        assert all(s != psdp.PSDP_OK for s in statuses[2:]), statuses
