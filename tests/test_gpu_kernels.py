"""GPU checks of the block product kernel on its own (psdp_block_product):
MFMA FP64 / FP32 / BF16 against FP64 products of the same rounded inputs,
ragged sizes, split-K reproducibility."""
import numpy as np
import pytest

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


def _round(a, prec):
    import torch
    if prec == "fp64":
        return a
    a32 = a.astype(np.float32)
    if prec == "fp32":
        return a32.astype(np.float64)
    return torch.from_numpy(a32).to(torch.bfloat16).to(torch.float64).numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n,k", [(50, 8), (130, 24), (257, 72), (1000, 144), (1100, 17)])
def test_block_product_matches_rounded_fp64(proj, prec, n, k):
    from gpu_util import to_dev, to_host
    rng = np.random.default_rng(1000 + n + k)
    G = rng.standard_normal((n, n))
    X = G + G.T
    S = rng.standard_normal((n, k)) / np.sqrt(n)
    Y = to_host(proj.block_product(to_dev(X), to_dev(S), prec=prec))
    Xs = np.tril(X) + np.tril(X, -1).T
    ref = _round(Xs, prec) @ _round(S, prec)
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    tol = {"fp64": 1e-13, "fp32": 2e-6, "bf16": 2e-6}[prec]
    print(prec, n, k, err)
    assert err <= tol


def test_block_product_reproducible(proj):
    from gpu_util import to_dev, to_host
    rng = np.random.default_rng(7)
    n, k = 2100, 96
    G = rng.standard_normal((n, n))
    X, S = to_dev(G + G.T), to_dev(rng.standard_normal((n, k)))
    for prec in ("fp64", "fp32", "bf16"):
        Y1 = to_host(proj.block_product(X, S, prec=prec))
        Y2 = to_host(proj.block_product(X, S, prec=prec))
        assert np.array_equal(Y1, Y2)
