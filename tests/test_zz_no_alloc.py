"""GPU: psdp_block_product_noalloc, the block product for callers that cannot
allocate (its buffers live in a static device array), against
psdp_block_product through the C-ABI: the same kernels give the same bytes.
Two calls in a row, the second smaller, share the array; a request beyond the
array's capacity is refused before any launch."""
import ctypes

import numpy as np
import pytest

from workloads import random_spectrum_matrix, rng_for

pytestmark = pytest.mark.gpu


def _call(lib, fn, h, X, S, Y, prec):
    n, k = S.shape
    return getattr(lib, fn)(h, n, ctypes.c_void_p(X.data_ptr()), X.stride(1),
                            ctypes.c_void_p(S.data_ptr()), S.stride(1), k, prec,
                            ctypes.c_void_p(Y.data_ptr()), Y.stride(1))


def test_noalloc_product_matches_workspace_product():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_02767_amd as psdp
    from gpu_util import to_dev
    proj = psdp.Projector(0)
    lib, h = proj.lib, proj._h
    try:
        for n, k, prec in [(1000, 144, 0), (300, 40, 0), (1000, 96, 1), (257, 17, 2)]:
            print(f"n={n} k={k} prec={prec}", flush=True)
            X = to_dev(random_spectrum_matrix(n, max(1, n // 20), rng_for(94, n)).X)
            S = to_dev(rng_for(94, 1000 + n).standard_normal((n, k)))
            Y_ref = psdp._empty_f(n, k, X.device)
            Y = psdp._empty_f(n, k, X.device)
            Y.fill_(float("nan"))
            assert _call(lib, "psdp_block_product", h, X, S, Y_ref, prec) == 0
            assert _call(lib, "psdp_block_product_noalloc", h, X, S, Y, prec) == 0
            torch.cuda.synchronize()
            a, b = Y_ref.cpu().numpy(), Y.cpu().numpy()
            assert np.isfinite(b).all()
            assert np.array_equal(a, b), float(np.abs(a - b).max())
        # beyond the static array: refused before any launch
        big = 3000
        Xb = psdp._empty_f(big, big, torch.device("cuda", 0))
        Sb = psdp._empty_f(big, 144, torch.device("cuda", 0))
        Yb = psdp._empty_f(big, 144, torch.device("cuda", 0))
        assert _call(lib, "psdp_block_product_noalloc", h, Xb, Sb, Yb, 0) == psdp.PSDP_ERR_CAPACITY
    finally:
        proj.close()
