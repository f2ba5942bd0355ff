"""The FP64 matrix-core tile products (16x16x4 MFMA steps) used by the coarse
factorization, checked against numpy on the running GPU (operand layout)."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_tile_products(mode):
    from paper_2007_01941_amd import _lib
    rng = np.random.default_rng(mode)
    X, Y, C = (rng.normal(size=(16, 16)) for _ in range(3))
    t = [torch.as_tensor(a, device="cuda").contiguous() for a in (X, Y, C)]
    _lib.check(_lib.LIB.ba_selftest_tile_mma(ctypes.c_void_p(t[0].data_ptr()), ctypes.c_void_p(t[1].data_ptr()),
                                             ctypes.c_void_p(t[2].data_ptr()), mode,
                                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    got = t[2].cpu().numpy()
    ref = C + {0: X @ Y.T, 1: X.T @ Y, 2: X @ Y}[mode]
    print(f"[gpu] mode {mode}: max err {np.abs(got - ref).max():.2e}; transposed-layout err "
          f"{np.abs(got - (C + (ref - C).T)).max():.2e}", flush=True)
    if np.abs(got - ref).max() > 1e-12:
        np.set_printoptions(precision=3, linewidth=200)
        print("got - C:\n", got - C, "\nref - C:\n", ref - C, flush=True)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
