"""The entry point that allocates nothing (mstab_project_noalloc) against the
one it varies (mstab_project): two calls in a row, the second on a smaller
input, both through the C ABI; results bit-identical (same kernel, same
grid, same order of sums) and within the rounding bound of P^T y."""
import ctypes
import math

import numpy as np
import pytest

from paper_1604_06043_amd import inputs as I

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def test_project_noalloc_matches_project():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1604_06043_amd import mstab
    lib = mstab.load()
    torch.cuda.set_device(0)
    for N, s, seed in ((2097152, 8, 3), (4097, 5, 1), (1, 1, 0)):
        print(f"[noalloc project N={N} s={s}]", flush=True)
        y = np.random.default_rng(seed).standard_normal(N)
        yd = torch.tensor(y, device="cuda")
        got = np.array(mstab.mstab_project_noalloc(yd, s, seed))
        ref = np.array(mstab.mstab_project(yd, s, seed))
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), (got, ref)
        P = I.p_dense(seed, N, s)
        exact = P.T @ y
        bound = 4 * math.log2(N + 2) * EPS * (np.abs(P).T @ np.abs(y))
        assert np.all(np.abs(got - exact) <= bound + 1e-300)
    # sizes beyond the maximum are refused before any launch
    out = (ctypes.c_double * 8)()
    st = lib.mstab_project_noalloc(1 << 29, 4, 0, ctypes.c_void_p(yd.data_ptr()),
                                   ctypes.cast(out, ctypes.c_void_p), None)
    assert st == mstab.E_INVALID
    assert b"2^29" in lib.mstab_last_error(None)
    st = lib.mstab_project_noalloc(10, 9, 0, ctypes.c_void_p(yd.data_ptr()),
                                   ctypes.cast(out, ctypes.c_void_p), None)
    assert st == mstab.E_INVALID
