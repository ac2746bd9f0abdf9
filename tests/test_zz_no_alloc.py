"""tdvp_heff_apply_noalloc (scratch in a static device array, no device
allocation) against tdvp_heff_apply on the same inputs: two calls in a row,
the second with smaller sizes, in FP64 and FP32; and a size beyond the
scratch maximum is rejected with TDVP_ERR_ARG."""
import ctypes as C

import numpy as np
import pytest

from paper_2005_06104_amd import inputs as I

pytestmark = pytest.mark.gpu


def _operands(torch, ml, wl, wr, mr, seed, dtype):
    L = torch.tensor(I.random_complex((ml, wl, ml), seed), dtype=dtype, device="cuda")
    Rt = torch.tensor(I.random_complex((wr, mr, mr), seed + 1), dtype=dtype, device="cuda")
    Cv = torch.tensor(I.random_complex((ml, 2, mr), seed + 2), dtype=dtype, device="cuda")
    W = I.random_mpo_site(wl, wr, seed + 3)
    return L, Rt, Cv, W


def test_noalloc_matches_allocating_entry_point():
    import torch
    from paper_2005_06104_amd import tdvp as T
    ctx = T.Context(0)
    try:
        for prec, dtype in (("fp64", torch.complex128), ("fp32", torch.complex64)):
            for (ml, wl, wr, mr, seed) in ((150, 8, 8, 130, 1), (37, 3, 5, 21, 2)):
                L, Rt, Cv, W = _operands(torch, ml, wl, wr, mr, seed, dtype)
                Y_ref = torch.empty_like(Cv)
                T.tdvp_heff_apply(ctx, W, L, Rt, Cv, Y_ref, prec=prec)
                torch.cuda.synchronize()
                Y = torch.full_like(Cv, float("nan"))
                n0 = torch.cuda.memory_stats()["allocation.all.allocated"]
                T.tdvp_heff_apply_noalloc(ctx, W, L, Rt, Cv, Y, prec=prec)
                torch.cuda.synchronize()
                assert torch.cuda.memory_stats()["allocation.all.allocated"] == n0   # nothing allocated
                # the same kernels on the same partition: identical results
                assert torch.equal(Y, Y_ref), (prec, ml, mr)
        # beyond the scratch maximum: rejected before any work
        L, Rt, Cv, W = _operands(torch, 600, 8, 8, 600, 3, torch.complex128)
        with pytest.raises(T.TdvpError) as ei:
            T.tdvp_heff_apply_noalloc(ctx, W, L, Rt, Cv, torch.empty_like(Cv))
        assert ei.value.status == T.TDVP_ERR_ARG
    finally:
        ctx.close()
