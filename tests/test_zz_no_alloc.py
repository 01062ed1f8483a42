"""The allocation-free product (ddst_apply_noalloc) against ddst_apply.

Both run the same kernels on the same data (the allocation-free entry point
keeps its temporaries in a static per-GPU array), so their outputs agree to
the last bit up to the summation order, which is the same here: the bar is
1e-15 relative.  Two calls in a row, the second with a smaller operator, check
that nothing of the first call's contents leaks into the second; oversized
products are rejected with EINVAL.
"""
import numpy as np
import pytest
import torch

from problems import make_config

pytestmark = pytest.mark.gpu


def ddst():
    from paper_2510_25991_amd import ddst as mod
    return mod


def rel(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def check(op, seed, forms):
    g = torch.Generator(device="cuda").manual_seed(seed)
    x = torch.randn(op.n_ds * op.M, dtype=torch.float64, device="cuda", generator=g)
    for which in forms:
        for trans in (False, True):
            ref = op.apply(x, transpose=trans, which=which).reshape(-1)
            y = torch.full_like(x, float("nan"))
            op.apply_noalloc(x, y, transpose=trans, which=which)
            torch.cuda.synchronize()
            e = rel(y, ref)
            print(f"  {which} transpose={trans}: rel diff {e:.2e}", flush=True)
            assert e <= 1e-15


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_apply_matches_apply(precision):
    dd = ddst()
    big = make_config("cfg2", n=511, n_slabs=16)
    print(f"\n[gpu] no-alloc apply, {precision}: 511^2 16 slabs, then 127^2 8 slabs", flush=True)
    op1 = dd.Operator.from_problem(big, precision=precision)
    op1.compress(tol=1e-8, leaf=128, oversample=10, max_rank=64,
                 factor_dtype="fp32" if precision == "fp32" else "fp64")
    op1.compress_hbs(rank=16, factor_dtype="fp32" if precision == "fp32" else "fp64")
    check(op1, 1, ("dense", "hodlr", "hbs"))
    op1.close()
    small = make_config("cfg1", variant=2)
    op2 = dd.Operator.from_problem(small, precision=precision)
    op2.compress(tol=1e-8, leaf=32, oversample=10, max_rank=32,
                 factor_dtype="fp32" if precision == "fp32" else "fp64")
    check(op2, 2, ("dense", "hodlr"))
    op2.close()


def test_noalloc_rejects_oversized_and_other_forms():
    dd = ddst()
    print("\n[gpu] no-alloc apply: size limit and forms", flush=True)
    # 255 interfaces of 1023 nodes: the transposed dense product's partial
    # sums alone take 255 * 32 * 1024 * 8 bytes = 67 MB > 16 MiB
    p = make_config("cfg2", n=1023, n_slabs=256)
    op = dd.Operator.from_problem(p, precision="fp32")
    x = torch.zeros(op.n_ds * op.M, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    op.apply_noalloc(x, y, transpose=False)  # 2 * 255 * 1024 * 8 + jobs: fits
    with pytest.raises(dd.DDSTError) as e:
        op.apply_noalloc(x, y, transpose=True)
    assert e.value.code == dd.DDST_EINVAL
    L = dd.load_library()
    code = L.ddst_apply_noalloc(op._h, 0, dd.APPLY_MATFREE, dd._ptr(x), dd._ptr(y), dd._stream())
    assert code == dd.DDST_EINVAL
    code = L.ddst_apply_noalloc(op._h, 0, dd.APPLY_HODLR, dd._ptr(x), dd._ptr(y), dd._stream())
    assert code == dd.DDST_ESTATE  # not compressed
    op.close()
