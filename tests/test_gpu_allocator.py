"""Device memory from the caller's allocator (ddst_set_allocator), here
torch's caching allocator through the binding: every call gives the same
results as with hipMalloc, torch accounts for the library's memory while an
operator lives, and every block comes back when it is destroyed."""
import numpy as np
import pytest
import torch

from problems import make_config

pytestmark = pytest.mark.gpu


def ddst():
    from paper_2510_25991_amd import ddst as mod
    return mod


def run_all(dd, p):
    """Build, dense / matrix-free / compressed products, a solve and a
    two-right-hand-side solve; returns the outputs."""
    op = dd.Operator.from_problem(p, precision="fp32")
    x = torch.tensor(np.random.default_rng(41).standard_normal(p.n_ds * op.M), device="cuda")
    out = {"dense": op.apply(x), "matfree": op.apply(x, which="matfree")}
    out["u"], _, _ = op.solve(p.f)
    F = np.stack([p.f, 0.5 * p.f])
    out["U"], _ = op.solve_many(F)
    op.compress(tol=1e-6, max_rank=64)
    out["hodlr"] = op.apply(x, which="hodlr")
    held = torch.cuda.memory_allocated()
    op.close()
    return out, held


def test_torch_allocator_matches_hipmalloc():
    dd = ddst()
    p = make_config("cfg2", n=255, n_slabs=8)
    print("\n[gpu] allocator hooks: cfg2 255^2 8 slabs", flush=True)
    ref, _ = run_all(dd, p)
    base = torch.cuda.memory_allocated()
    dd.use_torch_allocator(True)
    try:
        got, held = run_all(dd, p)
        # the operator (transfer blocks, factors, compressed form, workspace)
        # was counted by torch while it lived, and nothing is left
        assert held - base > 50 * 2 ** 20
        assert dd.torch_allocator_blocks() == 0
        # what torch still holds beyond the base is the outputs of the calls
        outs = sum(-(-t.numel() * t.element_size() // 512) * 512 for t in got.values())
        assert torch.cuda.memory_allocated() - base <= outs
        # hooks cannot change while the library holds memory
        op = dd.Operator.from_problem(p, precision="fp32")
        with pytest.raises(dd.DDSTError) as ei:
            dd.use_torch_allocator(False)
        assert ei.value.code == dd.DDST_ESTATE
        op.close()
    finally:
        dd.use_torch_allocator(False)
    for k in ref:
        assert torch.equal(got[k], ref[k]), k
