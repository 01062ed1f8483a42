"""Many right-hand sides solved together (ddst_solve_many), through the C-ABI,
against the CPU FP64 oracle's global direct solves of each of them, and
against one-at-a-time solves on the GPU.

Tolerances: refined solutions 1e-10 (FP64 path) and 1e-8 (FP32 build +
FP64 refinement), as for single solves."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

from problems import make_config
from oracle import fd as ofd

pytestmark = pytest.mark.gpu

CASES = {
    "cfg1": lambda: make_config("cfg1", variant=2),              # 127^2, 8 slabs
    "cfg2s": lambda: make_config("cfg2", n=255, n_slabs=8),      # nonsymmetric, m=32
    "cfg4s": lambda: make_config("cfg4", n=23, n_slabs=4),       # 3D, M=529 -> ld 640
    "m2": lambda: make_config("cfg2", n=7, n_slabs=4),           # slab width m=2
    "two_slabs": lambda: make_config("cfg2", n=15, n_slabs=2),   # one interface
}
_PROBS = {}


def prob(name):
    if name not in _PROBS:
        _PROBS[name] = CASES[name]()
    return _PROBS[name]


def ddst():
    from paper_2510_25991_amd import ddst as mod
    return mod


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def banner(msg):
    print(f"\n[gpu] {msg}", flush=True)


def data(p, nrhs, seed):
    """Right-hand side 0 is the workload's own (f, g); the others are seeded
    N(0,1) loads with scaled copies of g (or zero boundary data)."""
    rng = np.random.default_rng(seed)
    shape = (p.n,) * p.dim
    f0 = p.f if p.f is not None else np.zeros(shape)
    F = np.stack([f0] + [rng.standard_normal(shape) for _ in range(nrhs - 1)])
    if p.g is None:
        return F, None
    G = np.stack([p.g] + [rng.uniform(-1, 1) * p.g for _ in range(nrhs - 1)])
    return F, G


def oracle_solutions(p, F, G):
    Ab = ofd.assemble(p)
    lu = spla.splu(Ab[0].tocsc())
    zero = np.zeros((p.n + 2,) * p.dim)
    return [lu.solve(ofd.rhs(p, Ab, f=F[v], g=zero if G is None else G[v]))
            for v in range(len(F))]


@pytest.mark.parametrize("name,precision,nrhs", [
    ("cfg2s", "fp32", 5), ("cfg2s", "fp64", 3), ("cfg1", "fp32", 9), ("cfg4s", "fp32", 4),
    ("cfg4s", "fp64", 2), ("m2", "fp32", 16), ("two_slabs", "fp64", 3)])
def test_solve_many_matches_oracle(name, precision, nrhs):
    p = prob(name)
    banner(f"solve_many {name} {precision} nrhs={nrhs}")
    tol = 1e-10 if precision == "fp64" else 1e-8
    dd = ddst()
    op = dd.Operator.from_problem(p, precision=precision)
    F, G = data(p, nrhs, seed=31)
    U, st = op.solve_many(F, G)
    refs = oracle_solutions(p, F, G)
    errs = [rel(U[v].cpu().numpy().ravel(), refs[v]) for v in range(nrhs)]
    _, _, st1 = op.solve(F[0], None if G is None else G[0])
    print(f"  max rel err {max(errs):.3e} outer {st['outer_iters']} gmres {st['gmres_iters']} "
          f"(one right-hand side: outer {st1['outer_iters']} gmres {st1['gmres_iters']})")
    assert st["status"] == 0 and st["converged"] == 1
    assert max(errs) <= tol
    op.close()


def test_solve_many_one_rhs_is_solve():
    p = prob("cfg2s")
    banner("solve_many with one right-hand side equals solve")
    dd = ddst()
    op = dd.Operator.from_problem(p, precision="fp32")
    u, _, st = op.solve(p.f, p.g)
    U, stm = op.solve_many(p.f[None], None if p.g is None else p.g[None])
    assert torch.equal(U[0], u)
    assert stm["gmres_iters"] == st["gmres_iters"]
    op.close()


def test_solve_many_zero_rhs_stays_zero():
    """A right-hand side of zeros among others: its block of every Krylov
    vector is zero, so its solution is exactly zero."""
    p = prob("cfg2s")
    banner("solve_many with a zero right-hand side")
    dd = ddst()
    op = dd.Operator.from_problem(p, precision="fp32")
    F, _ = data(p, 3, seed=32)
    F[1] = 0.0
    U, st = op.solve_many(F)
    assert float(U[1].abs().max()) == 0.0
    refs = oracle_solutions(p, F, None)
    assert rel(U[2].cpu().numpy().ravel(), refs[2]) <= 1e-8
    op.close()


@pytest.mark.parametrize("form", ["matfree", "hodlr"])
def test_solve_many_other_forms(form):
    p = prob("cfg2s")
    banner(f"solve_many through the {form} form")
    dd = ddst()
    op = dd.Operator.from_problem(p, precision="fp32")
    if form == "hodlr":
        op.compress(tol=1e-7, max_rank=100)
        opts = dd.SolveOptions(use_hodlr=True, max_outer=10)
    else:
        opts = dd.SolveOptions(matrix_free=True)
    F, G = data(p, 3, seed=33)
    U, st = op.solve_many(F, G, opts=opts)
    refs = oracle_solutions(p, F, G)
    errs = [rel(U[v].cpu().numpy().ravel(), refs[v]) for v in range(3)]
    print(f"  max rel err {max(errs):.3e} outer {st['outer_iters']} gmres {st['gmres_iters']}")
    assert st["status"] == 0 and max(errs) <= 1e-8
    op.close()


def test_solve_many_errors():
    import ctypes
    dd = ddst()
    p = prob("m2")
    op = dd.Operator.from_problem(p, precision="fp32")
    L = dd.load_library()
    U = torch.empty(17 * p.n ** 2, dtype=torch.float64, device="cuda")
    for nrhs in (0, dd.MAX_RHS + 1):
        code = L.ddst_solve_many(op._h, nrhs, None, None, None, ctypes.c_void_p(U.data_ptr()),
                                 None, None)
        assert code == dd.DDST_EINVAL
    op.close()


def test_solve_many_full_size_cfg2():
    """The benchmarked workload at full size (1023^2, 32 slabs, FP32 build):
    eight right-hand sides together; the workload's own against the oracle's
    global direct solve, all against one-at-a-time GPU solves."""
    p = make_config("cfg2")
    banner("solve_many full-size cfg2 1023^2 32 slabs fp32, 8 right-hand sides")
    dd = ddst()
    op = dd.Operator.from_problem(p, precision="fp32")
    F, _ = data(p, 8, seed=34)
    opts = dd.SolveOptions(tol=1e-9, max_outer=6)
    U, st = op.solve_many(F, opts=opts)
    worst = 0.0
    t_single = 0.0
    for v in range(8):
        u, _, s1 = op.solve(F[v], opts=opts)
        t_single += s1["t_solve_ms"]
        worst = max(worst, rel(U[v].cpu().numpy(), u.cpu().numpy()))
    ref = ofd.solve_global(p)
    err0 = rel(U[0].cpu().numpy().ravel(), ref)
    print(f"  together {st['t_solve_ms']:.1f} ms ({st['gmres_iters']} GMRES, "
          f"{st['outer_iters']} passes) vs one at a time {t_single:.1f} ms; "
          f"vs single solves {worst:.3e}, rhs 0 vs oracle {err0:.3e}")
    assert st["status"] == 0
    assert err0 <= 1e-8 and worst <= 2e-8
    op.close()
