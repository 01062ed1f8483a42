"""Matrix-free application of the equilibrium matrix S (Sections 2.2 and
5.1: S_{j,j+-1} applied by local solves with stored factors instead of formed
blocks), through the C-ABI, against the CPU FP64 oracle's dense S.

Tolerances as for the dense blocks (the matrix-free products use the same
stored plane factors): 1e-11 for FP64, max(1e-5, 4e-7 m^2) for FP32; refined
solutions 1e-10 (FP64) and 1e-8 (FP32 + FP64 refinement)."""
import numpy as np
import pytest
import torch

from tests.tol import fp32_block_tol

from problems import make_config, sensor_nodes
from oracle import adjoint as oadj
from oracle import dd as odd
from oracle import fd as ofd

pytestmark = pytest.mark.gpu

CASES = {
    "cfg1": lambda: make_config("cfg1", variant=2),              # 127^2, 8 slabs, m=16
    "cfg2s": lambda: make_config("cfg2", n=255, n_slabs=8),      # nonsymmetric, m=32
    "cfg4s": lambda: make_config("cfg4", n=23, n_slabs=4),       # 3D, M=529 -> ld 640
    "m2": lambda: make_config("cfg2", n=7, n_slabs=4),           # slab width m=2
    "three_slabs": lambda: make_config("cfg2", n=23, n_slabs=3),  # one slab with two chains
    "two_slabs": lambda: make_config("cfg2", n=15, n_slabs=2),   # no coupling: S = I
}
_PROBS, _ORACLES = {}, {}


def prob(name):
    if name not in _PROBS:
        _PROBS[name] = CASES[name]()
    return _PROBS[name]


def oracle(name):
    if name not in _ORACLES:
        _ORACLES[name] = odd.DDOracle(prob(name))
    return _ORACLES[name]


def ddst():
    from paper_2510_25991_amd import ddst as mod
    return mod


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def banner(msg):
    print(f"\n[gpu] {msg}", flush=True)


def block_tol(precision, m, M):
    return 1e-11 if precision == "fp64" else fp32_block_tol(m, M)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_matfree_apply_matches_oracle(name, precision):
    p = prob(name)
    banner(f"matrix-free apply {name} n={p.n} slabs={p.n_slabs} {precision}")
    op = ddst().Operator.from_problem(p, precision=precision)
    S = oracle(name).assemble_S()
    rng = np.random.default_rng(21)
    for trial in range(2):
        x = rng.standard_normal(S.shape[0])
        xd = torch.tensor(x, device="cuda")
        y = op.apply(xd, which="matfree").cpu().numpy().ravel()
        yt = op.apply(xd, transpose=True, which="matfree").cpu().numpy().ravel()
        e, et = rel(y, S @ x), rel(yt, S.T @ x)
        print(f"  trial {trial}: S x {e:.3e}  S^T x {et:.3e}")
        assert e <= block_tol(precision, p.m, p.M)
        assert et <= block_tol(precision, p.m, p.M)
    if p.n_ds == 1:
        assert np.array_equal(y, x)
    op.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-8)])
@pytest.mark.parametrize("name", list(CASES))
def test_matfree_solve_matches_global_direct(name, precision, tol):
    p = prob(name)
    banner(f"matrix-free solve {name} {precision}")
    ref = ofd.solve_global(p)
    dd = ddst()
    op = dd.Operator.from_problem(p, precision=precision)
    u, ug, st = op.solve(p.f, p.g, opts=dd.SolveOptions(matrix_free=True))
    ud, _, std = op.solve(p.f, p.g)
    err = rel(u.cpu().numpy().ravel(), ref)
    gerr = rel(ug.cpu().numpy(), oracle(name).interface_trace(ref))
    print(f"  rel err {err:.3e} interface {gerr:.3e} gmres {st['gmres_iters']} "
          f"(dense blocks: {std['gmres_iters']}) status {st['status']}")
    assert st["status"] == 0 and st["converged"] == 1
    assert err <= tol and gerr <= tol
    op.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_matfree_adjoint_matches_oracle(precision):
    p = make_config("cfg5", n=127, n_slabs=4)
    banner(f"matrix-free adjoint cfg5-shape n=127 {precision}")
    u_ref = ofd.solve_global(p)
    sens = sensor_nodes(2, p.n, 64, seed=1003)
    data = np.random.default_rng(1004).standard_normal(64) * 0.01
    gbar = oadj.sensor_loss_grad(u_ref, sens, data, p.N)
    gref, lref = oadj.gradient(p, u_ref, gbar)
    dd = ddst()
    op = dd.Operator.from_problem(p, precision=precision)
    opts = dd.SolveOptions(matrix_free=True)
    u, _, _ = op.solve(p.f, opts=opts)
    dk, lam, st = op.adjoint(u.reshape(-1), torch.tensor(gbar, device="cuda"), opts=opts,
                             want_lambda=True)
    print(f"  lambda err {rel(lam.cpu().numpy().ravel(), lref):.3e} "
          f"grad err {rel(dk.cpu().numpy(), gref):.3e}")
    assert rel(lam.cpu().numpy().ravel(), lref) <= 1e-8
    assert rel(dk.cpu().numpy(), gref) <= 1e-8
    # recomputed factors (the operator keeps none) serve the same chains
    op.release_factors()
    dk2, _ = op.adjoint(u.reshape(-1), torch.tensor(gbar, device="cuda"), opts=opts)
    assert rel(dk2.cpu().numpy(), gref) <= 1e-8
    op.close()


def test_matfree_errors():
    dd = ddst()
    p = prob("m2")
    op = dd.Operator.from_problem(p, precision="fp32")
    with pytest.raises(dd.DDSTError) as ei:
        op.solve(p.f, opts=dd.SolveOptions(matrix_free=True, use_hodlr=True))
    assert ei.value.code == dd.DDST_EINVAL
    with pytest.raises(ValueError):
        op.apply(torch.zeros(p.n_ds * op.M, dtype=torch.float64, device="cuda"), which="lu")
    op.release_factors()
    with pytest.raises(dd.DDSTError) as ei:
        op.apply(torch.zeros(p.n_ds * op.M, dtype=torch.float64, device="cuda"),
                 which="matfree")
    assert ei.value.code == dd.DDST_ESTATE
    op.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["cfg2s", "cfg4s", "m2", "two_slabs"])
def test_matfree_setup(name, precision):
    """The matrix-free set-up (no transfer chains, no blocks) holds the same
    slab factors and interface blocks as the full build: its matrix-free
    products are bit-identical, and its solves match the global direct one."""
    p = prob(name)
    banner(f"matrix-free set-up {name} {precision}")
    dd = ddst()
    full = dd.Operator.from_problem(p, precision=precision)
    op = dd.Operator.from_problem(p, precision=precision, transfer_blocks=False)
    x = torch.tensor(np.random.default_rng(22).standard_normal(p.n_ds * op.M), device="cuda")
    for trans in (False, True):
        a = op.apply(x, transpose=trans, which="matfree")
        b = full.apply(x, transpose=trans, which="matfree")
        assert torch.equal(a, b)
    _, _, st_full = full.solve(p.f, p.g)
    ref = ofd.solve_global(p)
    u, _, st = op.solve(p.f, p.g)
    err = rel(u.cpu().numpy().ravel(), ref)
    print(f"  rel err {err:.3e} gmres {st['gmres_iters']} build {st['t_build_ms']:.1f} ms "
          f"(with blocks {st_full['t_build_ms']:.1f} ms)")
    assert st["status"] == 0 and err <= (1e-10 if precision == "fp64" else 1e-8)
    assert st["bytes_transfer"] == 0 and st["bytes_factors"] == st_full["bytes_factors"]
    full.close()
    op.close()


def test_matfree_setup_errors():
    dd = ddst()
    p = prob("m2")
    with pytest.raises(dd.DDSTError) as ei:
        dd.Operator.from_problem(p, keep_factors=False, transfer_blocks=False)
    assert ei.value.code == dd.DDST_EINVAL
    op = dd.Operator.from_problem(p, transfer_blocks=False)
    x = torch.zeros(p.n_ds * op.M, dtype=torch.float64, device="cuda")
    for call in (lambda: op.apply(x, which="dense"), lambda: op.transfer(1),
                 lambda: op.compress()):
        with pytest.raises(dd.DDSTError) as ei:
            call()
        assert ei.value.code == dd.DDST_ESTATE
    op.close()


def test_matfree_full_size_cfg2():
    """The benchmarked workload at full size (1023^2, 32 slabs, FP32 factors):
    the matrix-free product against the dense blocks' product on every
    interface, and against the oracle's blocks on one interface."""
    p = make_config("cfg2")
    banner("matrix-free apply, full-size cfg2 1023^2 32 slabs fp32")
    dd = ddst()
    op = dd.Operator.from_problem(p, precision="fp32")
    rng = np.random.default_rng(23)
    x = rng.standard_normal(p.n_ds * op.M)
    xd = torch.tensor(x, device="cuda")
    tol = block_tol("fp32", p.m, p.M)
    for trans in (False, True):
        ym = op.apply(xd, transpose=trans, which="matfree").cpu().numpy()
        yd = op.apply(xd, transpose=trans, which="dense").cpu().numpy()
        print(f"  transpose={trans}: matrix-free vs dense {rel(ym, yd):.3e}")
        assert rel(ym, yd) <= 2 * tol
    ym = op.apply(xd, which="matfree").cpu().numpy()
    o = odd.DDOracle(p)
    j = 16
    X = x.reshape(p.n_ds, op.M)
    ref = (X[j - 1] - o.transfer_block(j, j - 1) @ X[j - 2]
           - o.transfer_block(j, j + 1) @ X[j])
    print(f"  interface {j} vs oracle blocks {rel(ym[j - 1], ref):.3e}")
    assert rel(ym[j - 1], ref) <= tol
    op.close()
