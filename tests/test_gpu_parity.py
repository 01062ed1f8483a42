"""Parity of the HIP path (through the C-ABI) against the CPU FP64 oracle.

Tolerances (entries of transfer blocks are <= 1 in magnitude; errors are
measured as max |GPU - oracle| / max |oracle|):
* FP64 path: transfer blocks and loads 1e-11 -- Gauss-Jordan inversion of the
  well-conditioned plane blocks (condition number O(10)) loses a few
  hundred ulps over <= 64 planes;
* FP32 path: transfer blocks 1.5 eps32 m sqrt(M) for slabs of m cells and
  interfaces of M nodes (tests/tol.py: m - 1 inverted plane blocks per
  sweep, each with a relative error of order eps32 sqrt(M); observed
  0.15-0.55 of eps32 m sqrt(M));
* refined solutions: 1e-10 (FP64) and 1e-8 (mixed FP32 + FP64 refinement,
  the accuracy target of the method's mixed-precision form);
* adjoint gradients: 1e-8 vs the oracle's transposed sparse solve.
"""
import numpy as np
import pytest
import torch

from problems import Problem, make_config, sensor_nodes, fd_directions
from oracle import adjoint as oadj
from oracle import dd as odd
from oracle import fd as ofd
from tests.tol import fp32_block_tol as _fp32_block_tol

pytestmark = pytest.mark.gpu

_ORACLES = {}


def oracle(name, prob):
    if name not in _ORACLES:
        _ORACLES[name] = odd.DDOracle(prob)
    return _ORACLES[name]


def ddst():
    from paper_2510_25991_amd import ddst as mod
    return mod


CASES = {
    # name: (problem factory) -- sizes span several 128-tiles and ragged tails
    "cfg1": lambda: make_config("cfg1", variant=2),                 # 127^2, 8 slabs, M=127
    "cfg2s": lambda: make_config("cfg2", n=255, n_slabs=8),         # M=255 -> ld 256, m=32
    # Helmholtz, M=191, m=4: double slabs 1/24 wide keep the local problems
    # definite (lambda_min(-Laplace) ~ 24^2 pi^2 > k^2 = 3600), as in the full
    # 64-slab configuration
    "cfg3s": lambda: make_config("cfg3", n=191, n_slabs=48),
    "cfg4s": lambda: make_config("cfg4", n=23, n_slabs=4),          # 3D, M=529 -> ld 640, m=6
    "m2": lambda: make_config("cfg2", n=7, n_slabs=4),              # minimum slab width m=2
    "two_slabs": lambda: make_config("cfg2", n=15, n_slabs=2),      # one interface, no blocks
}
_PROBS = {}


def prob(name):
    if name not in _PROBS:
        _PROBS[name] = CASES[name]()
    return _PROBS[name]


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def banner(msg):
    print(f"\n[gpu] {msg}", flush=True)


def fp32_block_tol(p):
    return _fp32_block_tol(p.m, p.M)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["cfg1", "cfg2s", "cfg3s", "cfg4s", "m2"])
def test_transfer_blocks(name, precision):
    p = prob(name)
    tol = 1e-11 if precision == "fp64" else fp32_block_tol(p)
    banner(f"transfer blocks {name} n={p.n} slabs={p.n_slabs} {precision}")
    op = ddst().Operator.from_problem(p, precision=precision)
    o = oracle(name, p)
    blocks = o.all_blocks()
    scale = max(np.abs(B).max() for B in blocks.values())
    worst = 0.0
    for j in range(1, p.n_ds + 1):
        SL, SR = (t.cpu().numpy() for t in op.transfer(j))
        refL = blocks.get((j, j - 1), np.zeros_like(SL))
        refR = blocks.get((j, j + 1), np.zeros_like(SR))
        worst = max(worst, np.abs(SL - refL).max() / scale, np.abs(SR - refR).max() / scale)
    print(f"  max rel block error {worst:.3e}")
    assert worst <= tol
    op.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["cfg1", "cfg3s", "cfg4s"])
def test_symmetric_elimination_matches_general(name, precision):
    """Symmetric operators (no convection) are eliminated on the lower
    triangle only by default; the general elimination of the same operator
    and the oracle's blocks agree with it to the same bound, and the
    operator with convection keeps the general elimination."""
    p = prob(name)
    tol = 1e-11 if precision == "fp64" else fp32_block_tol(p)
    banner(f"symmetric vs general elimination {name} {precision}")
    dd = ddst()
    op_s = dd.Operator.from_problem(p, precision=precision)
    op_g = dd.Operator.from_problem(p, precision=precision, symmetric_elimination=False)
    assert op_s.build_stats()["symmetric"] == 1
    assert op_g.build_stats()["symmetric"] == 0
    blocks = oracle(name, p).all_blocks()
    scale = max(np.abs(B).max() for B in blocks.values())
    e_sym = e_gen = e_both = 0.0
    for j in range(1, p.n_ds + 1):
        a = [t.cpu().numpy() for t in op_s.transfer(j)]
        b = [t.cpu().numpy() for t in op_g.transfer(j)]
        for side, jp in ((0, j - 1), (1, j + 1)):
            ref = blocks.get((j, jp), np.zeros_like(a[side]))
            e_sym = max(e_sym, np.abs(a[side] - ref).max() / scale)
            e_gen = max(e_gen, np.abs(b[side] - ref).max() / scale)
            e_both = max(e_both, np.abs(a[side] - b[side]).max() / scale)
    print(f"  vs oracle: symmetric {e_sym:.3e}, general {e_gen:.3e}; between {e_both:.3e}")
    assert e_sym <= tol and e_gen <= tol and e_both <= 2 * tol
    # the interface inverses come out symmetric
    for j in (1, p.n_ds):
        Si = op_s.center_inverse(j).cpu().numpy()
        assert np.abs(Si - Si.T).max() <= tol * np.abs(Si).max()
    op_s.close()
    op_g.close()
    conv = dd.Operator.from_problem(prob("cfg2s"), precision=precision)
    assert conv.build_stats()["symmetric"] == 0
    conv.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["cfg2s", "cfg4s"])
def test_loads_and_apply(name, precision):
    p = prob(name)
    tol = 1e-11 if precision == "fp64" else fp32_block_tol(p)
    banner(f"loads/apply {name} {precision}")
    op = ddst().Operator.from_problem(p, precision=precision)
    o = oracle(name, p)
    hh = op.loads(p.f).cpu().numpy()
    ref = o.loads(o.rhs())
    print(f"  loads rel err {rel(hh, ref):.3e} (bound {tol:.1e})")
    assert rel(hh, ref) <= tol
    S = o.assemble_S()
    x = np.random.default_rng(11).standard_normal(S.shape[0])
    y = op.apply(torch.tensor(x, device="cuda")).cpu().numpy().ravel()
    yt = op.apply(torch.tensor(x, device="cuda"), transpose=True).cpu().numpy().ravel()
    assert rel(y, S @ x) <= tol
    assert rel(yt, S.T @ x) <= tol
    op.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-8)])
@pytest.mark.parametrize("name", ["cfg1", "cfg2s", "cfg3s", "cfg4s", "m2", "two_slabs"])
def test_solve_matches_global_direct(name, precision, tol):
    p = prob(name)
    banner(f"solve {name} {precision}")
    ref = ofd.solve_global(p)
    op = ddst().Operator.from_problem(p, precision=precision)
    # the oscillatory case needs many more Krylov iterations (its count is
    # reported, not pinned)
    opts = ddst().SolveOptions(max_iter=1000 if name == "cfg3s" else 300)
    u, ug, st = op.solve(p.f, p.g, opts=opts, allow_notconv=True)
    err = rel(u.cpu().numpy().ravel(), ref)
    o = oracle(name, p)
    gerr = rel(ug.cpu().numpy(), o.interface_trace(ref))
    print(f"  rel err {err:.3e} interface {gerr:.3e} outer {st['outer_iters']} "
          f"gmres {st['gmres_iters']} resid {st['residual_rel']:.2e} status {st['status']}")
    assert st["status"] == 0 and st["converged"] == 1
    assert err <= tol and gerr <= tol
    op.close()


def test_manufactured_cfg1_test1():
    p = make_config("cfg1", variant=1)
    banner("cfg1 manufactured exp(x) sin(y) fp32")
    op = ddst().Operator.from_problem(p, precision="fp32")
    u, _, st = op.solve(p.f, p.g)
    ref = ofd.solve_global(p)
    assert rel(u.cpu().numpy().ravel(), ref) <= 1e-8
    xn = np.arange(1, p.n + 1) / (p.n + 1)
    X, Y = np.meshgrid(xn, xn, indexing="ij")
    # O(h^2) discretisation error, about 6e-7 at h = 1/128
    assert np.abs(u.cpu().numpy() - np.exp(X) * np.sin(Y)).max() < 2e-6
    op.close()


def test_zero_rhs_gives_zero():
    p = prob("cfg2s")
    banner("zero right-hand side")
    op = ddst().Operator.from_problem(p, precision="fp32")
    u, ug, st = op.solve(np.zeros((p.n, p.n)))
    assert float(u.abs().max()) == 0.0
    op.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_adjoint_matches_oracle(precision):
    p = make_config("cfg5", n=127, n_slabs=4)
    banner(f"adjoint cfg5-shape n=127 {precision}")
    u_ref = ofd.solve_global(p)
    sens = sensor_nodes(2, p.n, 64, seed=1003)
    data = np.random.default_rng(1004).standard_normal(64) * 0.01
    gbar = oadj.sensor_loss_grad(u_ref, sens, data, p.N)
    gref, lref = oadj.gradient(p, u_ref, gbar)
    op = ddst().Operator.from_problem(p, precision=precision)
    u, _, _ = op.solve(p.f)
    dk, lam, st = op.adjoint(u.reshape(-1), torch.tensor(gbar, device="cuda"), want_lambda=True)
    print(f"  lambda err {rel(lam.cpu().numpy().ravel(), lref):.3e} "
          f"grad err {rel(dk.cpu().numpy(), gref):.3e}")
    assert rel(lam.cpu().numpy().ravel(), lref) <= 1e-8
    assert rel(dk.cpu().numpy(), gref) <= 1e-8
    # recomputed factors give the same gradient
    op.release_factors()
    dk2, st2 = op.adjoint(u.reshape(-1), torch.tensor(gbar, device="cuda"))
    assert rel(dk2.cpu().numpy(), gref) <= 1e-8
    op.close()


def test_adjoint_central_differences_gpu():
    """Central FD of the sensor loss along seeded directions, every solve on
    the GPU (FP64 path), against the autograd backward."""
    p = make_config("cfg5", n=63, n_slabs=4)
    banner("adjoint vs central differences n=63")
    dd = ddst()
    sens = torch.tensor(sensor_nodes(2, p.n, 32, seed=1003), device="cuda")
    kap = torch.tensor(p.kappa, device="cuda", requires_grad=True)
    f = torch.tensor(p.f, device="cuda")
    opts = dd.SolveOptions(tol=1e-13, max_outer=3)
    data = torch.zeros(32, dtype=torch.float64, device="cuda")

    def loss(k):
        u = dd.ddst_solve(k, f, p.n_slabs, bvec=p.bvec, precision="fp64", opts=opts)
        return 0.5 * ((u.reshape(-1)[sens] - data) ** 2).sum()

    L = loss(kap)
    L.backward()
    grad = kap.grad.detach().cpu().numpy()
    dirs = fd_directions(p.kappa.shape, 5, seed=1007)
    eps = 1e-5 * float(np.abs(p.kappa).max())
    with torch.no_grad():
        for v in dirs:
            vt = torch.tensor(v, device="cuda")
            lp = float(loss(kap.detach() + eps * vt))
            lm = float(loss(kap.detach() - eps * vt))
            fdv = (lp - lm) / (2 * eps)
            ad = float(np.sum(grad * v))
            assert abs(fdv - ad) <= 1e-5 * abs(ad), (fdv, ad)


def test_autograd_load_gradient_and_second_backward():
    """The autograd function returns dL/df = lambda = A^{-T} dL/du (f enters
    A u = f linearly) beside dL/dkappa, both against the oracle's transposed
    sparse solve, and a second backward over the same graph (retain_graph)
    gives the same gradients (the operator lives as long as the graph)."""
    p = make_config("cfg5", n=63, n_slabs=4)
    banner("autograd: dL/df and a second backward")
    dd = ddst()
    sens = sensor_nodes(2, p.n, 32, seed=1003)
    kap = torch.tensor(p.kappa, device="cuda", requires_grad=True)
    f = torch.tensor(p.f, device="cuda", requires_grad=True)
    opts = dd.SolveOptions(tol=1e-13, max_outer=3)
    u = dd.ddst_solve(kap, f, p.n_slabs, bvec=p.bvec, precision="fp64", opts=opts)
    st = torch.tensor(sens, device="cuda")
    L = 0.5 * (u.reshape(-1)[st] ** 2).sum()
    gk1, gf1 = torch.autograd.grad(L, (kap, f), retain_graph=True)
    gk2, gf2 = torch.autograd.grad(L, (kap, f))
    ref = ofd.solve_global(p)
    gbar = np.zeros(p.N)
    gbar[sens] = ref[sens]
    gref, lref = oadj.gradient(p, ref, gbar)
    ek = rel(gk1.cpu().numpy().ravel(), gref.ravel())
    ef = rel(gf1.cpu().numpy().ravel(), lref.ravel())
    print(f"  dL/dkappa rel err {ek:.3e}; dL/df rel err {ef:.3e}")
    assert ek <= 1e-8 and ef <= 1e-9
    assert rel(gk2.cpu().numpy(), gk1.cpu().numpy()) <= 1e-13
    assert rel(gf2.cpu().numpy(), gf1.cpu().numpy()) <= 1e-13


def test_errors_are_reported():
    dd = ddst()
    banner("error paths")
    with pytest.raises(dd.DDSTError) as e:
        dd.Operator(2, 16, 4)  # (n+1) % n_slabs != 0
    assert e.value.code == dd.DDST_EINVAL
    k = np.ones((16, 16))
    k[3, 4] = 0.0
    with pytest.raises(dd.DDSTError) as e:
        dd.Operator(2, 15, 4, kappa=k)
    assert e.value.code == dd.DDST_EINVAL
    c = np.zeros((15, 15))
    c[2, 2] = np.nan
    with pytest.raises(dd.DDSTError) as e:
        dd.Operator(2, 15, 4, c=c)
    assert e.value.code == dd.DDST_EINVAL
    # a zeroth-order term far beyond the local spectrum makes the plane blocks
    # indefinite: the first pivot is negative
    with pytest.raises(dd.DDSTError) as e:
        dd.Operator(2, 31, 2, c=-20000.0 * np.ones((31, 31)))
    assert e.value.code == dd.DDST_EBREAKDOWN
    # the Helmholtz workload on four wide slabs: double slabs half a unit wide
    # are locally resonant-side (k^2 above their lowest Dirichlet eigenvalue),
    # the degenerate local case the method must detect
    h3 = make_config("cfg3", n=191, n_slabs=4)
    with pytest.raises(dd.DDSTError) as e:
        dd.Operator.from_problem(h3, precision="fp32")
    assert e.value.code == dd.DDST_EBREAKDOWN
    # too few GMRES iterations: outputs written, status ENOTCONV
    p = prob("cfg2s")
    op = dd.Operator.from_problem(p, precision="fp64")
    u, _, st = op.solve(p.f, opts=dd.SolveOptions(max_iter=2, max_outer=1), allow_notconv=True)
    assert st["status"] == dd.DDST_ENOTCONV and bool(torch.isfinite(u).all())
    op.release_factors()
    with pytest.raises(dd.DDSTError) as e:
        op.solve(p.f)
    assert e.value.code == dd.DDST_ESTATE
    op.close()


def test_build_is_deterministic():
    p = prob("cfg2s")
    banner("determinism of the batched build")
    dd = ddst()
    a = dd.Operator.from_problem(p, precision="fp32")
    b = dd.Operator.from_problem(p, precision="fp32")
    for j in (1, 4, p.n_ds):
        for x, y in zip(a.transfer(j), b.transfer(j)):
            assert torch.equal(x, y)
    a.close()
    b.close()


def test_profiler_counts_and_union():
    """Per-class timing: every class timed, then the update class alone.  The
    launch counts follow the schedule (per matrix batch and elimination step:
    pivot + panel, and the two update parts, one launch on the last step),
    the union of a class's launch intervals never exceeds their sum, and a
    class left out is not timed."""
    p = prob("cfg2s")
    banner("profiler: launch counts, union of intervals, class selection")
    dd = ddst()
    dd.profile_enable(True)
    op = dd.Operator.from_problem(p, precision="fp32")
    torch.cuda.synchronize()
    pr = dd.profile_read()
    busy = dd.profile_busy()
    dd.profile_enable(False)
    op.close()
    steps = -(-p.M // 128)  # elimination steps per inversion
    ninv = (p.m - 1) + 1    # plane steps of the sweeps + the interface centres
    assert pr["gj_panel"][0] == ninv * 2 * steps
    assert pr["gj_update"][0] == ninv * (2 * (steps - 1) + 1)
    for k, (n, ms, work) in pr.items():
        if n:
            assert ms > 0 and work > 0
            # the union is built from float ms offsets against a common
            # origin: allow their rounding (well under 1 us per launch)
            assert 0 < busy[k] <= ms + n * 1e-3, (k, busy[k], ms)
    dd.profile_enable(True, kinds=["gj_update"])
    op = dd.Operator.from_problem(p, precision="fp32")
    torch.cuda.synchronize()
    pr2 = dd.profile_read()
    dd.profile_enable(False)
    op.close()
    assert pr2["gj_update"][0] == pr["gj_update"][0]
    assert all(pr2[k][0] == 0 for k in pr2 if k != "gj_update")


def test_full_size_cfg2_sampled():
    """The benchmarked workload at full size (1023^2, 32 slabs, FP32 build,
    FP64 refinement): two sampled transfer blocks and the full solution."""
    p = make_config("cfg2")
    banner("full-size cfg2 1023^2 32 slabs fp32")
    dd = ddst()
    op = dd.Operator.from_problem(p, precision="fp32")
    o = odd.DDOracle(p)
    for j in (1, 16):
        SL, SR = (t.cpu().numpy() for t in op.transfer(j))
        refR = o.transfer_block(j, j + 1)
        print(f"  block S_{j},{j+1} rel err {rel(SR, refR):.3e}")
        assert rel(SR, refR) <= fp32_block_tol(p)
        if j > 1:
            assert rel(SL, o.transfer_block(j, j - 1)) <= fp32_block_tol(p)
    u, _, st = op.solve(p.f, allow_notconv=True)
    ref = ofd.solve_global(p)
    err = rel(u.cpu().numpy().ravel(), ref)
    print(f"  full cfg2 rel err {err:.3e} outer {st['outer_iters']} gmres {st['gmres_iters']} "
          f"last {st['last_gmres_iters']} relres {st['gmres_relres']:.2e} corr "
          f"{st['correction_rel']:.2e} status {st['status']} build {st['t_build_ms']:.1f} ms "
          f"solve {st['t_solve_ms']:.1f} ms")
    assert st["status"] == 0
    assert err <= 1e-8
    op.close()
