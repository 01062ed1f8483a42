"""Diagnostics of the equilibrium system on the GPU (Section 5.2, Tables
fd_poisson_fixedH, fd_shrinkingH and the Helmholtz block of fd_other_models):
unrestarted GMRES iteration counts at relative tolerance 1e-8 and
kappa_2(S_H) by power / inverse iteration, through the C-ABI, for the 3D
Poisson and constant-wavenumber Helmholtz problems on the unit cube.

Pins: kappa_2 against the separation-of-variables closed form (itself pinned
to both printed tables by the CPU tests) to 1e-8 relative, and against the
printed two-decimal values within 0.01 (the tables truncate some values,
8.9374 -> 8.93, and round others, 2.4499 -> 2.45); iteration counts against the printed ones within
+-3 (the paper does not state its right-hand side; seeded N(0,1) ones here).
The paper's grid has N = (1/h)^3 nodes: n = N^(1/3) - 1 interior nodes."""
import ctypes

import numpy as np
import pytest
import torch

from tests.golden.fixtures import paper_tables
from problems import Problem, make_config
from tests.test_oracle_pins import closed_form_kappa, mode_kappa

pytestmark = pytest.mark.gpu


def ddst():
    from paper_2510_25991_amd import ddst as mod
    return mod


def banner(msg):
    print(f"\n[gpu] {msg}", flush=True)


def rows():
    t = paper_tables()
    out = []
    for N, its, kap in t["fd_poisson_fixedH"]:
        out.append((round(N ** (1 / 3)) - 1, 8, its, kap))
    for hinv, its, kap in t["fd_shrinkingH"]:
        if hinv != 8:  # the H = 1/8 row of 64^3 is the table above's
            out.append((63, hinv, its, kap))
    return out


def check_row(n, n_slabs, its_paper, kap_paper, precision):
    ref = closed_form_kappa(n, n_slabs)
    kap = check_solves(Problem(3, n, n_slabs), precision, ref, lambda it: abs(it - its_paper) <= 3,
                       f"paper {its_paper}")
    assert abs(kap - kap_paper) < 0.01


def check_solves(p, precision, ref, its_ok, paper_note, indefinite=False, kap_tol=None):
    """GMRES on S for three seeded right-hand sides (true residual and the
    iteration-count check its_ok) and kappa_2(S) against the closed form ref;
    returns kappa_2."""
    dd = ddst()
    op = dd.Operator.from_problem(p, precision=precision, keep_factors=False,
                                  indefinite=indefinite)
    its = []
    for seed in range(3):
        b = torch.tensor(np.random.default_rng(seed).standard_normal(p.n_ds * op.M),
                         device="cuda")
        x, it, rr = op.gmres(b, tol=1e-8)
        assert rr <= 1e-8
        # the true residual of the returned solution
        res = op.apply(x.reshape(-1)).reshape(-1) - b
        assert float(res.norm() / b.norm()) <= 1.01e-8
        its.append(it)
    smax, smin, kap = op.cond_estimate()
    print(f"  GMRES iterations {its} ({paper_note}); kappa {kap:.8f} closed form {ref:.8f}; "
          f"pivot growth {op.build_stats()['pivot_growth']:.3e}")
    assert all(its_ok(it) for it in its)
    # FP32 blocks at m = 16 carry entry errors up to ~1e-4 relative (the
    # transfer-block tolerance), which move kappa_2 by ~6e-4 for Poisson and
    # by ~3e-3 for the near-resonant Helmholtz modes (N_lambda = 2)
    if kap_tol is None:
        kap_tol = 1e-8 if precision == "fp64" else 4e-3
    assert abs(kap - ref) <= kap_tol * ref
    op.close()
    return kap


@pytest.mark.parametrize("n,n_slabs,its_paper,kap_paper",
                         [r for r in rows() if r[0] <= 63])
def test_fd_poisson_tables(n, n_slabs, its_paper, kap_paper):
    banner(f"Poisson 3D n={n} H=1/{n_slabs}: iterations and kappa_2(S_H)")
    check_row(n, n_slabs, its_paper, kap_paper, "fp64")


def test_fd_poisson_fixedH_largest_row():
    n, n_slabs, its_paper, kap_paper = [r for r in rows() if r[0] == 127][0]
    banner(f"Poisson 3D n={n} H=1/{n_slabs} (FP32 blocks)")
    check_row(n, n_slabs, its_paper, kap_paper, "fp32")


def helmholtz(n, n_lambda):
    """-Laplace(u) - k^2 u, k = 2 pi N_lambda, H = 1/8 (Table fd_other_models)."""
    k2 = (2.0 * np.pi * n_lambda) ** 2
    return Problem(3, n, 8, c=-k2 * np.ones((n,) * 3)), k2


def check_helmholtz(n, n_lambda, precision, indefinite=False, kap_tol=None):
    """Iteration counts against the printed 128^3 ones within 15% (the
    right-hand side is not stated; observed 26 / 58-60 / 140-142 at
    32^3-64^3 and 25 / 67-68 / 140 at 128^3 against 27 / 61 / 141), kappa_2
    against the closed form."""
    its_paper = {r[0]: int(r[2]) for r in paper_tables()["fd_other_models_helmholtz"]}[n_lambda]
    p, k2 = helmholtz(n, n_lambda)
    check_solves(p, precision, closed_form_kappa(n, 8, k2),
                 lambda it: abs(it - its_paper) <= 0.15 * its_paper,
                 f"paper {its_paper} at 128^3", indefinite, kap_tol)


@pytest.mark.parametrize("n_lambda", [1, 2])
@pytest.mark.parametrize("n", [31, 63])
def test_fd_other_models_helmholtz(n, n_lambda):
    banner(f"Helmholtz 3D n={n} H=1/8 N_lambda={n_lambda}: iterations and kappa_2(S_H)")
    check_helmholtz(n, n_lambda, "fp64")


def test_fd_other_models_helmholtz_indefinite_rejected():
    """At N_lambda = 3, k^2 exceeds the lowest Dirichlet eigenvalue of a
    double slab 1/4 wide (about 177.6), so the local problems are indefinite
    and, by default, the elimination without pivoting reports them."""
    banner("Helmholtz 3D n=31 H=1/8 N_lambda=3: indefinite double slabs")
    dd = ddst()
    p, _ = helmholtz(31, 3)
    with pytest.raises(dd.DDSTError) as ei:
        dd.Operator.from_problem(p, precision="fp64", keep_factors=False)
    assert ei.value.code == dd.DDST_EBREAKDOWN


@pytest.mark.parametrize("n", [31, 63])
def test_fd_other_models_helmholtz_indefinite(n):
    """indefinite=True accepts negative pivots: the N_lambda = 3 row, with
    kappa_2 against the closed form (which holds for indefinite double slabs
    too, pinned on the CPU) and the iteration counts within 15% of the printed
    141 (at 128^3; 140-142 observed at 32^3 and 64^3)."""
    banner(f"Helmholtz 3D n={n} H=1/8 N_lambda=3 (indefinite local problems accepted)")
    dd = ddst()
    p, k2 = helmholtz(n, 3)
    op = dd.Operator.from_problem(p, precision="fp64", keep_factors=False, indefinite=True)
    its = []
    for seed in range(3):
        b = torch.tensor(np.random.default_rng(seed).standard_normal(p.n_ds * op.M),
                         device="cuda")
        x, it, rr = op.gmres(b, tol=1e-8)
        res = op.apply(x.reshape(-1)).reshape(-1) - b
        assert rr <= 1e-8 and float(res.norm() / b.norm()) <= 1.01e-8
        its.append(it)
    _, _, kap = op.cond_estimate()
    ref = closed_form_kappa(n, 8, k2)
    print(f"  GMRES iterations {its} (paper 141 at 128^3); kappa {kap:.8f} closed form {ref:.8f}; "
          f"pivot growth {op.build_stats()['pivot_growth']:.3e}")
    assert abs(kap - ref) <= 1e-7 * ref
    assert all(abs(it - 141) <= 0.15 * 141 for it in its)
    op.close()


def test_indefinite_solve_matches_global_direct():
    """The whole solve (FP32 blocks, FP64 refinement) of the N_lambda = 3
    Helmholtz problem with a seeded load against the oracle's sparse direct
    solve, and the adjoint gradient of a sensor loss against the oracle's."""
    from oracle import fd as ofd
    banner("indefinite Helmholtz 3D n=31 H=1/8: DD solve vs global direct")
    dd = ddst()
    p, _ = helmholtz(31, 3)
    p.f = np.random.default_rng(11).standard_normal((31,) * 3)
    ref = ofd.solve_global(p)
    op = dd.Operator.from_problem(p, precision="fp32", indefinite=True)
    u, _, st = op.solve(p.f)
    err = float(np.abs(u.cpu().numpy().ravel() - ref).max() / np.abs(ref).max())
    print(f"  rel err {err:.3e} outer {st['outer_iters']} gmres {st['gmres_iters']} "
          f"pivot growth {st['pivot_growth']:.3e}")
    assert st["status"] == 0 and err <= 1e-8
    # the adjoint recomputes the slab eliminations under the same sign rule
    from oracle import adjoint as oadj
    from problems import sensor_nodes
    sens = sensor_nodes(3, 31, 64, seed=1005)
    data = np.random.default_rng(1006).standard_normal(64) * 0.01
    gbar = oadj.sensor_loss_grad(ref, sens, data, p.N)
    gref, _ = oadj.gradient(p, ref, gbar)
    dk, sta = op.adjoint(u.reshape(-1), torch.tensor(gbar, device="cuda"))
    aerr = float(np.abs(dk.cpu().numpy().ravel() - gref.ravel()).max() / np.abs(gref).max())
    print(f"  adjoint rel err {aerr:.3e}")
    assert sta["status"] == 0 and aerr <= 1e-8
    op.close()


@pytest.mark.parametrize("dim,n,n_slabs,k2", [(2, 31, 4, (6 * np.pi) ** 2),
                                             (2, 255, 4, (20 * np.pi) ** 2),
                                             (3, 15, 4, (3 * np.pi) ** 2)])
def test_indefinite_transfer_blocks_match_oracle(dim, n, n_slabs, k2):
    """Transfer blocks (FP64) of shifted problems whose double slabs are past
    their first resonance, under indefinite=True, against the oracle's sparse
    local solves (which the CPU tests pin to the Chebyshev sine-basis form)."""
    from oracle import dd as odd
    banner(f"indefinite transfer blocks dim={dim} n={n} slabs={n_slabs} k^2={k2:.1f}")
    p = Problem(dim, n, n_slabs, c=-k2 * np.ones((n,) * dim))
    blocks = odd.DDOracle(p).all_blocks()
    scale = max(np.abs(B).max() for B in blocks.values())
    op = ddst().Operator.from_problem(p, precision="fp64", indefinite=True)
    worst = 0.0
    for j in range(1, p.n_ds + 1):
        SL, SR = (t.cpu().numpy() for t in op.transfer(j))
        refL = blocks.get((j, j - 1), np.zeros_like(SL))
        refR = blocks.get((j, j + 1), np.zeros_like(SR))
        worst = max(worst, np.abs(SL - refL).max() / scale, np.abs(SR - refR).max() / scale)
    print(f"  max rel block error {worst:.3e} pivot growth {op.build_stats()['pivot_growth']:.3e}")
    assert worst <= 1e-11  # the bar of the definite FP64 blocks; 6e-14-1.6e-12 observed
    # indefinite local problems keep the general elimination
    assert op.build_stats()["symmetric"] == 0
    op.close()


def singular_partial_slab_k2(n, k):
    """k^2 at which planes 1..k of a slab have a singular Schur complement
    for the lowest tangential mode (2D shifted Laplacian; pinned on the CPU
    by a dense Schur complement): z = cos(pi/(k+1)), z = 1 + (lambda_1 -
    k^2 h^2)/2."""
    h = 1.0 / (n + 1)
    return (4.0 * np.sin(np.pi * h / 2) ** 2 + 2.0 * (1.0 - np.cos(np.pi / (k + 1)))) / (h * h)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_singular_partial_slab_reported(precision):
    """k^2 ~ 401 on the 2D grid n = 31 with 4 slabs: the double slabs are
    nonsingular but the Schur complement of planes 1..4 of every slab is
    singular, and the elimination without pivoting would divide by a pivot
    of rounding size.  Under indefinite=True the FP64 build reports it as
    EBREAKDOWN through the pivot growth.  FP32 blocks round D_4 away from
    exact singularity by ~1e-7 ||A||: the build reports EBREAKDOWN (growth
    7e6 measured, limit 1e5), or builds with a pivot growth that shows it
    (>= 1e4, against <= 1e2 for the well-posed indefinite problems)."""
    dd = ddst()
    n = 31
    k2 = singular_partial_slab_k2(n, 4)
    banner(f"singular partial slab 2D n={n} 4 slabs k^2={k2:.4f} {precision}")
    p = Problem(2, n, 4, c=-k2 * np.ones((n, n)))
    try:
        op = dd.Operator.from_problem(p, precision=precision, indefinite=True)
    except dd.DDSTError as e:
        print(f"  EBREAKDOWN: {e}")
        assert e.code == dd.DDST_EBREAKDOWN
        return
    g = op.build_stats()["pivot_growth"]
    print(f"  built, pivot growth {g:.3e}")
    op.close()
    assert precision == "fp32", "the FP64 build must report the singular local problem"
    assert g >= 1e4


def test_indefinite_oscillatory_wide_slabs():
    """The 2D oscillatory workload (variable wavenumber, k^2 up to 3600) on
    four slabs of 48 cells: its double slabs are half the domain wide, far
    above their first resonance, and rejected by default; with indefinite=True
    the solve matches the oracle's global direct one."""
    from oracle import fd as ofd
    banner("oscillatory 2D n=191, 4 slabs: indefinite double slabs")
    dd = ddst()
    p = make_config("cfg3", n=191, n_slabs=4)
    with pytest.raises(dd.DDSTError) as ei:
        dd.Operator.from_problem(p, precision="fp32")
    assert ei.value.code == dd.DDST_EBREAKDOWN
    op = dd.Operator.from_problem(p, precision="fp32", indefinite=True)
    u, _, st = op.solve(p.f, opts=dd.SolveOptions(max_outer=20))
    ref = ofd.solve_global(p)
    err = float(np.abs(u.cpu().numpy().ravel() - ref).max() / np.abs(ref).max())
    print(f"  rel err {err:.3e} outer {st['outer_iters']} gmres {st['gmres_iters']} "
          f"pivot growth {st['pivot_growth']:.3e}")
    assert st["status"] == 0 and err <= 1e-8
    op.close()


@pytest.mark.parametrize("n_lambda,precision", [(1, "fp32"), (2, "fp64"), (3, "fp64")])
def test_fd_other_models_helmholtz_paper_size(n_lambda, precision):
    """The printed size.  N_lambda = 2 and 3 take FP64 blocks: their nearly
    resonant modes amplify the rounding of FP32 blocks (kappa_2 ~ 1.1e5 and
    2.7e5; FP32 blocks move it by 0.3% and 13%, and the iteration counts by
    10-15%); the estimate itself is good to a few 1e-6 there (inner GMRES at
    1e-12)."""
    banner(f"Helmholtz 3D n=127 H=1/8 N_lambda={n_lambda} ({precision} blocks)")
    if n_lambda == 3:
        check_helmholtz(127, 3, precision, indefinite=True, kap_tol=1e-5)
    else:
        check_helmholtz(127, n_lambda, precision, kap_tol=1e-5 if precision == "fp64" else None)


@pytest.mark.parametrize("n", [31, 63])
def test_fd_other_models_convection_diffusion(n):
    """Convection-diffusion block of Table fd_other_models (its velocity is
    not stated; b = (10, 0, 0) here): kappa_2 against the per-mode
    decomposition (pinned to the oracle on the CPU) and the iteration counts
    within 25% of the printed 20 (16-18 observed)."""
    banner(f"convection-diffusion 3D n={n} H=1/8 b=(10,0,0)")
    p = Problem(3, n, 8, bvec=(10.0, 0.0, 0.0))
    check_solves(p, "fp64", mode_kappa(n, 8, 0.0, 10.0), lambda it: abs(it - 20) <= 5,
                 "paper 20 for its unstated velocity")


@pytest.mark.parametrize("n", [31, 63])
def test_fd_other_models_variable_coefficient(n):
    """Variable-coefficient diffusion block of Table fd_other_models (its
    field is not stated; the 3D workload's log-normal field here): iteration
    counts within +-3 of the printed 19; kappa_2 has no closed form: at
    N = 32^3 it is checked against kappa_2 of the oracle's S (sparse local
    solves, about 15 s of CPU), at 64^3 only printed."""
    banner(f"variable-coefficient diffusion 3D n={n} H=1/8")
    p = make_config("cfg4", n=n, n_slabs=8)
    dd = ddst()
    op = dd.Operator.from_problem(p, precision="fp64", keep_factors=False)
    its = []
    for seed in range(3):
        b = torch.tensor(np.random.default_rng(seed).standard_normal(p.n_ds * op.M),
                         device="cuda")
        x, it, rr = op.gmres(b, tol=1e-8)
        res = op.apply(x.reshape(-1)).reshape(-1) - b
        assert float(res.norm() / b.norm()) <= 1.01e-8
        its.append(it)
    _, _, kap = op.cond_estimate()
    print(f"  GMRES iterations {its} (paper 19); kappa {kap:.8f}")
    assert all(abs(it - 19) <= 3 for it in its)
    op.close()
    if n == 31:
        from oracle import dd as odd
        from tests.test_oracle_pins import _kappa2
        ref = _kappa2(odd.DDOracle(p).assemble_S())
        print(f"  oracle kappa {ref:.8f}")
        assert abs(kap - ref) <= 1e-8 * ref


def test_gmres_forms_agree():
    """The same interface solve through the dense blocks, the matrix-free
    sweeps and the compressed form."""
    dd = ddst()
    p = Problem(3, 31, 8)
    banner("GMRES through dense, matrix-free and compressed S")
    op = dd.Operator.from_problem(p, precision="fp64")
    b = torch.tensor(np.random.default_rng(5).standard_normal(p.n_ds * op.M), device="cuda")
    xd, itd, _ = op.gmres(b, tol=1e-10)
    xm, itm, _ = op.gmres(b, tol=1e-10, which="matfree")
    op.compress(tol=1e-12, leaf=64, max_rank=100, factor_dtype="fp64")
    xh, ith, _ = op.gmres(b, tol=1e-10, which="hodlr")
    xt, itt, rt = op.gmres(b, tol=1e-10, transpose=True)
    rel = lambda a, c: float((a - c).abs().max() / c.abs().max())
    print(f"  iterations dense {itd} matrix-free {itm} compressed {ith} transposed {itt}; "
          f"matrix-free {rel(xm, xd):.2e} compressed {rel(xh, xd):.2e}")
    assert itm == itd and rel(xm, xd) <= 1e-12
    assert abs(ith - itd) <= 1 and rel(xh, xd) <= 1e-9
    res = op.apply(xt.reshape(-1), transpose=True).reshape(-1) - b
    assert float(res.norm() / b.norm()) <= 1.01e-10
    op.close()


def test_diagnostics_errors():
    dd = ddst()
    p = Problem(3, 15, 8)
    op = dd.Operator.from_problem(p, precision="fp64", transfer_blocks=False)
    b = torch.ones(p.n_ds * op.M, dtype=torch.float64, device="cuda")
    with pytest.raises(dd.DDSTError) as ei:
        op.gmres(b, tol=0.0, which="matfree")
    assert ei.value.code == dd.DDST_EINVAL
    with pytest.raises(dd.DDSTError) as ei:
        op.cond_estimate(which="dense")
    assert ei.value.code == dd.DDST_ESTATE
    # the matrix-free form serves the same diagnostics
    _, _, kap = op.cond_estimate(which="matfree")
    assert abs(kap - closed_form_kappa(15, 8)) <= 1e-8 * kap
    # the indefinite build option takes 0 or 1 only
    L = dd.load_library()
    h = ctypes.c_void_p()
    bad = dd.BuildOptsC(dd.FP64, 1, 0, 0, 2)
    code = L.ddst_build_transfer(ctypes.byref(op._prob), ctypes.byref(bad), dd._stream(),
                                 ctypes.byref(h))
    assert code == dd.DDST_EINVAL and not h.value
    op.close()
