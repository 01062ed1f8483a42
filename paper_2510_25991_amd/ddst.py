"""ctypes binding of libddst (argument marshalling only).

Every step of the method runs in the HIP library; this module only passes
device pointers of torch tensors, sizes and the current HIP stream.  It
fails loudly when the library is not built or no GPU is present -- there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libddst.so")

DDST_OK, DDST_ENOTCONV = 0, 1
DDST_EINVAL, DDST_ENOMEM, DDST_EHIP, DDST_EBREAKDOWN, DDST_ERANK, DDST_ESTATE = -1, -2, -3, -4, -5, -6
FP64, FP32 = 0, 1
ELIM_AUTO, ELIM_GENERAL = 0, 1
TREE_BINARY, TREE_QUAD = 0, 1
FACTOR_BF16, FACTOR_FP32, FACTOR_FP64 = 0, 1, 2
APPLY_DENSE, APPLY_HODLR, APPLY_MATFREE, APPLY_HBS = 0, 1, 2, 3
MAX_RHS = 16
_APPLY_FORMS = {"dense": APPLY_DENSE, "hodlr": APPLY_HODLR, "matfree": APPLY_MATFREE,
                "hbs": APPLY_HBS}


class DDSTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ddst error {code}: {msg}")
        self.code = code


class ProblemC(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("n_slabs", ctypes.c_int32),
                ("kappa", ctypes.c_void_p), ("bvec", ctypes.c_double * 3),
                ("c", ctypes.c_void_p)]


class BuildOptsC(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("keep_factors", ctypes.c_int32),
                ("transpose", ctypes.c_int32), ("skip_transfer", ctypes.c_int32),
                ("indefinite", ctypes.c_int32), ("elimination", ctypes.c_int32)]


class CompressOptsC(ctypes.Structure):
    _fields_ = [("tree", ctypes.c_int32), ("leaf", ctypes.c_int32),
                ("oversample", ctypes.c_int32), ("max_rank", ctypes.c_int32),
                ("factor_dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tol", ctypes.c_double), ("seed", ctypes.c_uint64)]


class SolveOptsC(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("inner_tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("max_outer", ctypes.c_int32),
                ("use_hodlr", ctypes.c_int32), ("matrix_free", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("use_hbs", ctypes.c_int32),
                ("basis_fp32", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


class HbsOptsC(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("oversample", ctypes.c_int32),
                ("leaf", ctypes.c_int32), ("factor_dtype", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class StatsC(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("gmres_iters", ctypes.c_int32),
                ("last_gmres_iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("gmres_relres", ctypes.c_double), ("residual_rel", ctypes.c_double),
                ("correction_rel", ctypes.c_double), ("t_build_ms", ctypes.c_double),
                ("t_compress_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double),
                ("t_adjoint_ms", ctypes.c_double), ("bytes_factors", ctypes.c_double),
                ("bytes_transfer", ctypes.c_double), ("bytes_hodlr", ctypes.c_double),
                ("max_rank", ctypes.c_int32), ("min_rank", ctypes.c_int32),
                ("pivot_growth", ctypes.c_double), ("symmetric", ctypes.c_int32),
                ("reserved_", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["ddst_build_transfer", "ddst_compress", "ddst_solve", "ddst_solve_many", "ddst_adjoint",
           "ddst_release_factors", "ddst_destroy", "ddst_last_error", "ddst_op_info",
           "ddst_get_transfer", "ddst_apply", "ddst_loads", "ddst_get_factor",
           "ddst_get_center_inverse", "ddst_test_gemm", "ddst_test_invert",
           "ddst_test_invert_sym",
           "ddst_profile_enable", "ddst_profile_select", "ddst_profile_read",
           "ddst_profile_busy", "ddst_compress_info", "ddst_gmres", "ddst_cond_est",
           "ddst_set_allocator", "ddst_build_stats", "ddst_apply_noalloc",
           "ddst_compress_hbs", "ddst_hbs_info", "ddst_sample_blocks"]
KERNEL_CLASSES = {0: "gj_panel", 1: "gj_update", 2: "gemm", 3: "assemble", 4: "gemv",
                  5: "gemv_many"}

_lib = None

# device allocator hooks (ddst_set_allocator): blocks from torch's caching
# allocator, kept alive here until the library frees them
_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_torch_blocks = {}


def _torch_alloc(nbytes, ctx):
    try:
        t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    except RuntimeError:
        return None  # NULL: the library reports ENOMEM
    _torch_blocks[t.data_ptr()] = t
    return t.data_ptr()


def _torch_free(ptr, ctx):
    _torch_blocks.pop(ptr, None)


_ALLOC_CB = _ALLOC_T(_torch_alloc)
_FREE_CB = _FREE_T(_torch_free)


def use_torch_allocator(on: bool = True):
    """Take the library's device memory from torch's caching allocator (on)
    or from hipMalloc again (off).  Call while no Operator exists."""
    L = load_library()
    if on:
        _check(L.ddst_set_allocator(_ALLOC_CB, _FREE_CB, None))
    else:
        _check(L.ddst_set_allocator(_ALLOC_T(), _FREE_T(), None))


def torch_allocator_blocks() -> int:
    """Library blocks currently held from torch's allocator."""
    return len(_torch_blocks)


def load_library(path: str = _LIB_PATH):
    """Load libddst.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2510_25991_amd.build_lib.build()")
    L = ctypes.CDLL(path)
    vp, i32, P = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER
    L.ddst_build_transfer.argtypes = [P(ProblemC), P(BuildOptsC), vp, P(vp)]
    L.ddst_compress.argtypes = [vp, P(CompressOptsC), vp]
    L.ddst_compress_hbs.argtypes = [vp, P(HbsOptsC), vp, vp, vp]
    L.ddst_hbs_info.argtypes = [vp, P(ctypes.c_double), P(i32), P(ctypes.c_double),
                                P(ctypes.c_double)]
    L.ddst_sample_blocks.argtypes = [vp, i32, vp, vp, vp, vp]
    L.ddst_solve.argtypes = [vp, vp, vp, P(SolveOptsC), vp, vp, P(StatsC), vp]
    L.ddst_solve_many.argtypes = [vp, i32, vp, vp, P(SolveOptsC), vp, P(StatsC), vp]
    L.ddst_set_allocator.argtypes = [_ALLOC_T, _FREE_T, vp]
    L.ddst_gmres.argtypes = [vp, i32, i32, vp, vp, ctypes.c_double, i32, P(i32),
                             P(ctypes.c_double), vp]
    L.ddst_cond_est.argtypes = [vp, i32, i32, ctypes.c_double, ctypes.c_double,
                                P(ctypes.c_double), P(ctypes.c_double), P(i32), vp]
    L.ddst_adjoint.argtypes = [vp, vp, vp, vp, P(SolveOptsC), vp, vp, P(StatsC), vp]
    L.ddst_release_factors.argtypes = [vp]
    L.ddst_destroy.argtypes = [vp]
    L.ddst_destroy.restype = None
    L.ddst_last_error.argtypes = []
    L.ddst_last_error.restype = ctypes.c_char_p
    L.ddst_op_info.argtypes = [vp, P(i32), P(i32), P(i32), P(i32)]
    L.ddst_build_stats.argtypes = [vp, P(StatsC)]
    L.ddst_get_transfer.argtypes = [vp, i32, vp, vp, vp]
    L.ddst_apply.argtypes = [vp, i32, i32, vp, vp, vp]
    L.ddst_apply_noalloc.argtypes = [vp, i32, i32, vp, vp, vp]
    L.ddst_loads.argtypes = [vp, vp, vp, vp, vp]
    L.ddst_get_factor.argtypes = [vp, i32, i32, vp, vp]
    L.ddst_get_center_inverse.argtypes = [vp, i32, vp, vp]
    L.ddst_test_gemm.argtypes = [i32, i32, i32, vp, vp, vp, vp, ctypes.c_double,
                                 ctypes.c_double, vp]
    L.ddst_test_invert.argtypes = [i32, i32, i32, vp, vp]
    L.ddst_test_invert_sym.argtypes = [i32, i32, i32, vp, vp]
    L.ddst_compress_info.argtypes = [vp, P(ctypes.c_double), P(i32), P(i32),
                                     P(ctypes.c_double)]
    L.ddst_profile_enable.argtypes = [i32]
    L.ddst_profile_select.argtypes = [ctypes.c_uint32]
    L.ddst_profile_busy.argtypes = [i32, P(ctypes.c_double)]
    L.ddst_profile_read.argtypes = [i32, P(ctypes.c_int64), P(ctypes.c_double),
                                    P(ctypes.c_double)]
    for name in EXPORTS:
        fn = getattr(L, name)
        if name not in ("ddst_destroy", "ddst_last_error"):
            fn.restype = ctypes.c_int
    _lib = L
    return L


def _check(code, allow_notconv=False):
    if code == DDST_OK or (allow_notconv and code == DDST_ENOTCONV):
        return code
    raise DDSTError(code, load_library().ddst_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _dev(x, device="cuda"):
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(x, dtype=torch.float64, device=device).contiguous()


@dataclasses.dataclass
class SolveOptions:
    tol: float = 1e-10
    inner_tol: Optional[float] = None      # default: 1e-4 (FP32), 1e-12 (FP64)
    max_iter: int = 300
    max_outer: int = 4
    use_hodlr: bool = False
    matrix_free: bool = False              # apply S by sweeps with the stored factors
    restart: int = 0                       # 0: unrestarted GMRES; k: restart every k
    use_hbs: bool = False                  # apply S through the sampled HBS form
    basis_fp32: bool = False               # FP32 Krylov basis for passes at tol >= 1e-6


class Operator:
    """A built equilibrium operator (transfer blocks + slab factors) on the GPU."""

    def __init__(self, dim, n, n_slabs, kappa=None, bvec=(0.0, 0.0, 0.0), c=None,
                 precision: str = "fp32", keep_factors: bool = True,
                 transfer_blocks: bool = True, indefinite: bool = False,
                 symmetric_elimination: bool = True):
        """transfer_blocks=False: the matrix-free set-up (slab factors and
        interface blocks only); solves then apply S matrix-free.
        indefinite=True: accept negative pivots (indefinite, nonsingular local
        problems); by default they are reported as DDST_EBREAKDOWN.
        symmetric_elimination=False: the general elimination even when the
        operator is symmetric (no convection)."""
        if not torch.cuda.is_available():
            raise RuntimeError("ddst needs a ROCm GPU; no device is visible")
        L = load_library()
        self.dim, self.n, self.n_slabs = int(dim), int(n), int(n_slabs)
        self.precision = precision
        self._kappa = _dev(kappa)
        self._c = _dev(c)
        b = list(bvec) + [0.0] * 3
        self._prob = ProblemC(self.dim, self.n, self.n_slabs, _ptr(self._kappa),
                              (ctypes.c_double * 3)(*[float(v) for v in b[:3]]), _ptr(self._c))
        self.transfer_blocks = bool(transfer_blocks)
        opts = BuildOptsC(FP32 if precision == "fp32" else FP64, 1 if keep_factors else 0, 0,
                          0 if transfer_blocks else 1, 1 if indefinite else 0,
                          ELIM_AUTO if symmetric_elimination else ELIM_GENERAL)
        h = ctypes.c_void_p()
        _check(L.ddst_build_transfer(ctypes.byref(self._prob), ctypes.byref(opts), _stream(),
                                     ctypes.byref(h)))
        self._h = h
        M, nds, ld, pr = (ctypes.c_int32() for _ in range(4))
        _check(L.ddst_op_info(self._h, ctypes.byref(M), ctypes.byref(nds), ctypes.byref(ld),
                              ctypes.byref(pr)))
        self.M, self.n_ds, self.ld = M.value, nds.value, ld.value

    @classmethod
    def from_problem(cls, prob, precision="fp32", keep_factors=True, transfer_blocks=True,
                     indefinite=False, symmetric_elimination=True):
        return cls(prob.dim, prob.n, prob.n_slabs, kappa=prob.kappa, bvec=prob.bvec, c=prob.c,
                   precision=precision, keep_factors=keep_factors,
                   transfer_blocks=transfer_blocks, indefinite=indefinite,
                   symmetric_elimination=symmetric_elimination)

    # -- lifetime --------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().ddst_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_stats(self):
        """Build figures (times, storage, ranks, pivot growth) as a dict."""
        st = StatsC()
        _check(load_library().ddst_build_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def release_factors(self):
        _check(load_library().ddst_release_factors(self._h))

    # -- operations --------------------------------------------------------
    def _solve_opts(self, opts: Optional[SolveOptions]):
        o = opts or SolveOptions()
        inner = o.inner_tol if o.inner_tol is not None else (1e-4 if self.precision == "fp32" else 1e-12)
        # an operator without transfer blocks applies S matrix-free
        mf = o.matrix_free or not (self.transfer_blocks or o.use_hodlr or o.use_hbs)
        return SolveOptsC(o.tol, inner, o.max_iter, o.max_outer, 1 if o.use_hodlr else 0,
                          1 if mf else 0, int(o.restart), 1 if o.use_hbs else 0,
                          1 if o.basis_fp32 else 0, 0)

    def solve(self, f=None, g=None, opts: Optional[SolveOptions] = None, want_gamma=True,
              allow_notconv=False):
        """Returns (u_vol (n,)*dim, u_gamma (n_ds, M), stats dict)."""
        f, g = _dev(f), _dev(g)
        N = self.n ** self.dim
        u = torch.empty(N, dtype=torch.float64, device="cuda")
        ug = torch.empty(self.n_ds * self.M, dtype=torch.float64, device="cuda") if want_gamma else None
        st = StatsC()
        o = self._solve_opts(opts)
        code = load_library().ddst_solve(self._h, _ptr(f), _ptr(g), ctypes.byref(o), _ptr(ug),
                                         _ptr(u), ctypes.byref(st), _stream())
        _check(code, allow_notconv)
        d = st.as_dict()
        d["status"] = code
        return (u.view((self.n,) * self.dim),
                None if ug is None else ug.view(self.n_ds, self.M), d)

    def solve_many(self, F, G=None, opts: Optional[SolveOptions] = None, allow_notconv=False):
        """Solves for nrhs right-hand sides at once: F (nrhs, n, ...) loads,
        G (nrhs, n+2, ...) boundary boxes or None.  Returns (U (nrhs, n, ...),
        stats dict)."""
        F = _dev(F)
        G = _dev(G)
        nrhs = int(F.shape[0])
        N = self.n ** self.dim
        U = torch.empty(nrhs * N, dtype=torch.float64, device="cuda")
        st = StatsC()
        o = self._solve_opts(opts)
        code = load_library().ddst_solve_many(self._h, nrhs, _ptr(F), _ptr(G), ctypes.byref(o),
                                              _ptr(U), ctypes.byref(st), _stream())
        _check(code, allow_notconv)
        d = st.as_dict()
        d["status"] = code
        return U.view((nrhs,) + (self.n,) * self.dim), d

    def adjoint(self, u, gbar, g=None, opts: Optional[SolveOptions] = None, want_lambda=False,
                allow_notconv=False):
        """dL/dkappa on the (n+1)^dim cells for dL/du = gbar."""
        u, gbar, g = _dev(u), _dev(gbar), _dev(g)
        dk = torch.empty((self.n + 1) ** self.dim, dtype=torch.float64, device="cuda")
        lam = torch.empty(self.n ** self.dim, dtype=torch.float64, device="cuda") if want_lambda else None
        st = StatsC()
        o = self._solve_opts(opts)
        code = load_library().ddst_adjoint(self._h, _ptr(u), _ptr(g), _ptr(gbar), ctypes.byref(o),
                                           _ptr(dk), _ptr(lam), ctypes.byref(st), _stream())
        _check(code, allow_notconv)
        d = st.as_dict()
        d["status"] = code
        dk = dk.view((self.n + 1,) * self.dim)
        if want_lambda:
            return dk, lam.view((self.n,) * self.dim), d
        return dk, d

    def transfer(self, j):
        """(S_{j,j-1}, S_{j,j+1}) as float64 M x M tensors (zeros if absent)."""
        a = torch.empty(self.M, self.M, dtype=torch.float64, device="cuda")
        b = torch.empty(self.M, self.M, dtype=torch.float64, device="cuda")
        _check(load_library().ddst_get_transfer(self._h, int(j), _ptr(a), _ptr(b), _stream()))
        return a, b

    def factor(self, slab, k):
        """G_k of the left-to-right elimination of single slab `slab`."""
        out = torch.empty(self.M, self.M, dtype=torch.float64, device="cuda")
        _check(load_library().ddst_get_factor(self._h, int(slab), int(k), _ptr(out), _stream()))
        return out

    def center_inverse(self, j):
        out = torch.empty(self.M, self.M, dtype=torch.float64, device="cuda")
        _check(load_library().ddst_get_center_inverse(self._h, int(j), _ptr(out), _stream()))
        return out

    def apply(self, x, transpose=False, which="dense"):
        """y = S x (or S^T x); which: "dense", "hodlr" or "matfree"."""
        if which not in _APPLY_FORMS:
            raise ValueError(f"which must be one of {sorted(_APPLY_FORMS)}")
        x = _dev(x).reshape(-1)
        y = torch.empty_like(x)
        _check(load_library().ddst_apply(self._h, 1 if transpose else 0, _APPLY_FORMS[which],
                                         _ptr(x), _ptr(y), _stream()))
        return y.view(self.n_ds, self.M)

    def apply_noalloc(self, x, y, transpose=False, which="dense"):
        """y = S x (or S^T x) into the caller's y (N_ds*M float64) without any
        allocation in the library; which: "dense", "hodlr" or "hbs"."""
        if which not in ("dense", "hodlr", "hbs"):
            raise ValueError("which must be 'dense', 'hodlr' or 'hbs'")
        _check(load_library().ddst_apply_noalloc(self._h, 1 if transpose else 0,
                                                 _APPLY_FORMS[which], _ptr(x), _ptr(y),
                                                 _stream()))
        return y

    def gmres(self, b, tol=1e-8, max_iter=1000, which="dense", transpose=False,
              allow_notconv=False):
        """x = S^{-1} b (or S^{-T} b) by unrestarted GMRES from zero; returns
        (x (n_ds, M), iterations, relative residual)."""
        if which not in _APPLY_FORMS:
            raise ValueError(f"which must be one of {sorted(_APPLY_FORMS)}")
        b = _dev(b).reshape(-1)
        x = torch.empty_like(b)
        it, rr = ctypes.c_int32(), ctypes.c_double()
        code = load_library().ddst_gmres(self._h, 1 if transpose else 0, _APPLY_FORMS[which],
                                         _ptr(b), _ptr(x), float(tol), int(max_iter),
                                         ctypes.byref(it), ctypes.byref(rr), _stream())
        _check(code, allow_notconv)
        return x.view(self.n_ds, self.M), it.value, rr.value

    def cond_estimate(self, which="dense", max_iter=500, tol=1e-10, gmres_tol=1e-12):
        """(sigma_max, sigma_min, kappa_2) of S by power and inverse iteration."""
        smax, smin, it = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        _check(load_library().ddst_cond_est(self._h, _APPLY_FORMS[which], int(max_iter),
                                            float(tol), float(gmres_tol), ctypes.byref(smax),
                                            ctypes.byref(smin), ctypes.byref(it), _stream()))
        return smax.value, smin.value, smax.value / smin.value

    def loads(self, f=None, g=None):
        f, g = _dev(f), _dev(g)
        out = torch.empty(self.n_ds * self.M, dtype=torch.float64, device="cuda")
        _check(load_library().ddst_loads(self._h, _ptr(f), _ptr(g), _ptr(out), _stream()))
        return out.view(self.n_ds, self.M)

    def compress(self, tol=1e-8, leaf=128, oversample=10, max_rank=112, tree=None,
                 factor_dtype="bf16", seed=0):
        tree = (TREE_BINARY if self.dim == 2 else TREE_QUAD) if tree is None else tree
        fd = {"bf16": FACTOR_BF16, "fp32": FACTOR_FP32, "fp64": FACTOR_FP64}[factor_dtype]
        o = CompressOptsC(tree, leaf, oversample, max_rank, fd, 0, tol, seed)
        _check(load_library().ddst_compress(self._h, ctypes.byref(o), _stream()))
        return self.compress_info()

    def compress_hbs(self, rank=64, oversample=10, leaf=0, factor_dtype="bf16", seed=0,
                     omega=None, psi=None):
        """Sampled HBS form of every transfer block (s = 3 rank + oversample
        probes per side, from omega / psi (M x s) if given, else drawn)."""
        fd = {"bf16": FACTOR_BF16, "fp32": FACTOR_FP32, "fp64": FACTOR_FP64}[factor_dtype]
        o = HbsOptsC(int(rank), int(oversample), int(leaf), fd, int(seed))
        om, ps = _dev(omega), _dev(psi)
        _check(load_library().ddst_compress_hbs(self._h, ctypes.byref(o), _ptr(om), _ptr(ps),
                                                _stream()))
        return self.hbs_info()

    def hbs_info(self):
        b, k, t1, t2 = ctypes.c_double(), ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
        _check(load_library().ddst_hbs_info(self._h, ctypes.byref(b), ctypes.byref(k),
                                            ctypes.byref(t1), ctypes.byref(t2)))
        return {"bytes": b.value, "rank": k.value, "sample_ms": t1.value, "compress_ms": t2.value}

    def sample_blocks(self, X):
        """(Y, Z): Y[b] = S_b X, Z[b] = S_b^T X for the 2 (N_ds - 1) transfer
        blocks (S_{s+1,s} at 2 (s - 1), S_{s,s+1} at 2 (s - 1) + 1), by the
        sampling chains."""
        X = _dev(X)
        ncols = int(X.shape[1])
        nb = 2 * max(self.n_ds - 1, 0)
        Y = torch.empty(max(nb, 1), self.M, ncols, dtype=torch.float64, device="cuda")
        Z = torch.empty_like(Y)
        _check(load_library().ddst_sample_blocks(self._h, ncols, _ptr(X), _ptr(Y), _ptr(Z),
                                                 _stream()))
        return Y[:nb], Z[:nb]

    def compress_info(self):
        b, mx, mn, ms = ctypes.c_double(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(load_library().ddst_compress_info(self._h, ctypes.byref(b), ctypes.byref(mx),
                                                 ctypes.byref(mn), ctypes.byref(ms)))
        return {"bytes": b.value, "max_rank": mx.value, "min_rank": mn.value, "ms": ms.value}


def _raw_ptr(t):
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("expected a contiguous CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def kernel_gemm(A, B, C, bscale=None, alpha=1.0, beta=0.0):
    """Batched C = alpha A diag(s) B + beta C with the build's MFMA kernel
    (A, B, C: (batch, ld, ld) float32 or float64 CUDA tensors, in place)."""
    prec = FP32 if A.dtype == torch.float32 else FP64
    batch, ld, _ = A.shape
    _check(load_library().ddst_test_gemm(prec, ld, batch, _raw_ptr(A), _raw_ptr(B), _raw_ptr(C),
                                         None if bscale is None else _raw_ptr(bscale),
                                         float(alpha), float(beta), _stream()))
    return C


def kernel_invert(A, symmetric=False):
    """In-place batched Gauss-Jordan inversion with the build's kernels
    (symmetric=True: the symmetric elimination, which reads only the lower
    triangle of each A_b)."""
    prec = FP32 if A.dtype == torch.float32 else FP64
    batch, ld, _ = A.shape
    f = load_library().ddst_test_invert_sym if symmetric else load_library().ddst_test_invert
    _check(f(prec, ld, batch, _raw_ptr(A), _stream()))
    return A


def profile_enable(on=True, kinds=None):
    """Start (clearing the counters) or stop per-launch timing; `kinds`
    restricts it to the named classes (names of KERNEL_CLASSES)."""
    if kinds is None or not on:
        _check(load_library().ddst_profile_enable(1 if on else 0))
        return
    ids = {v: k for k, v in KERNEL_CLASSES.items()}
    mask = 0
    for name in kinds:
        mask |= 1 << ids[name]
    _check(load_library().ddst_profile_select(mask))


def profile_read():
    """{class name: (launches, total ms, algorithmic work)}."""
    out = {}
    L = load_library()
    for k, name in KERNEL_CLASSES.items():
        n, ms, w = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(L.ddst_profile_read(k, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(w)))
        out[name] = (n.value, ms.value, w.value)
    return out


def profile_busy():
    """{class name: union of its launch intervals in ms}."""
    out = {}
    L = load_library()
    for k, name in KERNEL_CLASSES.items():
        b = ctypes.c_double()
        _check(L.ddst_profile_busy(k, ctypes.byref(b)))
        out[name] = b.value
    return out


class DDSTSolve(torch.autograd.Function):
    """u = A(kappa)^{-1} f through the DD solver; backward by the hand-written
    adjoint, which recomputes the slab factors (they are dropped after the
    forward solve to keep memory at the transfer blocks only).

    Gradients: dL/dkappa from the adjoint solution lambda = A^{-T} dL/du and
    the solution, and dL/df = lambda itself (f enters A u = f linearly).  The
    operator stays alive as long as the autograd graph does (it is released
    with the context), so backward may run more than once (retain_graph)."""

    @staticmethod
    def forward(ctx, kappa, f, n_slabs, bvec, g, precision, opts, indefinite=False):
        dim = kappa.dim()
        n = kappa.shape[0] - 1
        op = Operator(dim, n, n_slabs, kappa=kappa.detach(), bvec=bvec, precision=precision,
                      indefinite=indefinite)
        u, _, st = op.solve(f.detach(), g, opts=opts, want_gamma=False)
        op.release_factors()
        ctx.op, ctx.g, ctx.opts = op, g, opts
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, gbar):
        (u,) = ctx.saved_tensors
        need_k, need_f = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_k or need_f):
            return (None,) * 8
        dk, lam, _ = ctx.op.adjoint(u, gbar.contiguous(), g=ctx.g, opts=ctx.opts,
                                    want_lambda=True)
        return (dk if need_k else None, lam if need_f else None,
                None, None, None, None, None, None)


def ddst_solve(kappa, f, n_slabs, bvec=(0.0, 0.0, 0.0), g=None, precision="fp32", opts=None,
               indefinite=False):
    """Differentiable solve (gradients for kappa and f); indefinite as in
    Operator."""
    return DDSTSolve.apply(kappa, f, n_slabs, tuple(bvec), g, precision, opts, indefinite)
