"""Seeded synthetic workloads shaped like the paper's FD model problems.

Conventions (shared by every consumer):

* the domain is the unit square / cube, ``n`` interior nodes per axis,
  ``h = 1/(n+1)``; nodes ``i = 0..n+1`` per axis, ``0`` and ``n+1`` are on the
  physical boundary;
* slabs are cut along the first axis ``x``: ``n_slabs`` slabs of
  ``m = (n+1)/n_slabs`` cells; interfaces sit on node planes ``i = j*m``,
  ``j = 1..n_slabs-1`` (Section 2, equispaced slabs);
* interior nodal arrays have shape ``(n,)*dim`` in C order (x slowest), so a
  node plane ``x = const`` is a contiguous block of ``n**(dim-1)`` values;
* the cellwise coefficient ``kappa`` has shape ``(n+1,)*dim``; cell ``c``
  spans nodes ``c..c+1`` on every axis;
* boundary data ``g`` lives on the full node box ``(n+2,)*dim``; only its
  boundary entries are read.

The random fields follow one fixed recipe (a sum of seeded Fourier modes,
amplitude proportional to ``1/|k|^2``), the recipe stated for the
variable-coefficient workloads.  Every array is float64.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Problem:
    """One FD boundary value problem ``A u = f`` in the box, ``u = g`` on it."""

    dim: int
    n: int
    n_slabs: int
    kappa: Optional[np.ndarray] = None   # (n+1,)*dim cells, None => 1
    bvec: tuple = (0.0, 0.0, 0.0)        # constant convection velocity
    c: Optional[np.ndarray] = None       # (n,)*dim nodal zeroth order, None => 0
    f: Optional[np.ndarray] = None       # (n,)*dim load, None => 0
    g: Optional[np.ndarray] = None       # (n+2,)*dim node box, None => 0
    name: str = ""

    def __post_init__(self):
        if self.dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        if self.n_slabs < 2 or (self.n + 1) % self.n_slabs != 0:
            raise ValueError("(n+1) must be a multiple of n_slabs >= 2")
        self.bvec = tuple(float(v) for v in (list(self.bvec) + [0.0] * 3)[:3])

    @property
    def h(self) -> float:
        return 1.0 / (self.n + 1)

    @property
    def m(self) -> int:
        return (self.n + 1) // self.n_slabs

    @property
    def n_ds(self) -> int:
        return self.n_slabs - 1

    @property
    def M(self) -> int:
        return self.n ** (self.dim - 1)

    @property
    def N(self) -> int:
        return self.n ** self.dim

    def interface_planes(self):
        """Node-plane index (1-based along x) of every interface."""
        return [j * self.m for j in range(1, self.n_slabs)]

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def _half_space_modes(dim: int, kmax: int):
    """Integer wave vectors with 0 < |k| <= kmax, one of each +-k pair."""
    out = []
    rng = range(-kmax, kmax + 1)
    for k in itertools.product(rng, repeat=dim):
        if all(v == 0 for v in k):
            continue
        if sum(v * v for v in k) > kmax * kmax:
            continue
        first = next(v for v in k if v != 0)
        if first > 0:
            out.append(k)
    return np.array(out, dtype=np.int64)


def fourier_field(dim: int, n_cells: int, n_modes: int, kmax: int,
                  seed: int) -> np.ndarray:
    """G(x) = sum_i xi_i / |k_i|^2 cos(2 pi k_i . x + phi_i) at cell centres.

    ``k_i`` are drawn without replacement from the half-space integer vectors
    with ``0 < |k| <= kmax``; ``xi ~ N(0,1)``, ``phi ~ U[0, 2 pi)``.
    """
    rng = np.random.default_rng(seed)
    modes = _half_space_modes(dim, kmax)
    pick = rng.choice(len(modes), size=min(n_modes, len(modes)), replace=False)
    ks = modes[pick]
    xi = rng.standard_normal(len(ks))
    phi = rng.uniform(0.0, 2.0 * np.pi, len(ks))
    centres = (np.arange(n_cells) + 0.5) / n_cells
    grids = np.meshgrid(*([centres] * dim), indexing="ij")
    G = np.zeros((n_cells,) * dim)
    for k, a, p in zip(ks, xi, phi):
        arg = sum(2.0 * np.pi * k[d] * grids[d] for d in range(dim)) + p
        G += a / float(np.dot(k, k)) * np.cos(arg)
    return G


def box_boundary_values(dim: int, n: int, func) -> np.ndarray:
    """Evaluate ``func`` on the (n+2)^dim node box (boundary entries used)."""
    x = np.arange(n + 2) / (n + 1)
    grids = np.meshgrid(*([x] * dim), indexing="ij")
    return np.asarray(func(*grids), dtype=np.float64)


def sensor_nodes(dim: int, n: int, count: int, seed: int) -> np.ndarray:
    """``count`` distinct interior grid nodes, as flat C-order indices."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n ** dim, size=count, replace=False)).astype(np.int64)


def perturbed_kappa(prob, seed: int = 1009, amplitude: float = 0.1) -> np.ndarray:
    """The "true" coefficient behind synthetic sensor data of the adjoint
    workload: kappa * exp(amplitude * G') with G' an independent Fourier field
    of the same spectrum as the workload's (16 modes, |k| <= 8 in 2D; 32
    modes, |k| <= 6 in 3D).  Seed: 1005 + 4 for the adjoint configuration."""
    n_modes, kmax = (16, 8) if prob.dim == 2 else (32, 6)
    G = fourier_field(prob.dim, prob.n + 1, n_modes, kmax, seed=seed)
    base = np.ones((prob.n + 1,) * prob.dim) if prob.kappa is None else prob.kappa
    return np.asarray(base, dtype=np.float64) * np.exp(amplitude * G)


def fd_directions(shape, count: int, seed: int) -> np.ndarray:
    """Random cellwise directions ``v ~ N(0,1)``, normalised to max|v| = 1."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((count,) + tuple(shape))
    v /= np.abs(v.reshape(count, -1)).max(axis=1).reshape((count,) + (1,) * len(shape))
    return v


def _nodes(dim, n):
    x = np.arange(1, n + 1) / (n + 1)
    return np.meshgrid(*([x] * dim), indexing="ij")


def make_config(name: str, n: Optional[int] = None, n_slabs: Optional[int] = None,
                variant: int = 2) -> Problem:
    """Build one of the five workloads, optionally at a reduced size.

    ``cfg1`` 2D Poisson, 127^2, 8 slabs (variant 1: manufactured
    ``exp(x) sin(y)`` boundary data with f = 0; variant 2: f ~ N(0,1), g = 0).
    ``cfg2`` 2D variable-kappa convection-diffusion, 1023^2, 32 slabs.
    ``cfg3`` 2D Helmholtz-type, 2047^2, 64 slabs, k = 60, Gaussian source.
    ``cfg4`` 3D variable kappa, 127^3, 16 slabs.
    ``cfg5`` the cfg2 operator (the adjoint workload).
    Seeds: 1000+i for config i (coefficient field), +10 load, +2 FD
    directions, +3 sensors, +4 perturbation field (cfg5 reuses 1002).
    """
    defaults = {"cfg1": (2, 127, 8), "cfg2": (2, 1023, 32), "cfg3": (2, 2047, 64),
                "cfg4": (3, 127, 16), "cfg5": (2, 1023, 32)}
    if name not in defaults:
        raise KeyError(name)
    dim, n0, s0 = defaults[name]
    n = n0 if n is None else n
    if n_slabs is None:
        n_slabs = s0 if n == n0 else max(2, (n + 1) // ((n0 + 1) // s0))
    idx = int(name[-1])
    seed = 1000 + idx
    rng = np.random.default_rng(seed)
    X = _nodes(dim, n)
    if name == "cfg1":
        if variant == 1:
            g = box_boundary_values(dim, n, lambda x, y: np.exp(x) * np.sin(y))
            return Problem(dim, n, n_slabs, f=np.zeros((n,) * dim), g=g,
                           name="cfg1-manufactured")
        return Problem(dim, n, n_slabs, f=rng.standard_normal((n,) * dim),
                       name="cfg1-random")
    if name in ("cfg2", "cfg5"):
        G = fourier_field(2, n + 1, 16, 8, seed=1002)
        kappa = np.exp(0.5 * G)
        f = np.random.default_rng(1002 + 10).standard_normal((n,) * 2)
        return Problem(2, n, n_slabs, kappa=kappa, bvec=(10.0, 0.0, 0.0), f=f,
                       name=name)
    if name == "cfg3":
        k = 60.0
        r2 = (X[0] - 0.5) ** 2 + (X[1] - 0.5) ** 2
        c = -k * k * (1.0 - 0.5 * np.exp(-20.0 * r2))
        x0 = rng.uniform(0.25, 0.75, 2)
        sig = 0.02
        f = np.exp(-((X[0] - x0[0]) ** 2 + (X[1] - x0[1]) ** 2) / (2 * sig * sig))
        return Problem(2, n, n_slabs, c=c, f=f, name="cfg3")
    # cfg4
    G = fourier_field(3, n + 1, 32, 6, seed=seed)
    kappa = np.exp(0.5 * G)
    f = np.random.default_rng(seed + 10).standard_normal((n,) * 3)
    return Problem(3, n, n_slabs, kappa=kappa, f=f, name="cfg4")


def config_names():
    return ["cfg1", "cfg2", "cfg3", "cfg4", "cfg5"]
