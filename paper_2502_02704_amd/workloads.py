"""Seeded synthetic workloads: problem geometry and initial moments.

This module only *describes* inputs (grids, boundary conditions, initial
primitive moments rho, u, theta at x-cell centres).  It holds none of the
method's arithmetic, so that both the HIP path and the CPU oracle can be fed
from it without sharing any computation.

The initial data follow the shapes of the paper's tests (Section 5): Riemann
problems with Maxwellian initial data (Sod, Section 5.1), and smooth data on a
periodic domain.  The paper's exact settings are rescaled to x in [0, 1]; the
workloads below are the ones this library is benchmarked and tested on.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np

BC_NEUMANN = 0
BC_PERIODIC = 1


@dataclass(frozen=True)
class Problem:
    """Phase-space grid and model parameters of one 1D-3V BGK problem."""
    nx: int
    nv: Tuple[int, int, int]
    x_lo: float = 0.0
    x_hi: float = 1.0
    v_lo: Tuple[float, float, float] = (-8.0, -8.0, -8.0)
    v_hi: Tuple[float, float, float] = (8.0, 8.0, 8.0)
    bc: int = BC_NEUMANN
    eps: float = 1e-2
    cfl: float = 0.5
    sound_gamma: float = 5.0 / 3.0

    @property
    def nv3(self) -> int:
        return self.nv[0] * self.nv[1] * self.nv[2]

    @property
    def cells(self) -> int:
        return self.nx * self.nv3

    def with_eps(self, eps: float) -> "Problem":
        return replace(self, eps=eps)

    def x_centres(self) -> np.ndarray:
        dx = (self.x_hi - self.x_lo) / self.nx
        return self.x_lo + (np.arange(self.nx) + 0.5) * dx


@dataclass
class Workload:
    name: str
    problem: Problem
    W0: np.ndarray            # [nx][5] primitive (rho, ux, uy, uz, theta)
    T: float
    n_slices: int = 1
    k_max: int = 0
    tol: float = 0.0
    meta: dict = field(default_factory=dict)


def _iso(nv: int, L: float):
    return (nv, nv, nv), (-L, -L, -L), (L, L, L)


def riemann_W0(prob: Problem, left, right, x_split: float = 0.5) -> np.ndarray:
    """Piecewise-constant primitive moments: `left` for x_i < x_split."""
    x = prob.x_centres()
    W = np.empty((prob.nx, 5))
    W[x < x_split] = np.asarray(left, dtype=np.float64)
    W[x >= x_split] = np.asarray(right, dtype=np.float64)
    return W


SOD_LEFT = (1.0, 0.0, 0.0, 0.0, 1.0)
SOD_RIGHT = (0.125, 0.0, 0.0, 0.0, 0.8)


def c1_sod_small() -> Workload:
    """Nx=64, 16^3 on [-8,8]^3, Neumann, eps=1e-2, Sod, T=0.1, 8 slices, K=3."""
    nv, lo, hi = _iso(16, 8.0)
    p = Problem(nx=64, nv=nv, v_lo=lo, v_hi=hi, bc=BC_NEUMANN, eps=1e-2)
    return Workload("sod_nx64_nv16", p, riemann_W0(p, SOD_LEFT, SOD_RIGHT),
                    T=0.1, n_slices=8, k_max=3)


def c2_smooth_periodic(eps: float = 1e-2, nx: int = 512, nv: int = 32,
                       n_slices: int = 64) -> Workload:
    """Nx=512, 32^3 on [-8,8]^3, periodic, rho = 1 + 0.2 sin 2 pi x,
    u = (0.1 sin 2 pi x, 0, 0), theta = 1, T=0.2, 64 slices."""
    nvv, lo, hi = _iso(nv, 8.0)
    p = Problem(nx=nx, nv=nvv, v_lo=lo, v_hi=hi, bc=BC_PERIODIC, eps=eps)
    x = p.x_centres()
    W = np.zeros((nx, 5))
    W[:, 0] = 1.0 + 0.2 * np.sin(2 * np.pi * x)
    W[:, 1] = 0.1 * np.sin(2 * np.pi * x)
    W[:, 4] = 1.0
    return Workload(f"smooth_periodic_nx{nx}_nv{nv}_eps{eps:g}", p, W, T=0.2,
                    n_slices=n_slices, k_max=n_slices, tol=1e-6)


def c3_sod_large() -> Workload:
    """Nx=2048, 48^3 on [-10,10]^3, Neumann, eps=1e-3, Sod, T=0.15, 32 slices."""
    nv, lo, hi = _iso(48, 10.0)
    p = Problem(nx=2048, nv=nv, v_lo=lo, v_hi=hi, bc=BC_NEUMANN, eps=1e-3)
    return Workload("sod_nx2048_nv48", p, riemann_W0(p, SOD_LEFT, SOD_RIGHT),
                    T=0.15, n_slices=32, k_max=6)


def c3_slice_states(wk: Workload | None = None) -> np.ndarray:
    """Primitive moments [32][2048][5] handed to the 32 slices of the large
    Sod workload in one batched fine sweep: member b is the Sod data with its
    discontinuity at x = 0.5 + (b - 16)/256 (a cell face; every member
    distinct), a stand-in for the Riemann-fan states a parareal iterate
    carries at the slice starts (the fine solve's cost does not depend on
    the data)."""
    wk = wk or c3_sod_large()
    p = wk.problem
    return np.stack([riemann_W0(p, SOD_LEFT, SOD_RIGHT, x_split=0.5 + (b - 16) / 256.0)
                     for b in range(wk.n_slices)])


C4_SEED = 250202704


def c4_adjoint(nx: int = 256, nv: int = 24, T: float = 0.1,
               eps0: float = 1e-2, eps_target: float = 3e-3):
    """Seeded random 8-mode Fourier density on a periodic box.

    Returns (workload at eps0, rho0, eps_target, rng) where rng has already
    drawn the Fourier coefficients and is positioned for direction draws."""
    rng = np.random.default_rng(C4_SEED)
    a = rng.standard_normal(8)
    b = rng.standard_normal(8)
    nvv, lo, hi = _iso(nv, 8.0)
    p = Problem(nx=nx, nv=nvv, v_lo=lo, v_hi=hi, bc=BC_PERIODIC, eps=eps0)
    x = p.x_centres()
    s = np.zeros(nx)
    for m in range(1, 9):
        s += (a[m - 1] * np.sin(2 * np.pi * m * x) +
              b[m - 1] * np.cos(2 * np.pi * m * x)) / m
    rho0 = 1.0 + 0.3 * s / np.max(np.abs(s))
    W = np.zeros((nx, 5))
    W[:, 0] = rho0
    W[:, 4] = 1.0
    wl = Workload(f"adjoint_nx{nx}_nv{nv}", p, W, T=T,
                  meta={"eps_target": eps_target})
    return wl, rho0, eps_target, rng


C5_SEED = 250202705


def _ball(rng, radius: float) -> np.ndarray:
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    return d * radius * rng.uniform() ** (1.0 / 3.0)


def c5_uneven(n_instances: int = 32, nx_range=(128, 1024),
              nv_range=(16, 32), seed: int = C5_SEED) -> List[Workload]:
    """Independent Riemann problems of uneven size and Knudsen number.

    Per instance, drawn in this order: Nx ~ U{nx_range}, Nv ~ U{nv_range},
    log10 eps ~ U[-4, 0], rho_L, rho_R ~ U[0.1, 1], theta_L, theta_R ~
    U[0.1, 1], u_L, u_R uniform in the ball of radius 0.5.  Split at x=0.5,
    Neumann, box [-8,8]^3, T=0.1, CFL 0.5."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n_instances):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        nv = int(rng.integers(nv_range[0], nv_range[1] + 1))
        eps = 10.0 ** rng.uniform(-4.0, 0.0)
        rl, rr = rng.uniform(0.1, 1.0, size=2)
        tl, tr = rng.uniform(0.1, 1.0, size=2)
        ul, ur = _ball(rng, 0.5), _ball(rng, 0.5)
        nvv, lo, hi = _iso(nv, 8.0)
        p = Problem(nx=nx, nv=nvv, v_lo=lo, v_hi=hi, bc=BC_NEUMANN, eps=eps)
        W = riemann_W0(p, (rl, *ul, tl), (rr, *ur, tr))
        out.append(Workload(f"uneven_{q}_nx{nx}_nv{nv}", p, W, T=0.1))
    return out


def exterior_force(x) -> np.ndarray:
    """The exterior force of the paper's third test, E(x) = -5 x^4 (x-2)^4 (x-1)
    on [0, 2]: it pushes mass towards x = 1."""
    x = np.asarray(x, dtype=np.float64)
    return -5.0 * x ** 4 * (x - 2.0) ** 4 * (x - 1.0)


@dataclass
class ForceWorkload:
    name: str
    problem: Problem
    E: np.ndarray        # force at the x-cell centres
    W_beams: tuple       # primitive states of the two beams
    T: float
    n_slices: int

    def f0(self, lift) -> np.ndarray:
        """Initial phase-space field: the sum of the two beams' Maxwellians,
        each lifted with the given lifting routine."""
        p = self.problem
        return sum(lift(p, np.tile(np.asarray(w, dtype=np.float64), (p.nx, 1)))
                   for w in self.W_beams)

    def U0(self) -> np.ndarray:
        """Primitive moments of f0: the beams have equal densities and
        opposite x velocities, so rho = 2, u = 0, theta = 1 + 1/3 (continuous
        moments)."""
        p = self.problem
        W = np.zeros((p.nx, 5))
        W[:, 0] = 2.0
        W[:, 4] = 4.0 / 3.0
        return W


def c6_two_beam_force(nx: int = 100, nv=(256, 16, 16), eps: float = 1e-5,
                      n_slices: int = 20, T: float = 0.5) -> ForceWorkload:
    """Two opposite beams M(1, +e_x, 1) + M(1, -e_x, 1) under the exterior
    force E(x) = -5 x^4 (x-2)^4 (x-1), x in [0, 2] periodic, velocity box
    [-8, 8]^3 refined in v_x, eps = 1e-5, T = 0.5."""
    lo, hi = (-8.0,) * 3, (8.0,) * 3
    p = Problem(nx=nx, nv=tuple(nv), x_lo=0.0, x_hi=2.0, v_lo=lo, v_hi=hi,
                bc=BC_PERIODIC, eps=eps)
    E = exterior_force(p.x_centres())
    beams = ((1.0, 1.0, 0.0, 0.0, 1.0), (1.0, -1.0, 0.0, 0.0, 1.0))
    return ForceWorkload(f"two_beam_force_nx{nx}_nv{nv[0]}x{nv[1]}x{nv[2]}", p, E, beams,
                         T, n_slices)


def random_f(prob: Problem, seed: int, lo: float = 0.5, hi: float = 1.5) -> np.ndarray:
    """A strictly positive random phase-space field, for unit tests only."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(prob.nx, prob.nv3)) * 1e-3


def small_problem(nx: int = 8, nv=(4, 4, 4), bc: int = BC_NEUMANN,
                  eps: float = 1e-2, L: float = 6.0, cfl: float = 0.5) -> Problem:
    return Problem(nx=nx, nv=tuple(nv), v_lo=(-L,) * 3, v_hi=(L,) * 3, bc=bc,
                   eps=eps, cfl=cfl)


def all_configs():
    """The benchmarked and tested workload families, by name."""
    return {
        "sod_nx64_nv16": c1_sod_small,
        "smooth_periodic_nx512_nv32": c2_smooth_periodic,
        "sod_nx2048_nv48": c3_sod_large,
    }
