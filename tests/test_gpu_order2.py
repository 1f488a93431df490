"""Parity of the second-order fine transport (van Leer limited Lax-Wendroff
correction in x, the flux limiters Section 3.1 names) with the CPU oracle,
element by element at the 1e-12 normwise bar."""
import numpy as np
import pytest

import oracle
from paper_2502_02704_amd import bgk
from paper_2502_02704_amd import workloads as wl
from tests.gpu_util import TOL, rel_f, rel_V
from tests.test_gpu_parity import GRIDS, cuda, states

pytestmark = pytest.mark.gpu

ORDER2_TILES = [(0, 0, -1), (2, 1, 0), (4, 3, 0), (2, 16, 0), (4, 64, 0), (8, 8, 0)]
# with the exterior force: the v_x-column mapping too (pair = 2)
ORDER2_FORCE_TILES = ORDER2_TILES + [(0, 0, 2), (2, 1, 2), (4, 5, 2), (8, 16, 2),
                                     (0, 0, 3), (2, 3, 3), (4, 16, 3)]


@pytest.fixture(autouse=True)
def _reset_tiles():
    bgk.set_tiles(0, 0, -1)
    yield
    bgk.set_tiles(0, 0, -1)


@pytest.mark.parametrize("tiles", ORDER2_TILES)
@pytest.mark.parametrize("name", list(GRIDS))
def test_fine_steps_second_order(name, tiles):
    p = GRIDS[name]
    bgk.set_tiles(*tiles)
    _, f = states(p, 100)
    n, dt = oracle.n_steps(p, 0.004)
    n = min(n, 5)
    got = bgk.fine_steps(p, cuda(f), dt, n, fine_order=2).cpu().numpy()
    bgk.check_status()
    assert rel_f(got, oracle.fine_steps_opts(p, f, dt, n, fine_order=2)) < TOL


@pytest.mark.parametrize("tiles", ORDER2_FORCE_TILES)
@pytest.mark.parametrize("name", ["ragged_neumann", "wide_periodic", "even_z_ragged"])
def test_second_order_with_force(name, tiles):
    p = GRIDS[name]
    bgk.set_tiles(*tiles)
    _, f = states(p, 101)
    E = np.random.default_rng(102).uniform(-2, 2, p.nx)
    n, dt = oracle.n_steps(p, 0.004, E=E)
    n = min(n, 4)
    got = bgk.fine_steps(p, cuda(f), dt, n, E=E, fine_order=2).cpu().numpy()
    bgk.check_status()
    assert rel_f(got, oracle.fine_steps_opts(p, f, dt, n, E=E, fine_order=2)) < TOL


def test_step_profile_stays_monotone():
    # a sharp profile without relaxation: the limited scheme adds no extrema
    p = wl.Problem(nx=40, nv=(6, 2, 2), v_lo=(-3, -1, -1), v_hi=(3, 1, 1),
                   bc=wl.BC_PERIODIC, eps=float("inf"))
    x = p.x_centres()
    f = np.column_stack([np.where((x > 0.3) & (x < 0.6), 2.0, 0.5)] * p.nv3)
    dt = 0.9 / p.nx / 2.5
    got = bgk.fine_steps(p, cuda(f), dt, 12, fine_order=2).cpu().numpy()
    assert rel_f(got, oracle.fine_steps_opts(p, f, dt, 12, fine_order=2)) < TOL
    assert got.min() >= 0.5 - 1e-14 and got.max() <= 2.0 + 1e-14


@pytest.mark.parametrize("name", ["sod_nx64_nv16", "wide_periodic"])
def test_propagate_second_order(name):
    p = GRIDS[name]
    W, _ = states(p, 103)
    V = np.column_stack([W[:, 0], W[:, 0:1] * W[:, 1:4],
                         0.5 * W[:, 0] * (W[:, 1:4] ** 2).sum(1) + 1.5 * W[:, 0] * W[:, 4]])
    Vin = np.stack([V, V[::-1].copy()])
    got = bgk.fine_propagate_moments(p, cuda(Vin), 0.0043, fine_order=2).cpu().numpy()
    bgk.check_status()
    for b in range(2):
        ref = oracle.fine_propagate_moments_opts(p, Vin[b], 0.0043, fine_order=2)
        assert rel_V(got[b], ref) < TOL


def test_parareal_second_order_matches_oracle_and_serial():
    wk = wl.c2_smooth_periodic(eps=1e-2, nx=32, nv=16, n_slices=6)
    p, N = wk.problem, wk.n_slices
    V, err, kd = bgk.parareal_iterate(p, cuda(wk.W0), N, wk.T, 2, 0.0, fine_order=2)
    Vr, errr, kdr = oracle.parareal_iterate_opts(p, wk.W0, N, wk.T, 2, 0.0, fine_order=2)
    assert kd == kdr == 2
    assert rel_V(V.cpu().numpy(), Vr) < TOL
    VN, _, _ = bgk.parareal_iterate(p, cuda(wk.W0), N, wk.T, N, 0.0, fine_order=2)
    S = bgk.serial_fine(p, cuda(wk.W0), N, wk.T, fine_order=2).cpu().numpy()
    assert rel_V(VN.cpu().numpy(), S) < 1e-13
    assert rel_V(S, oracle.serial_fine_opts(p, wk.W0, N, wk.T, fine_order=2)) < TOL


def test_eight_elements_per_lane_runs_as_four():
    """The second-order flat kernels take 2 or 4 velocities per lane: a tile
    override of 8 runs with 4 (same results as the built-in choice)."""
    p = GRIDS["wide_periodic"]
    _, f = states(p, 104)
    bgk.set_tiles(8, 4, 0)
    got = bgk.fine_steps(p, cuda(f), 1e-3, 2, fine_order=2).cpu().numpy()
    bgk.check_status()
    assert rel_f(got, oracle.fine_steps_opts(p, f, 1e-3, 2, fine_order=2)) < TOL


def test_smooth_periodic_full_batch_second_order_sampled():
    """The benchmark batch (64 slices of 512 x 32^3, 25 steps) with the
    second-order transport in the launch configuration the bench times (the
    built-in tiles: four velocities per lane, 64-cell chunks, one step per
    pass); eight sampled members (first and last among them) against the
    oracle."""
    wk = wl.c2_smooth_periodic(eps=1e-2)
    p = wk.problem
    B = wk.n_slices
    x = p.x_centres()
    V = np.empty((B, p.nx, 5))
    for b in range(B):
        rho = 1 + 0.2 * np.sin(2 * np.pi * (x + b / B))
        u = 0.1 * np.sin(2 * np.pi * (x + b / B))
        V[b] = np.column_stack([rho, rho * u, 0 * x, 0 * x, 0.5 * rho * u * u + 1.5 * rho])
    span = wk.T / wk.n_slices
    got = bgk.fine_propagate_moments(p, cuda(V), span, fine_order=2).cpu().numpy()
    bgk.check_status()
    for b in (0, 9, 18, 27, 36, 45, 54, 63):
        ref = oracle.fine_propagate_moments_opts(p, V[b], span, fine_order=2)
        assert rel_V(got[b], ref) < TOL
