"""Four IMEX steps per read-write pass over f (Section 3.1's scheme, fused):
parity with the CPU oracle and with one step per pass, element by element on
the same seeded inputs at the 1e-12 normwise bar.  Before a pass the moments
of the second, third and fourth fields follow from sums of the previous
field weighted by 1 and by max(+-nu, 0) to the first, second and third
powers (linearity of the upwind transport).  These tests cover every step
count modulo 4 from the copy and from the lift, the closing steps evaluated
on the moments (one, two or three), both boundary conditions, the four-deep
ghost rows at nx = 4, ragged and single-cell chunks, and the large Sod batch
in the launch configuration of the benchmark."""
import numpy as np
import pytest
import torch

import oracle
from paper_2502_02704_amd import bgk
from paper_2502_02704_amd import workloads as wl
from tests.gpu_util import TOL, rel_f, rel_V
from tests.test_gpu_parity import cuda, states

pytestmark = pytest.mark.gpu

# grids whose v_x planes are whole tiles of 128 velocities (one pair per lane)
QUAD_GRIDS = {
    "uni_neumann": wl.Problem(nx=13, nv=(12, 8, 16), v_lo=(-6, -5, -7), v_hi=(6.5, 5, 7),
                              bc=wl.BC_NEUMANN, eps=3e-3),
    "uni_periodic": wl.Problem(nx=11, nv=(5, 16, 16), v_lo=(-6,) * 3, v_hi=(6,) * 3,
                               bc=wl.BC_PERIODIC, eps=0.5),
    "uni_nx4_neumann": wl.Problem(nx=4, nv=(4, 8, 16), v_lo=(-5,) * 3, v_hi=(5,) * 3,
                                  bc=wl.BC_NEUMANN, eps=1e-2),
    "uni_nx4_periodic": wl.Problem(nx=4, nv=(4, 8, 16), v_lo=(-5,) * 3, v_hi=(5,) * 3,
                                   bc=wl.BC_PERIODIC, eps=2e-2),
    "sod_nx64_nv16": wl.c1_sod_small().problem,
}
TILES = [(0, 0, -1), (2, 1, 1), (2, 2, 1), (2, 3, 1), (2, 5, 1), (2, 24, 1), (2, 64, 1)]


@pytest.fixture(autouse=True)
def _four():
    bgk.set_tiles(0, 0, -1)
    bgk.set_step_fusion(4)
    yield
    bgk.set_tiles(0, 0, -1)
    bgk.set_step_fusion(3)


def dt_of(p):
    return 0.45 * ((p.x_hi - p.x_lo) / p.nx) / max(abs(p.v_lo[0]), abs(p.v_hi[0]))


def conserved(W):
    return np.column_stack([W[:, 0], W[:, 0:1] * W[:, 1:4],
                            0.5 * W[:, 0] * (W[:, 1:4] ** 2).sum(1) + 1.5 * W[:, 0] * W[:, 4]])


def span_of(p, steps):
    dv = (p.v_hi[0] - p.v_lo[0]) / p.nv[0]
    vmax = max(abs(p.v_lo[0] + 0.5 * dv), abs(p.v_hi[0] - 0.5 * dv))
    return (steps - 0.5) * p.cfl * ((p.x_hi - p.x_lo) / p.nx) / vmax


@pytest.mark.parametrize("n", [4, 5, 6, 7, 8, 9, 11])
@pytest.mark.parametrize("name", list(QUAD_GRIDS))
def test_four_steps_per_pass(name, n):
    """Copy-mode start (a single step first), then quads and a remainder of
    pairs and a single: equal to the oracle and to one step per pass."""
    p = QUAD_GRIDS[name]
    _, f = states(p, 400 + n)
    dt = dt_of(p)
    ref = oracle.fine_steps(p, f, dt, n)
    bgk.set_step_fusion(1)
    single = bgk.fine_steps(p, cuda(f), dt, n).cpu().numpy()
    bgk.set_step_fusion(4)
    for tiles in TILES:
        bgk.set_tiles(*tiles)
        fused = bgk.fine_steps(p, cuda(f), dt, n).cpu().numpy()
        bgk.check_status()
        assert rel_f(fused, ref) < TOL, tiles
        assert rel_f(fused, single) < 1e-13, tiles


@pytest.mark.parametrize("span_steps", [4, 5, 6, 7, 8, 9, 10, 12])
@pytest.mark.parametrize("name", list(QUAD_GRIDS))
def test_four_steps_from_lift_and_closing_on_moments(name, span_steps):
    """Lift-mode start: a quad from the lifted Maxwellian, quads, then
    (n - 4) mod 4 closing steps on the moments (one: W1 + W2 projected; two:
    the three-step sums; three: the four-step sums); batched members against
    the oracle and against one step per pass."""
    p = QUAD_GRIDS[name]
    span = span_of(p, span_steps)
    n, _ = oracle.n_steps(p, span)
    assert n == span_steps
    Vin = np.stack([conserved(states(p, 420 + b)[0]) for b in range(2)])
    bgk.set_step_fusion(1)
    single = bgk.fine_propagate_moments(p, cuda(Vin), span).cpu().numpy()
    bgk.set_step_fusion(4)
    for tiles in [(0, 0, -1), (2, 1, 1), (2, 3, 1), (2, 16, 1)]:
        bgk.set_tiles(*tiles)
        got = bgk.fine_propagate_moments(p, cuda(Vin), span).cpu().numpy()
        bgk.check_status()
        for b in range(2):
            assert rel_V(got[b], oracle.fine_propagate_moments(p, Vin[b], span)) < TOL, tiles
            assert rel_V(got[b], single[b]) < 1e-13, tiles


def test_four_step_kernel_runs_and_is_timed():
    """On a quad-capable grid the propagation runs four-step passes (timing
    kinds BGK_PROF_FOUR_STEP_LIFT and BGK_PROF_FOUR_STEP, 2 and 4 algorithmic
    bytes per update): one from the lift, then (n - 4) // 4."""
    p = QUAD_GRIDS["sod_nx64_nv16"]
    V = np.stack([conserved(states(p, 442)[0])])
    n, _ = oracle.n_steps(p, 0.01)
    bgk.prof_enable(True)
    try:
        bgk.fine_propagate_moments(p, cuda(V), 0.01)
        ms, launches, upd, by = bgk.prof_read(bgk.PROF_FOUR_STEP)
        _, launches_l, upd_l, by_l = bgk.prof_read(bgk.PROF_FOUR_STEP_LIFT)
    finally:
        bgk.prof_enable(False)
    assert n >= 8 and launches_l == 1 and launches == (n - 4) // 4
    assert abs(by / upd - 4.0) < 1e-9 and abs(by_l / upd_l - 2.0) < 1e-9


def test_grids_without_whole_plane_tiles_fall_back():
    """Grids whose tiles straddle v_x planes, or nx < 4, run as under three
    steps per pass: same results."""
    for p in [wl.Problem(nx=21, nv=(7, 3, 6), v_lo=(-6, -5, -6), v_hi=(6, 5, 6),
                         bc=wl.BC_PERIODIC, eps=5e-2),
              wl.Problem(nx=3, nv=(4, 8, 16), v_lo=(-5,) * 3, v_hi=(5,) * 3,
                         bc=wl.BC_NEUMANN, eps=1e-2)]:
        _, f = states(p, 443)
        dt = dt_of(p)
        got4 = bgk.fine_steps(p, cuda(f), dt, 7).cpu().numpy()
        bgk.set_step_fusion(3)
        got3 = bgk.fine_steps(p, cuda(f), dt, 7).cpu().numpy()
        bgk.set_step_fusion(4)
        bgk.check_status()
        assert np.array_equal(got4, got3)
        assert rel_f(got4, oracle.fine_steps(p, f, dt, 7)) < TOL


def test_sod_large_32_slices_four_steps_sampled():
    """The benchmark's large Sod batch (32 slices of 2048 x 48^3) with four
    steps per pass over 23 steps (a quad from the lift, four quads, three
    steps closed on the moments): sampled slices against the oracle, mass
    and energy of every slice conserved."""
    wk = wl.c3_sod_large()
    p = wk.problem
    V = np.stack([conserved(w) for w in wl.c3_slice_states(wk)])
    n, dt = bgk.n_steps(p, wk.T / wk.n_slices)
    span = 23 * dt
    assert bgk.n_steps(p, span)[0] == 23
    bgk.free_workspaces()
    torch.cuda.empty_cache()
    bgk.prof_enable(True)
    try:
        got = bgk.fine_propagate_moments(p, cuda(V), span).cpu().numpy()
        _, quads, _, _ = bgk.prof_read(bgk.PROF_FOUR_STEP)
        _, quads_l, _, _ = bgk.prof_read(bgk.PROF_FOUR_STEP_LIFT)
    finally:
        bgk.prof_enable(False)
    bgk.check_status()
    bgk.free_workspaces()
    torch.cuda.empty_cache()
    assert (quads_l, quads) == (1, 4)
    dx = (p.x_hi - p.x_lo) / p.nx
    for b in range(V.shape[0]):
        for c in (0, 4):
            m0, m1 = V[b, :, c].sum() * dx, got[b, :, c].sum() * dx
            assert abs(m1 - m0) <= 1e-12 * abs(m0), (b, c)
    for b in (0, 17, 31):
        e = rel_V(got[b], oracle.fine_propagate_moments(p, V[b], span))
        print(f"slice {b}: {e:.2e}")
        assert e <= TOL
