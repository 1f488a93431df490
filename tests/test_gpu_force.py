"""Parity of the exterior-force path (Section 3.1 with E != 0: Rusanov
transport in v_x; the coarse Euler system with the force source) with the
CPU oracle, element by element on the same seeded inputs, at the 1e-12
normwise bar; step and substep counts bit-exact."""
import numpy as np
import pytest
import torch

import oracle
from paper_2502_02704_amd import bgk
from paper_2502_02704_amd import workloads as wl
from tests.gpu_util import TOL, rel_f, rel_V
from tests.test_gpu_parity import GRIDS, cuda, states

pytestmark = pytest.mark.gpu

# (elems, x chunk, lane mapping): 0 = flat velocity runs, 2 = v_x columns,
# 3 = v_x columns with two (v_y, v_z) points per lane, -1 = built-in (columns
# where a v_x plane fills a wave)
FORCE_TILES = [(0, 0, -1), (2, 1, 0), (4, 3, 0), (8, 16, 0), (2, 64, 0),
               (0, 0, 2), (2, 1, 2), (4, 3, 2), (8, 16, 2), (8, 64, 2),
               (0, 0, 3), (2, 1, 3), (4, 5, 3), (2, 64, 3)]


@pytest.fixture(autouse=True)
def _reset_tiles():
    bgk.set_tiles(0, 0, -1)
    yield
    bgk.set_tiles(0, 0, -1)


def force_of(p, seed, amp=2.0):
    return np.random.default_rng(seed).uniform(-amp, amp, p.nx)


def conserved(W):
    return np.column_stack([W[:, 0], W[:, 0:1] * W[:, 1:4],
                            0.5 * W[:, 0] * (W[:, 1:4] ** 2).sum(1) + 1.5 * W[:, 0] * W[:, 4]])


@pytest.mark.parametrize("tiles", FORCE_TILES)
@pytest.mark.parametrize("name", list(GRIDS))
def test_fine_steps_force(name, tiles):
    p = GRIDS[name]
    bgk.set_tiles(*tiles)
    _, f = states(p, 80)
    E = force_of(p, 81)
    n, dt = oracle.n_steps(p, 0.004, E=E)
    n = min(n, 5)
    got = bgk.fine_steps(p, cuda(f), dt, n, E=E).cpu().numpy()
    bgk.check_status()
    assert rel_f(got, oracle.fine_steps(p, f, dt, n, E=E)) < TOL


@pytest.mark.parametrize("name", ["sod_nx64_nv16", "asym_box", "even_z_ragged"])
def test_zero_force_matches_plain_path(name):
    p = GRIDS[name]
    _, f = states(p, 82)
    n, dt = oracle.n_steps(p, 0.003)
    got = bgk.fine_steps(p, cuda(f), dt, n, E=np.zeros(p.nx)).cpu().numpy()
    plain = bgk.fine_steps(p, cuda(f), dt, n).cpu().numpy()
    bgk.check_status()
    assert rel_f(got, plain) < 1e-13
    assert rel_f(got, oracle.fine_steps(p, f, dt, n)) < TOL


@pytest.mark.parametrize("name", ["ragged_neumann", "wide_periodic"])
def test_fine_step_span_force(name):
    p = GRIDS[name]
    _, f = states(p, 83)
    E = force_of(p, 84, amp=3.0)
    got, n = bgk.fine_step(p, cuda(f), 0.0057, E=E)
    ref, nr = oracle.fine_step(p, f, 0.0057, E=E)
    assert n == nr
    assert bgk.n_steps(p, 0.0057, E=E)[0] == oracle.n_steps(p, 0.0057, E=E)[0]
    assert rel_f(got.cpu().numpy(), ref) < TOL


@pytest.mark.parametrize("name", ["sod_nx64_nv16", "wide_periodic", "even_z_ragged"])
def test_propagate_moments_force(name):
    p = GRIDS[name]
    E = force_of(p, 85)
    Vin = np.stack([conserved(states(p, 86 + b)[0]) for b in range(3)])
    got = bgk.fine_propagate_moments(p, cuda(Vin), 0.0041, E=E).cpu().numpy()
    bgk.check_status()
    for b in range(3):
        assert rel_V(got[b], oracle.fine_propagate_moments(p, Vin[b], 0.0041, E=E)) < TOL


@pytest.mark.parametrize("bc", [wl.BC_NEUMANN, wl.BC_PERIODIC])
def test_euler_coarse_force(bc):
    p = wl.small_problem(nx=40, bc=bc)
    E = force_of(p, 87, amp=1.5)
    V = np.stack([conserved(states(p, 88 + b)[0]) for b in range(2)])
    got, nsub = bgk.euler_coarse_step(p, cuda(V), 0.02, E=E)
    got, nsub = got.cpu().numpy(), nsub.cpu().numpy()
    for b in range(2):
        ref, nr = oracle.euler_coarse_step(p, V[b], 0.02, E=E)
        assert nsub[b] == nr
        assert rel_V(got[b], ref) < TOL


def small_two_beam():
    return wl.c6_two_beam_force(nx=24, nv=(32, 12, 12), eps=1e-3, n_slices=4, T=0.04)


def test_parareal_force_matches_oracle():
    wk = small_two_beam()
    p, W0 = wk.problem, wk.U0()
    V, err, kd = bgk.parareal_iterate(p, cuda(W0), wk.n_slices, wk.T, 2, 0.0, E=wk.E)
    Vr, errr, kdr = oracle.parareal_iterate(p, W0, wk.n_slices, wk.T, 2, 0.0, E=wk.E)
    assert kd == kdr == 2
    assert rel_V(V.cpu().numpy(), Vr) < TOL
    assert np.allclose(err, errr, rtol=1e-6, atol=1e-13)


def test_parareal_force_k_equals_n_is_serial_fine():
    wk = small_two_beam()
    p, W0, N = wk.problem, wk.U0(), wk.n_slices
    V, _, kd = bgk.parareal_iterate(p, cuda(W0), N, wk.T, N, 0.0, E=wk.E)
    S = bgk.serial_fine(p, cuda(W0), N, wk.T, E=wk.E).cpu().numpy()
    assert kd == N
    assert rel_V(V.cpu().numpy(), S) < 1e-13
    assert rel_V(S, oracle.serial_fine(p, W0, N, wk.T, E=wk.E)) < TOL


def test_force_above_emax_is_reported():
    """A force larger than the Rusanov coefficient passed through the C ABI
    is flagged on the device and reported by bgk_status as invalid."""
    p = GRIDS["wide_periodic"]
    _, f = states(p, 89)
    E = torch.from_numpy(force_of(p, 90)).cuda()
    fin, fout = cuda(f), torch.empty_like(cuda(f))
    w = bgk.workspace(p, bgk.OP_FINE_STEP)
    L = bgk.load_library()
    emax = float(E.abs().max()) * 0.5
    rc = L.bgk_fine_steps_force(bgk.C.byref(bgk.problem_struct(p)), E.data_ptr(), emax,
                                fin.data_ptr(), fout.data_ptr(), 1e-4, 2, w.data_ptr(),
                                w.numel(), bgk._stream())
    assert rc == bgk.OK
    assert bgk.status(w) == bgk.E_INVALID
    assert bgk.status(w) == bgk.OK  # the flag is cleared by the read


def test_two_beam_exterior_force_full_grid():
    """The exterior-force test at its grid: Nx=100 on [0,2] periodic,
    256 x 16 x 16 velocities on [-8,8]^3, eps=1e-5, two opposite beams; one
    parareal slice of its 20 (21 steps) against the oracle."""
    wk = wl.c6_two_beam_force()
    p = wk.problem
    f0 = wk.f0(oracle.lift)
    f0g = sum(bgk.lift(p, cuda(np.tile(np.asarray(b), (p.nx, 1)))) for b in wk.W_beams)
    assert rel_f(f0g.cpu().numpy(), f0) < TOL
    span = wk.T / wk.n_slices
    got, n = bgk.fine_step(p, f0g, span, E=wk.E)
    bgk.check_status()
    ref, nr = oracle.fine_step(p, f0, span, E=wk.E)
    assert n == nr == 21
    assert rel_f(got.cpu().numpy(), ref) < TOL
    V, _ = bgk.moments(p, got)
    Vr, _ = oracle.moments(p, ref)
    assert rel_V(V.cpu().numpy(), Vr) < TOL


@pytest.mark.parametrize("tiles", [(4, 8, 2), (8, 2, 2), (2, 5, 2), (4, 8, 3), (2, 3, 3)])
def test_two_beam_columns_match_flat_mapping(tiles):
    """On the two-beam grid (256 x 16 x 16 velocities) the v_x-column force
    step and the flat-mapping one agree to rounding, over a lifted start and
    relaxed steps, and both agree with the oracle."""
    wk = wl.c6_two_beam_force(nx=24)
    p = wk.problem
    f0 = wk.f0(oracle.lift)
    n, dt = oracle.n_steps(p, 0.01, E=wk.E)
    n = min(n, 4)
    bgk.set_tiles(2, 8, 0)
    flat = bgk.fine_steps(p, cuda(f0), dt, n, E=wk.E).cpu().numpy()
    bgk.set_tiles(*tiles)
    col = bgk.fine_steps(p, cuda(f0), dt, n, E=wk.E).cpu().numpy()
    bgk.check_status()
    assert rel_f(col, flat) < 1e-14
    assert rel_f(col, oracle.fine_steps(p, f0, dt, n, E=wk.E)) < TOL


@pytest.mark.parametrize("mapping", [0, 2, 3])
def test_parareal_force_lane_mappings(mapping):
    """The parareal iterate with the force is the same on either lane
    mapping of the force step (batched slices, graph-captured iterations)."""
    wk = small_two_beam()
    p, W0 = wk.problem, wk.U0()
    bgk.set_tiles(0, 0, mapping)
    V, _, kd = bgk.parareal_iterate(p, cuda(W0), wk.n_slices, wk.T, 2, 0.0, E=wk.E)
    Vr, _, _ = oracle.parareal_iterate(p, W0, wk.n_slices, wk.T, 2, 0.0, E=wk.E)
    assert kd == 2
    assert rel_V(V.cpu().numpy(), Vr) < TOL


def test_two_beam_batched_slices_sampled():
    """The exterior-force propagation in the launch configuration the bench
    times: all 20 slices of the two-beam test batched (lift, 21 steps, one
    per pass on v_x columns, projection) with the built-in tiles; the members
    differ by a density scale; six sampled members (first and last among
    them) against the oracle."""
    wk = wl.c6_two_beam_force()
    p, N = wk.problem, wk.n_slices
    W = wk.U0()
    V1 = np.column_stack([W[:, 0], W[:, 0:1] * W[:, 1:4],
                          0.5 * W[:, 0] * (W[:, 1:4] ** 2).sum(1) + 1.5 * W[:, 0] * W[:, 4]])
    V = np.stack([V1 * (1.0 + 0.01 * b) for b in range(N)])
    span = wk.T / N
    got = bgk.fine_propagate_moments(p, cuda(V), span, E=wk.E).cpu().numpy()
    bgk.check_status()
    for b in (0, 4, 9, 13, 16, 19):
        assert rel_V(got[b], oracle.fine_propagate_moments(p, V[b], span, E=wk.E)) < TOL
