"""Parity of the Navier-Stokes coarse propagator (Section 1 system with the
BGK coefficients) and of parareal using it, against the CPU oracle: substep
counts bit-exact, moments at the 1e-12 normwise bar."""
import numpy as np
import pytest

import oracle
from paper_2502_02704_amd import bgk
from paper_2502_02704_amd import workloads as wl
from tests.gpu_util import TOL, rel_V
from tests.test_gpu_parity import cuda

pytestmark = pytest.mark.gpu


def smooth_states(p, seed, B):
    rng = np.random.default_rng(seed)
    x = p.x_centres()
    out = []
    for _ in range(B):
        a = rng.uniform(-1, 1, 6)
        rho = 1 + 0.3 * np.sin(2 * np.pi * x + a[0])
        u = np.column_stack([0.2 * np.cos(2 * np.pi * x + a[1]), 0.1 * np.sin(4 * np.pi * x + a[2]),
                             0.05 * np.cos(2 * np.pi * x + a[3])])
        th = 1 + 0.2 * np.cos(2 * np.pi * x + a[4])
        E = 0.5 * rho * (u ** 2).sum(1) + 1.5 * rho * th
        out.append(np.column_stack([rho, rho[:, None] * u, E]))
    return np.stack(out)


@pytest.mark.parametrize("force", [False, True])
@pytest.mark.parametrize("bc", [wl.BC_NEUMANN, wl.BC_PERIODIC])
@pytest.mark.parametrize("nx", [40, 64, 100, 200, 600, 1200])
def test_cns_coarse_matches_oracle(nx, bc, force):
    # 40 and 64 cells: one wave per conserved component; 100, 200 and 600:
    # one thread per cell (two, four and ten waves), scratch in LDS; 1200:
    # several cells per thread, scratch in global memory
    p = wl.small_problem(nx=nx, bc=bc, eps=0.02)
    V = smooth_states(p, nx + bc, 2)
    E = 0.6 * np.sin(2 * np.pi * p.x_centres()) if force else None
    got, nsub = bgk.euler_coarse_step(p, cuda(V), 0.01, E=E, coarse="cns")
    got, nsub = got.cpu().numpy(), nsub.cpu().numpy()
    for b in range(2):
        ref, nr = oracle.cns_coarse_step(p, V[b], 0.01, E=E)
        assert nsub[b] == nr
        assert rel_V(got[b], ref) < TOL


def test_cns_sod():
    p = wl.small_problem(nx=64, bc=wl.BC_NEUMANN, eps=1e-2)
    W0 = wl.riemann_W0(p, wl.SOD_LEFT, wl.SOD_RIGHT)
    V = np.column_stack([W0[:, 0], 0 * W0[:, :3], 1.5 * W0[:, 0] * W0[:, 4]])
    got, nsub = bgk.euler_coarse_step(p, cuda(V[None]), 0.05, coarse="cns")
    ref, nr = oracle.cns_coarse_step(p, V, 0.05)
    assert int(nsub[0]) == nr
    assert rel_V(got[0].cpu().numpy(), ref) < TOL


def small_smooth():
    return wl.c2_smooth_periodic(eps=1e-2, nx=32, nv=16, n_slices=6)


def test_parareal_cns_matches_oracle():
    wk = small_smooth()
    p = wk.problem
    V, err, kd = bgk.parareal_iterate(p, cuda(wk.W0), wk.n_slices, wk.T, 3, 0.0, coarse="cns")
    Vr, errr, kdr = oracle.parareal_iterate_cns(p, wk.W0, wk.n_slices, wk.T, 3, 0.0)
    assert kd == kdr == 3
    assert rel_V(V.cpu().numpy(), Vr) < TOL
    assert np.allclose(err, errr, rtol=1e-6, atol=1e-13)


def test_parareal_cns_k_equals_n_is_serial_fine():
    wk = small_smooth()
    p, N = wk.problem, wk.n_slices
    V, _, kd = bgk.parareal_iterate(p, cuda(wk.W0), N, wk.T, N, 0.0, coarse="cns")
    S = bgk.serial_fine(p, cuda(wk.W0), N, wk.T).cpu().numpy()
    assert kd == N
    assert rel_V(V.cpu().numpy(), S) < 1e-13


def test_parareal_cns_with_force_matches_oracle():
    wk = wl.c6_two_beam_force(nx=24, nv=(32, 12, 12), eps=1e-3, n_slices=4, T=0.04)
    p, W0 = wk.problem, wk.U0()
    V, err, kd = bgk.parareal_iterate(p, cuda(W0), 4, wk.T, 2, 0.0, E=wk.E, coarse="cns")
    Vr, errr, kdr = oracle.parareal_iterate_cns(p, W0, 4, wk.T, 2, 0.0, E=wk.E)
    assert kd == kdr == 2
    assert rel_V(V.cpu().numpy(), Vr) < TOL


def test_cns_needs_finite_eps():
    p = wl.small_problem(nx=8, eps=float("inf"))
    V = smooth_states(p, 1, 1)
    with pytest.raises(bgk.BgkError) as e:
        bgk.euler_coarse_step(p, cuda(V), 0.01, coarse="cns")
    assert e.value.code == bgk.E_INVALID


# ------------------------------------------- order-one (Chapman-Enskog) lift --
from tests.test_gpu_parity import GRIDS, states  # noqa: E402
from tests.gpu_util import rel_f  # noqa: E402


@pytest.mark.parametrize("name", list(GRIDS))
def test_lift_ce_matches_oracle(name):
    p = GRIDS[name]
    W, _ = states(p, 91)
    got = bgk.lift_ce(p, cuda(W)).cpu().numpy()
    bgk.check_status()
    assert rel_f(got, oracle.lift_ce(p, W)) < TOL


@pytest.mark.parametrize("name", ["sod_nx64_nv16", "wide_periodic", "even_z_ragged",
                                  "ragged_neumann"])
def test_propagate_with_order_one_lift(name):
    p = GRIDS[name]
    Vin = np.stack([smooth_states(p, 92, 1)[0], smooth_states(p, 93, 1)[0]])
    got = bgk.fine_propagate_moments(p, cuda(Vin), 0.0043, lift_order=1).cpu().numpy()
    bgk.check_status()
    for b in range(2):
        ref = oracle.fine_propagate_moments_opts(p, Vin[b], 0.0043, lift_order=1)
        assert rel_V(got[b], ref) < TOL


def test_parareal_order_one_lift_cns_matches_oracle():
    wk = small_smooth()
    p = wk.problem
    V, err, kd = bgk.parareal_iterate(p, cuda(wk.W0), wk.n_slices, wk.T, 3, 0.0,
                                      coarse="cns", lift_order=1)
    Vr, errr, kdr = oracle.parareal_iterate_opts(p, wk.W0, wk.n_slices, wk.T, 3, 0.0,
                                                 coarse="cns", lift_order=1)
    assert kd == kdr == 3
    assert rel_V(V.cpu().numpy(), Vr) < TOL
    assert np.allclose(err, errr, rtol=1e-6, atol=1e-13)


def test_parareal_order_one_lift_k_equals_n_is_serial_fine():
    wk = small_smooth()
    p, N = wk.problem, wk.n_slices
    V, _, kd = bgk.parareal_iterate(p, cuda(wk.W0), N, wk.T, N, 0.0, coarse="cns",
                                    lift_order=1)
    S = bgk.serial_fine(p, cuda(wk.W0), N, wk.T, lift_order=1).cpu().numpy()
    assert kd == N
    assert rel_V(V.cpu().numpy(), S) < 1e-13
    assert rel_V(S, oracle.serial_fine_opts(p, wk.W0, N, wk.T, lift_order=1)) < TOL


def test_order_one_lift_with_force():
    wk = wl.c6_two_beam_force(nx=24, nv=(32, 12, 12), eps=1e-3, n_slices=4, T=0.04)
    p = wk.problem
    W0 = wk.U0()
    x = p.x_centres()
    W0[:, 1] = 0.2 * np.sin(np.pi * x)  # a velocity gradient for the correction
    V, _, kd = bgk.parareal_iterate(p, cuda(W0), 4, wk.T, 2, 0.0, E=wk.E, coarse="cns",
                                    lift_order=1)
    Vr, _, kdr = oracle.parareal_iterate_opts(p, W0, 4, wk.T, 2, 0.0, E=wk.E, coarse="cns",
                                              lift_order=1)
    assert kd == kdr == 2
    assert rel_V(V.cpu().numpy(), Vr) < TOL
