"""Seeded sweep of random grid shapes through the HIP path against the oracle.

The fixed grids of the other parity tests are chosen by hand; here each case
draws its own: nx in [2, 70] (below three the fused passes fall back to
pairs), 3 to 14 velocity points per axis on an off-centre box whose spacing
keeps the Maxwellians resolved (odd and even v_z; every third case with v_x
planes of whole velocity tiles, which take the three- and four-step
passes), either boundary condition, eps from 1e-5 to 10 or
infinite (free transport), one to seven IMEX steps under every step fusion
setting (1 to 4 steps per pass) and tile shape.  Each case compares moments,
fine steps and the batched lift-propagate-project call with the oracle at the
1e-12 bar, and a batch of several drawn grids through the uneven batched call
(bit-exact step counts).  Further drawn cases cover the exterior force and the
second-order transport, the Euler and Navier-Stokes coarse steps (bit-exact
substep counts), the order-one lifting, the adjoint and parareal.
"""
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle
from paper_2502_02704_amd import bgk
from paper_2502_02704_amd import workloads as wl
from tests.gpu_util import TOL, rel_f, rel_s, rel_V, rel_W

pytestmark = pytest.mark.gpu

SEED = 250202790
N_CASES = 40
TILES = [(0, 0, -1), (2, 1, 0), (4, 5, 0), (8, 16, 0), (2, 1, 1), (4, 3, 1), (8, 64, 1)]


@pytest.fixture(autouse=True)
def _reset_tiles():
    bgk.set_tiles(0, 0, -1)
    bgk.set_step_fusion(3)
    yield
    bgk.set_tiles(0, 0, -1)
    bgk.set_step_fusion(3)


# (v_y, v_z) points whose planes are whole tiles of 128 or 256 velocities:
# such grids take the three- and four-step passes
WHOLE_TILE_PLANES = [(8, 16), (16, 8), (16, 16), (4, 32), (32, 4), (8, 32)]


def draw_problem(rng, whole_planes=False):
    """A grid of the sweep: spacing 0.45 to 1.1 per velocity axis around a
    shifted centre (thermal speed 0.7 to 1.1 stays resolved)."""
    nx = int(rng.integers(2, 71))
    nv = tuple(int(rng.integers(3, 15)) for _ in range(3))
    if whole_planes:
        nv = (int(rng.integers(3, 11)),) + WHOLE_TILE_PLANES[int(rng.integers(0, 6))]
    lo, hi = [], []
    for a in range(3):
        dv = rng.uniform(0.45, 1.1)
        c = rng.uniform(-0.6, 0.6)
        lo.append(c - 0.5 * nv[a] * dv)
        hi.append(c + 0.5 * nv[a] * dv)
    bc = int(rng.integers(0, 2))
    eps = float("inf") if rng.uniform() < 0.1 else float(10.0 ** rng.uniform(-5, 1))
    return wl.Problem(nx=nx, nv=nv, v_lo=tuple(lo), v_hi=tuple(hi), bc=bc, eps=eps)


def draw_states(rng, p):
    """Primitive moments near (1, 0, 0.8) with their lifted, perturbed field."""
    W = np.column_stack([rng.uniform(0.4, 1.4, p.nx), rng.uniform(-0.3, 0.3, (p.nx, 3)),
                         rng.uniform(0.5, 1.2, p.nx)])
    f = oracle.lift(p, W) * (1 + 0.2 * rng.uniform(-1, 1, (p.nx, p.nv3)))
    return W, f


def conserved(W):
    return np.column_stack([W[:, 0], W[:, 0:1] * W[:, 1:4],
                            0.5 * W[:, 0] * (W[:, 1:4] ** 2).sum(1) + 1.5 * W[:, 0] * W[:, 4]])


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("case", range(N_CASES))
def test_random_grid_matches_oracle(case):
    rng = np.random.default_rng(SEED + case)
    p = draw_problem(rng, whole_planes=case % 3 == 0)
    fusion = int(rng.integers(1, 5))
    tiles = TILES[int(rng.integers(0, len(TILES)))]
    n = int(rng.integers(1, 8))
    W, f = draw_states(rng, p)
    print(f"case {case}: nx={p.nx} nv={p.nv} bc={p.bc} eps={p.eps:.3g} steps={n} "
          f"fusion={fusion} tiles={tiles}", flush=True)
    bgk.set_step_fusion(fusion)
    bgk.set_tiles(*tiles)

    # moments of the perturbed field
    V, Wg = bgk.moments(p, cuda(f))
    bgk.check_status()
    Vr, Wr = oracle.moments(p, f)
    assert rel_V(V.cpu().numpy(), Vr) < TOL
    assert max(rel_W(Wg.cpu().numpy(), Wr)) < TOL

    # n IMEX steps at a step size inside the stability bound
    n_unit, dt1 = oracle.n_steps(p, 1.0)  # dt1 = 1 / n_unit: at most the stable step
    dt = 0.9 * dt1
    got = bgk.fine_steps(p, cuda(f), dt, n).cpu().numpy()
    bgk.check_status()
    assert rel_f(got, oracle.fine_steps(p, f, dt, n)) < TOL

    # lift, n steps and projection of a few slices in one batched call
    B = int(rng.integers(1, 4))
    Vin = np.stack([conserved(draw_states(rng, p)[0]) for _ in range(B)])
    span = n * dt1
    out = bgk.fine_propagate_moments(p, cuda(Vin), span).cpu().numpy()
    bgk.check_status()
    for b in range(B):
        assert rel_V(out[b], oracle.fine_propagate_moments(p, Vin[b], span)) < TOL


@pytest.mark.parametrize("batch", range(4))
def test_random_uneven_batch_matches_oracle(batch):
    """Several drawn grids (some with odd v_z, some with free transport)
    advanced over their own spans in one uneven batched call."""
    rng = np.random.default_rng(SEED + 1000 + batch)
    fusion = int(rng.integers(1, 5))
    m = int(rng.integers(2, 7))
    probs, fs, spans = [], [], []
    for i in range(m):
        p = draw_problem(rng, whole_planes=i % 2 == 1)
        # the batched call takes eps in (0, inf]; keep every instance relaxing
        # in half the cases
        if batch % 2 == 0 and p.eps == float("inf"):
            p = replace(p, eps=1e-2)
        probs.append(p)
        fs.append(draw_states(rng, p)[1])
        _, dt1 = oracle.n_steps(p, 1.0)
        spans.append(float(rng.integers(1, 9)) * dt1 * rng.uniform(0.7, 1.0))
    print(f"batch {batch}: fusion={fusion} grids=" +
          ", ".join(f"{p.nx}x{p.nv}" for p in probs), flush=True)
    bgk.set_step_fusion(fusion)
    outs, steps = bgk.fine_step_batched(probs, [cuda(f) for f in fs], spans)
    bgk.check_status()
    for q, p in enumerate(probs):
        ref, n = oracle.fine_step(p, fs[q], spans[q])
        assert int(steps[q]) == n
        assert rel_f(outs[q].cpu().numpy(), ref) < TOL


@pytest.mark.parametrize("case", range(12))
def test_random_force_and_second_order_match_oracle(case):
    """Drawn grids with a drawn exterior force (step size from the force's
    stability bound) under the first- and the second-order (van Leer
    limited) x transport."""
    rng = np.random.default_rng(SEED + 2000 + case)
    p = draw_problem(rng, whole_planes=case % 3 == 0)
    if p.eps == float("inf"):
        p = replace(p, eps=1e-3)
    E = rng.uniform(-2.0, 2.0, p.nx)
    n = int(rng.integers(1, 7))
    order = 1 + case % 2
    use_force = case % 4 != 3
    _, f = draw_states(rng, p)
    print(f"case {case}: nx={p.nx} nv={p.nv} bc={p.bc} eps={p.eps:.3g} steps={n} "
          f"order={order} force={use_force}", flush=True)
    Ef = E if use_force else None
    _, dt1 = oracle.n_steps(p, 1.0, E=Ef)
    dt = 0.9 * dt1
    got = bgk.fine_steps(p, cuda(f), dt, n, E=Ef, fine_order=order).cpu().numpy()
    bgk.check_status()
    ref = oracle.fine_steps_opts(p, f, dt, n, E=Ef, fine_order=order)
    assert rel_f(got, ref) < TOL


@pytest.mark.parametrize("case", range(12))
def test_random_coarse_steps_match_oracle(case):
    """The Euler and Navier-Stokes coarse propagators on drawn grids and
    drawn two-state data (bit-exact substep counts)."""
    rng = np.random.default_rng(SEED + 3000 + case)
    p = draw_problem(rng)
    p = replace(p, nx=int(rng.integers(2, 1300)) if case % 4 == 0 else p.nx,
                eps=float(10.0 ** rng.uniform(-5, 0)))
    coarse = "cns" if case % 2 else "euler"
    if coarse == "cns":
        # the viscous step limit cfl dx^2 / (2 eps (5/3) theta) keeps the
        # substep count in the thousands for eps <= 0.1
        p = replace(p, eps=min(p.eps, 0.1))
    B = int(rng.integers(1, 4))
    Vin = []
    for _ in range(B):
        left = (rng.uniform(0.5, 1.5), rng.uniform(-0.3, 0.3), rng.uniform(-0.2, 0.2), 0.0,
                rng.uniform(0.6, 1.2))
        right = (rng.uniform(0.1, 0.6), rng.uniform(-0.3, 0.3), 0.0, rng.uniform(-0.2, 0.2),
                 rng.uniform(0.5, 1.0))
        Vin.append(conserved(wl.riemann_W0(p, left, right, rng.uniform(0.3, 0.7))))
    Vin = np.stack(Vin)
    span = rng.uniform(0.005, 0.05)
    print(f"case {case}: nx={p.nx} bc={p.bc} eps={p.eps:.3g} batch={B} span={span:.4f} "
          f"coarse={coarse}", flush=True)
    got, nsub = bgk.euler_coarse_step(p, cuda(Vin), span, coarse=coarse)
    bgk.check_status()
    got, nsub = got.cpu().numpy(), nsub.cpu().numpy()
    for b in range(B):
        if coarse == "cns":
            ref, nr = oracle.cns_coarse_step(p, Vin[b], span)
        else:
            ref, nr = oracle.euler_coarse_step(p, Vin[b], span)
        assert int(nsub[b]) == nr
        assert rel_V(got[b], ref) < TOL


@pytest.mark.parametrize("case", range(8))
def test_random_lift_order_one_matches_oracle(case):
    """The order-one (Chapman-Enskog) lifting of drawn moments on drawn grids."""
    rng = np.random.default_rng(SEED + 4000 + case)
    p = draw_problem(rng, whole_planes=case % 2 == 0)
    p = replace(p, eps=float(10.0 ** rng.uniform(-5, -1)))
    W, _ = draw_states(rng, p)
    print(f"case {case}: nx={p.nx} nv={p.nv} bc={p.bc} eps={p.eps:.3g}", flush=True)
    got = bgk.lift_ce(p, cuda(W)).cpu().numpy()
    bgk.check_status()
    assert rel_f(got, oracle.lift_ce(p, W)) < TOL


@pytest.mark.parametrize("case", range(8))
def test_random_adjoint_matches_oracle(case):
    """The adjoint of drawn step sequences (checkpoint intervals 1 to 4) on
    drawn grids against the oracle's FP64 adjoint: f-bar at step 0 and the
    log-eps gradient."""
    rng = np.random.default_rng(SEED + 5000 + case)
    p = draw_problem(rng, whole_planes=case % 4 == 0)
    p = replace(p, nx=min(p.nx, 24), eps=float(10.0 ** rng.uniform(-4, 0)))
    n = int(rng.integers(1, 9))
    every = int(rng.integers(1, 5))
    _, f0 = draw_states(rng, p)
    _, dt1 = oracle.n_steps(p, 1.0)
    dt = 0.9 * dt1
    w = rng.standard_normal(f0.shape)
    print(f"case {case}: nx={p.nx} nv={p.nv} bc={p.bc} eps={p.eps:.3g} steps={n} "
          f"every={every}", flush=True)
    ck, _ = oracle.checkpoints(p, f0, dt, n, every)
    fb_ref, dle_ref = oracle.fine_adjoint(p, ck, every, n, dt, w)
    fb, dle = bgk.fine_adjoint(p, cuda(ck), every, n, dt, cuda(w))
    bgk.check_status()
    e_fb = rel_f(fb.cpu().numpy(), fb_ref)
    e_le = rel_s(dle.cpu(), dle_ref)
    print(f"  fbar_0 {e_fb:.2e}, log eps {e_le:.2e}", flush=True)
    assert e_fb < TOL
    assert e_le < TOL


@pytest.mark.parametrize("case", range(8))
def test_random_parareal_matches_oracle(case):
    """Algorithm 2 on drawn grids and drawn two-state data: the Euler or
    Navier-Stokes coarse model, the Maxwellian or order-one lifting, the
    first- or second-order fine transport, 2 to 6 slices and 1 to 3
    iterations (iterates at the 1e-12 bar, iteration count exact)."""
    rng = np.random.default_rng(SEED + 6000 + case)
    # resolved grids (8 to 14 points per axis over about [-6.5, 6.5]): the
    # coarse model's states and the order-one lifting stay physical
    nv = tuple(int(rng.integers(8, 15)) for _ in range(3))
    if case % 4 == 0:
        nv = (int(rng.integers(6, 11)), 16, 16)
    c = rng.uniform(-0.3, 0.3, 3)
    p = wl.Problem(nx=int(rng.integers(8, 49)), nv=nv, v_lo=tuple(c - 6.5),
                   v_hi=tuple(c + 6.5), bc=int(rng.integers(0, 2)),
                   eps=float(10.0 ** rng.uniform(-4, -2)))
    left = (rng.uniform(0.6, 1.2), rng.uniform(-0.2, 0.2), 0.0, 0.0, rng.uniform(0.7, 1.1))
    right = (rng.uniform(0.3, 0.7), rng.uniform(-0.2, 0.2), 0.0, 0.0, rng.uniform(0.6, 1.0))
    W0 = wl.riemann_W0(p, left, right, rng.uniform(0.35, 0.65))
    N = int(rng.integers(2, 7))
    T = N * rng.uniform(0.002, 0.006)
    K = int(rng.integers(1, 4))
    coarse = "cns" if case % 2 else "euler"
    lift_order = (case // 2) % 2
    fine_order = 2 if case in (5, 6) else 1
    print(f"case {case}: nx={p.nx} nv={p.nv} bc={p.bc} eps={p.eps:.3g} N={N} T={T:.4f} "
          f"K={K} coarse={coarse} lift={lift_order} order={fine_order}", flush=True)
    V, err, kd = bgk.parareal_iterate(p, cuda(W0), N, T, K, 0.0, coarse=coarse,
                                      lift_order=lift_order, fine_order=fine_order)
    bgk.check_status()
    Vr, errr, kr = oracle.parareal_iterate_opts(p, W0, N, T, K, 0.0, coarse=coarse,
                                                lift_order=lift_order, fine_order=fine_order)
    assert kd == kr == K
    assert rel_V(V.cpu().numpy(), Vr) < TOL
    assert np.allclose(err, errr, rtol=1e-6, atol=1e-13)
