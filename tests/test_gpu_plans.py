"""Plans (the library's caches between calls), the stream-wide status check
and tuned-tile files, through the C ABI on the GPU."""
import json

import numpy as np
import pytest
import torch

import oracle
from paper_2502_02704_amd import bgk
from paper_2502_02704_amd import workloads as wl
from tests.gpu_util import TOL, rel_V
from tests.test_gpu_parity import GRIDS, cuda, states

pytestmark = pytest.mark.gpu


def test_parareal_replays_through_a_plan():
    """Parareal iterations captured into a plan of their own and replayed
    from it equal the same calls on the default plan; destroying the plan
    releases its graphs and leaves the default plan's untouched."""
    wk = wl.c1_sod_small()
    p, W0 = wk.problem, cuda(wk.W0)
    V0, err0, _ = bgk.parareal_iterate(p, W0, wk.n_slices, wk.T, 3, 0.0)
    g_default = bgk.default_plan_info()[0]
    assert g_default > 0
    with bgk.Plan() as pl:
        assert pl.info() == (0, 0)
        outs = []
        for _ in range(3):
            V, err, kd = bgk.parareal_iterate(p, W0, wk.n_slices, wk.T, 3, 0.0)
            outs.append((V.cpu().numpy(), err))
        n_graphs = pl.info()[0]
        assert n_graphs >= 3  # the iterations of this call shape
        assert bgk.default_plan_info()[0] == n_graphs  # the thread's plan is this one
    assert bgk.default_plan_info()[0] == g_default
    for V, err in outs:
        assert np.array_equal(V, V0.cpu().numpy()) and err == err0
    Vr, _, _ = oracle.parareal_iterate(p, wk.W0, wk.n_slices, wk.T, 3, 0.0)
    assert rel_V(outs[-1][0], Vr) < TOL


def test_stream_check_reads_every_workspace_used():
    """A non-physical lift flags its workspace; a later healthy call on
    another workspace does not hide it from the stream-wide check, which
    clears both."""
    p = GRIDS["ragged_neumann"]
    W, f = states(p, 40)
    W[3, 4] = -0.5
    bgk.lift(p, cuda(W))              # BGK_OP_LIFT workspace: flagged
    bgk.moments(p, cuda(f))           # BGK_OP_MOMENTS workspace: healthy
    assert bgk.status() == bgk.E_NONPHYSICAL
    assert bgk.status() == bgk.OK


def test_autotuned_tiles_saved_loaded_and_used(tmp_path):
    """bgk_autotune on a grid class no other test uses stores its choice in
    the plan; the JSON file written from it carries this device's
    architecture; another plan loads it and its calls, which take the tuned
    shape, still match the oracle."""
    p = wl.Problem(nx=30, nv=(8, 16, 16), v_lo=(-6,) * 3, v_hi=(6,) * 3, bc=wl.BC_NEUMANN,
                   eps=5e-3)
    B = 3
    path = str(tmp_path / "tiles.json")
    with bgk.Plan() as pl:
        e, c, pr = bgk.autotune(p, B)
        assert pl.info()[1] == 1
        pl.save_tiles(path)
    entries = json.load(open(path))["entries"]
    assert len(entries) == 1
    en = entries[0]
    assert en["arch"].startswith("gfx") and en["nv"] == [8, 16, 16]
    assert (en["nx_bucket"], en["batch_bucket"], en["steps_per_pass"]) == (32, 4, 3)
    assert (en["elems"], en["chunk"], en["pair"]) == (e, c, pr)
    Vin = np.stack([np.column_stack([w[:, 0], w[:, 0:1] * w[:, 1:4],
                                     0.5 * w[:, 0] * (w[:, 1:4] ** 2).sum(1) + 1.5 * w[:, 0] * w[:, 4]])
                    for w in (states(p, 700 + b)[0] for b in range(B))])
    span = 0.003
    with bgk.Plan() as pl2:
        pl2.load_tiles(path)
        assert pl2.info()[1] == 1
        got = bgk.fine_propagate_moments(p, cuda(Vin), span).cpu().numpy()
        bgk.check_status()
    for b in range(B):
        assert rel_V(got[b], oracle.fine_propagate_moments(p, Vin[b], span)) < TOL


def test_force_bound_of_a_device_array():
    fk = wl.c6_two_beam_force()
    assert bgk._emax(fk.problem, cuda(fk.E)) == float(np.max(np.abs(fk.E)))
