"""The allocation-free entry point bgk_fine_propagate_moments_noalloc (its
workspace is a static device array) against bgk_fine_propagate_moments with
a caller workspace, through the C ABI: two calls in a row, the second on a
smaller grid and batch (the scratch keeps the first call's contents), both
also against the CPU oracle, at the 1e-12 normwise bar; the status output;
the size limit."""
import numpy as np
import pytest
import torch

import oracle
from paper_2502_02704_amd import bgk
from paper_2502_02704_amd import workloads as wl
from tests.gpu_util import TOL, rel_V

pytestmark = pytest.mark.gpu


def conserved(W):
    return np.column_stack([W[:, 0], W[:, 0:1] * W[:, 1:4],
                            0.5 * W[:, 0] * (W[:, 1:4] ** 2).sum(1) + 1.5 * W[:, 0] * W[:, 4]])


def members(W0, B):
    """B distinct primitive states around W0 (density, drift and temperature
    varied per member), as conserved moments [B][nx][5]."""
    out = []
    for b in range(B):
        W = W0.copy()
        W[:, 0] *= 1.0 + 0.03 * b
        W[:, 1] += 0.02 * b
        W[:, 4] *= 1.0 - 0.01 * b
        out.append(conserved(W))
    return np.stack(out)


def run_pair(p, V, span):
    Vd = torch.from_numpy(V).cuda()
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    got = bgk.fine_propagate_moments_noalloc(p, Vd, span, status=st)
    ref = bgk.fine_propagate_moments(p, Vd, span)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy(), int(st.item())


def test_noalloc_matches_workspace_call_twice_second_smaller():
    # first call: the small Sod workload's 8 slices (34.8 MiB of scratch)
    c1 = wl.c1_sod_small()
    p1, span1 = c1.problem, c1.T / c1.n_slices
    V1 = members(c1.W0, 8)
    got, ref, st = run_pair(p1, V1, span1)
    assert st == bgk.OK
    e = rel_V(got, ref)
    print(f"noalloc vs workspace call, 8 x 64 x 16^3: {e:.3e}")
    assert e <= TOL
    for b in (0, 7):
        eo = rel_V(got[b], oracle.fine_propagate_moments(p1, V1[b], span1))
        print(f"noalloc vs oracle, member {b}: {eo:.3e}")
        assert eo <= TOL
    # second call: a smaller grid and batch, laid out differently over the
    # same scratch
    p2 = wl.Problem(nx=13, nv=(12, 8, 16), v_lo=(-6, -5, -7), v_hi=(6.5, 5, 7),
                    bc=wl.BC_PERIODIC, eps=3e-3)
    x = p2.x_centres()
    W2 = np.column_stack([1 + 0.2 * np.sin(2 * np.pi * x), 0.1 * np.cos(2 * np.pi * x),
                          0 * x, 0 * x + 0.05, 0.9 + 0 * x])
    V2 = members(W2, 3)
    span2 = 0.01
    assert bgk.workspace_bytes(p2, bgk.OP_PROPAGATE, 3) < bgk.workspace_bytes(
        p1, bgk.OP_PROPAGATE, 8)
    got2, ref2, st2 = run_pair(p2, V2, span2)
    assert st2 == bgk.OK
    e2 = rel_V(got2, ref2)
    print(f"noalloc vs workspace call, 3 x 13 x 12x8x16: {e2:.3e}")
    assert e2 <= TOL
    for b in range(3):
        assert rel_V(got2[b], oracle.fine_propagate_moments(p2, V2[b], span2)) <= TOL


def test_noalloc_status_reports_each_call():
    c1 = wl.c1_sod_small()
    p, span = c1.problem, c1.T / c1.n_slices
    V = members(c1.W0, 2)
    V[1, 5, 0] = -0.25  # a negative density in one member's lift
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    bgk.fine_propagate_moments_noalloc(p, torch.from_numpy(V).cuda(), span, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == bgk.E_NONPHYSICAL
    # the next call starts from a cleared word
    bgk.fine_propagate_moments_noalloc(p, torch.from_numpy(members(c1.W0, 2)).cuda(), span,
                                       status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == bgk.OK


def test_noalloc_rejects_batches_beyond_the_scratch():
    c1 = wl.c1_sod_small()
    p, span = c1.problem, c1.T / c1.n_slices
    assert bgk.workspace_bytes(p, bgk.OP_PROPAGATE, 15) > bgk.NOALLOC_SCRATCH_BYTES
    V = torch.zeros((15, p.nx, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(bgk.BgkError) as e:
        bgk.fine_propagate_moments_noalloc(p, V, span)
    assert e.value.code == bgk.E_WORKSPACE
    assert "static scratch holds" in str(e.value)
