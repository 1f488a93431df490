"""The C ABI library loads on a host without GPU and exports every entry
point that include/bgk.h declares (no compute calls here)."""
import ctypes
import os
from dataclasses import replace
import re

import pytest

from paper_2502_02704_amd import bgk
from paper_2502_02704_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bgk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_lists_expected_entry_points():
    names = declared_functions()
    for must in ("bgk_fine_step", "bgk_moments", "euler_coarse_step", "parareal_iterate",
                 "bgk_fine_adjoint"):
        assert must in names
    assert sorted(bgk.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = bgk.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_host_only_calls():
    # argument validation, step counts and workspace sizes need no GPU
    c1 = wl.c1_sod_small()
    assert bgk.n_steps(c1.problem, c1.T / c1.n_slices)[0] == 12
    c3 = wl.c3_sod_large()
    assert bgk.n_steps(c3.problem, c3.T / c3.n_slices)[0] == 188
    assert bgk.workspace_bytes(c1.problem, bgk.OP_FINE_STEP) > 64 * 4096 * 8
    from dataclasses import replace
    assert bgk.workspace_bytes(replace(c1.problem, nx=1), bgk.OP_FINE_STEP) == 0
    assert bgk.workspace_bytes(replace(c1.problem, eps=0.0), bgk.OP_FINE_STEP) == 0
    assert bgk.workspace_bytes(replace(c1.problem, cfl=1.5), bgk.OP_FINE_STEP) == 0
    with pytest.raises(bgk.BgkError) as e:
        bgk.n_steps(replace(c1.problem, bc=7), 0.1)
    assert e.value.code == bgk.E_INVALID
    lib = bgk.load_library()
    assert lib.bgk_status_string(bgk.E_NONPHYSICAL).decode().startswith("non-physical")
    assert lib.bgk_set_tiles(3, 8, -1) == bgk.E_INVALID
    assert lib.bgk_set_tiles(4, 8, 4) == bgk.E_INVALID
    assert lib.bgk_set_tiles(4, 8, 3) == bgk.OK
    assert lib.bgk_set_tiles(4, 8, 2) == bgk.OK
    assert lib.bgk_set_tiles(0, 0, -1) == bgk.OK
    # nothing cached in a process that made no GPU call: no device call
    assert lib.bgk_release_graphs() == bgk.OK
    # steps per pass: 1, 2, 3 (the default) or 4
    for bad in (0, 5, -1):
        assert lib.bgk_set_step_fusion(bad) == bgk.E_INVALID
    for good in (1, 2, 4, 3):
        assert lib.bgk_set_step_fusion(good) == bgk.OK
    # timing kinds 0 .. BGK_PROF_FOUR_STEP_LIFT
    assert lib.bgk_prof_read(bgk.PROF_FOUR_STEP_LIFT, None, None, None, None) == bgk.OK
    assert lib.bgk_prof_read(bgk.PROF_FOUR_STEP_LIFT + 1, None, None, None, None) == bgk.E_INVALID


def test_problem_struct_layout_matches_oracle():
    import oracle
    assert ctypes.sizeof(bgk._Problem) == ctypes.sizeof(oracle._Problem)
    assert [f[0] for f in bgk._Problem._fields_] == [f[0] for f in oracle._Problem._fields_]


def test_host_side_validation_of_the_widened_entry_points():
    """Option and argument checks of the exterior-force, Navier-Stokes,
    order-one lifting and second-order calls fail before any device work."""
    from dataclasses import replace
    import oracle
    lib = bgk.load_library()
    fk = wl.c6_two_beam_force()
    p = fk.problem
    ps = ctypes.byref(bgk.problem_struct(p))
    span = fk.T / fk.n_slices
    # step rule with a force: library and oracle agree (host arithmetic only)
    assert bgk.n_steps(p, span, E=fk.E) == oracle.n_steps(p, span, E=fk.E)
    n, dt = ctypes.c_int32(), ctypes.c_double()
    assert lib.bgk_n_steps_force(ps, -1.0, span, ctypes.byref(n), ctypes.byref(dt)) == bgk.E_INVALID
    # a force call without its force array
    assert lib.bgk_fine_steps_force(ps, None, 1.0, None, None, 1e-3, 1, None, 0,
                                    None) == bgk.E_INVALID
    # the Navier-Stokes model and the order-one lifting need a finite eps
    pinf = ctypes.byref(bgk.problem_struct(replace(p, eps=float("inf"))))
    assert lib.euler_coarse_step_cns(pinf, None, 1, None, None, 0.1, None, None, 0,
                                     None) == bgk.E_INVALID
    assert lib.bgk_lift_ce(pinf, None, None, None, 0, None) == bgk.E_INVALID
    # option fields out of range
    o = bgk._Options()
    o.coarse = 7
    err = (ctypes.c_double * 1)()
    kd = ctypes.c_int32()
    assert lib.parareal_iterate_opts(ps, ctypes.byref(o), None, 4, 0.1, 1, 0.0, None, err,
                                     ctypes.byref(kd), None, 0, None) == bgk.E_INVALID
    o.coarse = 0
    o.fine_order = 3
    assert lib.bgk_fine_steps_opts(ps, ctypes.byref(o), None, None, 1e-3, 1, None, 0,
                                   None) == bgk.E_INVALID
    o.fine_order = 1
    o.lift_order = 2
    assert lib.bgk_serial_fine_opts(ps, ctypes.byref(o), None, 4, 0.1, None, None, 0,
                                    None) == bgk.E_INVALID


def test_options_struct_layout():
    # pointer, double, four int32: 32 bytes, as include/bgk.h lays it out
    assert ctypes.sizeof(bgk._Options) == 32
    assert [f[0] for f in bgk._Options._fields_] == ["E", "e_max", "coarse", "lift_order",
                                                      "fine_order", "reserved"]


def test_empty_and_oversized_batches_rejected():
    """Batch, slice and instance counts below one (and an uneven batch above
    its 4096-instance limit) are argument errors, found before any device
    work; the arrays passed here are never read."""
    lib = bgk.load_library()
    c1 = wl.c1_sod_small()
    ps = ctypes.byref(bgk.problem_struct(c1.problem))
    buf = (ctypes.c_double * 8)()
    a, b = ctypes.cast(buf, ctypes.c_void_p), ctypes.cast(ctypes.byref(buf, 32), ctypes.c_void_p)
    for batch in (0, -3):
        assert lib.bgk_fine_propagate_moments(ps, batch, a, b, 0.1, None, 0, None) == bgk.E_INVALID
        assert lib.euler_coarse_step(ps, batch, a, b, 0.1, None, None, 0, None) == bgk.E_INVALID
    err = (ctypes.c_double * 4)()
    kd = ctypes.c_int32()
    assert lib.parareal_iterate(ps, a, 0, 0.1, 2, 0.0, b, err, ctypes.byref(kd), None, 0,
                                None) == bgk.E_INVALID
    assert lib.parareal_iterate(ps, a, 4, 0.1, -1, 0.0, b, err, ctypes.byref(kd), None, 0,
                                None) == bgk.E_INVALID
    assert lib.bgk_serial_fine(ps, a, 0, 0.1, b, None, 0, None) == bgk.E_INVALID
    probs = (bgk._Problem * 1)(bgk.problem_struct(c1.problem))
    ptrs = (ctypes.c_void_p * 1)(a.value)
    outs = (ctypes.c_void_p * 1)(b.value)
    spans = (ctypes.c_double * 1)(0.1)
    for n in (0, 4097):
        assert lib.bgk_fine_step_batched(probs, n, ptrs, outs, spans, None, None, 0,
                                         None) == bgk.E_INVALID


def test_batched_workspace_holds_padded_copies_for_odd_nvz():
    """An instance with odd nv_z gets two padded fields in the uneven batch's
    workspace (each z row one point longer), an instance with even nv_z one
    field: the odd instance's workspace exceeds the even one's by at least
    the padded fields' bytes."""
    lib = bgk.load_library()
    base = wl.Problem(nx=40, nv=(6, 5, 8), v_lo=(-5,) * 3, v_hi=(5,) * 3, bc=wl.BC_NEUMANN,
                      eps=1e-2)
    odd = replace(base, nv=(6, 5, 7))

    def ws(p):
        arr = (bgk._Problem * 1)(bgk.problem_struct(p))
        return int(lib.bgk_workspace_bytes_batched(arr, 1))

    f_even = base.nx * 6 * 5 * 8 * 8
    assert ws(base) >= f_even
    # odd: two fields of nx * 6 * 5 * (7 + 1) doubles against one of the even grid's size
    assert ws(odd) - ws(base) >= 2 * f_even - f_even


def test_noalloc_size_limit_checked_on_the_host():
    """The allocation-free propagation rejects a batch whose workspace would
    exceed its static scratch, and an empty batch, before any device work
    (the arrays passed here are never read)."""
    lib = bgk.load_library()
    c1 = wl.c1_sod_small()
    ps = ctypes.byref(bgk.problem_struct(c1.problem))
    assert bgk.workspace_bytes(c1.problem, bgk.OP_PROPAGATE, 14) <= bgk.NOALLOC_SCRATCH_BYTES
    assert bgk.workspace_bytes(c1.problem, bgk.OP_PROPAGATE, 15) > bgk.NOALLOC_SCRATCH_BYTES
    buf = (ctypes.c_double * 8)()
    a, b = ctypes.cast(buf, ctypes.c_void_p), ctypes.cast(ctypes.byref(buf, 32), ctypes.c_void_p)
    assert lib.bgk_fine_propagate_moments_noalloc(ps, 15, a, b, 0.0125, None,
                                                  None) == bgk.E_WORKSPACE
    assert b"static scratch holds 67108864 bytes" in lib.bgk_last_error()
    assert lib.bgk_fine_propagate_moments_noalloc(ps, 0, a, b, 0.0125, None,
                                                  None) == bgk.E_INVALID


def test_survey_boundary_helpers_exported():
    """The helper calls of the boundary: workspace sizing, plans, the stream
    check, status strings and the last error."""
    lib = bgk.load_library()
    for name in ("bgk_workspace_bytes", "bgk_plan_create", "bgk_plan_destroy", "bgk_check",
                 "bgk_status_string", "bgk_last_error", "bgk_plan_use", "bgk_plan_info",
                 "bgk_plan_save_tiles", "bgk_plan_load_tiles", "bgk_force_bound"):
        assert hasattr(lib, name), name


def test_plans_and_tile_files_on_the_host(tmp_path):
    """A plan is created, selected, queried and destroyed without device
    work while it holds no graphs; an empty tile file round-trips; a file
    that is not a tile file, or an entry out of range, is an argument
    error."""
    lib = bgk.load_library()
    pl = bgk.Plan()
    assert pl.info() == (0, 0)
    pl.use()
    assert bgk.default_plan_info() == (0, 0)
    path = str(tmp_path / "tiles.json")
    pl.save_tiles(path)
    assert '"bgk_tiles": 1' in open(path).read()
    pl.load_tiles(path)
    assert pl.info() == (0, 0)
    bad = tmp_path / "bad.json"
    bad.write_text('{"something": 1}')
    assert lib.bgk_plan_load_tiles(pl.handle, str(bad).encode()) == bgk.E_INVALID
    bad.write_text('{"bgk_tiles": 1, "entries": [{"arch": "gfx950", "nv": [4, 4, 4], '
                   '"nx_bucket": 8, "batch_bucket": 1, "steps_per_pass": 3, "elems": 3, '
                   '"chunk": 4, "pair": 0, "ms": 1.0}]}')
    assert lib.bgk_plan_load_tiles(pl.handle, str(bad).encode()) == bgk.E_INVALID
    assert lib.bgk_plan_load_tiles(pl.handle, str(tmp_path / "missing.json").encode()) == bgk.E_INVALID
    assert lib.bgk_plan_use(None) == bgk.OK
    pl.destroy()
    assert lib.bgk_plan_destroy(None) == bgk.OK
    assert lib.bgk_plan_create(None) == bgk.E_INVALID


def test_force_bound_of_a_host_array():
    """bgk_force_bound on a host array: max |E_i| (the Rusanov coefficient),
    NaN if an entry is NaN."""
    import numpy as np
    lib = bgk.load_library()
    fk = wl.c6_two_beam_force()
    p = fk.problem
    assert bgk._emax(p, fk.E) == float(np.max(np.abs(fk.E)))
    E = fk.E.copy()
    E[7] = np.nan
    out = ctypes.c_double()
    assert lib.bgk_force_bound(ctypes.byref(bgk.problem_struct(p)), E.ctypes.data, 0,
                               ctypes.byref(out), None) == bgk.OK
    assert np.isnan(out.value)
    assert lib.bgk_force_bound(ctypes.byref(bgk.problem_struct(p)), None, 0,
                               ctypes.byref(out), None) == bgk.E_INVALID
