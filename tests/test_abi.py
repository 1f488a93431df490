"""The C ABI library loads on a host without GPU and exports every entry
point that include/bgk.h declares (no compute calls here)."""
import ctypes
import os
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
    assert lib.bgk_set_tiles(4, 8, 2) == bgk.E_INVALID
    assert lib.bgk_set_tiles(0, 0, -1) == bgk.OK


def test_problem_struct_layout_matches_oracle():
    import oracle
    assert ctypes.sizeof(bgk._Problem) == ctypes.sizeof(oracle._Problem)
    assert [f[0] for f in bgk._Problem._fields_] == [f[0] for f in oracle._Problem._fields_]
