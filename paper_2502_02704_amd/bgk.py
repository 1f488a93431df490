"""Thin ctypes binding of libbgk.so on torch device tensors.

Every function here marshals arguments (device pointers of FP64 torch
tensors, the current HIP stream, a cached workspace) and calls the C ABI of
``include/bgk.h`` under the same name; all arithmetic of the path runs in the
library's HIP kernels.  There is no CPU fallback: if ``libbgk.so`` is not
built, or no GPU is visible, the first call raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Dict, List, Sequence, Tuple

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbgk.so")

OK, E_INVALID, E_NONPHYSICAL, E_WORKSPACE, E_HIP = 0, -1, -2, -3, -4
OP_FINE_STEP, OP_MOMENTS, OP_LIFT, OP_COARSE, OP_PROPAGATE, OP_PARAREAL, OP_ADJOINT = range(7)

EXPORTS = [
    "bgk_workspace_bytes", "bgk_workspace_bytes_batched", "bgk_n_steps", "bgk_lift",
    "bgk_moments", "bgk_fine_steps", "bgk_fine_step", "bgk_fine_step_batched",
    "bgk_fine_propagate_moments", "euler_coarse_step", "parareal_iterate",
    "bgk_serial_fine", "bgk_fine_adjoint", "bgk_lift_adjoint_rho",
    "bgk_density_adjoint", "bgk_status", "bgk_status_string", "bgk_last_error",
    "bgk_set_tiles", "bgk_autotune", "bgk_prof_enable", "bgk_prof_read",
    "bgk_set_graphs", "bgk_release_graphs", "bgk_set_step_fusion", "bgk_n_steps_force", "bgk_fine_steps_force",
    "bgk_fine_step_force", "bgk_fine_propagate_moments_force", "euler_coarse_step_force",
    "parareal_iterate_force", "bgk_serial_fine_force", "euler_coarse_step_cns",
    "parareal_iterate_cns", "bgk_lift_ce", "bgk_fine_propagate_moments_opts",
    "parareal_iterate_opts", "bgk_serial_fine_opts", "bgk_fine_steps_opts",
    "bgk_fine_propagate_moments_noalloc", "bgk_check", "bgk_plan_create", "bgk_plan_use",
    "bgk_plan_destroy", "bgk_plan_info", "bgk_plan_save_tiles", "bgk_plan_load_tiles",
    "bgk_force_bound",
]


class _Options(C.Structure):
    _fields_ = [("E", C.c_void_p), ("e_max", C.c_double), ("coarse", C.c_int32),
                ("lift_order", C.c_int32), ("fine_order", C.c_int32), ("reserved", C.c_int32)]


COARSE = {"euler": 0, "cns": 1}


class BgkError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: status {code} ({msg})")
        self.code = code


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nv", C.c_int32 * 3),
                ("x_lo", C.c_double), ("x_hi", C.c_double),
                ("v_lo", C.c_double * 3), ("v_hi", C.c_double * 3),
                ("bc", C.c_int32), ("eps", C.c_double), ("cfl", C.c_double),
                ("sound_gamma", C.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libbgk.so and declare the C signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
    L = C.CDLL(path)
    P, D, I, V = C.POINTER(_Problem), C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_void_p
    Z = C.c_size_t
    sig = {
        "bgk_workspace_bytes": (Z, [P, C.c_int32, C.c_int32]),
        "bgk_workspace_bytes_batched": (Z, [P, C.c_int32]),
        "bgk_n_steps": (C.c_int, [P, C.c_double, I, D]),
        "bgk_lift": (C.c_int, [P, V, V, V, Z, V]),
        "bgk_moments": (C.c_int, [P, V, V, V, V, Z, V]),
        "bgk_fine_steps": (C.c_int, [P, V, V, C.c_double, C.c_int32, V, Z, V]),
        "bgk_fine_step": (C.c_int, [P, V, V, C.c_double, I, V, Z, V]),
        "bgk_fine_step_batched": (C.c_int, [P, C.c_int32, C.POINTER(V), C.POINTER(V),
                                            D, I, V, Z, V]),
        "bgk_fine_propagate_moments": (C.c_int, [P, C.c_int32, V, V, C.c_double, V, Z, V]),
        "euler_coarse_step": (C.c_int, [P, C.c_int32, V, V, C.c_double, V, V, Z, V]),
        "parareal_iterate": (C.c_int, [P, V, C.c_int32, C.c_double, C.c_int32, C.c_double,
                                       V, D, I, V, Z, V]),
        "bgk_serial_fine": (C.c_int, [P, V, C.c_int32, C.c_double, V, V, Z, V]),
        "bgk_fine_adjoint": (C.c_int, [P, V, C.c_int32, C.c_int32, C.c_double, V, V, V,
                                       V, Z, V]),
        "bgk_lift_adjoint_rho": (C.c_int, [P, V, V, V, V, Z, V]),
        "bgk_density_adjoint": (C.c_int, [P, V, V, V]),
        "bgk_status": (C.c_int, [V, V]),
        "bgk_status_string": (C.c_char_p, [C.c_int]),
        "bgk_last_error": (C.c_char_p, []),
        "bgk_set_tiles": (C.c_int, [C.c_int32, C.c_int32, C.c_int32]),
        "bgk_autotune": (C.c_int, [P, C.c_int32, V, Z, V, I, I, I]),
        "bgk_prof_enable": (C.c_int, [C.c_int32]),
        "bgk_set_graphs": (C.c_int, [C.c_int32]),
        "bgk_set_step_fusion": (C.c_int, [C.c_int32]),
        "bgk_release_graphs": (C.c_int, []),
        "bgk_prof_read": (C.c_int, [C.c_int32, D, C.POINTER(C.c_int64), D, D]),
        "bgk_n_steps_force": (C.c_int, [P, C.c_double, C.c_double, I, D]),
        "bgk_fine_steps_force": (C.c_int, [P, V, C.c_double, V, V, C.c_double, C.c_int32,
                                           V, Z, V]),
        "bgk_fine_step_force": (C.c_int, [P, V, C.c_double, V, V, C.c_double, I, V, Z, V]),
        "bgk_fine_propagate_moments_force": (C.c_int, [P, V, C.c_double, C.c_int32, V, V,
                                                       C.c_double, V, Z, V]),
        "euler_coarse_step_force": (C.c_int, [P, V, C.c_int32, V, V, C.c_double, V, V, Z,
                                              V]),
        "parareal_iterate_force": (C.c_int, [P, V, C.c_double, V, C.c_int32, C.c_double,
                                             C.c_int32, C.c_double, V, D, I, V, Z, V]),
        "bgk_serial_fine_force": (C.c_int, [P, V, C.c_double, V, C.c_int32, C.c_double, V,
                                            V, Z, V]),
        "euler_coarse_step_cns": (C.c_int, [P, V, C.c_int32, V, V, C.c_double, V, V, Z, V]),
        "parareal_iterate_cns": (C.c_int, [P, V, C.c_double, V, C.c_int32, C.c_double,
                                           C.c_int32, C.c_double, V, D, I, V, Z, V]),
        "bgk_lift_ce": (C.c_int, [P, V, V, V, Z, V]),
        "bgk_fine_steps_opts": (C.c_int, [P, C.POINTER(_Options), V, V, C.c_double, C.c_int32,
                                          V, Z, V]),
        "bgk_fine_propagate_moments_opts": (C.c_int, [P, C.POINTER(_Options), C.c_int32, V,
                                                      V, C.c_double, V, Z, V]),
        "parareal_iterate_opts": (C.c_int, [P, C.POINTER(_Options), V, C.c_int32,
                                            C.c_double, C.c_int32, C.c_double, V, D, I, V,
                                            Z, V]),
        "bgk_serial_fine_opts": (C.c_int, [P, C.POINTER(_Options), V, C.c_int32, C.c_double,
                                           V, V, Z, V]),
        "bgk_fine_propagate_moments_noalloc": (C.c_int, [P, C.c_int32, V, V, C.c_double, V,
                                                         V]),
        "bgk_check": (C.c_int, [V]),
        "bgk_plan_create": (C.c_int, [C.POINTER(V)]),
        "bgk_plan_use": (C.c_int, [V]),
        "bgk_plan_destroy": (C.c_int, [V]),
        "bgk_plan_info": (C.c_int, [V, I, I]),
        "bgk_plan_save_tiles": (C.c_int, [V, C.c_char_p]),
        "bgk_plan_load_tiles": (C.c_int, [V, C.c_char_p]),
        "bgk_force_bound": (C.c_int, [P, V, C.c_int32, D, V]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _gpu_lib():
    L = load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("libbgk needs a visible gfx950 GPU")
    return L


def problem_struct(p) -> _Problem:
    s = _Problem()
    s.nx = int(p.nx)
    for a in range(3):
        s.nv[a] = int(p.nv[a])
        s.v_lo[a] = float(p.v_lo[a])
        s.v_hi[a] = float(p.v_hi[a])
    s.x_lo, s.x_hi = float(p.x_lo), float(p.x_hi)
    s.bc = int(p.bc)
    s.eps = float(p.eps)
    s.cfl = float(p.cfl)
    s.sound_gamma = float(p.sound_gamma)
    return s


def _check(rc: int, where: str):
    if rc != OK:
        msg = load_library().bgk_last_error().decode()
        raise BgkError(rc, where, msg or load_library().bgk_status_string(rc).decode())


def _dev(t: torch.Tensor, name: str) -> int:
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _f64(x, device="cuda") -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(x, dtype=torch.float64, device=device).contiguous()


# ------------------------------------------------------------- workspaces --
_ws: Dict[tuple, torch.Tensor] = {}
_last_ws: List[torch.Tensor] = []


def _key(p):
    return (p.nx, tuple(p.nv), p.x_lo, p.x_hi, tuple(p.v_lo), tuple(p.v_hi))


def workspace_bytes(p, op: int, batch: int = 1) -> int:
    return int(load_library().bgk_workspace_bytes(C.byref(problem_struct(p)), op, batch))


def workspace(p, op: int, batch: int = 1) -> torch.Tensor:
    """Cached zero-initialised device workspace for (grid, op, batch)."""
    key = (_key(p), op, batch)
    w = _ws.get(key)
    if w is None:
        n = workspace_bytes(p, op, batch)
        if n == 0:
            raise BgkError(E_INVALID, "workspace_bytes", "invalid problem")
        w = torch.zeros(n, dtype=torch.uint8, device="cuda")
        _ws[key] = w
    _last_ws[:] = [w]
    return w


def _drain():
    """bgk_check on the current stream before workspaces are released (the
    library reads the status of every workspace a call used since the last
    check, so none may be freed before it)."""
    if _lib is not None and torch.cuda.is_available():
        _lib.bgk_check(C.c_void_p(_stream()))


def free_workspaces():
    _drain()
    _ws.clear()
    _last_ws.clear()
    _batched_ws.clear()


def status(ws: torch.Tensor | None = None) -> int:
    """Synchronise and return/clear the sticky status: of one workspace, or
    (ws None) of every workspace the calls on the current stream used since
    the last check (bgk_check)."""
    L = _gpu_lib()
    if ws is not None:
        return int(L.bgk_status(C.c_void_p(ws.data_ptr()), C.c_void_p(_stream())))
    return int(L.bgk_check(C.c_void_p(_stream())))


def check_status(ws: torch.Tensor | None = None):
    _check(status(ws), "device status")


# ------------------------------------------------------------ operations --
# Functions taking E=None also run the exterior-force variant of the method
# when E (force at the x centres, [nx], numpy or tensor) is given; its Rusanov
# coefficient e_max is max |E_i| of those values.
def _emax(p, E) -> float:
    """The library's Rusanov coefficient max_i |E_i| (bgk_force_bound)."""
    L = load_library()
    out = C.c_double()
    if isinstance(E, torch.Tensor) and E.is_cuda:
        Ed = E.detach().to(torch.float64).contiguous()
        rc = L.bgk_force_bound(C.byref(problem_struct(p)), Ed.data_ptr(), 1, C.byref(out),
                               _stream())
    else:
        Eh = np.ascontiguousarray(
            E.detach().cpu().numpy() if isinstance(E, torch.Tensor) else E, dtype=np.float64)
        if Eh.shape != (p.nx,):
            raise ValueError(f"E must have shape ({p.nx},)")
        rc = L.bgk_force_bound(C.byref(problem_struct(p)), Eh.ctypes.data, 0, C.byref(out), None)
    _check(rc, "bgk_force_bound")
    return out.value


def _force(p, E):
    """(device [nx] float64 tensor, e_max) of an exterior force."""
    Ed = _f64(E)
    if Ed.shape != (p.nx,):
        raise ValueError(f"E must have shape ({p.nx},)")
    return Ed, _emax(p, Ed)


def n_steps(p, t_span: float, E=None) -> Tuple[int, float]:
    n, dt = C.c_int32(), C.c_double()
    L = load_library()
    if E is None:
        rc = L.bgk_n_steps(C.byref(problem_struct(p)), t_span, C.byref(n), C.byref(dt))
    else:
        rc = L.bgk_n_steps_force(C.byref(problem_struct(p)), _emax(p, E), t_span, C.byref(n),
                                 C.byref(dt))
    _check(rc, "bgk_n_steps")
    return n.value, dt.value


def lift(p, W) -> torch.Tensor:
    L = _gpu_lib()
    W = _f64(W)
    f = torch.empty((p.nx, p.nv[0] * p.nv[1] * p.nv[2]), dtype=torch.float64, device="cuda")
    w = workspace(p, OP_LIFT)
    _check(L.bgk_lift(C.byref(problem_struct(p)), _dev(W, "W"), _dev(f, "f"),
                      w.data_ptr(), w.numel(), _stream()), "bgk_lift")
    return f


def lift_ce(p, W) -> torch.Tensor:
    """Lifting of order one (first Chapman-Enskog correction) of primitive W."""
    L = _gpu_lib()
    W = _f64(W)
    f = torch.empty((p.nx, p.nv[0] * p.nv[1] * p.nv[2]), dtype=torch.float64, device="cuda")
    w = workspace(p, OP_LIFT)
    _check(L.bgk_lift_ce(C.byref(problem_struct(p)), _dev(W, "W"), _dev(f, "f"),
                         w.data_ptr(), w.numel(), _stream()), "bgk_lift_ce")
    return f


def _options(p, E, coarse: str, lift_order: int, fine_order: int = 1):
    """(ctypes options, device force tensor kept alive by the caller)."""
    if coarse not in COARSE:
        raise ValueError("coarse must be 'euler' or 'cns'")
    o = _Options()
    Ed = None
    if E is not None:
        Ed, o.e_max = _force(p, E)
        o.E = Ed.data_ptr()
    o.coarse = COARSE[coarse]
    o.lift_order = int(lift_order)
    o.fine_order = int(fine_order)
    return o, Ed


def moments(p, f: torch.Tensor):
    L = _gpu_lib()
    V = torch.empty((p.nx, 5), dtype=torch.float64, device="cuda")
    W = torch.empty((p.nx, 5), dtype=torch.float64, device="cuda")
    w = workspace(p, OP_MOMENTS)
    _check(L.bgk_moments(C.byref(problem_struct(p)), _dev(f, "f"), V.data_ptr(),
                         W.data_ptr(), w.data_ptr(), w.numel(), _stream()), "bgk_moments")
    return V, W


def fine_steps(p, f: torch.Tensor, dt: float, n: int, out: torch.Tensor | None = None,
               E=None, fine_order: int = 1):
    """n IMEX steps of size dt; fine_order 2 = van Leer limited x transport."""
    L = _gpu_lib()
    out = torch.empty_like(f) if out is None else out
    w = workspace(p, OP_FINE_STEP)
    ps = C.byref(problem_struct(p))
    if fine_order != 1:
        o, Ed = _options(p, E, "euler", 0, fine_order)
        rc = L.bgk_fine_steps_opts(ps, C.byref(o), _dev(f, "f_in"), _dev(out, "f_out"), dt, n,
                                   w.data_ptr(), w.numel(), _stream())
    elif E is None:
        rc = L.bgk_fine_steps(ps, _dev(f, "f_in"), _dev(out, "f_out"), dt, n, w.data_ptr(),
                              w.numel(), _stream())
    else:
        Ed, emax = _force(p, E)
        rc = L.bgk_fine_steps_force(ps, _dev(Ed, "E"), emax, _dev(f, "f_in"),
                                    _dev(out, "f_out"), dt, n, w.data_ptr(), w.numel(),
                                    _stream())
    _check(rc, "bgk_fine_steps")
    return out


def fine_step(p, f: torch.Tensor, t_span: float, out: torch.Tensor | None = None, E=None):
    L = _gpu_lib()
    out = torch.empty_like(f) if out is None else out
    n = C.c_int32()
    w = workspace(p, OP_FINE_STEP)
    ps = C.byref(problem_struct(p))
    if E is None:
        rc = L.bgk_fine_step(ps, _dev(f, "f_in"), _dev(out, "f_out"), t_span, C.byref(n),
                             w.data_ptr(), w.numel(), _stream())
    else:
        Ed, emax = _force(p, E)
        rc = L.bgk_fine_step_force(ps, _dev(Ed, "E"), emax, _dev(f, "f_in"),
                                   _dev(out, "f_out"), t_span, C.byref(n), w.data_ptr(),
                                   w.numel(), _stream())
    _check(rc, "bgk_fine_step")
    return out, n.value


_batched_ws: Dict[tuple, torch.Tensor] = {}


def fine_step_batched(probs: Sequence, fs: Sequence[torch.Tensor], spans: Sequence[float],
                      outs: Sequence[torch.Tensor] | None = None):
    """Uneven batch: instance q advances fs[q] by spans[q] on its own grid
    (bgk_fine_step_batched).  Returns (outputs, step counts)."""
    L = _gpu_lib()
    n = len(probs)
    arr = (_Problem * n)(*[problem_struct(p) for p in probs])
    outs = [torch.empty_like(f) for f in fs] if outs is None else list(outs)
    fin = (C.c_void_p * n)(*[_dev(f, "f_in") for f in fs])
    fout = (C.c_void_p * n)(*[_dev(o, "f_out") for o in outs])
    sp = (C.c_double * n)(*[float(s) for s in spans])
    steps = (C.c_int32 * n)()
    nb = int(L.bgk_workspace_bytes_batched(arr, n))
    if nb == 0:
        raise BgkError(E_INVALID, "bgk_workspace_bytes_batched", "invalid problems")
    key = tuple(_key(p) for p in probs)
    w = _batched_ws.get(key)
    if w is None or w.numel() < nb:
        w = torch.zeros(nb, dtype=torch.uint8, device="cuda")
        _drain()
        _batched_ws.clear()
        _batched_ws[key] = w
    _last_ws[:] = [w]
    _check(L.bgk_fine_step_batched(arr, n, fin, fout, sp, steps, w.data_ptr(), w.numel(),
                                   _stream()), "bgk_fine_step_batched")
    return outs, list(steps)


def fine_propagate_moments(p, V_in: torch.Tensor, t_span: float, E=None,
                           lift_order: int = 0, fine_order: int = 1) -> torch.Tensor:
    """Batched P F L over the leading dimension of V_in ([B][nx][5] conserved);
    lift_order 1 lifts with the first Chapman-Enskog correction."""
    L = _gpu_lib()
    V_in = V_in.contiguous()
    B = V_in.shape[0] if V_in.dim() == 3 else 1
    out = torch.empty_like(V_in)
    w = workspace(p, OP_PROPAGATE, B)
    ps = C.byref(problem_struct(p))
    if lift_order != 0 or fine_order != 1:
        o, Ed = _options(p, E, "euler", lift_order, fine_order)
        rc = L.bgk_fine_propagate_moments_opts(ps, C.byref(o), B, _dev(V_in, "V_in"),
                                               _dev(out, "V_out"), t_span, w.data_ptr(),
                                               w.numel(), _stream())
    elif E is None:
        rc = L.bgk_fine_propagate_moments(ps, B, _dev(V_in, "V_in"), _dev(out, "V_out"),
                                          t_span, w.data_ptr(), w.numel(), _stream())
    else:
        Ed, emax = _force(p, E)
        rc = L.bgk_fine_propagate_moments_force(ps, _dev(Ed, "E"), emax, B,
                                                _dev(V_in, "V_in"), _dev(out, "V_out"),
                                                t_span, w.data_ptr(), w.numel(), _stream())
    _check(rc, "bgk_fine_propagate_moments")
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20  # BGK_NOALLOC_SCRATCH_BYTES


def fine_propagate_moments_noalloc(p, V_in: torch.Tensor, t_span: float,
                                   out: torch.Tensor | None = None,
                                   status: torch.Tensor | None = None) -> torch.Tensor:
    """bgk_fine_propagate_moments_noalloc: the batched P F L of
    fine_propagate_moments with the library's static scratch instead of a
    workspace.  `out` ([B][nx][5]) and `status` (int32 device scalar, receives
    BGK_OK or BGK_E_NONPHYSICAL) are optional caller-owned outputs."""
    L = _gpu_lib()
    V_in = V_in.contiguous()
    B = V_in.shape[0] if V_in.dim() == 3 else 1
    out = torch.empty_like(V_in) if out is None else out
    if status is not None and not (status.is_cuda and status.dtype == torch.int32):
        raise TypeError("status must be an int32 CUDA tensor")
    _check(L.bgk_fine_propagate_moments_noalloc(
        C.byref(problem_struct(p)), B, _dev(V_in, "V_in"), _dev(out, "V_out"), t_span,
        status.data_ptr() if status is not None else None, _stream()),
        "bgk_fine_propagate_moments_noalloc")
    return out


def euler_coarse_step(p, V: torch.Tensor, t_span: float, E=None, coarse: str = "euler"):
    """Coarse propagator over t_span for each member of V ([B][nx][5]);
    coarse = "euler" (Section 3.2) or "cns" (Navier-Stokes, BGK coefficients)."""
    L = _gpu_lib()
    V = V.contiguous()
    B = V.shape[0] if V.dim() == 3 else 1
    out = torch.empty_like(V)
    nsub = torch.zeros(B, dtype=torch.int32, device="cuda")
    w = workspace(p, OP_COARSE, B)
    ps = C.byref(problem_struct(p))
    if coarse not in ("euler", "cns"):
        raise ValueError("coarse must be 'euler' or 'cns'")
    if coarse == "cns":
        Ed = _force(p, E)[0] if E is not None else None
        rc = L.euler_coarse_step_cns(ps, _dev(Ed, "E") if Ed is not None else None, B,
                                     _dev(V, "V_in"), _dev(out, "V_out"), t_span,
                                     nsub.data_ptr(), w.data_ptr(), w.numel(), _stream())
    elif E is None:
        rc = L.euler_coarse_step(ps, B, _dev(V, "V_in"), _dev(out, "V_out"), t_span,
                                 nsub.data_ptr(), w.data_ptr(), w.numel(), _stream())
    else:
        Ed, _ = _force(p, E)
        rc = L.euler_coarse_step_force(ps, _dev(Ed, "E"), B, _dev(V, "V_in"),
                                       _dev(out, "V_out"), t_span, nsub.data_ptr(),
                                       w.data_ptr(), w.numel(), _stream())
    _check(rc, "euler_coarse_step")
    return out, nsub


def parareal_iterate(p, W0, n_slices: int, T: float, k_max: int, tol: float, E=None,
                     coarse: str = "euler", lift_order: int = 0, fine_order: int = 1):
    """Algorithm 2; coarse = "euler" or "cns" (Navier-Stokes coarse propagator);
    lift_order 1 = the order-one (Chapman-Enskog) lifting."""
    L = _gpu_lib()
    W0 = _f64(W0)
    V = torch.empty((n_slices + 1, p.nx, 5), dtype=torch.float64, device="cuda")
    err = (C.c_double * max(k_max, 1))()
    kd = C.c_int32()
    w = workspace(p, OP_PARAREAL, n_slices)
    ps = C.byref(problem_struct(p))
    if coarse not in ("euler", "cns"):
        raise ValueError("coarse must be 'euler' or 'cns'")
    if lift_order != 0 or fine_order != 1:
        o, Ed = _options(p, E, coarse, lift_order, fine_order)
        rc = L.parareal_iterate_opts(ps, C.byref(o), _dev(W0, "W0"), n_slices, T, k_max, tol,
                                     _dev(V, "V_out"), err, C.byref(kd), w.data_ptr(),
                                     w.numel(), _stream())
    elif coarse == "cns":
        Ed, emax = _force(p, E) if E is not None else (None, 0.0)
        rc = L.parareal_iterate_cns(ps, _dev(Ed, "E") if Ed is not None else None, emax,
                                    _dev(W0, "W0"), n_slices, T, k_max, tol, _dev(V, "V_out"),
                                    err, C.byref(kd), w.data_ptr(), w.numel(), _stream())
    elif E is None:
        rc = L.parareal_iterate(ps, _dev(W0, "W0"), n_slices, T, k_max, tol,
                                _dev(V, "V_out"), err, C.byref(kd), w.data_ptr(), w.numel(),
                                _stream())
    else:
        Ed, emax = _force(p, E)
        rc = L.parareal_iterate_force(ps, _dev(Ed, "E"), emax, _dev(W0, "W0"), n_slices, T,
                                      k_max, tol, _dev(V, "V_out"), err, C.byref(kd),
                                      w.data_ptr(), w.numel(), _stream())
    _check(rc, "parareal_iterate")
    return V, [err[i] for i in range(kd.value)], kd.value


def serial_fine(p, W0, n_slices: int, T: float, E=None, lift_order: int = 0,
                fine_order: int = 1) -> torch.Tensor:
    """The chained serial fine reference U^n = P F L(U^{n-1})."""
    L = _gpu_lib()
    W0 = _f64(W0)
    V = torch.empty((n_slices + 1, p.nx, 5), dtype=torch.float64, device="cuda")
    w = workspace(p, OP_PARAREAL, n_slices)
    ps = C.byref(problem_struct(p))
    if lift_order != 0 or fine_order != 1:
        o, Ed = _options(p, E, "euler", lift_order, fine_order)
        rc = L.bgk_serial_fine_opts(ps, C.byref(o), _dev(W0, "W0"), n_slices, T,
                                    _dev(V, "V_out"), w.data_ptr(), w.numel(), _stream())
    elif E is None:
        rc = L.bgk_serial_fine(ps, _dev(W0, "W0"), n_slices, T, _dev(V, "V_out"),
                               w.data_ptr(), w.numel(), _stream())
    else:
        Ed, emax = _force(p, E)
        rc = L.bgk_serial_fine_force(ps, _dev(Ed, "E"), emax, _dev(W0, "W0"), n_slices, T,
                                     _dev(V, "V_out"), w.data_ptr(), w.numel(), _stream())
    _check(rc, "bgk_serial_fine")
    return V


def fine_adjoint(p, f_ckpt: torch.Tensor, ckpt_every: int, n: int, dt: float,
                 fbar_T: torch.Tensor, dlog_eps: torch.Tensor | None = None):
    L = _gpu_lib()
    fbar0 = torch.empty_like(fbar_T)
    dle = torch.zeros(1, dtype=torch.float64, device="cuda") if dlog_eps is None else dlog_eps
    w = workspace(p, OP_ADJOINT, ckpt_every)
    _check(L.bgk_fine_adjoint(C.byref(problem_struct(p)), _dev(f_ckpt, "f_ckpt"), ckpt_every,
                              n, dt, _dev(fbar_T, "fbar_T"), _dev(fbar0, "fbar_0"),
                              _dev(dle, "dlog_eps"), w.data_ptr(), w.numel(), _stream()),
           "bgk_fine_adjoint")
    return fbar0, dle


def lift_adjoint_rho(p, W, fbar: torch.Tensor) -> torch.Tensor:
    L = _gpu_lib()
    W = _f64(W)
    rb = torch.empty(p.nx, dtype=torch.float64, device="cuda")
    w = workspace(p, OP_LIFT)
    _check(L.bgk_lift_adjoint_rho(C.byref(problem_struct(p)), _dev(W, "W"), _dev(fbar, "fbar"),
                                  _dev(rb, "rhobar"), w.data_ptr(), w.numel(), _stream()),
           "bgk_lift_adjoint_rho")
    return rb


def density_adjoint(p, rhobar: torch.Tensor) -> torch.Tensor:
    L = _gpu_lib()
    fbar = torch.empty((p.nx, p.nv[0] * p.nv[1] * p.nv[2]), dtype=torch.float64, device="cuda")
    _check(L.bgk_density_adjoint(C.byref(problem_struct(p)), _dev(rhobar.contiguous(), "rhobar"),
                                 _dev(fbar, "fbar"), _stream()), "bgk_density_adjoint")
    return fbar


def set_tiles(elems: int = 0, chunk: int = 0, pair: int = -1):
    """Tile shape of the step kernels (0 / -1: built-in).  pair: 1 paired
    v_z lanes, 0 one velocity per lane slot; the exterior-force step on v_x
    columns with 2 one, 3 two (v_y, v_z) points per lane."""
    _check(load_library().bgk_set_tiles(elems, chunk, pair), "bgk_set_tiles")


def autotune(p, batch: int = 1) -> Tuple[int, int, int]:
    L = _gpu_lib()
    w = workspace(p, OP_PROPAGATE, batch)
    e, c, pr = C.c_int32(), C.c_int32(), C.c_int32()
    _check(L.bgk_autotune(C.byref(problem_struct(p)), batch, w.data_ptr(), w.numel(),
                          _stream(), C.byref(e), C.byref(c), C.byref(pr)), "bgk_autotune")
    return e.value, c.value, pr.value


class Plan:
    """A library plan (captured graphs, tuned tiles, the workspace registry
    of bgk_check); `with Plan() as pl:` makes it the calling thread's plan
    for the block and destroys it afterwards."""

    def __init__(self):
        h = C.c_void_p()
        _check(load_library().bgk_plan_create(C.byref(h)), "bgk_plan_create")
        self.handle = h

    def use(self):
        _check(load_library().bgk_plan_use(self.handle), "bgk_plan_use")

    def info(self) -> Tuple[int, int]:
        g, t = C.c_int32(), C.c_int32()
        _check(load_library().bgk_plan_info(self.handle, C.byref(g), C.byref(t)),
               "bgk_plan_info")
        return g.value, t.value

    def save_tiles(self, path: str):
        _check(load_library().bgk_plan_save_tiles(self.handle, path.encode()),
               "bgk_plan_save_tiles")

    def load_tiles(self, path: str):
        _check(load_library().bgk_plan_load_tiles(self.handle, path.encode()),
               "bgk_plan_load_tiles")

    def destroy(self):
        if self.handle:
            _drain()
            _check(load_library().bgk_plan_destroy(self.handle), "bgk_plan_destroy")
            self.handle = None

    def __enter__(self):
        self.use()
        return self

    def __exit__(self, *exc):
        self.destroy()
        return False


def default_plan_info() -> Tuple[int, int]:
    """(graphs, tuned tile shapes) held by the calling thread's plan."""
    g, t = C.c_int32(), C.c_int32()
    _check(load_library().bgk_plan_info(None, C.byref(g), C.byref(t)), "bgk_plan_info")
    return g.value, t.value


def save_tiles(path: str):
    """The calling thread's plan's tuned tiles as JSON (bgk_plan_save_tiles)."""
    _check(load_library().bgk_plan_save_tiles(None, path.encode()), "bgk_plan_save_tiles")


def load_tiles(path: str):
    """Merge a tile file into the calling thread's plan (bgk_plan_load_tiles)."""
    _check(load_library().bgk_plan_load_tiles(None, path.encode()), "bgk_plan_load_tiles")


def release_graphs():
    """Destroy every cached HIP graph (synchronises the device)."""
    _check(load_library().bgk_release_graphs(), "bgk_release_graphs")


def set_graphs(on: bool = True):
    """Capture/replay launch-bound sequences as HIP graphs (default on)."""
    _check(load_library().bgk_set_graphs(1 if on else 0), "bgk_set_graphs")


def set_step_fusion(steps_per_pass: int = 3):
    """IMEX steps per read-write pass over f: 1, 2 (fused pairs), 3 (fused
    triples where every velocity tile lies in one v_x plane, else pairs;
    the default) or 4 (quads where the grid allows, else as 3)."""
    _check(load_library().bgk_set_step_fusion(steps_per_pass), "bgk_set_step_fusion")


def prof_enable(on: bool = True):
    _check(load_library().bgk_prof_enable(1 if on else 0), "bgk_prof_enable")


PROF_ALL, PROF_TWO_STEP, PROF_TWO_STEP_LIFT, PROF_ONE_STEP = 0, 1, 2, 3
PROF_THREE_STEP, PROF_THREE_STEP_LIFT = 4, 5
PROF_FOUR_STEP, PROF_FOUR_STEP_LIFT = 6, 7


def prof_read(kind: int = PROF_ALL):
    """(kernel milliseconds, launches, phase-space updates, algorithmic bytes)
    of the step-kernel launches of `kind` since prof_enable(True)."""
    ms, n, cells, by = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
    _check(load_library().bgk_prof_read(kind, C.byref(ms), C.byref(n), C.byref(cells),
                                        C.byref(by)), "bgk_prof_read")
    return ms.value, n.value, cells.value, by.value


# ------------------------------------------------------------- autograd --
class KineticDensity(torch.autograd.Function):
    """rho(T) of the fine propagator started from the lifted Maxwellian
    M[rho0, u0, theta0], differentiable in rho0 and log(eps).

    forward: lift -> n IMEX steps (checkpoints every `ckpt_every` steps)
    -> density; backward: density adjoint -> fine adjoint (recomputing each
    checkpoint segment) -> lift adjoint.  All steps run in libbgk kernels."""

    @staticmethod
    def forward(ctx, rho0, log_eps, prob, u0, theta0, T, ckpt_every):
        from dataclasses import replace
        eps = math.exp(float(log_eps.detach().cpu()))
        p = replace(prob, eps=eps)
        nx = p.nx
        W = torch.zeros((nx, 5), dtype=torch.float64, device="cuda")
        W[:, 0] = rho0.detach()
        W[:, 1:4] = _f64(u0).reshape(-1, 3) if not isinstance(u0, float) else u0
        W[:, 4] = theta0
        n, dt = n_steps(p, T)
        f = lift(p, W)
        n_ck = (n + ckpt_every - 1) // ckpt_every
        ck = torch.empty((n_ck,) + tuple(f.shape), dtype=torch.float64, device="cuda")
        for c in range(n_ck):
            ck[c].copy_(f)
            m = min(ckpt_every, n - c * ckpt_every)
            f = fine_steps(p, f, dt, m)
        _, Wt = moments(p, f)
        ctx.save_for_backward(ck, W)
        ctx.p, ctx.n, ctx.dt, ctx.ckpt_every = p, n, dt, ckpt_every
        return Wt[:, 0].clone()

    @staticmethod
    def backward(ctx, grad_rho):
        ck, W = ctx.saved_tensors
        p = ctx.p
        fbar = density_adjoint(p, grad_rho.contiguous().to(torch.float64))
        fbar0, dle = fine_adjoint(p, ck, ctx.ckpt_every, ctx.n, ctx.dt, fbar)
        rb = lift_adjoint_rho(p, W, fbar0)
        return rb, dle.reshape(()), None, None, None, None, None


def kinetic_density(rho0, log_eps, prob, u0=0.0, theta0=1.0, T=0.1, ckpt_every=16):
    return KineticDensity.apply(rho0, log_eps, prob, u0, theta0, T, ckpt_every)
