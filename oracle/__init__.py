"""ctypes front end of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Plain FP64 CPU reference of the method of Laidin & Rey (arXiv 2502.02704):
lifting and projection (Section 2.1, 3.3), IMEX upwind/BGK fine propagator
(Section 3.1), Rusanov Euler coarse propagator (Section 3.2), optimised
parareal (Algorithm 2) and the adjoint of the fine propagator.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

OK = 0
E_INVALID = -1
E_NONPHYSICAL = -2


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"oracle {where} failed with status {code}")
        self.code = code


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nv", C.c_int32 * 3),
                ("x_lo", C.c_double), ("x_hi", C.c_double),
                ("v_lo", C.c_double * 3), ("v_hi", C.c_double * 3),
                ("bc", C.c_int32), ("eps", C.c_double), ("cfl", C.c_double),
                ("sound_gamma", C.c_double)]


_lib = None
_lib_path = LIB_PATH


def use_library(path: str | None = None) -> None:
    """Load the oracle from another build of the same source (the host-tuned
    build the benchmark times); None returns to the portable build."""
    global _lib, _lib_path
    _lib = None
    _lib_path = path or LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if _lib_path == LIB_PATH and not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_lib_path)
        P = C.POINTER(_Problem)
        D = C.POINTER(C.c_double)
        I = C.POINTER(C.c_int32)
        sig = {
            "bgk_oracle_n_steps": [P, C.c_double, I, D],
            "bgk_oracle_lift": [P, D, D],
            "bgk_oracle_moments": [P, D, D, D],
            "bgk_oracle_transport": [P, D, C.c_double, D],
            "bgk_oracle_relax": [P, D, C.c_double, D],
            "bgk_oracle_fine_steps": [P, D, D, C.c_double, C.c_int32],
            "bgk_oracle_fine_step": [P, D, D, C.c_double, I],
            "bgk_oracle_fine_propagate_moments": [P, D, D, C.c_double],
            "bgk_oracle_euler_coarse_step": [P, D, D, C.c_double, I],
            "bgk_oracle_parareal_iterate": [P, D, C.c_int32, C.c_double, C.c_int32,
                                            C.c_double, D, D, I],
            "bgk_oracle_serial_fine": [P, D, C.c_int32, C.c_double, D],
            "bgk_oracle_fine_adjoint": [P, D, C.c_int32, C.c_int32, C.c_double, D,
                                        D, D],
            "bgk_oracle_lift_adjoint_rho": [P, D, D, D],
            "bgk_oracle_n_steps_force": [P, D, C.c_double, I, D],
            "bgk_oracle_transport_force": [P, D, D, C.c_double, D],
            "bgk_oracle_fine_steps_force": [P, D, D, D, C.c_double, C.c_int32],
            "bgk_oracle_fine_step_force": [P, D, D, D, C.c_double, I],
            "bgk_oracle_fine_propagate_moments_force": [P, D, D, D, C.c_double],
            "bgk_oracle_euler_coarse_step_force": [P, D, D, D, C.c_double, I],
            "bgk_oracle_parareal_iterate_force": [P, D, D, C.c_int32, C.c_double,
                                                  C.c_int32, C.c_double, D, D, I],
            "bgk_oracle_serial_fine_force": [P, D, D, C.c_int32, C.c_double, D],
            "bgk_oracle_cns_coarse_step": [P, D, D, D, C.c_double, I],
            "bgk_oracle_lift_ce": [P, D, D],
            "bgk_oracle_transport_opts": [P, D, C.c_int32, D, C.c_double, D],
            "bgk_oracle_fine_steps_opts": [P, D, C.c_int32, D, D, C.c_double, C.c_int32],
            "bgk_oracle_fine_propagate_moments_opts": [P, D, C.c_int32, C.c_int32, D, D,
                                                       C.c_double],
            "bgk_oracle_parareal_iterate_opts": [P, D, C.c_int32, C.c_int32, C.c_int32, D,
                                                 C.c_int32, C.c_double, C.c_int32,
                                                 C.c_double, D, D, I],
            "bgk_oracle_serial_fine_opts": [P, D, C.c_int32, C.c_int32, D, C.c_int32,
                                            C.c_double, D],
            "bgk_oracle_parareal_iterate_cns": [P, D, D, C.c_int32, C.c_double, C.c_int32,
                                                C.c_double, D, D, I],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.bgk_oracle_set_threads.argtypes = [C.c_int]
        L.bgk_oracle_set_threads.restype = None
        L.bgk_oracle_get_threads.argtypes = []
        L.bgk_oracle_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _prob(p) -> _Problem:
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


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _arr(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _chk(rc, where):
    if rc != OK:
        raise OracleError(rc, where)


def set_threads(n: int) -> None:
    lib().bgk_oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().bgk_oracle_get_threads())


def _force(p, E):
    """Exterior force at the x-cell centres as a contiguous [nx] array."""
    E = _arr(E)
    if E.shape != (p.nx,):
        raise ValueError(f"E must have shape ({p.nx},)")
    return E


def n_steps(p, t_span: float, E=None):
    n = C.c_int32()
    dt = C.c_double()
    if E is None:
        rc = lib().bgk_oracle_n_steps(C.byref(_prob(p)), t_span, C.byref(n), C.byref(dt))
    else:
        rc = lib().bgk_oracle_n_steps_force(C.byref(_prob(p)), _d(_force(p, E)), t_span,
                                            C.byref(n), C.byref(dt))
    _chk(rc, "n_steps")
    return n.value, dt.value


def lift(p, W) -> np.ndarray:
    W = _arr(W)
    f = np.empty((p.nx, p.nv[0] * p.nv[1] * p.nv[2]))
    _chk(lib().bgk_oracle_lift(C.byref(_prob(p)), _d(W), _d(f)), "lift")
    return f


def moments(p, f):
    f = _arr(f)
    V = np.empty((p.nx, 5))
    W = np.empty((p.nx, 5))
    _chk(lib().bgk_oracle_moments(C.byref(_prob(p)), _d(f), _d(V), _d(W)),
         "moments")
    return V, W


def transport(p, f, dt: float, E=None) -> np.ndarray:
    f = _arr(f)
    out = np.empty_like(f)
    if E is None:
        rc = lib().bgk_oracle_transport(C.byref(_prob(p)), _d(f), dt, _d(out))
    else:
        E = _force(p, E)
        rc = lib().bgk_oracle_transport_force(C.byref(_prob(p)), _d(E), _d(f), dt, _d(out))
    _chk(rc, "transport")
    return out


def relax(p, f_star, dt: float) -> np.ndarray:
    f_star = _arr(f_star)
    out = np.empty_like(f_star)
    _chk(lib().bgk_oracle_relax(C.byref(_prob(p)), _d(f_star), dt, _d(out)),
         "relax")
    return out


def fine_steps(p, f, dt: float, n: int, E=None) -> np.ndarray:
    f = _arr(f)
    out = np.empty_like(f)
    if E is None:
        rc = lib().bgk_oracle_fine_steps(C.byref(_prob(p)), _d(f), _d(out), dt, n)
    else:
        E = _force(p, E)
        rc = lib().bgk_oracle_fine_steps_force(C.byref(_prob(p)), _d(E), _d(f), _d(out),
                                               dt, n)
    _chk(rc, "fine_steps")
    return out


def fine_step(p, f, t_span: float, E=None):
    f = _arr(f)
    out = np.empty_like(f)
    n = C.c_int32()
    if E is None:
        rc = lib().bgk_oracle_fine_step(C.byref(_prob(p)), _d(f), _d(out), t_span,
                                        C.byref(n))
    else:
        E = _force(p, E)
        rc = lib().bgk_oracle_fine_step_force(C.byref(_prob(p)), _d(E), _d(f), _d(out),
                                              t_span, C.byref(n))
    _chk(rc, "fine_step")
    return out, n.value


def fine_propagate_moments(p, V, t_span: float, E=None) -> np.ndarray:
    V = _arr(V)
    out = np.empty_like(V)
    if E is None:
        rc = lib().bgk_oracle_fine_propagate_moments(C.byref(_prob(p)), _d(V), _d(out),
                                                     t_span)
    else:
        E = _force(p, E)
        rc = lib().bgk_oracle_fine_propagate_moments_force(C.byref(_prob(p)), _d(E), _d(V),
                                                           _d(out), t_span)
    _chk(rc, "PFL")
    return out


def euler_coarse_step(p, V, t_span: float, E=None):
    V = _arr(V)
    out = np.empty_like(V)
    n = C.c_int32()
    if E is None:
        rc = lib().bgk_oracle_euler_coarse_step(C.byref(_prob(p)), _d(V), _d(out), t_span,
                                                C.byref(n))
    else:
        E = _force(p, E)
        rc = lib().bgk_oracle_euler_coarse_step_force(C.byref(_prob(p)), _d(E), _d(V),
                                                      _d(out), t_span, C.byref(n))
    _chk(rc, "euler")
    return out, n.value


def lift_ce(p, W) -> np.ndarray:
    """Lifting of order one (first Chapman-Enskog correction)."""
    W = _arr(W)
    f = np.empty((p.nx, p.nv[0] * p.nv[1] * p.nv[2]))
    _chk(lib().bgk_oracle_lift_ce(C.byref(_prob(p)), _d(W), _d(f)), "lift_ce")
    return f


# coarse models of the parareal iteration; "fine" (the fine propagator as G)
# exists to pin the correction: with G = F one iteration gives the serial chain
COARSE = {"euler": 0, "cns": 1, "fine": 2}


def transport_opts(p, f, dt: float, E=None, fine_order: int = 1) -> np.ndarray:
    """One explicit transport; fine_order 2 adds the van Leer limited
    Lax-Wendroff correction in x."""
    f = _arr(f)
    out = np.empty_like(f)
    Ea = _force(p, E) if E is not None else None
    _chk(lib().bgk_oracle_transport_opts(C.byref(_prob(p)), _d(Ea) if Ea is not None else None,
                                         fine_order, _d(f), dt, _d(out)), "transport_opts")
    return out


def fine_steps_opts(p, f, dt: float, n: int, E=None, fine_order: int = 1) -> np.ndarray:
    f = _arr(f)
    out = np.empty_like(f)
    Ea = _force(p, E) if E is not None else None
    _chk(lib().bgk_oracle_fine_steps_opts(C.byref(_prob(p)), _d(Ea) if Ea is not None else None,
                                          fine_order, _d(f), _d(out), dt, n), "steps_opts")
    return out


def fine_propagate_moments_opts(p, V, t_span: float, E=None, lift_order: int = 0,
                                fine_order: int = 1):
    V = _arr(V)
    out = np.empty_like(V)
    Ea = _force(p, E) if E is not None else None
    _chk(lib().bgk_oracle_fine_propagate_moments_opts(
        C.byref(_prob(p)), _d(Ea) if Ea is not None else None, lift_order, fine_order, _d(V),
        _d(out), t_span), "PFL_opts")
    return out


def parareal_iterate_opts(p, W0, n_slices: int, T: float, k_max: int, tol: float, E=None,
                          coarse: str = "euler", lift_order: int = 0, fine_order: int = 1):
    W0 = _arr(W0)
    V = np.empty((n_slices + 1, p.nx, 5))
    err = np.zeros(max(k_max, 1))
    kd = C.c_int32()
    Ea = _force(p, E) if E is not None else None
    _chk(lib().bgk_oracle_parareal_iterate_opts(
        C.byref(_prob(p)), _d(Ea) if Ea is not None else None, COARSE[coarse], lift_order,
        fine_order, _d(W0), n_slices, T, k_max, tol, _d(V), _d(err), C.byref(kd)),
        "parareal_opts")
    return V, err[:kd.value].copy(), kd.value


def serial_fine_opts(p, W0, n_slices: int, T: float, E=None, lift_order: int = 0,
                     fine_order: int = 1):
    W0 = _arr(W0)
    V = np.empty((n_slices + 1, p.nx, 5))
    Ea = _force(p, E) if E is not None else None
    _chk(lib().bgk_oracle_serial_fine_opts(
        C.byref(_prob(p)), _d(Ea) if Ea is not None else None, lift_order, fine_order, _d(W0),
        n_slices, T, _d(V)), "serial_opts")
    return V


def cns_coarse_step(p, V, t_span: float, E=None):
    """Navier-Stokes coarse propagator (BGK coefficients); E optional."""
    V = _arr(V)
    out = np.empty_like(V)
    n = C.c_int32()
    Ea = _force(p, E) if E is not None else None
    Ep = _d(Ea) if Ea is not None else None
    _chk(lib().bgk_oracle_cns_coarse_step(C.byref(_prob(p)), Ep, _d(V), _d(out), t_span,
                                          C.byref(n)), "cns")
    return out, n.value


def parareal_iterate_cns(p, W0, n_slices: int, T: float, k_max: int, tol: float, E=None):
    """Algorithm 2 with the Navier-Stokes coarse propagator."""
    W0 = _arr(W0)
    V = np.empty((n_slices + 1, p.nx, 5))
    err = np.zeros(max(k_max, 1))
    kd = C.c_int32()
    Ea = _force(p, E) if E is not None else None
    Ep = _d(Ea) if Ea is not None else None
    _chk(lib().bgk_oracle_parareal_iterate_cns(C.byref(_prob(p)), Ep, _d(W0), n_slices, T,
                                               k_max, tol, _d(V), _d(err), C.byref(kd)),
         "parareal_cns")
    return V, err[:kd.value].copy(), kd.value


def parareal_iterate(p, W0, n_slices: int, T: float, k_max: int, tol: float, E=None):
    W0 = _arr(W0)
    V = np.empty((n_slices + 1, p.nx, 5))
    err = np.zeros(max(k_max, 1))
    kd = C.c_int32()
    if E is None:
        rc = lib().bgk_oracle_parareal_iterate(C.byref(_prob(p)), _d(W0), n_slices, T,
                                               k_max, tol, _d(V), _d(err), C.byref(kd))
    else:
        E = _force(p, E)
        rc = lib().bgk_oracle_parareal_iterate_force(C.byref(_prob(p)), _d(E), _d(W0),
                                                     n_slices, T, k_max, tol, _d(V),
                                                     _d(err), C.byref(kd))
    _chk(rc, "parareal")
    return V, err[:kd.value].copy(), kd.value


def serial_fine(p, W0, n_slices: int, T: float, E=None) -> np.ndarray:
    W0 = _arr(W0)
    V = np.empty((n_slices + 1, p.nx, 5))
    if E is None:
        rc = lib().bgk_oracle_serial_fine(C.byref(_prob(p)), _d(W0), n_slices, T, _d(V))
    else:
        E = _force(p, E)
        rc = lib().bgk_oracle_serial_fine_force(C.byref(_prob(p)), _d(E), _d(W0), n_slices,
                                                T, _d(V))
    _chk(rc, "serial_fine")
    return V


def fine_adjoint(p, f_ckpt, ckpt_every: int, n: int, dt: float, fbar_T):
    f_ckpt = _arr(f_ckpt)
    fbar_T = _arr(fbar_T)
    fbar0 = np.empty_like(fbar_T)
    dle = C.c_double(0.0)
    _chk(lib().bgk_oracle_fine_adjoint(C.byref(_prob(p)), _d(f_ckpt), ckpt_every,
                                       n, dt, _d(fbar_T), _d(fbar0),
                                       C.byref(dle)), "fine_adjoint")
    return fbar0, dle.value


def lift_adjoint_rho(p, W, fbar) -> np.ndarray:
    W = _arr(W)
    fbar = _arr(fbar)
    out = np.empty(p.nx)
    _chk(lib().bgk_oracle_lift_adjoint_rho(C.byref(_prob(p)), _d(W), _d(fbar),
                                           _d(out)), "lift_adjoint_rho")
    return out


def checkpoints(p, f0, dt: float, n: int, every: int) -> np.ndarray:
    """Forward states at steps 0, every, 2*every, ... (< n)."""
    f = _arr(f0)
    out = []
    for s in range(0, n, every):
        out.append(f.copy())
        m = min(every, n - s)
        f = fine_steps(p, f, dt, m)
    return np.stack(out), f
