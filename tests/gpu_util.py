"""Shared helpers of the GPU parity tests (comparison norms)."""
import numpy as np


def rel_f(got, ref):
    """Normwise relative max-norm error of a phase-space field."""
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def rel_V(got, ref):
    """Normwise errors of conserved moments [..., 5]: density by max|rho|,
    momentum by sqrt(max|rho| * 2 max|E|), energy by max|E|."""
    got = np.asarray(got).reshape(-1, 5)
    ref = np.asarray(ref).reshape(-1, 5)
    r = np.max(np.abs(ref[:, 0]))
    e = np.max(np.abs(ref[:, 4]))
    m = np.sqrt(r * 2 * e)
    d = np.abs(got - ref)
    return max(np.max(d[:, 0]) / r, np.max(d[:, 1:4]) / m, np.max(d[:, 4]) / e)


def rel_W(got, ref):
    """Normwise errors of primitive moments [..., 5]: density by max|rho|,
    velocity by the thermal speed sqrt(max theta), temperature by max theta.
    Returns (rho, u, theta) errors."""
    got = np.asarray(got).reshape(-1, 5)
    ref = np.asarray(ref).reshape(-1, 5)
    d = np.abs(got - ref)
    th = np.max(np.abs(ref[:, 4]))
    return (float(np.max(d[:, 0]) / np.max(np.abs(ref[:, 0]))),
            float(np.max(d[:, 1:4]) / np.sqrt(th)), float(np.max(d[:, 4]) / th))


TOL = 1e-12  # parity bar on f and moments (max norm, normwise relative)
