"""Shared helpers of the GPU parity tests (comparison norms).

Every norm evaluated here is also recorded in ERRORS, so that the test
session can report, per test, the largest error it measured against the
bar (the margin of each parity check)."""
import numpy as np

ERRORS = []  # errors measured by the running test (cleared per test)


def rel_f(got, ref):
    """Normwise relative max-norm error of a phase-space field."""
    e = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    ERRORS.append(e)
    return e


def rel_V(got, ref):
    """Normwise errors of conserved moments [..., 5]: density by max|rho|,
    momentum by sqrt(max|rho| * 2 max|E|), energy by max|E|."""
    got = np.asarray(got).reshape(-1, 5)
    ref = np.asarray(ref).reshape(-1, 5)
    r = np.max(np.abs(ref[:, 0]))
    e = np.max(np.abs(ref[:, 4]))
    m = np.sqrt(r * 2 * e)
    d = np.abs(got - ref)
    err = float(max(np.max(d[:, 0]) / r, np.max(d[:, 1:4]) / m, np.max(d[:, 4]) / e))
    ERRORS.append(err)
    return err


def rel_W(got, ref):
    """Normwise errors of primitive moments [..., 5]: density by max|rho|,
    velocity by the thermal speed sqrt(max theta), temperature by max theta.
    Returns (rho, u, theta) errors."""
    got = np.asarray(got).reshape(-1, 5)
    ref = np.asarray(ref).reshape(-1, 5)
    d = np.abs(got - ref)
    th = np.max(np.abs(ref[:, 4]))
    errs = (float(np.max(d[:, 0]) / np.max(np.abs(ref[:, 0]))),
            float(np.max(d[:, 1:4]) / np.sqrt(th)), float(np.max(d[:, 4]) / th))
    ERRORS.append(max(errs))
    return errs


def rel_s(got, ref):
    """Relative error of a scalar."""
    e = float(abs(float(got) - float(ref)) / abs(float(ref)))
    ERRORS.append(e)
    return e


TOL = 1e-12  # parity bar on f and moments (max norm, normwise relative)
