"""Independent vectorised numpy re-derivation of one IMEX fine step and one
Rusanov Euler substep, used only as a brute-force cross-check of the C oracle
on tiny grids.  Written from the paper's Section 3.1-3.3 definitions without
looking at the oracle's loops: whole-array operations, moments by tensor
contraction, Maxwellian by broadcasting, ghost cells by np.pad / np.roll.
"""
import numpy as np


def axes(p):
    out = []
    for a in range(3):
        dv = (p.v_hi[a] - p.v_lo[a]) / p.nv[a]
        out.append(p.v_lo[a] + dv * (np.arange(p.nv[a]) + 0.5))
    return out


def vgrid(p):
    vx, vy, vz = axes(p)
    VX, VY, VZ = np.meshgrid(vx, vy, vz, indexing="ij")
    return VX.ravel(), VY.ravel(), VZ.ravel()


def dv3(p):
    return np.prod([(p.v_hi[a] - p.v_lo[a]) / p.nv[a] for a in range(3)])


def maxwell(p, rho, u, th):
    VX, VY, VZ = vgrid(p)
    d2 = ((VX[None] - u[:, 0:1]) ** 2 + (VY[None] - u[:, 1:2]) ** 2 +
          (VZ[None] - u[:, 2:3]) ** 2)
    return rho[:, None] * np.exp(-d2 / (2 * th[:, None])) / (2 * np.pi * th[:, None]) ** 1.5


def prim(p, f):
    VX, VY, VZ = vgrid(p)
    w = dv3(p)
    rho = f.sum(1) * w
    u = np.stack([(f * VX).sum(1), (f * VY).sum(1), (f * VZ).sum(1)], 1) * w / rho[:, None]
    c2 = ((VX[None] - u[:, 0:1]) ** 2 + (VY[None] - u[:, 1:2]) ** 2 +
          (VZ[None] - u[:, 2:3]) ** 2)
    th = (c2 * f).sum(1) * w / (3 * rho)
    return rho, u, th


def transport(p, f, dt):
    VX, _, _ = vgrid(p)
    if p.bc == 1:
        fl = np.roll(f, 1, axis=0)
        fr = np.roll(f, -1, axis=0)
    else:
        fp = np.pad(f, ((1, 1), (0, 0)), mode="edge")
        fl, fr = fp[:-2], fp[2:]
    dx = (p.x_hi - p.x_lo) / p.nx
    up = np.where(VX > 0, VX, 0.0)[None]
    um = np.where(VX < 0, VX, 0.0)[None]
    flux_r = up * f + um * fr
    flux_l = up * fl + um * f
    return f - dt / dx * (flux_r - flux_l)


def transport_force(p, f, dt, E):
    """x transport followed by the v_x Rusanov flux difference of an
    exterior force E (one value per x cell), no flux through the ends of the
    v_x range: planes of constant v_x are slices of a [nx, nvx, nvy*nvz] view."""
    g = transport(p, f, dt)
    nvx = p.nv[0]
    F = f.reshape(p.nx, nvx, -1)
    dvx = (p.v_hi[0] - p.v_lo[0]) / nvx
    a = np.max(np.abs(E))
    Ec = np.asarray(E)[:, None, None]
    faces = np.zeros((p.nx, nvx + 1, F.shape[2]))
    faces[:, 1:-1] = 0.5 * Ec * (F[:, :-1] + F[:, 1:]) - 0.5 * a * (F[:, 1:] - F[:, :-1])
    return g - dt / dvx * (faces[:, 1:] - faces[:, :-1]).reshape(p.nx, -1)


def step_force(p, f, dt, E):
    g = transport_force(p, f, dt, E)
    rho, u, th = prim(p, g)
    M = maxwell(p, rho, u, th)
    lam = dt / p.eps
    return (g + lam * M) / (1 + lam)


def step(p, f, dt):
    g = transport(p, f, dt)
    rho, u, th = prim(p, g)
    M = maxwell(p, rho, u, th)
    lam = dt / p.eps
    return (g + lam * M) / (1 + lam)


def euler_substep(p, V, dt, E=None):
    rho = V[:, 0]
    u = V[:, 1:4] / rho[:, None]
    th = (2 * V[:, 4] / rho - (u ** 2).sum(1)) / 3
    pr = rho * th
    h = np.stack([rho * u[:, 0], rho * u[:, 0] ** 2 + pr, rho * u[:, 0] * u[:, 1],
                  rho * u[:, 0] * u[:, 2], u[:, 0] * (V[:, 4] + pr)], 1)
    s = np.abs(u[:, 0]) + np.sqrt(p.sound_gamma * th)
    if p.bc == 1:
        idxL = np.arange(-1, p.nx) % p.nx
        idxR = np.arange(0, p.nx + 1) % p.nx
    else:
        idxL = np.clip(np.arange(-1, p.nx), 0, p.nx - 1)
        idxR = np.clip(np.arange(0, p.nx + 1), 0, p.nx - 1)
    S = np.maximum(s[idxL], s[idxR])[:, None]
    H = 0.5 * (h[idxL] + h[idxR]) - 0.5 * S * (V[idxR] - V[idxL])
    dx = (p.x_hi - p.x_lo) / p.nx
    out = V - dt / dx * (H[1:] - H[:-1])
    if E is not None:
        out[:, 1] += dt * V[:, 0] * E
        out[:, 4] += dt * V[:, 1] * E
    return out, s.max()


def cns_substep(p, V, dt, E=None):
    """Euler substep plus the Navier-Stokes viscous and heat fluxes with BGK
    coefficients (mu = rho theta, kappa = 5/2 rho theta), central face
    differences, arrays of faces built with np.roll / edge padding.
    Returns (V_new, smax, theta_max)."""
    out, smax = euler_substep(p, V, dt, E)
    rho = V[:, 0]
    u = V[:, 1:4] / rho[:, None]
    th = (2 * V[:, 4] / rho - (u ** 2).sum(1)) / 3
    if p.bc == 1:
        L = np.arange(-1, p.nx) % p.nx
        R = np.arange(0, p.nx + 1) % p.nx
    else:
        L = np.clip(np.arange(-1, p.nx), 0, p.nx - 1)
        R = np.clip(np.arange(0, p.nx + 1), 0, p.nx - 1)
    dx = (p.x_hi - p.x_lo) / p.nx
    mu = 0.5 * (rho[L] * th[L] + rho[R] * th[R])
    du = u[R] - u[L]
    uf = 0.5 * (u[L] + u[R])
    D = np.zeros((p.nx + 1, 5))
    D[:, 1] = (4.0 / 3.0) * mu * du[:, 0]
    D[:, 2] = mu * du[:, 1]
    D[:, 3] = mu * du[:, 2]
    D[:, 4] = mu * ((4.0 / 3.0) * uf[:, 0] * du[:, 0] + uf[:, 1] * du[:, 1] +
                    uf[:, 2] * du[:, 2]) + 2.5 * mu * (th[R] - th[L])
    D *= p.eps / dx
    out = out + dt / dx * (D[1:] - D[:-1])
    return out, smax, th.max()


def lift_ce(p, W):
    """First-order Chapman-Enskog lifting: the Maxwellian of W times
    1 - eps P(c), the x-derivatives of u and theta by central differences
    (np.roll for periodic, edge padding for Neumann)."""
    if p.bc == 1:
        Wl, Wr = np.roll(W, 1, axis=0), np.roll(W, -1, axis=0)
    else:
        Wp = np.pad(W, ((1, 1), (0, 0)), mode="edge")
        Wl, Wr = Wp[:-2], Wp[2:]
    dx = (p.x_hi - p.x_lo) / p.nx
    g = (Wr - Wl) / (2 * dx)
    VX, VY, VZ = vgrid(p)
    th = W[:, 4:5]
    cx, cy, cz = VX[None] - W[:, 1:2], VY[None] - W[:, 2:3], VZ[None] - W[:, 3:4]
    c2 = cx ** 2 + cy ** 2 + cz ** 2
    P = (g[:, 1:2] * (cx ** 2 - c2 / 3) + g[:, 2:3] * cx * cy + g[:, 3:4] * cx * cz +
         g[:, 4:5] * cx * (c2 / (2 * th) - 2.5)) / th
    return maxwell(p, W[:, 0], W[:, 1:4], W[:, 4]) * (1 - p.eps * P)


def transport2(p, f, dt):
    """x transport with the van Leer limited Lax-Wendroff correction: face
    fluxes from whole-array shifts (two ghost layers)."""
    if p.bc == 1:
        sh = lambda k: np.roll(f, -k, axis=0)  # noqa: E731  f[i + k]
    else:
        fp = np.pad(f, ((2, 2), (0, 0)), mode="edge")
        sh = lambda k: fp[2 + k: 2 + k + p.nx]  # noqa: E731
    VX, _, _ = vgrid(p)
    dx = (p.x_hi - p.x_lo) / p.nx
    nu = VX * dt / dx

    def lim(a, b):
        prod = a * b
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(prod > 0, 2 * prod / (a + b), 0.0)

    def face(k):  # flux through the face between cells i+k and i+k+1
        fm, f0, f1, f2 = sh(k - 1), sh(k), sh(k + 1), sh(k + 2)
        pos = VX * (f0 + 0.5 * (1 - nu) * lim(f0 - fm, f1 - f0))
        neg = VX * (f1 - 0.5 * (1 + nu) * lim(f2 - f1, f1 - f0))
        return np.where(VX > 0, pos, np.where(VX < 0, neg, 0.0))

    return f - dt / dx * (face(0) - face(-1))
