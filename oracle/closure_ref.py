"""Plain FP64 reference of the learned-closure form (2D-2V).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the CPU
baseline of the benchmark may use this module; nothing in the library
imports it.  It shares no code with the GPU kernels.

The closure form is not part of the paper.  It rests on the moment update
of the HOFKS step (eq. (UK) with (mom)): with f* = lam f + mu E,
    U^{n+1}_j = sum_k w m_k f*(j - k, k) - mu sum_k w m_k E(j - k, k) + U_E
              = lam sum_k w m_k E(j - k, k) + U_E + N_j,
    N_j = lam sum_k w m_k (f - E)(j - k, k),
so a closure cell needs, besides the Euler part U_E = mu MUSCL(U^n)
(section 4.3), only the transported equilibrium and an estimate of N.
Readings used here (not fixed by the paper):
  * network inputs: 3 x 3 stencil of (rho_c/rho_j - 1, (u_c - u_j)/c_j,
    theta_c/theta_j - 1), c = sqrt(gamma theta), then log10(tau/dt) in
    [-8, 8]; the network estimate is taken relative to its output on the
    uniform stencil (zeros), where N vanishes;
  * targets N_j / (lam s_j) with s_j = (rho, rho c, rho c, E) of cell j.
Periodic grids only.
"""
import numpy as np


def primitives(U, gam=2.0):
    """rho, u (2 x nc), theta, sound speed of U (4 x nc)"""
    rho = U[0]
    u = U[1:3] / rho
    th = (2.0 * U[3] - rho * (u * u).sum(0)) / (2.0 * rho)
    return rho, u, th, np.sqrt(gam * th)


def scales(U, gam=2.0):
    rho, _, _, c = primitives(U, gam)
    return np.stack([rho, rho * c, rho * c, U[3]])


def features(U, n, ftau, gam=2.0):
    """network inputs (nc x 37) of every cell of a periodic nx x ny grid"""
    nx, ny = n
    rho, u, th, c = primitives(U, gam)
    fields = [rho, u[0], u[1], th]
    grid = [a.reshape(ny, nx) for a in fields]
    x = np.empty((nx * ny, 37))
    for cidx in range(9):
        dy, dx = cidx // 3 - 1, cidx % 3 - 1
        # value of the neighbour (x + dx, y + dy) at cell (x, y)
        nb = [np.roll(g, shift=(-dy, -dx), axis=(0, 1)).reshape(-1) for g in grid]
        x[:, 4 * cidx + 0] = nb[0] / rho - 1.0
        x[:, 4 * cidx + 1] = (nb[1] - u[0]) / c
        x[:, 4 * cidx + 2] = (nb[2] - u[1]) / c
        x[:, 4 * cidx + 3] = nb[3] / th - 1.0
    x[:, 36] = min(8.0, max(-8.0, float(ftau)))
    return x


def uniform_input(ftau):
    """inputs of a uniform stencil"""
    x = np.zeros((1, 37))
    x[0, 36] = min(8.0, max(-8.0, float(ftau)))
    return x


def moment_flux(o, F):
    """sum_k w m_k F(j - k, k) on the periodic grid of oracle `o`: the
    moments of the pieces F (nv x nc) after one exact shift"""
    nx, ny = o.n[0], o.n[1]
    vel = o.velocities
    dv = o.dv
    w = dv ** 2
    out = np.zeros((4, nx * ny))
    for k in range(o.nv):
        vx, vy = vel[k]
        kx, ky = int(round(vx / dv)), int(round(vy / dv))
        sh = np.roll(F[k].reshape(ny, nx), shift=(ky, kx), axis=(0, 1)).reshape(-1)
        out[0] += w * sh
        out[1] += w * vx * sh
        out[2] += w * vy * sh
        out[3] += w * 0.5 * (vx * vx + vy * vy) * sh
    return out


def equilibria(o, U):
    """E[U] of every cell (nv x nc), from the oracle's projection"""
    return np.stack([o.equilibrium(U[:, j]) for j in range(U.shape[1])], axis=1)


def targets(o, f, U, gam=2.0):
    """N / (lam s) = sum_k w m_k (f - E)(j - k, k) / s_j  (nc x 4)"""
    return (moment_flux(o, f - equilibria(o, U)) / scales(U, gam)).T


def closure_step(o, U, tau, nhat=None):
    """U^{n+1} of every cell taken as a closure cell:
    lam sum_k w m_k E(j - k, k) + mu MUSCL_dt(U) + nhat"""
    lam = np.exp(-o.dt / tau) if tau > 0 else 0.0
    mu = -np.expm1(-o.dt / tau) if tau > 0 else 1.0
    UE, _ = o.muscl(U, o.dt)
    out = lam * moment_flux(o, equilibria(o, U)) + mu * UE
    if nhat is not None:
        out = out + nhat
    return out
