"""Pins of the FP64 closure reference (oracle/closure_ref.py) on the CPU.

The closure update must reproduce the oracle's HOFKS step exactly when it is
given the true non-equilibrium term, reduce to the MUSCL solve at tau = 0,
conserve the totals, and its inputs must follow the stencil ordering.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Oracle
from oracle import closure_ref as C


def small_grid(tau, n=12, nv=8, dv=0.5, seed=3):
    o = Oracle(2, (n, n), 1.0 / n, nv, dv, bc=(0, 0), tau=tau)
    rho, u, th = W.perturbed_gas(n, 2, 0.15, 0.1, 2, (seed, seed + 10))
    o.init_macro(rho, u, th)
    return o


def test_features_of_uniform_state():
    n = 6
    U = np.zeros((4, n * n))
    U[0] = 2.0
    U[1] = 2.0 * 0.3
    U[2] = -2.0 * 0.1
    U[3] = 0.5 * 2.0 * (0.09 + 0.01) + 2.0 * 0.7  # theta = 0.7
    x = C.features(U, (n, n), -1.25)
    np.testing.assert_allclose(x[:, :36], 0.0, atol=1e-15)
    np.testing.assert_array_equal(x[:1], C.uniform_input(-1.25))
    assert (x[:, 36] == -1.25).all()
    assert C.features(U, (n, n), 30.0)[0, 36] == 8.0


def test_feature_stencil_order():
    """rho grows with x and y: stencil cell c = 3 (dy + 1) + (dx + 1)"""
    nx, ny = 7, 5
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    rho = (1.0 + 0.1 * X + 0.01 * Y).reshape(-1)
    U = np.zeros((4, nx * ny))
    U[0] = rho
    U[3] = rho  # theta = 1
    x = C.features(U, (nx, ny), 0.0)
    j = 2 * nx + 3  # cell (3, 2)
    for c in range(9):
        dy, dx = c // 3 - 1, c % 3 - 1
        nb = 1.0 + 0.1 * (3 + dx) + 0.01 * (2 + dy)
        assert x[j, 4 * c] == pytest.approx(nb / rho[j] - 1.0, rel=1e-13, abs=1e-16)


def test_shift_direction_of_moment_flux():
    """a piece at cell j0 with velocity index k arrives at j0 + k"""
    o = Oracle(2, (8, 8), 1.0 / 8, 4, 1.0, bc=(0, 0), tau=1.0)
    vel = o.velocities
    k = int(np.where((vel[:, 0] == 1.0) & (vel[:, 1] == -2.0))[0][0])
    F = np.zeros((o.nv, 64))
    F[k, 3 * 8 + 2] = 1.0  # cell (2, 3)
    mf = C.moment_flux(o, F)
    dest = ((3 - 2) % 8) * 8 + (2 + 1) % 8
    assert np.flatnonzero(mf[0]).tolist() == [dest]
    np.testing.assert_allclose(mf[:, dest], [1.0, 1.0, -2.0, 2.5])


def test_targets_vanish_at_equilibrium():
    o = small_grid(1e-2)
    t = C.targets(o, o.f, o.U)
    assert np.abs(t).max() < 1e-13


def test_closure_step_with_exact_term_is_the_hofks_step():
    """lam KFVS(E) + U_E + lam s t reproduces the oracle step"""
    tau = 2e-2
    o = small_grid(tau)
    o.step(2)  # away from equilibrium
    U0, f0 = o.U.copy(), o.f.copy()
    lam = np.exp(-o.dt / tau)
    nhat = lam * C.scales(U0) * C.targets(o, f0, U0).T
    Uc = C.closure_step(o, U0, tau, nhat)
    o.step(1)
    err = np.abs(Uc - o.U).max(axis=1) / np.abs(o.U).max(axis=1)
    assert err.max() < 1e-12, err
    # without the term the update differs by O(lam |N|)
    Uz = C.closure_step(o, U0, tau)
    assert np.abs(Uz - o.U).max() > 1e3 * np.abs(Uc - o.U).max()


def test_closure_step_at_tau_zero_is_muscl():
    o = small_grid(0.0)
    U0 = o.U.copy()
    UE, _ = o.muscl(U0, o.dt)
    np.testing.assert_array_equal(C.closure_step(o, U0, 0.0), UE)


def test_closure_step_conserves_totals():
    tau = 5e-3
    o = small_grid(tau)
    U = o.U.copy()
    tot0 = U.sum(axis=1)
    for _ in range(3):
        U = C.closure_step(o, U, tau)
    np.testing.assert_allclose(U.sum(axis=1), tot0, rtol=1e-13, atol=1e-13)
