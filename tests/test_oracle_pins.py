"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine, a closed form, an invariant, an exact solution or a textbook value.
Section numbers refer to arXiv:1212.0204.
"""
import math
import os

import numpy as np
import pytest
from scipy.stats import norm

import workloads as W
from oracle import ENONPHYS, Oracle, OracleError
from tests import exact_riemann as XR


def moment_matrix(o):
    """C of section 4.1: rows w*(1, v_k, |v_k|^2/2), built here from the node
    list the oracle reports (the node list itself is pinned below)."""
    v = o.velocities
    w = o.dv ** o.d
    rows = [np.ones(o.nv)] + [v[:, a] for a in range(o.d)] + [0.5 * (v ** 2).sum(1)]
    return w * np.array(rows)


def primitives(U, d):
    rho = U[0]
    u = U[1:1 + d] / rho
    theta = (2.0 * U[d + 1] - rho * (u ** 2).sum(0)) / (d * rho)
    return rho, u, theta


# ------------------------------------------------------------- section 3, 4.1
@pytest.mark.parametrize("d,nv", [(1, 8), (1, 7), (2, 6), (3, 4)])
def test_velocity_lattice(d, nv):
    dv = 0.375
    o = Oracle(d, [4] * d, 0.1, nv, dv)
    k1 = np.arange(nv) - nv // 2
    if nv % 2:
        assert k1[0] == -k1[-1]  # odd: symmetric set
    else:
        assert k1[0] == -nv // 2 and k1[-1] == nv // 2 - 1
    grids = np.meshgrid(*([k1 * dv] * d), indexing="ij")
    expect = np.stack([g.transpose(list(range(d))[::-1]).reshape(-1) for g in grids], 1)
    assert np.array_equal(o.velocities, expect)
    assert o.dt == 0.1 / dv  # dt v_k = k dx


@pytest.mark.parametrize("d,nv,dv", [(1, 16, 0.5), (2, 8, 0.75), (3, 6, 1.0)])
def test_projection_matrix_is_inverse_gram(d, nv, dv):
    o = Oracle(d, [3] * d, 0.1, nv, dv)
    C = moment_matrix(o)
    np.testing.assert_allclose(o.A, np.linalg.inv(C @ C.T), rtol=1e-12, atol=0)


def test_maxwellian_matches_normal_pdf():
    o = Oracle(2, [2, 2], 0.1, 12, 0.5)
    rho, u, th = 1.7, np.array([0.3, -0.6]), 0.8
    U = np.array([rho, rho * u[0], rho * u[1], 0.5 * rho * (u @ u) + rho * th])
    v = o.velocities
    expect = rho * norm.pdf(v[:, 0], u[0], math.sqrt(th)) * norm.pdf(v[:, 1], u[1], math.sqrt(th))
    np.testing.assert_allclose(o.maxwellian(U), expect, rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("d,nv,dv", [(1, 12, 0.75), (2, 8, 0.9), (3, 6, 1.1)])
def test_equilibrium_is_min_norm_correction(d, nv, dv):
    """eq. (minimMax): E = M + C^T (C C^T)^{-1} (U - C M) is the minimum-norm
    correction with C E = U; compare with numpy's min-norm least squares."""
    o = Oracle(d, [2] * d, 0.1, nv, dv)
    rng = np.random.default_rng(7)
    for _ in range(3):
        rho = rng.uniform(0.5, 2.0)
        u = rng.uniform(-0.5, 0.5, d)
        th = rng.uniform(0.5, 1.5)
        U = np.concatenate([[rho], rho * u, [0.5 * rho * (u @ u) + 0.5 * d * rho * th]])
        M = o.maxwellian(U)
        E = o.equilibrium(U)
        C = moment_matrix(o)
        y = np.linalg.lstsq(C, U - C @ M, rcond=None)[0]  # min-norm solution
        np.testing.assert_allclose(E, M + y, rtol=0, atol=1e-13 * np.abs(M).max())
        np.testing.assert_allclose(C @ E, U, rtol=1e-13, atol=1e-14)
        # the correction is not negligible on these coarse velocity grids
        assert np.abs(C @ M - U).max() > 1e-8


def test_equilibrium_correction_vanishes_with_resolution():
    """|U - C M| -> 0 as dv -> 0 on a fixed box (the trapezoid rule of a
    Gaussian), so E -> M (section 4.1 remark on truncation)."""
    U = np.array([1.0, 0.2, 0.5 * 0.04 + 0.5 * 0.25])  # theta = 1/4
    errs = []
    for nv, dv in [(16, 1.0), (32, 0.5), (64, 0.25)]:
        o = Oracle(1, [2], 0.1, nv, dv)
        errs.append(np.abs(o.equilibrium(U) - o.maxwellian(U)).max())
    assert errs[0] > 1e-4 and errs[2] < 1e-12 and errs[1] < errs[0]


# ----------------------------------------------------- section 4.2: transport
@pytest.mark.parametrize("d,n,nv", [(1, (37,), 9), (2, (11, 7), 6), (3, (5, 4, 6), 4)])
def test_free_transport_is_exact_periodic_shift(d, n, nv):
    """tau = +inf: lambda = 1, the scheme is the exact transport of the
    piecewise-constant pieces (sections 4.2, 4.3.1): f^n(j,k) = f^0(j - k n, k)."""
    o = Oracle(d, n, 0.05, nv, 0.5, tau=math.inf)
    rng = np.random.default_rng(3)
    f0 = rng.uniform(0.0, 1.0, (o.nv, o.nc))
    o.set_f(f0)
    steps = 3
    o.step(steps)
    kint = np.rint(o.velocities / 0.5).astype(int)
    expect = np.empty_like(f0)
    shape = tuple(n[::-1])
    for k in range(o.nv):
        plane = f0[k].reshape(shape)
        shift = tuple(int(kint[k, a]) * steps for a in range(d))[::-1]
        expect[k] = np.roll(plane, shift, axis=tuple(range(d))).reshape(-1)
    assert np.array_equal(o.f, expect)


def test_free_transport_outflow_replicates_boundary():
    """outflow: pieces entering through a boundary copy the boundary cell's
    piece of the same velocity (zero gradient); checked one step at a time."""
    nx, nv = 23, 8
    o = Oracle(1, (nx,), 0.05, nv, 0.5, bc=(1,), tau=math.inf)
    rng = np.random.default_rng(5)
    f = rng.uniform(0.0, 1.0, (nv, nx))
    o.set_f(f)
    for _ in range(3):
        o.step(1)
        nxt = np.empty_like(f)
        for k in range(nv):
            kk = k - nv // 2
            src = np.clip(np.arange(nx) - kk, 0, nx - 1)
            nxt[k] = f[k, src]
        f = nxt
        assert np.array_equal(o.f, f)


# -------------------------------------------------- section 4.2: relaxation
@pytest.mark.parametrize("tau", [0.05, 0.4, 3.0])
def test_homogeneous_relaxation_closed_form(tau):
    """Spatially uniform f: transport is the identity, U_E = U_M, and the
    scheme reduces to f^n = E + lambda^n (f^0 - E) with U constant."""
    d, nv, dv = 2, 10, 0.6
    o = Oracle(d, (4, 3), 0.1, nv, dv, tau=tau)
    v = o.velocities
    bump = (np.exp(-((v[:, 0] - 1.0) ** 2 + v[:, 1] ** 2)) +
            0.5 * np.exp(-((v[:, 0] + 0.7) ** 2 + (v[:, 1] - 0.4) ** 2) / 0.5))
    f0 = np.repeat(bump[:, None], o.nc, axis=1)
    o.set_f(f0)
    C = moment_matrix(o)
    U0 = C @ bump
    rho, u, th = primitives(U0[:, None], d)
    M = rho[0] * norm.pdf(v[:, 0], u[0, 0], math.sqrt(th[0])) * \
        norm.pdf(v[:, 1], u[1, 0], math.sqrt(th[0]))
    E = M + np.linalg.lstsq(C, U0 - C @ M, rcond=None)[0]
    lam = math.exp(-o.dt / tau)
    for n in range(1, 5):
        o.step(1)
        expect = E + lam ** n * (bump - E)
        np.testing.assert_allclose(o.f, np.repeat(expect[:, None], o.nc, 1),
                                   rtol=0, atol=1e-13)
        np.testing.assert_allclose(o.U, np.repeat(U0[:, None], o.nc, 1),
                                   rtol=1e-13, atol=1e-14)


# --------------------------------------------------------- invariants (4.2)
@pytest.mark.parametrize("tau", [0.0, 1e-3, 1e-2, 1.0, math.inf])
@pytest.mark.parametrize("d", [1, 2])
def test_periodic_conservation_and_moment_consistency(d, tau):
    """Relaxation and exact transport conserve (section 4.2 remark); the HOFKS
    correction gives P(f^{n+1}) = U^{n+1} (eq. mom with eq. minim_full)."""
    if d == 1:
        n, nv, dv = (48,), 24, 0.5
        rho, u, th = W.sod_tube(48, left=(1.0, 0.2, 1.0), right=(0.5, -0.1, 0.6))
    else:
        n, nv, dv = (12, 10), 12, 0.75
        rho, u, th = W.perturbed_gas(12, 2, 0.2, 0.1, 3, (11, 12))
        rho, th, u = rho[:120], th[:120], u[:, :120]
    o = Oracle(d, n, 1.0 / n[0], nv, dv, tau=tau)
    o.init_macro(rho, u, th)
    tot0 = o.U.sum(1)
    o.step(6)
    U = o.U
    scale = np.abs(o.U).max(1)
    np.testing.assert_allclose(U.sum(1), tot0, rtol=0, atol=1e-13 * scale.max() * o.nc)
    np.testing.assert_allclose(moment_matrix(o) @ o.f, U, rtol=0, atol=1e-12 * scale.max())


def test_fks_scheme_moments_are_transported_moments():
    """scheme 1 (no Euler coupling): U_E := U_M, so the correction vanishes."""
    rho, u, th = W.sod_tube(40)
    o = Oracle(1, (40,), 1 / 40, 16, 0.5, bc=(1,), tau=1e-2, scheme=1)
    o.init_macro(rho, u, th)
    o.step(2)
    assert np.abs(o.delta).max() == 0.0
    np.testing.assert_allclose(moment_matrix(o) @ o.f, o.U, rtol=0, atol=1e-13)


# --------------------------------------------------- section 4.3.2: MUSCL
def test_muscl_uniform_state_is_steady():
    o = Oracle(2, (6, 5), 0.1, 8, 0.5)
    U = np.tile(np.array([[1.3], [0.2], [-0.4], [2.0]]), (1, 30))
    Un, ns = o.muscl(U, 0.05)
    np.testing.assert_allclose(Un, U, rtol=1e-15, atol=1e-15)


def test_muscl_smooth_advection_second_order_in_space():
    """uniform velocity and pressure: the Euler system advects rho.  Eq.
    (discmom) is a forward-Euler step, first order in time; with dt ~ dx^2
    (as for Table 1 of section 5.2) the MUSCL of section 4.3.2 shows its
    second spatial order on smooth data (L1 rate ~2)."""
    errs = []
    for nx in (40, 80, 160):
        x = (np.arange(nx) + 0.5) / nx
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
        uu, p = 1.0, 1.0
        o = Oracle(1, (nx,), 1.0 / nx, 8, 0.5)
        U = np.stack([rho, rho * uu, 0.5 * rho * uu ** 2 + p / (3.0 - 1.0)])  # gamma = 3
        t = 0.1
        nsteps = int(math.ceil(t / (0.5 / nx ** 2)))
        for _ in range(nsteps):
            U, ns = o.muscl(U, t / nsteps)
            assert ns == 1
        ex = 1.0 + 0.2 * np.sin(2 * np.pi * (x - uu * t))
        errs.append(np.abs(U[0] - ex).mean())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > 1.7, (errs, rates)


def test_muscl_forward_euler_is_first_order_at_fixed_cfl():
    """the same problem at the scheme's own CFL 1/2 (eq. Time2): the time
    error dominates and the rate drops to ~1."""
    errs = []
    for nx in (50, 100, 200):
        x = (np.arange(nx) + 0.5) / nx
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
        o = Oracle(1, (nx,), 1.0 / nx, 8, 0.5)
        U = np.stack([rho, rho, 0.5 * rho + 0.5])
        Un, ns = o.muscl(U, 0.25)
        errs.append(np.abs(Un[0] - (1.0 + 0.2 * np.sin(2 * np.pi * (x - 0.25)))).mean())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert 0.8 < rates.min() and rates.max() < 1.5, (errs, rates)


def test_tau_zero_sod_converges_to_exact_riemann():
    """tau = 0: HOFKS returns the MUSCL Euler solution (Theorem 1 discussion,
    section 5.3 remark); the 1D-1V gas has gamma = (d+2)/d = 3 (eq. sys1).
    The L1 density error against the exact Riemann solution decreases under
    refinement at a first-order-like rate (shock-dominated)."""
    left, right = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    errs = []
    for nx in (100, 200, 400):
        rho, u, th = W.sod_tube(nx)
        o = Oracle(1, (nx,), 1.0 / nx, 16, 0.25 * 400 / nx, bc=(1,), tau=0.0)
        o.init_macro(rho, u, th)
        t_end = 0.16
        steps = int(round(t_end / o.dt))
        assert abs(steps * o.dt - t_end) < 1e-12
        o.step(steps)
        x = (np.arange(nx) + 0.5) / nx
        rex, _, _ = XR.solution(left, right, 3.0, x, t_end)
        errs.append(np.abs(o.U[0] - rex).mean())
    assert errs[0] > errs[1] > errs[2]
    assert math.log2(errs[0] / errs[2]) / 2 > 0.5, errs
    assert errs[2] < 6e-3


# --------------------------------------- section 4.3.3: a WENO Euler solve
def test_weno_uniform_state_is_steady():
    o = Oracle(2, (7, 5), 0.1, 8, 0.5, scheme=3)
    U = np.tile(np.array([[1.3], [0.2], [-0.4], [2.0]]), (1, 35))
    Un, ns = o.weno(U, 0.05)
    assert ns >= 1
    np.testing.assert_allclose(Un, U, rtol=1e-15, atol=1e-15)


def _weno_advection_errors(sizes, dt_of):
    errs = []
    for nx in sizes:
        x = (np.arange(nx) + 0.5) / nx
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
        o = Oracle(1, (nx,), 1.0 / nx, 8, 0.5, scheme=3)
        U = np.stack([rho, rho, 0.5 * rho + 0.5])  # u = 1, p = 1, gamma = 3
        t, T = 0.0, 0.25
        h = dt_of(nx)
        while t < T - 1e-15:
            step = min(h, T - t) if h else T - t
            U, _ = o.weno(U, step)
            t += step
        errs.append(np.abs(U[0] - (1.0 + 0.2 * np.sin(2 * np.pi * (x - T)))).mean())
    return np.array(errs)


def test_weno_smooth_advection_fifth_order_in_space():
    """smooth density advected at uniform velocity and pressure: with
    dt ~ dx^(5/3) the third-order Runge-Kutta error is O(dx^5), so the
    fifth-order WENO reconstruction shows its spatial order (L1 rate > 4.5;
    a wrong linear weight or candidate coefficient leaves <= 3)"""
    errs = _weno_advection_errors((32, 64, 128), lambda nx: 0.4 * (1.0 / nx) ** (5.0 / 3.0))
    rates = np.log2(errs[:-1] / errs[1:])
    assert rates.min() > 4.5, (errs, rates)


def test_weno_at_its_own_cfl_is_high_order():
    """the same problem in one call (the solver's own sub-steps at CFL 0.4):
    still well above MUSCL's second order (rate > 4)"""
    errs = _weno_advection_errors((32, 64, 128), lambda nx: None)
    rates = np.log2(errs[:-1] / errs[1:])
    assert rates.min() > 4.0, (errs, rates)


def test_weno_substeps_from_the_reduced_cfl():
    """s is the smallest count with dt_s sum_a alpha_a <= 0.4 dx at t^n (a
    CFL tighter than MUSCL's 1/2, section 4.3.3)"""
    nx = 200
    rho, u, th = W.sod_tube(nx)
    o = Oracle(1, (nx,), 1.0 / nx, 64, 0.25, bc=(1,), tau=0.0, scheme=3)
    o.init_macro(rho, u, th)
    U0 = o.U
    _, s = o.weno(U0, o.dt)
    a0 = _lf_speeds(U0, 1).sum()
    assert (o.dt / s) * a0 <= 0.4 * o.dx * (1 + 1e-15)
    assert (o.dt / (s - 1)) * a0 > 0.4 * o.dx


def test_tau_zero_sod_weno_converges_to_exact_riemann():
    """tau = 0 with the WENO Euler solve: the L1 density error against the
    exact Riemann solution (gamma = 3) decreases under refinement and stays
    below the MUSCL scheme's on every grid"""
    left, right = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    for nx in (100, 200, 400):
        errs = {}
        for scheme in (0, 3):
            rho, u, th = W.sod_tube(nx)
            o = Oracle(1, (nx,), 1.0 / nx, 16, 0.25 * 400 / nx, bc=(1,), tau=0.0, scheme=scheme)
            o.init_macro(rho, u, th)
            t_end = 0.16
            o.step(int(round(t_end / o.dt)))
            x = (np.arange(nx) + 0.5) / nx
            rex, _, _ = XR.solution(left, right, 3.0, x, t_end)
            errs[scheme] = np.abs(o.U[0] - rex).mean()
        assert errs[3] < errs[0], (nx, errs)
        if nx == 100:
            e100 = errs[3]
        if nx == 400:
            assert errs[3] < 0.5 * e100 and errs[3] < 5e-3, (e100, errs)


def test_exact_riemann_solver_textbook_sod():
    """the exact solver itself: Sod's problem at gamma = 1.4 against the
    textbook star state stored in tests/golden (5 digits)."""
    vals = {}
    path = os.path.join(os.path.dirname(__file__), "golden", "sod_star_state_gamma14.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            vals[k] = [float(x) for x in v]
    ps, us = XR.star_state(tuple(vals["left"]), tuple(vals["right"]), vals["gamma"][0])
    assert abs(ps - vals["p_star"][0]) < 5e-6 and abs(us - vals["u_star"][0]) < 5e-6


@pytest.mark.parametrize("scheme", [0, 3])
def test_mirror_symmetry_odd_velocity_set(scheme):
    """odd n_v gives a symmetric velocity set; mirrored data stay mirrored
    (pins the orientation of the shift, fluxes and slopes; scheme 3: of the
    upwind-biased WENO stencils)."""
    nx, nv = 60, 15
    x = (np.arange(nx) + 0.5) / nx
    rho = np.where(np.abs(x - 0.5) < 0.2, 1.0, 0.3) + 0.1 * x * (1 - x)
    u = (0.3 * np.sin(2 * np.pi * x))[None, :]  # odd about the centre
    th = np.where(np.abs(x - 0.5) < 0.2, 1.0, 0.7)
    o = Oracle(1, (nx,), 1 / nx, nv, 8.0 / nv, bc=(1,), tau=3e-3, scheme=scheme)
    o.init_macro(rho, u, th)
    o.step(5)
    U = o.U
    np.testing.assert_allclose(U[0], U[0][::-1], rtol=1e-12)
    np.testing.assert_allclose(U[1], -U[1][::-1], rtol=0, atol=1e-12)
    np.testing.assert_allclose(U[2], U[2][::-1], rtol=1e-12)


# ------------------------------------------------------- Theorem 1 (4.3.1)
def test_theorem1_delta_is_second_order_in_dt():
    """From smooth equilibrium data, U_E - U_M = O(dt^2) (Theorem 1).  With
    dv fixed, dt = dx/dv, so halving dx should divide max|delta| by ~4.  A
    wrong gamma or a wrong flux would leave an O(dt) mismatch."""
    res = []
    for nx in (256, 512, 1024):
        x = (np.arange(nx) + 0.5) / nx
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
        u = (0.1 + 0.1 * np.cos(2 * np.pi * x))[None, :]
        th = 1.0 + 0.1 * np.sin(4 * np.pi * x)
        o = Oracle(1, (nx,), 1 / nx, 48, 0.25, tau=0.0)
        o.init_macro(rho, u, th)
        o.step(1)
        res.append(np.abs(o.delta).max())
    rates = np.log2(np.array(res[:-1]) / np.array(res[1:]))
    assert rates.min() > 1.85, (res, rates)


# ------------------------------------------------------------ failure modes
def test_nonphysical_state_is_reported():
    o = Oracle(1, (4,), 0.25, 8, 0.5, tau=1e-2)
    with pytest.raises(OracleError) as e:
        o.init_macro(np.array([1.0, 0.0, 1.0, 1.0]), np.zeros((1, 4)), np.ones(4))
    assert e.value.status == ENONPHYS
    o.init_macro(np.ones(4), np.zeros((1, 4)), np.ones(4))
    o.set_f(np.full((8, 4), np.nan))
    with pytest.raises(OracleError):
        o.step(1)


def test_bad_descriptors_rejected():
    with pytest.raises(OracleError):
        Oracle(4, (2,), 0.1, 8, 0.5)
    with pytest.raises(OracleError):
        Oracle(1, (2,), 0.1, 1, 0.5)
    with pytest.raises(OracleError):
        Oracle(1, (2,), 0.1, 8, 0.5, tau=-1.0)


# -------------------------------------------- closure network (not in the paper)
def test_mlp_gradient_matches_central_differences():
    """back-propagated gradient of the FP64 closure network vs central finite
    differences of its own forward pass"""
    from oracle import mlp_forward, mlp_loss_grad, mlp_nparam
    rng = np.random.default_rng(12)
    p = 0.2 * rng.standard_normal(mlp_nparam())
    x = rng.standard_normal((5, 37))
    t = rng.standard_normal((5, 4))
    loss, g = mlp_loss_grad(p, x, t)
    assert abs(loss - ((mlp_forward(p, x) - t) ** 2).mean()) < 1e-14
    idx = rng.choice(p.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp_loss_grad(pp, x, t)[0] - mlp_loss_grad(pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_mlp_zero_weights_give_bias_and_adam_descends():
    from oracle import mlp_adam, mlp_forward, mlp_loss_grad, mlp_nparam
    n = mlp_nparam()
    p = np.zeros(n)
    p[-4:] = [0.1, -0.2, 0.3, -0.4]  # output bias
    x = np.random.default_rng(0).standard_normal((3, 37))
    np.testing.assert_array_equal(mlp_forward(p, x), np.tile(p[-4:], (3, 1)))
    rng = np.random.default_rng(1)
    p = 0.3 * rng.standard_normal(n)
    x = rng.standard_normal((64, 37))
    t = np.tanh(x[:, :4])
    m, v = np.zeros(n), np.zeros(n)
    l0 = mlp_loss_grad(p, x, t)[0]
    for k in range(1, 51):
        _, g = mlp_loss_grad(p, x, t)
        mlp_adam(p, g, m, v, 1e-3, k)
    assert mlp_loss_grad(p, x, t)[0] < 0.7 * l0


def _torch_net(p):
    """the closure network as a float64 torch.nn composition, with its
    parameters taken from the documented flat layout (W row-major (out, in),
    then b, for 37 -> 64 -> 64 -> 64 -> 4)"""
    import torch
    sizes = [(37, 64), (64, 64), (64, 64), (64, 4)]
    layers, o = [], 0
    for li, (nin, nout) in enumerate(sizes):
        lin = torch.nn.Linear(nin, nout, dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(p[o:o + nin * nout].reshape(nout, nin)))
            o += nin * nout
            lin.bias.copy_(torch.from_numpy(p[o:o + nout]))
            o += nout
        layers.append(lin)
        if li < 3:
            layers.append(torch.nn.Tanh())
    assert o == p.size
    return torch.nn.Sequential(*layers)


def _torch_flat_grad(net):
    import torch
    return torch.cat([torch.cat([l.weight.grad.reshape(-1), l.bias.grad])
                      for l in net if isinstance(l, torch.nn.Linear)]).numpy()


def test_mlp_forward_and_gradient_match_torch_float64():
    """forward pass, MSE loss and its gradient against torch.nn (Linear, Tanh)
    in float64 with autograd: a transposed weight layout, a wrong activation
    derivative or a wrong loss scale fails here"""
    import torch
    from oracle import mlp_forward, mlp_loss_grad, mlp_nparam
    rng = np.random.default_rng(21)
    p = 0.25 * rng.standard_normal(mlp_nparam())
    x = rng.standard_normal((33, 37))
    t = rng.standard_normal((33, 4))
    net = _torch_net(p)
    xt = torch.from_numpy(x)
    y = net(xt)
    np.testing.assert_allclose(mlp_forward(p, x), y.detach().numpy(), rtol=1e-12, atol=1e-13)
    loss_t = torch.nn.functional.mse_loss(y, torch.from_numpy(t))
    loss_t.backward()
    loss, g = mlp_loss_grad(p, x, t)
    assert abs(loss - loss_t.item()) <= 1e-13 * abs(loss_t.item())
    gt = _torch_flat_grad(net)
    np.testing.assert_allclose(g, gt, rtol=1e-11, atol=1e-14 * np.abs(gt).max())


def test_mlp_adam_matches_torch_optim_adam():
    """five Adam steps (bias-corrected, Kingma & Ba) against torch.optim.Adam
    in float64 on the same gradients"""
    import torch
    from oracle import mlp_adam, mlp_loss_grad, mlp_nparam
    rng = np.random.default_rng(22)
    n = mlp_nparam()
    p = 0.3 * rng.standard_normal(n)
    x = rng.standard_normal((40, 37))
    t = rng.standard_normal((40, 4))
    pt = torch.from_numpy(p.copy()).requires_grad_(True)
    opt = torch.optim.Adam([pt], lr=3e-3, betas=(0.85, 0.995), eps=1e-7)
    m, v = np.zeros(n), np.zeros(n)
    po = p.copy()
    for k in range(1, 6):
        _, g = mlp_loss_grad(po, x, t)
        mlp_adam(po, g, m, v, 3e-3, k, b1=0.85, b2=0.995, eps=1e-7)
        opt.zero_grad()
        pt.grad = torch.from_numpy(mlp_loss_grad(pt.detach().numpy().copy(), x, t)[1])
        opt.step()
        np.testing.assert_allclose(po, pt.detach().numpy(), rtol=1e-13, atol=1e-15)


# ---------------------------------------------- sub-steps and eq. (Time2)
def _lf_speeds(U, d):
    """global Lax-Friedrichs speeds max_j |u_a| + c, c = sqrt(gamma p / rho)"""
    rho = U[0]
    u = U[1:1 + d] / rho
    p = (2.0 * U[d + 1] - rho * (u ** 2).sum(0)) / d
    c = np.sqrt((d + 2.0) / d * p / rho)
    return np.array([(np.abs(u[a]) + c).max() for a in range(d)])


@pytest.mark.parametrize("d", [1, 2])
def test_substeps_meet_time2_at_tn_and_reevaluate_speeds(d):
    """eq. (Time2): the MUSCL solve is stable for dt_s sum_a alpha_a <= dx / 2.
    The lattice dt = dx/dv is larger, so the oracle sub-cycles (reading R11):
    s is the smallest count that meets the bound with the speeds of U^n
    (computed here independently), the sub-steps are equal, and each takes
    the Lax-Friedrichs speeds of its own state -- replayed here one sub-step
    at a time, the solve must equal the s-step solve bit for bit.  The bound
    is met at the first sub-step only; the largest ratio reached at a later
    sub-step is printed (R11 fixes s from U^n)."""
    if d == 1:
        nx, dv = 200, 0.25
        rho, u, th = W.sod_tube(nx)
        o = Oracle(1, (nx,), 1.0 / nx, 64, dv, bc=(1,), tau=0.0)
    else:
        nx, dv = 48, 0.5
        rho, u, th = W.perturbed_gas(nx, 2, 0.2, 0.1, 4, (61, 62))
        u = 0.2 * np.stack([np.sin(np.arange(nx * nx) * 0.07), np.cos(np.arange(nx * nx) * 0.05)])
        o = Oracle(2, (nx, nx), 1.0 / nx, 16, dv, tau=0.0)
    o.init_macro(rho, u, th)
    U0 = o.U
    dt, dx = o.dt, o.dx
    Us, s = o.muscl(U0, dt)
    a0 = _lf_speeds(U0, d).sum()
    assert s > 1
    assert (dt / s) * a0 <= 0.5 * dx * (1 + 1e-15)
    assert (dt / (s - 1)) * a0 > 0.5 * dx
    U = U0.copy()
    cfl = []
    for i in range(s):
        cfl.append((dt / s) * _lf_speeds(U, d).sum() / dx)
        U = o.muscl_substep(U, dt / s)
    np.testing.assert_array_equal(U, Us)
    print(f"d={d}: s={s}, dt_s sum alpha / dx at the sub-steps: first {cfl[0]:.4f}, "
          f"largest {max(cfl):.4f}")


def test_tube_pool_matches_in_process_oracle():
    """the worker pool the batch tests use gives the in-process oracle's
    moments bit for bit (one thread per tube either way)"""
    from oracle import set_threads
    from tests.oracle_pool import run_tube, run_tubes
    tubes = W.batched_tubes(count=6, seed=99, nx_range=(200, 400))
    res = run_tubes(tubes, 3, workers=2)
    for t, (U, bad) in zip(tubes, res):
        U1, bad1 = run_tube((t, 3))
        assert bad == bad1
        if not bad:
            np.testing.assert_array_equal(U, U1)
    set_threads(os.cpu_count() or 1)


# -------------------------------- section 4.2: transport off the lattice
def _exact_piecewise_transport(f0, n, nv, dv, dt, dx, nsteps, d):
    """f at the cell centres after nsteps free-transport steps: each f_k is
    the piecewise-constant initial function (cells [p dx, (p+1) dx))
    translated by v_k t, evaluated at x_j (periodic); computed here from the
    positions, not from step-by-step offsets"""
    ks = np.arange(nv) - nv // 2
    t = nsteps * dt
    out = np.empty_like(f0)
    nc = int(np.prod(n))
    cells = np.stack(np.unravel_index(np.arange(nc), tuple(reversed(n)))[::-1], 1)  # (nc, d) x first
    for k in range(nv ** d):
        idx = np.unravel_index(k, (nv,) * d)[::-1]  # x-fastest velocity index
        src = np.empty_like(cells)
        for a in range(d):
            y = (cells[:, a] + 0.5) * dx - ks[idx[a]] * dv * t
            src[:, a] = np.floor(y / dx).astype(int) % n[a]
        j = np.ravel_multi_index(tuple(src[:, a] for a in reversed(range(d))), tuple(reversed(n)))
        out[k] = f0[k, j]
    return out


@pytest.mark.parametrize("d,n,nv,frac", [(1, (41,), 12, 0.37), (2, (13, 9), 6, math.sqrt(2) / 3),
                                         (3, (7, 5, 6), 4, 0.61)])
def test_offlattice_free_transport_is_exact(d, n, nv, frac):
    """tau = +inf with a free time step dt = frac dx/dv: f^n at every cell
    centre is the initial piecewise-constant f_k translated by v_k n dt
    (section 4.2, no reconstruction), bit for bit"""
    dv = 0.5
    dx = 1.0 / n[0]
    dt = frac * dx / dv
    rng = np.random.default_rng(5 + d)
    f0 = rng.uniform(0.0, 1.0, (nv ** d, int(np.prod(n))))
    o = Oracle(d, n, dx, nv, dv, tau=math.inf, dt=dt)
    assert o.dt == dt
    o.set_f(f0)
    for steps in (1, 3, 7):
        o.step(steps - o.nstep)
        np.testing.assert_array_equal(o.f, _exact_piecewise_transport(f0, n, nv, dv, dt, dx, steps, d))


@pytest.mark.parametrize("tau", [0.0, 1e-3, 1e-2, 1.0, math.inf])
@pytest.mark.parametrize("scheme", [0, 1, 3])
def test_offlattice_conservation_and_consistency(tau, scheme):
    """off-lattice transport keeps every piece, so periodic totals are
    conserved to rounding for every tau and scheme, and P(f^n) = U^n"""
    n, nv, dv = (24, 20), 12, 0.5
    dx = 1.0 / 24
    rho, u, th = W.perturbed_gas(24, 2, 0.2, 0.1, 3, (71, 72))
    rho = rho.reshape(24, 24)[:20].reshape(-1)
    th = th.reshape(24, 24)[:20].reshape(-1)
    u = 0.2 * np.stack([np.sin(np.arange(480) * 0.1), np.cos(np.arange(480) * 0.07)])
    o = Oracle(2, n, dx, nv, dv, tau=tau, scheme=scheme, dt=0.43 * dx / dv)
    o.init_macro(rho, u, th)
    tot0 = o.U.sum(1)
    o.step(6)
    U = o.U
    scale = np.abs(U[0]).sum()
    assert (np.abs(U.sum(1) - tot0) / scale).max() < 1e-13
    np.testing.assert_allclose(moment_matrix(o) @ o.f, U, rtol=0, atol=1e-13)


@pytest.mark.parametrize("tau", [0.0, 1e-2, math.inf])
def test_offlattice_at_the_lattice_step_is_the_lattice_scheme(tau):
    """dt = dx/dv given explicitly reproduces the lattice run bit for bit"""
    n, nv, dv = (30, 11), 10, 0.5
    dx = 1.0 / 30
    rng = np.random.default_rng(8)
    fields = (1.0 + 0.2 * rng.uniform(-1, 1, 330), 0.1 * rng.uniform(-1, 1, (2, 330)),
              1.0 + 0.2 * rng.uniform(-1, 1, 330))
    a = Oracle(2, n, dx, nv, dv, bc=(1, 0), tau=tau)
    b = Oracle(2, n, dx, nv, dv, bc=(1, 0), tau=tau, dt=dx / dv)
    a.init_macro(*fields)
    b.init_macro(*fields)
    a.step(5)
    b.step(5)
    np.testing.assert_array_equal(a.U, b.U)
    np.testing.assert_array_equal(a.f, b.f)


def test_offlattice_rejects_a_step_beyond_the_lattice():
    with pytest.raises(OracleError):
        Oracle(1, (10,), 0.1, 8, 0.5, dt=0.21)


# ------------------------------------------- Strang splitting (section 4.2)
@pytest.mark.parametrize("tau", [0.05, 0.4, 3.0])
def test_strang_homogeneous_relaxation_closed_form(tau):
    """a spatially uniform non-equilibrium f: transport is the identity and
    R_{dt/2} (R_dt)^{n-1} R_{dt/2} = R_{n dt}, so the f read after n Strang
    steps is E + lambda^n (f0 - E) and U stays constant"""
    o = Oracle(1, (8,), 0.125, 24, 0.5, tau=tau, scheme=1, strang=True)
    v = o.velocities[:, 0]
    g = np.exp(-0.5 * (v - 1.0) ** 2) + 0.6 * np.exp(-2.0 * (v + 1.5) ** 2)
    f0 = np.tile(g[:, None], (1, 8))
    o.set_f(f0)
    U0 = o.U
    E = o.equilibrium(U0[:, 0])
    for n in (1, 2, 5):
        o.step(n - o.nstep)
        lam = math.exp(-o.dt / tau)
        expect = E[:, None] + lam ** n * (f0 - E[:, None])
        np.testing.assert_allclose(o.f, expect, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(o.U, U0, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("scheme", [0, 1, 3])
def test_strang_conservation_and_consistency(scheme):
    """periodic totals conserved and P(f) = U for the f read after the
    pending half relaxation"""
    n, nv, dv = (20, 18), 12, 0.5
    dx = 1.0 / 20
    rng = np.random.default_rng(91)
    fields = (1.0 + 0.2 * rng.uniform(-1, 1, 360), 0.1 * rng.uniform(-1, 1, (2, 360)),
              1.0 + 0.2 * rng.uniform(-1, 1, 360))
    o = Oracle(2, n, dx, nv, dv, tau=2e-2, scheme=scheme, strang=True)
    o.init_macro(*fields)
    tot0 = o.U.sum(1)
    o.step(5)
    U = o.U
    assert (np.abs(U.sum(1) - tot0) / np.abs(U[0]).sum()).max() < 1e-13
    np.testing.assert_allclose(moment_matrix(o) @ o.f, U, rtol=0, atol=1e-13)


def test_strang_fks_moments_from_equilibrium_equal_first_order():
    """R_{dt/2} leaves an equilibrium and all moments unchanged, so from
    equilibrium data the FKS moment trajectory of Strang splitting is the
    first-order one; only the distribution read out differs"""
    nx = 40
    rho, u, th = W.sod_tube(nx)
    a = Oracle(1, (nx,), 1.0 / nx, 16, 0.5, bc=(1,), tau=0.05, scheme=1)
    b = Oracle(1, (nx,), 1.0 / nx, 16, 0.5, bc=(1,), tau=0.05, scheme=1, strang=True)
    a.init_macro(rho, u, th)
    b.init_macro(rho, u, th)
    a.step(6)
    b.step(6)
    np.testing.assert_allclose(a.U, b.U, rtol=1e-14, atol=1e-15)  # to the rounding of lambda
    assert np.abs(a.f - b.f).max() > 1e-6
