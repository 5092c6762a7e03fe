"""Pin of the FP64 C oracle against a 50-digit brute-force statement of the
scheme on tiny grids (arXiv:1212.0204, sections 4.1-4.3).

The brute force (tests/brute_force.py) is written separately from the oracle:
it solves the normal equations of eq. (minimMax) and (minim_full) by LU in
50-digit arithmetic, evaluates the MUSCL flux of section 4.3.2 literally
(chi, phi, sigma) face by face, and walks the grid through cell tuples.  On
1D 5 cells x 5 velocities and 2D 3 x 3 cells x 3^2 velocities, three steps
from a non-equilibrium start, every scheme, tau and boundary, the oracle must
agree to 1e-13 normwise on U and on f.  A dropped term, a wrong sign or
index, or a transposed operand in the oracle fails here.  For the WENO
solve (scheme 3) the brute force derives the candidate reconstructions, the
linear weights and the smoothness indicators from their definitions (cell
averages of quadratics, the quartic through five averages, integrals of the
squared derivatives) instead of typing their coefficients.
"""
import math

import numpy as np
import pytest

from oracle import Oracle
from tests.brute_force import Brute

TOL = 1e-13

CASES_1D = [((5,), (0,)), ((5,), (1,))]
CASES_2D = [((3, 3), (0, 0)), ((3, 3), (1, 0)), ((3, 3), (1, 1))]


def _start(d, n, nv, dv, seed):
    """a non-equilibrium f0: the Maxwellian of random (rho, u, theta) per cell
    times a random factor in [0.8, 1.2] per piece (FP64 values, handed to both
    sides bit for bit)"""
    rng = np.random.default_rng(seed)
    nc = int(np.prod(n))
    rho = rng.uniform(0.6, 1.4, nc)
    u = rng.uniform(-0.3, 0.3, (d, nc))
    th = rng.uniform(0.7, 1.3, nc)
    ks = np.arange(nv) - nv // 2
    grids = np.meshgrid(*([ks * dv] * d), indexing="ij")
    vel = np.stack([g.transpose(list(range(d))[::-1]).reshape(-1) for g in grids], 1)
    f0 = np.empty((nv ** d, nc))
    for j in range(nc):
        q = ((vel - u[:, j]) ** 2).sum(1)
        f0[:, j] = rho[j] * (2 * np.pi * th[j]) ** (-d / 2) * np.exp(-q / (2 * th[j]))
    f0 *= rng.uniform(0.8, 1.2, f0.shape)
    return f0, (rho, u, th)


def _compare(o, b, d):
    Ub = np.array(b.U_array())
    fb = np.array(b.f_array())
    Uo, fo = o.U, o.f
    errU = [np.abs(Uo[r] - Ub[r]).max() / np.abs(Ub[r]).max() if np.abs(Ub[r]).max() > 0
            else np.abs(Uo[r]).max() for r in range(d + 2)]
    errf = np.abs(fo - fb).max() / np.abs(fb).max()
    return max(errU), errf


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
@pytest.mark.parametrize("tau", [0.0, 1e-2, 1.0, math.inf])
@pytest.mark.parametrize("n,bc", CASES_1D + CASES_2D)
def test_oracle_matches_brute_force(n, bc, tau, scheme):
    d = len(n)
    nv = 5 if d == 1 else 3
    dv = 1.25
    dx = 1.0 / n[0]
    f0, _ = _start(d, n, nv, dv, seed=1000 + 10 * d + sum(bc))
    o = Oracle(d, n, dx, nv, dv, bc=bc, tau=tau, scheme=scheme)
    b = Brute(d, n, dx, nv, dv, bc, tau, scheme)
    o.set_f(f0)
    b.set_f(f0)
    o.step(3)
    b.step(3)
    eU, ef = _compare(o, b, d)
    assert eU < TOL and ef < TOL, (eU, ef)


@pytest.mark.parametrize("n,bc", [((5,), (1,)), ((3, 3), (0, 1))])
def test_oracle_matches_brute_force_from_equilibrium(n, bc):
    """initial data f0 = E[U0] (section 4.2), then two HOFKS steps"""
    d = len(n)
    nv = 5 if d == 1 else 3
    _, (rho, u, th) = _start(d, n, nv, 1.25, seed=77)
    o = Oracle(d, n, 1.0 / n[0], nv, 1.25, bc=bc, tau=0.05)
    b = Brute(d, n, 1.0 / n[0], nv, 1.25, bc, 0.05)
    o.init_macro(rho, u, th)
    b.init_macro(rho, u.tolist(), th)
    eU, ef = _compare(o, b, d)
    assert eU < TOL and ef < TOL
    o.step(2)
    b.step(2)
    eU, ef = _compare(o, b, d)
    assert eU < TOL and ef < TOL, (eU, ef)


@pytest.mark.parametrize("scheme", [0, 1, 3])
@pytest.mark.parametrize("tau", [0.0, 0.05, math.inf])
@pytest.mark.parametrize("n,bc", [((5,), (0,)), ((5,), (1,)), ((3, 3), (0, 1))])
def test_oracle_matches_brute_force_off_lattice(n, bc, tau, scheme):
    """a free time step dt = 0.37 dx/dv (section 4.2 transport of the
    piecewise-constant pieces at accumulated offsets v_k n dt): four steps,
    so that the per-step shifts take both of their values"""
    d = len(n)
    nv = 5 if d == 1 else 3
    dv = 1.25
    dx = 1.0 / n[0]
    dt = 0.37 * dx / dv
    f0, _ = _start(d, n, nv, dv, seed=2000 + 10 * d + sum(bc))
    o = Oracle(d, n, dx, nv, dv, bc=bc, tau=tau, scheme=scheme, dt=dt)
    b = Brute(d, n, dx, nv, dv, bc, tau, scheme, dt=dt)
    o.set_f(f0)
    b.set_f(f0)
    o.step(4)
    b.step(4)
    eU, ef = _compare(o, b, d)
    assert eU < TOL and ef < TOL, (eU, ef)


@pytest.mark.parametrize("scheme", [0, 1, 3])
@pytest.mark.parametrize("tau", [0.05, 1.0, 0.0])
@pytest.mark.parametrize("n,bc,offl", [((5,), (1,), False), ((5,), (0,), True), ((3, 3), (0, 1), False)])
def test_oracle_matches_brute_force_strang(n, bc, offl, tau, scheme):
    """Strang splitting R_{dt/2} T R_{dt/2} per step.  For FKS the brute
    force applies the two half relaxations literally (an equilibrium formed
    at each); the oracle merges consecutive halves into one relaxation and
    applies the last half when f is read.  For HOFKS and its WENO variant
    both use the merged form (the merged relaxation's equilibrium part is
    the one the Euler solve advances)."""
    d = len(n)
    nv = 5 if d == 1 else 3
    dv = 1.25
    dx = 1.0 / n[0]
    dt = 0.37 * dx / dv if offl else None
    f0, _ = _start(d, n, nv, dv, seed=3000 + 10 * d + sum(bc))
    o = Oracle(d, n, dx, nv, dv, bc=bc, tau=tau, scheme=scheme, dt=dt, strang=True)
    b = Brute(d, n, dx, nv, dv, bc, tau, scheme, dt=dt, strang=True)
    o.set_f(f0)
    b.set_f(f0)
    o.step(3)
    b.step(3)
    eU, ef = _compare(o, b, d)
    assert eU < TOL and ef < TOL, (eU, ef)
