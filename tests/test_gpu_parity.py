"""Parity of the HIP path (through the C ABI) with the CPU oracle.

The plain FP64 form must match the oracle to 1e-12 normwise per moment (and
on f); the FP32 precision form to 1e-5 on moments.  Free transport must be
bit-exact.  Every case prints its name, sizes and seed before running.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import Oracle
from tests.helpers import moment_errors, rel_inf

gpu = pytest.mark.gpu
TOL64 = 1e-12
TOL32 = 1e-5


def _solver(**kw):
    from paper_1212_0204_amd import Solver
    return Solver(**kw)


def announce(*a):
    print("CASE", *a, flush=True)


def run_pair(d, n, dx, nv, dv, bc, tau, steps, fields=None, f0=None, precision=0, scheme=0):
    o = Oracle(d, n, dx, nv, dv, bc=bc, tau=tau, scheme=scheme)
    s = _solver(dim=d, n_cells=n, dx=dx, n_vel=nv, dv=dv, bc=bc, precision=precision,
                scheme=scheme, tau=tau)
    if f0 is not None:
        o.set_f(f0)
        s.set_state_f(f0)
    else:
        o.init_macro(*fields)
        s.set_state_macro(*fields)
    o.step(steps)
    s.step(steps)
    return o, s


# ------------------------------------------------------------------- FP64
@gpu
def test_sod_tube_fp64_full_config():
    """1D-1V Sod: 200 cells x 64 velocities, tau = 1e-2, 100 steps, outflow."""
    wl = W.SOD_1D
    announce("sod1d", wl)
    o, s = run_pair(1, wl.n, wl.dx, wl.nv, wl.dv, wl.bc, wl.tau, wl.steps, W.initial_fields(wl))
    err = moment_errors(s.read_moments(), o.U, 1)
    assert err.max() < TOL64, err
    assert rel_inf(s.read_f(), o.f) < TOL64
    assert s.counters()[0] == o.substeps


@gpu
@pytest.mark.parametrize("tau", [0.0, 1e-4, 1e-2, 1.0])
def test_sod_tube_fp64_tau_sweep(tau):
    announce("sod1d tau", tau)
    rho, u, th = W.sod_tube(130)
    o, s = run_pair(1, (130,), 1 / 130, 24, 0.5, (1,), tau, 12, (rho, u, th))
    assert moment_errors(s.read_moments(), o.U, 1).max() < TOL64
    assert rel_inf(s.read_f(), o.f) < TOL64


@gpu
@pytest.mark.parametrize("d,n,nv", [(1, (97,), 16), (2, (70, 37), 10), (3, (23, 9, 11), 6)])
def test_free_transport_bit_exact(d, n, nv):
    """tau = +inf: pieces move by exactly k cells per step; bit-exact."""
    announce("free transport", d, n, nv)
    rng = np.random.default_rng(100 + d)
    f0 = rng.uniform(0.0, 1.0, (nv ** d, int(np.prod(n))))
    o, s = run_pair(d, n, 1.0 / n[0], nv, 0.5, (0,) * d, math.inf, 5, f0=f0)
    assert np.array_equal(s.read_f(), o.f)


@gpu
@pytest.mark.parametrize("n,bc,tau,scheme", [
    ((70, 37), (0, 0), 1e-3, 0),     # ragged x tile, several rows
    ((300, 20), (0, 0), 1e-2, 0),    # two x segments, ragged tail
    ((48, 40), (1, 1), 5e-3, 0),     # outflow on both axes
    ((64, 32), (0, 1), 0.0, 0),      # tau = 0: Euler only
    ((64, 32), (0, 0), 1e-2, 1),     # FKS
    ((64, 32), (0, 0), 1e-2, 2),     # unlimited
    ((67, 9), (0, 0), 1e-3, 0),      # odd x: a lane with one cell, pairs across the seam
    ((129, 5), (1, 0), 2e-3, 0),     # odd x over two 128-cell segments, outflow clamps
])
def test_2d_fp64(n, bc, tau, scheme):
    announce("2d fp64", n, bc, tau, scheme)
    rho, u, th = W.perturbed_gas(max(n), 2, 0.2, 0.1, 4, (21, 22))
    nn = max(n)
    rho = rho.reshape(nn, nn)[:n[1], :n[0]].reshape(-1)
    th = th.reshape(nn, nn)[:n[1], :n[0]].reshape(-1)
    u = 0.1 * np.stack([np.sin(np.linspace(0, 6, n[0] * n[1])), np.cos(np.linspace(0, 5, n[0] * n[1]))])
    o, s = run_pair(2, n, 1.0 / n[0], 16, 0.5, bc, tau, 8, (rho, u, th), scheme=scheme)
    assert moment_errors(s.read_moments(), o.U, 2).max() < TOL64
    assert rel_inf(s.read_f(), o.f) < TOL64
    if scheme != 1 and tau != math.inf:
        assert s.counters()[0] == o.substeps


@gpu
def test_3d_fp64():
    announce("3d fp64 (23, 9, 11) x 8^3")
    n = (23, 9, 11)
    rng = np.random.default_rng(31)
    nc = int(np.prod(n))
    rho = 1.0 + 0.2 * rng.uniform(-1, 1, nc)
    th = 1.0 + 0.2 * rng.uniform(-1, 1, nc)
    u = 0.2 * rng.uniform(-1, 1, (3, nc))
    o, s = run_pair(3, n, 1.0 / 23, 8, 0.75, (0, 1, 0), 1e-2, 4, (rho, u, th))
    assert moment_errors(s.read_moments(), o.U, 3).max() < TOL64
    assert rel_inf(s.read_f(), o.f) < TOL64


@gpu
@pytest.mark.parametrize("n,nv,bc,tau,prec", [
    ((70, 10, 6), 10, (1, 1, 1), 5e-3, 0),   # two x segments, ragged y blocks, outflow
    ((40, 7, 9), 16, (0, 0, 1), 1e-2, 0),    # periodic y shorter than the largest shift
    ((30, 5, 4), 24, (0, 1, 0), 2e-3, 0),    # the 24-node lattice of the 3D workload
    ((66, 9, 5), 16, (1, 0, 0), 1e-3, 1),    # FP32 form, ragged x and y
])
def test_3d_row_blocks(n, nv, bc, tau, prec):
    """3D steps with an Euler solve (blocks of four y rows sharing staged
    upstream rows): every block shape, ragged tail and boundary"""
    announce("3d row blocks", n, nv, bc, tau, prec)
    rng = np.random.default_rng(37)
    nc = int(np.prod(n))
    rho = 1.0 + 0.2 * rng.uniform(-1, 1, nc)
    th = 1.0 + 0.2 * rng.uniform(-1, 1, nc)
    u = 0.2 * rng.uniform(-1, 1, (3, nc))
    o, s = run_pair(3, n, 1.0 / n[0], nv, 0.5, bc, tau, 3, (rho, u, th), precision=prec)
    tol = TOL64 if prec == 0 else TOL32
    assert moment_errors(s.read_moments(), o.U, 3).max() < tol
    assert rel_inf(s.read_f(), o.f) < tol


@gpu
def test_gas2d_full_size_three_steps():
    """the 256^2 x 32^2 perturbed-gas workload at full size, 3 steps"""
    wl = W.GAS_2D
    announce("gas2d full", wl)
    o, s = run_pair(2, wl.n, wl.dx, wl.nv, wl.dv, wl.bc, wl.tau, 3, W.initial_fields(wl))
    assert moment_errors(s.read_moments(), o.U, 2).max() < TOL64
    f = s.read_f()
    fo = o.f
    assert rel_inf(f, fo) < TOL64


@gpu
def test_gas2d_full_size_conservation_200_steps():
    """periodic conservation of mass, momentum and energy over the whole run"""
    wl = W.GAS_2D
    announce("gas2d conservation", wl)
    s = _solver(dim=2, n_cells=wl.n, dx=wl.dx, n_vel=wl.nv, dv=wl.dv, bc=wl.bc, tau=wl.tau)
    s.set_state_macro(*W.initial_fields(wl))
    U0 = s.read_moments()
    s.step(wl.steps)
    U = s.read_moments()
    tot0, tot = U0.sum(1), U.sum(1)
    scale = np.abs(U0[0]).max() * U0.shape[1]  # momentum is measured in rho * 1 units
    assert (np.abs(tot - tot0) / scale).max() < 1e-13



@gpu
def test_gas3d_fp32_full_size_conservation():
    """the FP32 3D form at its full size (64^3 cells x 24^3 velocities, 14.5
    GB of pieces per buffer): periodic totals stay fixed over 3 steps to the
    FP32 rounding of the pieces, and U stays physical"""
    wl = W.GAS_3D
    announce("gas3d fp32 conservation", wl)
    s = _solver(dim=3, n_cells=wl.n, dx=wl.dx, n_vel=wl.nv, dv=wl.dv, bc=wl.bc, tau=wl.tau,
                precision=1)
    s.set_state_macro(*W.initial_fields(wl))
    U0 = s.read_moments()
    s.step(3)
    U = s.read_moments()
    tot0, tot = U0.sum(1), U.sum(1)
    scale = np.abs(U0[0]).max() * U0.shape[1]
    assert (np.abs(tot - tot0) / scale).max() < 1e-6
    assert np.isfinite(U).all() and U[0].min() > 0


# ------------------------------------------------------------------- FP32
@gpu
@pytest.mark.parametrize("d,n,nv,dv,tau", [(2, (70, 37), 16, 0.5, 1e-3), (3, (20, 12, 10), 12, 0.5, 1e-3),
                                           (1, (200,), 64, 0.25, 1e-2)])
def test_precision_form_moments(d, n, nv, dv, tau):
    announce("fp32", d, n, nv, tau)
    nc = int(np.prod(n))
    if d == 1:
        fields = W.sod_tube(n[0])
        bc = (1,)
    else:
        rng = np.random.default_rng(41)
        fields = (1.0 + 0.1 * rng.uniform(-1, 1, nc), 0.05 * rng.uniform(-1, 1, (d, nc)),
                  1.0 + 0.1 * rng.uniform(-1, 1, nc))
        bc = (0,) * d
    o, s = run_pair(d, n, 1.0 / n[0], nv, dv, bc, tau, 10, fields, precision=1)
    err = moment_errors(s.read_moments(), o.U, d)
    print("fp32 moment errors", err)
    assert err.max() < TOL32, err


# ----------------------------------------------------------- error paths
@gpu
def test_nonphysical_state_is_reported():
    from paper_1212_0204_amd import HofksError
    announce("nonphysical")
    s = _solver(dim=1, n_cells=(64,), dx=1 / 64, n_vel=8, dv=0.5, bc=(0,), tau=1e-2)
    with pytest.raises(HofksError) as e:
        s.set_state_macro(np.r_[np.ones(63), -1.0], np.zeros((1, 64)), np.ones(64))
    assert e.value.status == -4
    f = np.full((8, 64), 0.1)
    f[3, 5] = np.nan
    with pytest.raises(HofksError) as e:  # reported at the first synchronising call
        s.set_state_f(f)
        s.step(1)
        s.read_moments()
    assert e.value.status == -4


@gpu
def test_step_before_state_is_rejected():
    from paper_1212_0204_amd import HofksError
    s = _solver(dim=1, n_cells=(64,), dx=1 / 64, n_vel=8, dv=0.5, bc=(0,), tau=1e-2)
    with pytest.raises(HofksError) as e:
        s.step(1)
    assert e.value.status == -5


@gpu
def test_tau_change_mid_run_matches_oracle():
    announce("tau change")
    rho, u, th = W.sod_tube(96)
    o = Oracle(1, (96,), 1 / 96, 16, 0.5, bc=(1,), tau=1e-2)
    s = _solver(dim=1, n_cells=(96,), dx=1 / 96, n_vel=16, dv=0.5, bc=(1,), tau=1e-2)
    o.init_macro(rho, u, th)
    s.set_state_macro(rho, u, th)
    for tau in (1e-2, 1e-3, math.inf, 0.0, 1e-1):
        o.set_tau(tau)
        s.set_tau(tau)
        o.step(3)
        s.step(3)
    assert moment_errors(s.read_moments(), o.U, 1).max() < TOL64
    assert rel_inf(s.read_f(), o.f) < TOL64


@gpu
def test_grid_autotune_then_parity(tmp_path):
    """the autotuner picks a kinetic configuration (and reuses a cached one);
    results after re-initialisation still match the oracle"""
    announce("grid autotune")
    n = (96, 40)
    rho, u, th = W.perturbed_gas(96, 2, 0.2, 0.1, 4, (51, 52))
    rho = rho.reshape(96, 96)[:40].reshape(-1)
    th = th.reshape(96, 96)[:40].reshape(-1)
    u = u[:, :96 * 40]
    s = _solver(dim=2, n_cells=n, dx=1 / 96, n_vel=16, dv=0.5, bc=(0, 0), tau=1e-3)
    s.set_state_macro(rho, u, th)
    cache = str(tmp_path / "tune.jsonl")
    ng, unr, seq = s.autotune(steps=2, cache_path=cache)
    assert ng in (2, 4, 8) and unr in (4, 8, 16) and seq in (0, 1)
    assert s.autotune(steps=2, cache_path=cache) == (ng, unr, seq)
    s.set_state_macro(rho, u, th)
    s.step(6)
    o = Oracle(2, n, 1 / 96, 16, 0.5, bc=(0, 0), tau=1e-3)
    o.init_macro(rho, u, th)
    o.step(6)
    assert moment_errors(s.read_moments(), o.U, 2).max() < TOL64


@gpu
@pytest.mark.parametrize("d,n,nv,prec,bc", [(2, (70, 37), 10, 0, (0, 0)), (3, (20, 12, 10), 6, 1, (0, 1, 0)),
                                             (1, (150,), 16, 0, (1,))])
def test_checkpoint_resume_is_exact(d, n, nv, prec, bc):
    """a state image taken after 3 steps, restored into a fresh context,
    continues bit for bit like the original run"""
    announce("checkpoint", d, n, nv, prec, bc)
    from paper_1212_0204_amd import HofksError, Solver
    rng_fields = W.perturbed_gas(n[0], d, 0.2, 0.1, 2, (11, 12)) if d > 1 else W.sod_tube(n[0])
    if d == 2 and n[0] != n[1] or d == 3:
        rho = 1.0 + 0.1 * np.sin(np.arange(int(np.prod(n))) * 0.37)
        rng_fields = (rho, np.zeros((d, rho.size)), np.ones(rho.size))
    dx = 1.0 / n[0]
    s1 = Solver(d, n, dx, nv, 0.5, bc=bc, precision=prec, tau=2e-2)
    s1.set_state_macro(*rng_fields)
    s1.step(3)
    img = s1.read_state()
    s1.step(4)
    Ua, fa = s1.read_moments(), s1.read_f()
    s2 = Solver(d, n, dx, nv, 0.5, bc=bc, precision=prec, tau=1.0)
    s2.write_state(img)
    assert s2.counters()[1] == 3
    s2.step(4)
    assert np.array_equal(s2.read_moments(), Ua)
    assert np.array_equal(s2.read_f(), fa)
    s3 = Solver(d, n, dx, nv + 2, 0.5, bc=bc, precision=prec, tau=2e-2)
    with pytest.raises(HofksError):
        s3.write_state(img)


@gpu
@pytest.mark.parametrize("d,n,nv,prec", [(2, (70, 37), 16, 0), (3, (20, 12, 10), 8, 1)])
def test_steps_in_one_call_equal_single_steps(d, n, nv, prec):
    """within one step call the next step's Euler solve forks before the
    records of the current step are formed; the results are bit for bit
    those of single-step calls"""
    announce("one call vs single steps", d, n, nv, prec)
    from paper_1212_0204_amd import Solver
    nc = int(np.prod(n))
    rng = np.random.default_rng(19)
    fields = (1.0 + 0.2 * rng.uniform(-1, 1, nc), 0.1 * rng.uniform(-1, 1, (d, nc)),
              1.0 + 0.2 * rng.uniform(-1, 1, nc))
    runs = []
    for split in (False, True):
        s = Solver(d, n, 1.0 / n[0], nv, 0.5, bc=(0,) * d, precision=prec, tau=1e-3)
        s.set_state_macro(*fields)
        if split:
            for _ in range(6):
                s.step(1)
        else:
            s.step(6)
        runs.append((s.read_moments(), s.read_f()))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])


# ------------------------------------------- relaxation weight lambda = 1/2
def _lam_half_tau(dx, dv):
    """tau with lambda = exp(-dt/tau) = 1/2 on the lattice dt = dx/dv, so that
    the relaxed pieces carry half of U^{n+1}"""
    return (dx / dv) / math.log(2.0)


def _random_fields(d, nc, seed, amp=0.2):
    rng = np.random.default_rng(seed)
    return (1.0 + amp * rng.uniform(-1, 1, nc), 0.1 * rng.uniform(-1, 1, (d, nc)),
            1.0 + amp * rng.uniform(-1, 1, nc))


@gpu
@pytest.mark.parametrize("d,n,nv,bc", [
    (2, (70, 37), 16, (0, 0)),        # ragged x tile, several rows
    (2, (131, 19), 12, (1, 0)),       # three x segments, outflow x
    (3, (66, 9, 5), 12, (0, 1, 0)),   # ragged x and y row blocks
    (3, (20, 12, 10), 8, (1, 1, 1)),
])
def test_precision_form_at_lambda_half(d, n, nv, bc):
    """FP32 pieces where they carry half of U^{n+1} (lambda = 1/2): the FP32
    relaxation and shift of the 2D and 3D kinetic kernels reach the moments;
    1e-5 per moment and on f after 6 steps"""
    dv = 0.5
    dx = 1.0 / n[0]
    tau = _lam_half_tau(dx, dv)
    announce("fp32 lambda 1/2", d, n, nv, bc, f"tau={tau:.4g}")
    nc = int(np.prod(n))
    o, s = run_pair(d, n, dx, nv, dv, bc, tau, 6, _random_fields(d, nc, 43), precision=1)
    assert abs(o.lam - 0.5) < 1e-12
    err = moment_errors(s.read_moments(), o.U, d)
    ef = rel_inf(s.read_f(), o.f)
    print("fp32 lambda=1/2 moment errors", err, "f", ef)
    assert err.max() < TOL32, err
    assert ef < TOL32, ef


@gpu
@pytest.mark.parametrize("n,nv,bc", [((70, 10, 6), 10, (1, 1, 1)), ((30, 5, 4), 24, (0, 1, 0))])
def test_3d_fp64_at_lambda_half(n, nv, bc):
    """the 3D kinetic kernel (blocks of four y rows) in FP64 where the
    relaxed pieces carry half of U^{n+1}: 1e-12"""
    dv, dx = 0.5, 1.0 / n[0]
    tau = _lam_half_tau(dx, dv)
    announce("3d fp64 lambda 1/2", n, nv, bc)
    o, s = run_pair(3, n, dx, nv, dv, bc, tau, 4, _random_fields(3, int(np.prod(n)), 47))
    err = moment_errors(s.read_moments(), o.U, 3)
    print("3d fp64 lambda=1/2 moment errors", err)
    assert err.max() < TOL64, err
    assert rel_inf(s.read_f(), o.f) < TOL64


@gpu
@pytest.mark.parametrize("lam", [0.0, 0.5])
def test_gas3d_reduced_grid_fp32(lam):
    """the 3D FP32 workload's velocity grid (24^3, dv = 1/2) and field recipe
    on a 32^3 grid, 3 steps, against the oracle: with the workload's tau
    (lambda ~ 1e-14, the Euler part dominates) and with lambda = 1/2"""
    wl = W.GAS_3D
    n = (32, 32, 32)
    dx = 1.0 / 32
    rho, u, th = W.perturbed_gas(32, 3, 0.1, 0.1, 4, (3, 33))
    tau = _lam_half_tau(dx, wl.dv) if lam else wl.tau
    announce("gas3d reduced 32^3 x 24^3 fp32", f"tau={tau:.4g}")
    o, s = run_pair(3, n, dx, wl.nv, wl.dv, wl.bc, tau, 3, (rho, u, th), precision=1)
    err = moment_errors(s.read_moments(), o.U, 3)
    ef = rel_inf(s.read_f(), o.f)
    print(f"gas3d 32^3 fp32 lambda={o.lam:.3g} moment errors", err, "f", ef)
    assert err.max() < TOL32, err
    assert ef < TOL32, ef


# ------------------------------------------------ persistent Euler tail
@gpu
@pytest.mark.parametrize("d,n,nv,bc,tau", [
    (1, (130,), 24, (1,), 1e-2),
    (1, (256,), 16, (0,), 1e-2),   # the largest 1D grid of one tail block
    (1, (257,), 16, (1,), 1e-2),   # two blocks: arrival counters
    (1, (700,), 24, (1,), 1e-2),
    (2, (70, 37), 16, (0, 0), 1e-3),
    (2, (48, 40), 16, (1, 1), 5e-3),
    (3, (23, 9, 11), 8, (0, 1, 0), 1e-2),
])
def test_euler_tail_every_substep(d, n, nv, bc, tau):
    """one single-sub-step Euler launch per step: every further sub-step runs
    in the persistent kernel (grid barrier, per-block speed maxima); the
    library's tail counter shows that it ran; 1e-12 against the oracle"""
    announce("euler tail", d, n, nv, bc, tau)
    from paper_1212_0204_amd import Solver
    nc = int(np.prod(n))
    fields = W.sod_tube(n[0]) if d == 1 else _random_fields(d, nc, 53)
    dx = 1.0 / n[0]
    o = Oracle(d, n, dx, nv, 0.5, bc=bc, tau=tau)
    s = Solver(d, n, dx, nv, 0.5, bc=bc, tau=tau)
    s.set_euler_launches(1)
    o.init_macro(*fields)
    s.set_state_macro(*fields)
    expect = 0
    for _ in range(5):  # the tail runs every sub-step after the first
        o.step(1)
        expect += o.substeps - 1
    s.step(5)
    tail = s.tail_substeps()
    assert tail == expect and tail > 0, (tail, expect)
    err = moment_errors(s.read_moments(), o.U, d)
    assert err.max() < TOL64, err
    assert rel_inf(s.read_f(), o.f) < TOL64
    assert s.counters()[0] == o.substeps


@gpu
def test_disk_substeps_grow_within_one_call():
    """a disk-shaped Riemann problem (section 5, 2D Sod geometry) on a 40^2
    periodic grid, lambda ~ 0.29: the sub-step count jumps from 12 to 18
    at the second step, inside one step call, beyond the one spare launch,
    so the persistent tail runs the extra sub-steps; 1e-12 after 8 steps"""
    n = (40, 40)
    dx = 2.0 / 40
    rho, u, th = W.disk_2d(40, 2.0, (1.0, 1.0), 0.3)
    announce("disk 40^2 substep growth")
    from paper_1212_0204_amd import Solver
    o = Oracle(2, n, dx, 16, 0.5, bc=(0, 0), tau=0.08)
    s = Solver(2, n, dx, 16, 0.5, bc=(0, 0), tau=0.08)
    o.init_macro(rho, u, th)
    s.set_state_macro(rho, u, th)
    o.step(8)
    s.step(8)
    tail = s.tail_substeps()
    print("tail sub-steps", tail)
    assert tail >= 5
    err = moment_errors(s.read_moments(), o.U, 2)
    assert err.max() < TOL64, err
    assert rel_inf(s.read_f(), o.f) < TOL64


@gpu
@pytest.mark.parametrize("before", [0, 1])
def test_long_call_follows_a_moving_substep_count(before):
    """the 40^2 periodic disk at tau = 0.02, whose sub-step count moves
    between 12 and 18 over 70 steps: in one 70-step call the host reads the
    count of earlier steps back and sizes the per-sub-step launches from it
    (with the spare launch dropped while two reads agree); with the Euler
    solve beside (0) or before (1) the kinetic kernel.  1e-12 against the
    oracle and against the same run in single-step calls, and fewer tail
    sub-steps than those calls, whose count stays at the initial one"""
    n = (40, 40)
    dx = 2.0 / 40
    rho, u, th = W.disk_2d(40, 2.0, (1.0, 1.0), 0.3)
    announce("disk 40^2 long call, euler before", before)
    from paper_1212_0204_amd import Solver
    o = Oracle(2, n, dx, 16, 0.5, bc=(0, 0), tau=0.02)
    o.init_macro(rho, u, th)
    o.step(70)
    runs = []
    for calls in (1, 70):
        s = Solver(2, n, dx, 16, 0.5, bc=(0, 0), tau=0.02)
        s.set_launch_config(4, 4, before)
        s.set_state_macro(rho, u, th)
        for _ in range(70 // calls):
            s.step(calls)
        s.sync()
        runs.append((s.read_moments(), s.read_f(), s.tail_substeps(), s.counters()))
        s.close()
    (U1, f1, t1, c1), (U70, f70, t70, c70) = runs
    print("tail sub-steps: single-step calls", t1, "one call", t70)
    assert c1 == c70 == (o.substeps, 70), (c1, c70, o.substeps)
    assert 0 < t70 < t1, (t70, t1)
    for U, f in ((U1, f1), (U70, f70)):
        err = moment_errors(U, o.U, 2)
        assert err.max() < TOL64, err
        assert rel_inf(f, o.f) < TOL64
    assert moment_errors(U70, U1, 2).max() < TOL64


# ------------------------------------------ WENO Euler solve (scheme 3)
@gpu
@pytest.mark.parametrize("d,n,nv,bc,tau,prec,launches", [
    (1, (200,), 64, (1,), 1e-2, 0, 0),         # the Sod tube workload's lattice
    (1, (130,), 24, (1,), 0.0, 0, 0),          # tau = 0: Euler only
    (1, (97,), 16, (0,), 1.0, 0, 1),           # periodic; persistent tail for every later sub-step
    (2, (70, 37), 16, (0, 0), 1e-3, 0, 0),     # ragged tiles
    (2, (48, 40), 16, (1, 1), 5e-3, 0, 1),     # outflow both axes; tail
    (2, (67, 9), 12, (0, 0), 2e-2, 1, 0),      # FP32 pieces
    (3, (23, 9, 11), 8, (0, 1, 0), 1e-2, 0, 0),
    (3, (20, 12, 10), 8, (1, 1, 1), 5e-3, 1, 1),
])
def test_weno_scheme_parity(d, n, nv, bc, tau, prec, launches):
    """HOFKS with the WENO Euler solve (scheme 3) against the oracle: 1e-12
    in FP64, 1e-5 with FP32 pieces, on U and f; sub-step counts equal; with
    one single-sub-step launch per step the persistent tail runs the rest"""
    announce("weno", d, n, nv, bc, tau, prec, launches)
    from paper_1212_0204_amd import Solver
    nc = int(np.prod(n))
    fields = W.sod_tube(n[0]) if d == 1 else _random_fields(d, nc, 59)
    dx = 1.0 / n[0]
    dv = 0.25 if nv == 64 else 0.5
    o = Oracle(d, n, dx, nv, dv, bc=bc, tau=tau, scheme=3)
    s = Solver(d, n, dx, nv, dv, bc=bc, tau=tau, precision=prec, scheme=3)
    if launches:
        s.set_euler_launches(launches)
    o.init_macro(*fields)
    s.set_state_macro(*fields)
    steps = 20 if d == 1 else 5
    o.step(steps)
    s.step(steps)
    tol = TOL64 if prec == 0 else TOL32
    err = moment_errors(s.read_moments(), o.U, d)
    print("weno moment errors", err, "substeps", o.substeps, "tail", s.tail_substeps())
    assert err.max() < tol, err
    assert rel_inf(s.read_f(), o.f) < tol
    assert s.counters()[0] == o.substeps
    if launches:
        assert s.tail_substeps() > 0


# ------------------------------------- off-lattice velocities (section 4.2)
@gpu
@pytest.mark.parametrize("d,n,nv,frac", [(1, (97,), 16, 0.37), (2, (70, 37), 12, math.sqrt(2) / 3),
                                         (3, (23, 9, 11), 8, 0.61)])
def test_offlattice_free_transport_bit_exact(d, n, nv, frac):
    """tau = +inf with dt = frac dx/dv: the pieces follow their accumulated
    offsets v_k n dt; bit-exact against the oracle over 9 steps"""
    announce("off-lattice free transport", d, n, nv, frac)
    dx, dv = 1.0 / n[0], 0.5
    rng = np.random.default_rng(200 + d)
    f0 = rng.uniform(0.0, 1.0, (nv ** d, int(np.prod(n))))
    from paper_1212_0204_amd import Solver
    o = Oracle(d, n, dx, nv, dv, bc=(0,) * d, tau=math.inf, dt=frac * dx / dv)
    s = Solver(d, n, dx, nv, dv, bc=(0,) * d, tau=math.inf, dt=frac * dx / dv)
    o.set_f(f0)
    s.set_state_f(f0)
    o.step(9)
    s.step(9)
    assert np.array_equal(s.read_f(), o.f)


@gpu
@pytest.mark.parametrize("d,n,nv,bc,tau,frac,prec,scheme", [
    (1, (200,), 64, (1,), 1e-2, 1.0 / 32, 0, 0),   # the Sod lattice at kinetic CFL 1
    (1, (130,), 24, (1,), 2e-3, 0.45, 0, 3),       # with the WENO Euler solve
    (2, (70, 37), 16, (0, 0), 1e-2, 0.3, 0, 0),
    (2, (48, 40), 16, (1, 1), 5e-3, 0.7, 0, 1),    # FKS, outflow
    (2, (67, 19), 12, (0, 1), None, 0.55, 1, 0),   # FP32 pieces at lambda = 1/2
    (3, (20, 12, 10), 8, (0, 1, 0), 1e-2, 0.4, 0, 0),
    (3, (23, 9, 11), 8, (1, 1, 1), None, 0.6, 1, 0),
])
def test_offlattice_parity(d, n, nv, bc, tau, frac, prec, scheme):
    """HOFKS with a free time step: per-step shifts of floor(c) or ceil(c)
    cells; 1e-12 (FP64) or 1e-5 (FP32 pieces) on U and f after 12 steps"""
    dx = 1.0 / n[0]
    dv = 0.25 if nv == 64 else 0.5
    dt = frac * dx / dv
    if tau is None:  # lambda = 1/2
        tau = dt / math.log(2.0)
    announce("off-lattice", d, n, nv, bc, tau, frac, prec, scheme)
    from paper_1212_0204_amd import Solver
    nc = int(np.prod(n))
    fields = W.sod_tube(n[0]) if d == 1 else _random_fields(d, nc, 61)
    o = Oracle(d, n, dx, nv, dv, bc=bc, tau=tau, scheme=scheme, dt=dt)
    s = Solver(d, n, dx, nv, dv, bc=bc, tau=tau, precision=prec, scheme=scheme, dt=dt)
    o.init_macro(*fields)
    s.set_state_macro(*fields)
    o.step(12)
    s.step(12)
    assert abs(s.dt - dt) == 0
    tol = TOL64 if prec == 0 else TOL32
    err = moment_errors(s.read_moments(), o.U, d)
    print("off-lattice moment errors", err, "substeps", o.substeps)
    assert err.max() < tol, err
    assert rel_inf(s.read_f(), o.f) < tol
    if scheme != 1:
        assert s.counters()[0] == o.substeps


@gpu
def test_offlattice_checkpoint_resume_is_exact():
    """the per-step shifts depend on the step count, which the state image
    carries: a restored run continues bit for bit"""
    from paper_1212_0204_amd import HofksError, Solver
    announce("off-lattice checkpoint")
    n, dx, nv, dv = (70, 37), 1.0 / 70, 12, 0.5
    dt = 0.41 * dx / dv
    fields = _random_fields(2, 70 * 37, 67)
    s1 = Solver(2, n, dx, nv, dv, tau=3e-2, dt=dt)
    s1.set_state_macro(*fields)
    s1.step(5)
    img = s1.read_state()
    s1.step(6)
    s2 = Solver(2, n, dx, nv, dv, tau=1.0, dt=dt)
    s2.write_state(img)
    s2.step(6)
    assert np.array_equal(s2.read_moments(), s1.read_moments())
    assert np.array_equal(s2.read_f(), s1.read_f())
    s3 = Solver(2, n, dx, nv, dv, tau=3e-2)  # the lattice dt: another grid
    with pytest.raises(HofksError):
        s3.write_state(img)


# ---------------------------------------- Strang splitting (section 4.2)
@gpu
@pytest.mark.parametrize("d,n,nv,bc,tau,prec,scheme,frac", [
    (1, (200,), 64, (1,), 1e-2, 0, 0, None),
    (1, (130,), 24, (1,), 0.05, 0, 1, 0.6),        # FKS, off-lattice
    (2, (70, 37), 16, (0, 0), None, 0, 0, None),   # lambda = 1/2
    (2, (48, 40), 16, (1, 1), 5e-3, 0, 3, None),   # WENO
    (2, (67, 19), 12, (0, 1), None, 1, 0, 0.55),   # FP32 pieces, off-lattice
    (3, (20, 12, 10), 8, (0, 1, 0), None, 0, 0, None),
])
def test_strang_parity(d, n, nv, bc, tau, prec, scheme, frac):
    """Strang splitting: the first step relaxes by half, the read f carries
    the pending half relaxation; 1e-12 (FP64) or 1e-5 (FP32) on U and f
    after 1 and after 8 steps"""
    dx = 1.0 / n[0]
    dv = 0.25 if nv == 64 else 0.5
    dt = frac * dx / dv if frac else None
    h = dt if dt else dx / dv
    if tau is None:
        tau = h / math.log(2.0)
    announce("strang", d, n, nv, bc, tau, prec, scheme, frac)
    from paper_1212_0204_amd import Solver
    nc = int(np.prod(n))
    fields = W.sod_tube(n[0]) if d == 1 else _random_fields(d, nc, 71)
    o = Oracle(d, n, dx, nv, dv, bc=bc, tau=tau, scheme=scheme, dt=dt, strang=True)
    s = Solver(d, n, dx, nv, dv, bc=bc, tau=tau, precision=prec, scheme=scheme, dt=dt, strang=True)
    o.init_macro(*fields)
    s.set_state_macro(*fields)
    tol = TOL64 if prec == 0 else TOL32
    for steps in (1, 7):
        o.step(steps)
        s.step(steps)
        err = moment_errors(s.read_moments(), o.U, d)
        ef = rel_inf(s.read_f(), o.f)
        print("strang moment errors", err, "f", ef)
        assert err.max() < tol, err
        assert ef < tol, ef


@gpu
def test_strang_tau_change_and_checkpoint():
    """a tau change between steps merges the two different half relaxations;
    a state image taken in between continues bit for bit"""
    announce("strang tau change + checkpoint")
    from paper_1212_0204_amd import Solver
    rho, u, th = W.sod_tube(96)
    o = Oracle(1, (96,), 1 / 96, 16, 0.5, bc=(1,), tau=1e-2, strang=True)
    s = Solver(1, (96,), 1 / 96, 16, 0.5, bc=(1,), tau=1e-2, strang=True)
    o.init_macro(rho, u, th)
    s.set_state_macro(rho, u, th)
    img = None
    for i, tau in enumerate((1e-2, 0.2, math.inf, 0.0, 3e-2)):
        o.set_tau(tau)
        s.set_tau(tau)
        if i == 2:
            img = s.read_state()
        o.step(3)
        s.step(3)
    assert moment_errors(s.read_moments(), o.U, 1).max() < TOL64
    assert rel_inf(s.read_f(), o.f) < TOL64
    s2 = Solver(1, (96,), 1 / 96, 16, 0.5, bc=(1,), tau=1.0, strang=True)
    s2.write_state(img)
    for tau in (math.inf, 0.0, 3e-2):
        s2.set_tau(tau)
        s2.step(3)
    assert np.array_equal(s2.read_moments(), s.read_moments())
    assert np.array_equal(s2.read_f(), s.read_f())


@gpu
@pytest.mark.parametrize("d,n,nv,prec,cfg", [
    (2, (70, 37), 16, 0, (4, 4)), (2, (67, 19), 12, 1, (8, 16)), (3, (20, 12, 10), 8, 1, (4, 8)),
    (1, (130,), 24, 0, (4, 8)),
])
def test_euler_before_or_beside_the_kinetic_kernel(d, n, nv, prec, cfg):
    """the Euler solve before the kinetic kernel (one stream) or beside it
    (a second stream): bit-identical results, and the oracle's"""
    announce("euler placement", d, n, nv, prec, cfg)
    from paper_1212_0204_amd import Solver
    nc = int(np.prod(n))
    fields = W.sod_tube(n[0]) if d == 1 else _random_fields(d, nc, 73)
    bc = (1,) if d == 1 else (0,) * d
    runs = []
    for before in (0, 1):
        s = Solver(d, n, 1.0 / n[0], nv, 0.5, bc=bc, tau=2e-2, precision=prec)
        s.set_launch_config(cfg[0], cfg[1], before)
        s.set_state_macro(*fields)
        s.step(3)
        s.step(4)
        runs.append((s.read_moments(), s.read_f()))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    o = Oracle(d, n, 1.0 / n[0], nv, 0.5, bc=bc, tau=2e-2)
    o.init_macro(*fields)
    o.step(7)
    assert moment_errors(runs[1][0], o.U, d).max() < (TOL64 if prec == 0 else TOL32)


@gpu
def test_kernel_timing_records_the_masked_groups_only():
    """the timing mask: events around the kinetic launches only, then around
    the Euler and update groups only; the launch counts follow the mask and
    the results do not depend on it; a mask outside 0..15 is rejected"""
    announce("kernel timing mask")
    from paper_1212_0204_amd import Solver, _lib
    n = (40, 36)
    fields = _random_fields(2, 40 * 36, 91)
    s = Solver(2, n, 1.0 / 40, 16, 0.5, bc=(0, 0), tau=1e-3)
    s.set_state_macro(*fields)
    s.kernel_timing(enable=True, groups=(1,))
    s.step(5)
    ms, cnt = s.kernel_timing(enable=True, groups=(0, 2))
    assert cnt[1] == 5 and cnt[0] == cnt[2] == cnt[3] == 0 and ms[1] > 0, (ms, cnt)
    s.step(5)
    ms, cnt = s.kernel_timing(enable=False)
    assert cnt[0] > 0 and cnt[2] > 0 and cnt[1] == cnt[3] == 0, (ms, cnt)
    U = s.read_moments()
    s.step(1)
    assert s.kernel_timing(enable=False)[1] == [0, 0, 0, 0]
    for bad in (16, -1):
        assert _lib.lib().hofks_kernel_timing(s._h, bad, None, None) != 0
    r = Solver(2, n, 1.0 / 40, 16, 0.5, bc=(0, 0), tau=1e-3)
    r.set_state_macro(*fields)
    r.step(10)
    assert np.array_equal(r.read_moments(), U)
