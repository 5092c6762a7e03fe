"""Seeded synthetic inputs shared by the GPU path and the oracle.

This module holds no arithmetic of the kinetic scheme: it only draws the
initial macroscopic fields (density rho, mean velocity u, temperature theta)
and names the grid sizes of each workload.  The paper's test problems are
analytic initial-value problems (section 5: Sod tubes, a disk-shaped 2D Sod
problem); the workloads below have their shapes and value ranges, with the
sizes of the throughput study.  Every random draw goes through
``numpy.random.default_rng(seed)``.

Layouts: cells are x-fastest; ``u`` is component-major ``(d, Nc)``.
"""
from dataclasses import dataclass, field
import math

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    d: int
    n: tuple            # cells per axis
    length: float       # domain edge, the domain is [0, length]^d
    nv: int             # velocity nodes per axis
    dv: float           # velocity step
    tau: float
    steps: int
    bc: tuple           # per axis: 0 periodic, 1 outflow
    precision: int = 0  # 0 FP64 pieces, 1 FP32 pieces
    extra: dict = field(default_factory=dict)

    @property
    def dx(self):
        return self.length / self.n[0]

    @property
    def nc(self):
        return int(np.prod(self.n))

    @property
    def nvel(self):
        return self.nv ** self.d

    @property
    def cv(self):
        """cell-velocity pairs updated per step"""
        return self.nc * self.nvel


def cell_centres(n, length):
    dx = length / n
    return (np.arange(n) + 0.5) * dx


# --------------------------------------------------------------------- 1D Sod
def sod_tube(nx, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), length=1.0,
             x_interface=0.5):
    """Riemann data: ``left``/``right`` are (rho, u, p); theta = p / rho."""
    x = cell_centres(nx, length)
    L = x < x_interface
    rho = np.where(L, left[0], right[0]).astype(np.float64)
    u = np.where(L, left[1], right[1]).astype(np.float64)[None, :]
    p = np.where(L, left[2], right[2]).astype(np.float64)
    return rho, u, p / rho


# ------------------------------------------------ smooth random Fourier fields
def fourier_field(n, d, max_mode, seed, length=1.0):
    """g(x) = sum_m a_m cos(2 pi m.x / L + phi_m) over the integer modes with
    1 <= max_a |m_a| <= max_mode, a_m ~ N(0,1)/|m|, phi_m ~ U[0, 2 pi),
    normalised so that max |g| = 1.  Sampled at cell centres, x-fastest."""
    rng = np.random.default_rng(seed)
    rng_axis = np.arange(-max_mode, max_mode + 1)
    modes = np.array(np.meshgrid(*([rng_axis] * d), indexing="ij")).reshape(d, -1).T
    modes = modes[np.abs(modes).max(axis=1) >= 1]
    amp = rng.standard_normal(len(modes)) / np.linalg.norm(modes, axis=1)
    phase = rng.uniform(0.0, 2.0 * np.pi, len(modes))
    x = cell_centres(n, length)
    grids = np.meshgrid(*([x] * d), indexing="ij")  # grids[a] varies along axis a
    g = np.zeros((n,) * d)
    for m, a, ph in zip(modes, amp, phase):
        arg = ph + sum(2.0 * np.pi * m[ax] * grids[ax] / length for ax in range(d))
        g += a * np.cos(arg)
    g /= np.abs(g).max()
    # meshgrid 'ij' puts axis 0 = x first; store x-fastest (C order of (z, y, x))
    return np.ascontiguousarray(np.transpose(g, list(range(d))[::-1])).reshape(-1)


def perturbed_gas(n, d, rho_amp, theta_amp, max_mode, seeds):
    """rho = 1 + rho_amp g1, theta = 1 + theta_amp g2, u = 0 (periodic box)."""
    nc = n ** d
    rho = np.ones(nc)
    theta = np.ones(nc)
    if rho_amp:
        rho = 1.0 + rho_amp * fourier_field(n, d, max_mode, seeds[0])
    if theta_amp:
        theta = 1.0 + theta_amp * fourier_field(n, d, max_mode, seeds[1])
    return rho, np.zeros((d, nc)), theta


# ------------------------------------------------------------- 2D disk (Sod)
def disk_2d(n, length=2.0, centre=(1.0, 1.0), radius=0.2,
            inside=(1.0, 1.0), outside=(0.125, 0.1)):
    """Disk-shaped Riemann data (section 5, 2D Sod): (rho, p) inside/outside."""
    x = cell_centres(n, length)
    X, Y = np.meshgrid(x, x, indexing="xy")  # Y varies along rows -> x-fastest
    r2 = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2
    ins = (r2 <= radius * radius).reshape(-1)
    rho = np.where(ins, inside[0], outside[0]).astype(np.float64)
    p = np.where(ins, inside[1], outside[1]).astype(np.float64)
    return rho, np.zeros((2, n * n)), p / rho


def planar_2d(n, length, angle, offset, left, right):
    """Planar Riemann data across the line through the domain centre shifted
    by `offset` along the normal (cos a, sin a); (rho, p) left/right, u = 0.
    The domain is periodic, so the data also jumps at the edges."""
    x = cell_centres(n, length)
    X, Y = np.meshgrid(x, x, indexing="xy")
    s = (X - 0.5 * length) * np.cos(angle) + (Y - 0.5 * length) * np.sin(angle) - offset
    lhs = (s < 0.0).reshape(-1)
    rho = np.where(lhs, left[0], right[0]).astype(np.float64)
    p = np.where(lhs, left[1], right[1]).astype(np.float64)
    return rho, np.zeros((2, n * n)), p / rho


@dataclass(frozen=True)
class ClosureRun:
    """One 2D-2V run that feeds the closure network (periodic square)."""
    kind: str            # "gas", "disk" or "planar"
    n: int
    length: float
    nv: int
    dv: float
    tau: float
    inside: tuple        # disk/planar: (rho, p) inside / left; gas: (rho_amp, theta_amp)
    outside: tuple
    geom: tuple          # disk: (cx, cy, r); planar: (angle, offset); gas: (modes, seed)

    def fields(self):
        if self.kind == "gas":
            modes, seed = self.geom
            return perturbed_gas(self.n, 2, self.inside[0], self.inside[1], modes,
                                 (seed, seed + 1))
        if self.kind == "disk":
            cx, cy, r = self.geom
            return disk_2d(self.n, self.length, (cx, cy), r, self.inside, self.outside)
        return planar_2d(self.n, self.length, self.geom[0], self.geom[1], self.inside,
                         self.outside)


def closure_runs(seed, count, n=128, dx=1.0 / 256, nv=32, dv=0.5, tau_range=(3e-4, 1e-2)):
    """Runs with the spacing of the 512^2 disk (dx = 1/256) and tau
    log-uniform: index i % 3 == 0 a smooth perturbed gas (density and
    temperature amplitudes U(0.05, 0.3), Fourier modes up to 2..6), 1 a disk
    and 2 a planar front at a random angle with rho ~ U(0.1, 1) and
    theta ~ U(0.6, 1.2) on each side (the velocity grid, |v| <= 8, spans six
    thermal widths)."""
    rng = np.random.default_rng(seed)
    length = n * dx
    out = []
    for i in range(count):
        tau = float(10.0 ** rng.uniform(np.log10(tau_range[0]), np.log10(tau_range[1])))
        if i % 3 == 0:
            amp = (float(rng.uniform(0.05, 0.3)), float(rng.uniform(0.05, 0.3)))
            geom = (int(rng.integers(2, 7)), int(rng.integers(1000, 100000)))
            out.append(ClosureRun("gas", n, length, nv, dv, tau, amp, (), geom))
            continue
        rl, rr = rng.uniform(0.1, 1.0, 2)
        pl, pr = rl * rng.uniform(0.6, 1.2), rr * rng.uniform(0.6, 1.2)
        if i % 3 == 1:
            geom = (float(rng.uniform(0.35, 0.65) * length), float(rng.uniform(0.35, 0.65) * length),
                    float(rng.uniform(0.1, 0.3) * length))
            kind = "disk"
        else:
            geom = (float(rng.uniform(0.0, np.pi)), float(rng.uniform(-0.1, 0.1) * length))
            kind = "planar"
        out.append(ClosureRun(kind, n, length, nv, dv, tau, (float(rl), float(pl)),
                              (float(rr), float(pr)), geom))
    return out


# -------------------------------------------------------- batched shock tubes
@dataclass(frozen=True)
class Tube:
    nx: int
    nv: int
    dv: float
    tau: float
    left: tuple   # (rho, u, p)
    right: tuple

    @property
    def dx(self):
        return 1.0 / self.nx


def batched_tubes(count=512, seed=4, nx_range=(200, 4000), nv_choices=(32, 64, 128),
                  log_tau_range=(-5.0, 0.0), state_range=(0.1, 1.0), v_cover=6.0):
    """Independent 1D outflow shock tubes on [0, 1] with an interface at 0.5.

    N_x ~ U{nx_range}, n_v ~ nv_choices, tau = 10^U(log_tau_range), left/right
    rho and p ~ U(state_range), u = 0.  dv is the smallest power of two with
    (n_v/2) dv >= v_cover * sqrt(theta_max) of the tube."""
    rng = np.random.default_rng(seed)
    tubes = []
    for _ in range(count):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        nv = int(rng.choice(nv_choices))
        tau = float(10.0 ** rng.uniform(*log_tau_range))
        rl, pl, rr, pr = rng.uniform(*state_range, size=4)
        th_max = max(pl / rl, pr / rr)
        need = v_cover * math.sqrt(th_max) / (nv / 2)
        dv = 2.0 ** math.ceil(math.log2(need))
        tubes.append(Tube(nx, nv, dv, tau, (float(rl), 0.0, float(pl)),
                          (float(rr), 0.0, float(pr))))
    return tubes


# ------------------------------------------------------------ named workloads
SOD_1D = Workload("sod1d_200x64_fp64", 1, (200,), 1.0, 64, 0.25, 1e-2, 100, (1,))
GAS_2D = Workload("gas2d_256sq_x_32sq_fp64", 2, (256, 256), 1.0, 32, 0.5, 1e-3, 200, (0, 0))
GAS_3D = Workload("gas3d_64cube_x_24cube_fp32", 3, (64, 64, 64), 1.0, 24, 0.5, 1e-3, 50,
                  (0, 0, 0), precision=1)
DISK_2D = Workload("disk2d_512sq_x_32sq_fp32", 2, (512, 512), 2.0, 32, 0.5, 1e-4, 100,
                   (0, 0), precision=1)


def initial_fields(wl: Workload):
    """(rho, u, theta) of a named workload."""
    if wl.name.startswith("sod1d"):
        return sod_tube(wl.n[0])
    if wl.name.startswith("gas2d"):
        return perturbed_gas(wl.n[0], 2, 0.2, 0.0, 8, (2, None))
    if wl.name.startswith("gas3d"):
        return perturbed_gas(wl.n[0], 3, 0.1, 0.1, 4, (3, 33))
    if wl.name.startswith("disk2d"):
        return disk_2d(wl.n[0], wl.length)
    raise KeyError(wl.name)
