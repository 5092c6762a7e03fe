"""``Solver``: one grid + velocity set on one GPU, through the C ABI.

Argument marshalling only: arrays are handed to the library as host pointers,
the workspace is a torch uint8 tensor on the current device and kernels run on
torch's current HIP stream.
"""
import ctypes
import math

import numpy as np
import torch

from . import _lib


class HofksError(RuntimeError):
    def __init__(self, status, what, msg=""):
        name = _lib.STATUS_NAMES.get(status, str(status))
        super().__init__(f"{what}: {name} {msg}".strip())
        self.status = status


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Solver:
    """HOFKS on a Cartesian grid of ``n_cells`` (x first) with ``n_vel`` velocity
    nodes per axis spaced ``dv``; the time step is ``dx / dv`` (the lattice) unless
    a smaller ``dt`` is given.

    precision: 0 FP64 pieces; 1 FP32 pieces with FP64 compensated moment sums.
    scheme: 0 HOFKS; 1 FKS (no Euler coupling); 2 HOFKS with phi == 1;
    3 HOFKS with the WENO Euler solve.
    bc per axis: 0 periodic, 1 outflow.
    dt: None for the lattice dt = dx/dv; 0 < dt <= dx/dv for off-lattice
    transport.
    strang: Strang splitting R_{dt/2} T_dt R_{dt/2} instead of the
    first-order relaxation-then-transport step.
    """

    def __init__(self, dim, n_cells, dx, n_vel, dv, bc=None, precision=0, scheme=0,
                 tau=math.inf, stream=None, dt=None, strang=False):
        L = _lib.lib()
        # held here so that close() still works while the interpreter tears
        # down module globals
        self._destroy = L.hofks_destroy
        if not torch.cuda.is_available():
            raise RuntimeError("the HOFKS library needs a ROCm GPU")
        n = (list(n_cells) + [1, 1, 1])[:3]
        b = (list(bc if bc is not None else [0, 0, 0]) + [0, 0, 0])[:3]
        self.desc = _lib.GridDesc(dim, (ctypes.c_int * 3)(*n), float(dx), int(n_vel), float(dv),
                                  (ctypes.c_int * 3)(*b), int(precision), int(scheme),
                                  float(dt or 0.0), int(bool(strang)))
        self.d, self.nm = dim, dim + 2
        self.nc = int(np.prod(n[:dim]))
        self.nv = int(n_vel) ** dim
        size = ctypes.c_size_t(0)
        self._check(L.hofks_workspace_size(ctypes.byref(self.desc), ctypes.byref(size)),
                    "workspace_size", None)
        self.workspace_bytes = size.value
        self.workspace = torch.empty(size.value, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p(0)
        self._check(L.hofks_create(ctypes.byref(self.desc), ctypes.c_void_p(self.workspace.data_ptr()),
                                   size.value, ctypes.c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(h)), "create", None)
        self._h = h
        self.set_tau(tau)

    # ------------------------------------------------------------ plumbing
    def _check(self, st, what, h=-1):
        if st != 0:
            msg = ""
            hh = self._h if h == -1 else h
            if hh:
                msg = _lib.lib().hofks_last_error(hh).decode()
            raise HofksError(st, what, msg)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._destroy(h)
            self._h = None

    def __del__(self):
        self.close()

    # ------------------------------------------------------------ the ABI
    def set_tau(self, tau):
        self._check(_lib.lib().hofks_set_tau(self._h, float(tau)), "set_tau")

    def set_state_macro(self, rho, u, theta):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.nc)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.d, self.nc)
        theta = np.ascontiguousarray(theta, dtype=np.float64).reshape(self.nc)
        self._check(_lib.lib().hofks_set_state_macro(self._h, _dp(rho), _dp(u), _dp(theta)),
                    "set_state_macro")

    def set_state_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.nv, self.nc)
        self._check(_lib.lib().hofks_set_state_f(self._h, _dp(f), f.nbytes), "set_state_f")

    def step(self, n=1):
        self._check(_lib.lib().hofks_step(self._h, int(n)), "step")

    def sync(self):
        self._check(_lib.lib().hofks_sync(self._h), "sync")

    def read_moments(self):
        U = np.empty((self.nm, self.nc), dtype=np.float64)
        self._check(_lib.lib().hofks_read_moments(self._h, _dp(U)), "read_moments")
        return U

    def read_f(self):
        f = np.empty((self.nv, self.nc), dtype=np.float64)
        self._check(_lib.lib().hofks_read_f(self._h, _dp(f), f.nbytes), "read_f")
        return f

    def read_state(self):
        """host image of the state (bytes) to resume from with write_state"""
        n = ctypes.c_size_t(0)
        self._check(_lib.lib().hofks_state_bytes(self._h, ctypes.byref(n)), "state_bytes")
        buf = np.empty(n.value, dtype=np.uint8)
        self._check(_lib.lib().hofks_read_state(self._h, buf.ctypes.data_as(ctypes.c_void_p),
                                                buf.nbytes), "read_state")
        return buf

    def write_state(self, image):
        buf = np.ascontiguousarray(image, dtype=np.uint8)
        self._check(_lib.lib().hofks_write_state(self._h, buf.ctypes.data_as(ctypes.c_void_p),
                                                 buf.nbytes), "write_state")

    def counters(self):
        s, n = ctypes.c_int(0), ctypes.c_long(0)
        self._check(_lib.lib().hofks_read_counters(self._h, ctypes.byref(s), ctypes.byref(n)),
                    "read_counters")
        return s.value, n.value

    def tail_substeps(self):
        """Euler sub-steps run by the persistent tail since the state was set"""
        n = ctypes.c_long(0)
        self._check(_lib.lib().hofks_read_tail_substeps(self._h, ctypes.byref(n)),
                    "read_tail_substeps")
        return n.value

    def set_euler_launches(self, k):
        """single-sub-step Euler launches per step before the persistent tail
        (0: automatic)"""
        self._check(_lib.lib().hofks_set_euler_launches(self._h, int(k)), "set_euler_launches")

    def kernel_timing(self, enable=True, groups=(0, 1, 2, 3)):
        """(ms[4], launches[4]) of the Euler, kinetic, per-cell update and
        closure-network groups since the previous call; keeps recording
        the listed groups while ``enable``."""
        mask = sum(1 << int(g) for g in set(groups)) if enable else 0
        ms = np.zeros(4)
        cnt = (ctypes.c_int * 4)()
        self._check(_lib.lib().hofks_kernel_timing(self._h, mask, _dp(ms), cnt),
                    "kernel_timing")
        return ms, list(cnt)

    @property
    def dt(self):
        return _lib.lib().hofks_dt(self._h)

    def set_launch_config(self, wavefronts, loads, euler_before):
        """a launch configuration without timing (see hofks_set_launch_config)"""
        self._check(_lib.lib().hofks_set_launch_config(self._h, int(wavefronts), int(loads),
                                                       int(euler_before)), "set_launch_config")

    def autotune(self, steps=4, cache_path=None):
        """time the candidate launch configurations (advances the state: set
        it again afterwards); returns the chosen (wavefronts, loads ahead,
        Euler solve before the kinetic kernel) for a grid, (cells per item,
        cells per Euler part, 0) for a batch"""
        ch = (ctypes.c_int * 3)()
        cp = cache_path.encode() if cache_path else None
        self._check(_lib.lib().hofks_autotune(self._h, int(steps), cp, ch), "autotune")
        return int(ch[0]), int(ch[1]), int(ch[2])

    # ------------------------------------------------ closure form (2D-2V)
    def closure_enable(self, net, threshold=1e-3):
        """run the following steps in the closure form with ``net`` (a
        ``ClosureNet``; its packed weights must stay alive)"""
        self._net = net
        self._check(_lib.lib().hofks_closure_enable(
            self._h, ctypes.c_void_p(net.packed.data_ptr()), float(net.sigma), float(threshold)),
            "closure_enable")

    def closure_disable(self):
        self._check(_lib.lib().hofks_closure_disable(self._h), "closure_disable")
        self._net = None

    def closure_snapshot(self):
        """one plain step; returns the network inputs of U^n and the targets
        N / (lambda s) as FP32 device tensors (nc x 37, nc x 4)"""
        x = torch.empty((self.nc, 37), dtype=torch.float32, device="cuda")
        t = torch.empty((self.nc, 4), dtype=torch.float32, device="cuda")
        self._check(_lib.lib().hofks_closure_snapshot(
            self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr())),
            "closure_snapshot")
        return x, t

    def closure_stats(self):
        """(closure steps, kinetic cell-steps among them)"""
        s, k = ctypes.c_long(0), ctypes.c_ulonglong(0)
        self._check(_lib.lib().hofks_closure_stats(self._h, ctypes.byref(s), ctypes.byref(k)),
                    "closure_stats")
        return s.value, k.value


class Batch(Solver):
    """Independent 1D-1V outflow tubes in FP32 pieces, advanced together (an
    Euler launch beside a kinetic launch, then an update launch, per step;
    replayed from a captured graph).

    ``tubes``: sequence of (n_cells, dx, n_vel, dv, tau).  Host arrays are
    concatenated over tubes (see include/hofks.h)."""

    def __init__(self, tubes, stream=None):
        L = _lib.lib()
        # held here so that close() still works while the interpreter tears
        # down module globals
        self._destroy = L.hofks_destroy
        if not torch.cuda.is_available():
            raise RuntimeError("the HOFKS library needs a ROCm GPU")
        n = len(tubes)
        descs = (_lib.GridDesc * n)()
        taus = np.empty(n)
        for i, (nx, dx, nv, dv, tau) in enumerate(tubes):
            descs[i] = _lib.GridDesc(1, (ctypes.c_int * 3)(nx, 1, 1), float(dx), int(nv), float(dv),
                                     (ctypes.c_int * 3)(1, 0, 0), 1, 0)
            taus[i] = tau
        self._descs, self.tubes = descs, list(tubes)
        self.d, self.nm = 1, 3
        self.nx = np.array([t[0] for t in tubes])
        self.nvs = np.array([t[2] for t in tubes])
        self.nc = int(self.nx.sum())
        self.ncv = int((self.nx * self.nvs).sum())
        self._h = None
        size = ctypes.c_size_t(0)
        self._check(L.hofks_batch_workspace_size(descs, n, ctypes.byref(size)),
                    "batch_workspace_size", None)
        self.workspace_bytes = size.value
        self.workspace = torch.empty(size.value, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p(0)
        self._check(L.hofks_batch_create(descs, _dp(taus), n,
                                         ctypes.c_void_p(self.workspace.data_ptr()), size.value,
                                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                    "batch_create", None)
        self._h = h

    def set_state_macro(self, rho, u, theta):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.nc)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.nc)
        theta = np.ascontiguousarray(theta, dtype=np.float64).reshape(self.nc)
        self._check(_lib.lib().hofks_set_state_macro(self._h, _dp(rho), _dp(u), _dp(theta)),
                    "set_state_macro")

    def read_moments(self):
        """list of (3, Nx_i) arrays"""
        U = np.empty(3 * self.nc, dtype=np.float64)
        self._check(_lib.lib().hofks_read_moments(self._h, _dp(U)), "read_moments")
        out, o = [], 0
        for nx in self.nx:
            out.append(U[o:o + 3 * nx].reshape(3, nx))
            o += 3 * nx
        return out

    def read_f(self):
        """list of (n_vel_i, Nx_i) arrays"""
        f = np.empty(self.ncv, dtype=np.float64)
        self._check(_lib.lib().hofks_read_f(self._h, _dp(f), f.nbytes), "read_f")
        out, o = [], 0
        for nx, nv in zip(self.nx, self.nvs):
            out.append(f[o:o + nx * nv].reshape(nv, nx))
            o += nx * nv
        return out

    def set_launch_config(self, cells, euler_part):
        """a batch launch configuration without timing (see
        hofks_batch_set_launch_config)"""
        self._check(_lib.lib().hofks_batch_set_launch_config(self._h, int(cells), int(euler_part)),
                    "batch_set_launch_config")

    def tube_flags(self):
        fl = (ctypes.c_int * len(self.tubes))()
        self._check(_lib.lib().hofks_batch_tube_flags(self._h, fl), "batch_tube_flags")
        return np.array(list(fl))
