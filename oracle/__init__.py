"""Plain FP64 CPU oracle of the HOFKS step (arXiv:1212.0204, section 4.3).

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It loads its own
shared object built from ``oracle/hofks_oracle.c`` (plain C, ``gcc -O2
-ffp-contract=off``) and shares nothing with the GPU library.

Layouts (see the C file's header): moments are component-major ``(d+2, Nc)``,
the distribution is velocity-plane major ``(Nv, Nc)``; cells and velocity
nodes are x-fastest.
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OK, EINVAL, ENONPHYS = 0, -1, -4


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"oracle {what}: status {status}")
        self.status = status


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libhofks_oracle.so")
        if not os.path.exists(path) or any(
                os.path.getmtime(path) < os.path.getmtime(src) for src in _build.SOURCES):
            _build.build()
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        d, i, vp = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        dp = P(ctypes.c_double)
        lib.or_create.restype = vp
        lib.or_create.argtypes = [i, P(i), d, i, d, P(i), i, d, d, i, P(i)]
        lib.or_nstep.argtypes = [vp]
        lib.or_nstep.restype = ctypes.c_long
        lib.or_destroy.argtypes = [vp]
        lib.or_set_tau.argtypes = [vp, d]
        lib.or_init_macro.argtypes = [vp, dp, dp, dp]
        lib.or_set_f.argtypes = [vp, dp]
        lib.or_step.argtypes = [vp, i]
        for name in ("or_get_U", "or_get_f", "or_get_delta", "or_get_A",
                     "or_get_velocities"):
            getattr(lib, name).argtypes = [vp, dp]
        lib.or_last_substeps.argtypes = [vp]
        lib.or_set_threads.argtypes = [i]
        lib.or_max_threads.restype = i
        lib.or_dt.argtypes = [vp]
        lib.or_dt.restype = d
        lib.or_lambda.argtypes = [vp]
        lib.or_lambda.restype = d
        lib.or_maxwellian.argtypes = [vp, dp, dp]
        lib.or_equilibrium.argtypes = [vp, dp, dp]
        lib.or_muscl.argtypes = [vp, dp, d, P(i)]
        lib.or_muscl_substep.argtypes = [vp, dp, d]
        lib.or_weno.argtypes = [vp, dp, d, P(i)]
        lib.mlp_nparam.restype = i
        lib.mlp_forward.argtypes = [dp, dp, dp, i]
        lib.mlp_loss_grad.argtypes = [dp, dp, dp, i, dp]
        lib.mlp_loss_grad.restype = d
        lib.mlp_adam.argtypes = [dp, dp, dp, dp, d, d, d, d, i]
        _LIB = lib
    return _LIB


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """One grid + velocity set + tau, stepped with the plain FP64 scheme.

    ``scheme``: 0 HOFKS (section 4.3), 1 FKS with the Euler coupling removed
    (U_E := U_M), 2 HOFKS with the Van Leer limiter replaced by phi == 1,
    3 HOFKS with the WENO Euler solve (section 4.3.3).
    ``bc`` per axis: 0 periodic, 1 outflow (zero gradient).
    ``dt``: None for the lattice dt = dx/dv; a smaller value for off-lattice
    transport (pieces at accumulated offsets v_k n dt, section 4.2).
    ``strang``: Strang splitting R_{dt/2} T_dt R_{dt/2} instead of the
    first-order relax-then-transport step; ``f`` is then read after the
    pending half relaxation.
    """

    def __init__(self, d, n, dx, nv, dv, bc=None, tau=math.inf, scheme=0, dt=None,
                 strang=False):
        n = (list(n) + [1, 1, 1])[:3]
        bc = (list(bc if bc is not None else [0] * 3) + [0, 0, 0])[:3]
        self.d, self.n, self.nv1, self.dx, self.dv = d, n[:d], nv, dx, dv
        self.nm = d + 2
        self.nc = int(np.prod(n[:d]))
        self.nv = nv ** d
        self.scheme = scheme
        st = ctypes.c_int(0)
        ia = (ctypes.c_int * 3)(*n)
        ba = (ctypes.c_int * 3)(*bc)
        self._h = _lib().or_create(d, ia, float(dx), nv, float(dv), ba,
                                   scheme, float(tau), float(dt or 0.0), int(bool(strang)),
                                   ctypes.byref(st))
        if not self._h:
            raise OracleError(st.value, "create")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib().or_destroy(h)
            self._h = None

    # -- set-up -----------------------------------------------------------
    def set_tau(self, tau):
        st = _lib().or_set_tau(self._h, float(tau))
        if st:
            raise OracleError(st, "set_tau")

    def init_macro(self, rho, u, theta):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.nc)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.d, self.nc)
        theta = np.ascontiguousarray(theta, dtype=np.float64).reshape(self.nc)
        st = _lib().or_init_macro(self._h, _dp(rho), _dp(u), _dp(theta))
        if st:
            raise OracleError(st, "init_macro")

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.nv, self.nc)
        _lib().or_set_f(self._h, _dp(f))

    # -- stepping ---------------------------------------------------------
    def step(self, n=1):
        st = _lib().or_step(self._h, int(n))
        if st:
            raise OracleError(st, "step")

    # -- read-out ---------------------------------------------------------
    def _get(self, name, shape):
        out = np.empty(shape, dtype=np.float64)
        getattr(_lib(), name)(self._h, _dp(out))
        return out

    @property
    def U(self):
        return self._get("or_get_U", (self.nm, self.nc))

    @property
    def f(self):
        return self._get("or_get_f", (self.nv, self.nc))

    @property
    def delta(self):
        return self._get("or_get_delta", (self.nm, self.nc))

    @property
    def A(self):
        return self._get("or_get_A", (self.nm, self.nm))

    @property
    def velocities(self):
        return self._get("or_get_velocities", (self.nv, self.d))

    @property
    def substeps(self):
        return _lib().or_last_substeps(self._h)

    @property
    def dt(self):
        return _lib().or_dt(self._h)

    @property
    def nstep(self):
        return _lib().or_nstep(self._h)

    @property
    def lam(self):
        return _lib().or_lambda(self._h)

    # -- standalone pieces ------------------------------------------------
    def maxwellian(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        M = np.empty(self.nv)
        st = _lib().or_maxwellian(self._h, _dp(U), _dp(M))
        if st:
            raise OracleError(st, "maxwellian")
        return M

    def equilibrium(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        E = np.empty(self.nv)
        st = _lib().or_equilibrium(self._h, _dp(U), _dp(E))
        if st:
            raise OracleError(st, "equilibrium")
        return E

    def muscl(self, U, dt):
        U = np.array(U, dtype=np.float64).reshape(self.nm, self.nc).copy()
        ns = ctypes.c_int(0)
        st = _lib().or_muscl(self._h, _dp(U), float(dt), ctypes.byref(ns))
        if st:
            raise OracleError(st, "muscl")
        return U, ns.value

    def weno(self, U, dt):
        """the WENO solve of scheme 3 over dt: (U after dt, sub-steps)"""
        U = np.array(U, dtype=np.float64).reshape(self.nm, self.nc).copy()
        ns = ctypes.c_int(0)
        st = _lib().or_weno(self._h, _dp(U), float(dt), ctypes.byref(ns))
        if st:
            raise OracleError(st, "weno")
        return U, ns.value

    def muscl_substep(self, U, h):
        """one sub-step of length h with the speeds of U (no sub-cycling)"""
        U = np.array(U, dtype=np.float64).reshape(self.nm, self.nc).copy()
        st = _lib().or_muscl_substep(self._h, _dp(U), float(h))
        if st:
            raise OracleError(st, "muscl_substep")
        return U


# ------------------------------------------------------ closure network (FP64)
MLP_NIN, MLP_NH, MLP_NOUT = 37, 64, 4


def mlp_nparam():
    return _lib().mlp_nparam()


def mlp_forward(params, x):
    """y = MLP(x) for x of shape (n, 37); FP64"""
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, MLP_NIN)
    y = np.empty((x.shape[0], MLP_NOUT))
    _lib().mlp_forward(_dp(p), _dp(x), _dp(y), x.shape[0])
    return y


def mlp_loss_grad(params, x, t):
    """(loss, gradient) of L = mean (y - t)^2 over samples and outputs"""
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, MLP_NIN)
    t = np.ascontiguousarray(t, dtype=np.float64).reshape(-1, MLP_NOUT)
    g = np.empty(mlp_nparam())
    loss = _lib().mlp_loss_grad(_dp(p), _dp(x), _dp(t), x.shape[0], _dp(g))
    return loss, g


def mlp_adam(params, grad, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """one Adam step in place on params, m, v (FP64 arrays)"""
    g = np.ascontiguousarray(grad, dtype=np.float64)
    _lib().mlp_adam(_dp(params), _dp(g), _dp(m), _dp(v), lr, b1, b2, eps, int(step))


def set_threads(n):
    """threads of the oracle's OpenMP loops"""
    _lib().or_set_threads(int(n))


def max_threads():
    return _lib().or_max_threads()
