"""Brute-force HOFKS in 50-digit arithmetic (mpmath), for tiny grids.

TEST INFRASTRUCTURE: a second, independent statement of what one step of the
scheme computes (arXiv:1212.0204, sections 3, 4.1, 4.2 and 4.3), used only to
pin the FP64 C oracle on grids of a few cells.  It shares no code with the
oracle or the GPU library: every quantity is formed here from the paper's
definitions with the readings listed in the design notes (lattice
k in {-n/2 .. n/2-1}, w = dv^d, energy row |v|^2/2, gamma = (d+2)/d,
U_E = (1 - lambda) Euler_dt(U^n) with s = max(1, ceil(2 dt sum_a alpha_a / dx))
equal sub-steps, global Lax-Friedrichs speeds re-evaluated every sub-step,
zero-gradient outflow ghosts).

Where the oracle inverts C C^T once, this file solves the normal equations
(C C^T) y = r with mpmath's LU solver for every correction, and where the
oracle walks cells with index arithmetic, this file keeps cells and velocities
as tuples.
"""
import itertools

import mpmath as mp

mp.mp.dps = 50


def _velocity_tuples(d, nv):
    ks = [i - nv // 2 for i in range(nv)]
    # x-fastest order (k = (iz n + iy) n + ix), like the arrays compared
    out = []
    for idx in itertools.product(range(nv), repeat=d):
        out.append(tuple(ks[i] for i in reversed(idx)))
    return out


def _cell_tuples(n):
    d = len(n)
    out = []
    for idx in itertools.product(*[range(m) for m in reversed(n)]):
        out.append(tuple(reversed(idx)))
    return out


def _cell_average_quadratic(offsets):
    """coefficients (a, b, c) of p(xi) = a + b xi + c xi^2 as linear maps of
    the cell averages of p over the cells at `offsets` (xi in cell widths,
    cell m = [m - 1/2, m + 1/2]): the 3 x 3 inverse of the averaging map"""
    A = mp.matrix(3, 3)
    for row, m in enumerate(offsets):
        A[row, 0] = 1
        A[row, 1] = mp.mpf(m)
        A[row, 2] = mp.mpf(m) ** 2 + mp.mpf(1) / 12
    return A ** -1


def _reconstruction_at(xi, offsets):
    """row vector giving p(xi) from the averages of a polynomial of degree
    len(offsets) - 1 over the cells at `offsets`"""
    k = len(offsets)
    A = mp.matrix(k, k)
    for row, m in enumerate(offsets):
        for pw in range(k):
            # average of xi^pw over [m - 1/2, m + 1/2]
            A[row, pw] = ((m + mp.mpf(1) / 2) ** (pw + 1) - (m - mp.mpf(1) / 2) ** (pw + 1)) / (pw + 1)
    Ainv = A ** -1
    return [sum(xi ** pw * Ainv[pw, col] for pw in range(k)) for col in range(k)]


class Weno5:
    """fifth-order WENO (Jiang and Shu) from its definitions: three quadratic
    candidates matching cell averages on the stencils {-2..0}, {-1..1},
    {0..2} around a cell, linear weights that recombine them into the quartic
    through all five averages, and smoothness indicators
    sum_l int (d^l p / dxi^l)^2 over the cell (l = 1, 2), eps = 1e-6"""

    STENCILS = [(-2, -1, 0), (-1, 0, 1), (0, 1, 2)]

    def __init__(self):
        self.eps = mp.mpf("1e-6")
        self.coef = [_cell_average_quadratic(st) for st in self.STENCILS]
        self.cand = {}
        self.lin = {}
        for side in (1, -1):
            xi = mp.mpf(side) / 2
            rows = [_reconstruction_at(xi, st) for st in self.STENCILS]
            big = _reconstruction_at(xi, (-2, -1, 0, 1, 2))
            # d with sum_r d_r rows_r == big on the five cells (the first,
            # third and fifth columns determine d; the others must agree)
            M = mp.matrix(5, 3)
            for r, st in enumerate(self.STENCILS):
                for c, m in enumerate(st):
                    M[m + 2, r] = rows[r][c]
            Msub = mp.matrix(3, 3)
            for i, row in enumerate((0, 2, 4)):
                for c in range(3):
                    Msub[i, c] = M[row, c]
            d = mp.lu_solve(Msub, mp.matrix([big[0], big[2], big[4]]))
            assert max(abs((M * d)[i] - big[i]) for i in range(5)) < mp.mpf("1e-40")
            self.cand[side] = rows
            self.lin[side] = [d[i] for i in range(3)]

    def face(self, v, side):
        """value at the face (side +1: right, -1: left) of the middle cell of
        v = averages of cells -2..2"""
        q, w = [], []
        for r, st in enumerate(self.STENCILS):
            vals = [v[m + 2] for m in st]
            q.append(sum(c * x for c, x in zip(self.cand[side][r], vals)))
            ab = self.coef[r] * mp.matrix(vals)
            b, c = ab[1], ab[2]
            beta = b * b + c * c / 3 + 4 * c * c  # int p'^2 + int p''^2 over the cell
            w.append(self.lin[side][r] / (self.eps + beta) ** 2)
        return sum(wi * qi for wi, qi in zip(w, q)) / sum(w)


class Brute:
    """scheme 0 HOFKS, 1 FKS (U_E := U_M), 2 HOFKS with phi == 1, 3 HOFKS
    with the WENO Euler solve (three-stage SSP Runge-Kutta, CFL 0.4)"""

    def __init__(self, d, n, dx, nv, dv, bc, tau, scheme=0, dt=None, strang=False):
        self.d, self.n, self.bc, self.scheme = d, tuple(n), tuple(bc), scheme
        self.dx, self.dv = mp.mpf(dx), mp.mpf(dv)
        self.dt = self.dx / self.dv  # lattice: v_k dt = k dx
        # off-lattice (section 4.2): a free dt; the pieces of f_k move by
        # v_k dt per step and the centre x_j lies, after n steps, in the piece
        # whose cell [x_p - dx/2, x_p + dx/2) contains x_j - v_k n dt
        self.offl = dt is not None
        if self.offl:
            self.dt = mp.mpf(dt)
        self.nstep = 0
        self.K = _velocity_tuples(d, nv)
        self.V = [tuple(k * self.dv for k in kk) for kk in self.K]
        self.cells = _cell_tuples(n)
        self.w = self.dv ** d
        self.gam = mp.mpf(d + 2) / d
        # rows of C: w (1, v, |v|^2/2)
        self.m = [[mp.mpf(1)] + list(v) + [sum(c * c for c in v) / 2] for v in self.V]
        nm = d + 2
        self.CCt = mp.matrix(nm, nm)
        for r in range(nm):
            for s in range(nm):
                self.CCt[r, s] = sum(self.w * mk[r] * self.w * mk[s] for mk in self.m)
        self.set_tau(tau)
        self.f = None
        self.U = None
        self.weno = Weno5() if scheme == 3 else None
        # Strang splitting R_{dt/2} T R_{dt/2}: the state kept here is the
        # synchronised f (after the second half relaxation)
        self.strang = strang

    # --------------------------------------------------------------- set-up
    def set_tau(self, tau):
        self.tau = tau
        if tau == float("inf"):
            self.lam, self.mu = mp.mpf(1), mp.mpf(0)
        elif tau == 0:
            self.lam, self.mu = mp.mpf(0), mp.mpf(1)
        else:
            self.lam = mp.exp(-self.dt / mp.mpf(tau))
            self.mu = 1 - self.lam

    def half_relax(self):
        """R_{dt/2} of the whole grid: f <- l f + (1 - l) E[U], l = exp(-dt/(2 tau));
        U is unchanged (C E[U] = U)"""
        if self.tau == float("inf"):
            return
        l = mp.mpf(0) if self.tau == 0 else mp.exp(-self.dt / (2 * mp.mpf(self.tau)))
        for j, U in enumerate(self.U):
            E = self.equilibrium(U)
            self.f[j] = [l * fk + (1 - l) * ek for fk, ek in zip(self.f[j], E)]

    def moments(self, g):
        nm = self.d + 2
        return [sum(self.w * mk[r] * gk for mk, gk in zip(self.m, g)) for r in range(nm)]

    def prim(self, U):
        d = self.d
        rho = U[0]
        u = [U[1 + a] / rho for a in range(d)]
        th = (2 * U[d + 1] - rho * sum(c * c for c in u)) / (d * rho)
        if not (rho > 0 and th > 0):
            raise ValueError("non-physical state")
        return rho, u, th

    def equilibrium(self, U):
        """eq. (minimMax): M + C^T y with (C C^T) y = U - C M"""
        rho, u, th = self.prim(U)
        M = [rho / (2 * mp.pi * th) ** (mp.mpf(self.d) / 2) *
             mp.exp(-sum((vi - ui) ** 2 for vi, ui in zip(v, u)) / (2 * th)) for v in self.V]
        CM = self.moments(M)
        y = mp.lu_solve(self.CCt, mp.matrix([U[r] - CM[r] for r in range(self.d + 2)]))
        return [Mk + sum(self.w * mk[r] * y[r] for r in range(self.d + 2))
                for Mk, mk in zip(M, self.m)]

    def init_macro(self, rho, u, theta):
        d = self.d
        self.nstep = 0
        self.U, self.f = [], []
        for j in range(len(self.cells)):
            r = mp.mpf(float(rho[j]))
            uu = [mp.mpf(float(u[a][j])) for a in range(d)]
            th = mp.mpf(float(theta[j]))
            U = [r] + [r * c for c in uu] + [r * sum(c * c for c in uu) / 2 + d * r * th / 2]
            self.U.append(U)
            self.f.append(self.equilibrium(U))

    def _piece(self, k, n):
        """cells between x_j and the piece holding it after n steps"""
        if not self.offl:
            return k * n
        y = mp.mpf(1) / 2 - k * self.dv * n * self.dt / self.dx  # (x_j - v_k n dt)/dx - j + 1/2
        return -int(mp.floor(y))

    def set_f(self, f):
        """f[k][j] (velocity-plane major); U = P(f)"""
        self.nstep = 0
        self.f = [[mp.mpf(float(f[k][j])) for k in range(len(self.K))]
                  for j in range(len(self.cells))]
        self.U = [self.moments(fj) for fj in self.f]

    # --------------------------------------------------------- neighbours
    def _wrap(self, a, i):
        N = self.n[a]
        if self.bc[a] == 0:
            return i % N
        return min(max(i, 0), N - 1)

    def _index(self, c):
        return self.cells.index(tuple(c))

    def _shifted(self, cell, a, off):
        c = list(cell)
        c[a] = self._wrap(a, c[a] + off)
        return self._index(c)

    # ----------------------------------------------------------- Euler
    def flux(self, U, a):
        rho, u, th = self.prim(U)
        p = rho * th
        F = [U[1 + a]] + [U[1 + b] * u[a] + (p if a == b else 0) for b in range(self.d)]
        F.append((U[self.d + 1] + p) * u[a])
        return F, abs(u[a]) + mp.sqrt(self.gam * p / rho)

    def speeds(self, Us):
        return [max(self.flux(U, a)[1] for U in Us) for a in range(self.d)]

    @staticmethod
    def phi(chi):
        # Van Leer limiter of section 4.3.2; zero numerator for chi <= 0
        if chi <= 0:
            return mp.mpf(0)
        return (abs(chi) + chi) / (1 + chi)

    def sigma(self, Wm1, W0, Wp1):
        """sigma_j = (W_{j+1} - W_j) phi(chi_j), chi_j = (W_j - W_{j-1})/(W_{j+1} - W_j)"""
        den = Wp1 - W0
        if self.scheme == 2:
            return den
        if den == 0:
            return mp.mpf(0)
        return den * self.phi((W0 - Wm1) / den)

    def face_flux(self, Us, cell, a, alpha, side):
        """psi of the face of `cell` on `side` (+1 right, -1 left) along axis a;
        its four stencil cells are taken relative to `cell` and each mapped
        onto the grid (periodic wrap, or the outflow ghost = boundary cell)"""
        nm = self.d + 2
        offs = (-1, 0, 1, 2) if side > 0 else (-2, -1, 0, 1)
        idx = [self._shifted(cell, a, o) for o in offs]
        F = [self.flux(Us[i], a)[0] for i in idx]
        Wp = [[F[q][r] + alpha * Us[idx[q]][r] for r in range(nm)] for q in range(4)]
        Wm = [[F[q][r] - alpha * Us[idx[q]][r] for r in range(nm)] for q in range(4)]
        psi = []
        for r in range(nm):
            sp = self.sigma(Wp[0][r], Wp[1][r], Wp[2][r])   # sigma^+ of the left cell
            sm = self.sigma(Wm[1][r], Wm[2][r], Wm[3][r])   # sigma^- of the right cell
            psi.append((F[1][r] + F[2][r]) / 2 - alpha * (Us[idx[2]][r] - Us[idx[1]][r]) / 2 +
                       (sp - sm) / 4)
        return psi

    def weno_rhs(self, Us, alpha):
        """L(U) = -(1/dx) sum_a (fh_{j+1/2} - fh_{j-1/2}); fh = WENO value of
        (F + alpha U)/2 from the left of the face + WENO value of
        (F - alpha U)/2 from the right of the face"""
        nm = self.d + 2
        out = []
        for cell in self.cells:
            div = [mp.mpf(0)] * nm
            for a in range(self.d):
                idx = {o: self._shifted(cell, a, o) for o in range(-3, 4)}
                F = {o: self.flux(Us[i], a)[0] for o, i in idx.items()}
                for r in range(nm):
                    fp = {o: (F[o][r] + alpha[a] * Us[idx[o]][r]) / 2 for o in idx}
                    fm = {o: (F[o][r] - alpha[a] * Us[idx[o]][r]) / 2 for o in idx}
                    right = self.weno.face([fp[o] for o in range(-2, 3)], 1) + \
                        self.weno.face([fm[o] for o in range(-1, 4)], -1)
                    left = self.weno.face([fp[o] for o in range(-3, 2)], 1) + \
                        self.weno.face([fm[o] for o in range(-2, 3)], -1)
                    div[r] += right - left
            out.append([-x / self.dx for x in div])
        return out

    def euler(self, Us, dt):
        if self.scheme == 3:
            return self.euler_weno(Us, dt)
        return self.euler_muscl(Us, dt)

    def euler_weno(self, Us, dt):
        """s = max(1, ceil(dt sum alpha / (0.4 dx))) sub-steps, each by the
        Shu-Osher three-stage SSP Runge-Kutta method with the speeds of the
        sub-step's initial state"""
        alpha = self.speeds(Us)
        s = max(1, int(mp.ceil(dt * sum(alpha) / (mp.mpf(2) / 5 * self.dx))))
        h = dt / s
        nm = self.d + 2
        for it in range(s):
            if it:
                alpha = self.speeds(Us)
            L0 = self.weno_rhs(Us, alpha)
            U1 = [[u[r] + h * l[r] for r in range(nm)] for u, l in zip(Us, L0)]
            L1 = self.weno_rhs(U1, alpha)
            U2 = [[(3 * u[r] + u1[r] + h * l[r]) / 4 for r in range(nm)] for u, u1, l in zip(Us, U1, L1)]
            L2 = self.weno_rhs(U2, alpha)
            Us = [[(u[r] + 2 * (u2[r] + h * l[r])) / 3 for r in range(nm)] for u, u2, l in zip(Us, U2, L2)]
        return Us, s

    def euler_muscl(self, Us, dt):
        """eq. (discmom) over dt in s equal sub-steps"""
        alpha = self.speeds(Us)
        s = max(1, int(mp.ceil(2 * dt * sum(alpha) / self.dx)))
        h = dt / s
        for it in range(s):
            if it:
                alpha = self.speeds(Us)
            new = []
            for j, cell in enumerate(self.cells):
                div = [mp.mpf(0)] * (self.d + 2)
                for a in range(self.d):
                    right = self.face_flux(Us, cell, a, alpha[a], +1)
                    left = self.face_flux(Us, cell, a, alpha[a], -1)
                    div = [dv + rr - ll for dv, rr, ll in zip(div, right, left)]
                new.append([Us[j][r] - h / self.dx * div[r] for r in range(self.d + 2)])
            Us = new
        return Us, s

    # ------------------------------------------------------------ one step
    def step(self, nsteps=1):
        for _ in range(nsteps):
            if self.strang and self.scheme == 1:
                # FKS: R_{dt/2}, transport, R_{dt/2} applied literally
                self.half_relax()
                saved = (self.lam, self.mu)
                self.lam, self.mu = mp.mpf(1), mp.mpf(0)
                self._step()
                self.lam, self.mu = saved
                self.half_relax()
            elif self.strang:
                # HOFKS: the two half relaxations between transports act as
                # one full relaxation R_dt, whose equilibrium part the Euler
                # solve advances; the first step has only the half after the
                # initial data, and the last half is applied on reading f
                saved = (self.lam, self.mu)
                if self.nstep == 0 and self.tau != float("inf"):
                    self.lam = mp.mpf(0) if self.tau == 0 else \
                        mp.exp(-self.dt / (2 * mp.mpf(self.tau)))
                    self.mu = 1 - self.lam
                self._step()
                self.lam, self.mu = saved
            else:
                self._step()

    def f_synchronised(self):
        """f at t^n: for the merged Strang form, the pending R_{dt/2}"""
        if not (self.strang and self.scheme != 1 and self.nstep > 0):
            return self.f
        keep = [list(fj) for fj in self.f]
        self.half_relax()
        out, self.f = self.f, keep
        return out

    def _step(self):
        lam, mu, d = self.lam, self.mu, self.d
        ncell = len(self.cells)
        E = [self.equilibrium(U) for U in self.U] if lam != 1 else None
        fK = [[None] * len(self.K) for _ in range(ncell)]
        Ustar, UM = [], []
        n = self.nstep
        self.nstep += 1
        for j, cell in enumerate(self.cells):
            fs_parts, e_parts = [], []
            for q, kk in enumerate(self.K):
                sh = [self._piece(kk[a], n + 1) - self._piece(kk[a], n) for a in range(d)]
                src = self._index([self._wrap(a, cell[a] - sh[a]) for a in range(d)])
                fn = self.f[src][q]
                if lam == 1:
                    fK[j][q] = fn
                    e_parts.append(mp.mpf(0))
                else:
                    Es = E[src][q]
                    fK[j][q] = Es if lam == 0 else lam * fn + mu * Es
                    e_parts.append(mu * Es)
                fs_parts.append(lam * fn)
            Ustar.append(self.moments(fs_parts))
            UM.append(self.moments(e_parts))
        if lam == 1:
            UE = [[mp.mpf(0)] * (d + 2) for _ in range(ncell)]
        elif self.scheme == 1:
            UE = [list(u) for u in UM]
        else:
            Ue, _ = self.euler([list(u) for u in self.U], self.dt)
            UE = [[mu * x for x in u] for u in Ue]
        newf = []
        for j in range(ncell):
            if lam != 1 and self.scheme != 1:
                y = mp.lu_solve(self.CCt, mp.matrix([UE[j][r] - UM[j][r] for r in range(d + 2)]))
                newf.append([fK[j][q] + sum(self.w * self.m[q][r] * y[r] for r in range(d + 2))
                             for q in range(len(self.K))])
            else:
                newf.append(fK[j])
        self.f = newf
        self.U = [[Ustar[j][r] + UE[j][r] for r in range(d + 2)] for j in range(ncell)]

    # ------------------------------------------------------------- read-out
    def U_array(self):
        return [[float(self.U[j][r]) for j in range(len(self.cells))] for r in range(self.d + 2)]

    def f_array(self):
        f = self.f_synchronised()
        return [[float(f[j][q]) for j in range(len(self.cells))] for q in range(len(self.K))]
