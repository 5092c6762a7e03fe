/*
 * hofks_oracle.c -- plain, slow, FP64 CPU oracle of one HOFKS time step
 * (Dimarco & Loubere, "Towards an ultra efficient kinetic scheme. Part II:
 * the high order case", arXiv:1212.0204).
 *
 * TEST INFRASTRUCTURE.  This file is the checker of the GPU library, not part
 * of it.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load or call it; the product path never does.  It shares no
 * code, header, table or constant with the HIP library.
 *
 * What it computes, in the paper's order (section 4.3.1), for one step
 * t^n -> t^{n+1} given f^n on the grid and the carried moments U^n:
 *
 *   1. E^n = E[U^n] for every cell: the Maxwellian of eq. (M) corrected by the
 *      least-squares projection of eq. (minimMax), with the (d+2) x N matrix C
 *      of the discrete collision invariants m_k = (1, v_k, |v_k|^2/2) times the
 *      quadrature weight Delta v^d (eq. (DM)); C^T (C C^T)^{-1} is formed once
 *      (end of section 4.1).
 *   2. relaxation R_dt: f* = lambda f^n + (1 - lambda) E^n, lambda = exp(-dt/tau)
 *      (section 4.3.1, operator R).
 *   3. transport T_dt: exact shift of the piecewise-constant pieces,
 *      f_K(x_j, v_k) = f*(x_j - v_k dt).  On the lattice v_k dt = k dx used here
 *      this is the integer cell offset j - k (operator T).
 *   4. moments of the kinetic solution split as in eq. (UK):
 *      U_* = P(T(lambda f^n)),  U_M = P(T((1 - lambda) E^n)).
 *   5. U_E: the Euler system (eq. sys1) advanced over dt from U^n by the MUSCL
 *      flux-split scheme of section 4.3.2 (eq. discmom, Van Leer limiter),
 *      scaled by (1 - lambda) so that it replaces U_M.
 *   6. consistency correction (eq. minim_full, solved like eq. minimMax):
 *      f^{n+1} = f_K + C^T (C C^T)^{-1} (U_E - U_M),  U^{n+1} = U_* + U_E (eq. mom).
 *
 * Readings where the paper is silent or ambiguous (each also listed in the
 * design notes of the repository):
 *   - quadrature weight w = dv^d (eq. (DM) writes dv for d = 1);
 *   - velocity nodes v_k = k dv with k in {-n/2 .. n/2-1} per axis for even n,
 *     {-(n-1)/2 .. (n-1)/2} for odd n (so dt = dx/dv makes v_k dt = k dx);
 *   - theta from the energy, theta = (2E - rho|u|^2)/(d rho), eq. (E);
 *   - gamma = (d+2)/d, the closure of eq. (sys1);
 *   - U_E = (1 - lambda) MUSCL_dt(U^n): every step restarts the Euler solve
 *     from the carried moments U^n (Theorem 1 needs U_E(t) = U_M(t));
 *   - alpha = global Lax-Friedrichs speed per direction, max over cells of
 *     |u_a| + sqrt(gamma p / rho), re-evaluated at every sub-step;
 *   - the lattice fixes dt = dx/dv, above the MUSCL bound of eq. (Time2), so
 *     the Euler solve takes s = max(1, ceil(2 dt sum_a alpha_a / dx)) equal
 *     sub-steps of dt/s, s taken from the state at t^n;
 *   - Van Leer phi(chi) = (|chi|+chi)/(1+chi) is taken as 0 for chi <= 0 (its
 *     numerator vanishes there; this also covers the 0/0 at chi = -1), and
 *     sigma = 0 where the slope ratio's denominator is 0 (the limit of
 *     den * phi(num/den));
 *   - multi-D: unsplit sum of the directional fluxes;
 *   - boundaries: periodic wrap, or outflow = zero-gradient (the ghost value is
 *     the boundary cell's value, for the pieces and for the Euler ghosts);
 *   - lambda = 1 (tau = +inf) skips every E term, so free transport is an exact
 *     copy; lambda = 0 (tau = 0) skips every f^n term.
 *
 * Scheme 3 replaces the MUSCL solve by a WENO solve (section 4.3.3 names WENO
 * as a higher-order Euler solver for HOFKS; its details follow the standard
 * finite-difference form of Jiang and Shu): the same global Lax-Friedrichs
 * splitting F +- alpha U, the fifth-order WENO reconstruction of each split
 * flux at the faces (upwind-biased: left-biased for the + part, right-biased
 * for the - part, smoothness indicators with eps = 1e-6 and linear weights
 * 1/10, 6/10, 3/10), and the three-stage strong-stability-preserving
 * Runge-Kutta method of Shu and Osher in time.  Readings: the CFL number is
 * tighter than MUSCL's 1/2 (eq. (Time2) reduced, as the paper says a WENO
 * solver needs): s = max(1, ceil(dt sum_a alpha_a / (0.4 dx))) equal
 * sub-steps from the speeds of U^n; alpha is taken from each sub-step's
 * initial state and kept for its three stages; outflow ghosts (three per
 * side) copy the boundary cell.
 *
 * Off-lattice velocities (dt given, dt <= dx/dv): the transport of section
 * 4.2 moves every piecewise-constant function f_k by v_k dt per step with no
 * reconstruction, so after n steps the discontinuities of f_k sit at
 * x_{p-1/2} + v_k n dt and the cell centre x_j lies in the piece that started
 * in cell j - o_k(n), o_k(n) = ceil(c_k n - 1/2), c_k = v_k dt / dx (pieces
 * are the half-open cells [x_{p-1/2}, x_{p+1/2})).  The value at the centre
 * is what the relaxation and the moments see (section 4.2), so a step
 * t^n -> t^{n+1} reads the upstream cell j - (o_k(n+1) - o_k(n)) per axis:
 * an integer shift that is floor(c_k) or ceil(c_k) by step.  c_k n is formed
 * as ((k dv) dt / dx) * n, each operation rounded (no contraction).  With
 * dt = dx/dv this is the lattice shift k.
 *
 * Strang splitting (strang = 1; section 4.2 names it as the alternative to
 * the first-order splitting): a step is R_{dt/2} T_dt R_{dt/2} with the
 * HOFKS coupling on its transport.  A relaxation keeps the moments, so E is
 * the same for two consecutive half relaxations and R_{a} R_{b} = R_{a+b}:
 * n Strang steps are the first-order steps with the first relaxation weight
 * lambda = exp(-dt/(2 tau)) and a pending half relaxation R_{dt/2} of the
 * stored f, applied when f is read (the moments are unchanged by it).  With
 * a change of tau between steps the step after it relaxes by
 * exp(-dt/(2 tau_old)) exp(-dt/(2 tau_new)).  So the step n uses
 * lambda = exp(-e), e = dt/2 (1/tau_{n-1}) + dt/2 (1/tau_n), with the first
 * term absent at the first step (1/tau = 0 for tau = +inf, +inf for 0).
 *
 * Layouts: U and u are component-major, U[r*Nc + j]; f is velocity-plane major,
 * f[k*Nc + j]; cells are x-fastest, j = (jz*Ny + jy)*Nx + jx; velocities are
 * x-fastest, k = (iz*n + iy)*n + ix with k_a = i_a - n/2 (integer division).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENONPHYS (-4)

typedef struct or_state {
  int d, nm;            /* space = velocity dimension, nm = d + 2 moments   */
  int n[3];             /* cells per axis (unused axes 1)                   */
  int nc;               /* number of cells                                   */
  double dx, dv, dt, w; /* cell size, velocity step, time step, dv^d         */
  int nv1, nv;          /* nodes per velocity axis, total velocity nodes     */
  int bc[3];            /* 0 periodic, 1 outflow                             */
  int scheme;           /* 0 HOFKS, 1 FKS (U_E := U_M), 2 HOFKS unlimited,
                           3 HOFKS with the WENO Euler solve                 */
  double tau, lam, mu;  /* relaxation time, exp(-dt/tau), 1 - exp(-dt/tau)   */
  int offl;             /* 1: dt given (off-lattice transport), 0: dt = dx/dv */
  int strang;           /* 1: Strang splitting, 0: first order (relax, shift) */
  double inv_prev;      /* 1/tau of the previous step (Strang)                */
  long nstep;           /* steps taken since the initial data (off-lattice)  */
  double *cvel;         /* nv1: c = v dt / dx per node of one axis            */
  int *shift;           /* nv1: cells moved by the current step, per node     */
  int *kint;            /* nv x d integer velocity indices k_a               */
  double *m;            /* nv x nm collision invariants m_k                  */
  double A[25];         /* (C C^T)^{-1}, nm x nm                             */
  double *f, *fnew, *E; /* nv x nc                                           */
  double *U;            /* nm x nc                                           */
  double *delta;        /* nm x nc, U_E - U_M of the last step               */
  int last_substeps;
} or_state;

/* ---------------------------------------------------------------- helpers */

static int cell_index(const or_state *S, const int *c) {
  return (c[2] * S->n[1] + c[1]) * S->n[0] + c[0];
}

static void cell_coords(const or_state *S, int j, int *c) {
  c[0] = j % S->n[0];
  c[1] = (j / S->n[0]) % S->n[1];
  c[2] = j / (S->n[0] * S->n[1]);
}

/* map a possibly out-of-range coordinate on axis a onto a real cell:
 * periodic wrap or zero-gradient clamp (the ghost takes the boundary value) */
static int map_axis(const or_state *S, int a, int i) {
  int N = S->n[a];
  if (S->bc[a] == 0) {
    i %= N;
    if (i < 0) i += N;
    return i;
  }
  if (i < 0) return 0;
  if (i >= N) return N - 1;
  return i;
}

/* cell that the piece of velocity k arriving in cell j came from: x_j - v_k dt
 * = x_{j-k} on the lattice v_k dt = k dx */
static int upstream(const or_state *S, int j, int k) {
  int c[3], s[3];
  cell_coords(S, j, c);
  for (int a = 0; a < 3; ++a) {
    int ka = (a < S->d) ? S->kint[k * S->d + a] : 0;
    if (S->offl && a < S->d) ka = S->shift[ka + S->nv1 / 2];
    s[a] = map_axis(S, a, c[a] - ka);
  }
  return cell_index(S, s);
}

/* neighbour of cell j at offset off along axis a (with the boundary map) */
static int neighbour(const or_state *S, int j, int a, int off) {
  int c[3];
  cell_coords(S, j, c);
  c[a] = map_axis(S, a, c[a] + off);
  return cell_index(S, c);
}

/* plain Gauss-Jordan inverse with partial pivoting of an n x n matrix */
static int invert(int n, const double *Min, double *Minv) {
  double a[5][10];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j)
      a[i][j] = (j < n) ? Min[i * n + j] : (j - n == i ? 1.0 : 0.0);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int i = col + 1; i < n; ++i)
      if (fabs(a[i][col]) > fabs(a[piv][col])) piv = i;
    if (a[piv][col] == 0.0) return OR_EINVAL;
    if (piv != col)
      for (int j = 0; j < 2 * n; ++j) {
        double t = a[col][j];
        a[col][j] = a[piv][j];
        a[piv][j] = t;
      }
    double p = a[col][col];
    for (int j = 0; j < 2 * n; ++j) a[col][j] /= p;
    for (int i = 0; i < n; ++i) {
      if (i == col) continue;
      double fct = a[i][col];
      if (fct == 0.0) continue;
      for (int j = 0; j < 2 * n; ++j) a[i][j] -= fct * a[col][j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Minv[i * n + j] = a[i][j + n];
  return OR_OK;
}

/* ------------------------------------------------- section 3: DVM, moments */

/* primitive variables of a moment vector, eq. (Mo)-(E) with R5 */
static int primitives(const or_state *S, const double *U, double *rho,
                      double *u, double *theta) {
  int d = S->d;
  double r = U[0], usq = 0.0;
  for (int a = 0; a < d; ++a) {
    u[a] = U[1 + a] / r;
    usq += u[a] * u[a];
  }
  double th = (2.0 * U[d + 1] - r * usq) / (d * r);
  *rho = r;
  *theta = th;
  if (!(r > 0.0) || !(th > 0.0) || !isfinite(r) || !isfinite(th))
    return OR_ENONPHYS;
  for (int a = 0; a < d; ++a)
    if (!isfinite(u[a])) return OR_ENONPHYS;
  return OR_OK;
}

/* Maxwellian of eq. (M) sampled on the velocity nodes */
static int maxwellian(const or_state *S, const double *U, double *M) {
  double rho, u[3], th;
  int st = primitives(S, U, &rho, u, &th);
  if (st) return st;
  double pref = rho / pow(2.0 * M_PI * th, 0.5 * S->d);
  for (int k = 0; k < S->nv; ++k) {
    double q = 0.0;
    for (int a = 0; a < S->d; ++a) {
      double dvel = u[a] - S->m[k * S->nm + 1 + a];
      q += dvel * dvel;
    }
    M[k] = pref * exp(-q / (2.0 * th));
  }
  return OR_OK;
}

/* conservative Maxwellian of eq. (minimMax):
 *   E = M + C^T (C C^T)^{-1} (U - C M),  (C g)_r = sum_k w m_k[r] g_k */
static int equilibrium(const or_state *S, const double *U, double *E) {
  int nm = S->nm, st = maxwellian(S, U, E);
  if (st) return st;
  double CM[5] = {0, 0, 0, 0, 0}, c[5];
  for (int k = 0; k < S->nv; ++k)
    for (int r = 0; r < nm; ++r) CM[r] += S->w * S->m[k * nm + r] * E[k];
  for (int r = 0; r < nm; ++r) {
    c[r] = 0.0;
    for (int s = 0; s < nm; ++s) c[r] += S->A[r * nm + s] * (U[s] - CM[s]);
  }
  for (int k = 0; k < S->nv; ++k) {
    double corr = 0.0;
    for (int r = 0; r < nm; ++r) corr += S->w * S->m[k * nm + r] * c[r];
    E[k] += corr;
  }
  return OR_OK;
}

/* ------------------------------------- section 4.3.2: MUSCL for eq. (sys1) */

/* Euler flux along axis a, eq. (sys1) with p = rho theta, gamma = (d+2)/d */
static int euler_flux(const or_state *S, const double *U, int a, double *F,
                      double *speed) {
  double rho, u[3], th;
  int st = primitives(S, U, &rho, u, &th);
  if (st) return st;
  int d = S->d;
  double p = rho * th;
  double gam = (d + 2.0) / d;
  F[0] = U[1 + a];
  for (int b = 0; b < d; ++b) F[1 + b] = U[1 + b] * u[a] + (a == b ? p : 0.0);
  F[d + 1] = (U[d + 1] + p) * u[a];
  if (speed) *speed = fabs(u[a]) + sqrt(gam * p / rho);
  return OR_OK;
}

/* Van Leer limited slope sigma = den * phi(num / den) (section 4.3.2) */
static double limited_slope(double num, double den, int unlimited) {
  if (unlimited) return den; /* phi == 1 */
  if (den == 0.0) return 0.0;
  double chi = num / den;
  if (!(chi > 0.0)) return 0.0;
  double phi = (fabs(chi) + chi) / (1.0 + chi);
  return den * phi;
}

/* alpha_a = max over the cells of |u_a| + c (global Lax-Friedrichs speed) */
static int lf_speeds(const or_state *S, const double *U, double *alpha) {
  int nm = S->nm, nc = S->nc;
  for (int a = 0; a < S->d; ++a) alpha[a] = 0.0;
  double Uj[5], F[5];
  for (int j = 0; j < nc; ++j) {
    for (int r = 0; r < nm; ++r) Uj[r] = U[r * nc + j];
    for (int a = 0; a < S->d; ++a) {
      double sp;
      int st = euler_flux(S, Uj, a, F, &sp);
      if (st) return st;
      if (sp > alpha[a]) alpha[a] = sp;
    }
  }
  return OR_OK;
}

/* numerical flux psi through the face between cells j+base and j+base+1
 * along axis a (base = 0: face j+1/2, base = -1: face j-1/2); the stencil is
 * j+base-1 .. j+base+2, with out-of-range cells mapped by the boundary rule */
static int muscl_flux(const or_state *S, const double *U, int j, int a,
                      int base, double alpha, double *psi) {
  int nm = S->nm, nc = S->nc;
  double Us[4][5], Fs[4][5];
  for (int q = 0; q < 4; ++q) {
    int idx = neighbour(S, j, a, base - 1 + q);
    for (int r = 0; r < nm; ++r) Us[q][r] = U[r * nc + idx];
    int st = euler_flux(S, Us[q], a, Fs[q], NULL);
    if (st) return st;
  }
  int unl = (S->scheme == 2);
  for (int r = 0; r < nm; ++r) {
    /* W^{+-} = F +- alpha U at the four stencil cells */
    double Wp[4], Wm[4];
    for (int q = 0; q < 4; ++q) {
      Wp[q] = Fs[q][r] + alpha * Us[q][r];
      Wm[q] = Fs[q][r] - alpha * Us[q][r];
    }
    /* sigma^+ of the left cell from (q0, q1, q2); sigma^- of the right cell
     * from (q1, q2, q3) */
    double sp = limited_slope(Wp[1] - Wp[0], Wp[2] - Wp[1], unl);
    double sm = limited_slope(Wm[2] - Wm[1], Wm[3] - Wm[2], unl);
    psi[r] = 0.5 * (Fs[1][r] + Fs[2][r]) - 0.5 * alpha * (Us[2][r] - Us[1][r]) +
             0.25 * (sp - sm);
  }
  return OR_OK;
}

/* one forward-Euler sub-step of eq. (discmom) of length dts with the speeds
 * alpha; U (nm x nc) is read, Unew written */
static int muscl_substep(const or_state *S, const double *U, double *Unew,
                         const double *alpha, double dts) {
  int nm = S->nm, nc = S->nc, d = S->d, st = OR_OK;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < nc; ++j) {
    double div[5] = {0, 0, 0, 0, 0}, pr[5], pl[5];
    for (int a = 0; a < d; ++a) {
      int l1 = muscl_flux(S, U, j, a, 0, alpha[a], pr);
      int l2 = muscl_flux(S, U, j, a, -1, alpha[a], pl);
      if (l1 || l2) {
#pragma omp atomic write
        st = OR_ENONPHYS;
      }
      for (int r = 0; r < nm; ++r) div[r] += pr[r] - pl[r];
    }
    for (int r = 0; r < nm; ++r)
      Unew[r * nc + j] = U[r * nc + j] - dts / S->dx * div[r];
  }
  return st;
}

/* eq. (discmom) applied with s sub-steps over dt; U is nm x nc, updated */
static int muscl_solve(const or_state *S, double *U, double dt, int *nsub) {
  int nm = S->nm, nc = S->nc, d = S->d;
  double alpha[3];
  int st = lf_speeds(S, U, alpha);
  if (st) return st;
  double sum = 0.0;
  for (int a = 0; a < d; ++a) sum += alpha[a];
  int s = (int)ceil(2.0 * dt * sum / S->dx);
  if (s < 1) s = 1;
  if (nsub) *nsub = s;
  double dts = dt / s;
  double *Unew = (double *)malloc(sizeof(double) * nm * nc);
  if (!Unew) return OR_EINVAL;
  for (int it = 0; it < s && st == OR_OK; ++it) {
    if (it > 0) st = lf_speeds(S, U, alpha);
    if (st) break;
    st = muscl_substep(S, U, Unew, alpha, dts);
    memcpy(U, Unew, sizeof(double) * nm * nc);
  }
  free(Unew);
  return st;
}

/* ------------------------------- section 4.3.3: a WENO solve of eq. (sys1) */

/* fifth-order WENO value at the face between v[2] and v[3] of the
 * upwind-biased stencil v[0..4] (cells i-2 .. i+2 for the face i+1/2):
 * three third-order candidates, weighted by their smoothness */
static double weno5(const double *v) {
  const double q0 = (2.0 * v[0] - 7.0 * v[1] + 11.0 * v[2]) / 6.0;
  const double q1 = (-v[1] + 5.0 * v[2] + 2.0 * v[3]) / 6.0;
  const double q2 = (2.0 * v[2] + 5.0 * v[3] - v[4]) / 6.0;
  const double b0 = 13.0 / 12.0 * (v[0] - 2.0 * v[1] + v[2]) * (v[0] - 2.0 * v[1] + v[2]) +
                    0.25 * (v[0] - 4.0 * v[1] + 3.0 * v[2]) * (v[0] - 4.0 * v[1] + 3.0 * v[2]);
  const double b1 = 13.0 / 12.0 * (v[1] - 2.0 * v[2] + v[3]) * (v[1] - 2.0 * v[2] + v[3]) +
                    0.25 * (v[1] - v[3]) * (v[1] - v[3]);
  const double b2 = 13.0 / 12.0 * (v[2] - 2.0 * v[3] + v[4]) * (v[2] - 2.0 * v[3] + v[4]) +
                    0.25 * (3.0 * v[2] - 4.0 * v[3] + v[4]) * (3.0 * v[2] - 4.0 * v[3] + v[4]);
  const double eps = 1e-6;
  const double a0 = 0.1 / ((eps + b0) * (eps + b0));
  const double a1 = 0.6 / ((eps + b1) * (eps + b1));
  const double a2 = 0.3 / ((eps + b2) * (eps + b2));
  return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

/* WENO numerical flux through the face between cells j+base and j+base+1
 * along axis a: the + part F + alpha U reconstructed from the five cells
 * j+base-2 .. j+base+2, the - part F - alpha U from j+base+3 .. j+base-1
 * (mirrored), each halved */
static int weno_flux(const or_state *S, const double *U, int j, int a, int base,
                     double alpha, double *fh) {
  int nm = S->nm, nc = S->nc;
  double Us[6][5], Fs[6][5];
  for (int q = 0; q < 6; ++q) {
    int idx = neighbour(S, j, a, base - 2 + q);
    for (int r = 0; r < nm; ++r) Us[q][r] = U[r * nc + idx];
    int st = euler_flux(S, Us[q], a, Fs[q], NULL);
    if (st) return st;
  }
  for (int r = 0; r < nm; ++r) {
    double vp[5], vm[5];
    for (int q = 0; q < 5; ++q) {
      vp[q] = 0.5 * (Fs[q][r] + alpha * Us[q][r]);
      vm[q] = 0.5 * (Fs[5 - q][r] - alpha * Us[5 - q][r]);
    }
    fh[r] = weno5(vp) + weno5(vm);
  }
  return OR_OK;
}

/* L(U) = -(1/dx) sum_a (fh_{a,j+1/2} - fh_{a,j-1/2}) into out */
static int weno_rhs(const or_state *S, const double *U, const double *alpha, double *out) {
  int nm = S->nm, nc = S->nc, d = S->d, st = OR_OK;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < nc; ++j) {
    double div[5] = {0, 0, 0, 0, 0}, fr[5], fl[5];
    for (int a = 0; a < d; ++a) {
      int l1 = weno_flux(S, U, j, a, 0, alpha[a], fr);
      int l2 = weno_flux(S, U, j, a, -1, alpha[a], fl);
      if (l1 || l2) {
#pragma omp atomic write
        st = OR_ENONPHYS;
      }
      for (int r = 0; r < nm; ++r) div[r] += fr[r] - fl[r];
    }
    for (int r = 0; r < nm; ++r) out[r * nc + j] = -div[r] / S->dx;
  }
  return st;
}

/* one sub-step of length h by the three-stage SSP Runge-Kutta method:
 * U1 = U + h L(U), U2 = 3/4 U + 1/4 (U1 + h L(U1)),
 * U <- 1/3 U + 2/3 (U2 + h L(U2)), with the speeds alpha of U */
static int weno_substep(const or_state *S, double *U, const double *alpha, double h,
                        double *U1, double *U2, double *L) {
  int n = S->nm * S->nc, st;
  st = weno_rhs(S, U, alpha, L);
  if (st) return st;
  for (int i = 0; i < n; ++i) U1[i] = U[i] + h * L[i];
  st = weno_rhs(S, U1, alpha, L);
  if (st) return st;
  for (int i = 0; i < n; ++i) U2[i] = 0.75 * U[i] + 0.25 * (U1[i] + h * L[i]);
  st = weno_rhs(S, U2, alpha, L);
  if (st) return st;
  for (int i = 0; i < n; ++i) U[i] = U[i] / 3.0 + 2.0 / 3.0 * (U2[i] + h * L[i]);
  return OR_OK;
}

/* the WENO solve over dt in s equal sub-steps, s from the speeds of U */
static int weno_solve(const or_state *S, double *U, double dt, int *nsub) {
  int n = S->nm * S->nc, d = S->d;
  double alpha[3];
  int st = lf_speeds(S, U, alpha);
  if (st) return st;
  double sum = 0.0;
  for (int a = 0; a < d; ++a) sum += alpha[a];
  int s = (int)ceil(2.5 * dt * sum / S->dx);
  if (s < 1) s = 1;
  if (nsub) *nsub = s;
  double h = dt / s;
  double *buf = (double *)malloc(sizeof(double) * 3 * n);
  if (!buf) return OR_EINVAL;
  for (int it = 0; it < s && st == OR_OK; ++it) {
    if (it > 0) st = lf_speeds(S, U, alpha);
    if (st) break;
    st = weno_substep(S, U, alpha, h, buf, buf + n, buf + 2 * n);
  }
  free(buf);
  return st;
}

/* ---------------------------------------------- section 4.3.1: HOFKS step */

/* 1/tau with 1/inf = 0 and 1/0 = inf */
static double inv_tau(double tau) {
  if (isinf(tau)) return 0.0;
  if (tau == 0.0) return INFINITY;
  return 1.0 / tau;
}

/* Strang: exp(-e) and 1 - exp(-e), e = dt/2 (1/tau_prev) + dt/2 (1/tau) */
static void strang_weights(double dt, double ip, double in, double *lam, double *mu) {
  const double e = 0.5 * dt * ip + 0.5 * dt * in;
  *lam = exp(-e);
  *mu = -expm1(-e);
}

static int step_once(or_state *S) {
  const int nm = S->nm, nc = S->nc, nv = S->nv;
  double lam = S->lam, mu = S->mu;
  if (S->strang)
    strang_weights(S->dt, S->nstep > 1 ? S->inv_prev : 0.0, inv_tau(S->tau), &lam, &mu);
  const double w = S->w;
  int st = OR_OK;

  /* 1. E^n = E[U^n] in every cell (not needed when lambda == 1) */
  if (lam != 1.0) {
#pragma omp parallel
    {
      double Uj[5];
      double *Ej = (double *)malloc(sizeof(double) * nv);
#pragma omp for schedule(static)
      for (int j = 0; j < nc; ++j) {
        for (int r = 0; r < nm; ++r) Uj[r] = S->U[r * nc + j];
        int lst = equilibrium(S, Uj, Ej);
        if (lst) {
#pragma omp atomic write
          st = lst;
        }
        for (int k = 0; k < nv; ++k) S->E[(size_t)k * nc + j] = Ej[k];
      }
      free(Ej);
    }
    if (st) return st;
  }

  /* 2-4. relax, shift, and the two moment sums of eq. (UK) */
  double *sF = (double *)calloc((size_t)nm * nc, sizeof(double)); /* sum m F~ */
  double *sE = (double *)calloc((size_t)nm * nc, sizeof(double)); /* sum m E~ */
  double *UE = (double *)malloc(sizeof(double) * nm * nc);
  if (!sF || !sE || !UE) {
    free(sF);
    free(sE);
    free(UE);
    return OR_EINVAL;
  }
  for (int k = 0; k < nv; ++k) {
    const double *mk = S->m + (size_t)k * nm;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < nc; ++j) {
      int src = upstream(S, j, k);
      double F = S->f[(size_t)k * nc + src]; /* f^n(x_j - v_k dt)  */
      double fK;
      if (lam == 1.0) {
        fK = F; /* free transport: exact copy */
      } else {
        double Ek = S->E[(size_t)k * nc + src]; /* E^n(x_j - v_k dt) */
        fK = (lam == 0.0) ? Ek : lam * F + mu * Ek;
        for (int r = 0; r < nm; ++r) sE[r * nc + j] += mk[r] * Ek;
      }
      S->fnew[(size_t)k * nc + j] = fK;
      for (int r = 0; r < nm; ++r) sF[r * nc + j] += mk[r] * F;
    }
  }

  /* U_* = P(T(lambda f^n)),  U_M = P(T((1-lambda) E^n)) */
  double *Ustar = sF, *UM = sE;
  for (int i = 0; i < nm * nc; ++i) {
    Ustar[i] = (lam == 0.0) ? 0.0 : lam * (w * sF[i]);
    UM[i] = (lam == 1.0) ? 0.0 : mu * (w * sE[i]);
  }

  /* 5. U_E: Euler over dt from U^n, scaled by (1 - lambda) (R8) */
  S->last_substeps = 0;
  if (lam == 1.0) {
    for (int i = 0; i < nm * nc; ++i) UE[i] = 0.0;
  } else if (S->scheme == 1) {
    memcpy(UE, UM, sizeof(double) * nm * nc); /* FKS: keep the kinetic U_M */
  } else {
    memcpy(UE, S->U, sizeof(double) * nm * nc);
    st = (S->scheme == 3) ? weno_solve(S, UE, S->dt, &S->last_substeps)
                          : muscl_solve(S, UE, S->dt, &S->last_substeps);
    if (st) {
      free(sF);
      free(sE);
      free(UE);
      return st;
    }
    for (int i = 0; i < nm * nc; ++i) UE[i] *= mu;
  }

  /* 6. correction of the transported equilibrium part (eq. minim_full) and
   *    the hybrid moments of eq. (mom) */
  for (int i = 0; i < nm * nc; ++i) S->delta[i] = UE[i] - UM[i];
  if (lam != 1.0 && S->scheme != 1) {
    double *cj = (double *)malloc(sizeof(double) * nm * nc);
    for (int j = 0; j < nc; ++j)
      for (int r = 0; r < nm; ++r) {
        double acc = 0.0;
        for (int s = 0; s < nm; ++s) acc += S->A[r * nm + s] * S->delta[s * nc + j];
        cj[r * nc + j] = acc;
      }
    for (int k = 0; k < nv; ++k) {
      const double *mk = S->m + (size_t)k * nm;
#pragma omp parallel for schedule(static)
      for (int j = 0; j < nc; ++j) {
        double corr = 0.0;
        for (int r = 0; r < nm; ++r) corr += w * mk[r] * cj[r * nc + j];
        S->fnew[(size_t)k * nc + j] += corr;
      }
    }
    free(cj);
  }
  for (int i = 0; i < nm * nc; ++i) S->U[i] = Ustar[i] + UE[i];

  double *t = S->f;
  S->f = S->fnew;
  S->fnew = t;
  free(sF);
  free(sE);
  free(UE);
  return OR_OK;
}

/* ------------------------------------------------------------- public API */

void or_destroy(or_state *S) {
  if (!S) return;
  free(S->cvel);
  free(S->shift);
  free(S->kint);
  free(S->m);
  free(S->f);
  free(S->fnew);
  free(S->E);
  free(S->U);
  free(S->delta);
  free(S);
}

/* tau > 0 finite, +inf (free transport) or 0 (instant relaxation) */
static int set_tau(or_state *S, double tau) {
  if (!(tau >= 0.0)) return OR_EINVAL;
  S->tau = tau;
  if (isinf(tau)) {
    S->lam = 1.0;
    S->mu = 0.0;
  } else if (tau == 0.0) {
    S->lam = 0.0;
    S->mu = 1.0;
  } else {
    S->lam = exp(-S->dt / tau);
    S->mu = -expm1(-S->dt / tau);
  }
  return OR_OK;
}

or_state *or_create(int d, const int *n, double dx, int nv1, double dv,
                    const int *bc, int scheme, double tau, double dt, int strang,
                    int *status) {
  *status = OR_EINVAL;
  if (d < 1 || d > 3 || nv1 < 2 || !(dx > 0) || !(dv > 0) || scheme < 0 ||
      scheme > 3)
    return NULL;
  or_state *S = (or_state *)calloc(1, sizeof(or_state));
  S->d = d;
  S->nm = d + 2;
  S->nc = 1;
  for (int a = 0; a < 3; ++a) {
    S->n[a] = (a < d) ? n[a] : 1;
    S->bc[a] = (a < d) ? bc[a] : 0;
    if (S->n[a] < 1 || S->bc[a] < 0 || S->bc[a] > 1) {
      free(S);
      return NULL;
    }
    S->nc *= S->n[a];
  }
  S->dx = dx;
  S->dv = dv;
  S->dt = dx / dv; /* lattice: v_k dt = k dx */
  if (dt != 0.0) { /* off-lattice: a free time step up to the lattice's */
    if (!(dt > 0.0) || !(dt <= dx / dv)) {
      free(S);
      return NULL;
    }
    S->dt = dt;
    S->offl = 1;
  }
  if (strang < 0 || strang > 1) {
    free(S);
    return NULL;
  }
  S->strang = strang;
  S->w = pow(dv, d);
  S->nv1 = nv1;
  S->nv = 1;
  for (int a = 0; a < d; ++a) S->nv *= nv1;
  S->scheme = scheme;
  if (set_tau(S, tau)) {
    free(S);
    return NULL;
  }
  int nm = S->nm, nv = S->nv, nc = S->nc;
  S->cvel = (double *)malloc(sizeof(double) * nv1);
  S->shift = (int *)malloc(sizeof(int) * nv1);
  for (int i = 0; i < nv1; ++i) {
    double v = (double)(i - nv1 / 2) * dv;
    S->cvel[i] = v * S->dt / dx;
    S->shift[i] = i - nv1 / 2;
  }
  S->kint = (int *)malloc(sizeof(int) * nv * d);
  S->m = (double *)malloc(sizeof(double) * nv * nm);
  for (int k = 0; k < nv; ++k) {
    int rem = k;
    double vsq = 0.0;
    S->m[k * nm] = 1.0;
    for (int a = 0; a < d; ++a) {
      int ia = rem % nv1;
      rem /= nv1;
      int ka = ia - nv1 / 2;
      S->kint[k * d + a] = ka;
      double va = ka * dv;
      S->m[k * nm + 1 + a] = va;
      vsq += va * va;
    }
    S->m[k * nm + d + 1] = 0.5 * vsq;
  }
  /* C C^T with C[r][k] = w m_k[r] */
  double CCt[25];
  for (int r = 0; r < nm; ++r)
    for (int s = 0; s < nm; ++s) {
      double acc = 0.0;
      for (int k = 0; k < nv; ++k)
        acc += (S->w * S->m[k * nm + r]) * (S->w * S->m[k * nm + s]);
      CCt[r * nm + s] = acc;
    }
  if (invert(nm, CCt, S->A)) {
    or_destroy(S);
    return NULL;
  }
  size_t fsz = (size_t)nv * nc;
  S->f = (double *)calloc(fsz, sizeof(double));
  S->fnew = (double *)calloc(fsz, sizeof(double));
  S->E = (double *)calloc(fsz, sizeof(double));
  S->U = (double *)calloc((size_t)nm * nc, sizeof(double));
  S->delta = (double *)calloc((size_t)nm * nc, sizeof(double));
  if (!S->f || !S->fnew || !S->E || !S->U || !S->delta) {
    or_destroy(S);
    return NULL;
  }
  *status = OR_OK;
  return S;
}

int or_set_tau(or_state *S, double tau) { return set_tau(S, tau); }

/* initial data: U^0 from (rho, u, theta), f^0 = E[U^0] (section 4.2) */
int or_init_macro(or_state *S, const double *rho, const double *u,
                  const double *theta) {
  S->nstep = 0;
  int d = S->d, nm = S->nm, nc = S->nc, nv = S->nv, st = OR_OK;
  for (int j = 0; j < nc; ++j) {
    double usq = 0.0;
    S->U[j] = rho[j];
    for (int a = 0; a < d; ++a) {
      S->U[(1 + a) * nc + j] = rho[j] * u[a * nc + j];
      usq += u[a * nc + j] * u[a * nc + j];
    }
    S->U[(d + 1) * nc + j] = 0.5 * rho[j] * usq + 0.5 * d * rho[j] * theta[j];
  }
  double *Ej = (double *)malloc(sizeof(double) * nv);
  double Uj[5];
  for (int j = 0; j < nc && st == OR_OK; ++j) {
    for (int r = 0; r < nm; ++r) Uj[r] = S->U[r * nc + j];
    st = equilibrium(S, Uj, Ej);
    for (int k = 0; k < nv; ++k) S->f[(size_t)k * nc + j] = Ej[k];
  }
  free(Ej);
  return st;
}

/* arbitrary initial f; the carried moments become U = P(f), eq. (DM) */
int or_set_f(or_state *S, const double *f) {
  S->nstep = 0;
  int nm = S->nm, nc = S->nc, nv = S->nv;
  memcpy(S->f, f, sizeof(double) * nv * nc);
  for (int j = 0; j < nc; ++j)
    for (int r = 0; r < nm; ++r) {
      double acc = 0.0;
      for (int k = 0; k < nv; ++k) acc += S->m[k * nm + r] * f[(size_t)k * nc + j];
      S->U[r * nc + j] = S->w * acc;
    }
  return OR_OK;
}

/* o(n) = ceil(c n - 1/2): the piece holding a cell centre after n steps */
static long piece_offset(double c, long n) {
  volatile double cn = c * (double)n; /* rounded product, no contraction */
  return (long)ceil(cn - 0.5);
}

int or_step(or_state *S, int nsteps) {
  for (int i = 0; i < nsteps; ++i) {
    if (S->offl)
      for (int q = 0; q < S->nv1; ++q)
        S->shift[q] = (int)(piece_offset(S->cvel[q], S->nstep + 1) -
                            piece_offset(S->cvel[q], S->nstep));
    S->nstep++;
    int st = step_once(S);
    if (st) return st;
    S->inv_prev = inv_tau(S->tau);
  }
  return OR_OK;
}

void or_get_U(const or_state *S, double *U) {
  memcpy(U, S->U, sizeof(double) * S->nm * S->nc);
}
/* f at t^n.  With Strang splitting, after a step, the stored f still waits
 * for the half relaxation R_{dt/2} (with the tau of the last step) towards
 * E[U^n]; it is applied here (non-physical U gives NaN) */
void or_get_f(const or_state *S, double *f) {
  memcpy(f, S->f, sizeof(double) * (size_t)S->nv * S->nc);
  if (!S->strang || S->nstep == 0) return;
  double lh, mh;
  strang_weights(S->dt, S->inv_prev, 0.0, &lh, &mh);
  if (lh == 1.0) return;
  double Uj[5];
  double *Ej = (double *)malloc(sizeof(double) * S->nv);
  for (int j = 0; j < S->nc; ++j) {
    for (int r = 0; r < S->nm; ++r) Uj[r] = S->U[r * S->nc + j];
    int bad = equilibrium(S, Uj, Ej);
    for (int k = 0; k < S->nv; ++k) {
      double *p = f + (size_t)k * S->nc + j;
      *p = bad ? NAN : (lh == 0.0 ? Ej[k] : lh * *p + mh * Ej[k]);
    }
  }
  free(Ej);
}
void or_get_delta(const or_state *S, double *dl) {
  memcpy(dl, S->delta, sizeof(double) * S->nm * S->nc);
}
int or_last_substeps(const or_state *S) { return S->last_substeps; }

/* threads of the OpenMP loops (for timing with one thread and with all) */
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
double or_dt(const or_state *S) { return S->dt; }
long or_nstep(const or_state *S) { return S->nstep; }
double or_lambda(const or_state *S) { return S->lam; }
void or_get_A(const or_state *S, double *A) {
  memcpy(A, S->A, sizeof(double) * S->nm * S->nm);
}
void or_get_velocities(const or_state *S, double *v) {
  for (int k = 0; k < S->nv; ++k)
    for (int a = 0; a < S->d; ++a) v[k * S->d + a] = S->m[k * S->nm + 1 + a];
}

/* standalone pieces, for the pins */
int or_maxwellian(const or_state *S, const double *U, double *M) {
  return maxwellian(S, U, M);
}
int or_equilibrium(const or_state *S, const double *U, double *E) {
  return equilibrium(S, U, E);
}
int or_muscl(const or_state *S, double *U, double dt, int *nsub) {
  return muscl_solve(S, U, dt, nsub);
}
int or_weno(const or_state *S, double *U, double dt, int *nsub) {
  return weno_solve(S, U, dt, nsub);
}
/* a single sub-step of length h with the speeds of U (no sub-cycling) */
int or_muscl_substep(const or_state *S, double *U, double h) {
  double alpha[3];
  int st = lf_speeds(S, U, alpha);
  if (st) return st;
  double *Unew = (double *)malloc(sizeof(double) * S->nm * S->nc);
  if (!Unew) return OR_EINVAL;
  st = muscl_substep(S, U, Unew, alpha, h);
  memcpy(U, Unew, sizeof(double) * S->nm * S->nc);
  free(Unew);
  return st;
}
