// kernels.hpp -- gfx950 kernels of one HOFKS time step (arXiv:1212.0204).
//
// Data kept resident in HBM between steps (cells x-fastest):
//   g[k][j]    pieces of the distribution, one plane per velocity node k
//              (FP64, or FP32 in the precision form).  The distribution is
//              f(j,k) = g(j,k) + w m_k . cf(j): the consistency correction of
//              eq. (minim_full) is kept as d+2 coefficients per cell and
//              applied when the piece is next read, so every step reads and
//              writes each piece exactly once.
//   U[r][j]    moments U^n (FP64), two buffers (read / written by a step).
//   cf[r][j]   pending correction coefficients (C C^T)^{-1}(U_E - U_M).
//   rec[j][q]  per-cell record read by the pieces that leave cell j, in the
//              piece precision, two buffers:
//              q = 0 .. d+1      log prefactor, u_1..u_d, beta = 1/(2 theta)
//              q = d+2 .. 2d+3   p = w (lambda cf + (1-lambda) cE)
//              q = 2d+4 .. 3d+5  e = w cE
//              with cE = (C C^T)^{-1}(U - C M) the conservative correction of
//              eq. (minimMax); a piece of velocity v leaving cell j' relaxes to
//                f* = lambda g + (1-lambda) M + p.m(v),
//                E  = M + e.m(v),   M = exp(lp - beta |v - u|^2).
// One time step is two launches: k_euler runs the s Euler sub-steps of eq.
// (discmom) on U^n (co-resident blocks, barrier between sub-steps); k_kinetic
// relaxes, shifts and sums the pieces of a 64-cell tile over all velocities
// inside one block, then forms delta, U^{n+1}, cf and the next records of the
// tile's cells.  No block waits on another block of the same launch except
// the Euler barrier.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// stream the pieces with non-temporal loads and stores
#ifndef HOFKS_EULER_NT
#define HOFKS_EULER_NT 0
#endif
#ifndef HOFKS_NT
#define HOFKS_NT 1
#endif

namespace hofks {

constexpr int SMAX = 512;         // largest Euler sub-step count a plan may use
constexpr int ASTR = 4;           // doubles per row of Lax-Friedrichs speeds
// doubles per slot set: row 0 (speeds of U^n), rows 1..SMAX of sub-step
// speeds with NSLOT partial maxima each (slot = block index mod NSLOT, one
// 32-byte group per slot, so the atomics of one row spread over lines),
// then control words (barrier counters, each on its own 64-byte line)
constexpr int NSLOT = 8;
constexpr int CTRL_LINES = 10;
constexpr int SET_CTRL = ASTR + SMAX * NSLOT * ASTR;
constexpr int SET_D = SET_CTRL + CTRL_LINES * 8;
constexpr int FLAG_NONPHYS = 1;
constexpr int FLAG_SUBSTEP = 2;
constexpr int FLAG_SPIN = 4;      // a bounded wait gave up: results are invalid
constexpr unsigned SPIN_CAP = 1u << 20;  // ~1-2 s of polling

struct Geom {
  int n[3];
  int nc;
  int nv1, kofs, nv;  // nodes per axis, k_a = i_a - kofs, total nodes
  int bc[3];          // 0 periodic, 1 outflow
  int offl;           // 1: a free time step (off-lattice transport), 0: dt = dx/dv
  double dx, dv, dt, w, lam, mu, gam;
  double sfac;        // sub-steps s = ceil(sfac dt sum_a alpha_a / dx): 2 MUSCL, 2.5 WENO
  double lam_r, mu_r; // relaxation weights of the step that reads the records formed
                      // (equal to lam, mu except around Strang half relaxations)
};

struct Mat {
  double a[25];
};

// MODE_RETAU: as MODE_REFRESH, keeping the mark of cells without pieces
enum { MODE_STEP = 0, MODE_INIT = 1, MODE_INIT_FROM_SUMS = 2, MODE_REFRESH = 3, MODE_RETAU = 4 };

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int map_axis(int i, int N, int bc) {
  if (bc == 0) {
    i %= N;
    return i < 0 ? i + N : i;
  }
  return i < 0 ? 0 : (i >= N ? N - 1 : i);
}

// x index of the piece that reaches cell x with shift kx (|kx| <= N).  kx is
// the same for the whole wavefront, so the offset is formed in scalar code.
template <int BCX>
__device__ __forceinline__ int map_x(int xN, int kx, int N) {
  if (BCX == 0) {  // periodic: u = x - kx (+ N when kx > 0) lies in [0, 2N)
    const int off = kx > 0 ? kx - N : kx;
    const unsigned u = (unsigned)(xN - N - off);
    return (int)min(u, u - (unsigned)N);
  }
  const int t = xN - N - kx;  // outflow: clamp to the boundary cell
  return min(max(t, 0), N - 1);
}

__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ void atomic_max_pos(double* addr, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long*>(addr),
            static_cast<unsigned long long>(__double_as_longlong(v)));
}

__device__ __forceinline__ unsigned load_acquire(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Euler sub-step count of a step, from the speeds of U^n (same rule as the
// oracle: s = max(1, ceil(c dt sum_a alpha_a / dx)), c = 2 for the MUSCL
// bound dt_s sum alpha <= dx/2 of eq. (Time2), 2.5 for the WENO solve's 0.4)
template <int D>
__device__ __forceinline__ int substeps(const double* alpha0, const Geom& G, int s_cap,
                                        bool* over) {
  double sum = 0.0;
  for (int a = 0; a < D; ++a) sum += alpha0[a];
  double sv = ceil(G.sfac * G.dt * sum / G.dx);
  int s = (sv >= 1.0) ? (sv <= (double)s_cap ? (int)sv : s_cap + 1) : 1;
  *over = (s > s_cap);
  return s > s_cap ? s_cap : s;
}

// Blocks are dispatched to the NXCD accelerator dies round-robin (block b
// to die b mod NXCD), and each die has its own L2.  Tile index of block b
// such that every die takes one contiguous range of tiles: neighbouring
// rows, whose upstream records overlap, then share that die's L2.
constexpr unsigned NXCD = 8;
__device__ __forceinline__ int xcd_tile(unsigned b, unsigned nb) {
  const unsigned x = b % NXCD, i = b / NXCD;
  const unsigned per = nb / NXCD, rem = nb % NXCD;
  return (int)(x * per + (x < rem ? x : rem) + i);
}

// slot `slot` of speed row r of a set (row 0 has one slot)
__device__ __forceinline__ double* speed_row(double* S, int r, int slot) {
  return r == 0 ? S : S + ASTR + ((size_t)(r - 1) * NSLOT + slot) * ASTR;
}

// speeds of row r: the maximum over its slots
template <int D>
__device__ __forceinline__ void row_speeds(const double* S, int r, double* alpha) {
#pragma unroll
  for (int d = 0; d < D; ++d) alpha[d] = S[d];
  if (r == 0) return;
  const double* p = S + ASTR + (size_t)(r - 1) * NSLOT * ASTR;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    double m = p[d];
    for (int q = 1; q < NSLOT; ++q) m = fmax(m, p[q * ASTR + d]);
    alpha[d] = m;
  }
}

__device__ __forceinline__ void two_sum(double& s, double& c, double x) {
  double t = s + x;
  double z = t - s;
  c += (s - (t - z)) + (x - z);
  s = t;
}

template <typename T>
__device__ __forceinline__ T fast_exp(T x);
template <>
__device__ __forceinline__ double fast_exp<double>(double x) {
  return exp(x);
}
template <>
__device__ __forceinline__ float fast_exp<float>(float x) {
  return __expf(x);
}

// Record of a cell, array-of-structures: R = 3(d+2) values padded to RS so
// that a record is an odd number of 16-byte chunks.  Lanes of a wavefront
// read consecutive records with ds_read_b128; an odd chunk stride spreads
// eight consecutive lanes over all LDS banks.
template <int D, typename T>
__host__ __device__ constexpr int rec_values() {
  return 3 * (D + 2);
}
template <int D, typename T>
__host__ __device__ constexpr int rec_stride() {
  constexpr int per16 = 16 / (int)sizeof(T);
  constexpr int n16 = (rec_values<D, T>() + per16 - 1) / per16;
  return (n16 % 2 ? n16 : n16 + 1) * per16;
}
template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  using type = double2;
};
template <>
struct Vec16<float> {
  using type = float4;
};

// velocity node table of one axis: v, v^2, and FP32 copies (scalar loads);
// it is followed in memory by nv1 doubles c = v dt / dx, the cells a piece
// travels per step (read only by off-lattice steps)
struct VelNode {
  double v, v2;
  float vf, v2hf;  // (float)v, (float)(v^2 / 2)
  double v2h;      // v^2 / 2
};

// Cells moved by the pieces of velocity node i in the step t^n -> t^{n+1}
// (section 4.2: exact transport of piecewise-constant pieces).  On the
// lattice dt = dx/dv this is k = i - kofs.  Off the lattice the pieces sit
// at accumulated offsets v n dt, the cell centre x_j lies in the piece that
// started in cell j - o(n), o(n) = ceil(c n - 1/2), and the step moves by
// o(n+1) - o(n) (floor(c) or ceil(c)).  Products and differences are rounded
// one by one, as in the oracle.
__device__ __forceinline__ int node_shift(const VelNode* vt, int i, const Geom& G, long n) {
#pragma clang fp contract(off)
  if (!G.offl) return i - G.kofs;
  using CD = const __attribute__((address_space(4))) double;
  const double c = ((CD*)(vt + G.nv1))[i];
  const double a = c * (double)(n + 1) - 0.5;
  const double b = c * (double)n - 0.5;
  const int sh = (int)(ceil(a) - ceil(b));
  // |c| <= |i - kofs| (dt <= dx/dv), so the shift lies in the lattice's range
  // and within the staged record segment; the clamp only guards memory
  return min(max(sh, -G.kofs), G.nv1 - 1 - G.kofs);
}

// bounded wait: gives up (and flags) after SPIN_CAP sleeps, or at once when
// another wait of the launch has already given up
__device__ __forceinline__ void spin_until_geq(unsigned* p, unsigned target, int* flag) {
  unsigned it = 0;
  while (load_acquire(p) < target) {
    __builtin_amdgcn_s_sleep(2);
    ++it;
    if (it > SPIN_CAP ||
        ((it & 255u) == 0 &&
         (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & FLAG_SPIN))) {
      atomicOr(flag, FLAG_SPIN);
      break;
    }
  }
}

// barrier of the nb blocks of the Euler group (monotonic arrival counter)
__device__ __forceinline__ void group_barrier(unsigned* cnt, unsigned target, int* flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(cnt, 1u);
    spin_until_geq(cnt, target, flag);
    __threadfence();  // acquire: invalidates this compute unit's caches for all its waves
  }
  __syncthreads();
}

// ===================================================================== MUSCL
// Section 4.3.2: flux-split Lax-Friedrichs with Van Leer limited slopes of
// W+- = F +- alpha U, unsplit over the d directions, forward Euler in time.
// The face flux psi = (F_l + F_r)/2 - alpha (U_r - U_l)/2 + (s+_l - s-_r)/4
// is written as (W+_l + W-_r)/2 + (s+_l - s-_r)/4.

// W+- of one cell along axis a; false if the state is not physical
template <int D>
__device__ __forceinline__ bool split_flux(const double* U, int a, double alpha, double gam,
                                           double* Wp, double* Wm) {
  constexpr int NM = D + 2;
  const double rho = U[0], irho = 1.0 / rho;
  double usq = 0.0, u[3];
#pragma unroll
  for (int b = 0; b < D; ++b) {
    u[b] = U[1 + b] * irho;
    usq += u[b] * u[b];
  }
  // p = rho theta = (2E - rho |u|^2) / d
  const double p = (2.0 * U[NM - 1] - rho * usq) * (1.0 / D);
  double F[NM];
  F[0] = U[1 + a];
#pragma unroll
  for (int b = 0; b < D; ++b) F[1 + b] = U[1 + b] * u[a] + (a == b ? p : 0.0);
  F[NM - 1] = (U[NM - 1] + p) * u[a];
#pragma unroll
  for (int r = 0; r < NM; ++r) {
    Wp[r] = F[r] + alpha * U[r];
    Wm[r] = F[r] - alpha * U[r];
  }
  return (rho > 0.0) && (p > 0.0) && isfinite(rho) && isfinite(p) && isfinite(usq);
}

// |u_a| + c for every axis; false if the state is not physical
template <int D>
__device__ __forceinline__ bool lf_speeds(const double* U, double gam, double* sp) {
  constexpr int NM = D + 2;
  const double rho = U[0];
  double usq = 0.0, u[3];
#pragma unroll
  for (int b = 0; b < D; ++b) {
    u[b] = U[1 + b] / rho;
    usq += u[b] * u[b];
  }
  const double th = (2.0 * U[NM - 1] - rho * usq) / (D * rho);
  const bool ok = (rho > 0.0) && (th > 0.0) && isfinite(rho) && isfinite(th) && isfinite(usq);
  const double c = ok ? sqrt(gam * (rho * th) / rho) : 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) sp[a] = ok ? fabs(u[a]) + c : 0.0;
  return ok;
}

// Van Leer slope 2ab/(a+b) for ab > 0, else 0.  The quotient uses the
// hardware reciprocal refined by two Newton steps (error within a few ulp of
// the IEEE quotient); a + b cannot vanish when ab > 0.
__device__ __forceinline__ double vl_slope(double a, double b, int unlimited) {
  if (unlimited) return b;
  const double ab = a * b;
  if (!(ab > 0.0)) return 0.0;
  const double den = a + b;
  double r = __builtin_amdgcn_rcp(den);
  r = fma(fma(-den, r, 1.0), r, r);
  r = fma(fma(-den, r, 1.0), r, r);
  const double q = 2.0 * ab * r;
  return fma(fma(-den, q, 2.0 * ab), r, q);
}

// new value of cell j after one sub-step: in - dt_s/dx sum_a (psi_a+ - psi_a-).
// All stencil values are loaded before any flux is formed, so the loads of
// a sub-step overlap.  Each face is formed from its own four cells (both
// neighbours of a face get bit-identical fluxes, so the update conserves
// exactly up to the final sum).
template <int D>
__device__ __forceinline__ bool euler_cell(const double* __restrict__ in, int j,
                                           const double* alpha, double dts_dx, const Geom& G,
                                           int unl, double* Un) {
  constexpr int NM = D + 2;
  const int c[3] = {j % G.n[0], (j / G.n[0]) % G.n[1], j / (G.n[0] * G.n[1])};
  double St[D][5][NM];  // cells j-2 .. j+2 along each axis
#pragma unroll
  for (int a = 0; a < D; ++a) {
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      int cc[3] = {c[0], c[1], c[2]};
      cc[a] = map_axis(c[a] + q - 2, G.n[a], G.bc[a]);
      const int jj = (cc[2] * G.n[1] + cc[1]) * G.n[0] + cc[0];
#pragma unroll
      for (int r = 0; r < NM; ++r) St[a][q][r] = in[(size_t)r * G.nc + jj];
    }
  }
  double div[NM];
#pragma unroll
  for (int r = 0; r < NM; ++r) div[r] = 0.0;
  bool phys = true;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    double Wp[5][NM], Wm[5][NM];
#pragma unroll
    for (int q = 0; q < 5; ++q) phys &= split_flux<D>(St[a][q], a, alpha[a], G.gam, Wp[q], Wm[q]);
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      // face j-1/2 from cells 0..3, face j+1/2 from cells 1..4
      const double spl = vl_slope(Wp[1][r] - Wp[0][r], Wp[2][r] - Wp[1][r], unl);
      const double sml = vl_slope(Wm[2][r] - Wm[1][r], Wm[3][r] - Wm[2][r], unl);
      const double spr = vl_slope(Wp[2][r] - Wp[1][r], Wp[3][r] - Wp[2][r], unl);
      const double smr = vl_slope(Wm[3][r] - Wm[2][r], Wm[4][r] - Wm[3][r], unl);
      const double psil = 0.5 * (Wp[1][r] + Wm[2][r]) + 0.25 * (spl - sml);
      const double psir = 0.5 * (Wp[2][r] + Wm[3][r]) + 0.25 * (spr - smr);
      div[r] += psir - psil;
    }
  }
#pragma unroll
  for (int r = 0; r < NM; ++r) Un[r] = St[0][2][r] - dts_dx * div[r];
  return phys;
}

// ============================================================ cell record
// Maxwellian parameters of U (eq. M, theta from eq. E), separable discrete
// moments C M (sums along each velocity axis), cE = A (U - C M), and the
// record; speeds |u_a| + c for the next Euler solve.  Returns physicality.
template <int D, typename T>
__device__ __forceinline__ bool cell_record(const double* Un, const double* cfv, const Geom& G,
                                            const Mat& A, T* __restrict__ rec_j, double* speed,
                                            bool valid = true) {
  constexpr int NM = D + 2;
  const double rho = Un[0];
  double u[3] = {0.0, 0.0, 0.0}, usq = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    u[a] = Un[1 + a] / rho;
    usq += u[a] * u[a];
  }
  const double th = (2.0 * Un[NM - 1] - rho * usq) / (D * rho);
  const bool phys = (rho > 0.0) && (th > 0.0) && isfinite(rho) && isfinite(th) && isfinite(usq);
  double lp = 0.0, beta = 0.0, cE[NM];
#pragma unroll
  for (int r = 0; r < NM; ++r) cE[r] = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) speed[a] = 0.0;
  if (phys) {
    beta = 0.5 / th;
    const double pref = rho * pow(2.0 * M_PI * th, -0.5 * D);
    lp = log(rho) - 0.5 * D * log(2.0 * M_PI * th);
    // 1D sums of exp(-beta (v_i - u_a)^2) over the nodes: from the node
    // nearest to u_a outwards, each value is the previous one times a ratio
    // that itself changes by the constant factor exp(-2 beta dv^2); both are
    // recomputed every 16 nodes so that rounding stays within ~16 ulp.
    // Values only decrease away from the peak, so an underflow to zero is
    // where the true value is below the FP64 range.  Nodes v_i = (i - kofs) dv
    // are formed in place (the same rounding as the node table).
    double G0[3], G1[3], G2[3];
    const double dv = G.dv;
    auto vnode = [&](int i) { return (double)(i - G.kofs) * dv; };
    const double qf = exp(-2.0 * beta * dv * dv);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      int ip = (int)rint(u[a] / dv) + G.kofs;
      ip = ip < 0 ? 0 : (ip >= G.nv1 ? G.nv1 - 1 : ip);
      const double dp = vnode(ip) - u[a];
      const double ep = exp(-beta * dp * dp);
      double s0 = ep, s1 = vnode(ip) * ep, s2 = (vnode(ip) * vnode(ip)) * ep;
      double e = ep, r = exp(-beta * (2.0 * dp * dv + dv * dv));
      for (int i = ip + 1; i < G.nv1; ++i) {
        if (((i - ip) & 15) == 0) {
          const double d = vnode(i) - u[a];
          e = exp(-beta * d * d);
          r = exp(-beta * (2.0 * d * dv + dv * dv));
        } else {
          e *= r;
          r *= qf;
        }
        s0 += e;
        s1 += vnode(i) * e;
        s2 += (vnode(i) * vnode(i)) * e;
      }
      e = ep;
      r = exp(-beta * (dv * dv - 2.0 * dp * dv));
      for (int i = ip - 1; i >= 0; --i) {
        if (((ip - i) & 15) == 0) {
          const double d = vnode(i) - u[a];
          e = exp(-beta * d * d);
          r = exp(-beta * (dv * dv - 2.0 * d * dv));
        } else {
          e *= r;
          r *= qf;
        }
        s0 += e;
        s1 += vnode(i) * e;
        s2 += (vnode(i) * vnode(i)) * e;
      }
      G0[a] = s0;
      G1[a] = s1;
      G2[a] = s2;
    }
    double CM[NM];
    double all0 = 1.0;
#pragma unroll
    for (int a = 0; a < D; ++a) all0 *= G0[a];
    CM[0] = G.w * pref * all0;
    double en = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double oth = 1.0;
#pragma unroll
      for (int b2 = 0; b2 < D; ++b2)
        if (b2 != a) oth *= G0[b2];
      CM[1 + a] = G.w * pref * G1[a] * oth;
      en += G2[a] * oth;
    }
    CM[NM - 1] = G.w * pref * 0.5 * en;
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int s2 = 0; s2 < NM; ++s2) acc += A.a[r * NM + s2] * (Un[s2] - CM[s2]);
      cE[r] = acc;
    }
    const double c = sqrt(G.gam * (rho * th) / rho);
#pragma unroll
    for (int a = 0; a < D; ++a) speed[a] = fabs(u[a]) + c;
  }
  const bool need_eq = G.mu_r != 0.0;
  constexpr int RS = rec_stride<D, T>();
  T rv[RS];
#pragma unroll
  for (int q = 0; q < RS; ++q) rv[q] = (T)0;
  rv[0] = (T)lp;
#pragma unroll
  for (int a = 0; a < D; ++a) rv[1 + a] = (T)u[a];
  rv[D + 1] = (T)(valid ? beta : -beta);  // negative: pieces of this cell not kept
#pragma unroll
  for (int r = 0; r < NM; ++r) {
    rv[NM + r] = (T)(need_eq ? G.w * (G.lam_r * cfv[r] + G.mu_r * cE[r]) : G.w * (G.lam_r * cfv[r]));
    rv[2 * NM + r] = (T)(G.w * cE[r]);
  }
#pragma unroll
  for (int q = 0; q < RS; ++q) rec_j[q] = rv[q];
  return phys;
}

// ================================================================ step
template <typename T>
struct StepArgs {
  const T* g_in;
  T* g_out;
  const T* rec_in;
  T* rec_out;
  const VelNode* vt;
  const double* U_in;
  double* U_out;
  double* UE0;
  double* UE1;
  double* UE2;        // WENO solve: Runge-Kutta stage values (scheme 3 only)
  double* UE3;
  double* cf;
  double* set_r;      // speeds of U^n (row 0) and of the sub-steps; control
  double* set_w;      // speeds of U^{n+1} (row 0), written by the kinetic epilogue
  double* set_z;      // the set of the step after next, cleared by the Euler kernel
  double* bmax;       // [2][GE][ASTR] per-block speed maxima of the Euler sub-steps
  int* flag;
  int nseg, GE, s_cap, unlimited;
  // closure form only
  const unsigned char* mode;  // 1: the cell runs the kinetic step, 0: closure
  const float4* nhat;         // network estimate of the non-equilibrium term
  unsigned char* dfl;         // lam max|delta| / s above thr (kinetic cells)
  float* tgt;                 // optional: training targets N / (lam s) per cell
  unsigned long long* kcount;  // kinetic cell-steps (accumulated)
  double thr;
  double* sums;  // [2 (d+2)][nc]: moment sums of f* and of E, for k_cell_update
  long nstep;    // n of the step t^n -> t^{n+1} (off-lattice shifts)
};

// Euler sub-step i (eq. (discmom) with the flux of section 4.3), one cell per
// thread over the whole grid: sub-step 0 also clears the set of the step
// after next and records s; launches with i >= s return at once.  The
// speeds of the result are reduced per block and folded into row i+1 with
// one atomic maximum per block on slot (block mod NSLOT).  Sub-step i reads
// UE[i % 2] (U^n for i = 0) and writes UE[(i + 1) % 2].
template <int D, typename T>
__global__ __launch_bounds__(256) void k_euler_sub(StepArgs<T> a, Geom G, int i) {
  constexpr int NM = D + 2;
  double* S = a.set_r;
  bool over;
  const int s = substeps<D>(S, G, a.s_cap, &over);
  if (i == 0) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < SET_D; q += gridDim.x * blockDim.x)
      a.set_z[q] = 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (over) atomicOr(a.flag, FLAG_SUBSTEP);
      a.flag[1] = s;
    }
  }
  if (i >= s) return;
  double alpha[3];
  row_speeds<D>(S, i, alpha);
  const double dts_dx = (G.dt / s) / G.dx;
  const double* in = (i == 0) ? a.U_in : ((i & 1) ? a.UE1 : a.UE0);
  double* out = ((i + 1) & 1) ? a.UE1 : a.UE0;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  bool phys = true;
  double mx[3] = {0.0, 0.0, 0.0};
  if (j < G.nc) {
    double Un[NM];
    phys = euler_cell<D>(in, j, alpha, dts_dx, G, a.unlimited, Un);
#pragma unroll
    for (int r = 0; r < NM; ++r) out[(size_t)r * G.nc + j] = Un[r];
    if (i + 1 < s) {
      double sp[3];
      phys &= lf_speeds<D>(Un, G.gam, sp);
#pragma unroll
      for (int d2 = 0; d2 < D; ++d2) mx[d2] = sp[d2];
    }
  }
  if (!phys) atomicOr(a.flag, FLAG_NONPHYS);
  if (i + 1 < s) {
    __shared__ double wm[4][ASTR];
#pragma unroll
    for (int d2 = 0; d2 < D; ++d2) {
      const double m = wave_max(mx[d2]);
      if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6][d2] = m;
    }
    __syncthreads();
    if (threadIdx.x < D) {
      double m = wm[0][threadIdx.x];
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, wm[w][threadIdx.x]);
      atomic_max_pos(speed_row(S, i + 1, blockIdx.x % NSLOT) + threadIdx.x, m);
    }
  }
}

// Euler tail: GE co-resident blocks continue from sub-step K to s when the
// sub-step launches of the step stopped short (grid-strided over cells);
// the speeds of sub-step i+1 are reduced through per-block maxima into slot
// 0 of row i+1 and the blocks meet at a barrier between sub-steps.
template <int D, typename T, int TPB>
__global__ __launch_bounds__(TPB) void k_euler(StepArgs<T> a, Geom G, int K) {
  constexpr int NM = D + 2;
  double* S = a.set_r;
  unsigned* ctrl = reinterpret_cast<unsigned*>(S + SET_CTRL);
  bool over;
  const int s = substeps<D>(S, G, a.s_cap, &over);
  if (K >= s) return;  // the sub-step launches covered every sub-step
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(a.flag + 2, s - K);  // tail sub-steps run
  const double dts_dx = (G.dt / s) / G.dx;
  __shared__ double wmax[TPB / 64][ASTR];
  double alpha[3];
  row_speeds<D>(S, K, alpha);
  for (int i = K; i < s; ++i) {
    const double* in = (i == 0) ? a.U_in : ((i & 1) ? a.UE1 : a.UE0);
    double* out = ((i + 1) & 1) ? a.UE1 : a.UE0;
    bool phys = true;
    double mx[3] = {0.0, 0.0, 0.0};
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < G.nc; j += a.GE * blockDim.x) {
      double Un[NM];
      phys &= euler_cell<D>(in, j, alpha, dts_dx, G, a.unlimited, Un);
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        if (HOFKS_EULER_NT)
          __builtin_nontemporal_store(Un[r], out + (size_t)r * G.nc + j);
        else
          out[(size_t)r * G.nc + j] = Un[r];
      }
      if (i + 1 < s) {
        double sp[3];
        phys &= lf_speeds<D>(Un, G.gam, sp);
#pragma unroll
        for (int d2 = 0; d2 < D; ++d2) mx[d2] = fmax(mx[d2], sp[d2]);
      }
    }
    if (!phys) atomicOr(a.flag, FLAG_NONPHYS);
    if (i + 1 < s) {
      // block maxima into bmax[block]; two-level barrier: blocks arrive on
      // one of 8 group counters, the last of each group on the top counter,
      // and the very last block reduces all maxima into row i+1 of set_r
      // and releases everyone through the generation word
      double* bm = a.bmax;
#pragma unroll
      for (int d2 = 0; d2 < D; ++d2) {
        const double m = wave_max(mx[d2]);
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6][d2] = m;
      }
      __syncthreads();
      if (a.GE == 1) {
        // the whole grid is this block: its maxima are the sub-step's speeds
        // and the block barrier orders the sub-steps (the same values as
        // through the arrival counters)
#pragma unroll
        for (int d2 = 0; d2 < D; ++d2) {
          double m = wmax[0][d2];
          for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, wmax[w][d2]);
          alpha[d2] = m;
        }
        if (threadIdx.x == 0)
#pragma unroll
          for (int d2 = 0; d2 < D; ++d2) speed_row(S, i + 1, 0)[d2] = alpha[d2];
        __syncthreads();
        continue;
      }
      if (threadIdx.x < D) {
        double m = wmax[0][threadIdx.x];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, wmax[w][threadIdx.x]);
        bm[(size_t)blockIdx.x * ASTR + threadIdx.x] = m;
      }
      __syncthreads();
      __shared__ int s_last;
      unsigned* gen = ctrl;  // line 0: generation
      if (threadIdx.x == 0) {
        const unsigned g = blockIdx.x & 7u;
        const unsigned ng = (a.GE - g + 7) / 8;  // blocks in group g
        const unsigned ngroups = a.GE < 8 ? a.GE : 8;
        unsigned* top = ctrl + 16;               // line 1: top counter
        unsigned* sub = ctrl + 32 + 16 * g;      // lines 2..9: group counters
        __threadfence();
        int last = 0;
        const unsigned nb = (unsigned)(i - K + 1);  // barriers of this launch so far
        const unsigned old = atomicAdd(sub, 1u);
        if (old == nb * ng - 1) {
          const unsigned t = atomicAdd(top, 1u);
          last = (t == nb * ngroups - 1);
        }
        s_last = last;
      }
      __syncthreads();
      if (s_last) {  // the whole last block reduces the block maxima
        __threadfence();
        double m[3] = {0.0, 0.0, 0.0};
        for (int b = threadIdx.x; b < a.GE; b += blockDim.x)
#pragma unroll
          for (int d2 = 0; d2 < D; ++d2)
            m[d2] = fmax(m[d2], __hip_atomic_load(bm + (size_t)b * ASTR + d2, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT));
#pragma unroll
        for (int d2 = 0; d2 < D; ++d2) {
          const double w = wave_max(m[d2]);
          if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6][d2] = w;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
#pragma unroll
          for (int d2 = 0; d2 < D; ++d2) {
            double w = wmax[0][d2];
            for (int q = 1; q < (int)(blockDim.x >> 6); ++q) w = fmax(w, wmax[q][d2]);
            __hip_atomic_store(speed_row(S, i + 1, 0) + d2, w, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
          }
          __threadfence();
          __hip_atomic_store(gen, (unsigned)(i - K + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      if (threadIdx.x == 0) {
        spin_until_geq(gen, (unsigned)(i - K + 1), a.flag);
        __threadfence();
#pragma unroll
        for (int d2 = 0; d2 < D; ++d2)
          wmax[0][d2] = __hip_atomic_load(speed_row(S, i + 1, 0) + d2, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
#pragma unroll
      for (int d2 = 0; d2 < D; ++d2) alpha[d2] = wmax[0][d2];
      __syncthreads();
    }
  }
}

// Closure form, per cell after the moment sums: closure cells add the
// network estimate N^ to U^{n+1}; kinetic cells report whether
// lam max|delta| / s exceeds the threshold; a snapshot step stores the
// training target N / (lam s) with N = w (sum f* - sum E), s from U^n.
template <int D, typename T>
__device__ __forceinline__ void closure_epilogue(const StepArgs<T>& a, const Geom& G, int dest,
                                                 bool kin, const double* SK, const double* CK,
                                                 const double* SE, const double* CE, bool comp,
                                                 const double* delta, double* Un) {
  static_assert(D == 2, "closure form is 2D-2V");
  if (!kin) {
    const float4 nh = a.nhat[dest];
    Un[0] += nh.x;
    Un[1] += nh.y;
    Un[2] += nh.z;
    Un[3] += nh.w;
  }
  if (a.tgt) {
    const double rho = a.U_in[dest];
    const double ux = a.U_in[(size_t)G.nc + dest] / rho, uy = a.U_in[2 * (size_t)G.nc + dest] / rho;
    const double En = a.U_in[3 * (size_t)G.nc + dest];
    const double th = (2.0 * En - rho * (ux * ux + uy * uy)) / (2.0 * rho);
    const double c = sqrt(G.gam * th);
    const double sc[4] = {rho, rho * c, rho * c, En};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double N = G.w * ((comp ? SK[r] + CK[r] : SK[r]) - (comp ? SE[r] + CE[r] : SE[r]));
      a.tgt[(size_t)dest * 4 + r] = (float)(N / (G.lam * sc[r]));
    }
  }
  unsigned char df = 0;
  if (kin) {
    const double rho = Un[0];
    const double ux = Un[1] / rho, uy = Un[2] / rho;
    const double th = (2.0 * Un[3] - rho * (ux * ux + uy * uy)) / (2.0 * rho);
    const double c = sqrt(G.gam * th);
    const double sc[4] = {rho, rho * c, rho * c, Un[3]};
    double m = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) m = fmax(m, fabs(delta[r]) / sc[r]);
    df = (unsigned char)!(G.lam * m <= a.thr);
  }
  a.dfl[dest] = df;
}

// wave-local LDS hand-off: LDS operations of one wavefront complete in order;
// this keeps the compiler from moving them across and waits for them
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Record of one upstream cell as the piece loop reads it: the terms of the
// transverse velocities (v_y, v_z: fixed over a velocity row) folded in,
//   [a0, u_x, beta | P0, p_1, p_{d+1} | E0, e_1, e_{d+1}],
//   log M = a0 - |beta| (v_x - u_x)^2,   p . m(v) = P0 + p_1 v_x + p_{d+1} v_x^2 / 2,
// with a0 = lp - |beta| sum_{a>1} (v_a - u_a)^2 and
// P0 = p_0 + sum_{a>1} p_a v_a + p_{d+1} sum_{a>1} v_a^2 / 2 (the same for e).
// In 1D it is the record itself.  Nine values padded to an odd number of
// 16-byte chunks.  A staged row segment holds its cells in reverse order, so
// that the pieces of increasing k_x read increasing addresses (constant
// offsets in the LDS reads).
template <typename T>
__host__ __device__ constexpr int row_rec_stride() {
  return rec_stride<1, T>();
}

// read the nine values of a row record from LDS (16-byte chunks, the last
// partial chunk as single values)
template <typename T>
__device__ __forceinline__ void read_row_rec(const T* p, T (&r)[9]) {
  using V = typename Vec16<T>::type;
  const V* q = reinterpret_cast<const V*>(p);
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const V t = q[c];
      r[2 * c] = t.x;
      r[2 * c + 1] = t.y;
    }
    r[8] = p[8];
  } else {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const V t = q[c];
      r[4 * c] = t.x;
      r[4 * c + 1] = t.y;
      r[4 * c + 2] = t.z;
      r[4 * c + 3] = t.w;
    }
    r[8] = p[8];
  }
}

// velocity node i through the scalar cache (the table is written only when
// a context is created)
__device__ __forceinline__ VelNode vel_node(const VelNode* vt, int i) {
  using CVN = const __attribute__((address_space(4))) VelNode;
  CVN* p = (CVN*)vt + i;
  VelNode r;
  r.v = p->v;
  r.v2 = p->v2;
  r.vf = p->vf;
  r.v2hf = p->v2hf;
  r.v2h = p->v2h;
  return r;
}

// Kinetic kernel.  One block = 64 consecutive x cells of one row (one lane
// per cell) and NG wavefronts, each taking 1/NG of the velocities (of the
// velocity rows (k_y, k_z) in 2D/3D, of k_x in 1D).  Per velocity row a
// wavefront stages the row records of the upstream row segment in its own
// LDS slice; its k_x loop issues UNR piece loads g(j - k, k) (coalesced
// along x) before using them, relaxes each piece, writes it to cell j of the
// new buffer and sums the moments of f* and of E.  The partial sums are
// combined in LDS and written for the per-cell update (k_cell_update; the
// Euler solve runs on another stream meanwhile), or, for steps without an
// Euler solve, the first wavefront forms U^{n+1}, cf and the next record of
// its 64 cells.  (NG, UNR) is chosen per grid by the autotuner.
template <int D, typename T, bool FT, bool COMP, int BCX, int UNR, bool EUL, int NG,
          bool CLOS = false, bool OFFL = false>
__global__ __launch_bounds__(64 * NG) void k_kinetic(StepArgs<T> a, Geom G, Mat A) {
  constexpr int NM = D + 2;
  constexpr int RS = rec_stride<D, T>();
  constexpr int PER16 = 16 / (int)sizeof(T);
  constexpr int NCH = (rec_values<D, T>() + PER16 - 1) / PER16;  // chunks of a record
  constexpr int C16 = RS / PER16;
  constexpr int FS = row_rec_stride<T>();
  using V = typename Vec16<T>::type;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int SW = 64 + G.nv1 - 1;

  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int seg = tile % a.nseg;
  const int row = tile / a.nseg;
  const int lane = threadIdx.x & 63;
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int Nx = G.n[0];
  const int x0 = seg * 64;
  const int x = x0 + lane;
  const bool active = x < Nx;
  const int jy = row % G.n[1], jz = row / G.n[1];
  const int dest = row * Nx + x;
  const unsigned dboff = (unsigned)dest * (unsigned)sizeof(T);
  const int xN = x + Nx;
  const int lofs = G.nv1 - 1 - G.kofs;
  const int xlo = x0 - lofs;
  const T lam = (T)G.lam, mu = (T)G.mu;
  const int nvr = G.nv / G.nv1;
  // closure form: kinetic lanes, and whether any cell of the tile is kinetic
  // (all wavefronts of the block hold the same 64 cells)
  const bool kin = !CLOS || (active && a.mode[dest] != 0);
  const bool tile_kin = !CLOS || __ballot(kin) != 0;
  // velocity rows of this wavefront (2D/3D) or k_x range (1D)
  const int vr0 = (D >= 2) ? grp * nvr / NG : 0;
  const int vr1 = (D >= 2) ? (grp + 1) * nvr / NG : 1;
  const int ixa = (D >= 2) ? 0 : grp * G.nv1 / NG;
  const int ixb = (D >= 2) ? G.nv1 : (grp + 1) * G.nv1 / NG;
  T* Lw = lds + (D >= 2 ? (size_t)grp * SW * FS : 0);

  double SK[NM], SE[NM], CK[NM], CE[NM];
#pragma unroll
  for (int r = 0; r < NM; ++r) SK[r] = SE[r] = CK[r] = CE[r] = 0.0;

  for (int vr = vr0; vr < vr1; ++vr) {
    const int iy = (D >= 2) ? vr % G.nv1 : 0;
    const int iz = (D >= 3) ? vr / G.nv1 : 0;
    const int ky = OFFL ? node_shift(a.vt, iy, G, a.nstep) : iy - G.kofs;
    const int kz = OFFL ? node_shift(a.vt, iz, G, a.nstep) : iz - G.kofs;
    const double vy = (D >= 2) ? vel_node(a.vt, iy).v : 0.0;
    const double vz = (D >= 3) ? vel_node(a.vt, iz).v : 0.0;
    const double hrow = (D >= 2 ? 0.5 * vel_node(a.vt, iy).v2 : 0.0) +
                        (D >= 3 ? 0.5 * vel_node(a.vt, iz).v2 : 0.0);
    const int uy = (D >= 2) ? map_axis(jy - ky, G.n[1], G.bc[1]) : 0;
    const int uz = (D >= 3) ? map_axis(jz - kz, G.n[2], G.bc[2]) : 0;
    const int ubase = (uz * G.n[1] + uy) * Nx;

    // stage the row records of the upstream row segment
    {
      const V* recv = reinterpret_cast<const V*>(a.rec_in);
      if (D >= 2) {
        const T vyT = (T)vy, vzT = (T)vz, hT = (T)hrow;
        wave_lds_sync();
        for (int i = lane; i < SW; i += 64) {
          const V* src = recv + (size_t)(ubase + map_axis(xlo + i, Nx, G.bc[0])) * C16;
          T rv[NCH * PER16];
#pragma unroll
          for (int c = 0; c < NCH; ++c) {
            const V t = src[c];
            if constexpr (sizeof(T) == 8) {
              rv[2 * c] = t.x;
              rv[2 * c + 1] = t.y;
            } else {
              rv[4 * c] = t.x;
              rv[4 * c + 1] = t.y;
              rv[4 * c + 2] = t.z;
              rv[4 * c + 3] = t.w;
            }
          }
          // record: [lp, u_1..u_D, beta | p_0..p_{D+1} | e_0..e_{D+1}]
          const T beta = rv[D + 1];
          const T bq = CLOS ? fabs(beta) : beta;
          T q = (vyT - rv[2]) * (vyT - rv[2]);
          T P0 = rv[NM] + rv[NM + 2] * vyT;
          T E0 = rv[2 * NM] + rv[2 * NM + 2] * vyT;
          if (D >= 3) {
            q += (vzT - rv[3]) * (vzT - rv[3]);
            P0 += rv[NM + 3] * vzT;
            E0 += rv[2 * NM + 3] * vzT;
          }
          P0 += rv[2 * NM - 1] * hT;
          E0 += rv[3 * NM - 1] * hT;
          T* o = Lw + (size_t)(SW - 1 - i) * FS;
          const T f[9] = {rv[0] - bq * q, rv[1], beta, P0, rv[NM + 1], rv[2 * NM - 1],
                          E0, rv[2 * NM + 1], rv[3 * NM - 1]};
          if constexpr (sizeof(T) == 8) {
#pragma unroll
            for (int c = 0; c < 4; ++c) reinterpret_cast<V*>(o)[c] = V{f[2 * c], f[2 * c + 1]};
          } else {
#pragma unroll
            for (int c = 0; c < 2; ++c)
              reinterpret_cast<V*>(o)[c] = V{f[4 * c], f[4 * c + 1], f[4 * c + 2], f[4 * c + 3]};
          }
          o[8] = f[8];
        }
        wave_lds_sync();
      } else {
        // 1D: the record is the row record
        V* ldsv = reinterpret_cast<V*>(Lw);
        for (int idx = threadIdx.x; idx < SW * C16; idx += blockDim.x) {
          const int c = idx % C16, i = idx / C16;
          const int ux = map_axis(xlo + i, Nx, G.bc[0]);
          ldsv[(SW - 1 - i) * C16 + c] = recv[(size_t)ux * C16 + c];
        }
        __syncthreads();
      }
    }
    if (!active) continue;

    const size_t kbase = (size_t)vr * G.nv1;
    double aK0 = 0.0, aK1 = 0.0, aK2 = 0.0, aE0 = 0.0, aE1 = 0.0, aE2 = 0.0;

    if constexpr (CLOS) {
      if (!tile_kin) {
        // closure tile: every piece is the equilibrium of its upstream cell,
        // so only E is evaluated and summed once; the sums of f* equal those
        // of E
        for (int ix0 = ixa; ix0 < ixb; ix0 += UNR) {
          const T* Lb = Lw + (SW - 1 - lane - lofs - G.kofs + ix0) * FS;
#pragma unroll
          for (int u = 0; u < UNR; ++u) {
            const VelNode vn = vel_node(a.vt, ix0 + u);
            const T vxT = (sizeof(T) == 4) ? (T)vn.vf : (T)vn.v;
            const T vhT = (sizeof(T) == 4) ? (T)vn.v2hf : (T)vn.v2h;
            T rr[9];
            read_row_rec<T>(Lb + u * FS, rr);
            const T dx_ = vxT - rr[1];
            const T M = fast_exp<T>(rr[0] - fabs(rr[2]) * (dx_ * dx_));
            const T E = M + (rr[6] + rr[7] * vxT + rr[8] * vhT);
            const double Ed = (double)E;
            aE0 += Ed;
            aE1 += vn.v * Ed;
            aE2 += vn.v2h * Ed;
          }
        }
        aK0 = aE0;
        aK1 = aE1;
        aK2 = aE2;
        goto row_done;
      }
    }
    for (int ix0 = ixa; ix0 < ixb; ix0 += UNR) {
      T gv[UNR];
      int shx[UNR];  // off-lattice: cells moved by each piece of the group
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int ix = ix0 + u;
        const int kx = OFFL ? node_shift(a.vt, ix, G, a.nstep) : ix - G.kofs;
        shx[u] = kx;
        // plane base (uniform) + 32-bit byte offset of the upstream cell
        const char* gp = reinterpret_cast<const char*>(a.g_in + (kbase + ix) * (size_t)G.nc);
        const T* src = reinterpret_cast<const T*>(
            gp + (unsigned)(ubase + map_x<BCX>(xN, kx, Nx)) * (unsigned)sizeof(T));
        if (CLOS && !tile_kin)
          gv[u] = (T)0;
        else if (HOFKS_NT)
          gv[u] = __builtin_nontemporal_load(src);
        else
          gv[u] = *src;
      }
      // row records of the pieces of this group: cell lane - kx + lofs, at
      // position SW - 1 - lane + kx - lofs, for kx = ix0 + u - kofs
      const T* Lb = Lw + (SW - 1 - lane - lofs - G.kofs + ix0) * FS;
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int ix = ix0 + u;
        const VelNode vn = vel_node(a.vt, ix);
        const double vx = vn.v;
        const T vxT = (sizeof(T) == 4) ? (T)vn.vf : (T)vn.v;
        const T vhT = (sizeof(T) == 4) ? (T)vn.v2hf : (T)vn.v2h;
        T rv[9];
        read_row_rec<T>(OFFL ? Lw + (SW - 1 - lane - lofs + shx[u]) * FS : Lb + u * FS, rv);
        // row record: [a0, u_x, beta | P0, p_1, p_{d+1} | E0, e_1, e_{d+1}]
        const T pp = rv[3] + rv[4] * vxT + rv[5] * vhT;
        const T g = gv[u];
        T fs;
        if (FT) {
          fs = g + pp;
        } else {
          const T dx_ = vxT - rv[1];
          const T M = fast_exp<T>(rv[0] - (CLOS ? fabs(rv[2]) : rv[2]) * (dx_ * dx_));
          const T E = M + (rv[6] + rv[7] * vxT + rv[8] * vhT);
          fs = lam * g + (mu * M + pp);
          // closure form: closure cells, and upstream cells without pieces,
          // take the equilibrium
          if (CLOS) fs = (kin && rv[2] > (T)0) ? fs : E;
          const double Ed = (double)E;
          aE0 += Ed;
          aE1 += vx * Ed;
          aE2 += vn.v2h * Ed;
        }
        T* op = reinterpret_cast<T*>(reinterpret_cast<char*>(a.g_out + (kbase + ix) * (size_t)G.nc) +
                                     dboff);
        if (CLOS && !kin) {
        } else if (HOFKS_NT) {
          __builtin_nontemporal_store(fs, op);
        } else {
          *op = fs;
        }
        const double fd = (double)fs;
        aK0 += fd;
        aK1 += vx * fd;
        aK2 += vn.v2h * fd;
      }
    }
  row_done:
    // fold the row into the totals: m = (1, v_x, v_y, v_z, |v|^2/2)
    double rk[NM + 2], re[NM + 2];  // padded: the D >= 3 branch indexes [3]
    rk[0] = aK0;
    rk[1] = aK1;
    re[0] = aE0;
    re[1] = aE1;
    if (D >= 2) {
      rk[2] = vy * aK0;
      re[2] = vy * aE0;
    }
    if (D >= 3) {
      rk[3] = vz * aK0;
      re[3] = vz * aE0;
    }
    rk[NM - 1] = aK2 + hrow * aK0;
    re[NM - 1] = aE2 + hrow * aE0;
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      if (COMP) {
        two_sum(SK[r], CK[r], rk[r]);
        two_sum(SE[r], CE[r], re[r]);
      } else {
        SK[r] += rk[r];
        SE[r] += re[r];
      }
    }
  }

  // ---------------------------------------------- combine the wavefronts
  __syncthreads();
  double* red = reinterpret_cast<double*>(lds_raw);
  if (grp > 0) {
    double* q = red + ((size_t)(grp - 1) * 64 + lane) * (2 * NM);
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      q[r] = COMP ? SK[r] + CK[r] : SK[r];
      q[NM + r] = COMP ? SE[r] + CE[r] : SE[r];
    }
  }
  __syncthreads();
  if (grp != 0) return;
#pragma unroll
  for (int r = 0; r < NM; ++r) {
    if (COMP) {
      SK[r] += CK[r];
      SE[r] += CE[r];
      CK[r] = CE[r] = 0.0;
    }
  }
  for (int g2 = 1; g2 < NG; ++g2) {
    const double* q = red + ((size_t)(g2 - 1) * 64 + lane) * (2 * NM);
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      if (COMP) {
        two_sum(SK[r], CK[r], q[r]);
        two_sum(SE[r], CE[r], q[NM + r]);
      } else {
        SK[r] += q[r];
        SE[r] += q[NM + r];
      }
    }
  }

  if constexpr (EUL) {
    // the Euler solve of the step runs on another stream meanwhile: store the
    // sums; k_cell_update forms delta, U^{n+1}, cf and the next record
    if (active) {
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        a.sums[(size_t)r * G.nc + dest] = COMP ? SK[r] + CK[r] : SK[r];
        a.sums[(size_t)(NM + r) * G.nc + dest] = COMP ? SE[r] + CE[r] : SE[r];
      }
    }
    return;
  }

  // ------------------------------------------------- per-cell update
  const bool need_eq = G.mu != 0.0;
  bool phys = true;
  double speed[3] = {0.0, 0.0, 0.0};
  if (active) {
    double delta[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) delta[r] = 0.0;
    if (EUL) {
      bool over;
      const int s = substeps<D>(a.set_r, G, a.s_cap, &over);
      const double* UEs = (s & 1) ? a.UE1 : a.UE0;
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        const double UM = G.mu * (G.w * (COMP ? SE[r] + CE[r] : SE[r]));
        const double UEv = G.mu * UEs[(size_t)r * G.nc + dest];
        delta[r] = UEv - UM;
      }
    }
    double Un[NM], cfv[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) Un[r] = G.w * (COMP ? SK[r] + CK[r] : SK[r]) + delta[r];
    if constexpr (CLOS) closure_epilogue<D>(a, G, dest, kin, SK, CK, SE, CE, COMP, delta, Un);
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int s2 = 0; s2 < NM; ++s2) acc += A.a[r * NM + s2] * delta[s2];
      cfv[r] = acc;
    }
    phys = cell_record<D, T>(Un, cfv, G, A, a.rec_out + (size_t)dest * RS, speed, kin);
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      a.U_out[(size_t)r * G.nc + dest] = Un[r];
      a.cf[(size_t)r * G.nc + dest] = cfv[r];
    }
  }
  if (active && need_eq && !phys) atomicOr(a.flag, FLAG_NONPHYS);
  if (CLOS) {
    const unsigned long long bk = __ballot(kin);
    if (lane == 0 && grp == 0 && bk) atomicAdd(a.kcount, (unsigned long long)__popcll(bk));
  }
  if (EUL) {
#pragma unroll
    for (int d2 = 0; d2 < D; ++d2) {
      const double m = wave_max(phys ? speed[d2] : 0.0);
      if (lane == 0) atomic_max_pos(a.set_w + d2, m);
    }
  }
}

// Per-cell update of a step after its kinetic sums and its Euler solve
// (eqs. (UK), (mom), (minim_full)): delta = U_E - U_M, U^{n+1} = U_* + U_E,
// cf = A delta, the next record and the speeds of U^{n+1}; in the closure
// form also N^ for closure cells, the delta marks and the kinetic count.
// The per-cell launches give each die a contiguous range of cells (blocks
// reach the dies round-robin), as the kinetic and Euler tiles, so that most
// of what a cell reads was written on its own die.
template <int D, typename T, bool CLOS>
__global__ __launch_bounds__(256) void k_cell_update(StepArgs<T> a, Geom G, Mat A) {
  constexpr int NM = D + 2;
  constexpr int RS = rec_stride<D, T>();
  const int j = xcd_tile(blockIdx.x, gridDim.x) * (int)blockDim.x + threadIdx.x;
  const bool active = j < G.nc;
  const bool kin = !CLOS || (active && a.mode[j] != 0);
  bool phys = true;
  double speed[3] = {0.0, 0.0, 0.0};
  if (active) {
    double SK[NM], SE[NM], Z[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      SK[r] = a.sums[(size_t)r * G.nc + j];
      SE[r] = a.sums[(size_t)(NM + r) * G.nc + j];
      Z[r] = 0.0;
    }
    bool over;
    const int s = substeps<D>(a.set_r, G, a.s_cap, &over);
    const double* UEs = (s & 1) ? a.UE1 : a.UE0;
    double delta[NM], Un[NM], cfv[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      const double UM = G.mu * (G.w * SE[r]);
      const double UEv = G.mu * UEs[(size_t)r * G.nc + j];
      delta[r] = UEv - UM;
    }
#pragma unroll
    for (int r = 0; r < NM; ++r) Un[r] = G.w * SK[r] + delta[r];
    if constexpr (CLOS) closure_epilogue<D>(a, G, j, kin, SK, Z, SE, Z, false, delta, Un);
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int s2 = 0; s2 < NM; ++s2) acc += A.a[r * NM + s2] * delta[s2];
      cfv[r] = acc;
    }
    phys = cell_record<D, T>(Un, cfv, G, A, a.rec_out + (size_t)j * RS, speed, kin);
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      a.U_out[(size_t)r * G.nc + j] = Un[r];
      a.cf[(size_t)r * G.nc + j] = cfv[r];
    }
  }
  if (active && G.mu != 0.0 && !phys) atomicOr(a.flag, FLAG_NONPHYS);
  const int lane = threadIdx.x & 63;
  if (CLOS) {
    const unsigned long long bk = __ballot(kin);
    if (lane == 0 && bk) atomicAdd(a.kcount, (unsigned long long)__popcll(bk));
  }
  // speeds of U^{n+1}: maximum over the block, then one atomic per axis (the
  // atomics of all blocks go to the same address and are serialised there)
  __shared__ double wm[4][ASTR];
#pragma unroll
  for (int d2 = 0; d2 < D; ++d2) {
    const double m = wave_max(phys ? speed[d2] : 0.0);
    if (lane == 0) wm[threadIdx.x >> 6][d2] = m;
  }
  __syncthreads();
  if (threadIdx.x < D) {
    double m = wm[0][threadIdx.x];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, wm[w][threadIdx.x]);
    atomic_max_pos(a.set_w + threadIdx.x, m);
  }
}

// The per-cell update in two launches, so that the Euler solve of the next
// step (which needs U^{n+1} and its speeds only) can start while the next
// records are formed.  First: delta, U^{n+1}, cf and the speeds of U^{n+1}
// (the same formulas as `k_cell_update`; |u_a| + c as in `lf_speeds`).
template <int D, typename T>
__global__ __launch_bounds__(256) void k_cell_update_u(StepArgs<T> a, Geom G, Mat A) {
  constexpr int NM = D + 2;
  const int j = xcd_tile(blockIdx.x, gridDim.x) * (int)blockDim.x + threadIdx.x;
  const bool active = j < G.nc;
  bool phys = true;
  double speed[3] = {0.0, 0.0, 0.0};
  if (active) {
    double SK[NM], SE[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      SK[r] = a.sums[(size_t)r * G.nc + j];
      SE[r] = a.sums[(size_t)(NM + r) * G.nc + j];
    }
    bool over;
    const int s = substeps<D>(a.set_r, G, a.s_cap, &over);
    const double* UEs = (s & 1) ? a.UE1 : a.UE0;
    double delta[NM], Un[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      const double UM = G.mu * (G.w * SE[r]);
      const double UEv = G.mu * UEs[(size_t)r * G.nc + j];
      delta[r] = UEv - UM;
    }
#pragma unroll
    for (int r = 0; r < NM; ++r) Un[r] = G.w * SK[r] + delta[r];
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int s2 = 0; s2 < NM; ++s2) acc += A.a[r * NM + s2] * delta[s2];
      a.U_out[(size_t)r * G.nc + j] = Un[r];
      a.cf[(size_t)r * G.nc + j] = acc;
    }
    phys = lf_speeds<D>(Un, G.gam, speed);
  }
  if (active && G.mu != 0.0 && !phys) atomicOr(a.flag, FLAG_NONPHYS);
  const int lane = threadIdx.x & 63;
  __shared__ double wm[4][ASTR];
#pragma unroll
  for (int d2 = 0; d2 < D; ++d2) {
    const double m = wave_max(phys ? speed[d2] : 0.0);
    if (lane == 0) wm[threadIdx.x >> 6][d2] = m;
  }
  __syncthreads();
  if (threadIdx.x < D) {
    double m = wm[0][threadIdx.x];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, wm[w][threadIdx.x]);
    atomic_max_pos(a.set_w + threadIdx.x, m);
  }
}

// Second: the next record of every cell from U^{n+1} and cf.
template <int D, typename T>
__global__ __launch_bounds__(256) void k_cell_record(StepArgs<T> a, Geom G, Mat A) {
  constexpr int NM = D + 2;
  constexpr int RS = rec_stride<D, T>();
  const int j = xcd_tile(blockIdx.x, gridDim.x) * (int)blockDim.x + threadIdx.x;
  if (j >= G.nc) return;
  double Un[NM], cfv[NM], speed[3];
#pragma unroll
  for (int r = 0; r < NM; ++r) {
    Un[r] = a.U_out[(size_t)r * G.nc + j];
    cfv[r] = a.cf[(size_t)r * G.nc + j];
  }
  (void)cell_record<D, T>(Un, cfv, G, A, a.rec_out + (size_t)j * RS, speed, true);
}

// ======================================================= set-up / refresh
// MODE_INIT: U given, the pieces g hold sampled values with sums S (chunk 0
// of part): project onto U as in eq. (minim1), cf = A (U - w S).
// MODE_INIT_FROM_SUMS: U = w S (cf = 0).  MODE_REFRESH: U and cf given
// (after a change of tau).  Writes the record and the speeds of U (row 0 of
// `set`).
template <int D, typename T>
__global__ __launch_bounds__(256) void k_cell_init(double* __restrict__ U, double* __restrict__ cf,
                                                   T* __restrict__ rec,
                                                   const VelNode* __restrict__ vt,
                                                   const double* __restrict__ part,
                                                   double* __restrict__ set, int* __restrict__ flag,
                                                   Geom G, Mat A, int mode) {
  constexpr int NM = D + 2;
  constexpr int RS = rec_stride<D, T>();
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = j < G.nc;
  bool phys = true;
  double speed[3] = {0.0, 0.0, 0.0};
  if (act) {
    double Un[NM], cfv[NM];
    if (mode == MODE_REFRESH || mode == MODE_RETAU) {
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        Un[r] = U[(size_t)r * G.nc + j];
        cfv[r] = cf[(size_t)r * G.nc + j];
      }
    } else {
      double S[NM];
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        S[r] = part[(size_t)r * G.nc + j];
        Un[r] = (mode == MODE_INIT) ? U[(size_t)r * G.nc + j] : G.w * S[r];
      }
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int s2 = 0; s2 < NM; ++s2) acc += A.a[r * NM + s2] * (Un[s2] - G.w * S[s2]);
        cfv[r] = acc;
      }
    }
    const bool valid = mode != MODE_RETAU || !(rec[(size_t)j * RS + D + 1] < (T)0);
    phys = cell_record<D, T>(Un, cfv, G, A, rec + (size_t)j * RS, speed, valid);
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      U[(size_t)r * G.nc + j] = Un[r];
      cf[(size_t)r * G.nc + j] = cfv[r];
    }
  }
  if (act && (G.mu != 0.0 || mode == MODE_INIT) && !phys) atomicOr(flag, FLAG_NONPHYS);
#pragma unroll
  for (int d2 = 0; d2 < D; ++d2) {
    const double m = wave_max(phys ? speed[d2] : 0.0);
    if ((threadIdx.x & 63) == 0) atomic_max_pos(set + d2, m);
  }
}

// ============================================================ set-up kernels
template <int D>
__global__ void k_prim_to_moments(const double* __restrict__ prim, double* __restrict__ U,
                                  int nc) {
  constexpr int NM = D + 2;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nc) return;
  const double rho = prim[j], th = prim[(size_t)(D + 1) * nc + j];
  double usq = 0.0;
  U[j] = rho;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double ua = prim[(size_t)(1 + a) * nc + j];
    U[(size_t)(1 + a) * nc + j] = rho * ua;
    usq += ua * ua;
  }
  U[(size_t)(NM - 1) * nc + j] = 0.5 * rho * usq + 0.5 * D * rho * th;
}

// g(j,k) = M_k of cell j (the pointwise Maxwellian of the record)
template <int D, typename T>
__global__ void k_fill_maxwellian(T* __restrict__ g, const T* __restrict__ rec, Geom G) {
  constexpr int RS = rec_stride<D, T>();
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)G.nv * G.nc) return;
  const int j = (int)(idx % G.nc);
  int k = (int)(idx / G.nc);
  double q = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double v = (k % G.nv1 - G.kofs) * G.dv;
    k /= G.nv1;
    const double d = v - (double)rec[(size_t)j * RS + 1 + a];
    q += d * d;
  }
  g[idx] = (T)exp((double)rec[(size_t)j * RS] - (double)rec[(size_t)j * RS + D + 1] * q);
}

// S_r(j) = sum_k m_k[r] g(j,k) into part chunk 0
template <int D, typename T>
__global__ void k_piece_sums(const T* __restrict__ g, double* __restrict__ part, Geom G) {
  constexpr int NM = D + 2;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= G.nc) return;
  double S[NM];
#pragma unroll
  for (int r = 0; r < NM; ++r) S[r] = 0.0;
  for (int k = 0; k < G.nv; ++k) {
    const double val = (double)g[(size_t)k * G.nc + j];
    int kk = k;
    double vsq = 0.0;
    S[0] += val;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double v = (kk % G.nv1 - G.kofs) * G.dv;
      kk /= G.nv1;
      S[1 + a] += v * val;
      vsq += v * v;
    }
    S[NM - 1] += 0.5 * vsq * val;
  }
#pragma unroll
  for (int r = 0; r < NM; ++r) part[(size_t)r * G.nc + j] = S[r];
}

// out(j, k) = g(j,k) + w m_k . cf(j) for planes [k0, k0 + nk); with `rec`
// given, cells whose record marks their pieces as not kept (closure form)
// give their equilibrium E(j, k) instead
template <int D, typename T>
__global__ void k_materialize(const T* __restrict__ g, const double* __restrict__ cf,
                              double* __restrict__ out, int k0, int nk, Geom G,
                              const T* __restrict__ rec = nullptr, double blend = 1.0,
                              const T* __restrict__ rec_e = nullptr) {
  constexpr int NM = D + 2;
  constexpr int RS = rec_stride<D, T>();
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nk * G.nc) return;
  const int j = (int)(idx % G.nc);
  int k = k0 + (int)(idx / G.nc);
  const bool eq = rec && rec[(size_t)j * RS + D + 1] < (T)0;
  double corr = eq ? (double)rec[(size_t)j * RS + 2 * NM] : cf[j], vsq = 0.0, q = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double v = (k % G.nv1 - G.kofs) * G.dv;
    k /= G.nv1;
    if (eq) {
      corr += v * (double)rec[(size_t)j * RS + 2 * NM + 1 + a];
      const double du = v - (double)rec[(size_t)j * RS + 1 + a];
      q += du * du;
    } else {
      corr += v * cf[(size_t)(1 + a) * G.nc + j];
    }
    vsq += v * v;
  }
  if (eq) {  // e = w cE is stored, so no factor w here
    corr += 0.5 * vsq * (double)rec[(size_t)j * RS + 3 * NM - 1];
    const double M = exp((double)rec[(size_t)j * RS] + (double)rec[(size_t)j * RS + D + 1] * q);
    out[idx] = M + corr;
    return;
  }
  corr += 0.5 * vsq * cf[(size_t)(NM - 1) * G.nc + j];
  const double fv = (double)g[(size_t)(k0 + (int)(idx / G.nc)) * G.nc + j] + G.w * corr;
  if (!rec_e) {
    out[idx] = fv;
    return;
  }
  // Strang splitting: the pending half relaxation towards E of U^n,
  // E = exp(lp - beta |v - u|^2) + e . m(v) from the record of the cell
  const T* r = rec_e + (size_t)j * RS;
  int kk = k0 + (int)(idx / G.nc);
  double qq = 0.0, ec = (double)r[2 * NM], v2 = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double v = (kk % G.nv1 - G.kofs) * G.dv;
    kk /= G.nv1;
    const double du = v - (double)r[1 + a];
    qq += du * du;
    ec += v * (double)r[2 * NM + 1 + a];
    v2 += v * v;
  }
  ec += 0.5 * v2 * (double)r[3 * NM - 1];
  const double E = exp((double)r[0] - (double)r[D + 1] * qq) + ec;
  out[idx] = blend == 0.0 ? E : blend * fv + (1.0 - blend) * E;
}

// g planes [k0, k0+nk) <- FP64 staging (storage precision conversion)
template <typename T>
__global__ void k_store_planes(T* __restrict__ g, const double* __restrict__ src, size_t count) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) g[idx] = (T)src[idx];
}

__global__ void k_zero(double* __restrict__ p, size_t n) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) p[idx] = 0.0;
}

__global__ void k_zero_int(int* __restrict__ p, int n) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) p[idx] = 0;
}

}  // namespace hofks
