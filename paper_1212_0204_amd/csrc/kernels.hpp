// kernels.hpp -- gfx950 kernels of one HOFKS time step (arXiv:1212.0204).
//
// Data kept resident in HBM between steps (all component-major, cells
// x-fastest):
//   g[k][j]   pieces of the distribution, one plane per velocity node k
//             (FP64, or FP32 in the precision form).  The true distribution is
//             f(j,k) = g(j,k) + w m_k . cf(j): the consistency correction of
//             eq. (minim_full) is kept as d+2 coefficients per cell and applied
//             when the piece is next read, so every step reads and writes each
//             piece exactly once.
//   U[r][j]   moments U^n (FP64).
//   cf[r][j]  pending correction coefficients (C C^T)^{-1}(U_E - U_M).
//   rec[q][j] per-cell record read by the pieces that leave cell j:
//             q = 0 .. d+1         log prefactor, u_1..u_d, beta = 1/(2 theta)
//             q = d+2 .. 2d+3      p = w (lambda cf + (1-lambda) cE)
//             q = 2d+4 .. 3d+5     e = w cE
//             with cE = (C C^T)^{-1}(U - C M) the conservative correction of
//             eq. (minimMax); a piece of velocity v leaving cell j' relaxes to
//               f* = lambda g + (1-lambda) M + p.m(v),
//               E  = M + e.m(v),  M = exp(lp - beta |v - u|^2).
// Per step: k_muscl (s sub-steps of eq. discmom on U^n), k_kinetic (relax +
// shift + moment sums over all velocities of every cell), k_cell_update
// (delta, U^{n+1}, cf, the next records and the next Lax-Friedrichs speeds).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hofks {

constexpr int SMAX = 512;  // largest Euler sub-step count a plan may use
constexpr int SLOT_STRIDE = 4;
constexpr int FLAG_NONPHYS = 1;
constexpr int FLAG_SUBSTEP = 2;

struct Geom {
  int n[3];
  int nc;
  int nv1, kofs, nv;  // nodes per axis, k_a = i_a - kofs, total nodes
  int bc[3];          // 0 periodic, 1 outflow
  double dx, dv, dt, w, lam, mu, gam;
};

struct Mat {
  double a[25];
};

enum { MODE_STEP = 0, MODE_INIT = 1, MODE_INIT_FROM_SUMS = 2, MODE_REFRESH = 3 };

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int map_axis(int i, int N, int bc) {
  if (bc == 0) {
    i %= N;
    return i < 0 ? i + N : i;
  }
  return i < 0 ? 0 : (i >= N ? N - 1 : i);
}

// |i - in-range| <= N guaranteed by the plan
__device__ __forceinline__ int map_near(int i, int N, int bc) {
  if (bc == 0) return i < 0 ? i + N : (i >= N ? i - N : i);
  return i < 0 ? 0 : (i >= N ? N - 1 : i);
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

// Euler sub-step count of a step, from the speeds of U^n (same rule as the
// oracle: s = max(1, ceil(2 dt sum_a alpha_a / dx)))
template <int D>
__device__ __forceinline__ int substeps(const double* alpha0, const Geom& G, int s_cap,
                                        bool* over) {
  double sum = 0.0;
  for (int a = 0; a < D; ++a) sum += alpha0[a];
  double sv = ceil(2.0 * G.dt * sum / G.dx);
  int s = (sv >= 1.0) ? (sv <= (double)s_cap ? (int)sv : s_cap + 1) : 1;
  *over = (s > s_cap);
  return s > s_cap ? s_cap : s;
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

// ===================================================================== MUSCL
// Section 4.3.2: flux-split Lax-Friedrichs with Van Leer limited slopes of
// W+- = F +- alpha U, unsplit over the d directions, forward Euler in time.

template <int D>
__device__ __forceinline__ bool euler_flux(const double* U, int a, double gam, double* F,
                                           double* speed) {
  constexpr int NM = D + 2;
  double rho = U[0], usq = 0.0, u[3];
#pragma unroll
  for (int b = 0; b < D; ++b) {
    u[b] = U[1 + b] / rho;
    usq += u[b] * u[b];
  }
  double th = (2.0 * U[NM - 1] - rho * usq) / (D * rho);
  double p = rho * th;
  F[0] = U[1 + a];
#pragma unroll
  for (int b = 0; b < D; ++b) F[1 + b] = U[1 + b] * u[a] + (a == b ? p : 0.0);
  F[NM - 1] = (U[NM - 1] + p) * u[a];
  if (speed) *speed = fabs(u[a]) + sqrt(gam * p / rho);
  return (rho > 0.0) && (th > 0.0) && isfinite(rho) && isfinite(th) && isfinite(usq);
}

__device__ __forceinline__ double vl_slope(double a, double b, int unlimited) {
  if (unlimited) return b;
  double ab = a * b;
  return ab > 0.0 ? 2.0 * ab / (a + b) : 0.0;
}

// flux through a face from the four cells around it (indices 0..3 of Uq/Fq)
template <int NM>
__device__ __forceinline__ void face_flux(const double (*Uq)[NM], const double (*Fq)[NM],
                                          double alpha, int unl, double* psi) {
#pragma unroll
  for (int r = 0; r < NM; ++r) {
    double wp0 = Fq[0][r] + alpha * Uq[0][r], wp1 = Fq[1][r] + alpha * Uq[1][r],
           wp2 = Fq[2][r] + alpha * Uq[2][r];
    double wm1 = Fq[1][r] - alpha * Uq[1][r], wm2 = Fq[2][r] - alpha * Uq[2][r],
           wm3 = Fq[3][r] - alpha * Uq[3][r];
    double sp = vl_slope(wp1 - wp0, wp2 - wp1, unl);
    double sm = vl_slope(wm2 - wm1, wm3 - wm2, unl);
    psi[r] = 0.5 * (Fq[1][r] + Fq[2][r]) - 0.5 * alpha * (Uq[2][r] - Uq[1][r]) +
             0.25 * (sp - sm);
  }
}

// one Euler sub-step i of the current step (slot set `set`)
template <int D>
__global__ __launch_bounds__(256) void k_muscl(const double* __restrict__ U,
                                               double* __restrict__ UE0,
                                               double* __restrict__ UE1,
                                               double* __restrict__ slots, int set, int i,
                                               int s_cap, int* __restrict__ flag, Geom G,
                                               int unlimited) {
  constexpr int NM = D + 2;
  double* srow = slots + (size_t)set * (SMAX + 1) * SLOT_STRIDE;
  bool over;
  const int s = substeps<D>(srow, G, s_cap, &over);
  if (i >= s) return;
  const double* in = (i == 0) ? U : ((i & 1) ? UE1 : UE0);
  double* out = ((i + 1) & 1) ? UE1 : UE0;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const double dts = G.dt / s;
  bool phys = true;
  double speed_out[3] = {0.0, 0.0, 0.0};
  if (j < G.nc) {
    int c[3] = {j % G.n[0], (j / G.n[0]) % G.n[1], j / (G.n[0] * G.n[1])};
    double div[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) div[r] = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double alpha = srow[i * SLOT_STRIDE + a];
      double Uq[5][NM], Fq[5][NM];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        int cc[3] = {c[0], c[1], c[2]};
        cc[a] = map_axis(c[a] + q - 2, G.n[a], G.bc[a]);
        int jj = (cc[2] * G.n[1] + cc[1]) * G.n[0] + cc[0];
#pragma unroll
        for (int r = 0; r < NM; ++r) Uq[q][r] = in[(size_t)r * G.nc + jj];
        phys &= euler_flux<D>(Uq[q], a, G.gam, Fq[q], nullptr);
      }
      double pl[NM], pr[NM];
      face_flux<NM>(Uq, Fq, alpha, unlimited, pl);          // face j-1/2
      face_flux<NM>(Uq + 1, Fq + 1, alpha, unlimited, pr);  // face j+1/2
#pragma unroll
      for (int r = 0; r < NM; ++r) div[r] += pr[r] - pl[r];
    }
    double Un[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      Un[r] = in[(size_t)r * G.nc + j] - dts / G.dx * div[r];
      out[(size_t)r * G.nc + j] = Un[r];
    }
    if (i + 1 < s) {
      double F[NM];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double sp;
        phys &= euler_flux<D>(Un, a, G.gam, F, &sp);
        speed_out[a] = phys ? sp : 0.0;
      }
    }
  }
  if (!phys) atomicOr(flag, FLAG_NONPHYS);
  if (i + 1 < s) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double m = wave_max(speed_out[a]);
      if ((threadIdx.x & 63) == 0) atomic_max_pos(srow + (i + 1) * SLOT_STRIDE + a, m);
    }
  }
}

// =================================================================== kinetic
// One block = TX x TR destination cells (TX consecutive x, TR rows), one
// chunk of velocity rows.  For every velocity row (k_y, k_z) the records of
// the upstream row segment are staged in LDS; the inner loop over k_x reads
// the piece g(j - k, k) (coalesced along x), relaxes it, writes it to cell j
// of the new buffer and accumulates the moment sums of f* and of E.
template <int D, typename T, bool FT, bool COMP>
__global__ __launch_bounds__(256) void k_kinetic(const T* __restrict__ g_in,
                                                 T* __restrict__ g_out,
                                                 const T* __restrict__ rec,
                                                 double* __restrict__ part,
                                                 double* __restrict__ zero_slots, Geom G,
                                                 int TX, int TR, int nseg, int nrowgrp,
                                                 int nchunk, int nvr) {
  constexpr int NM = D + 2;
  constexpr int R = 3 * NM;
  extern __shared__ unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int SW = TX + G.nv1 - 1;

  if (zero_slots != nullptr && blockIdx.x == 0) {
    for (int q = threadIdx.x; q < (SMAX + 1) * SLOT_STRIDE; q += blockDim.x) zero_slots[q] = 0.0;
  }

  int b = blockIdx.x;
  const int seg = b % nseg;
  b /= nseg;
  const int rg = b % nrowgrp;
  const int chunk = b / nrowgrp;
  const int tx = threadIdx.x % TX, tr = threadIdx.x / TX;
  const int x0 = seg * TX;
  const int x = x0 + tx;
  const int nrows = G.n[1] * G.n[2];
  const int row = rg * TR + tr;
  const bool active = (x < G.n[0]) && (row < nrows) && (tr < TR);
  const int jy = active ? row % G.n[1] : 0;
  const int jz = active ? row / G.n[1] : 0;
  const int dest = row * G.n[0] + x;
  const int vr0 = (int)((long)chunk * nvr / nchunk);
  const int vr1 = (int)((long)(chunk + 1) * nvr / nchunk);
  const int xlo = x0 - (G.nv1 - 1 - G.kofs);
  const int lofs = G.nv1 - 1 - G.kofs;

  double SK[NM], SE[NM], CK[NM], CE[NM];
#pragma unroll
  for (int r = 0; r < NM; ++r) SK[r] = SE[r] = CK[r] = CE[r] = 0.0;

  for (int vr = vr0; vr < vr1; ++vr) {
    const int iy = (D >= 2) ? vr % G.nv1 : 0;
    const int iz = (D >= 3) ? vr / G.nv1 : 0;
    const int ky = iy - G.kofs, kz = iz - G.kofs;
    const double vy = (D >= 2) ? ky * G.dv : 0.0;
    const double vz = (D >= 3) ? kz * G.dv : 0.0;
    const double hrow = 0.5 * (vy * vy + vz * vz);

    __syncthreads();
    for (int idx = threadIdx.x; idx < TR * SW; idx += blockDim.x) {
      const int r_ = idx / SW, i = idx - r_ * SW;
      const int rw = rg * TR + r_;
      if (rw < nrows) {
        const int ry = rw % G.n[1], rz = rw / G.n[1];
        const int uy = (D >= 2) ? map_axis(ry - ky, G.n[1], G.bc[1]) : 0;
        const int uz = (D >= 3) ? map_axis(rz - kz, G.n[2], G.bc[2]) : 0;
        const int ux = map_axis(xlo + i, G.n[0], G.bc[0]);
        const int cell = (uz * G.n[1] + uy) * G.n[0] + ux;
#pragma unroll
        for (int q = 0; q < R; ++q) lds[(r_ * R + q) * SW + i] = rec[(size_t)q * G.nc + cell];
      }
    }
    __syncthreads();
    if (!active) continue;

    const int uy = (D >= 2) ? map_axis(jy - ky, G.n[1], G.bc[1]) : 0;
    const int uz = (D >= 3) ? map_axis(jz - kz, G.n[2], G.bc[2]) : 0;
    const int ubase = (uz * G.n[1] + uy) * G.n[0];
    const T* L = lds + tr * R * SW;
    const size_t kbase = (size_t)vr * G.nv1;
    const T lam = (T)G.lam, mu = (T)G.mu;
    const T vyT = (T)vy, vzT = (T)vz;
    double aK0 = 0.0, aK1 = 0.0, aK2 = 0.0, aE0 = 0.0, aE1 = 0.0, aE2 = 0.0;

    for (int ix = 0; ix < G.nv1; ++ix) {
      const int kx = ix - G.kofs;
      const double vx = kx * G.dv;
      const int li = tx - kx + lofs;
      const int xs = map_near(x - kx, G.n[0], G.bc[0]);
      const size_t plane = (kbase + ix) * (size_t)G.nc;
      const T g = g_in[plane + ubase + xs];
      const T vxT = (T)vx;
      const T vhT = (T)(hrow + 0.5 * vx * vx);
      // pending correction + relaxation poly p.m(v)
      T pp = L[(NM + 0) * SW + li] + L[(NM + 1) * SW + li] * vxT;
      if (D >= 2) pp += L[(NM + 2) * SW + li] * vyT;
      if (D >= 3) pp += L[(NM + 3) * SW + li] * vzT;
      pp += L[(2 * NM - 1) * SW + li] * vhT;
      T fs;
      if (FT) {
        fs = g + pp;
      } else {
        T q = (vxT - L[1 * SW + li]) * (vxT - L[1 * SW + li]);
        if (D >= 2) q += (vyT - L[2 * SW + li]) * (vyT - L[2 * SW + li]);
        if (D >= 3) q += (vzT - L[3 * SW + li]) * (vzT - L[3 * SW + li]);
        const T M = fast_exp<T>(L[0 * SW + li] - L[(D + 1) * SW + li] * q);
        T pe = L[(2 * NM + 0) * SW + li] + L[(2 * NM + 1) * SW + li] * vxT;
        if (D >= 2) pe += L[(2 * NM + 2) * SW + li] * vyT;
        if (D >= 3) pe += L[(2 * NM + 3) * SW + li] * vzT;
        pe += L[(3 * NM - 1) * SW + li] * vhT;
        const T E = M + pe;
        fs = lam * g + (mu * M + pp);
        const double Ed = (double)E;
        aE0 += Ed;
        aE1 += vx * Ed;
        aE2 += (vx * vx) * Ed;
      }
      g_out[plane + dest] = fs;
      const double fd = (double)fs;
      aK0 += fd;
      aK1 += vx * fd;
      aK2 += (vx * vx) * fd;
    }
    // fold the row into the totals: m = (1, v_x, v_y, v_z, |v|^2/2)
    double rk[NM], re[NM];
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
    rk[NM - 1] = 0.5 * aK2 + hrow * aK0;
    re[NM - 1] = 0.5 * aE2 + hrow * aE0;
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
  if (!active) return;
  double* P = part + (size_t)chunk * 2 * NM * G.nc;
#pragma unroll
  for (int r = 0; r < NM; ++r) {
    P[(size_t)r * G.nc + dest] = COMP ? SK[r] + CK[r] : SK[r];
    if (!FT) P[(size_t)(NM + r) * G.nc + dest] = COMP ? SE[r] + CE[r] : SE[r];
  }
}

// =============================================================== cell update
// Per cell: sums of the velocity chunks -> U_K, U_M; delta = U_E - U_M;
// U^{n+1} = U_K + delta (= U_* + U_E); cf = A delta; then the record of the
// new state (Maxwellian parameters, separable discrete moments C M, cE) and
// the Lax-Friedrichs speeds of U^{n+1} for the next Euler solve.
template <int D, typename T>
__global__ __launch_bounds__(256) void k_cell_update(
    double* __restrict__ U, double* __restrict__ cf, double* __restrict__ rec,
    T* __restrict__ recT, const double* __restrict__ part, int nchunk,
    const double* __restrict__ UE0, const double* __restrict__ UE1, double* __restrict__ slots,
    int set, int aset, int s_cap, int* __restrict__ flag, Geom G, Mat A, int mode, int fks) {
  constexpr int NM = D + 2;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = j < G.nc;
  const bool need_eq = G.mu != 0.0;
  bool phys = true;
  double speed[3] = {0.0, 0.0, 0.0};
  if (act) {
    double Un[NM], cfv[NM];
    if (mode == MODE_STEP) {
      double SK[NM], SE[NM];
#pragma unroll
      for (int r = 0; r < NM; ++r) SK[r] = SE[r] = 0.0;
      for (int c = 0; c < nchunk; ++c) {
        const double* P = part + (size_t)c * 2 * NM * G.nc;
#pragma unroll
        for (int r = 0; r < NM; ++r) {
          SK[r] += P[(size_t)r * G.nc + j];
          if (need_eq) SE[r] += P[(size_t)(NM + r) * G.nc + j];
        }
      }
      double delta[NM];
      if (!need_eq) {
#pragma unroll
        for (int r = 0; r < NM; ++r) delta[r] = 0.0;
      } else if (fks) {
#pragma unroll
        for (int r = 0; r < NM; ++r) delta[r] = 0.0;
      } else {
        bool over;
        const int s = substeps<D>(slots + (size_t)set * (SMAX + 1) * SLOT_STRIDE, G, s_cap, &over);
        if (over && j == 0) atomicOr(flag, FLAG_SUBSTEP);
        if (j == 0) flag[1] = s;
        const double* UEs = (s & 1) ? UE1 : UE0;
#pragma unroll
        for (int r = 0; r < NM; ++r) {
          double UM = G.mu * (G.w * SE[r]);
          double UEv = G.mu * UEs[(size_t)r * G.nc + j];
          delta[r] = UEv - UM;
        }
      }
#pragma unroll
      for (int r = 0; r < NM; ++r) Un[r] = G.w * SK[r] + delta[r];
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int s2 = 0; s2 < NM; ++s2) acc += A.a[r * NM + s2] * delta[s2];
        cfv[r] = acc;
      }
    } else if (mode == MODE_REFRESH) {
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        Un[r] = U[(size_t)r * G.nc + j];
        cfv[r] = cf[(size_t)r * G.nc + j];
      }
    } else {
      // MODE_INIT: U given; MODE_INIT_FROM_SUMS: U = w S.  The pieces g hold
      // sampled values whose sums S are in chunk 0 of part; project them onto
      // U as in eq. (minim1): cf = A (U - w S).
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

    // Maxwellian parameters of U^{n+1} (eq. M with theta from eq. E)
    const double rho = Un[0];
    double u[3] = {0.0, 0.0, 0.0}, usq = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      u[a] = Un[1 + a] / rho;
      usq += u[a] * u[a];
    }
    const double th = (2.0 * Un[NM - 1] - rho * usq) / (D * rho);
    phys = (rho > 0.0) && (th > 0.0) && isfinite(rho) && isfinite(th) && isfinite(usq);
    double lp = 0.0, beta = 0.0, cE[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) cE[r] = 0.0;
    if (phys) {
      beta = 0.5 / th;
      const double pref = rho * pow(2.0 * M_PI * th, -0.5 * D);
      lp = log(rho) - 0.5 * D * log(2.0 * M_PI * th);
      // separable discrete moments of the Maxwellian: sums along each axis
      double G0[3], G1[3], G2[3];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int i = 0; i < G.nv1; ++i) {
          const double v = (i - G.kofs) * G.dv;
          const double e = exp(-beta * (v - u[a]) * (v - u[a]));
          s0 += e;
          s1 += v * e;
          s2 += v * v * e;
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
      const double p = rho * th;
#pragma unroll
      for (int a = 0; a < D; ++a) speed[a] = fabs(u[a]) + sqrt(G.gam * p / rho);
    }
    // record
    double rv[3 * NM];
    rv[0] = lp;
#pragma unroll
    for (int a = 0; a < D; ++a) rv[1 + a] = u[a];
    rv[D + 1] = beta;
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      rv[NM + r] = need_eq ? G.w * (G.lam * cfv[r] + G.mu * cE[r]) : G.w * (G.lam * cfv[r]);
      rv[2 * NM + r] = G.w * cE[r];
    }
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      U[(size_t)r * G.nc + j] = Un[r];
      cf[(size_t)r * G.nc + j] = cfv[r];
    }
#pragma unroll
    for (int q = 0; q < 3 * NM; ++q) {
      rec[(size_t)q * G.nc + j] = rv[q];
      if (recT != nullptr) recT[(size_t)q * G.nc + j] = (T)rv[q];
    }
  }
  if (act && (need_eq || mode == MODE_INIT) && !phys) atomicOr(flag, FLAG_NONPHYS);
  if (need_eq && !fks) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double m = wave_max(phys ? speed[a] : 0.0);
      if ((threadIdx.x & 63) == 0)
        atomic_max_pos(slots + (size_t)aset * (SMAX + 1) * SLOT_STRIDE + a, m);
    }
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
__global__ void k_fill_maxwellian(T* __restrict__ g, const double* __restrict__ rec, Geom G) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)G.nv * G.nc) return;
  const int j = (int)(idx % G.nc);
  int k = (int)(idx / G.nc);
  double q = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double v = (k % G.nv1 - G.kofs) * G.dv;
    k /= G.nv1;
    const double d = v - rec[(size_t)(1 + a) * G.nc + j];
    q += d * d;
  }
  g[idx] = (T)exp(rec[j] - rec[(size_t)(D + 1) * G.nc + j] * q);
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

// out(j, k) = g(j,k) + w m_k . cf(j) for planes [k0, k0 + nk)
template <int D, typename T>
__global__ void k_materialize(const T* __restrict__ g, const double* __restrict__ cf,
                              double* __restrict__ out, int k0, int nk, Geom G) {
  constexpr int NM = D + 2;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nk * G.nc) return;
  const int j = (int)(idx % G.nc);
  int k = k0 + (int)(idx / G.nc);
  double corr = cf[j], vsq = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double v = (k % G.nv1 - G.kofs) * G.dv;
    k /= G.nv1;
    corr += v * cf[(size_t)(1 + a) * G.nc + j];
    vsq += v * v;
  }
  corr += 0.5 * vsq * cf[(size_t)(NM - 1) * G.nc + j];
  out[idx] = (double)g[(size_t)(k0 + (int)(idx / G.nc)) * G.nc + j] + G.w * corr;
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
