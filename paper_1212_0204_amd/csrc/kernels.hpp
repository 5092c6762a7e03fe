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
// One launch of k_step advances one time step: its first blocks run the s
// Euler sub-steps of eq. (discmom) on U^n (grid barrier between sub-steps),
// the other blocks relax, shift and sum the pieces tile by tile, and the last
// velocity chunk to finish a tile forms delta, U^{n+1}, cf and the next
// records of the tile's cells once the Euler group is done.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hofks {

constexpr int SMAX = 512;         // largest Euler sub-step count a plan may use
constexpr int ASTR = 4;           // doubles per row of Lax-Friedrichs speeds
constexpr int SET_D = (SMAX + 1) * ASTR + 8;  // doubles per slot set (+ 16 control ints)
constexpr int FLAG_NONPHYS = 1;
constexpr int FLAG_SUBSTEP = 2;
constexpr int FLAG_SPIN = 4;      // a bounded wait gave up: results are invalid
constexpr unsigned SPIN_CAP = 1u << 20;  // ~1-2 s of polling

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

template <int BCX>
__device__ __forceinline__ int map_x(int xN, int kx, int N) {
  if (BCX == 0) {  // periodic: t = x + N - k in [0, 2N)
    const unsigned t = (unsigned)(xN - kx);
    return (int)min(t, t - (unsigned)N);
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

// velocity node table of one axis: v, v^2, and FP32 copies (scalar loads)
struct VelNode {
  double v, v2;
  float vf, v2hf;  // (float)v, (float)(v^2 / 2)
  float pad0, pad1;
};

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
  }
  __syncthreads();
  __threadfence();  // acquire for every wave: the next sub-step reads other blocks' cells
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
  double rho = U[0], usq = 0.0, u[3];
#pragma unroll
  for (int b = 0; b < D; ++b) {
    u[b] = U[1 + b] / rho;
    usq += u[b] * u[b];
  }
  const double th = (2.0 * U[NM - 1] - rho * usq) / (D * rho);
  const double p = rho * th;
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
  return (rho > 0.0) && (th > 0.0) && isfinite(rho) && isfinite(th) && isfinite(usq);
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

__device__ __forceinline__ double vl_slope(double a, double b, int unlimited) {
  if (unlimited) return b;
  const double ab = a * b;
  return ab > 0.0 ? 2.0 * ab / (a + b) : 0.0;
}

// new value of cell j after one sub-step: in - dt_s/dx sum_a (psi_a+ - psi_a-).
// Each face is formed from its own four cells (both neighbours of a face get
// bit-identical fluxes, so the update conserves exactly up to the final sum).
template <int D>
__device__ __forceinline__ bool euler_cell(const double* __restrict__ in, int j,
                                           const double* alpha, double dts_dx, const Geom& G,
                                           int unl, double* Un) {
  constexpr int NM = D + 2;
  const int c[3] = {j % G.n[0], (j / G.n[0]) % G.n[1], j / (G.n[0] * G.n[1])};
  double div[NM];
#pragma unroll
  for (int r = 0; r < NM; ++r) div[r] = 0.0;
  bool phys = true;
#pragma unroll 1
  for (int a = 0; a < D; ++a) {
#pragma unroll 1
    for (int side = -1; side <= 0; ++side) {
      // face between cells j+side and j+side+1: stencil j+side-1 .. j+side+2
      double Wp[3][NM], Wm[3][NM];  // W+ of cells 0..2, W- of cells 1..3
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int cc[3] = {c[0], c[1], c[2]};
        cc[a] = map_axis(c[a] + side - 1 + q, G.n[a], G.bc[a]);
        const int jj = (cc[2] * G.n[1] + cc[1]) * G.n[0] + cc[0];
        double Uq[NM], wp[NM], wm[NM];
#pragma unroll
        for (int r = 0; r < NM; ++r) Uq[r] = in[(size_t)r * G.nc + jj];
        phys &= split_flux<D>(Uq, a, alpha[a], G.gam, wp, wm);
#pragma unroll
        for (int r = 0; r < NM; ++r) {
          if (q < 3) Wp[q][r] = wp[r];
          if (q > 0) Wm[q - 1][r] = wm[r];
        }
      }
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        const double sp = vl_slope(Wp[1][r] - Wp[0][r], Wp[2][r] - Wp[1][r], unl);
        const double sm = vl_slope(Wm[1][r] - Wm[0][r], Wm[2][r] - Wm[1][r], unl);
        const double psi = 0.5 * (Wp[1][r] + Wm[1][r]) + 0.25 * (sp - sm);
        div[r] += side == 0 ? psi : -psi;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NM; ++r) Un[r] = in[(size_t)r * G.nc + j] - dts_dx * div[r];
  return phys;
}

// ============================================================ cell record
// Maxwellian parameters of U (eq. M, theta from eq. E), separable discrete
// moments C M (sums along each velocity axis), cE = A (U - C M), and the
// record; speeds |u_a| + c for the next Euler solve.  Returns physicality.
template <int D, typename T>
__device__ __forceinline__ bool cell_record(const double* Un, const double* cfv, const Geom& G,
                                            const Mat& A, const VelNode* __restrict__ vt,
                                            T* __restrict__ rec_j, double* speed) {
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
    double G0[3], G1[3], G2[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int i = 0; i < G.nv1; ++i) {
        const double v = vt[i].v;
        const double e = exp(-beta * (v - u[a]) * (v - u[a]));
        s0 += e;
        s1 += v * e;
        s2 += vt[i].v2 * e;
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
  const bool need_eq = G.mu != 0.0;
  constexpr int RS = rec_stride<D, T>();
  T rv[RS];
#pragma unroll
  for (int q = 0; q < RS; ++q) rv[q] = (T)0;
  rv[0] = (T)lp;
#pragma unroll
  for (int a = 0; a < D; ++a) rv[1 + a] = (T)u[a];
  rv[D + 1] = (T)beta;
#pragma unroll
  for (int r = 0; r < NM; ++r) {
    rv[NM + r] = (T)(need_eq ? G.w * (G.lam * cfv[r] + G.mu * cE[r]) : G.w * (G.lam * cfv[r]));
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
  double* cf;
  double* part;       // nchunk x 2(d+2) x nc velocity-chunk sums
  int* tile_cnt;      // chunks finished per tile
  double* set_r;      // speeds of U^n (row 0) and of the sub-steps; control
  double* set_w;      // speeds of U^{n+1} (row 0), written by the epilogues
  double* set_z;      // the set of the step after next, cleared here
  int* flag;
  int TX, TR, nseg, nrowgrp, nchunk, nvr, GE, s_cap, unlimited, fks;
};

// Euler group: blocks 0 .. GE-1 advance U^n over dt with s sub-steps; the
// speeds of sub-step i+1 are reduced with atomics into row i+1 of set_r.
template <int D, typename T>
__device__ void euler_group(const StepArgs<T>& a, const Geom& G) {
  constexpr int NM = D + 2;
  double* S = a.set_r;
  unsigned* ctrl = reinterpret_cast<unsigned*>(S + (SMAX + 1) * ASTR);
  bool over;
  const int s = substeps<D>(S, G, a.s_cap, &over);
  if (blockIdx.x == 0) {
    for (int q = threadIdx.x; q < SET_D; q += blockDim.x) a.set_z[q] = 0.0;
    if (threadIdx.x == 0) {
      if (over) atomicOr(a.flag, FLAG_SUBSTEP);
      a.flag[1] = s;
    }
  }
  const double dts_dx = (G.dt / s) / G.dx;
  for (int i = 0; i < s; ++i) {
    const double* in = (i == 0) ? a.U_in : ((i & 1) ? a.UE1 : a.UE0);
    double* out = ((i + 1) & 1) ? a.UE1 : a.UE0;
    double alpha[3];
#pragma unroll
    for (int d2 = 0; d2 < D; ++d2)
      alpha[d2] = __hip_atomic_load(S + i * ASTR + d2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool phys = true;
    double mx[3] = {0.0, 0.0, 0.0};
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < G.nc; j += a.GE * blockDim.x) {
      double Un[NM];
      phys &= euler_cell<D>(in, j, alpha, dts_dx, G, a.unlimited, Un);
#pragma unroll
      for (int r = 0; r < NM; ++r) out[(size_t)r * G.nc + j] = Un[r];
      if (i + 1 < s) {
        double sp[3];
        phys &= lf_speeds<D>(Un, G.gam, sp);
#pragma unroll
        for (int d2 = 0; d2 < D; ++d2) mx[d2] = fmax(mx[d2], sp[d2]);
      }
    }
    if (!phys) atomicOr(a.flag, FLAG_NONPHYS);
    if (i + 1 < s) {
#pragma unroll
      for (int d2 = 0; d2 < D; ++d2) {
        const double m = wave_max(mx[d2]);
        if ((threadIdx.x & 63) == 0) atomic_max_pos(S + (i + 1) * ASTR + d2, m);
      }
    }
    group_barrier(ctrl, (unsigned)((i + 1) * a.GE), a.flag);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    __threadfence();
    __hip_atomic_store(ctrl + 1, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One kinetic block = TX x TR destination cells (TX consecutive x, TR rows)
// and one chunk of velocity rows.  For every velocity row (k_y, k_z) the
// records of the upstream row segment are staged in LDS; the loop over k_x
// issues the loads of UNR pieces g(j - k, k) (coalesced along x) before using
// them, relaxes each piece, writes it to cell j of the new buffer and sums
// the moments of f* and of E.  The last chunk to finish a tile then forms the
// new state of the tile's cells.
template <int D, typename T, bool FT, bool COMP, int BCX, int UNR, bool EUL>
__global__ __launch_bounds__(256) void k_step(StepArgs<T> a, Geom G, Mat A) {
  if (EUL && (int)blockIdx.x < a.GE) {
    euler_group<D, T>(a, G);
    return;
  }
  constexpr int NM = D + 2;
  constexpr int RS = rec_stride<D, T>();
  constexpr int PER16 = 16 / (int)sizeof(T);
  constexpr int NCH = (rec_values<D, T>() + PER16 - 1) / PER16;  // chunks read per piece
  using V = typename Vec16<T>::type;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  __shared__ int s_last;
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int TX = a.TX, TR = a.TR;
  const int SW = TX + G.nv1 - 1;

  int b = (int)blockIdx.x - (EUL ? a.GE : 0);
  const int tile = b % (a.nseg * a.nrowgrp);
  const int seg = b % a.nseg;
  b /= a.nseg;
  const int rg = b % a.nrowgrp;
  const int chunk = b / a.nrowgrp;
  const int tx = threadIdx.x % TX, tr = threadIdx.x / TX;
  const int x0 = seg * TX;
  const int x = x0 + tx;
  const int Nx = G.n[0];
  const int xN = x + Nx;
  const int nrows = G.n[1] * G.n[2];
  const int row = rg * TR + tr;
  const bool active = (x < Nx) && (row < nrows) && (tr < TR);
  const int jy = active ? row % G.n[1] : 0;
  const int jz = active ? row / G.n[1] : 0;
  const int dest = row * Nx + x;
  const int vr0 = (int)((long)chunk * a.nvr / a.nchunk);
  const int vr1 = (int)((long)(chunk + 1) * a.nvr / a.nchunk);
  const int xlo = x0 - (G.nv1 - 1 - G.kofs);
  const int lofs = G.nv1 - 1 - G.kofs;
  const T lam = (T)G.lam, mu = (T)G.mu;

  double SK[NM], SE[NM], CK[NM], CE[NM];
#pragma unroll
  for (int r = 0; r < NM; ++r) SK[r] = SE[r] = CK[r] = CE[r] = 0.0;

  for (int vr = vr0; vr < vr1; ++vr) {
    const int iy = (D >= 2) ? vr % G.nv1 : 0;
    const int iz = (D >= 3) ? vr / G.nv1 : 0;
    const int ky = iy - G.kofs, kz = iz - G.kofs;
    const double vy = (D >= 2) ? a.vt[iy].v : 0.0;
    const double vz = (D >= 3) ? a.vt[iz].v : 0.0;
    const double hrow = (D >= 2 ? 0.5 * a.vt[iy].v2 : 0.0) + (D >= 3 ? 0.5 * a.vt[iz].v2 : 0.0);

    // stage the records of the upstream row segments (16-byte chunks)
    __syncthreads();
    {
      constexpr int C16 = RS / PER16;
      const int total = TR * SW * C16;
      V* ldsv = reinterpret_cast<V*>(lds);
      const V* recv = reinterpret_cast<const V*>(a.rec_in);
      for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int c = idx % C16;
        const int cellslot = idx / C16;
        const int r_ = cellslot / SW, i = cellslot - r_ * SW;
        const int rw = rg * TR + r_;
        if (rw < nrows) {
          const int ry = rw % G.n[1], rz = rw / G.n[1];
          const int uy = (D >= 2) ? map_axis(ry - ky, G.n[1], G.bc[1]) : 0;
          const int uz = (D >= 3) ? map_axis(rz - kz, G.n[2], G.bc[2]) : 0;
          const int ux = map_axis(xlo + i, Nx, G.bc[0]);
          const int cell = (uz * G.n[1] + uy) * Nx + ux;
          ldsv[idx] = recv[(size_t)cell * C16 + c];
        }
      }
    }
    __syncthreads();
    if (!active) continue;

    const int uy = (D >= 2) ? map_axis(jy - ky, G.n[1], G.bc[1]) : 0;
    const int uz = (D >= 3) ? map_axis(jz - kz, G.n[2], G.bc[2]) : 0;
    const int ubase = (uz * G.n[1] + uy) * Nx;
    const T* Lrow = lds + (size_t)tr * SW * RS;
    const size_t kbase = (size_t)vr * G.nv1;
    const T vyT = (T)vy, vzT = (T)vz;
    const T hrowT = (T)hrow;
    double aK0 = 0.0, aK1 = 0.0, aK2 = 0.0, aE0 = 0.0, aE1 = 0.0, aE2 = 0.0;

    for (int ix0 = 0; ix0 < G.nv1; ix0 += UNR) {
      T gv[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int ix = ix0 + u;
        const int kx = ix - G.kofs;
        const T* gp = a.g_in + (kbase + ix) * (size_t)G.nc;
        gv[u] = gp[ubase + map_x<BCX>(xN, kx, Nx)];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int ix = ix0 + u;
        const int kx = ix - G.kofs;
        const VelNode vn = a.vt[ix];
        const double vx = vn.v;
        const T vxT = (sizeof(T) == 4) ? (T)vn.vf : (T)vn.v;
        const T vhT = (sizeof(T) == 4) ? (T)(hrowT + (T)vn.v2hf) : (T)(hrow + 0.5 * vn.v2);
        const V* rp = reinterpret_cast<const V*>(Lrow + (tx - kx + lofs) * RS);
        T rv[NCH * PER16];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const V t = rp[c];
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
        T pp = rv[NM + 0] + rv[NM + 1] * vxT;
        if (D >= 2) pp += rv[NM + 2] * vyT;
        if (D >= 3) pp += rv[NM + 3] * vzT;
        pp += rv[2 * NM - 1] * vhT;
        const T g = gv[u];
        T fs;
        if (FT) {
          fs = g + pp;
        } else {
          const T dx_ = vxT - rv[1];
          T q = dx_ * dx_;
          if (D >= 2) {
            const T dy_ = vyT - rv[2];
            q += dy_ * dy_;
          }
          if (D >= 3) {
            const T dz_ = vzT - rv[3];
            q += dz_ * dz_;
          }
          const T M = fast_exp<T>(rv[0] - rv[D + 1] * q);
          T pe = rv[2 * NM + 0] + rv[2 * NM + 1] * vxT;
          if (D >= 2) pe += rv[2 * NM + 2] * vyT;
          if (D >= 3) pe += rv[2 * NM + 3] * vzT;
          pe += rv[3 * NM - 1] * vhT;
          const T E = M + pe;
          fs = lam * g + (mu * M + pp);
          const double Ed = (double)E;
          aE0 += Ed;
          aE1 += vx * Ed;
          aE2 += vn.v2 * Ed;
        }
        T* op = a.g_out + (kbase + ix) * (size_t)G.nc;
        op[dest] = fs;
        const double fd = (double)fs;
        aK0 += fd;
        aK1 += vx * fd;
        aK2 += vn.v2 * fd;
      }
    }
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
  if (active) {
    double* P = a.part + (size_t)chunk * 2 * NM * G.nc;
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      P[(size_t)r * G.nc + dest] = COMP ? SK[r] + CK[r] : SK[r];
      if (!FT) P[(size_t)(NM + r) * G.nc + dest] = COMP ? SE[r] + CE[r] : SE[r];
    }
  }

  // ------------------------------------------------ last chunk of the tile
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const int old = atomicAdd(a.tile_cnt + tile, 1);
    s_last = (old == a.nchunk - 1);
    if (s_last) atomicExch(a.tile_cnt + tile, 0);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();

  const bool need_eq = G.mu != 0.0;
  int s = 0;
  if (EUL) {
    unsigned* ctrl = reinterpret_cast<unsigned*>(a.set_r + (SMAX + 1) * ASTR);
    if (threadIdx.x == 0) spin_until_geq(ctrl + 1, 1u, a.flag);
    __syncthreads();
    __threadfence();
    bool over;
    s = substeps<D>(a.set_r, G, a.s_cap, &over);
  }
  bool phys = true;
  double speed[3] = {0.0, 0.0, 0.0};
  if (active) {
    double SKt[NM], SEt[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) SKt[r] = SEt[r] = 0.0;
    for (int c = 0; c < a.nchunk; ++c) {
      const double* P = a.part + (size_t)c * 2 * NM * G.nc;
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        SKt[r] += P[(size_t)r * G.nc + dest];
        if (!FT) SEt[r] += P[(size_t)(NM + r) * G.nc + dest];
      }
    }
    double delta[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) delta[r] = 0.0;
    if (EUL) {
      const double* UEs = (s & 1) ? a.UE1 : a.UE0;
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        const double UM = G.mu * (G.w * SEt[r]);
        const double UEv = G.mu * UEs[(size_t)r * G.nc + dest];
        delta[r] = UEv - UM;
      }
    }
    double Un[NM], cfv[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) Un[r] = G.w * SKt[r] + delta[r];
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int s2 = 0; s2 < NM; ++s2) acc += A.a[r * NM + s2] * delta[s2];
      cfv[r] = acc;
    }
    phys = cell_record<D, T>(Un, cfv, G, A, a.vt, a.rec_out + (size_t)dest * RS, speed);
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      a.U_out[(size_t)r * G.nc + dest] = Un[r];
      a.cf[(size_t)r * G.nc + dest] = cfv[r];
    }
  }
  if (active && need_eq && !phys) atomicOr(a.flag, FLAG_NONPHYS);
  if (EUL) {
#pragma unroll
    for (int d2 = 0; d2 < D; ++d2) {
      const double m = wave_max(phys ? speed[d2] : 0.0);
      if ((threadIdx.x & 63) == 0) atomic_max_pos(a.set_w + d2, m);
    }
  }
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
    if (mode == MODE_REFRESH) {
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
    phys = cell_record<D, T>(Un, cfv, G, A, vt, rec + (size_t)j * RS, speed);
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
