// weno.hpp -- the WENO Euler solve of HOFKS scheme 3 (section 4.3.3 of
// arXiv:1212.0204 names WENO as a higher-order solver for the Euler part,
// with a tighter CFL than eq. (Time2)).
//
// Finite-difference WENO5 (Jiang and Shu) on the global Lax-Friedrichs split
// flux h+- = (F_a(U) +- alpha_a U) / 2: the + part is reconstructed at face
// j+1/2 from cells j-2 .. j+2, the - part from cells j+3 .. j-1 (mirrored);
// time by the three-stage SSP Runge-Kutta method of Shu and Osher,
//   U1 = U + h L(U),  U2 = 3/4 U + 1/4 (U1 + h L(U1)),
//   U  <- 1/3 U + 2/3 (U2 + h L(U2)),   L(V) = -(1/dx) sum_a (fh_{j+1/2} - fh_{j-1/2}),
// with alpha from the speeds of each sub-step's initial state (row i of the
// speed set) for all three stages.  The s sub-steps of dt/s follow from
// s = max(1, ceil(dt sum_a alpha_a / (0.4 dx))) (G.sfac = 2.5).
//
// Buffers: sub-step i reads X = U^n (i = 0) or UE[i % 2]; stage 0 writes
// UE2, stage 1 writes UE3, stage 2 writes UE[(i + 1) % 2], so that after s
// sub-steps the result is in UE[s % 2] as for the MUSCL solve.
#pragma once
#include "kernels.hpp"

namespace hofks {

// fifth-order WENO value at the right face of v2 from v0 .. v4 (cells
// j-2 .. j+2): third-order candidates on {j-2..j}, {j-1..j+1}, {j..j+2},
// linear weights 1/10, 6/10, 3/10, smoothness indicators, eps = 1e-6.  The
// nonlinear weights d_k / (eps + b_k)^2 are brought to one denominator, so
// that one division forms the value.
__device__ __forceinline__ double weno5(double v0, double v1, double v2, double v3, double v4) {
  const double q0 = (2.0 * v0 - 7.0 * v1 + 11.0 * v2) * (1.0 / 6.0);
  const double q1 = (-v1 + 5.0 * v2 + 2.0 * v3) * (1.0 / 6.0);
  const double q2 = (2.0 * v2 + 5.0 * v3 - v4) * (1.0 / 6.0);
  const double s0 = v0 - 2.0 * v1 + v2, t0 = v0 - 4.0 * v1 + 3.0 * v2;
  const double s1 = v1 - 2.0 * v2 + v3, t1 = v1 - v3;
  const double s2 = v2 - 2.0 * v3 + v4, t2 = 3.0 * v2 - 4.0 * v3 + v4;
  constexpr double c13 = 13.0 / 12.0, eps = 1e-6;
  const double e0 = eps + (c13 * s0 * s0 + 0.25 * t0 * t0);
  const double e1 = eps + (c13 * s1 * s1 + 0.25 * t1 * t1);
  const double e2 = eps + (c13 * s2 * s2 + 0.25 * t2 * t2);
  const double E0 = e0 * e0, E1 = e1 * e1, E2 = e2 * e2;
  // a_k = d_k / E_k  ->  a_k E0 E1 E2 = d_k prod_{l != k} E_l
  const double w0 = 0.1 * (E1 * E2), w1 = 0.6 * (E0 * E2), w2 = 0.3 * (E0 * E1);
  return (w0 * q0 + w1 * q1 + w2 * q2) / (w0 + w1 + w2);
}

// L(V) at cell j (times -dx: the flux divergence summed over the axes);
// false if a stencil state is not physical
template <int D>
__device__ __forceinline__ bool weno_div(const double* __restrict__ V, int j, const double* alpha,
                                         const Geom& G, double* div) {
  constexpr int NM = D + 2;
  const int c[3] = {j % G.n[0], (j / G.n[0]) % G.n[1], j / (G.n[0] * G.n[1])};
  bool phys = true;
#pragma unroll
  for (int r = 0; r < NM; ++r) div[r] = 0.0;
#pragma unroll 1
  for (int a = 0; a < D; ++a) {
    double hp[7][NM], hm[7][NM];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      int cc[3] = {c[0], c[1], c[2]};
      cc[a] = map_axis(c[a] + q - 3, G.n[a], G.bc[a]);
      const int jj = (cc[2] * G.n[1] + cc[1]) * G.n[0] + cc[0];
      double Uq[NM];
#pragma unroll
      for (int r = 0; r < NM; ++r) Uq[r] = V[(size_t)r * G.nc + jj];
      double Wp[NM], Wm[NM];
      phys &= split_flux<D>(Uq, a, alpha[a], G.gam, Wp, Wm);
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        hp[q][r] = 0.5 * Wp[r];
        hm[q][r] = 0.5 * Wm[r];
      }
    }
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      const double fr = weno5(hp[1][r], hp[2][r], hp[3][r], hp[4][r], hp[5][r]) +
                        weno5(hm[6][r], hm[5][r], hm[4][r], hm[3][r], hm[2][r]);
      const double fl = weno5(hp[0][r], hp[1][r], hp[2][r], hp[3][r], hp[4][r]) +
                        weno5(hm[5][r], hm[4][r], hm[3][r], hm[2][r], hm[1][r]);
      div[r] += fr - fl;
    }
  }
  return phys;
}

// buffers of stage `st` of sub-step i
template <typename T>
__device__ __forceinline__ void weno_buffers(const StepArgs<T>& a, int i, int st, const double** X,
                                             const double** V, double** out) {
  *X = (i == 0) ? a.U_in : ((i & 1) ? a.UE1 : a.UE0);
  *V = st == 0 ? *X : (st == 1 ? a.UE2 : a.UE3);
  *out = st == 0 ? a.UE2 : (st == 1 ? a.UE3 : (((i + 1) & 1) ? a.UE1 : a.UE0));
}

// the new value of cell j after stage st (the Shu-Osher combination)
template <int D>
__device__ __forceinline__ bool weno_cell(const double* __restrict__ X, const double* __restrict__ V,
                                          int j, const double* alpha, double h, int st,
                                          const Geom& G, double* Un) {
  constexpr int NM = D + 2;
  double div[NM];
  const bool phys = weno_div<D>(V, j, alpha, G, div);
#pragma unroll
  for (int r = 0; r < NM; ++r) {
    const double L = -div[r] / G.dx;
    const double x = X[(size_t)r * G.nc + j];
    const double v = st == 0 ? x : V[(size_t)r * G.nc + j];
    if (st == 0)
      Un[r] = v + h * L;
    else if (st == 1)
      Un[r] = 0.75 * x + 0.25 * (v + h * L);
    else
      Un[r] = x / 3.0 + 2.0 / 3.0 * (v + h * L);
  }
  return phys;
}

// Stage st of sub-step i over the whole grid, one cell per thread (one
// launch per stage: the kernel boundary is the grid-wide barrier).  Stage 0
// of sub-step 0 also records s and clears the set of the step after next;
// launches with i >= s return at once; stage 2 folds the speeds of its
// result into row i+1 (one atomic maximum per block, slot block mod NSLOT).
template <int D, typename T>
__global__ __launch_bounds__(256) void k_weno_stage(StepArgs<T> a, Geom G, int i, int st) {
  constexpr int NM = D + 2;
  double* S = a.set_r;
  bool over;
  const int s = substeps<D>(S, G, a.s_cap, &over);
  if (i == 0 && st == 0) {
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
  const double h = G.dt / s;
  const double *X, *V;
  double* out;
  weno_buffers(a, i, st, &X, &V, &out);
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const bool want = st == 2 && i + 1 < s;
  bool phys = true;
  double mx[3] = {0.0, 0.0, 0.0};
  if (j < G.nc) {
    double Un[NM];
    phys = weno_cell<D>(X, V, j, alpha, h, st, G, Un);
#pragma unroll
    for (int r = 0; r < NM; ++r) out[(size_t)r * G.nc + j] = Un[r];
    if (want) {
      double sp[3];
      phys &= lf_speeds<D>(Un, G.gam, sp);
#pragma unroll
      for (int d2 = 0; d2 < D; ++d2) mx[d2] = sp[d2];
    }
  }
  if (!phys) atomicOr(a.flag, FLAG_NONPHYS);
  if (want) {
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

// WENO tail: GE co-resident blocks run the stages of sub-steps K .. s-1
// (grid-strided over cells) with a barrier after every stage but the last;
// after stage 2 of a sub-step the blocks' speed maxima are reduced by the
// last block to arrive into slot 0 of row i+1, as in k_euler.  nb counts the
// barriers of this launch, the same in every block.
template <int D, typename T, int TPB>
__global__ __launch_bounds__(TPB) void k_weno_tail(StepArgs<T> a, Geom G, int K) {
  constexpr int NM = D + 2;
  double* S = a.set_r;
  unsigned* ctrl = reinterpret_cast<unsigned*>(S + SET_CTRL);
  bool over;
  const int s = substeps<D>(S, G, a.s_cap, &over);
  if (K >= s) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(a.flag + 2, s - K);
  const double h = G.dt / s;
  __shared__ double wmax[TPB / 64][ASTR];
  __shared__ int s_last;
  double alpha[3];
  row_speeds<D>(S, K, alpha);
  unsigned nb = 0;
  for (int i = K; i < s; ++i) {
    for (int st = 0; st < 3; ++st) {
      const double *X, *V;
      double* out;
      weno_buffers(a, i, st, &X, &V, &out);
      const bool want = st == 2 && i + 1 < s;
      bool phys = true;
      double mx[3] = {0.0, 0.0, 0.0};
      for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < G.nc; j += a.GE * blockDim.x) {
        double Un[NM];
        phys &= weno_cell<D>(X, V, j, alpha, h, st, G, Un);
#pragma unroll
        for (int r = 0; r < NM; ++r) out[(size_t)r * G.nc + j] = Un[r];
        if (want) {
          double sp[3];
          phys &= lf_speeds<D>(Un, G.gam, sp);
#pragma unroll
          for (int d2 = 0; d2 < D; ++d2) mx[d2] = fmax(mx[d2], sp[d2]);
        }
      }
      if (!phys) atomicOr(a.flag, FLAG_NONPHYS);
      if (st == 2 && i + 1 == s) break;  // the last stage: no barrier
      ++nb;
      double* bm = a.bmax;
      if (want) {
#pragma unroll
        for (int d2 = 0; d2 < D; ++d2) {
          const double m = wave_max(mx[d2]);
          if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6][d2] = m;
        }
        __syncthreads();
        if (threadIdx.x < D) {
          double m = wmax[0][threadIdx.x];
          for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, wmax[w][threadIdx.x]);
          bm[(size_t)blockIdx.x * ASTR + threadIdx.x] = m;
        }
      }
      __syncthreads();
      unsigned* gen = ctrl;  // line 0: generation
      if (threadIdx.x == 0) {
        const unsigned g = blockIdx.x & 7u;
        const unsigned ng = (a.GE - g + 7) / 8;
        const unsigned ngroups = a.GE < 8 ? a.GE : 8;
        unsigned* top = ctrl + 16;
        unsigned* sub = ctrl + 32 + 16 * g;
        __threadfence();
        int last = 0;
        const unsigned old = atomicAdd(sub, 1u);
        if (old == nb * ng - 1) {
          const unsigned t = atomicAdd(top, 1u);
          last = (t == nb * ngroups - 1);
        }
        s_last = last;
      }
      __syncthreads();
      if (s_last) {
        __threadfence();
        if (want) {
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
        }
        __syncthreads();
        if (threadIdx.x == 0) {
          if (want) {
#pragma unroll
            for (int d2 = 0; d2 < D; ++d2) {
              double w = wmax[0][d2];
              for (int q = 1; q < (int)(blockDim.x >> 6); ++q) w = fmax(w, wmax[q][d2]);
              __hip_atomic_store(speed_row(S, i + 1, 0) + d2, w, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
            }
          }
          __threadfence();
          __hip_atomic_store(gen, nb, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      if (threadIdx.x == 0) {
        spin_until_geq(gen, nb, a.flag);
        __threadfence();
        if (want) {
#pragma unroll
          for (int d2 = 0; d2 < D; ++d2)
            wmax[0][d2] = __hip_atomic_load(speed_row(S, i + 1, 0) + d2, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      __syncthreads();
      if (want) {
#pragma unroll
        for (int d2 = 0; d2 < D; ++d2) alpha[d2] = wmax[0][d2];
      }
      __syncthreads();
    }
  }
}

}  // namespace hofks

namespace hofks {

// Stage st of sub-step i on a 2D grid with LDS tiles: one block advances a
// 16 x 16 tile.  The stage input V of the tile and three halo cells on each
// side (22 x 22) goes to LDS; for each axis the split fluxes of the 22 x 16
// cells the faces need are formed once, then each face value (17 faces per
// line, both split parts) once, and every cell adds the difference of its
// two faces.  Same arithmetic per face as `weno_div`; buffers, speeds and
// the sub-step count as `k_weno_stage`.
constexpr int WT = 16;          // tile edge
constexpr int WH = WT + 6;      // with three halo cells per side
constexpr int WF = WT + 1;      // faces per tile line

template <typename T>
__global__ __launch_bounds__(256) void k_weno_stage_tile(StepArgs<T> a, Geom G, int i, int st,
                                                         int ntx) {
  constexpr int NM = 4;
  double* S = a.set_r;
  const int Nx = G.n[0], Ny = G.n[1];
  // contiguous ranges of tiles per die, as the MUSCL tiles
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int X0 = (tile % ntx) * WT, Y0 = (tile / ntx) * WT;
  const int t = threadIdx.x;
  __shared__ double Vt[NM][WH * WH];        // stage input, tile + halo
  __shared__ double Hs[2][NM][WH * WT];     // split fluxes along one axis
  __shared__ double Fc[NM][WF * WT];        // face values along one axis

  bool over;
  const int s = substeps<2>(S, G, a.s_cap, &over);
  if (i == 0 && st == 0) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < SET_D; q += gridDim.x * blockDim.x)
      a.set_z[q] = 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (over) atomicOr(a.flag, FLAG_SUBSTEP);
      a.flag[1] = s;
    }
  }
  if (i >= s) return;
  double alpha[3];
  row_speeds<2>(S, i, alpha);
  const double h = G.dt / s;
  const double *X, *V;
  double* out;
  weno_buffers(a, i, st, &X, &V, &out);
  for (int q = t; q < WH * WH; q += 256) {
    const int hx = q % WH, hy = q / WH;
    const int gx = map_axis(X0 + hx - 3, Nx, G.bc[0]);
    const int gy = map_axis(Y0 + hy - 3, Ny, G.bc[1]);
    const size_t j = (size_t)gy * Nx + gx;
#pragma unroll
    for (int r = 0; r < NM; ++r) Vt[r][q] = V[(size_t)r * G.nc + j];
  }
  __syncthreads();
  bool phys = true;
  const int lx = t % WT, ly = t / WT;
  const int gx = X0 + lx, gy = Y0 + ly;
  const bool own = gx < Nx && gy < Ny;
  double div[NM] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
  for (int ax = 0; ax < 2; ++ax) {
    // split fluxes of the cells along ax: x -> (x = -3..18, y = 0..15),
    // y -> (x = 0..15, y = -3..18); entry e = line * WH + position
    for (int q = t; q < WH * WT; q += 256) {
      const int line = q / WH, pos = q % WH;
      const int hx = ax == 0 ? pos : line + 3, hy = ax == 0 ? line + 3 : pos;
      double Uq[NM];
#pragma unroll
      for (int r = 0; r < NM; ++r) Uq[r] = Vt[r][hy * WH + hx];
      double Wp[NM], Wm[NM];
      phys &= split_flux<2>(Uq, ax, alpha[ax], G.gam, Wp, Wm);
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        Hs[0][r][q] = 0.5 * Wp[r];
        Hs[1][r][q] = 0.5 * Wm[r];
      }
    }
    __syncthreads();
    // face f of a line lies between cells f - 1 and f (f = 0..16): the +
    // part from cells f-3 .. f+1, the - part from cells f+2 .. f-2
    for (int q = t; q < WF * WT * NM; q += 256) {
      const int r = q / (WF * WT), e = q % (WF * WT);
      const int line = e / WF, f = e % WF;
      const double* hp = &Hs[0][r][line * WH + f];  // cell f - 3 at offset 0
      const double* hm = &Hs[1][r][line * WH + f];
      Fc[r][e] = weno5(hp[0], hp[1], hp[2], hp[3], hp[4]) + weno5(hm[5], hm[4], hm[3], hm[2], hm[1]);
    }
    __syncthreads();
    if (own) {
      const int line = ax == 0 ? ly : lx, c = ax == 0 ? lx : ly;
#pragma unroll
      for (int r = 0; r < NM; ++r) div[r] += Fc[r][line * WF + c + 1] - Fc[r][line * WF + c];
    }
    __syncthreads();  // Hs and Fc are rewritten for the next axis
  }
  double mx[2] = {0.0, 0.0};
  const bool want = st == 2 && i + 1 < s;
  if (own) {
    const size_t j = (size_t)gy * Nx + gx;
    double Un[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      const double L = -div[r] / G.dx;
      const double x = X[(size_t)r * G.nc + j];
      const double v = Vt[r][(ly + 3) * WH + lx + 3];
      if (st == 0)
        Un[r] = v + h * L;
      else if (st == 1)
        Un[r] = 0.75 * x + 0.25 * (v + h * L);
      else
        Un[r] = x / 3.0 + 2.0 / 3.0 * (v + h * L);
      out[(size_t)r * G.nc + j] = Un[r];
    }
    if (want) {
      double sp[3];
      phys &= lf_speeds<2>(Un, G.gam, sp);
      mx[0] = sp[0];
      mx[1] = sp[1];
    }
  }
  if (!phys) atomicOr(a.flag, FLAG_NONPHYS);
  if (want) {
    __shared__ double wm4[4][ASTR];
#pragma unroll
    for (int d2 = 0; d2 < 2; ++d2) {
      const double m = wave_max(mx[d2]);
      if ((t & 63) == 0) wm4[t >> 6][d2] = m;
    }
    __syncthreads();
    if (t < 2) {
      double m = wm4[0][t];
      for (int w = 1; w < 4; ++w) m = fmax(m, wm4[w][t]);
      atomic_max_pos(speed_row(S, i + 1, blockIdx.x % NSLOT) + t, m);
    }
  }
}

}  // namespace hofks
