// Learned closure of near-equilibrium cells (2D-2V, not part of the paper).
//
// In a closure cell the moment update of eq. (UK) + (mom) is taken as
//   U^{n+1} = lam * sum_k w m_k E^n(j - k, k) + U_E + N^,
// where the first term is the transported equilibrium (the kinetic flux of
// E, no pieces needed), U_E the MUSCL Euler part and N^ the network's
// estimate of the non-equilibrium term
//   N = sum_k w m_k (f*^n - E^n)(j - k, k) = lam * sum_k w m_k (f^n - E^n)(j - k, k).
// N carries the factor lam exactly, so the network predicts
//   y = N / (lam * s_j),   s_j = (rho, rho c, rho c, E) of cell j,  c = sqrt(gam theta)
// from the 3 x 3 stencil of U^n, and N^ = lam * sigma * (y - y0) (.) s_j,
// y0 the output for a uniform stencil (N vanishes for a uniform state).
//
// Inputs (37): for each stencil cell c = 3 (dy + 1) + (dx + 1) the values
// rho_c / rho_j - 1, (u_c - u_j) / c_j (two components), theta_c / theta_j - 1
// (zero for a uniform state, which keeps the small differences resolved in
// BF16), then log10(tau / dt) clamped to [-8, 8].
//
// A cell runs the kinetic step (relaxation, shift, moments, correction)
// when its indicator r = lam * sigma * max|y - y0| exceeds the threshold, or
// when its last kinetic step had lam * max|delta| / s above it (every cell
// counts as such after the state is set), or when such a cell lies within
// n_v / 2 cells in each axis (the reach of one shift).
// Closure cells keep no pieces: a kinetic cell reading an upstream piece of
// a cell whose pieces were not written by the last step uses the
// equilibrium E of that cell instead (a negative beta in its record marks
// it).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "mlp.hpp"

namespace hofks {

struct ClosureArgs {
  const double* U;           // U^n, [4][nc]
  const void* packed;        // network, packed BF16 (see mlp.hpp)
  float4* nhat;              // N^ per cell (physical units)
  unsigned char* flagged;    // indicator above threshold (before dilation)
  const unsigned char* dfl;  // delta indicator of the last kinetic step
  const float* y0;           // network output for a uniform stencil
  float ftau;                // log10(tau / dt), clamped
  double lam, sigma, thr;
};

// primitive state (rho, u_x, u_y, theta) of cell j of a 2D grid
__device__ __forceinline__ void prim2(const double* __restrict__ U, int nc, int j, double* p) {
  const double rho = U[j];
  const double ux = U[(size_t)nc + j] / rho, uy = U[2 * (size_t)nc + j] / rho;
  p[0] = rho;
  p[1] = ux;
  p[2] = uy;
  p[3] = (2.0 * U[3 * (size_t)nc + j] - rho * (ux * ux + uy * uy)) / (2.0 * rho);
}

// the four inputs of stencil cell c of the cell with primitive state pc
__device__ __forceinline__ void stencil_inputs(const double* __restrict__ U, const Geom& G, int x,
                                               int y, int c, const double* pc, double cs,
                                               float* out) {
  const int xx = map_axis(x + c % 3 - 1, G.n[0], G.bc[0]);
  const int yy = map_axis(y + c / 3 - 1, G.n[1], G.bc[1]);
  double p[4];
  prim2(U, G.nc, yy * G.n[0] + xx, p);
  out[0] = (float)(p[0] / pc[0] - 1.0);
  out[1] = (float)((p[1] - pc[1]) / cs);
  out[2] = (float)((p[2] - pc[2]) / cs);
  out[3] = (float)(p[3] / pc[3] - 1.0);
}

// x[j][37] for every cell (training snapshots)
__global__ __launch_bounds__(256) void k_closure_features(const double* __restrict__ U,
                                                          float* __restrict__ xo, Geom G,
                                                          float ftau) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= G.nc) return;
  const int x = j % G.n[0], y = j / G.n[0];
  double pc[4];
  prim2(U, G.nc, j, pc);
  const double cs = sqrt(G.gam * pc[3]);
  float* o = xo + (size_t)j * mlp::NIN;
  for (int c = 0; c < 9; ++c) stencil_inputs(U, G, x, y, c, pc, cs, o + 4 * c);
  o[36] = ftau;
}

// y0: the network on the uniform stencil (zeros, then log10(tau/dt)); one
// wavefront
__global__ __launch_bounds__(64) void k_closure_center(const void* __restrict__ packed,
                                                       float* __restrict__ y0, float ftau) {
  using namespace mlp;
  const int lane = threadIdx.x & 63, q = lane >> 4;
  FwdW W;
  load_fwd(packed, W, lane);
  // input 36 (element 4 of lane quarter 0 in the second K step) is the tau
  // feature, the others zero
  const s4 z = pack4(f4{0.0f, 0.0f, 0.0f, 0.0f});
  const s8 xf[2] = {cat8(z, z), cat8(z, pack4(f4{q == 0 ? ftau : 0.0f, 0.0f, 0.0f, 0.0f}))};
  const f4 y = forward16<false>(W, biases(packed), xf, nullptr, lane);
  if (lane == 0) {
    y0[0] = y[0];
    y0[1] = y[1];
    y0[2] = y[2];
    y0[3] = y[3];
  }
}

// network over all cells: N^ and the indicator; one wavefront per 16 cells
__global__ __launch_bounds__(256) void k_closure_mlp(ClosureArgs a, Geom G) {
  using namespace mlp;
  const int lane = threadIdx.x & 63, q = lane >> 4;
  FwdW W;
  load_fwd(a.packed, W, lane);
  const float* bias = biases(a.packed);
  const long ntile = (G.nc + 15) / 16;
  const long wave = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const long nwave = (long)gridDim.x * (blockDim.x >> 6);
  for (long tile = wave; tile < ntile; tile += nwave) {
    const int j = (int)(tile * 16 + (lane & 15));
    const bool act = j < G.nc;
    const int jc = act ? j : G.nc - 1;
    const int x = jc % G.n[0], y = jc / G.n[0];
    double pc[4];
    prim2(a.U, G.nc, jc, pc);
    const double cs = sqrt(G.gam * pc[3]);
    // K step s of lane quarter q: stencil cells 8 s + 2 q and 8 s + 2 q + 1
    // (four inputs each; cell 9 is the tau feature, cells beyond are zero)
    s8 xf[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      s4 half[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = 8 * s + 2 * q + h;
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        if (c < 9)
          stencil_inputs(a.U, G, x, y, c, pc, cs, v);
        else if (c == 9)
          v[0] = a.ftau;
        half[h] = pack4(f4{v[0], v[1], v[2], v[3]});
      }
      xf[s] = cat8(half[0], half[1]);
    }
    f4 yv = forward16<false>(W, bias, xf, nullptr, lane);
    if (lane < 16 && act) {
      yv[0] -= a.y0[0];
      yv[1] -= a.y0[1];
      yv[2] -= a.y0[2];
      yv[3] -= a.y0[3];
      const double ls = a.lam * a.sigma;
      const double sc[4] = {pc[0], pc[0] * cs, pc[0] * cs,
                            a.U[3 * (size_t)G.nc + j]};
      float4 nh;
      nh.x = (float)(ls * yv[0] * sc[0]);
      nh.y = (float)(ls * yv[1] * sc[1]);
      nh.z = (float)(ls * yv[2] * sc[2]);
      nh.w = (float)(ls * yv[3] * sc[3]);
      a.nhat[j] = nh;
      const float m = fmaxf(fmaxf(fabsf(yv[0]), fabsf(yv[1])), fmaxf(fabsf(yv[2]), fabsf(yv[3])));
      const double r = ls * (double)m;
      a.flagged[j] = (unsigned char)(!(r <= a.thr) || a.dfl[j] != 0);
    }
  }
}

// out = in dilated by h cells along one axis (a box filter of OR)
template <int AXIS>
__global__ __launch_bounds__(256) void k_dilate(const unsigned char* __restrict__ in,
                                                unsigned char* __restrict__ out, Geom G, int h) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= G.nc) return;
  const int x = j % G.n[0], y = j / G.n[0];
  // every load of the window is issued (no early exit), so they overlap
  unsigned char any = 0;
#pragma unroll 8
  for (int d = -h; d <= h; ++d) {
    const int jj = AXIS == 0 ? y * G.n[0] + map_axis(x + d, G.n[0], G.bc[0])
                             : map_axis(y + d, G.n[1], G.bc[1]) * G.n[0] + x;
    any |= in[jj];
  }
  out[j] = any;
}

__global__ void k_fill_u8(unsigned char* __restrict__ p, int n, unsigned char v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace hofks
