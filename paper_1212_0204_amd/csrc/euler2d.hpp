// Euler sub-step on a 2D grid with LDS tiles (section 4.3.2, eq. (discmom)
// with the limited slopes of the MUSCL flux).  One block advances a 16 x 16
// tile of cells: it loads the tile and two halo cells on every side into
// LDS, then for each axis in turn evaluates the split fluxes
// W+- = F_a(U) +- alpha_a U once per cell (x: the 20 x 16 cells the x faces
// need; y: the 16 x 20 cells the y faces need) into one buffer, every thread
// adding the difference of its cell's two faces along that axis; then the
// new value.  The per-cell form `euler_cell` evaluates ten fluxes and reads
// 36 values from memory per cell; here it is 2.5 fluxes and about 1.6
// values.  Same arithmetic per face; the speeds, the sub-step count and the
// output buffers follow `k_euler_sub`.
#pragma once
#include "kernels.hpp"

namespace hofks {

constexpr int ET = 16;      // tile edge (cells)
constexpr int EH = ET + 4;  // tile edge with two halo cells on each side

template <typename T>
__global__ __launch_bounds__(256) void k_euler_sub_tile(StepArgs<T> a, Geom G, int i, int ntx) {
  constexpr int NM = 4;
  double* S = a.set_r;
  const int Nx = G.n[0], Ny = G.n[1];
  const int X0 = (int)(blockIdx.x % ntx) * ET, Y0 = (int)(blockIdx.x / ntx) * ET;
  const int t = threadIdx.x;
  const double* in = (i == 0) ? a.U_in : ((i & 1) ? a.UE1 : a.UE0);
  double* out = ((i + 1) & 1) ? a.UE1 : a.UE0;

  __shared__ double Ut[NM][EH][EH];
  // split fluxes along one axis at a time (x, then y) in one buffer:
  // x: [+/-][r][y][x + 2] over 16 x 20 cells; y: [+/-][r][y + 2][x] over 20 x 16
  __shared__ double Wb[2][NM][ET * EH];

  // tile + halo (periodic wrap or outflow clamp, as the per-cell form),
  // loaded before the speeds of the sub-step are read so that the two
  // memory round trips overlap (both buffers exist whatever s is)
  constexpr int NQ = (EH * EH + 255) / 256;
  double Uload[NQ][NM];
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = t + k * 256;
    if (q < EH * EH) {
      const int hx = q % EH, hy = q / EH;
      const int gx = map_axis(X0 + hx - 2, Nx, G.bc[0]);
      const int gy = map_axis(Y0 + hy - 2, Ny, G.bc[1]);
      const size_t j = (size_t)gy * Nx + gx;
#pragma unroll
      for (int r = 0; r < NM; ++r) Uload[k][r] = in[(size_t)r * G.nc + j];
    }
  }
  bool over;
  const int s = substeps<2>(S, G, a.s_cap, &over);
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
  row_speeds<2>(S, i, alpha);
  const double dts_dx = (G.dt / s) / G.dx;
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = t + k * 256;
    if (q < EH * EH) {
#pragma unroll
      for (int r = 0; r < NM; ++r) Ut[r][q / EH][q % EH] = Uload[k][r];
    }
  }
  __syncthreads();
  bool phys = true;
  const int lx = t % ET, ly = t / ET;
  const int gx = X0 + lx, gy = Y0 + ly;
  const bool own = gx < Nx && gy < Ny;
  double div[NM] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ax = 0; ax < 2; ++ax) {
    if (ax == 1) __syncthreads();  // the x faces have been read
    // fluxes along ax: x for cells (x = -2..17, y = 0..15), y for (x = 0..15, y = -2..17)
    for (int q = t; q < ET * EH; q += blockDim.x) {
      const int hx = ax == 0 ? q % EH : q % ET + 2;
      const int hy = ax == 0 ? q / EH + 2 : q / ET;
      double Uq[NM];
#pragma unroll
      for (int r = 0; r < NM; ++r) Uq[r] = Ut[r][hy][hx];
      double Wp[NM], Wm[NM];
      phys &= split_flux<2>(Uq, ax, alpha[ax], G.gam, Wp, Wm);
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        Wb[0][r][q] = Wp[r];
        Wb[1][r][q] = Wm[r];
      }
    }
    __syncthreads();
    if (own) {
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        // cells l-2 .. l+2 along ax: x -> entries ly*EH + lx + k, y -> (ly + k)*ET + lx
        double wp[5], wm[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const int e = ax == 0 ? ly * EH + lx + k : (ly + k) * ET + lx;
          wp[k] = Wb[0][r][e];
          wm[k] = Wb[1][r][e];
        }
        const double spl = vl_slope(wp[1] - wp[0], wp[2] - wp[1], a.unlimited);
        const double sml = vl_slope(wm[2] - wm[1], wm[3] - wm[2], a.unlimited);
        const double spr = vl_slope(wp[2] - wp[1], wp[3] - wp[2], a.unlimited);
        const double smr = vl_slope(wm[3] - wm[2], wm[4] - wm[3], a.unlimited);
        const double psil = 0.5 * (wp[1] + wm[2]) + 0.25 * (spl - sml);
        const double psir = 0.5 * (wp[2] + wm[3]) + 0.25 * (spr - smr);
        div[r] += psir - psil;
      }
    }
  }
  double mx[2] = {0.0, 0.0};
  if (own) {
    double Un[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) Un[r] = Ut[r][ly + 2][lx + 2] - dts_dx * div[r];
    const size_t j = (size_t)gy * Nx + gx;
#pragma unroll
    for (int r = 0; r < NM; ++r) out[(size_t)r * G.nc + j] = Un[r];
    if (i + 1 < s) {
      double sp[3];
      phys &= lf_speeds<2>(Un, G.gam, sp);
      mx[0] = sp[0];
      mx[1] = sp[1];
    }
  }
  if (!phys) atomicOr(a.flag, FLAG_NONPHYS);
  if (i + 1 < s) {
    __shared__ double wm4[4][ASTR];
#pragma unroll
    for (int d2 = 0; d2 < 2; ++d2) {
      const double m = wave_max(mx[d2]);
      if ((t & 63) == 0) wm4[t >> 6][d2] = m;
    }
    __syncthreads();
    if (t < 2) {
      double m = wm4[0][t];
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, wm4[w][t]);
      atomic_max_pos(speed_row(S, i + 1, blockIdx.x % NSLOT) + t, m);
    }
  }
}

}  // namespace hofks
