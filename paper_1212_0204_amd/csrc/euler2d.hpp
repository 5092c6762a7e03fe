// Euler sub-step on a 2D grid with LDS tiles (section 4.3.2, eq. (discmom)
// with the limited slopes of the MUSCL flux).  One block advances a 16 x 16
// tile of cells: it loads the tile and two halo cells on every side into
// LDS, evaluates the split fluxes W+- = F_a(U) +- alpha_a U once per cell and
// axis (x fluxes for the 20 x 16 cells the x faces need, y fluxes for the
// 16 x 20 cells the y faces need), then every thread forms the four faces of
// its cell and the new value.  The per-cell form `euler_cell` evaluates ten
// fluxes and reads 36 values from memory per cell; here it is 2.5 fluxes and
// about 1.6 values.  Same arithmetic per face; the speeds, the sub-step
// count and the output buffers follow `k_euler_sub`.
#pragma once
#include "kernels.hpp"

namespace hofks {

constexpr int ET = 16;      // tile edge (cells)
constexpr int EH = ET + 4;  // tile edge with two halo cells on each side

template <typename T>
__global__ __launch_bounds__(256) void k_euler_sub_tile(StepArgs<T> a, Geom G, int i, int ntx) {
  constexpr int NM = 4;
  double* S = a.set_r;
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
  const double* in = (i == 0) ? a.U_in : ((i & 1) ? a.UE1 : a.UE0);
  double* out = ((i + 1) & 1) ? a.UE1 : a.UE0;
  const int Nx = G.n[0], Ny = G.n[1];
  const int X0 = (int)(blockIdx.x % ntx) * ET, Y0 = (int)(blockIdx.x / ntx) * ET;
  const int t = threadIdx.x;

  __shared__ double Ut[NM][EH][EH];
  __shared__ double Wx[2][NM][ET][EH];  // [+/-][r][y][x + 2]
  __shared__ double Wy[2][NM][EH][ET];  // [+/-][r][y + 2][x]

  // tile + halo (periodic wrap or outflow clamp, as the per-cell form)
  for (int q = t; q < EH * EH; q += blockDim.x) {
    const int hx = q % EH, hy = q / EH;
    const int gx = map_axis(X0 + hx - 2, Nx, G.bc[0]);
    const int gy = map_axis(Y0 + hy - 2, Ny, G.bc[1]);
    const size_t j = (size_t)gy * Nx + gx;
#pragma unroll
    for (int r = 0; r < NM; ++r) Ut[r][hy][hx] = in[(size_t)r * G.nc + j];
  }
  __syncthreads();
  bool phys = true;
  // x fluxes of cells (x = -2..17, y = 0..15), y fluxes of (x = 0..15, y = -2..17)
  for (int q = t; q < 2 * ET * EH; q += blockDim.x) {
    const int ax = q < ET * EH ? 0 : 1;
    const int qq = ax == 0 ? q : q - ET * EH;
    const int hx = ax == 0 ? qq % EH : qq % ET + 2;
    const int hy = ax == 0 ? qq / EH + 2 : qq / ET;
    double Uq[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) Uq[r] = Ut[r][hy][hx];
    double Wp[NM], Wm[NM];
    phys &= split_flux<2>(Uq, ax, alpha[ax], G.gam, Wp, Wm);
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      if (ax == 0) {
        Wx[0][r][hy - 2][hx] = Wp[r];
        Wx[1][r][hy - 2][hx] = Wm[r];
      } else {
        Wy[0][r][hy][hx - 2] = Wp[r];
        Wy[1][r][hy][hx - 2] = Wm[r];
      }
    }
  }
  __syncthreads();
  const int lx = t % ET, ly = t / ET;
  const int gx = X0 + lx, gy = Y0 + ly;
  double mx[2] = {0.0, 0.0};
  if (gx < Nx && gy < Ny) {
    double div[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      // along x: cells lx-2 .. lx+2 are entries lx .. lx+4 of row ly
      const double* wp = &Wx[0][r][ly][lx];
      const double* wm = &Wx[1][r][ly][lx];
      double spl = vl_slope(wp[1] - wp[0], wp[2] - wp[1], a.unlimited);
      double sml = vl_slope(wm[2] - wm[1], wm[3] - wm[2], a.unlimited);
      double spr = vl_slope(wp[2] - wp[1], wp[3] - wp[2], a.unlimited);
      double smr = vl_slope(wm[3] - wm[2], wm[4] - wm[3], a.unlimited);
      double psil = 0.5 * (wp[1] + wm[2]) + 0.25 * (spl - sml);
      double psir = 0.5 * (wp[2] + wm[3]) + 0.25 * (spr - smr);
      div[r] = psir - psil;
      // along y: cells ly-2 .. ly+2 are rows ly .. ly+4 of column lx
      double yp[5], ym[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        yp[k] = Wy[0][r][ly + k][lx];
        ym[k] = Wy[1][r][ly + k][lx];
      }
      spl = vl_slope(yp[1] - yp[0], yp[2] - yp[1], a.unlimited);
      sml = vl_slope(ym[2] - ym[1], ym[3] - ym[2], a.unlimited);
      spr = vl_slope(yp[2] - yp[1], yp[3] - yp[2], a.unlimited);
      smr = vl_slope(ym[3] - ym[2], ym[4] - ym[3], a.unlimited);
      psil = 0.5 * (yp[1] + ym[2]) + 0.25 * (spl - sml);
      psir = 0.5 * (yp[2] + ym[3]) + 0.25 * (spr - smr);
      div[r] += psir - psil;
    }
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
