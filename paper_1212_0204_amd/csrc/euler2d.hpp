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
  // contiguous ranges of tiles per die (blocks reach the dies round-robin),
  // so that the halo of most tiles was written on the same die
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int X0 = (tile % ntx) * ET, Y0 = (tile / ntx) * ET;
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

// Euler sub-step on a 3D grid with LDS tiles: one block of 256 threads
// advances an 8 x 4 x 4 tile, loaded with two halo cells on every side
// (an 12 x 8 x 8 box) into LDS; for each axis in turn the split fluxes of
// the cells the faces along that axis need are evaluated once, one per
// thread, then every cell thread forms its two faces and adds their
// difference.  Same arithmetic per face as `euler_cell`; few registers
// (at most 64), so that the sub-step blocks find room beside the blocks of
// the kinetic kernel running at the same time.
constexpr int E3X = 8, E3Y = 4, E3Z = 4;  // tile (cells)
constexpr int E3C = E3X * E3Y * E3Z;      // 128 cells
constexpr int B3X = E3X + 4, B3Y = E3Y + 4, B3Z = E3Z + 4;  // box with halo

template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_num_vgpr(64))) void k_euler_sub_tile3(StepArgs<T> a, Geom G, int i, int ntx,
                                                           int nty) {
  constexpr int NM = 5;
  double* S = a.set_r;
  const int Nx = G.n[0], Ny = G.n[1], Nz = G.n[2];
  const int tb = xcd_tile(blockIdx.x, gridDim.x);  // contiguous ranges of tiles per die
  const int X0 = (tb % ntx) * E3X, Y0 = ((tb / ntx) % nty) * E3Y, Z0 = (tb / ntx / nty) * E3Z;
  const int t = threadIdx.x;
  const double* in = (i == 0) ? a.U_in : ((i & 1) ? a.UE1 : a.UE0);
  double* out = ((i + 1) & 1) ? a.UE1 : a.UE0;

  __shared__ double Ub[NM][B3Z * B3Y * B3X];  // box: [z][y][x]
  __shared__ double Wb[2][NM][256];          // split fluxes along one axis

  bool over;
  const int s = substeps<3>(S, G, a.s_cap, &over);
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
  row_speeds<3>(S, i, alpha);
  const double dts_dx = (G.dt / s) / G.dx;
  // box (periodic wrap or outflow clamp, as the per-cell form)
  for (int q = t; q < B3Z * B3Y * B3X; q += 256) {
    const int hx = q % B3X, hy = (q / B3X) % B3Y, hz = q / (B3X * B3Y);
    const int gx = map_axis(X0 + hx - 2, Nx, G.bc[0]);
    const int gy = map_axis(Y0 + hy - 2, Ny, G.bc[1]);
    const int gz = map_axis(Z0 + hz - 2, Nz, G.bc[2]);
    const size_t j = ((size_t)gz * Ny + gy) * Nx + gx;
#pragma unroll
    for (int r = 0; r < NM; ++r) Ub[r][q] = in[(size_t)r * G.nc + j];
  }
  __syncthreads();
  bool phys = true;
  const int lx = t % E3X, ly = (t / E3X) % E3Y, lz = t / (E3X * E3Y);  // cell of t < 128
  const int gx = X0 + lx, gy = Y0 + ly, gz = Z0 + lz;
  const bool own = t < E3C && gx < Nx && gy < Ny && gz < Nz;
  double div[NM] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int ax = 0; ax < 3; ++ax) {
    if (ax > 0) __syncthreads();  // the fluxes of the previous axis have been read
    // entries: the tile extended by two cells on each side along ax
    const int ex = ax == 0 ? B3X : E3X, ey = ax == 1 ? B3Y : E3Y;
    const int ne = ex * ey * (ax == 2 ? B3Z : E3Z);
    if (t < ne) {
      const int qx = t % ex, qy = (t / ex) % ey, qz = t / (ex * ey);
      const int hx = ax == 0 ? qx : qx + 2, hy = ax == 1 ? qy : qy + 2, hz = ax == 2 ? qz : qz + 2;
      const int b = (hz * B3Y + hy) * B3X + hx;
      double Uq[NM];
#pragma unroll
      for (int r = 0; r < NM; ++r) Uq[r] = Ub[r][b];
      double Wp[NM], Wm[NM];
      phys &= split_flux<3>(Uq, ax, alpha[ax], G.gam, Wp, Wm);
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        Wb[0][r][t] = Wp[r];
        Wb[1][r][t] = Wm[r];
      }
    }
    __syncthreads();
    if (own) {
      // entries of the cells l-2 .. l+2 along ax
      const int e0 = ax == 0 ? (lz * E3Y + ly) * B3X + lx
                   : ax == 1 ? (lz * B3Y + ly) * E3X + lx : (lz * E3Y + ly) * E3X + lx;
      const int es = ax == 0 ? 1 : ax == 1 ? E3X : E3X * E3Y;
      // one moment at a time (few live registers)
#pragma unroll 1
      for (int r = 0; r < NM; ++r) {
        double wp[5], wm[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          wp[k] = Wb[0][r][e0 + k * es];
          wm[k] = Wb[1][r][e0 + k * es];
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
  double mx[3] = {0.0, 0.0, 0.0};
  if (own) {
    const int b = ((lz + 2) * B3Y + ly + 2) * B3X + lx + 2;
    double Un[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) Un[r] = Ub[r][b] - dts_dx * div[r];
    const size_t j = ((size_t)gz * Ny + gy) * Nx + gx;
#pragma unroll
    for (int r = 0; r < NM; ++r) out[(size_t)r * G.nc + j] = Un[r];
    if (i + 1 < s) phys &= lf_speeds<3>(Un, G.gam, mx);
  }
  if (!phys) atomicOr(a.flag, FLAG_NONPHYS);
  if (i + 1 < s) {
    __shared__ double wm4[4][ASTR];
#pragma unroll
    for (int d2 = 0; d2 < 3; ++d2) {
      const double m = wave_max(mx[d2]);
      if ((t & 63) == 0) wm4[t >> 6][d2] = m;
    }
    __syncthreads();
    if (t < 3) {
      double m = wm4[0][t];
      for (int w = 1; w < 4; ++w) m = fmax(m, wm4[w][t]);
      atomic_max_pos(speed_row(S, i + 1, blockIdx.x % NSLOT) + t, m);
    }
  }
}

}  // namespace hofks
