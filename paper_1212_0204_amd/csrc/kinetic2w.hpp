// Kinetic kernel for 2D-2V FP64 steps with an Euler solve (relaxation,
// shift and moment sums of section 4.3.1, eq. (UK)) with two cells per lane:
// a wavefront covers 128 consecutive x cells of one row and reads and
// writes each velocity plane in 16-byte pieces per lane (1 KB per
// instruction instead of 512 B), which the memory system serves about a
// tenth faster.  One block = 128 cells of a row and NG wavefronts, each
// taking 1/NG of the velocity rows, as in `k_kinetic`.
//
// Per velocity row a wavefront stages the row records (transverse terms
// folded in, nine values, see `row_rec_stride`) of the upstream row segment
// in its LDS slice, split by the parity of the cell index: the two records a
// lane reads for one piece pair lie in different halves, and within a half
// the lanes read consecutive records (an odd number of 16-byte chunks apart,
// so no LDS bank conflicts).  The pair of upstream cells (x - k, x + 1 - k)
// is contiguous except where it straddles the periodic seam or leaves an
// outflow boundary; those lanes load the two pieces separately.
#pragma once
#include "kernels.hpp"

namespace hofks {

constexpr int W2_CELLS = 128;  // cells per block row segment
typedef double w2v __attribute__((ext_vector_type(2)));  // a lane's two pieces

template <int BCX, int UNR, int NG>
__global__ __launch_bounds__(64 * NG) void k_kinetic2w(StepArgs<double> a, Geom G, int nsegw) {
  using T = double;
  constexpr int NM = 4;
  constexpr int RS = rec_stride<2, T>();
  constexpr int NCH = (rec_values<2, T>() + 1) / 2;  // 16-byte chunks of a record
  constexpr int C16 = RS / 2;
  constexpr int FS = row_rec_stride<T>();
  using V = double2;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int SW = W2_CELLS + G.nv1 - 1;  // upstream cells of a segment
  const int SP = (SW + 1) / 2;           // records per parity half

  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int seg = tile % nsegw;
  const int row = tile / nsegw;
  const int lane = threadIdx.x & 63;
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int Nx = G.n[0];
  const int x0 = seg * W2_CELLS;
  const int xl = x0 + 2 * lane;  // the lane's first cell
  const bool act0 = xl < Nx, act1 = xl + 1 < Nx;
  const int jy = row % G.n[1];
  const int dest = row * Nx + xl;
  const int lofs = G.nv1 - 1 - G.kofs;
  const int xlo = x0 - lofs;
  const T lam = (T)G.lam, mu = (T)G.mu;
  const int nvr = G.nv1;
  const int vr0 = grp * nvr / NG, vr1 = (grp + 1) * nvr / NG;
  T* Lw = lds + (size_t)grp * 2 * SP * FS;

  double SK[2][NM], SE[2][NM];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int r = 0; r < NM; ++r) SK[c][r] = SE[c][r] = 0.0;

  for (int vr = vr0; vr < vr1; ++vr) {
    const int iy = vr;
    const int ky = iy - G.kofs;
    const double vy = vel_node(a.vt, iy).v;
    const double hrow = vel_node(a.vt, iy).v2h;
    const int uy = map_axis(jy - ky, G.n[1], G.bc[1]);
    const int ubase = uy * Nx;

    // stage the row records of the upstream row segment: cell i of the
    // segment (x = xlo + i) at half i % 2, position i / 2
    {
      const V* recv = reinterpret_cast<const V*>(a.rec_in);
      const T vyT = (T)vy, hT = (T)hrow;
      wave_lds_sync();
      for (int i = lane; i < SW; i += 64) {
        const V* src = recv + (size_t)(ubase + map_axis(xlo + i, Nx, G.bc[0])) * C16;
        T rv[NCH * 2];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const V t = src[c];
          rv[2 * c] = t.x;
          rv[2 * c + 1] = t.y;
        }
        // record: [lp, u_x, u_y, beta | p_0..p_3 | e_0..e_3]
        const T beta = rv[3];
        const T q = (vyT - rv[2]) * (vyT - rv[2]);
        const T P0 = rv[NM] + rv[NM + 2] * vyT + rv[2 * NM - 1] * hT;
        const T E0 = rv[2 * NM] + rv[2 * NM + 2] * vyT + rv[3 * NM - 1] * hT;
        T* o = Lw + (size_t)((i & 1) * SP + (i >> 1)) * FS;
        const T f[9] = {rv[0] - beta * q, rv[1], beta, P0, rv[NM + 1], rv[2 * NM - 1],
                        E0, rv[2 * NM + 1], rv[3 * NM - 1]};
#pragma unroll
        for (int c = 0; c < 4; ++c) reinterpret_cast<V*>(o)[c] = V{f[2 * c], f[2 * c + 1]};
        o[8] = f[8];
      }
      wave_lds_sync();
    }
    if (!act0) continue;

    const size_t kbase = (size_t)vr * G.nv1;
    double aK[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    double aE[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int ix0 = 0; ix0 < G.nv1; ix0 += UNR) {
      w2v gv[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int kx = ix0 + u - G.kofs;
        const char* gp = reinterpret_cast<const char*>(a.g_in + (kbase + ix0 + u) * (size_t)G.nc) +
                         (size_t)ubase * sizeof(T);
        // upstream cells of the pair, mapped as the single-cell form does
        const int m0 = map_x<BCX>(xl + Nx, kx, Nx);
        const int m1 = map_x<BCX>(xl + 1 + Nx, kx, Nx);
        if (m1 == m0 + 1) {
          gv[u] = __builtin_nontemporal_load(
              reinterpret_cast<const w2v*>(gp + (unsigned)m0 * (unsigned)sizeof(T)));
        } else {
          gv[u].x = __builtin_nontemporal_load(
              reinterpret_cast<const T*>(gp + (unsigned)m0 * (unsigned)sizeof(T)));
          gv[u].y = __builtin_nontemporal_load(
              reinterpret_cast<const T*>(gp + (unsigned)m1 * (unsigned)sizeof(T)));
        }
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int ix = ix0 + u;
        const int kx = ix - G.kofs;
        const VelNode vn = vel_node(a.vt, ix);
        const T vxT = (T)vn.v;
        const T vhT = (T)vn.v2h;
        T fs[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          // segment index of the upstream cell: 2 lane + (c - kx + lofs)
          const int d = c - kx + lofs;
          const T* rec = Lw + (size_t)((d & 1) * SP + lane + (d >> 1)) * FS;
          T rv[9];
          read_row_rec<T>(rec, rv);
          // row record: [a0, u_x, beta | P0, p_1, p_3 | E0, e_1, e_3]
          const T pp = rv[3] + rv[4] * vxT + rv[5] * vhT;
          const T dx_ = vxT - rv[1];
          const T M = fast_exp<T>(rv[0] - rv[2] * (dx_ * dx_));
          const T E = M + (rv[6] + rv[7] * vxT + rv[8] * vhT);
          const T g = c == 0 ? gv[u].x : gv[u].y;
          fs[c] = lam * g + (mu * M + pp);
          aE[c][0] += E;
          aE[c][1] += vn.v * E;
          aE[c][2] += vn.v2h * E;
          aK[c][0] += fs[c];
          aK[c][1] += vn.v * fs[c];
          aK[c][2] += vn.v2h * fs[c];
        }
        char* op = reinterpret_cast<char*>(a.g_out + (kbase + ix) * (size_t)G.nc) +
                   (size_t)dest * sizeof(T);
        if (act1) {
          __builtin_nontemporal_store(w2v{fs[0], fs[1]}, reinterpret_cast<w2v*>(op));
        } else {
          __builtin_nontemporal_store(fs[0], reinterpret_cast<T*>(op));
        }
      }
    }
    // fold the row into the totals: m = (1, v_x, v_y, |v|^2/2)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      SK[c][0] += aK[c][0];
      SK[c][1] += aK[c][1];
      SK[c][2] += vy * aK[c][0];
      SK[c][3] += aK[c][2] + hrow * aK[c][0];
      SE[c][0] += aE[c][0];
      SE[c][1] += aE[c][1];
      SE[c][2] += vy * aE[c][0];
      SE[c][3] += aE[c][2] + hrow * aE[c][0];
    }
  }

  // combine the wavefronts in LDS (fixed order), then the sums per cell
  __syncthreads();
  double* red = reinterpret_cast<double*>(lds_raw);
  if (grp > 0) {
    double* q = red + ((size_t)(grp - 1) * 64 + lane) * (4 * NM);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        q[c * 2 * NM + r] = SK[c][r];
        q[c * 2 * NM + NM + r] = SE[c][r];
      }
  }
  __syncthreads();
  if (grp != 0 || !act0) return;
  for (int g2 = 1; g2 < NG; ++g2) {
    const double* q = red + ((size_t)(g2 - 1) * 64 + lane) * (4 * NM);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < NM; ++r) {
        SK[c][r] += q[c * 2 * NM + r];
        SE[c][r] += q[c * 2 * NM + NM + r];
      }
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if (c == 1 && !act1) break;
#pragma unroll
    for (int r = 0; r < NM; ++r) {
      a.sums[(size_t)r * G.nc + dest + c] = SK[c][r];
      a.sums[(size_t)(NM + r) * G.nc + dest + c] = SE[c][r];
    }
  }
}

}  // namespace hofks
