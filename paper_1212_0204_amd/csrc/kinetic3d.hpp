// Kinetic kernel for 3D-3V steps with an Euler solve (relaxation, shift and
// moment sums of section 4.3.1, eq. (UK)), organised around the reuse of
// staged upstream records.  One block holds RY = 4 consecutive y rows of 64
// cells at one z (one wavefront per row, one lane per cell).  For velocity
// row (k_y, k_z) wavefront w needs the records of upstream row
// y + w - k_y at z - k_z; for consecutive k_y the four rows slide by one, so
// the block keeps them in a ring of RY + 1 LDS slots and stages one new row
// per k_y step while the pieces of the current step are processed: 27 row
// segments per k_z instead of 96.  Since k_z is fixed while a ring is in use,
// staging folds the v_z terms into the record (12 values instead of 15):
//   log M = lp - beta |v - u|^2  ->  a0 - beta ((v_x - u_x)^2 + (v_y - u_y)^2),
//   p . m(v)                     ->  P0 + p_1 v_x + p_2 v_y + p_4 (v_x^2 + v_y^2)/2,
// with a0 = lp - beta (v_z - u_z)^2 and P0 = p_0 + p_3 v_z + p_4 v_z^2 / 2 (the
// same for e).  Each lane sums its cell's moments over all velocities and
// writes them for the per-cell update (k_cell_update).
#pragma once
#include "kernels.hpp"

namespace hofks {

constexpr int RY = 4;

// 16-byte chunks of one folded record (12 values), odd so that the lanes of
// a wavefront reading consecutive records hit distinct LDS banks
template <typename T>
__host__ __device__ constexpr int fold3_chunks() {
  return ((12 * (int)sizeof(T) / 16) | 1);
}

template <typename T, bool COMP, int BCX, int UNR>
__global__ __launch_bounds__(64 * RY) void k_kinetic3(StepArgs<T> a, Geom G, int nyb) {
  constexpr int D = 3, NM = 5;
  constexpr int RS = rec_stride<D, T>();
  constexpr int PER16 = 16 / (int)sizeof(T);
  constexpr int NCH = (rec_values<D, T>() + PER16 - 1) / PER16;
  constexpr int C16 = RS / PER16;
  constexpr int NF = 12 / PER16;            // chunks of a folded record
  constexpr int FC = fold3_chunks<T>();     // their stride
  constexpr int FS = FC * PER16;            // in values
  using V = typename Vec16<T>::type;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int SW = 64 + G.nv1 - 1;
  const int nseg = (G.n[0] + 63) / 64;

  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int seg = tile % nseg;
  const int yb = (tile / nseg) % nyb, z = tile / nseg / nyb;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int Nx = G.n[0], Ny = G.n[1], Nz = G.n[2];
  const int x0 = seg * 64, x = x0 + lane, y = yb * RY + w;
  const bool active = x < Nx && y < Ny;
  const int dest = (z * Ny + (y < Ny ? y : Ny - 1)) * Nx + x;
  const unsigned dboff = (unsigned)dest * (unsigned)sizeof(T);
  const int xN = x + Nx;
  const int lofs = G.nv1 - 1 - G.kofs;
  const int xlo = x0 - lofs;
  const T lam = (T)G.lam, mu = (T)G.mu;
  const V* recv = reinterpret_cast<const V*>(a.rec_in);
  const int nslot = RY + 1;

  // stage the folded records of upstream row r (unwrapped) at plane uz into
  // its slot, one record per thread, cells in reverse order (the pieces of
  // increasing k_x then read increasing addresses)
  auto stage = [&](int r, int uz, T vzT, T vz2hT) {
    const int slot = ((r % nslot) + nslot) % nslot;
    V* dst = reinterpret_cast<V*>(lds + (size_t)slot * SW * FS);
    const int uy = map_axis(r, Ny, G.bc[1]);
    const size_t base = (size_t)(uz * Ny + uy) * Nx;
    for (int i = threadIdx.x; i < SW; i += blockDim.x) {
      const V* src = recv + (base + map_axis(xlo + i, Nx, G.bc[0])) * C16;
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
      // record: [lp, u_x, u_y, u_z, beta | p_0..p_4 | e_0..e_4]
      const T dz_ = vzT - rv[3];
      T o[12];
      o[0] = rv[0] - rv[4] * (dz_ * dz_);
      o[1] = rv[1];
      o[2] = rv[2];
      o[3] = rv[4];
      o[4] = rv[NM] + rv[NM + 3] * vzT + rv[2 * NM - 1] * vz2hT;
      o[5] = rv[NM + 1];
      o[6] = rv[NM + 2];
      o[7] = rv[2 * NM - 1];
      o[8] = rv[2 * NM] + rv[2 * NM + 3] * vzT + rv[3 * NM - 1] * vz2hT;
      o[9] = rv[2 * NM + 1];
      o[10] = rv[2 * NM + 2];
      o[11] = rv[3 * NM - 1];
#pragma unroll
      for (int c = 0; c < NF; ++c) {
        V t;
        if constexpr (sizeof(T) == 8) {
          t.x = o[2 * c];
          t.y = o[2 * c + 1];
        } else {
          t.x = o[4 * c];
          t.y = o[4 * c + 1];
          t.z = o[4 * c + 2];
          t.w = o[4 * c + 3];
        }
        dst[(size_t)(SW - 1 - i) * FC + c] = t;
      }
    }
  };

  double SK[NM], SE[NM], CK[NM], CE[NM];
#pragma unroll
  for (int r = 0; r < NM; ++r) SK[r] = SE[r] = CK[r] = CE[r] = 0.0;

  for (int iz = 0; iz < G.nv1; ++iz) {
    const int kz = iz - G.kofs;
    const int uz = map_axis(z - kz, Nz, G.bc[2]);
    const double vz = vel_node(a.vt, iz).v;
    const T vzT = (T)vz, vz2hT = (T)vel_node(a.vt, iz).v2h;
    // rows of the first k_y step: yb RY - ky .. + RY - 1 with ky = -kofs
    __syncthreads();  // the previous k_z's slots are no longer read
    for (int q = 0; q < RY; ++q) stage(yb * RY + G.kofs + q, uz, vzT, vz2hT);
    __syncthreads();
    for (int iy = 0; iy < G.nv1; ++iy) {
      const int ky = iy - G.kofs;
      // the row the next k_y step adds (the slot last read one step ago)
      if (iy + 1 < G.nv1) stage(yb * RY - ky - 1, uz, vzT, vz2hT);
      const int r = y - ky;  // unwrapped upstream row of this wavefront
      const int slot = ((r % nslot) + nslot) % nslot;
      const T* Lw = lds + (size_t)slot * SW * FS;
      const int uy = map_axis(r, Ny, G.bc[1]);
      const int ubase = (uz * Ny + uy) * Nx;
      const double vy = vel_node(a.vt, iy).v;
      const double hrow = vel_node(a.vt, iy).v2h + vel_node(a.vt, iz).v2h;
      const size_t kbase = ((size_t)iz * G.nv1 + iy) * G.nv1;
      const T vyT = (T)vy, vy2hT = (T)vel_node(a.vt, iy).v2h;
      double aK0 = 0.0, aK1 = 0.0, aK2 = 0.0, aE0 = 0.0, aE1 = 0.0, aE2 = 0.0;
      if (active) {
#pragma unroll 1
        for (int ix0 = 0; ix0 < G.nv1; ix0 += UNR) {
          T gv[UNR];
#pragma unroll
          for (int u = 0; u < UNR; ++u) {
            const int ix = ix0 + u;
            const char* gp = reinterpret_cast<const char*>(a.g_in + (kbase + ix) * (size_t)G.nc);
            const T* src = reinterpret_cast<const T*>(
                gp + (unsigned)(ubase + map_x<BCX>(xN, ix - G.kofs, Nx)) * (unsigned)sizeof(T));
            gv[u] = HOFKS_NT ? __builtin_nontemporal_load(src) : *src;
          }
          const T* Lb = Lw + (SW - 1 - lane - lofs - G.kofs + ix0) * FS;
#pragma unroll
          for (int u = 0; u < UNR; ++u) {
            const int ix = ix0 + u;
            const VelNode vn = vel_node(a.vt, ix);
            const double vx = vn.v;
            const T vxT = (sizeof(T) == 4) ? (T)vn.vf : (T)vn.v;
            const T vhT = (sizeof(T) == 4) ? (T)(vy2hT + (T)vn.v2hf) : (T)(vy2hT + vn.v2h);
            const V* rp = reinterpret_cast<const V*>(Lb + u * FS);
            T rv[12];
#pragma unroll
            for (int c = 0; c < NF; ++c) {
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
            // folded record: [a0, u_x, u_y, beta | P0, p_1, p_2, p_4 | E0, e_1, e_2, e_4]
            const T pp = rv[4] + rv[5] * vxT + rv[6] * vyT + rv[7] * vhT;
            const T dx_ = vxT - rv[1], dy_ = vyT - rv[2];
            const T M = fast_exp<T>(rv[0] - rv[3] * (dx_ * dx_ + dy_ * dy_));
            const T pe = rv[8] + rv[9] * vxT + rv[10] * vyT + rv[11] * vhT;
            const T E = M + pe;
            const T fs = lam * gv[u] + (mu * M + pp);
            T* op = reinterpret_cast<T*>(
                reinterpret_cast<char*>(a.g_out + (kbase + ix) * (size_t)G.nc) + dboff);
            if (HOFKS_NT)
              __builtin_nontemporal_store(fs, op);
            else
              *op = fs;
            const double fd = (double)fs, Ed = (double)E;
            aK0 += fd;
            aK1 += vx * fd;
            aK2 += vn.v2h * fd;
            aE0 += Ed;
            aE1 += vx * Ed;
            aE2 += vn.v2h * Ed;
          }
        }
        // fold the row: m = (1, v_x, v_y, v_z, |v|^2/2)
        const double rk[NM] = {aK0, aK1, vy * aK0, vz * aK0, aK2 + hrow * aK0};
        const double re[NM] = {aE0, aE1, vy * aE0, vz * aE0, aE2 + hrow * aE0};
#pragma unroll
        for (int q = 0; q < NM; ++q) {
          if (COMP) {
            two_sum(SK[q], CK[q], rk[q]);
            two_sum(SE[q], CE[q], re[q]);
          } else {
            SK[q] += rk[q];
            SE[q] += re[q];
          }
        }
      }
      __syncthreads();  // the next row is staged; this step's slots are read
    }
  }
  if (active) {
#pragma unroll
    for (int q = 0; q < NM; ++q) {
      a.sums[(size_t)q * G.nc + dest] = COMP ? SK[q] + CK[q] : SK[q];
      a.sums[(size_t)(NM + q) * G.nc + dest] = COMP ? SE[q] + CE[q] : SE[q];
    }
  }
}

}  // namespace hofks
