// batch.hpp -- batched persistent form: many independent 1D-1V tubes (each
// with its own cells, velocity grid, dt and tau) advanced together.  A step is
// two launches: the Euler launch runs every tube's s MUSCL sub-steps, one
// 1024-thread block per tube (largest first); the kinetic launch is a
// persistent grid pulling items from a queue, an item being a CELLS-cell
// segment of one tube with all its velocities split over 1024/CELLS groups of
// threads, ending with the per-cell update of the segment.
#pragma once
#include "kernels.hpp"

namespace hofks {

struct TubeDev {
  long long g[2];    // piece offsets (floats); g[p] holds f^n when step % 2 == p
  long long rec[2];  // record offsets (floats)
  long long U[2];    // moment offsets (doubles), 3 x Nx each
  long long UE[2];   // Euler sub-step buffers (doubles)
  long long cf;      // pending correction (doubles)
  int vt;            // first velocity node of the tube in the node arena
  int Nx, nv1, kofs;
  double dx, dv, dt, w, lam, mu, gam;
  double A[9];
};

struct BatchArgs {
  float* gar;             // piece arena
  float* rar;             // record arena
  double* dar;            // moment arena
  const VelNode* vtar;    // velocity node arena
  const TubeDev* tubes;
  const int* euler_order; // tubes, most Euler work first
  const int2* items;      // kinetic items (tube, segment), most work first
  int ntubes, nitems;
  int* queue;             // work counters by step parity
  double* alpha;          // [tube][parity][ASTR]: speeds of U^n / U^{n+1}
  int* done;              // unused
  int* tube_s;            // sub-steps of the current step, per tube
  int* tflag;             // per-tube error bits
  int* flag;              // launch-wide bits (bounded waits)
  int parity;
  int s_cap;
};

__device__ __forceinline__ Geom tube_geom(const TubeDev& T) {
  Geom G;
  G.n[0] = T.Nx;
  G.n[1] = G.n[2] = 1;
  G.nc = T.Nx;
  G.nv1 = T.nv1;
  G.kofs = T.kofs;
  G.nv = T.nv1;
  G.bc[0] = 1;
  G.bc[1] = G.bc[2] = 0;
  G.dx = T.dx;
  G.dv = T.dv;
  G.dt = T.dt;
  G.w = T.w;
  G.lam = T.lam;
  G.mu = T.mu;
  G.gam = T.gam;
  return G;
}

// max over a 1024-thread block, result in every thread
__device__ __forceinline__ double block_max_1024(double v, double* red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double m = red[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = fmax(m, red[i]);
  return m;
}

__device__ void batch_euler_item(const BatchArgs& a, int t, double* red) {
  t = __builtin_amdgcn_readfirstlane(t);
  const TubeDev T = a.tubes[t];
  const Geom G = tube_geom(T);
  const int p = a.parity;
  double* alpha_r = a.alpha + ((size_t)t * 2 + p) * ASTR;
  double* alpha_w = a.alpha + ((size_t)t * 2 + (p ^ 1)) * ASTR;
  double alpha = __hip_atomic_load(alpha_r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  bool over;
  const int s = substeps<1>(&alpha, G, a.s_cap, &over);
  if (threadIdx.x == 0) {
    alpha_w[0] = 0.0;  // the kinetic launch reduces the speeds of U^{n+1} here
    a.tube_s[t] = s;
    if (over) atomicOr(a.tflag + t, FLAG_SUBSTEP);
  }
  const bool need = G.mu != 0.0;
  if (need) {
    const double* U = a.dar + T.U[p];
    double* UE0 = a.dar + T.UE[0];
    double* UE1 = a.dar + T.UE[1];
    const double dts_dx = (G.dt / s) / G.dx;
    bool phys = true;
    for (int i = 0; i < s; ++i) {
      const double* in = (i == 0) ? U : ((i & 1) ? UE1 : UE0);
      double* out = ((i + 1) & 1) ? UE1 : UE0;
      double mx = 0.0;
      for (int j = threadIdx.x; j < G.nc; j += blockDim.x) {
        double Un[3];
        phys &= euler_cell<1>(in, j, &alpha, dts_dx, G, 0, Un);
        out[j] = Un[0];
        out[(size_t)G.nc + j] = Un[1];
        out[2 * (size_t)G.nc + j] = Un[2];
        double sp;
        phys &= lf_speeds<1>(Un, G.gam, &sp);
        mx = fmax(mx, sp);
      }
      alpha = block_max_1024(mx, red);  // also orders this sub-step's writes
    }
    if (!phys) atomicOr(a.tflag + t, FLAG_NONPHYS);
  }
}

template <int CELLS, int UNR>
__device__ void batch_kinetic_item(const BatchArgs& a, int it, unsigned char* lds_raw) {
  constexpr int VG = 1024 / CELLS;
  constexpr int RS = rec_stride<1, float>();
  constexpr int C16 = RS / 4;
  it = __builtin_amdgcn_readfirstlane(it);
  const int2 item = a.items[it];
  const int t = __builtin_amdgcn_readfirstlane(item.x);
  const TubeDev T = a.tubes[t];
  const Geom G = tube_geom(T);
  const int p = a.parity;
  const float* gin = a.gar + T.g[p];
  float* gout = a.gar + T.g[p ^ 1];
  const float* recin = a.rar + T.rec[p];
  float* recout = a.rar + T.rec[p ^ 1];
  const VelNode* vt = a.vtar + T.vt;
  const int Nx = G.n[0];
  const int cl = threadIdx.x % CELLS, vg = threadIdx.x / CELLS;
  const int x0 = __builtin_amdgcn_readfirstlane(item.y) * CELLS;
  const int x = x0 + cl;
  const bool active = x < Nx;
  const int SW = CELLS + G.nv1 - 1;
  const int lofs = G.nv1 - 1 - G.kofs;
  const int xlo = x0 - lofs;
  float* lds = reinterpret_cast<float*>(lds_raw);

  // records of the upstream segment (outflow: clamped to the tube)
  __syncthreads();
  {
    float4* ldsv = reinterpret_cast<float4*>(lds);
    const float4* recv = reinterpret_cast<const float4*>(recin);
    for (int idx = threadIdx.x; idx < SW * C16; idx += blockDim.x) {
      const int c = idx % C16, i = idx / C16;
      const int ux = min(max(xlo + i, 0), Nx - 1);
      ldsv[idx] = recv[(size_t)ux * C16 + c];
    }
  }
  __syncthreads();

  const float lam = (float)G.lam, mu = (float)G.mu;
  double aK0 = 0.0, aK1 = 0.0, aK2 = 0.0, aE0 = 0.0, aE1 = 0.0, aE2 = 0.0;
  if (active) {
    const int per = G.nv1 / VG;
    const int ixa = vg * per;
    const int xN = x + Nx;
    for (int ix0 = ixa; ix0 < ixa + per; ix0 += UNR) {
      float gv[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int ix = ix0 + u;
        gv[u] = gin[(size_t)ix * Nx + map_x<1>(xN, ix - G.kofs, Nx)];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int ix = ix0 + u;
        const int kx = ix - G.kofs;
        const VelNode vn = vt[ix];
        const float vxT = vn.vf, vhT = vn.v2hf;
        const float4* rp = reinterpret_cast<const float4*>(lds + (cl - kx + lofs) * RS);
        const float4 r0 = rp[0], r1 = rp[1], r2 = rp[2];
        // record: [lp, u, beta | p0 p1 p2 | e0 e1 e2 | pad]
        const float pp = r0.w + r1.x * vxT + r1.y * vhT;
        const float dxv = vxT - r0.y;
        const float M = __expf(r0.x - r0.z * (dxv * dxv));
        const float pe = r1.z + r1.w * vxT + r2.x * vhT;
        const float E = M + pe;
        const float fs = lam * gv[u] + (mu * M + pp);
        gout[(size_t)ix * Nx + x] = fs;
        const double fd = (double)fs, Ed = (double)E;
        aK0 += fd;
        aK1 += vn.v * fd;
        aK2 += vn.v2 * fd;
        aE0 += Ed;
        aE1 += vn.v * Ed;
        aE2 += vn.v2 * Ed;
      }
    }
  }
  // combine the velocity groups in LDS (fixed order)
  __syncthreads();
  double* red = reinterpret_cast<double*>(lds_raw);
  if (vg > 0) {
    double* q = red + ((size_t)(vg - 1) * CELLS + cl) * 6;
    q[0] = aK0;
    q[1] = aK1;
    q[2] = aK2;
    q[3] = aE0;
    q[4] = aE1;
    q[5] = aE2;
  }
  __syncthreads();
  if (vg != 0) return;
  bool phys = true;
  double speed = 0.0;
  if (active) {
    double S[6] = {aK0, aK1, aK2, aE0, aE1, aE2}, C[6] = {0, 0, 0, 0, 0, 0};
    for (int g2 = 1; g2 < VG; ++g2) {
      const double* q = red + ((size_t)(g2 - 1) * CELLS + cl) * 6;
#pragma unroll
      for (int r = 0; r < 6; ++r) two_sum(S[r], C[r], q[r]);
    }
#pragma unroll
    for (int r = 0; r < 6; ++r) S[r] += C[r];
    const double SK[3] = {S[0], S[1], 0.5 * S[2]};
    const double SE[3] = {S[3], S[4], 0.5 * S[5]};
    const int s = a.tube_s[t];
    const double* UEs = a.dar + T.UE[s & 1];
    double delta[3] = {0.0, 0.0, 0.0};
    if (G.mu != 0.0) {
#pragma unroll
      for (int r = 0; r < 3; ++r)
        delta[r] = G.mu * UEs[(size_t)r * Nx + x] - G.mu * (G.w * SE[r]);
    }
    double Un[3], cfv[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) Un[r] = G.w * SK[r] + delta[r];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      cfv[r] = T.A[3 * r] * delta[0] + T.A[3 * r + 1] * delta[1] + T.A[3 * r + 2] * delta[2];
    Mat A;
#pragma unroll
    for (int q = 0; q < 9; ++q) A.a[q] = T.A[q];
    phys = cell_record<1, float>(Un, cfv, G, A, vt, recout + (size_t)x * RS, &speed);
    double* Uo = a.dar + T.U[p ^ 1];
    double* cf = a.dar + T.cf;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      Uo[(size_t)r * Nx + x] = Un[r];
      cf[(size_t)r * Nx + x] = cfv[r];
    }
    if (!phys && G.mu != 0.0) atomicOr(a.tflag + t, FLAG_NONPHYS);
  }
  const double m = wave_max(phys ? speed : 0.0);
  if ((threadIdx.x & 63) == 0) atomic_max_pos(a.alpha + ((size_t)t * 2 + (p ^ 1)) * ASTR, m);
}

// Euler launch: one 1024-thread block per tube, the tubes with the most
// Euler work first.
__global__ __launch_bounds__(1024) void k_batch_euler(BatchArgs a) {
  __shared__ double red[16];
  batch_euler_item(a, a.euler_order[blockIdx.x], red);
}

// Kinetic launch: persistent blocks pull (tube, segment) items from a queue,
// the items with the most work first; the Euler launch of the step is done.
template <int CELLS, int UNR>
__global__ __launch_bounds__(1024) void k_batch_kinetic(BatchArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  __shared__ int s_item;
  const int p = a.parity;
  if (blockIdx.x == 0 && threadIdx.x == 0) a.queue[p ^ 1] = 0;  // for the next step
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(a.queue + p, 1);
    __syncthreads();
    const int item = s_item;
    if (item >= a.nitems) break;
    batch_kinetic_item<CELLS, UNR>(a, item, lds_raw);
  }
}

}  // namespace hofks
