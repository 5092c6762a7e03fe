// batch.hpp -- batched persistent form: many independent 1D-1V tubes (each
// with its own cells, velocity grid, dt and tau) advanced together.  A step is
// two launches: a persistent grid pulls from one queue first the Euler solves
// of the tubes (one 1024-thread block per tube, s MUSCL sub-steps with the
// tube's moments in registers, largest first) and then the kinetic items (a CELLS-cell segment of one tube with
// all its velocities split over 1024/CELLS groups of threads, writing the
// moment sums of its cells), so the two run side by side; the update launch
// then forms U^{n+1} and the next records cell by cell.
#pragma once
#include "kernels.hpp"

namespace hofks {

struct TubeDev {
  long long g[2];    // piece offsets (floats); g[p] holds f^n when step % 2 == p
  long long rec[2];  // record offsets (floats)
  long long U[2];    // moment offsets (doubles), 3 x Nx each
  long long UE[2];   // Euler sub-step buffers (doubles)
  long long cf;      // pending correction (doubles)
  long long S;       // moment sums of f* and E per cell (doubles), 6 x Nx
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
  G.offl = 0;
  G.dx = T.dx;
  G.dv = T.dv;
  G.dt = T.dt;
  G.w = T.w;
  G.lam = T.lam;
  G.mu = T.mu;
  G.gam = T.gam;
  G.sfac = 2.0;
  G.lam_r = T.lam;
  G.mu_r = T.mu;
  return G;
}

// max over the block (up to 1024 threads), result in every thread
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

// Euler solve of one tube by segments of EUL_TPB cells (eq. (discmom) with
// the limited slopes of section 4.3.2): per sub-step and segment the block
// evaluates the split fluxes W+- of the segment and two cells on each side
// once into LDS, then the face fluxes psi of the segment's faces into LDS,
// then the new cell values, written out of place to the other sub-step
// buffer.  Every flux and every face is computed once (the global-memory
// form evaluates five fluxes and two faces per cell).  Same arithmetic per
// face as `euler_cell`; the result is UE[s % 2].
constexpr int EUL_TPB = 1024;
constexpr size_t EUL_LDS = (size_t)((EUL_TPB + 4) * 6 + (EUL_TPB + 1) * 3) * sizeof(double);
constexpr size_t EUL_REG_LDS = 2 * EUL_LDS;  // the register form alternates two sets

__device__ void batch_euler_seg(const BatchArgs& a, int t, double* L, double* red) {
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
  if (G.mu == 0.0) return;
  const int Nx = G.nc;
  double* Wl = L;                           // [EUL_TPB + 4][6]: W+ (3), W- (3)
  double* Pl = L + (EUL_TPB + 4) * 6;       // [EUL_TPB + 1][3]: face fluxes
  const double* U0 = a.dar + (p ? T.U[1] : T.U[0]);
  double* UE0 = a.dar + T.UE[0];
  double* UE1 = a.dar + T.UE[1];
  const double dts_dx = (G.dt / s) / G.dx;
  bool phys = true;
  for (int i = 0; i < s; ++i) {
    const double* in = (i == 0) ? U0 : ((i & 1) ? UE1 : UE0);
    double* out = ((i + 1) & 1) ? UE1 : UE0;
    double mx = 0.0;
    for (int x0 = 0; x0 < Nx; x0 += EUL_TPB) {
      // fluxes of cells x0-2 .. x0+EUL_TPB+1 (outflow: clamped)
      for (int q = threadIdx.x; q < EUL_TPB + 4; q += blockDim.x) {
        const int jj = min(max(x0 - 2 + q, 0), Nx - 1);
        const double Uq[3] = {in[jj], in[(size_t)Nx + jj], in[2 * (size_t)Nx + jj]};
        double Wp[3], Wm[3];
        phys &= split_flux<1>(Uq, 0, alpha, G.gam, Wp, Wm);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          Wl[q * 6 + r] = Wp[r];
          Wl[q * 6 + 3 + r] = Wm[r];
        }
      }
      __syncthreads();
      // face f between cells x0+f-1 and x0+f uses the fluxes of cells
      // x0+f-2 .. x0+f+1, i.e. entries f .. f+3
      for (int f = threadIdx.x; f <= EUL_TPB; f += blockDim.x) {
        const double* w = Wl + f * 6;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const double spl = vl_slope(w[6 + r] - w[r], w[12 + r] - w[6 + r], 0);
          const double sml = vl_slope(w[15 + r] - w[9 + r], w[21 + r] - w[15 + r], 0);
          Pl[f * 3 + r] = 0.5 * (w[6 + r] + w[15 + r]) + 0.25 * (spl - sml);
        }
      }
      __syncthreads();
      const int j = x0 + threadIdx.x;
      if (threadIdx.x < EUL_TPB && j < Nx) {
        const int c = threadIdx.x;
        double Un[3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
          Un[r] = in[(size_t)r * Nx + j] - dts_dx * (Pl[(c + 1) * 3 + r] - Pl[c * 3 + r]);
#pragma unroll
        for (int r = 0; r < 3; ++r) out[(size_t)r * Nx + j] = Un[r];
        if (i + 1 < s) {
          double sp;
          phys &= lf_speeds<1>(Un, G.gam, &sp);
          mx = fmax(mx, sp);
        }
      }
      __syncthreads();  // the next segment overwrites the LDS tiles
    }
    if (i + 1 < s) alpha = block_max_1024(mx, red);  // also orders this sub-step's writes
  }
  if (!phys) atomicOr(a.tflag + t, FLAG_NONPHYS);
}

// Euler solve of one tube of at most EUL_TPB * EUL_CPT cells with the
// moments held in registers for all s sub-steps: thread t owns cells
// t + k EUL_TPB (slab k).  Per sub-step and slab the owners write the split
// fluxes W+- of their cells (and of the two cells beyond each end of the
// slab, which they also own, or the boundary cell for the clamped outflow
// entries) into LDS, the faces of the slab are formed once each, and every
// owner updates its cell; memory is read once at the start and written once
// at the end (UE[s % 2]).  Same arithmetic per flux and face as
// `batch_euler_seg` and `euler_cell`.
constexpr int EUL_CPT = 4;

__device__ void batch_euler_reg(const BatchArgs& a, int t, double* L, double* red) {
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
  if (G.mu == 0.0) return;
  const int Nx = G.nc;
  const int nslab = (Nx + EUL_TPB - 1) / EUL_TPB;
  // two sets of LDS entries, alternating between slabs, so that a slab's
  // writes need no barrier after the previous slab's reads (the barriers
  // inside each slab already separate slab k's reads from slab k+2's writes)
  double* Wl0 = L;                       // [EUL_TPB + 4][6]: W+ (3), W- (3)
  double* Pl0 = L + (EUL_TPB + 4) * 6;   // [EUL_TPB + 1][3]: face fluxes
  double* Wl1 = L + EUL_LDS / sizeof(double);
  double* Pl1 = Wl1 + (EUL_TPB + 4) * 6;
  const int tid = threadIdx.x;
  const double* U0 = a.dar + (p ? T.U[1] : T.U[0]);
  double Ur[EUL_CPT][3], Un[EUL_CPT][3];
#pragma unroll
  for (int k = 0; k < EUL_CPT; ++k) {
    const int c = k * EUL_TPB + tid;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      Ur[k][r] = c < Nx ? U0[(size_t)r * Nx + c] : 0.0;
      Un[k][r] = Ur[k][r];
    }
  }
  const double dts_dx = (G.dt / s) / G.dx;
  bool phys = true;
  for (int i = 0; i < s; ++i) {
    double mx = 0.0;
#pragma unroll
    for (int k = 0; k < EUL_CPT; ++k) {
      if (k >= nslab) break;
      double* Wl = (k & 1) ? Wl1 : Wl0;
      double* Pl = (k & 1) ? Pl1 : Pl0;
      const int x0 = k * EUL_TPB;
      const int end = min(x0 + EUL_TPB, Nx);
      const int nent = end - x0 + 4;  // flux entries of cells x0-2 .. end+1
      // entries written by this thread: those whose (clamped) cell it owns,
      // among its cells of slabs k-1, k and k+1
#pragma unroll
      for (int dk = -1; dk <= 1; ++dk) {
        const int kk = k + dk;
        if (kk < 0 || kk >= EUL_CPT) continue;
        const int c = kk * EUL_TPB + tid;
        if (c >= Nx) continue;
        int qlo = c - x0 + 2, qhi = qlo;
        if (c == 0) qlo = 0;
        if (c == Nx - 1) qhi = nent - 1;
        qlo = max(qlo, 0);
        qhi = min(qhi, nent - 1);
        if (qlo > qhi) continue;
        double Wp[3], Wm[3];
        if (k > 0 && (dk < 0 || (dk == 0 && tid < 2))) {
          // cells x0-2, x0-1, x0 and x0+1: this thread formed their split
          // fluxes in the previous slab's pass, in the other set of entries
          const double* Wq = ((k & 1) ? Wl0 : Wl1) + (c - x0 + EUL_TPB + 2) * 6;
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            Wp[r] = Wq[r];
            Wm[r] = Wq[3 + r];
          }
        } else {
          phys &= split_flux<1>(Ur[kk], 0, alpha, G.gam, Wp, Wm);
        }
        for (int q = qlo; q <= qhi; ++q) {
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            Wl[q * 6 + r] = Wp[r];
            Wl[q * 6 + 3 + r] = Wm[r];
          }
        }
        if (k == 0 && c == 0) {
          // the tube's left face: entries 0..2 all hold cell 0, so both
          // limited slopes vanish and the flux is the mean of W+ and W- of
          // cell 0 (the value the face loop below would give)
#pragma unroll
          for (int r = 0; r < 3; ++r) Pl[r] = 0.5 * (Wp[r] + Wm[r]) + 0.25 * (0.0 - 0.0);
        }
      }
      __syncthreads();
      // face f between cells x0+f-1 and x0+f uses entries f .. f+3; face 0
      // of a later slab is the previous slab's last face, kept in the other
      // set, so the 1024 threads form the at most 1024 remaining faces at once
      for (int f = tid + 1; f <= end - x0; f += blockDim.x) {
        const double* w = Wl + f * 6;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const double spl = vl_slope(w[6 + r] - w[r], w[12 + r] - w[6 + r], 0);
          const double sml = vl_slope(w[15 + r] - w[9 + r], w[21 + r] - w[15 + r], 0);
          Pl[f * 3 + r] = 0.5 * (w[6 + r] + w[15 + r]) + 0.25 * (spl - sml);
        }
      }
      __syncthreads();
      if (x0 + tid < Nx) {
        const double* Pleft = (tid == 0 && k > 0) ? ((k & 1) ? Pl0 : Pl1) + EUL_TPB * 3 : Pl + tid * 3;
#pragma unroll
        for (int r = 0; r < 3; ++r)
          Un[k][r] = Ur[k][r] - dts_dx * (Pl[(tid + 1) * 3 + r] - Pleft[r]);
        if (i + 1 < s) {
          double sp;
          phys &= lf_speeds<1>(Un[k], G.gam, &sp);
          mx = fmax(mx, sp);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < EUL_CPT; ++k)
#pragma unroll
      for (int r = 0; r < 3; ++r) Ur[k][r] = Un[k][r];
    if (i + 1 < s) alpha = block_max_1024(mx, red);
  }
  double* out = a.dar + ((s & 1) ? T.UE[1] : T.UE[0]);
#pragma unroll
  for (int k = 0; k < EUL_CPT; ++k) {
    const int c = k * EUL_TPB + tid;
    if (c < Nx) {
#pragma unroll
      for (int r = 0; r < 3; ++r) out[(size_t)r * Nx + c] = Ur[k][r];
    }
  }
  if (!phys) atomicOr(a.tflag + t, FLAG_NONPHYS);
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
  // (selects, not indexes: a dynamic index would put the tube record in scratch)
  const float* gin = a.gar + (p ? T.g[1] : T.g[0]);
  float* gout = a.gar + (p ? T.g[0] : T.g[1]);
  const float* recin = a.rar + (p ? T.rec[1] : T.rec[0]);
  float* recout = a.rar + (p ? T.rec[0] : T.rec[1]);
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
        const char* gp = reinterpret_cast<const char*>(gin + (size_t)ix * Nx);
        gv[u] = *reinterpret_cast<const float*>(
            gp + (unsigned)map_x<1>(xN, ix - G.kofs, Nx) * (unsigned)sizeof(float));
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int ix = ix0 + u;
        const int kx = ix - G.kofs;
        const VelNode vn = vel_node(vt, ix);
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
        *reinterpret_cast<float*>(reinterpret_cast<char*>(gout + (size_t)ix * Nx) +
                                  (unsigned)x * (unsigned)sizeof(float)) = fs;
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
  if (vg != 0 || !active) return;
  double S[6] = {aK0, aK1, aK2, aE0, aE1, aE2}, C[6] = {0, 0, 0, 0, 0, 0};
  for (int g2 = 1; g2 < VG; ++g2) {
    const double* q = red + ((size_t)(g2 - 1) * CELLS + cl) * 6;
#pragma unroll
    for (int r = 0; r < 6; ++r) two_sum(S[r], C[r], q[r]);
  }
  double* Sg = a.dar + T.S;
#pragma unroll
  for (int r = 0; r < 6; ++r) Sg[(size_t)r * Nx + x] = S[r] + C[r];
}

// Per-cell update of one item after the Euler solve of its tube: delta,
// U^{n+1}, cf and the next record from the moment sums (eqs. (UK), (mom),
// (minim_full)); the speeds of U^{n+1} go to the tube's next speed row.
__device__ void batch_update_item(const BatchArgs& a, int it) {
  constexpr int RS = rec_stride<1, float>();
  it = __builtin_amdgcn_readfirstlane(it);
  const int2 item = a.items[it];
  const int t = __builtin_amdgcn_readfirstlane(item.x);
  const TubeDev T = a.tubes[t];
  const Geom G = tube_geom(T);
  const int p = a.parity;
  const int Nx = G.n[0];
  const int x = item.y * (int)blockDim.x + (int)threadIdx.x;
  bool phys = true;
  double speed = 0.0;
  if (x < Nx) {
    const double* Sg = a.dar + T.S;
    double S[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) S[r] = Sg[(size_t)r * Nx + x];
    const double SK[3] = {S[0], S[1], 0.5 * S[2]};
    const double SE[3] = {S[3], S[4], 0.5 * S[5]};
    const int s = a.tube_s[t];
    const double* UEs = a.dar + ((s & 1) ? T.UE[1] : T.UE[0]);
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
    float* recout = a.rar + (p ? T.rec[0] : T.rec[1]);
    phys = cell_record<1, float>(Un, cfv, G, A, recout + (size_t)x * RS, &speed);
    double* Uo = a.dar + (p ? T.U[0] : T.U[1]);
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

// Step launch: persistent 1024-thread blocks pull work from one queue: the
// Euler solves of the tubes first (most Euler work first), then the kinetic
// items (relaxation, shift and moment sums of a (tube, segment), most work
// first), which need nothing from the Euler solves.  (1024, 4): four waves
// per SIMD.
template <int CELLS, int UNR>
__global__ __launch_bounds__(1024, 4) void k_batch_step(BatchArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  __shared__ double red[16];
  __shared__ int s_item;
  const int p = a.parity;
  if (blockIdx.x == 0 && threadIdx.x == 0) a.queue[p ^ 1] = 0;  // for the next step
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(a.queue + p, 1);
    __syncthreads();
    const int w = s_item;
    if (w < a.ntubes) {
      const int tb = a.euler_order[w];
      if (a.tubes[tb].Nx <= EUL_TPB * EUL_CPT)
        batch_euler_reg(a, tb, reinterpret_cast<double*>(lds_raw), red);
      else
        batch_euler_seg(a, tb, reinterpret_cast<double*>(lds_raw), red);
    } else if (w < a.ntubes + a.nitems)
      batch_kinetic_item<CELLS, UNR>(a, w - a.ntubes, lds_raw);
    else
      break;
  }
}

// Update launch: one block of CELLS threads per kinetic item.
__global__ __launch_bounds__(512) void k_batch_update(BatchArgs a) {
  batch_update_item(a, blockIdx.x);
}

}  // namespace hofks
