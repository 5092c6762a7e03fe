// batch.hpp -- batched form: many independent 1D-1V tubes (each with its own
// cells, velocity grid, dt and tau) advanced together.  A step is three
// launches: the Euler launch (one block per Euler item: a tube's whole Euler
// solve, or one part of a long tube split over several blocks that meet
// after every sub-step; most work first) and the kinetic launch (one block
// per CELLS-cell segment of a tube with all its velocities split over
// 1024/CELLS groups of threads, writing the moment sums of its cells) run
// side by side on two streams; the update launch then forms U^{n+1} and the
// next records cell by cell.
#pragma once
#include "kernels.hpp"
#include "slope.hpp"

namespace hofks {

constexpr int UPD_CELLS = 256;  // cells per update item (one thread each)

struct TubeDev {
  long long g[2];    // piece offsets (floats); g[p] holds f^n when step % 2 == p
  long long rec[2];  // record offsets (floats)
  long long U[2];    // moment offsets (doubles), 3 x Nx each
  long long UE[2];   // Euler sub-step buffers (doubles)
  long long cf;      // pending correction (doubles)
  long long S;       // moment sums of f* and E per cell (doubles), 6 x Nx
  long long X;       // part exchange rows (doubles), 2 x ceil(Nx / 1024) x XSTR
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
  const int4* eitems;     // Euler items, most work first: (tube, 0, 0, 0) whole,
                          // (tube, part, parts, 1) one part, (tube, tube or -1, CPT, 2) a pair
  const int2* items;      // kinetic items (tube, segment) dealt to the dies; tube -1: none
  const int2* uitems;     // update items (tube, UPD_CELLS-cell segment), the same dies
  int neuler, nitems;
  int part_cells;         // cells per part of a split Euler solve (1024 or 2048)
  unsigned* ebar;         // [tube][parity]: arrivals at the part barriers
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

// 1/x from the hardware reciprocal refined by two Newton steps (within a
// few ulp of the IEEE quotient, and a shorter dependency chain)
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

// max(v, v of the lane that DPP control CTRL selects) for the rows in
// ROW_MASK; lanes without a source keep v
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_max(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, ROW_MASK, 0xF,
                                             false);
  return fmax(v, __longlong_as_double(((long long)hi << 32) | (unsigned)lo));
}

// maximum over the wavefront, in every lane: row shifts by 1, 2, 4 and 8
// leave each row's maximum in its lane 15, the row broadcasts carry rows 0
// and 2 into rows 1 and 3 and then row 1 into rows 2 and 3, and lane 63 is
// read back (cross-lane moves of the ALU instead of LDS permutes)
__device__ __forceinline__ double wave_max_dpp(double v) {
  v = dpp_max<0x111, 0xF>(v);
  v = dpp_max<0x112, 0xF>(v);
  v = dpp_max<0x114, 0xF>(v);
  v = dpp_max<0x118, 0xF>(v);
  v = dpp_max<0x142, 0xA>(v);
  v = dpp_max<0x143, 0xC>(v);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Flux F(U) of one 1D cell from U and 1/rho, with the expressions of
// split_flux (W+- = F +- alpha U); false if the state is not physical
__device__ __forceinline__ bool flux1(const double* U, double irho, double* F) {
  const double rho = U[0];
  const double u = U[1] * irho;
  const double usq = u * u;
  const double p = fma(-rho, usq, 2.0 * U[2]);
  F[0] = U[1];
  F[1] = fma(U[1], u, p);
  F[2] = (U[2] + p) * u;
  return (rho > 0.0) && (p > 0.0) && isfinite(rho) && isfinite(p) && isfinite(usq);
}

// Lax-Friedrichs speed |u| + sqrt(gam p / rho) of one 1D cell (p = rho
// theta) from U and 1/rho; 0 and false if the state is not physical
__device__ __forceinline__ bool speed1(const double* U, double irho, double gam, double* sp) {
  const double rho = U[0];
  const double u = U[1] * irho;
  const double usq = u * u;
  const double p = fma(-rho, usq, 2.0 * U[2]);
  const bool ok = (rho > 0.0) && (p > 0.0) && isfinite(rho) && isfinite(p) && isfinite(usq);
  *sp = ok ? fabs(u) + sqrt(gam * p * irho) : 0.0;
  return ok;
}

// W+ (w[0..2]) and W- (w[3..5]) of one cell
__device__ __forceinline__ void wsplit(const double* U, const double* F, double alpha, double* w) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    w[r] = fma(alpha, U[r], F[r]);
    w[3 + r] = fma(-alpha, U[r], F[r]);
  }
}

// face flux between the cells of entries 1 and 2 of a four-entry window
// (the face arithmetic of section 4.3.2 as in the other Euler forms)
__device__ __forceinline__ void face4(const double* w0, const double* w1, const double* w2,
                                      const double* w3, double* fc) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double spl = vl_slope_sel(w1[r] - w0[r], w2[r] - w1[r]);
    const double sml = vl_slope_sel(w2[3 + r] - w1[3 + r], w3[3 + r] - w2[3 + r]);
    fc[r] = fma(0.25, spl - sml, 0.5 * (w1[r] + w2[3 + r]));
  }
}

// Euler solve of one tube by segments of EUL_TPB cells (eq. (discmom) with
// the limited slopes of section 4.3.2): per sub-step and segment the block
// evaluates the split fluxes W+- of the segment and two cells on each side
// once into LDS, then the face fluxes psi of the segment's faces into LDS,
// then the new cell values, written out of place to the other sub-step
// buffer.  Every flux and every face is computed once (the global-memory
// form evaluates five fluxes and two faces per cell).  Same helpers (flux1,
// wsplit, vl_slope_sel, speed1) as the register and part forms, so all
// three give the same bits; the result is UE[s % 2].
constexpr int EUL_TPB = 1024;
constexpr size_t EUL_LDS = (size_t)((EUL_TPB + 4) * 6 + (EUL_TPB + 1) * 3) * sizeof(double);

__device__ void batch_euler_seg(const BatchArgs& a, int t, double* L, double* red) {
  t = __builtin_amdgcn_readfirstlane(t);
  if (a.tflag[t] != 0) return;  // a flagged tube is no longer advanced
  const TubeDev T = a.tubes[t];
  const Geom G = tube_geom(T);
  const int p = a.parity;
  double* alpha_r = a.alpha + ((size_t)t * 2 + p) * ASTR;
  double* alpha_w = a.alpha + ((size_t)t * 2 + (p ^ 1)) * ASTR;
  double alpha = __hip_atomic_load(alpha_r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  bool over;
  const int s = substeps<1>(&alpha, G, a.s_cap, &over);
  if (threadIdx.x == 0) {
    alpha_w[0] = 0.0;  // the update launch reduces the speeds of U^{n+1} here
    a.tube_s[t] = s;
    if (over) atomicOr(a.tflag + t, FLAG_SUBSTEP);
  }
  if (G.mu == 0.0 || over) return;  // over the cap: flagged, not solved
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
        double F[3], w[6];
        phys &= flux1(Uq, rcp_nr(Uq[0]), F);
        wsplit(Uq, F, alpha, w);
        const double* Wp = w;
        const double* Wm = w + 3;
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
          const double spl = vl_slope_sel(w[6 + r] - w[r], w[12 + r] - w[6 + r]);
          const double sml = vl_slope_sel(w[15 + r] - w[9 + r], w[21 + r] - w[15 + r]);
          Pl[f * 3 + r] = fma(0.25, spl - sml, 0.5 * (w[6 + r] + w[15 + r]));
        }
      }
      __syncthreads();
      const int j = x0 + threadIdx.x;
      if (threadIdx.x < EUL_TPB && j < Nx) {
        const int c = threadIdx.x;
        double Un[3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
          Un[r] = fma(-dts_dx, Pl[(c + 1) * 3 + r] - Pl[c * 3 + r], in[(size_t)r * Nx + j]);
#pragma unroll
        for (int r = 0; r < 3; ++r) out[(size_t)r * Nx + j] = Un[r];
        if (i + 1 < s) {
          double sp;
          phys &= speed1(Un, rcp_nr(Un[0]), G.gam, &sp);
          mx = fmax(mx, sp);
        }
      }
      __syncthreads();  // the next segment overwrites the LDS tiles
    }
    if (i + 1 < s) alpha = block_max_1024(mx, red);  // also orders this sub-step's writes
  }
  if (!phys) atomicOr(a.tflag + t, FLAG_NONPHYS);
}

// Euler solve of one tube of at most NT * CPT cells with every cell's
// moments (and 1/rho) in registers for all s sub-steps, by NT threads of
// the block: thread t of the group owns the CPT consecutive cells
// t CPT .. t CPT + CPT - 1, so a face stencil reaches at most two cells into
// each neighbouring thread.  After every sub-step a thread leaves U and 1/rho
// of its first two and last two cells in its LDS slots, which the
// neighbouring lanes of its wavefront read during the next sub-step (a
// wavefront's LDS operations complete in order, so lanes of one wavefront
// need no barrier); at the ends of a wavefront the cells come from the edge
// set that each wavefront leaves for its neighbours (one set per sub-step
// parity, so one block barrier per sub-step suffices, which also publishes
// the wavefront speed maxima that make alpha).  A thread forms the split
// fluxes of each stencil entry as it enters a four-entry window, the left
// faces of its cells and the right face of its last cell (which its right
// neighbour forms too, from the same values with the same arithmetic), and
// updates its cells.  Outflow ends: entries before cell 0 repeat cell 0,
// those past cell Nx - 1 repeat cell Nx - 1.
//
// With NT = 512 the two halves of the block solve two tubes (t0, t1; t1 may
// be -1) side by side: the solve is bound by the latency of its
// per-sub-step dependency chain, so two tubes on one compute unit overlap
// their chains.  Each half has its own LDS region and alpha; the block
// barrier is shared, so the block runs max(s0, s1) sub-steps and a half
// that is done only keeps meeting the barrier.
constexpr int RUN_SLOT = 4;  // doubles per exchanged cell: U, 1/rho
// LDS of one group of NT threads: per-thread slots [4 cells][RUN_SLOT][NT],
// the wavefront edge sets [2][NT/64][4 cells][RUN_SLOT] and the wavefront
// speed maxima [2][NT/64]
__host__ __device__ constexpr int run_lds_group(int nt) {
  return 4 * RUN_SLOT * nt + 2 * (nt / 64) * 4 * RUN_SLOT + 2 * (nt / 64);
}
constexpr size_t RUN_LDS = (size_t)(2 * run_lds_group(512)) * sizeof(double);
static_assert(run_lds_group(1024) <= 2 * run_lds_group(512), "one 1024-thread group fits");

template <int CPT, int NT>
__device__ void batch_euler_run(const BatchArgs& a, int t0, int t1, double* Lall) {
  constexpr int WAVES = NT / 64;
  __shared__ int s_grp[2];
  const int grp = (int)threadIdx.x / NT;
  const int tid = (int)threadIdx.x % NT, lane = tid & 63, wv = tid >> 6;
  int t = grp == 0 ? t0 : t1;
  t = __builtin_amdgcn_readfirstlane(t);
  if (t >= 0 && a.tflag[t] != 0) t = -1;  // a flagged tube is no longer advanced
  const TubeDev T = a.tubes[t < 0 ? t0 : t];
  const Geom G = tube_geom(T);
  const int p = a.parity;
  double alpha = t < 0 ? 0.0
                       : __hip_atomic_load(a.alpha + ((size_t)t * 2 + p) * ASTR,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  bool over = false;
  const int s_sub = t < 0 ? 0 : substeps<1>(&alpha, G, a.s_cap, &over);
  if (tid == 0 && t >= 0) {
    // the update launch reduces the speeds of U^{n+1} into the other row
    a.alpha[((size_t)t * 2 + (p ^ 1)) * ASTR] = 0.0;
    a.tube_s[t] = s_sub;
    if (over) atomicOr(a.tflag + t, FLAG_SUBSTEP);
  }
  // sub-steps this group runs (none over the cap: flagged, not solved)
  const int s = (t < 0 || G.mu == 0.0 || over) ? 0 : s_sub;
  if (tid == 0) s_grp[grp] = s;
  __syncthreads();
  const int smax = NT == 1024 ? s : max(s_grp[0], s_grp[1]);
  if (smax == 0) return;
  const int Nx = G.nc;
  const int c0 = tid * CPT;          // first cell of the thread
  const int wfirst = wv * 64 * CPT;  // first cell of the wavefront
  double* L = Lall + (size_t)grp * run_lds_group(NT);
  double* SL = L;                          // [4][RUN_SLOT][NT]
  double* EX = L + 4 * RUN_SLOT * NT;      // [2][WAVES][4][RUN_SLOT]
  double* WM = EX + 2 * WAVES * 4 * RUN_SLOT;  // [2][WAVES]
  const double* U0 = a.dar + (p ? T.U[1] : T.U[0]);
  double U[CPT][3], ir[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const bool ok = s > 0 && c0 + j < Nx;  // idle cells hold a finite placeholder
#pragma unroll
    for (int r = 0; r < 3; ++r) U[j][r] = ok ? U0[(size_t)r * Nx + c0 + j] : 1.0;
    ir[j] = rcp_nr(U[j][0]);
  }
  // own cells 0, 1 into slots 0, 1 and cells CPT-2, CPT-1 into slots 2, 3;
  // the wavefront's first two and last two cells into edge set b
  auto publish = [&](int b) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int j = k < 2 ? k : CPT - 4 + k;
      if (j < 0 || j >= CPT) continue;
#pragma unroll
      for (int r = 0; r < 3; ++r) SL[(k * RUN_SLOT + r) * NT + tid] = U[j][r];
      SL[(k * RUN_SLOT + 3) * NT + tid] = ir[j];
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int q = c0 + j - wfirst;
      const int slot = q < 2 ? q : (q >= 64 * CPT - 2 ? q - (64 * CPT - 4) : -1);
      if (slot >= 0) {
        double* e = EX + ((b * WAVES + wv) * 4 + slot) * RUN_SLOT;
#pragma unroll
        for (int r = 0; r < 3; ++r) e[r] = U[j][r];
        e[3] = ir[j];
      }
    }
  };
  if (s > 0) publish(0);
  __syncthreads();
  const double dts_dx = s > 0 ? (G.dt / s) / G.dx : 0.0;
  bool phys = true;
  for (int i = 0; i < smax; ++i) {
    const int b = i & 1;
    if (i < s) {
      if (i > 0) {
        double m[WAVES];
#pragma unroll
        for (int q = 0; q < WAVES; ++q) m[q] = WM[b * WAVES + q];
#pragma unroll
        for (int h = WAVES / 2; h >= 1; h /= 2)
#pragma unroll
          for (int q = 0; q < h; ++q) m[q] = fmax(m[q], m[q + h]);
        alpha = m[0];
      }
      // split fluxes of an entry from U and 1/rho
      auto entry = [&](const double* Uq, double irq, double* w) {
        double F[3];
        (void)flux1(Uq, irq, F);
        wsplit(Uq, F, alpha, w);
      };
      auto own_entry = [&](int j, double* w) {
        double F[3];
        const bool ph = flux1(U[j], ir[j], F);
        phys &= ph || c0 + j >= Nx;
        wsplit(U[j], F, alpha, w);
      };
      // a neighbour's cell: from its slot k in the thread nb lanes away, or,
      // past the wavefront's end, from edge slot es of wavefront ew
      auto remote_entry = [&](int k, int nb, bool edge, int ew, int es, double* w) {
        const double* src = edge ? EX + ((b * WAVES + ew) * 4 + es) * RUN_SLOT
                                 : SL + k * RUN_SLOT * NT + (tid + nb);
        const int stride = edge ? 1 : NT;
        const double Uq[3] = {src[0], src[stride], src[2 * stride]};
        entry(Uq, src[3 * stride], w);
      };
      // stencil entries k = 0 .. CPT + 3 are the cells c0 - 2 + k: the left
      // pair from lane - 1's slots 2, 3 (lanes - 2 and - 1 when CPT = 1), the
      // right pair from lane + 1's slots 0, 1 (lanes + 1 and + 2)
      auto left_entry = [&](int e, double* w) {
        const int dl = CPT >= 2 ? 1 : 2 - e;
        const bool edge = lane < dl;
        remote_entry(CPT >= 2 ? 2 + e : 0, edge ? 0 : -dl, edge, max(wv - 1, 0),
                     4 + (c0 - 2 + e - wfirst), w);
      };
      auto right_entry = [&](int e, double* w) {
        const int dr = CPT >= 2 ? 1 : 1 + e;
        const bool edge = lane >= 64 - dr;
        remote_entry(CPT >= 2 ? e : 0, edge ? 0 : dr, edge, min(wv + 1, WAVES - 1),
                     c0 + CPT + e - (wfirst + 64 * CPT), w);
      };
      // window of face 0: entries 0 .. 3
      double W0[6], W1[6], W2[6], W3[6];
      own_entry(0, W2);
      left_entry(1, W1);
      left_entry(0, W0);
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        W1[q] = c0 - 1 < 0 ? W2[q] : W1[q];
        W0[q] = c0 - 2 < 0 ? W1[q] : W0[q];
      }
      if (CPT >= 2)
        own_entry(CPT >= 2 ? 1 : 0, W3);
      else
        right_entry(0, W3);
      if (c0 + 1 >= Nx) {
#pragma unroll
        for (int q = 0; q < 6; ++q) W3[q] = W2[q];
      }
      double fprev[3];
      face4(W0, W1, W2, W3, fprev);
#pragma unroll
      for (int j = 1; j <= CPT; ++j) {
        // entry j + 3 (cell c0 + j + 1) enters the window
        double Wn[6];
        const int k = j + 3;
        if (k - 2 < CPT)
          own_entry(k - 2 < CPT ? k - 2 : 0, Wn);
        else
          right_entry(k - 2 - CPT, Wn);
        const bool past = c0 + j + 1 >= Nx;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          W0[q] = W1[q];
          W1[q] = W2[q];
          W2[q] = W3[q];
          W3[q] = past ? W2[q] : Wn[q];
        }
        double fc[3];
        face4(W0, W1, W2, W3, fc);
#pragma unroll
        for (int r = 0; r < 3; ++r) U[j - 1][r] = fma(-dts_dx, fc[r] - fprev[r], U[j - 1][r]);
#pragma unroll
        for (int r = 0; r < 3; ++r) fprev[r] = fc[r];
      }
      if (i + 1 < s) {
        // 1/rho and the speeds of the new values; slots, edge cells and
        // wavefront maxima out before the block barrier
        double mx = 0.0;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
          ir[j] = rcp_nr(U[j][0]);
          double sp;
          const bool ps = speed1(U[j], ir[j], G.gam, &sp);
          if (c0 + j < Nx) {
            phys &= ps;
            mx = fmax(mx, sp);
          }
        }
        publish(b ^ 1);
        const double wm = wave_max_dpp(mx);
        if (lane == 0) WM[(b ^ 1) * WAVES + wv] = wm;
      }
    }
    if (i + 1 < smax) __syncthreads();
  }
  if (s == 0) return;
  double* out = a.dar + ((s & 1) ? T.UE[1] : T.UE[0]);
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int c = c0 + j;
    if (c < Nx) {
#pragma unroll
      for (int r = 0; r < 3; ++r) out[(size_t)r * Nx + c] = U[j][r];
    }
  }
  if (!phys) atomicOr(a.tflag + t, FLAG_NONPHYS);
}

// Euler solve of one part of a tube, cells c0 .. c1-1 with c0 = part * PC
// and PC = part_cells (1024 or 2048): thread t owns cells c0 + t and
// c0 + 1024 + t, whose moments stay in registers for all s sub-steps.  Per
// sub-step the owners write the split fluxes W+- of their cells into LDS (one
// array per component; the tube's boundary cells also fill the clamped
// outflow entries), four threads write those of the two cells beyond each
// end of the part (held by the neighbouring parts), the faces c0 .. c1 are
// formed once each, and the owners update their cells.  Between sub-steps a
// part publishes its first two and last two cells and the largest speed of
// its cells in the tube's exchange row of the sub-step's parity; after the
// barrier of the tube's parts every part reads its halo cells and the speeds
// of all parts, so all parts take the same alpha (a maximum is exact in any
// order).  A face shared by two parts is formed by both from the same values
// with the same arithmetic, as in the whole-tube forms.  Two exchange rows
// suffice: a part overwrites a row only after passing the barrier that
// follows every part's reads of it.  The parts of a tube are consecutive
// blocks of the Euler launch, which start in block order, and a tube has at
// most PART_MAX parts, fewer than the compute units: only the tube of the
// last started block can be waiting for a part not yet started, and the
// other blocks finish and free a compute unit for it.
constexpr int XSTR = 16;       // doubles per part in an exchange row: 4 cells x 3, speed
constexpr int PART_MAX = 64;   // parts per tube at most
__host__ __device__ constexpr size_t part_lds(int pc) {
  return (size_t)(6 * (pc + 4) + 3 * (pc + 1)) * sizeof(double);
}

__device__ void batch_euler_part(const BatchArgs& a, int t, int part, int P, double* L,
                                 double* red) {
  t = __builtin_amdgcn_readfirstlane(t);
  part = __builtin_amdgcn_readfirstlane(part);
  P = __builtin_amdgcn_readfirstlane(P);
  const TubeDev T = a.tubes[t];
  const Geom G = tube_geom(T);
  const int p = a.parity;
  double alpha = __hip_atomic_load(a.alpha + ((size_t)t * 2 + p) * ASTR, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
  bool over;
  const int s = substeps<1>(&alpha, G, a.s_cap, &over);
  if (part == 0 && threadIdx.x == 0) {
    // the update launch reduces the speeds of U^{n+1} into the other row
    a.alpha[((size_t)t * 2 + (p ^ 1)) * ASTR] = 0.0;
    a.tube_s[t] = s;
    a.ebar[2 * t + (p ^ 1)] = 0u;  // the next step's barriers
    if (over) atomicOr(a.tflag + t, FLAG_SUBSTEP);
  }
  if (G.mu == 0.0 || over) return;  // every part sees the same alpha and s
  const int Nx = G.nc, PC = a.part_cells;
  const int c0 = part * PC, c1 = min(c0 + PC, Nx), n = c1 - c0;
  const int WS = PC + 4, FS = PC + 1;
  double* Wl = L;           // [6][WS]: W+ (3), W- (3) of cells c0-2 .. c1+1
  double* Pl = L + 6 * WS;  // [3][FS]: faces c0 .. c1
  const int tid = threadIdx.x;
  const double* U0 = a.dar + (p ? T.U[1] : T.U[0]);
  double Ur[2][3];
  bool own[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int c = c0 + k * 1024 + tid;
    own[k] = k * 1024 < PC && c < c1;
#pragma unroll
    for (int r = 0; r < 3; ++r) Ur[k][r] = own[k] ? U0[(size_t)r * Nx + c] : 0.0;
  }
  // halo entries: thread e < 4 fills entry q_h (0, 1, n + 2, n + 3), cell
  // c0 - 2 + q_h clamped to the tube, when that cell lies outside the part:
  // the last two cells of part - 1 (slots 2, 3) or the first two of part + 1
  // (slots 0, 1; slot 0 when the clamp folds c1 + 1 onto c1)
  const int q_h = tid < 2 ? tid : n + tid;
  const int c_h = min(max(c0 - 2 + q_h, 0), Nx - 1);
  const bool halo = tid < 4 && (c_h < c0 || c_h >= c1);
  const int h_part = c_h < c0 ? part - 1 : part + 1;
  const int h_slot = c_h < c0 ? 3 - (c0 - 1 - c_h) : c_h - c1;
  double Uh[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) Uh[r] = halo ? U0[(size_t)r * Nx + c_h] : 0.0;
  const double dts_dx = (G.dt / s) / G.dx;
  const int nw = (int)(blockDim.x >> 6);
  bool phys = true;
  for (int i = 0; i < s; ++i) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (!own[k]) continue;
      const int c = c0 + k * 1024 + tid;
      double F[3], w[6];
      phys &= flux1(Ur[k], rcp_nr(Ur[k][0]), F);
      wsplit(Ur[k], F, alpha, w);
      const double* Wp = w;
      const double* Wm = w + 3;
      int qlo = c - c0 + 2, qhi = qlo;
      if (c == 0) qlo = 0;
      if (c == Nx - 1) qhi = n + 3;
      for (int q = qlo; q <= qhi; ++q) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          Wl[r * WS + q] = Wp[r];
          Wl[(3 + r) * WS + q] = Wm[r];
        }
      }
    }
    if (halo) {
      double F[3], w[6];
      phys &= flux1(Uh, rcp_nr(Uh[0]), F);
      wsplit(Uh, F, alpha, w);
      const double* Wp = w;
      const double* Wm = w + 3;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        Wl[r * WS + q_h] = Wp[r];
        Wl[(3 + r) * WS + q_h] = Wm[r];
      }
    }
    __syncthreads();
    // face f between cells c0 + f - 1 and c0 + f from entries f .. f + 3
    for (int f = tid; f <= n; f += blockDim.x) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double* wp = Wl + r * WS + f;
        const double* wm = Wl + (3 + r) * WS + f;
        const double spl = vl_slope_sel(wp[1] - wp[0], wp[2] - wp[1]);
        const double sml = vl_slope_sel(wm[2] - wm[1], wm[3] - wm[2]);
        Pl[r * FS + f] = fma(0.25, spl - sml, 0.5 * (wp[1] + wm[2]));
      }
    }
    __syncthreads();
    double mx = 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (!own[k]) continue;
      const int j = k * 1024 + tid;
#pragma unroll
      for (int r = 0; r < 3; ++r)
        Ur[k][r] = fma(-dts_dx, Pl[r * FS + j + 1] - Pl[r * FS + j], Ur[k][r]);
      if (i + 1 < s) {
        double sp;
        phys &= speed1(Ur[k], rcp_nr(Ur[k][0]), G.gam, &sp);
        mx = fmax(mx, sp);
      }
    }
    if (i + 1 == s) break;
    double* row = a.dar + T.X + (size_t)((i & 1) * P) * XSTR;
    if (P > 1) {
      // publish the part's first two and last two cells
      bool wrote = false;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (!own[k]) continue;
        const int c = c0 + k * 1024 + tid;
        if (c - c0 < 2) {
#pragma unroll
          for (int r = 0; r < 3; ++r) row[part * XSTR + (c - c0) * 3 + r] = Ur[k][r];
          wrote = true;
        }
        if (c1 - 1 - c < 2) {
#pragma unroll
          for (int r = 0; r < 3; ++r) row[part * XSTR + (3 - (c1 - 1 - c)) * 3 + r] = Ur[k][r];
          wrote = true;
        }
      }
      if (wrote) __threadfence();
    }
    const double wmx = wave_max(mx);
    if ((tid & 63) == 0) red[tid >> 6] = wmx;
    __syncthreads();
    if (P == 1) {
      double m = red[0];
      for (int q = 1; q < nw; ++q) m = fmax(m, red[q]);
      alpha = m;
    } else {
      if (tid == 0) {
        double m = red[0];
        for (int q = 1; q < nw; ++q) m = fmax(m, red[q]);
        row[part * XSTR + 12] = m;
        __threadfence();
        atomicAdd(a.ebar + 2 * t + p, 1u);
        spin_until_geq(a.ebar + 2 * t + p, (unsigned)(P * (i + 1)), a.flag);
        __threadfence();
        double am = 0.0;
        for (int q = 0; q < P; ++q)
          am = fmax(am, __hip_atomic_load(row + q * XSTR + 12, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT));
        red[16] = am;
      }
      __syncthreads();
      alpha = red[16];
      if (halo) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
          Uh[r] = __hip_atomic_load(row + h_part * XSTR + h_slot * 3 + r, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  double* out = a.dar + ((s & 1) ? T.UE[1] : T.UE[0]);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (!own[k]) continue;
    const int c = c0 + k * 1024 + tid;
#pragma unroll
    for (int r = 0; r < 3; ++r) out[(size_t)r * Nx + c] = Ur[k][r];
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
  if (t < 0) return;  // padding of a die's item list
  if (a.tflag[t] != 0) return;  // a flagged tube is no longer advanced
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
  const int2 item = a.uitems[it];
  const int t = __builtin_amdgcn_readfirstlane(item.x);
  if (t < 0) return;  // padding of a die's item list
  if (a.tflag[t] != 0) return;  // a flagged tube is no longer advanced
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

// Euler launch: one 1024-thread block per Euler item (a whole tube or one
// part of a split tube), most work first; it runs beside the kinetic
// launch, on its own stream.
__global__ __launch_bounds__(1024) void k_batch_euler(BatchArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  __shared__ double red[32];
  const int4 e = a.eitems[blockIdx.x];
  double* L = reinterpret_cast<double*>(lds_raw);
  if (e.w == 1) {
    batch_euler_part(a, e.x, e.y, e.z, L, red);
  } else if (e.w == 2) {  // two tubes of at most 512 * e.z cells side by side
    if (e.z == 1)
      batch_euler_run<1, 512>(a, e.x, e.y, L);
    else if (e.z == 2)
      batch_euler_run<2, 512>(a, e.x, e.y, L);
    else if (e.z == 3)
      batch_euler_run<3, 512>(a, e.x, e.y, L);
    else
      batch_euler_run<4, 512>(a, e.x, e.y, L);
  } else {
    const int nx = a.tubes[e.x].Nx;
    if (nx <= 1024)
      batch_euler_run<1, 1024>(a, e.x, -1, L);
    else if (nx <= 2048)
      batch_euler_run<2, 1024>(a, e.x, -1, L);
    else if (nx <= 3072)
      batch_euler_run<3, 1024>(a, e.x, -1, L);
    else if (nx <= 4096)
      batch_euler_run<4, 1024>(a, e.x, -1, L);
    else
      batch_euler_seg(a, e.x, L, red);
  }
}

// Kinetic launch: one 1024-thread block per kinetic item (relaxation, shift
// and moment sums of a (tube, segment)), most work first; it needs nothing
// from the Euler solves.
template <int CELLS, int UNR>
__global__ __launch_bounds__(1024) void k_batch_kinetic(BatchArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  batch_kinetic_item<CELLS, UNR>(a, blockIdx.x, lds_raw);
}

// Update launch: one block of UPD_CELLS threads per update item.
__global__ __launch_bounds__(1024) void k_batch_update(BatchArgs a) {
  batch_update_item(a, blockIdx.x);
}

}  // namespace hofks
