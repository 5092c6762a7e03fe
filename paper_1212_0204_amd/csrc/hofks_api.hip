// hofks_api.hip -- host side of the C ABI declared in include/hofks.h.
//
// The plan fixes the lattice (dt = dx/dv, velocity nodes k dv), forms
// A = (C C^T)^{-1} once in FP64 (end of section 4.1 of arXiv:1212.0204),
// carves the caller's workspace and chooses the kinetic kernel's tiling.
// Every arithmetic step of the scheme runs in the kernels of kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <new>
#include <type_traits>
#include <utility>
#include <vector>

#include "hofks.h"
#include "batch.hpp"
#include "closure.hpp"
#include "euler2d.hpp"
#include "kernels.hpp"
#include "kinetic2w.hpp"
#include "kinetic3d.hpp"
#include "mlp.hpp"
#include "weno.hpp"
#include "train.hpp"
#include "probe.hpp"

using namespace hofks;

namespace {

struct Plan {
  int d, nm, R;
  Geom G;
  Mat A;
  int prec;
  size_t tsize;  // bytes per stored piece
  int TX, TR, nseg, nrowgrp, nchunk, nvr, GE, ETPB;
  int ncu;  // compute units of the device
  size_t lds;
  int RS;  // record stride (values)
  // workspace offsets (bytes)
  size_t off_g[2], off_U[2], off_UE[4], off_rec[2], off_vt, off_cf, off_part, off_slots,
      off_tiles, off_flag;
  size_t off_clos;  // closure form (2D): N^, indicator, dilation, mode, delta marks, count
  size_t off_sums;  // kinetic moment sums per cell, 2 (d+2) doubles
  size_t total;
};

#ifndef HOFKS_EULER_TPB_MAX
#define HOFKS_EULER_TPB_MAX 256
#endif

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Gauss-Jordan inverse with partial pivoting (n <= 5)
bool invert(int n, const double* M, double* Minv) {
  double a[5][10];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j) a[i][j] = (j < n) ? M[i * n + j] : (j - n == i ? 1.0 : 0.0);
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int i = c + 1; i < n; ++i)
      if (std::fabs(a[i][c]) > std::fabs(a[p][c])) p = i;
    if (a[p][c] == 0.0) return false;
    if (p != c)
      for (int j = 0; j < 2 * n; ++j) std::swap(a[c][j], a[p][j]);
    const double piv = a[c][c];
    for (int j = 0; j < 2 * n; ++j) a[c][j] /= piv;
    for (int i = 0; i < n; ++i) {
      if (i == c || a[i][c] == 0.0) continue;
      const double fct = a[i][c];
      for (int j = 0; j < 2 * n; ++j) a[i][j] -= fct * a[c][j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Minv[i * n + j] = a[i][j + n];
  return true;
}

int fmt_err(char* buf, const char* f, ...) {
  if (!buf) return 0;
  va_list ap;
  va_start(ap, f);
  vsnprintf(buf, 512, f, ap);
  va_end(ap);
  return 0;
}

// LDS of a kinetic block with ng wavefronts: the staged record segments and
// the partial sums of the extra wavefronts
size_t kin_lds(const Plan& P, int ng) {
  const size_t sw = 64 + P.G.nv1 - 1;
  const size_t fs = P.tsize == 8 ? row_rec_stride<double>() : row_rec_stride<float>();
  const size_t stage = (P.d >= 2 ? ng : 1) * sw * fs * P.tsize;
  const size_t red = (size_t)(ng - 1) * 64 * 2 * P.nm * sizeof(double);
  return std::max(stage, red);
}

int rec_stride_rt(int d, int prec) {
  if (prec) return d == 1 ? rec_stride<1, float>() : d == 2 ? rec_stride<2, float>() : rec_stride<3, float>();
  return d == 1 ? rec_stride<1, double>() : d == 2 ? rec_stride<2, double>() : rec_stride<3, double>();
}

hofks_status make_plan(const hofks_grid_desc* desc, Plan* P, char* err) {
  if (!desc || !P) return HOFKS_EINVAL;
  std::memset(P, 0, sizeof(*P));
  const int d = desc->dim;
  if (d < 1 || d > 3) return fmt_err(err, "dim must be 1, 2 or 3"), HOFKS_EINVAL;
  if (!(desc->dx > 0.0) || !std::isfinite(desc->dx))
    return fmt_err(err, "dx must be positive"), HOFKS_EINVAL;
  if (!(desc->dv > 0.0) || !std::isfinite(desc->dv))
    return fmt_err(err, "dv must be positive"), HOFKS_EINVAL;
  if (desc->n_vel < 2 || desc->n_vel > 256)
    return fmt_err(err, "n_vel must be in [2, 256]"), HOFKS_EINVAL;
  if (desc->precision < 0 || desc->precision > 1)
    return fmt_err(err, "precision must be 0 or 1"), HOFKS_EINVAL;
  if (desc->scheme < 0 || desc->scheme > 3)
    return fmt_err(err, "scheme must be 0, 1, 2 or 3"), HOFKS_EINVAL;
  if (desc->splitting < 0 || desc->splitting > 1)
    return fmt_err(err, "splitting must be 0 or 1"), HOFKS_EINVAL;
  Geom& G = P->G;
  G.nc = 1;
  for (int a = 0; a < 3; ++a) {
    G.n[a] = a < d ? desc->n_cells[a] : 1;
    G.bc[a] = a < d ? desc->bc[a] : 0;
    if (G.n[a] < 1 || G.n[a] > (1 << 20)) return fmt_err(err, "bad n_cells[%d]", a), HOFKS_EINVAL;
    if (G.bc[a] != 0 && G.bc[a] != 1) return fmt_err(err, "bad bc[%d]", a), HOFKS_EINVAL;
    if ((long)G.nc * G.n[a] > (1L << 30)) return fmt_err(err, "too many cells"), HOFKS_EINVAL;
    G.nc *= G.n[a];
  }
  G.nv1 = desc->n_vel;
  G.kofs = G.nv1 / 2;
  G.nv = 1;
  for (int a = 0; a < d; ++a) G.nv *= G.nv1;
  if (G.bc[0] == 0 && (G.kofs > G.n[0] || G.nv1 - 1 - G.kofs > G.n[0]))
    return fmt_err(err, "periodic x axis shorter than the largest shift n_vel/2"), HOFKS_EINVAL;
  G.dx = desc->dx;
  G.dv = desc->dv;
  G.dt = desc->dx / desc->dv;  // lattice: v_k dt = k dx
  G.offl = 0;
  if (desc->dt != 0.0) {  // a free time step: off-lattice transport (section 4.2)
    if (!(desc->dt > 0.0) || !(desc->dt <= G.dt))
      return fmt_err(err, "dt must lie in (0, dx/dv]"), HOFKS_EINVAL;
    if (d >= 2 && G.nv1 % 4 != 0)
      return fmt_err(err, "off-lattice transport in 2D/3D needs n_vel a multiple of 4"), HOFKS_EINVAL;
    G.dt = desc->dt;
    G.offl = 1;
  }
  G.w = std::pow(desc->dv, d);
  G.lam = G.lam_r = 1.0;
  G.mu = G.mu_r = 0.0;
  G.gam = (d + 2.0) / d;
  G.sfac = desc->scheme == 3 ? 2.5 : 2.0;
  P->d = d;
  P->nm = d + 2;
  P->R = 3 * P->nm;
  P->prec = desc->precision;
  P->tsize = desc->precision ? sizeof(float) : sizeof(double);

  // A = (C C^T)^{-1}, C[r][k] = w m_k[r], m_k = (1, v_k, |v_k|^2/2)
  const int nm = P->nm;
  double CCt[25] = {0};
  for (int k = 0; k < G.nv; ++k) {
    double m[5], vsq = 0.0;
    int kk = k;
    m[0] = 1.0;
    for (int a = 0; a < d; ++a) {
      const double v = (kk % G.nv1 - G.kofs) * G.dv;
      kk /= G.nv1;
      m[1 + a] = v;
      vsq += v * v;
    }
    m[nm - 1] = 0.5 * vsq;
    for (int r = 0; r < nm; ++r)
      for (int s = 0; s < nm; ++s) CCt[r * nm + s] += (G.w * m[r]) * (G.w * m[s]);
  }
  if (!invert(nm, CCt, P->A.a)) return fmt_err(err, "C C^T is singular"), HOFKS_EINVAL;

  // kinetic tiling: one block per 64 consecutive x cells of a row, four
  // wavefronts over the velocities
  const int Nx = G.n[0];
  const int nrows = G.n[1] * G.n[2];
  P->TX = 64;
  P->TR = 1;
  P->nseg = (Nx + 63) / 64;
  P->nrowgrp = nrows;
  P->nchunk = 1;
  P->nvr = G.nv / G.nv1;
  P->RS = rec_stride_rt(d, P->prec);
  const size_t sw = 64 + G.nv1 - 1;
  (void)sw;
  P->lds = kin_lds(*P, 2);
  if (P->lds > 65536) return fmt_err(err, "velocity grid too wide for the LDS tile"), HOFKS_EINVAL;
  // Euler kernel: at most one block per compute unit (co-resident), grid-
  // strided over cells
  int ncu = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      ncu < 1)
    ncu = 256;
  // threads per Euler block: up to one cell per thread when the grid is
  // large enough to fill every compute unit with wider blocks
  P->ncu = ncu;
  const int ge = std::min(256, ncu);
  P->ETPB = 256;
  for (int tpb = HOFKS_EULER_TPB_MAX; tpb > 256; tpb /= 2)
    if ((long)G.nc >= (long)ge * tpb) {
      P->ETPB = tpb;
      break;
    }
  P->GE = (int)std::min<long>(ge, ((long)G.nc + P->ETPB - 1) / P->ETPB);

  size_t off = 0;
  const size_t gbytes = (size_t)G.nv * G.nc * P->tsize;
  const size_t ubytes = (size_t)nm * G.nc * sizeof(double);
  P->off_g[0] = off;
  off = align256(off + gbytes);
  P->off_g[1] = off;
  off = align256(off + gbytes);
  P->off_U[0] = off;
  off = align256(off + ubytes);
  P->off_U[1] = off;
  off = align256(off + ubytes);
  P->off_UE[0] = off;
  off = align256(off + ubytes);
  P->off_UE[1] = off;
  off = align256(off + ubytes);
  if (desc->scheme == 3) {  // Runge-Kutta stage values of the WENO solve
    P->off_UE[2] = off;
    off = align256(off + ubytes);
    P->off_UE[3] = off;
    off = align256(off + ubytes);
  }
  P->off_rec[0] = off;
  off = align256(off + (size_t)P->RS * G.nc * P->tsize);
  P->off_rec[1] = off;
  off = align256(off + (size_t)P->RS * G.nc * P->tsize);
  P->off_vt = off;  // node table, then c = v dt/dx per node
  off = align256(off + (size_t)G.nv1 * (sizeof(VelNode) + sizeof(double)));
  P->off_cf = off;
  off = align256(off + ubytes);
  P->off_part = off;
  off = align256(off + (size_t)P->nchunk * 2 * nm * G.nc * sizeof(double));
  P->off_slots = off;
  off = align256(off + 3 * (size_t)SET_D * sizeof(double));
  P->off_tiles = off;  // per-block speed maxima of the Euler kernel
  off = align256(off + (size_t)2 * 256 * ASTR * sizeof(double));
  P->off_flag = off;
  off = align256(off + 64);
  P->off_sums = off;
  off = align256(off + (size_t)2 * nm * G.nc * sizeof(double));
  if (d == 2) {
    P->off_clos = off;
    off = align256(off + (size_t)G.nc * sizeof(float4));
    off = align256(off + 4 * (size_t)G.nc);
    off = align256(off + 256);
  }
  P->total = off;
  return HOFKS_OK;
}

}  // namespace

struct hofks_ctx {
  Plan P;
  hofks_grid_desc desc;
  hipStream_t stream;
  unsigned char* ws;
  void* g[2];
  int cur;                 // piece buffer holding f^n
  double *U[2], *UE[4], *cf, *part, *slots;
  void* rec[2];
  VelNode* vt;
  int* tiles;
  int* flag;
  double tau;
  int s_cap;
  int s_known;  // Euler sub-steps of the last step seen by the host
  int s_margin;  // spare single-sub-step launches beyond s_known (0 or 1)
  int euler_k;  // > 0: per-sub-step Euler launches before the tail (0: s_known + 1)
  bool euler_seq;   // the Euler solve runs on the caller's stream before the kinetic kernel
  bool strang;      // Strang splitting: half relaxations around each transport
  double inv_prev;  // 1/tau of the last step taken (Strang)
  long steps;
  bool ready;
  int kng, kunr;  // kinetic kernel: wavefronts per block, loads issued ahead
  int kring;      // 3D steps with an Euler solve: k_kinetic3 (blocks of RY rows)
  int kwide;      // 2D FP64 steps with an Euler solve: k_kinetic2w (two cells per lane)
  bool fork_next;     // the current step is followed by another in this call
  bool fork_pending;  // ev_fork already marks the next step's fork point
  // optional per-kernel timing: hipEvents around the launch groups whose
  // bits are set (bit g: group g)
  unsigned timing;
  std::vector<hipEvent_t> ev_pool;
  struct MarkRec {
    int group, count;
    hipEvent_t a, b;
  };
  std::vector<MarkRec> ev_marks;
  size_t ev_next;
  struct Batch* batch;  // non-null for a batch of independent tubes
  // the Euler solve of a step runs on `aux`, forked from and joined to the
  // caller's stream with two events, beside the kinetic kernel
  hipStream_t aux;
  hipEvent_t ev_fork, ev_join;
  // the Euler sub-step count of a recent step, read back during long step
  // calls: the auxiliary stream copies it to pinned host memory after the
  // step's Euler launches and marks the copy (ev_peek)
  hipEvent_t ev_peek;
  int* peek_h;
  bool peek_now;      // copy the count of the step being queued
  bool peek_pending;
  long peek_at;     // step after which the pending read was queued
  long peek_next;   // first step at which the next read may be queued
  int peek_every;   // steps between reads: 8 while the count moves, doubling to 64 while not
  // closure form (2D-2V): network (caller's device memory), scale of its
  // output, indicator threshold; per-cell arrays in the workspace
  const void* clos_w;
  double clos_sigma, clos_thr;
  bool clos_on;
  bool clos_dirty;  // some record marks a cell without pieces
  float4* nhat;
  unsigned char *cflag, *ctmp, *cmode, *cdfl;
  unsigned long long* kcount;
  float* clos_y0;
  float clos_y0_ftau;  // log10(tau/dt) input of the stored y0
  bool clos_y0_ok;     // y0 holds the network's output on the uniform stencil
  long clos_steps;
  char err[512];
};

namespace {

hofks_status hip_fail(hofks_ctx* c, hipError_t e, const char* what) {
  fmt_err(c->err, "%s: %s", what, hipGetErrorString(e));
  return HOFKS_EDEVICE;
}

#define HIPCHK(c, call)                                    \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_fail((c), e_, #call); \
  } while (0)

unsigned nblk(size_t n, unsigned b = 256) { return (unsigned)((n + b - 1) / b); }

// 1/tau with 1/inf = 0 and 1/0 = inf
double inv_tau(double tau) {
  if (std::isinf(tau)) return 0.0;
  if (tau == 0.0) return INFINITY;
  return 1.0 / tau;
}

// Strang splitting: exp(-e), 1 - exp(-e) with e = dt/2 ip + dt/2 in
void strang_weights(double dt, double ip, double in, double* lam, double* mu) {
  const double e = 0.5 * dt * ip + 0.5 * dt * in;
  *lam = std::exp(-e);
  *mu = -std::expm1(-e);
}

// relaxation weights of the next step (lam, mu) and of the one after it
// (lam_r, mu_r: the weights the records formed by the next step are for).
// First-order splitting: lambda = exp(-dt/tau) for both.  Strang splitting:
// the half relaxation closing the previous step (its tau) merged with the
// half opening the next (none before the first step after the state is set).
void set_step_weights(hofks_ctx* c) {
  Geom& G = c->P.G;
  const double tau = c->tau;
  if (!c->strang) {
    if (std::isinf(tau)) {
      G.lam = 1.0;
      G.mu = 0.0;
    } else if (tau == 0.0) {
      G.lam = 0.0;
      G.mu = 1.0;
    } else {
      G.lam = std::exp(-G.dt / tau);
      G.mu = -std::expm1(-G.dt / tau);
    }
    G.lam_r = G.lam;
    G.mu_r = G.mu;
    return;
  }
  const double in = inv_tau(tau);
  strang_weights(G.dt, c->steps > 0 ? c->inv_prev : 0.0, in, &G.lam, &G.mu);
  strang_weights(G.dt, in, in, &G.lam_r, &G.mu_r);
}


double* slot_set(hofks_ctx* c, int set) { return c->slots + (size_t)set * SET_D; }
int rpar(const hofks_ctx* c) { return (int)(c->steps & 1); }   // buffer holding U^n, rec^n
int rset(const hofks_ctx* c) { return (int)(c->steps % 3); }   // speeds of U^n

// timing groups: 0 the Euler sub-steps (auxiliary stream), 1 the kinetic
// kernel, 2 the per-cell update, 3 the closure network and its indicator
hipEvent_t next_event(hofks_ctx* c) {
  if (c->ev_next == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_next++];
}

struct Mark {
  hofks_ctx* c;
  int group, count;
  hipStream_t st;
  hipEvent_t a = nullptr;
  Mark(hofks_ctx* c_, int g, int n = 1, hipStream_t s_ = nullptr)
      : c(c_), group(g), count(n), st(s_ ? s_ : c_->stream) {
    if (c->timing >> group & 1u) {
      a = next_event(c);
      if (a) (void)hipEventRecord(a, st);
    }
  }
  ~Mark() {
    if (a) {
      hipEvent_t b = next_event(c);
      if (b) {
        (void)hipEventRecord(b, st);
        c->ev_marks.push_back({group, count, a, b});
      }
    }
  }
};

// ---------------------------------------------------------------- launchers
template <int D, typename T>
hofks_status launch_cell_init(hofks_ctx* c, int mode) {
  const Plan& P = c->P;
  const int rp = rpar(c);
  Geom Gi = P.G;  // the records formed here are read by the next step
  Gi.lam_r = Gi.lam;
  Gi.mu_r = Gi.mu;
  hipLaunchKernelGGL((k_cell_init<D, T>), dim3(nblk(P.G.nc)), dim3(256), 0, c->stream, c->U[rp],
                     c->cf, (T*)c->rec[rp], c->vt, c->part, slot_set(c, rset(c)), c->flag, Gi,
                     P.A, mode);
  HIPCHK(c, hipGetLastError());
  return HOFKS_OK;
}

// unroll depth that divides the k_x range of one wavefront
int kin_unroll(const Plan& P, int ng, int unr) {
  const int per = P.d >= 2 ? P.G.nv1 : P.G.nv1 / ng;
  const bool even = P.d >= 2 || P.G.nv1 % ng == 0;
  return (even && per % unr == 0) ? unr : 1;
}

// 3D steps with an Euler solve: blocks of RY y rows sharing a ring of
// staged upstream rows (k_kinetic3)
size_t kin3_lds(const Plan& P) {
  const int fc = P.tsize == 4 ? fold3_chunks<float>() : fold3_chunks<double>();
  return (size_t)(RY + 1) * (64 + P.G.nv1 - 1) * fc * 16;
}

template <typename T>
void dispatch_kin3(hofks_ctx* c, const StepArgs<T>& a) {
  constexpr bool CP = sizeof(T) == 4;
  const Plan& P = c->P;
  const int nyb = (P.G.n[1] + RY - 1) / RY;
  const dim3 grid((unsigned)((long)P.nseg * nyb * P.G.n[2]));
  const size_t lds = kin3_lds(P);
  const int nv = P.G.nv1;
  const int unr = nv % c->kunr == 0 ? c->kunr : nv % 12 == 0 ? 12 : nv % 8 == 0 ? 8 : 1;
#define K(BCX, U)                                                                 \
  hipLaunchKernelGGL((k_kinetic3<T, CP, BCX, U>), grid, dim3(64 * RY), lds, c->stream, a, \
                     P.G, nyb)
#define KB(U) \
  if (P.G.bc[0] == 0) K(0, U); else K(1, U);
  if (unr == 16) { KB(16) } else if (unr == 12) { KB(12) } else if (unr == 8) { KB(8) } else { KB(1) }
#undef KB
#undef K
}

// 2D FP64 steps with an Euler solve: two cells per lane (k_kinetic2w)
size_t kin2w_lds(const Plan& P, int ng) {
  const size_t sp = (W2_CELLS + P.G.nv1) / 2;  // records per parity half
  const size_t stage = (size_t)ng * 2 * sp * row_rec_stride<double>() * sizeof(double);
  const size_t red = (size_t)(ng - 1) * 64 * 16 * sizeof(double);
  return std::max(stage, red);
}

void dispatch_kin2w(hofks_ctx* c, const StepArgs<double>& a) {
  const Plan& P = c->P;
  const int nsegw = (P.G.n[0] + W2_CELLS - 1) / W2_CELLS;
  const dim3 grid((unsigned)((long)nsegw * P.G.n[1]));
  const int ng = c->kng == 2 ? 2 : 4, unr = P.G.nv1 % 8 == 0 && c->kunr == 8 ? 8 : 4;
  const size_t lds = kin2w_lds(P, ng);
#define K(BCX, NG, U)                                                                    \
  hipLaunchKernelGGL((k_kinetic2w<BCX, U, NG>), grid, dim3(64 * NG), lds, c->stream, a, \
                     P.G, nsegw)
#define KB(NG, U) \
  if (P.G.bc[0] == 0) K(0, NG, U); else K(1, NG, U);
  if (ng == 2) {
    if (unr == 8) { KB(2, 8) } else { KB(2, 4) }
  } else {
    if (unr == 8) { KB(4, 8) } else { KB(4, 4) }
  }
#undef KB
#undef K
}

template <int D, typename T, bool FT, bool EUL>
void dispatch_kin(hofks_ctx* c, const StepArgs<T>& a, dim3 grid) {
  constexpr bool CP = sizeof(T) == 4;  // compensated sums in the FP32 form
  const Plan& P = c->P;
  if constexpr (D == 3 && EUL && !FT) {
    if (c->kring) {
      dispatch_kin3<T>(c, a);
      return;
    }
  }
  if constexpr (D == 2 && EUL && !FT && sizeof(T) == 8) {
    if (c->kwide) {
      dispatch_kin2w(c, a);
      return;
    }
  }
  const int bcx = P.G.bc[0];
  if (P.G.offl) {  // four wavefronts; four loads ahead in 2D/3D (n_vel % 4 == 0)
    const size_t lds0 = kin_lds(P, 4);
#define KO(BCX, U)                                                                               \
  hipLaunchKernelGGL((k_kinetic<D, T, FT, CP, BCX, U, EUL, 4, false, true>), grid, dim3(256), lds0, \
                     c->stream, a, P.G, P.A)
    if constexpr (D >= 2) {
      if (bcx == 0) KO(0, 4); else KO(1, 4);
    } else {
      if (bcx == 0) KO(0, 1); else KO(1, 1);
    }
#undef KO
    return;
  }
  int ng = c->kng, unr = kin_unroll(P, c->kng, c->kunr);
  if (FT || !EUL) {  // free transport and FKS steps: one configuration
    ng = 4;
    unr = kin_unroll(P, 4, 8);
  }
  const size_t lds = kin_lds(P, ng);
#define K(BCX, NG, U)                                                                       \
  hipLaunchKernelGGL((k_kinetic<D, T, FT, CP, BCX, U, EUL, NG>), grid, dim3(64 * NG), lds, \
                     c->stream, a, P.G, P.A)
#define KB(NG, U) \
  if (bcx == 0) K(0, NG, U); else K(1, NG, U);
  if (FT || !EUL) {
    if (unr == 8) { KB(4, 8) } else { KB(4, 1) }
  } else if (ng == 2) {
    if (unr == 16) { KB(2, 16) } else if (unr == 8) { KB(2, 8) } else { KB(2, 1) }
  } else if (ng == 8 && D >= 2) {
    if (unr == 16) { KB(8, 16) } else if (unr == 8) { KB(8, 8) } else { KB(8, 1) }
  } else {
    if (unr == 16) { KB(4, 16) } else if (unr == 8) { KB(4, 8) } else { KB(4, 1) }
  }
#undef KB
#undef K
}

template <typename T>
hofks_status launch_closure_step(hofks_ctx* c, StepArgs<T>& a, float* snap_x, float* snap_t);

template <int D, typename T>
void launch_euler(hofks_ctx* c, const StepArgs<T>& a, hipStream_t st);

// Euler launches of the step on the auxiliary stream, after everything
// already queued on the caller's stream
// the step's sub-step count to the host on the auxiliary stream, after its
// Euler launches there (or, with the Euler solve on the caller's stream, after
// an event that follows them), beside the update
hofks_status queue_peek(hofks_ctx* c) {
  c->peek_now = false;
  if (c->euler_seq) {  // the auxiliary stream is idle in this form
    HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
    HIPCHK(c, hipStreamWaitEvent(c->aux, c->ev_fork, 0));
  }
  HIPCHK(c, hipMemcpyAsync(c->peek_h, c->flag + 1, sizeof(int), hipMemcpyDeviceToHost, c->aux));
  HIPCHK(c, hipEventRecord(c->ev_peek, c->aux));
  c->peek_pending = true;
  c->peek_at = c->steps;
  c->peek_next = c->steps + c->peek_every;
  return HOFKS_OK;
}

template <int D, typename T>
hofks_status fork_euler(hofks_ctx* c, const StepArgs<T>& a) {
  if (c->euler_seq) {  // before the kinetic kernel, on the caller's stream
    {
      Mark m0(c, 0, 1, c->stream);
      launch_euler<D, T>(c, a, c->stream);
      HIPCHK(c, hipGetLastError());
    }
    return c->peek_now ? queue_peek(c) : HOFKS_OK;
  }
  // within one hofks_step call the previous step recorded the fork point
  // right after U^{n+1} was formed, before its records
  if (c->fork_pending)
    c->fork_pending = false;
  else
    HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
  HIPCHK(c, hipStreamWaitEvent(c->aux, c->ev_fork, 0));
  {
    Mark m0(c, 0, 1, c->aux);
    launch_euler<D, T>(c, a, c->aux);
    HIPCHK(c, hipGetLastError());
  }
  HIPCHK(c, hipEventRecord(c->ev_join, c->aux));
  return c->peek_now ? queue_peek(c) : HOFKS_OK;
}

// join the Euler launches and run the per-cell update on the caller's stream
template <int D, typename T, bool CLOS>
hofks_status join_update(hofks_ctx* c, const StepArgs<T>& a) {
  const Plan& P = c->P;
  if (!c->euler_seq) HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
  Mark m(c, 2);
  if constexpr (CLOS) {
    hipLaunchKernelGGL((k_cell_update<D, T, CLOS>), dim3(nblk(P.G.nc)), dim3(256), 0, c->stream,
                       a, P.G, P.A);
  } else {
    // U^{n+1}, cf and speeds; the fork point of the next step of this call;
    // then the records, beside the next step's Euler solve
    hipLaunchKernelGGL((k_cell_update_u<D, T>), dim3(nblk(P.G.nc)), dim3(256), 0, c->stream, a,
                       P.G, P.A);
    if (c->fork_next && !c->euler_seq) {
      HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
      c->fork_pending = true;
    }
    hipLaunchKernelGGL((k_cell_record<D, T>), dim3(nblk(P.G.nc)), dim3(256), 0, c->stream, a,
                       P.G, P.A);
  }
  HIPCHK(c, hipGetLastError());
  return HOFKS_OK;
}

// Euler solve of a step: one launch per sub-step for the first K = (last
// known count + margin) sub-steps (the kernel boundary is the grid-wide
// barrier), then a persistent tail that runs any further sub-steps with an
// in-kernel barrier (it returns at once when K >= s).  The spare launch (margin
// 1) absorbs a count that grows by one; each launch with i >= s still costs a
// kernel boundary on the solve's critical path, so it is dropped while the
// read-back sees a steady count, and a single sub-step left to the tail is
// about as cheap.
template <int D, typename T>
void launch_euler(hofks_ctx* c, const StepArgs<T>& a, hipStream_t st) {
  const Plan& P = c->P;
  // a 1D grid within one tail block runs every sub-step after the first in
  // the tail, whose barrier is then the block's own
  const bool one_block = D == 1 && P.GE == 1 && c->desc.scheme != 3;
  const int K = std::max(
      1, std::min(c->s_cap, c->euler_k > 0 ? c->euler_k
                            : one_block    ? 1
                                           : c->s_known + c->s_margin));
  if (c->desc.scheme == 3) {  // WENO: three Runge-Kutta stage launches per sub-step
    if constexpr (D == 2) {  // 16 x 16 LDS tiles
      const int ntx = (P.G.n[0] + WT - 1) / WT, nty = (P.G.n[1] + WT - 1) / WT;
      for (int i = 0; i < K; ++i)
        for (int stg = 0; stg < 3; ++stg)
          hipLaunchKernelGGL((k_weno_stage_tile<T>), dim3(ntx * nty), dim3(256), 0, st, a, P.G, i,
                             stg, ntx);
    } else {
      for (int i = 0; i < K; ++i)
        for (int stg = 0; stg < 3; ++stg)
          hipLaunchKernelGGL((k_weno_stage<D, T>), dim3(nblk(P.G.nc)), dim3(256), 0, st, a, P.G, i,
                             stg);
    }
    hipLaunchKernelGGL((k_weno_tail<D, T, 256>), dim3(P.GE), dim3(256), 0, st, a, P.G, K);
    return;
  }
  if constexpr (D == 2) {  // 16 x 16 LDS tiles
    const int ntx = (P.G.n[0] + ET - 1) / ET, nty = (P.G.n[1] + ET - 1) / ET;
    for (int i = 0; i < K; ++i)
      hipLaunchKernelGGL((k_euler_sub_tile<T>), dim3(ntx * nty), dim3(256), 0, st, a, P.G, i, ntx);
  } else if constexpr (D == 3) {  // 8 x 4 x 4 LDS tiles
    const int ntx = (P.G.n[0] + E3X - 1) / E3X, nty = (P.G.n[1] + E3Y - 1) / E3Y;
    const int ntz = (P.G.n[2] + E3Z - 1) / E3Z;
    for (int i = 0; i < K; ++i)
      hipLaunchKernelGGL((k_euler_sub_tile3<T>), dim3(ntx * nty * ntz), dim3(256), 0, st, a, P.G,
                         i, ntx, nty);
  } else {
    for (int i = 0; i < K; ++i)
      hipLaunchKernelGGL((k_euler_sub<D, T>), dim3(nblk(P.G.nc)), dim3(256), 0, st, a, P.G, i);
  }
  if (P.ETPB == 1024)
    hipLaunchKernelGGL((k_euler<D, T, 1024>), dim3(P.GE), dim3(1024), 0, st, a, P.G, K);
  else if (P.ETPB == 512)
    hipLaunchKernelGGL((k_euler<D, T, 512>), dim3(P.GE), dim3(512), 0, st, a, P.G, K);
  else
    hipLaunchKernelGGL((k_euler<D, T, 256>), dim3(P.GE), dim3(256), 0, st, a, P.G, K);
}

template <int D, typename T>
hofks_status launch_step(hofks_ctx* c, float* snap_x = nullptr, float* snap_t = nullptr) {
  const Plan& P = c->P;
  const int rp = rpar(c);
  const long n = c->steps;
  StepArgs<T> a;
  a.g_in = (const T*)c->g[c->cur];
  a.g_out = (T*)c->g[c->cur ^ 1];
  a.rec_in = (const T*)c->rec[rp];
  a.rec_out = (T*)c->rec[rp ^ 1];
  a.vt = c->vt;
  a.U_in = c->U[rp];
  a.U_out = c->U[rp ^ 1];
  a.UE0 = c->UE[0];
  a.UE1 = c->UE[1];
  a.UE2 = c->UE[2];
  a.UE3 = c->UE[3];
  a.cf = c->cf;
  a.set_r = slot_set(c, (int)(n % 3));
  a.set_w = slot_set(c, (int)((n + 1) % 3));
  a.set_z = slot_set(c, (int)((n + 2) % 3));
  a.bmax = (double*)c->tiles;
  a.flag = c->flag;
  a.nseg = P.nseg;
  a.GE = P.GE;
  a.s_cap = c->s_cap;
  a.unlimited = (int)(c->desc.scheme == 2);
  a.mode = nullptr;
  a.nhat = nullptr;
  a.dfl = nullptr;
  a.tgt = nullptr;
  a.kcount = nullptr;
  a.thr = 0.0;
  a.sums = (double*)(c->ws + P.off_sums);
  a.nstep = n;
  const bool ft = (P.G.mu == 0.0);
  const bool eul = !ft && c->desc.scheme != 1;
  if (c->clos_dirty && !eul) {
    fmt_err(c->err, "after closure steps, run a step with finite tau and the HOFKS scheme first");
    return HOFKS_ESTATE;
  }
  if constexpr (D == 2) {
    if ((c->clos_on || snap_x || c->clos_dirty) && eul)
      return launch_closure_step<T>(c, a, snap_x, snap_t);
  }
  if (eul) {
    hofks_status st = fork_euler<D, T>(c, a);
    if (st) return st;
  }
  const dim3 grid((unsigned)((long)P.nseg * P.nrowgrp));
  {
    Mark m(c, 1);
    if (ft)
      dispatch_kin<D, T, true, false>(c, a, grid);
    else if (eul)
      dispatch_kin<D, T, false, true>(c, a, grid);
    else
      dispatch_kin<D, T, false, false>(c, a, grid);
    HIPCHK(c, hipGetLastError());
  }
  if (eul) return join_update<D, T, false>(c, a);
  return HOFKS_OK;
}

// closure step (2D): indicator and N^ from the network (or, for a training
// snapshot, every cell kinetic and the inputs of U^n stored), dilation by
// the reach of one shift, Euler solve, kinetic kernel in its closure form
template <typename T>
hofks_status launch_closure_step(hofks_ctx* c, StepArgs<T>& a, float* snap_x, float* snap_t) {
  const Plan& P = c->P;
  const int nc = P.G.nc;
  const double rt = c->tau / P.G.dt;
  const float ftau = (float)std::min(8.0, std::max(-8.0, std::log10(rt)));
  a.mode = c->cmode;
  a.nhat = c->nhat;
  a.dfl = c->cdfl;
  a.kcount = c->kcount;
  a.thr = c->clos_thr;
  {
    hofks_status st = fork_euler<2, T>(c, a);
    if (st) return st;
  }
  const bool all_kin = snap_x || !c->clos_on;  // snapshot, or clearing the marks
  if (all_kin) {
    a.tgt = snap_t;
    Mark m2(c, 3);
    hipLaunchKernelGGL(k_fill_u8, dim3(nblk(nc)), dim3(256), 0, c->stream, c->cmode, nc,
                       (unsigned char)1);
    if (snap_x)
      hipLaunchKernelGGL(k_closure_features, dim3(nblk(nc)), dim3(256), 0, c->stream,
                         (const double*)a.U_in, snap_x, P.G, ftau);
  } else {
    Mark m2(c, 3);
    ClosureArgs ca;
    ca.U = a.U_in;
    ca.packed = c->clos_w;
    ca.nhat = c->nhat;
    ca.flagged = c->cflag;
    ca.dfl = c->cdfl;
    ca.y0 = c->clos_y0;
    ca.ftau = ftau;
    ca.lam = P.G.lam;
    ca.sigma = c->clos_sigma;
    ca.thr = c->clos_thr;
    if (!c->clos_y0_ok || c->clos_y0_ftau != ftau) {  // once per network and tau
      hipLaunchKernelGGL(k_closure_center, dim3(1), dim3(64), 0, c->stream, c->clos_w,
                         c->clos_y0, ftau);
      c->clos_y0_ok = true;
      c->clos_y0_ftau = ftau;
    }
    // one resident round of blocks (two per compute unit at this kernel's
    // register use), each wavefront looping over 16-cell tiles, so that the
    // network weights are loaded into registers once per wavefront
    const unsigned tiles = (unsigned)((nc + 15) / 16);
    const unsigned grid = std::min(2u * (unsigned)P.ncu, (tiles + 3) / 4);
    hipLaunchKernelGGL(k_closure_mlp, dim3(grid), dim3(256), 0, c->stream, ca, P.G);
    const int h = P.G.nv1 / 2;
    hipLaunchKernelGGL((k_dilate<0>), dim3(nblk(nc)), dim3(256), 0, c->stream,
                       (const unsigned char*)c->cflag, c->ctmp, P.G, h);
    hipLaunchKernelGGL((k_dilate<1>), dim3(nblk(nc)), dim3(256), 0, c->stream,
                       (const unsigned char*)c->ctmp, c->cmode, P.G, h);
  }
  HIPCHK(c, hipGetLastError());
  const dim3 grid((unsigned)((long)P.nseg * P.nrowgrp));
  Mark m(c, 1);
  constexpr bool CP = sizeof(T) == 4;
  const int ng = c->kng;
  const bool u16 = P.G.nv1 % 16 == 0;
  const size_t lds = kin_lds(P, ng);
#define KC(BCX, NG, U)                                                                          \
  hipLaunchKernelGGL((k_kinetic<2, T, false, CP, BCX, U, true, NG, true>), grid, dim3(64 * NG), \
                     lds, c->stream, a, P.G, P.A)
#define KCB(NG, U) \
  if (P.G.bc[0] == 0) KC(0, NG, U); else KC(1, NG, U);
  if (ng == 2) {
    if (u16) { KCB(2, 16) } else { KCB(2, 1) }
  } else if (ng == 8) {
    if (u16) { KCB(8, 16) } else { KCB(8, 1) }
  } else {
    if (u16) { KCB(4, 16) } else { KCB(4, 1) }
  }
#undef KCB
#undef KC
  HIPCHK(c, hipGetLastError());
  hofks_status st = join_update<2, T, true>(c, a);
  if (st) return st;
  if (!all_kin) c->clos_steps++;
  c->clos_dirty = !all_kin;
  return HOFKS_OK;
}

// Within a long step call on a 2D or 3D grid the host reads back the Euler
// sub-step count of a step some steps behind the one it queues, so that the
// per-sub-step Euler launches of the later steps follow a count that grows
// during the call (otherwise the persistent tail, slower per sub-step beside
// the kinetic kernel, runs the growth).  Reads are 8 steps apart while the
// count moves and up to 64 while it does not; while two reads agree the spare
// Euler launch is dropped.  The host waits for the step a
// read follows only when it is PEEK_LAG steps ahead of it, so the device
// keeps that many steps queued; the wait polls (a blocking wait wakes up
// late).  On 1D grids the tail is the faster form.
constexpr long PEEK_LAG = 16;
constexpr int PEEK_MIN = 8, PEEK_MAX = 64;

hofks_status peek_substeps(hofks_ctx* c) {
  if (c->peek_pending) {
    hipError_t q = hipEventQuery(c->ev_peek);
    if (q == hipErrorNotReady) {
      (void)hipGetLastError();  // clear the status the query leaves
      if (c->steps - c->peek_at < PEEK_LAG) return HOFKS_OK;
      do {
        q = hipEventQuery(c->ev_peek);
        if (q == hipErrorNotReady) (void)hipGetLastError();
      } while (q == hipErrorNotReady);
    }
    if (q != hipSuccess) return fmt_err(c->err, "step count read-back failed"), HOFKS_EDEVICE;
    const int sv = *c->peek_h;
    c->peek_every = (sv > 0 && sv != c->s_known) ? PEEK_MIN : std::min(PEEK_MAX, 2 * c->peek_every);
    if (sv > 0) c->s_known = sv;
    c->peek_pending = false;
  }
  return HOFKS_OK;
}

// whether the step about to be queued copies its sub-step count back
bool peek_due(const hofks_ctx* c) {
  // (a step count set back by a new state leaves peek_next far ahead: read)
  return !c->peek_pending && (c->steps >= c->peek_next || c->peek_next - c->steps > PEEK_MAX);
}

template <int D, typename T>
hofks_status step_impl(hofks_ctx* c, int nsteps) {
  c->fork_pending = false;
  hofks_status st = HOFKS_OK;
  for (int it = 0; it < nsteps && !st; ++it) {
    c->fork_next = it + 1 < nsteps;
    if (c->strang) set_step_weights(c);
    const bool peek = c->euler_k == 0 && D >= 2 && nsteps > PEEK_LAG;
    if (peek) st = peek_substeps(c);
    if (st) break;
    c->peek_now = peek && peek_due(c);
    c->s_margin = peek && c->peek_every > PEEK_MIN ? 0 : 1;  // two reads agreed
    st = launch_step<D, T>(c);
    if (st) break;
    c->cur ^= 1;
    c->steps++;
    c->inv_prev = inv_tau(c->tau);
  }
  if (c->strang) set_step_weights(c);
  c->fork_next = c->fork_pending = false;
  c->s_margin = 1;
  return st;
}

template <typename F>
hofks_status dispatch(hofks_ctx* c, F&& f) {
  const int d = c->P.d;
  if (c->P.prec) {
    if (d == 1) return f(std::integral_constant<int, 1>(), float());
    if (d == 2) return f(std::integral_constant<int, 2>(), float());
    return f(std::integral_constant<int, 3>(), float());
  }
  if (d == 1) return f(std::integral_constant<int, 1>(), double());
  if (d == 2) return f(std::integral_constant<int, 2>(), double());
  return f(std::integral_constant<int, 3>(), double());
}

hofks_status zero_doubles(hofks_ctx* c, double* p, size_t n) {
  hipLaunchKernelGGL(k_zero, dim3(nblk(n)), dim3(256), 0, c->stream, p, n);
  HIPCHK(c, hipGetLastError());
  return HOFKS_OK;
}

hofks_status zero_ints(hofks_ctx* c, int* p, int n) {
  hipLaunchKernelGGL(k_zero_int, dim3(nblk((size_t)n)), dim3(256), 0, c->stream, p, n);
  HIPCHK(c, hipGetLastError());
  return HOFKS_OK;
}

// a sub-step count read back for an earlier step, still in flight, would
// later replace a newer one: wait for it and drop it
hofks_status drop_peek(hofks_ctx* c) {
  if (c->peek_pending) {
    HIPCHK(c, hipEventSynchronize(c->ev_peek));
    c->peek_pending = false;
  }
  return HOFKS_OK;
}

hofks_status read_flag(hofks_ctx* c) {
  int h[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(h, c->flag, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  hofks_status st = drop_peek(c);
  if (st) return st;
  if (h[1] > 0) c->s_known = h[1];
  if (h[0] & FLAG_SPIN) {
    fmt_err(c->err, "a bounded wait of the step kernel gave up; results are invalid");
    return HOFKS_EDEVICE;
  }
  if (h[0] & FLAG_NONPHYS) {
    fmt_err(c->err, "non-physical moments (rho <= 0, theta <= 0 or non-finite) were met");
    return HOFKS_ENONPHYS;
  }
  if (h[0] & FLAG_SUBSTEP) {
    fmt_err(c->err, "Euler sub-step count exceeded the planned cap %d", c->s_cap);
    return HOFKS_ESTATE;
  }
  return HOFKS_OK;
}

// sub-step cap from the speeds of U^n (row 0 of the read set)
hofks_status plan_substeps(hofks_ctx* c) {
  double a[ASTR];
  HIPCHK(c, hipMemcpyAsync(a, slot_set(c, rset(c)), sizeof(a), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double sum = 0.0;
  for (int k = 0; k < c->P.d; ++k) sum += a[k];
  const double sv = std::ceil(c->P.G.sfac * c->P.G.dt * sum / c->P.G.dx);
  const int s0 = (sv >= 1.0 && sv < SMAX) ? (int)sv : (sv >= SMAX ? SMAX : 1);
  c->s_cap = std::min(SMAX, std::max(2 * s0, s0 + 8));
  hofks_status st = drop_peek(c);  // the count of the previous state
  if (st) return st;
  c->s_known = s0;
  c->peek_every = PEEK_MIN;
  c->peek_next = 0;
  return HOFKS_OK;
}

// records and speeds of the current U and cf with the current lambda
hofks_status refresh(hofks_ctx* c) {
  hofks_status st = zero_doubles(c, c->slots, 3 * (size_t)SET_D);
  if (st) return st;
  st = dispatch(c, [&](auto D, auto t) {
    return launch_cell_init<decltype(D)::value, decltype(t)>(c, MODE_RETAU);
  });
  if (st) return st;
  return plan_substeps(c);
}

// common start of both state set-ups
hofks_status reset_counters(hofks_ctx* c) {
  c->cur = 0;
  c->steps = 0;
  c->inv_prev = 0.0;
  set_step_weights(c);  // Strang: the first step opens with a half relaxation
  hofks_status st = zero_ints(c, c->flag, 16);
  if (st) return st;
  if (c->cdfl) {  // closure form: every cell marked kinetic for its first
                  // step, no count, every cell keeps pieces
    c->clos_dirty = false;
    c->clos_steps = 0;
    hipLaunchKernelGGL(k_fill_u8, dim3(nblk(c->P.G.nc)), dim3(256), 0, c->stream, c->cdfl,
                       c->P.G.nc, (unsigned char)1);
    st = zero_doubles(c, (double*)c->kcount, 1);
    if (st) return st;
  }
  return zero_doubles(c, c->slots, 3 * (size_t)SET_D);
}

// batch helpers (defined with the batch code below)
hofks_status batch_set_state(hofks_ctx*, const double*, const double*, const double*);
hofks_status batch_step(hofks_ctx*, int, bool);
hofks_status batch_read_flag(hofks_ctx*);
hofks_status batch_read_moments(hofks_ctx*, double*);
hofks_status batch_read_f(hofks_ctx*, double*, size_t);
hofks_status batch_max_substeps(hofks_ctx*, int*);
double batch_dt(const hofks_ctx*);
}  // namespace

// ====================================================================== ABI
extern "C" {

hofks_status hofks_workspace_size(const hofks_grid_desc* desc, size_t* bytes) {
  if (!bytes) return HOFKS_EINVAL;
  Plan P;
  hofks_status st = make_plan(desc, &P, nullptr);
  if (st) return st;
  *bytes = P.total;
  return HOFKS_OK;
}

hofks_status hofks_create(const hofks_grid_desc* desc, void* dev_ws, size_t ws_bytes,
                          void* hip_stream, hofks_ctx** out) {
  if (!out) return HOFKS_EINVAL;
  *out = nullptr;
  hofks_ctx* c = new (std::nothrow) hofks_ctx();
  if (!c) return HOFKS_EINVAL;
  hofks_status st = make_plan(desc, &c->P, c->err);
  if (st) {
    delete c;
    return st;
  }
  if (!dev_ws || ws_bytes < c->P.total || ((uintptr_t)dev_ws & 255)) {
    delete c;
    return HOFKS_ESIZE;
  }
  c->desc = *desc;
  c->strang = desc->splitting == 1;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (unsigned char*)dev_ws;
  const Plan& P = c->P;
  for (int i = 0; i < 2; ++i) {
    c->g[i] = c->ws + P.off_g[i];
    c->U[i] = (double*)(c->ws + P.off_U[i]);
    c->UE[i] = (double*)(c->ws + P.off_UE[i]);
    c->rec[i] = (void*)(c->ws + P.off_rec[i]);
  }
  for (int i = 2; i < 4; ++i)
    c->UE[i] = desc->scheme == 3 ? (double*)(c->ws + P.off_UE[i]) : nullptr;
  c->cur = 0;
  c->vt = (VelNode*)(c->ws + P.off_vt);
  c->cf = (double*)(c->ws + P.off_cf);
  c->part = (double*)(c->ws + P.off_part);
  c->slots = (double*)(c->ws + P.off_slots);
  c->tiles = (int*)(c->ws + P.off_tiles);
  c->flag = (int*)(c->ws + P.off_flag);
  if (P.d == 2) {
    unsigned char* b = c->ws + P.off_clos;
    const size_t nc = P.G.nc;
    c->nhat = (float4*)b;
    b += align256(nc * sizeof(float4));
    c->cflag = b;
    c->ctmp = b + nc;
    c->cmode = b + 2 * nc;
    c->cdfl = b + 3 * nc;
    b += align256(4 * nc);
    c->kcount = (unsigned long long*)b;
    c->clos_y0 = (float*)(b + 16);
  }
  // the fork and join events order the two streams of this device only, so
  // they need no system-scope fence (no host or peer reads between them)
  constexpr unsigned evf = hipEventDisableTiming | hipEventDisableSystemFence;
  if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, evf) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, evf) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_peek, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->peek_h), sizeof(int), hipHostMallocDefault) !=
          hipSuccess) {
    hofks_destroy(c);
    return HOFKS_EDEVICE;
  }
  *c->peek_h = 0;
  c->peek_pending = false;
  c->peek_every = PEEK_MIN;
  c->peek_next = 0;
  c->tau = INFINITY;
  c->s_cap = 1;
  c->s_known = 1;
  c->s_margin = 1;
  // kinetic configuration before any tuning: wider unroll in 2D/3D, two
  // wavefronts per block for the FP64 2D grid
  c->kng = (P.d == 2 && !P.prec) ? 2 : 4;
  c->kunr = P.d >= 2 ? 16 : 8;
  if (kin_lds(P, c->kng) > 65536) c->kng = 2;
  c->kring = P.d == 3 && kin3_lds(P) <= 65536;
  c->kwide = P.d == 2 && !P.prec && P.G.nv1 % 4 == 0 && kin2w_lds(P, 4) <= 65536;
  if (c->kwide) {
    c->kng = 4;
    c->kunr = 4;
  }
  if (P.G.offl) {  // off-lattice: the generic kinetic kernel with per-step shifts
    c->kring = c->kwide = 0;
    c->kng = 4;
  }
  // velocity node table of one axis (the lattice, used by every kernel)
  std::vector<VelNode> tab(P.G.nv1);
  for (int i = 0; i < P.G.nv1; ++i) {
    const double v = (i - P.G.kofs) * P.G.dv;
    tab[i] = VelNode{v, v * v, (float)v, (float)(0.5 * v * v), 0.5 * v * v};
  }
  std::vector<double> ctab(P.G.nv1);
  for (int i = 0; i < P.G.nv1; ++i) ctab[i] = ((i - P.G.kofs) * P.G.dv) * P.G.dt / P.G.dx;
  if (reset_counters(c) != HOFKS_OK ||
      hipMemcpyAsync(c->vt, tab.data(), tab.size() * sizeof(VelNode), hipMemcpyHostToDevice,
                     c->stream) != hipSuccess ||
      hipMemcpyAsync(c->vt + P.G.nv1, ctab.data(), ctab.size() * sizeof(double),
                     hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    delete c;
    return HOFKS_EDEVICE;
  }
  *out = c;
  return HOFKS_OK;
}

hofks_status hofks_set_tau(hofks_ctx* c, double tau) {
  if (!c) return HOFKS_EINVAL;
  if (c->batch) return fmt_err(c->err, "tube relaxation times are fixed at creation"), HOFKS_EINVAL;
  if (!(tau >= 0.0)) return fmt_err(c->err, "tau must be >= 0 or +inf"), HOFKS_EINVAL;
  c->tau = tau;
  set_step_weights(c);
  if (c->ready) return refresh(c);
  return HOFKS_OK;
}

hofks_status hofks_set_state_macro(hofks_ctx* c, const double* rho, const double* u,
                                   const double* theta) {
  if (!c || !rho || !theta || !u) return HOFKS_EINVAL;
  if (c->batch) return batch_set_state(c, rho, u, theta);
  const Plan& P = c->P;
  const size_t nc = P.G.nc;
  hofks_status st = reset_counters(c);
  if (st) return st;
  double* prim = c->UE[0];  // (d+2) x nc staging: rho | u | theta
  HIPCHK(c, hipMemcpyAsync(prim, rho, nc * 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(prim + nc, u, nc * 8 * P.d, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(prim + nc * (P.d + 1), theta, nc * 8, hipMemcpyHostToDevice, c->stream));
  st = zero_doubles(c, c->cf, (size_t)P.nm * nc);
  if (st) return st;
  st = dispatch(c, [&](auto D, auto t) -> hofks_status {
    constexpr int DD = decltype(D)::value;
    using T = decltype(t);
    hipLaunchKernelGGL((k_prim_to_moments<DD>), dim3(nblk(nc)), dim3(256), 0, c->stream, prim,
                       c->U[0], (int)nc);
    // Maxwellian parameters of U^0, then sample M into the pieces, sum the
    // stored pieces and project onto U^0 (f^0 = E[U^0], section 4.2)
    hofks_status s2 = launch_cell_init<DD, T>(c, MODE_REFRESH);
    if (s2) return s2;
    const size_t tot = (size_t)P.G.nv * nc;
    hipLaunchKernelGGL((k_fill_maxwellian<DD, T>), dim3(nblk(tot)), dim3(256), 0, c->stream,
                       (T*)c->g[0], (const T*)c->rec[0], P.G);
    hipLaunchKernelGGL((k_piece_sums<DD, T>), dim3(nblk(nc)), dim3(256), 0, c->stream,
                       (const T*)c->g[0], c->part, P.G);
    HIPCHK(c, hipGetLastError());
    s2 = zero_doubles(c, c->slots, 3 * (size_t)SET_D);
    if (s2) return s2;
    return launch_cell_init<DD, T>(c, MODE_INIT);
  });
  if (st) return st;
  c->ready = true;
  st = plan_substeps(c);
  if (st) return st;
  return read_flag(c);
}

hofks_status hofks_set_state_f(hofks_ctx* c, const double* f, size_t bytes) {
  if (!c || !f) return HOFKS_EINVAL;
  if (c->batch) return fmt_err(c->err, "not available for batches"), HOFKS_EINVAL;
  const Plan& P = c->P;
  const size_t nc = P.G.nc, tot = (size_t)P.G.nv * nc;
  if (bytes < tot * 8) return HOFKS_ESIZE;
  hofks_status st = reset_counters(c);
  if (st) return st;
  // stage FP64 planes through the idle piece buffer, store in piece precision
  const size_t per = std::max<size_t>(1, (tot * P.tsize) / (nc * 8));
  double* stage = (double*)c->g[1];
  for (size_t k0 = 0; k0 < (size_t)P.G.nv; k0 += per) {
    const size_t nk = std::min(per, (size_t)P.G.nv - k0);
    HIPCHK(c, hipMemcpyAsync(stage, f + k0 * nc, nk * nc * 8, hipMemcpyHostToDevice, c->stream));
    st = dispatch(c, [&](auto, auto t) -> hofks_status {
      using T = decltype(t);
      hipLaunchKernelGGL((k_store_planes<T>), dim3(nblk(nk * nc)), dim3(256), 0, c->stream,
                         (T*)c->g[0] + k0 * nc, stage, nk * nc);
      HIPCHK(c, hipGetLastError());
      return HOFKS_OK;
    });
    if (st) return st;
  }
  st = dispatch(c, [&](auto D, auto t) -> hofks_status {
    constexpr int DD = decltype(D)::value;
    using T = decltype(t);
    hipLaunchKernelGGL((k_piece_sums<DD, T>), dim3(nblk(nc)), dim3(256), 0, c->stream,
                       (const T*)c->g[0], c->part, P.G);
    HIPCHK(c, hipGetLastError());
    return launch_cell_init<DD, T>(c, MODE_INIT_FROM_SUMS);
  });
  if (st) return st;
  c->ready = true;
  st = plan_substeps(c);
  if (st) return st;
  return read_flag(c);
}

hofks_status hofks_step(hofks_ctx* c, int n) {
  if (!c || n < 0) return HOFKS_EINVAL;
  if (!c->ready) return fmt_err(c->err, "set the state before stepping"), HOFKS_ESTATE;
  if (c->batch) return batch_step(c, n, true);
  return dispatch(c, [&](auto D, auto t) {
    return step_impl<decltype(D)::value, decltype(t)>(c, n);
  });
}

hofks_status hofks_sync(hofks_ctx* c) {
  if (!c) return HOFKS_EINVAL;
  if (c->batch) return batch_read_flag(c);
  return read_flag(c);
}

hofks_status hofks_read_moments(hofks_ctx* c, double* U) {
  if (!c || !U) return HOFKS_EINVAL;
  if (c->batch) return batch_read_moments(c, U);
  HIPCHK(c, hipMemcpyAsync(U, c->U[rpar(c)], (size_t)c->P.nm * c->P.G.nc * 8,
                           hipMemcpyDeviceToHost, c->stream));
  return read_flag(c);
}

hofks_status hofks_read_f(hofks_ctx* c, double* f, size_t bytes) {
  if (!c || !f) return HOFKS_EINVAL;
  if (c->batch) return batch_read_f(c, f, bytes);
  const Plan& P = c->P;
  const size_t nc = P.G.nc, tot = (size_t)P.G.nv * nc;
  if (bytes < tot * 8) return HOFKS_ESIZE;
  const size_t per = std::max<size_t>(1, (tot * P.tsize) / (nc * 8));
  double* stage = (double*)c->g[c->cur ^ 1];
  // Strang splitting: f at t^n includes the pending half relaxation of the
  // last step towards E[U^n] (the stored pieces wait for it)
  double blend = 1.0, mh = 0.0;
  if (c->strang && c->steps > 0) strang_weights(P.G.dt, c->inv_prev, 0.0, &blend, &mh);
  for (size_t k0 = 0; k0 < (size_t)P.G.nv; k0 += per) {
    const size_t nk = std::min(per, (size_t)P.G.nv - k0);
    hofks_status st = dispatch(c, [&](auto D, auto t) -> hofks_status {
      constexpr int DD = decltype(D)::value;
      using T = decltype(t);
      hipLaunchKernelGGL((k_materialize<DD, T>), dim3(nblk(nk * nc)), dim3(256), 0, c->stream,
                         (const T*)c->g[c->cur], c->cf, stage, (int)k0, (int)nk, P.G,
                         c->clos_dirty ? (const T*)c->rec[rpar(c)] : nullptr, blend,
                         blend < 1.0 ? (const T*)c->rec[rpar(c)] : nullptr);
      HIPCHK(c, hipGetLastError());
      return HOFKS_OK;
    });
    if (st) return st;
    HIPCHK(c, hipMemcpyAsync(f + k0 * nc, stage, nk * nc * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return read_flag(c);
}

// ------------------------------------------------------------ checkpoint
// Host image of the state: a header (shape, tau, step count, speeds of U^n)
// then U^n, the pending correction cf, the records and the pieces (the
// Eulerian pieces g; f = g + w m.cf).  Enough to continue stepping exactly.
struct StateHeader {
  char magic[8];
  int version, dim, n[3], nv1, precision, scheme, bc[3], splitting;
  double dx, dv, tau, dt, inv_prev;
  long long steps;
  double speeds[ASTR];
};

size_t state_bytes(const Plan& P) {
  return sizeof(StateHeader) + 2 * (size_t)P.nm * P.G.nc * sizeof(double) +
         (size_t)P.RS * P.G.nc * P.tsize + (size_t)P.G.nv * P.G.nc * P.tsize;
}

hofks_status hofks_state_bytes(hofks_ctx* c, size_t* bytes) {
  if (!c || !bytes) return HOFKS_EINVAL;
  if (c->batch) return fmt_err(c->err, "not available for batches"), HOFKS_EINVAL;
  *bytes = state_bytes(c->P);
  return HOFKS_OK;
}

hofks_status hofks_read_state(hofks_ctx* c, void* host, size_t bytes) {
  if (!c || !host) return HOFKS_EINVAL;
  if (c->batch) return fmt_err(c->err, "not available for batches"), HOFKS_EINVAL;
  if (!c->ready) return fmt_err(c->err, "no state to read"), HOFKS_ESTATE;
  if (c->clos_dirty)
    return fmt_err(c->err, "closure cells hold no pieces: run a step without the closure first"),
           HOFKS_ESTATE;
  const Plan& P = c->P;
  if (bytes < state_bytes(P)) return HOFKS_ESIZE;
  hofks_status st = read_flag(c);
  if (st) return st;
  StateHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, "HOFKSST1", 8);
  h.version = 2;
  h.dim = P.d;
  for (int a = 0; a < 3; ++a) {
    h.n[a] = P.G.n[a];
    h.bc[a] = P.G.bc[a];
  }
  h.nv1 = P.G.nv1;
  h.precision = P.prec;
  h.scheme = c->desc.scheme;
  h.dx = P.G.dx;
  h.dv = P.G.dv;
  h.tau = c->tau;
  h.dt = P.G.dt;
  h.splitting = c->desc.splitting;
  h.inv_prev = c->inv_prev;
  h.steps = c->steps;
  HIPCHK(c, hipMemcpyAsync(h.speeds, slot_set(c, rset(c)), sizeof(h.speeds), hipMemcpyDeviceToHost,
                           c->stream));
  unsigned char* o = (unsigned char*)host + sizeof(StateHeader);
  const size_t ub = (size_t)P.nm * P.G.nc * sizeof(double);
  const size_t rb = (size_t)P.RS * P.G.nc * P.tsize, gb = (size_t)P.G.nv * P.G.nc * P.tsize;
  const int rp = rpar(c);
  HIPCHK(c, hipMemcpyAsync(o, c->U[rp], ub, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(o + ub, c->cf, ub, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(o + 2 * ub, c->rec[rp], rb, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(o + 2 * ub + rb, c->g[c->cur], gb, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::memcpy(host, &h, sizeof(h));
  return HOFKS_OK;
}

hofks_status hofks_write_state(hofks_ctx* c, const void* host, size_t bytes) {
  if (!c || !host) return HOFKS_EINVAL;
  if (c->batch) return fmt_err(c->err, "not available for batches"), HOFKS_EINVAL;
  const Plan& P = c->P;
  if (bytes < state_bytes(P)) return HOFKS_ESIZE;
  StateHeader h;
  std::memcpy(&h, host, sizeof(h));
  bool same = std::memcmp(h.magic, "HOFKSST1", 8) == 0 && h.version == 2 && h.dim == P.d &&
              h.nv1 == P.G.nv1 && h.precision == P.prec && h.scheme == c->desc.scheme &&
              h.dx == P.G.dx && h.dv == P.G.dv && h.dt == P.G.dt &&
              h.splitting == c->desc.splitting && h.steps >= 0;
  for (int a = 0; a < 3; ++a) same = same && h.n[a] == P.G.n[a] && h.bc[a] == P.G.bc[a];
  if (!same) return fmt_err(c->err, "state image does not match this grid"), HOFKS_EINVAL;
  hofks_status st = hofks_set_tau(c, h.tau);  // lambda of the stored records
  if (st) return st;
  st = reset_counters(c);
  if (st) return st;
  c->steps = h.steps;
  c->inv_prev = h.inv_prev;
  set_step_weights(c);
  c->cur = 0;
  const unsigned char* o = (const unsigned char*)host + sizeof(StateHeader);
  const size_t ub = (size_t)P.nm * P.G.nc * sizeof(double);
  const size_t rb = (size_t)P.RS * P.G.nc * P.tsize, gb = (size_t)P.G.nv * P.G.nc * P.tsize;
  const int rp = rpar(c);
  HIPCHK(c, hipMemcpyAsync(c->U[rp], o, ub, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->cf, o + ub, ub, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->rec[rp], o + 2 * ub, rb, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->g[0], o + 2 * ub + rb, gb, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(slot_set(c, rset(c)), h.speeds, sizeof(h.speeds),
                           hipMemcpyHostToDevice, c->stream));
  c->ready = true;
  st = plan_substeps(c);
  if (st) return st;
  return read_flag(c);
}

hofks_status hofks_read_counters(hofks_ctx* c, int* substeps, long* steps) {
  if (!c) return HOFKS_EINVAL;
  int h[2] = {0, 0};
  if (c->batch) {
    hofks_status st = batch_max_substeps(c, h + 1);
    if (st) return st;
  } else {
    HIPCHK(c, hipMemcpyAsync(h, c->flag, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  if (substeps) *substeps = h[1];
  if (steps) *steps = c->steps;
  return HOFKS_OK;
}

hofks_status hofks_kernel_timing(hofks_ctx* c, int enable, double* ms, int* launches) {
  if (!c) return HOFKS_EINVAL;
  if (enable < 0 || enable > 15) return fmt_err(c->err, "timing group mask %d", enable), HOFKS_EINVAL;
  if (ms || launches) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int cnt[4] = {0, 0, 0, 0};
    for (auto& m : c->ev_marks) {
      float t = 0.0f;
      HIPCHK(c, hipEventElapsedTime(&t, m.a, m.b));
      acc[m.group] += t;
      cnt[m.group] += m.count;
    }
    for (int g = 0; g < 4; ++g) {
      if (ms) ms[g] = acc[g];
      if (launches) launches[g] = cnt[g];
    }
  }
  c->ev_marks.clear();
  c->ev_next = 0;
  c->timing = (unsigned)enable;
  return HOFKS_OK;
}

hofks_status hofks_read_tail_substeps(hofks_ctx* c, long* n) {
  if (!c || !n) return HOFKS_EINVAL;
  if (c->batch) {
    *n = 0;
    return HOFKS_OK;
  }
  int h[3] = {0, 0, 0};
  HIPCHK(c, hipMemcpyAsync(h, c->flag, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *n = h[2];
  return HOFKS_OK;
}

hofks_status hofks_set_euler_launches(hofks_ctx* c, int k) {
  if (!c || k < 0) return HOFKS_EINVAL;
  if (c->batch) return fmt_err(c->err, "not available for batches"), HOFKS_EINVAL;
  c->euler_k = k;
  return HOFKS_OK;
}

double hofks_dt(const hofks_ctx* c) {
  if (!c) return 0.0;
  return c->batch ? batch_dt(c) : c->P.G.dt;
}

const char* hofks_last_error(const hofks_ctx* c) { return c ? c->err : "null context"; }

}  // extern "C"

// ================================================================== batches
// A batch of independent 1D-1V outflow tubes in FP32 pieces.  Host-side plan:
// per-tube offsets into four arenas (pieces, records, FP64 moments, velocity
// nodes), the Euler/kinetic work order, the tuned item width and grid, and a
// captured graph of consecutive step launches.
struct Batch {
  int n = 0;
  std::vector<hofks_grid_desc> descs;
  std::vector<double> taus;
  std::vector<TubeDev> tubes;
  long long g_floats = 0, r_floats = 0, d_doubles = 0;
  int nvt = 0, items_max = 0, eitems_max = 0;
  long long total_cells = 0, total_cv = 0;
  size_t off_gar = 0, off_rar = 0, off_dar = 0, off_vt = 0, off_tubes = 0, off_eitems = 0,
         off_items = 0, off_uitems = 0, off_alpha = 0, off_s = 0, off_tflag = 0,
         off_flag = 0, off_ebar = 0, total = 0;
  // device pointers
  float *gar = nullptr, *rar = nullptr;
  double *dar = nullptr, *alpha = nullptr;
  VelNode* vtar = nullptr;
  TubeDev* tubes_d = nullptr;
  int *tube_s = nullptr, *tflag = nullptr, *flag = nullptr;
  unsigned* ebar = nullptr;
  int4* eitems = nullptr;
  int2* items = nullptr;
  int2* uitems = nullptr;  // update items: 256-cell segments on their tube's die
  // launch configuration; part = cells per part of a split Euler solve (0:
  // every tube whole in one block)
  int cells = 256, unr = 8, nitems = 0, nuitems = 0, neuler = 0, ncu = 256, part = 0;
  size_t lds = 0;
  // graph of GRAPH_STEPS launches starting at parity 0
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_cells = 0, graph_part = -1;
};

namespace {

constexpr int GRAPH_STEPS = 16;

hofks_status batch_plan(const hofks_grid_desc* descs, const double* taus, int n, Batch* B,
                        char* err) {
  if (!descs || n < 1 || n > (1 << 20)) return fmt_err(err, "bad tube count"), HOFKS_EINVAL;
  B->n = n;
  B->descs.assign(descs, descs + n);
  B->taus.assign(n, INFINITY);
  if (taus) B->taus.assign(taus, taus + n);
  B->tubes.resize(n);
  long long go = 0, ro = 0, dof = 0;
  int vto = 0, nitems = 0, eitems = 0;
  constexpr int RS = rec_stride<1, float>();
  for (int i = 0; i < n; ++i) {
    const hofks_grid_desc& d = descs[i];
    if (d.dim != 1 || d.precision != 1 || d.bc[0] != 1 || d.scheme != 0 || d.dt != 0.0 ||
        d.splitting != 0)
      return fmt_err(err, "tube %d: batches hold 1D outflow HOFKS tubes in FP32", i), HOFKS_EINVAL;
    Plan P;
    hofks_status st = make_plan(&d, &P, err);
    if (st) return st;
    if (d.n_vel % 8 != 0 || d.n_vel > 256)
      return fmt_err(err, "tube %d: n_vel must be a multiple of 8", i), HOFKS_EINVAL;
    const double tau = B->taus[i];
    if (!(tau >= 0.0)) return fmt_err(err, "tube %d: tau must be >= 0 or +inf", i), HOFKS_EINVAL;
    TubeDev& T = B->tubes[i];
    const long long Nx = P.G.n[0], nv = P.G.nv1;
    T.g[0] = go;
    T.g[1] = go + nv * Nx;
    go += 2 * nv * Nx;
    T.rec[0] = ro;
    T.rec[1] = ro + RS * Nx;
    ro += 2 * RS * Nx;
    T.U[0] = dof;
    T.U[1] = dof + 3 * Nx;
    T.UE[0] = dof + 6 * Nx;
    T.UE[1] = dof + 9 * Nx;
    T.cf = dof + 12 * Nx;
    T.S = dof + 15 * Nx;
    T.X = dof + 21 * Nx;
    dof += 21 * Nx + 2LL * XSTR * ((Nx + 1023) / 1024);
    T.vt = vto;
    vto += (int)nv;
    T.Nx = (int)Nx;
    T.nv1 = (int)nv;
    T.kofs = P.G.kofs;
    T.dx = P.G.dx;
    T.dv = P.G.dv;
    T.dt = P.G.dt;
    T.w = P.G.w;
    T.gam = P.G.gam;
    if (std::isinf(tau)) {
      T.lam = 1.0;
      T.mu = 0.0;
    } else if (tau == 0.0) {
      T.lam = 0.0;
      T.mu = 1.0;
    } else {
      T.lam = std::exp(-T.dt / tau);
      T.mu = -std::expm1(-T.dt / tau);
    }
    for (int q = 0; q < 9; ++q) T.A[q] = P.A.a[q];
    nitems += (int)((Nx + 255) / 256);
    eitems += (int)((Nx + 1023) / 1024);
    B->total_cells += Nx;
    B->total_cv += Nx * nv;
  }
  B->g_floats = go;
  B->r_floats = ro;
  B->d_doubles = dof;
  B->nvt = vto;
  // the die lists of the kinetic items are padded to equal length: at most
  // NXCD entries per item
  B->items_max = (int)NXCD * nitems;
  B->eitems_max = eitems;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  B->off_gar = take(sizeof(float) * go);
  B->off_rar = take(sizeof(float) * ro);
  B->off_dar = take(sizeof(double) * dof);
  B->off_vt = take(sizeof(VelNode) * vto);
  B->off_tubes = take(sizeof(TubeDev) * n);
  B->off_eitems = take(sizeof(int4) * eitems);
  B->off_items = take(sizeof(int2) * B->items_max);
  B->off_uitems = take(sizeof(int2) * B->items_max);
  B->off_alpha = take(sizeof(double) * n * 2 * ASTR);
  B->off_s = take(sizeof(int) * n);
  B->off_tflag = take(sizeof(int) * n);
  B->off_flag = take(64);
  B->off_ebar = take(sizeof(unsigned) * 2 * n);
  B->total = off;
  return HOFKS_OK;
}

Geom host_tube_geom(const TubeDev& T) {
  Geom G{};
  G.n[0] = T.Nx;
  G.n[1] = G.n[2] = 1;
  G.nc = T.Nx;
  G.nv1 = T.nv1;
  G.kofs = T.kofs;
  G.nv = T.nv1;
  G.bc[0] = 1;
  G.dx = T.dx;
  G.dv = T.dv;
  G.dt = T.dt;
  G.w = T.w;
  G.lam = G.lam_r = T.lam;
  G.mu = G.mu_r = T.mu;
  G.gam = T.gam;
  G.sfac = 2.0;
  return G;
}

int unroll_for(const Batch* B, int cells) {
  const int vg = 1024 / cells;
  int u = 8;
  for (const TubeDev& T : B->tubes) {
    const int per = T.nv1 / vg;
    while (u > 1 && per % u) u /= 2;
  }
  return u;
}

size_t lds_for(const Batch* B, int cells) {
  int nvmax = 0;
  for (const TubeDev& T : B->tubes) nvmax = std::max(nvmax, T.nv1);
  const size_t recb = (size_t)(cells + nvmax - 1) * rec_stride<1, float>() * sizeof(float);
  const size_t redb = (size_t)(1024 / cells - 1) * cells * 6 * sizeof(double);
  return std::max(recb, redb);
}

// work order, on the host from the speeds of U^n: Euler items by decreasing
// work per item (cells of the item times s; the parts of a split tube next
// to each other), kinetic items by decreasing per-item work (n_v).  With
// B->part > 0 a tube longer than part cells is split into ceil(Nx / part)
// parts when that is at most PART_MAX and the compute units, else it stays
// whole.
hofks_status batch_order(hofks_ctx* c) {
  Batch* B = c->batch;
  std::vector<double> al((size_t)B->n * 2 * ASTR);
  HIPCHK(c, hipMemcpyAsync(al.data(), B->alpha, al.size() * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int p = (int)(c->steps & 1);
  std::vector<double> work(B->n);
  std::vector<int> parts(B->n);
  // the parts of a tube must be co-resident: at most one block per compute
  // unit runs (the Euler tiles take most of the LDS)
  const int pmax = std::min(PART_MAX, B->ncu);
  for (int i = 0; i < B->n; ++i) {
    const TubeDev& T = B->tubes[i];
    const double s = std::max(1.0, std::ceil(2.0 * T.dt * al[((size_t)i * 2 + p) * ASTR] / T.dx));
    const int np = B->part > 0 ? (T.Nx + B->part - 1) / B->part : 0;
    parts[i] = (np >= 2 && np <= pmax) ? np : 0;
    work[i] = (double)(parts[i] ? std::min(T.Nx, B->part) : T.Nx) * s;
  }
  std::vector<int> order(B->n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  // whole tubes of at most 2048 cells run two to a block (neighbours in the
  // work order, so of similar work); the others one to a block or in parts
  std::vector<std::pair<double, int4>> ew;
  int pend = -1;
  for (int i : order) {
    if (parts[i]) {
      for (int k = 0; k < parts[i]; ++k) ew.push_back({work[i], make_int4(i, k, parts[i], 1)});
    } else if (B->tubes[i].Nx > 2 * 1024) {
      ew.push_back({work[i], make_int4(i, 0, 0, 0)});
    } else if (pend < 0) {
      pend = i;
    } else {
      const int cpt = (std::max(B->tubes[pend].Nx, B->tubes[i].Nx) + 511) / 512;
      ew.push_back({std::max(work[pend], work[i]), make_int4(pend, i, cpt, 2)});
      pend = -1;
    }
  }
  if (pend >= 0) ew.push_back({work[pend], make_int4(pend, -1, (B->tubes[pend].Nx + 511) / 512, 2)});
  std::stable_sort(ew.begin(), ew.end(),
                   [](const std::pair<double, int4>& a, const std::pair<double, int4>& b) {
                     return a.first > b.first;
                   });
  // kinetic items: the tubes are dealt to the NXCD dies by kinetic work
  // (largest first, each to the least loaded die), a die's list holds its
  // tubes' segments in order, and block b of the kinetic launch takes entry
  // b / NXCD of die b mod NXCD's list (blocks go to the dies round-robin), so
  // neighbouring segments, whose upstream pieces and records overlap, meet
  // in one L2.  Short lists are padded with empty items (tube -1).
  std::vector<int> korder(B->n);
  std::iota(korder.begin(), korder.end(), 0);
  auto kwork = [&](int i) { return (double)B->tubes[i].Nx * B->tubes[i].nv1; };
  std::stable_sort(korder.begin(), korder.end(), [&](int a, int b) { return kwork(a) > kwork(b); });
  std::vector<std::vector<int2>> die(NXCD);
  std::vector<double> load(NXCD, 0.0);
  std::vector<int> tdie(B->n, 0);
  for (int i : korder) {
    const int d = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    for (int sg = 0; sg * B->cells < B->tubes[i].Nx; ++sg) die[d].push_back(make_int2(i, sg));
    load[d] += kwork(i);
    tdie[i] = d;
  }
  // Euler items on their tube's die (the die of its kinetic and update
  // items, whose U^n it reads and which read its result): block p of the
  // Euler launch takes the next item of die p mod NXCD, in work order, or
  // the heaviest item left when that die has none; split solves keep the
  // plain work order (their parts start together)
  std::vector<int4> eitems;
  if (B->part > 0) {
    for (const auto& w : ew) eitems.push_back(w.second);
  } else {
    std::vector<std::vector<std::pair<double, int4>>> dq(NXCD);
    for (const auto& w : ew) dq[tdie[w.second.x]].push_back(w);
    std::vector<size_t> head(NXCD, 0);
    for (size_t pos = 0; pos < ew.size(); ++pos) {
      int d = (int)(pos % NXCD);
      if (head[d] == dq[d].size()) {
        d = -1;
        for (int e = 0; e < (int)NXCD; ++e)
          if (head[e] < dq[e].size() && (d < 0 || dq[e][head[e]].first > dq[d][head[d]].first))
            d = e;
      }
      eitems.push_back(dq[d][head[d]++].second);
    }
  }
  if ((int)eitems.size() > B->eitems_max)
    return fmt_err(c->err, "batch Euler item list exceeds its workspace"), HOFKS_EINVAL;
  size_t len = 0;
  for (const auto& l : die) len = std::max(len, l.size());
  std::vector<int2> items;
  for (size_t q = 0; q < len; ++q)
    for (unsigned d = 0; d < NXCD; ++d)
      items.push_back(q < die[d].size() ? die[d][q] : make_int2(-1, 0));
  if ((int)items.size() > B->items_max)
    return fmt_err(c->err, "batch item list exceeds its workspace"), HOFKS_EINVAL;
  // update items: the same dies, in segments of UPD_CELLS cells
  std::vector<std::vector<int2>> udie(NXCD);
  for (int i : korder)
    for (int sg = 0; sg * UPD_CELLS < B->tubes[i].Nx; ++sg) udie[tdie[i]].push_back(make_int2(i, sg));
  size_t ulen = 0;
  for (const auto& l : udie) ulen = std::max(ulen, l.size());
  std::vector<int2> uitems;
  for (size_t q = 0; q < ulen; ++q)
    for (unsigned d = 0; d < NXCD; ++d)
      uitems.push_back(q < udie[d].size() ? udie[d][q] : make_int2(-1, 0));
  if ((int)uitems.size() > B->items_max)
    return fmt_err(c->err, "batch update item list exceeds its workspace"), HOFKS_EINVAL;
  B->nuitems = (int)uitems.size();
  B->nitems = (int)items.size();
  B->neuler = (int)eitems.size();
  HIPCHK(c, hipMemcpyAsync(B->eitems, eitems.data(), sizeof(int4) * eitems.size(),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(B->items, items.data(), sizeof(int2) * items.size(),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(B->uitems, uitems.data(), sizeof(int2) * uitems.size(),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HOFKS_OK;
}

BatchArgs batch_args(hofks_ctx* c, int parity) {
  Batch* B = c->batch;
  BatchArgs a;
  a.gar = B->gar;
  a.rar = B->rar;
  a.dar = B->dar;
  a.vtar = B->vtar;
  a.tubes = B->tubes_d;
  a.eitems = B->eitems;
  a.items = B->items;
  a.uitems = B->uitems;
  a.neuler = B->neuler;
  a.nitems = B->nitems;
  a.part_cells = B->part > 0 ? B->part : 1024;
  a.ebar = B->ebar;
  a.alpha = B->alpha;
  a.tube_s = B->tube_s;
  a.tflag = B->tflag;
  a.flag = B->flag;
  a.parity = parity;
  a.s_cap = SMAX;
  return a;
}

size_t batch_euler_lds(const Batch* B) {
  return std::max(std::max(RUN_LDS, EUL_LDS), B->part > 0 ? part_lds(B->part) : (size_t)0);
}

// one step: the Euler launch on `stream` and the kinetic launch on the
// context's second stream, forked from and joined to `stream`, then the
// update launch
hofks_status batch_launch(hofks_ctx* c, hipStream_t stream, int parity) {
  Batch* B = c->batch;
  const BatchArgs a = batch_args(c, parity);
  HIPCHK(c, hipEventRecord(c->ev_fork, stream));
  HIPCHK(c, hipStreamWaitEvent(c->aux, c->ev_fork, 0));
  hipLaunchKernelGGL(k_batch_euler, dim3(B->neuler), dim3(1024), batch_euler_lds(B), stream, a);
#define BL(CELLS, UNR) \
  hipLaunchKernelGGL((k_batch_kinetic<CELLS, UNR>), dim3(B->nitems), dim3(1024), B->lds, c->aux, a)
  const int u = B->unr;
  switch (B->cells) {
    case 1024:
      if (u == 8) BL(1024, 8); else if (u == 4) BL(1024, 4); else if (u == 2) BL(1024, 2); else BL(1024, 1);
      break;
    case 512:
      if (u == 8) BL(512, 8); else if (u == 4) BL(512, 4); else if (u == 2) BL(512, 2); else BL(512, 1);
      break;
    default:
      if (u == 8) BL(256, 8); else if (u == 4) BL(256, 4); else if (u == 2) BL(256, 2); else BL(256, 1);
  }
#undef BL
  HIPCHK(c, hipEventRecord(c->ev_join, c->aux));
  HIPCHK(c, hipStreamWaitEvent(stream, c->ev_join, 0));
  hipLaunchKernelGGL(k_batch_update, dim3(B->nuitems), dim3(UPD_CELLS), 0, stream, a);
  HIPCHK(c, hipGetLastError());
  return HOFKS_OK;
}

hofks_status batch_configure(hofks_ctx* c, int cells, int part) {
  Batch* B = c->batch;
  B->cells = cells;
  B->part = part;
  B->unr = unroll_for(B, cells);
  B->lds = lds_for(B, cells);
  return batch_order(c);
}

hofks_status batch_capture(hofks_ctx* c) {
  Batch* B = c->batch;
  if (B->gexec && B->graph_cells == B->cells && B->graph_part == B->part)
    return HOFKS_OK;
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->gexec = nullptr;
  B->graph = nullptr;
  if (!B->cap) HIPCHK(c, hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
  HIPCHK(c, hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < GRAPH_STEPS; ++i) {
    hofks_status st = batch_launch(c, B->cap, i & 1);
    if (st) {
      hipGraph_t g;
      (void)hipStreamEndCapture(B->cap, &g);
      return st;
    }
  }
  HIPCHK(c, hipStreamEndCapture(B->cap, &B->graph));
  HIPCHK(c, hipGraphInstantiate(&B->gexec, B->graph, nullptr, nullptr, 0));
  B->graph_cells = B->cells;
  B->graph_part = B->part;
  return HOFKS_OK;
}

hofks_status batch_step(hofks_ctx* c, int n, bool use_graph) {
  Batch* B = c->batch;
  if (use_graph) {
    hofks_status st = batch_capture(c);
    if (st) return st;
  }
  while (n > 0) {
    const int p = (int)(c->steps & 1);
    if (use_graph && p == 0 && n >= GRAPH_STEPS) {
      {
        Mark m(c, 1, GRAPH_STEPS);
        HIPCHK(c, hipGraphLaunch(B->gexec, c->stream));
      }
      c->steps += GRAPH_STEPS;
      n -= GRAPH_STEPS;
      continue;
    }
    hofks_status st;
    {
      Mark m(c, 1);
      st = batch_launch(c, c->stream, p);
    }
    if (st) return st;
    c->steps += 1;
    n -= 1;
  }
  return HOFKS_OK;
}

hofks_status batch_read_flag(hofks_ctx* c) {
  Batch* B = c->batch;
  int h = 0;
  std::vector<int> tf(B->n);
  HIPCHK(c, hipMemcpyAsync(&h, B->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(tf.data(), B->tflag, sizeof(int) * B->n, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (h & FLAG_SPIN) {
    fmt_err(c->err, "a bounded wait of the batch kernel gave up; results are invalid");
    return HOFKS_EDEVICE;
  }
  int bad = 0, first = -1, bits = 0;
  for (int i = 0; i < B->n; ++i)
    if (tf[i]) {
      ++bad;
      bits |= tf[i];
      if (first < 0) first = i;
    }
  // flagged tubes are reported through hofks_batch_tube_flags and excluded
  // by the caller; the other tubes stay readable
  if (bad)
    fmt_err(c->err, "%d tube(s) flagged (first: %d, bits %d); see hofks_batch_tube_flags", bad,
            first, bits);
  return HOFKS_OK;
}

hofks_status batch_set_state(hofks_ctx* c, const double* rho, const double* u,
                             const double* theta) {
  Batch* B = c->batch;
  c->steps = 0;
  c->cur = 0;
  hofks_status st = zero_ints(c, B->flag, 16);
  if (st) return st;
  st = zero_ints(c, B->tflag, B->n);
  if (st) return st;
  st = zero_ints(c, reinterpret_cast<int*>(B->ebar), 2 * B->n);
  if (st) return st;
  st = zero_doubles(c, B->alpha, (size_t)B->n * 2 * ASTR);
  if (st) return st;
  long long cell0 = 0;
  for (int i = 0; i < B->n; ++i) {
    const TubeDev& T = B->tubes[i];
    const Geom G = host_tube_geom(T);
    Mat A;
    for (int q = 0; q < 9; ++q) A.a[q] = T.A[q];
    const size_t nx = T.Nx;
    double* prim = B->dar + T.UE[0];  // rho | u | theta staging (3 x Nx)
    double* U0 = B->dar + T.U[0];
    double* cf = B->dar + T.cf;
    double* part = B->dar + T.UE[1];
    float* rec0 = B->rar + T.rec[0];
    float* g0 = B->gar + T.g[0];
    const VelNode* vt = B->vtar + T.vt;
    double* al = B->alpha + (size_t)i * 2 * ASTR;
    HIPCHK(c, hipMemcpyAsync(prim, rho + cell0, nx * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(prim + nx, u + cell0, nx * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(prim + 2 * nx, theta + cell0, nx * 8, hipMemcpyHostToDevice, c->stream));
    st = zero_doubles(c, cf, 3 * nx);
    if (st) return st;
    hipLaunchKernelGGL((k_prim_to_moments<1>), dim3(nblk(nx)), dim3(256), 0, c->stream, prim, U0,
                       (int)nx);
    hipLaunchKernelGGL((k_cell_init<1, float>), dim3(nblk(nx)), dim3(256), 0, c->stream, U0, cf,
                       rec0, vt, part, al, B->tflag + i, G, A, (int)MODE_REFRESH);
    hipLaunchKernelGGL((k_fill_maxwellian<1, float>), dim3(nblk(nx * T.nv1)), dim3(256), 0,
                       c->stream, g0, (const float*)rec0, G);
    hipLaunchKernelGGL((k_piece_sums<1, float>), dim3(nblk(nx)), dim3(256), 0, c->stream,
                       (const float*)g0, part, G);
    st = zero_doubles(c, al, ASTR);
    if (st) return st;
    hipLaunchKernelGGL((k_cell_init<1, float>), dim3(nblk(nx)), dim3(256), 0, c->stream, U0, cf,
                       rec0, vt, part, al, B->tflag + i, G, A, (int)MODE_INIT);
    HIPCHK(c, hipGetLastError());
    cell0 += (long long)nx;
  }
  c->ready = true;
  st = batch_order(c);
  if (st) return st;
  return batch_read_flag(c);
}

// single grid: choose (wavefronts per kinetic block, loads issued ahead)
hofks_status grid_autotune(hofks_ctx* c, int steps, const char* cache_path, int* choice) {
  const Plan& P = c->P;
  if (P.G.offl) {  // one configuration (four wavefronts, fixed loads ahead)
    if (choice) {
      choice[0] = 4;
      choice[1] = P.d >= 2 ? 4 : 1;
      choice[2] = c->euler_seq;
    }
    return HOFKS_OK;
  }
  std::ostringstream key;
  key << "gfx950:grid:d=" << P.d << ":n=" << P.G.n[0] << "x" << P.G.n[1] << "x" << P.G.n[2]
      << ":nv=" << P.G.nv1 << ":prec=" << P.prec << ":bc=" << P.G.bc[0] << P.G.bc[1] << P.G.bc[2]
      << ":scheme=" << c->desc.scheme;
  int best_ng = 0, best_unr = 0, best_seq = 0;
  if (cache_path && *cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    const std::string k = "\"key\": \"" + key.str() + "\"";
    while (std::getline(in, line)) {
      if (line.find(k) == std::string::npos) continue;
      const size_t pn = line.find("\"ng\": "), pu = line.find("\"unr\": ");
      const size_t ps = line.find("\"seq\": ");
      if (pn == std::string::npos || pu == std::string::npos || ps == std::string::npos) continue;
      const int ng = std::atoi(line.c_str() + pn + 6), unr = std::atoi(line.c_str() + pu + 7);
      const int sq = std::atoi(line.c_str() + ps + 7);
      if ((ng == 2 || ng == 4 || (ng == 8 && P.d >= 2)) &&
          (unr == 8 || unr == 16 || (unr == 4 && c->kwide)) && (sq == 0 || sq == 1)) {
        best_ng = ng;
        best_unr = unr;
        best_seq = sq;
      }
    }
  }
  if (!best_ng) {
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    // two cells per lane (2D FP64): loads ahead 4 or 8, at most four wavefronts
    const int cand_w[4][2] = {{4, 4}, {2, 4}, {4, 8}, {2, 8}};
    const int cand_n[6][2] = {{4, 8}, {2, 16}, {4, 16}, {2, 8}, {8, 16}, {8, 8}};
    const int ncand = c->kwide ? 4 : 6;
    for (int k = 0; k < ncand; ++k) {
      const int* cd = c->kwide ? cand_w[k] : cand_n[k];
      if (c->kwide && kin2w_lds(P, cd[0]) > 65536) continue;
      if (!c->kwide && (kin_lds(P, cd[0]) > 65536 || (cd[0] == 8 && P.d < 2))) continue;
      if (c->kring && cd[0] != RY) continue;  // 3D: blocks of RY rows, only the unroll varies
      c->kng = cd[0];
      c->kunr = cd[1];
      hofks_status st = hofks_step(c, 1);
      if (st) return st;
      HIPCHK(c, hipEventRecord(e0, c->stream));
      st = hofks_step(c, steps);
      if (st) return st;
      HIPCHK(c, hipEventRecord(e1, c->stream));
      HIPCHK(c, hipEventSynchronize(e1));
      float ms = 0.0f;
      HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) {
        best_ms = ms;
        best_ng = cd[0];
        best_unr = cd[1];
      }
    }
    // the Euler solve before the kinetic kernel instead of beside it: it
    // then has the chip to itself and does not slow the kinetic kernel
    if (best_ng) {
      c->kng = best_ng;
      c->kunr = best_unr;
      c->euler_seq = !c->euler_seq;
      hofks_status st = hofks_step(c, 1);
      if (st) return st;
      HIPCHK(c, hipEventRecord(e0, c->stream));
      st = hofks_step(c, steps);
      if (st) return st;
      HIPCHK(c, hipEventRecord(e1, c->stream));
      HIPCHK(c, hipEventSynchronize(e1));
      float ms = 0.0f;
      HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) best_ms = ms;
      else c->euler_seq = !c->euler_seq;
      best_seq = c->euler_seq;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (cache_path && *cache_path) {
      std::ofstream o(cache_path, std::ios::app);
      o << "{\"key\": \"" << key.str() << "\", \"ng\": " << best_ng << ", \"unr\": " << best_unr
        << ", \"seq\": " << best_seq << ", \"ms_per_step\": " << best_ms / steps << "}\n";
    }
  }
  c->kng = best_ng;
  c->kunr = best_unr;
  c->euler_seq = best_seq != 0;
  if (choice) {
    choice[0] = best_ng;
    choice[1] = best_unr;
    choice[2] = best_seq;
  }
  return read_flag(c);
}

}  // namespace

extern "C" {

hofks_status hofks_batch_workspace_size(const hofks_grid_desc* descs, int n, size_t* bytes) {
  if (!bytes) return HOFKS_EINVAL;
  Batch B;
  hofks_status st = batch_plan(descs, nullptr, n, &B, nullptr);
  if (st) return st;
  *bytes = B.total;
  return HOFKS_OK;
}

hofks_status hofks_batch_create(const hofks_grid_desc* descs, const double* taus, int n,
                                void* dev_ws, size_t ws_bytes, void* hip_stream,
                                hofks_ctx** out) {
  if (!out) return HOFKS_EINVAL;
  *out = nullptr;
  hofks_ctx* c = new (std::nothrow) hofks_ctx();
  if (!c) return HOFKS_EINVAL;
  Batch* B = new (std::nothrow) Batch();
  if (!B) {
    delete c;
    return HOFKS_EINVAL;
  }
  c->batch = B;
  hofks_status st = batch_plan(descs, taus, n, B, c->err);
  if (st) {
    delete B;
    delete c;
    return st;
  }
  if (!dev_ws || ws_bytes < B->total || ((uintptr_t)dev_ws & 255)) {
    delete B;
    delete c;
    return HOFKS_ESIZE;
  }
  c->desc = descs[0];
  c->stream = (hipStream_t)hip_stream;
  c->ws = (unsigned char*)dev_ws;
  B->gar = (float*)(c->ws + B->off_gar);
  B->rar = (float*)(c->ws + B->off_rar);
  B->dar = (double*)(c->ws + B->off_dar);
  B->vtar = (VelNode*)(c->ws + B->off_vt);
  B->tubes_d = (TubeDev*)(c->ws + B->off_tubes);
  B->eitems = (int4*)(c->ws + B->off_eitems);
  B->items = (int2*)(c->ws + B->off_items);
  B->uitems = (int2*)(c->ws + B->off_uitems);
  B->alpha = (double*)(c->ws + B->off_alpha);
  B->tube_s = (int*)(c->ws + B->off_s);
  B->tflag = (int*)(c->ws + B->off_tflag);
  B->flag = (int*)(c->ws + B->off_flag);
  B->ebar = (unsigned*)(c->ws + B->off_ebar);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&B->ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    B->ncu = 256;
  // the Euler tiles take more than the default 64 KB of LDS
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_euler),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024) !=
      hipSuccess) {
    delete B;
    delete c;
    return HOFKS_EDEVICE;
  }
  {
    constexpr unsigned evf = hipEventDisableTiming | hipEventDisableSystemFence;
    if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, evf) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, evf) != hipSuccess) {
      hofks_destroy(c);
      return HOFKS_EDEVICE;
    }
  }
  std::vector<VelNode> tab;
  tab.reserve(B->nvt);
  for (const TubeDev& T : B->tubes)
    for (int i = 0; i < T.nv1; ++i) {
      const double v = (i - T.kofs) * T.dv;
      tab.push_back(VelNode{v, v * v, (float)v, (float)(0.5 * v * v), 0.5 * v * v});
    }
  if (hipMemcpyAsync(B->vtar, tab.data(), sizeof(VelNode) * tab.size(), hipMemcpyHostToDevice,
                     c->stream) != hipSuccess ||
      hipMemcpyAsync(B->tubes_d, B->tubes.data(), sizeof(TubeDev) * B->n, hipMemcpyHostToDevice,
                     c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    hofks_destroy(c);
    return HOFKS_EDEVICE;
  }
  B->cells = 512;
  B->unr = unroll_for(B, 512);
  B->lds = lds_for(B, 512);
  *out = c;
  return HOFKS_OK;
}

hofks_status hofks_batch_tube_flags(hofks_ctx* c, int* flags) {
  if (!c || !c->batch || !flags) return HOFKS_EINVAL;
  HIPCHK(c, hipMemcpyAsync(flags, c->batch->tflag, sizeof(int) * c->batch->n,
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HOFKS_OK;
}

hofks_status hofks_set_launch_config(hofks_ctx* c, int wavefronts, int loads, int euler_before) {
  if (!c || c->batch || euler_before < 0 || euler_before > 1) return HOFKS_EINVAL;
  const Plan& P = c->P;
  const bool ok_w = c->kwide ? ((wavefronts == 2 || wavefronts == 4) && (loads == 4 || loads == 8) &&
                                kin2w_lds(P, wavefronts) <= 65536)
                             : ((wavefronts == 2 || wavefronts == 4 || (wavefronts == 8 && P.d >= 2)) &&
                                (loads == 8 || loads == 16) && kin_lds(P, wavefronts) <= 65536);
  if (!ok_w || (c->kring && wavefronts != RY))
    return fmt_err(c->err, "launch configuration not available for this grid"), HOFKS_EINVAL;
  c->kng = wavefronts;
  c->kunr = loads;
  c->euler_seq = euler_before != 0;
  return HOFKS_OK;
}

hofks_status hofks_batch_set_launch_config(hofks_ctx* c, int cells, int euler_part) {
  if (!c || !c->batch || !c->ready) return HOFKS_EINVAL;
  if ((cells != 256 && cells != 512 && cells != 1024) ||
      (euler_part != 0 && euler_part != 1024 && euler_part != 2048))
    return fmt_err(c->err, "launch configuration not available for a batch"), HOFKS_EINVAL;
  return batch_configure(c, cells, euler_part);
}

// Batch: pick the item width (cells per kinetic item), then the part size of
// the split Euler solves, by timing `steps` steps of each candidate on the
// current state (which is advanced).  With a cache file, a matching line is
// reused without timing; otherwise the result is appended.
hofks_status hofks_autotune(hofks_ctx* c, int steps, const char* cache_path, int* choice) {
  if (!c || !c->ready || steps < 1) return HOFKS_EINVAL;
  if (!c->batch) return grid_autotune(c, steps, cache_path, choice);
  Batch* B = c->batch;
  std::ostringstream key;
  key << "gfx950:batch2:n=" << B->n << ":cells=" << B->total_cells << ":cv=" << B->total_cv
      << ":ncu=" << B->ncu;
  int best_cells = 0, best_part = 0;
  if (cache_path && *cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      const std::string k = "\"key\": \"" + key.str() + "\"";
      if (line.find(k) == std::string::npos) continue;
      int cc = 0, pp = -1;
      const size_t pc = line.find("\"cells\": "), pe = line.find("\"euler_part\": ");
      if (pc != std::string::npos && pe != std::string::npos) {
        cc = std::atoi(line.c_str() + pc + 9);
        pp = std::atoi(line.c_str() + pe + 14);
      }
      if ((cc == 256 || cc == 512 || cc == 1024) && (pp == 0 || pp == 1024 || pp == 2048)) {
        best_cells = cc;
        best_part = pp;
      }
    }
  }
  if (!best_cells) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hofks_status st = HOFKS_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
      st = hip_fail(c, hipErrorOutOfMemory, "hipEventCreate");
    // times one candidate: a warm-up step, then `steps` steps
    auto time_cfg = [&](int cells, int part, float* ms) -> hofks_status {
      hofks_status r = batch_configure(c, cells, part);
      if (!r) r = batch_step(c, 1, false);
      if (r) return r;
      HIPCHK(c, hipEventRecord(e0, c->stream));
      r = batch_step(c, steps, false);
      if (r) return r;
      HIPCHK(c, hipEventRecord(e1, c->stream));
      HIPCHK(c, hipEventSynchronize(e1));
      HIPCHK(c, hipEventElapsedTime(ms, e0, e1));
      return HOFKS_OK;
    };
    // the state evolves while the candidates run, so every candidate is
    // timed in two rounds and keeps its better time
    const int ccand[3] = {256, 512, 1024}, pcand[3] = {0, 1024, 2048};
    float cms[3] = {1e30f, 1e30f, 1e30f}, pms[3] = {1e30f, 1e30f, 1e30f};
    float best_ms = 1e30f;
    for (int round = 0; round < 2 && !st; ++round)
      for (int k = 0; k < 3 && !st; ++k) {
        float ms = 0.0f;
        st = time_cfg(ccand[k], best_part, &ms);
        cms[k] = std::min(cms[k], ms);
      }
    for (int k = 0; k < 3; ++k)
      if (cms[k] < best_ms) {
        best_ms = cms[k];
        best_cells = ccand[k];
      }
    for (int round = 0; round < 2 && !st; ++round)
      for (int k = 0; k < 3 && !st; ++k) {
        float ms = 0.0f;
        st = time_cfg(best_cells, pcand[k], &ms);
        pms[k] = std::min(pms[k], ms);
      }
    best_ms = 1e30f;
    for (int k = 0; k < 3; ++k)
      if (pms[k] < best_ms) {
        best_ms = pms[k];
        best_part = pcand[k];
      }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) return st;
    if (cache_path && *cache_path) {
      std::ofstream o(cache_path, std::ios::app);
      o << "{\"key\": \"" << key.str() << "\", \"cells\": " << best_cells
        << ", \"euler_part\": " << best_part << ", \"ms_per_step\": " << best_ms / steps
        << "}\n";
    }
  }
  hofks_status st = batch_configure(c, best_cells, best_part);
  if (st) return st;
  if (choice) {
    choice[0] = best_cells;
    choice[1] = best_part;
    choice[2] = 0;
  }
  return batch_read_flag(c);
}

}  // extern "C"

namespace {

hofks_status batch_read_moments(hofks_ctx* c, double* U) {
  Batch* B = c->batch;
  const int p = (int)(c->steps & 1);
  long long o = 0;
  for (const TubeDev& T : B->tubes) {
    HIPCHK(c, hipMemcpyAsync(U + o, B->dar + T.U[p], sizeof(double) * 3 * T.Nx,
                             hipMemcpyDeviceToHost, c->stream));
    o += 3LL * T.Nx;
  }
  return batch_read_flag(c);
}

hofks_status batch_read_f(hofks_ctx* c, double* f, size_t bytes) {
  Batch* B = c->batch;
  if (bytes < sizeof(double) * (size_t)B->total_cv) return HOFKS_ESIZE;
  const int p = (int)(c->steps & 1);
  long long o = 0;
  for (const TubeDev& T : B->tubes) {
    const Geom G = host_tube_geom(T);
    // stage FP64 planes in the idle piece buffer of the tube (half its planes
    // fit at a time)
    double* stage = reinterpret_cast<double*>(B->gar + T.g[p ^ 1]);
    const int per = std::max(1, T.nv1 / 2);
    for (int k0 = 0; k0 < T.nv1; k0 += per) {
      const int nk = std::min(per, T.nv1 - k0);
      hipLaunchKernelGGL((k_materialize<1, float>), dim3(nblk((size_t)nk * T.Nx)), dim3(256), 0,
                         c->stream, (const float*)(B->gar + T.g[p]), B->dar + T.cf, stage, k0,
                         nk, G);
      HIPCHK(c, hipGetLastError());
      HIPCHK(c, hipMemcpyAsync(f + o + (long long)k0 * T.Nx, stage,
                               sizeof(double) * (size_t)nk * T.Nx, hipMemcpyDeviceToHost,
                               c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    o += (long long)T.nv1 * T.Nx;
  }
  return batch_read_flag(c);
}

// largest sub-step count of the last step over the tubes that are not flagged
hofks_status batch_max_substeps(hofks_ctx* c, int* out) {
  std::vector<int> ts(c->batch->n), tf(c->batch->n);
  HIPCHK(c, hipMemcpyAsync(ts.data(), c->batch->tube_s, sizeof(int) * ts.size(),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(tf.data(), c->batch->tflag, sizeof(int) * tf.size(),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int m = 0;
  for (size_t i = 0; i < ts.size(); ++i)
    if (!tf[i]) m = std::max(m, ts[i]);
  *out = m;
  return HOFKS_OK;
}

double batch_dt(const hofks_ctx* c) { return c->batch->tubes[0].dt; }

void batch_free(hofks_ctx* c) {
  Batch* B = c->batch;
  if (!B) return;
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  delete B;
  c->batch = nullptr;
}

}  // namespace

// ============================================================ closure ABI
extern "C" {

hofks_status hofks_closure_enable(hofks_ctx* c, const void* packed, double sigma,
                                  double threshold) {
  if (!c) return HOFKS_EINVAL;
  if (c->batch || c->P.d != 2)
    return fmt_err(c->err, "the closure form is defined for 2D-2V grids"), HOFKS_EINVAL;
  if (c->desc.scheme != 0) return fmt_err(c->err, "the closure form needs the HOFKS scheme"), HOFKS_EINVAL;
  if (c->P.G.offl) return fmt_err(c->err, "the closure form needs the lattice dt = dx/dv"), HOFKS_EINVAL;
  if (c->strang) return fmt_err(c->err, "the closure form needs first-order splitting"), HOFKS_EINVAL;
  if (!packed || ((uintptr_t)packed & 15))
    return fmt_err(c->err, "network weights: 16-byte aligned device pointer expected"), HOFKS_EINVAL;
  if (!std::isfinite(sigma) || std::isnan(threshold))
    return fmt_err(c->err, "sigma must be finite and the threshold a number"), HOFKS_EINVAL;
  c->clos_w = packed;
  c->clos_sigma = sigma;
  c->clos_thr = threshold;
  c->clos_on = true;
  c->clos_y0_ok = false;
  return HOFKS_OK;
}

hofks_status hofks_closure_set_weights(hofks_ctx* c, const void* packed, size_t bytes) {
  if (!c || !packed || ((uintptr_t)packed & 15)) return HOFKS_EINVAL;
  if (bytes != mlp::PACKED_BYTES) return HOFKS_ESIZE;
  c->clos_w = packed;
  c->clos_y0_ok = false;  // the output on the uniform stencil is evaluated again
  return HOFKS_OK;
}

hofks_status hofks_closure_disable(hofks_ctx* c) {
  if (!c) return HOFKS_EINVAL;
  c->clos_on = false;
  return HOFKS_OK;
}

hofks_status hofks_closure_snapshot(hofks_ctx* c, float* x, float* t) {
  if (!c || !x || !t) return HOFKS_EINVAL;
  if (c->batch || c->P.d != 2)
    return fmt_err(c->err, "the closure form is defined for 2D-2V grids"), HOFKS_EINVAL;
  if (!c->ready) return fmt_err(c->err, "set the state before stepping"), HOFKS_ESTATE;
  if (c->desc.scheme != 0) return fmt_err(c->err, "the closure form needs the HOFKS scheme"), HOFKS_EINVAL;
  if (c->P.G.offl) return fmt_err(c->err, "the closure form needs the lattice dt = dx/dv"), HOFKS_EINVAL;
  if (c->strang) return fmt_err(c->err, "the closure form needs first-order splitting"), HOFKS_EINVAL;
  if (!(c->P.G.lam >= 1e-12) || !(c->P.G.mu > 0.0))
    return fmt_err(c->err, "training targets need 1e-12 <= lambda < 1 (finite tau, not too small)"),
           HOFKS_EINVAL;
  if (((uintptr_t)x & 3) || ((uintptr_t)t & 3)) return HOFKS_EINVAL;
  hofks_status st = dispatch(c, [&](auto D, auto tt) -> hofks_status {
    if constexpr (decltype(D)::value == 2) {
      return launch_step<2, decltype(tt)>(c, x, t);
    }
    return HOFKS_EINVAL;
  });
  if (st) return st;
  c->cur ^= 1;
  c->steps++;
  return HOFKS_OK;
}

hofks_status hofks_closure_stats(hofks_ctx* c, long* closure_steps,
                                 unsigned long long* kinetic_cell_steps) {
  if (!c) return HOFKS_EINVAL;
  unsigned long long k = 0;
  if (c->kcount) {
    HIPCHK(c, hipMemcpyAsync(&k, c->kcount, sizeof(k), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  if (closure_steps) *closure_steps = c->clos_steps;
  if (kinetic_cell_steps) *kinetic_cell_steps = k;
  return HOFKS_OK;
}

int hofks_mlp_nparam(void) { return mlp::NPARAM; }

size_t hofks_mlp_packed_bytes(void) { return mlp::PACKED_BYTES; }

hofks_status hofks_mlp_pack(const float* params, void* packed, void* stream) {
  if (!params || !packed || ((uintptr_t)packed & 15)) return HOFKS_EINVAL;
  const int n = mlp::PACK_VALUES + mlp::NBIAS;
  hipLaunchKernelGGL(mlp::k_mlp_pack, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, params,
                     packed);
  return hipGetLastError() == hipSuccess ? HOFKS_OK : HOFKS_EDEVICE;
}

hofks_status hofks_mlp_forward(const void* packed, const float* x, float* y, long n,
                               void* stream) {
  if (!packed || ((uintptr_t)packed & 15) || n < 0) return HOFKS_EINVAL;
  if (n == 0) return HOFKS_OK;
  if (!x || !y || ((uintptr_t)y & 15) || ((uintptr_t)x & 3)) return HOFKS_EINVAL;
  const long tiles = (n + 15) / 16;
  const unsigned grid = (unsigned)std::min<long>(2048, (tiles + 3) / 4);
  hipLaunchKernelGGL(mlp::k_mlp_forward, dim3(grid), dim3(256), 0, (hipStream_t)stream, packed,
                     x, y, n);
  return hipGetLastError() == hipSuccess ? HOFKS_OK : HOFKS_EDEVICE;
}

size_t hofks_mlp_grad_work_bytes(long n) {
  return n < 1 ? 0 : (size_t)mlp::grad_blocks(n) * mlp::PART_STRIDE * sizeof(float);
}

namespace {
// deterministic gradient into grad/loss with the partials in `part`
hofks_status mlp_grad_launch(const void* packed, const float* x, const float* t, const int* idx,
                             long n, float* grad, float* loss, float* part, hipStream_t s) {
  const int nb = mlp::grad_blocks(n);
  hipLaunchKernelGGL(mlp::k_mlp_grad, dim3(nb), dim3(64 * mlp::GRAD_WAVES), mlp::GRAD_LDS, s,
                     packed, x, t, idx, n, part);
  hipLaunchKernelGGL(mlp::k_mlp_grad_reduce, dim3(nblk(mlp::NPARAM + 1)), dim3(256), 0, s,
                     (const float*)part, nb, grad, loss);
  return hipGetLastError() == hipSuccess ? HOFKS_OK : HOFKS_EDEVICE;
}

bool mlp_grad_args_ok(const void* packed, const float* x, const float* t, long n,
                      const float* grad, const float* loss) {
  return packed && !((uintptr_t)packed & 15) && grad && loss && n >= 1 && x && t;
}
}  // namespace

hofks_status hofks_mlp_grad(const void* packed, const float* x, const float* t, const int* idx,
                            long n, float* grad, float* loss, void* work, size_t work_bytes,
                            void* stream) {
  if (!mlp_grad_args_ok(packed, x, t, n, grad, loss) || !work || ((uintptr_t)work & 255))
    return HOFKS_EINVAL;
  if (work_bytes < hofks_mlp_grad_work_bytes(n)) return HOFKS_ESIZE;
  return mlp_grad_launch(packed, x, t, idx, n, grad, loss, (float*)work, (hipStream_t)stream);
}

}  // extern "C"

namespace {
// Scratch of hofks_mlp_grad_noalloc: the per-block partial gradients of the
// largest grid, in device memory the library holds for the life of the
// process (one copy on every GPU it runs on).  Host code never passes the
// array's name to a kernel: its device address on the current device is
// looked up once per device with hipGetSymbolAddress and kept here.
__device__ __align__(256) float scratch[mlp::GRAD_WORK_MAX / sizeof(float)];

constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_ptr[SCRATCH_DEVICES];

hofks_status scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_DEVICES) return HOFKS_EDEVICE;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HOFKS_EDEVICE;
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return HOFKS_OK;
}
}  // namespace

extern "C" {

hofks_status hofks_mlp_grad_noalloc(const void* packed, const float* x, const float* t,
                                    const int* idx, long n, float* grad, float* loss,
                                    void* stream) {
  if (!mlp_grad_args_ok(packed, x, t, n, grad, loss)) return HOFKS_EINVAL;
  if (hofks_mlp_grad_work_bytes(n) > sizeof(scratch)) return HOFKS_ESIZE;
  void* work = nullptr;
  const hofks_status st = scratch_address(&work);
  if (st) return st;
  return mlp_grad_launch(packed, x, t, idx, n, grad, loss, (float*)work, (hipStream_t)stream);
}

hofks_status hofks_stream_probe(int mode, const void* src, void* dst, size_t bytes,
                                void* stream) {
  if (mode < 0 || mode > 2 || bytes < 16 || (bytes & 15) || ((uintptr_t)src & 15) ||
      ((uintptr_t)dst & 15) || (mode != 1 && !src) || (mode != 0 && !dst) || (mode == 0 && !dst))
    return HOFKS_EINVAL;
  const size_t nvec = bytes / 16;
  int ncu = 256, dev = 0;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t per_block = (size_t)PROBE_TPB * PROBE_UNR;
  const unsigned grid =
      (unsigned)std::min<size_t>((size_t)ncu * 8, (nvec + per_block - 1) / per_block);
  hipStream_t s = (hipStream_t)stream;
  auto* in = (const pv4*)src;
  auto* out = (pv4*)dst;
  if (mode == 0)
    hipLaunchKernelGGL(k_stream_probe<0>, dim3(grid), dim3(PROBE_TPB), 0, s, in, out, nvec,
                       (unsigned*)dst);
  else if (mode == 1)
    hipLaunchKernelGGL(k_stream_probe<1>, dim3(grid), dim3(PROBE_TPB), 0, s, in, out, nvec,
                       nullptr);
  else
    hipLaunchKernelGGL(k_stream_probe<2>, dim3(grid), dim3(PROBE_TPB), 0, s, in, out, nvec,
                       nullptr);
  return hipGetLastError() == hipSuccess ? HOFKS_OK : HOFKS_EDEVICE;
}

size_t hofks_closure_prepare_work_bytes(long n) {
  if (n < 1) return 0;
  const size_t ntiles = (size_t)((n + train::SCAN_TILE - 1) / train::SCAN_TILE);
  return align256(sizeof(train::PrepState)) + align256(ntiles * sizeof(int));
}

hofks_status hofks_closure_prepare(const float* x, const float* t, long n, float clip,
                                   float* x_out, float* t_out, double* scales, int* kept,
                                   void* work, size_t work_bytes, void* stream) {
  if (!x || !t || n < 1 || !(clip > 0.0f) || !x_out || !t_out || !scales || !kept || !work ||
      ((uintptr_t)work & 255) || n > (1L << 30))
    return HOFKS_EINVAL;
  if (work_bytes < hofks_closure_prepare_work_bytes(n)) return HOFKS_ESIZE;
  hipStream_t s = (hipStream_t)stream;
  auto* st = (train::PrepState*)work;
  int* tiles = (int*)((unsigned char*)work + align256(sizeof(train::PrepState)));
  const unsigned ntiles = (unsigned)((n + train::SCAN_TILE - 1) / train::SCAN_TILE);
  const unsigned gh = (unsigned)std::min<long>(1024, (n + train::TB - 1) / train::TB);
  const int nbm = (int)std::min<long>(train::MOM_BLOCKS, (n + train::TB - 1) / train::TB);
  hipLaunchKernelGGL(train::k_prep_init, dim3(1), dim3(256), 0, s, st, n);
  for (int shift = 24; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(train::k_prep_hist, dim3(gh), dim3(train::TB), 0, s, t, n, st, shift);
    hipLaunchKernelGGL(train::k_prep_select, dim3(1), dim3(256), 0, s, st, shift);
  }
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(train::k_prep_moments, dim3(nbm), dim3(train::TB), 0, s, t, n, st, pass);
    hipLaunchKernelGGL(train::k_prep_moments_final, dim3(1), dim3(64), 0, s, st, nbm, pass);
  }
  hipLaunchKernelGGL(train::k_prep_count, dim3(ntiles), dim3(train::TB), 0, s, t, n,
                     (const train::PrepState*)st, clip, tiles);
  hipLaunchKernelGGL(train::k_prep_scan_tiles, dim3(1), dim3(64), 0, s, tiles, (int)ntiles, st);
  hipLaunchKernelGGL(train::k_prep_compact, dim3(ntiles), dim3(train::TB), 0, s, x, t, n,
                     (const train::PrepState*)st, clip, (const int*)tiles, x_out, t_out);
  hipLaunchKernelGGL(train::k_prep_export, dim3(1), dim3(64), 0, s, (const train::PrepState*)st,
                     scales, kept);
  return hipGetLastError() == hipSuccess ? HOFKS_OK : HOFKS_EDEVICE;
}

hofks_status hofks_mlp_fold_scales(float* params, const double* scales, void* stream) {
  if (!params || !scales) return HOFKS_EINVAL;
  hipLaunchKernelGGL(train::k_fold_scales, dim3(1), dim3(256), 0, (hipStream_t)stream, params,
                     scales);
  return hipGetLastError() == hipSuccess ? HOFKS_OK : HOFKS_EDEVICE;
}

hofks_status hofks_closure_train_step(float* params, float* m, float* v, void* packed,
                                      const float* x, const float* t, const int* idx, long n,
                                      float lr, float beta1, float beta2, float eps, int step,
                                      float* grad, float* loss, void* work, size_t work_bytes,
                                      void* stream) {
  if (!params || !m || !v || step < 1 || !mlp_grad_args_ok(packed, x, t, n, grad, loss) ||
      !work || ((uintptr_t)work & 255))
    return HOFKS_EINVAL;
  if (work_bytes < hofks_mlp_grad_work_bytes(n)) return HOFKS_ESIZE;
  hipStream_t s = (hipStream_t)stream;
  hofks_status st = mlp_grad_launch(packed, x, t, idx, n, grad, loss, (float*)work, s);
  if (st) return st;
  st = hofks_mlp_adam(params, grad, m, v, lr, beta1, beta2, eps, step, stream);
  if (st) return st;
  return hofks_mlp_pack(params, packed, stream);
}

hofks_status hofks_mlp_adam(float* params, const float* grad, float* m, float* v, float lr,
                            float b1, float b2, float eps, int step, void* stream) {
  if (!params || !grad || !m || !v || step < 1) return HOFKS_EINVAL;
  const float c1 = (float)(1.0 - std::pow((double)b1, step));
  const float c2 = (float)(1.0 - std::pow((double)b2, step));
  hipLaunchKernelGGL(mlp::k_mlp_adam, dim3(nblk(mlp::NPARAM)), dim3(256), 0, (hipStream_t)stream,
                     params, grad, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? HOFKS_OK : HOFKS_EDEVICE;
}

}  // extern "C"

extern "C" void hofks_destroy(hofks_ctx* c) {
  if (!c) return;
  batch_free(c);
  if (c->aux) (void)hipStreamSynchronize(c->aux);  // a read-back may be in flight
  if (c->ev_peek) (void)hipEventDestroy(c->ev_peek);
  if (c->peek_h) (void)hipHostFree(c->peek_h);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->aux) {
    (void)hipStreamSynchronize(c->aux);
    (void)hipStreamDestroy(c->aux);
  }
  delete c;
}
