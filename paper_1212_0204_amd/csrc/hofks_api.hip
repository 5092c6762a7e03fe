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
#include <new>
#include <type_traits>
#include <utility>
#include <vector>

#include "hofks.h"
#include "kernels.hpp"

using namespace hofks;

namespace {

struct Plan {
  int d, nm, R;
  Geom G;
  Mat A;
  int prec;
  size_t tsize;  // bytes per stored piece
  int TX, TR, nseg, nrowgrp, nchunk, nvr;
  size_t lds;
  // workspace offsets (bytes)
  size_t off_g[2], off_U, off_UE[2], off_rec, off_recT, off_cf, off_part, off_slots, off_flag;
  size_t total;
};

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
  if (desc->scheme < 0 || desc->scheme > 2)
    return fmt_err(err, "scheme must be 0, 1 or 2"), HOFKS_EINVAL;
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
  G.w = std::pow(desc->dv, d);
  G.lam = 1.0;
  G.mu = 0.0;
  G.gam = (d + 2.0) / d;
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

  // kinetic tiling: TX consecutive cells along x (a multiple of the 64-wide
  // wavefront), TR rows per 256-thread block, velocity rows split in chunks
  // so that the grid holds ~8 blocks per compute unit
  const int Nx = G.n[0];
  P->TX = Nx >= 192 ? 256 : (Nx > 64 ? 128 : 64);
  P->TR = 256 / P->TX;
  P->nseg = (Nx + P->TX - 1) / P->TX;
  const int nrows = G.n[1] * G.n[2];
  P->nrowgrp = (nrows + P->TR - 1) / P->TR;
  P->nvr = G.nv / G.nv1;
  const long base = (long)P->nseg * P->nrowgrp;
  long nch = (2048 + base - 1) / base;
  P->nchunk = (int)std::max(1L, std::min<long>(nch, P->nvr));
  P->lds = (size_t)P->TR * P->R * (P->TX + G.nv1 - 1) * P->tsize;
  if (P->lds > 65536) return fmt_err(err, "velocity grid too wide for the LDS tile"), HOFKS_EINVAL;

  size_t off = 0;
  const size_t gbytes = (size_t)G.nv * G.nc * P->tsize;
  const size_t ubytes = (size_t)nm * G.nc * sizeof(double);
  P->off_g[0] = off;
  off = align256(off + gbytes);
  P->off_g[1] = off;
  off = align256(off + gbytes);
  P->off_U = off;
  off = align256(off + ubytes);
  P->off_UE[0] = off;
  off = align256(off + ubytes);
  P->off_UE[1] = off;
  off = align256(off + ubytes);
  P->off_rec = off;
  off = align256(off + (size_t)P->R * G.nc * sizeof(double));
  P->off_recT = off;
  if (P->prec) off = align256(off + (size_t)P->R * G.nc * sizeof(float));
  P->off_cf = off;
  off = align256(off + ubytes);
  P->off_part = off;
  off = align256(off + (size_t)P->nchunk * 2 * nm * G.nc * sizeof(double));
  P->off_slots = off;
  off = align256(off + 2 * (SMAX + 1) * SLOT_STRIDE * sizeof(double));
  P->off_flag = off;
  off = align256(off + 64);
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
  int cur;
  double *U, *UE[2], *rec, *cf, *part, *slots;
  void* recT;
  int* flag;
  double tau;
  int s_cap;
  long steps;
  bool ready;
  // optional per-kernel timing: hipEvents around each launch group
  bool timing;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_marks;  // (group, start, stop)
  size_t ev_next;
  char err[512];
};

namespace {

hofks_status hip_fail(hofks_ctx* c, hipError_t e, const char* what) {
  fmt_err(c->err, "%s: %s", what, hipGetErrorString(e));
  return HOFKS_EDEVICE;
}

#define HIPCHK(c, call)                                   \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return hip_fail((c), e_, #call); \
  } while (0)

unsigned nblk(size_t n, unsigned b = 256) { return (unsigned)((n + b - 1) / b); }

double* slot_set(hofks_ctx* c, int set) {
  return c->slots + (size_t)set * (SMAX + 1) * SLOT_STRIDE;
}

// timing groups: 0 Euler sub-steps, 1 kinetic, 2 cell update
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
  int group;
  hipEvent_t a = nullptr;
  Mark(hofks_ctx* c_, int g) : c(c_), group(g) {
    if (c->timing) {
      a = next_event(c);
      if (a) (void)hipEventRecord(a, c->stream);
    }
  }
  ~Mark() {
    if (c->timing && a) {
      hipEvent_t b = next_event(c);
      if (b) {
        (void)hipEventRecord(b, c->stream);
        c->ev_marks.push_back({group, {a, b}});
      }
    }
  }
};

// ---------------------------------------------------------------- launchers
template <int D, typename T>
hofks_status launch_cell_update(hofks_ctx* c, int mode, int set, int aset) {
  const Plan& P = c->P;
  hipLaunchKernelGGL((k_cell_update<D, T>), dim3(nblk(P.G.nc)), dim3(256), 0, c->stream, c->U,
                     c->cf, c->rec, (T*)(P.prec ? c->recT : nullptr), c->part, P.nchunk, c->UE[0],
                     c->UE[1], c->slots, set, aset, c->s_cap, c->flag, P.G, P.A, mode,
                     (int)(c->desc.scheme == 1));
  HIPCHK(c, hipGetLastError());
  return HOFKS_OK;
}

template <int D, typename T>
hofks_status launch_kinetic(hofks_ctx* c, int set) {
  const Plan& P = c->P;
  const T* gin = (const T*)c->g[c->cur];
  T* gout = (T*)c->g[c->cur ^ 1];
  const T* rec = P.prec ? (const T*)c->recT : (const T*)c->rec;
  const dim3 grid((unsigned)((long)P.nseg * P.nrowgrp * P.nchunk));
  const bool ft = (P.G.mu == 0.0);
  const bool comp = (P.prec == 1);
  double* zs = slot_set(c, set ^ 1);
#define KLAUNCH(FT, CP)                                                                       \
  hipLaunchKernelGGL((k_kinetic<D, T, FT, CP>), grid, dim3(256), P.lds, c->stream, gin, gout, \
                     rec, c->part, zs, P.G, P.TX, P.TR, P.nseg, P.nrowgrp, P.nchunk, P.nvr)
  if (ft) {
    if (comp) KLAUNCH(true, true); else KLAUNCH(true, false);
  } else {
    if (comp) KLAUNCH(false, true); else KLAUNCH(false, false);
  }
#undef KLAUNCH
  HIPCHK(c, hipGetLastError());
  return HOFKS_OK;
}

template <int D, typename T>
hofks_status step_impl(hofks_ctx* c, int nsteps) {
  const Plan& P = c->P;
  const bool need_euler = (P.G.mu != 0.0) && (c->desc.scheme != 1);
  for (int it = 0; it < nsteps; ++it) {
    const int set = (int)(c->steps & 1);
    if (need_euler) {
      Mark m(c, 0);
      for (int i = 0; i < c->s_cap; ++i) {
        hipLaunchKernelGGL((k_muscl<D>), dim3(nblk(P.G.nc)), dim3(256), 0, c->stream, c->U,
                           c->UE[0], c->UE[1], c->slots, set, i, c->s_cap, c->flag, P.G,
                           (int)(c->desc.scheme == 2));
      }
      HIPCHK(c, hipGetLastError());
    }
    hofks_status st;
    {
      Mark m(c, 1);
      st = launch_kinetic<D, T>(c, set);
    }
    if (st) return st;
    {
      Mark m(c, 2);
      st = launch_cell_update<D, T>(c, MODE_STEP, set, set ^ 1);
    }
    if (st) return st;
    c->cur ^= 1;
    c->steps++;
  }
  return HOFKS_OK;
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

hofks_status read_flag(hofks_ctx* c) {
  int h[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(h, c->flag, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
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

// after the records and the speeds of slot set `set` row 0 are final: size
// the number of sub-step launches per step
hofks_status plan_substeps(hofks_ctx* c, int set) {
  double a[SLOT_STRIDE];
  HIPCHK(c, hipMemcpyAsync(a, slot_set(c, set), sizeof(a), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double sum = 0.0;
  for (int k = 0; k < c->P.d; ++k) sum += a[k];
  double sv = std::ceil(2.0 * c->P.G.dt * sum / c->P.G.dx);
  int s0 = (sv >= 1.0 && sv < SMAX) ? (int)sv : (sv >= SMAX ? SMAX : 1);
  c->s_cap = std::min(SMAX, std::max(2 * s0, s0 + 8));
  return HOFKS_OK;
}

// records of the current U and cf with the current lambda (after set_tau)
hofks_status refresh(hofks_ctx* c) {
  const int set = (int)(c->steps & 1);
  hofks_status st = zero_doubles(c, slot_set(c, set), SLOT_STRIDE);
  if (st) return st;
  st = dispatch(c, [&](auto D, auto t) {
    return launch_cell_update<decltype(D)::value, decltype(t)>(c, MODE_REFRESH, set, set);
  });
  if (st) return st;
  return plan_substeps(c, set);
}

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
  c->stream = (hipStream_t)hip_stream;
  c->ws = (unsigned char*)dev_ws;
  const Plan& P = c->P;
  c->g[0] = c->ws + P.off_g[0];
  c->g[1] = c->ws + P.off_g[1];
  c->cur = 0;
  c->U = (double*)(c->ws + P.off_U);
  c->UE[0] = (double*)(c->ws + P.off_UE[0]);
  c->UE[1] = (double*)(c->ws + P.off_UE[1]);
  c->rec = (double*)(c->ws + P.off_rec);
  c->recT = P.prec ? (void*)(c->ws + P.off_recT) : nullptr;
  c->cf = (double*)(c->ws + P.off_cf);
  c->part = (double*)(c->ws + P.off_part);
  c->slots = (double*)(c->ws + P.off_slots);
  c->flag = (int*)(c->ws + P.off_flag);
  c->tau = INFINITY;
  c->s_cap = 1;
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, c->stream, c->flag, 16);
  if (hipGetLastError() != hipSuccess) {
    delete c;
    return HOFKS_EDEVICE;
  }
  *out = c;
  return HOFKS_OK;
}

hofks_status hofks_set_tau(hofks_ctx* c, double tau) {
  if (!c) return HOFKS_EINVAL;
  if (!(tau >= 0.0)) return fmt_err(c->err, "tau must be >= 0 or +inf"), HOFKS_EINVAL;
  c->tau = tau;
  Geom& G = c->P.G;
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
  if (c->ready) return refresh(c);
  return HOFKS_OK;
}

hofks_status hofks_set_state_macro(hofks_ctx* c, const double* rho, const double* u,
                                   const double* theta) {
  if (!c || !rho || !theta || !u) return HOFKS_EINVAL;
  const Plan& P = c->P;
  const size_t nc = P.G.nc;
  double* prim = c->UE[0];  // (d+2) x nc staging: rho | u | theta
  HIPCHK(c, hipMemcpyAsync(prim, rho, nc * 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(prim + nc, u, nc * 8 * P.d, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(prim + nc * (P.d + 1), theta, nc * 8, hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, c->stream, c->flag, 16);
  hofks_status st = zero_doubles(c, c->slots, 2 * (SMAX + 1) * SLOT_STRIDE);
  if (st) return st;
  st = zero_doubles(c, c->cf, (size_t)P.nm * nc);
  if (st) return st;
  c->cur = 0;
  c->steps = 0;
  st = dispatch(c, [&](auto D, auto t) -> hofks_status {
    constexpr int DD = decltype(D)::value;
    using T = decltype(t);
    hipLaunchKernelGGL((k_prim_to_moments<DD>), dim3(nblk(nc)), dim3(256), 0, c->stream, prim,
                       c->U, (int)nc);
    // Maxwellian parameters of U^0, then sample M into the pieces, sum the
    // stored pieces and project onto U^0 (f^0 = E[U^0], section 4.2)
    hofks_status s2 = launch_cell_update<DD, T>(c, MODE_REFRESH, 0, 0);
    if (s2) return s2;
    const size_t tot = (size_t)P.G.nv * nc;
    hipLaunchKernelGGL((k_fill_maxwellian<DD, T>), dim3(nblk(tot)), dim3(256), 0, c->stream,
                       (T*)c->g[0], c->rec, P.G);
    hipLaunchKernelGGL((k_piece_sums<DD, T>), dim3(nblk(nc)), dim3(256), 0, c->stream,
                       (const T*)c->g[0], c->part, P.G);
    HIPCHK(c, hipGetLastError());
    return HOFKS_OK;
  });
  if (st) return st;
  st = zero_doubles(c, c->slots, 2 * (SMAX + 1) * SLOT_STRIDE);
  if (st) return st;
  st = dispatch(c, [&](auto D, auto t) {
    return launch_cell_update<decltype(D)::value, decltype(t)>(c, MODE_INIT, 0, 0);
  });
  if (st) return st;
  c->ready = true;
  st = plan_substeps(c, 0);
  if (st) return st;
  return read_flag(c);
}

hofks_status hofks_set_state_f(hofks_ctx* c, const double* f, size_t bytes) {
  if (!c || !f) return HOFKS_EINVAL;
  const Plan& P = c->P;
  const size_t nc = P.G.nc, tot = (size_t)P.G.nv * nc;
  if (bytes < tot * 8) return HOFKS_ESIZE;
  // stage FP64 planes through the idle piece buffer, store in piece precision
  const size_t per = std::max<size_t>(1, (tot * P.tsize) / (nc * 8));
  double* stage = (double*)c->g[1];
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, c->stream, c->flag, 16);
  c->cur = 0;
  c->steps = 0;
  for (size_t k0 = 0; k0 < (size_t)P.G.nv; k0 += per) {
    const size_t nk = std::min(per, (size_t)P.G.nv - k0);
    HIPCHK(c, hipMemcpyAsync(stage, f + k0 * nc, nk * nc * 8, hipMemcpyHostToDevice, c->stream));
    hofks_status st = dispatch(c, [&](auto, auto t) -> hofks_status {
      using T = decltype(t);
      hipLaunchKernelGGL((k_store_planes<T>), dim3(nblk(nk * nc)), dim3(256), 0, c->stream,
                         (T*)c->g[0] + k0 * nc, stage, nk * nc);
      HIPCHK(c, hipGetLastError());
      return HOFKS_OK;
    });
    if (st) return st;
  }
  hofks_status st = zero_doubles(c, c->slots, 2 * (SMAX + 1) * SLOT_STRIDE);
  if (st) return st;
  st = dispatch(c, [&](auto D, auto t) -> hofks_status {
    constexpr int DD = decltype(D)::value;
    using T = decltype(t);
    hipLaunchKernelGGL((k_piece_sums<DD, T>), dim3(nblk(nc)), dim3(256), 0, c->stream,
                       (const T*)c->g[0], c->part, P.G);
    HIPCHK(c, hipGetLastError());
    return launch_cell_update<DD, T>(c, MODE_INIT_FROM_SUMS, 0, 0);
  });
  if (st) return st;
  c->ready = true;
  st = plan_substeps(c, 0);
  if (st) return st;
  return read_flag(c);
}

hofks_status hofks_step(hofks_ctx* c, int n) {
  if (!c || n < 0) return HOFKS_EINVAL;
  if (!c->ready) return fmt_err(c->err, "set the state before stepping"), HOFKS_ESTATE;
  return dispatch(c, [&](auto D, auto t) {
    return step_impl<decltype(D)::value, decltype(t)>(c, n);
  });
}

hofks_status hofks_sync(hofks_ctx* c) {
  if (!c) return HOFKS_EINVAL;
  return read_flag(c);
}

hofks_status hofks_read_moments(hofks_ctx* c, double* U) {
  if (!c || !U) return HOFKS_EINVAL;
  HIPCHK(c, hipMemcpyAsync(U, c->U, (size_t)c->P.nm * c->P.G.nc * 8, hipMemcpyDeviceToHost,
                           c->stream));
  return read_flag(c);
}

hofks_status hofks_read_f(hofks_ctx* c, double* f, size_t bytes) {
  if (!c || !f) return HOFKS_EINVAL;
  const Plan& P = c->P;
  const size_t nc = P.G.nc, tot = (size_t)P.G.nv * nc;
  if (bytes < tot * 8) return HOFKS_ESIZE;
  const size_t per = std::max<size_t>(1, (tot * P.tsize) / (nc * 8));
  double* stage = (double*)c->g[c->cur ^ 1];
  for (size_t k0 = 0; k0 < (size_t)P.G.nv; k0 += per) {
    const size_t nk = std::min(per, (size_t)P.G.nv - k0);
    hofks_status st = dispatch(c, [&](auto D, auto t) -> hofks_status {
      constexpr int DD = decltype(D)::value;
      using T = decltype(t);
      hipLaunchKernelGGL((k_materialize<DD, T>), dim3(nblk(nk * nc)), dim3(256), 0, c->stream,
                         (const T*)c->g[c->cur], c->cf, stage, (int)k0, (int)nk, P.G);
      HIPCHK(c, hipGetLastError());
      return HOFKS_OK;
    });
    if (st) return st;
    HIPCHK(c, hipMemcpyAsync(f + k0 * nc, stage, nk * nc * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return read_flag(c);
}

hofks_status hofks_read_counters(hofks_ctx* c, int* substeps, long* steps) {
  if (!c) return HOFKS_EINVAL;
  int h[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(h, c->flag, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (substeps) *substeps = h[1];
  if (steps) *steps = c->steps;
  return HOFKS_OK;
}

hofks_status hofks_kernel_timing(hofks_ctx* c, int enable, double* ms, int* launches) {
  if (!c) return HOFKS_EINVAL;
  if (ms || launches) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double acc[3] = {0.0, 0.0, 0.0};
    int cnt[3] = {0, 0, 0};
    for (auto& m : c->ev_marks) {
      float t = 0.0f;
      HIPCHK(c, hipEventElapsedTime(&t, m.second.first, m.second.second));
      acc[m.first] += t;
      cnt[m.first] += 1;
    }
    for (int g = 0; g < 3; ++g) {
      if (ms) ms[g] = acc[g];
      if (launches) launches[g] = cnt[g];
    }
  }
  c->ev_marks.clear();
  c->ev_next = 0;
  c->timing = enable != 0;
  return HOFKS_OK;
}

double hofks_dt(const hofks_ctx* c) { return c ? c->P.G.dt : 0.0; }

const char* hofks_last_error(const hofks_ctx* c) { return c ? c->err : "null context"; }

void hofks_destroy(hofks_ctx* c) {
  if (!c) return;
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"
