// train.hpp -- preparation of the closure network's training data on the
// GPU.  Not part of the paper: the learned closure predicts the
// non-equilibrium term of eq. (UK) in near-equilibrium cells, and its four
// targets differ in scale by orders of magnitude, so each is divided by a
// robust scale before training and the scales are folded into the output
// layer afterwards.
//
// Robust scale of output c (n samples): q_c = the k-th smallest |t_c| with
// k = ceil(995 n / 1000) (found by a four-pass radix selection on the FP32
// bit patterns, which order like the values for |t| >= 0), then the sample
// standard deviation (n - 1 divisor) of the t_c with |t_c| <= q_c, at least
// 1e-12.  Samples whose normalised targets all lie within +-clip are kept,
// in their original order (a block scan of the keep flags).  Every sum runs
// in a fixed order (per-block FP64 partials, then the partials in block
// order), so the result does not depend on scheduling.
#pragma once
#include <hip/hip_runtime.h>

#include "mlp.hpp"

namespace hofks {
namespace train {

constexpr int NOUT = mlp::NOUT, NIN = mlp::NIN;
constexpr int TB = 256;             // threads per block
constexpr int MOM_BLOCKS = 512;     // blocks of the moment passes
constexpr int SCAN_ITEMS = 4;       // keep flags per thread in the scan
constexpr int SCAN_TILE = TB * SCAN_ITEMS;

// state of the selection and the statistics, in the work area
struct PrepState {
  unsigned prefix[NOUT];    // selected high bits so far
  unsigned krem[NOUT];      // rank still to find among the matching keys (1-based)
  unsigned hist[NOUT][256];
  double q[NOUT];           // k-th smallest |t_c|
  double count[NOUT];       // samples with |t_c| <= q_c
  double mean[NOUT];
  double scale[NOUT];
  double part[MOM_BLOCKS][NOUT][2];  // per-block (count, sum) or (sum of squares)
  int kept;
};

__device__ __forceinline__ unsigned key_of(float v) { return __float_as_uint(fabsf(v)); }

__global__ void k_prep_init(PrepState* st, long n) {
  const int i = threadIdx.x;
  if (i < NOUT) {
    st->prefix[i] = 0u;
    st->krem[i] = (unsigned)((995 * n + 999) / 1000);
  }
  for (int b = i; b < NOUT * 256; b += blockDim.x) (&st->hist[0][0])[b] = 0u;
  if (i == 0) st->kept = 0;
}

// histogram of the 8-bit digit at `shift` of the keys whose higher bits equal
// the selected prefix
__global__ __launch_bounds__(TB) void k_prep_hist(const float* __restrict__ t, long n,
                                                  PrepState* st, int shift) {
  __shared__ unsigned h[NOUT][256];
  for (int b = threadIdx.x; b < NOUT * 256; b += TB) (&h[0][0])[b] = 0u;
  __syncthreads();
  unsigned pre[NOUT];
#pragma unroll
  for (int c = 0; c < NOUT; ++c) pre[c] = st->prefix[c];
  for (long i = (long)blockIdx.x * TB + threadIdx.x; i < n; i += (long)gridDim.x * TB) {
#pragma unroll
    for (int c = 0; c < NOUT; ++c) {
      const unsigned k = key_of(t[i * NOUT + c]);
      const bool match = shift == 24 || (k >> (shift + 8)) == pre[c];
      if (match) atomicAdd(&h[c][(k >> shift) & 255u], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < NOUT * 256; b += TB) {
    const unsigned v = (&h[0][0])[b];
    if (v) atomicAdd(&st->hist[0][0] + b, v);
  }
}

// pick the digit holding rank krem, extend the prefix, clear the histogram
__global__ void k_prep_select(PrepState* st, int shift) {
  const int c = threadIdx.x;
  if (c < NOUT) {
    unsigned acc = 0, k = st->krem[c];
    int d = 0;
    for (; d < 255; ++d) {
      const unsigned h = st->hist[c][d];
      if (acc + h >= k) break;
      acc += h;
    }
    st->krem[c] = k - acc;
    st->prefix[c] = (st->prefix[c] << 8) | (unsigned)d;
    if (shift == 0) st->q[c] = (double)__uint_as_float(st->prefix[c]);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < NOUT * 256; b += blockDim.x) (&st->hist[0][0])[b] = 0u;
}

// block sum in a fixed order (wavefront shuffles, then the wavefronts)
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < TB / 64; ++w) s += red[w];
  return s;
}

// pass 0: count and sum of the t_c with |t_c| <= q_c; pass 1: sum of squared
// deviations from the mean.  One partial per block.
__global__ __launch_bounds__(TB) void k_prep_moments(const float* __restrict__ t, long n,
                                                     PrepState* st, int pass) {
  __shared__ double red[TB / 64];
  double a[NOUT], b[NOUT], q[NOUT], mean[NOUT];
#pragma unroll
  for (int c = 0; c < NOUT; ++c) {
    a[c] = b[c] = 0.0;
    q[c] = st->q[c];
    mean[c] = pass ? st->mean[c] : 0.0;
  }
  for (long i = (long)blockIdx.x * TB + threadIdx.x; i < n; i += (long)gridDim.x * TB) {
#pragma unroll
    for (int c = 0; c < NOUT; ++c) {
      const double v = (double)t[i * NOUT + c];
      if (fabs(v) <= q[c]) {
        if (pass == 0) {
          a[c] += 1.0;
          b[c] += v;
        } else {
          a[c] += (v - mean[c]) * (v - mean[c]);
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NOUT; ++c) {
    const double sa = block_sum(a[c], red);
    const double sb = pass == 0 ? block_sum(b[c], red) : 0.0;
    if (threadIdx.x == 0) {
      st->part[blockIdx.x][c][0] = sa;
      st->part[blockIdx.x][c][1] = sb;
    }
  }
}

// partials in block order: the mean (pass 0), the scale (pass 1)
__global__ void k_prep_moments_final(PrepState* st, int nblocks, int pass) {
  const int c = threadIdx.x;
  if (c >= NOUT) return;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < nblocks; ++k) {
    a += st->part[k][c][0];
    b += st->part[k][c][1];
  }
  if (pass == 0) {
    st->count[c] = a;
    st->mean[c] = a > 0.0 ? b / a : 0.0;
  } else {
    const double m = st->count[c];
    const double sd = m > 1.0 ? sqrt(a / (m - 1.0)) : 0.0;
    st->scale[c] = sd > 1e-12 ? sd : 1e-12;
  }
}

__device__ __forceinline__ bool keep_sample(const float* __restrict__ t, long i, const float* sc,
                                            float clip) {
  bool k = true;
#pragma unroll
  for (int c = 0; c < NOUT; ++c) k &= fabsf(t[i * NOUT + c] / sc[c]) <= clip;
  return k;
}

// per-tile counts of kept samples
__global__ __launch_bounds__(TB) void k_prep_count(const float* __restrict__ t, long n,
                                                   const PrepState* st, float clip,
                                                   int* __restrict__ tile_count) {
  float sc[NOUT];
#pragma unroll
  for (int c = 0; c < NOUT; ++c) sc[c] = (float)st->scale[c];
  int cnt = 0;
  const long base = (long)blockIdx.x * SCAN_TILE + (long)threadIdx.x * SCAN_ITEMS;
#pragma unroll
  for (int e = 0; e < SCAN_ITEMS; ++e)
    if (base + e < n && keep_sample(t, base + e, sc, clip)) ++cnt;
  __shared__ int red[TB / 64];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) tile_count[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// exclusive scan of the tile counts (one block, sequential chunks)
__global__ void k_prep_scan_tiles(int* __restrict__ tile_count, int ntiles, PrepState* st) {
  if (threadIdx.x != 0) return;
  int acc = 0;
  for (int i = 0; i < ntiles; ++i) {
    const int c = tile_count[i];
    tile_count[i] = acc;
    acc += c;
  }
  st->kept = acc;
}

// write the kept samples in order: x rows copied, targets divided by the scales
__global__ __launch_bounds__(TB) void k_prep_compact(const float* __restrict__ x,
                                                     const float* __restrict__ t, long n,
                                                     const PrepState* st, float clip,
                                                     const int* __restrict__ tile_off,
                                                     float* __restrict__ xo,
                                                     float* __restrict__ to) {
  float sc[NOUT];
#pragma unroll
  for (int c = 0; c < NOUT; ++c) sc[c] = (float)st->scale[c];
  const long base = (long)blockIdx.x * SCAN_TILE + (long)threadIdx.x * SCAN_ITEMS;
  bool kp[SCAN_ITEMS];
  int cnt = 0;
#pragma unroll
  for (int e = 0; e < SCAN_ITEMS; ++e) {
    kp[e] = base + e < n && keep_sample(t, base + e, sc, clip);
    cnt += kp[e];
  }
  // exclusive scan of cnt over the block's threads (in thread order)
  __shared__ int sc_w[TB / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) sc_w[w] = incl;
  __syncthreads();
  int woff = 0;
  for (int k = 0; k < w; ++k) woff += sc_w[k];
  int pos = tile_off[blockIdx.x] + woff + incl - cnt;
#pragma unroll
  for (int e = 0; e < SCAN_ITEMS; ++e) {
    if (!kp[e]) continue;
    const long i = base + e;
    for (int q = 0; q < NIN; ++q) xo[(size_t)pos * NIN + q] = x[i * NIN + q];
#pragma unroll
    for (int c = 0; c < NOUT; ++c) to[(size_t)pos * NOUT + c] = t[i * NOUT + c] / sc[c];
    ++pos;
  }
}

__global__ void k_prep_export(const PrepState* st, double* __restrict__ scales,
                              int* __restrict__ kept) {
  const int c = threadIdx.x;
  if (c < NOUT) scales[c] = st->scale[c];
  if (c == 0 && kept) *kept = st->kept;
}

// output layer times the scales: W4 row c and b4[c] multiplied by s_c
__global__ void k_fold_scales(float* __restrict__ p, const double* __restrict__ scales) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NOUT * mlp::NH) p[mlp::OW4 + i] *= (float)scales[i / mlp::NH];
  if (i < NOUT) p[mlp::OB4 + i] *= (float)scales[i];
}

}  // namespace train
}  // namespace hofks
