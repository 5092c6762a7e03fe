// Closure network on the matrix cores: a multilayer perceptron 37 -> 64 ->
// 64 -> 64 -> 4 (tanh hidden layers, linear output) with BF16 weights and
// activations and FP32 accumulation, evaluated on the matrix cores: the
// forward pass with gfx950's v_mfma_f32_16x16x32_bf16, the backward products
// with v_mfma_f32_16x16x16_bf16.  The network is not part of the
// paper; it is the learned closure of the near-equilibrium cells (the
// non-equilibrium part of the moment update, eq. (UK)).
//
// One wavefront carries 16 samples through the whole network.  A layer is
// out^T = W a^T: the rows of an MFMA tile are output neurons, its columns
// samples, and the K dimension runs over input neurons.  The accumulator of
// a tile (lane j + 16q holds rows 4q..4q+3 of column j) is half of the B
// operand of the next layer's 32-deep K step: step s takes the accumulators
// of tiles 2s and 2s+1 of the same lane (its K order is neuron
// 16 (2s + e/4) + 4q + e%4 for element e of lane quarter q, and the weight
// fragments are packed in that order), so activations never leave registers.
//
// Flat FP32 parameter layout (shared with the host and the trainer):
//   W1[64][37] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[4][64] b4[4]
// Packed BF16 layout (what the kernels read): 26 forward fragments of 64
// lanes x 8 values -- W1 (4 output tiles x 2 K steps of 32 inputs), W2 and
// W3 (4 x 2), W4 (1 x 2) -- then 36 transposed fragments of 64 lanes x 4
// values for the backward pass -- W2, W3 (4 x 4), W4 (4 x 1) -- followed by
// the biases in FP32 (b1, b2, b3, b4 padded to 16).
#pragma once
#include <hip/hip_runtime.h>

namespace hofks {
namespace mlp {

constexpr int NIN = 37, NH = 64, NOUT = 4;
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH;
constexpr int OW3 = OB2 + NH, OB3 = OW3 + NH * NH, OW4 = OB3 + NH, OB4 = OW4 + NOUT * NH;
constexpr int NPARAM = OB4 + NOUT;  // 11012
constexpr int F_L1 = 0, F_L2 = 8, F_L3 = 16, F_L4 = 24, NFWD = 26;  // forward (K = 32)
constexpr int F_T2 = 0, F_T3 = 16, F_T4 = 32, NTR = 36;            // transposed (K = 16)
constexpr int NBIAS = 3 * NH + 16;
constexpr size_t FWD_BYTES = (size_t)NFWD * 64 * 16;
constexpr size_t FRAG_BYTES = FWD_BYTES + (size_t)NTR * 64 * 8;
constexpr size_t PACKED_BYTES = FRAG_BYTES + NBIAS * sizeof(float);
constexpr int PACK_VALUES = NFWD * 64 * 8 + NTR * 64 * 4;  // BF16 values before the biases

typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (inputs are finite here)
__device__ __forceinline__ short to_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ s4 pack4(f4 v) {
  s4 r;
  r.x = to_bf16(v.x);
  r.y = to_bf16(v.y);
  r.z = to_bf16(v.z);
  r.w = to_bf16(v.w);
  return r;
}

__device__ __forceinline__ float tanh_fast(float z) {
  const float e = __expf(2.0f * z);
  return 1.0f - __fdividef(2.0f, e + 1.0f);
}

__device__ __forceinline__ f4 mfma(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// 16 x 16 x 32: lane l holds A row l % 16 and B column l % 16, K elements
// 8 (l / 16) .. + 7; the accumulator as in the 16-deep form
__device__ __forceinline__ f4 mfma32(s8 a, s8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                  __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

__device__ __forceinline__ s8 cat8(s4 lo, s4 hi) {
  return s8{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
}

// element e (0..7) of lane L of forward fragment f, from the flat params:
// rows are output neurons 16 t + L % 16, K element k = 8 (L / 16) + e of
// step s is input 32 s + k of the first layer, and hidden neuron
// 16 (2 s + e / 4) + 4 (L / 16) + e % 4 of the others
__device__ inline float fwd_value(const float* __restrict__ p, int f, int L, int e) {
  const int i = L & 15, kq = L >> 4;
  const int hid_in = 4 * kq + (e & 3);  // + 16 (2 s + e / 4)
  if (f < F_L2) {  // W1: tile t of outputs, K step s of inputs
    const int t = f / 2, s = f % 2, o = 16 * t + i, in = 32 * s + 8 * kq + e;
    return in < NIN ? p[OW1 + o * NIN + in] : 0.0f;
  }
  if (f < F_L4) {  // W2, W3
    const int base = f < F_L3 ? OW2 : OW3, ff = f < F_L3 ? f - F_L2 : f - F_L3;
    const int t = ff / 2, s = ff % 2, o = 16 * t + i, in = 16 * (2 * s + (e >> 2)) + hid_in;
    return p[base + o * NH + in];
  }
  {  // W4 (rows 4..15 of the tile are zero)
    const int s = f - F_L4, o = i, in = 16 * (2 * s + (e >> 2)) + hid_in;
    return o < NOUT ? p[OW4 + o * NH + in] : 0.0f;
  }
}

// element e (0..3) of lane L of transposed fragment f (backward pass, K = 16)
__device__ inline float tr_value(const float* __restrict__ p, int f, int L, int e) {
  const int i = L & 15, kq = L >> 4;
  if (f < F_T4) {  // W2^T, W3^T: rows are inputs, K runs over outputs
    const int base = f < F_T3 ? OW2 : OW3, ff = f < F_T3 ? f - F_T2 : f - F_T3;
    const int t = ff / 4, s = ff % 4, in = 16 * t + i, o = 16 * s + 4 * kq + e;
    return p[base + o * NH + in];
  }
  {  // W4^T: K runs over the 4 outputs (padded to 16)
    const int t = f - F_T4, in = 16 * t + i, o = 4 * kq + e;
    return o < NOUT ? p[OW4 + o * NH + in] : 0.0f;
  }
}

// flat FP32 parameters -> packed BF16 fragments + FP32 biases
__global__ void k_mlp_pack(const float* __restrict__ p, void* __restrict__ packed) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int NF = NFWD * 64 * 8;
  if (idx < NF) {
    const int e = idx & 7, L = (idx >> 3) & 63, f = idx >> 9;
    reinterpret_cast<short*>(packed)[idx] = to_bf16(fwd_value(p, f, L, e));
  } else if (idx < PACK_VALUES) {
    const int k = idx - NF, e = k & 3, L = (k >> 2) & 63, f = k >> 8;
    reinterpret_cast<short*>(packed)[idx] = to_bf16(tr_value(p, f, L, e));
  } else if (idx < PACK_VALUES + NBIAS) {
    const int b = idx - PACK_VALUES;
    float v;
    if (b < NH) v = p[OB1 + b];
    else if (b < 2 * NH) v = p[OB2 + b - NH];
    else if (b < 3 * NH) v = p[OB3 + b - 2 * NH];
    else v = (b - 3 * NH) < NOUT ? p[OB4 + b - 3 * NH] : 0.0f;
    reinterpret_cast<float*>(reinterpret_cast<char*>(packed) + FRAG_BYTES)[b] = v;
  }
}

__device__ __forceinline__ const s8* fwd_frags(const void* packed) {
  return reinterpret_cast<const s8*>(packed);
}
__device__ __forceinline__ const s4* tr_frags(const void* packed) {
  return reinterpret_cast<const s4*>(reinterpret_cast<const char*>(packed) + FWD_BYTES);
}
__device__ __forceinline__ const float* biases(const void* packed) {
  return reinterpret_cast<const float*>(reinterpret_cast<const char*>(packed) + FRAG_BYTES);
}

// bias of rows 16 t + 4 q .. + 3 of a layer (the accumulator start)
__device__ __forceinline__ f4 bias_frag(const float* b, int t, int lane) {
  return *reinterpret_cast<const f4*>(b + 16 * t + 4 * (lane >> 4));
}

// forward fragments of one wavefront, kept in registers by the caller
struct FwdW {
  s8 w[NFWD];
};

__device__ __forceinline__ void load_fwd(const void* packed, FwdW& W, int lane) {
  const s8* F = fwd_frags(packed);
#pragma unroll
  for (int f = 0; f < NFWD; ++f) W.w[f] = F[f * 64 + lane];
}

// Hidden activations of one 16-sample tile (post-tanh, FP32 and BF16).
struct Acts {
  f4 a[3][4];
  s4 b[3][4];
};

// 16 samples through the network: x holds the two K fragments of the
// inputs (features 32 s + 8 q .. + 7 of sample j in lane j + 16 q).  Returns
// the output tile: lanes 0..15 hold outputs 0..3 of their sample.
template <bool KEEP>
__device__ __forceinline__ f4 forward16(const FwdW& W, const float* __restrict__ bias,
                                        const s8 (&x)[2], Acts* acts, int lane) {
  s4 b[4];
  f4 h[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    h[t] = bias_frag(bias, t, lane);
#pragma unroll
    for (int s = 0; s < 2; ++s) h[t] = mfma32(W.w[F_L1 + 2 * t + s], x[s], h[t]);
  }
#pragma unroll
  for (int l = 0; l < 3; ++l) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int r = 0; r < 4; ++r) h[t][r] = tanh_fast(h[t][r]);
      b[t] = pack4(h[t]);
      if (KEEP) {
        acts->a[l][t] = h[t];
        acts->b[l][t] = b[t];
      }
    }
    if (l == 2) break;
    const int base = l == 0 ? F_L2 : F_L3;
    const float* bl = bias + NH * (l + 1);
    const s8 bk[2] = {cat8(b[0], b[1]), cat8(b[2], b[3])};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      h[t] = bias_frag(bl, t, lane);
#pragma unroll
      for (int s = 0; s < 2; ++s) h[t] = mfma32(W.w[base + 2 * t + s], bk[s], h[t]);
    }
  }
  f4 y = bias_frag(bias + 3 * NH, 0, lane);
#pragma unroll
  for (int s = 0; s < 2; ++s) y = mfma32(W.w[F_L4 + s], cat8(b[2 * s], b[2 * s + 1]), y);
  return y;
}

// inputs of one 16-sample tile from row `row` of a row-major [.][37] FP32
// array (zero where `ok` is false)
__device__ __forceinline__ void load_x(const float* __restrict__ x, long row, bool ok, int lane,
                                       s8 (&xf)[2]) {
  const int q = lane >> 4;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    f4 lo, hi;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int in = 32 * s + 8 * q + e;
      lo[e] = (ok && in < NIN) ? x[row * NIN + in] : 0.0f;
      hi[e] = (ok && in + 4 < NIN) ? x[row * NIN + in + 4] : 0.0f;
    }
    xf[s] = cat8(pack4(lo), pack4(hi));
  }
}

// y[n][4] = MLP(x[n][37]); grid-stride over 16-sample tiles
__global__ __launch_bounds__(256) void k_mlp_forward(const void* __restrict__ packed,
                                                     const float* __restrict__ x,
                                                     float* __restrict__ y, long n) {
  const int lane = threadIdx.x & 63;
  FwdW W;
  load_fwd(packed, W, lane);
  const float* bias = biases(packed);
  const long ntile = (n + 15) / 16;
  const long wave = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const long nwave = (long)gridDim.x * (blockDim.x >> 6);
  for (long tile = wave; tile < ntile; tile += nwave) {
    const long j = tile * 16 + (lane & 15);
    s8 xf[2];
    load_x(x, j, j < n, lane, xf);
    const f4 out = forward16<false>(W, bias, xf, nullptr, lane);
    if (lane < 16 && j < n) *reinterpret_cast<f4*>(y + j * NOUT) = out;
  }
}

// ------------------------------------------------------------------ training
// Gradient of L = (1/(4n)) sum (y - t)^2 with respect to the flat FP32
// parameters (evaluated at the packed BF16 weights); sample j of the batch
// is row idx[j] of x and t (row j without idx).  Each wavefront takes
// 16-sample tiles; weight gradients are 16 x 16 MFMA tiles with the samples
// as K, which needs activations and deltas with 4 consecutive samples per
// lane: they pass through a small LDS transpose.  Per-block gradients are
// summed in LDS and added to `grad` (zeroed beforehand) at the end.

constexpr int TR_ROW = 16;  // bf16 per transposed row (16 samples)

// LDS hand-off inside one wavefront (its LDS operations complete in order)
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// store an accumulator-layout tile (rows 4q+r, column j) into rows
// [16 t, 16 t + 16) of a transposed [neuron][sample] LDS array
__device__ __forceinline__ void tr_store(short* T, int t, s4 v, int lane) {
  const int j = lane & 15, q = lane >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) T[(16 * t + 4 * q + r) * TR_ROW + j] = v[r];
}

// an input fragment (features 32 s + 8 q + e of sample j) into rows
// 32 s + 8 q + e of the transposed array
__device__ __forceinline__ void tr_store8(short* T, int s, s8 v, int lane) {
  const int j = lane & 15, q = lane >> 4;
#pragma unroll
  for (int e = 0; e < 8; ++e) T[(32 * s + 8 * q + e) * TR_ROW + j] = v[e];
}

// fragment with rows 16 t + i and K = samples 4 q .. 4 q + 3
__device__ __forceinline__ s4 tr_load(const short* T, int t, int lane) {
  const int i = lane & 15, q = lane >> 4;
  return *reinterpret_cast<const s4*>(T + (16 * t + i) * TR_ROW + 4 * q);
}

// gradient tile (rows = outputs 16 T + 4 q + r, column = input 16 U + j)
// into the wavefront's own LDS gradient of a layer with nout x nin weights
// (the lanes of a tile touch distinct entries, and one wavefront's LDS
// operations complete in order, so plain adds accumulate in a fixed order)
__device__ __forceinline__ void add_wgrad(float* gl, int ow, int nout, int nin, int T, int U,
                                          f4 v, int lane) {
  const int j = lane & 15, q = lane >> 4;
  const int in = 16 * U + j;
  if (in >= nin) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int o = 16 * T + 4 * q + r;
    if (o < nout) gl[ow + o * nin + in] += v[r];
  }
}

// sum over the 16 sample columns of an accumulator tile; lanes j == 0 add
// rows 4 q + r to the bias gradient
__device__ __forceinline__ void add_bgrad(float* gl, int ob, int nout, int t, f4 v, int lane) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float s = v[r];
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    s += __shfl_xor(s, 4);
    s += __shfl_xor(s, 8);
    v[r] = s;
  }
  if ((lane & 15) == 0) {
    const int q = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 16 * t + 4 * q + r;
      if (o < nout) gl[ob + o] += v[r];
    }
  }
}

// Gradient in a fixed summation order (bit-reproducible): every wavefront
// keeps its own gradient in LDS, the block adds its wavefronts in order and
// writes one partial gradient (and loss) per block to the work area; a
// second launch sums the partials over the blocks in block order.
constexpr int GRAD_WAVES = 2;
constexpr int GRAD_BLOCKS = 128;                 // largest grid of the gradient kernel
constexpr int PART_STRIDE = (NPARAM + 1 + 63) & ~63;  // partial gradient + loss, floats
constexpr size_t GRAD_LDS = (size_t)GRAD_WAVES * NPARAM * sizeof(float) +
                            (size_t)GRAD_WAVES * 2 * NH * TR_ROW * sizeof(short);
// work area of one gradient call (bytes) for n samples
__host__ __device__ constexpr int grad_blocks(long n) {
  return (int)((n + 15) / 16 < (long)GRAD_BLOCKS * GRAD_WAVES
                   ? ((n + 15) / 16 + GRAD_WAVES - 1) / GRAD_WAVES
                   : GRAD_BLOCKS);
}
constexpr size_t GRAD_WORK_MAX = (size_t)GRAD_BLOCKS * PART_STRIDE * sizeof(float);

__global__ __launch_bounds__(64 * GRAD_WAVES) void k_mlp_grad(const void* __restrict__ packed,
                                                              const float* __restrict__ x,
                                                              const float* __restrict__ t,
                                                              const int* __restrict__ idx,
                                                              long n, float* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float* gl = reinterpret_cast<float*>(lds_raw) + (size_t)wv * NPARAM;
  short* TA = reinterpret_cast<short*>(lds_raw + GRAD_WAVES * NPARAM * sizeof(float)) +
              wv * 2 * NH * TR_ROW;
  short* TZ = TA + NH * TR_ROW;
  for (int i = threadIdx.x; i < GRAD_WAVES * NPARAM; i += blockDim.x)
    reinterpret_cast<float*>(lds_raw)[i] = 0.0f;
  __syncthreads();

  FwdW W;
  load_fwd(packed, W, lane);
  const float* bias = biases(packed);
  const s4* F = tr_frags(packed);
  const float inv = 1.0f / (4.0f * (float)n);
  float lsum = 0.0f;
  const long ntile = (n + 15) / 16;
  const long wave = (long)blockIdx.x * GRAD_WAVES + wv;
  const long nwave = (long)gridDim.x * GRAD_WAVES;
  const int q = lane >> 4;
  for (long tile = wave; tile < ntile; tile += nwave) {
    const long j = tile * 16 + (lane & 15);
    const long row = j < n ? (idx ? (long)idx[j] : j) : 0;
    s8 xf[2];
    load_x(x, row, j < n, lane, xf);
    Acts A;
    const f4 y = forward16<true>(W, bias, xf, &A, lane);
    // output delta: rows 0..3 (lanes 0..15) of valid samples
    f4 dz;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float d = 0.0f;
      if (q == 0 && j < n) {
        const float e = y[r] - t[row * NOUT + r];
        lsum += e * e;
        d = 2.0f * e * inv;
      }
      dz[r] = d;
    }
    // layer 4: gradients and delta of a3
    s4 bz = pack4(dz);
    add_bgrad(gl, OB4, NOUT, 0, dz, lane);
    tr_store(TZ, 0, bz, lane);
#pragma unroll
    for (int u = 0; u < 4; ++u) tr_store(TA, u, A.b[2][u], lane);
    wave_sync_lds();
    {
      const s4 az = tr_load(TZ, 0, lane);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const f4 g = mfma(az, tr_load(TA, u, lane), f4{0.f, 0.f, 0.f, 0.f});
        add_wgrad(gl, OW4, NOUT, NH, 0, u, g, lane);
      }
    }
    f4 d[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      d[u] = mfma(F[(F_T4 + u) * 64 + lane], bz, f4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
      for (int r = 0; r < 4; ++r) d[u][r] *= 1.0f - A.a[2][u][r] * A.a[2][u][r];
    }
    // layers 3 and 2: d holds dL/dz of the layer's outputs
#pragma unroll
    for (int l = 2; l >= 1; --l) {
      const int ow = l == 2 ? OW3 : OW2, ob = l == 2 ? OB3 : OB2;
      const int ft = l == 2 ? F_T3 : F_T2;
      s4 bd[4];
      wave_sync_lds();
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        bd[u] = pack4(d[u]);
        add_bgrad(gl, ob, NH, u, d[u], lane);
        tr_store(TZ, u, bd[u], lane);
        tr_store(TA, u, A.b[l - 1][u], lane);
      }
      wave_sync_lds();
#pragma unroll
      for (int T = 0; T < 4; ++T) {
        const s4 az = tr_load(TZ, T, lane);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const f4 g = mfma(az, tr_load(TA, u, lane), f4{0.f, 0.f, 0.f, 0.f});
          add_wgrad(gl, ow, NH, NH, T, u, g, lane);
        }
      }
      f4 dn[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        dn[u] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) dn[u] = mfma(F[(ft + 4 * u + s) * 64 + lane], bd[s], dn[u]);
#pragma unroll
        for (int r = 0; r < 4; ++r) dn[u][r] *= 1.0f - A.a[l - 1][u][r] * A.a[l - 1][u][r];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) d[u] = dn[u];
    }
    // layer 1: gradients only (inputs are data)
    wave_sync_lds();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      add_bgrad(gl, OB1, NH, u, d[u], lane);
      tr_store(TZ, u, pack4(d[u]), lane);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) tr_store8(TA, s, xf[s], lane);
    wave_sync_lds();
#pragma unroll
    for (int T = 0; T < 4; ++T) {
      const s4 az = tr_load(TZ, T, lane);
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const f4 g = mfma(az, tr_load(TA, s, lane), f4{0.f, 0.f, 0.f, 0.f});
        add_wgrad(gl, OW1, NH, NIN, T, s, g, lane);
      }
    }
    wave_sync_lds();
  }
  // the block's loss and gradient: wavefronts added in order
  float ls = lsum;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) ls += __shfl_xor(ls, o);
  __shared__ float wl[GRAD_WAVES];
  if (lane == 0) wl[wv] = ls * inv;
  __syncthreads();
  const float* g0 = reinterpret_cast<const float*>(lds_raw);
  float* out = part + (size_t)blockIdx.x * PART_STRIDE;
  for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) {
    float v = g0[i];
#pragma unroll
    for (int w = 1; w < GRAD_WAVES; ++w) v += g0[(size_t)w * NPARAM + i];
    out[i] = v;
  }
  if (threadIdx.x == 0) {
    float l = wl[0];
#pragma unroll
    for (int w = 1; w < GRAD_WAVES; ++w) l += wl[w];
    out[NPARAM] = l;
  }
}

// grad[i] = sum over blocks b = 0, 1, ... of the partials (in that order);
// thread NPARAM sums the loss
__global__ void k_mlp_grad_reduce(const float* __restrict__ part, int nblocks,
                                  float* __restrict__ grad, float* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > NPARAM) return;
  // 16 partials loaded at a time, then added in block order (the same sums
  // as one at a time, with the loads' latencies overlapped)
  float v = 0.0f;
  int b = 0;
  for (; b + 16 <= nblocks; b += 16) {
    float t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t[u] = part[(size_t)(b + u) * PART_STRIDE + i];
#pragma unroll
    for (int u = 0; u < 16; ++u) v += t[u];
  }
  for (; b < nblocks; ++b) v += part[(size_t)b * PART_STRIDE + i];
  if (i < NPARAM)
    grad[i] = v;
  else
    *loss = v;
}

// Adam with bias correction on the FP32 master parameters (c1 = 1 - b1^k,
// c2 = 1 - b2^k from the host)
__global__ void k_mlp_adam(float* __restrict__ p, const float* __restrict__ g,
                           float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                           float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_mlp_zero(float* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

}  // namespace mlp
}  // namespace hofks
