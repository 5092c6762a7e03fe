// probe.hpp -- streaming probes of the HBM bandwidth the kinetic kernels are
// measured against: the same 16-byte non-temporal accesses the piece loops
// use, without any arithmetic.  mode 0 reads `bytes` (folding them into one
// word per thread so that the loads are kept), mode 1 writes them, mode 2
// copies them.  Blocks take contiguous chunks of 16-byte vectors, four per
// thread per iteration, so every wavefront issues 4 KB of requests at once.
#pragma once
#include <hip/hip_runtime.h>

namespace hofks {

constexpr int PROBE_TPB = 256;
constexpr int PROBE_UNR = 4;
typedef unsigned pv4 __attribute__((ext_vector_type(4)));

template <int MODE>
__global__ __launch_bounds__(PROBE_TPB) void k_stream_probe(const pv4* __restrict__ src,
                                                            pv4* __restrict__ dst, size_t nvec,
                                                            unsigned* __restrict__ sink) {
  const size_t stride = (size_t)gridDim.x * PROBE_TPB * PROBE_UNR;
  unsigned acc = 0;
  for (size_t base = (size_t)blockIdx.x * PROBE_TPB * PROBE_UNR + threadIdx.x; base < nvec;
       base += stride) {
    pv4 v[PROBE_UNR];
#pragma unroll
    for (int u = 0; u < PROBE_UNR; ++u) {
      const size_t i = base + (size_t)u * PROBE_TPB;
      if (MODE != 1 && i < nvec) v[u] = __builtin_nontemporal_load(src + i);
      if (MODE == 1) v[u] = pv4{(unsigned)i, 0u, 0u, 0u};
    }
#pragma unroll
    for (int u = 0; u < PROBE_UNR; ++u) {
      const size_t i = base + (size_t)u * PROBE_TPB;
      if (i >= nvec) continue;
      if (MODE == 0)
        acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
      else
        __builtin_nontemporal_store(v[u], dst + i);
    }
  }
  // the read probe keeps its loads alive through a store that is taken
  // only for one improbable value
  if (MODE == 0 && acc == 0x9e3779b9u) sink[0] = acc;
}

}  // namespace hofks
