// Achievable HBM bandwidth of the part: the roofline denominator measured beside the published 8 TB/s.
// Three streaming kernels over caller-sized buffers (1 GiB and more, far beyond the 256 MB Infinity
// Cache).  Each block streams one contiguous chunk of the arrays (DRAM-page friendly: on this part a
// grid-stride walk reads ~20% slower), each lane moving 16-byte vectors with U loads in flight, and the
// accesses are non-temporal (the data is touched once):
//   read   s += a[i]        (one partial sum per block is written, so the loads stay live)
//   copy   b[i] = a[i]
//   triad  a[i] = b[i] + q c[i]
// Bytes moved per launch: n, 2 n and 3 n bytes for arrays of n bytes.
#include "kernels.hpp"

namespace gmrf {

constexpr int kBwThreads = 256;
typedef float f4 __attribute__((ext_vector_type(4)));

// [b0, b1): the block's contiguous share of n4 16-byte elements
__device__ __forceinline__ void bw_chunk(size_t n4, size_t& b0, size_t& b1) {
  const size_t per = (n4 + gridDim.x - 1) / gridDim.x;
  b0 = min(n4, (size_t)blockIdx.x * per);
  b1 = min(n4, b0 + per);
}

template <int U>
__global__ __launch_bounds__(kBwThreads) void k_bw_read(const f4* __restrict__ a, size_t n4, float* __restrict__ out) {
  size_t b0, b1;
  bw_chunk(n4, b0, b1);
  size_t i = b0 + threadIdx.x;
  float acc = 0.f;
  for (; i + (U - 1) * kBwThreads < b1; i += U * kBwThreads) {
    f4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(&a[i + u * kBwThreads]);
#pragma unroll
    for (int u = 0; u < U; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  for (; i < b1; i += kBwThreads) {
    const f4 v = a[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  __shared__ float red[kBwThreads / kWave];
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int w = 0; w < kBwThreads / kWave; ++w) t += red[w];
    out[blockIdx.x] = t;
  }
}

template <int U>
__global__ __launch_bounds__(kBwThreads) void k_bw_copy(const f4* __restrict__ a, f4* __restrict__ b, size_t n4) {
  size_t b0, b1;
  bw_chunk(n4, b0, b1);
  size_t i = b0 + threadIdx.x;
  for (; i + (U - 1) * kBwThreads < b1; i += U * kBwThreads) {
    f4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(&a[i + u * kBwThreads]);
#pragma unroll
    for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], &b[i + u * kBwThreads]);
  }
  for (; i < b1; i += kBwThreads) b[i] = a[i];
}

template <int U>
__global__ __launch_bounds__(kBwThreads) void k_bw_triad(f4* __restrict__ a, const f4* __restrict__ b,
                                                         const f4* __restrict__ c, float q, size_t n4) {
  size_t b0, b1;
  bw_chunk(n4, b0, b1);
  size_t i = b0 + threadIdx.x;
  for (; i + (U - 1) * kBwThreads < b1; i += U * kBwThreads) {
    f4 x[U], y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      x[u] = __builtin_nontemporal_load(&b[i + u * kBwThreads]);
      y[u] = __builtin_nontemporal_load(&c[i + u * kBwThreads]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) __builtin_nontemporal_store(x[u] + q * y[u], &a[i + u * kBwThreads]);
  }
  for (; i < b1; i += kBwThreads) a[i] = b[i] + q * c[i];
}

// which 0 read (a, out), 1 copy (a -> b), 2 triad (b, c -> a); n4 = elements of 16 bytes per array
void launch_bandwidth(int which, int blocks, void* a, void* b, void* c, float* out, size_t n4, hipStream_t st) {
  if (which == 0)
    hipLaunchKernelGGL(k_bw_read<16>, dim3(blocks), dim3(kBwThreads), 0, st, (const f4*)a, n4, out);
  else if (which == 1)
    hipLaunchKernelGGL(k_bw_copy<8>, dim3(blocks), dim3(kBwThreads), 0, st, (const f4*)a, (f4*)b, n4);
  else
    hipLaunchKernelGGL(k_bw_triad<8>, dim3(blocks), dim3(kBwThreads), 0, st, (f4*)a, (const f4*)b, (const f4*)c,
                       0.5f, n4);
}

}  // namespace gmrf
