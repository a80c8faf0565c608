// Elementwise kernels of the Lanczos recurrence (Algorithm 1), the full
// reorthogonalisation, the final combination x_m = ||z|| V_m y and the Rademacher probes
// of the Hutchinson estimator (Section 6).  All memory-bound: coalesced strided loops, FP64
// arithmetic on values loaded from the storage type T, deterministic partial sums.
#include <stdint.h>

#include <algorithm>

#include "kernels.hpp"

namespace gmrf {

// Element e of block b, thread t, step q: b*chunk + q*NT + t  (each wave-load coalesced).
#define EW_LOOP(q) for (int q = 0; q < kEwPerThread; ++q)

// ---- init: slot 0 <- z (storage type), partial sums of ||z||^2 ------------------------------
template <typename T>
__global__ __launch_bounds__(kEwThreads) void k_init_from_f64(const double* __restrict__ Z, long zld,
                                                              long L, T* __restrict__ V0, LzState S) {
  __shared__ double lds[kEwThreads / kWave];
  const int r = blockIdx.y;
  const long len = lz_len(S, r, L);
  if ((long)blockIdx.x * kEwChunk >= len) return;
  const long base = (long)blockIdx.x * kEwChunk + threadIdx.x;
  const int64_t* ext = S.col_ext ? S.col_ext : S.col_off;
  const double* z = Z + (ext ? (size_t)ext[r] : (size_t)r * zld);
  T* v = V0 + lz_off(S, r, L);
  double acc = 0.0;
  EW_LOOP(q) {
    const long e = base + (long)q * kEwThreads;
    if (e < len) {
      const T t = (T)z[e];
      v[e] = t;
      acc += ip_weight(S, e) * (double)t * (double)t;
    }
  }
  const double s = block_sum<kEwThreads>(acc, lds);
  if (threadIdx.x == 0) S.part_b[(size_t)r * S.pstride + blockIdx.x] = s;
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
//   (hi0, lo0) = M0 c0, (hi1, lo1) = M1 c2, c <- (hi1^c1^k0, lo1, hi0^c3^k1, lo0), key += W.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Rademacher probe entries: lane l of a wave generates the four Philox words of block
// (wave_base + l) (256 entries); the wave then writes its 64 x 256 entries with coalesced
// stores, reading each word from its owner lane.  With a colouring (Section 6.1) entries whose
// node is not of class `cls` are zero: the probe restricted to one colour class.
template <typename OutT>
__device__ __forceinline__ void rademacher_wave(uint64_t seed, int p, long n, long wave_block0,
                                                OutT* out, double& acc, const int32_t* colour = nullptr,
                                                int cls = 0) {
  const int lane = threadIdx.x & (kWave - 1);
  uint64_t c[4] = {(uint64_t)(wave_block0 + lane), (uint64_t)p, 0ull, 0ull};
  philox4x64_10(c, seed, 0ull);
  const long e0 = wave_block0 * 256;
  for (int q = 0; q < 256; ++q) {
    // entry e0 + 64 q + lane lies in block (wave_block0 + q/4), word q%4, bit lane
    const int src = q >> 2, wsel = q & 3;
    const uint64_t wv = wsel == 0 ? c[0] : wsel == 1 ? c[1] : wsel == 2 ? c[2] : c[3];
    const uint32_t lo = __shfl((uint32_t)(wv & 0xffffffffu), src, kWave);
    const uint32_t hi = __shfl((uint32_t)(wv >> 32), src, kWave);
    const uint64_t word = ((uint64_t)hi << 32) | lo;
    const long e = e0 + 64L * q + lane;
    if (e < n) {
      const int bit = (int)((word >> lane) & 1ull);
      const bool on = colour == nullptr || colour[e] == cls;
      const OutT v = !on ? (OutT)0 : bit ? (OutT)-1 : (OutT)1;
      out[e] = v;
      acc += on ? 1.0 : 0.0;
    }
  }
}

__global__ __launch_bounds__(256) void k_rademacher_i8(uint64_t seed, long n, int8_t* __restrict__ out) {
  const int p = blockIdx.y;
  const long wave_block0 = ((long)blockIdx.x * (256 / kWave) + threadIdx.x / kWave) * kWave;
  if (wave_block0 * 256 >= n) return;
  double acc = 0.0;
  rademacher_wave<int8_t>(seed, p, n, wave_block0, out + (size_t)p * n, acc);
}

// Probe columns q = p0, p0 + 1, ... straight into Krylov slot 0 (storage type, column q - p0); ||v||^2
// partials per block.  Column q is probe q / K restricted to colour class q mod K (K = 1, colour = NULL:
// the plain probe q).
template <typename T>
__global__ __launch_bounds__(256) void k_init_rademacher(uint64_t seed, long n, int p0, T* __restrict__ V0,
                                                         LzState S, const int32_t* __restrict__ colour, int K) {
  __shared__ double lds[256 / kWave];
  const int p = blockIdx.y;
  const int q = p0 + p;
  const long wave_block0 = ((long)blockIdx.x * (256 / kWave) + threadIdx.x / kWave) * kWave;
  double acc = 0.0;
  if (wave_block0 * 256 < n)
    rademacher_wave<T>(seed, q / K, n, wave_block0, V0 + (size_t)p * n, acc, colour, q % K);
  const double s = block_sum<256>(acc, lds);
  if (threadIdx.x == 0) S.part_b[(size_t)p * S.pstride + blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kEwThreads) void k_init_from_i8(const int8_t* __restrict__ P, long L,
                                                             T* __restrict__ V0, LzState S) {
  __shared__ double lds[kEwThreads / kWave];
  const int r = blockIdx.y;
  const long base = (long)blockIdx.x * kEwChunk + threadIdx.x;
  double acc = 0.0;
  EW_LOOP(q) {
    const long e = base + (long)q * kEwThreads;
    if (e < L) {
      const T t = (T)P[(size_t)r * L + e];
      V0[(size_t)r * L + e] = t;
      acc += (double)t * (double)t;
    }
  }
  const double s = block_sum<kEwThreads>(acc, lds);
  if (threadIdx.x == 0) S.part_b[(size_t)r * S.pstride + blockIdx.x] = s;
}

// ---- update: alpha_j from the op kernel's partials, w_j = q - alpha_j v_j into slot j ------
template <typename T>
__global__ __launch_bounds__(kEwThreads) void k_update(const T* __restrict__ Qb, const T* __restrict__ Vj,
                                                       T* __restrict__ W, long L, int j, int with_norm,
                                                       LzState S) {
  __shared__ double lds[kEwThreads / kWave];
  __shared__ int flag[1];
  const int r = blockIdx.y;
  const long len = lz_len(S, r, L);
  if ((long)blockIdx.x * kEwChunk >= len) return;
  if (!block_active(S, r, flag)) return;
  const double a = sum_partials<kEwThreads>(S.part_a + (size_t)r * S.pstride, lz_pa(S, r), lds);
  if (blockIdx.x == 0 && threadIdx.x == 0) S.alpha[lz_ia(S, r, j)] = a;
  const double sc = 1.0 / S.beta[lz_ib(S, r, j - 1)];
  const size_t off = lz_off(S, r, L);
  const T* vj = Vj + off;
  T* w = W + off;
  const T* q = Qb + off;
  const long base = (long)blockIdx.x * kEwChunk + threadIdx.x;
  double acc = 0.0;
  EW_LOOP(qq) {
    const long e = base + (long)qq * kEwThreads;
    if (e < len) {
      const double v = (double)(T)((double)vj[e] * sc);
      const T t = (T)((double)q[e] - a * v);
      w[e] = t;
      acc += ip_weight(S, e) * (double)t * (double)t;
    }
  }
  if (with_norm) {
    const double s = block_sum<kEwThreads>(acc, lds);
    if (threadIdx.x == 0) S.part_b[(size_t)r * S.pstride + blockIdx.x] = s;
  }
}

// ---- weighted ||v||^2 partials of slot 0 (after an FFT-based init) ------------------------------
template <typename T>
__global__ __launch_bounds__(kEwThreads) void k_norm_partials(const T* __restrict__ V0, long L, LzState S) {
  __shared__ double lds[kEwThreads / kWave];
  const int r = blockIdx.y;
  const long base = (long)blockIdx.x * kEwChunk + threadIdx.x;
  double acc = 0.0;
  EW_LOOP(q) {
    const long e = base + (long)q * kEwThreads;
    if (e < L) {
      const double t = (double)V0[(size_t)r * L + e];
      acc += ip_weight(S, e) * t * t;
    }
  }
  const double s = block_sum<kEwThreads>(acc, lds);
  if (threadIdx.x == 0) S.part_b[(size_t)r * S.pstride + blockIdx.x] = s;
}

// ---- closes runs that reached m_max ----------------------------------------------------------
__global__ __launch_bounds__(256) void k_finalize(LzState S) {
  __shared__ double lds[256 / kWave];
  __shared__ int flag[1];
  double a, b, c;
  lz_open<256>(S, blockIdx.x, S.m_max + 1, threadIdx.x == 0, lds, flag, a, b, c);
}

// ---- full reorthogonalisation, classical Gram-Schmidt ------------------------------------------
// pass: h_t = v_{t+1}^T w for t < j (partials per block), then w -= sum_t h_t v_{t+1}.
// Dot kernel: the block's chunk of w is staged in LDS; wave g takes basis vectors
// t = g, g + NW, ... and reduces each with wave shuffles only.
// grid.z splits t < j into slices of tslice vectors (short vectors: the dot of every basis vector in
// flight at once instead of a chain of j / NW per wave); each h_t is still formed by one wave alone, so
// the result does not depend on the split.
template <typename T>
__global__ __launch_bounds__(kEwThreads) void k_reorth_dot(const T* __restrict__ V, long L, int j,
                                                           double* __restrict__ part_h, int hstride,
                                                           int tslice, LzState S) {
  __shared__ double wl[kEwChunk];
  __shared__ int flag[1];
  const int r = blockIdx.y;
  if (!block_active(S, r, flag)) return;
  const size_t vs = lz_slot(S, L);
  const long base = (long)blockIdx.x * kEwChunk;
  const T* w = V + (size_t)j * vs + (size_t)r * L;
  for (int i = threadIdx.x; i < kEwChunk; i += kEwThreads) {
    const long e = base + i;
    wl[i] = (e < L) ? ip_weight(S, e) * (double)w[e] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), g = threadIdx.x / kWave;
  constexpr int NW = kEwThreads / kWave;
  const int t1 = min(j, (int)(blockIdx.z + 1) * tslice);
  for (int t = (int)blockIdx.z * tslice + g; t < t1; t += NW) {
    const T* vt = V + (size_t)t * vs + (size_t)r * L;
    const double sc = 1.0 / S.beta[lz_ib(S, r, t)];
    double acc = 0.0;
    for (int i = lane; i < kEwChunk; i += kWave) {
      const long e = base + i;
      if (e < L) acc += (double)(T)((double)vt[e] * sc) * wl[i];
    }
    acc = wave_sum(acc);
    if (lane == 0) part_h[((size_t)r * hstride + t) * gridDim.x + blockIdx.x] = acc;
  }
}

__global__ __launch_bounds__(256) void k_reorth_reduce(const double* __restrict__ part_h, int hstride,
                                                       int P, int j, double* __restrict__ h,
                                                       LzState S) {
  const int r = blockIdx.x;
  if (!S.active[r]) return;
  for (int t = threadIdx.x; t < j; t += 256) {
    const double* p = part_h + ((size_t)r * hstride + t) * P;
    double s = 0.0;
    for (int b = 0; b < P; ++b) s += p[b];
    h[(size_t)r * hstride + t] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(kEwThreads) void k_reorth_update(T* __restrict__ V, long L, int j,
                                                              const double* __restrict__ h,
                                                              int hstride, int with_norm,
                                                              LzState S) {
  __shared__ double cl[1024];
  __shared__ double lds[kEwThreads / kWave];
  __shared__ int flag[1];
  const int r = blockIdx.y;
  if (!block_active(S, r, flag)) return;
  const size_t vs = lz_slot(S, L);
  T* w = V + (size_t)j * vs + (size_t)r * L;
  const long base = (long)blockIdx.x * kEwChunk + threadIdx.x;
  double acc[kEwPerThread];
  EW_LOOP(q) {
    const long e = base + (long)q * kEwThreads;
    acc[q] = (e < L) ? (double)w[e] : 0.0;
  }
  for (int t0 = 0; t0 < j; t0 += 1024) {
    const int tn = min(1024, j - t0);
    __syncthreads();
    for (int t = threadIdx.x; t < tn; t += kEwThreads) cl[t] = h[(size_t)r * hstride + t0 + t];
    __syncthreads();
    for (int t = 0; t < tn; ++t) {
      const T* vt = V + (size_t)(t0 + t) * vs + (size_t)r * L;
      const double sc = 1.0 / S.beta[lz_ib(S, r, t0 + t)];
      const double ht = cl[t];
      EW_LOOP(q) {
        const long e = base + (long)q * kEwThreads;
        if (e < L) acc[q] -= ht * (double)(T)((double)vt[e] * sc);
      }
    }
  }
  double nrm = 0.0;
  EW_LOOP(q) {
    const long e = base + (long)q * kEwThreads;
    if (e < L) {
      const T t = (T)acc[q];
      w[e] = t;
      nrm += ip_weight(S, e) * (double)t * (double)t;
    }
  }
  if (with_norm) {
    const double s = block_sum<kEwThreads>(nrm, lds);
    if (threadIdx.x == 0) S.part_b[(size_t)r * S.pstride + blockIdx.x] = s;
  }
}

// Short vectors (L <= kRoSmallL), dot half: block (x, r, z) covers the kEwChunk elements of chunk x for
// the basis vectors of slice z; wave g holds its 512 elements of w in registers (8 per lane) and
// reduces each v_{t+1}^T w over them, the four wave sums added in wave order through LDS.  No load
// waits on another: active[] is not written during the reorthogonalisation, so it is read directly.
constexpr int kRoDotTs = 64;   // basis vectors per LDS round

// Qb != nullptr (first pass only): the kernel also does the update step that precedes the
// reorthogonalisation.  Every block forms alpha_j from the operator's partial sums and
// w_j = q - alpha_j v_j for its elements (the update kernel's arithmetic); the blocks of slice 0 store w_j
// and alpha_j, so no block reads slot j in this launch.
template <typename T>
__global__ __launch_bounds__(kEwThreads) void k_reorth_dot_short(const T* V, T* Wj, const T* __restrict__ Qb, long L,
                                                                 int j, double* __restrict__ part_h, int hstride,
                                                                 int tslice, LzState S) {
  constexpr int NW = kEwThreads / kWave;
  constexpr int PER = kEwChunk / kEwThreads;
  __shared__ double red[NW][kRoDotTs];
  __shared__ double lds[NW];
  const int r = blockIdx.y;
  if (!S.active[r]) return;
  const size_t vs = lz_slot(S, L);
  const int lane = threadIdx.x & (kWave - 1), g = threadIdx.x / kWave;
  const long base = (long)blockIdx.x * kEwChunk + (long)g * (kWave * PER) + lane;
  const T* w = V + (size_t)j * vs + (size_t)r * L;
  double wv[PER];
  if (Qb) {
    const double a = sum_partials<kEwThreads>(S.part_a + (size_t)r * S.pstride, lz_pa(S, r), lds);
    if (blockIdx.x == 0 && blockIdx.z == 0 && threadIdx.x == 0) S.alpha[lz_ia(S, r, j)] = a;
    const double sc = 1.0 / S.beta[lz_ib(S, r, j - 1)];
    const T* vj = V + (size_t)(j - 1) * vs + (size_t)r * L;
    const T* q = Qb + (size_t)r * L;
    T* wr = Wj + (size_t)r * L;
#pragma unroll
    for (int qq = 0; qq < PER; ++qq) {
      const long e = base + (long)qq * kWave;
      wv[qq] = 0.0;
      if (e < L) {
        const double v = (double)(T)((double)vj[e] * sc);
        const T t = (T)((double)q[e] - a * v);
        if (blockIdx.z == 0) wr[e] = t;
        wv[qq] = ip_weight(S, e) * (double)t;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const long e = base + (long)q * kWave;
      wv[q] = (e < L) ? ip_weight(S, e) * (double)w[e] : 0.0;
    }
  }
  const int t1 = min(j, (int)(blockIdx.z + 1) * tslice);
  for (int t0 = (int)blockIdx.z * tslice; t0 < t1; t0 += kRoDotTs) {
    const int tn = min(kRoDotTs, t1 - t0);
    for (int u = 0; u < tn; ++u) {
      const int t = t0 + u;
      const T* vt = V + (size_t)t * vs + (size_t)r * L;
      const double sc = 1.0 / S.beta[lz_ib(S, r, t)];
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const long e = base + (long)q * kWave;
        if (e < L) acc += (double)(T)((double)vt[e] * sc) * wv[q];
      }
      acc = wave_sum(acc);
      if (lane == 0) red[g][u] = acc;
    }
    __syncthreads();
    if ((int)threadIdx.x < tn) {
      double s = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) s += red[w2][threadIdx.x];
      part_h[((size_t)r * hstride + t0 + threadIdx.x) * gridDim.x + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// Short vectors (L <= kRoSmallL): w -= sum_t h_t v_{t+1} with the t sum split over the 16 waves of a
// 1024-thread block (wave g takes t = g, g + 16, ...) over a 512-element chunk, the 16 partial sums
// added in wave order through LDS, so every element's chain is j / 16 long instead of j.  h_t is
// summed here from the dot kernel's P block partials (in block order), with no reduce launch.
constexpr int kRoThreads = 1024;
constexpr int kRoWaves = kRoThreads / kWave;
constexpr int kRoChunk = 512;
constexpr int kRoPer = kRoChunk / kWave;
constexpr long kRoSmallL = 65536;

template <typename T>
__global__ __launch_bounds__(kRoThreads) void k_reorth_update_short(T* __restrict__ V, long L, int j,
                                                                    const double* __restrict__ part_h,
                                                                    int hstride, int P, int with_norm, LzState S) {
  __shared__ double red[kRoWaves][kRoChunk];
  __shared__ double lds[kRoWaves];
  const int r = blockIdx.y;
  if (!S.active[r]) return;   // not written during the reorthogonalisation: every thread reads the same value
  const size_t vs = lz_slot(S, L);
  T* w = V + (size_t)j * vs + (size_t)r * L;
  const long base = (long)blockIdx.x * kRoChunk;
  const int lane = threadIdx.x & (kWave - 1), g = threadIdx.x / kWave;
  const long ew = base + threadIdx.x;
  const double w0 = ((int)threadIdx.x < kRoChunk && ew < L) ? (double)w[ew] : 0.0;   // in flight during the t loop
  double acc[kRoPer];
#pragma unroll
  for (int q = 0; q < kRoPer; ++q) acc[q] = 0.0;
  for (int t = g; t < j; t += kRoWaves) {
    const T* vt = V + (size_t)t * vs + (size_t)r * L;
    const double sc = 1.0 / S.beta[lz_ib(S, r, t)];
    const double* ph = part_h + ((size_t)r * hstride + t) * P;
    double ht = 0.0;
    for (int b = 0; b < P; ++b) ht += ph[b];
#pragma unroll
    for (int q = 0; q < kRoPer; ++q) {
      const long e = base + lane + q * kWave;
      if (e < L) acc[q] += ht * (double)(T)((double)vt[e] * sc);
    }
  }
#pragma unroll
  for (int q = 0; q < kRoPer; ++q) red[g][lane + q * kWave] = acc[q];
  __syncthreads();
  double nrm = 0.0;
  if ((int)threadIdx.x < kRoChunk) {
    double s = 0.0;
#pragma unroll
    for (int w2 = 0; w2 < kRoWaves; ++w2) s += red[w2][threadIdx.x];
    if (ew < L) {
      const T t = (T)(w0 - s);
      w[ew] = t;
      nrm = ip_weight(S, ew) * (double)t * (double)t;
    }
  }
  if (with_norm) {
    const double s = block_sum<kRoThreads>(nrm, lds);
    if (threadIdx.x == 0) S.part_b[(size_t)r * S.pstride + blockIdx.x] = s;
  }
}

// ---- x_m = ||z|| V_m y  (Algorithm 1, final step) ---------------------------------------------
// out[r*old + e] = beta_0 sum_{t < m} y_t v_{t+1}[e]; NaN for a column whose status is ENOTSPD
// or EINVAL, zero for m = 0.
template <typename T, typename OutT>
__global__ __launch_bounds__(kEwThreads) void k_combine(const T* __restrict__ V, long L,
                                                        const double* __restrict__ y, int ldy,
                                                        OutT* __restrict__ out, long old, LzState S) {
  __shared__ double cl[1024];
  const int r = blockIdx.y;
  const long len = lz_len(S, r, L);
  if ((long)blockIdx.x * kEwChunk >= len) return;
  const int m = S.m_used[r];
  const int st = S.status[r];
  const double beta0 = S.beta[lz_ib(S, r, 0)];
  const size_t vs = lz_slot(S, L);
  const size_t voff = lz_off(S, r, L);
  const int64_t* ext = S.col_ext ? S.col_ext : S.col_off;
  const size_t ooff = ext ? (size_t)ext[r] : (size_t)r * old;
  const long base = (long)blockIdx.x * kEwChunk + threadIdx.x;
  double acc[kEwPerThread];
  EW_LOOP(q) acc[q] = 0.0;
  const bool bad = (st == kENOTSPD || st == kEINVAL);
  if constexpr (sizeof(T) == 8) {
    // FP64 columns at even offsets: each thread takes pairs of elements with one 16-byte non-temporal load per
    // basis vector (the basis is read once); every element's sum is the same as below, in t order
    if (!bad && ((voff | vs) & 1) == 0 && (len & 1) == 0 && ((uintptr_t)V & 15) == 0) {
      typedef double d2 __attribute__((ext_vector_type(2)));
      constexpr int NP = kEwPerThread / 2;
      const long pbase = (long)blockIdx.x * kEwChunk + 2 * (long)threadIdx.x;
      double pacc[NP][2];
#pragma unroll
      for (int p = 0; p < NP; ++p) pacc[p][0] = pacc[p][1] = 0.0;
      for (int t0 = 0; t0 < m; t0 += 1024) {
        const int tn = min(1024, m - t0);
        __syncthreads();
        for (int t = threadIdx.x; t < tn; t += kEwThreads)
          cl[t] = beta0 * y[(size_t)r * ldy + t0 + t] / S.beta[lz_ib(S, r, t0 + t)];
        __syncthreads();
        int t = 0;
        for (; t + 3 < tn; t += 4) {
          const double* v0 = (const double*)V + (size_t)(t0 + t) * vs + voff;
          d2 x[4][NP];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int p = 0; p < NP; ++p) {
              const long e = pbase + (long)p * 2 * kEwThreads;
              x[u][p] = (e < len) ? __builtin_nontemporal_load((const d2*)(v0 + (size_t)u * vs + e)) : d2{0.0, 0.0};
            }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double ct = cl[t + u];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
              pacc[p][0] += ct * x[u][p].x;
              pacc[p][1] += ct * x[u][p].y;
            }
          }
        }
        for (; t < tn; ++t) {
          const double* vt = (const double*)V + (size_t)(t0 + t) * vs + voff;
          const double ct = cl[t];
#pragma unroll
          for (int p = 0; p < NP; ++p) {
            const long e = pbase + (long)p * 2 * kEwThreads;
            if (e < len) {
              const d2 xv = *(const d2*)(vt + e);
              pacc[p][0] += ct * xv.x;
              pacc[p][1] += ct * xv.y;
            }
          }
        }
      }
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const long e = pbase + (long)p * 2 * kEwThreads;
        if (e < len) {
          out[ooff + e] = (OutT)pacc[p][0];
          out[ooff + e + 1] = (OutT)pacc[p][1];
        }
      }
      return;
    }
  }
  if (!bad) {
    for (int t0 = 0; t0 < m; t0 += 1024) {
      const int tn = min(1024, m - t0);
      __syncthreads();
      for (int t = threadIdx.x; t < tn; t += kEwThreads)
        cl[t] = beta0 * y[(size_t)r * ldy + t0 + t] / S.beta[lz_ib(S, r, t0 + t)];
      __syncthreads();
      // four basis vectors' loads in flight, then the sums in t order
      int t = 0;
      for (; t + 3 < tn; t += 4) {
        const T* v0 = V + (size_t)(t0 + t) * vs + voff;
        double x[4][kEwPerThread];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          EW_LOOP(q) {
            const long e = base + (long)q * kEwThreads;
            x[u][q] = (e < len) ? (double)v0[(size_t)u * vs + e] : 0.0;
          }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double ct = cl[t + u];
          EW_LOOP(q) acc[q] += ct * x[u][q];
        }
      }
      for (; t < tn; ++t) {
        const T* vt = V + (size_t)(t0 + t) * vs + voff;
        const double ct = cl[t];
        EW_LOOP(q) {
          const long e = base + (long)q * kEwThreads;
          if (e < len) acc[q] += ct * (double)vt[e];
        }
      }
    }
  }
  const double nanv = __longlong_as_double(0x7ff8000000000000ll);
  EW_LOOP(q) {
    const long e = base + (long)q * kEwThreads;
    if (e < len) out[ooff + e] = (OutT)(bad ? nanv : acc[q]);
  }
}

// FP32 storage with 16-byte aligned columns: the same sums with one float4 load per thread and basis
// vector (1024 elements per block, so short columns of an uneven batch leave few lanes idle) and four
// basis vectors in flight.  Each element still accumulates beta_0 y_t / beta_t v_{t+1}[e] in t order,
// as k_combine does.
#ifndef GMRF_CB_VEC
#define GMRF_CB_VEC 1
#endif
#ifndef GMRF_CB_T
#define GMRF_CB_T 4
#endif
constexpr int kCbVec = GMRF_CB_VEC;                      // float4 loads per thread and basis vector
constexpr int kCbT = GMRF_CB_T;                          // basis vectors in flight
constexpr int kCbChunk = kEwThreads * kCbVec * 4;        // elements per block

template <typename OutT>
__global__ __launch_bounds__(kEwThreads) void k_combine_f32v(const float* __restrict__ V, long L,
                                                             const double* __restrict__ y, int ldy,
                                                             OutT* __restrict__ out, long old, LzState S) {
  __shared__ double cl[1024];
  const int r = blockIdx.y;
  const long len = lz_len(S, r, L);
  if ((long)blockIdx.x * kCbChunk >= len) return;
  const int m = S.m_used[r];
  const int st = S.status[r];
  const double beta0 = S.beta[lz_ib(S, r, 0)];
  const size_t vs = lz_slot(S, L);
  const size_t voff = lz_off(S, r, L);
  const int64_t* ext = S.col_ext ? S.col_ext : S.col_off;
  const size_t ooff = ext ? (size_t)ext[r] : (size_t)r * old;
  const long base = (long)blockIdx.x * kCbChunk + (long)threadIdx.x * 4;
  double acc[kCbVec][4];
#pragma unroll
  for (int q = 0; q < kCbVec; ++q)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[q][i] = 0.0;
  auto load = [&](const float* v, long e) {
    if (e + 3 < len) return *(const float4*)(v + e);
    float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
    if (e < len) x.x = v[e];
    if (e + 1 < len) x.y = v[e + 1];
    if (e + 2 < len) x.z = v[e + 2];
    return x;
  };
  auto add = [&](double c, const float4* x) {
#pragma unroll
    for (int q = 0; q < kCbVec; ++q) {
      acc[q][0] += c * (double)x[q].x;
      acc[q][1] += c * (double)x[q].y;
      acc[q][2] += c * (double)x[q].z;
      acc[q][3] += c * (double)x[q].w;
    }
  };
  const bool bad = (st == kENOTSPD || st == kEINVAL);
  if (!bad) {
    for (int t0 = 0; t0 < m; t0 += 1024) {
      const int tn = min(1024, m - t0);
      __syncthreads();
      for (int t = threadIdx.x; t < tn; t += kEwThreads)
        cl[t] = beta0 * y[(size_t)r * ldy + t0 + t] / S.beta[lz_ib(S, r, t0 + t)];
      __syncthreads();
      int t = 0;
      for (; t + kCbT - 1 < tn; t += kCbT) {
        const float* va = V + (size_t)(t0 + t) * vs + voff;
        float4 xa[kCbT][kCbVec];
#pragma unroll
        for (int u = 0; u < kCbT; ++u)
#pragma unroll
          for (int q = 0; q < kCbVec; ++q) xa[u][q] = load(va + (size_t)u * vs, base + (long)q * kEwThreads * 4);
#pragma unroll
        for (int u = 0; u < kCbT; ++u) add(cl[t + u], xa[u]);
      }
      for (; t < tn; ++t) {
        const float* va = V + (size_t)(t0 + t) * vs + voff;
        float4 xa[kCbVec];
#pragma unroll
        for (int q = 0; q < kCbVec; ++q) xa[q] = load(va, base + (long)q * kEwThreads * 4);
        add(cl[t], xa);
      }
    }
  }
  const double nanv = __longlong_as_double(0x7ff8000000000000ll);
#pragma unroll
  for (int q = 0; q < kCbVec; ++q)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long e = base + (long)q * kEwThreads * 4 + i;
      if (e < len) out[ooff + e] = (OutT)(bad ? nanv : acc[q][i]);
    }
}

// The combine one basis vector at a time (the second pass of the two-pass sampler): with slot t holding
// w_t = beta_t v_{t+1}, out[r] = beta_0 y_0 v_1 for t = 0 and out[r] += beta_0 y_t v_{t+1} for 0 < t < m_used.
// NaN for a column whose status is ENOTSPD or EINVAL, zero for m_used = 0.
template <typename T, typename OutT>
__global__ __launch_bounds__(kEwThreads) void k_accumulate(const T* __restrict__ Vt, long L,
                                                           const double* __restrict__ y, int ldy, LzState S, int t,
                                                           OutT* __restrict__ out, long old) {
  const int r = blockIdx.y;
  const int m = S.m_used[r];
  const int st = S.status[r];
  const bool bad = (st == kENOTSPD || st == kEINVAL);
  if (t > 0 && (bad || t >= m)) return;
  const double c = (bad || t >= m) ? 0.0 : S.beta[lz_ib(S, r, 0)] * y[(size_t)r * ldy + t] / S.beta[lz_ib(S, r, t)];
  const double nanv = __longlong_as_double(0x7ff8000000000000ll);
  const T* v = Vt + (size_t)r * L;
  OutT* o = out + (size_t)r * old;
  const long base = (long)blockIdx.x * kEwChunk + threadIdx.x;
  EW_LOOP(q) {
    const long e = base + (long)q * kEwThreads;
    if (e < L) {
      const double cv = c * (double)v[e];
      o[e] = t == 0 ? (OutT)(bad ? nanv : cv) : (OutT)((double)o[e] + cv);
    }
  }
}

// ---- Hutchinson aggregate (Section 6): Gamma_p = sum_{c < K} ||v_pc||^2 e_1^T log(T_m) e_1 + shift over
// the K colour classes of probe p (columns p K .. p K + K - 1; K = 1 without a colouring, Section 6.1);
// an empty class (||v_pc|| = 0) adds nothing.  out[0] = mean, out[1] = sd / sqrt(N) (NaN for N = 1),
// out[2 + p] = Gamma_p.
__device__ __forceinline__ double probe_gamma(const double* g, const double* beta, int ldb, int p, int K,
                                              double shift) {
  double gam = shift;
  for (int c = 0; c < K; ++c) {
    const int q = p * K + c;
    const double b0 = beta[(size_t)q * ldb];
    if (b0 != 0.0) gam += b0 * b0 * g[q];
  }
  return gam;
}

__global__ __launch_bounds__(256) void k_hutchinson(const double* __restrict__ g, const double* __restrict__ beta,
                                                    int ldb, int np, int K, double shift, double* __restrict__ out) {
  __shared__ double lds[256 / kWave];
  double s = 0.0;
  for (int p = threadIdx.x; p < np; p += 256) {
    const double gam = probe_gamma(g, beta, ldb, p, K, shift);
    out[2 + p] = gam;
    s += gam;
  }
  const double mean = block_sum<256>(s, lds) / np;
  double v = 0.0;
  for (int p = threadIdx.x; p < np; p += 256) {
    const double d = probe_gamma(g, beta, ldb, p, K, shift) - mean;
    v += d * d;
  }
  const double ss = block_sum<256>(v, lds);
  if (threadIdx.x == 0) {
    out[0] = mean;
    out[1] = np > 1 ? sqrt(ss / (np - 1) / np) : __longlong_as_double(0x7ff8000000000000ll);
  }
}

void launch_hutchinson_aggregate(const double* g, const double* beta, int ldb, int np, int K, double shift,
                                 double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_hutchinson, dim3(1), dim3(256), 0, st, g, beta, ldb, np, K, shift, out);
}

// ---- host launchers ---------------------------------------------------------------------------
static inline dim3 ew_grid(long L, int k) { return dim3((unsigned)((L + kEwChunk - 1) / kEwChunk), (unsigned)k); }
// in batch mode L is the longest column; shorter columns' surplus blocks return at once
// Stop poll: out[r] = active[r], out[k + r] = rho_{j-1} of column r, one contiguous block for a single copy.
__global__ __launch_bounds__(256) void k_poll_gather(LzState S, int j, double* __restrict__ out) {
  for (int r = blockIdx.x * 256 + threadIdx.x; r < S.k; r += gridDim.x * 256) {
    out[r] = (double)S.active[r];
    out[S.k + r] = S.rho[lz_ia(S, r, j - 1)];
  }
}

void launch_poll_gather(const LzState& S, int j, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_poll_gather, dim3((unsigned)std::min(64, (S.k + 255) / 256)), dim3(256), 0, st, S, j, out);
}

int ew_blocks(long L) { return (int)((L + kEwChunk - 1) / kEwChunk); }

template <typename T>
void launch_init_from_f64(const double* Z, long zld, long L, T* V0, const LzState& S, hipStream_t st) {
  hipLaunchKernelGGL(k_init_from_f64<T>, ew_grid(L, S.k), dim3(kEwThreads), 0, st, Z, zld, L, V0, S);
}
template <typename T>
void launch_init_from_i8(const int8_t* P, long L, T* V0, const LzState& S, hipStream_t st) {
  hipLaunchKernelGGL(k_init_from_i8<T>, ew_grid(L, S.k), dim3(kEwThreads), 0, st, P, L, V0, S);
}
int rademacher_blocks(long n) {
  const long nb256 = (n + 255) / 256;       // Philox blocks
  const long waves = (nb256 + kWave - 1) / kWave;
  return (int)((waves + 3) / 4);
}
template <typename T>
void launch_init_rademacher(uint64_t seed, long n, int p0, T* V0, const LzState& S, hipStream_t st,
                            const int32_t* colour, int K) {
  hipLaunchKernelGGL(k_init_rademacher<T>, dim3(rademacher_blocks(n), S.k), dim3(256), 0, st, seed, n, p0, V0, S,
                     colour, K);
}
void launch_rademacher_i8(uint64_t seed, long n, int nprobes, int8_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_rademacher_i8, dim3(rademacher_blocks(n), nprobes), dim3(256), 0, st, seed, n, out);
}
template <typename T>
void launch_update(const T* Qb, const T* Vj, T* W, long L, int j, int with_norm, const LzState& S, hipStream_t st) {
  hipLaunchKernelGGL(k_update<T>, ew_grid(L, S.k), dim3(kEwThreads), 0, st, Qb, Vj, W, L, j, with_norm, S);
}
template <typename T>
void launch_norm_partials(const T* V0, long L, const LzState& S, hipStream_t st) {
  hipLaunchKernelGGL(k_norm_partials<T>, ew_grid(L, S.k), dim3(kEwThreads), 0, st, V0, L, S);
}
void launch_finalize(const LzState& S, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(S.k), dim3(256), 0, st, S);
}
int reorth_blocks(long L) { return L <= kRoSmallL ? (int)((L + kRoChunk - 1) / kRoChunk) : ew_blocks(L); }

bool reorth_takes_update(long L) { return L <= kRoSmallL; }

static size_t lz_slot_h(const LzState& S, long L) { return S.slot_stride ? (size_t)S.slot_stride : (size_t)S.k * L; }

template <typename T>
void launch_reorth(T* V, long L, int j, double* part_h, double* h, int hstride, const LzState& S,
                   hipStream_t st, const T* Qb) {
  const dim3 g = ew_grid(L, S.k);
  // t slices for the dot kernel: enough blocks for about two per compute unit, with at least
  // kEwThreads / kWave vectors per slice (one per block for short vectors)
  constexpr int NW = kEwThreads / kWave;
  const bool short_v = L <= kRoSmallL;
  const int tmin = short_v ? 1 : NW;
  const long blocks = (long)g.x * S.k;
  int nz = (int)std::min<long>((j + tmin - 1) / tmin, std::max<long>(1, (512 + blocks - 1) / blocks));
  const int tslice = ((j + nz - 1) / nz + tmin - 1) / tmin * tmin;
  nz = (j + tslice - 1) / tslice;
  const dim3 gd(g.x, g.y, (unsigned)nz);
  const dim3 gu((unsigned)reorth_blocks(L), S.k);
  for (int pass = 0; pass < 2; ++pass) {
    if (short_v)
      hipLaunchKernelGGL(k_reorth_dot_short<T>, gd, dim3(kEwThreads), 0, st, (const T*)V, V + (size_t)j * lz_slot_h(S, L),
                         pass == 0 ? Qb : (const T*)nullptr, L, j, part_h, hstride, tslice, S);
    else
      hipLaunchKernelGGL(k_reorth_dot<T>, gd, dim3(kEwThreads), 0, st, V, L, j, part_h, hstride, tslice, S);
    if (short_v) {
      hipLaunchKernelGGL(k_reorth_update_short<T>, gu, dim3(kRoThreads), 0, st, V, L, j, part_h, hstride,
                         (int)g.x, pass == 1 ? 1 : 0, S);
    } else {
      hipLaunchKernelGGL(k_reorth_reduce, dim3(S.k), dim3(256), 0, st, part_h, hstride, (int)g.x, j, h, S);
      hipLaunchKernelGGL(k_reorth_update<T>, g, dim3(kEwThreads), 0, st, V, L, j, h, hstride,
                         pass == 1 ? 1 : 0, S);
    }
  }
}
template <typename T, typename OutT>
void launch_accumulate(const T* Vt, long L, const double* y, int ldy, const LzState& S, int t, OutT* out, long old,
                       hipStream_t st) {
  hipLaunchKernelGGL((k_accumulate<T, OutT>), ew_grid(L, S.k), dim3(kEwThreads), 0, st, Vt, L, y, ldy, S, t, out, old);
}

template <typename T, typename OutT>
void launch_combine(const T* V, long L, const double* y, int ldy, OutT* out, long old, const LzState& S,
                    hipStream_t st) {
  // float4 loads need every column to start on a 16-byte boundary: batch offsets are padded to four
  // elements, plain columns start at r * L
  if constexpr (sizeof(T) == 4) {
    if ((S.col_off != nullptr || L % 4 == 0) && ((uintptr_t)V & 15) == 0 && ((S.slot_stride ? (size_t)S.slot_stride : (size_t)S.k * (size_t)L) % 4) == 0) {
      const dim3 g((unsigned)((L + kCbChunk - 1) / kCbChunk), S.k);
      hipLaunchKernelGGL((k_combine_f32v<OutT>), g, dim3(kEwThreads), 0, st, (const float*)V, L, y, ldy, out, old, S);
      return;
    }
  }
  hipLaunchKernelGGL((k_combine<T, OutT>), ew_grid(L, S.k), dim3(kEwThreads), 0, st, V, L, y, ldy, out, old, S);
}

#define INST(T)                                                                                  \
  template void launch_init_from_f64<T>(const double*, long, long, T*, const LzState&, hipStream_t); \
  template void launch_init_from_i8<T>(const int8_t*, long, T*, const LzState&, hipStream_t);      \
  template void launch_init_rademacher<T>(uint64_t, long, int, T*, const LzState&, hipStream_t, const int32_t*, int);        \
  template void launch_update<T>(const T*, const T*, T*, long, int, int, const LzState&, hipStream_t); \
  template void launch_norm_partials<T>(const T*, long, const LzState&, hipStream_t);              \
  template void launch_reorth<T>(T*, long, int, double*, double*, int, const LzState&, hipStream_t, const T*); \
  template void launch_combine<T, double>(const T*, long, const double*, int, double*, long,       \
                                          const LzState&, hipStream_t);                           \
  template void launch_accumulate<T, double>(const T*, long, const double*, int, const LzState&, int, double*, \
                                             long, hipStream_t);
INST(double)
INST(float)
#undef INST
template void launch_accumulate<float, float>(const float*, long, const double*, int, const LzState&, int, float*,
                                              long, hipStream_t);
template void launch_combine<float, float>(const float*, long, const double*, int, float*, long,
                                           const LzState&, hipStream_t);

}  // namespace gmrf
