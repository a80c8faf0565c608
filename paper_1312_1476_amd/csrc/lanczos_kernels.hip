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
  // every load issued before the first use, from a clamped index (a load behind a bounds branch waits for
  // its own data); only the stores and the sum are masked
  double zv[kEwPerThread];
  EW_LOOP(q) zv[q] = z[min(base + (long)q * kEwThreads, len - 1)];
  EW_LOOP(q) {
    const long e = base + (long)q * kEwThreads;
    const T t = (T)zv[q];
    if (e < len) v[e] = t;
    const double tm = (e < len) ? (double)t : 0.0;   // the operand is masked, so the sum keeps its fused form
    acc += ip_weight(S, e) * tm * tm;
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
  int8_t pv[kEwPerThread];
  EW_LOOP(q) pv[q] = P[(size_t)r * L + min(base + (long)q * kEwThreads, L - 1)];   // clamped, masked below
  EW_LOOP(q) {
    const long e = base + (long)q * kEwThreads;
    const T t = (T)pv[q];
    if (e < L) V0[(size_t)r * L + e] = t;
    const double tm = (e < L) ? (double)t : 0.0;
    acc += tm * tm;
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
  const size_t off = lz_off(S, r, L);
  const T* vj = Vj + off;
  T* w = W + off;
  const T* q = Qb + off;
  const long base = (long)blockIdx.x * kEwChunk + threadIdx.x;
  // the elements' loads go out first, with the scalars' (clamped indices, masked below: a load behind a
  // bounds branch waits for its own data)
  T va[kEwPerThread], qa[kEwPerThread];
  EW_LOOP(qq) {
    const long ec = min(base + (long)qq * kEwThreads, len - 1);
    va[qq] = vj[ec];
    qa[qq] = q[ec];
  }
  double a, bj1;
  if (!lz_update_scalars<kEwThreads>(S, r, j, lds, flag, a, bj1)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) S.alpha[lz_ia(S, r, j)] = a;
  const double sc = 1.0 / bj1;
  double acc = 0.0;
  EW_LOOP(qq) {
    const long e = base + (long)qq * kEwThreads;
    const double v = (double)(T)((double)va[qq] * sc);
    const T t = (T)((double)qa[qq] - a * v);
    if (e < len) w[e] = t;
    const double tm = (e < len) ? (double)t : 0.0;   // the operand is masked, so the sum keeps its fused form
    acc += ip_weight(S, e) * tm * tm;
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
  double tv[kEwPerThread];
  EW_LOOP(q) tv[q] = (double)V0[(size_t)r * L + min(base + (long)q * kEwThreads, L - 1)];   // clamped, masked below
  EW_LOOP(q) {
    const long e = base + (long)q * kEwThreads;
    const double tm = (e < L) ? tv[q] : 0.0;
    acc += ip_weight(S, e) * tm * tm;
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
  // loads from clamped indices, masked in the sums (a load behind a bounds branch waits for its own data)
  double acc[kEwPerThread];
  EW_LOOP(q) acc[q] = (double)w[min(base + (long)q * kEwThreads, L - 1)];
  for (int t0 = 0; t0 < j; t0 += 1024) {
    const int tn = min(1024, j - t0);
    __syncthreads();
    for (int t = threadIdx.x; t < tn; t += kEwThreads) cl[t] = h[(size_t)r * hstride + t0 + t];
    __syncthreads();
    for (int t = 0; t < tn; ++t) {
      const T* vt = V + (size_t)(t0 + t) * vs + (size_t)r * L;
      const double sc = 1.0 / S.beta[lz_ib(S, r, t0 + t)];
      const double ht = cl[t];
      double xv[kEwPerThread];
      EW_LOOP(q) xv[q] = (double)vt[min(base + (long)q * kEwThreads, L - 1)];
      EW_LOOP(q) acc[q] -= ht * ((base + (long)q * kEwThreads < L) ? (double)(T)(xv[q] * sc) : 0.0);
    }
  }
  double nrm = 0.0;
  EW_LOOP(q) {
    const long e = base + (long)q * kEwThreads;
    const T t = (T)acc[q];
    if (e < L) w[e] = t;
    const double tm = (e < L) ? (double)t : 0.0;
    nrm += ip_weight(S, e) * tm * tm;
  }
  if (with_norm) {
    const double s = block_sum<kEwThreads>(nrm, lds);
    if (threadIdx.x == 0) S.part_b[(size_t)r * S.pstride + blockIdx.x] = s;
  }
}

// Short vectors (L <= kRoSmallL): block (x, r) owns chunk x of column r, the kWave * EPL elements
// e = x * kWave * EPL + i * kWave + lane (i < EPL), and takes every basis vector over it; wave g of the
// block takes the basis vectors t = t0 + g + 8 u (u < 16) of each sweep of 128.  The update of one pass and
// the dots of the next then touch only the block's own elements and share one launch, so one step of CGS2
// is three launches:
//   MODE 0  the dots h_t = v_{t+1}^T w, t < j, of w = slot j; given q, w is first formed here as
//           w_j = q - alpha_j v_j from the operator's partial sums (the update step of Algorithm 1);
//   MODE 1  w -= sum_t h_t v_{t+1}, h_t the sum of MODE 0's block partials, then the dots of the result
//           (the second pass);
//   MODE 2  the same update with the second pass's h_t, then the partial sums of ||w||^2.
// Each launch re-reads its share of the basis and the other blocks' dot partials from beyond L2 (on a 64^2
// lattice about 80 KB per block at j = 81), so every load a sweep needs is issued at its start, and with
// j <= 128 the dots of MODE 1 take the basis values its update loaded: one round of loads per launch.  The
// 64-element chunks balance the two kinds of traffic (8 j (L / P + P) bytes per block, least at P = sqrt L).
// Sums over lanes take the 16 values of a wave's share at once (wave_sum16: lane swaps and DPP permutes; a
// select between register-array elements chosen by lane compiles to compare-and-select chains).  An element's update is summed per wave in t order, then over the waves in
// wave order through LDS.  Every sum has a fixed order, so results are bitwise reproducible.
constexpr int kCsThreads = 512;
constexpr int kCsWaves = kCsThreads / kWave;
constexpr int kCsGroup = 16;                   // basis vectors per wave and sweep (values folded together)
constexpr int kCsSpan = kCsWaves * kCsGroup;   // basis vectors per sweep
constexpr long kRoSmallL = 16384;
constexpr int kCsMaxChunks = 128;              // chunks per column (partials per h_t: at most two per lane)

// Elements per lane and basis vector: chunks as small as kCsMaxChunks allows.
int cgs_epl(long L) { return L <= (long)kWave * kCsMaxChunks ? 1 : 2; }

// The basis values (clamped indices, masked where used) of wave gu's share of the sweep at t0, and beta_t of
// its basis vector u = lane & 15 (a vector load issued with the others; lanes take 1 / beta by shuffles).
template <typename T, int EPL>
__device__ __forceinline__ void cgs_load(const T* Vr, size_t vs, long L, long base, int lane, int gu, int t0, int j,
                                         const LzState& S, int r, double (&vv)[kCsGroup][EPL], double& bl) {
  bl = S.beta[lz_ib(S, r, min(t0 + gu + (lane & (kCsGroup - 1)) * kCsWaves, j - 1))];
#pragma unroll
  for (int u = 0; u < kCsGroup; ++u) {
    const int tc = min(t0 + gu + u * kCsWaves, j - 1);
#pragma unroll
    for (int i = 0; i < EPL; ++i) vv[u][i] = (double)Vr[(size_t)tc * vs + min(base + i * kWave + lane, L - 1)];
  }
}

// Partials of the sweep's h_t (lane l holds block partials l and l + 64), summed after the loads are issued.
__device__ __forceinline__ void cgs_load_h(const double* pin, int hstride, int P, int r, int lane, int gu, int t0,
                                           int j, double (&p)[kCsGroup]) {
  double pv[2][kCsGroup];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int u = 0; u < kCsGroup; ++u) {
      const int tc = min(t0 + gu + u * kCsWaves, j - 1);
      pv[q][u] = pin[((size_t)r * hstride + tc) * P + min(lane + q * kWave, P - 1)];
    }
#pragma unroll
  for (int u = 0; u < kCsGroup; ++u) {
    p[u] = (lane < P) ? pv[0][u] : 0.0;
    p[u] += (lane + kWave < P) ? pv[1][u] : 0.0;
  }
}

template <typename T, int EPL, int MODE>
__global__ __launch_bounds__(kCsThreads) void k_cgs_short(T* __restrict__ V, const T* __restrict__ Qb, long L, int j,
                                                          const double* __restrict__ pin, double* __restrict__ pout,
                                                          int hstride, LzState S) {
  constexpr int kChunk = kWave * EPL;
  __shared__ double red[kCsWaves][kChunk];
  __shared__ double wl[kChunk];   // the weighted w the dots take
  __shared__ double lds[kCsWaves];
  const int r = blockIdx.y;
  const int act = S.active[r];    // not written during the reorthogonalisation: the same on every thread
  const int P = (int)gridDim.x, x = (int)blockIdx.x;
  const int tid = (int)threadIdx.x, lane = tid & (kWave - 1);
  const int gu = __builtin_amdgcn_readfirstlane(tid / kWave);
  const size_t vs = lz_slot(S, L);
  const T* Vr = V + (size_t)r * L;
  T* w = V + (size_t)j * vs + (size_t)r * L;
  const long base = (long)x * kChunk;
  const long eo = base + tid;                 // the element thread tid < kChunk writes
  const long ec = min(eo, L - 1);
  double vv[kCsGroup][EPL], bl;
  if constexpr (MODE == 0) {
    cgs_load<T, EPL>(Vr, vs, L, base, lane, gu, 0, j, S, r, vv, bl);
    if (!act) return;
    if (Qb) {
      const double bprev = S.beta[lz_ib(S, r, j - 1)];
      const double vj = (double)V[(size_t)(j - 1) * vs + (size_t)r * L + ec];
      const double qv = (double)Qb[(size_t)r * L + ec];
      const double a = sum_partials<kCsThreads>(S.part_a + (size_t)r * S.pstride, lz_pa(S, r), lds);
      if (x == 0 && tid == 0) S.alpha[lz_ia(S, r, j)] = a;
      if (tid < kChunk) {
        double wt = 0.0;
        if (eo < L) {
          const double v = (double)(T)(vj * (1.0 / bprev));
          const T t = (T)(qv - a * v);
          w[eo] = t;
          wt = ip_weight(S, eo) * (double)t;
        }
        wl[tid] = wt;
      }
    } else {
      const double wv0 = (double)w[ec];
      if (tid < kChunk) wl[tid] = (eo < L) ? ip_weight(S, eo) * wv0 : 0.0;
    }
  } else {
    const double w0 = (double)w[ec];
    double acc[EPL];
#pragma unroll
    for (int i = 0; i < EPL; ++i) acc[i] = 0.0;
    for (int t0 = 0; t0 < j; t0 += kCsSpan) {
      double p[kCsGroup];
      cgs_load<T, EPL>(Vr, vs, L, base, lane, gu, t0, j, S, r, vv, bl);
      cgs_load_h(pin, hstride, P, r, lane, gu, t0, j, p);
      if (!act) return;
      wave_sum16(p);
      const double il = 1.0 / bl;
#pragma unroll
      for (int u = 0; u < kCsGroup; ++u) {
        const double h = lane_read(p[u & 3], 16 * (u >> 2));
        const bool ok = t0 + gu + u * kCsWaves < j;
        const double s = lane_read(il, u);
#pragma unroll
        for (int i = 0; i < EPL; ++i) acc[i] += (ok && base + i * kWave + lane < L) ? h * (double)(T)(vv[u][i] * s) : 0.0;
      }
    }
#pragma unroll
    for (int i = 0; i < EPL; ++i) red[gu][i * kWave + lane] = acc[i];
    __syncthreads();
    double nrm = 0.0;
    if (tid < kChunk) {
      double s = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < kCsWaves; ++w2) s += red[w2][tid];
      double wt = 0.0;
      if (eo < L) {
        const T t = (T)(w0 - s);
        w[eo] = t;
        const double q = ip_weight(S, eo);
        wt = q * (double)t;
        nrm = q * (double)t * (double)t;
      }
      wl[tid] = wt;
    }
    if constexpr (MODE == 2) {
      const double s = block_sum<kCsThreads>(nrm, lds);
      if (tid == 0) S.part_b[(size_t)r * S.pstride + x] = s;
      return;
    }
  }
  if constexpr (MODE != 2) {
    __syncthreads();
    double wv[EPL];
#pragma unroll
    for (int i = 0; i < EPL; ++i) wv[i] = wl[i * kWave + lane];
    for (int t0 = 0; t0 < j; t0 += kCsSpan) {
      // the values of the last sweep are still in registers when there was only one (MODE 0: the first)
      if ((MODE == 0 && t0 > 0) || (MODE == 1 && j > kCsSpan)) cgs_load<T, EPL>(Vr, vs, L, base, lane, gu, t0, j, S, r, vv, bl);
      const double il = 1.0 / bl;
      double p[kCsGroup];
#pragma unroll
      for (int u = 0; u < kCsGroup; ++u) {
        const bool ok = t0 + gu + u * kCsWaves < j;
        const double s = lane_read(il, u);
        p[u] = 0.0;
#pragma unroll
        for (int i = 0; i < EPL; ++i) p[u] += ok ? (double)(T)(vv[u][i] * s) * wv[i] : 0.0;
      }
      wave_sum16(p);
      // lane i < 4 of row q writes value 4 q + i
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t = t0 + gu + (4 * (lane >> 4) + i) * kCsWaves;
        if ((lane & 15) == i && t < j) pout[((size_t)r * hstride + t) * P + x] = p[i];
      }
    }
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
        // clamped indices, masked in the sums (a load behind a bounds branch waits for its own data)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          EW_LOOP(q) x[u][q] = (double)v0[(size_t)u * vs + min(base + (long)q * kEwThreads, len - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double ct = cl[t + u];
          EW_LOOP(q) acc[q] += ct * ((base + (long)q * kEwThreads < len) ? x[u][q] : 0.0);   // fused, as before
        }
      }
      for (; t < tn; ++t) {
        const T* vt = V + (size_t)(t0 + t) * vs + voff;
        const double ct = cl[t];
        double xt[kEwPerThread];
        EW_LOOP(q) xt[q] = (double)vt[min(base + (long)q * kEwThreads, len - 1)];
        EW_LOOP(q) acc[q] += ct * ((base + (long)q * kEwThreads < len) ? xt[q] : 0.0);
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
  // both loads of every element issued first, from clamped indices (a load behind a bounds branch waits for
  // its own data); only the stores are masked
  double vv[kEwPerThread], ov[kEwPerThread];
  EW_LOOP(q) vv[q] = (double)v[min(base + (long)q * kEwThreads, L - 1)];
  if (t > 0) {
    EW_LOOP(q) ov[q] = (double)o[min(base + (long)q * kEwThreads, L - 1)];
  } else {
    EW_LOOP(q) ov[q] = 0.0;
  }
  EW_LOOP(q) {
    const long e = base + (long)q * kEwThreads;
    const double cv = c * vv[q];
    const OutT res = t == 0 ? (OutT)(bad ? nanv : cv) : (OutT)(ov[q] + cv);
    if (e < L) o[e] = res;
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
int reorth_blocks(long L) {
  return L <= kRoSmallL ? (int)((L + (long)kWave * cgs_epl(L) - 1) / ((long)kWave * cgs_epl(L))) : ew_blocks(L);
}

bool reorth_takes_update(long L) { return L <= kRoSmallL; }

int reorth_partial_sets(long L) { return L <= kRoSmallL ? 2 : 1; }

template <typename T, int EPL>
static void launch_cgs_short(T* V, long L, int j, double* ph0, double* ph1, int hstride, const LzState& S,
                             hipStream_t st, const T* Qb) {
  const dim3 g((unsigned)reorth_blocks(L), S.k);
  hipLaunchKernelGGL((k_cgs_short<T, EPL, 0>), g, dim3(kCsThreads), 0, st, V, Qb, L, j, (const double*)nullptr, ph0,
                     hstride, S);
  hipLaunchKernelGGL((k_cgs_short<T, EPL, 1>), g, dim3(kCsThreads), 0, st, V, (const T*)nullptr, L, j,
                     (const double*)ph0, ph1, hstride, S);
  hipLaunchKernelGGL((k_cgs_short<T, EPL, 2>), g, dim3(kCsThreads), 0, st, V, (const T*)nullptr, L, j,
                     (const double*)ph1, (double*)nullptr, hstride, S);
}

template <typename T>
void launch_reorth(T* V, long L, int j, double* part_h, double* h, int hstride, const LzState& S,
                   hipStream_t st, const T* Qb) {
  if (L <= kRoSmallL) {
    // two sets of partials, [k][hstride][P] each: the first pass's dots and the second's
    double* ph1 = part_h + (size_t)S.k * hstride * reorth_blocks(L);
    if (cgs_epl(L) == 1) launch_cgs_short<T, 1>(V, L, j, part_h, ph1, hstride, S, st, Qb);
    else launch_cgs_short<T, 2>(V, L, j, part_h, ph1, hstride, S, st, Qb);
    return;
  }
  const dim3 g = ew_grid(L, S.k);
  // t slices for the dot kernel: enough blocks for about two per compute unit, with at least
  // kEwThreads / kWave vectors per slice
  constexpr int NW = kEwThreads / kWave;
  const long blocks = (long)g.x * S.k;
  int nz = (int)std::min<long>((j + NW - 1) / NW, std::max<long>(1, (512 + blocks - 1) / blocks));
  const int tslice = ((j + nz - 1) / nz + NW - 1) / NW * NW;
  nz = (j + tslice - 1) / tslice;
  const dim3 gd(g.x, g.y, (unsigned)nz);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_reorth_dot<T>, gd, dim3(kEwThreads), 0, st, V, L, j, part_h, hstride, tslice, S);
    hipLaunchKernelGGL(k_reorth_reduce, dim3(S.k), dim3(256), 0, st, part_h, hstride, (int)g.x, j, h, S);
    hipLaunchKernelGGL(k_reorth_update<T>, g, dim3(kEwThreads), 0, st, V, L, j, h, hstride, pass == 1 ? 1 : 0, S);
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
