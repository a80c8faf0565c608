// LDS FFT shared by the transform kernels and the preconditioned Lanczos step: Stockham
// autosort (radix-4 stages, one radix-2 stage when log2 N is odd), after Govindaraju et al.,
// "High performance discrete Fourier transforms on graphics processors" (SC'08).  Stage with
// span Ns: item j gathers v_r = x[j + r N/R], multiplies by w^{r (j mod Ns) N/(Ns R)}
// (w = e^{-2 pi i / N}), takes an R-point DFT and scatters y_r to
// x[(j / Ns) Ns R + (j mod Ns) + r Ns].  Each thread stages its items in registers between two
// barriers, so one LDS buffer suffices.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "fft.hpp"

namespace gmrf {

template <typename T> struct C2 { T x, y; };

template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

constexpr int kFftThreads = 1024;
template <typename T> struct FftCfg {
  static constexpr int ELEMS = 65536 / (int)sizeof(C2<T>);          // complex values per block
  static constexpr int MAXIT = ELEMS / (4 * kFftThreads);            // radix-4 items per thread
};

__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }

// nf sequences of length N in LDS: element e of sequence f at buf[f * fs + e * es].
// INTER: items enumerate f fastest (interleaved sequences, es = nf, fs = 1), else e fastest.
// EARLY_TW: each stage requests its twiddles together with its LDS reads, before the barrier, so
// that a twiddle table in global memory costs one latency per stage instead of two.  NT threads; a
// block of NT < kFftThreads threads transforms at most 4 MAXIT NT points (a proportionally smaller
// buffer).
template <typename T, bool INTER, bool EARLY_TW = false, int NT = kFftThreads>
__device__ void lds_fft(C2<T>* buf, int N, int nf, int fs, int es, const C2<T>* __restrict__ tw, bool inv) {
  constexpr int MAXIT = FftCfg<T>::MAXIT;
  const int logN = ilog2(N);
  int Ns = 1;
  const int n4 = N >> 2;
  for (int s = 0; s < logN / 2; ++s) {
    const int items = nf * n4;
    C2<T> v[MAXIT][4];
    C2<T> wv[EARLY_TW ? MAXIT : 1][3];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
      const int item = threadIdx.x + it * NT;
      if (item < items) {
        const int f = INTER ? item % nf : item / n4;
        const int j = INTER ? item / nf : item % n4;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[it][r] = buf[f * fs + (j + r * n4) * es];
        if (EARLY_TW) {
          const int k = j & (Ns - 1);
          const int step = N / (Ns * 4);
#pragma unroll
          for (int r = 1; r < 4; ++r) wv[EARLY_TW ? it : 0][r - 1] = tw[r * k * step];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
      const int item = threadIdx.x + it * NT;
      if (item < items) {
        const int f = INTER ? item % nf : item / n4;
        const int j = INTER ? item / nf : item % n4;
        const int k = j & (Ns - 1);
        const int step = N / (Ns * 4);
#pragma unroll
        for (int r = 1; r < 4; ++r) {
          C2<T> w = EARLY_TW ? wv[EARLY_TW ? it : 0][r - 1] : tw[r * k * step];
          if (inv) w.y = -w.y;
          v[it][r] = cmul(v[it][r], w);
        }
        const C2<T> a0 = v[it][0], a1 = v[it][1], a2 = v[it][2], a3 = v[it][3];
        const C2<T> s02 = {a0.x + a2.x, a0.y + a2.y}, d02 = {a0.x - a2.x, a0.y - a2.y};
        const C2<T> s13 = {a1.x + a3.x, a1.y + a3.y}, d13 = {a1.x - a3.x, a1.y - a3.y};
        // forward: y1 = d02 - i d13, y3 = d02 + i d13; inverse swaps them
        const C2<T> mi = {d13.y, -d13.x};   // -i * d13
        C2<T> y[4];
        y[0] = {s02.x + s13.x, s02.y + s13.y};
        y[2] = {s02.x - s13.x, s02.y - s13.y};
        const C2<T> p = {d02.x + mi.x, d02.y + mi.y}, q = {d02.x - mi.x, d02.y - mi.y};
        y[1] = inv ? q : p;
        y[3] = inv ? p : q;
        const int idxD = (j / Ns) * Ns * 4 + k;
#pragma unroll
        for (int r = 0; r < 4; ++r) buf[f * fs + (idxD + r * Ns) * es] = y[r];
      }
    }
    __syncthreads();
    Ns *= 4;
  }
  if (logN & 1) {
    const int n2 = N >> 1;
    const int items = nf * n2;
    C2<T> v[2 * MAXIT][2];
    C2<T> wv[EARLY_TW ? 2 * MAXIT : 1];
#pragma unroll
    for (int it = 0; it < 2 * MAXIT; ++it) {
      const int item = threadIdx.x + it * NT;
      if (item < items) {
        const int f = INTER ? item % nf : item / n2;
        const int j = INTER ? item / nf : item % n2;
        v[it][0] = buf[f * fs + j * es];
        v[it][1] = buf[f * fs + (j + n2) * es];
        if (EARLY_TW) wv[EARLY_TW ? it : 0] = tw[(j & (Ns - 1)) * (N / (Ns * 2))];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 2 * MAXIT; ++it) {
      const int item = threadIdx.x + it * NT;
      if (item < items) {
        const int f = INTER ? item % nf : item / n2;
        const int j = INTER ? item / nf : item % n2;
        const int k = j & (Ns - 1);
        C2<T> w = EARLY_TW ? wv[EARLY_TW ? it : 0] : tw[k * (N / (Ns * 2))];
        if (inv) w.y = -w.y;
        const C2<T> b = cmul(v[it][1], w), a = v[it][0];
        const int idxD = (j / Ns) * Ns * 2 + k;
        buf[f * fs + idxD * es] = {a.x + b.x, a.y + b.y};
        buf[f * fs + (idxD + Ns) * es] = {a.x - b.x, a.y - b.y};
      }
    }
    __syncthreads();
  }
}

#ifndef GMRF_XCD_COLS
#define GMRF_XCD_COLS 1        // column blocks of one XCD take adjacent columns
#endif
// Column block of launch block b (of nb) in the column passes.  Blocks are dispatched to the 8 XCDs
// round robin (b mod 8); giving the blocks of one XCD consecutive column groups keeps the rows'
// shared 128-byte lines in that XCD's L2 when a block covers fewer columns than a line holds (FP64
// sides of 1024 and more: LGCP column pass 869 -> 565 us at 4096^2, 1208 -> 712 us at 2048^2 x 8).
__device__ __forceinline__ int xcd_col_block(int b, int nb) {
  if (!GMRF_XCD_COLS || (nb & 7) != 0) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// Multiply the LDS tile (columns c0.., row-major [k1][c]) by lambda^{-1/2} * scale.  Column 0 holds
// X[k1, 0] + i X[k1, N2/2]: with m0 = mult(k1, 0), mN = mult(k1, N2/2) and k1' = -k1 mod N1,
//   S'[k1] = (m0 + mN)/2 S[k1] + (m0 - mN)/2 conj(S[k1']).
template <typename T, int NT = kFftThreads>
__device__ void apply_mult(C2<T>* buf, int nf, int c0, int N1, int H, const T* __restrict__ mult, T scale) {
  __syncthreads();
  // at most ELEMS NT / kFftThreads values, a compile-time count per thread: every multiplier load is issued
  // before the first is used (a load behind a bounds branch would wait for its own data)
  constexpr int MI = FftCfg<T>::ELEMS / kFftThreads;
  const int cnt = nf * N1;
  T mv[MI];
#pragma unroll
  for (int it = 0; it < MI; ++it) {
    const int idx = min((int)threadIdx.x + it * NT, cnt - 1);
    const int k1 = idx / nf, cg = c0 + idx % nf;
    mv[it] = mult[(size_t)k1 * mult_stride(H) + cg];
  }
#pragma unroll
  for (int it = 0; it < MI; ++it) {
    const int idx = (int)threadIdx.x + it * NT;
    if (idx >= cnt || c0 + idx % nf == 0) continue;
    const T m = mv[it] * scale;
    buf[idx] = {buf[idx].x * m, buf[idx].y * m};
  }
  if (c0 == 0) {
    for (int k1 = threadIdx.x; k1 <= N1 / 2; k1 += NT) {
      const int kb = (N1 - k1) & (N1 - 1);
      const T m0 = mult[(size_t)k1 * mult_stride(H)] * scale, mN = mult[(size_t)k1 * mult_stride(H) + H] * scale;
      const T p = (m0 + mN) * (T)0.5, q = (m0 - mN) * (T)0.5;
      const C2<T> a = buf[k1 * nf], b = buf[kb * nf];
      buf[k1 * nf] = {p * a.x + q * b.x, p * a.y - q * b.y};
      if (kb != k1) buf[kb * nf] = {p * b.x + q * a.x, p * b.y - q * a.y};
    }
  }
  __syncthreads();
}

}  // namespace gmrf
