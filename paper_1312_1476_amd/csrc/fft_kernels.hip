// 2D FFT kernels of the block-circulant preconditioner (Proposition 1, Section 5.1), in the
// packed half-spectrum layout described in fft.hpp.  Power-of-two sides N1, N2 in [8, 4096].
//
// LDS FFT: Stockham autosort (radix-4 stages, one radix-2 stage when log2 N is odd), after
// Govindaraju et al., "High performance discrete Fourier transforms on graphics processors"
// (SC'08).  Stage with span Ns: item j gathers v_r = x[j + r N/R], multiplies by
// w^{r (j mod Ns) N/(Ns R)} (w = e^{-2 pi i / N}), takes an R-point DFT and scatters y_r to
// x[(j / Ns) Ns R + (j mod Ns) + r Ns].  Each thread stages its items in registers between
// two barriers, so one LDS buffer suffices.
//
// Row pass: two real rows a, b form one complex sequence a + i b; one length-N2 FFT gives both
// half spectra, A_k = (Z_k + conj Z_{N-k}) / 2 and B_k = -i (Z_k - conj Z_{N-k}) / 2.
// Column pass: nf packed columns of one field per block, LDS laid out row-major [k1][c] so
// global loads and LDS traffic stay contiguous; the diagonal multiplier and the Lanczos
// epilogue are fused into it.
#include "fft.hpp"

#include <cmath>
#include <vector>

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
template <typename T, bool INTER>
__device__ void lds_fft(C2<T>* buf, int N, int nf, int fs, int es, const C2<T>* __restrict__ tw, bool inv) {
  constexpr int MAXIT = FftCfg<T>::MAXIT;
  const int logN = ilog2(N);
  int Ns = 1;
  const int n4 = N >> 2;
  for (int s = 0; s < logN / 2; ++s) {
    const int items = nf * n4;
    C2<T> v[MAXIT][4];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
      const int item = threadIdx.x + it * kFftThreads;
      if (item < items) {
        const int f = INTER ? item % nf : item / n4;
        const int j = INTER ? item / nf : item % n4;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[it][r] = buf[f * fs + (j + r * n4) * es];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
      const int item = threadIdx.x + it * kFftThreads;
      if (item < items) {
        const int f = INTER ? item % nf : item / n4;
        const int j = INTER ? item / nf : item % n4;
        const int k = j & (Ns - 1);
        const int step = N / (Ns * 4);
#pragma unroll
        for (int r = 1; r < 4; ++r) {
          C2<T> w = tw[r * k * step];
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
#pragma unroll
    for (int it = 0; it < 2 * MAXIT; ++it) {
      const int item = threadIdx.x + it * kFftThreads;
      if (item < items) {
        const int f = INTER ? item % nf : item / n2;
        const int j = INTER ? item / nf : item % n2;
        v[it][0] = buf[f * fs + j * es];
        v[it][1] = buf[f * fs + (j + n2) * es];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 2 * MAXIT; ++it) {
      const int item = threadIdx.x + it * kFftThreads;
      if (item < items) {
        const int f = INTER ? item % nf : item / n2;
        const int j = INTER ? item / nf : item % n2;
        const int k = j & (Ns - 1);
        C2<T> w = tw[k * (N / (Ns * 2))];
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

// ---- row passes ----------------------------------------------------------------------------------
// Real rows (N1 x N2 per field, field r at in + r * ild) -> packed rows (N1 x H complex, field r at
// out + r * old complex), scaled by `scale`.
template <typename Tin, typename T>
__global__ __launch_bounds__(kFftThreads) void k_rows_r2c(const Tin* __restrict__ in, long ild,
                                                          C2<T>* __restrict__ out, long old, int N1, int N2,
                                                          int np, const C2<T>* __restrict__ tw, T scale,
                                                          const int* __restrict__ active) {
  __shared__ C2<T> buf[FftCfg<T>::ELEMS];
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int H = N2 / 2;
  const int row0 = 2 * np * blockIdx.x;
  const Tin* src = in + (size_t)r * ild;
  for (int idx = threadIdx.x; idx < np * N2; idx += kFftThreads) {
    const int p = idx / N2, t = idx % N2;
    const size_t ra = (size_t)(row0 + 2 * p) * N2;
    buf[p * N2 + t] = {(T)src[ra + t], (T)src[ra + N2 + t]};
  }
  __syncthreads();
  lds_fft<T, false>(buf, N2, np, N2, 1, tw, false);
  C2<T>* dst = out + (size_t)r * old;
  const T h = (T)0.5 * scale;
  for (int idx = threadIdx.x; idx < np * H; idx += kFftThreads) {
    const int p = idx / H, c = idx % H;
    const C2<T>* Z = buf + p * N2;
    C2<T> pa, pb;
    if (c == 0) {
      const C2<T> z0 = Z[0], zn = Z[H];
      pa = {z0.x * scale, zn.x * scale};
      pb = {z0.y * scale, zn.y * scale};
    } else {
      const C2<T> zk = Z[c], zm = Z[N2 - c];
      // A = (zk + conj zm) / 2, B = -i (zk - conj zm) / 2
      pa = {(zk.x + zm.x) * h, (zk.y - zm.y) * h};
      pb = {(zk.y + zm.y) * h, (zm.x - zk.x) * h};
    }
    dst[(size_t)(row0 + 2 * p) * H + c] = pa;
    dst[(size_t)(row0 + 2 * p + 1) * H + c] = pb;
  }
}

// Packed rows -> real rows (unnormalised inverse, times `scale`).
template <typename T, typename Tout>
__global__ __launch_bounds__(kFftThreads) void k_rows_c2r(const C2<T>* __restrict__ in, long ild,
                                                          Tout* __restrict__ out, long old, int N1, int N2,
                                                          int np, const C2<T>* __restrict__ tw, T scale,
                                                          const int* __restrict__ active) {
  __shared__ C2<T> buf[FftCfg<T>::ELEMS];
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int H = N2 / 2;
  const int row0 = 2 * np * blockIdx.x;
  const C2<T>* src = in + (size_t)r * ild;
  for (int idx = threadIdx.x; idx < np * N2; idx += kFftThreads) {
    const int p = idx / N2, k = idx % N2;
    const C2<T>* PA = src + (size_t)(row0 + 2 * p) * H;
    const C2<T>* PB = PA + H;
    C2<T> a, b;
    if (k == 0) {
      a = {PA[0].x, (T)0};
      b = {PB[0].x, (T)0};
    } else if (k == H) {
      a = {PA[0].y, (T)0};
      b = {PB[0].y, (T)0};
    } else if (k < H) {
      a = PA[k];
      b = PB[k];
    } else {
      a = {PA[N2 - k].x, -PA[N2 - k].y};
      b = {PB[N2 - k].x, -PB[N2 - k].y};
    }
    buf[p * N2 + k] = {a.x - b.y, a.y + b.x};   // A + i B
  }
  __syncthreads();
  lds_fft<T, false>(buf, N2, np, N2, 1, tw, true);
  Tout* dst = out + (size_t)r * old;
  for (int idx = threadIdx.x; idx < np * N2; idx += kFftThreads) {
    const int p = idx / N2, t = idx % N2;
    const size_t ra = (size_t)(row0 + 2 * p) * N2;
    const C2<T> z = buf[p * N2 + t];
    dst[ra + t] = (Tout)(z.x * scale);
    dst[ra + N2 + t] = (Tout)(z.y * scale);
  }
}

// ---- column pass -------------------------------------------------------------------------------------
enum ColMode : int {
  kColFwdInit = 0,   // FFT, times scale                                  (z_hat = F z)
  kColFwdLz = 1,     // FFT, times lambda^{-1/2}, Lanczos epilogue          (operator, second half)
  kColInvLz = 2,     // opener; v_j times lambda^{-1/2} scale, inverse FFT  (operator, first half)
  kColInvOut = 3,    // times lambda^{-1/2} scale, inverse FFT              (x = F^H Lambda^{-1/2} u)
  kColApply = 4      // FFT, times lambda^{-1/2} scale, inverse FFT         (M^{-1/2} on its own)
};

// Multiply the LDS tile (columns c0.., row-major [k1][c]) by lambda^{-1/2} * scale.  Column 0 holds
// X[k1, 0] + i X[k1, N2/2]: with m0 = mult(k1, 0), mN = mult(k1, N2/2) and k1' = -k1 mod N1,
//   S'[k1] = (m0 + mN)/2 S[k1] + (m0 - mN)/2 conj(S[k1']).
template <typename T>
__device__ void apply_mult(C2<T>* buf, int nf, int c0, int N1, int H, const T* __restrict__ mult, T scale) {
  __syncthreads();
  for (int idx = threadIdx.x; idx < nf * N1; idx += kFftThreads) {
    const int k1 = idx / nf, c = idx % nf, cg = c0 + c;
    if (cg == 0) continue;
    const T m = mult[(size_t)k1 * (H + 1) + cg] * scale;
    buf[idx] = {buf[idx].x * m, buf[idx].y * m};
  }
  if (c0 == 0) {
    for (int k1 = threadIdx.x; k1 <= N1 / 2; k1 += kFftThreads) {
      const int kb = (N1 - k1) & (N1 - 1);
      const T m0 = mult[(size_t)k1 * (H + 1)] * scale, mN = mult[(size_t)k1 * (H + 1) + H] * scale;
      const T p = (m0 + mN) * (T)0.5, q = (m0 - mN) * (T)0.5;
      const C2<T> a = buf[k1 * nf], b = buf[kb * nf];
      buf[k1 * nf] = {p * a.x + q * b.x, p * a.y - q * b.y};
      if (kb != k1) buf[kb * nf] = {p * b.x + q * a.x, p * b.y - q * a.y};
    }
  }
  __syncthreads();
}

// Band-pass hand-off between the two column passes of the preconditioned operator.
//   pband[((rhs * N1 + row) * ntiles + tile) * 4 + t]: per column tile, the partial sums of
//     u(row, {0, 1, N2-2, N2-1}[t]) over the tile's packed columns (written by the opener);
//   edge_in[(rhs * 6 + q) * H + c]: packed row spectra of u for rows {0,1,2,N1-3,N1-2,N1-1};
//   bcoef[(rhs * N1 + row) * 2 + {0,1}]: (d0, d1) of interior rows (written by the band pass);
//   edge_out[(rhs * 4 + q) * H + c]: packed row spectra of D u for rows {0,1,N1-2,N1-1}.
template <typename T>
struct BandIO {
  const C2<T>* tw2;        // N2-point twiddles
  double* pband;
  C2<T>* edge_in;
  double* bcoef;
  C2<T>* edge_out;
};

__device__ __forceinline__ int edge_in_slot(int row, int N1) {
  return row <= 2 ? row : (row >= N1 - 3 ? row - (N1 - 6) : -1);
}
__device__ __forceinline__ int edge_out_slot(int row, int N1) {
  return row <= 1 ? row : (row >= N1 - 2 ? row - (N1 - 4) : -1);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kFftThreads) void k_cols(const C2<T>* __restrict__ in, C2<T>* __restrict__ out,
                                                      int N1, int H, int nf, const C2<T>* __restrict__ tw,
                                                      const T* __restrict__ mult, T scale, LzState S, int j,
                                                      const C2<T>* __restrict__ Xj, const C2<T>* __restrict__ Xprev,
                                                      BandIO<T> bio) {
  __shared__ C2<T> buf[FftCfg<T>::ELEMS];
  __shared__ double red[kFftThreads / kWave];
  __shared__ int flag[1];
  // per-column coefficients of the band hand-off (tiles of at most kCoefCols columns use them)
  constexpr int kCoefCols = 64;
  __shared__ C2<T> coefA[(MODE == kColFwdLz) ? kCoefCols : 1], coefB[(MODE == kColFwdLz) ? kCoefCols : 1];
  __shared__ double coefW[(MODE == kColInvLz) ? 8 * kCoefCols : 1];
  const int r = blockIdx.y;
  const int c0 = blockIdx.x * nf;
  const size_t fsz = (size_t)N1 * H;   // complex values per field
  double s_cur = 1.0, s_prev = 0.0, bprev = 0.0;
  if (MODE == kColInvLz) {
    if (!lz_open<kFftThreads>(S, r, j, blockIdx.x == 0, red, flag, s_cur, s_prev, bprev)) return;
  } else if (MODE == kColFwdLz) {
    if (!block_active(S, r, flag)) return;
    s_cur = 1.0 / S.beta[lz_ib(S, r, j - 1)];
    if (j > 1) {
      s_prev = 1.0 / S.beta[lz_ib(S, r, j - 2)];
      bprev = S.beta[lz_ib(S, r, j - 1)];
    }
  }
  const C2<T>* src = in + (size_t)r * fsz;
  const bool use_coef = nf <= kCoefCols;
  if (MODE == kColFwdLz && bio.bcoef) {
    // row spectra of D u: closed form X_c = d0 A_c + d1 B_c on interior rows, with
    // A_c = 1 - conj w^c, B_c = w^c - conj w^{2c} (A_0 = 2i, B_0 = -2i covers X_{N2/2} = 2(d0 - d1));
    // stored spectra on the edge rows
    auto coef = [&](int cg, C2<T>& A, C2<T>& Bc) {
      if (cg == 0) {
        A = {(T)0, (T)2};
        Bc = {(T)0, (T)-2};
      } else {
        const C2<T> w1 = bio.tw2[cg], w2 = bio.tw2[2 * cg];
        A = {(T)1 - w1.x, w1.y};
        Bc = {w1.x - w2.x, w1.y + w2.y};
      }
    };
    if (use_coef) {
      for (int c = threadIdx.x; c < nf; c += kFftThreads) coef(c0 + c, coefA[c], coefB[c]);
      __syncthreads();
    }
    for (int idx = threadIdx.x; idx < nf * N1; idx += kFftThreads) {
      const int k1 = idx / nf, c = idx % nf, cg = c0 + c;
      const int q = edge_out_slot(k1, N1);
      C2<T> v;
      if (q >= 0) {
        v = bio.edge_out[((size_t)r * 4 + q) * H + cg];
      } else {
        const double d0 = bio.bcoef[((size_t)r * N1 + k1) * 2], d1 = bio.bcoef[((size_t)r * N1 + k1) * 2 + 1];
        C2<T> A, Bc;
        if (use_coef) {
          A = coefA[c];
          Bc = coefB[c];
        } else {
          coef(cg, A, Bc);
        }
        v = {(T)(d0 * (double)A.x + d1 * (double)Bc.x), (T)(d0 * (double)A.y + d1 * (double)Bc.y)};
      }
      buf[idx] = v;
    }
  } else {
    for (int idx = threadIdx.x; idx < nf * N1; idx += kFftThreads) {
      const int k1 = idx / nf, c = idx % nf;
      C2<T> v = src[(size_t)k1 * H + c0 + c];
      if (MODE == kColInvLz) v = {(T)((double)v.x * s_cur), (T)((double)v.y * s_cur)};
      buf[idx] = v;
    }
  }
  if (MODE == kColInvLz || MODE == kColInvOut) apply_mult(buf, nf, c0, N1, H, mult, scale);
  else __syncthreads();
  const bool inverse_first = (MODE == kColInvLz || MODE == kColInvOut);
  lds_fft<T, true>(buf, N1, nf, 1, nf, tw, inverse_first);
  if (MODE == kColApply) {
    apply_mult(buf, nf, c0, N1, H, mult, scale);
    lds_fft<T, true>(buf, N1, nf, 1, nf, tw, true);
  }
  if (MODE == kColFwdLz) apply_mult(buf, nf, c0, N1, H, mult, (T)1);
  if (MODE == kColInvLz && bio.pband) {
    // u at columns {0, 1, N2-2, N2-1} from this tile's packed columns:
    //   X_0 + (-1)^t X_{N2/2} (column 0), 2 Re(X_c e^{+2 pi i c t / N2}) (columns c >= 1)
    const int ntiles = gridDim.x;
    // contribution of column cg to u(., t) is a px + b py with (a, b) = weight(cg, t)
    auto weight = [&](int cg, int t, double& a, double& b) {
      if (cg == 0) {
        a = 1.0;
        b = (t & 1) ? -1.0 : 1.0;
      } else {
        const C2<T> w1 = bio.tw2[cg], w2 = bio.tw2[2 * cg];
        if (t == 0) { a = 2.0; b = 0.0; }
        else if (t == 1) { a = 2.0 * (double)w1.x; b = 2.0 * (double)w1.y; }
        else if (t == 2) { a = 2.0 * (double)w2.x; b = -2.0 * (double)w2.y; }
        else { a = 2.0 * (double)w1.x; b = -2.0 * (double)w1.y; }
      }
    };
    if (use_coef) {
      for (int item = threadIdx.x; item < 4 * nf; item += kFftThreads) {
        const int t = item / nf, c = item % nf;
        weight(c0 + c, t, coefW[2 * item], coefW[2 * item + 1]);
      }
      __syncthreads();
    }
    for (int item = threadIdx.x; item < N1 * 4; item += kFftThreads) {
      const int k1 = item >> 2, t = item & 3;
      double acc = 0.0;
      for (int c = 0; c < nf; ++c) {
        const C2<T> x = buf[k1 * nf + c];
        double a, b;
        if (use_coef) {
          a = coefW[2 * (t * nf + c)];
          b = coefW[2 * (t * nf + c) + 1];
        } else {
          weight(c0 + c, t, a, b);
        }
        acc += a * (double)x.x + b * (double)x.y;
      }
      bio.pband[(((size_t)r * N1 + k1) * ntiles + blockIdx.x) * 4 + t] = acc;
    }
    for (int idx = threadIdx.x; idx < 6 * nf; idx += kFftThreads) {
      const int q = idx / nf, c = idx % nf;
      const int k1 = q < 3 ? q : N1 - 6 + q;
      bio.edge_in[((size_t)r * 6 + q) * H + c0 + c] = buf[k1 * nf + c];
    }
    return;
  }
  C2<T>* dst = out + (size_t)r * fsz;
  if (MODE == kColFwdLz) {
    const C2<T>* vj = Xj + (size_t)r * fsz;
    const C2<T>* vp = Xprev + (size_t)r * fsz;
    double acc = 0.0;
    for (int idx = threadIdx.x; idx < nf * N1; idx += kFftThreads) {
      const int k1 = idx / nf, c = idx % nf;
      const size_t gi = (size_t)k1 * H + c0 + c;
      const C2<T> a = buf[idx];   // Lambda^{-1/2} F D F^H Lambda^{-1/2} v_j
      const C2<T> v = vj[gi];
      const double vx = (double)(T)((double)v.x * s_cur), vy = (double)(T)((double)v.y * s_cur);
      double qx = vx - (double)a.x, qy = vy - (double)a.y;   // A v_j = v_j - (...)
      if (j > 1) {
        const C2<T> p = vp[gi];
        qx -= bprev * (double)(T)((double)p.x * s_prev);
        qy -= bprev * (double)(T)((double)p.y * s_prev);
      }
      const C2<T> qt = {(T)qx, (T)qy};
      dst[gi] = qt;
      acc += ((c0 + c) == 0 ? 1.0 : 2.0) * (vx * (double)qt.x + vy * (double)qt.y);
    }
    const double sblk = block_sum<kFftThreads>(acc, red);
    if (threadIdx.x == 0) S.part_a[(size_t)r * S.pstride + blockIdx.x] = sblk;
  } else {
    const T sc = (MODE == kColFwdInit) ? scale : (T)1;
    for (int idx = threadIdx.x; idx < nf * N1; idx += kFftThreads) {
      const int k1 = idx / nf, c = idx % nf;
      const C2<T> a = buf[idx];
      dst[(size_t)k1 * H + c0 + c] = {a.x * sc, a.y * sc};
    }
  }
}

// ---- host side -----------------------------------------------------------------------------------------
template <typename T>
static int col_nf(const FftPlan& p) {
  return std::min(p.H, FftCfg<T>::ELEMS / p.N1);
}
template <typename T>
static int row_np(const FftPlan& p) {
  return std::min(p.N1 / 2, FftCfg<T>::ELEMS / p.N2);
}

gmrf_status fft_plan_create(FftPlan& p, int N1, int N2) {
  p.N1 = N1;
  p.N2 = N2;
  p.H = N2 / 2;
  auto table = [](int N, std::vector<double>& t) {
    t.resize(2 * (size_t)N);
    for (int k = 0; k < N; ++k) {
      // e^{-2 pi i k / N}, reduced to the first octant-free form by symmetry of k / N
      const double a = 2.0 * M_PI * (double)k / (double)N;
      t[2 * k] = std::cos(a);
      t[2 * k + 1] = -std::sin(a);
    }
  };
  std::vector<double> t1, t2;
  table(N1, t1);
  table(N2, t2);
  std::vector<float> f1(t1.begin(), t1.end()), f2(t2.begin(), t2.end());
  if (hipMalloc(&p.tw64_1, t1.size() * 8) != hipSuccess || hipMalloc(&p.tw64_2, t2.size() * 8) != hipSuccess ||
      hipMalloc(&p.tw32_1, f1.size() * 4) != hipSuccess || hipMalloc(&p.tw32_2, f2.size() * 4) != hipSuccess)
    return GMRF_ENOMEM;
  if (hipMemcpy(p.tw64_1, t1.data(), t1.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p.tw64_2, t2.data(), t2.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p.tw32_1, f1.data(), f1.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p.tw32_2, f2.data(), f2.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
    return GMRF_EDEVICE;
  return GMRF_OK;
}

void fft_plan_destroy(FftPlan& p) {
  if (p.tw64_1) (void)hipFree(p.tw64_1);
  if (p.tw64_2) (void)hipFree(p.tw64_2);
  if (p.tw32_1) (void)hipFree(p.tw32_1);
  if (p.tw32_2) (void)hipFree(p.tw32_2);
  p = FftPlan{};
}

// column blocks per field (the alpha partial count of the preconditioned operator); sized for
// the FP32 tile, which the FP64 path shares by construction (same nf for both is not needed:
// each path asks for its own count through fft_col_blocks_t)
template <typename T>
static int col_blocks_t(const FftPlan& p) { return p.H / col_nf<T>(p); }
int fft_col_blocks(const FftPlan& p) { return std::max(col_blocks_t<double>(p), col_blocks_t<float>(p)); }

template <typename T> static const C2<T>* tw1(const FftPlan& p);
template <typename T> static const C2<T>* tw2(const FftPlan& p);
template <> const C2<double>* tw1<double>(const FftPlan& p) { return (const C2<double>*)p.tw64_1; }
template <> const C2<double>* tw2<double>(const FftPlan& p) { return (const C2<double>*)p.tw64_2; }
template <> const C2<float>* tw1<float>(const FftPlan& p) { return (const C2<float>*)p.tw32_1; }
template <> const C2<float>* tw2<float>(const FftPlan& p) { return (const C2<float>*)p.tw32_2; }

template <typename Tin, typename T>
static void rows_r2c(const FftPlan& p, const Tin* in, long ild, T* out, long old_complex, T scale, const int* active,
                     int k, hipStream_t st) {
  const int np = row_np<T>(p);
  hipLaunchKernelGGL((k_rows_r2c<Tin, T>), dim3(p.N1 / (2 * np), k), dim3(kFftThreads), 0, st, in, ild,
                     (C2<T>*)out, old_complex, p.N1, p.N2, np, tw2<T>(p), scale, active);
}
template <typename T, typename Tout>
static void rows_c2r(const FftPlan& p, const T* in, long ild_complex, Tout* out, long old, T scale,
                     const int* active, int k, hipStream_t st) {
  const int np = row_np<T>(p);
  hipLaunchKernelGGL((k_rows_c2r<T, Tout>), dim3(p.N1 / (2 * np), k), dim3(kFftThreads), 0, st,
                     (const C2<T>*)in, ild_complex, out, old, p.N1, p.N2, np, tw2<T>(p), scale, active);
}
template <typename T, int MODE>
static void cols(const FftPlan& p, const T* in, T* out, const T* mult, T scale, const LzState& S, int j,
                 const T* Xj, const T* Xprev, int k, hipStream_t st, BandIO<T> bio = BandIO<T>{}) {
  const int nf = col_nf<T>(p);
  hipLaunchKernelGGL((k_cols<T, MODE>), dim3(p.H / nf, k), dim3(kFftThreads), 0, st, (const C2<T>*)in,
                     (C2<T>*)out, p.N1, p.H, nf, tw1<T>(p), mult, scale, S, j, (const C2<T>*)Xj,
                     (const C2<T>*)Xprev, bio);
}


// ---- band pass of the preconditioned operator --------------------------------------------------------
// D = M - Q (M the periodic version of Q) is nonzero only within one point of the boundary, so for
// interior rows r = 2..N1-3 the row of D u is supported on columns {0, 1, N2-2, N2-1} and, with
// e_r = u(r,0) - u(r,N2-1),
//   order 1:  d0 = tau e_r,  d1 = 0
//   order 2:  d0 = tau [K_f(Eu)(r,0) + K_p u(r,0) - K_p u(r,N2-1)],  d1 = -tau e_r,
// D u(r, N2-2) = -d1 and D u(r, N2-1) = -d0.  Such a row needs u only at those four columns of
// rows r-1..r+1: the opening column pass leaves their partial sums per column tile, here summed in
// tile order.  Its forward row transform is closed form (X_0 = 0, X_{N2/2} = 2 (d0 - d1),
// X_c = d0 (1 - conj w^c) + d1 (w^c - conj w^{2c}), w = e^{-2 pi i / N2}) and is evaluated by the
// closing column pass.  Blocks 0 and 1 of each field handle the edge rows {0, 1} and {N1-2, N1-1}
// (full rows, y-wrap terms): each takes the inverse FFTs of rows {0, 1, 2, N1-3, N1-2, N1-1}
// (batched in LDS), tabulates E u and K_p u, forms D u = tau [K_f (E u) + E (K_p u)] (order 2;
// tau E u for order 1) on its two rows and takes their forward FFT.

constexpr int kBandRowsPerBlock = 64;   // interior rows per band block

// u(row, band column t) from the opener's per-tile partial sums, in tile order
__device__ __forceinline__ double band_sum(const double* pb, int row, int ntiles, int t) {
  const double* p = pb + (size_t)row * ntiles * 4 + t;
  double s = 0.0;
  for (int i = 0; i < ntiles; ++i) s += p[4 * i];
  return s;
}

// Edge rows.  Slots 0..5 hold rows {0, 1, 2, N1-3, N1-2, N1-1}; the output slots 0..3 rows
// {0, 1, N1-2, N1-1}.  E u is needed on all six rows, K_p u on the four output rows.
__device__ __forceinline__ int slot_row(int s, int N1) { return s < 3 ? s : N1 - 6 + s; }
__device__ __forceinline__ int row_slot(int r, int N1) { return r <= 2 ? r : r - (N1 - 6); }

template <typename T, int ORDER>
__global__ __launch_bounds__(kFftThreads) void k_band(int N1, int N2, int ntiles, const C2<T>* __restrict__ tw,
                                                      T k2, T tau, BandIO<T> bio, T* __restrict__ scratch,
                                                      const int* __restrict__ active, int periodic) {
  __shared__ C2<T> buf[FftCfg<T>::ELEMS];
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int H = N2 / 2;
  C2<T>* E = bio.edge_out + (size_t)r * 4 * H;
  double* B = bio.bcoef + (size_t)r * N1 * 2;
  const int half = blockIdx.x < 2 ? (int)blockIdx.x : -1;   // edge block: 0 top, 1 bottom
  if (periodic) {
    // a periodic Q is its own preconditioner: D = 0
    if (half >= 0) {
      for (int i = threadIdx.x; i < 2 * H; i += kFftThreads) E[(size_t)half * 2 * H + i] = {(T)0, (T)0};
    } else {
      const int r0 = 2 + (blockIdx.x - 2) * kBandRowsPerBlock, r1 = min(N1 - 2, r0 + kBandRowsPerBlock);
      for (int i = threadIdx.x; i < 2 * (r1 - r0); i += kFftThreads) B[2 * r0 + i] = 0.0;
    }
    return;
  }
  if (half < 0) {
    // ---- interior rows r0..r1-1: (d0, d1) ----
    const int r0 = 2 + (blockIdx.x - 2) * kBandRowsPerBlock, r1 = min(N1 - 2, r0 + kBandRowsPerBlock);
    double* ub = (double*)buf;   // [(r1 - r0 + 2) rows][4]
    const double* pb = bio.pband + (size_t)r * N1 * ntiles * 4;
    const int nq = r1 - r0 + 2;
    for (int item = threadIdx.x; item < nq * 4; item += kFftThreads) {
      const int q = item >> 2, t = item & 3;
      ub[item] = band_sum(pb, r0 - 1 + q, ntiles, t);
    }
    __syncthreads();
    const double kk = (double)k2, tt = (double)tau;
    for (int row = r0 + threadIdx.x; row < r1; row += kFftThreads) {
      const double* cu = ub + 4 * (row - r0 + 1);
      const double u0 = cu[0], u1 = cu[1], um2 = cu[2], um1 = cu[3];
      const double e = u0 - um1;
      double d0, d1;
      if (ORDER == 1) {
        d0 = tt * e;
        d1 = 0.0;
      } else {
        const double a0 = cu[-4], a3 = cu[-1], b0 = cu[4], b3 = cu[7];
        const double em = a0 - a3, ep = b0 - b3;
        const double kfe0 = kk * e + e + (e - em) + (e - ep);
        const double kp0 = kk * u0 + (u0 - u1) + (u0 - um1) + (u0 - a0) + (u0 - b0);
        const double kpm1 = kk * um1 + (um1 - um2) + (um1 - u0) + (um1 - a3) + (um1 - b3);
        d0 = tt * (kfe0 + kp0 - kpm1);
        d1 = -tt * e;
      }
      B[2 * row] = d0;
      B[2 * row + 1] = d1;
    }
    return;
  }
  // ---- edge rows: block `half` produces output slots 2 half, 2 half + 1 ----
  T* U = scratch + ((size_t)r * 2 + half) * 20 * N2;   // 6 rows u, 6 rows E u, 4 rows K_p u, 4 rows D u
  T* EU = U + (size_t)6 * N2;
  T* KP = EU + (size_t)6 * N2;
  T* DU = KP + (size_t)4 * N2;
  const C2<T>* Cin = bio.edge_in + (size_t)r * 6 * H;
  const int np = min(3, FftCfg<T>::ELEMS / N2);   // row pairs per LDS pass
  for (int p0 = 0; p0 < 3; p0 += np) {
    const int npp = min(np, 3 - p0);
    for (int idx = threadIdx.x; idx < npp * N2; idx += kFftThreads) {
      const int pr = p0 + idx / N2, k = idx % N2;
      const C2<T>* PA = Cin + (size_t)(2 * pr) * H;
      const C2<T>* PB = PA + H;
      C2<T> a, b;
      if (k == 0) { a = {PA[0].x, (T)0}; b = {PB[0].x, (T)0}; }
      else if (k == H) { a = {PA[0].y, (T)0}; b = {PB[0].y, (T)0}; }
      else if (k < H) { a = PA[k]; b = PB[k]; }
      else { a = {PA[N2 - k].x, -PA[N2 - k].y}; b = {PB[N2 - k].x, -PB[N2 - k].y}; }
      buf[idx] = {a.x - b.y, a.y + b.x};
    }
    __syncthreads();
    lds_fft<T, false>(buf, N2, npp, N2, 1, tw, true);
    for (int idx = threadIdx.x; idx < npp * N2; idx += kFftThreads) {
      const int pr = p0 + idx / N2, t = idx % N2;
      U[(size_t)(2 * pr) * N2 + t] = buf[idx].x;
      U[(size_t)(2 * pr + 1) * N2 + t] = buf[idx].y;
    }
    __syncthreads();
  }
  // E u on the six rows, K_p u on the four output rows (wrap in both directions)
  for (int idx = threadIdx.x; idx < 10 * N2; idx += kFftThreads) {
    const int q = idx / N2, c = idx % N2;
    const int cm = c == 0 ? N2 - 1 : c - 1, cp = c == N2 - 1 ? 0 : c + 1;
    if (q < 6) {
      const int row = slot_row(q, N1);
      const T v = U[(size_t)q * N2 + c];
      T acc = (T)0;
      if (c == 0) acc += v - U[(size_t)q * N2 + N2 - 1];
      if (c == N2 - 1) acc += v - U[(size_t)q * N2];
      if (row == 0) acc += v - U[(size_t)5 * N2 + c];
      if (row == N1 - 1) acc += v - U[c];
      EU[(size_t)q * N2 + c] = acc;
    } else {
      const int o = q - 6;                         // output slot 0..3 -> rows 0, 1, N1-2, N1-1
      const int row = o < 2 ? o : N1 - 4 + o;
      const int s = row_slot(row, N1);
      const int sm = row_slot(row == 0 ? N1 - 1 : row - 1, N1), sp = row_slot(row == N1 - 1 ? 0 : row + 1, N1);
      const T v = U[(size_t)s * N2 + c];
      KP[(size_t)o * N2 + c] = k2 * v + (v - U[(size_t)s * N2 + cm]) + (v - U[(size_t)s * N2 + cp]) +
                               (v - U[(size_t)sm * N2 + c]) + (v - U[(size_t)sp * N2 + c]);
    }
  }
  __syncthreads();
  // D u = tau [K_f (E u) + E (K_p u)] (order 2), tau E u (order 1), on this block's two rows
  for (int idx = threadIdx.x; idx < 2 * N2; idx += kFftThreads) {
    const int o = 2 * half + idx / N2, c = idx % N2;
    const int row = o < 2 ? o : N1 - 4 + o;
    const int s = row_slot(row, N1);
    T d;
    if (ORDER == 1) {
      d = tau * EU[(size_t)s * N2 + c];
    } else {
      const T e = EU[(size_t)s * N2 + c];
      T kfe = k2 * e;
      if (c > 0) kfe += e - EU[(size_t)s * N2 + c - 1];
      if (c < N2 - 1) kfe += e - EU[(size_t)s * N2 + c + 1];
      if (row > 0) kfe += e - EU[(size_t)row_slot(row - 1, N1) * N2 + c];
      if (row < N1 - 1) kfe += e - EU[(size_t)row_slot(row + 1, N1) * N2 + c];
      const T kp = KP[(size_t)o * N2 + c];
      T ekp = (T)0;
      if (c == 0) ekp += kp - KP[(size_t)o * N2 + N2 - 1];
      if (c == N2 - 1) ekp += kp - KP[(size_t)o * N2];
      if (row == 0) ekp += kp - KP[(size_t)3 * N2 + c];
      if (row == N1 - 1) ekp += kp - KP[c];
      d = tau * (kfe + ekp);
    }
    DU[(size_t)(idx / N2) * N2 + c] = d;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < N2; t += kFftThreads) buf[t] = {DU[t], DU[(size_t)N2 + t]};
  __syncthreads();
  lds_fft<T, false>(buf, N2, 1, N2, 1, tw, false);
  C2<T>* PA = E + (size_t)(2 * half) * H;
  C2<T>* PB = PA + H;
  const T h = (T)0.5;
  for (int c = threadIdx.x; c < H; c += kFftThreads) {
    if (c == 0) {
      PA[0] = {buf[0].x, buf[H].x};
      PB[0] = {buf[0].y, buf[H].y};
    } else {
      const C2<T> zk = buf[c], zm = buf[N2 - c];
      PA[c] = {(zk.x + zm.x) * h, (zk.y - zm.y) * h};
      PB[c] = {(zk.y + zm.y) * h, (zm.x - zk.x) * h};
    }
  }
}

template <typename T>
static void band(const FftPlan& p, const StencilGeom& g, int order, BandIO<T> bio, T* scratch, const int* active,
                 int k, hipStream_t st) {
  const int ntiles = p.H / col_nf<T>(p);
  const dim3 grid(2 + (p.N1 - 4 + kBandRowsPerBlock - 1) / kBandRowsPerBlock, k);
  if (order == 1)
    hipLaunchKernelGGL((k_band<T, 1>), grid, dim3(kFftThreads), 0, st, p.N1, p.N2, ntiles, tw2<T>(p),
                       (T)g.kappa2, (T)g.tau, bio, scratch, active, g.periodic);
  else
    hipLaunchKernelGGL((k_band<T, 2>), grid, dim3(kFftThreads), 0, st, p.N1, p.N2, ntiles, tw2<T>(p),
                       (T)g.kappa2, (T)g.tau, bio, scratch, active, g.periodic);
}

// device bytes of the band hand-off buffers for k fields
template <typename T>
static size_t band_bytes(const FftPlan& p, int k) {
  const size_t ntiles = p.H / col_nf<T>(p);
  return (size_t)k * ((size_t)p.N1 * ntiles * 4 * 8 + (size_t)6 * p.H * sizeof(C2<T>) + (size_t)p.N1 * 2 * 8 +
                      (size_t)4 * p.H * sizeof(C2<T>) + (size_t)40 * p.N2 * sizeof(T));
}

template <typename T>
static BandIO<T> band_io(const FftPlan& p, void* base, int k) {
  const size_t ntiles = p.H / col_nf<T>(p);
  char* b = (char*)base;
  BandIO<T> io{};
  io.tw2 = tw2<T>(p);
  io.pband = (double*)b;
  b += (size_t)k * p.N1 * ntiles * 4 * 8;
  io.bcoef = (double*)b;
  b += (size_t)k * p.N1 * 2 * 8;
  io.edge_in = (C2<T>*)b;
  b += (size_t)k * 6 * p.H * sizeof(C2<T>);
  io.edge_out = (C2<T>*)b;
  return io;
}

size_t fft_band_bytes(const FftPlan& p, int storage, int k) {
  return storage == GMRF_F64 ? band_bytes<double>(p, k) : band_bytes<float>(p, k);
}

template <typename T>
void fft_apply_inv_sqrt_M(const FftPlan& p, const T* mult, const T* X, T* Y, T* tmp, int k, hipStream_t st) {
  const long n = (long)p.N1 * p.N2;
  LzState S{};
  rows_r2c<T, T>(p, X, n, tmp, n / 2, (T)1, nullptr, k, st);
  cols<T, kColApply>(p, tmp, tmp, mult, (T)(1.0 / (double)n), S, 0, nullptr, nullptr, k, st);
  rows_c2r<T, T>(p, tmp, n / 2, Y, n, (T)1, nullptr, k, st);
}

template <typename T>
void fft_forward_init(const FftPlan& p, const double* Z, T* V0, T* tmp, const LzState& S, int k, hipStream_t st) {
  const long n = (long)p.N1 * p.N2;
  rows_r2c<double, T>(p, Z, n, tmp, n / 2, (T)1, nullptr, k, st);
  cols<T, kColFwdInit>(p, tmp, V0, nullptr, (T)(1.0 / std::sqrt((double)n)), S, 0, nullptr, nullptr, k, st);
  launch_norm_partials<T>(V0, n, S, st);
}

template <typename T>
void fft_forward_init_probes(const FftPlan& p, uint64_t seed, const int8_t* probes, T* real_tmp, T* V0, T* tmp,
                             const LzState& S, int k, hipStream_t st) {
  const long n = (long)p.N1 * p.N2;
  if (probes) launch_init_from_i8<T>(probes, n, real_tmp, S, st);
  else launch_init_rademacher<T>(seed, n, real_tmp, S, st);
  rows_r2c<T, T>(p, real_tmp, n, tmp, n / 2, (T)1, nullptr, k, st);
  cols<T, kColFwdInit>(p, tmp, V0, nullptr, (T)(1.0 / std::sqrt((double)n)), S, 0, nullptr, nullptr, k, st);
  launch_norm_partials<T>(V0, n, S, st);
}

template <typename T>
void fft_lanczos_operator(const FftPlan& p, const StencilGeom& g, int order, const void* mult, const T* Xj,
                          const T* Xprev, T* Qb, void* scratch, const LzState& S, int j, int k, hipStream_t st) {
  const long n = (long)p.N1 * p.N2;
  const T* m = (const T*)mult;
  // A = M^{-1/2} Q M^{-1/2} = I - M^{-1/2} D M^{-1/2} with D = M - Q supported near the boundary
  // scratch: band hand-off buffers followed by the edge-row work rows (40 N2 per field)
  const BandIO<T> bio = band_io<T>(p, scratch, k);
  T* edge_rows = (T*)((char*)scratch + band_bytes<T>(p, k) - (size_t)k * 40 * p.N2 * sizeof(T));
  cols<T, kColInvLz>(p, Xj, nullptr, m, (T)(1.0 / (double)n), S, j, nullptr, nullptr, k, st, bio);
  band<T>(p, g, order, bio, edge_rows, S.active, k, st);
  cols<T, kColFwdLz>(p, nullptr, Qb, m, (T)1, S, j, Xj, Xprev, k, st, bio);
}

template <typename T>
void fft_backward_output(const FftPlan& p, const void* mult, const T* U, double* X, T* tmp, const LzState& S,
                         int k, hipStream_t st) {
  const long n = (long)p.N1 * p.N2;
  cols<T, kColInvOut>(p, U, tmp, (const T*)mult, (T)(1.0 / std::sqrt((double)n)), S, 0, nullptr, nullptr, k, st);
  rows_c2r<T, double>(p, tmp, n / 2, X, n, (T)1, nullptr, k, st);
}

template <typename T>
void fft_col_pass_lz(const FftPlan& p, int forward, const void* mult, const T* Xj, const T* Xprev, T* Qb,
                     void* scratch, const LzState& S, int j, int k, hipStream_t st) {
  const long n = (long)p.N1 * p.N2;
  const BandIO<T> bio = band_io<T>(p, scratch, k);
  if (forward) cols<T, kColFwdLz>(p, nullptr, Qb, (const T*)mult, (T)1, S, j, Xj, Xprev, k, st, bio);
  else cols<T, kColInvLz>(p, Xj, nullptr, (const T*)mult, (T)(1.0 / (double)n), S, j, nullptr, nullptr, k, st, bio);
}
template void fft_col_pass_lz<double>(const FftPlan&, int, const void*, const double*, const double*, double*,
                                      void*, const LzState&, int, int, hipStream_t);
template void fft_col_pass_lz<float>(const FftPlan&, int, const void*, const float*, const float*, float*,
                                     void*, const LzState&, int, int, hipStream_t);

int fft_col_blocks_for(const FftPlan& p, int storage) {
  return storage == GMRF_F64 ? col_blocks_t<double>(p) : col_blocks_t<float>(p);
}

#define INST(T)                                                                                            \
  template void fft_apply_inv_sqrt_M<T>(const FftPlan&, const T*, const T*, T*, T*, int, hipStream_t);     \
  template void fft_forward_init<T>(const FftPlan&, const double*, T*, T*, const LzState&, int, hipStream_t); \
  template void fft_forward_init_probes<T>(const FftPlan&, uint64_t, const int8_t*, T*, T*, T*, const LzState&, int, hipStream_t); \
  template void fft_lanczos_operator<T>(const FftPlan&, const StencilGeom&, int, const void*, const T*, const T*, T*, void*, const LzState&, int, int, hipStream_t); \
  template void fft_backward_output<T>(const FftPlan&, const void*, const T*, double*, T*, const LzState&, int, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace gmrf
