// Preconditioned Lanczos step for Q + diag(H) on a periodic 2D lattice with M = the lattice part
// Q (Section 5.1 with alpha_n = 0: the sMMALA proposal of the log-Gaussian Cox process, Section 3).
//
// In the unitary spectral basis of fft.hpp, A_hat = I + Lambda^{-1/2} F H F^H Lambda^{-1/2}: two 2D
// transforms per step (Section 5.1 counts four for the real-space form).  One step is two launches,
// each keeping one axis of both transforms on chip:
//   row pass:    T1 holds the column-inverse transform of Lambda^{-1/2} w_{j-1}.  Opens iteration j
//                (beta_{j-1}, stopping rule); inverse row transforms give y = F^H Lambda^{-1/2} v_j in
//                real space (v_j = w_{j-1} / beta_{j-1}); partial sums of y^T H y; forward row transforms
//                of H y into T2.
//   column pass: forward column transforms of T2 give F H y;  w_j = v_j + Lambda^{-1/2} F H y -
//                alpha_j v_j - beta_{j-1} v_{j-1} with alpha_j = v_j^T A_hat v_j - <w_{j-1}, v_{j-1}>
//                = 1 + y^T H y - <w_{j-1}, v_{j-1}> (Algorithm 1's alpha_j, ||v_j|| = 1); w_j is written
//                with its ||w_j||^2 and <w_j, v_j> partial sums, then the column-inverse transform of
//                Lambda^{-1/2} w_j goes to T1 for the next row pass.
// Per step: 7 s E bytes (row pass 2, column pass 5) plus the diagonal once per field.
#include "fft.hpp"
#include "fft_lds.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <cmath>

namespace gmrf {

// The FP64 row pass requests each FFT stage's twiddles before the barrier (measured 5% faster at
// 512^2 x 32 and 4096^2); elsewhere the extra registers cost more than the latency they hide
// (FP32 column pass 59 -> 84 us).
template <typename T> constexpr bool kRowsEarlyTw = sizeof(T) == 8;

// Threads per block of each pass: 512 (half the LDS of a 1024-thread block, four blocks per CU, so their
// load, transform and store phases overlap more than two large blocks do) when the pass's tile still fits:
// a row for the row pass, at least four columns (64 bytes of each row) for the column pass; else 1024.
// Measured at 512^2 x 32 FP64: row pass 76.2 -> 66.8 us, column pass 127.8 -> 116.9 us; at 2048^2 the
// one-column tiles of small column blocks were slower (711 -> 809 us), so that pass stays large there.
#ifndef GMRF_LGCP_SMALL
#define GMRF_LGCP_SMALL 1
#endif
template <typename T>
static int lgcp_rows_nt(const FftPlan& p) {
  return (GMRF_LGCP_SMALL && p.N2 <= FftCfg<T>::ELEMS / 2) ? kFftThreads / 2 : kFftThreads;
}
template <typename T>
static int lgcp_cols_nt(const FftPlan& p) {
  return (GMRF_LGCP_SMALL && 4 * p.N1 <= FftCfg<T>::ELEMS / 2) ? kFftThreads / 2 : kFftThreads;
}
template <typename T>
static int lgcp_row_np(const FftPlan& p) {
  const int elems = FftCfg<T>::ELEMS / (kFftThreads / lgcp_rows_nt<T>(p));
  return std::min(p.N1 / 2, elems / p.N2);
}
template <typename T>
static int lgcp_col_nf(const FftPlan& p) {
  const int elems = FftCfg<T>::ELEMS / (kFftThreads / lgcp_cols_nt<T>(p));
  return std::min(p.H, elems / p.N1);
}

// ---- row pass ------------------------------------------------------------------------------------------
// Grid (N1 / (2 np), k): np row pairs of field r per block.  Partial sums of y^T H y go to
// part_a[r][blockIdx.x]; the opener block also stores <w_{j-1}, v_{j-1}> (the column pass's part_c
// partials, Pc of them; 0 when use_c = 0 or j = 1) at part_a[r][gridDim.x].
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_lgcp_rows(const C2<T>* __restrict__ T1, C2<T>* __restrict__ T2,
                                                           const T* __restrict__ d, int N1, int N2, int np,
                                                           const C2<T>* __restrict__ tw, LzState S, int j,
                                                           int use_c, int Pc, double inv_sqrt_n) {
  __shared__ C2<T> buf[FftCfg<T>::ELEMS * NT / kFftThreads];
  __shared__ double red[3 * (NT / kWave)];   // lz_open_with takes three sets
  __shared__ int flag;
  const int r = blockIdx.y;
  const bool writer = blockIdx.x == 0;
  double s_cur, s_prev, bprev, qa, c;
  // the <w_{j-1}, v_{j-1}> partials (the writer's) load with the opener's
  const bool with_c = writer && use_c && j > 1;
  if (!lz_open_with<NT>(S, r, j, writer, red, &flag, nullptr, 0, with_c ? S.part_c + (size_t)r * S.pstride : nullptr,
                        Pc, s_cur, s_prev, bprev, qa, c))
    return;
  if (writer && threadIdx.x == 0) S.part_a[(size_t)r * S.pstride + gridDim.x] = c;
  const int H = N2 / 2;
  const int row0 = 2 * np * blockIdx.x;
  const size_t fsz = (size_t)N1 * H;
  const C2<T>* src = T1 + (size_t)r * fsz;
  // packed rows (A + i B of rows 2p, 2p+1) -> full-length sequence A + i B.  At most ELEMS NT / kFftThreads
  // values, a compile-time count per thread: all loads are issued first, from the one packed index each
  // value needs (a load behind a branch would wait for its own data), and the cases are selects.
  constexpr int MI = FftCfg<T>::ELEMS / kFftThreads;
  const int cnt = np * N2;
  C2<T> ra[MI], rb[MI];
#pragma unroll
  for (int it = 0; it < MI; ++it) {
    const int idx = min((int)threadIdx.x + it * NT, cnt - 1);
    const int p = idx / N2, k = idx % N2;
    const int ks = (k == 0 || k == H) ? 0 : (k < H ? k : N2 - k);
    const C2<T>* PA = src + (size_t)(row0 + 2 * p) * H;
    ra[it] = PA[ks];
    rb[it] = PA[H + ks];
  }
#pragma unroll
  for (int it = 0; it < MI; ++it) {
    const int idx = (int)threadIdx.x + it * NT;
    if (idx >= cnt) continue;
    const int k = idx % N2;
    const C2<T> a = k == 0 ? C2<T>{ra[it].x, (T)0} : k == H ? C2<T>{ra[it].y, (T)0}
                  : k < H ? ra[it] : C2<T>{ra[it].x, -ra[it].y};
    const C2<T> b = k == 0 ? C2<T>{rb[it].x, (T)0} : k == H ? C2<T>{rb[it].y, (T)0}
                  : k < H ? rb[it] : C2<T>{rb[it].x, -rb[it].y};
    buf[idx] = {a.x - b.y, a.y + b.x};
  }
  __syncthreads();
  lds_fft<T, false, kRowsEarlyTw<T>, NT>(buf, N2, np, N2, 1, tw, true);
  // y = (1 / (beta_{j-1} sqrt n)) * (real rows), u = H y, partial y^T H y
  const T sc = (T)(s_cur * inv_sqrt_n);
  double acc = 0.0;
  T da[MI], db[MI];
#pragma unroll
  for (int it = 0; it < MI; ++it) {
    const int idx = min((int)threadIdx.x + it * NT, cnt - 1);
    const size_t rr = (size_t)(row0 + 2 * (idx / N2)) * N2 + idx % N2;
    da[it] = d[rr];
    db[it] = d[rr + N2];
  }
#pragma unroll
  for (int it = 0; it < MI; ++it) {
    const int idx = (int)threadIdx.x + it * NT;
    if (idx >= cnt) continue;
    const C2<T> z = buf[idx];
    const T ya = z.x * sc, yb = z.y * sc;
    const T ua = da[it] * ya, ub = db[it] * yb;
    acc += (double)ya * (double)ua + (double)yb * (double)ub;
    buf[idx] = {ua, ub};
  }
  __syncthreads();
  lds_fft<T, false, kRowsEarlyTw<T>, NT>(buf, N2, np, N2, 1, tw, false);
  // unpack the two half spectra of rows 2p, 2p+1 into packed rows of T2
  C2<T>* dst = T2 + (size_t)r * fsz;
  for (int idx = threadIdx.x; idx < np * H; idx += NT) {
    const int p = idx / H, c = idx % H;
    const C2<T>* Z = buf + p * N2;
    C2<T> pa, pb;
    if (c == 0) {
      const C2<T> z0 = Z[0], zn = Z[H];
      pa = {z0.x, zn.x};
      pb = {z0.y, zn.y};
    } else {
      const C2<T> zk = Z[c], zm = Z[N2 - c];
      pa = {(zk.x + zm.x) * (T)0.5, (zk.y - zm.y) * (T)0.5};
      pb = {(zk.y + zm.y) * (T)0.5, (zm.x - zk.x) * (T)0.5};
    }
    dst[(size_t)(row0 + 2 * p) * H + c] = pa;
    dst[(size_t)(row0 + 2 * p + 1) * H + c] = pb;
  }
  const double tot = block_sum<NT>(acc, red);
  if (threadIdx.x == 0) S.part_a[(size_t)r * S.pstride + blockIdx.x] = tot;
}

// ---- column pass ---------------------------------------------------------------------------------------
// MODE 0: T1 <- column-inverse transform of Lambda^{-1/2} X (X = slot 0, or a reorthogonalised w_j).
// MODE 1: the column pass of step j (X = T2, Vj = slot j-1, Vp = slot j-2, W = slot j).
// Grid (H / nf, k): nf packed columns of field r per block, all N1 rows.
template <typename T, int MODE, int NT>
__global__ __launch_bounds__(NT) void k_lgcp_cols(const C2<T>* __restrict__ X, const C2<T>* __restrict__ Vj,
                                                           const C2<T>* __restrict__ Vp, C2<T>* __restrict__ W,
                                                           C2<T>* __restrict__ T1, int N1, int H, int nf,
                                                           const C2<T>* __restrict__ tw, const T* __restrict__ mult,
                                                           LzState S, int j, int Pr, double inv_sqrt_n) {
  __shared__ C2<T> buf[FftCfg<T>::ELEMS * NT / kFftThreads];
  __shared__ double red[NT / kWave];
  __shared__ double sh[4];
  __shared__ int flag;
  const int r = blockIdx.y;
  const int c0 = xcd_col_block(blockIdx.x, gridDim.x) * nf;
  const size_t fsz = (size_t)N1 * H;
  const size_t foff = (size_t)r * fsz;
  double alpha = 0.0, s_cur = 0.0, s_prev = 0.0, bprev = 0.0;
  if (MODE == 1) {
    if (!block_active(S, r, &flag)) return;
    const double yhy = sum_partials<NT>(S.part_a + (size_t)r * S.pstride, Pr, red);
    if (threadIdx.x == 0) {
      const double a = 1.0 + yhy - S.part_a[(size_t)r * S.pstride + Pr];
      sh[0] = a;
      sh[1] = S.beta[lz_ib(S, r, j - 1)];
      sh[2] = j > 1 ? S.beta[lz_ib(S, r, j - 2)] : 1.0;
      if (blockIdx.x == 0) S.alpha[lz_ia(S, r, j)] = a;
    }
    __syncthreads();
    alpha = sh[0];
    s_cur = 1.0 / sh[1];
    s_prev = j > 1 ? 1.0 / sh[2] : 0.0;
    bprev = j > 1 ? sh[1] : 0.0;
  }
  // at most ELEMS NT / kFftThreads values, a compile-time count per thread: every load of a loop is issued
  // before the first is used (a load behind a bounds branch would wait for its own data)
  constexpr int MI = FftCfg<T>::ELEMS / kFftThreads;
  const int cnt = nf * N1;
  {
    C2<T> xv[MI];
#pragma unroll
    for (int it = 0; it < MI; ++it) {
      const int idx = min((int)threadIdx.x + it * NT, cnt - 1);
      xv[it] = X[foff + (size_t)(idx / nf) * H + c0 + idx % nf];
    }
#pragma unroll
    for (int it = 0; it < MI; ++it) {
      const int idx = (int)threadIdx.x + it * NT;
      if (idx < cnt) buf[idx] = xv[it];
    }
  }
  if (MODE == 1) {
    __syncthreads();
    lds_fft<T, true, false, NT>(buf, N1, nf, 1, nf, tw, false);
    apply_mult<T, NT>(buf, nf, c0, N1, H, mult, (T)inv_sqrt_n);
    const T sc = (T)s_cur, sp = (T)s_prev, al = (T)alpha, bp = (T)bprev;
    double nb = 0.0, nc = 0.0;
    for (int idx = threadIdx.x; idx < cnt; idx += NT) {
      const int k1 = idx / nf, c = idx % nf;
      const size_t g = foff + (size_t)k1 * H + c0 + c;
      const C2<T> xv = Vj[g];
      const C2<T> v = {xv.x * sc, xv.y * sc};
      C2<T> vp = {(T)0, (T)0};
      if (j > 1) {
        const C2<T> xp = Vp[g];
        vp = {xp.x * sp, xp.y * sp};
      }
      const C2<T> a = buf[idx];
      const C2<T> w = {v.x + a.x - al * v.x - bp * vp.x, v.y + a.y - al * v.y - bp * vp.y};
      const double wt = (c0 + c == 0) ? 1.0 : 2.0;
      nb += wt * ((double)w.x * (double)w.x + (double)w.y * (double)w.y);
      nc += wt * ((double)w.x * (double)v.x + (double)w.y * (double)v.y);
      W[g] = w;
      buf[idx] = w;
    }
    const double sb = block_sum<NT>(nb, red);
    const double scc = block_sum<NT>(nc, red);
    if (threadIdx.x == 0) {
      S.part_b[(size_t)r * S.pstride + blockIdx.x] = sb;
      S.part_c[(size_t)r * S.pstride + blockIdx.x] = scc;
    }
  }
  apply_mult<T, NT>(buf, nf, c0, N1, H, mult, (T)1);
  lds_fft<T, true, false, NT>(buf, N1, nf, 1, nf, tw, true);
  for (int idx = threadIdx.x; idx < nf * N1; idx += NT) {
    const int k1 = idx / nf, c = idx % nf;
    T1[foff + (size_t)k1 * H + c0 + c] = buf[idx];
  }
}

// Y += diag(d) X, column r of X and Y at offset r * n.
template <typename T>
__global__ __launch_bounds__(kEwThreads) void k_add_diag(const T* __restrict__ d, const T* __restrict__ X,
                                                         T* __restrict__ Y, long n) {
  const size_t off = (size_t)blockIdx.y * (size_t)n;
  for (long i = (long)blockIdx.x * kEwThreads + threadIdx.x; i < n; i += (long)gridDim.x * kEwThreads)
    Y[off + i] += d[i] * X[off + i];
}

// ---- host side -----------------------------------------------------------------------------------------
LgcpCounts lgcp_counts(const FftPlan& p, int storage) {
  LgcpCounts c;
  if (storage == GMRF_F64) {
    c.Pr = p.N1 / (2 * lgcp_row_np<double>(p));
    c.Pc = p.H / lgcp_col_nf<double>(p);
  } else {
    c.Pr = p.N1 / (2 * lgcp_row_np<float>(p));
    c.Pc = p.H / lgcp_col_nf<float>(p);
  }
  return c;
}

template <typename T> static const C2<T>* twid1(const FftPlan& p);
template <typename T> static const C2<T>* twid2(const FftPlan& p);
template <> const C2<double>* twid1<double>(const FftPlan& p) { return (const C2<double>*)p.tw64_1; }
template <> const C2<double>* twid2<double>(const FftPlan& p) { return (const C2<double>*)p.tw64_2; }
template <> const C2<float>* twid1<float>(const FftPlan& p) { return (const C2<float>*)p.tw32_1; }
template <> const C2<float>* twid2<float>(const FftPlan& p) { return (const C2<float>*)p.tw32_2; }

template <typename T>
void lgcp_col_init(const FftPlan& p, const void* mult, const T* X, T* T1, int k, hipStream_t st) {
  const int nf = lgcp_col_nf<T>(p);
  LzState S{};
  if (lgcp_cols_nt<T>(p) == kFftThreads)
    hipLaunchKernelGGL((k_lgcp_cols<T, 0, kFftThreads>), dim3(p.H / nf, k), dim3(kFftThreads), 0, st,
                       (const C2<T>*)X, nullptr, nullptr, nullptr, (C2<T>*)T1, p.N1, p.H, nf, twid1<T>(p),
                       (const T*)mult, S, 0, 0, 0.0);
  else
    hipLaunchKernelGGL((k_lgcp_cols<T, 0, kFftThreads / 2>), dim3(p.H / nf, k), dim3(kFftThreads / 2), 0, st,
                       (const C2<T>*)X, nullptr, nullptr, nullptr, (C2<T>*)T1, p.N1, p.H, nf, twid1<T>(p),
                       (const T*)mult, S, 0, 0, 0.0);
}

template <typename T>
void lgcp_lanczos_step(const FftPlan& p, const void* mult, const T* d, T* T1, T* T2, const T* Xj, const T* Xprev,
                       T* W, const LzState& S, int j, int use_c, int k, hipStream_t st, int only) {
  const double inv_sqrt_n = 1.0 / std::sqrt((double)p.N1 * (double)p.N2);
  const LgcpCounts c = lgcp_counts(p, sizeof(T) == 8 ? GMRF_F64 : GMRF_F32);
  if (only != 2) {
    const int np = lgcp_row_np<T>(p);
    if (lgcp_rows_nt<T>(p) == kFftThreads)
      hipLaunchKernelGGL((k_lgcp_rows<T, kFftThreads>), dim3(c.Pr, k), dim3(kFftThreads), 0, st, (const C2<T>*)T1,
                         (C2<T>*)T2, d, p.N1, p.N2, np, twid2<T>(p), S, j, use_c, c.Pc, inv_sqrt_n);
    else
      hipLaunchKernelGGL((k_lgcp_rows<T, kFftThreads / 2>), dim3(c.Pr, k), dim3(kFftThreads / 2), 0, st,
                         (const C2<T>*)T1, (C2<T>*)T2, d, p.N1, p.N2, np, twid2<T>(p), S, j, use_c, c.Pc, inv_sqrt_n);
  }
  if (only != 1) {
    const int nf = lgcp_col_nf<T>(p);
    if (lgcp_cols_nt<T>(p) == kFftThreads)
      hipLaunchKernelGGL((k_lgcp_cols<T, 1, kFftThreads>), dim3(c.Pc, k), dim3(kFftThreads), 0, st, (const C2<T>*)T2,
                         (const C2<T>*)Xj, (const C2<T>*)Xprev, (C2<T>*)W, (C2<T>*)T1, p.N1, p.H, nf, twid1<T>(p),
                         (const T*)mult, S, j, c.Pr, inv_sqrt_n);
    else
      hipLaunchKernelGGL((k_lgcp_cols<T, 1, kFftThreads / 2>), dim3(c.Pc, k), dim3(kFftThreads / 2), 0, st,
                         (const C2<T>*)T2, (const C2<T>*)Xj, (const C2<T>*)Xprev, (C2<T>*)W, (C2<T>*)T1, p.N1, p.H,
                         nf, twid1<T>(p), (const T*)mult, S, j, c.Pr, inv_sqrt_n);
  }
}

template <typename T>
void launch_add_diag(const T* d, const T* X, T* Y, long n, int k, hipStream_t st) {
  const long blocks = std::min<long>((n + kEwThreads - 1) / kEwThreads, 1024);
  hipLaunchKernelGGL((k_add_diag<T>), dim3((unsigned)blocks, k), dim3(kEwThreads), 0, st, d, X, Y, n);
}

#define INST(T)                                                                                                \
  template void lgcp_col_init<T>(const FftPlan&, const void*, const T*, T*, int, hipStream_t);                 \
  template void lgcp_lanczos_step<T>(const FftPlan&, const void*, const T*, T*, T*, const T*, const T*, T*,    \
                                     const LzState&, int, int, int, hipStream_t, int);           \
  template void launch_add_diag<T>(const T*, const T*, T*, long, int, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace gmrf
