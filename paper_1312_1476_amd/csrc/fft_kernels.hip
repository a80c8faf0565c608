// 2D FFT kernels of the block-circulant preconditioner (Proposition 1, Section 5.1), in the
// packed half-spectrum layout described in fft.hpp.  Power-of-two sides N1, N2 in [8, 4096].
// These are the transforms around the Lanczos loop (z_hat = F z, x = F^H Lambda^{-1/2} u_hat,
// M^{-1/2} on its own); the loop itself never takes a full 2D FFT (see precond_step.hip).
//
// Row pass: two real rows a, b form one complex sequence a + i b; one length-N2 FFT gives both
// half spectra, A_k = (Z_k + conj Z_{N-k}) / 2 and B_k = -i (Z_k - conj Z_{N-k}) / 2.
// Column pass: nf packed columns of one field per block, LDS laid out row-major [k1][c] so
// global loads and LDS traffic stay contiguous; the diagonal multiplier is fused into it.
#include "fft.hpp"
#include "fft_lds.hpp"

#include <cmath>
#include <vector>

namespace gmrf {

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
  // at most ELEMS values, a compile-time count per thread: every load is issued before the first is used
  // (one load per loop iteration would wait for its own data)
  constexpr int MI = FftCfg<T>::ELEMS / kFftThreads;
  const int cnt = np * N2;
  Tin sa[MI], sb[MI];
#pragma unroll
  for (int it = 0; it < MI; ++it) {
    const int idx = min((int)threadIdx.x + it * kFftThreads, cnt - 1);
    const size_t ra = (size_t)(row0 + 2 * (idx / N2)) * N2 + idx % N2;
    sa[it] = src[ra];
    sb[it] = src[ra + N2];
  }
#pragma unroll
  for (int it = 0; it < MI; ++it) {
    const int idx = (int)threadIdx.x + it * kFftThreads;
    if (idx < cnt) buf[idx] = {(T)sa[it], (T)sb[it]};
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
  // packed rows -> A + i B: every load issued first, from the one packed index each value needs (a load
  // behind a branch waits for its own data); the four cases are selects
  constexpr int MI = FftCfg<T>::ELEMS / kFftThreads;
  const int cnt = np * N2;
  C2<T> ra[MI], rb[MI];
#pragma unroll
  for (int it = 0; it < MI; ++it) {
    const int idx = min((int)threadIdx.x + it * kFftThreads, cnt - 1);
    const int p = idx / N2, k = idx % N2;
    const int ks = (k == 0 || k == H) ? 0 : (k < H ? k : N2 - k);
    const C2<T>* PA = src + (size_t)(row0 + 2 * p) * H;
    ra[it] = PA[ks];
    rb[it] = PA[H + ks];
  }
#pragma unroll
  for (int it = 0; it < MI; ++it) {
    const int idx = (int)threadIdx.x + it * kFftThreads;
    if (idx >= cnt) continue;
    const int k = idx % N2;
    const C2<T> a = k == 0 ? C2<T>{ra[it].x, (T)0} : k == H ? C2<T>{ra[it].y, (T)0}
                  : k < H ? ra[it] : C2<T>{ra[it].x, -ra[it].y};
    const C2<T> b = k == 0 ? C2<T>{rb[it].x, (T)0} : k == H ? C2<T>{rb[it].y, (T)0}
                  : k < H ? rb[it] : C2<T>{rb[it].x, -rb[it].y};
    buf[idx] = {a.x - b.y, a.y + b.x};   // A + i B
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
  kColFwdMult = 1,   // FFT, times lambda^{-1/2} scale                      (Lambda^{-1/2} F b)
  kColInvOut = 3,    // times lambda^{-1/2} scale, inverse FFT              (x = F^H Lambda^{-1/2} u)
  kColApply = 4      // FFT, times lambda^{-1/2} scale, inverse FFT         (M^{-1/2} on its own)
};

template <typename T, int MODE>
__global__ __launch_bounds__(kFftThreads) void k_cols(const C2<T>* __restrict__ in, C2<T>* __restrict__ out,
                                                      int N1, int H, int nf, const C2<T>* __restrict__ tw,
                                                      const T* __restrict__ mult, T scale) {
  __shared__ C2<T> buf[FftCfg<T>::ELEMS];
  const int r = blockIdx.y;
  const int c0 = xcd_col_block(blockIdx.x, gridDim.x) * nf;
  const size_t fsz = (size_t)N1 * H;   // complex values per field
  const C2<T>* src = in + (size_t)r * fsz;
  {
    // every load issued before the first is used (one load per loop iteration would wait for its own data)
    constexpr int MI = FftCfg<T>::ELEMS / kFftThreads;
    const int cnt = nf * N1;
    C2<T> xv[MI];
#pragma unroll
    for (int it = 0; it < MI; ++it) {
      const int idx = min((int)threadIdx.x + it * kFftThreads, cnt - 1);
      xv[it] = src[(size_t)(idx / nf) * H + c0 + idx % nf];
    }
#pragma unroll
    for (int it = 0; it < MI; ++it) {
      const int idx = (int)threadIdx.x + it * kFftThreads;
      if (idx < cnt) buf[idx] = xv[it];
    }
  }
  if (MODE == kColInvOut) apply_mult(buf, nf, c0, N1, H, mult, scale);
  else __syncthreads();
  lds_fft<T, true>(buf, N1, nf, 1, nf, tw, MODE == kColInvOut);
  if (MODE == kColFwdMult) apply_mult(buf, nf, c0, N1, H, mult, scale);
  if (MODE == kColApply) {
    apply_mult(buf, nf, c0, N1, H, mult, scale);
    lds_fft<T, true>(buf, N1, nf, 1, nf, tw, true);
  }
  C2<T>* dst = out + (size_t)r * fsz;
  const T sc = (MODE == kColFwdInit) ? scale : (T)1;
  for (int idx = threadIdx.x; idx < nf * N1; idx += kFftThreads) {
    const int k1 = idx / nf, c = idx % nf;
    const C2<T> a = buf[idx];
    dst[(size_t)k1 * H + c0 + c] = {a.x * sc, a.y * sc};
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
  std::vector<double> m1(N1), m2(N2);
  for (int k = 0; k < N1; ++k) m1[k] = periodic_mu(k, N1);
  for (int k = 0; k < N2; ++k) m2[k] = periodic_mu(k, N2);
  if (hipMalloc(&p.tw64_1, t1.size() * 8) != hipSuccess || hipMalloc(&p.tw64_2, t2.size() * 8) != hipSuccess ||
      hipMalloc(&p.tw32_1, f1.size() * 4) != hipSuccess || hipMalloc(&p.tw32_2, f2.size() * 4) != hipSuccess ||
      hipMalloc(&p.mu1, m1.size() * 8) != hipSuccess || hipMalloc(&p.mu2, m2.size() * 8) != hipSuccess)
    return GMRF_ENOMEM;
  if (hipMemcpy(p.mu1, m1.data(), m1.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p.mu2, m2.data(), m2.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
    return GMRF_EDEVICE;
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
  if (p.mu1) (void)hipFree(p.mu1);
  if (p.mu2) (void)hipFree(p.mu2);
  p = FftPlan{};
}

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
static void cols(const FftPlan& p, const T* in, T* out, const T* mult, T scale, int k, hipStream_t st) {
  const int nf = col_nf<T>(p);
  hipLaunchKernelGGL((k_cols<T, MODE>), dim3(p.H / nf, k), dim3(kFftThreads), 0, st, (const C2<T>*)in,
                     (C2<T>*)out, p.N1, p.H, nf, tw1<T>(p), mult, scale);
}

template <typename T>
void fft_apply_inv_sqrt_M(const FftPlan& p, const T* mult, const T* X, T* Y, T* tmp, int k, hipStream_t st) {
  const long n = (long)p.N1 * p.N2;
  rows_r2c<T, T>(p, X, n, tmp, n / 2, (T)1, nullptr, k, st);
  cols<T, kColApply>(p, tmp, tmp, mult, (T)(1.0 / (double)n), k, st);
  rows_c2r<T, T>(p, tmp, n / 2, Y, n, (T)1, nullptr, k, st);
}

template <typename T>
void fft_forward_init(const FftPlan& p, const double* Z, T* V0, T* tmp, const LzState& S, int k, hipStream_t st) {
  const long n = (long)p.N1 * p.N2;
  rows_r2c<double, T>(p, Z, n, tmp, n / 2, (T)1, nullptr, k, st);
  cols<T, kColFwdInit>(p, tmp, V0, nullptr, (T)(1.0 / std::sqrt((double)n)), k, st);
  launch_norm_partials<T>(V0, n, S, st);
}

template <typename T>
void fft_forward_init_mult(const FftPlan& p, const void* mult, const double* B, T* V0, T* tmp, const LzState& S, int k,
                           hipStream_t st) {
  const long n = (long)p.N1 * p.N2;
  rows_r2c<double, T>(p, B, n, tmp, n / 2, (T)1, nullptr, k, st);
  cols<T, kColFwdMult>(p, tmp, V0, (const T*)mult, (T)(1.0 / std::sqrt((double)n)), k, st);
  launch_norm_partials<T>(V0, n, S, st);
}

template <typename T>
void fft_forward_init_probes(const FftPlan& p, uint64_t seed, int p0, const int8_t* probes, T* real_tmp, T* V0,
                             T* tmp, const LzState& S, int k, hipStream_t st, const int32_t* colour, int K) {
  const long n = (long)p.N1 * p.N2;
  if (probes) launch_init_from_i8<T>(probes, n, real_tmp, S, st);
  else launch_init_rademacher<T>(seed, n, p0, real_tmp, S, st, colour, K);
  rows_r2c<T, T>(p, real_tmp, n, tmp, n / 2, (T)1, nullptr, k, st);
  cols<T, kColFwdInit>(p, tmp, V0, nullptr, (T)(1.0 / std::sqrt((double)n)), k, st);
  launch_norm_partials<T>(V0, n, S, st);
}

template <typename T>
void fft_backward_output(const FftPlan& p, const void* mult, const T* U, double* X, T* tmp, const LzState& S,
                         int k, hipStream_t st) {
  const long n = (long)p.N1 * p.N2;
  cols<T, kColInvOut>(p, U, tmp, (const T*)mult, (T)(1.0 / std::sqrt((double)n)), k, st);
  rows_c2r<T, double>(p, tmp, n / 2, X, n, (T)1, nullptr, k, st);
}

#define INST(T)                                                                                            \
  template void fft_apply_inv_sqrt_M<T>(const FftPlan&, const T*, const T*, T*, T*, int, hipStream_t);     \
  template void fft_forward_init<T>(const FftPlan&, const double*, T*, T*, const LzState&, int, hipStream_t); \
  template void fft_forward_init_mult<T>(const FftPlan&, const void*, const double*, T*, T*, const LzState&, int, hipStream_t); \
  template void fft_forward_init_probes<T>(const FftPlan&, uint64_t, int, const int8_t*, T*, T*, T*, const LzState&, int, hipStream_t, const int32_t*, int); \
  template void fft_backward_output<T>(const FftPlan&, const void*, const T*, double*, T*, const LzState&, int, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace gmrf
