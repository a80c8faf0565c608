// The m x m tridiagonal step (FP64): y = T^{-1/2} e_1 for the sample (Algorithm 1, final
// step) and e_1^T log(T) e_1 for the Gauss quadrature of the log-det estimator (Section 6).
//
// The caption of Algorithm 1 suggests replacing T^{-1/2} by a rational approximation.  This
// file uses one that needs no eigenvectors, so clustered or repeated Ritz values cost
// nothing extra and every shift is independent (one GPU thread each):
//   lambda^{-1/2} = (2/pi) int_R e^s / (e^{2s} + lambda) ds,
//   log(lambda)   = int_R e^s ( 1/(1 + e^s) - 1/(lambda + e^s) ) ds,
// discretised by the trapezoidal rule in s.  The integrands are analytic in the strips
// |Im s| < pi/2 and |Im s| < pi, so steps h = 1/4 and h = 1/2 give errors near 1e-16; the
// truncation points sit 37 e-folds beyond the spectrum [lo, hi] of T (for the log, beyond
// [min(lo, 1), max(hi, 1)], where its integrand's tails begin), whose upper end is a
// Gershgorin bound and whose lower end comes from Sturm counts (LDL^T inertia of T - x I)
// at x = hi * 2^{-t/2}, t = 0..255, which also certifies that T is positive definite.
// Each node needs (T + sigma I)^{-1} e_1: with the backward pivots
//   d_{m-1} = alpha_{m-1} + sigma,  d_i = alpha_i + sigma - beta_i^2 / d_{i+1},
// its entries are y_0 = 1/d_0, y_{i+1} = -(beta_i / d_{i+1}) y_i, and (T+sigma)^{-1}_{00} = 1/d_0.
// Sums over nodes are fixed-order (lanes, wave butterflies, node blocks in order): deterministic.
// Up to kTriLdsM steps T and the output accumulator are staged in LDS; longer recurrences (unpreconditioned
// runs on ill-conditioned fields take a few thousand steps) read T from global memory and accumulate in the
// output row, with the same arithmetic in the same order, so both forms give the same bits.
#include "kernels.hpp"

namespace gmrf {

constexpr int kTriThreads = 256;
// T^{-1/2} e_1 takes 512 threads: one node block holds every quadrature node up to an eigenvalue
// spread of e^107, so the per-node recurrences over m run once
constexpr int kTriInvThreads = 512;
constexpr int kTriLdsM = 1024;      // T in LDS up to this many steps
constexpr int kTriMaxM = 16384;     // longest recurrence the tridiagonal step accepts
constexpr double kPad = 37.0;

struct TriArgs {
  const double* alpha;
  int lda, a_off;
  const double* beta;
  int ldb, b_off;
  const int* m;         // nullptr: use m_fixed
  int m_fixed;
  const int* status_in; // nullptr or per-RHS status; a non-OK entry is skipped
  double* out;          // y (ldy per RHS) or scalar per RHS
  int ldy;
  int* status_out;      // may be nullptr; only written (ENOTSPD) when T is not SPD
  double* scratch;      // [k][scr_m][kTriInvThreads] for the sample
  int scr_m;
};

// Spectrum bracket of T (LDS copies a, b of length m): returns false if T is not SPD.
template <int NT>
__device__ bool tri_bracket(const double* a, const double* b, int m, double* red, int* ired,
                            double& lo, double& hi) {
  double g = 0.0;
  for (int i = threadIdx.x; i < m; i += NT) {
    const double bl = i > 0 ? fabs(b[i - 1]) : 0.0, br = i + 1 < m ? fabs(b[i]) : 0.0;
    g = fmax(g, a[i] + bl + br);
  }
  hi = block_max<NT>(g, red);
  // Sturm count at x_t = hi 2^{-t/2}: number of negative pivots of T - x I
  const int t = threadIdx.x;
  const double x = hi * exp2(-0.5 * (double)t);
  int neg = 0;
  double d = a[0] - x;
  if (d <= 0.0) ++neg;
  for (int i = 1; i < m; ++i) {
    if (d == 0.0) d = -1e-300;
    d = a[i] - x - b[i - 1] * b[i - 1] / d;
    if (d <= 0.0) ++neg;
  }
  int cand = (neg == 0) ? t : 1 << 30;
  cand = wave_min_int(cand);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) ired[threadIdx.x / kWave] = cand;
  __syncthreads();
  int best = 1 << 30;
  for (int w = 0; w < NT / kWave; ++w) best = min(best, ired[w]);
  if (!(hi > 0.0) || !isfinite(hi) || best >= (1 << 30)) return false;
  lo = hi * exp2(-0.5 * (double)best);
  return true;
}

// T of column r: copied into the LDS arrays sa, sb (LDS form) or read in place (b[m-1] is never read)
template <bool LDS>
__device__ void tri_view(const TriArgs& A, int r, int m, double* sa, double* sb, const double*& a, const double*& b) {
  const double* ga = A.alpha + (size_t)r * A.lda + A.a_off;
  const double* gb = A.beta + (size_t)r * A.ldb + A.b_off;
  if constexpr (LDS) {
    for (int i = threadIdx.x; i < m; i += kTriThreads) {
      sa[i] = ga[i];
      sb[i] = (i + 1 < m) ? gb[i] : 0.0;
    }
    __syncthreads();
    a = sa;
    b = sb;
  } else {
    a = ga;
    b = gb;
  }
}

// Per node (one thread each): the backward pivots leave q_i = beta_i / d_{i+1} in the scratch rows, the
// forward recurrence overwrites row i with w y_i (loads taken eight rows ahead, no cross-lane work in the
// chain); then each thread sums whole rows over the block's nodes in node order, and the accumulator adds
// the node blocks in order.
template <bool LDS>
__global__ __launch_bounds__(kTriInvThreads) void k_tri_invsqrt(TriArgs A) {
  constexpr int LM = LDS ? kTriLdsM : 1;
  __shared__ double sa[LM], sb[LM], sacc[LM];
  __shared__ double red[kTriInvThreads / kWave];
  __shared__ int ired[kTriInvThreads / kWave];
  const int r = blockIdx.x;
  // m never exceeds the LDS copy, the scratch rows or the output row
  const int m = min(min(A.m ? A.m[r] : A.m_fixed, LDS ? kTriLdsM : kTriMaxM), min(A.scr_m, A.ldy));
  double* y = A.out + (size_t)r * A.ldy;
  if (A.status_in && A.status_in[r] != kOK && A.status_in[r] != kENOCONV) return;
  if (m <= 0) return;
  const double *a, *b;
  tri_view<LDS>(A, r, m, sa, sb, a, b);
  double* acc = LDS ? sacc : y;     // the node blocks' sums, in order
  double lo, hi;
  const bool spd = tri_bracket<kTriInvThreads>(a, b, m, red, ired, lo, hi);
  if (!spd) {
    if (threadIdx.x == 0 && A.status_out) A.status_out[r] = kENOTSPD;
    return;
  }
  const double h = 0.25;
  const double s_lo = 0.5 * log(lo) - kPad, s_hi = 0.5 * log(hi) + kPad;
  const int nq = (int)ceil((s_hi - s_lo) / h) + 1;
  constexpr int AH = 8;   // rows loaded ahead in the forward recurrence
  // each row's sum is kept by the thread that adds to it (thread i mod kTriInvThreads), which also clears it
  for (int i = threadIdx.x; i < m; i += kTriInvThreads) acc[i] = 0.0;
  double* rs = A.scratch + (size_t)r * A.scr_m * kTriInvThreads;
  for (int base = 0; base < nq; base += kTriInvThreads) {
    const int l = base + threadIdx.x;
    const double s = s_lo + h * (double)l;
    const double es = exp(s);
    const double sigma = es * es;
    const double wgt = l < nq ? (2.0 / M_PI) * h * es : 0.0;
    // backward pivots; row i holds q_i = beta_i / d_{i+1}
    double d = a[m - 1] + sigma;
    for (int i = m - 2; i >= 0; --i) {
      const double q = b[i] / d;
      rs[(size_t)i * kTriInvThreads + threadIdx.x] = q;
      d = a[i] + sigma - b[i] * q;
    }
    // forward: y_0 = 1 / d_0, y_i = -q_{i-1} y_{i-1}; row i-1 then receives w y_{i-1}
    double yi = 1.0 / d;
    for (int i0 = 1; i0 < m; i0 += AH) {
      double qv[AH];
#pragma unroll
      for (int u = 0; u < AH; ++u) qv[u] = i0 + u < m ? rs[(size_t)(i0 + u - 1) * kTriInvThreads + threadIdx.x] : 0.0;
#pragma unroll
      for (int u = 0; u < AH; ++u) {
        if (i0 + u < m) {
          rs[(size_t)(i0 + u - 1) * kTriInvThreads + threadIdx.x] = wgt * yi;
          yi = -qv[u] * yi;
        }
      }
    }
    rs[(size_t)(m - 1) * kTriInvThreads + threadIdx.x] = wgt * yi;
    __syncthreads();   // the block's rows are complete in memory
    // row sums: thread t takes rows t, t + kTriInvThreads, ... and adds the row's nodes in order, 16 bytes per
    // load with all of a row's loads independent (no cross-lane step in the chain)
    for (int i = threadIdx.x; i < m; i += kTriInvThreads) {
      const double2* row = (const double2*)(rs + (size_t)i * kTriInvThreads);
      double v = 0.0;
#pragma unroll 16
      for (int c = 0; c < kTriInvThreads / 2; ++c) {
        const double2 pr = row[c];
        v += pr.x;
        v += pr.y;
      }
      acc[i] += v;
    }
    __syncthreads();   // the rows are rewritten by the next node block
  }
  if constexpr (LDS)
    for (int i = threadIdx.x; i < m; i += kTriInvThreads) y[i] = acc[i];
}

template <bool LDS>
__global__ __launch_bounds__(kTriThreads) void k_tri_log(TriArgs A) {
  constexpr int LM = LDS ? kTriLdsM : 1;
  __shared__ double sa[LM], sb[LM];
  __shared__ double red[kTriThreads / kWave];
  __shared__ int ired[kTriThreads / kWave];
  const int r = blockIdx.x;
  const int m = min(A.m ? A.m[r] : A.m_fixed, min(LDS ? kTriLdsM : kTriMaxM, A.lda));
  if (A.status_in && A.status_in[r] != kOK && A.status_in[r] != kENOCONV) return;
  if (m <= 0) return;
  const double *a, *b;
  tri_view<LDS>(A, r, m, sa, sb, a, b);
  double lo, hi;
  const bool spd = tri_bracket<kTriThreads>(a, b, m, red, ired, lo, hi);
  if (!spd) {
    if (threadIdx.x == 0) {
      if (A.status_out) A.status_out[r] = kENOTSPD;
      A.out[(size_t)r * A.ldy] = __longlong_as_double(0x7ff8000000000000ll);
    }
    return;
  }
  // the integrand decays like e^s below min(log lo, 0) and like e^{-s} above max(log hi, 0): the window
  // covers both ends of the spectrum and the switch of 1/(1 + e^s) at s = 0
  const double h = 0.5;
  const double s_lo = fmin(log(lo), 0.0) - kPad, s_hi = fmax(log(hi), 0.0) + kPad;
  const int nq = (int)ceil((s_hi - s_lo) / h) + 1;
  double acc = 0.0;
  for (int l = threadIdx.x; l < nq; l += kTriThreads) {
    const double s = s_lo + h * (double)l;
    const double sigma = exp(s);
    double d = a[m - 1] + sigma;
    for (int i = m - 2; i >= 0; --i) d = a[i] + sigma - b[i] * b[i] / d;
    acc += h * sigma * (1.0 / (1.0 + sigma) - 1.0 / d);
  }
  const double tot = block_sum<kTriThreads>(acc, red);
  if (threadIdx.x == 0) A.out[(size_t)r * A.ldy] = tot;
}

// y = T^{-1} e_1 for the linear solve x_m = ||b|| V_m T_m^{-1} e_1: backward pivots d_{m-1} = alpha_{m-1},
// d_i = alpha_i - beta_i^2 / d_{i+1}, then y_0 = 1 / d_0, y_{i+1} = -(beta_i / d_{i+1}) y_i (the sigma = 0
// case of the shifted solves above).  One thread per right-hand side; a non-positive pivot is ENOTSPD.
__global__ __launch_bounds__(kTriThreads) void k_tri_solve(TriArgs A, int k) {
  const int r = blockIdx.x * kTriThreads + threadIdx.x;
  if (r >= k) return;
  const int m = A.m ? A.m[r] : A.m_fixed;
  double* y = A.out + (size_t)r * A.ldy;
  if ((A.status_in && A.status_in[r] != kOK && A.status_in[r] != kENOCONV) || m <= 0) return;
  const double* al = A.alpha + (size_t)r * A.lda + A.a_off;
  const double* be = A.beta + (size_t)r * A.ldb + A.b_off;
  // pass 1: backward pivots into y (reused as scratch), checking definiteness
  double d = al[m - 1];
  bool ok = d > 0.0;
  y[m - 1] = d;
  for (int i = m - 2; i >= 0; --i) {
    d = al[i] - be[i] * be[i] / d;
    ok = ok && d > 0.0;
    y[i] = d;
  }
  if (!ok) {
    if (A.status_out) A.status_out[r] = kENOTSPD;
    return;
  }
  // pass 2: y_0 = 1 / d_0, y_{i+1} = -(beta_i / d_{i+1}) y_i
  double yi = 1.0 / y[0];
  y[0] = yi;
  for (int i = 0; i + 1 < m; ++i) {
    yi = -(be[i] / y[i + 1]) * yi;
    y[i + 1] = yi;
  }
}

void launch_tri_solve(const double* alpha, int lda, int a_off, const double* beta, int ldb, int b_off, const int* m,
                      int m_fixed, const int* status_in, double* y, int ldy, int* status_out, int k, hipStream_t st) {
  TriArgs A{alpha, lda, a_off, beta, ldb, b_off, m, m_fixed, status_in, y, ldy, status_out, nullptr, 0};
  hipLaunchKernelGGL(k_tri_solve, dim3((k + kTriThreads - 1) / kTriThreads), dim3(kTriThreads), 0, st, A, k);
}

int tri_max_m() { return kTriMaxM; }
size_t tri_scratch_doubles(int k, int m_cap) { return (size_t)k * m_cap * kTriInvThreads; }

void launch_tri_invsqrt(const double* alpha, int lda, int a_off, const double* beta, int ldb, int b_off,
                        const int* m, int m_fixed, const int* status_in, double* y, int ldy,
                        int* status_out, double* scratch, int scr_m, int k, hipStream_t st) {
  TriArgs A{alpha, lda, a_off, beta, ldb, b_off, m, m_fixed, status_in, y, ldy, status_out, scratch, scr_m};
  // the form follows the caller's capacity (scratch rows), never the data, so a column gets the same form
  // whichever m it stopped at
  if (scr_m <= kTriLdsM) hipLaunchKernelGGL(k_tri_invsqrt<true>, dim3(k), dim3(kTriInvThreads), 0, st, A);
  else hipLaunchKernelGGL(k_tri_invsqrt<false>, dim3(k), dim3(kTriInvThreads), 0, st, A);
}

void launch_tri_log(const double* alpha, int lda, int a_off, const double* beta, int ldb, int b_off,
                    const int* m, int m_fixed, const int* status_in, double* out, int ldo,
                    int* status_out, int k, hipStream_t st) {
  TriArgs A{alpha, lda, a_off, beta, ldb, b_off, m, m_fixed, status_in, out, ldo, status_out, nullptr, 0};
  // the row holds lda - a_off steps: the form follows that capacity
  if (lda - a_off <= kTriLdsM) hipLaunchKernelGGL(k_tri_log<true>, dim3(k), dim3(kTriThreads), 0, st, A);
  else hipLaunchKernelGGL(k_tri_log<false>, dim3(k), dim3(kTriThreads), 0, st, A);
}

}  // namespace gmrf
