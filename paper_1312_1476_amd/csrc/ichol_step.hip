// Incomplete-Cholesky preconditioned Lanczos step (Section 5.2, Proposition 1 with F = L):
// A v = L^{-1} Q L^{-T} v as a backward solve, the operator, a forward solve; then the opener below and
// the update kernel finish Algorithm 1's step.  The triangular solves are sequential by nature: rows run
// level by level (a level holds rows whose dependencies all lie in earlier levels), one block per
// right-hand side with a barrier between levels, so no block ever waits on another.
#include "ichol.hpp"
#include "kernels.hpp"

namespace gmrf {

constexpr int kTrsvThreads = 1024;
constexpr int64_t kTrsvLdsRows = 8192;   // x of up to this many rows is kept in LDS (64 KB of FP64)
constexpr size_t kTrsvLdsMaxBytes = 160 * 1024;   // whole solve in LDS up to the CU's LDS size

// x = T^{-1} b, T = D + N with N strictly triangular, stored in level order (TrsvDev).  Only the x
// values carry the dependency between levels; every row's indices and values are known in advance.
// XLDS: x lives in LDS (n <= kTrsvLdsRows) and is written out once at the end.
template <typename T, typename OutT, bool XLDS>
__global__ __launch_bounds__(kTrsvThreads) void k_trsv_levels(const int32_t* __restrict__ lvl_ptr,
                                                              const int32_t* __restrict__ rows,
                                                              const int64_t* __restrict__ rp,
                                                              const int32_t* __restrict__ ci,
                                                              const T* __restrict__ va, const T* __restrict__ dinv,
                                                              int nlev, long n, const T* __restrict__ B, long bld,
                                                              OutT* X, long xld, const int* __restrict__ active) {
  extern __shared__ double xs[];
  const int r = blockIdx.x;
  if (active && !active[r]) return;   // one value per block: the whole block returns or none does
  const T* b = B + (size_t)r * bld;
  OutT* x = X + (size_t)r * xld;
  for (int lev = 0; lev < nlev; ++lev) {
    const int e0 = lvl_ptr[lev], e1 = lvl_ptr[lev + 1];
    for (int p = e0 + (int)threadIdx.x; p < e1; p += kTrsvThreads) {
      const int i = rows[p];
      double s = (double)b[i];
      const int64_t q1 = rp[p + 1];
      int64_t e = rp[p];
      for (; e + 3 < q1; e += 4) {   // four entries' loads issued before the sums (same order)
        int c[4];
        double xv[4], lv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          c[u] = ci[e + u];
          lv[u] = (double)va[e + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = XLDS ? xs[c[u]] : (double)x[c[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) s -= lv[u] * xv[u];
      }
      for (; e < q1; ++e) s -= (double)va[e] * (XLDS ? xs[ci[e]] : (double)x[ci[e]]);
      s *= (double)dinv[p];
      if (XLDS) xs[i] = s;
      else x[i] = (OutT)s;
    }
    __syncthreads();   // this level's x are visible to the block before the next level reads them
  }
  if (XLDS)
    for (long i = threadIdx.x; i < n; i += kTrsvThreads) x[i] = (OutT)xs[i];
}

// The same solve with the whole factor in LDS as well (values, column indices, row starts, level
// pointers and 1 / l_ii), staged once per block: every level's loads are then LDS loads, not two
// dependent L2 round trips.  x starts as b in LDS (a row's own entry is read only by itself).  Same
// arithmetic in the same order as k_trsv_levels.
template <typename T, typename OutT>
__global__ __launch_bounds__(kTrsvThreads) void k_trsv_lds(const int32_t* __restrict__ lvl_ptr,
                                                           const int32_t* __restrict__ rows,
                                                           const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const T* __restrict__ va, const T* __restrict__ dinv,
                                                           int nlev, long n, long nnz, const T* __restrict__ B,
                                                           long bld, OutT* X, long xld,
                                                           const int* __restrict__ active) {
  extern __shared__ double smem[];
  const int r = blockIdx.x;
  if (active && !active[r]) return;   // one value per block: the whole block returns or none does
  double* xs = smem;
  T* sd = (T*)(xs + n);
  T* sv = sd + n;
  int32_t* srp = (int32_t*)(sv + nnz);
  int32_t* sci = srp + n + 1;
  int32_t* srow = sci + nnz;
  int32_t* slv = srow + n;
  const T* b = B + (size_t)r * bld;
  for (long i = threadIdx.x; i < n; i += kTrsvThreads) {
    xs[i] = (double)b[i];
    sd[i] = dinv[i];
    srow[i] = rows[i];
  }
  for (long i = threadIdx.x; i <= n; i += kTrsvThreads) srp[i] = (int32_t)rp[i];
  for (long e = threadIdx.x; e < nnz; e += kTrsvThreads) {
    sv[e] = va[e];
    sci[e] = ci[e];
  }
  for (int l = threadIdx.x; l <= nlev; l += kTrsvThreads) slv[l] = lvl_ptr[l];
  __syncthreads();
  for (int lev = 0; lev < nlev; ++lev) {
    const int e0 = slv[lev], e1 = slv[lev + 1];
    for (int p = e0 + (int)threadIdx.x; p < e1; p += kTrsvThreads) {
      const int i = srow[p];
      double s = xs[i];
      const int q1 = srp[p + 1];
      int e = srp[p];
      for (; e + 3 < q1; e += 4) {   // four entries' index and x loads issued before the sums (same order)
        int c[4];
        double xv[4], lv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[u] = sci[e + u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          xv[u] = xs[c[u]];
          lv[u] = (double)sv[e + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) s -= lv[u] * xv[u];
      }
      for (; e < q1; ++e) s -= (double)sv[e] * xs[sci[e]];
      xs[i] = s * (double)sd[p];
    }
    __syncthreads();   // this level's x are visible to the block before the next level reads them
  }
  OutT* x = X + (size_t)r * xld;
  for (long i = threadIdx.x; i < n; i += kTrsvThreads) x[i] = (OutT)xs[i];
}

// LDS bytes of k_trsv_lds for a solve (0: does not fit)
template <typename T>
static size_t trsv_lds_bytes(const TrsvDev& d, int64_t n) {
  const size_t b = (size_t)n * 8 + (size_t)(n + d.nnz) * sizeof(T) + (size_t)(2 * n + 1 + d.nnz + d.nlev + 1) * 4;
  return b <= kTrsvLdsMaxBytes ? b : 0;
}

// Opener of iteration j plus q = AX / beta_{j-1} - beta_{j-1} v_{j-1} and partial sums of v_j^T q.
template <typename T>
__global__ __launch_bounds__(kEwThreads) void k_pre_lz(const T* __restrict__ AX, const T* __restrict__ Xj,
                                                       const T* __restrict__ Xprev, T* __restrict__ Qb, long L,
                                                       LzState S, int j) {
  __shared__ double lds[kEwThreads / kWave];
  __shared__ int flag;
  const int r = blockIdx.y;
  double s_cur, s_prev, bprev;
  if (!lz_open<kEwThreads>(S, r, j, blockIdx.x == 0, lds, &flag, s_cur, s_prev, bprev)) return;
  const size_t off = (size_t)r * L;
  const long base = (long)blockIdx.x * kEwChunk + threadIdx.x;
  double acc = 0.0;
  for (int q = 0; q < kEwPerThread; ++q) {
    const long e = base + (long)q * kEwThreads;
    if (e < L) {
      const double v = (double)(T)((double)Xj[off + e] * s_cur);
      double qv = (double)AX[off + e] * s_cur;
      if (j > 1) qv -= bprev * (double)(T)((double)Xprev[off + e] * s_prev);
      const T qt = (T)qv;
      Qb[off + e] = qt;
      acc += v * (double)qt;
    }
  }
  const double s = block_sum<kEwThreads>(acc, lds);
  if (threadIdx.x == 0) S.part_a[(size_t)r * S.pstride + blockIdx.x] = s;
}

template <typename T, typename OutT>
void launch_trsv(const IcholDev& f, bool upper, const T* B, long bld, OutT* X, long xld, const int* active, int k,
                 hipStream_t st) {
  const TrsvDev& d = upper ? f.bwd : f.fwd;
  const size_t lb = trsv_lds_bytes<T>(d, f.n);
  if (lb) {
    // the launch needs more than the default dynamic LDS; set once (thread-safe static initialisation)
    static const bool attr_set = [] {
      const bool ok = hipFuncSetAttribute((const void*)k_trsv_lds<T, OutT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)kTrsvLdsMaxBytes) == hipSuccess;
      (void)hipGetLastError();
      return ok;
    }();
    if (attr_set || lb <= 65536) {
      hipLaunchKernelGGL((k_trsv_lds<T, OutT>), dim3(k), dim3(kTrsvThreads), lb, st, d.lvl_ptr, d.rows, d.rp, d.ci,
                         (const T*)d.va, (const T*)d.dinv, d.nlev, (long)f.n, (long)d.nnz, B, bld, X, xld, active);
      return;
    }
  }
  if (f.n <= kTrsvLdsRows)
    hipLaunchKernelGGL((k_trsv_levels<T, OutT, true>), dim3(k), dim3(kTrsvThreads), (size_t)f.n * sizeof(double), st,
                       d.lvl_ptr, d.rows, d.rp, d.ci, (const T*)d.va, (const T*)d.dinv, d.nlev, (long)f.n, B, bld,
                       X, xld, active);
  else
    hipLaunchKernelGGL((k_trsv_levels<T, OutT, false>), dim3(k), dim3(kTrsvThreads), 0, st, d.lvl_ptr, d.rows, d.rp,
                       d.ci, (const T*)d.va, (const T*)d.dinv, d.nlev, (long)f.n, B, bld, X, xld, active);
}

template <typename T>
void launch_pre_lz(const T* AX, const T* Xj, const T* Xprev, T* Qb, long L, const LzState& S, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_pre_lz<T>, dim3((unsigned)ew_blocks(L), S.k), dim3(kEwThreads), 0, st, AX, Xj, Xprev, Qb, L,
                     S, j);
}

template void launch_trsv<double, double>(const IcholDev&, bool, const double*, long, double*, long, const int*, int,
                                          hipStream_t);
template void launch_trsv<float, float>(const IcholDev&, bool, const float*, long, float*, long, const int*, int,
                                        hipStream_t);
template void launch_trsv<float, double>(const IcholDev&, bool, const float*, long, double*, long, const int*, int,
                                         hipStream_t);
template void launch_pre_lz<double>(const double*, const double*, const double*, double*, long, const LzState&, int,
                                    hipStream_t);
template void launch_pre_lz<float>(const float*, const float*, const float*, float*, long, const LzState&, int,
                                   hipStream_t);

}  // namespace gmrf
