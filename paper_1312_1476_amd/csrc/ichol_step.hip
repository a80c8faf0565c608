// Incomplete-Cholesky preconditioned Lanczos step (Section 5.2, Proposition 1 with F = L):
// A v = L^{-1} Q L^{-T} v as a backward solve, the operator, a forward solve; then the opener below and
// the update kernel finish Algorithm 1's step.  The triangular solves are sequential by nature: rows run
// level by level (a level holds rows whose dependencies all lie in earlier levels), one block per
// right-hand side, so no block ever waits on another: a barrier separates the levels, or, where every
// level fits one wave, that wave takes them all in order.
#include "ichol.hpp"
#include "kernels.hpp"

namespace gmrf {

constexpr int kTrsvThreads = 1024;
constexpr int64_t kTrsvLdsRows = 8192;   // x of up to this many rows is kept in LDS (64 KB of FP64)
constexpr size_t kTrsvLdsMaxBytes = 160 * 1024;   // whole solve in LDS up to the CU's LDS size

// x = T^{-1} b, T = D + N with N strictly triangular, stored in level order (TrsvDev).  Only the x
// values carry the dependency between levels; every row's indices and values are known in advance.
// G lanes share a row: lane g takes the row's entries g, g + G, ..., four of them per round with all
// loads issued before the sums, and the G partial sums are added across the lanes by DPP (lane 0 of
// the group starts from b_i).  G = 1 is one thread per row with the entries summed in order.  The
// level's rows go in passes of kTrsvThreads / G.
template <int G>
__device__ __forceinline__ double trsv_group_sum(double v) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "a lane group lies within one DPP row");
  if (G >= 2) v += dpp<kDppQuadXor1>(v);
  if (G >= 4) v += dpp<kDppQuadXor2>(v);
  if (G >= 8) v += dpp<kDppRowHalfMirror>(v);
  if (G >= 16) v += dpp<kDppRowMirror>(v);
  return v;
}

// s -= sum over the entries q of the row taken by lane g (g, g + G, ... below q1) of va[q] x[ci[q]]; an
// entry past the row's end is loaded from the round's first entry (in range) and counts with value 0.
template <int G, typename Idx, typename LoadC, typename LoadV, typename LoadX>
__device__ __forceinline__ double trsv_row(double s, Idx q0, Idx q1, int g, LoadC lc, LoadV lv_, LoadX lx) {
  for (Idx e = q0 + g; e < q1; e += 4 * G) {
    int c[4];
    double xv[4], lv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const Idx eu = e + u * G;
      const Idx ec = eu < q1 ? eu : e;
      c[u] = lc(ec);
      const double v = lv_(ec);
      lv[u] = eu < q1 ? v : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) xv[u] = lx(c[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) s -= lv[u] * xv[u];
  }
  return s;
}

// XLDS: x lives in LDS (n <= kTrsvLdsRows) and is written out once at the end.
template <typename T, typename OutT, bool XLDS, int G>
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
  const int g = (int)threadIdx.x % G;
  for (int lev = 0; lev < nlev; ++lev) {
    const int e0 = lvl_ptr[lev], e1 = lvl_ptr[lev + 1];
    for (int pb = e0; pb < e1; pb += kTrsvThreads / G) {   // the same trip count in every lane
      const int p = pb + (int)threadIdx.x / G;
      const bool live = p < e1;
      const int pc = live ? p : e0;   // a lane past the level's end works on its first row and writes nothing
      const int i = rows[pc];
      const int64_t q0 = rp[pc], q1 = live ? rp[pc + 1] : q0;
      const double bi = (double)b[i];
      double s = g == 0 ? bi : 0.0;
      s = trsv_row<G>(s, q0, q1, g, [&](int64_t q) { return ci[q]; }, [&](int64_t q) { return (double)va[q]; },
                      [&](int c) { return XLDS ? xs[c] : (double)x[c]; });
      s = trsv_group_sum<G>(s);
      const double di = (double)dinv[pc];
      if (live && g == 0) {
        s *= di;
        if (XLDS) xs[i] = s;
        else x[i] = (OutT)s;
      }
    }
    __syncthreads();   // this level's x are visible to the block before the next level reads them
  }
  if (XLDS)
    for (long i = threadIdx.x; i < n; i += kTrsvThreads) x[i] = (OutT)xs[i];
}

// The same solve with the factor's tables in LDS (row starts, rows, level pointers and 1 / l_ii),
// staged once per block, and with VLDS the entries too (values and column indices): every level's
// loads are then LDS loads, or without VLDS one L2 round for the entries, instead of three dependent
// rounds.  x starts as b in LDS (a row's own entry is read only by its own lane group).  Same
// arithmetic in the same order as k_trsv_levels with the same G.
// WAVE: 0 block form, 1 one wave with one pass per level, 2 one wave with up to two passes per level.
template <typename T, typename OutT, int G, bool VLDS, int WAVE>
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
  if (n <= 0 || (active && !active[r])) return;   // one value per block: the whole block returns or none does
  const long nv = VLDS ? nnz : 0;      // entries staged in LDS
  double* xs = smem;
  T* sd = (T*)(xs + n);
  T* sv = sd + n;
  int32_t* srp = (int32_t*)(sv + nv);
  int32_t* sci = srp + n + 1;
  int32_t* srow = sci + nv;
  int32_t* slv = srow + n;
  const T* b = B + (size_t)r * bld;
  // Staging in two passes, per-row tables (n + 1 >= nlev + 1 positions) and entries: a thread's loads
  // of a trip are issued before its LDS stores (clamped addresses, stores masked), so a pass costs a
  // memory round per kSU or kSE loop trips instead of one per trip.
  constexpr int kSU = 4, kSE = 8;
  for (long base = threadIdx.x; base <= n; base += kSU * kTrsvThreads) {
    double bv[kSU];
    T dv[kSU];
    int32_t rw[kSU], lp[kSU];
    int64_t rs[kSU];
#pragma unroll
    for (int u = 0; u < kSU; ++u) {
      const long t = base + (long)u * kTrsvThreads;
      const long tr = min(t, n - 1);
      bv[u] = (double)b[tr];
      dv[u] = dinv[tr];
      rw[u] = rows[tr];
      rs[u] = rp[min(t, n)];
      lp[u] = lvl_ptr[min(t, (long)nlev)];
    }
#pragma unroll
    for (int u = 0; u < kSU; ++u) {
      const long t = base + (long)u * kTrsvThreads;
      if (t < n) {
        xs[t] = bv[u];
        sd[t] = dv[u];
        srow[t] = rw[u];
      }
      if (t <= n) srp[t] = (int32_t)rs[u];
      if (t <= nlev) slv[t] = lp[u];
    }
  }
  for (long base = threadIdx.x; base < nv; base += kSE * kTrsvThreads) {
    T v[kSE];
    int32_t c[kSE];
#pragma unroll
    for (int u = 0; u < kSE; ++u) {
      const long e = min(base + (long)u * kTrsvThreads, nv - 1);
      v[u] = va[e];
      c[u] = ci[e];
    }
#pragma unroll
    for (int u = 0; u < kSE; ++u) {
      const long e = base + (long)u * kTrsvThreads;
      if (e < nv) {
        sv[e] = v[u];
        sci[e] = c[u];
      }
    }
  }
  __syncthreads();
  const int32_t* fc = VLDS ? sci : ci;
  const T* fv = VLDS ? sv : va;
  const int g = (int)threadIdx.x % G;
  if constexpr (WAVE > 0) {
    // Every level fits one wave (kWave / G rows a pass, a wide level in further passes): wave 0 solves
    // all of them and the other waves wait at the closing barrier.  Between levels the wave needs no block barrier: a
    // wave's LDS operations execute in order, so the next level's reads see this level's x stores;
    // wavefront-scope fences around the wave barrier keep the compiler from moving memory accesses
    // across it.  The next level's tables are read at the end of a level, as below.
    if (threadIdx.x < kWave) {
      const int slot = (int)threadIdx.x / G;
      const int nlast = (int)n - 1;
      int e0 = slv[0], e1 = slv[min(1, nlev)];
      int pn = min(e0 + slot, nlast);
      int i = srow[pn], q0 = srp[pn], q1n = srp[pn + 1];
      double di = (double)sd[pn];
      for (int lev = 0; lev < nlev; ++lev) {
        const bool live = e0 + slot < e1;
        const double bi = xs[i];
        double s = g == 0 ? bi : 0.0;
        s = trsv_row<G>(s, q0, live ? q1n : q0, g, [&](int q) { return fc[q]; },
                        [&](int q) { return (double)fv[q]; }, [&](int c) { return xs[c]; });
        s = trsv_group_sum<G>(s);
        if (live && g == 0) xs[i] = s * di;
        if constexpr (WAVE == 2) {
          for (int pb = e0 + kWave / G; pb < e1; pb += kWave / G) {   // further passes of a wide level
            const int p = pb + slot;
            const bool lp = p < e1;
            const int pc = lp ? p : e0;
            const int ip = srow[pc];
            const int p0 = srp[pc], p1 = lp ? srp[pc + 1] : p0;
            const double bp = xs[ip];
            double sp = g == 0 ? bp : 0.0;
            sp = trsv_row<G>(sp, p0, p1, g, [&](int q) { return fc[q]; }, [&](int q) { return (double)fv[q]; },
                             [&](int c) { return xs[c]; });
            sp = trsv_group_sum<G>(sp);
            const double dp = (double)sd[pc];
            if (lp && g == 0) xs[ip] = sp * dp;
          }
        }
        if (lev + 1 < nlev) {   // the next level's tables
          const int e2 = slv[lev + 2];
          pn = min(e1 + slot, nlast);
          i = srow[pn];
          q0 = srp[pn];
          q1n = srp[pn + 1];
          di = (double)sd[pn];
          e0 = e1;
          e1 = e2;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __syncthreads();   // the solve is complete before the block writes x out
  } else {
    // A level's first pass takes positions e0 + slot.  Their tables (row, entry range, 1 / l_ii) do not
    // depend on x, so they are read at the end of the previous level, after its x stores and before
    // its barrier: a level then starts with its entries' loads.  A position past the level's end is
    // clamped to a valid one and its lane writes nothing; further passes of a wide level read their
    // tables in place.
    const int slot = (int)threadIdx.x / G;
    const int nlast = (int)n - 1;
    int e0 = 0, e1 = 0, i = 0, q0 = 0, q1n = 0;
    double di = 0.0;
    if (nlev > 0) {
      e0 = slv[0];
      e1 = slv[1];
      const int pn = min(e0 + slot, nlast);
      i = srow[pn];
      q0 = srp[pn];
      q1n = srp[pn + 1];
      di = (double)sd[pn];
    }
    for (int lev = 0; lev < nlev; ++lev) {
      {
        const bool live = e0 + slot < e1;
        const double bi = xs[i];
        double s = g == 0 ? bi : 0.0;
        s = trsv_row<G>(s, q0, live ? q1n : q0, g, [&](int q) { return fc[q]; }, [&](int q) { return (double)fv[q]; },
                        [&](int c) { return xs[c]; });
        s = trsv_group_sum<G>(s);
        if (live && g == 0) xs[i] = s * di;
      }
      for (int pb = e0 + kTrsvThreads / G; pb < e1; pb += kTrsvThreads / G) {   // the same trip count in every lane
        const int p = pb + slot;
        const bool live = p < e1;
        const int pc = live ? p : e0;   // a lane past the level's end works on its first row and writes nothing
        const int ip = srow[pc];
        const int p0 = srp[pc], p1 = live ? srp[pc + 1] : p0;
        const double bi = xs[ip];
        double s = g == 0 ? bi : 0.0;
        s = trsv_row<G>(s, p0, p1, g, [&](int q) { return fc[q]; }, [&](int q) { return (double)fv[q]; },
                        [&](int c) { return xs[c]; });
        s = trsv_group_sum<G>(s);
        const double dp = (double)sd[pc];
        if (live && g == 0) xs[ip] = s * dp;
      }
      if (lev + 1 < nlev) {   // the next level's first-pass tables
        const int e2 = slv[lev + 2];
        const int pn = min(e1 + slot, nlast);
        i = srow[pn];
        q0 = srp[pn];
        q1n = srp[pn + 1];
        di = (double)sd[pn];
        e0 = e1;
        e1 = e2;
      }
      __syncthreads();   // this level's x are visible to the block before the next level reads them
    }
  }
  OutT* x = X + (size_t)r * xld;
  for (long t = threadIdx.x; t < n; t += kTrsvThreads) x[t] = (OutT)xs[t];
}

// LDS bytes of k_trsv_lds for a solve, with the entries (VLDS) or without (0: does not fit)
template <typename T>
static size_t trsv_lds_bytes(const TrsvDev& d, int64_t n, bool vlds) {
  if (d.nnz >= ((int64_t)1 << 31)) return 0;   // row starts are staged as 32-bit offsets
  const int64_t nv = vlds ? d.nnz : 0;
  const size_t b = (size_t)n * 8 + (size_t)(n + nv) * sizeof(T) + (size_t)(2 * n + 1 + nv + d.nlev + 1) * 4;
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

// Lanes per row G and the form of the LDS solve.  A round of four loads per lane covers 4 G entries of a
// row; one wave holds kWave / G rows a pass.  Block form: the least G whose round covers the longest row.
// One wave (no barrier between levels): among the G whose wave holds the widest level in at most two
// passes, the fewest rounds, then the fewest passes; taken when it needs no more rounds than the block
// form's G (on Section 5.2's matrix a second round cost more than the barriers it saved: droptol 1e-4
// at G = 8, 3.87 -> 4.69 ms per batch).
struct TrsvShape {
  int g_block = 16;   // G of the block form (and of the large-matrix kernel)
  int g_wave = 0;     // G of the one-wave form, 0: not taken
  int passes = 0;     // passes per level of the one-wave form (1 or 2)
};
static TrsvShape trsv_shape(const TrsvDev& d) {
  static constexpr int kG[4] = {1, 4, 8, 16};
  auto rounds = [&](int G) { return (d.max_row + 4 * G - 1) / (4 * G); };
  auto passes = [&](int G) { return (d.max_width + kWave / G - 1) / (kWave / G); };
  TrsvShape sh;
  for (int G : kG)
    if (4 * G >= d.max_row) {
      sh.g_block = G;
      break;
    }
  int best = 0;
  for (int G : kG) {
    if (passes(G) > 2) continue;
    if (best == 0 || rounds(G) < rounds(best) || (rounds(G) == rounds(best) && passes(G) < passes(best))) best = G;
  }
  if (best && rounds(best) <= rounds(sh.g_block)) {
    sh.g_wave = best;
    sh.passes = passes(best);
  }
  return sh;
}

// k_trsv_lds above the default dynamic LDS size needs the attribute; set once per instance
// (thread-safe static initialisation)
template <typename T, typename OutT, int G, bool VLDS, int WAVE>
static bool trsv_lds_launch(const IcholDev& f, const TrsvDev& d, size_t lb, const T* B, long bld, OutT* X, long xld,
                            const int* active, int k, hipStream_t st) {
  static const bool attr_set = [] {
    const bool ok = hipFuncSetAttribute((const void*)k_trsv_lds<T, OutT, G, VLDS, WAVE>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTrsvLdsMaxBytes) ==
                    hipSuccess;
    (void)hipGetLastError();
    return ok;
  }();
  if (!attr_set && lb > 65536) return false;
  hipLaunchKernelGGL((k_trsv_lds<T, OutT, G, VLDS, WAVE>), dim3(k), dim3(kTrsvThreads), lb, st, d.lvl_ptr,
                     d.rows, d.rp, d.ci, (const T*)d.va, (const T*)d.dinv, d.nlev, (long)f.n, (long)d.nnz, B, bld, X,
                     xld, active);
  return true;
}

template <typename T, typename OutT, int G, bool VLDS>
static bool trsv_lds_form(const IcholDev& f, const TrsvDev& d, int wave, size_t lb, const T* B, long bld, OutT* X,
                          long xld, const int* active, int k, hipStream_t st) {
  switch (wave) {
    case 1: return trsv_lds_launch<T, OutT, G, VLDS, 1>(f, d, lb, B, bld, X, xld, active, k, st);
    case 2: return trsv_lds_launch<T, OutT, G, VLDS, 2>(f, d, lb, B, bld, X, xld, active, k, st);
    default: return trsv_lds_launch<T, OutT, G, VLDS, 0>(f, d, lb, B, bld, X, xld, active, k, st);
  }
}

template <typename T, typename OutT, int G>
static void launch_trsv_g(const IcholDev& f, const TrsvDev& d, int wave, const T* B, long bld, OutT* X, long xld,
                          const int* active, int k, hipStream_t st) {
  size_t lb = trsv_lds_bytes<T>(d, f.n, true);
  if (lb && trsv_lds_form<T, OutT, G, true>(f, d, wave, lb, B, bld, X, xld, active, k, st)) return;
  lb = trsv_lds_bytes<T>(d, f.n, false);
  if (lb && trsv_lds_form<T, OutT, G, false>(f, d, wave, lb, B, bld, X, xld, active, k, st)) return;
  if (f.n <= kTrsvLdsRows)
    hipLaunchKernelGGL((k_trsv_levels<T, OutT, true, G>), dim3(k), dim3(kTrsvThreads), (size_t)f.n * sizeof(double),
                       st, d.lvl_ptr, d.rows, d.rp, d.ci, (const T*)d.va, (const T*)d.dinv, d.nlev, (long)f.n, B, bld,
                       X, xld, active);
  else
    hipLaunchKernelGGL((k_trsv_levels<T, OutT, false, G>), dim3(k), dim3(kTrsvThreads), 0, st, d.lvl_ptr, d.rows,
                       d.rp, d.ci, (const T*)d.va, (const T*)d.dinv, d.nlev, (long)f.n, B, bld, X, xld, active);
}

template <typename T, typename OutT>
void launch_trsv(const IcholDev& f, bool upper, const T* B, long bld, OutT* X, long xld, const int* active, int k,
                 hipStream_t st) {
  const TrsvDev& d = upper ? f.bwd : f.fwd;
  const TrsvShape sh = trsv_shape(d);
  // the one-wave form exists only for the LDS kernels
  const bool lds = trsv_lds_bytes<T>(d, f.n, true) || trsv_lds_bytes<T>(d, f.n, false);
  const int wave = lds && sh.g_wave ? sh.passes : 0;
  switch (wave ? sh.g_wave : sh.g_block) {
    case 1: launch_trsv_g<T, OutT, 1>(f, d, wave, B, bld, X, xld, active, k, st); break;
    case 4: launch_trsv_g<T, OutT, 4>(f, d, wave, B, bld, X, xld, active, k, st); break;
    case 8: launch_trsv_g<T, OutT, 8>(f, d, wave, B, bld, X, xld, active, k, st); break;
    default: launch_trsv_g<T, OutT, 16>(f, d, wave, B, bld, X, xld, active, k, st); break;
  }
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
