// Operator kernels: q = Q v for the lattice precisions (matrix free) and for CSR matrices
// (Section 2: the method touches Q only through products Q v).
//
// Lattice operators, with L the graph Laplacian of the grid (free) or torus (periodic):
//   order 1: Q = tau (kappa2 I + L)      order 2: Q = tau (kappa2 I + L)^2
// K = kappa2 I + L is evaluated in difference form, K v_p = kappa2 v_p + sum_{nb}(v_p - v_nb),
// so smooth fields cancel exactly in FP32; order 2 applies K twice inside LDS (tile + 2-point
// halo -> K on tile + 1 -> K on tile), the 13-point operator in 2D.
//
// In Lanczos mode the kernel opens iteration j (scalar step, see lz_open), reads
// v_j = slot(j-1)/beta_{j-1} with the scale folded into the load, and fuses the first part
// of Algorithm 1's loop body:  q = Q v_j - beta_{j-1} v_{j-1},  partial sums of v_j^T q.
#include "kernels.hpp"

#include <algorithm>

namespace gmrf {

template <int DIM> struct TileShape;
template <> struct TileShape<1> { static constexpr int TZ = 1, TY = 1, TX = 256; };
template <> struct TileShape<2> { static constexpr int TZ = 1, TY = 16, TX = 64; };
template <> struct TileShape<3> { static constexpr int TZ = 4, TY = 8, TX = 32; };

__device__ __forceinline__ int wrap_idx(int c, int n) {
  c %= n;
  return c < 0 ? c + n : c;
}

// K = kappa2 I + L at local point (lz, ly, lx) of an LDS box A of dims (AY, AX) per plane
// whose origin sits at global (gz - lz, gy - ly, gx - lx).  Neighbour validity: periodic
// always, free only inside the lattice.
template <typename T, int DIM>
__device__ __forceinline__ T apply_K(const T* A, int AY, int AX, int lz, int ly, int lx, int gz,
                                     int gy, int gx, const StencilGeom& g, T k2) {
  const int c = (lz * AY + ly) * AX + lx;
  const T v = A[c];
  T acc = k2 * v;
  const bool per = g.periodic != 0;
  if (per || gx - 1 >= 0) acc += v - A[c - 1];
  if (per || gx + 1 < g.n2) acc += v - A[c + 1];
  if (DIM >= 2) {
    if (per || gy - 1 >= 0) acc += v - A[c - AX];
    if (per || gy + 1 < g.n1) acc += v - A[c + AX];
  }
  if (DIM >= 3) {
    if (per || gz - 1 >= 0) acc += v - A[c - AX * AY];
    if (per || gz + 1 < g.n0) acc += v - A[c + AX * AY];
  }
  return acc;
}

template <typename T, int ORDER, int DIM, bool LZ>
__global__ __launch_bounds__(256) void k_stencil(StencilGeom g0, const T* __restrict__ X, long xld,
                                                 T* __restrict__ Y, long yld,
                                                 const T* __restrict__ Xprev, LzState S, int j,
                                                 const int* __restrict__ active) {
  using TS = TileShape<DIM>;
  constexpr int HZ = DIM >= 3 ? ORDER : 0, HY = DIM >= 2 ? ORDER : 0, HX = ORDER;
  constexpr int RZ = TS::TZ + 2 * HZ, RY = TS::TY + 2 * HY, RX = TS::TX + 2 * HX;
  constexpr int EZ = DIM >= 3 ? 1 : 0, EY = DIM >= 2 ? 1 : 0;
  constexpr int QZ = TS::TZ + 2 * EZ, QY = TS::TY + 2 * EY, QX = TS::TX + 2;  // K-stage box
  __shared__ T vs[RZ * RY * RX];
  __shared__ T ts[ORDER == 2 ? QZ * QY * QX : 1];
  __shared__ double red[256 / kWave];
  __shared__ int flag[1];

  const int r = blockIdx.y;
  // uneven batches: each column has its own lattice and offset; surplus tiles return
  const StencilGeom g = (LZ && S.col_geom) ? S.col_geom[r] : g0;
  if ((int)blockIdx.x >= g.tiles_x * g.tiles_y * g.tiles_z) return;
  double s_cur = 1.0, s_prev = 0.0, bprev = 0.0;
  if (LZ) {
    if (!lz_open<256>(S, r, j, blockIdx.x == 0, red, flag, s_cur, s_prev, bprev)) return;
  } else if (active && !active[r]) {
    return;
  }
  const int bid = blockIdx.x;
  const int tx = bid % g.tiles_x, ty = (bid / g.tiles_x) % g.tiles_y, tz = bid / (g.tiles_x * g.tiles_y);
  const int x0 = tx * TS::TX, y0 = ty * TS::TY, z0 = tz * TS::TZ;
  const size_t roff = (LZ && S.col_off) ? (size_t)S.col_off[r] : (size_t)r * xld;
  const T* src = X + roff;
  const bool per = g.periodic != 0;

  // The box with its halo, every load of a thread issued before the first is used: indices outside the
  // lattice (or the box) read element 0 of the column and are masked afterwards, so no load sits behind a
  // branch (each would then wait for its own data).
  constexpr int NF = RZ * RY * RX, NFI = (NF + 255) / 256;
  T fv[NFI];
  bool fok[NFI];
#pragma unroll
  for (int it = 0; it < NFI; ++it) {
    const int idx = (int)threadIdx.x + it * 256;
    const int lx = idx % RX, ly = (idx / RX) % RY, lz = idx / (RX * RY);
    int gx = x0 + lx - HX, gy = y0 + ly - HY, gz = z0 + lz - HZ;
    bool ok;
    if (per) {
      gx = wrap_idx(gx, g.n2);
      gy = wrap_idx(gy, g.n1);
      gz = wrap_idx(gz, g.n0);
      ok = idx < NF;
    } else {
      ok = idx < NF && gx >= 0 && gx < g.n2 && gy >= 0 && gy < g.n1 && gz >= 0 && gz < g.n0;
    }
    fok[it] = ok;
    fv[it] = src[ok ? ((size_t)gz * g.n1 + gy) * g.n2 + gx : 0];
  }
#pragma unroll
  for (int it = 0; it < NFI; ++it) {
    const int idx = (int)threadIdx.x + it * 256;
    const T val = fok[it] ? (LZ ? (T)((double)fv[it] * s_cur) : fv[it]) : (T)0;
    if (idx < NF) vs[idx] = val;
  }
  __syncthreads();
  const T k2 = (T)g.kappa2;
  const T* A = vs;
  int AY = RY, AX = RX, oz = HZ, oy = HY, ox = HX;   // box origin offset vs tile origin
  if (ORDER == 2) {
    for (int idx = threadIdx.x; idx < QZ * QY * QX; idx += 256) {
      const int lx = idx % QX, ly = (idx / QX) % QY, lz = idx / (QX * QY);
      const int gx = x0 + lx - 1, gy = y0 + ly - EY, gz = z0 + lz - EZ;
      const bool in = per || (gx >= 0 && gx < g.n2 && gy >= 0 && gy < g.n1 && gz >= 0 && gz < g.n0);
      T t = (T)0;
      if (in) t = apply_K<T, DIM>(vs, RY, RX, lz + (HZ - EZ), ly + (HY - EY), lx + (HX - 1), gz, gy, gx, g, k2);
      ts[idx] = t;
    }
    __syncthreads();
    A = ts;
    AY = QY;
    AX = QX;
    oz = EZ;
    oy = EY;
    ox = 1;
  }
  const T tau = (T)g.tau;
  T* dst = Y + ((LZ && S.col_off) ? roff : (size_t)r * yld);
  const T* prv = LZ ? Xprev + roff : nullptr;
  double acc = 0.0;
  constexpr int TP = TS::TZ * TS::TY * TS::TX, TPI = (TP + 255) / 256;
  // v_{j-1} at the thread's outputs, requested before the first output is formed (clamped like the box)
  T pv[TPI];
#pragma unroll
  for (int it = 0; it < TPI; ++it) {
    const int idx = (int)threadIdx.x + it * 256;
    const int lx = idx % TS::TX, ly = (idx / TS::TX) % TS::TY, lz = idx / (TS::TX * TS::TY);
    const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
    const bool in = idx < TP && gx < g.n2 && gy < g.n1 && gz < g.n0;
    if constexpr (LZ) pv[it] = prv[in ? ((size_t)gz * g.n1 + gy) * g.n2 + gx : 0];   // a valid vector at j = 1 too
    else pv[it] = (T)0;
  }
#pragma unroll
  for (int it = 0; it < TPI; ++it) {
    const int idx = (int)threadIdx.x + it * 256;
    const int lx = idx % TS::TX, ly = (idx / TS::TX) % TS::TY, lz = idx / (TS::TX * TS::TY);
    const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
    if (idx >= TP || gx >= g.n2 || gy >= g.n1 || gz >= g.n0) continue;
    const T kv = apply_K<T, DIM>(A, AY, AX, lz + oz, ly + oy, lx + ox, gz, gy, gx, g, k2);
    const T out = tau * kv;
    const size_t gi = ((size_t)gz * g.n1 + gy) * g.n2 + gx;
    if (LZ) {
      double q = (double)out;
      if (j > 1) q -= bprev * (double)(T)((double)pv[it] * s_prev);
      const T qt = (T)q;
      dst[gi] = qt;
      const T vj = vs[((lz + HZ) * RY + (ly + HY)) * RX + (lx + HX)];
      acc += (double)vj * (double)qt;
    } else {
      dst[gi] = out;
    }
  }
  if (LZ) {
    const double s = block_sum<256>(acc, red);
    if (threadIdx.x == 0) S.part_a[(size_t)r * S.pstride + blockIdx.x] = s;
  }
}

// XCD-aware tile order (kTuneXcd): the dispatcher hands workgroup i (linear over the grid) to XCD i mod 8,
// each XCD with its own L2.  Logical (tile, column) ids are assigned so that every XCD works through one
// contiguous range of them: neighbouring strips and bands, whose halo rows and columns overlap, then meet
// in one L2.  The map is a bijection of the grid.
constexpr int kXcds = 8;
__device__ __forceinline__ void xcd_order(bool on, int& tile, int& col) {
  if (!on) {
    tile = blockIdx.x;
    col = blockIdx.y;
    return;
  }
  const int gx = gridDim.x, nb = gx * gridDim.y;
  const int i = blockIdx.x + blockIdx.y * gx;
  const int q = nb / kXcds, rm = nb % kXcds, x = i % kXcds, k = i / kXcds;
  const int L = (x < rm ? x * (q + 1) : rm * (q + 1) + (x - rm) * q) + k;
  tile = L % gx;
  col = L / gx;
}

// ---- 3D first-order lattices: z-march ----------------------------------------------------------
// A block owns a segment of `band` whole rows of the plane (at most kZSeg points) and walks a run of `zc`
// planes along z.  Each thread keeps its points of planes z - 1, z and z + 1 in registers (plane z + 1 and
// the next plane's two halo rows are requested while plane z is evaluated), so every value of v is read
// from memory once per run plus the runs' first and last planes; only the plane's own segment and its
// halo rows pass through LDS for the x and y neighbours.  The box tiles above read about twice their
// outputs.  The terms of K v are those of apply_K in the same order, so Q v is bitwise the same.
constexpr int kZThreads = 256;
constexpr int kZEpt = 4;                        // points per thread per plane
constexpr int kZSeg = kZThreads * kZEpt;        // points per segment
constexpr int kZMaxN2 = kZSeg / 2;              // the two halo rows are loaded kZEpt per thread too
constexpr long kZMinPoints = 1L << 20;          // lattices from this size march (smaller ones: box tiles)

template <typename T, int VE> struct ZVec;
template <typename T> struct ZVec<T, 1> { typedef T type; };
template <> struct ZVec<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct ZVec<float, 2> { typedef float type __attribute__((ext_vector_type(2))); };

// One block's run.  VE points per load (2 when the row length is even: every pair lies in one row and
// starts at an even offset), so a thread holds kZEpt / VE groups of VE consecutive points; the terms of
// every point and the order of every sum depend only on VE, which each block takes from its own lattice.
template <typename T, bool LZ, int VE>
__device__ __forceinline__ void z3_run(const StencilGeom& g, int tile, T* pl, const T* __restrict__ src,
                                       T* __restrict__ dst, const T* __restrict__ prv, int j, double s_cur,
                                       double s_prev, double bprev, double& acc) {
  using V = typename ZVec<T, VE>::type;
  constexpr int NS = kZEpt / VE;
  const int n0 = g.n0, n1 = g.n1, n2 = g.n2;
  const int seg = tile % g.tiles_x, zi = tile / g.tiles_x;
  const int y0 = seg * g.band, rows = min(g.band, n1 - y0), E = rows * n2;
  const int z0 = zi * g.zc, z1 = min(n0, z0 + g.zc);
  const bool per = g.periodic != 0;
  const size_t plane = (size_t)n1 * n2, sbase = (size_t)y0 * n2;
  const int yup = y0 > 0 ? y0 - 1 : (per ? n1 - 1 : -1);               // halo rows (-1: none)
  const int ydn = y0 + rows < n1 ? y0 + rows : (per ? 0 : -1);
  const T k2 = (T)g.kappa2, tau = (T)g.tau;
  const bool prev_term = LZ && j > 1;
  auto first = [&](int i) { return VE * ((int)threadIdx.x + i * kZThreads); };   // first point of group i

  int lx[kZEpt], ly[kZEpt];
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int v = 0; v < VE; ++v) {
      const int e = first(i) + v;
      ly[i * VE + v] = e / n2;
      lx[i * VE + v] = e - ly[i * VE + v] * n2;
    }
  auto get = [&](const T* p, size_t gi, T* out, double scale, bool scaled) {
    const V raw = *(const V*)(p + gi);
#pragma unroll
    for (int v = 0; v < VE; ++v) {
      T x;
      if constexpr (VE == 1) x = raw;
      else x = raw[v];
      out[v] = scaled ? (T)((double)x * scale) : x;
    }
  };
  // In the Lanczos step every load reads a valid address (indices outside the lattice read element 0 of the
  // column) and the value is masked afterwards, so no load sits behind a branch, where each would wait for
  // its own data (3D samples 10-20% faster).  The operator alone keeps its loads behind the bounds tests:
  // masked, it took 121.9 -> 133.6 us at 128^3 x 32 FP32.  The values, and so the bits, are the same.
  auto masked = [&](const T* p, size_t gi, bool ok, T* out, double scale, bool scaled) {
    if constexpr (LZ) {
      T tmp[VE];
      get(p, ok ? gi : 0, tmp, scale, scaled);
#pragma unroll
      for (int v = 0; v < VE; ++v) out[v] = ok ? tmp[v] : (T)0;
    } else if (ok) {
      get(p, gi, out, scale, scaled);
    } else {
#pragma unroll
      for (int v = 0; v < VE; ++v) out[v] = (T)0;
    }
  };
  // the segment of plane z (zeros for a plane beyond a free boundary)
  auto load_seg = [&](int z, T* vv) {
    const int zz = z < 0 ? (per ? z + n0 : -1) : (z >= n0 ? (per ? z - n0 : -1) : z);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int e = first(i);
      masked(src, (size_t)max(zz, 0) * plane + sbase + e, zz >= 0 && e < E, vv + i * VE, s_cur, LZ);
    }
  };
  // the halo rows of plane z (0 <= z < n0): points [0, n2) the row above, [n2, 2 n2) the row below
  auto load_halo = [&](int z, T* h) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int e = first(i);
      const int row = e < n2 ? yup : ydn;
      masked(src, (size_t)z * plane + (size_t)max(row, 0) * n2 + (e < n2 ? e : e - n2), e < 2 * n2 && row >= 0,
             h + i * VE, s_cur, LZ);
    }
  };
  // v_{j-1} (the Lanczos step passes a valid vector at j = 1 too)
  auto load_prev = [&](int z, T* pp) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int e = first(i);
      if constexpr (LZ) masked(prv, (size_t)z * plane + sbase + e, prev_term && e < E, pp + i * VE, s_prev, true);
      else
#pragma unroll
        for (int v = 0; v < VE; ++v) pp[i * VE + v] = (T)0;
    }
  };

  T vp[kZEpt], vc[kZEpt], vn[kZEpt], hc[kZEpt], hn[kZEpt], pc[kZEpt], pn[kZEpt];
  load_seg(z0 - 1, vp);
  load_seg(z0, vc);
  load_halo(z0, hc);
  load_prev(z0, pc);
  for (int z = z0; z < z1; ++z) {
    // the next plane's values (in the Lanczos step the last plane of the run reloads its own halo rows and
    // v_{j-1}, unused, rather than branch around the loads)
    load_seg(z + 1, vn);
    if (LZ || z + 1 < z1) {
      load_halo(min(z + 1, z1 - 1), hn);
      load_prev(min(z + 1, z1 - 1), pn);
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int e0 = first(i);
#pragma unroll
      for (int v = 0; v < VE; ++v) {
        const int e = e0 + v;
        if (e < E) pl[n2 + e] = vc[i * VE + v];
        if (e < 2 * n2) pl[e < n2 ? e : (rows + 1) * n2 + (e - n2)] = hc[i * VE + v];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int e0 = first(i);
      if (e0 >= E) continue;
      T outv[VE];
#pragma unroll
      for (int v = 0; v < VE; ++v) {
        const int q = i * VE + v, e = e0 + v;
        const int x = lx[q], y = y0 + ly[q], c = n2 + e;
        const T vv = vc[q];
        T a = k2 * vv;
        if (per || x - 1 >= 0) a += vv - pl[x > 0 ? c - 1 : c + n2 - 1];
        if (per || x + 1 < n2) a += vv - pl[x + 1 < n2 ? c + 1 : c - n2 + 1];
        if (per || y - 1 >= 0) a += vv - pl[c - n2];
        if (per || y + 1 < n1) a += vv - pl[c + n2];
        if (per || z - 1 >= 0) a += vv - vp[q];
        if (per || z + 1 < n0) a += vv - vn[q];
        const T out = tau * a;
        if (LZ) {
          double qd = (double)out;
          if (prev_term) qd -= bprev * (double)pc[q];
          const T qt = (T)qd;
          outv[v] = qt;
          acc += (double)vv * (double)qt;
        } else {
          outv[v] = out;
        }
      }
      V ov;
      if constexpr (VE == 1) ov = outv[0];
      else
#pragma unroll
        for (int v = 0; v < VE; ++v) ov[v] = outv[v];
      *(V*)(dst + (size_t)z * plane + sbase + e0) = ov;
    }
    __syncthreads();   // the plane buffer is rewritten next
#pragma unroll
    for (int q = 0; q < kZEpt; ++q) {
      vp[q] = vc[q];
      vc[q] = vn[q];
      hc[q] = hn[q];
      pc[q] = pn[q];
    }
  }
}

template <typename T, bool LZ>
__global__ __launch_bounds__(kZThreads) void k_stencil3z(StencilGeom g0, const T* __restrict__ X, long xld,
                                                         T* __restrict__ Y, long yld, const T* __restrict__ Xprev,
                                                         LzState S, int j, const int* __restrict__ active) {
  __shared__ __align__(16) T pl[kZSeg + 2 * kZMaxN2];       // halo row above, the segment, halo row below
  __shared__ double red[kZThreads / kWave];
  __shared__ int flag[1];
  // XCD-contiguous order: the segments and runs that share halo rows and planes meet in one L2
  int tile, r;
  xcd_order(true, tile, r);
  const StencilGeom g = (LZ && S.col_geom) ? S.col_geom[r] : g0;
  if (tile >= g.tiles_x * g.tiles_z) return;
  double s_cur = 1.0, s_prev = 0.0, bprev = 0.0;
  if (LZ) {
    if (!lz_open<kZThreads>(S, r, j, tile == 0, red, flag, s_cur, s_prev, bprev)) return;
  } else if (active && !active[r]) {
    return;
  }
  const size_t roff = (LZ && S.col_off) ? (size_t)S.col_off[r] : (size_t)r * xld;
  const T* src = X + roff;
  T* dst = Y + ((LZ && S.col_off) ? roff : (size_t)r * yld);
  const T* prv = LZ ? Xprev + roff : nullptr;
  double acc = 0.0;
  if (g.n2 % 2 == 0) z3_run<T, LZ, 2>(g, tile, pl, src, dst, prv, j, s_cur, s_prev, bprev, acc);
  else z3_run<T, LZ, 1>(g, tile, pl, src, dst, prv, j, s_cur, s_prev, bprev, acc);
  if (LZ) {
    const double bs = block_sum<kZThreads>(acc, red);
    if (threadIdx.x == 0) S.part_a[(size_t)r * S.pstride + tile] = bs;
  }
}

// ---- 2D lattices: row-streaming waves ---------------------------------------------------------
// One wave per 64-column strip (kWave - 2 ORDER output columns, the strips overlap by ORDER columns
// on each side) walks down a band of kS2Band rows.  Vertical neighbours stay in registers; each row
// of v (and, for order 2, of K v) passes through a small per-wave LDS row buffer for its left and
// right neighbours, so the row loop has no block barrier.  Rows are requested S2Ahead rows ahead,
// unconditionally (row index clamped or wrapped), so that several rows are in flight per wave.
// Free boundary: a missing neighbour is replaced by the point itself, so its difference is exactly 0
// (same terms in the same order as k_stencil).
constexpr int kS2Waves = 4;     // waves per block (bands stacked vertically)
constexpr int kS2Band = 32;     // output rows per wave
// Output rows per wave of the one-pass kernel: each band re-reads 2 (ORDER + 1) halo rows, so the 13-point
// step keeps 32-row bands while the 5-point step takes 24, which shortens each wave's row chain and
// spreads large grids over more blocks (measured, FP64 5-point 2048^2 x 8: 32 / 24 / 16 rows -> 194.7 /
// 184.2 / 182.0 us; 256^2 x 8 FP32: 20.2 / 16.2 / 13.3 us; the 256-field batch 43.6 / 42.1 / 45.2 ms;
// 13-point 1024^2 x 64 FP32: 222.4 / 228.3 / 254.5 us, 64 rows 216.3 us but slower on small grids)
#ifndef GMRF_S2F_BAND1
#define GMRF_S2F_BAND1 24
#endif
#ifndef GMRF_S2F_BAND2
#define GMRF_S2F_BAND2 32
#endif
__host__ __device__ constexpr int s2f_band(int order) { return order == 1 ? GMRF_S2F_BAND1 : GMRF_S2F_BAND2; }
#ifndef GMRF_L2D_FEPL4
#define GMRF_L2D_FEPL4 1       // the one-pass kernel may take four FP32 columns per lane (else two)
#endif

// rows requested ahead per wave: a row is 64 elements, so FP32 rows carry half the bytes of FP64 rows
#ifndef GMRF_S2_AHEAD64
#define GMRF_S2_AHEAD64 4
#endif
#ifndef GMRF_S2_AHEAD32
#define GMRF_S2_AHEAD32 8
#endif
template <typename T> struct S2Ahead;
template <> struct S2Ahead<double> { static constexpr int value = GMRF_S2_AHEAD64; };
template <> struct S2Ahead<float> { static constexpr int value = GMRF_S2_AHEAD32; };

// Elements of a lane: EPL adjacent columns (one vector load) when the geometry allows it (row length and
// field offsets multiples of EPL): 4 for FP32 storage (16-byte loads), 2 for FP64, else 1.  With EPL > 1
// the strips start EPL columns left of their first output, so lanes hold aligned groups and a group never
// straddles the lattice edge.
template <typename T, int EPL> struct VecE;
template <typename T> struct VecE<T, 1> {
  typedef T type;
  __device__ static T get(const type& v, int) { return v; }
};
template <> struct VecE<double, 2> {
  typedef double type __attribute__((ext_vector_type(2)));
  __device__ static double get(const type& v, int e) { return v[e]; }
};
template <> struct VecE<float, 2> {
  typedef float type __attribute__((ext_vector_type(2)));
  __device__ static float get(const type& v, int e) { return v[e]; }
};
template <> struct VecE<float, 4> {
  typedef float type __attribute__((ext_vector_type(4)));
  __device__ static float get(const type& v, int e) { return v[e]; }
};
// largest EPL of the 2D operator kernel per storage type (sizes its LDS row slots)
template <typename T> constexpr int kS2MaxEpl = sizeof(T) == 4 ? 4 : 2;
__host__ __device__ inline int s2_halo(int order, int epl) { return epl >= 2 ? epl : order; }
__host__ __device__ inline int s2_out(int order, int epl) { return kWave * epl - 2 * s2_halo(order, epl); }

template <typename T, int ORDER, bool LZ, int EPL, bool NTS>
__device__ __forceinline__ void s2_strip(const StencilGeom& g, int tx, int ty, int w, int lane,
                                         const T* __restrict__ src, T* __restrict__ dst,
                                         const T* __restrict__ prv, int j, double s_cur, double s_prev,
                                         double bprev, T* vbuf, T* tbuf, double& acc) {
  using VE = VecE<T, EPL>;
  using VT = typename VE::type;
  constexpr int HX = EPL >= 2 ? EPL : ORDER;
  constexpr int OX = kWave * EPL - 2 * HX;
  constexpr int RW = kWave * EPL;                               // row-slot width
  const int n1 = g.n1, n2 = g.n2;
  const bool per = g.periodic != 0;
  const int xb = tx * OX - HX + lane * EPL;                     // first column of this lane
  // column of the lane's load: clamped (free) or wrapped (periodic), group-aligned when EPL > 1
  const int xl = per ? ((xb % n2) + n2) % n2 : min(max(xb, 0), n2 - EPL);
  bool hl[EPL], hr[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    hl[e] = per || xb + e > 0;
    hr[e] = per || xb + e < n2 - 1;
  }
  const bool olane = lane * EPL >= HX && lane * EPL < RW - HX && xb >= 0 && xb < n2;
  const int lm = (lane * EPL - 1) & (RW - 1), lp = (lane * EPL + EPL) & (RW - 1);
  const int band = g.band > 0 ? g.band : kS2Band;
  const int y_lo = (ty * kS2Waves + w) * band;
  const int y_hi = min(y_lo + band, n1);
  const int count = y_hi > y_lo ? y_hi - y_lo + 2 * ORDER : 0;   // input rows y_lo - ORDER .. y_hi + ORDER - 1
  if (count == 0) return;
  const int ys = y_lo - ORDER;
  const int xp = min(max(xb, 0), n2 - EPL);                       // v_{j-1} column (clamped, aligned)
  const bool tiny = n1 <= 2 * ORDER;
  auto rowi = [&](int y) {
    if (!per) return min(max(y, 0), n1 - 1);
    if (tiny) return ((y % n1) + n1) % n1;
    return y < 0 ? y + n1 : (y >= n1 ? y - n1 : y);
  };
  auto ld = [&](int i) { return *(const VT*)(src + (size_t)rowi(ys + min(i, count - 1)) * n2 + xl); };
  auto ldp = [&](int i) {
    const int yo = min(max(ys + min(i, count - 1) - ORDER, 0), n1 - 1);
    return *(const VT*)(prv + (size_t)yo * n2 + xp);
  };
  const T k2 = (T)g.kappa2, tau = (T)g.tau;
  // K at row yc of element e: centre c[e], vertical u[e], d[e]; horizontal from the row slot b and the
  // lane's own neighbouring element
  auto kop = [&](const T (&c)[EPL], const T (&u)[EPL], const T (&d)[EPL], const T* b, int yc, T (&out)[EPL]) {
    const T bl = b[lm], br = b[lp];
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const T v = c[e];
      const T ln = e > 0 ? c[e > 0 ? e - 1 : 0] : bl;
      const T rn = e < EPL - 1 ? c[e < EPL - 1 ? e + 1 : 0] : br;
      const T l = hl[e] ? ln : v, rr = hr[e] ? rn : v;
      const T uu = (per || yc > 0) ? u[e] : v, dd = (per || yc < n1 - 1) ? d[e] : v;
      T a = k2 * v;
      a += v - l;
      a += v - rr;
      a += v - uu;
      a += v - dd;
      out[e] = a;
    }
  };
  T v0[EPL], v1[EPL], t0[EPL], t1[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) v0[e] = v1[e] = t0[e] = t1[e] = (T)0;
  constexpr int LEAD = 2 * ORDER;   // input rows consumed before the first output
  auto store_row = [&](T* buf, int par, const T (&val)[EPL]) {
    VT vv;
    if constexpr (EPL == 1) {
      vv = val[0];
    } else {
#pragma unroll
      for (int e = 0; e < EPL; ++e) vv[e] = val[e];
    }
    *(VT*)(buf + par * RW + lane * EPL) = vv;
  };
  auto step = [&](int i, int par, bool T2, bool OUT, const VT& raw, const VT& rawp) {
    T v2[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) v2[e] = LZ ? (T)((double)VE::get(raw, e) * s_cur) : VE::get(raw, e);
    store_row(vbuf, par, v2);
    const int yi = ys + i;
    T oc[EPL], vc[EPL];
    int yo;
    if (ORDER == 1) {
      yo = yi - 1;
#pragma unroll
      for (int e = 0; e < EPL; ++e) vc[e] = v1[e];
      if (OUT) {
        kop(v1, v0, v2, vbuf + (par ^ 1) * RW, yo, oc);
#pragma unroll
        for (int e = 0; e < EPL; ++e) oc[e] = tau * oc[e];
      }
    } else {
      T t2[EPL];
#pragma unroll
      for (int e = 0; e < EPL; ++e) t2[e] = (T)0;
      if (T2) {
        kop(v1, v0, v2, vbuf + (par ^ 1) * RW, yi - 1, t2);
        store_row(tbuf, par ^ 1, t2);
      }
      yo = yi - 2;
#pragma unroll
      for (int e = 0; e < EPL; ++e) vc[e] = v0[e];
      if (OUT) {
        kop(t1, t0, t2, tbuf + par * RW, yo, oc);
#pragma unroll
        for (int e = 0; e < EPL; ++e) oc[e] = tau * oc[e];
      }
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        t0[e] = t1[e];
        t1[e] = t2[e];
      }
    }
    if (OUT && olane) {
      T res[EPL];
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        if (LZ) {
          double q = (double)oc[e];
          if (j > 1) q -= bprev * (double)(T)((double)VE::get(rawp, e) * s_prev);
          res[e] = (T)q;
          acc += (double)vc[e] * (double)res[e];
        } else {
          res[e] = oc[e];
        }
      }
      VT vv;
      if constexpr (EPL == 1) {
        vv = res[0];
      } else {
#pragma unroll
        for (int e = 0; e < EPL; ++e) vv[e] = res[e];
      }
      if constexpr (NTS) __builtin_nontemporal_store(vv, (VT*)(dst + (size_t)yo * n2 + xb));
      else *(VT*)(dst + (size_t)yo * n2 + xb) = vv;
    }
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      v0[e] = v1[e];
      v1[e] = v2[e];
    }
  };
  // AHEAD register sets take turns (unrolled, no copies between them): row i lives in set i % AHEAD and
  // is computed while rows i + 1 .. i + AHEAD - 1 are in flight; 16-byte lanes (FP64 pairs, FP32 groups
  // of four) take the FP64 depth
  constexpr int AHEAD = EPL * sizeof(T) >= 16 ? GMRF_S2_AHEAD64 : S2Ahead<T>::value;
  static_assert(AHEAD >= LEAD && AHEAD % 2 == 0, "prefetch depth");
  VT q[AHEAD], p[AHEAD];
#pragma unroll
  for (int d = 0; d < AHEAD; ++d) {
    q[d] = ld(d);
    p[d] = LZ ? ldp(d) : q[d];
  }
#pragma unroll
  for (int d = 0; d < LEAD; ++d) {   // warm-up rows: no output
    step(d, d & 1, d >= 2, false, q[d], p[d]);
    q[d] = ld(d + AHEAD);
    if (LZ) p[d] = ldp(d + AHEAD);
  }
  int i = LEAD;
  for (; i + AHEAD <= count; i += AHEAD) {
#pragma unroll
    for (int d = 0; d < AHEAD; ++d) {
      const int c = (LEAD + d) % AHEAD;
      step(i + d, (LEAD + d) & 1, true, true, q[c], p[c]);
      q[c] = ld(i + d + AHEAD);
      if (LZ) p[c] = ldp(i + d + AHEAD);
    }
  }
#pragma unroll
  for (int d = 0; d < AHEAD; ++d) {   // tail: the rows left, already requested
    const int c = (LEAD + d) % AHEAD;
    if (i + d < count) step(i + d, (LEAD + d) & 1, true, true, q[c], p[c]);
  }
}

// NTS: non-temporal stores of q (kTuneNtStore; a template parameter so that the store keeps its cache policy)
template <typename T, int ORDER, bool LZ, bool NTS>
__global__ __launch_bounds__(256) void k_stencil2d(StencilGeom g0, const T* __restrict__ X, long xld,
                                                   T* __restrict__ Y, long yld, const T* __restrict__ Xprev,
                                                   LzState S, int j, const int* __restrict__ active) {
  __shared__ __align__(16) T vrow[kS2Waves][2][kS2MaxEpl<T> * kWave];
  __shared__ __align__(16) T trow[kS2Waves][2][kS2MaxEpl<T> * kWave];
  __shared__ double red[256 / kWave];
  __shared__ int flag[1];
  int tile, r;
  xcd_order((g0.tune & kTuneXcd) != 0, tile, r);
  const StencilGeom g = (LZ && S.col_geom) ? S.col_geom[r] : g0;
  if (tile >= g.tiles_x * g.tiles_y) return;
  double s_cur = 1.0, s_prev = 0.0, bprev = 0.0;
  if (LZ) {
    if (!lz_open<256>(S, r, j, tile == 0, red, flag, s_cur, s_prev, bprev)) return;
  } else if (active && !active[r]) {
    return;
  }
  const int tx = tile % g.tiles_x, ty = tile / g.tiles_x;
  // wave index read as a scalar: the row loop's bounds are then uniform and its branches scalar
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
  const size_t roff = (LZ && S.col_off) ? (size_t)S.col_off[r] : (size_t)r * xld;
  const T* src = X + roff;
  T* dst = Y + ((LZ && S.col_off) ? roff : (size_t)r * yld);
  const T* prv = LZ ? Xprev + roff : nullptr;
  double acc = 0.0;
  if constexpr (kS2MaxEpl<T> == 4) {
    if (g.epl == 4) {
      s2_strip<T, ORDER, LZ, 4, NTS>(g, tx, ty, w, lane, src, dst, prv, j, s_cur, s_prev, bprev, &vrow[w][0][0],
                                &trow[w][0][0], acc);
      goto done;
    }
  }
  if (g.epl == 2)
    s2_strip<T, ORDER, LZ, 2, NTS>(g, tx, ty, w, lane, src, dst, prv, j, s_cur, s_prev, bprev, &vrow[w][0][0],
                              &trow[w][0][0], acc);
  else
    s2_strip<T, ORDER, LZ, 1, NTS>(g, tx, ty, w, lane, src, dst, prv, j, s_cur, s_prev, bprev, &vrow[w][0][0],
                              &trow[w][0][0], acc);
done:
  if (LZ) {
    const double bs = block_sum<256>(acc, red);
    if (threadIdx.x == 0) S.part_a[(size_t)r * S.pstride + tile] = bs;
  }
}

// ---- 2D lattices: one pass per Lanczos step ----------------------------------------------------
// alpha_j is known before the pass (Algorithm 1's alpha_j = v_j^T (Q v_j - beta_{j-1} v_{j-1})):
//   v_j^T Q v_j = w_{j-1}^T Q w_{j-1} / beta_{j-1}^2,   beta_{j-1} v_j^T v_{j-1} = <w_{j-1}, v_{j-1}>,
// with w^T Q w = tau ||K w||^2 (order 2, Q = tau K^2) or tau (kappa2 ||w||^2 + sum over the lattice's
// edges of (w_a - w_b)^2) (order 1) -- sums of squares, formed by the previous pass while it wrote
// w_{j-1}.  One pass therefore reads v_j (= slot j-1 / beta_{j-1}) and v_{j-1} and writes
//   w_j = Q v_j - alpha_j v_j - beta_{j-1} v_{j-1}
// with the partial sums of ||w_j||^2, <w_j, v_j> and w_j^T Q w_j for the next pass: 3 s E bytes per step
// instead of 6 s E for an operator pass plus an update pass.  K w needs w around each output point, so
// each strip forms w on a one-point halo: v is read with a halo of ORDER + 1 points.
// MODE 1: the quadratic form of the input alone (slot 0 before iteration 1), into out_a.
// halo: w needs v one point beyond K w's output, K one more for order 2; group-aligned for EPL > 1
__host__ __device__ inline int s2f_halo(int order, int epl) {
  return epl == 4 ? 4 : (epl == 2 ? (order == 2 ? 4 : 2) : order + 1);
}
__host__ __device__ inline int s2f_out(int order, int epl) { return kWave * epl - 2 * s2f_halo(order, epl); }

template <typename T, int ORDER, int MODE, int EPL, bool NTS>
__device__ __forceinline__ void s2f_strip(const StencilGeom& g, int tx, int ty, int w, int lane,
                                          const T* __restrict__ src, T* __restrict__ dst,
                                          const T* __restrict__ prv, int j, double s_cur, double s_prev,
                                          double bprev, double alpha, T* vbuf, T* tbuf, T* wbuf, double& acc_b,
                                          double& acc_c, double& acc_a) {
  using VE = VecE<T, EPL>;
  using VT = typename VE::type;
  constexpr int HX = EPL == 4 ? 4 : (EPL == 2 ? (ORDER == 2 ? 4 : 2) : ORDER + 1);
  constexpr int OX = kWave * EPL - 2 * HX;
  constexpr int RW = kWave * EPL;
  constexpr int HV = ORDER + 1;                                 // rows of v above and below the band
  const int n1 = g.n1, n2 = g.n2;
  const bool per = g.periodic != 0;
  const int xb = tx * OX - HX + lane * EPL;
  const int xl = per ? ((xb % n2) + n2) % n2 : min(max(xb, 0), n2 - EPL);
  bool hl[EPL], hr[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    hl[e] = per || xb + e > 0;
    hr[e] = per || xb + e < n2 - 1;
  }
  const bool olane = lane * EPL >= HX && lane * EPL < RW - HX && xb >= 0 && xb < n2;
  const int lm = (lane * EPL - 1) & (RW - 1), lp = (lane * EPL + EPL) & (RW - 1);
  constexpr int BAND = s2f_band(ORDER);
  const int y_lo = (ty * kS2Waves + w) * BAND;   // the one-pass kernel keeps full bands (ftiles_y)
  const int y_hi = min(y_lo + BAND, n1);
  const int count = y_hi > y_lo ? y_hi - y_lo + 2 * HV : 0;
  if (count == 0) return;
  const int ys = y_lo - HV;
  const bool tiny = n1 <= 2 * HV;
  auto rowi = [&](int y) {
    if (!per) return min(max(y, 0), n1 - 1);
    if (tiny) return ((y % n1) + n1) % n1;
    return y < 0 ? y + n1 : (y >= n1 ? y - n1 : y);
  };
  auto ld = [&](int i) { return *(const VT*)(src + (size_t)rowi(ys + min(i, count - 1)) * n2 + xl); };
  // v_{j-1} at the row of w formed at input row i (ys + i - ORDER), wrapped or clamped like v: w is also
  // formed on the halo, where a periodic lattice needs the wrapped values
  auto ldp = [&](int i) { return *(const VT*)(prv + (size_t)rowi(ys + min(i, count - 1) - ORDER) * n2 + xl); };
  const T k2 = (T)g.kappa2, tau = (T)g.tau;
  const double dk2 = g.kappa2, dtau = g.tau;
  auto kop = [&](const T (&c)[EPL], const T (&u)[EPL], const T (&d)[EPL], const T* b, int yc, T (&out)[EPL]) {
    const T bl = b[lm], br = b[lp];
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const T v = c[e];
      const T ln = e > 0 ? c[e > 0 ? e - 1 : 0] : bl;
      const T rn = e < EPL - 1 ? c[e < EPL - 1 ? e + 1 : 0] : br;
      const T l = hl[e] ? ln : v, rr = hr[e] ? rn : v;
      const T uu = (per || yc > 0) ? u[e] : v, dd = (per || yc < n1 - 1) ? d[e] : v;
      T a = k2 * v;
      a += v - l;
      a += v - rr;
      a += v - uu;
      a += v - dd;
      out[e] = a;
    }
  };
  // quadratic-form terms of the points of row yc held in c (row yc + 1 in d, right neighbours from b)
  auto qform = [&](const T (&c)[EPL], const T (&u)[EPL], const T (&d)[EPL], const T* b, int yc) {
    if (ORDER == 2) {
      T kw[EPL];
      kop(c, u, d, b, yc, kw);
#pragma unroll
      for (int e = 0; e < EPL; ++e) acc_a += dtau * ((double)kw[e] * (double)kw[e]);
    } else {
      const T br = b[lp];
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const double v = (double)c[e];
        const double rn = (double)(e < EPL - 1 ? c[e < EPL - 1 ? e + 1 : 0] : br);
        double q = dk2 * v * v;
        if (hr[e]) q += (v - rn) * (v - rn);
        if (per || yc < n1 - 1) q += (v - (double)d[e]) * (v - (double)d[e]);
        acc_a += dtau * q;
      }
    }
  };
  auto store_row = [&](T* buf, int par, const T (&val)[EPL]) {
    VT vv;
    if constexpr (EPL == 1) {
      vv = val[0];
    } else {
#pragma unroll
      for (int e = 0; e < EPL; ++e) vv[e] = val[e];
    }
    *(VT*)(buf + par * RW + lane * EPL) = vv;
  };
  T v0[EPL], v1[EPL], t0[EPL], t1[EPL], wa[EPL], wb[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) v0[e] = v1[e] = t0[e] = t1[e] = wa[e] = wb[e] = (T)0;
  // Input row i (row ys + i).  par = i & 1 picks the LDS row slots; the stages run from i >= 2 (K v, order
  // 2), i >= 2 ORDER (w at row ys + i - ORDER) and i >= 2 ORDER + 2 (K w at row ys + i - ORDER - 1).
  auto step = [&](int i, int par, const VT& raw, const VT& rawp) {
    T v2[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) v2[e] = MODE == 0 ? (T)((double)VE::get(raw, e) * s_cur) : VE::get(raw, e);
    store_row(vbuf, par, v2);
    const int yi = ys + i;
    if (MODE == 1) {
      // quadratic form of the input itself: row yi - 1
      const int yc = yi - 1;
      if (i >= 2 && olane && yc >= y_lo && yc < y_hi) qform(v1, v0, v2, vbuf + (par ^ 1) * RW, yc);
    } else {
      T q[EPL], vw[EPL];
      bool haw = false;
      const int yw = yi - ORDER;
      if (ORDER == 1) {
        if (i >= 2) {
          kop(v1, v0, v2, vbuf + (par ^ 1) * RW, yw, q);
          haw = true;
        }
#pragma unroll
        for (int e = 0; e < EPL; ++e) vw[e] = v1[e];
      } else {
        T t2[EPL];
#pragma unroll
        for (int e = 0; e < EPL; ++e) t2[e] = (T)0;
        if (i >= 2) {
          kop(v1, v0, v2, vbuf + (par ^ 1) * RW, yi - 1, t2);
          store_row(tbuf, par ^ 1, t2);
        }
        if (i >= 4) {
          kop(t1, t0, t2, tbuf + par * RW, yw, q);
          haw = true;
        }
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          vw[e] = v0[e];
          t0[e] = t1[e];
          t1[e] = t2[e];
        }
      }
      if (haw) {
        T wn[EPL];
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          double qq = (double)(tau * q[e]);
          if (j > 1) qq -= bprev * (double)(T)((double)VE::get(rawp, e) * s_prev);
          const T qt = (T)qq;
          wn[e] = (T)((double)qt - alpha * (double)vw[e]);
        }
        const int wpar = (ORDER == 1) ? (par ^ 1) : par;   // slot of index i - ORDER
        store_row(wbuf, wpar, wn);
        if (olane && yw >= y_lo && yw < y_hi) {
          VT vv;
          if constexpr (EPL == 1) {
            vv = wn[0];
          } else {
#pragma unroll
            for (int e = 0; e < EPL; ++e) vv[e] = wn[e];
          }
          if constexpr (NTS) __builtin_nontemporal_store(vv, (VT*)(dst + (size_t)yw * n2 + xb));
          else *(VT*)(dst + (size_t)yw * n2 + xb) = vv;
#pragma unroll
          for (int e = 0; e < EPL; ++e) {
            acc_b += (double)wn[e] * (double)wn[e];
            acc_c += (double)wn[e] * (double)vw[e];
          }
        }
        // K w at the row above (its lower neighbour wn just formed)
        const int yk = yw - 1;
        if (i >= 2 * ORDER + 2 && olane && yk >= y_lo && yk < y_hi) qform(wb, wa, wn, wbuf + (wpar ^ 1) * RW, yk);
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          wa[e] = wb[e];
          wb[e] = wn[e];
        }
      }
    }
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      v0[e] = v1[e];
      v1[e] = v2[e];
    }
  };
  constexpr int AHEAD = EPL * sizeof(T) >= 16 ? GMRF_S2_AHEAD64 : S2Ahead<T>::value;
  VT qv[AHEAD], pv[AHEAD];
#pragma unroll
  for (int d = 0; d < AHEAD; ++d) {
    qv[d] = ld(d);
    pv[d] = MODE == 0 ? ldp(d) : qv[d];
  }
  int i = 0;
  for (; i + AHEAD <= count; i += AHEAD) {
#pragma unroll
    for (int d = 0; d < AHEAD; ++d) {
      step(i + d, d & 1, qv[d], pv[d]);
      qv[d] = ld(i + d + AHEAD);
      if (MODE == 0) pv[d] = ldp(i + d + AHEAD);
    }
  }
#pragma unroll
  for (int d = 0; d < AHEAD; ++d)
    if (i + d < count) step(i + d, d & 1, qv[d], pv[d]);
}

#ifndef GMRF_L2D_WAVES
#define GMRF_L2D_WAVES 2       // lower bound on waves per SIMD given to the compiler; 4 caps registers at
                               // 128 and spills in the FP64 13-point case (measured 14% slower)
#endif
template <typename T, int ORDER, int MODE, bool NTS>
__global__ __launch_bounds__(256, GMRF_L2D_WAVES) void k_lanczos2d(StencilGeom g0, const T* __restrict__ X, long xld,
                                                   T* __restrict__ W, const T* __restrict__ Xprev, LzState S,
                                                   int j, double* __restrict__ out_a, double* __restrict__ out_b,
                                                   double* __restrict__ out_c) {
  constexpr int NW = 256 / kWave;
  __shared__ __align__(16) T vrow[kS2Waves][2][kS2MaxEpl<T> * kWave];
  __shared__ __align__(16) T trow[kS2Waves][2][kS2MaxEpl<T> * kWave];
  __shared__ __align__(16) T wrow[kS2Waves][2][kS2MaxEpl<T> * kWave];
  __shared__ double red[3 * NW];
  __shared__ int flag[1];
  int r, tile;
  xcd_order(!S.work && (g0.tune & kTuneXcd), tile, r);
  if (S.work) {
    const int2 wt = S.work[blockIdx.x];
    r = wt.x;
    tile = wt.y;
  }
  const StencilGeom g = S.col_geom ? S.col_geom[r] : g0;
  if (tile >= g.ftiles_x * g.ftiles_y) return;
  double s_cur = 1.0, s_prev = 0.0, bprev = 0.0, alpha = 0.0;
  if (MODE == 0) {
    // the scalar step, and alpha_j from the previous pass's partial sums (fixed order; the same in every
    // block), their loads issued together
    double qf, cc;
    if (!lz_open_with<256>(S, r, j, tile == 0, red, flag, S.part_a + (size_t)r * S.pstride, lz_pa(S, r),
                           j > 1 ? S.part_c + (size_t)r * S.pstride : nullptr, lz_pa(S, r), s_cur, s_prev, bprev,
                           qf, cc))
      return;
    alpha = qf * s_cur * s_cur - cc;
    if (tile == 0 && threadIdx.x == 0) S.alpha[lz_ia(S, r, j)] = alpha;
  }
  const int tx = tile % g.ftiles_x, ty = tile / g.ftiles_x;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x & (kWave - 1);
  const size_t roff = S.col_off ? (size_t)S.col_off[r] : (size_t)r * xld;
  double acc_b = 0.0, acc_c = 0.0, acc_a = 0.0;
  const T* prv = MODE == 0 ? Xprev + roff : nullptr;
  if constexpr (kS2MaxEpl<T> == 4) {
    if (g.fepl == 4) {
      s2f_strip<T, ORDER, MODE, 4, NTS>(g, tx, ty, w, lane, X + roff, W + roff, prv, j, s_cur, s_prev, bprev, alpha,
                                   &vrow[w][0][0], &trow[w][0][0], &wrow[w][0][0], acc_b, acc_c, acc_a);
      goto sums;
    }
  }
  if (g.fepl == 2)
    s2f_strip<T, ORDER, MODE, 2, NTS>(g, tx, ty, w, lane, X + roff, W + roff, prv, j, s_cur, s_prev, bprev, alpha,
                                 &vrow[w][0][0], &trow[w][0][0], &wrow[w][0][0], acc_b, acc_c, acc_a);
  else
    s2f_strip<T, ORDER, MODE, 1, NTS>(g, tx, ty, w, lane, X + roff, W + roff, prv, j, s_cur, s_prev, bprev, alpha,
                                 &vrow[w][0][0], &trow[w][0][0], &wrow[w][0][0], acc_b, acc_c, acc_a);
sums:
  // block sums in fixed order
  const double sa = block_sum<256>(acc_a, red);
  if (MODE == 0) {
    const double sb = block_sum<256>(acc_b, red);
    const double sc = block_sum<256>(acc_c, red);
    if (threadIdx.x == 0) {
      out_b[(size_t)r * S.pstride + tile] = sb;
      out_c[(size_t)r * S.pstride + tile] = sc;
    }
  }
  if (threadIdx.x == 0) out_a[(size_t)r * S.pstride + tile] = sa;
}

// ---- CSR: one thread per row ----------------------------------------------------------------
// One thread per row and KB columns per block: the row's entries (indices and values) are loaded once for
// its KB right-hand sides.  Every column's sums are formed as with one column per block (entries in row
// order; the block's partial sum over the same 256 rows), so the result bits do not depend on KB.
template <typename T, bool LZ, int KB>
__global__ __launch_bounds__(256) void k_csr(long n, const int64_t* __restrict__ rp,
                                             const int32_t* __restrict__ ci, const T* __restrict__ va,
                                             const T* __restrict__ X, long xld, T* __restrict__ Y,
                                             long yld, const T* __restrict__ Xprev, LzState S, int j, int k) {
  __shared__ double red[KB * (256 / kWave)];
  __shared__ int flag[KB];
  const int r0 = blockIdx.y * KB;
  double s_cur[KB], s_prev[KB], bprev[KB];
  bool act[KB];
#pragma unroll
  for (int c = 0; c < KB; ++c) {
    act[c] = r0 + c < k;    // uniform over the block
    s_cur[c] = 1.0;
    s_prev[c] = 0.0;
    bprev[c] = 0.0;
  }
  if (LZ) lz_open_multi<256, KB>(S, r0, k, j, blockIdx.x == 0, red, flag, act, s_cur, s_prev, bprev);
  bool any = false;
#pragma unroll
  for (int c = 0; c < KB; ++c) any = any || act[c];
  if (!any) return;
  const long row = (long)blockIdx.x * 256 + threadIdx.x;
  T s[KB];
#pragma unroll
  for (int c = 0; c < KB; ++c) s[c] = (T)0;
  auto term = [&](int c, T a, int32_t col) {
    const T raw = X[(size_t)(r0 + c) * xld + col];
    s[c] += a * (LZ ? (T)((double)raw * s_cur[c]) : raw);
  };
  if (row < n) {
    const int64_t e1 = rp[row + 1];
    int64_t e = rp[row];
    for (; e + 3 < e1; e += 4) {   // four entries' loads issued before the sums (same order)
      int32_t cc[4];
      T a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        cc[u] = ci[e + u];
        a[u] = va[e + u];
      }
#pragma unroll
      for (int c = 0; c < KB; ++c) {
        if (!act[c]) continue;
        T raw[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) raw[u] = X[(size_t)(r0 + c) * xld + cc[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) s[c] += a[u] * (LZ ? (T)((double)raw[u] * s_cur[c]) : raw[u]);
      }
    }
    for (; e < e1; ++e) {
      const int32_t c1 = ci[e];
      const T a1 = va[e];
#pragma unroll
      for (int c = 0; c < KB; ++c)
        if (act[c]) term(c, a1, c1);
    }
  }
#pragma unroll
  for (int c = 0; c < KB; ++c) {
    if (!act[c]) continue;
    const int r = r0 + c;
    double acc = 0.0;
    if (row < n) {
      if (LZ) {
        double q = (double)s[c];
        if (j > 1) q -= bprev[c] * (double)(T)((double)Xprev[(size_t)r * xld + row] * s_prev[c]);
        const T qt = (T)q;
        Y[(size_t)r * yld + row] = qt;
        acc = (double)(T)((double)X[(size_t)r * xld + row] * s_cur[c]) * (double)qt;
      } else {
        Y[(size_t)r * yld + row] = s[c];
      }
    }
    if (LZ) {
      const double bs = block_sum<256>(acc, red);
      if (threadIdx.x == 0) S.part_a[(size_t)r * S.pstride + blockIdx.x] = bs;
    }
  }
}

// ---- host side --------------------------------------------------------------------------------
void stencil_geom_tiles(StencilGeom& g, int dim, int order, int epl, int vbytes) {
  int TZ, TY, TX;
  g.epl = 1;
  // groups need a row length that is a multiple of the group: 4 for FP32, 2 for FP64.  A strip of 4-column
  // lanes covers 256 - 8 columns, so short rows leave much of the last strip idle: FP32 takes groups of
  // four only while its strips cover at most 15% more columns than those of pairs (measured: 2048 columns
  // 30.4 -> 26.1 us, 1024 columns 16.0 -> 15.0 us with fours; 512 columns 17.3 -> 19.5 us, so pairs)
  auto cover = [&](int e) {
    const int ox = s2_out(order, e);
    return (double)((g.n2 + ox - 1) / ox) * (kWave * e);
  };
  // the one-pass kernel by the same rule with its own strip width
  auto fcover = [&](int e) {
    const int ox = s2f_out(order, e);
    return (double)((g.n2 + ox - 1) / ox) * (kWave * e);
  };
  g.fepl = 1;
  // band of the operator kernel: 32 rows per wave from 256 rows up; shorter lattices take 16 or 8, so that
  // their few tiles still spread over more waves with shorter row chains (the one-pass kernel keeps 32:
  // with many columns in flight its halo rows cost more than the shorter chains save)
  g.band = kS2Band;
  if (dim == 2)
    while (g.band > 8 && g.n1 < 8 * g.band) g.band >>= 1;
  if (dim == 2) {
    if (epl > 0) g.epl = epl;
    else if (g.n2 % 2 != 0) g.epl = 1;
    else g.epl = (vbytes == 4 && g.n2 % 4 == 0 && cover(4) <= 1.15 * cover(2)) ? 4 : 2;
    if (epl > 0) g.fepl = epl;
    else if (g.n2 % 2 != 0) g.fepl = 1;
    else g.fepl = (GMRF_L2D_FEPL4 && vbytes == 4 && g.n2 % 4 == 0 && fcover(4) <= 1.15 * fcover(2)) ? 4 : 2;
  }
  if (dim == 1) { TZ = TileShape<1>::TZ; TY = TileShape<1>::TY; TX = TileShape<1>::TX; }
  else if (dim == 2) { TZ = 1; TY = kS2Waves * g.band; TX = s2_out(order, g.epl); }   // k_stencil2d
  else { TZ = TileShape<3>::TZ; TY = TileShape<3>::TY; TX = TileShape<3>::TX; }
  g.zc = 0;
  if (dim == 3 && order == 1 && g.n2 <= kZMaxN2 && (long)g.n0 * g.n1 * g.n2 >= kZMinPoints) {
    // z-march: segments of whole rows (at most kZSeg points), runs of planes sized so that a lattice
    // gives about 256 blocks per column (runs of at least 8 planes: each run also reads its neighbours).
    // Smaller lattices keep the box tiles: a run walks its planes one after another, which costs more
    // latency than the box tiles' extra reads when there are few points per column (measured at 64^3:
    // 6.7 against 15.2 us for one column, 3.3 against 5.0 TB/s for 32)
    g.band = std::max(1, std::min(g.n1, kZSeg / g.n2));
    g.tiles_x = (g.n1 + g.band - 1) / g.band;
    g.tiles_y = 1;
    const int runs = std::max(1, std::min(g.n0, (256 + g.tiles_x - 1) / g.tiles_x));
    g.zc = std::max(std::min(8, g.n0), (g.n0 + runs - 1) / runs);
    g.tiles_z = (g.n0 + g.zc - 1) / g.zc;
    g.ftiles_x = g.ftiles_y = 0;
    return;
  }
  g.tiles_x = (g.n2 + TX - 1) / TX;
  g.ftiles_x = dim == 2 ? (g.n2 + s2f_out(order, g.fepl) - 1) / s2f_out(order, g.fepl) : 0;   // k_lanczos2d
  g.ftiles_y = dim == 2 ? (g.n1 + kS2Waves * s2f_band(order) - 1) / (kS2Waves * s2f_band(order)) : 0;
  g.tiles_y = (g.n1 + TY - 1) / TY;
  g.tiles_z = (g.n0 + TZ - 1) / TZ;
}

// 2D operator kernel with rows per wave `band` and columns per lane `epl` instead of the lattice's rule (the
// caller checks that epl suits the storage type and the row length)
void stencil_geom_shape(StencilGeom& g, int order, int band, int epl) {
  g.band = band;
  g.epl = epl;
  g.tiles_x = (g.n2 + s2_out(order, epl) - 1) / s2_out(order, epl);
  g.tiles_y = (g.n1 + kS2Waves * band - 1) / (kS2Waves * band);
  g.tiles_z = 1;
}

int stencil_blocks(const StencilGeom& g) { return g.tiles_x * g.tiles_y * g.tiles_z; }

template <typename T, int ORDER, int DIM, bool LZ>
static void launch_stencil_t(const StencilGeom& g, const T* X, long xld, T* Y, long yld,
                             const T* Xprev, const LzState& S, int j, int k, hipStream_t st,
                             const int* active = nullptr) {
  if constexpr (DIM == 2) {
    if (g.tune & kTuneNtStore)
      hipLaunchKernelGGL((k_stencil2d<T, ORDER, LZ, true>), dim3(stencil_blocks(g), k), dim3(256), 0, st, g, X, xld,
                         Y, yld, Xprev, S, j, active);
    else
      hipLaunchKernelGGL((k_stencil2d<T, ORDER, LZ, false>), dim3(stencil_blocks(g), k), dim3(256), 0, st, g, X, xld,
                         Y, yld, Xprev, S, j, active);
  }
  else if (DIM == 3 && ORDER == 1 && g.zc > 0)
    hipLaunchKernelGGL((k_stencil3z<T, LZ>), dim3(stencil_blocks(g), k), dim3(kZThreads), 0, st, g, X, xld, Y, yld,
                       Xprev, S, j, active);
  else
    hipLaunchKernelGGL((k_stencil<T, ORDER, DIM, LZ>), dim3(stencil_blocks(g), k), dim3(256), 0, st, g,
                       X, xld, Y, yld, Xprev, S, j, active);
}

template <typename T>
void launch_stencil(const StencilGeom& g, int order, int dim, bool lz, const T* X, long xld, T* Y,
                    long yld, const T* Xprev, const LzState& S, int j, int k, hipStream_t st) {
#define CASE(O, D)                                                                      \
  if (order == O && dim == D) {                                                          \
    if (lz) launch_stencil_t<T, O, D, true>(g, X, xld, Y, yld, Xprev, S, j, k, st);      \
    else launch_stencil_t<T, O, D, false>(g, X, xld, Y, yld, Xprev, S, j, k, st);        \
    return;                                                                              \
  }
  CASE(1, 1) CASE(1, 2) CASE(1, 3) CASE(2, 1) CASE(2, 2) CASE(2, 3)
#undef CASE
}

// Uneven batch: S.col_geom / S.col_off describe each column's lattice; the grid covers the
// largest field's tiles.
template <typename T>
void launch_stencil_batch(int order, int dim, int max_tiles, const T* X, T* Y, const T* Xprev, const LzState& S,
                          int j, hipStream_t st, bool zmarch) {
  StencilGeom g{};
  if (zmarch) {   // 3D first-order fields whose rows fit a segment (every field of the batch)
    hipLaunchKernelGGL((k_stencil3z<T, true>), dim3(max_tiles, S.k), dim3(kZThreads), 0, st, g, X, 0L, Y, 0L, Xprev,
                       S, j, (const int*)nullptr);
    return;
  }
#define CASEB(O, D)                                                                                          \
  if (order == O && dim == D) {                                                                               \
    hipLaunchKernelGGL((k_stencil<T, O, D, true>), dim3(max_tiles, S.k), dim3(256), 0, st, g, X, 0L, Y, 0L, \
                       Xprev, S, j, (const int*)nullptr);                                                    \
    return;                                                                                                   \
  }
#define CASEB2(O)                                                                                            \
  if (order == O && dim == 2) {                                                                               \
    hipLaunchKernelGGL((k_stencil2d<T, O, true, false>), dim3(max_tiles, S.k), dim3(256), 0, st, g, X, 0L, Y, 0L, \
                       Xprev, S, j, (const int*)nullptr);                                                    \
    return;                                                                                                   \
  }
  CASEB(1, 1) CASEB2(1) CASEB(1, 3) CASEB(2, 1) CASEB2(2) CASEB(2, 3)
#undef CASEB
#undef CASEB2
}
template void launch_stencil_batch<double>(int, int, int, const double*, double*, const double*, const LzState&,
                                           int, hipStream_t, bool);
template void launch_stencil_batch<float>(int, int, int, const float*, float*, const float*, const LzState&, int,
                                          hipStream_t, bool);

int lanczos2d_blocks(const StencilGeom& g) { return g.ftiles_x * g.ftiles_y; }

template <typename T>
void launch_lanczos2d(const StencilGeom& g, int order, int mode, int grid_x, const T* X, long xld, T* W,
                      const T* Xprev, const LzState& S, int j, int k, double* out_a, double* out_b, double* out_c,
                      hipStream_t st) {
  const dim3 grid(grid_x > 0 ? grid_x : lanczos2d_blocks(g), k);
#define CASEL(O, M)                                                                                             \
  if (order == O && mode == M) {                                                                                 \
    if (g.tune & kTuneNtStore)                                                                                   \
      hipLaunchKernelGGL((k_lanczos2d<T, O, M, true>), grid, dim3(256), 0, st, g, X, xld, W, Xprev, S, j, out_a, \
                         out_b, out_c);                                                                          \
    else                                                                                                         \
      hipLaunchKernelGGL((k_lanczos2d<T, O, M, false>), grid, dim3(256), 0, st, g, X, xld, W, Xprev, S, j, out_a,\
                         out_b, out_c);                                                                          \
    return;                                                                                                      \
  }
  CASEL(1, 0) CASEL(2, 0) CASEL(1, 1) CASEL(2, 1)
#undef CASEL
}
template void launch_lanczos2d<double>(const StencilGeom&, int, int, int, const double*, long, double*,
                                       const double*, const LzState&, int, int, double*, double*, double*,
                                       hipStream_t);
template void launch_lanczos2d<float>(const StencilGeom&, int, int, int, const float*, long, float*, const float*,
                                      const LzState&, int, int, double*, double*, double*, hipStream_t);

int csr_blocks(long n) { return (int)((n + 255) / 256); }

template <typename T, int KB>
static void launch_csr_kb(long n, const int64_t* rp, const int32_t* ci, const T* va, bool lz, const T* X,
                          long xld, T* Y, long yld, const T* Xprev, const LzState& S, int j, int k,
                          hipStream_t st) {
  const dim3 grid(csr_blocks(n), (k + KB - 1) / KB);
  if (lz)
    hipLaunchKernelGGL((k_csr<T, true, KB>), grid, dim3(256), 0, st, n, rp, ci, va, X, xld, Y, yld, Xprev, S, j, k);
  else
    hipLaunchKernelGGL((k_csr<T, false, KB>), grid, dim3(256), 0, st, n, rp, ci, va, X, xld, Y, yld, Xprev, S, j, k);
}

// Columns per block (no result bit depends on it): 8 or 4 where the grid keeps at least kCsrMinBlocks blocks,
// else 1.  Blocking saves re-reads of the matrix on large matrices; on small ones (the 900-row matrix of
// Section 5.2 with 32 columns: 16 blocks at 8 columns each) the fewer, longer blocks are latency-bound.
#ifndef GMRF_CSR_MAX_KB
#define GMRF_CSR_MAX_KB 8
#endif
constexpr long kCsrMinBlocks = 512;
template <typename T>
void launch_csr(long n, const int64_t* rp, const int32_t* ci, const T* va, bool lz, const T* X,
                long xld, T* Y, long yld, const T* Xprev, const LzState& S, int j, int k,
                hipStream_t st) {
  const long rb = csr_blocks(n);
  if (GMRF_CSR_MAX_KB >= 8 && k >= 8 && rb * ((k + 7) / 8) >= kCsrMinBlocks)
    launch_csr_kb<T, 8>(n, rp, ci, va, lz, X, xld, Y, yld, Xprev, S, j, k, st);
  else if (GMRF_CSR_MAX_KB >= 4 && k >= 4 && rb * ((k + 3) / 4) >= kCsrMinBlocks)
    launch_csr_kb<T, 4>(n, rp, ci, va, lz, X, xld, Y, yld, Xprev, S, j, k, st);
  else
    launch_csr_kb<T, 1>(n, rp, ci, va, lz, X, xld, Y, yld, Xprev, S, j, k, st);
}

template void launch_stencil<double>(const StencilGeom&, int, int, bool, const double*, long, double*,
                                     long, const double*, const LzState&, int, int, hipStream_t);
template void launch_stencil<float>(const StencilGeom&, int, int, bool, const float*, long, float*,
                                    long, const float*, const LzState&, int, int, hipStream_t);
template void launch_csr<double>(long, const int64_t*, const int32_t*, const double*, bool,
                                 const double*, long, double*, long, const double*, const LzState&,
                                 int, int, hipStream_t);
template void launch_csr<float>(long, const int64_t*, const int32_t*, const float*, bool,
                                const float*, long, float*, long, const float*, const LzState&, int,
                                int, hipStream_t);

}  // namespace gmrf
