// Preconditioned Lanczos step in the spectral basis (Proposition 1 with Algorithm 1, Section 5.1).
//
// The Krylov vectors are packed half spectra (fft.hpp) and the operator is
//     A_hat = I - Lambda^{-1/2} F D F^H Lambda^{-1/2},   D = M - Q,
// where D, the difference between the periodic and the free-boundary precision, is nonzero only
// within one point of the lattice boundary.  A step therefore needs
//   * u = F^H Lambda^{-1/2} v_j only at the four boundary columns {0, 1, N2-2, N2-1} of every row
//     and on the six boundary rows {0, 1, 2, N1-3, N1-2, N1-1};
//   * D u, supported on those columns and rows;
//   * Lambda^{-1/2} F D u, whose column transform is closed form in the D u coefficients,
// and no full 2D FFT is taken inside the loop.  u on the boundary comes from dot products of
// Y = lambda^{-1/2} v_j / n: per spectral row k1 the four dots G_t(k1) = sum_c gamma_t(c) Y(k1, c),
// whose inverse DFT over k1 is u(., col_t), and per packed column c the six dots
// h_q(c) = sum_k1 e^{+2 pi i k1 r_q / N1} Y(k1, c), the packed row spectra of u on the boundary
// rows r_q.  The kernel that writes w_j forms these dots for the next step while w_j is in
// registers (they are linear, so they are taken on w_j and scaled by 1 / beta_j once beta_j is
// known).  Two launches per step:
//
// k_band  opens iteration j (scalar step and stopping rule, beta_{j-1} from the partial sums),
//         scales the dots by 1 / beta_{j-1}; block 2 of each field inverts the G_t (four length-N1
//         FFTs), forms the interior coefficients (d0, d1) of D u and their DFTs D0, D1 over the
//         rows; blocks 0 and 1 invert the boundary rows, form D u there (wrap and corner terms) and
//         its packed row spectra E_q.  Each block adds its share of <u, D u>.
// k_step  (reads slots j-1 and j-2, writes slot j) evaluates the 2D spectrum of D u as
//         Z(k1, c) = A_c D0(k1) + B_c D1(k1) + sum_q e^{-2 pi i k1 r_q / N1} E_q(c),
//         A_c = 1 - conj w^c, B_c = w^c - conj w^{2c} (w = e^{-2 pi i / N2}), and writes
//         w_j = v_j - lambda^{-1/2} Z - alpha_j v_j - beta_{j-1} v_{j-1}
//         in one pass: alpha_j is known beforehand from
//         v_j^T A v_j = ||v_j||^2 - n <u, D u>  (Parseval, ||v_j|| = 1),
//         minus <w_{j-1}, v_{j-1}> = beta_{j-1} v_j^T v_{j-1}, the term by which Algorithm 1's
//         alpha_j = v_j^T (A v_j - beta_{j-1} v_{j-1}) differs in floating point.  It leaves the
//         ||w_j||^2 and <w_j, v_j> partial sums and the dots of lambda^{-1/2} w_j / n.
// k_dots  the dots alone, for slot 0 and for a w_j that full reorthogonalisation changed.
//
// Packed column 0 (X_0 + i X_{N2/2}) couples k1 with -k1 through the multiplier; one extra block
// per field handles it, so the other lanes carry no special case.
//
// Interior rows r = 2..N1-3 of D u are supported on columns {0, 1, N2-2, N2-1}: with
// e_r = u(r,0) - u(r,N2-1),
//   order 1:  d0 = tau e_r,  d1 = 0
//   order 2:  d0 = tau [K_f(Eu)(r,0) + K_p u(r,0) - K_p u(r,N2-1)],  d1 = -tau e_r,
// D u(r,0) = d0, D u(r,1) = d1, D u(r,N2-2) = -d1, D u(r,N2-1) = -d0, and the packed row spectrum
// is d0 A_c + d1 B_c (column 0: X_0 = 0 and X_{N2/2} = 2 (d0 - d1)).  On the boundary rows
// D u = tau [K_f (E u) + E (K_p u)] (order 2) or tau E u (order 1), E the wrap-edge Laplacian.
#include "fft.hpp"
#include "fft_lds.hpp"

#include <algorithm>

namespace gmrf {

// Launch shape of the streaming kernels (build-time overridable for tuning).
#ifndef GMRF_STEP_ROWS
#define GMRF_STEP_ROWS 64
#endif
#ifndef GMRF_STEP_WAVES
#define GMRF_STEP_WAVES 4
#endif
#ifndef GMRF_STEP_PREFETCH
#define GMRF_STEP_PREFETCH 0
#endif
#ifndef GMRF_STREAM_NT
#define GMRF_STREAM_NT 0     // 1: non-temporal loads of the Krylov vectors, 2: loads and stores
#endif
constexpr int kStepThreads = 512;              // threads per streaming block
constexpr int kStepWaves = GMRF_STEP_WAVES;    // waves per SIMD asked of the compiler
constexpr int kStepRows = GMRF_STEP_ROWS;      // spectral rows per block (column dots are partial per block)
constexpr int kBandBlocks = 3;                 // per field: top edge, bottom edge, interior

// One packed column per lane; a row segment of LG = min(H, 64) lanes (one wave when the row holds
// 64 packed columns or more).  A block covers one column tile of LG columns, RPS = NT / LG rows at
// a time and `rows` rows in all; CT column tiles per row, NB row blocks per field, plus one block
// per field for column 0.
struct SpecTile {
  int LG, CT, RPS, R, NB;
};
__host__ __device__ inline SpecTile spec_tile(int N1, int H, int NT, int rows) {
  SpecTile t;
  t.LG = H < kWave ? H : kWave;
  t.CT = H / t.LG;
  t.RPS = NT / t.LG;
  t.R = N1 < rows ? N1 : rows;
  t.NB = N1 / t.R;
  return t;
}

template <typename T>
struct StepIO {
  double* gpart;       // [k][N1][CT + 1][8]  row dots G_0, A, B, G_2 (re, im) per row segment; segment CT: column 0
  C2<double>* cpart;   // [k][NB][6][H]       column dots P0, P1, R1, P2, R2, H3 per row block (column 0: zero)
  double* c0dots;      // [k][12]             column dots of column 0 over all rows
  double* ub;          // [k][N1][4]          u at the boundary columns (general band kernel)
  C2<double>* dtab;    // [k][N1][2]          D0(k1), D1(k1)
  C2<T>* etab;         // [k][4][H]           packed row spectra of D u on rows 0, 1, N1-2, N1-1
  C2<T>* hin;          // [k][2][6][H]        per edge block: packed row spectra of u on the boundary rows
  T* work;             // [k][2][20 N2]       per edge block: u (6 rows), E u (6), K_p u (4), D u (4)
  int CT, NB;
};

template <typename T>
__device__ __forceinline__ double rnd(double v) { return (double)(T)v; }

// Krylov vectors stream through once per step; optionally with non-temporal loads and stores, which keep
// them from evicting the tables every block re-reads (multipliers, boundary spectra) from L2.
template <typename T> struct Vec2;
template <> struct Vec2<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct Vec2<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <typename T>
__device__ __forceinline__ C2<T> stream_load(const C2<T>* p) {
  if constexpr (GMRF_STREAM_NT >= 1) {
    const typename Vec2<T>::type v = __builtin_nontemporal_load((const typename Vec2<T>::type*)p);
    return {v.x, v.y};
  } else {
    return *p;
  }
}
template <typename T>
__device__ __forceinline__ void stream_store(C2<T>* p, C2<T> a) {
  if constexpr (GMRF_STREAM_NT >= 2) {
    typename Vec2<T>::type v;
    v.x = a.x;
    v.y = a.y;
    __builtin_nontemporal_store(v, (typename Vec2<T>::type*)p);
  } else {
    *p = a;
  }
}

// Row index that is the same on every lane of a row segment: with full-wave segments it is read
// from the first lane, so row-indexed tables come through scalar loads.
template <int LG>
__device__ __forceinline__ int seg_uniform(int v) {
  if constexpr (LG == kWave) return __builtin_amdgcn_readfirstlane(v);
  else return v;
}

// Sum of 8 values over groups of LG adjacent lanes (LG a power of two, 2..64), halving the value
// set at the first three exchanges (named scalars, so that the lane-dependent choice stays a
// register select).  Afterwards a lane holds the full sums of values base..base+NV-1 in
// a0..a{NV-1}, NV = max(1, 8 / LG); lanes with (lane & LOW) == 0 hold distinct sets.
template <int LG>
struct GroupReduce {
  static constexpr int NV = LG >= 8 ? 1 : 8 / LG;
  static constexpr int LOW = LG >= 16 ? LG / 8 - 1 : 0;
  __device__ static __forceinline__ void pair(bool up, double& lo, double hi, int o) {
    const double send = up ? lo : hi;
    const double keep = up ? hi : lo;
    lo = keep + __shfl_xor(send, o, kWave);
  }
  __device__ static __forceinline__ int run(double& a0, double& a1, double& a2, double& a3, double& a4, double& a5,
                                            double& a6, double& a7, int lane) {
    int base = 0;
    if constexpr (LG >= 2) {
      constexpr int o = LG / 2;
      const bool up = (lane & o) != 0;
      pair(up, a0, a4, o);
      pair(up, a1, a5, o);
      pair(up, a2, a6, o);
      pair(up, a3, a7, o);
      if (up) base += 4;
    }
    if constexpr (LG >= 4) {
      constexpr int o = LG / 4;
      const bool up = (lane & o) != 0;
      pair(up, a0, a2, o);
      pair(up, a1, a3, o);
      if (up) base += 2;
    }
    if constexpr (LG >= 8) {
      constexpr int o = LG / 8;
      const bool up = (lane & o) != 0;
      pair(up, a0, a1, o);
      if (up) base += 1;
    }
    if constexpr (LG >= 16) a0 += __shfl_xor(a0, LG / 16, kWave);
    if constexpr (LG >= 32) a0 += __shfl_xor(a0, LG / 32, kWave);
    if constexpr (LG >= 64) a0 += __shfl_xor(a0, LG / 64, kWave);
    return base;
  }
};

// Full-wave version (LG = 64) of GroupReduce: the exchanges at distance 32 and 16 use the gfx950
// lane swaps (after v_permlane32_swap(lo, hi) a lane's lo + hi is the pair sum of its half: lower
// lanes get lo[i] + lo[i+32], upper lanes hi[i-32] + hi[i]; likewise per 16-lane row with
// v_permlane16_swap), the one at distance 8 the DPP row mirror (lane i <-> 15 - i), and the last three
// a half-row mirror and two quad permutes.  No LDS traffic; LOW = 7, base from lane bits 5, 4, 3.
__device__ __forceinline__ int wave_reduce8(double& a0, double& a1, double& a2, double& a3, double& a4, double& a5,
                                            double& a6, double& a7, int lane) {
  swap32(a0, a4);
  swap32(a1, a5);
  swap32(a2, a6);
  swap32(a3, a7);
  a0 += a4;
  a1 += a5;
  a2 += a6;
  a3 += a7;
  swap16(a0, a2);
  swap16(a1, a3);
  a0 += a2;
  a1 += a3;
  const bool up = (lane & 8) != 0;
  const double send = up ? a0 : a1, keep = up ? a1 : a0;
  a0 = keep + dpp<kDppRowMirror>(send);
  a0 += dpp<kDppRowHalfMirror>(a0);
  a0 += dpp<kDppQuadXor2>(a0);
  a0 += dpp<kDppQuadXor1>(a0);
  return ((lane & 32) ? 4 : 0) + ((lane & 16) ? 2 : 0) + (up ? 1 : 0);
}

// ---- dot products of lambda^{-1/2} x / n -----------------------------------------------------------------
// Band-column weights of packed column c >= 1: G_0 += 2 y, A += ga y, B += gb y, G_2 += g2 y with
// ga = 2 Re w^c, gb = 2 Im w^c, g2 = 2 w^{2c}; then G_1 = A - i B, G_3 = A + i B.  Column 0
// (X_0 + i X_{N2/2}): G_0 = G_2 += (1 - i) y, A += (1 + i) y.
struct DotCoef {
  double ga, gb, g2x, g2y;
  __device__ __forceinline__ void init(const C2<double>* __restrict__ tw2, int c) {
    const C2<double> w1 = tw2[c], w2 = tw2[2 * c];
    ga = 2.0 * w1.x;
    gb = 2.0 * w1.y;
    g2x = 2.0 * w2.x;
    g2y = 2.0 * w2.y;
  }
};

// Row-dot values of one element y (before the reduction over the row) and its column dots:
// e^{+i theta}, e^{+2 i theta} through cos/sin pairs, e^{-3 i theta} directly (theta = 2 pi k1 / N1).
__device__ __forceinline__ void dot_elem(const DotCoef& g, double yx, double yy, C2<double> t1, C2<double> t2,
                                         C2<double> t3, double (&ca)[12], double& r0, double& r1, double& r2,
                                         double& r3, double& r4, double& r5, double& r6, double& r7) {
  r0 = 2.0 * yx;
  r1 = 2.0 * yy;
  r2 = g.ga * yx;
  r3 = g.ga * yy;
  r4 = g.gb * yx;
  r5 = g.gb * yy;
  r6 = g.g2x * yx - g.g2y * yy;
  r7 = g.g2x * yy + g.g2y * yx;
  const double c1 = t1.x, s1 = -t1.y, c2 = t2.x, s2 = -t2.y;
  ca[0] += yx;
  ca[1] += yy;
  ca[2] += c1 * yx;
  ca[3] += c1 * yy;
  ca[4] += s1 * yx;
  ca[5] += s1 * yy;
  ca[6] += c2 * yx;
  ca[7] += c2 * yy;
  ca[8] += s2 * yx;
  ca[9] += s2 * yy;
  ca[10] += t3.x * yx - t3.y * yy;
  ca[11] += t3.x * yy + t3.y * yx;
}

// Reduce r0..r7 over the row segment and store them as segment `seg` of row k1.
template <int LG>
__device__ __forceinline__ void store_row_dots(double* __restrict__ gp, int lane, double r0, double r1, double r2,
                                               double r3, double r4, double r5, double r6, double r7) {
  int base;
  if constexpr (LG == kWave) base = wave_reduce8(r0, r1, r2, r3, r4, r5, r6, r7, lane);
  else base = GroupReduce<LG>::run(r0, r1, r2, r3, r4, r5, r6, r7, lane);
  constexpr int LOW = LG == kWave ? 7 : GroupReduce<LG>::LOW;
  constexpr int NV = LG == kWave ? 1 : GroupReduce<LG>::NV;
  if ((lane & LOW) == 0) {
    gp[base] = r0;
    if constexpr (NV >= 2) gp[base + 1] = r1;
    if constexpr (NV >= 4) {
      gp[base + 2] = r2;
      gp[base + 3] = r3;
    }
  }
}

// Column dots of the block: lanes sharing a column (ro = 0..nro-1) combine in ro order through
// xch (NT * 4 doubles) and store row block rb's partials.
template <int NT>
__device__ __forceinline__ void store_col_dots(const double (&ca)[12], double* xch, int tid, int ro, int tlane,
                                               int LG, int nro, C2<double>* __restrict__ cp, int H, int c) {
#pragma unroll
  for (int round = 0; round < 3; ++round) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) xch[tid * 4 + i] = ca[round * 4 + i];
    __syncthreads();
    if (ro == 0) {
      double sacc[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) sacc[i] = xch[tid * 4 + i];
      for (int o = 1; o < nro; ++o) {
#pragma unroll
        for (int i = 0; i < 4; ++i) sacc[i] += xch[(o * LG + tlane) * 4 + i];
      }
      cp[(size_t)(2 * round) * H + c] = {sacc[0], sacc[1]};
      cp[(size_t)(2 * round + 1) * H + c] = {sacc[2], sacc[3]};
    }
  }
}

// Column 0 over all rows: y(k1) = scale (p x(k1) + q conj x(-k1)), p = (m0 + mN)/2, q = (m0 - mN)/2;
// its row-dot contributions as segment CT, its column dots into c0dots.
template <typename T, int NT>
__device__ void col0_dots(const C2<T>* __restrict__ x, int N1, int H, const T* __restrict__ mult, double scale,
                          const C2<double>* __restrict__ tw1, double* __restrict__ gpart, int CT,
                          double* __restrict__ c0d, double* red) {
  const int ms = mult_stride(H);
  double ca[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) ca[i] = 0.0;
  for (int k1 = threadIdx.x; k1 < N1; k1 += NT) {
    const int kb = (N1 - k1) & (N1 - 1);
    const C2<T> a = x[(size_t)k1 * H], b = x[(size_t)kb * H];
    const double m0 = (double)mult[(size_t)k1 * ms], mN = (double)mult[(size_t)k1 * ms + H];
    const double p = 0.5 * (m0 + mN) * scale, q = 0.5 * (m0 - mN) * scale;
    const double yx = p * (double)a.x + q * (double)b.x, yy = p * (double)a.y - q * (double)b.y;
    double* gp = gpart + ((size_t)k1 * (CT + 1) + CT) * 8;
    gp[0] = yx + yy;   // G_0 += (1 - i) y
    gp[1] = yy - yx;
    gp[2] = yx - yy;   // A += (1 + i) y
    gp[3] = yy + yx;
    gp[4] = 0.0;
    gp[5] = 0.0;
    gp[6] = yx + yy;   // G_2 += (1 - i) y
    gp[7] = yy - yx;
    const C2<double> t1 = tw1[k1], t2 = tw1[(2 * k1) & (N1 - 1)], t3 = tw1[(3 * k1) & (N1 - 1)];
    const double c1 = t1.x, s1 = -t1.y, c2 = t2.x, s2 = -t2.y;
    ca[0] += yx;
    ca[1] += yy;
    ca[2] += c1 * yx;
    ca[3] += c1 * yy;
    ca[4] += s1 * yx;
    ca[5] += s1 * yy;
    ca[6] += c2 * yx;
    ca[7] += c2 * yy;
    ca[8] += s2 * yx;
    ca[9] += s2 * yy;
    ca[10] += t3.x * yx - t3.y * yy;
    ca[11] += t3.x * yy + t3.y * yx;
  }
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    const double v = block_sum<NT>(ca[i], red);
    if (threadIdx.x == 0) c0d[i] = v;
  }
}

// Dots of y = lambda^{-1/2} x scale for k fields (grid: NB * CT + 1 blocks per field).
template <typename T, int LG>
__global__ __launch_bounds__(kStepThreads, kStepWaves) void k_dots(const C2<T>* __restrict__ X, int N1, int H,
                                                                   const T* __restrict__ mult, double scale,
                                                                   const C2<double>* __restrict__ tw1,
                                                                   const C2<double>* __restrict__ tw2, LzState S,
                                                                   StepIO<T> io) {
  constexpr int NT = kStepThreads;
  __shared__ double red[NT / kWave];
  __shared__ int flag[1];
  __shared__ double xch[NT * 4];
  const int r = blockIdx.y;
  if (!block_active(S, r, flag)) return;
  const SpecTile tl = spec_tile(N1, H, NT, kStepRows);
  const C2<T>* src = X + (size_t)r * N1 * H;
  double* gpart = io.gpart + (size_t)r * N1 * (tl.CT + 1) * 8;
  if ((int)blockIdx.x == tl.NB * tl.CT) {
    col0_dots<T, NT>(src, N1, H, mult, scale, tw1, gpart, tl.CT, io.c0dots + (size_t)r * 12, red);
    return;
  }
  const int rb = blockIdx.x / tl.CT, ct = blockIdx.x - rb * tl.CT;
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int tlane = tid % LG, ro = tid / LG;
  const int c = ct * LG + tlane;
  const double sc = c == 0 ? 0.0 : scale;   // column 0 belongs to the extra block
  DotCoef g;
  g.init(tw2, c);
  const int ms = mult_stride(H);
  double ca[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) ca[i] = 0.0;
  const int nsteps = ro < tl.R ? (tl.R - ro + tl.RPS - 1) / tl.RPS : 0;
  for (int s = 0; s < nsteps; ++s) {
    const int k1 = seg_uniform<LG>(rb * tl.R + ro + s * tl.RPS);
    const C2<T> x = src[(size_t)k1 * H + c];
    const double f = (double)mult[(size_t)k1 * ms + c] * sc;
    double r0, r1, r2, r3, r4, r5, r6, r7;
    dot_elem(g, f * (double)x.x, f * (double)x.y, tw1[k1], tw1[(2 * k1) & (N1 - 1)], tw1[(3 * k1) & (N1 - 1)], ca,
             r0, r1, r2, r3, r4, r5, r6, r7);
    store_row_dots<LG>(gpart + ((size_t)k1 * (tl.CT + 1) + ct) * 8, lane, r0, r1, r2, r3, r4, r5, r6, r7);
  }
  store_col_dots<NT>(ca, xch, tid, ro, tlane, LG, min(tl.RPS, tl.R),
                     io.cpart + ((size_t)r * tl.NB + rb) * 6 * H, H, c);
}

// ---- band kernel -------------------------------------------------------------------------------------
// Opens iteration j (every block of the field reaches the same decision; block 0 stores it) and, for
// the interior block, stores <w_{j-1}, v_{j-1}> next to the <u, D u> partials.
template <int NT>
__device__ __forceinline__ bool band_open(const LzState& S, int r, int j, int use_c, double* red, int* flag,
                                          double& s_cur) {
  double s_prev, bprev, qa, c;
  const bool with_c = blockIdx.x == 2 && use_c && j > 1;   // the <w_{j-1}, v_{j-1}> partials load with the opener's
  if (!lz_open_with<NT>(S, r, j, blockIdx.x == 0, red, flag, nullptr, 0,
                        with_c ? S.part_c + (size_t)r * S.pstride : nullptr, lz_pb(S, r), s_cur, s_prev, bprev, qa, c))
    return false;
  if (blockIdx.x == 2 && threadIdx.x == 0) S.part_a[(size_t)r * S.pstride + kBandBlocks] = c;
  return true;
}

// G_t(k1) = s_cur * (sum of the row-dot segments), t = 0..3 (G_1 = A - i B, G_3 = A + i B).
__device__ __forceinline__ void band_row_dot(const double* __restrict__ gp, int k1, int RH, int t, double s_cur,
                                             double& gx, double& gy) {
  const double* g = gp + (size_t)k1 * RH * 8;
  gx = 0.0;
  gy = 0.0;
  if (t == 0 || t == 2) {
    const int o = t == 0 ? 0 : 6;
    for (int sg = 0; sg < RH; ++sg) {
      gx += g[sg * 8 + o];
      gy += g[sg * 8 + o + 1];
    }
  } else {
    double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0;
    for (int sg = 0; sg < RH; ++sg) {
      ax += g[sg * 8 + 2];
      ay += g[sg * 8 + 3];
      bx += g[sg * 8 + 4];
      by += g[sg * 8 + 5];
    }
    gx = t == 1 ? ax + by : ax - by;
    gy = t == 1 ? ay - bx : ay + bx;
  }
  gx *= s_cur;
  gy *= s_cur;
}

// Column dot q of packed column c: s_cur * (sum over the row blocks, plus column 0's own sums).
template <typename T>
__device__ __forceinline__ void band_col_dot(const StepIO<T>& io, int r, int H, int q, int c, double s_cur,
                                             double& sx, double& sy) {
  const int NB = io.NB;
  const C2<double>* cp = io.cpart + (size_t)r * NB * 6 * H + (size_t)q * H + c;
  sx = 0.0;
  sy = 0.0;
  for (int b0 = 0; b0 < NB; b0 += 8) {
    C2<double> v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = (b0 + i < NB) ? cp[(size_t)(b0 + i) * 6 * H] : C2<double>{0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      sx += v[i].x;
      sy += v[i].y;
    }
  }
  if (c == 0) {
    sx += io.c0dots[(size_t)r * 12 + 2 * q];
    sy += io.c0dots[(size_t)r * 12 + 2 * q + 1];
  }
  sx *= s_cur;
  sy *= s_cur;
}

// Boundary-row slots 0..5 hold rows {0, 1, 2, N1-3, N1-2, N1-1}; output slots 0..3 rows {0, 1, N1-2, N1-1}.
__device__ __forceinline__ int slot_row(int s, int N1) { return s < 3 ? s : N1 - 6 + s; }
__device__ __forceinline__ int row_slot(int r, int N1) { return r <= 2 ? r : r - (N1 - 6); }

// General version: u, E u, K_p u and D u of the boundary rows go through global scratch (any side
// up to 4096).
template <typename T, int ORDER>
__global__ __launch_bounds__(kFftThreads) void k_band_global(int N1, int N2, const C2<T>* __restrict__ tw1,
                                                      const C2<T>* __restrict__ tw2, T k2, T tau, LzState S,
                                                      int j, int use_c, int periodic, StepIO<T> io) {
  constexpr int NT = kFftThreads;
  __shared__ C2<T> buf[FftCfg<T>::ELEMS];
  __shared__ double red[3 * (NT / kWave)];   // lz_open_with takes three sets
  __shared__ int flag[1];
  const int r = blockIdx.y;
  double s_cur;
  if (!band_open<NT>(S, r, j, use_c, red, flag, s_cur)) return;
  const int H = N2 / 2;
  const int tid = threadIdx.x;
  double* pa = S.part_a + (size_t)r * S.pstride;
  C2<T>* E = io.etab + (size_t)r * 4 * H;
  C2<double>* Dt = io.dtab + (size_t)r * N1 * 2;
  if (periodic) {
    // a periodic Q is its own preconditioner: D = 0
    if (blockIdx.x < 2) {
      for (int i = tid; i < 2 * H; i += NT) E[(size_t)blockIdx.x * 2 * H + i] = {(T)0, (T)0};
    } else {
      for (int i = tid; i < 2 * N1; i += NT) Dt[i] = {0.0, 0.0};
    }
    if (tid == 0) pa[blockIdx.x] = 0.0;
    return;
  }
  if (blockIdx.x == 2) {
    // ---- interior: u at the boundary columns, (d0, d1), D0 and D1 ----
    const int RH = io.CT + 1;
    const double* gp = io.gpart + (size_t)r * N1 * RH * 8;
    double* ub = io.ub + (size_t)r * N1 * 4;
    const int nb = min(4, FftCfg<T>::ELEMS / N1);
    for (int t0 = 0; t0 < 4; t0 += nb) {
      const int nbb = min(nb, 4 - t0);
      for (int idx = tid; idx < nbb * N1; idx += NT) {
        const int t = t0 + idx / N1, k1 = idx % N1;
        double gx, gy;
        band_row_dot(gp, k1, RH, t, s_cur, gx, gy);
        buf[idx] = {(T)gx, (T)gy};
      }
      __syncthreads();
      lds_fft<T, false>(buf, N1, nbb, N1, 1, tw1, true);
      for (int idx = tid; idx < nbb * N1; idx += NT) {
        const int t = t0 + idx / N1, k1 = idx % N1;
        ub[(size_t)k1 * 4 + t] = (double)buf[idx].x;
      }
      __threadfence_block();
      __syncthreads();
    }
    const double kk = (double)k2, tt = (double)tau;
    double acc = 0.0;
    for (int row = tid; row < N1; row += NT) {
      double d0 = 0.0, d1 = 0.0;
      if (row >= 2 && row < N1 - 2) {
        const double* cu = ub + 4 * row;
        const double u0 = cu[0], u1 = cu[1], um2 = cu[2], um1 = cu[3];
        const double e = u0 - um1;
        if (ORDER == 1) {
          d0 = tt * e;
        } else {
          const double a0 = cu[-4], a3 = cu[-1], b0 = cu[4], b3 = cu[7];
          const double em = a0 - a3, ep = b0 - b3;
          const double kfe0 = kk * e + e + (e - em) + (e - ep);
          const double kp0 = kk * u0 + (u0 - u1) + (u0 - um1) + (u0 - a0) + (u0 - b0);
          const double kpm1 = kk * um1 + (um1 - um2) + (um1 - u0) + (um1 - a3) + (um1 - b3);
          d0 = tt * (kfe0 + kp0 - kpm1);
          d1 = -tt * e;
        }
        acc += d0 * (u0 - um1) + d1 * (u1 - um2);
      }
      buf[row] = {(T)d0, (T)d1};
    }
    const double uDu = block_sum<NT>(acc, red);
    if (tid == 0) pa[2] = uDu;
    lds_fft<T, false>(buf, N1, 1, N1, 1, tw1, false);
    // d0, d1 real: one complex FFT of d0 + i d1 gives both spectra
    for (int k = tid; k < N1; k += NT) {
      const C2<T> zk = buf[k], zm = buf[(N1 - k) & (N1 - 1)];
      Dt[2 * k] = {0.5 * ((double)zk.x + (double)zm.x), 0.5 * ((double)zk.y - (double)zm.y)};
      Dt[2 * k + 1] = {0.5 * ((double)zk.y + (double)zm.y), 0.5 * ((double)zm.x - (double)zk.x)};
    }
    return;
  }
  // ---- boundary rows: block `half` produces output slots 2 half, 2 half + 1 ----
  const int half = blockIdx.x;
  T* U = io.work + ((size_t)r * 2 + half) * 20 * N2;
  T* EU = U + (size_t)6 * N2;
  T* KP = EU + (size_t)6 * N2;
  T* DU = KP + (size_t)4 * N2;
  C2<T>* Cin = io.hin + ((size_t)r * 2 + half) * 6 * H;
  {
    for (int c = tid; c < H; c += NT) {
      double s[12];
#pragma unroll
      for (int q = 0; q < 6; ++q) band_col_dot(io, r, H, q, c, s_cur, s[2 * q], s[2 * q + 1]);
      // slots: P0, P1 + i R1, P2 + i R2, H3, P2 - i R2, P1 - i R1
      Cin[c] = {(T)s[0], (T)s[1]};
      Cin[H + c] = {(T)(s[2] - s[5]), (T)(s[3] + s[4])};
      Cin[2 * H + c] = {(T)(s[6] - s[9]), (T)(s[7] + s[8])};
      Cin[3 * H + c] = {(T)s[10], (T)s[11]};
      Cin[4 * H + c] = {(T)(s[6] + s[9]), (T)(s[7] - s[8])};
      Cin[5 * H + c] = {(T)(s[2] + s[5]), (T)(s[3] - s[4])};
    }
  }
  __threadfence_block();
  __syncthreads();
  const int np = min(3, FftCfg<T>::ELEMS / N2);   // row pairs per LDS pass
  for (int p0 = 0; p0 < 3; p0 += np) {
    const int npp = min(np, 3 - p0);
    for (int idx = tid; idx < npp * N2; idx += NT) {
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
    lds_fft<T, false>(buf, N2, npp, N2, 1, tw2, true);
    for (int idx = tid; idx < npp * N2; idx += NT) {
      const int pr = p0 + idx / N2, t = idx % N2;
      U[(size_t)(2 * pr) * N2 + t] = buf[idx].x;
      U[(size_t)(2 * pr + 1) * N2 + t] = buf[idx].y;
    }
    __threadfence_block();
    __syncthreads();
  }
  // E u on the six rows, K_p u on the four output rows (wrap in both directions)
  for (int idx = tid; idx < 10 * N2; idx += NT) {
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
      const int o = q - 6;
      const int row = o < 2 ? o : N1 - 4 + o;
      const int s = row_slot(row, N1);
      const int sm = row_slot(row == 0 ? N1 - 1 : row - 1, N1), sp = row_slot(row == N1 - 1 ? 0 : row + 1, N1);
      const T v = U[(size_t)s * N2 + c];
      KP[(size_t)o * N2 + c] = k2 * v + (v - U[(size_t)s * N2 + cm]) + (v - U[(size_t)s * N2 + cp]) +
                               (v - U[(size_t)sm * N2 + c]) + (v - U[(size_t)sp * N2 + c]);
    }
  }
  __threadfence_block();
  __syncthreads();
  double acc = 0.0;
  for (int idx = tid; idx < 2 * N2; idx += NT) {
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
    acc += (double)U[(size_t)s * N2 + c] * (double)d;
  }
  __threadfence_block();
  const double uDu = block_sum<NT>(acc, red);
  if (tid == 0) pa[half] = uDu;
  for (int t = tid; t < N2; t += NT) buf[t] = {DU[t], DU[(size_t)N2 + t]};
  __syncthreads();
  lds_fft<T, false>(buf, N2, 1, N2, 1, tw2, false);
  C2<T>* PA = E + (size_t)(2 * half) * H;
  C2<T>* PB = PA + H;
  const T hh = (T)0.5;
  for (int c = tid; c < H; c += NT) {
    if (c == 0) {
      PA[0] = {buf[0].x, buf[H].x};
      PB[0] = {buf[0].y, buf[H].y};
    } else {
      const C2<T> zk = buf[c], zm = buf[N2 - c];
      PA[c] = {(zk.x + zm.x) * hh, (zk.y - zm.y) * hh};
      PB[c] = {(zk.y + zm.y) * hh, (zm.x - zk.x) * hh};
    }
  }
}

// On-chip version for 4 N1 <= E and 4 N2 <= E (E = complex values of the LDS FFT buffer): the
// boundary-row spectra, u on the six rows and D u on the block's two rows stay in LDS, D u is
// taken straight from u (E u and K_p u evaluated where needed), and the partial sums are loaded
// in batches.  Same arithmetic as k_band_global.
template <typename T, int ORDER>
struct BoundaryRows {
  // u on boundary slot s (rows {0, 1, 2, N1-3, N1-2, N1-1}) after the paired inverse FFTs
  const C2<T>* buf;
  int N1, N2;
  T k2;
  __device__ T U(int s, int c) const {
    const C2<T> z = buf[(s >> 1) * N2 + c];
    return (s & 1) ? z.y : z.x;
  }
  // (E u)(slot s, c): wrap-edge Laplacian
  __device__ T EU(int s, int c) const {
    const int row = slot_row(s, N1);
    const T v = U(s, c);
    T acc = (T)0;
    if (c == 0) acc += v - U(s, N2 - 1);
    if (c == N2 - 1) acc += v - U(s, 0);
    if (row == 0) acc += v - U(5, c);
    if (row == N1 - 1) acc += v - U(0, c);
    return acc;
  }
  // (K_p u)(output slot o, c), rows {0, 1, N1-2, N1-1}
  __device__ T KP(int o, int c) const {
    const int row = o < 2 ? o : N1 - 4 + o;
    const int sl = row_slot(row, N1);
    const int sm = row_slot(row == 0 ? N1 - 1 : row - 1, N1), sp = row_slot(row == N1 - 1 ? 0 : row + 1, N1);
    const int cm = c == 0 ? N2 - 1 : c - 1, cp = c == N2 - 1 ? 0 : c + 1;
    const T v = U(sl, c);
    return k2 * v + (v - U(sl, cm)) + (v - U(sl, cp)) + (v - U(sm, c)) + (v - U(sp, c));
  }
  // (D u)(output slot o, c)
  __device__ T DU(int o, int c, T tau) const {
    const int row = o < 2 ? o : N1 - 4 + o;
    const int sl = row_slot(row, N1);
    if (ORDER == 1) return tau * EU(sl, c);
    const T e = EU(sl, c);
    T kfe = k2 * e;
    if (c > 0) kfe += e - EU(sl, c - 1);
    if (c < N2 - 1) kfe += e - EU(sl, c + 1);
    if (row > 0) kfe += e - EU(row_slot(row - 1, N1), c);
    if (row < N1 - 1) kfe += e - EU(row_slot(row + 1, N1), c);
    const T kp = KP(o, c);
    T ekp = (T)0;
    if (c == 0) ekp += kp - KP(o, N2 - 1);
    if (c == N2 - 1) ekp += kp - KP(o, 0);
    if (row == 0) ekp += kp - KP(3, c);
    if (row == N1 - 1) ekp += kp - KP(0, c);
    return tau * (kfe + ekp);
  }
};

template <typename T, int ORDER>
__global__ __launch_bounds__(kFftThreads) void k_band_lds(int N1, int N2, const C2<T>* __restrict__ tw1,
                                                          const C2<T>* __restrict__ tw2, T k2, T tau, LzState S,
                                                          int j, int use_c, int periodic, StepIO<T> io) {
  constexpr int NT = kFftThreads;
  constexpr int EX = FftCfg<T>::ELEMS;
  constexpr int TWL = 3 * EX / 16;   // twiddles an N-point stage reads: indices below 3N/4, N <= EX/4
  __shared__ C2<T> buf[EX];
  __shared__ C2<T> aux[EX];
  __shared__ C2<T> tl1[TWL], tl2[TWL];
  __shared__ double red[3 * (NT / kWave)];   // lz_open_with takes three sets
  __shared__ int flag[1];
  const int r = blockIdx.y;
  const int tid = threadIdx.x;
  // FFT twiddles staged in LDS (every stage reads them)
  for (int i = tid; i < 3 * N1 / 4; i += NT) tl1[i] = tw1[i];
  for (int i = tid; i < 3 * N2 / 4; i += NT) tl2[i] = tw2[i];
  double s_cur;
  if (!band_open<NT>(S, r, j, use_c, red, flag, s_cur)) return;
  const int H = N2 / 2;
  double* pa = S.part_a + (size_t)r * S.pstride;
  C2<T>* E = io.etab + (size_t)r * 4 * H;
  C2<double>* Dt = io.dtab + (size_t)r * N1 * 2;
  if (periodic) {
    if (blockIdx.x < 2) {
      for (int i = tid; i < 2 * H; i += NT) E[(size_t)blockIdx.x * 2 * H + i] = {(T)0, (T)0};
    } else {
      for (int i = tid; i < 2 * N1; i += NT) Dt[i] = {0.0, 0.0};
    }
    if (tid == 0) pa[blockIdx.x] = 0.0;
    return;
  }
  if (blockIdx.x == 2) {
    // ---- interior ----
    const int RH = io.CT + 1;
    const double* gp = io.gpart + (size_t)r * N1 * RH * 8;
    for (int k1 = tid; k1 < N1; k1 += NT) {
      // the row's segments are contiguous: G_0, A, B, G_2 summed in segment order
      const double* g = gp + (size_t)k1 * RH * 8;
      double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 4
      for (int sg = 0; sg < RH; ++sg) {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] += g[sg * 8 + i];
      }
      buf[k1] = {(T)(a[0] * s_cur), (T)(a[1] * s_cur)};
      buf[N1 + k1] = {(T)((a[2] + a[5]) * s_cur), (T)((a[3] - a[4]) * s_cur)};   // A - i B
      buf[2 * N1 + k1] = {(T)(a[6] * s_cur), (T)(a[7] * s_cur)};
      buf[3 * N1 + k1] = {(T)((a[2] - a[5]) * s_cur), (T)((a[3] + a[4]) * s_cur)};   // A + i B
    }
    __syncthreads();
    lds_fft<T, false>(buf, N1, 4, N1, 1, tl1, true);
    // u(row, col_t) = Re buf[t N1 + row]
    auto ub = [&](int row, int t) { return (double)buf[t * N1 + row].x; };
    const double kk = (double)k2, tt = (double)tau;
    double acc = 0.0;
    for (int row = tid; row < N1; row += NT) {
      double d0 = 0.0, d1 = 0.0;
      if (row >= 2 && row < N1 - 2) {
        const double u0 = ub(row, 0), u1 = ub(row, 1), um2 = ub(row, 2), um1 = ub(row, 3);
        const double e = u0 - um1;
        if (ORDER == 1) {
          d0 = tt * e;
        } else {
          const double a0 = ub(row - 1, 0), a3 = ub(row - 1, 3), b0 = ub(row + 1, 0), b3 = ub(row + 1, 3);
          const double em = a0 - a3, ep = b0 - b3;
          const double kfe0 = kk * e + e + (e - em) + (e - ep);
          const double kp0 = kk * u0 + (u0 - u1) + (u0 - um1) + (u0 - a0) + (u0 - b0);
          const double kpm1 = kk * um1 + (um1 - um2) + (um1 - u0) + (um1 - a3) + (um1 - b3);
          d0 = tt * (kfe0 + kp0 - kpm1);
          d1 = -tt * e;
        }
        acc += d0 * (u0 - um1) + d1 * (u1 - um2);
      }
      aux[row] = {(T)d0, (T)d1};
    }
    const double uDu = block_sum<NT>(acc, red);
    if (tid == 0) pa[2] = uDu;
    lds_fft<T, false>(aux, N1, 1, N1, 1, tl1, false);
    for (int k = tid; k < N1; k += NT) {
      const C2<T> zk = aux[k], zm = aux[(N1 - k) & (N1 - 1)];
      Dt[2 * k] = {0.5 * ((double)zk.x + (double)zm.x), 0.5 * ((double)zk.y - (double)zm.y)};
      Dt[2 * k + 1] = {0.5 * ((double)zk.y + (double)zm.y), 0.5 * ((double)zm.x - (double)zk.x)};
    }
    return;
  }
  // ---- boundary rows ----
  const int half = blockIdx.x;
  C2<T>* hs = aux;                      // [6][H] raw column dots P0, P1, R1, P2, R2, H3
  T* du = (T*)(aux + 3 * N2);           // [2][N2]
  for (int idx = tid; idx < 6 * H; idx += NT) {
    double sx, sy;
    band_col_dot(io, r, H, idx / H, idx % H, s_cur, sx, sy);
    hs[idx] = {(T)sx, (T)sy};
  }
  __syncthreads();
  // packed row spectrum of u on slot s: P0, P1 + i R1, P2 + i R2, H3, P2 - i R2, P1 - i R1
  auto slot = [&](int sl, int c) -> C2<T> {
    switch (sl) {
      case 0: return hs[c];
      case 1: return {hs[H + c].x - hs[2 * H + c].y, hs[H + c].y + hs[2 * H + c].x};
      case 2: return {hs[3 * H + c].x - hs[4 * H + c].y, hs[3 * H + c].y + hs[4 * H + c].x};
      case 3: return hs[5 * H + c];
      case 4: return {hs[3 * H + c].x + hs[4 * H + c].y, hs[3 * H + c].y - hs[4 * H + c].x};
      default: return {hs[H + c].x + hs[2 * H + c].y, hs[H + c].y - hs[2 * H + c].x};
    }
  };
  for (int idx = tid; idx < 3 * N2; idx += NT) {
    const int pr = idx / N2, k = idx % N2;
    C2<T> a, b;
    if (k == 0) {
      a = {slot(2 * pr, 0).x, (T)0};
      b = {slot(2 * pr + 1, 0).x, (T)0};
    } else if (k == H) {
      a = {slot(2 * pr, 0).y, (T)0};
      b = {slot(2 * pr + 1, 0).y, (T)0};
    } else if (k < H) {
      a = slot(2 * pr, k);
      b = slot(2 * pr + 1, k);
    } else {
      const C2<T> pa2 = slot(2 * pr, N2 - k), pb2 = slot(2 * pr + 1, N2 - k);
      a = {pa2.x, -pa2.y};
      b = {pb2.x, -pb2.y};
    }
    buf[idx] = {a.x - b.y, a.y + b.x};
  }
  __syncthreads();
  lds_fft<T, false>(buf, N2, 3, N2, 1, tl2, true);
  const BoundaryRows<T, ORDER> br{buf, N1, N2, k2};
  double acc = 0.0;
  for (int idx = tid; idx < 2 * N2; idx += NT) {
    const int ol = idx / N2, c = idx % N2;
    const int o = 2 * half + ol;
    const int row = o < 2 ? o : N1 - 4 + o;
    const T d = br.DU(o, c, tau);
    du[idx] = d;
    acc += (double)br.U(row_slot(row, N1), c) * (double)d;
  }
  const double uDu = block_sum<NT>(acc, red);
  if (tid == 0) pa[half] = uDu;
  for (int t = tid; t < N2; t += NT) buf[t] = {du[t], du[N2 + t]};
  __syncthreads();
  lds_fft<T, false>(buf, N2, 1, N2, 1, tl2, false);
  C2<T>* PA = E + (size_t)(2 * half) * H;
  C2<T>* PB = PA + H;
  const T hh = (T)0.5;
  for (int c = tid; c < H; c += NT) {
    if (c == 0) {
      PA[0] = {buf[0].x, buf[H].x};
      PB[0] = {buf[0].y, buf[H].y};
    } else {
      const C2<T> zk = buf[c], zm = buf[N2 - c];
      PA[c] = {(zk.x + zm.x) * hh, (zk.y - zm.y) * hh};
      PB[c] = {(zk.y + zm.y) * hh, (zm.x - zk.x) * hh};
    }
  }
}

// ---- step kernel ----------------------------------------------------------------------------------------
// Per-lane coefficients of the closed form for packed column c >= 1.
struct CloseCoef {
  double Ax, Ay, Bx, By, E0x, E0y, S1x, S1y, T1x, T1y, F2x, F2y;
  template <typename T>
  __device__ __forceinline__ void init(const C2<double>* __restrict__ tw2, const C2<T>* __restrict__ E, int H, int c) {
    const C2<double> w1 = tw2[c], w2 = tw2[2 * c];
    Ax = 1.0 - w1.x;
    Ay = w1.y;
    Bx = w1.x - w2.x;
    By = w1.y + w2.y;
    const C2<T> e0 = E[c], e1 = E[H + c], em2 = E[2 * H + c], em1 = E[3 * H + c];
    E0x = (double)e0.x;
    E0y = (double)e0.y;
    S1x = (double)e1.x + (double)em1.x;
    S1y = (double)e1.y + (double)em1.y;
    // i (E_{N1-1} - E_1)
    T1x = (double)e1.y - (double)em1.y;
    T1y = (double)em1.x - (double)e1.x;
    F2x = (double)em2.x;
    F2y = (double)em2.y;
  }
  // Z(k1, c); sgn = -1 evaluates it at row -k1 (cos even, sin odd in k1)
  __device__ __forceinline__ void z(C2<double> D0, C2<double> D1, double c1, double s1, double c2, double s2,
                                    double& zx, double& zy) const {
    zx = Ax * D0.x - Ay * D0.y + Bx * D1.x - By * D1.y + E0x + c1 * S1x + s1 * T1x + c2 * F2x - s2 * F2y;
    zy = Ax * D0.y + Ay * D0.x + Bx * D1.y + By * D1.x + E0y + c1 * S1y + s1 * T1y + c2 * F2y + s2 * F2x;
  }
};

// Scalars of iteration j and alpha_j = ||v_j||^2 - <w_{j-1}, v_{j-1}> - n <u, D u> from the fixed-order
// partial sums (||v_j|| = 1 by construction), gathered by thread 0 into LDS (flag, sh[0..2]) in one round
// trip; block 0 stores alpha_j.  The caller issues its own loads before the barrier that publishes them.
__device__ __forceinline__ void step_scalars(const LzState& S, int r, int j, double n, int* flag, double* sh) {
  const double* pa = S.part_a + (size_t)r * S.pstride;
  const int act = S.active[r];
  const double bj = S.beta[lz_ib(S, r, j - 1)];
  const double bp = j > 1 ? S.beta[lz_ib(S, r, j - 2)] : 1.0;
  double band = 0.0;
  for (int i = 0; i < kBandBlocks; ++i) band += pa[i];
  const double a = 1.0 - pa[kBandBlocks] - n * band;
  flag[0] = act;
  sh[0] = a;
  sh[1] = bj;
  sh[2] = bp;
  if (act && blockIdx.x == 0) S.alpha[lz_ia(S, r, j)] = a;
}
// A value known to be the same on every lane, kept in scalar registers.
__device__ __forceinline__ double uniform_d(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ void step_read_scalars(int j, const double* sh, double& s_cur, double& s_prev,
                                                  double& bprev, double& alpha) {
  alpha = uniform_d(sh[0]);
  const double b1 = uniform_d(sh[1]), b2 = uniform_d(sh[2]);
  s_cur = 1.0 / b1;
  s_prev = j > 1 ? 1.0 / b2 : 0.0;
  bprev = j > 1 ? b1 : 0.0;
}

// Sum over the wave of two values: afterwards lanes 0..31 hold the total of a, lanes 32..63 that of b
// (v_permlane32_swap pairs the halves, v_permlane16_swap the rows, then a row mirror, a half-row
// mirror and two quad permutes; no LDS traffic).
__device__ __forceinline__ double wave_sum2(double a, double b) {
  swap32(a, b);
  double v = a + b;
  double u = v;
  swap16(v, u);
  v += u;
  v += dpp<kDppRowMirror>(v);
  v += dpp<kDppRowHalfMirror>(v);
  v += dpp<kDppQuadXor2>(v);
  v += dpp<kDppQuadXor1>(v);
  return v;
}

template <int NT>
__device__ __forceinline__ void step_norms(const LzState& S, int r, double nb, double nc, double* red) {
  const double sb = block_sum<NT>(nb, red);
  const double sc = block_sum<NT>(nc, red);
  if (threadIdx.x == 0) {
    S.part_b[(size_t)r * S.pstride + blockIdx.x] = sb;
    S.part_c[(size_t)r * S.pstride + blockIdx.x] = sc;
  }
}

// Column 0 of w_j over all rows (the extra block of each field).
template <typename T, int NT>
__device__ void step_col0(const C2<T>* __restrict__ vj, const C2<T>* __restrict__ vp, C2<T>* __restrict__ wo, int N1,
                          int H, const T* __restrict__ mult, const C2<double>* __restrict__ tw1,
                          const C2<T>* __restrict__ E, const C2<double>* __restrict__ Dt, int j, double s_cur,
                          double s_prev, double bprev, double alpha, double& nb, double& nc) {
  const int ms = mult_stride(H);
  // A_0 = 2i, B_0 = -2i carry X_{N2/2} = 2 (d0 - d1); the E terms of packed column 0
  const double E0x = (double)E[0].x, E0y = (double)E[0].y;
  const double S1x = (double)E[H].x + (double)E[3 * H].x, S1y = (double)E[H].y + (double)E[3 * H].y;
  const double T1x = (double)E[H].y - (double)E[3 * H].y, T1y = (double)E[3 * H].x - (double)E[H].x;
  const double F2x = (double)E[2 * H].x, F2y = (double)E[2 * H].y;
  auto zval = [&](C2<double> D0, C2<double> D1, double c1, double s1, double c2, double s2, double& zx, double& zy) {
    zx = -2.0 * D0.y + 2.0 * D1.y + E0x + c1 * S1x + s1 * T1x + c2 * F2x - s2 * F2y;
    zy = 2.0 * D0.x - 2.0 * D1.x + E0y + c1 * S1y + s1 * T1y + c2 * F2y + s2 * F2x;
  };
  for (int k1 = threadIdx.x; k1 < N1; k1 += NT) {
    const int kb = (N1 - k1) & (N1 - 1);
    const C2<double> t1 = tw1[k1], t2 = tw1[(2 * k1) & (N1 - 1)];
    const double c1 = t1.x, s1 = -t1.y, c2 = t2.x, s2 = -t2.y;
    double zx, zy, mx, my;
    zval(Dt[2 * k1], Dt[2 * k1 + 1], c1, s1, c2, s2, zx, zy);
    zval(Dt[2 * kb], Dt[2 * kb + 1], c1, -s1, c2, -s2, mx, my);
    const double m0 = (double)mult[(size_t)k1 * ms], mN = (double)mult[(size_t)k1 * ms + H];
    const double p = 0.5 * (m0 + mN), q = 0.5 * (m0 - mN);
    const double px = p * zx + q * mx, py = p * zy - q * my;
    const size_t gi = (size_t)k1 * H;
    const C2<T> x = vj[gi];
    const C2<T> xp = j > 1 ? vp[gi] : C2<T>{(T)0, (T)0};
    const double vx = rnd<T>((double)x.x * s_cur), vy = rnd<T>((double)x.y * s_cur);
    const double ux = rnd<T>((double)xp.x * s_prev), uy = rnd<T>((double)xp.y * s_prev);
    const C2<T> out = {(T)(vx - px - bprev * ux - alpha * vx), (T)(vy - py - bprev * uy - alpha * vy)};
    wo[gi] = out;
    nb += (double)out.x * (double)out.x + (double)out.y * (double)out.y;
    nc += (double)out.x * vx + (double)out.y * vy;
  }
}

// One Lanczos step in the spectral basis (grid: NB * CT + 1 blocks per field).  DOTS: also the dots of
// lambda^{-1/2} w_j / n for the next band kernel.
// lambda_M^{-1/2} of packed column c >= 1 at row k1, in registers: b = kappa2 + mu1(k1) + mu2(c),
// order 1: (tau b)^{-1/2}, order 2: tau^{-1/2} / b (hardware reciprocal and reciprocal square root, two
// Newton steps each).
struct MultEval {
  const double* mu1;
  double kappa2, tau, rtau;   // rtau = tau^{-1/2}
  int order;
  __device__ __forceinline__ double operator()(double mu2c, int k1) const { return eval(kappa2 + mu1[k1] + mu2c); }
  __device__ __forceinline__ double eval(double b) const {
    if (order == 2) {
      double y = __builtin_amdgcn_rcp(b);
      y = y * (2.0 - b * y);
      y = y * (2.0 - b * y);
      return rtau * y;
    }
    const double x = tau * b;
    double y = __builtin_amdgcn_rsq(x);
    y = y * (1.5 - 0.5 * x * y * y);
    y = y * (1.5 - 0.5 * x * y * y);
    return y;
  }
};

// Per-row values of a block's rows, staged in LDS once per block: cos/sin of theta, 2 theta, e^{-3 i theta}
// (theta = 2 pi k1 / N1), D0(k1), D1(k1) and mu1(k1).
constexpr int kRowTab = 12;
// s_waitcnt operand: vector memory count 0, export and LDS/scalar counts left at their maxima
constexpr int kWaitVm0 = (7 << 4) | (15 << 8);
enum { RT_C1 = 0, RT_S1, RT_C2, RT_S2, RT_T3X, RT_T3Y, RT_D0X, RT_D0Y, RT_D1X, RT_D1Y, RT_MU1 };

template <typename T, int LG, bool DOTS>
__global__ __launch_bounds__(kStepThreads, kStepWaves) void k_step(const C2<T>* __restrict__ Xj,
                                                                   const C2<T>* __restrict__ Xprev,
                                                                   C2<T>* __restrict__ W, int N1, int H,
                                                                   const T* __restrict__ mult, MultEval me,
                                                                   const double* __restrict__ mu2,
                                                                   const C2<double>* __restrict__ tw1,
                                                                   const C2<double>* __restrict__ tw2, LzState S,
                                                                   int j, double n, StepIO<T> io) {
  constexpr int NT = kStepThreads;
  constexpr int NW = NT / kWave;
  __shared__ double red[2 * NW];
  __shared__ int flag[1];
  __shared__ double sh[3];
  __shared__ __align__(16) double rowtab[kStepRows * kRowTab];
  __shared__ double xch[DOTS ? 12 * NT : 1];
  const int r = blockIdx.y;
  const SpecTile tl = spec_tile(N1, H, NT, kStepRows);
  const size_t fsz = (size_t)N1 * H;
  const C2<T>* vj = Xj + (size_t)r * fsz;
  const C2<T>* vp = Xprev + (size_t)r * fsz;
  C2<T>* wo = W + (size_t)r * fsz;
  const C2<T>* E = io.etab + (size_t)r * 4 * H;
  const C2<double>* Dt = io.dtab + (size_t)r * N1 * 2;
  double* gpart = io.gpart + (size_t)r * N1 * (tl.CT + 1) * 8;
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  double s_cur, s_prev, bprev, alpha;
  double nb = 0.0, nc = 0.0;
  if ((int)blockIdx.x == tl.NB * tl.CT) {
    if (tid == 0) step_scalars(S, r, j, n, flag, sh);
    __syncthreads();
    if (!flag[0]) return;
    step_read_scalars(j, sh, s_cur, s_prev, bprev, alpha);
    step_col0<T, NT>(vj, vp, wo, N1, H, mult, tw1, E, Dt, j, s_cur, s_prev, bprev, alpha, nb, nc);
    __threadfence_block();   // column 0 of w_j is read back by other threads of this block
    step_norms<NT>(S, r, nb, nc, red);
    if (DOTS) col0_dots<T, NT>(wo, N1, H, mult, 1.0 / n, tw1, gpart, tl.CT, io.c0dots + (size_t)r * 12, red);
    return;
  }
  const int rb = blockIdx.x / tl.CT, ct = blockIdx.x - rb * tl.CT;
  const int row0 = rb * tl.R;
  const int tlane = tid % LG, ro = tid / LG;
  const int c = ct * LG + tlane;
  const bool live = c != 0;   // column 0 belongs to the extra block
  const int cc = live ? c : 1;
  const int nsteps = ro < tl.R ? (tl.R - ro + tl.RPS - 1) / tl.RPS : 0;
  auto row_of = [&](int s) { return seg_uniform<LG>(row0 + ro + s * tl.RPS); };
  // Everything the block needs before its first row is requested at once, ahead of the one barrier:
  // the iteration scalars (thread 0), the per-row table (one thread per row), the per-column
  // coefficients and the first row of v_j and v_{j-1}.
  const C2<T> zero = {(T)0, (T)0};
  C2<T> xa = zero, xpa = zero, xb = zero, xpb = zero;
  if (nsteps > 0) {
    const int g0 = row_of(0) * H + cc;
    xa = stream_load(vj + g0);
    xpa = stream_load(vp + g0);
  }
  if (tid == 0) step_scalars(S, r, j, n, flag, sh);
  for (int i = tid - (NT - kWave); i >= 0 && i < tl.R; i += kWave) {
    // the last wave fills the table (thread 0's scalar gather runs in the first)
    const int k1 = row0 + i;
    const C2<double> t1 = tw1[k1], t2 = tw1[(2 * k1) & (N1 - 1)], t3 = tw1[(3 * k1) & (N1 - 1)];
    const C2<double> d0 = Dt[2 * k1], d1 = Dt[2 * k1 + 1];
    double* rt = rowtab + i * kRowTab;
    rt[RT_C1] = t1.x;
    rt[RT_S1] = -t1.y;
    rt[RT_C2] = t2.x;
    rt[RT_S2] = -t2.y;
    rt[RT_T3X] = t3.x;
    rt[RT_T3Y] = t3.y;
    rt[RT_D0X] = d0.x;
    rt[RT_D0Y] = d0.y;
    rt[RT_D1X] = d1.x;
    rt[RT_D1Y] = d1.y;
    rt[RT_MU1] = me.mu1[k1];
  }
  CloseCoef g;
  g.init<T>(tw2, E, H, cc);
  const double mu2c = mu2[cc];
  __syncthreads();
  if (!flag[0]) return;
  step_read_scalars(j, sh, s_cur, s_prev, bprev, alpha);
  const double inv_n = 1.0 / n;
  const double b0 = me.kappa2 + mu2c;   // kappa2 + mu2(c), per lane, formed before the loop
  double ca[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) ca[i] = 0.0;
  // Loads are issued unconditionally (row index clamped; at j = 1 Xprev is a valid vector whose value is
  // not used): the hardware wait counter is in order, and a load that some paths skip would make the
  // compiler wait for every load in flight.
  auto load_row = [&](int s, C2<T>& a, C2<T>& ap) {
    const int gi = row_of(min(s, nsteps - 1)) * H + cc;
    a = stream_load(vj + gi);
    ap = stream_load(vp + gi);
  };
  auto do_row = [&](int s, C2<T> x, C2<T> xp) {
    const int k1 = row_of(s);
    const double* rt = rowtab + (k1 - row0) * kRowTab;
    const C2<double> t1 = {rt[RT_C1], rt[RT_S1]}, t2 = {rt[RT_C2], rt[RT_S2]};
    const C2<double> D0 = {rt[RT_D0X], rt[RT_D0Y]}, D1 = {rt[RT_D1X], rt[RT_D1Y]};
    const double m = me.eval(b0 + rt[RT_MU1]);
    double zx, zy;
    g.z(D0, D1, t1.x, t1.y, t2.x, t2.y, zx, zy);
    const double vx = rnd<T>((double)x.x * s_cur), vy = rnd<T>((double)x.y * s_cur);
    const double ux = j > 1 ? rnd<T>((double)xp.x * s_prev) : 0.0;
    const double uy = j > 1 ? rnd<T>((double)xp.y * s_prev) : 0.0;
    const C2<T> out = {(T)(vx - m * zx - bprev * ux - alpha * vx), (T)(vy - m * zy - bprev * uy - alpha * vy)};
    if (live) {
      stream_store(wo + (k1 * H + cc), out);
      nb += 2.0 * ((double)out.x * (double)out.x + (double)out.y * (double)out.y);
      nc += 2.0 * ((double)out.x * vx + (double)out.y * vy);
    }
    if (DOTS) {
      const double f = live ? m * inv_n : 0.0;
      const double yx = f * (double)out.x, yy = f * (double)out.y;
      // band-column weights through the closed-form coefficients (w^c = 1 - conj A_c,
      // w^{2c} = w^c - conj(B_c - w^c)): with r0 = 2 y,
      //   2 Re w^c y = r0 - A_x r0,  2 Im w^c y = A_y r0,  2 w^{2c} y = (1 - A_x - B_x) r0 - i (B_y - A_y) r0
      const double r0 = 2.0 * yx, r1 = 2.0 * yy;
      const double r2 = r0 - g.Ax * r0, r3 = r1 - g.Ax * r1;
      const double r4 = g.Ay * r0, r5 = g.Ay * r1;
      const double r6 = r2 + r5 - g.Bx * r0 - g.By * r1;
      const double r7 = r3 - r4 - g.Bx * r1 + g.By * r0;
      ca[0] += yx;
      ca[1] += yy;
      ca[2] += t1.x * yx;
      ca[3] += t1.x * yy;
      ca[4] += t1.y * yx;
      ca[5] += t1.y * yy;
      ca[6] += t2.x * yx;
      ca[7] += t2.x * yy;
      ca[8] += t2.y * yx;
      ca[9] += t2.y * yy;
      const double t3x = rt[RT_T3X], t3y = rt[RT_T3Y];
      ca[10] += t3x * yx - t3y * yy;
      ca[11] += t3x * yy + t3y * yx;
      store_row_dots<LG>(gpart + ((k1 * (tl.CT + 1) + ct) * 8), lane, r0, r1, r2, r3, r4, r5, r6, r7);
    }
  };
  // Two register sets take turns (no copies between them), so that one row's loads are in flight while
  // the other row is computed.  The loads issued before the loop are drained first: the wait counter
  // is in order, and a wait for them inside the loop would also wait for the row in flight.
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  for (int s = 0; s < nsteps; s += 2) {
    load_row(s + 1, xb, xpb);
    do_row(s, xa, xpa);
    load_row(s + 2, xa, xpa);
    if (s + 1 < nsteps) do_row(s + 1, xb, xpb);
  }
  // Epilogue, one barrier: per-wave sums of ||w||^2 and <w, v_j>, and the column dots of every
  // (value, column) pair, combined below in fixed order.
  const double ws = wave_sum2(nb, nc);
  const int w = tid / kWave;
  if (lane == 0) red[2 * w] = ws;
  if (lane == 32) red[2 * w + 1] = ws;
  if (DOTS) {
#pragma unroll
    for (int i = 0; i < 12; ++i) xch[i * NT + tid] = ca[i];
  }
  __syncthreads();
  if (tid == 0) {
    double sb = 0.0, sc = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      sb += red[2 * i];
      sc += red[2 * i + 1];
    }
    S.part_b[(size_t)r * S.pstride + blockIdx.x] = sb;
    S.part_c[(size_t)r * S.pstride + blockIdx.x] = sc;
  }
  if (DOTS) {
    // slot q (P0, P1, R1, P2, R2, H3) of column ct * LG + t: values 2q and 2q + 1 summed over the row groups
    const int nro = min(tl.RPS, tl.R);
    C2<double>* cp = io.cpart + ((size_t)r * tl.NB + rb) * 6 * H;
    for (int pq = tid; pq < 6 * LG; pq += NT) {
      const int q = pq / LG, t = pq - q * LG;
      double sx = 0.0, sy = 0.0;
      for (int o = 0; o < nro; ++o) {
        sx += xch[(2 * q) * NT + o * LG + t];
        sy += xch[(2 * q + 1) * NT + o * LG + t];
      }
      cp[(size_t)q * H + ct * LG + t] = {sx, sy};
    }
  }
}

// ---- host side -----------------------------------------------------------------------------------------
PrecondStepCounts precond_step_counts(const FftPlan& p) {
  const SpecTile t = spec_tile(p.N1, p.H, kStepThreads, kStepRows);
  PrecondStepCounts c;
  c.Pband = kBandBlocks;
  c.Ps = t.NB * t.CT + 1;
  return c;
}

template <typename T>
static StepIO<T> step_io(const FftPlan& p, void* base, int k, size_t* total) {
  const SpecTile t = spec_tile(p.N1, p.H, kStepThreads, kStepRows);
  StepIO<T> io{};
  io.CT = t.CT;
  io.NB = t.NB;
  const size_t N1 = p.N1, H = p.H, N2 = p.N2, K = k;
  size_t off = 0;
  char* b = (char*)base;
  auto take = [&](size_t bytes) {
    char* q = b ? b + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return q;
  };
  io.gpart = (double*)take(K * N1 * (t.CT + 1) * 8 * sizeof(double));
  io.cpart = (C2<double>*)take(K * t.NB * 6 * H * sizeof(C2<double>));
  io.c0dots = (double*)take(K * 12 * sizeof(double));
  io.ub = (double*)take(K * N1 * 4 * sizeof(double));
  io.dtab = (C2<double>*)take(K * N1 * 2 * sizeof(C2<double>));
  io.etab = (C2<T>*)take(K * 4 * H * sizeof(C2<T>));
  io.hin = (C2<T>*)take(K * 2 * 6 * H * sizeof(C2<T>));
  io.work = (T*)take(K * 2 * 20 * N2 * sizeof(T));
  if (total) *total = off;
  return io;
}

size_t precond_step_bytes(const FftPlan& p, int storage, int k) {
  size_t total = 0;
  if (storage == GMRF_F64) step_io<double>(p, nullptr, k, &total);
  else step_io<float>(p, nullptr, k, &total);
  return total;
}

template <typename T> static const C2<T>* twT1(const FftPlan& p);
template <typename T> static const C2<T>* twT2(const FftPlan& p);
template <> const C2<double>* twT1<double>(const FftPlan& p) { return (const C2<double>*)p.tw64_1; }
template <> const C2<double>* twT2<double>(const FftPlan& p) { return (const C2<double>*)p.tw64_2; }
template <> const C2<float>* twT1<float>(const FftPlan& p) { return (const C2<float>*)p.tw32_1; }
template <> const C2<float>* twT2<float>(const FftPlan& p) { return (const C2<float>*)p.tw32_2; }

template <typename T, int LG>
static void launch_stream(const FftPlan& p, const StencilGeom& g, int order, const T* m, const T* X, const T* Xprev,
                          T* W, const StepIO<T>& io, const LzState& S, int j, int k, hipStream_t st, int kind) {
  const double n = (double)p.N1 * (double)p.N2;
  MultEval me{p.mu1, g.kappa2, g.tau, 1.0 / std::sqrt(g.tau), order};
  const C2<double>* t1 = (const C2<double>*)p.tw64_1;
  const C2<double>* t2 = (const C2<double>*)p.tw64_2;
  const dim3 grid(precond_step_counts(p).Ps, k);
  if (kind == 0)
    hipLaunchKernelGGL((k_dots<T, LG>), grid, dim3(kStepThreads), 0, st, (const C2<T>*)X, p.N1, p.H, m, 1.0 / n, t1,
                       t2, S, io);
  else if (kind == 1)
    hipLaunchKernelGGL((k_step<T, LG, true>), grid, dim3(kStepThreads), 0, st, (const C2<T>*)X, (const C2<T>*)Xprev,
                       (C2<T>*)W, p.N1, p.H, m, me, (const double*)p.mu2, t1, t2, S, j, n, io);
  else
    hipLaunchKernelGGL((k_step<T, LG, false>), grid, dim3(kStepThreads), 0, st, (const C2<T>*)X, (const C2<T>*)Xprev,
                       (C2<T>*)W, p.N1, p.H, m, me, (const double*)p.mu2, t1, t2, S, j, n, io);
}

// kind 0: dots of X; 1: step with dots; 2: step without dots
template <typename T>
static void stream(const FftPlan& p, const StencilGeom& g, int order, const T* m, const T* X, const T* Xprev, T* W,
                   const StepIO<T>& io, const LzState& S, int j, int k, hipStream_t st, int kind) {
  switch (spec_tile(p.N1, p.H, kStepThreads, 1).LG) {
    case 4: launch_stream<T, 4>(p, g, order, m, X, Xprev, W, io, S, j, k, st, kind); break;
    case 8: launch_stream<T, 8>(p, g, order, m, X, Xprev, W, io, S, j, k, st, kind); break;
    case 16: launch_stream<T, 16>(p, g, order, m, X, Xprev, W, io, S, j, k, st, kind); break;
    case 32: launch_stream<T, 32>(p, g, order, m, X, Xprev, W, io, S, j, k, st, kind); break;
    default: launch_stream<T, 64>(p, g, order, m, X, Xprev, W, io, S, j, k, st, kind); break;
  }
}

template <typename T>
void precond_dots(const FftPlan& p, const void* mult, const T* X, void* scratch, const LzState& S, int k,
                  hipStream_t st) {
  const StepIO<T> io = step_io<T>(p, scratch, k, nullptr);
  stream<T>(p, StencilGeom{}, 0, (const T*)mult, X, nullptr, nullptr, io, S, 0, k, st, 0);
}

template <typename T>
void precond_lanczos_step(const FftPlan& p, const StencilGeom& g, int order, const void* mult, const T* Xj,
                          const T* Xprev, T* W, void* scratch, const LzState& S, int j, int use_c, int dots, int k,
                          hipStream_t st, int only) {
  const StepIO<T> io = step_io<T>(p, scratch, k, nullptr);
  const T* m = (const T*)mult;
  if (only < 0 || only == 1) {
    const dim3 grid(kBandBlocks, k);
    constexpr int EX = FftCfg<T>::ELEMS;
    const bool onchip = 4 * p.N1 <= EX && 4 * p.N2 <= EX;
    const T k2 = (T)g.kappa2, tau = (T)g.tau;
    if (onchip && order == 1)
      hipLaunchKernelGGL((k_band_lds<T, 1>), grid, dim3(kFftThreads), 0, st, p.N1, p.N2, twT1<T>(p), twT2<T>(p), k2,
                         tau, S, j, use_c, g.periodic, io);
    else if (onchip)
      hipLaunchKernelGGL((k_band_lds<T, 2>), grid, dim3(kFftThreads), 0, st, p.N1, p.N2, twT1<T>(p), twT2<T>(p), k2,
                         tau, S, j, use_c, g.periodic, io);
    else if (order == 1)
      hipLaunchKernelGGL((k_band_global<T, 1>), grid, dim3(kFftThreads), 0, st, p.N1, p.N2, twT1<T>(p), twT2<T>(p),
                         k2, tau, S, j, use_c, g.periodic, io);
    else
      hipLaunchKernelGGL((k_band_global<T, 2>), grid, dim3(kFftThreads), 0, st, p.N1, p.N2, twT1<T>(p), twT2<T>(p),
                         k2, tau, S, j, use_c, g.periodic, io);
  }
  if (only < 0 || only == 2) stream<T>(p, g, order, m, Xj, Xprev, W, io, S, j, k, st, dots ? 1 : 2);
  if (only == 0) stream<T>(p, g, order, m, Xj, nullptr, nullptr, io, S, 0, k, st, 0);
}

#define INST(T)                                                                                                  \
  template void precond_dots<T>(const FftPlan&, const void*, const T*, void*, const LzState&, int, hipStream_t); \
  template void precond_lanczos_step<T>(const FftPlan&, const StencilGeom&, int, const void*, const T*, const T*, \
                                        T*, void*, const LzState&, int, int, int, int, hipStream_t, int);
INST(double)
INST(float)
#undef INST

}  // namespace gmrf
