// Preconditioned Lanczos step in the spectral basis (Proposition 1 with Algorithm 1, Section 5.1).
//
// The Krylov vectors are packed half spectra (fft.hpp) and the operator is
//     A_hat = I - Lambda^{-1/2} F D F^H Lambda^{-1/2},   D = M - Q,
// where D, the difference between the periodic and the free-boundary precision, is nonzero only
// within one point of the lattice boundary.  One step therefore needs
//   * u = F^H Lambda^{-1/2} v_j only at the four boundary columns {0, 1, N2-2, N2-1} of every row
//     and on the six boundary rows {0, 1, 2, N1-3, N1-2, N1-1};
//   * D u, supported on those columns and rows;
//   * Lambda^{-1/2} F D u, whose column transform is closed form in the D u coefficients,
// and no full 2D FFT is taken inside the loop.  Three launches per step:
//
// k_open  (streams slot j-1 once) opens iteration j (scalar step and stopping rule) and, with
//         Y = lambda^{-1/2} v_j / n, accumulates per spectral row k1 the dots
//         G_t(k1) = sum_c gamma_t(c) Y(k1, c), whose inverse DFT over k1 is u(., col_t), and per
//         packed column c the dots h_q(c) = sum_k1 e^{+2 pi i k1 r_q / N1} Y(k1, c), the packed
//         row spectra of u on the boundary rows r_q; plus ||v_j||^2.
// k_band  (small) block 2 of each field inverts the G_t (four length-N1 FFTs), forms the interior
//         coefficients (d0, d1) of D u and their DFTs D0, D1 over the rows; blocks 0 and 1
//         invert the boundary rows, form D u there (wrap and corner terms) and its packed row
//         spectra E_q.  Each block adds its share of <u, D u>.
// k_close (reads slots j-1 and j-2, writes slot j) evaluates the 2D spectrum of D u as
//         Z(k1, c) = A_c D0(k1) + B_c D1(k1) + sum_q e^{-2 pi i k1 r_q / N1} E_q(c),
//         A_c = 1 - conj w^c, B_c = w^c - conj w^{2c} (w = e^{-2 pi i / N2}), and writes
//         w_j = v_j - lambda^{-1/2} Z - alpha_j v_j - beta_{j-1} v_{j-1}
//         in one pass: alpha_j is known beforehand from
//         v_j^T A v_j = ||v_j||^2 - n <u, D u>  (Parseval),
//         minus <w_{j-1}, v_{j-1}> = beta_{j-1} v_j^T v_{j-1}, the term by which Algorithm 1's
//         alpha_j = v_j^T (A v_j - beta_{j-1} v_{j-1}) differs in floating point.  It leaves the
//         ||w_j||^2 and <w_j, v_j> partial sums for iteration j+1.
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

constexpr int kStepThreads = 512;   // opening and closing passes
constexpr int kStepWaves = 4;       // waves per SIMD asked of the compiler (two blocks per CU)
constexpr int kOpenRows = 64;       // spectral rows per opening block (column dots are partial per block)
constexpr int kCloseRows = 16;      // spectral rows per closing block
constexpr int kBandBlocks = 3;      // per field: top edge, bottom edge, interior

// Two packed columns per lane; a row segment of LG = min(H/2, 64) lanes (one wave when the row
// holds 128 columns or more) covers 2 LG columns.  A block of NT lanes covers one column tile of
// RPS = NT / LG rows at a time and `rows` rows in all; CT column tiles per row.
struct SpecTile {
  int LPR, LG, CT, RPS, R, NB;
};
__host__ __device__ inline SpecTile spec_tile(int N1, int H, int NT, int rows) {
  SpecTile t;
  t.LPR = H / 2;
  t.LG = t.LPR < kWave ? t.LPR : kWave;
  t.CT = t.LPR / t.LG;
  t.RPS = NT / t.LG;
  t.R = N1 < rows ? N1 : rows;
  t.NB = N1 / t.R;
  return t;
}

template <typename T>
struct StepIO {
  double* gpart;       // [k][N1][RH][8]  row dots G_0, A, B, G_2 (re, im) per row segment
  C2<double>* cpart;   // [k][NBo][6][H]  column dots P0, P1, R1, P2, R2, H3 per opening row block
  double* ub;          // [k][N1][4]      u at the boundary columns
  C2<double>* dtab;    // [k][N1][2]      D0(k1), D1(k1)
  C2<T>* etab;         // [k][4][H]       packed row spectra of D u on rows 0, 1, N1-2, N1-1
  C2<T>* hin;          // [k][2][6][H]    per edge block: packed row spectra of u on the boundary rows
  T* work;             // [k][2][20 N2]   per edge block: u (6 rows), E u (6), K_p u (4), D u (4)
  int RH, NBo;
};

template <typename T>
__device__ __forceinline__ double rnd(double v) { return (double)(T)v; }

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

// ---- opening pass ------------------------------------------------------------------------------------
template <typename T, int LG>
__global__ __launch_bounds__(kStepThreads, kStepWaves) void k_open(const C2<T>* __restrict__ X, int N1, int H,
                                                                   const T* __restrict__ mult, double scale,
                                                                   const C2<double>* __restrict__ tw1,
                                                                   const C2<double>* __restrict__ tw2, LzState S,
                                                                   int j, int use_c, int Po, StepIO<T> io) {
  constexpr int NT = kStepThreads;
  __shared__ double red[NT / kWave];
  __shared__ int flag[1];
  __shared__ double xch[NT * 8];
  const int r = blockIdx.y;
  double s_cur, s_prev, bprev;
  if (!lz_open<NT>(S, r, j, blockIdx.x == 0, red, flag, s_cur, s_prev, bprev)) return;
  double* pa = S.part_a + (size_t)r * S.pstride;
  if (blockIdx.x == 0) {
    // <w_{j-1}, v_{j-1}> from the previous closing pass
    const double c = (use_c && j > 1) ? sum_partials<NT>(S.part_c + (size_t)r * S.pstride, lz_pb(S, r), red) : 0.0;
    if (threadIdx.x == 0) pa[kBandBlocks + Po] = c;
  }
  const SpecTile tl = spec_tile(N1, H, NT, kOpenRows);
  const int rb = blockIdx.x / tl.CT, ct = blockIdx.x - rb * tl.CT;
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int tlane = tid % LG, ro = tid / LG;
  const int c0 = 2 * (ct * LG + tlane);
  const C2<T>* src = X + (size_t)r * N1 * H;
  // Band-column weights, as complex coefficients so that column 0 (X_0 + i X_{N2/2}) takes the same
  // arithmetic: G_0 += g0 Y, A += ga Y, B += gb Y, G_2 += g2 Y; G_1 = A - i B, G_3 = A + i B.
  //   c >= 1: g0 = 2, ga = 2 Re w^c, gb = 2 Im w^c, g2 = 2 w^{2c};  c = 0: g0 = g2 = 1 - i, ga = 1 + i, gb = 0.
  const bool col0 = (c0 == 0);
  double g0x, g0y, gax, gay, gbx, g2x0, g2y0;   // column c0
  double ga1, gb1, g2x1, g2y1;                  // column c0 + 1 (never 0)
  {
    const C2<double> w1 = tw2[c0], w2 = tw2[2 * c0];
    g0x = col0 ? 1.0 : 2.0;
    g0y = col0 ? -1.0 : 0.0;
    gax = col0 ? 1.0 : 2.0 * w1.x;
    gay = col0 ? 1.0 : 0.0;
    gbx = col0 ? 0.0 : 2.0 * w1.y;
    g2x0 = col0 ? 1.0 : 2.0 * w2.x;
    g2y0 = col0 ? -1.0 : 2.0 * w2.y;
    const C2<double> u1 = tw2[c0 + 1], u2 = tw2[2 * c0 + 2];
    ga1 = 2.0 * u1.x;
    gb1 = 2.0 * u1.y;
    g2x1 = 2.0 * u2.x;
    g2y1 = 2.0 * u2.y;
  }
  // column 0 couples k1 with -k1: Y = p v(k1) + q conj v(-k1), p = (m0 + mN) / 2, q = (m0 - mN) / 2;
  // other lanes read their own element again with q = 0
  const double wv0 = col0 ? 1.0 : 2.0;
  const double zq = col0 ? 1.0 : 0.0;
  const int moff = col0 ? H : c0;
  double ca[24];
#pragma unroll
  for (int i = 0; i < 24; ++i) ca[i] = 0.0;
  double vv = 0.0;
  const int nsteps = ro < tl.R ? (tl.R - ro + tl.RPS - 1) / tl.RPS : 0;
  for (int s = 0; s < nsteps; ++s) {
    const int k1 = seg_uniform<LG>(rb * tl.R + ro + s * tl.RPS);
    const int kb = (N1 - k1) & (N1 - 1);
    const C2<T>* rowp = src + (size_t)k1 * H + c0;
    const C2<T> x0 = rowp[0], x1 = rowp[1];
    const C2<T> xm = src[col0 ? (size_t)kb * H : (size_t)k1 * H + c0];
    const T* mrow = mult + (size_t)k1 * (H + 1);
    const double mA = (double)mrow[c0], mB = (double)mrow[moff], m1 = (double)mrow[c0 + 1] * scale;
    const double p = 0.5 * (mA + mB) * scale, q = 0.5 * (mA - mB) * scale * zq;
    const double v0x = rnd<T>((double)x0.x * s_cur), v0y = rnd<T>((double)x0.y * s_cur);
    const double v1x = rnd<T>((double)x1.x * s_cur), v1y = rnd<T>((double)x1.y * s_cur);
    const double vmx = rnd<T>((double)xm.x * s_cur), vmy = rnd<T>((double)xm.y * s_cur);
    vv += wv0 * (v0x * v0x + v0y * v0y) + 2.0 * (v1x * v1x + v1y * v1y);
    const double y0x = p * v0x + q * vmx, y0y = p * v0y - q * vmy;
    const double y1x = m1 * v1x, y1y = m1 * v1y;
    // row dots
    double r0 = 2.0 * y1x + g0x * y0x - g0y * y0y;
    double r1 = 2.0 * y1y + g0x * y0y + g0y * y0x;
    double r2 = ga1 * y1x + gax * y0x - gay * y0y;
    double r3 = ga1 * y1y + gax * y0y + gay * y0x;
    double r4 = gb1 * y1x + gbx * y0x;
    double r5 = gb1 * y1y + gbx * y0y;
    double r6 = g2x1 * y1x - g2y1 * y1y + g2x0 * y0x - g2y0 * y0y;
    double r7 = g2x1 * y1y + g2y1 * y1x + g2x0 * y0y + g2y0 * y0x;
    const int base = GroupReduce<LG>::run(r0, r1, r2, r3, r4, r5, r6, r7, lane);
    if ((lane & GroupReduce<LG>::LOW) == 0) {
      double* gp = io.gpart + (((size_t)r * N1 + k1) * tl.CT + ct) * 8 + base;
      constexpr int NV = GroupReduce<LG>::NV;
      gp[0] = r0;
      if constexpr (NV >= 2) gp[1] = r1;
      if constexpr (NV >= 4) {
        gp[2] = r2;
        gp[3] = r3;
      }
    }
    // column dots: e^{+i theta}, e^{+2 i theta} through cos/sin pairs, e^{-3 i theta} directly
    const C2<double> t1 = tw1[k1], t2 = tw1[(2 * k1) & (N1 - 1)], t3 = tw1[(3 * k1) & (N1 - 1)];
    const double c1 = t1.x, s1 = -t1.y, c2 = t2.x, s2 = -t2.y;
    const double yv[2][2] = {{y0x, y0y}, {y1x, y1y}};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const double yx = yv[e][0], yy = yv[e][1];
      double* a = ca + 12 * e;
      a[0] += yx;
      a[1] += yy;
      a[2] += c1 * yx;
      a[3] += c1 * yy;
      a[4] += s1 * yx;
      a[5] += s1 * yy;
      a[6] += c2 * yx;
      a[7] += c2 * yy;
      a[8] += s2 * yx;
      a[9] += s2 * yy;
      a[10] += t3.x * yx - t3.y * yy;
      a[11] += t3.x * yy + t3.y * yx;
    }
  }
  const double vsum = block_sum<NT>(vv, red);
  if (tid == 0) pa[kBandBlocks + blockIdx.x] = vsum;
  // column dots: lanes sharing a column pair (different ro) combine in ro order
  const int nro = min(tl.RPS, tl.R);
  double* cp = (double*)(io.cpart + ((size_t)r * io.NBo + rb) * 6 * H);
#pragma unroll
  for (int round = 0; round < 3; ++round) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) xch[tid * 8 + i] = ca[round * 8 + i];
    __syncthreads();
    if (ro == 0) {
      double sacc[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) sacc[i] = xch[tid * 8 + i];
      for (int o = 1; o < nro; ++o) {
#pragma unroll
        for (int i = 0; i < 8; ++i) sacc[i] += xch[(o * LG + tlane) * 8 + i];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int f = round * 8 + i, e = f / 12, qq = (f % 12) / 2, comp = f & 1;
        cp[((size_t)qq * H + c0 + e) * 2 + comp] = sacc[i];
      }
    }
  }
}

// ---- band kernel -------------------------------------------------------------------------------------
// Boundary-row slots 0..5 hold rows {0, 1, 2, N1-3, N1-2, N1-1}; output slots 0..3 rows {0, 1, N1-2, N1-1}.
__device__ __forceinline__ int slot_row(int s, int N1) { return s < 3 ? s : N1 - 6 + s; }
__device__ __forceinline__ int row_slot(int r, int N1) { return r <= 2 ? r : r - (N1 - 6); }

template <typename T, int ORDER>
__global__ __launch_bounds__(kFftThreads) void k_band(int N1, int N2, const C2<T>* __restrict__ tw1,
                                                      const C2<T>* __restrict__ tw2, T k2, T tau, LzState S,
                                                      int periodic, StepIO<T> io) {
  constexpr int NT = kFftThreads;
  __shared__ C2<T> buf[FftCfg<T>::ELEMS];
  __shared__ double red[NT / kWave];
  __shared__ int flag[1];
  const int r = blockIdx.y;
  if (!block_active(S, r, flag)) return;
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
    const int RH = io.RH;
    const double* gp = io.gpart + (size_t)r * N1 * RH * 8;
    double* ub = io.ub + (size_t)r * N1 * 4;
    const int nb = min(4, FftCfg<T>::ELEMS / N1);
    for (int t0 = 0; t0 < 4; t0 += nb) {
      const int nbb = min(nb, 4 - t0);
      for (int idx = tid; idx < nbb * N1; idx += NT) {
        const int t = t0 + idx / N1, k1 = idx % N1;
        const double* g = gp + (size_t)k1 * RH * 8;
        double gx = 0.0, gy = 0.0;
        if (t == 0 || t == 2) {
          const int o = t == 0 ? 0 : 6;
          for (int s = 0; s < RH; ++s) {
            gx += g[s * 8 + o];
            gy += g[s * 8 + o + 1];
          }
        } else {
          double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0;
          for (int s = 0; s < RH; ++s) {
            ax += g[s * 8 + 2];
            ay += g[s * 8 + 3];
            bx += g[s * 8 + 4];
            by += g[s * 8 + 5];
          }
          // t = 1: A - i B, t = 3: A + i B
          gx = t == 1 ? ax + by : ax - by;
          gy = t == 1 ? ay - bx : ay + bx;
        }
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
    const C2<double>* cp = io.cpart + (size_t)r * io.NBo * 6 * H;
    for (int c = tid; c < H; c += NT) {
      double s[12];
#pragma unroll
      for (int i = 0; i < 12; ++i) s[i] = 0.0;
      for (int b = 0; b < io.NBo; ++b) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const C2<double> v = cp[((size_t)b * 6 + q) * H + c];
          s[2 * q] += v.x;
          s[2 * q + 1] += v.y;
        }
      }
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

// ---- closing pass ------------------------------------------------------------------------------------
template <typename T, int LG>
__global__ __launch_bounds__(kStepThreads, kStepWaves) void k_close(const C2<T>* __restrict__ Xj,
                                                                    const C2<T>* __restrict__ Xprev,
                                                                    C2<T>* __restrict__ W, int N1, int H,
                                                                    const T* __restrict__ mult,
                                                                    const C2<double>* __restrict__ tw1,
                                                                    const C2<double>* __restrict__ tw2, LzState S,
                                                                    int j, int Po, double n, StepIO<T> io) {
  constexpr int NT = kStepThreads;
  __shared__ double red[NT / kWave];
  __shared__ int flag[1];
  __shared__ double alpha_sh[1];
  const int r = blockIdx.y;
  if (!block_active(S, r, flag)) return;
  const double bj = S.beta[lz_ib(S, r, j - 1)];
  const double s_cur = 1.0 / bj;
  const double s_prev = j > 1 ? 1.0 / S.beta[lz_ib(S, r, j - 2)] : 0.0;
  const double bprev = j > 1 ? bj : 0.0;
  if (threadIdx.x == 0) {
    // alpha_j = ||v_j||^2 - <w_{j-1}, v_{j-1}> - n <u, D u>, partial sums in fixed order
    const double* pa = S.part_a + (size_t)r * S.pstride;
    double vv = 0.0, band = 0.0;
    for (int i = 0; i < Po; ++i) vv += pa[kBandBlocks + i];
    for (int i = 0; i < kBandBlocks; ++i) band += pa[i];
    const double a = vv - pa[kBandBlocks + Po] - n * band;
    alpha_sh[0] = a;
    if (blockIdx.x == 0) S.alpha[lz_ia(S, r, j)] = a;
  }
  __syncthreads();
  const double alpha = alpha_sh[0];
  const SpecTile tl = spec_tile(N1, H, NT, kCloseRows);
  const int rb = blockIdx.x / tl.CT, ct = blockIdx.x - rb * tl.CT;
  const int tid = threadIdx.x;
  const int tlane = tid % LG, ro = tid / LG;
  const int c0 = 2 * (ct * LG + tlane);
  const bool col0 = (c0 == 0);
  // per-column coefficients of the closed form
  double Ax[2], Ay[2], Bx[2], By[2], E0x[2], E0y[2], S1x[2], S1y[2], T1x[2], T1y[2], F2x[2], F2y[2];
  const C2<T>* E = io.etab + (size_t)r * 4 * H;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int c = c0 + e;
    const C2<double> w1 = tw2[c], w2 = tw2[2 * c];
    const bool z = (c == 0);
    Ax[e] = z ? 0.0 : 1.0 - w1.x;
    Ay[e] = z ? 2.0 : w1.y;
    Bx[e] = z ? 0.0 : w1.x - w2.x;
    By[e] = z ? -2.0 : w1.y + w2.y;
    const C2<T> e0 = E[c], e1 = E[H + c], em2 = E[2 * H + c], em1 = E[3 * H + c];
    E0x[e] = (double)e0.x;
    E0y[e] = (double)e0.y;
    S1x[e] = (double)e1.x + (double)em1.x;
    S1y[e] = (double)e1.y + (double)em1.y;
    // i (E_{N1-1} - E_1)
    T1x[e] = (double)e1.y - (double)em1.y;
    T1y[e] = (double)em1.x - (double)e1.x;
    F2x[e] = (double)em2.x;
    F2y[e] = (double)em2.y;
  }
  const double wv0 = col0 ? 1.0 : 2.0;
  const double zq = col0 ? 1.0 : 0.0;
  const int moff = col0 ? H : c0;
  const C2<double>* Dt = io.dtab + (size_t)r * N1 * 2;
  const size_t fsz = (size_t)N1 * H;
  const C2<T>* vj = Xj + (size_t)r * fsz;
  const C2<T>* vp = Xprev + (size_t)r * fsz;
  C2<T>* wo = W + (size_t)r * fsz;
  double nb = 0.0, nc = 0.0;
  const int nsteps = ro < tl.R ? (tl.R - ro + tl.RPS - 1) / tl.RPS : 0;
#pragma unroll 2
  for (int s = 0; s < nsteps; ++s) {
    const int k1 = seg_uniform<LG>(rb * tl.R + ro + s * tl.RPS);
    const int kb = (N1 - k1) & (N1 - 1);
    const size_t gi = (size_t)k1 * H + c0;
    const C2<T> xa = vj[gi], xb = vj[gi + 1];
    C2<T> pa0 = {(T)0, (T)0}, pa1 = {(T)0, (T)0};
    if (j > 1) {
      pa0 = vp[gi];
      pa1 = vp[gi + 1];
    }
    const C2<double> D0 = Dt[2 * k1], D1 = Dt[2 * k1 + 1], M0 = Dt[2 * kb], M1 = Dt[2 * kb + 1];
    const C2<double> t1 = tw1[k1], t2 = tw1[(2 * k1) & (N1 - 1)];
    const double c1 = t1.x, s1 = -t1.y, c2 = t2.x, s2 = -t2.y;
    const T* mrow = mult + (size_t)k1 * (H + 1);
    const double mA = (double)mrow[c0], mB = (double)mrow[moff], m1 = (double)mrow[c0 + 1];
    double zx[2], zy[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      zx[e] = Ax[e] * D0.x - Ay[e] * D0.y + Bx[e] * D1.x - By[e] * D1.y + E0x[e] + c1 * S1x[e] + s1 * T1x[e] +
              c2 * F2x[e] - s2 * F2y[e];
      zy[e] = Ax[e] * D0.y + Ay[e] * D0.x + Bx[e] * D1.y + By[e] * D1.x + E0y[e] + c1 * S1y[e] + s1 * T1y[e] +
              c2 * F2y[e] + s2 * F2x[e];
    }
    // column 0 couples k1 with -k1: Z at the mirrored row (cos even, sin odd in k1), weight q = 0
    // on the other lanes
    const double mx = Ax[0] * M0.x - Ay[0] * M0.y + Bx[0] * M1.x - By[0] * M1.y + E0x[0] + c1 * S1x[0] -
                      s1 * T1x[0] + c2 * F2x[0] + s2 * F2y[0];
    const double my = Ax[0] * M0.y + Ay[0] * M0.x + Bx[0] * M1.y + By[0] * M1.x + E0y[0] + c1 * S1y[0] -
                      s1 * T1y[0] + c2 * F2y[0] - s2 * F2x[0];
    const double p = 0.5 * (mA + mB), q = 0.5 * (mA - mB) * zq;
    const double px[2] = {p * zx[0] + q * mx, m1 * zx[1]};
    const double py[2] = {p * zy[0] - q * my, m1 * zy[1]};
    const C2<T> xv[2] = {xa, xb}, xp[2] = {pa0, pa1};
    const double wgt[2] = {wv0, 2.0};
    C2<T> out[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const double vx = rnd<T>((double)xv[e].x * s_cur), vy = rnd<T>((double)xv[e].y * s_cur);
      const double ux = rnd<T>((double)xp[e].x * s_prev), uy = rnd<T>((double)xp[e].y * s_prev);
      const double qx = vx - px[e] - bprev * ux, qy = vy - py[e] - bprev * uy;
      out[e] = {(T)(qx - alpha * vx), (T)(qy - alpha * vy)};
      const double wx = (double)out[e].x, wy = (double)out[e].y;
      nb += wgt[e] * (wx * wx + wy * wy);
      nc += wgt[e] * (wx * vx + wy * vy);
    }
    wo[gi] = out[0];
    wo[gi + 1] = out[1];
  }
  const double sb = block_sum<NT>(nb, red);
  const double sc = block_sum<NT>(nc, red);
  if (tid == 0) {
    S.part_b[(size_t)r * S.pstride + blockIdx.x] = sb;
    S.part_c[(size_t)r * S.pstride + blockIdx.x] = sc;
  }
}

// ---- host side -----------------------------------------------------------------------------------------
PrecondStepCounts precond_step_counts(const FftPlan& p) {
  const SpecTile to = spec_tile(p.N1, p.H, kStepThreads, kOpenRows);
  const SpecTile tc = spec_tile(p.N1, p.H, kStepThreads, kCloseRows);
  PrecondStepCounts c;
  c.Pband = kBandBlocks;
  c.Po = to.NB * to.CT;
  c.Pc = tc.NB * tc.CT;
  return c;
}

template <typename T>
static StepIO<T> step_io(const FftPlan& p, void* base, int k, size_t* total) {
  const SpecTile to = spec_tile(p.N1, p.H, kStepThreads, kOpenRows);
  StepIO<T> io{};
  io.RH = to.CT;
  io.NBo = to.NB;
  const size_t N1 = p.N1, H = p.H, N2 = p.N2, K = k;
  size_t off = 0;
  char* b = (char*)base;
  auto take = [&](size_t bytes) {
    char* q = b ? b + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return q;
  };
  io.gpart = (double*)take(K * N1 * io.RH * 8 * sizeof(double));
  io.cpart = (C2<double>*)take(K * io.NBo * 6 * H * sizeof(C2<double>));
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
static void launch_open_close(const FftPlan& p, const T* m, const T* Xj, const T* Xprev, T* W, const StepIO<T>& io,
                              const PrecondStepCounts& cnt, const LzState& S, int j, int use_c, int k,
                              hipStream_t st, bool open) {
  const double n = (double)p.N1 * (double)p.N2;
  const C2<double>* t1 = (const C2<double>*)p.tw64_1;
  const C2<double>* t2 = (const C2<double>*)p.tw64_2;
  if (open)
    hipLaunchKernelGGL((k_open<T, LG>), dim3(cnt.Po, k), dim3(kStepThreads), 0, st, (const C2<T>*)Xj, p.N1, p.H, m,
                       1.0 / n, t1, t2, S, j, use_c, cnt.Po, io);
  else
    hipLaunchKernelGGL((k_close<T, LG>), dim3(cnt.Pc, k), dim3(kStepThreads), 0, st, (const C2<T>*)Xj,
                       (const C2<T>*)Xprev, (C2<T>*)W, p.N1, p.H, m, t1, t2, S, j, cnt.Po, n, io);
}

template <typename T>
static void open_close(const FftPlan& p, const T* m, const T* Xj, const T* Xprev, T* W, const StepIO<T>& io,
                       const PrecondStepCounts& cnt, const LzState& S, int j, int use_c, int k, hipStream_t st,
                       bool open) {
  switch (spec_tile(p.N1, p.H, kStepThreads, 1).LG) {
    case 2: launch_open_close<T, 2>(p, m, Xj, Xprev, W, io, cnt, S, j, use_c, k, st, open); break;
    case 4: launch_open_close<T, 4>(p, m, Xj, Xprev, W, io, cnt, S, j, use_c, k, st, open); break;
    case 8: launch_open_close<T, 8>(p, m, Xj, Xprev, W, io, cnt, S, j, use_c, k, st, open); break;
    case 16: launch_open_close<T, 16>(p, m, Xj, Xprev, W, io, cnt, S, j, use_c, k, st, open); break;
    case 32: launch_open_close<T, 32>(p, m, Xj, Xprev, W, io, cnt, S, j, use_c, k, st, open); break;
    default: launch_open_close<T, 64>(p, m, Xj, Xprev, W, io, cnt, S, j, use_c, k, st, open); break;
  }
}

template <typename T>
void precond_lanczos_step(const FftPlan& p, const StencilGeom& g, int order, const void* mult, const T* Xj,
                          const T* Xprev, T* W, void* scratch, const LzState& S, int j, int use_c, int k,
                          hipStream_t st, int only) {
  const StepIO<T> io = step_io<T>(p, scratch, k, nullptr);
  const PrecondStepCounts cnt = precond_step_counts(p);
  const T* m = (const T*)mult;
  if (only < 0 || only == 0) open_close<T>(p, m, Xj, Xprev, W, io, cnt, S, j, use_c, k, st, true);
  if (only < 0 || only == 1) {
    const dim3 grid(kBandBlocks, k);
    if (order == 1)
      hipLaunchKernelGGL((k_band<T, 1>), grid, dim3(kFftThreads), 0, st, p.N1, p.N2, twT1<T>(p), twT2<T>(p),
                         (T)g.kappa2, (T)g.tau, S, g.periodic, io);
    else
      hipLaunchKernelGGL((k_band<T, 2>), grid, dim3(kFftThreads), 0, st, p.N1, p.N2, twT1<T>(p), twT2<T>(p),
                         (T)g.kappa2, (T)g.tau, S, g.periodic, io);
  }
  if (only < 0 || only == 2) open_close<T>(p, m, Xj, Xprev, W, io, cnt, S, j, use_c, k, st, false);
}

template void precond_lanczos_step<double>(const FftPlan&, const StencilGeom&, int, const void*, const double*,
                                           const double*, double*, void*, const LzState&, int, int, int,
                                           hipStream_t, int);
template void precond_lanczos_step<float>(const FftPlan&, const StencilGeom&, int, const void*, const float*,
                                          const float*, float*, void*, const LzState&, int, int, int,
                                          hipStream_t, int);

}  // namespace gmrf
