// Shared device-side definitions of the gfx950 Krylov sampler: the Lanczos state, the
// deterministic reductions and the per-iteration scalar step of Algorithm 1.
//
// Vector layout: each right-hand side r owns one contiguous vector of L storage elements
// (a real lattice field, or a packed 2D half spectrum viewed as 2*N1*(N2/2) reals).  The
// Krylov basis keeps w_j = beta_j v_{j+1} unnormalised in slot j (slot 0 holds z), so
// v_{t+1} = V[t] / beta_t is formed on the fly by whichever kernel reads it: the division of
// Algorithm 1's normalisation step costs no pass over memory.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmrf {

enum : int { kOK = 0, kEINVAL = 1, kENOTSPD = 2, kENOCONV = 3 };

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kEwThreads = 256;  // elementwise kernels: threads per block
constexpr int kEwPerThread = 8;  // elements per thread
constexpr int kEwChunk = kEwThreads * kEwPerThread;  // elements per block

// Lattice geometry as a 3D box (n0, n1, n2), n2 contiguous; 1D/2D lattices have leading 1s.
struct StencilGeom {
  int n0, n1, n2;
  int periodic;
  double kappa2, tau;
  int tiles_x, tiles_y, tiles_z;
  int epl;                 // 2D operator kernel: elements per lane (1, 2, or 4 for FP32)
  int fepl;                // 2D one-pass Lanczos kernel: elements per lane (1 or 2)
  int ftiles_x;            // 2D one-pass Lanczos kernel: strips per row
  int band;                // 2D operator kernel: output rows per wave (0: kS2Band)
  int ftiles_y;            // 2D one-pass Lanczos kernel: bands of kS2Waves x s2f_band(order) rows
  int tune;                // launch options that leave every result bit unchanged (kTune* bits)
  int zc;                  // 3D first-order lattices: planes per z-march block (0: box tiles)
};

// Launch options chosen by the autotuner.  None of them changes what a thread computes or the order of
// any sum (partial sums are indexed by logical tile), so results are bitwise the same under every choice.
enum : int {
  kTuneXcd = 1,   // XCD-contiguous tile order: workgroup i runs on XCD i mod 8, each XCD takes one range
  kTuneNtStore = 2,   // non-temporal stores of the kernel's output vector (selects a kernel instantiation)
  // the operator kernel alone (Y = Q X, no partial sums): its tile shape, which changes no output bit either,
  // since every output point's terms and their order are the same in every tiling
  kTuneBandShift = 2,     // 2 bits: rows per wave 0 = the lattice's rule, 1 = 8, 2 = 16, 3 = 32
  kTuneEplShift = 4,      // 2 bits: columns per lane 0 = the lattice's rule, 1 = 1, 2 = 2, 3 = 4 (FP32)
  kTuneGeomMask = 0x3C,
};

// Per-call Lanczos state, all device memory.  Index conventions (1-based j as in
// Algorithm 1): alpha[r*(m_max+1) + j] = alpha_j, beta[r*(m_max+2) + j] = beta_j with
// beta_0 = ||z||, dpiv[r*(m_max+1) + j] = d_j (LDL^T pivot of T_j), rho[..+ j] = rho_j.
struct LzState {
  int k;
  int m_max;
  double tol;           // <= 0: run exactly m_max steps
  double* alpha;
  double* beta;
  double* dpiv;
  double* rho;
  int* m_used;
  int* status;
  int* active;
  double* part_a;       // [k][pstride] partial sums of v_j^T q (op kernels)
  double* part_b;       // [k][pstride] partial sums of ||w||^2 (elementwise kernels)
  double* part_c;       // [k][pstride] partial sums of <w, v_j> (preconditioned closing pass)
  int Pa;               // number of partials the op kernel writes per RHS
  int Pb;               // number of partials the elementwise kernels write per RHS
  int pstride;
  int weighted;         // 1: packed half-spectrum inner product (column 0 weight 1, else 2)
  int H;                // packed columns per spectral row (weighted mode)
  // Uneven batches (many fields in one launch): per-column tables, all nullptr otherwise.
  const int64_t* col_off;         // offset of column r inside a slot (default r * L)
  const int64_t* col_ext;         // offset of column r in the caller's Z and X (default col_off)
  const int* col_len;             // length of column r (default L)
  const int* col_pa;              // op-kernel partials of column r (default Pa)
  const int* col_pb;              // elementwise partials of column r (default Pb)
  const StencilGeom* col_geom;    // lattice of column r (default: the kernel's geometry)
  int64_t slot_stride;            // elements per Krylov slot (default k * L)
  // One-pass 2D step over an uneven batch: block b works on column work[b].x, tile work[b].y (the
  // tiles of the columns still running; nullptr: column blockIdx.y, tile blockIdx.x).
  const int2* work;
};

__device__ __forceinline__ size_t lz_off(const LzState& S, int r, long L) {
  return S.col_off ? (size_t)S.col_off[r] : (size_t)r * (size_t)L;
}
__device__ __forceinline__ long lz_len(const LzState& S, int r, long L) { return S.col_len ? (long)S.col_len[r] : L; }
__device__ __forceinline__ int lz_pa(const LzState& S, int r) { return S.col_pa ? S.col_pa[r] : S.Pa; }
__device__ __forceinline__ int lz_pb(const LzState& S, int r) { return S.col_pb ? S.col_pb[r] : S.Pb; }
__device__ __forceinline__ size_t lz_slot(const LzState& S, long L) {
  return S.slot_stride ? (size_t)S.slot_stride : (size_t)S.k * (size_t)L;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
  return v;
}

// gfx950 cross-lane exchanges of doubles.  swap32(a, b): v_permlane32_swap on both halves, after which a lane's
// a + b is the sum over its pair of lanes 32 apart of a (lanes 0..31) or of b (lanes 32..63); swap16 likewise
// per 16-lane row with v_permlane16_swap (even rows: a, odd rows: b).  dpp<CTRL>: a DPP lane permutation.
__device__ __forceinline__ void swap32(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
  a = __hiloint2double((int)hi[0], (int)lo[0]);
  b = __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ void swap16(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
  a = __hiloint2double((int)hi[0], (int)lo[0]);
  b = __hiloint2double((int)hi[1], (int)lo[1]);
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
constexpr int kDppRowMirror = 0x140, kDppRowHalfMirror = 0x141, kDppQuadXor2 = 0x4E, kDppQuadXor1 = 0xB1;

// Sum over the wave of 16 values per lane with no lane-dependent selects: afterwards every lane of 16-lane
// row q (q = lane / 16) holds in v[i], i < 4, the total of value 4 q + i (v_permlane32_swap pairs the
// halves, v_permlane16_swap the rows, then a row mirror, a half-row mirror and two quad permutes).
__device__ __forceinline__ void wave_sum16(double (&v)[16]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    swap32(v[i], v[i + 8]);
    v[i] += v[i + 8];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    swap16(v[i], v[i + 4]);
    v[i] += v[i + 4];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] += dpp<kDppRowMirror>(v[i]);
    v[i] += dpp<kDppRowHalfMirror>(v[i]);
    v[i] += dpp<kDppQuadXor2>(v[i]);
    v[i] += dpp<kDppQuadXor1>(v[i]);
  }
}

// Value of v on lane l (l uniform), for every lane.
__device__ __forceinline__ double lane_read(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Sum over the block; every thread receives the same value.  Fixed association order
// (butterfly inside a wave, then waves in index order), hence bitwise reproducible.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* lds) {
  constexpr int NW = NT / kWave;
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += lds[i];
  return s;
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double* lds) {
  constexpr int NW = NT / kWave;
  v = wave_max(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
  __syncthreads();
  double s = lds[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) s = fmax(s, lds[i]);
  return s;
}

// Sum of P partials in fixed order: thread t adds p[t], p[t+NT], ... then block_sum.
template <int NT>
__device__ __forceinline__ double sum_partials(const double* p, int P, double* lds) {
  double s = 0.0;
  for (int i = threadIdx.x; i < P; i += NT) s += p[i];
  return block_sum<NT>(s, lds);
}

__device__ __forceinline__ int lz_ia(const LzState& S, int r, int j) { return r * (S.m_max + 1) + j; }
__device__ __forceinline__ int lz_ib(const LzState& S, int r, int j) { return r * (S.m_max + 2) + j; }

// Block-uniform read of active[r]: the opener's writer block may clear it while other
// blocks of the same launch read it, so one thread reads and broadcasts through LDS.
__device__ __forceinline__ bool block_active(const LzState& S, int r, int* lds_flag) {
  __syncthreads();
  if (threadIdx.x == 0) lds_flag[0] = S.active[r];
  __syncthreads();
  return lds_flag[0] != 0;
}

// The loads of the scalar step for column r, all issued before any wait: active[r] (by one thread, broadcast
// with the partial sums' block reduction), this thread's share of the ||w_{j-1}||^2 partials (summed in
// sum_partials' order), and the scalars of iteration j-1, which no block of this launch writes.
struct LzOpenIn {
  int act0;
  double ps, a, bm1, dm1, rm1;
};
template <int NT>
__device__ __forceinline__ LzOpenIn lz_open_load(const LzState& S, int r, int j) {
  LzOpenIn o;
  const int tid = (int)threadIdx.x;
  o.act0 = (tid == 0) ? S.active[r] : 0;
  o.a = 0.0;
  o.bm1 = 0.0;
  o.dm1 = 1.0;
  o.rm1 = 1.0;
  if (j >= 2) {
    const int jm = j - 1;
    o.a = S.alpha[lz_ia(S, r, jm)];
    o.bm1 = S.beta[lz_ib(S, r, jm - 1)];
    o.rm1 = S.rho[lz_ia(S, r, jm - 1)];
    if (jm >= 2) o.dm1 = S.dpiv[lz_ia(S, r, jm - 1)];
  }
  const double* pb = S.part_b + (size_t)r * S.pstride;
  const int P = lz_pb(S, r);
  o.ps = 0.0;
  for (int i = tid; i < P; i += NT) o.ps += pb[i];
  return o;
}

// The decision of the scalar step from beta_{j-1}^2 = bsq and the loaded scalars (see lz_open).
__device__ __forceinline__ bool lz_decide(const LzState& S, int r, int j, bool writer, double bsq, const LzOpenIn& o,
                                          double& s_cur, double& s_prev, double& bprev) {
  const double b = sqrt(bsq);
  if (j == 1) {
    bool ok = (b > 0.0) && isfinite(b);
    if (writer) {
      S.beta[lz_ib(S, r, 0)] = b;
      S.rho[lz_ia(S, r, 0)] = 1.0;
      if (!ok) {
        S.m_used[r] = 0;
        S.status[r] = (b == 0.0) ? kOK : kEINVAL;
        S.active[r] = 0;
      }
    }
    s_cur = ok ? 1.0 / b : 0.0;
    s_prev = 0.0;
    bprev = 0.0;
    return ok;
  }
  const int jm = j - 1;                        // iteration being closed
  const double a = o.a;
  const double bpp = (jm >= 2) ? o.bm1 : 0.0;   // beta_{j-2}
  const double d = (jm == 1) ? a : a - bpp * bpp / o.dm1;
  const double rh = o.rm1 * b / d;
  int st = kOK;
  bool stop = false;
  if (!(a > 0.0) || !(d > 0.0) || !isfinite(b)) {
    st = kENOTSPD;
    stop = true;
  } else if (b <= 64.0 * 2.220446049250313e-16 * (fabs(a) + bpp) || (S.tol > 0.0 && rh <= S.tol)) {
    stop = true;
  } else if (j > S.m_max) {
    stop = true;
    st = (S.tol > 0.0) ? kENOCONV : kOK;
  }
  if (writer) {
    S.beta[lz_ib(S, r, jm)] = b;
    S.dpiv[lz_ia(S, r, jm)] = d;
    S.rho[lz_ia(S, r, jm)] = rh;
    if (stop) {
      S.m_used[r] = jm;
      S.status[r] = st;
      S.active[r] = 0;
    }
  }
  if (stop) return false;
  s_cur = 1.0 / b;
  s_prev = 1.0 / o.bm1;
  bprev = b;
  return true;
}

// Scalar step that opens iteration j for RHS r (Algorithm 1 with the Theorem 1 stopping
// quantity).  Every block working on RHS r calls it with identical inputs and so reaches
// the same decision; only `writer` stores it.  For j >= 2 it finishes iteration j-1:
//   beta_{j-1} = ||w_{j-1}|| from the partial sums, d_{j-1} = alpha_{j-1} - beta_{j-2}^2/d_{j-2},
//   rho_{j-1} = rho_{j-2} beta_{j-1} / d_{j-1}; stop on non-positive alpha or pivot
//   (not SPD), on breakdown beta_{j-1} <= 64 eps (|alpha_{j-1}| + beta_{j-2}), or on
//   rho_{j-1} <= tol.  For j = 1 it forms beta_0 = ||z|| (zero z: x = 0 with m = 0;
//   non-finite z: EINVAL).  With j = m_max + 1 it also closes a run that hit m_max.
// On continuation it returns s_cur = 1/beta_{j-1} (scale of slot j-1, giving v_j),
// s_prev = 1/beta_{j-2} (slot j-2, giving v_{j-1}) and bprev = beta_{j-1}.
template <int NT>
__device__ bool lz_open(const LzState& S, int r, int j, bool writer, double* lds, int* lds_flag,
                        double& s_cur, double& s_prev, double& bprev) {
  constexpr int NW = NT / kWave;
  const int tid = (int)threadIdx.x;
  const LzOpenIn o = lz_open_load<NT>(S, r, j);
  const double ps = wave_sum(o.ps);
  __syncthreads();
  if ((tid & (kWave - 1)) == 0) lds[tid / kWave] = ps;
  if (tid == 0) lds_flag[0] = o.act0;
  __syncthreads();
  if (!lds_flag[0]) return false;
  double bsq = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) bsq += lds[i];
  return lz_decide(S, r, j, writer, bsq, o, s_cur, s_prev, bprev);
}

// lz_open plus the sums of up to two more partial sets of column r (pa: Pa values, pc: Pc values; nullptr:
// 0), in sum_partials' order, all loaded before the first wait and reduced under the same two barriers.
// lds: 3 * NT / 64 doubles.
template <int NT>
__device__ bool lz_open_with(const LzState& S, int r, int j, bool writer, double* lds, int* lds_flag,
                             const double* pa, int Pa, const double* pc, int Pc, double& s_cur, double& s_prev,
                             double& bprev, double& qa, double& qc) {
  constexpr int NW = NT / kWave;
  const int tid = (int)threadIdx.x;
  const LzOpenIn o = lz_open_load<NT>(S, r, j);
  double sa = 0.0, sc = 0.0;
  if (pa)
    for (int i = tid; i < Pa; i += NT) sa += pa[i];
  if (pc)
    for (int i = tid; i < Pc; i += NT) sc += pc[i];
  const double ps = wave_sum(o.ps);
  sa = wave_sum(sa);
  sc = wave_sum(sc);
  __syncthreads();
  if ((tid & (kWave - 1)) == 0) {
    lds[tid / kWave] = ps;
    lds[NW + tid / kWave] = sa;
    lds[2 * NW + tid / kWave] = sc;
  }
  if (tid == 0) lds_flag[0] = o.act0;
  __syncthreads();
  if (!lds_flag[0]) return false;
  double bsq = 0.0;
  qa = 0.0;
  qc = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    bsq += lds[i];
    qa += lds[NW + i];
    qc += lds[2 * NW + i];
  }
  return lz_decide(S, r, j, writer, bsq, o, s_cur, s_prev, bprev);
}

// The update step's scalars of column r at step j, loaded together: active[r] (one thread, broadcast),
// alpha_j = the sum of the operator's Pa partials (sum_partials' order) and beta_{j-1}.  lds: NT / 64
// doubles.  Returns false for a column that has stopped.
template <int NT>
__device__ bool lz_update_scalars(const LzState& S, int r, int j, double* lds, int* lds_flag, double& a,
                                  double& bj1) {
  constexpr int NW = NT / kWave;
  const int tid = (int)threadIdx.x;
  const int act0 = (tid == 0) ? S.active[r] : 0;
  bj1 = S.beta[lz_ib(S, r, j - 1)];
  const double* pa = S.part_a + (size_t)r * S.pstride;
  const int Pa = lz_pa(S, r);
  double sa = 0.0;
  for (int i = tid; i < Pa; i += NT) sa += pa[i];
  sa = wave_sum(sa);
  __syncthreads();
  if ((tid & (kWave - 1)) == 0) lds[tid / kWave] = sa;
  if (tid == 0) lds_flag[0] = act0;
  __syncthreads();
  if (!lds_flag[0]) return false;
  a = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) a += lds[i];
  return true;
}

// lz_open for the KB columns r0 .. r0 + KB - 1 (those below k) of one block at once: every column's loads
// are issued before the first wait and the reductions share two barriers.  lds: KB * NT / 64 doubles,
// lds_flag: KB ints.  act[c] is true on return where column r0 + c continues.
template <int NT, int KB>
__device__ void lz_open_multi(const LzState& S, int r0, int k, int j, bool writer, double* lds, int* lds_flag,
                              bool (&act)[KB], double (&s_cur)[KB], double (&s_prev)[KB], double (&bprev)[KB]) {
  constexpr int NW = NT / kWave;
  const int tid = (int)threadIdx.x;
  LzOpenIn o[KB];
#pragma unroll
  for (int c = 0; c < KB; ++c) o[c] = lz_open_load<NT>(S, min(r0 + c, k - 1), j);
  __syncthreads();
#pragma unroll
  for (int c = 0; c < KB; ++c) {
    const double ps = wave_sum(o[c].ps);
    if ((tid & (kWave - 1)) == 0) lds[c * NW + tid / kWave] = ps;
    if (tid == 0) lds_flag[c] = (r0 + c < k) ? o[c].act0 : 0;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < KB; ++c) {
    act[c] = lds_flag[c] != 0;
    if (!act[c]) continue;
    double bsq = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) bsq += lds[c * NW + i];
    act[c] = lz_decide(S, r0 + c, j, writer, bsq, o[c], s_cur[c], s_prev[c], bprev[c]);
  }
}

// Inner-product weight of storage element e (real index) of a vector.
__device__ __forceinline__ double ip_weight(const LzState& S, long e) {
  if (!S.weighted) return 1.0;
  const long c = (e >> 1) % S.H;
  return c == 0 ? 1.0 : 2.0;
}

}  // namespace gmrf
