// 2D FFT machinery for the block-circulant preconditioner of Proposition 1 (Section 5.1):
// M = periodic version of the lattice precision, applied as M^{-1/2} v = F^H lambda_M^{-1/2} F v.
//
// Spectral Lanczos.  F is the unitary 2D DFT.  Since A = M^{-1/2} Q M^{-1/2} is real symmetric,
// running Algorithm 1 on A_hat = F A F^H from z_hat = F z produces the same alpha_j, beta_j and
// u_m = F^H u_hat_m (inner products are preserved by a unitary map).  With the Krylov vectors
// held in the spectral basis, each step applies
//     A_hat v_hat = Lambda^{-1/2} F Q F^H Lambda^{-1/2} v_hat
// i.e. one inverse and one forward 2D FFT around the stencil: two FFTs per step instead of the
// four of the real-space formulation (Section 5.1 counts four), and x = F^H Lambda^{-1/2} u_hat_m.
//
// Packed half spectrum of a real N1 x N2 field (N2 even): per row, columns c = 1..N2/2-1 hold the
// row-DFT coefficients, column 0 holds X[0] + i X[N2/2] (both real for a real row); the column
// FFT then acts on all N2/2 packed columns alike.  Unitary inner products become
//     <a, b> = sum_{c = 0} Re(conj a b) + 2 sum_{c >= 1} Re(conj a b),
// and the diagonal multiplier couples k1 with -k1 in column 0 only.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "../../include/gmrf.h"
#include "common.hpp"
#include "kernels.hpp"

namespace gmrf {

struct FftPlan {
  int N1 = 0, N2 = 0, H = 0;
  double* tw64_1 = nullptr;   // e^{-2 pi i k / N1}, k < N1 (interleaved re, im)
  double* tw64_2 = nullptr;   // e^{-2 pi i k / N2}, k < N2
  float* tw32_1 = nullptr;
  float* tw32_2 = nullptr;
  double* mu1 = nullptr;      // 4 sin^2(pi min(k, N1-k) / N1), k < N1: eigenvalues of the periodic second difference
  double* mu2 = nullptr;      // same for N2
};

// mu(k) of the periodic second difference on N points, evaluated at min(k, N - k) so that mu(k) = mu(N - k)
// exactly (shared by the multiplier table and the kernels that evaluate the multiplier in registers).
inline double periodic_mu(int k, int N) {
  const double s = std::sin(M_PI * (double)std::min(k, N - k) / N);
  return 4.0 * s * s;
}

// lambda_M^{-1/2} table, [N1][mult_stride(H)]: entries 0..H-1 for packed columns (column 0 -> k2 = 0),
// entry H -> k2 = N2/2, entry H+1 padding so that every row starts on a 16-byte boundary.
__host__ __device__ constexpr int mult_stride(int H) { return H + 2; }

gmrf_status fft_plan_create(FftPlan& p, int N1, int N2);
void fft_plan_destroy(FftPlan& p);

// Y = M^{-1/2} X for k real fields (storage T); tmp holds k packed spectra.
template <typename T>
void fft_apply_inv_sqrt_M(const FftPlan& p, const T* mult, const T* X, T* Y, T* tmp, int k, hipStream_t st);

// slot 0 <- F z (unitary, packed), partial sums of ||z_hat||^2 (ew tiling) into S.part_b.
template <typename T>
void fft_forward_init(const FftPlan& p, const double* Z, T* V0, T* tmp, const LzState& S, int k, hipStream_t st);

// slot 0 <- Lambda^{-1/2} F b (the spectral start vector of a preconditioned solve), with its norm partials.
template <typename T>
void fft_forward_init_mult(const FftPlan& p, const void* mult, const double* B, T* V0, T* tmp, const LzState& S, int k,
                           hipStream_t st);

// same for Rademacher probe columns p0 .. p0 + k - 1 (from seed, or from an int8 block when probes != nullptr;
// with a colouring, column q is probe q / K restricted to class q mod K).
template <typename T>
void fft_forward_init_probes(const FftPlan& p, uint64_t seed, int p0, const int8_t* probes, T* real_tmp, T* V0,
                             T* tmp, const LzState& S, int k, hipStream_t st, const int32_t* colour = nullptr,
                             int K = 1);

// Preconditioned Lanczos step (precond_step.hip).  Opens iteration j (beta_{j-1} from the partial
// sums, stopping rule), applies A_hat = I - Lambda^{-1/2} F D F^H Lambda^{-1/2} to v_j = Xj / beta_{j-1}
// and writes w_j = A_hat v_j - alpha_j v_j - beta_{j-1} v_{j-1} to W with its partial sums.  The
// boundary values of u = F^H Lambda^{-1/2} v_j come from dot products of v_j left in scratch by the
// previous step (dots = 1) or by precond_dots (slot 0; a w_j changed by reorthogonalisation, after
// which use_c = 0 because its <w, v> partials are stale).
// scratch: precond_step_bytes(p, storage, k) bytes.  only = -1 runs the band and the step kernels;
// 1 the band kernel, 2 the step kernel, 0 the dots kernel on Xj (timing).
struct PrecondStepCounts {
  int Pband;   // <u, D u> partials per field (part_a[0..Pband)), then <w_{j-1}, v_{j-1}> at part_a[Pband]
  int Ps;      // step blocks per field: ||w_j||^2 and <w_j, v_j> partials (part_b, part_c)
};
PrecondStepCounts precond_step_counts(const FftPlan& p);
size_t precond_step_bytes(const FftPlan& p, int storage, int k);
template <typename T>
void precond_lanczos_step(const FftPlan& p, const StencilGeom& g, int order, const void* mult, const T* Xj,
                          const T* Xprev, T* W, void* scratch, const LzState& S, int j, int use_c, int dots, int k,
                          hipStream_t st, int only = -1);
template <typename T>
void precond_dots(const FftPlan& p, const void* mult, const T* X, void* scratch, const LzState& S, int k,
                  hipStream_t st);

// Preconditioned step for Q + diag(H) with M = Q on a periodic lattice (lgcp_step.hip): a row pass
// (opens iteration j; y = F^H Lambda^{-1/2} v_j, y^T H y partial sums in part_a[0..Pr), <w_{j-1}, v_{j-1}>
// at part_a[Pr]; row transforms of H y into T2) and a column pass (w_j into W with its ||w||^2 and
// <w, v_j> partials over Pc blocks; T1 <- column-inverse transform of Lambda^{-1/2} w_j).  T1 must hold
// that transform of slot j - 1 on entry (lgcp_col_init for slot 0 and after a reorthogonalisation, which
// also sets use_c = 0).  d: the diagonal H (n values, storage dtype).  only = 1: row pass, 2: column pass.
struct LgcpCounts {
  int Pr;   // row-pass blocks per field
  int Pc;   // column-pass blocks per field
};
LgcpCounts lgcp_counts(const FftPlan& p, int storage);
template <typename T>
void lgcp_col_init(const FftPlan& p, const void* mult, const T* X, T* T1, int k, hipStream_t st);
template <typename T>
void lgcp_lanczos_step(const FftPlan& p, const void* mult, const T* d, T* T1, T* T2, const T* Xj, const T* Xprev,
                       T* W, const LzState& S, int j, int use_c, int k, hipStream_t st, int only = 0);

// X (FP64, real, n x k) = F^H Lambda^{-1/2} U_hat for the combined spectral vectors U_hat.
template <typename T>
void fft_backward_output(const FftPlan& p, const void* mult, const T* U, double* X, T* tmp, const LzState& S,
                         int k, hipStream_t st);

}  // namespace gmrf
