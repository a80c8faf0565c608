// Internal launcher declarations shared by the kernel translation units and the host
// runtime (gmrf_api.cpp).  Not part of the public C ABI (include/gmrf.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace gmrf {

// lanczos_kernels.hip
int ew_blocks(long L);
int rademacher_blocks(long n);
template <typename T> void launch_init_from_f64(const double* Z, long zld, long L, T* V0, const LzState& S, hipStream_t st);
template <typename T> void launch_init_from_i8(const int8_t* P, long L, T* V0, const LzState& S, hipStream_t st);
// column q = p0 + r of V0 <- probe q / K restricted to colour class q mod K (colour NULL, K = 1: probe q)
template <typename T> void launch_init_rademacher(uint64_t seed, long n, int p0, T* V0, const LzState& S, hipStream_t st,
                                                  const int32_t* colour = nullptr, int K = 1);
void launch_rademacher_i8(uint64_t seed, long n, int nprobes, int8_t* out, hipStream_t st);
template <typename T> void launch_update(const T* Qb, const T* Vj, T* W, long L, int j, int with_norm, const LzState& S, hipStream_t st);
void launch_hutchinson_aggregate(const double* g, const double* beta, int ldb, int np, int K, double shift, double* out, hipStream_t st);
void launch_finalize(const LzState& S, hipStream_t st);
// out[r] = active[r], out[k + r] = rho_{j-1} of column r (2 k doubles, device)
void launch_poll_gather(const LzState& S, int j, double* out, hipStream_t st);
template <typename T> void launch_norm_partials(const T* V0, long L, const LzState& S, hipStream_t st);
// norm partials per column the reorthogonalisation's last pass writes (vectors of L elements)
int reorth_blocks(long L);
// Qb != nullptr: the reorthogonalisation also does the update step before it (w_j = q - alpha_j v_j into
// slot j, alpha_j), where reorth_takes_update(L); the caller then launches no update kernel
bool reorth_takes_update(long L);
// sets of [k][hstride][reorth_blocks(L)] partials part_h must hold (the short-vector form keeps the two
// passes' dots apart; h is then unused)
int reorth_partial_sets(long L);
template <typename T> void launch_reorth(T* V, long L, int j, double* part_h, double* h, int hstride, const LzState& S, hipStream_t st, const T* Qb = nullptr);
// out (+)= beta_0 y_t v_{t+1} from slot t (t = 0 writes); S: the state of the pass that produced y
template <typename T, typename OutT> void launch_accumulate(const T* Vt, long L, const double* y, int ldy, const LzState& S, int t, OutT* out, long old, hipStream_t st);
template <typename T, typename OutT> void launch_combine(const T* V, long L, const double* y, int ldy, OutT* out, long old, const LzState& S, hipStream_t st);

// operator_kernels.hip
// epl: elements per lane of the 2D operator kernel (0: the widest the row length allows for vbytes-byte
// storage, 4 for FP32 and 2 for FP64; 1 for fields at arbitrary offsets); the one-pass kernel takes at
// most 2
void stencil_geom_tiles(StencilGeom& g, int dim, int order, int epl = 0, int vbytes = 8);
// One-pass Lanczos step on a 2D lattice (k_lanczos2d): mode 0 reads v_j = X / beta_{j-1} and v_{j-1} = Xprev
// (S holds the previous pass's partial sums), writes w_j to W and this pass's partial sums to out_*; mode 1
// writes the partial sums of X^T Q X to out_a.  grid_x = 0: the lattice's own block count.
int lanczos2d_blocks(const StencilGeom& g);
template <typename T>
void launch_lanczos2d(const StencilGeom& g, int order, int mode, int grid_x, const T* X, long xld, T* W,
                      const T* Xprev, const LzState& S, int j, int k, double* out_a, double* out_b, double* out_c,
                      hipStream_t st);
int stencil_blocks(const StencilGeom& g);
void stencil_geom_shape(StencilGeom& g, int order, int band, int epl);
template <typename T> void launch_stencil(const StencilGeom& g, int order, int dim, bool lz, const T* X, long xld, T* Y, long yld, const T* Xprev, const LzState& S, int j, int k, hipStream_t st);
template <typename T> void launch_stencil_batch(int order, int dim, int max_tiles, const T* X, T* Y, const T* Xprev, const LzState& S, int j, hipStream_t st, bool zmarch);
int csr_blocks(long n);
template <typename T> void launch_csr(long n, const int64_t* rp, const int32_t* ci, const T* va, bool lz, const T* X, long xld, T* Y, long yld, const T* Xprev, const LzState& S, int j, int k, hipStream_t st);

// lgcp_step.hip: Y += diag(d) X for k columns of length n (the diagonal term of Q + diag(d))
template <typename T> void launch_add_diag(const T* d, const T* X, T* Y, long n, int k, hipStream_t st);

// tridiag_kernels.hip
int tri_max_m();
size_t tri_scratch_doubles(int k, int m_cap);
void launch_tri_invsqrt(const double* alpha, int lda, int a_off, const double* beta, int ldb, int b_off,
                        const int* m, int m_fixed, const int* status_in, double* y, int ldy,
                        int* status_out, double* scratch, int scr_m, int k, hipStream_t st);
// y = T^{-1} e_1 (the linear solve's tridiagonal step); status_out[r] = ENOTSPD when T is not SPD
void launch_tri_solve(const double* alpha, int lda, int a_off, const double* beta, int ldb, int b_off, const int* m,
                      int m_fixed, const int* status_in, double* y, int ldy, int* status_out, int k, hipStream_t st);
void launch_tri_log(const double* alpha, int lda, int a_off, const double* beta, int ldb, int b_off,
                    const int* m, int m_fixed, const int* status_in, double* out, int ldo,
                    int* status_out, int k, hipStream_t st);

// bandwidth.hip: which 0 read of a, 1 copy a -> b, 2 triad a = b + q c; n4 = 16-byte elements per array
void launch_bandwidth(int which, int blocks, void* a, void* b, void* c, float* out, size_t n4, hipStream_t st);

}  // namespace gmrf
