// Incomplete-Cholesky preconditioning (Section 5.2): host factorisation (ichol.cpp) and the GPU
// level-scheduled triangular solves and step opener (ichol_step.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "common.hpp"

namespace gmrf {

// Host result of the factorisation: L = strictly lower part + diag, by rows (lrp, lci, lva) and L^T's
// strictly upper part by rows (urp, uci, uva); level sets of the forward and backward solves.
struct IcholHost {
  int64_t n = 0;
  double shift = 0.0;       // diagonal shift the factorisation needed (0 if none)
  double logdet_M = 0.0;    // log det (L L^T) = 2 sum log l_ii
  std::vector<double> diag;
  std::vector<int64_t> lrp, urp;
  std::vector<int32_t> lci, uci;
  std::vector<double> lva, uva;
  std::vector<int32_t> flev_ptr, flev_rows, blev_ptr, blev_rows;
};

// false: breakdown at every shift of the sequence.  Q: symmetric CSR (host).
bool ichol_factor(int64_t n, const int64_t* rp, const int32_t* ci, const double* va, double droptol, IcholHost& out);

// One triangular solve on the device, stored in level order: position p (levels are the ranges
// lvl_ptr[l] .. lvl_ptr[l+1]) holds row rows[p], its strictly-triangular entries rp[p] .. rp[p+1] of
// (ci, va) (column = original row index) and dinv[p] = 1 / l_ii; values in the storage dtype.
struct TrsvDev {
  int32_t* lvl_ptr = nullptr;
  int32_t* rows = nullptr;
  int64_t* rp = nullptr;
  int32_t* ci = nullptr;
  void* va = nullptr;
  void* dinv = nullptr;
  int nlev = 0;
  int64_t nnz = 0;      // strictly-triangular entries
  int max_row = 0;      // most strictly-triangular entries in one row
  int max_width = 0;    // most rows in one level
};
struct IcholDev {
  TrsvDev fwd, bwd;     // L y = b, L^T x = y
  int64_t n = 0;
};

// X[:, r] = L^{-1} B[:, r] (lower) or L^{-T} B[:, r] (upper) for the k columns with active[r] != 0
// (active may be null: all columns); X and B distinct.
template <typename T, typename OutT>
void launch_trsv(const IcholDev& f, bool upper, const T* B, long bld, OutT* X, long xld, const int* active, int k,
                 hipStream_t st);
// Opens iteration j (beta_{j-1}, stopping rule) and writes q = AX / beta_{j-1} - beta_{j-1} v_{j-1} with
// v_{j-1} = Xprev / beta_{j-2}, and the partial sums of v_j^T q (v_j = Xj / beta_{j-1}) for the update
// kernel; AX = L^{-1} Q L^{-T} Xj.  Elementwise tiling (ew_blocks(L) partials per column).
template <typename T>
void launch_pre_lz(const T* AX, const T* Xj, const T* Xprev, T* Qb, long L, const LzState& S, int j, hipStream_t st);

}  // namespace gmrf
