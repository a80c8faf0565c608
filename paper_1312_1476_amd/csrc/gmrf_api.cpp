// Host runtime behind include/gmrf.h: operator handles, the device scratch pool with its
// HBM budget, and the host-driven Lanczos loop that enqueues the gfx950 kernels.
//
// One iteration j of Algorithm 1 is two launches on the caller's stream (plus six for full
// reorthogonalisation): the operator kernel opens the iteration (scalar step of the previous
// one, stop decision), applies Q and fuses q -= beta v_{j-1} with the alpha partials; the
// update kernel forms w_j = q - alpha_j v_j and the ||w_j||^2 partials.  The host only polls
// the per-column `active` flags every few iterations, so the GPU never idles on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/gmrf.h"
#include "fft.hpp"
#include "ichol.hpp"
#include "kernels.hpp"

using namespace gmrf;

// ---- errors ----------------------------------------------------------------------------------
static thread_local std::string g_last_error;

static gmrf_status fail(gmrf_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(GMRF_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ---- device check --------------------------------------------------------------------------------
static gmrf_status check_device() {
  int dev = 0, count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
    return fail(GMRF_EDEVICE, "no HIP device available");
  if (hipGetDevice(&dev) != hipSuccess) return fail(GMRF_EDEVICE, "hipGetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(GMRF_EDEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(GMRF_EDEVICE, "device %d is %s; this library is built for gfx950 only", dev, prop.gcnArchName);
  return GMRF_OK;
}

// ---- scratch pool ---------------------------------------------------------------------------------
// Calls take their scratch from here in blocks rounded to 2 MiB.  By default a block comes from a cache of
// freed blocks (a cached block at most 25% larger than asked is reused) or from hipMalloc.  Device
// allocation and release are slow and irregular on this part when memory has been used before (seconds
// for some 100 GB requests, and hipFree waits for the whole device), so a server with a varied mix of
// request sizes reserves one region up front (gmrf_pool_reserve): blocks are then carved from it (large
// ones best fit from the bottom, small ones from the top) in an address-ordered list of free ranges that
// merges neighbours when a block comes back, and the pool calls into the device allocator no more.
namespace {
using Clock = std::chrono::steady_clock;

constexpr size_t kPoolSmallBlock = (size_t)64 << 20;   // region blocks up to this size come from the top

struct Pool {
  std::mutex mu;
  std::multimap<size_t, void*> free_blocks;
  size_t in_use = 0;
  size_t cached = 0;
  size_t budget = 0;
  char* region = nullptr;
  size_t region_size = 0;
  std::map<size_t, size_t> holes;     // free ranges of the region: offset -> length
  uint64_t n_alloc = 0, n_free = 0;
  double t_alloc = 0.0, t_free = 0.0;

  hipError_t dev_alloc(void** p, size_t bytes) {
    const auto t0 = Clock::now();
    const hipError_t e = hipMalloc(p, bytes);
    t_alloc += std::chrono::duration<double>(Clock::now() - t0).count();
    ++n_alloc;
    return e;
  }
  void dev_free(void* p) {
    const auto t0 = Clock::now();
    (void)hipFree(p);
    t_free += std::chrono::duration<double>(Clock::now() - t0).count();
    ++n_free;
  }
  void drop_cache() {
    for (auto& kv : free_blocks) dev_free(kv.second);
    free_blocks.clear();
    cached = 0;
  }
  size_t largest_hole() const {
    size_t b = 0;
    for (auto& h : holes) b = std::max(b, h.second);
    return b;
  }
  bool region_idle() const { return holes.size() == 1 && holes.begin()->second == region_size; }

  gmrf_status get(size_t bytes, void** out, size_t* actual) {
    bytes = rounded(bytes);
    std::lock_guard<std::mutex> lk(mu);
    if (budget && in_use + bytes > budget)
      return fail(GMRF_ENOMEM, "HBM budget %zu B exceeded (in use %zu B, request %zu B)", budget, in_use, bytes);
    if (region) {
      // small blocks (scalars, partial sums, one-vector buffers) from the top end of the highest range that
      // holds them, large ones (Krylov bases) best fit from the bottom: the small blocks of running calls
      // then do not split the ranges that the next large basis needs
      const bool small = bytes <= kPoolSmallBlock;
      auto pick = holes.end();
      for (auto it = holes.begin(); it != holes.end(); ++it) {
        if (it->second < bytes) continue;
        if (small) pick = it;                                             // the last fitting range: highest
        else if (pick == holes.end() || it->second < pick->second) pick = it;
      }
      if (pick == holes.end())
        return fail(GMRF_ENOMEM, "reserved region of %zu B has no free range of %zu B (largest %zu B)", region_size,
                    bytes, largest_hole());
      const size_t off = pick->first, len = pick->second;
      holes.erase(pick);
      size_t at = off;
      if (small) {
        at = off + len - bytes;
        if (len > bytes) holes.emplace(off, len - bytes);
      } else if (len > bytes) {
        holes.emplace(off + bytes, len - bytes);
      }
      *out = region + at;
      *actual = bytes;
      in_use += bytes;
      return GMRF_OK;
    }
    auto it = free_blocks.lower_bound(bytes);
    if (it != free_blocks.end() && it->first <= bytes + bytes / 4) {
      *out = it->second;
      *actual = it->first;
      in_use += it->first;
      cached -= it->first;
      free_blocks.erase(it);
      return GMRF_OK;
    }
    // cached blocks count against the budget: release them before allocating fresh memory
    if (budget && in_use + cached + bytes > budget) drop_cache();
    void* p = nullptr;
    if (dev_alloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      drop_cache();
      if (dev_alloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GMRF_ENOMEM, "hipMalloc of %zu B failed", bytes);
      }
    }
    *out = p;
    *actual = bytes;
    in_use += bytes;
    return GMRF_OK;
  }
  static size_t rounded(size_t bytes) { return (bytes + (2u << 20) - 1) & ~((size_t)(2u << 20) - 1); }
  // `bytes` is the size the block was handed out with
  void put(void* p, size_t bytes) {
    std::lock_guard<std::mutex> lk(mu);
    in_use -= std::min(in_use, bytes);
    char* c = static_cast<char*>(p);
    if (region && c >= region && c < region + region_size) {
      size_t off = (size_t)(c - region), len = bytes;
      auto nx = holes.lower_bound(off);
      if (nx != holes.end() && off + len == nx->first) {
        len += nx->second;
        nx = holes.erase(nx);
      }
      if (nx != holes.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
          pv->second += len;
          return;
        }
      }
      holes.emplace(off, len);
      return;
    }
    free_blocks.emplace(bytes, p);
    cached += bytes;
  }
};
Pool& pool() {
  static Pool* p = new Pool();
  return *p;
}

// Scratch of one call; returned to the pool (after the stream has drained) on destruction.  With an arena
// (a caller-provided device range) the call's buffers are carved from it in order instead, 256-byte
// aligned, and nothing is allocated or returned.
struct Workspace {
  hipStream_t stream;
  std::vector<std::pair<void*, size_t>> blocks;
  char* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  explicit Workspace(hipStream_t s) : stream(s) {}
  Workspace(hipStream_t s, void* base, size_t cap) : stream(s), arena(static_cast<char*>(base)), arena_cap(cap) {}
  ~Workspace() {
    if (!blocks.empty()) (void)hipStreamSynchronize(stream);
    for (auto& b : blocks) pool().put(b.first, b.second);
  }
  template <typename T>
  gmrf_status alloc(size_t count, T** out) {
    if (arena) {
      const size_t b = (std::max<size_t>(count * sizeof(T), 256) + 255) & ~(size_t)255;
      if (b > arena_cap - arena_used)
        return fail(GMRF_ENOMEM, "the call needs more than the %zu B of static scratch (%zu B used, %zu B more asked)",
                    arena_cap, arena_used, b);
      *out = reinterpret_cast<T*>(arena + arena_used);
      arena_used += b;
      return GMRF_OK;
    }
    void* p = nullptr;
    size_t actual = 0;
    gmrf_status s = pool().get(std::max<size_t>(count * sizeof(T), 256), &p, &actual);
    if (s != GMRF_OK) return s;
    blocks.emplace_back(p, actual);
    *out = static_cast<T*>(p);
    return GMRF_OK;
  }
};
}  // namespace

void free_ichol(gmrf::IcholDev& f);

// ---- operator handle -------------------------------------------------------------------------------
struct gmrf_op {
  int kind = 0;           // 0 lattice, 1 csr
  int ndim = 0;
  int64_t shape[3] = {1, 1, 1};
  int order = 1;
  double kappa2 = 0.0, tau = 1.0;
  int bc = GMRF_FREE;
  int storage = GMRF_F64;
  int64_t n = 0;
  StencilGeom geom{};
  int dim = 1;
  // CSR (device; the pattern is also kept on the host for the distance colouring)
  std::vector<int64_t> h_rp;
  std::vector<int32_t> h_ci;
  std::vector<double> h_va;
  // incomplete-Cholesky preconditioner (CSR handles)
  int ic = 0;
  IcholDev icd{};
  double ic_logdet = 0.0;     // log det (L L^T)
  double ic_shift = 0.0;
  int64_t ic_nnz = 0;
  int64_t* rp = nullptr;
  int32_t* ci = nullptr;
  void* va = nullptr;
  int64_t nnz = 0;
  // circulant preconditioner
  int precond = 0;
  FftPlan plan{};
  double logdet_M = 0.0;
  double* mult64 = nullptr;  // lambda_M^{-1/2} tables (device)
  float* mult32 = nullptr;
  // diagonal term: Q + diag(d) (device, both storage dtypes)
  int has_diag = 0;
  double* diag64 = nullptr;
  float* diag32 = nullptr;
  size_t resident_bytes = 0;
};

extern "C" {

const char* gmrf_last_error(void) { return g_last_error.c_str(); }

const char* gmrf_strerror(gmrf_status s) {
  switch (s) {
    case GMRF_OK: return "ok";
    case GMRF_EINVAL: return "invalid argument";
    case GMRF_ENOTSPD: return "operator is not symmetric positive definite";
    case GMRF_ENOCONV: return "tolerance not reached within m_max steps";
    case GMRF_ENOMEM: return "out of device memory or over the HBM budget";
    case GMRF_EDEVICE: return "no usable gfx950 device or HIP runtime error";
    case GMRF_EUNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

gmrf_status gmrf_set_hbm_budget(size_t bytes) {
  std::lock_guard<std::mutex> lk(pool().mu);
  pool().budget = bytes;
  // cached free blocks go back to the device, so that what the caller sees free afterwards is free
  pool().drop_cache();
  return GMRF_OK;
}

gmrf_status gmrf_pool_reserve(size_t bytes) {
  if (bytes) {
    gmrf_status ds = check_device();
    if (ds != GMRF_OK) return ds;
  }
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  if (P.region && !P.region_idle())
    return fail(GMRF_EINVAL, "the reserved region still holds scratch of running calls");
  P.drop_cache();
  if (P.region) {
    P.dev_free(P.region);
    P.region = nullptr;
    P.region_size = 0;
    P.holes.clear();
  }
  if (bytes == 0) return GMRF_OK;
  bytes = Pool::rounded(bytes);
  void* p = nullptr;
  if (P.dev_alloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(GMRF_ENOMEM, "hipMalloc of the %zu B region failed", bytes);
  }
  P.region = static_cast<char*>(p);
  P.region_size = bytes;
  P.holes.emplace(0, bytes);
  return GMRF_OK;
}

gmrf_status gmrf_pool_query(gmrf_pool_info* info) {
  if (!info) return fail(GMRF_EINVAL, "info is null");
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  info->reserved_bytes = P.region_size;
  info->largest_free_range = P.largest_hole();
  info->in_use = P.in_use;
  info->cached = P.cached;
  info->device_allocs = P.n_alloc;
  info->device_frees = P.n_free;
  info->alloc_seconds = P.t_alloc;
  info->free_seconds = P.t_free;
  return GMRF_OK;
}

size_t gmrf_hbm_in_use(void) {
  std::lock_guard<std::mutex> lk(pool().mu);
  return pool().in_use;
}

gmrf_status gmrf_op_create_lattice(int ndim, const int64_t* shape, int order, double kappa2, double tau,
                                   gmrf_boundary bc, gmrf_dtype storage, gmrf_op** out) {
  if (!out) return fail(GMRF_EINVAL, "out is NULL");
  *out = nullptr;
  if (ndim < 1 || ndim > 3 || !shape) return fail(GMRF_EINVAL, "ndim must be 1..3");
  if (order != 1 && order != 2) return fail(GMRF_EINVAL, "order must be 1 or 2");
  if (!(tau > 0.0) || !std::isfinite(tau) || !std::isfinite(kappa2))
    return fail(GMRF_EINVAL, "tau must be > 0 and finite, kappa2 finite");
  if (bc != GMRF_FREE && bc != GMRF_PERIODIC) return fail(GMRF_EINVAL, "bad boundary");
  if (storage != GMRF_F64 && storage != GMRF_F32) return fail(GMRF_EINVAL, "bad storage dtype");
  int64_t n = 1;
  for (int d = 0; d < ndim; ++d) {
    if (shape[d] < 1 || shape[d] > (1 << 24)) return fail(GMRF_EINVAL, "shape[%d] out of range", d);
    n *= shape[d];
  }
  if (n > ((int64_t)1 << 31)) return fail(GMRF_EINVAL, "lattice too large (n > 2^31)");
  gmrf_status ds = check_device();
  if (ds != GMRF_OK) return ds;
  auto op = new gmrf_op();
  op->kind = 0;
  op->ndim = ndim;
  for (int d = 0; d < 3; ++d) op->shape[d] = 1;
  for (int d = 0; d < ndim; ++d) op->shape[3 - ndim + d] = shape[d];
  op->order = order;
  op->kappa2 = kappa2;
  op->tau = tau;
  op->bc = bc;
  op->storage = storage;
  op->n = n;
  op->dim = ndim;
  op->geom.n0 = (int)op->shape[0];
  op->geom.n1 = (int)op->shape[1];
  op->geom.n2 = (int)op->shape[2];
  op->geom.periodic = bc == GMRF_PERIODIC;
  op->geom.kappa2 = kappa2;
  op->geom.tau = tau;
  stencil_geom_tiles(op->geom, ndim, order, 0, storage == GMRF_F64 ? 8 : 4);
  *out = op;
  return GMRF_OK;
}

gmrf_status gmrf_op_create_csr(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                               const double* values, gmrf_dtype storage, gmrf_op** out) {
  if (!out) return fail(GMRF_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || n > ((int64_t)1 << 31) || !row_ptr || !col_idx || !values)
    return fail(GMRF_EINVAL, "bad CSR arguments");
  if (storage != GMRF_F64 && storage != GMRF_F32) return fail(GMRF_EINVAL, "bad storage dtype");
  if (row_ptr[0] != 0) return fail(GMRF_EINVAL, "row_ptr[0] must be 0");
  for (int64_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return fail(GMRF_EINVAL, "row_ptr not non-decreasing at %lld", (long long)i);
  const int64_t nnz = row_ptr[n];
  for (int64_t e = 0; e < nnz; ++e)
    if (col_idx[e] < 0 || col_idx[e] >= n) return fail(GMRF_EINVAL, "column index out of range at %lld", (long long)e);
  for (int64_t e = 0; e < nnz; ++e)
    if (!std::isfinite(values[e])) return fail(GMRF_EINVAL, "non-finite value at %lld", (long long)e);
  gmrf_status ds = check_device();
  if (ds != GMRF_OK) return ds;
  auto op = std::make_unique<gmrf_op>();
  op->kind = 1;
  op->n = n;
  op->nnz = nnz;
  op->storage = storage;
  op->shape[2] = n;
  const size_t vb = storage == GMRF_F64 ? 8 : 4;
  HIP_TRY(hipMalloc(&op->rp, (n + 1) * sizeof(int64_t)));
  HIP_TRY(hipMalloc(&op->ci, std::max<int64_t>(nnz, 1) * sizeof(int32_t)));
  HIP_TRY(hipMalloc(&op->va, std::max<int64_t>(nnz, 1) * vb));
  HIP_TRY(hipMemcpy(op->rp, row_ptr, (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  if (nnz) HIP_TRY(hipMemcpy(op->ci, col_idx, nnz * sizeof(int32_t), hipMemcpyHostToDevice));
  if (nnz) {
    if (storage == GMRF_F64) {
      HIP_TRY(hipMemcpy(op->va, values, nnz * 8, hipMemcpyHostToDevice));
    } else {
      std::vector<float> tmp(values, values + nnz);
      HIP_TRY(hipMemcpy(op->va, tmp.data(), nnz * 4, hipMemcpyHostToDevice));
    }
  }
  op->resident_bytes = (n + 1) * 8 + nnz * (4 + vb);
  op->h_rp.assign(row_ptr, row_ptr + n + 1);
  op->h_ci.assign(col_idx, col_idx + nnz);
  op->h_va.assign(values, values + nnz);
  *out = op.release();
  return GMRF_OK;
}

void gmrf_op_destroy(gmrf_op* Q) {
  if (!Q) return;
  if (Q->rp) (void)hipFree(Q->rp);
  if (Q->ci) (void)hipFree(Q->ci);
  if (Q->va) (void)hipFree(Q->va);
  if (Q->mult64) (void)hipFree(Q->mult64);
  if (Q->mult32) (void)hipFree(Q->mult32);
  if (Q->diag64) (void)hipFree(Q->diag64);
  if (Q->diag32) (void)hipFree(Q->diag32);
  free_ichol(Q->icd);
  fft_plan_destroy(Q->plan);
  delete Q;
}

gmrf_status gmrf_op_size(const gmrf_op* Q, int64_t* n) {
  if (!Q || !n) return fail(GMRF_EINVAL, "NULL argument");
  *n = Q->n;
  return GMRF_OK;
}

}  // extern "C"

// ---- circulant preconditioner: lambda_M^{-1/2} table on the packed spectrum ----------------------
// M = periodic version of the lattice precision; lambda_M(k1, k2) = tau (kappa2 + mu1 + mu2)^order
// with mu = 4 sin^2(pi k / N) (cycle spectra).  The table stores lambda^{-1/2} for every packed
// coefficient: [k1][c] for c = 1..N2/2-1 and, in column 0, the pair (k2 = 0, k2 = N2/2).
static gmrf_status build_precond(gmrf_op* Q) {
  const int N1 = (int)Q->shape[1], N2 = (int)Q->shape[2];
  const int H = N2 / 2;
  std::vector<double> mu1(N1), mu2(N2);
  for (int k = 0; k < N1; ++k) mu1[k] = periodic_mu(k, N1);
  for (int k = 0; k < N2; ++k) mu2[k] = periodic_mu(k, N2);
  auto lam = [&](int k1, int k2) {
    const double b = Q->kappa2 + mu1[k1] + mu2[k2];
    return Q->order == 1 ? Q->tau * b : Q->tau * b * b;
  };
  // table layout: [k1][mult_stride(H)]: entries 0..H-1 for columns (col 0 -> k2 = 0), entry H -> k2 = N2/2
  const int ms = mult_stride(H);
  std::vector<double> t((size_t)N1 * ms, 0.0);
  double ld = 0.0;
  for (int k1 = 0; k1 < N1; ++k1) {
    for (int c = 0; c < H; ++c) t[(size_t)k1 * ms + c] = 1.0 / std::sqrt(lam(k1, c));
    t[(size_t)k1 * ms + H] = 1.0 / std::sqrt(lam(k1, H));
    for (int k2 = 0; k2 < N2; ++k2) {
      const double l = lam(k1, k2);
      if (!(l > 0.0)) return fail(GMRF_ENOTSPD, "periodic preconditioner is singular (kappa2 <= 0)");
      ld += std::log(l);
    }
  }
  Q->logdet_M = ld;
  HIP_TRY(hipMalloc(&Q->mult64, t.size() * sizeof(double)));
  HIP_TRY(hipMemcpy(Q->mult64, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
  std::vector<float> t32(t.begin(), t.end());
  HIP_TRY(hipMalloc(&Q->mult32, t32.size() * sizeof(float)));
  HIP_TRY(hipMemcpy(Q->mult32, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice));
  Q->resident_bytes += t.size() * 12;
  return GMRF_OK;
}

static bool pow2_in(int64_t v, int64_t lo, int64_t hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

extern "C" gmrf_status gmrf_op_set_circulant_precond(gmrf_op* Q, int enable) {
  if (!Q) return fail(GMRF_EINVAL, "NULL operator");
  if (!enable) {
    Q->precond = 0;
    return GMRF_OK;
  }
  if (Q->kind != 0 || Q->ndim != 2)
    return fail(GMRF_EUNSUPPORTED, "circulant preconditioning needs a 2D lattice operator");
  if (Q->has_diag && Q->bc != GMRF_PERIODIC)
    return fail(GMRF_EUNSUPPORTED, "with a diagonal term the preconditioner M = Q needs a periodic lattice");
  if (!pow2_in(Q->shape[1], 8, 4096) || !pow2_in(Q->shape[2], 8, 4096))
    return fail(GMRF_EUNSUPPORTED, "circulant preconditioning needs power-of-two sides in [8, 4096]");
  if (!Q->mult64) {
    gmrf_status s = build_precond(Q);
    if (s != GMRF_OK) return s;
    s = fft_plan_create(Q->plan, (int)Q->shape[1], (int)Q->shape[2]);
    if (s != GMRF_OK) return fail(s, "FFT plan creation failed");
  }
  Q->precond = 1;
  return GMRF_OK;
}

extern "C" gmrf_status gmrf_op_set_diagonal(gmrf_op* Q, const double* d) {
  if (!Q) return fail(GMRF_EINVAL, "NULL operator");
  if (!d) {
    Q->has_diag = 0;
    return GMRF_OK;
  }
  if (Q->kind != 0) return fail(GMRF_EUNSUPPORTED, "a diagonal term needs a lattice operator");
  if (Q->precond && Q->bc != GMRF_PERIODIC)
    return fail(GMRF_EUNSUPPORTED, "with circulant preconditioning a diagonal term needs a periodic lattice");
  const size_t n = (size_t)Q->n;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(d[i])) return fail(GMRF_EINVAL, "non-finite diagonal value at %zu", i);
  if (!Q->diag64) {
    HIP_TRY(hipMalloc(&Q->diag64, n * sizeof(double)));
    HIP_TRY(hipMalloc(&Q->diag32, n * sizeof(float)));
    Q->resident_bytes += n * 12;
  }
  std::vector<float> d32(d, d + n);
  HIP_TRY(hipMemcpy(Q->diag64, d, n * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(Q->diag32, d32.data(), n * sizeof(float), hipMemcpyHostToDevice));
  Q->has_diag = 1;
  return GMRF_OK;
}

// ---- incomplete-Cholesky preconditioner (Section 5.2) -----------------------------------------------
namespace {
void free_trsv(TrsvDev& d) {
  for (void* p : {(void*)d.lvl_ptr, (void*)d.rows, (void*)d.rp, (void*)d.ci, d.va, d.dinv})
    if (p) (void)hipFree(p);
  d = TrsvDev{};
}
}  // namespace
void free_ichol(IcholDev& f) {
  free_trsv(f.fwd);
  free_trsv(f.bwd);
}
namespace {
template <typename V>
gmrf_status upload(const std::vector<V>& h, V** d) {
  HIP_TRY(hipMalloc(d, std::max<size_t>(h.size(), 1) * sizeof(V)));
  if (!h.empty()) HIP_TRY(hipMemcpy(*d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice));
  return GMRF_OK;
}
gmrf_status upload_vals(const std::vector<double>& h, int storage, void** d) {
  if (storage == GMRF_F64) return upload(h, (double**)d);
  std::vector<float> f(h.begin(), h.end());
  return upload(f, (float**)d);
}
// One solve in level order: position p = row lvl_rows[p] of (rp, ci, va), 1 / diagonal alongside.
gmrf_status upload_trsv(const std::vector<int64_t>& rp, const std::vector<int32_t>& ci, const std::vector<double>& va,
                        const std::vector<double>& diag, const std::vector<int32_t>& lvl_ptr,
                        const std::vector<int32_t>& lvl_rows, int storage, TrsvDev& d) {
  const size_t n = lvl_rows.size();
  d.max_row = 0;
  std::vector<int64_t> prp(n + 1, 0);
  std::vector<int32_t> pci;
  std::vector<double> pva, pdinv(n);
  pci.reserve(ci.size());
  pva.reserve(va.size());
  for (size_t p = 0; p < n; ++p) {
    const int32_t i = lvl_rows[p];
    for (int64_t e = rp[(size_t)i]; e < rp[(size_t)i + 1]; ++e) {
      pci.push_back(ci[(size_t)e]);
      pva.push_back(va[(size_t)e]);
    }
    prp[p + 1] = (int64_t)pci.size();
    pdinv[p] = 1.0 / diag[(size_t)i];
    d.max_row = std::max(d.max_row, (int)(prp[p + 1] - prp[p]));
  }
  gmrf_status s;
  if ((s = upload(lvl_ptr, &d.lvl_ptr)) != GMRF_OK || (s = upload(lvl_rows, &d.rows)) != GMRF_OK ||
      (s = upload(prp, &d.rp)) != GMRF_OK || (s = upload(pci, &d.ci)) != GMRF_OK ||
      (s = upload_vals(pva, storage, &d.va)) != GMRF_OK || (s = upload_vals(pdinv, storage, &d.dinv)) != GMRF_OK)
    return s;
  d.nlev = (int)lvl_ptr.size() - 1;
  d.nnz = (int64_t)pci.size();
  d.max_width = 0;
  for (int l = 0; l < d.nlev; ++l) d.max_width = std::max(d.max_width, lvl_ptr[(size_t)l + 1] - lvl_ptr[(size_t)l]);
  return GMRF_OK;
}
}  // namespace

extern "C" gmrf_status gmrf_op_set_ichol_precond(gmrf_op* Q, int enable, double droptol, double* shift_used) {
  if (!Q) return fail(GMRF_EINVAL, "NULL operator");
  if (!enable) {
    Q->ic = 0;
    return GMRF_OK;
  }
  if (Q->kind != 1) return fail(GMRF_EUNSUPPORTED, "incomplete-Cholesky preconditioning needs a CSR operator");
  if (std::isnan(droptol)) return fail(GMRF_EINVAL, "droptol is NaN");
  IcholHost h;
  if (!ichol_factor(Q->n, Q->h_rp.data(), Q->h_ci.data(), Q->h_va.data(), droptol, h))
    return fail(GMRF_ENOTSPD, "incomplete Cholesky broke down for every diagonal shift up to 2^30 * 1e-3");
  IcholDev& d = Q->icd;
  free_ichol(d);
  d.n = Q->n;
  gmrf_status s;
  if ((s = upload_trsv(h.lrp, h.lci, h.lva, h.diag, h.flev_ptr, h.flev_rows, Q->storage, d.fwd)) != GMRF_OK ||
      (s = upload_trsv(h.urp, h.uci, h.uva, h.diag, h.blev_ptr, h.blev_rows, Q->storage, d.bwd)) != GMRF_OK)
    return s;
  Q->ic_logdet = h.logdet_M;
  Q->ic_shift = h.shift;
  Q->ic_nnz = (int64_t)h.lva.size() + Q->n;
  Q->ic = 1;
  if (shift_used) *shift_used = h.shift;
  return GMRF_OK;
}

extern "C" gmrf_status gmrf_ichol_info(const gmrf_op* Q, int64_t* nnz_L, int32_t* levels, double* shift) {
  if (!Q || !Q->ic) return fail(GMRF_EINVAL, "no incomplete-Cholesky preconditioner on this operator");
  if (nnz_L) *nnz_L = Q->ic_nnz;
  if (levels) *levels = Q->icd.fwd.nlev;
  if (shift) *shift = Q->ic_shift;
  return GMRF_OK;
}

// ---- sizes ------------------------------------------------------------------------------------------
namespace {
// Q + diag(d) preconditioned by its periodic lattice part: two FFT passes per step (lgcp_step.hip).
bool lgcp_path(const gmrf_op* Q) { return Q->precond && Q->has_diag; }
const void* diag_of(const gmrf_op* Q) {
  return Q->storage == GMRF_F64 ? (const void*)Q->diag64 : (const void*)Q->diag32;
}

// 2D lattice operators without preconditioning or reorthogonalisation run one pass per Lanczos step
// (k_lanczos2d: alpha_j from the quadratic form the previous pass formed).
bool fused_path(const gmrf_op* Q, int reorth) {
  return !Q->precond && !Q->has_diag && Q->kind == 0 && Q->dim == 2 && !reorth;
}

struct Sizes {
  long L;          // storage elements per vector
  int slots;       // Krylov slots kept
  int Pa, Pb, pstride;
  int Pb_first;    // ||w||^2 partials written by the init kernel (read by the opener of iteration 1)
  size_t vec_bytes;
};

Sizes sizes_for(const gmrf_op* Q, int64_t k, int m_max, int reorth, bool ring3) {
  Sizes z{};
  z.L = (long)Q->n;  // packed half spectrum has exactly n reals too
  z.slots = ring3 ? 3 : m_max + 1;
  z.Pb_first = ew_blocks(z.L);
  if (lgcp_path(Q)) {
    const LgcpCounts c = lgcp_counts(Q->plan, Q->storage);
    z.Pa = c.Pr + 1;                              // y^T H y per row block, <w_{j-1}, v_{j-1}>
    z.Pb = reorth ? reorth_blocks(z.L) : c.Pc;
    z.pstride = std::max(std::max(z.Pa, z.Pb), std::max(z.Pb_first, c.Pc));
  } else if (Q->precond) {
    const PrecondStepCounts c = precond_step_counts(Q->plan);
    z.Pa = c.Pband + 1;                           // <u, D u> per band block, <w_{j-1}, v_{j-1}>
    z.Pb = reorth ? reorth_blocks(z.L) : c.Ps;    // the reorthogonalisation rewrites the norm partials
  } else if (fused_path(Q, reorth)) {
    z.Pa = lanczos2d_blocks(Q->geom);             // the one-pass kernel's partial sums
    z.Pb = z.Pa;
  } else if (Q->ic) {
    z.Pa = ew_blocks(z.L);                        // the opener's v_j^T q partials (elementwise tiling)
    z.Pb = reorth ? reorth_blocks(z.L) : ew_blocks(z.L);
  } else {
    z.Pa = Q->kind == 0 ? stencil_blocks(Q->geom) : csr_blocks((long)Q->n);
    z.Pb = reorth ? reorth_blocks(z.L) : ew_blocks(z.L);
  }
  z.pstride = std::max(std::max(std::max(z.Pa, z.Pb), z.Pb_first), z.pstride);
  if (Q->precond && !lgcp_path(Q)) z.pstride = std::max(z.pstride, precond_step_counts(Q->plan).Ps);   // step kernel
  z.vec_bytes = (size_t)z.L * (Q->storage == GMRF_F64 ? 8 : 4);
  (void)k;
  return z;
}

int groups_for(const gmrf_op* Q, int64_t k);

size_t call_bytes(const gmrf_op* Q, int64_t k, int m_max, int reorth, bool ring3) {
  Sizes z = sizes_for(Q, k, m_max, reorth, ring3);
  size_t b = (size_t)z.slots * k * z.vec_bytes;       // Krylov basis
  b += (size_t)k * z.vec_bytes;                       // q
  if (Q->precond || Q->ic) b += (size_t)k * z.vec_bytes;                               // FFT / solve scratch
  if (Q->precond && !lgcp_path(Q)) b += precond_step_bytes(Q->plan, Q->storage, (int)k);   // band tables
  b += (size_t)k * (m_max + 2) * 8 * 4 + (size_t)k * 32;  // scalars, flags, poll values
  b += (fused_path(Q, reorth) ? 6 : 3) * (size_t)k * z.pstride * 8;   // partials (two sets when fused)
  if (reorth) b += (size_t)k * (m_max + 1) * ((size_t)z.Pb * reorth_partial_sets(z.L) + 1) * 8;
  if (!ring3) b += (size_t)k * m_max * 8 + tri_scratch_doubles((int)k, m_max) * 8;
  return b;
}
}  // namespace

// Allocations of one call are rounded up to the pool's granularity; kPoolAllocs bounds the number of blocks a
// column group's call takes (basis, work vectors, FFT or solve scratch, band tables, scalars, poll values, flags,
// reorthogonalisation partials, tridiagonal output and scratch, two-pass accumulator).
constexpr size_t kPoolGranule = (size_t)2 << 20;
constexpr int kPoolAllocs = 12;

extern "C" gmrf_status gmrf_op_bytes(const gmrf_op* Q, int64_t k, int32_t m_max, int reorth, size_t* bytes) {
  if (!Q || !bytes || k < 1 || m_max < 1) return fail(GMRF_EINVAL, "bad arguments");
  const int G = groups_for(Q, k);
  size_t b = 0;
  for (int g = 0; g < G; ++g) {
    const int64_t kg = k * (g + 1) / G - k * g / G;
    b += call_bytes(Q, kg, m_max, reorth, false) + kPoolAllocs * kPoolGranule;
  }
  *bytes = b + Q->resident_bytes;
  return GMRF_OK;
}

extern "C" gmrf_status gmrf_op_bytes_two_pass(const gmrf_op* Q, int64_t k, int32_t m_max, size_t* bytes) {
  if (!Q || !bytes || k < 1 || m_max < 1) return fail(GMRF_EINVAL, "bad arguments");
  const int G = groups_for(Q, k);
  size_t b = 0;
  for (int g = 0; g < G; ++g) {
    const int64_t kg = k * (g + 1) / G - k * g / G;
    const Sizes z = sizes_for(Q, kg, m_max, 0, true);
    b += call_bytes(Q, kg, m_max, 0, true);                                  // pass 1: three slots, scalars
    b += (size_t)kg * (m_max + 2) * 8 * 4 + (size_t)kg * 32 + 3 * (size_t)kg * z.pstride * 8;   // pass 2 scalars
    b += (size_t)kg * m_max * 8 + tri_scratch_doubles((int)kg, m_max) * 8;    // y and its scratch
    if (Q->precond || Q->ic) b += (size_t)kg * z.vec_bytes;                  // the u_m accumulator
    b += kPoolAllocs * kPoolGranule;
  }
  *bytes = b + Q->resident_bytes;
  return GMRF_OK;
}

// ---- autotuner table: launch options that leave every result bit unchanged --------------------------------
// The table maps (kernel, order, storage, shape class, columns class) to kTune* bits (common.hpp: tile order and
// store policy for both kernels, tile shape for the operator kernel alone); shape class =
// ceil(log2) of each lattice side, columns class = ceil(log2 k).  Entries come from gmrf_autotune, which times every
// candidate with HIP events on scratch data of the call's shape and keeps the fastest, or from gmrf_tune_import.
// A key without an entry launches with no options (linear tile order, ordinary stores).  Since no option changes a
// result bit, results never depend on the table's state: a field gets identical bits alone and in a batch whatever
// was tuned.
namespace {
enum { kTuneKernelSpmm = 0, kTuneKernelLanczos2d = 1, kTuneKernels = 2 };
constexpr int kTuneCandidates[4] = {0, kTuneXcd, kTuneNtStore, kTuneXcd | kTuneNtStore};
struct TuneKey {
  int kernel, order, storage, c1, c2, ck;
  bool operator<(const TuneKey& o) const {
    return std::tie(kernel, order, storage, c1, c2, ck) < std::tie(o.kernel, o.order, o.storage, o.c1, o.c2, o.ck);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int>& tune_table() {
  static std::map<TuneKey, int>* t = new std::map<TuneKey, int>();
  return *t;
}
int clog2(int64_t v) {
  int c = 0;
  while (((int64_t)1 << c) < v) ++c;
  return c;
}
TuneKey tune_key(int kernel, const gmrf_op* Q, int64_t k) {
  return {kernel, Q->order, Q->storage, clog2(Q->shape[1]), clog2(Q->shape[2]), clog2(k)};
}
bool tunable(const gmrf_op* Q) { return Q->kind == 0 && Q->dim == 2; }
int tune_lookup(int kernel, const gmrf_op* Q, int64_t k) {
  if (!tunable(Q)) return 0;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = tune_table().find(tune_key(kernel, Q, k));
  return it == tune_table().end() ? 0 : it->second;
}
// tile shape coded in kTuneGeomMask bits: (rows per wave, columns per lane), 0 where the code asks for the rule
// or does not suit the operator (four columns per lane: FP32 rows of a multiple of 4; two: even rows)
void geom_code(const gmrf_op* Q, int bits, int& band, int& epl) {
  static const int bands[4] = {0, 8, 16, 32}, epls[4] = {0, 1, 2, 4};
  band = bands[(bits >> kTuneBandShift) & 3];
  epl = epls[(bits >> kTuneEplShift) & 3];
  if ((epl == 4 && (Q->storage != GMRF_F32 || Q->shape[2] % 4 != 0)) || (epl == 2 && Q->shape[2] % 2 != 0)) epl = 0;
}
// the operator's geometry with the launch options of `kernel` for k columns (tune >= 0: those options instead);
// tile-shape bits apply to the operator kernel alone
StencilGeom tuned_geom(int kernel, const gmrf_op* Q, int64_t k, int tune = -1) {
  StencilGeom g = Q->geom;
  g.tune = tune >= 0 ? tune : tune_lookup(kernel, Q, k);
  if (kernel == kTuneKernelSpmm && (g.tune & kTuneGeomMask) && tunable(Q)) {
    int band, epl;
    geom_code(Q, g.tune, band, epl);
    stencil_geom_shape(g, Q->order, band ? band : g.band, epl ? epl : g.epl);
  }
  return g;
}
}  // namespace

// ---- operator application --------------------------------------------------------------------------
template <typename T>
static void op_apply_lz(const gmrf_op* Q, const T* X, T* Y, const T* Xprev, const LzState& S, int j, int k,
                        hipStream_t st) {
  if (Q->kind == 0)
    launch_stencil<T>(Q->geom, Q->order, Q->dim, true, X, Q->n, Y, Q->n, Xprev, S, j, k, st);
  else
    launch_csr<T>((long)Q->n, Q->rp, Q->ci, (const T*)Q->va, true, X, Q->n, Y, Q->n, Xprev, S, j, k, st);
}

template <typename T>
static void op_apply_plain(const gmrf_op* Q, const T* X, T* Y, int k, hipStream_t st, int tune = -1) {
  LzState S{};
  if (Q->kind == 0) {
    // caller buffers may not be aligned for the 2D kernel's element pairs: then one element per lane
    StencilGeom g = tuned_geom(kTuneKernelSpmm, Q, k, tune);
    if (g.epl > 1 && (((uintptr_t)X | (uintptr_t)Y) % (g.epl * sizeof(T))) != 0) stencil_geom_tiles(g, Q->dim, Q->order, 1);
    launch_stencil<T>(g, Q->order, Q->dim, false, X, Q->n, Y, Q->n, nullptr, S, 0, k, st);
    if (Q->has_diag) launch_add_diag<T>((const T*)diag_of(Q), X, Y, (long)Q->n, k, st);
    return;
  }
  launch_csr<T>((long)Q->n, Q->rp, Q->ci, (const T*)Q->va, false, X, Q->n, Y, Q->n, nullptr, S, 0, k, st);
}

extern "C" gmrf_status gmrf_op_apply(const gmrf_op* Q, const void* X, void* Y, int64_t k, void* stream) {
  if (!Q || !X || !Y || k < 1 || k > 65535) return fail(GMRF_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  if (Q->storage == GMRF_F64) op_apply_plain<double>(Q, (const double*)X, (double*)Y, (int)k, st);
  else op_apply_plain<float>(Q, (const float*)X, (float*)Y, (int)k, st);
  HIP_TRY(hipGetLastError());
  return GMRF_OK;
}

extern "C" gmrf_status gmrf_precond_apply(const gmrf_op* Q, const void* X, void* Y, int64_t k, void* stream) {
  if (!Q || !X || !Y || k < 1 || k > 65535) return fail(GMRF_EINVAL, "bad arguments");
  if (!Q->precond) return fail(GMRF_EINVAL, "circulant preconditioning is not enabled on this operator");
  hipStream_t st = (hipStream_t)stream;
  Workspace ws(st);
  gmrf_status s;
  if (Q->storage == GMRF_F64) {
    double* tmp;
    if ((s = ws.alloc(Q->n * k, &tmp)) != GMRF_OK) return s;
    fft_apply_inv_sqrt_M<double>(Q->plan, Q->mult64, (const double*)X, (double*)Y, tmp, (int)k, st);
  } else {
    float* tmp;
    if ((s = ws.alloc(Q->n * k, &tmp)) != GMRF_OK) return s;
    fft_apply_inv_sqrt_M<float>(Q->plan, Q->mult32, (const float*)X, (float*)Y, tmp, (int)k, st);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return GMRF_OK;
}

// ---- the Lanczos driver --------------------------------------------------------------------------------
namespace {

const void* precond_mult(const gmrf_op* Q) {
  return Q->storage == GMRF_F64 ? (const void*)Q->mult64 : (const void*)Q->mult32;
}

struct Scalars {
  double *alpha, *beta, *dpiv, *rho;
  int *m_used, *status, *active;
  double *part_a, *part_b;
};

template <typename T>
struct Run {
  const gmrf_op* Q;
  int k, m_max, reorth;
  double tol;
  hipStream_t st;
  Sizes z;
  LzState S{};
  T* V = nullptr;        // slots x k x L
  T* Qb = nullptr;       // k x L
  T* F1 = nullptr;       // FFT intermediates (preconditioned)
  void* band = nullptr;  // hand-off buffers between the kernels of a preconditioned step
  int pb_first = 0;      // partial count of the init kernel (iteration 1's opener)
  double* part_h = nullptr;
  double* h = nullptr;
  double* pollv = nullptr;        // 2 k doubles: active flags and rho_{j-1}, gathered for a stop poll
  bool ring3 = false;
  bool fused = false;             // one pass per step (k_lanczos2d); partial sums alternate between ps[0], ps[1]
  double* ps[2][3] = {};          // {quadratic form, ||w||^2, <w, v>} partial sums
  StencilGeom geom2d{};           // the operator's geometry with the one-pass kernel's tuned launch options

  T* slot(int t) const {
    const int s = ring3 ? (t % 3) : t;
    return V + (size_t)s * k * z.L;
  }
};

template <typename T>
gmrf_status setup_state(Run<T>& R, Workspace& ws);

template <typename T>
gmrf_status setup(Run<T>& R, Workspace& ws) {
  const gmrf_op* Q = R.Q;
  R.z = sizes_for(Q, R.k, R.m_max, R.reorth, R.ring3);
  const int k = R.k, m = R.m_max;
  gmrf_status s;
  if ((s = ws.alloc((size_t)R.z.slots * k * R.z.L, &R.V)) != GMRF_OK) return s;
  if ((s = ws.alloc((size_t)k * R.z.L, &R.Qb)) != GMRF_OK) return s;
  if (Q->precond || Q->ic) {
    if ((s = ws.alloc((size_t)k * R.z.L, &R.F1)) != GMRF_OK) return s;
  }
  if (Q->precond && !lgcp_path(Q)) {
    char* band;
    if ((s = ws.alloc(precond_step_bytes(Q->plan, Q->storage, k), &band)) != GMRF_OK) return s;
    R.band = band;
  }
  R.fused = fused_path(Q, R.reorth);
  R.geom2d = tuned_geom(kTuneKernelLanczos2d, Q, k);
  return setup_state<T>(R, ws);
}

// The scalar state of a run (coefficients, pivots, partial sums, flags), zeroed and active: a second
// pass over the same vector buffers takes a fresh one.
template <typename T>
gmrf_status setup_state(Run<T>& R, Workspace& ws) {
  const gmrf_op* Q = R.Q;
  const int k = R.k, m = R.m_max;
  gmrf_status s;
  double* dbuf;
  const int nsets = R.fused ? 6 : 3;
  const size_t nd = (size_t)k * (m + 1) * 3 + (size_t)k * (m + 2) + nsets * (size_t)k * R.z.pstride;
  if ((s = ws.alloc(nd, &dbuf)) != GMRF_OK) return s;
  if ((s = ws.alloc((size_t)2 * k, &R.pollv)) != GMRF_OK) return s;
  int* ibuf;
  if ((s = ws.alloc((size_t)3 * k, &ibuf)) != GMRF_OK) return s;
  LzState& S = R.S;
  S.k = k;
  S.m_max = m;
  S.tol = R.tol;
  S.alpha = dbuf;
  S.dpiv = S.alpha + (size_t)k * (m + 1);
  S.rho = S.dpiv + (size_t)k * (m + 1);
  S.beta = S.rho + (size_t)k * (m + 1);
  S.part_a = S.beta + (size_t)k * (m + 2);
  S.part_b = S.part_a + (size_t)k * R.z.pstride;
  S.part_c = S.part_b + (size_t)k * R.z.pstride;
  if (R.fused) {
    for (int q = 0; q < 6; ++q) R.ps[q / 3][q % 3] = S.part_a + (size_t)q * k * R.z.pstride;
  }
  S.m_used = ibuf;
  S.status = ibuf + k;
  S.active = ibuf + 2 * k;
  S.Pa = R.z.Pa;
  S.Pb = R.z.Pb;
  S.pstride = R.z.pstride;
  R.pb_first = R.z.Pb_first;
  S.weighted = Q->precond ? 1 : 0;
  S.H = Q->precond ? (int)(Q->shape[2] / 2) : 1;
  HIP_TRY(hipMemsetAsync(dbuf, 0, nd * sizeof(double), R.st));
  HIP_TRY(hipMemsetAsync(ibuf, 0, 2 * k * sizeof(int), R.st));
  HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)S.active, 1, k, R.st));
  if (R.reorth) {
    if ((s = ws.alloc((size_t)k * (m + 1) * R.z.Pb * reorth_partial_sets(R.z.L), &R.part_h)) != GMRF_OK) return s;
    if ((s = ws.alloc((size_t)k * (m + 1), &R.h)) != GMRF_OK) return s;
  }
  return GMRF_OK;
}

// After slot 0 and its norm partial sums are in place: the quadratic form of slot 0 (set 0) for the
// one-pass kernel's alpha_1.
template <typename T>
void fused_init(Run<T>& R) {
  if (!R.fused) return;
  launch_lanczos2d<T>(R.geom2d, R.Q->order, 1, 0, R.slot(0), R.z.L, nullptr, nullptr, R.S, 0, R.k, R.ps[0][0],
                      nullptr, nullptr, R.st);
}

// pinned polling buffer per host thread
int* poll_buffer(int k) {
  static thread_local int* buf = nullptr;
  static thread_local int cap = 0;
  if (cap < k) {
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    if (hipHostMalloc((void**)&buf, (size_t)std::max(k, 64) * sizeof(int), hipHostMallocDefault) != hipSuccess)
      return nullptr;
    cap = std::max(k, 64);
  }
  return buf;
}

// pinned buffer for the residuals read at a poll, per host thread
double* poll_rho_buffer(int k) {
  static thread_local double* buf = nullptr;
  static thread_local int cap = 0;
  if (cap < k) {
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    if (hipHostMalloc((void**)&buf, (size_t)std::max(k, 64) * sizeof(double), hipHostMallocDefault) != hipSuccess)
      return nullptr;
    cap = std::max(k, 64);
  }
  return buf;
}

// One iteration j: operator (opener) + update (+ reorth).  The opener of iteration 1 reduces the
// partial sums of the init kernel, later openers those of the previous iteration.
template <typename T>
void iterate(Run<T>& R, int j) {
  const gmrf_op* Q = R.Q;
  T* xj = R.slot(j - 1);
  T* xp = j >= 2 ? R.slot(j - 2) : R.slot(0);
  R.S.Pb = (j == 1) ? R.pb_first : R.z.Pb;
  // plain and incomplete-Cholesky steps with short vectors: the first reorthogonalisation launch also does
  // the update step
  const bool upd_in_reorth = R.reorth && !Q->precond && !R.fused && reorth_takes_update(R.z.L);
  if (R.fused) {
    // reads the partial sums in R.S (pass j - 1's; iteration 1: the init kernels' set 0) and writes the other
    // set, which R.S then points to (the next pass and k_finalize read it)
    const int wset = j & 1;
    launch_lanczos2d<T>(R.geom2d, Q->order, 0, 0, xj, R.z.L, R.slot(j), xp, R.S, j, R.k, R.ps[wset][0],
                        R.ps[wset][1], R.ps[wset][2], R.st);
    R.S.part_a = R.ps[wset][0];
    R.S.part_b = R.ps[wset][1];
    R.S.part_c = R.ps[wset][2];
  } else if (lgcp_path(Q)) {
    // T1 = R.F1 holds the column-inverse transform of Lambda^{-1/2} slot j-1; T2 = R.Qb
    lgcp_lanczos_step<T>(Q->plan, precond_mult(Q), (const T*)diag_of(Q), R.F1, R.Qb, xj, xp, R.slot(j), R.S, j,
                         R.reorth ? 0 : 1, R.k, R.st);
  } else if (Q->precond) {
    precond_lanczos_step<T>(Q->plan, Q->geom, Q->order, precond_mult(Q), xj, xp, R.slot(j), R.band, R.S, j,
                            R.reorth ? 0 : 1, R.reorth ? 0 : 1, R.k, R.st);
  } else if (Q->ic) {
    // A slot_{j-1} = L^{-1} Q L^{-T} slot_{j-1} (F1 <- L^{-T} slot, Qb <- Q F1, F1 <- L^{-1} Qb), then the opener
    launch_trsv<T, T>(Q->icd, true, xj, R.z.L, R.F1, R.z.L, R.S.active, R.k, R.st);
    launch_csr<T>((long)Q->n, Q->rp, Q->ci, (const T*)Q->va, false, R.F1, Q->n, R.Qb, Q->n, nullptr, R.S, 0, R.k, R.st);
    launch_trsv<T, T>(Q->icd, false, R.Qb, R.z.L, R.F1, R.z.L, R.S.active, R.k, R.st);
    launch_pre_lz<T>(R.F1, xj, xp, R.Qb, R.z.L, R.S, j, R.st);
    if (!upd_in_reorth) launch_update<T>(R.Qb, xj, R.slot(j), R.z.L, j, R.reorth ? 0 : 1, R.S, R.st);
  } else {
    op_apply_lz<T>(Q, xj, R.Qb, xp, R.S, j, R.k, R.st);
    if (!upd_in_reorth) launch_update<T>(R.Qb, xj, R.slot(j), R.z.L, j, R.reorth ? 0 : 1, R.S, R.st);
  }
  if (R.reorth) {
    launch_reorth<T>(R.V, R.z.L, j, R.part_h, R.h, R.m_max + 1, R.S, R.st, upd_in_reorth ? R.Qb : nullptr);
    if (lgcp_path(Q)) lgcp_col_init<T>(Q->plan, precond_mult(Q), R.slot(j), R.F1, R.k, R.st);
    else if (Q->precond) precond_dots<T>(Q->plan, precond_mult(Q), R.slot(j), R.band, R.S, R.k, R.st);
  }
  R.S.Pb = R.z.Pb;
}

// Iteration j of all groups, launches interleaved across the groups' streams.
template <typename T>
void iterate_all(std::vector<Run<T>>& Rs, int j, const std::vector<char>& live) {
  for (size_t g = 0; g < Rs.size(); ++g)
    if (live[g]) iterate<T>(Rs[g], j);
}

// Runs iterations of all groups (each on its own stream) until every column stopped or m_max, then closes
// the columns that hit m_max.  Groups whose columns all stopped launch no more.
// host_poll: host buffer of 2 x (columns) doubles for the stop polls (nullptr: the thread's pinned buffer).
template <typename T>
gmrf_status run_loop(std::vector<Run<T>>& Rs, const std::function<gmrf_status(int)>& on_done = nullptr,
                     double* host_poll = nullptr) {
  int ktot = 0;
  for (auto& R : Rs) ktot += R.k;
  double* ph = host_poll ? host_poll : poll_rho_buffer(2 * ktot);   // per group: k active flags, then k residuals
  if (!ph) return fail(GMRF_ENOMEM, "pinned host buffer allocation failed");
  std::vector<char> live(Rs.size(), 1);
  const int m_max = Rs[0].m_max;
  const bool predict = Rs[0].S.tol > 0.0;
  // Stop polls: every 8, 16, then 32 steps, or sooner where the residuals predict the last column's
  // stop.  rho_{j-1} of every column is read with the active flags; its geometric rate since the previous
  // poll (rho_0 = 1 before the first) gives each running column's remaining steps.  Polls only decide
  // when the host stops launching steps that every column would skip; results do not depend on them.
  std::vector<double> rho_prev((size_t)ktot, 1.0);
  int j_prev = 1, interval = 8, next_poll = 8;
  for (int j = 1; j <= m_max; ++j) {
    iterate_all<T>(Rs, j, live);
    if (j == next_poll && j < m_max) {
      HIP_TRY(hipGetLastError());
      int off = 0;
      for (size_t g = 0; g < Rs.size(); ++g) {
        if (live[g]) {
          launch_poll_gather(Rs[g].S, j, Rs[g].pollv, Rs[g].st);
          HIP_TRY(hipMemcpyAsync(ph + 2 * off, Rs[g].pollv, 2 * (size_t)Rs[g].k * sizeof(double),
                                 hipMemcpyDeviceToHost, Rs[g].st));
        }
        off += Rs[g].k;
      }
      bool any = false;
      double need = 0.0;   // steps until the slowest running column is predicted to stop (0: unknown)
      bool known = predict;
      off = 0;
      for (size_t g = 0; g < Rs.size(); ++g) {
        if (live[g]) {
          HIP_TRY(hipStreamSynchronize(Rs[g].st));
          bool a = false;
          const double* act = ph + 2 * off;
          const double* rh = act + Rs[g].k;
          for (int r = 0; r < Rs[g].k; ++r) {
            if (act[r] == 0.0) continue;
            a = true;
            if (!known) continue;
            const double rn = rh[r], rp = rho_prev[(size_t)(off + r)];
            if (!(rn > 0.0) || !(rp > rn) || !std::isfinite(rn)) {
              known = false;
              continue;
            }
            const double rate = std::log(rn / rp) / (double)(j - j_prev);
            need = std::max(need, std::log(Rs[g].S.tol / rn) / rate);
          }
          if (predict)
            for (int r = 0; r < Rs[g].k; ++r) rho_prev[(size_t)(off + r)] = rh[r];
          live[g] = a;
          if (!a) {
            // every column of this group has stopped: its closing work can overlap the other groups' steps
            launch_finalize(Rs[g].S, Rs[g].st);
            if (on_done) {
              gmrf_status e = on_done((int)g);
              if (e != GMRF_OK) return e;
            }
          }
        }
        any |= live[g] != 0;
        off += Rs[g].k;
      }
      if (!any) break;
      j_prev = j;
      interval = std::min(interval * 2, 32);
      int step = interval;
      if (known && need > 0.0) step = std::max(1, std::min(step, (int)std::ceil(need)));
      next_poll = j + step;
    }
  }
  for (size_t g = 0; g < Rs.size(); ++g) {
    if (!live[g]) continue;   // closed above
    launch_finalize(Rs[g].S, Rs[g].st);
    if (on_done) {
      gmrf_status e = on_done((int)g);
      if (e != GMRF_OK) return e;
    }
  }
  HIP_TRY(hipGetLastError());
  return GMRF_OK;
}

// Independent column groups of one call run side by side: with the preconditioned step the band
// kernel of one group (a few blocks, latency-bound) overlaps the streaming step kernel of the other.
// Column groups of a preconditioned call, each on its own stream (at least 4 columns per group).
#ifndef GMRF_PRECOND_GROUPS
#define GMRF_PRECOND_GROUPS 2
#endif
constexpr int kMaxGroups = 4;
static_assert(GMRF_PRECOND_GROUPS >= 1 && GMRF_PRECOND_GROUPS <= kMaxGroups, "column groups");
int groups_for(const gmrf_op* Q, int64_t k) {
  if (!Q->precond || lgcp_path(Q)) return 1;
  return (int)std::max<int64_t>(1, std::min<int64_t>(GMRF_PRECOND_GROUPS, k / 4));
}

// Side streams of the calling host thread on the current device (default priority, created once).
// Created on first use only: the process has few hardware queues, and streams beyond them share one, where
// work on one stream waits behind work on the other.
gmrf_status side_streams(hipStream_t* out, int count) {
  static thread_local std::map<int, std::vector<hipStream_t>> cache;
  if (count > kMaxGroups) return fail(GMRF_EINVAL, "at most %d side streams", kMaxGroups);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::vector<hipStream_t>& v = cache[dev];
  while ((int)v.size() < count) {
    hipStream_t x;
    HIP_TRY(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    v.push_back(x);
  }
  for (int i = 0; i < count; ++i) out[i] = v[(size_t)i];
  return GMRF_OK;
}

// Fork: the group streams start after the work already queued on `st`; join: `st` continues after
// everything queued on the group streams.
struct ForkJoin {
  hipStream_t st;
  std::vector<hipStream_t> gs;
  gmrf_status fork(hipStream_t s, int G) {
    st = s;
    gs.assign(G, s);
    if (G == 1) return GMRF_OK;
    gmrf_status e = side_streams(gs.data(), G);
    if (e != GMRF_OK) return e;
    hipEvent_t ev;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(ev, st));
    for (auto g : gs) HIP_TRY(hipStreamWaitEvent(g, ev, 0));
    HIP_TRY(hipEventDestroy(ev));
    return GMRF_OK;
  }
  gmrf_status join() {
    if (gs.size() <= 1) return GMRF_OK;
    for (auto g : gs) {
      hipEvent_t ev;
      HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      HIP_TRY(hipEventRecord(ev, g));
      HIP_TRY(hipStreamWaitEvent(st, ev, 0));
      HIP_TRY(hipEventDestroy(ev));
    }
    return GMRF_OK;
  }
};

}  // namespace

// slot 0 <- z (preconditioned: z in the unitary spectral basis, with what the first step needs)
template <typename T>
static void init_from_z(Run<T>& R, const double* Zg) {
  const gmrf_op* Q = R.Q;
  if (Q->precond) {
    fft_forward_init<T>(Q->plan, Zg, R.slot(0), R.F1, R.S, R.k, R.st);
    if (lgcp_path(Q)) lgcp_col_init<T>(Q->plan, precond_mult(Q), R.slot(0), R.F1, R.k, R.st);
    else precond_dots<T>(Q->plan, precond_mult(Q), R.slot(0), R.band, R.S, R.k, R.st);
  } else {
    launch_init_from_f64<T>(Zg, Q->n, R.z.L, R.slot(0), R.S, R.st);
    fused_init<T>(R);
  }
}

// slot 0 <- the start vector of the preconditioned solve: Lambda^{-1/2} F b (circulant, LGCP), L^{-1} b
// (incomplete Cholesky), b otherwise; the iterate is mapped back by the same output step as a sample.
template <typename T>
static void init_for_solve(Run<T>& R, const double* Bg) {
  const gmrf_op* Q = R.Q;
  if (Q->precond) {
    fft_forward_init_mult<T>(Q->plan, precond_mult(Q), Bg, R.slot(0), R.F1, R.S, R.k, R.st);
    if (lgcp_path(Q)) lgcp_col_init<T>(Q->plan, precond_mult(Q), R.slot(0), R.F1, R.k, R.st);
    else precond_dots<T>(Q->plan, precond_mult(Q), R.slot(0), R.band, R.S, R.k, R.st);
  } else if (Q->ic) {
    launch_init_from_f64<T>(Bg, Q->n, R.z.L, R.F1, R.S, R.st);
    launch_trsv<T, T>(Q->icd, false, R.F1, R.z.L, R.slot(0), R.z.L, nullptr, R.k, R.st);
    launch_norm_partials<T>(R.slot(0), R.z.L, R.S, R.st);
  } else {
    init_from_z<T>(R, Bg);
  }
}

// solve = false: samples x_m = ||z|| V_m T_m^{-1/2} e_1 (Algorithm 1); solve = true: the Lanczos form of the
// conjugate-gradient iterate x_m = ||b|| V_m T_m^{-1} e_1 for Q x = b, preconditioned the same way.
// arena (device, arena_cap bytes) non-null: every scratch buffer of the call is carved from it, the columns run
// as one group on the caller's stream and the stop polls read into host_poll (2 k doubles); nothing is allocated.
template <typename T>
static gmrf_status sample_impl(const gmrf_op* Q, const double* Z, int64_t k, double tol, int m_max, int reorth,
                               double* X, gmrf_info* info, double* alpha_out, double* beta_out,
                               hipStream_t st, bool solve = false, void* arena = nullptr, size_t arena_cap = 0,
                               double* host_poll = nullptr) {
  const int G = arena ? 1 : groups_for(Q, k);
  ForkJoin fj;
  gmrf_status s = fj.fork(st, G);
  if (s != GMRF_OK) return s;
  std::vector<int64_t> c0(G + 1);
  for (int g = 0; g <= G; ++g) c0[g] = k * g / G;
  std::vector<std::unique_ptr<Workspace>> ws;
  std::vector<Run<T>> Rs(G);
  std::vector<double*> ys(G, nullptr), scrs(G, nullptr);
  for (int g = 0; g < G; ++g) {
    ws.emplace_back(arena ? new Workspace(fj.gs[g], arena, arena_cap) : new Workspace(fj.gs[g]));
    Run<T>& R = Rs[g];
    R.Q = Q;
    R.k = (int)(c0[g + 1] - c0[g]);
    R.m_max = m_max;
    R.reorth = reorth;
    R.tol = tol;
    R.st = fj.gs[g];
    if ((s = setup<T>(R, *ws[g])) != GMRF_OK) return s;
    // the closing buffers too: every buffer of the call is taken before its first kernel, so that a call
    // whose scratch does not fit (budget, reserved region, arena) is refused without running
    if ((s = ws[g]->alloc((size_t)R.k * m_max, &ys[g])) != GMRF_OK) return s;
    if (!solve && (s = ws[g]->alloc(tri_scratch_doubles(R.k, m_max), &scrs[g])) != GMRF_OK) return s;
  }
  for (int g = 0; g < G; ++g) {
    if (solve) init_for_solve<T>(Rs[g], Z + (size_t)c0[g] * Q->n);
    else init_from_z<T>(Rs[g], Z + (size_t)c0[g] * Q->n);
  }
  // y = T_m^{-1/2} e_1 (or T_m^{-1} e_1), then x_m = ||z|| V_m y, enqueued as soon as the group's columns stop
  auto close_group = [&](int g) -> gmrf_status {
    Run<T>& R = Rs[g];
    if (solve) {
      launch_tri_solve(R.S.alpha, m_max + 1, 1, R.S.beta, m_max + 2, 1, R.S.m_used, 0, R.S.status, ys[g], m_max,
                       R.S.status, R.k, R.st);
    } else {
      launch_tri_invsqrt(R.S.alpha, m_max + 1, 1, R.S.beta, m_max + 2, 1, R.S.m_used, 0, R.S.status, ys[g], m_max,
                         R.S.status, scrs[g], m_max, R.k, R.st);
    }
    double* Xg = X + (size_t)c0[g] * Q->n;
    if (Q->precond) {
      launch_combine<T, T>(R.V, R.z.L, ys[g], m_max, R.Qb, R.z.L, R.S, R.st);
      fft_backward_output<T>(Q->plan, precond_mult(Q), R.Qb, Xg, R.F1, R.S, R.k, R.st);
    } else if (Q->ic) {
      // x = L^{-T} u_m
      launch_combine<T, T>(R.V, R.z.L, ys[g], m_max, R.Qb, R.z.L, R.S, R.st);
      launch_trsv<T, double>(Q->icd, true, R.Qb, R.z.L, Xg, Q->n, nullptr, R.k, R.st);
    } else {
      launch_combine<T, double>(R.V, R.z.L, ys[g], m_max, Xg, Q->n, R.S, R.st);
    }
    return GMRF_OK;
  };
  if ((s = run_loop<T>(Rs, close_group, host_poll)) != GMRF_OK) return s;
  HIP_TRY(hipGetLastError());
  // results to host
  std::vector<int> mu(k), stt(k);
  std::vector<double> rho((size_t)k * (m_max + 1)), beta((size_t)k * (m_max + 2)), alpha;
  if (alpha_out) alpha.resize((size_t)k * (m_max + 1));
  for (int g = 0; g < G; ++g) {
    Run<T>& R = Rs[g];
    const size_t o = (size_t)c0[g];
    HIP_TRY(hipMemcpyAsync(mu.data() + o, R.S.m_used, R.k * sizeof(int), hipMemcpyDeviceToHost, R.st));
    HIP_TRY(hipMemcpyAsync(stt.data() + o, R.S.status, R.k * sizeof(int), hipMemcpyDeviceToHost, R.st));
    HIP_TRY(hipMemcpyAsync(rho.data() + o * (m_max + 1), R.S.rho, (size_t)R.k * (m_max + 1) * 8,
                           hipMemcpyDeviceToHost, R.st));
    HIP_TRY(hipMemcpyAsync(beta.data() + o * (m_max + 2), R.S.beta, (size_t)R.k * (m_max + 2) * 8,
                           hipMemcpyDeviceToHost, R.st));
    if (alpha_out)
      HIP_TRY(hipMemcpyAsync(alpha.data() + o * (m_max + 1), R.S.alpha, (size_t)R.k * (m_max + 1) * 8,
                             hipMemcpyDeviceToHost, R.st));
  }
  if ((s = fj.join()) != GMRF_OK) return s;
  for (int g = 0; g < G; ++g) HIP_TRY(hipStreamSynchronize(Rs[g].st));
  double lam_lb = NAN;
  if (Q->kind == 0 && !Q->precond && Q->kappa2 > 0.0)
    lam_lb = Q->order == 1 ? Q->tau * Q->kappa2 : Q->tau * Q->kappa2 * Q->kappa2;
  gmrf_status ret = GMRF_OK;
  for (int r = 0; r < k; ++r) {
    const int m = mu[r];
    const double rr = rho[(size_t)r * (m_max + 1) + std::max(m, 0)];
    if (info) {
      info[r].m_used = m;
      info[r].status = stt[r];
      info[r].rel_residual = m > 0 ? rr : 0.0;
      // Theorem 1: ||x - x_m|| / ||z|| <= lambda_min^{-1/2} rho_m for a sample; ||x - x_m|| / ||b|| <= rho_m /
      // lambda_min for a solve
      info[r].err_bound = (m > 0 && std::isfinite(lam_lb)) ? (solve ? rr / lam_lb : rr / std::sqrt(lam_lb)) : NAN;
    }
    if (stt[r] == kENOTSPD) ret = GMRF_ENOTSPD;
    if (stt[r] == kEINVAL && ret == GMRF_OK) ret = GMRF_EINVAL;
    if (alpha_out)
      for (int j = 1; j <= m_max; ++j)
        alpha_out[(size_t)r * m_max + j - 1] = j <= m ? alpha[(size_t)r * (m_max + 1) + j] : 0.0;
    if (beta_out)
      for (int j = 0; j <= m_max; ++j)
        beta_out[(size_t)r * (m_max + 1) + j] = j <= m ? beta[(size_t)r * (m_max + 2) + j] : 0.0;
  }
  if (ret == GMRF_ENOTSPD) fail(ret, "at least one column is not positive definite (see info)");
  if (ret == GMRF_EINVAL) fail(ret, "at least one column of Z is not finite (see info)");
  return ret;
}

// Two passes over the recurrence, three Krylov slots (Section 1's O(n) storage): pass 1 runs the
// stopping rule and keeps only the coefficients; y = T_m^{-1/2} e_1; pass 2 runs the same launches from z
// again (bitwise the same vectors: every reduction has a fixed order) and adds beta_0 y_t v_{t+1} into
// the output as each vector appears.
template <typename T>
static gmrf_status sample_two_pass_impl(const gmrf_op* Q, const double* Z, int64_t k, double tol, int m_max,
                                        double* X, gmrf_info* info, hipStream_t st) {
  const int G = groups_for(Q, k);
  ForkJoin fj;
  gmrf_status s = fj.fork(st, G);
  if (s != GMRF_OK) return s;
  std::vector<int64_t> c0(G + 1);
  for (int g = 0; g <= G; ++g) c0[g] = k * g / G;
  std::vector<std::unique_ptr<Workspace>> ws;
  std::vector<Run<T>> Rs(G), R2s(G);
  std::vector<double*> ys(G);
  std::vector<T*> U(G, nullptr);
  for (int g = 0; g < G; ++g) {
    ws.emplace_back(new Workspace(fj.gs[g]));
    Run<T>& R = Rs[g];
    R.Q = Q;
    R.k = (int)(c0[g + 1] - c0[g]);
    R.m_max = m_max;
    R.reorth = 0;
    R.tol = tol;
    R.st = fj.gs[g];
    R.ring3 = true;
    if ((s = setup<T>(R, *ws[g])) != GMRF_OK) return s;
    init_from_z<T>(R, Z + (size_t)c0[g] * Q->n);
  }
  if ((s = run_loop<T>(Rs)) != GMRF_OK) return s;
  for (int g = 0; g < G; ++g) {
    Run<T>& R = Rs[g];
    double* scr;
    if ((s = ws[g]->alloc((size_t)R.k * m_max, &ys[g])) != GMRF_OK) return s;
    if ((s = ws[g]->alloc(tri_scratch_doubles(R.k, m_max), &scr)) != GMRF_OK) return s;
    launch_tri_invsqrt(R.S.alpha, m_max + 1, 1, R.S.beta, m_max + 2, 1, R.S.m_used, 0, R.S.status, ys[g], m_max,
                       R.S.status, scr, m_max, R.k, R.st);
  }
  std::vector<int> mu(k), stt(k);
  std::vector<double> rho((size_t)k * (m_max + 1));
  for (int g = 0; g < G; ++g) {
    Run<T>& R = Rs[g];
    const size_t o = (size_t)c0[g];
    HIP_TRY(hipMemcpyAsync(mu.data() + o, R.S.m_used, R.k * sizeof(int), hipMemcpyDeviceToHost, R.st));
    HIP_TRY(hipMemcpyAsync(stt.data() + o, R.S.status, R.k * sizeof(int), hipMemcpyDeviceToHost, R.st));
    HIP_TRY(hipMemcpyAsync(rho.data() + o * (m_max + 1), R.S.rho, (size_t)R.k * (m_max + 1) * 8,
                           hipMemcpyDeviceToHost, R.st));
  }
  for (int g = 0; g < G; ++g) HIP_TRY(hipStreamSynchronize(Rs[g].st));
  // pass 2: the same vector buffers, fresh scalars
  for (int g = 0; g < G; ++g) {
    Run<T>& R1 = Rs[g];
    Run<T>& R = R2s[g];
    R = R1;
    if ((s = setup_state<T>(R, *ws[g])) != GMRF_OK) return s;
    const bool via_u = Q->precond || Q->ic;   // accumulate u_m, then map it to x
    if (via_u && (s = ws[g]->alloc((size_t)R.k * R.z.L, &U[g])) != GMRF_OK) return s;
    int mg = 0;
    for (int r = 0; r < R.k; ++r) mg = std::max(mg, mu[(size_t)c0[g] + r]);
    double* Xg = X + (size_t)c0[g] * Q->n;
    init_from_z<T>(R, Z + (size_t)c0[g] * Q->n);
    auto acc = [&](int t) {
      if (via_u) launch_accumulate<T, T>(R.slot(t), R.z.L, ys[g], m_max, R1.S, t, U[g], R.z.L, R.st);
      else launch_accumulate<T, double>(R.slot(t), R.z.L, ys[g], m_max, R1.S, t, Xg, Q->n, R.st);
    };
    acc(0);
    for (int j = 1; j < mg; ++j) {
      iterate<T>(R, j);
      acc(j);
    }
    if (Q->precond) fft_backward_output<T>(Q->plan, precond_mult(Q), U[g], Xg, R.F1, R1.S, R.k, R.st);
    if (Q->ic) launch_trsv<T, double>(Q->icd, true, U[g], R.z.L, Xg, Q->n, nullptr, R.k, R.st);
  }
  HIP_TRY(hipGetLastError());
  if ((s = fj.join()) != GMRF_OK) return s;
  for (int g = 0; g < G; ++g) HIP_TRY(hipStreamSynchronize(R2s[g].st));
  gmrf_status ret = GMRF_OK;
  for (int r = 0; r < k; ++r) {
    const int m = mu[r];
    if (info) {
      info[r].m_used = m;
      info[r].status = stt[r];
      info[r].rel_residual = m > 0 ? rho[(size_t)r * (m_max + 1) + m] : 0.0;
      info[r].err_bound = NAN;
    }
    if (stt[r] == kENOTSPD) ret = GMRF_ENOTSPD;
    if (stt[r] == kEINVAL && ret == GMRF_OK) ret = GMRF_EINVAL;
  }
  if (ret == GMRF_ENOTSPD) fail(ret, "at least one column is not positive definite (see info)");
  if (ret == GMRF_EINVAL) fail(ret, "at least one column of Z is not finite (see info)");
  return ret;
}

extern "C" gmrf_status gmrf_sample_two_pass(const gmrf_op* Q, const double* Z, int64_t k, double tol, int32_t m_max,
                                            double* X, gmrf_info* info, void* stream) {
  if (!Q || !Z || !X) return fail(GMRF_EINVAL, "NULL argument");
  if (k < 1 || k > 65535) return fail(GMRF_EINVAL, "k must be in 1..65535");
  if (m_max < 1 || m_max > tri_max_m()) return fail(GMRF_EINVAL, "m_max must be in 1..%d", tri_max_m());
  if (!std::isfinite(tol)) return fail(GMRF_EINVAL, "tol must be finite");
  if (Q->has_diag && !Q->precond)
    return fail(GMRF_EUNSUPPORTED, "Q + diag(d) is sampled with circulant preconditioning only (else pass it as CSR)");
  hipStream_t st = (hipStream_t)stream;
  if (Q->storage == GMRF_F64) return sample_two_pass_impl<double>(Q, Z, k, tol, m_max, X, info, st);
  return sample_two_pass_impl<float>(Q, Z, k, tol, m_max, X, info, st);
}

extern "C" gmrf_status gmrf_sample_ex(const gmrf_op* Q, const double* Z, int64_t k, double tol, int32_t m_max,
                                      int reorth, double* X, gmrf_info* info, double* alpha, double* beta,
                                      void* stream) {
  if (!Q || !Z || !X) return fail(GMRF_EINVAL, "NULL argument");
  if (k < 1 || k > 65535) return fail(GMRF_EINVAL, "k must be in 1..65535");
  if (m_max < 1 || m_max > tri_max_m()) return fail(GMRF_EINVAL, "m_max must be in 1..%d", tri_max_m());
  if (!std::isfinite(tol)) return fail(GMRF_EINVAL, "tol must be finite");
  if (reorth != 0 && reorth != 1) return fail(GMRF_EINVAL, "reorth must be 0 or 1");
  if (Q->has_diag && !Q->precond)
    return fail(GMRF_EUNSUPPORTED, "Q + diag(d) is sampled with circulant preconditioning only (else pass it as CSR)");
  hipStream_t st = (hipStream_t)stream;
  if (Q->storage == GMRF_F64) return sample_impl<double>(Q, Z, k, tol, m_max, reorth, X, info, alpha, beta, st);
  return sample_impl<float>(Q, Z, k, tol, m_max, reorth, X, info, alpha, beta, st);
}

extern "C" gmrf_status gmrf_solve(const gmrf_op* Q, const double* B, int64_t k, double tol, int32_t m_max, int reorth,
                                  double* X, gmrf_info* info, void* stream) {
  if (!Q || !B || !X) return fail(GMRF_EINVAL, "NULL argument");
  if (k < 1 || k > 65535) return fail(GMRF_EINVAL, "k must be in 1..65535");
  if (m_max < 1 || m_max > tri_max_m()) return fail(GMRF_EINVAL, "m_max must be in 1..%d", tri_max_m());
  if (!std::isfinite(tol)) return fail(GMRF_EINVAL, "tol must be finite");
  if (reorth != 0 && reorth != 1) return fail(GMRF_EINVAL, "reorth must be 0 or 1");
  if (Q->has_diag && !Q->precond)
    return fail(GMRF_EUNSUPPORTED, "Q + diag(d) is solved with circulant preconditioning only (else pass it as CSR)");
  hipStream_t st = (hipStream_t)stream;
  if (Q->storage == GMRF_F64)
    return sample_impl<double>(Q, B, k, tol, m_max, reorth, X, info, nullptr, nullptr, st, true);
  return sample_impl<float>(Q, B, k, tol, m_max, reorth, X, info, nullptr, nullptr, st, true);
}

extern "C" gmrf_status gmrf_sample(const gmrf_op* Q, const double* Z, int64_t k, double tol, int32_t m_max,
                                   int reorth, double* X, gmrf_info* info, void* stream) {
  return gmrf_sample_ex(Q, Z, k, tol, m_max, reorth, X, info, nullptr, nullptr, stream);
}

// ---- allocation-free sampling -----------------------------------------------------------------------------------
// Every scratch buffer of gmrf_sample_noalloc lives in one static device array per GPU.  In host code the name
// `scratch` is only a host-side stand-in for the symbol: its device address (its own on every GPU) is taken once
// per device with hipGetSymbolAddress, and only that address reaches kernels, memsets and copies.
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
constexpr int kNoAllocMaxK = 256;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;                   // guards the address table and serialises the calls of the process
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call there); caller holds g_scratch_mu.
gmrf_status static_scratch(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GMRF_EDEVICE, "device ordinal %d out of range", dev);
  if (!g_scratch_addr[dev]) {
    gmrf_status ds = check_device();
    if (ds != GMRF_OK) return ds;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(GMRF_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return GMRF_OK;
}
}  // namespace

extern "C" gmrf_status gmrf_sample_noalloc(const gmrf_op* Q, const double* Z, int64_t k, double tol, int32_t m_max,
                                           int reorth, double* X, gmrf_info* info, void* stream) {
  if (!Q || !Z || !X) return fail(GMRF_EINVAL, "NULL argument");
  if (k < 1 || k > kNoAllocMaxK) return fail(GMRF_EINVAL, "k must be in 1..%d", kNoAllocMaxK);
  if (m_max < 1 || m_max > tri_max_m()) return fail(GMRF_EINVAL, "m_max must be in 1..%d", tri_max_m());
  if (!std::isfinite(tol)) return fail(GMRF_EINVAL, "tol must be finite");
  if (reorth != 0 && reorth != 1) return fail(GMRF_EINVAL, "reorth must be 0 or 1");
  if (Q->has_diag && !Q->precond)
    return fail(GMRF_EUNSUPPORTED, "Q + diag(d) is sampled with circulant preconditioning only (else pass it as CSR)");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  void* base = nullptr;
  gmrf_status s = static_scratch(&base);
  if (s != GMRF_OK) return s;
  double poll[2 * kNoAllocMaxK];
  hipStream_t st = (hipStream_t)stream;
  s = Q->storage == GMRF_F64
          ? sample_impl<double>(Q, Z, k, tol, m_max, reorth, X, info, nullptr, nullptr, st, false, base,
                                kStaticScratchBytes, poll)
          : sample_impl<float>(Q, Z, k, tol, m_max, reorth, X, info, nullptr, nullptr, st, false, base,
                               kStaticScratchBytes, poll);
  // a refused or failed call may have queued memsets into the array: let them finish before the next caller
  if (s != GMRF_OK && s != GMRF_ENOTSPD && s != GMRF_EINVAL) (void)hipStreamSynchronize(st);
  return s;
}

// ---- log-determinant ------------------------------------------------------------------------------------
// np probes; with a colouring (device, K classes) every probe runs as K columns, one per class
// (Section 6.1), and the aggregate sums each probe's K quadratures.
template <typename T>
static gmrf_status logdet_impl(const gmrf_op* Q, int np, int m, uint64_t seed, const int8_t* probes,
                               const int32_t* colour, int K, double* logdet, double* std_err, double* per_probe,
                               hipStream_t st) {
  const int ncol = np * K;
  const int G = groups_for(Q, ncol);
  ForkJoin fj;
  gmrf_status s = fj.fork(st, G);
  if (s != GMRF_OK) return s;
  std::vector<int> c0(G + 1);
  for (int g = 0; g <= G; ++g) c0[g] = (int)((int64_t)ncol * g / G);
  std::vector<std::unique_ptr<Workspace>> ws;
  std::vector<Run<T>> Rs(G);
  for (int g = 0; g < G; ++g) {
    ws.emplace_back(new Workspace(fj.gs[g]));
    Run<T>& R = Rs[g];
    R.Q = Q;
    R.k = c0[g + 1] - c0[g];
    R.m_max = m;
    R.reorth = 0;
    R.tol = 0.0;
    R.st = fj.gs[g];
    R.ring3 = true;
    if ((s = setup<T>(R, *ws[g])) != GMRF_OK) return s;
    const int8_t* pg = probes ? probes + (size_t)c0[g] * Q->n : nullptr;
    if (Q->precond) {
      // probes in real space, then into the spectral basis
      T* pr;
      if ((s = ws[g]->alloc((size_t)R.k * Q->n, &pr)) != GMRF_OK) return s;
      fft_forward_init_probes<T>(Q->plan, seed, c0[g], pg, pr, R.slot(0), R.F1, R.S, R.k, R.st, colour, K);
      if (lgcp_path(Q)) lgcp_col_init<T>(Q->plan, precond_mult(Q), R.slot(0), R.F1, R.k, R.st);
      else precond_dots<T>(Q->plan, precond_mult(Q), R.slot(0), R.band, R.S, R.k, R.st);
    } else if (pg) {
      launch_init_from_i8<T>(pg, R.z.L, R.slot(0), R.S, R.st);
    } else {
      LzState S2 = R.S;
      S2.Pb = rademacher_blocks(R.z.L);
      launch_init_rademacher<T>(seed, R.z.L, c0[g], R.slot(0), S2, R.st, colour, K);
      R.pb_first = S2.Pb;  // opener of iteration 1 reduces the probe partials
    }
    if (!Q->precond) fused_init<T>(R);
  }
  const std::vector<char> live(G, 1);
  for (int j = 1; j <= m; ++j) iterate_all<T>(Rs, j, live);
  // per-column quadrature e_1^T log(T_m) e_1 and ||v||^2 = beta_0^2, gathered for the aggregate
  double *g_all, *b0_all;
  if ((s = ws[0]->alloc((size_t)ncol + 2 + np, &g_all)) != GMRF_OK) return s;
  if ((s = ws[0]->alloc((size_t)ncol, &b0_all)) != GMRF_OK) return s;
  for (int g = 0; g < G; ++g) {
    Run<T>& R = Rs[g];
    launch_finalize(R.S, R.st);
    launch_tri_log(R.S.alpha, m + 1, 1, R.S.beta, m + 2, 1, R.S.m_used, 0, R.S.status, g_all + c0[g], 1,
                   R.S.status, R.k, R.st);
    HIP_TRY(hipMemcpy2DAsync(b0_all + c0[g], sizeof(double), R.S.beta, (size_t)(m + 2) * sizeof(double),
                             sizeof(double), R.k, hipMemcpyDeviceToDevice, R.st));
  }
  if ((s = fj.join()) != GMRF_OK) return s;
  double* agg = g_all + ncol;
  const double shift = Q->precond ? Q->logdet_M : Q->ic ? Q->ic_logdet : 0.0;   // log det M (Section 6.2)
  launch_hutchinson_aggregate(g_all, b0_all, 1, np, K, shift, agg, st);
  HIP_TRY(hipGetLastError());
  std::vector<double> gam(np), out(2);
  std::vector<int> stt(ncol);
  HIP_TRY(hipMemcpyAsync(gam.data(), agg + 2, np * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(out.data(), agg, 16, hipMemcpyDeviceToHost, st));
  for (int g = 0; g < G; ++g)
    HIP_TRY(hipMemcpyAsync(stt.data() + c0[g], Rs[g].S.status, Rs[g].k * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int q = 0; q < ncol; ++q)
    if (stt[q] == kENOTSPD) return fail(GMRF_ENOTSPD, "probe %d: operator is not positive definite", q / K);
  if (logdet) *logdet = out[0];
  if (std_err) *std_err = out[1];
  if (per_probe) std::memcpy(per_probe, gam.data(), np * sizeof(double));
  return GMRF_OK;
}

extern "C" gmrf_status gmrf_logdet(const gmrf_op* Q, int32_t n_probes, int32_t m, uint64_t seed,
                                   const int8_t* probes, double* logdet, double* std_err, double* per_probe,
                                   void* stream) {
  if (!Q) return fail(GMRF_EINVAL, "NULL operator");
  if (n_probes < 1 || n_probes > 65535) return fail(GMRF_EINVAL, "n_probes must be in 1..65535");
  if (m < 1 || m > tri_max_m()) return fail(GMRF_EINVAL, "m must be in 1..%d", tri_max_m());
  if (Q->has_diag && !Q->precond)
    return fail(GMRF_EUNSUPPORTED, "Q + diag(d) is handled with circulant preconditioning only (else pass it as CSR)");
  hipStream_t st = (hipStream_t)stream;
  if (Q->storage == GMRF_F64)
    return logdet_impl<double>(Q, n_probes, m, seed, probes, nullptr, 1, logdet, std_err, per_probe, st);
  return logdet_impl<float>(Q, n_probes, m, seed, probes, nullptr, 1, logdet, std_err, per_probe, st);
}

extern "C" gmrf_status gmrf_logdet_coloured(const gmrf_op* Q, int32_t n_probes, int32_t m, uint64_t seed,
                                            const int32_t* colour, int32_t n_colours, double* logdet,
                                            double* std_err, double* per_probe, void* stream) {
  if (!Q || !colour) return fail(GMRF_EINVAL, "NULL argument");
  if (n_probes < 1 || n_colours < 1 || (int64_t)n_probes * n_colours > 65535)
    return fail(GMRF_EINVAL, "need n_probes >= 1, n_colours >= 1 and n_probes * n_colours <= 65535");
  if (m < 1 || m > tri_max_m()) return fail(GMRF_EINVAL, "m must be in 1..%d", tri_max_m());
  if (Q->has_diag && !Q->precond)
    return fail(GMRF_EUNSUPPORTED, "Q + diag(d) is handled with circulant preconditioning only (else pass it as CSR)");
  for (int64_t i = 0; i < Q->n; ++i)
    if (colour[i] < 0 || colour[i] >= n_colours)
      return fail(GMRF_EINVAL, "colour[%lld] = %d is outside 0..%d", (long long)i, colour[i], n_colours - 1);
  hipStream_t st = (hipStream_t)stream;
  Workspace ws(st);
  int32_t* dcol;
  gmrf_status s = ws.alloc((size_t)Q->n, &dcol);
  if (s != GMRF_OK) return s;
  HIP_TRY(hipMemcpyAsync(dcol, colour, (size_t)Q->n * sizeof(int32_t), hipMemcpyHostToDevice, st));
  if (Q->storage == GMRF_F64)
    return logdet_impl<double>(Q, n_probes, m, seed, nullptr, dcol, n_colours, logdet, std_err, per_probe, st);
  return logdet_impl<float>(Q, n_probes, m, seed, nullptr, dcol, n_colours, logdet, std_err, per_probe, st);
}

// Distance-p colouring (Section 6.1): first fit in node order, a node taking the smallest colour not
// used by an already coloured node within p steps of it in the graph of Q (the graph of Q^p).  Lattice
// handles: Q couples nodes within lattice (L1) distance `order`, so the neighbours are the nodes within
// L1 distance p * order (wrapped on periodic axes); CSR handles: breadth-first search to depth p.
extern "C" gmrf_status gmrf_distance_colouring(const gmrf_op* Q, int32_t p, int32_t* colour, int32_t* n_colours) {
  if (!Q || !colour || !n_colours || p < 0) return fail(GMRF_EINVAL, "bad arguments");
  const int64_t n = Q->n;
  std::vector<int32_t> col((size_t)n, -1);
  std::vector<uint8_t> used;
  int32_t K = 1;
  auto first_fit = [&](int64_t i, const std::vector<int64_t>& nb) {
    used.assign((size_t)K + 1, 0);
    for (int64_t j : nb)
      if (col[(size_t)j] >= 0) used[(size_t)col[(size_t)j]] = 1;
    int32_t c = 0;
    while (used[(size_t)c]) ++c;
    col[(size_t)i] = c;
    K = std::max(K, c + 1);
  };
  std::vector<int64_t> nb;
  if (p == 0) {
    std::fill(col.begin(), col.end(), 0);
  } else if (Q->kind == 0) {
    const int D = p * Q->order;
    const int64_t N0 = Q->shape[0], N1 = Q->shape[1], N2 = Q->shape[2];
    const bool per = Q->bc == GMRF_PERIODIC;
    // offsets of the L1 ball of radius D, per axis clipped to the lattice (a periodic axis reaches at
    // most its whole cycle)
    std::vector<std::array<int, 3>> off;
    for (int a = -D; a <= D; ++a)
      for (int b = -(D - std::abs(a)); b <= D - std::abs(a); ++b)
        for (int c = -(D - std::abs(a) - std::abs(b)); c <= D - std::abs(a) - std::abs(b); ++c)
          if (a || b || c) off.push_back({a, b, c});
    std::vector<int64_t> stamp((size_t)n, -1);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t i0 = i / (N1 * N2), i1 = (i / N2) % N1, i2 = i % N2;
      nb.clear();
      for (const auto& o : off) {
        int64_t j0 = i0 + o[0], j1 = i1 + o[1], j2 = i2 + o[2];
        if (per) {
          j0 = ((j0 % N0) + N0) % N0;
          j1 = ((j1 % N1) + N1) % N1;
          j2 = ((j2 % N2) + N2) % N2;
        } else if (j0 < 0 || j0 >= N0 || j1 < 0 || j1 >= N1 || j2 < 0 || j2 >= N2) {
          continue;
        }
        const int64_t j = (j0 * N1 + j1) * N2 + j2;
        if (j != i && stamp[(size_t)j] != i) {
          stamp[(size_t)j] = i;
          nb.push_back(j);
        }
      }
      first_fit(i, nb);
    }
  } else {
    std::vector<int64_t> stamp((size_t)n, -1), frontier, next;
    for (int64_t i = 0; i < n; ++i) {
      nb.clear();
      frontier.assign(1, i);
      stamp[(size_t)i] = i;
      for (int d = 0; d < p && !frontier.empty(); ++d) {
        next.clear();
        for (int64_t u : frontier)
          for (int64_t e = Q->h_rp[(size_t)u]; e < Q->h_rp[(size_t)u + 1]; ++e) {
            const int64_t v = Q->h_ci[(size_t)e];
            if (stamp[(size_t)v] != i) {
              stamp[(size_t)v] = i;
              next.push_back(v);
              nb.push_back(v);
            }
          }
        frontier.swap(next);
      }
      first_fit(i, nb);
    }
  }
  std::memcpy(colour, col.data(), (size_t)n * sizeof(int32_t));
  *n_colours = K;
  return GMRF_OK;
}

extern "C" gmrf_status gmrf_rademacher(uint64_t seed, int64_t n, int32_t n_probes, int8_t* out, void* stream) {
  if (n < 1 || n_probes < 1 || n_probes > 65535 || !out) return fail(GMRF_EINVAL, "bad arguments");
  gmrf_status ds = check_device();
  if (ds != GMRF_OK) return ds;
  launch_rademacher_i8(seed, (long)n, n_probes, out, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return GMRF_OK;
}

extern "C" gmrf_status gmrf_tridiag_invsqrt_e1(const double* alpha, const double* beta, const int32_t* m,
                                               int32_t k, int32_t ld, double* y, int32_t* status,
                                               void* stream) {
  if (!alpha || !beta || !m || !y || k < 1 || k > 65535 || ld < 1 || ld > tri_max_m())
    return fail(GMRF_EINVAL, "bad arguments (ld must be <= %d)", tri_max_m());
  hipStream_t st = (hipStream_t)stream;
  Workspace ws(st);
  double* scr;
  gmrf_status s = ws.alloc(tri_scratch_doubles(k, ld), &scr);
  if (s != GMRF_OK) return s;
  launch_tri_invsqrt(alpha, ld, 0, beta, ld, 0, m, 0, nullptr, y, ld, status, scr, ld, k, st);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return GMRF_OK;
}

extern "C" gmrf_status gmrf_tridiag_log_e1(const double* alpha, const double* beta, const int32_t* m,
                                           int32_t k, int32_t ld, double* out, int32_t* status,
                                           void* stream) {
  if (!alpha || !beta || !m || !out || k < 1 || k > 65535 || ld < 1 || ld > tri_max_m())
    return fail(GMRF_EINVAL, "bad arguments (ld must be <= %d)", tri_max_m());
  launch_tri_log(alpha, ld, 0, beta, ld, 0, m, 0, nullptr, out, 1, status, k, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return GMRF_OK;
}

// ---- single-kernel timing (for the roofline of the step's dominant kernels) ----------------------------
// which: 0 = lattice/CSR operator Y = Q X (SpMM over k columns, storage dtype)
//        1 = step kernel of the preconditioned step (writes w_j and its dot products)
//        2 = dot-product kernel of the preconditioned step (reads one vector)
//        3 = update w = q - alpha v (unpreconditioned path)
//        4 = band kernel of the preconditioned step
// Buffers are allocated and filled (Krylov slots with seeded +-1 values, scratch with zeros) before the
// first event; `reps` launches run between two HIP events recorded on `stream`.  bytes = algorithmic bytes of one launch (each input read once, each
// output written once; the small hand-off tables between the kernels of a step are not counted).
template <typename T>
static gmrf_status kernel_bench_impl(const gmrf_op* Q, int which, int k, int reps, double* avg_us, double* bytes,
                                     hipStream_t st, int tune = -1) {
  Workspace ws(st);
  Run<T> R;
  R.Q = Q;
  R.k = k;
  R.m_max = 4;
  R.reorth = 0;
  R.tol = 0.0;
  R.st = st;
  gmrf_status s = setup<T>(R, ws);
  if (s != GMRF_OK) return s;
  // seeded +-1 vectors in every slot (representative bit patterns, unlike zero fill); then beta_j = 1 and
  // partial sums = 1: every column active, no stop decision triggers
  {
    LzState S2 = R.S;
    S2.Pb = rademacher_blocks(R.z.L);
    if (S2.Pb > R.z.pstride) return fail(GMRF_EDEVICE, "kernel bench: partial-sum stride too small");
    for (int s = 0; s < R.z.slots; ++s) launch_init_rademacher<T>(0x5eed + s, R.z.L, 0, R.slot(s), S2, st);
    std::vector<double> ones((size_t)k * (R.m_max + 2), 1.0);
    HIP_TRY(hipMemcpyAsync(R.S.beta, ones.data(), ones.size() * 8, hipMemcpyHostToDevice, st));
    std::vector<double> pones((size_t)k * R.z.pstride, 1.0);
    HIP_TRY(hipMemcpyAsync(R.S.part_b, pones.data(), pones.size() * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(R.S.part_a, pones.data(), pones.size() * 8, hipMemcpyHostToDevice, st));
    if (R.band) HIP_TRY(hipMemsetAsync(R.band, 0, precond_step_bytes(Q->plan, Q->storage, k), st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  R.S.Pb = R.pb_first;
  if (which == 7) {
    // the one-pass step at j = 2 closes iteration 1 first: alpha_1 = 1 keeps every column positive definite
    std::vector<double> aones((size_t)k * (R.m_max + 1), 1.0);
    HIP_TRY(hipMemcpyAsync(R.S.alpha, aones.data(), aones.size() * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  const size_t vb = (size_t)k * R.z.vec_bytes;
  std::function<void()> launch;
  double b = 0.0;
  const void* mult = Q->storage == GMRF_F64 ? (const void*)Q->mult64 : (const void*)Q->mult32;
  if (which == 0) {
    launch = [&]() { op_apply_plain<T>(Q, R.slot(0), R.Qb, k, st, tune); };
    b = 2.0 * vb + (Q->kind == 1 ? (double)Q->resident_bytes : 0.0);
  } else if (which == 7) {
    if (!R.fused) return fail(GMRF_EINVAL, "kernel 7 needs a 2D lattice without preconditioning or diagonal term");
    // step 2 from slots 1 and 0 into slot 2, reading partial-sum set 0 (seeded) and writing set 1
    const StencilGeom g = tuned_geom(kTuneKernelLanczos2d, Q, k, tune);
    launch = [&, g]() {
      launch_lanczos2d<T>(g, Q->order, 0, 0, R.slot(1), R.z.L, R.slot(2), R.slot(0), R.S, 2, k, R.ps[1][0],
                          R.ps[1][1], R.ps[1][2], st);
    };
    b = 3.0 * vb;   // read v_j, v_{j-1}; write w_j
  } else if (which == 1 || which == 2 || which == 4) {
    if (!Q->precond || lgcp_path(Q))
      return fail(GMRF_EINVAL, "kernel %d needs circulant preconditioning without a diagonal term", which);
    if (which == 1) {
      launch = [&]() {
        precond_lanczos_step<T>(Q->plan, Q->geom, Q->order, mult, R.slot(1), R.slot(0), R.slot(2), R.band, R.S, 2, 1,
                                1, k, st, 2);
      };
      b = 3.0 * vb;   // read v_j, v_{j-1}; write w_j
    } else if (which == 2) {
      launch = [&]() {
        precond_lanczos_step<T>(Q->plan, Q->geom, Q->order, mult, R.slot(0), R.slot(0), R.slot(1), R.band, R.S, 1, 1,
                                1, k, st, 0);
      };
      b = 1.0 * vb;   // read one vector (writes only the dot partial sums)
    } else {
      launch = [&]() {
        precond_lanczos_step<T>(Q->plan, Q->geom, Q->order, mult, R.slot(0), R.slot(0), R.slot(1), R.band, R.S, 1, 1,
                                1, k, st, 1);
      };
      b = 0.0;
    }
  } else if (which == 3) {
    launch = [&]() { launch_update<T>(R.Qb, R.slot(0), R.slot(1), R.z.L, 1, 1, R.S, st); };
    b = 3.0 * vb;
  } else if (which == 5 || which == 6) {
    if (!lgcp_path(Q)) return fail(GMRF_EINVAL, "kernel %d needs a diagonal term and circulant preconditioning", which);
    // the row pass opens iteration 1 (no stop decision on the seeded sums); the column pass runs as step 2 so
    // that it reads v_{j-1}
    const int only = which == 5 ? 1 : 2, jj = which == 5 ? 1 : 2;
    HIP_TRY(hipMemsetAsync(R.F1, 0, vb, st));
    HIP_TRY(hipMemsetAsync(R.Qb, 0, vb, st));
    launch = [&, only, jj]() {
      lgcp_lanczos_step<T>(Q->plan, mult, (const T*)diag_of(Q), R.F1, R.Qb, R.slot(1), R.slot(0), R.slot(2), R.S,
                           jj, 1, k, st, only);
    };
    // row pass: read T1, write T2, read the diagonal once; column pass: read T2, v_j, v_{j-1}, write w_j, T1
    b = which == 5 ? 2.0 * vb + (double)R.z.vec_bytes : 5.0 * vb;
  } else {
    return fail(GMRF_EINVAL, "unknown kernel id %d", which);
  }
  for (int i = 0; i < 3; ++i) launch();
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, st));
  for (int i = 0; i < reps; ++i) launch();
  HIP_TRY(hipEventRecord(e1, st));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(hipGetLastError());
  *avg_us = 1000.0 * ms / reps;
  *bytes = b;
  return GMRF_OK;
}

extern "C" gmrf_status gmrf_kernel_bench(const gmrf_op* Q, int which, int64_t k, int32_t reps, double* avg_us,
                                         double* bytes, void* stream) {
  if (!Q || !avg_us || !bytes || k < 1 || k > 65535 || reps < 1) return fail(GMRF_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  if (Q->storage == GMRF_F64) return kernel_bench_impl<double>(Q, which, (int)k, reps, avg_us, bytes, st);
  return kernel_bench_impl<float>(Q, which, (int)k, reps, avg_us, bytes, st);
}

// ---- autotuner -----------------------------------------------------------------------------------------------
// Times every candidate option set of the tunable kernels that calls on Q with k columns launch (the 2D operator's
// SpMM; the one-pass Lanczos step where the operator takes it) with `reps` launches between HIP events on scratch
// data of that shape, and records the fastest (ties: the earlier candidate) in the table.
template <typename T>
static gmrf_status autotune_impl(const gmrf_op* Q, int k, int reps, int32_t* chosen, hipStream_t st) {
  const int kernels[kTuneKernels] = {kTuneKernelSpmm, kTuneKernelLanczos2d};
  const int which[kTuneKernels] = {0, 7};
  for (int t = 0; t < kTuneKernels; ++t) {
    if (t == 1 && !fused_path(Q, 0)) {
      if (chosen) chosen[t] = -1;
      continue;
    }
    // candidates: the four option sets, and for the operator kernel each with every tile shape that suits the
    // operator (rows per wave 8 / 16 / 32 or the rule, columns per lane 1 / 2 / 4 or the rule)
    std::vector<int> cand;
    for (int c = 0; c < 4; ++c) {
      if (kernels[t] != kTuneKernelSpmm) {
        cand.push_back(kTuneCandidates[c]);
        continue;
      }
      for (int bc = 0; bc < 4; ++bc)
        for (int ec = 0; ec < 4; ++ec) {
          const int bits = kTuneCandidates[c] | (bc << kTuneBandShift) | (ec << kTuneEplShift);
          int band, epl;
          geom_code(Q, bits, band, epl);
          if (ec != 0 && epl == 0) continue;   // a lane width the operator cannot take
          cand.push_back(bits);
        }
    }
    int best = 0;
    double best_us = 0.0;
    for (size_t c = 0; c < cand.size(); ++c) {
      double us = 0.0, b = 0.0;
      gmrf_status s = kernel_bench_impl<T>(Q, which[t], k, reps, &us, &b, st, cand[c]);
      if (s != GMRF_OK) return s;
      if (c == 0 || us < best_us) {
        best = cand[c];
        best_us = us;
      }
    }
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      tune_table()[tune_key(kernels[t], Q, k)] = best;
    }
    if (chosen) chosen[t] = best;
  }
  return GMRF_OK;
}

extern "C" gmrf_status gmrf_autotune(const gmrf_op* Q, int64_t k, int32_t reps, int32_t* chosen, void* stream) {
  if (!Q || k < 1 || k > 65535 || reps < 1) return fail(GMRF_EINVAL, "bad arguments");
  if (!tunable(Q)) {
    if (chosen) chosen[0] = chosen[1] = -1;
    return GMRF_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  if (Q->storage == GMRF_F64) return autotune_impl<double>(Q, (int)k, reps, chosen, st);
  return autotune_impl<float>(Q, (int)k, reps, chosen, st);
}

extern "C" gmrf_status gmrf_tune_export(int32_t* entries, int32_t cap, int32_t* count) {
  if (!count || cap < 0 || (cap > 0 && !entries)) return fail(GMRF_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  *count = (int32_t)tune_table().size();
  int i = 0;
  for (const auto& kv : tune_table()) {
    if (i >= cap) break;
    const TuneKey& q = kv.first;
    const int32_t e[7] = {q.kernel, q.order, q.storage, q.c1, q.c2, q.ck, kv.second};
    std::memcpy(entries + 7 * i, e, sizeof(e));
    ++i;
  }
  return GMRF_OK;
}

extern "C" gmrf_status gmrf_tune_import(const int32_t* entries, int32_t count) {
  if (count < 0 || (count > 0 && !entries)) return fail(GMRF_EINVAL, "bad arguments");
  for (int i = 0; i < count; ++i) {
    const int32_t* e = entries + 7 * i;
    const int allowed = kTuneXcd | kTuneNtStore | (e[0] == kTuneKernelSpmm ? kTuneGeomMask : 0);
    if (e[0] < 0 || e[0] >= kTuneKernels || (e[1] != 1 && e[1] != 2) || (e[2] != GMRF_F64 && e[2] != GMRF_F32) ||
        e[3] < 0 || e[3] > 31 || e[4] < 0 || e[4] > 31 || e[5] < 0 || e[5] > 31 || (e[6] & ~allowed) != 0)
      return fail(GMRF_EINVAL, "tuning entry %d is not valid", i);
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (int i = 0; i < count; ++i) {
    const int32_t* e = entries + 7 * i;
    tune_table()[TuneKey{e[0], e[1], e[2], e[3], e[4], e[5]}] = e[6];
  }
  return GMRF_OK;
}

extern "C" gmrf_status gmrf_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_table().clear();
  return GMRF_OK;
}

// ---- achievable HBM bandwidth --------------------------------------------------------------------------------------
extern "C" gmrf_status gmrf_bandwidth_bench(int which, size_t bytes, int32_t blocks, int32_t reps, double* gbs,
                                            double* avg_us, void* stream) {
  if (which < 0 || which > 2 || bytes < ((size_t)1 << 20) || bytes % 16 != 0 || blocks < 0 || reps < 1 || !gbs ||
      !avg_us)
    return fail(GMRF_EINVAL, "bad arguments");
  gmrf_status ds = check_device();
  if (ds != GMRF_OK) return ds;
  hipStream_t st = (hipStream_t)stream;
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int nb = blocks > 0 ? blocks : 32 * cus;
  void *a = nullptr, *b = nullptr, *c = nullptr;
  float* out = nullptr;
  gmrf_status s = GMRF_OK;
  auto release = [&]() {
    (void)hipStreamSynchronize(st);
    for (void* p : {a, b, c, (void*)out})
      if (p) (void)hipFree(p);
  };
  if (hipMalloc(&a, bytes) != hipSuccess || (which >= 1 && hipMalloc(&b, bytes) != hipSuccess) ||
      (which == 2 && hipMalloc(&c, bytes) != hipSuccess) || hipMalloc(&out, (size_t)nb * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    release();
    return fail(GMRF_ENOMEM, "bandwidth bench: hipMalloc of %zu B failed", bytes);
  }
  for (void* p : {a, b, c})
    if (p && hipMemsetAsync(p, 0, bytes, st) != hipSuccess) s = fail(GMRF_EDEVICE, "hipMemsetAsync failed");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (s == GMRF_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    s = fail(GMRF_EDEVICE, "hipEventCreate failed");
  float ms = 0.f;
  if (s == GMRF_OK) {
    const size_t n4 = bytes / 16;
    for (int i = 0; i < 2; ++i) launch_bandwidth(which, nb, a, b, c, out, n4, st);
    (void)hipEventRecord(e0, st);
    for (int i = 0; i < reps; ++i) launch_bandwidth(which, nb, a, b, c, out, n4, st);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
        hipGetLastError() != hipSuccess)
      s = fail(GMRF_EDEVICE, "bandwidth bench: launch or timing failed");
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  release();
  if (s != GMRF_OK) return s;
  *avg_us = 1000.0 * ms / reps;
  *gbs = (double)(which + 1) * (double)bytes / (*avg_us * 1e3);
  return GMRF_OK;
}

// ---- uneven batch: many fields, one set of launches per Lanczos step ----------------------------------
template <typename T>
static gmrf_status sample_batch_impl(int nf, const gmrf_op* const* ops, const int64_t* kf, const double* Z, double tol,
                                     int m_max, double* X, gmrf_info* info, hipStream_t st) {
  const gmrf_op* Q0 = ops[0];
  std::vector<int64_t> off, ext;   // column offsets inside a Krylov slot, and in the caller's Z and X
  std::vector<int> len, pa, pb, pbf, field;
  const bool fused = Q0->kind == 0 && Q0->dim == 2;   // one pass per step (k_lanczos2d)
  std::vector<StencilGeom> geom;
  int64_t tot = 0, tot_ext = 0;
  int max_tiles = 1;
  long max_len = 1;
  int big = 0;                 // the field with the most elements: its tuned store policy serves the batch's launches
  int64_t big_elems = 0;
  for (int f = 0; f < nf; ++f) {
    const gmrf_op* Q = ops[f];
    // inside the Krylov slots every column starts at an even offset, so that the 2D kernel's element
    // pairs (even row length) stay aligned: each field is then tiled as it is when sampled alone
    const StencilGeom gf = Q->geom;
    const int tiles = fused ? lanczos2d_blocks(gf) : stencil_blocks(gf);
    max_tiles = std::max(max_tiles, tiles);
    max_len = std::max<long>(max_len, (long)Q->n);
    if (Q->n * kf[f] > big_elems) {
      big_elems = Q->n * kf[f];
      big = f;
    }
    for (int64_t r = 0; r < kf[f]; ++r) {
      off.push_back(tot);
      ext.push_back(tot_ext);
      len.push_back((int)Q->n);
      pa.push_back(tiles);
      pb.push_back(ew_blocks((long)Q->n));     // the init kernel's (and the update kernel's) norm partials
      pbf.push_back(tiles);                    // the one-pass kernel's norm partials
      geom.push_back(gf);
      field.push_back(f);
      tot += (Q->n + 3) & ~(int64_t)3;         // column starts 16-byte aligned for the 2D kernels' vector loads
      tot_ext += Q->n;
    }
  }
  const int K = (int)off.size();
  Workspace ws(st);
  gmrf_status s;
  T *V, *Qb;
  if ((s = ws.alloc((size_t)(m_max + 1) * tot, &V)) != GMRF_OK) return s;
  if ((s = ws.alloc((size_t)tot, &Qb)) != GMRF_OK) return s;
  const int pstride = std::max(max_tiles, ew_blocks(max_len));
  double* dbuf;
  const size_t nd = (size_t)K * (m_max + 1) * 3 + (size_t)K * (m_max + 2) + 6 * (size_t)K * pstride;
  if ((s = ws.alloc(nd, &dbuf)) != GMRF_OK) return s;
  int* ibuf;
  if ((s = ws.alloc((size_t)7 * K, &ibuf)) != GMRF_OK) return s;
  int64_t* doff;
  if ((s = ws.alloc((size_t)2 * K, &doff)) != GMRF_OK) return s;
  int64_t* dext = doff + K;
  StencilGeom* dgeom;
  if ((s = ws.alloc((size_t)K, &dgeom)) != GMRF_OK) return s;
  LzState S{};
  S.k = K;
  S.m_max = m_max;
  S.tol = tol;
  S.alpha = dbuf;
  S.dpiv = S.alpha + (size_t)K * (m_max + 1);
  S.rho = S.dpiv + (size_t)K * (m_max + 1);
  S.beta = S.rho + (size_t)K * (m_max + 1);
  S.part_a = S.beta + (size_t)K * (m_max + 2);
  S.part_b = S.part_a + (size_t)K * pstride;
  S.part_c = S.part_b + (size_t)K * pstride;
  double* ps[2][3];
  for (int q = 0; q < 6; ++q) ps[q / 3][q % 3] = S.part_a + (size_t)q * K * pstride;
  S.m_used = ibuf;
  S.status = ibuf + K;
  S.active = ibuf + 2 * K;
  int* dlen = ibuf + 3 * K;
  int* dpa = ibuf + 4 * K;
  int* dpb = ibuf + 5 * K;
  int* dpbf = ibuf + 6 * K;
  S.Pa = max_tiles;
  S.Pb = ew_blocks(max_len);
  S.pstride = pstride;
  S.col_off = doff;
  S.col_ext = dext;
  S.col_len = dlen;
  S.col_pa = dpa;
  S.col_pb = dpb;
  S.col_geom = dgeom;
  S.slot_stride = tot;
  HIP_TRY(hipMemsetAsync(dbuf, 0, nd * sizeof(double), st));
  HIP_TRY(hipMemsetAsync(ibuf, 0, 2 * K * sizeof(int), st));
  HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)S.active, 1, K, st));
  HIP_TRY(hipMemcpyAsync(doff, off.data(), K * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(dext, ext.data(), K * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(dlen, len.data(), K * sizeof(int), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(dpa, pa.data(), K * sizeof(int), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(dpb, pb.data(), K * sizeof(int), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(dpbf, pbf.data(), K * sizeof(int), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(dgeom, geom.data(), K * sizeof(StencilGeom), hipMemcpyHostToDevice, st));
  auto slot = [&](int t) { return V + (size_t)t * tot; };
  // launch options of the batch's one-pass steps: the store policy tuned for its largest field (the work list
  // fixes the tile order); no option changes a result bit
  StencilGeom gbatch = Q0->geom;
  gbatch.tune = tune_lookup(kTuneKernelLanczos2d, ops[big], kf[big]) & kTuneNtStore;
  launch_init_from_f64<T>(Z, 0, max_len, slot(0), S, st);
  if (fused)
    launch_lanczos2d<T>(gbatch, Q0->order, 1, max_tiles, slot(0), 0, nullptr, nullptr, S, 0, K, ps[0][0], nullptr,
                        nullptr, st);
  int* pbuf = poll_buffer(K);
  if (!pbuf) return fail(GMRF_ENOMEM, "pinned host buffer allocation failed");
  // one-pass step: a flat list of (column, tile) over the columns still running, rebuilt at every poll,
  // so that the grid shrinks as columns stop instead of launching max_tiles blocks for every column
  std::vector<int2> work;
  int2* dwork = nullptr;
  int nwork = 0;
  auto build_work = [&](const int* act) -> gmrf_status {
    work.clear();
    for (int r = 0; r < K; ++r) {
      if (act && !act[r]) continue;
      for (int t = 0; t < pa[r]; ++t) work.push_back(make_int2(r, t));
    }
    nwork = (int)work.size();
    if (nwork) HIP_TRY(hipMemcpyAsync(dwork, work.data(), work.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    return GMRF_OK;
  };
  if (fused) {
    size_t cap = 0;
    for (int r = 0; r < K; ++r) cap += (size_t)pa[r];
    if ((s = ws.alloc(cap, &dwork)) != GMRF_OK) return s;
    if ((s = build_work(nullptr)) != GMRF_OK) return s;
    S.work = dwork;
  }
  int poll = 8;
  for (int j = 1; j <= m_max; ++j) {
    if (fused) {
      // S holds pass j - 1's partial sums (iteration 1: the init kernels' set 0); this pass writes the other set
      const int wset = j & 1;
      if (nwork)
        launch_lanczos2d<T>(gbatch, Q0->order, 0, nwork, slot(j - 1), 0, slot(j), j >= 2 ? slot(j - 2) : slot(0),
                            S, j, 1, ps[wset][0], ps[wset][1], ps[wset][2], st);
      S.part_a = ps[wset][0];
      S.part_b = ps[wset][1];
      S.part_c = ps[wset][2];
      S.col_pb = dpbf;
    } else {
      launch_stencil_batch<T>(Q0->order, Q0->dim, max_tiles, slot(j - 1), Qb, j >= 2 ? slot(j - 2) : slot(0), S, j,
                              st, Q0->geom.zc > 0);
      launch_update<T>(Qb, slot(j - 1), slot(j), max_len, j, 1, S, st);
    }
    if (j % poll == 0 && j < m_max) {
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(pbuf, S.active, K * sizeof(int), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      bool any = false;
      for (int r = 0; r < K; ++r) any |= pbuf[r] != 0;
      if (!any) break;
      if (fused && (s = build_work(pbuf)) != GMRF_OK) return s;
      poll = std::min(poll * 2, 32);
    }
  }
  S.work = nullptr;
  launch_finalize(S, st);
  double *y, *scr;
  if ((s = ws.alloc((size_t)K * m_max, &y)) != GMRF_OK) return s;
  if ((s = ws.alloc(tri_scratch_doubles(K, m_max), &scr)) != GMRF_OK) return s;
  launch_tri_invsqrt(S.alpha, m_max + 1, 1, S.beta, m_max + 2, 1, S.m_used, 0, S.status, y, m_max, S.status, scr,
                     m_max, K, st);
  launch_combine<T, double>(V, max_len, y, m_max, X, 0, S, st);
  HIP_TRY(hipGetLastError());
  std::vector<int> mu(K), stt(K);
  std::vector<double> rho((size_t)K * (m_max + 1));
  HIP_TRY(hipMemcpyAsync(mu.data(), S.m_used, K * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(stt.data(), S.status, K * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(rho.data(), S.rho, rho.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  gmrf_status ret = GMRF_OK;
  for (int r = 0; r < K; ++r) {
    const gmrf_op* Q = ops[field[r]];
    double lam_lb = NAN;
    if (Q->kappa2 > 0.0) lam_lb = Q->order == 1 ? Q->tau * Q->kappa2 : Q->tau * Q->kappa2 * Q->kappa2;
    const int m = mu[r];
    const double rr = rho[(size_t)r * (m_max + 1) + std::max(m, 0)];
    if (info) {
      info[r].m_used = m;
      info[r].status = stt[r];
      info[r].rel_residual = m > 0 ? rr : 0.0;
      info[r].err_bound = (m > 0 && std::isfinite(lam_lb)) ? rr / std::sqrt(lam_lb) : NAN;
    }
    if (stt[r] == kENOTSPD) ret = GMRF_ENOTSPD;
    if (stt[r] == kEINVAL && ret == GMRF_OK) ret = GMRF_EINVAL;
  }
  if (ret != GMRF_OK) fail(ret, "at least one column is not positive definite or not finite (see info)");
  return ret;
}

extern "C" gmrf_status gmrf_sample_batch(int32_t n_fields, const gmrf_op* const* ops, const int64_t* k,
                                         const double* Z, double tol, int32_t m_max, double* X, gmrf_info* info,
                                         void* stream) {
  if (n_fields < 1 || !ops || !k || !Z || !X) return fail(GMRF_EINVAL, "bad arguments");
  if (m_max < 1 || m_max > tri_max_m()) return fail(GMRF_EINVAL, "m_max must be in 1..%d", tri_max_m());
  if (!std::isfinite(tol)) return fail(GMRF_EINVAL, "tol must be finite");
  int64_t K = 0;
  for (int f = 0; f < n_fields; ++f) {
    const gmrf_op* Q = ops[f];
    if (!Q) return fail(GMRF_EINVAL, "field %d: NULL operator", f);
    if (Q->kind != 0 || Q->precond || Q->has_diag)
      return fail(GMRF_EUNSUPPORTED, "field %d: batches take lattice operators without preconditioning or diagonal", f);
    if (Q->ndim != ops[0]->ndim || Q->order != ops[0]->order || Q->storage != ops[0]->storage)
      return fail(GMRF_EINVAL, "field %d: all fields must share ndim, order and storage", f);
    if ((Q->geom.zc > 0) != (ops[0]->geom.zc > 0))
      return fail(GMRF_EUNSUPPORTED, "field %d: 3D first-order fields of one batch must all have their last "
                  "(contiguous) side <= 512, or all > 512", f);
    if (k[f] < 1) return fail(GMRF_EINVAL, "field %d: k must be >= 1", f);
    K += k[f];
  }
  if (K > 65535) return fail(GMRF_EINVAL, "at most 65535 columns per batch");
  hipStream_t st = (hipStream_t)stream;
  if (ops[0]->storage == GMRF_F64) return sample_batch_impl<double>(n_fields, ops, k, Z, tol, m_max, X, info, st);
  return sample_batch_impl<float>(n_fields, ops, k, Z, tol, m_max, X, info, st);
}
