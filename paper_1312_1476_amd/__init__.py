"""MI355X (gfx950) Krylov sampler and Lanczos log-determinant for Gaussian Markov random fields.

Simpson, Turner, Strickland & Pettitt, "Scalable iterative methods for sampling from massive
Gaussian random vectors" (arXiv 1312.1476): Algorithm 1 (Lanczos approximation of
Q^{-1/2} z), Proposition 1 with the block-circulant preconditioner of Section 5.1, and the
Hutchinson log-determinant with Lanczos quadrature of Section 6.

This module only marshals arguments to the C ABI of libgmrf.so (include/gmrf.h); every
step of the computation runs in the library's HIP kernels.  Device buffers are torch CUDA
(HIP) tensors; blocks of vectors are (k, n) tensors, row r being right-hand side r (the
column-major n x k block of the C ABI).
"""
import ctypes as C

import numpy as np

from . import _abi
from ._abi import GMRF_F32, GMRF_F64, GMRF_FREE, GMRF_PERIODIC, GmrfError, Info, check, lib

__all__ = ["Operator", "rademacher", "tridiag_invsqrt_e1", "tridiag_log_e1", "set_hbm_budget",
           "hbm_in_use", "kernel_bench", "bandwidth_bench", "autotune", "tune_table", "save_tune", "load_tune",
           "clear_tune", "sample_batch", "GmrfError", "STATUS"]

STATUS = _abi.STATUS_NAMES


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def _storage_code(storage):
    if storage in ("f64", "float64", GMRF_F64):
        return GMRF_F64
    if storage in ("f32", "float32", GMRF_F32):
        return GMRF_F32
    raise ValueError("storage must be 'f64' or 'f32'")


class Operator:
    """A device-resident precision operator (gmrf_op handle)."""

    def __init__(self, handle, n, storage, shape=None, order=None):
        self._h = handle
        self.n = int(n)
        self.storage = storage
        self.shape = shape          # lattice shape (None for CSR)
        self.order = order          # lattice order 1 or 2 (None for CSR)
        self.precond = False        # circulant or incomplete-Cholesky preconditioning enabled
        self.has_diag = False       # Q + diag(d)

    # -- construction ---------------------------------------------------------------------
    @classmethod
    def lattice(cls, shape, order=1, kappa2=1.0, tau=1.0, boundary="free", storage="f64"):
        shape = tuple(int(s) for s in shape)
        arr = (C.c_int64 * len(shape))(*shape)
        h = C.c_void_p()
        bc = GMRF_PERIODIC if boundary == "periodic" else GMRF_FREE
        sc = _storage_code(storage)
        check(lib().gmrf_op_create_lattice(len(shape), arr, int(order), float(kappa2), float(tau), bc, sc,
                                           C.byref(h)), "gmrf_op_create_lattice")
        return cls(h, int(np.prod(shape)), sc, shape, int(order))

    @classmethod
    def csr(cls, n, indptr, indices, data, storage="f64"):
        rp = np.ascontiguousarray(indptr, dtype=np.int64)
        ci = np.ascontiguousarray(indices, dtype=np.int32)
        va = np.ascontiguousarray(data, dtype=np.float64)
        h = C.c_void_p()
        sc = _storage_code(storage)
        check(lib().gmrf_op_create_csr(int(n), rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p),
                                       va.ctypes.data_as(C.c_void_p), sc, C.byref(h)), "gmrf_op_create_csr")
        return cls(h, n, sc)

    def set_diagonal(self, d):
        """Q <- Q + diag(d) (host array of n values; None removes the term).  With circulant
        preconditioning on a periodic 2D lattice the preconditioner stays M = Q."""
        if d is None:
            check(lib().gmrf_op_set_diagonal(self._h, None), "gmrf_op_set_diagonal")
            self.has_diag = False
            return self
        arr = np.ascontiguousarray(d, dtype=np.float64)
        if arr.shape != (self.n,):
            raise ValueError(f"diagonal must have shape ({self.n},)")
        check(lib().gmrf_op_set_diagonal(self._h, arr.ctypes.data_as(C.c_void_p)), "gmrf_op_set_diagonal")
        self.has_diag = True
        return self

    def set_ichol_precond(self, droptol=-1.0, enable=True):
        """Incomplete-Cholesky preconditioning of a CSR operator (droptol < 0: IC(0)); returns the
        diagonal shift the factorisation needed."""
        sh = C.c_double()
        check(lib().gmrf_op_set_ichol_precond(self._h, 1 if enable else 0, float(droptol), C.byref(sh)),
              "gmrf_op_set_ichol_precond")
        self.precond = bool(enable)
        return sh.value

    def ichol_info(self):
        """(nonzeros of L, forward-solve levels, diagonal shift) of the incomplete-Cholesky factor."""
        nnz, lev, sh = C.c_int64(), C.c_int32(), C.c_double()
        check(lib().gmrf_ichol_info(self._h, C.byref(nnz), C.byref(lev), C.byref(sh)), "gmrf_ichol_info")
        return nnz.value, lev.value, sh.value

    def set_circulant_precond(self, enable=True):
        check(lib().gmrf_op_set_circulant_precond(self._h, 1 if enable else 0), "gmrf_op_set_circulant_precond")
        self.precond = bool(enable)
        return self

    def close(self):
        if self._h is not None and self._h.value:
            lib().gmrf_op_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def torch_dtype(self):
        torch = _torch()
        return torch.float64 if self.storage == GMRF_F64 else torch.float32

    def bytes(self, k, m_max, reorth=False):
        """Device bytes of one sample call with a stored Krylov basis (and of the handle)."""
        out = C.c_size_t()
        check(lib().gmrf_op_bytes(self._h, int(k), int(m_max), int(bool(reorth)), C.byref(out)), "gmrf_op_bytes")
        return out.value

    def bytes_two_pass(self, k, m_max):
        """Device bytes of one two-pass sample call (three Krylov slots) and of the handle."""
        out = C.c_size_t()
        check(lib().gmrf_op_bytes_two_pass(self._h, int(k), int(m_max), C.byref(out)), "gmrf_op_bytes_two_pass")
        return out.value

    # -- kernels -----------------------------------------------------------------------------
    def _check_block(self, X, dtype, name):
        if X.dim() != 2 or X.shape[1] != self.n or not X.is_contiguous() or X.dtype != dtype or not X.is_cuda:
            raise ValueError(f"{name} must be a contiguous CUDA ({dtype}) tensor of shape (k, {self.n})")

    def apply(self, X, out=None, stream=None):
        """Y = Q X in the storage dtype (rows of X are vectors)."""
        torch = _torch()
        self._check_block(X, self.torch_dtype, "X")
        Y = out if out is not None else torch.empty_like(X)
        check(lib().gmrf_op_apply(self._h, _dptr(X), _dptr(Y), X.shape[0], _stream_ptr(stream)), "gmrf_op_apply")
        return Y

    def precond_apply(self, X, out=None, stream=None):
        """Y = M^{-1/2} X (circulant preconditioning must be enabled)."""
        torch = _torch()
        self._check_block(X, self.torch_dtype, "X")
        Y = out if out is not None else torch.empty_like(X)
        check(lib().gmrf_precond_apply(self._h, _dptr(X), _dptr(Y), X.shape[0], _stream_ptr(stream)),
              "gmrf_precond_apply")
        return Y

    def sample(self, Z, tol=1e-8, m_max=200, reorth=False, out=None, coeffs=False, stream=None):
        """X[r] = x_m for z = Z[r] (FP64 CUDA tensors of shape (k, n)).  Returns (X, info) or,
        with coeffs=True, (X, info, alpha, beta) as numpy arrays."""
        torch = _torch()
        self._check_block(Z, torch.float64, "Z")
        k = Z.shape[0]
        X = out if out is not None else torch.empty_like(Z)
        info = (Info * k)()
        if coeffs:
            alpha = np.zeros((k, m_max))
            beta = np.zeros((k, m_max + 1))
            st = lib().gmrf_sample_ex(self._h, _dptr(Z), k, float(tol), int(m_max), int(bool(reorth)), _dptr(X),
                                      info, alpha.ctypes.data_as(C.c_void_p), beta.ctypes.data_as(C.c_void_p),
                                      _stream_ptr(stream))
        else:
            st = lib().gmrf_sample(self._h, _dptr(Z), k, float(tol), int(m_max), int(bool(reorth)), _dptr(X), info,
                                   _stream_ptr(stream))
        if st not in (_abi.GMRF_OK, _abi.GMRF_ENOTSPD, _abi.GMRF_EINVAL) or (
                st == _abi.GMRF_EINVAL and not any(i.status == _abi.GMRF_EINVAL for i in info)):
            raise GmrfError(st, "gmrf_sample")
        infos = [dict(m_used=i.m_used, status=STATUS[i.status], rel_residual=i.rel_residual,
                      err_bound=i.err_bound) for i in info]
        if coeffs:
            return X, infos, alpha, beta
        return X, infos

    def sample_noalloc(self, Z, tol=1e-8, m_max=200, reorth=False, out=None, stream=None):
        """As sample(), through gmrf_sample_noalloc: the library allocates nothing, its scratch being a
        static 128 MiB device array (the caller passes the output block `out`, else one is made here).
        Returns (X, info)."""
        torch = _torch()
        self._check_block(Z, torch.float64, "Z")
        k = Z.shape[0]
        X = out if out is not None else torch.empty_like(Z)
        self._check_block(X, torch.float64, "out")
        info = (Info * k)()
        st = lib().gmrf_sample_noalloc(self._h, _dptr(Z), k, float(tol), int(m_max), int(bool(reorth)), _dptr(X),
                                       info, _stream_ptr(stream))
        if st not in (_abi.GMRF_OK, _abi.GMRF_ENOTSPD, _abi.GMRF_EINVAL) or (
                st == _abi.GMRF_EINVAL and not any(i.status == _abi.GMRF_EINVAL for i in info)):
            raise GmrfError(st, "gmrf_sample_noalloc")
        return X, [dict(m_used=i.m_used, status=STATUS[i.status], rel_residual=i.rel_residual,
                        err_bound=i.err_bound) for i in info]

    def solve(self, B, tol=1e-8, m_max=200, reorth=False, out=None, stream=None):
        """X[r] ~= Q^{-1} B[r] (FP64 CUDA tensors of shape (k, n)) by the Lanczos form of (preconditioned)
        conjugate gradients; rel_residual in info is ||b - Q x|| / ||b||.  Returns (X, info)."""
        torch = _torch()
        self._check_block(B, torch.float64, "B")
        k = B.shape[0]
        X = out if out is not None else torch.empty_like(B)
        info = (Info * k)()
        st = lib().gmrf_solve(self._h, _dptr(B), k, float(tol), int(m_max), int(bool(reorth)), _dptr(X), info,
                              _stream_ptr(stream))
        if st not in (_abi.GMRF_OK, _abi.GMRF_ENOTSPD, _abi.GMRF_EINVAL) or (
                st == _abi.GMRF_EINVAL and not any(i.status == _abi.GMRF_EINVAL for i in info)):
            raise GmrfError(st, "gmrf_solve")
        return X, [dict(m_used=i.m_used, status=STATUS[i.status], rel_residual=i.rel_residual,
                        err_bound=i.err_bound) for i in info]

    def sample_two_pass(self, Z, tol=1e-8, m_max=200, out=None, stream=None):
        """As sample(), in O(n) device memory: the recurrence runs twice and no Krylov basis is kept
        (no reorthogonalisation).  Returns (X, info)."""
        torch = _torch()
        self._check_block(Z, torch.float64, "Z")
        k = Z.shape[0]
        X = out if out is not None else torch.empty_like(Z)
        info = (Info * k)()
        st = lib().gmrf_sample_two_pass(self._h, _dptr(Z), k, float(tol), int(m_max), _dptr(X), info,
                                        _stream_ptr(stream))
        if st not in (_abi.GMRF_OK, _abi.GMRF_ENOTSPD, _abi.GMRF_EINVAL) or (
                st == _abi.GMRF_EINVAL and not any(i.status == _abi.GMRF_EINVAL for i in info)):
            raise GmrfError(st, "gmrf_sample_two_pass")
        return X, [dict(m_used=i.m_used, status=STATUS[i.status], rel_residual=i.rel_residual,
                        err_bound=i.err_bound) for i in info]

    def logdet(self, n_probes, m, seed=0, probes=None, stream=None):
        """Hutchinson estimate (mean, standard error, per-probe values as numpy)."""
        torch = _torch()
        mean, se = C.c_double(), C.c_double()
        per = np.zeros(n_probes)
        pp = C.c_void_p(0)
        if probes is not None:
            if probes.dtype != torch.int8 or tuple(probes.shape) != (n_probes, self.n) or not probes.is_contiguous():
                raise ValueError("probes must be a contiguous int8 CUDA tensor of shape (n_probes, n)")
            pp = _dptr(probes)
        check(lib().gmrf_logdet(self._h, int(n_probes), int(m), C.c_uint64(seed & (2 ** 64 - 1)), pp,
                                C.byref(mean), C.byref(se), per.ctypes.data_as(C.c_void_p), _stream_ptr(stream)),
              "gmrf_logdet")
        return mean.value, se.value, per

    def logdet_coloured(self, n_probes, m, colour, seed=0, stream=None):
        """Coloured Hutchinson estimate (Section 6.1) for a partition `colour` (n integers in
        0..K-1): (mean, standard error, per-probe values as numpy)."""
        col = np.ascontiguousarray(colour, dtype=np.int32)
        if col.shape != (self.n,):
            raise ValueError(f"colour must have shape ({self.n},)")
        K = int(col.max()) + 1 if col.size else 1
        mean, se = C.c_double(), C.c_double()
        per = np.zeros(n_probes)
        check(lib().gmrf_logdet_coloured(self._h, int(n_probes), int(m), C.c_uint64(seed & (2 ** 64 - 1)),
                                         col.ctypes.data_as(C.c_void_p), K, C.byref(mean), C.byref(se),
                                         per.ctypes.data_as(C.c_void_p), _stream_ptr(stream)),
              "gmrf_logdet_coloured")
        return mean.value, se.value, per

    def distance_colouring(self, p):
        """Distance-p colouring of the lattice points (graph of Q^p, first fit): int32 numpy array."""
        col = np.zeros(self.n, dtype=np.int32)
        K = C.c_int32()
        check(lib().gmrf_distance_colouring(self._h, int(p), col.ctypes.data_as(C.c_void_p), C.byref(K)),
              "gmrf_distance_colouring")
        return col


TUNE_KERNELS = ("spmv", "lz2d")
TUNE_OPTIONS = {1: "xcd_order", 2: "nt_store"}


def _options(bits):
    """Names of the launch options in tuning bits: tile order and store policy, and for the operator kernel its
    tile shape (rows per wave "band8/16/32", columns per lane "lanes1/2/4"; absent: the lattice's rule)."""
    if bits < 0:
        return None
    out = [name for b, name in TUNE_OPTIONS.items() if bits & b]
    band, epl = (bits >> 2) & 3, (bits >> 4) & 3
    if band:
        out.append(f"band{(0, 8, 16, 32)[band]}")
    if epl:
        out.append(f"lanes{(0, 1, 2, 4)[epl]}")
    return out


def autotune(op, k, reps=20, stream=None):
    """Time the candidate launch options of the operator's tunable kernels for k columns and record the
    fastest in the library's table (results are bitwise the same under every choice).  Returns
    {kernel: [options]} (None: kernel not used by this operator)."""
    chosen = (C.c_int32 * 2)()
    check(lib().gmrf_autotune(op._h, int(k), int(reps), chosen, _stream_ptr(stream)), "gmrf_autotune")
    return {name: _options(chosen[i]) for i, name in enumerate(TUNE_KERNELS)}


def tune_table():
    """The library's tuning table: a list of dicts (kernel, order, storage, side classes, columns class,
    options)."""
    n = C.c_int32()
    check(lib().gmrf_tune_export(None, 0, C.byref(n)), "gmrf_tune_export")
    buf = (C.c_int32 * (7 * max(1, n.value)))()
    check(lib().gmrf_tune_export(buf, n.value, C.byref(n)), "gmrf_tune_export")
    out = []
    for i in range(n.value):
        e = list(buf[7 * i:7 * i + 7])
        out.append({"kernel": TUNE_KERNELS[e[0]], "order": e[1], "storage": "f64" if e[2] == GMRF_F64 else "f32",
                    "log2_n1": e[3], "log2_n2": e[4], "log2_k": e[5], "options": _options(e[6]), "bits": e[6]})
    return out


def save_tune(path):
    """Persist the tuning table as JSON."""
    import json
    with open(path, "w") as f:
        json.dump(tune_table(), f, indent=1)


def load_tune(path):
    """Add the entries of a JSON tuning table written by save_tune."""
    import json
    with open(path) as f:
        rows = json.load(f)
    flat = []
    for r in rows:
        flat += [TUNE_KERNELS.index(r["kernel"]), int(r["order"]), GMRF_F64 if r["storage"] == "f64" else GMRF_F32,
                 int(r["log2_n1"]), int(r["log2_n2"]), int(r["log2_k"]), int(r["bits"])]
    arr = (C.c_int32 * max(1, len(flat)))(*flat)
    check(lib().gmrf_tune_import(arr, len(rows)), "gmrf_tune_import")


def clear_tune():
    check(lib().gmrf_tune_clear(), "gmrf_tune_clear")


BANDWIDTH_KERNELS = {"read": 0, "copy": 1, "triad": 2}


def bandwidth_bench(kind, nbytes=1 << 30, blocks=0, reps=20, stream=None):
    """Achievable HBM bandwidth: `kind` in read / copy / triad over arrays of `nbytes` bytes each.
    Returns {"gbs", "avg_us", "bytes_per_launch"}."""
    which = BANDWIDTH_KERNELS[kind]
    gbs, us = C.c_double(), C.c_double()
    check(lib().gmrf_bandwidth_bench(which, C.c_size_t(int(nbytes)), int(blocks), int(reps), C.byref(gbs), C.byref(us),
                                     _stream_ptr(stream)), "gmrf_bandwidth_bench")
    return {"gbs": gbs.value, "avg_us": us.value, "bytes_per_launch": (which + 1) * int(nbytes)}


def sample_batch(ops, Zs, tol=1e-8, m_max=300, stream=None):
    """Uneven batch: field f is ops[f] with right-hand sides Zs[f] ((k_f, n_f) FP64 CUDA
    tensors).  All fields run in one set of launches per Lanczos step.  Returns ([X_f], info)
    with info in field-then-column order."""
    torch = _torch()
    if len(ops) != len(Zs) or not ops:
        raise ValueError("need one Z block per operator")
    for op, Zf in zip(ops, Zs):
        op._check_block(Zf, torch.float64, "Z")
    Z = torch.cat([Zf.reshape(-1) for Zf in Zs])
    X = torch.empty_like(Z)
    ks = (C.c_int64 * len(ops))(*[Zf.shape[0] for Zf in Zs])
    hs = (C.c_void_p * len(ops))(*[op._h.value for op in ops])
    K = sum(Zf.shape[0] for Zf in Zs)
    info = (Info * K)()
    st = lib().gmrf_sample_batch(len(ops), hs, ks, _dptr(Z), float(tol), int(m_max), _dptr(X), info,
                                 _stream_ptr(stream))
    if st not in (_abi.GMRF_OK, _abi.GMRF_ENOTSPD, _abi.GMRF_EINVAL) or (
            st == _abi.GMRF_EINVAL and not any(i.status == _abi.GMRF_EINVAL for i in info)):
        raise GmrfError(st, "gmrf_sample_batch")
    out, o = [], 0
    for Zf in Zs:
        out.append(X[o:o + Zf.numel()].view(Zf.shape))
        o += Zf.numel()
    infos = [dict(m_used=i.m_used, status=STATUS[i.status], rel_residual=i.rel_residual,
                  err_bound=i.err_bound) for i in info]
    return out, infos


def rademacher(seed, n, n_probes, stream=None):
    """(n_probes, n) int8 CUDA tensor of +-1 probes from the Philox4x64-10 rule."""
    torch = _torch()
    out = torch.empty((n_probes, n), dtype=torch.int8, device="cuda")
    check(lib().gmrf_rademacher(C.c_uint64(seed & (2 ** 64 - 1)), int(n), int(n_probes), _dptr(out),
                                _stream_ptr(stream)), "gmrf_rademacher")
    return out


def _tri_args(alpha, beta, m):
    torch = _torch()
    for t, nm in ((alpha, "alpha"), (beta, "beta")):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2:
            raise ValueError(f"{nm} must be a contiguous (k, ld) float64 CUDA tensor")
    if m.dtype != torch.int32 or not m.is_cuda:
        raise ValueError("m must be an int32 CUDA tensor")
    return alpha.shape[0], alpha.shape[1]


def tridiag_invsqrt_e1(alpha, beta, m, stream=None):
    """y[r] = T_r^{-1/2} e_1 for tridiag(beta[r], alpha[r], beta[r]) of size m[r]."""
    torch = _torch()
    k, ld = _tri_args(alpha, beta, m)
    y = torch.zeros_like(alpha)
    status = torch.zeros(k, dtype=torch.int32, device=alpha.device)
    check(lib().gmrf_tridiag_invsqrt_e1(_dptr(alpha), _dptr(beta), _dptr(m), k, ld, _dptr(y), _dptr(status),
                                        _stream_ptr(stream)), "gmrf_tridiag_invsqrt_e1")
    return y, status


def tridiag_log_e1(alpha, beta, m, stream=None):
    """out[r] = e_1^T log(T_r) e_1."""
    torch = _torch()
    k, ld = _tri_args(alpha, beta, m)
    out = torch.zeros(k, dtype=torch.float64, device=alpha.device)
    status = torch.zeros(k, dtype=torch.int32, device=alpha.device)
    check(lib().gmrf_tridiag_log_e1(_dptr(alpha), _dptr(beta), _dptr(m), k, ld, _dptr(out), _dptr(status),
                                    _stream_ptr(stream)), "gmrf_tridiag_log_e1")
    return out, status


KERNELS = {"spmv": 0, "lz_step": 1, "lz_dots": 2, "update": 3, "lz_band": 4, "lgcp_rows": 5, "lgcp_cols": 6,
           "lz2d": 7}


def kernel_bench(op, kernel, k, reps=50, stream=None):
    """Average duration (us) and algorithmic bytes of one launch of a path kernel, timed with
    HIP events on `stream` (default: torch's current stream)."""
    us, nb = C.c_double(), C.c_double()
    check(lib().gmrf_kernel_bench(op._h, KERNELS[kernel], int(k), int(reps), C.byref(us), C.byref(nb),
                                  _stream_ptr(stream)), "gmrf_kernel_bench")
    return {"kernel": kernel, "avg_us": us.value, "bytes": nb.value,
            "achieved_gbs": nb.value / (us.value * 1e-6) / 1e9}


def set_hbm_budget(nbytes):
    check(lib().gmrf_set_hbm_budget(int(nbytes)), "gmrf_set_hbm_budget")


def hbm_in_use():
    return int(lib().gmrf_hbm_in_use())


def pool_reserve(nbytes):
    """Reserve one device region of nbytes for the library's scratch (0 releases it); calls then
    allocate nothing from the device."""
    check(lib().gmrf_pool_reserve(int(nbytes)), "gmrf_pool_reserve")


def pool_info():
    """The scratch pool's state and device-allocator counters, as a dict."""
    info = _abi.PoolInfo()
    check(lib().gmrf_pool_query(C.byref(info)), "gmrf_pool_query")
    return {f: getattr(info, f) for f, _ in _abi.PoolInfo._fields_}
