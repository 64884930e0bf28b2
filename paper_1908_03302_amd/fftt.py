"""ctypes binding of libfftt (include/fftt.h): argument marshalling only.

Device buffers are torch tensors (memory and streams only); every operation
runs in the library's HIP kernels.  Loading fails loudly when the library has
not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfftt.so")

FFTT_OK = 0
FFTT_NOT_CONVERGED = 1
FP64, FP32, FP32_BF16TABLE = 0, 1, 2
_STATUS = {0: "FFTT_OK", -1: "FFTT_E_INVALID", -2: "FFTT_E_NOMEM", -3: "FFTT_E_DEVICE",
           -4: "FFTT_E_STATE", -5: "FFTT_E_UNSUPPORTED", 1: "FFTT_NOT_CONVERGED"}

EXPORTS = ["fftt_create", "fftt_destroy", "fftt_last_error", "fftt_set_stream",
           "fftt_set_geometry", "fftt_set_kernel_table", "fftt_build_table_from_pulse",
           "fftt_prepare", "fftt_work_count", "fftt_apply_J", "fftt_apply_JT", "fftt_solve",
           "fftt_psf", "fftt_profile", "fftt_kernel_time", "fftt_set_tuning", "fftt_get_tuning",
           "fftt_autotune", "fftt_set_kernel_series", "fftt_build_series_from_pulse",
           "fftt_coverage", "fftt_hessian_lowrank", "fftt_lowrank_diag",
           "fftt_set_geometry_2d", "fftt_hessian_apply", "fftt_apply_JT_noalloc"]
TUNE_WAVES_PER_BLOCK, TUNE_UNROLL_JT, TUNE_UNROLL_J, TUNE_SPLIT_JT, TUNE_SPLIT_J = 0, 1, 2, 3, 4
TUNE_STAGED, TUNE_UNROLL_JT_STAGED, TUNE_UNROLL_J_STAGED = 5, 6, 7
TUNE_STAGED_TABLE = 8
TUNE_RECIPROCITY = 9
TUNE_STAGED_BLOCK = 10
TUNE_KERNEL_EVAL = 11
TUNE_PSF_MATH = 12
TUNE_HESS_BATCHED = 13
TUNE_RHS_BATCHED = 14
TUNE_ENTRY_ORDER = 15


class SolveOpts(C.Structure):
    _fields_ = [("method", C.c_int32), ("prec", C.c_int32), ("alpha", C.c_double),
                ("noise_sigma", C.c_double), ("max_iter", C.c_int32), ("use_x0", C.c_int32),
                ("target_misfit", C.c_double), ("rel_tol", C.c_double),
                ("use_graph", C.c_int32), ("precond", C.c_int32)]


class SolveReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("misfit", C.c_double), ("rel_resid", C.c_double),
                ("time_ms", C.c_double)]


class FFTTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


_lib = None


def load():
    """Load libfftt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfftt.so is not built (%s); run `python -m "
                           "paper_1908_03302_amd.build`" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
    L.fftt_create.argtypes = [C.POINTER(vp), C.c_int, vp]
    L.fftt_destroy.argtypes = [vp]
    L.fftt_destroy.restype = None
    L.fftt_last_error.argtypes = [vp]
    L.fftt_last_error.restype = C.c_char_p
    L.fftt_set_stream.argtypes = [vp, vp]
    L.fftt_set_geometry.argtypes = [vp, C.c_double, dp, i64, C.POINTER(C.c_int32), i64, dp, dp,
                                    C.POINTER(C.c_int64), C.POINTER(C.c_uint8)]
    L.fftt_set_kernel_table.argtypes = [vp, C.c_int32, dp, i64, C.c_double]
    L.fftt_set_geometry_2d.argtypes = [vp, C.c_double, dp, i64, C.POINTER(C.c_int32), i64, dp,
                                       dp, C.POINTER(C.c_int64), C.c_double, C.c_double, i64,
                                       C.POINTER(C.c_uint8)]
    L.fftt_build_table_from_pulse.argtypes = [C.c_double, dp, i64, C.c_double, i64, C.c_double,
                                              dp, dp]
    L.fftt_set_kernel_series.argtypes = [vp, C.c_int32, dp, C.c_int32, C.c_double, C.c_double]
    L.fftt_build_series_from_pulse.argtypes = [C.c_double, dp, i64, C.c_double, C.c_double,
                                               C.c_double, C.c_int32, dp, C.POINTER(C.c_int32),
                                               dp]
    L.fftt_prepare.argtypes = [vp]
    L.fftt_work_count.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int64)]
    L.fftt_apply_J.argtypes = [vp, C.c_int, vp, vp, C.c_int32]
    L.fftt_apply_JT.argtypes = [vp, C.c_int, vp, vp, C.c_int32]
    L.fftt_apply_JT_noalloc.argtypes = [vp, C.c_int, vp, vp, C.c_int32]
    L.fftt_solve.argtypes = [vp, C.POINTER(SolveOpts), vp, vp, C.POINTER(SolveReport)]
    L.fftt_psf.argtypes = [vp, C.c_int, C.POINTER(C.c_int64), C.c_int32, C.c_double, vp]
    L.fftt_coverage.argtypes = [vp, C.c_int, C.c_int32, vp]
    L.fftt_hessian_lowrank.argtypes = [vp, C.c_int, C.c_double, vp, C.c_int32, C.c_int32,
                                       C.c_int32, dp, vp, C.POINTER(C.c_int32)]
    L.fftt_lowrank_diag.argtypes = [vp, C.c_int, dp, vp, C.c_int32, C.c_double, vp, vp]
    L.fftt_hessian_apply.argtypes = [vp, C.c_int, C.c_double, vp, C.c_int32, vp]
    L.fftt_profile.argtypes = [vp, C.c_int32]
    L.fftt_set_tuning.argtypes = [vp, C.c_int32, C.c_int32]
    L.fftt_get_tuning.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32)]
    L.fftt_autotune.argtypes = [vp, C.c_int, C.c_double]
    L.fftt_kernel_time.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    for name in EXPORTS:
        getattr(L, name).restype = getattr(L, name).restype or C.c_int
    L.fftt_destroy.restype = None
    L.fftt_last_error.restype = C.c_char_p
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def build_table_from_pulse(c0, f, dt, n, r_max=0.0):
    """Tabulate h on n nodes over [0, r_max] (r_max <= 0: automatic)."""
    L = load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    h = np.empty(int(n))
    rm = C.c_double(0.0)
    st = L.fftt_build_table_from_pulse(float(c0), _dp(f), f.size, float(dt), int(n),
                                       float(r_max), _dp(h), C.byref(rm))
    if st != FFTT_OK:
        raise FFTTError(st, "fftt_build_table_from_pulse failed")
    return h, rm.value


def build_series_from_pulse(c0, f, dt, r_max, tol=1e-8, max_terms=64):
    """Sine-series coefficients a_1..a_n and beta of h(R) = sum a_m sin(m beta R)."""
    L = load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    a = np.empty(int(max_terms))
    n = C.c_int32(0)
    beta = C.c_double(0.0)
    st = L.fftt_build_series_from_pulse(float(c0), _dp(f), f.size, float(dt), float(r_max),
                                        float(tol), int(max_terms), _dp(a), C.byref(n),
                                        C.byref(beta))
    if st != FFTT_OK:
        raise FFTTError(st, "fftt_build_series_from_pulse failed")
    return a[:n.value].copy(), beta.value


def _dtype_for(prec):
    import torch
    return torch.float64 if prec == FP64 else torch.float32


class Context:
    """One fftt_ctx bound to a device and (per call) torch's current stream."""

    def __init__(self, device: int = 0):
        import torch
        self._torch = torch
        self.L = load()
        self.device = int(device)
        h = C.c_void_p()
        st = self.L.fftt_create(C.byref(h), self.device, None)
        if st != FFTT_OK:
            raise FFTTError(st, "fftt_create(device=%d) failed" % device)
        self.h = h
        self.M = self.N = self.n_bands = 0

    def close(self):
        if getattr(self, "h", None):
            self.L.fftt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st not in (FFTT_OK, FFTT_NOT_CONVERGED):
            raise FFTTError(st, "%s: %s" % (what, self.L.fftt_last_error(self.h).decode()))
        return st

    def _bind_stream(self):
        s = self._torch.cuda.current_stream(self.device).cuda_stream
        self.L.fftt_set_stream(self.h, C.c_void_p(s))

    # -- set-up -------------------------------------------------------
    def set_geometry(self, c0, tx, pairs, origin, spacing, dims, mask=None):
        tx = np.ascontiguousarray(tx, dtype=np.float64).reshape(-1, 3)
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        o = np.ascontiguousarray(origin, dtype=np.float64)
        s = np.ascontiguousarray(spacing, dtype=np.float64)
        d = np.ascontiguousarray(dims, dtype=np.int64)
        mp = C.POINTER(C.c_uint8)()
        if mask is not None:
            self._mask = np.ascontiguousarray(mask, dtype=np.uint8)
            mp = self._mask.ctypes.data_as(C.POINTER(C.c_uint8))
        self._check(self.L.fftt_set_geometry(
            self.h, float(c0), _dp(tx), tx.shape[0],
            pairs.ctypes.data_as(C.POINTER(C.c_int32)), pairs.shape[0], _dp(o), _dp(s),
            d.ctypes.data_as(C.POINTER(C.c_int64)), mp), "set_geometry")
        self.M = pairs.shape[0]
        self.N = int(np.prod(d))

    def set_geometry_2d(self, c0, tx, pairs, origin, spacing, dims, z0, z1, nz, mask=None):
        """2D approximation: in-plane grid (origin, spacing, dims of length 2),
        the model constant over [z0, z1], midpoint rule on nz layers."""
        tx = np.ascontiguousarray(tx, dtype=np.float64).reshape(-1, 3)
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        o = np.ascontiguousarray(origin, dtype=np.float64)
        s = np.ascontiguousarray(spacing, dtype=np.float64)
        d = np.ascontiguousarray(dims, dtype=np.int64)
        mp = C.POINTER(C.c_uint8)()
        if mask is not None:
            self._mask = np.ascontiguousarray(mask, dtype=np.uint8)
            mp = self._mask.ctypes.data_as(C.POINTER(C.c_uint8))
        self._check(self.L.fftt_set_geometry_2d(
            self.h, float(c0), _dp(tx), tx.shape[0],
            pairs.ctypes.data_as(C.POINTER(C.c_int32)), pairs.shape[0], _dp(o), _dp(s),
            d.ctypes.data_as(C.POINTER(C.c_int64)), float(z0), float(z1), int(nz), mp),
            "set_geometry_2d")
        self.M = pairs.shape[0]
        self.N = int(np.prod(d))

    def set_kernel_table(self, band, h, r_max):
        h = np.ascontiguousarray(h, dtype=np.float64)
        self._check(self.L.fftt_set_kernel_table(self.h, int(band), _dp(h), h.size,
                                                 float(r_max)), "set_kernel_table")
        self.n_bands = max(self.n_bands, int(band) + 1)

    def set_kernel_series(self, band, a, beta, r_max):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self._check(self.L.fftt_set_kernel_series(self.h, int(band), _dp(a), a.size, float(beta),
                                                  float(r_max)), "set_kernel_series")

    def prepare(self):
        self._bind_stream()
        self._check(self.L.fftt_prepare(self.h), "prepare")

    def work_count(self):
        """(pv of the operator, pv the kernels evaluate, evaluated lanes)."""
        pv, pve, lanes = C.c_int64(), C.c_int64(), C.c_int64()
        self._bind_stream()
        self._check(self.L.fftt_work_count(self.h, C.byref(pv), C.byref(pve), C.byref(lanes)),
                    "work_count")
        return pv.value, pve.value, lanes.value

    def set_tuning(self, waves_per_block=None, unroll_jt=None, unroll_j=None, split_jt=None,
                   split_j=None, staged=None, unroll_jt_staged=None, unroll_j_staged=None,
                   staged_table=None, reciprocity=None, staged_block=None, kernel_eval=None,
                   psf_math=None, hess_batched=None, rhs_batched=None, entry_order=None):
        for key, v in ((TUNE_WAVES_PER_BLOCK, waves_per_block), (TUNE_UNROLL_JT, unroll_jt),
                       (TUNE_UNROLL_J, unroll_j), (TUNE_SPLIT_JT, split_jt),
                       (TUNE_SPLIT_J, split_j), (TUNE_STAGED, staged),
                       (TUNE_UNROLL_JT_STAGED, unroll_jt_staged),
                       (TUNE_UNROLL_J_STAGED, unroll_j_staged),
                       (TUNE_STAGED_TABLE, staged_table),
                       (TUNE_RECIPROCITY, reciprocity),
                       (TUNE_STAGED_BLOCK, staged_block), (TUNE_KERNEL_EVAL, kernel_eval),
                       (TUNE_PSF_MATH, psf_math), (TUNE_HESS_BATCHED, hess_batched),
                       (TUNE_RHS_BATCHED, rhs_batched), (TUNE_ENTRY_ORDER, entry_order)):
            if v is not None:
                self._check(self.L.fftt_set_tuning(self.h, key, int(v)), "set_tuning")

    TUNING_KEYS = {"waves_per_block": TUNE_WAVES_PER_BLOCK, "unroll_jt": TUNE_UNROLL_JT,
                   "unroll_j": TUNE_UNROLL_J, "split_jt": TUNE_SPLIT_JT, "split_j": TUNE_SPLIT_J,
                   "staged": TUNE_STAGED, "unroll_jt_staged": TUNE_UNROLL_JT_STAGED,
                   "unroll_j_staged": TUNE_UNROLL_J_STAGED, "staged_table": TUNE_STAGED_TABLE,
                   "reciprocity": TUNE_RECIPROCITY, "staged_block": TUNE_STAGED_BLOCK,
                   "kernel_eval": TUNE_KERNEL_EVAL, "psf_math": TUNE_PSF_MATH,
                   "hess_batched": TUNE_HESS_BATCHED, "rhs_batched": TUNE_RHS_BATCHED,
                   "entry_order": TUNE_ENTRY_ORDER}

    def get_tuning(self):
        """All tuning keys and their current values."""
        out = {}
        for name, key in self.TUNING_KEYS.items():
            v = C.c_int32()
            self._check(self.L.fftt_get_tuning(self.h, key, C.byref(v)), "get_tuning")
            out[name] = v.value
        return out

    def autotune(self, prec=FP32, max_seconds=5.0):
        """Time candidate launch shapes and keep the fastest; returns them."""
        self._bind_stream()
        self._check(self.L.fftt_autotune(self.h, int(prec), float(max_seconds)), "autotune")
        return self.get_tuning()

    def profile(self, enable=True):
        self._check(self.L.fftt_profile(self.h, 1 if enable else 0), "profile")

    def kernel_time(self, which):
        """(total ms, launches) of kernel family which (0 J, 1 J^T, 2 reduction)."""
        ms, n = C.c_double(), C.c_int64()
        self._check(self.L.fftt_kernel_time(self.h, int(which), C.byref(ms), C.byref(n)),
                    "kernel_time")
        return ms.value, n.value

    # -- operators ----------------------------------------------------
    def _tensor(self, t, prec, n, what):
        torch = self._torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("%s must be a CUDA/HIP tensor" % what)
        if t.dtype != _dtype_for(prec):
            raise TypeError("%s must be %s for this precision" % (what, _dtype_for(prec)))
        if not t.is_contiguous() or t.numel() != n:
            raise ValueError("%s must be contiguous with %d elements" % (what, n))
        return C.c_void_p(t.data_ptr())

    def apply_J(self, dc, dT=None, prec=FP32, n_rhs=1):
        torch = self._torch
        if dT is None:
            dT = torch.empty(n_rhs * self.n_bands * self.M, dtype=_dtype_for(prec),
                             device=dc.device)
        self._bind_stream()
        self._check(self.L.fftt_apply_J(
            self.h, int(prec), self._tensor(dc, prec, n_rhs * self.N, "dc"),
            self._tensor(dT, prec, n_rhs * self.n_bands * self.M, "dT"), int(n_rhs)), "apply_J")
        return dT

    def apply_JT(self, dT, dc=None, prec=FP32, n_rhs=1):
        torch = self._torch
        if dc is None:
            dc = torch.empty(n_rhs * self.N, dtype=_dtype_for(prec), device=dT.device)
        self._bind_stream()
        self._check(self.L.fftt_apply_JT(
            self.h, int(prec), self._tensor(dT, prec, n_rhs * self.n_bands * self.M, "dT"),
            self._tensor(dc, prec, n_rhs * self.N, "dc"), int(n_rhs)), "apply_JT")
        return dc

    def apply_JT_noalloc(self, dT, dc, prec=FP32, n_rhs=1):
        """J^T through the entry point that allocates nothing (its work
        memory is the library's fixed scratch array); dc must be given."""
        self._bind_stream()
        self._check(self.L.fftt_apply_JT_noalloc(
            self.h, int(prec), self._tensor(dT, prec, n_rhs * self.n_bands * self.M, "dT"),
            self._tensor(dc, prec, n_rhs * self.N, "dc"), int(n_rhs)), "apply_JT_noalloc")
        return dc

    def solve(self, d_obs, x, method=0, prec=FP32, alpha=1e-3, noise_sigma=1.0, max_iter=20,
              x0=False, target_misfit=0.0, rel_tol=0.0, graph=False, precond=False):
        o = SolveOpts(int(method), int(prec), float(alpha), float(noise_sigma), int(max_iter),
                      1 if x0 else 0, float(target_misfit), float(rel_tol), 1 if graph else 0,
                      1 if precond else 0)
        rep = SolveReport()
        self._bind_stream()
        st = self._check(self.L.fftt_solve(
            self.h, C.byref(o), self._tensor(d_obs, prec, self.n_bands * self.M, "d_obs"),
            self._tensor(x, prec, self.N, "x"), C.byref(rep)), "solve")
        return dict(iters=rep.iters, misfit=rep.misfit, rel_resid=rep.rel_resid,
                    time_ms=rep.time_ms, converged=(st == FFTT_OK))

    def coverage(self, kind=0, out=None, prec=FP32):
        """kind 0: sum_i |J_ij| (sensitivity coverage); 1: diag(J^T J); FP32 [N]."""
        torch = self._torch
        if out is None:
            out = torch.empty(self.N, dtype=torch.float32, device="cuda:%d" % self.device)
        self._bind_stream()
        self._check(self.L.fftt_coverage(self.h, int(prec), int(kind),
                                         self._tensor(out, FP32, self.N, "out")), "coverage")
        return out

    def hessian_lowrank(self, omega, k, q=1, noise_sigma=1.0, prec=FP32, eigvecs=None):
        """k leading Ritz pairs of J^T J / sigma^2 from the start block omega
        ([l][N] device tensor).  Returns (eigenvalues [k] numpy, eigenvectors
        [k][N] tensor, rank of the sampled range)."""
        torch = self._torch
        l = omega.numel() // max(self.N, 1)
        if eigvecs is None:
            eigvecs = torch.empty(k * self.N, dtype=_dtype_for(prec), device=omega.device)
        ev = np.zeros(int(k))
        r = C.c_int32(0)
        self._bind_stream()
        self._check(self.L.fftt_hessian_lowrank(
            self.h, int(prec), float(noise_sigma), self._tensor(omega, prec, l * self.N, "omega"),
            int(l), int(q), int(k), _dp(ev), self._tensor(eigvecs, prec, k * self.N, "eigvecs"),
            C.byref(r)), "hessian_lowrank")
        return ev, eigvecs, r.value

    def hessian_apply(self, x, n_vec, noise_sigma=1.0, prec=FP32, y=None):
        """y_k = J^T J x_k / sigma^2 for n_vec vectors ([n_vec][N] tensors)."""
        if y is None:
            y = self._torch.empty(n_vec * self.N, dtype=_dtype_for(prec), device=x.device)
        self._bind_stream()
        self._check(self.L.fftt_hessian_apply(
            self.h, int(prec), float(noise_sigma), self._tensor(x, prec, n_vec * self.N, "x"),
            int(n_vec), self._tensor(y, prec, n_vec * self.N, "y")), "hessian_apply")
        return y

    def lowrank_diag(self, eigvals, eigvecs, alpha, prec=FP32):
        """(posterior variance, resolution) diagonals [N] from k eigenpairs."""
        torch = self._torch
        ev = np.ascontiguousarray(eigvals, dtype=np.float64)
        k = ev.size
        var = torch.empty(self.N, dtype=_dtype_for(prec), device=eigvecs.device)
        res = torch.empty_like(var)
        self._bind_stream()
        self._check(self.L.fftt_lowrank_diag(
            self.h, int(prec), _dp(ev), self._tensor(eigvecs, prec, k * self.N, "eigvecs"),
            int(k), float(alpha), self._tensor(var, prec, self.N, "var"),
            self._tensor(res, prec, self.N, "res")), "lowrank_diag")
        return var, res

    def psf(self, voxels, noise_sigma, out=None, prec=FP32):
        torch = self._torch
        v = np.ascontiguousarray(voxels, dtype=np.int64)
        if out is None:
            out = torch.empty(v.size * self.N, dtype=_dtype_for(prec),
                              device="cuda:%d" % self.device)
        self._bind_stream()
        self._check(self.L.fftt_psf(self.h, int(prec), v.ctypes.data_as(C.POINTER(C.c_int64)),
                                    v.size, float(noise_sigma),
                                    self._tensor(out, prec, v.size * self.N, "out")), "psf")
        return out


def context_for_workload(w, device=0, n_table=None, series=False):
    """Context with the workload's geometry and one table per band built by
    the library's own table builder (and with series=True also each band's
    sine series from the library's series builder)."""
    ctx = Context(device)
    if hasattr(w, "nz"):    # 2D approximation: in-plane grid, z range, layers
        ctx.set_geometry_2d(w.c0, w.tx, w.pairs, w.grid.origin[:2], w.grid.spacing[:2],
                            w.grid.dims[:2], w.z0, w.z1, w.nz, w.mask)
    else:
        ctx.set_geometry(w.c0, w.tx, w.pairs, w.grid.origin, w.grid.spacing, w.grid.dims,
                         w.mask)
    n = n_table or w.n_table
    for b, (p, r) in enumerate(zip(w.pulses, w.r_max)):
        h, rm = build_table_from_pulse(w.c0, p.samples, p.dt, n, r)
        ctx.set_kernel_table(b, h, rm)
        if series:
            a, beta = build_series_from_pulse(w.c0, p.samples, p.dt, rm)
            ctx.set_kernel_series(b, a, beta, rm)
    return ctx
