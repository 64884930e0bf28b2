"""CPU FP64 oracle for the finite-frequency traveltime Jacobian.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  Nothing here is shared
with the HIP path; the product must never import this package.

``fftt_oracle.c`` holds the plain FP64 arithmetic (paper Sec. II-C and
Sec. II-D); this module marshals numpy arrays into it.  ``solvers.py`` holds
the numpy-level reference solvers (CGLS, LSQR, PSF, TV objective).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fftt_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
MAX_BANDS = 8

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=c11", "-D_GNU_SOURCE",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Geom(C.Structure):
    _fields_ = [
        ("c0", C.c_double),
        ("tx", C.POINTER(C.c_double)), ("n_tx", C.c_int64),
        ("pairs", C.POINTER(C.c_int32)), ("n_pairs", C.c_int64),
        ("origin", C.c_double * 3), ("spacing", C.c_double * 3),
        ("dims", C.c_int64 * 3),
        ("mask", C.POINTER(C.c_uint8)),
        ("n_bands", C.c_int32), ("use_table", C.c_int32),
        ("nw", C.c_int64),
        ("qa", C.POINTER(C.c_double)), ("qb", C.POINTER(C.c_double)),
        ("n_tab", C.c_int64), ("tab", C.POINTER(C.c_double)),
        ("r_max", C.c_double * MAX_BANDS),
    ]


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        gp = C.POINTER(_Geom)
        L.orc_quad_coeffs.argtypes = [dp, C.c_int64, C.c_double, C.c_double,
                                      C.c_double, C.c_int64, dp, dp]
        L.orc_quad_coeffs.restype = C.c_int
        L.orc_spectrum.argtypes = [dp, C.c_int64, C.c_double, dp, C.c_int64, dp]
        L.orc_h.argtypes = [dp, dp, C.c_int64, dp, C.c_int64, dp]
        L.orc_table.argtypes = [dp, dp, C.c_int64, C.c_double, C.c_int64, dp]
        L.orc_rows.argtypes = [gp, i64p, C.c_int64, dp, dp]
        L.orc_cols.argtypes = [gp, i64p, C.c_int64, dp, dp]
        L.orc_apply_J.argtypes = [gp, dp, dp]
        L.orc_apply_JT.argtypes = [gp, dp, dp]
        L.orc_block.argtypes = [gp, C.c_int, i64p, C.c_int64, i64p, C.c_int64, dp]
        L.orc_count_pv.argtypes = [gp]
        L.orc_count_pv.restype = C.c_int64
        L.orc_kernel_points.argtypes = [dp, dp, C.c_double, dp, dp, C.c_int64,
                                        C.c_double, dp, C.c_int64, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- spectra
def spectrum(f, dt, w):
    f = _f64(f)
    w = _f64(w)
    S = np.empty_like(w)
    lib().orc_spectrum(_dp(f), f.size, float(dt), _dp(w), w.size, _dp(S))
    return S


def auto_nodes(f, dt, c0, r_max, decay=1e-22, nw_min=96):
    """Quadrature nodes for a sampled pulse.

    w_max: 1.2x the largest frequency (on a 4096-point scan up to Nyquist)
    where w^3 S(w) still exceeds ``decay`` of its peak.
    Node spacing: at most half of 2 pi / (r_max/c0 + pulse duration), so the
    trapezoid sum of the oscillatory integrand cannot alias.
    """
    f = _f64(f)
    w = np.linspace(0.0, math.pi / dt, 4096)
    g = w ** 3 * spectrum(f, dt, w)
    w_hi = w[np.flatnonzero(g > decay * g.max()).max()]
    w_max = 1.2 * w_hi
    duration = f.size * dt
    dw = 0.5 * 2.0 * math.pi / (r_max / c0 + duration)
    nw = max(nw_min, int(math.ceil(w_max / dw)) + 1)
    return w_max, nw


def quad_coeffs(f, dt, c0, r_max=None, w_max=None, nw=None):
    """(a, b) with h(R) = sum_m a_m sin(b_m R)."""
    f = _f64(f)
    if w_max is None or nw is None:
        aw, an = auto_nodes(f, dt, c0, r_max if r_max is not None else 0.05)
        w_max = w_max or aw
        nw = nw or an
    a = np.empty(nw)
    b = np.empty(nw)
    rc = lib().orc_quad_coeffs(_dp(f), f.size, float(dt), float(c0), float(w_max),
                               int(nw), _dp(a), _dp(b))
    if rc != 0:
        raise ValueError("orc_quad_coeffs failed (%d)" % rc)
    return a, b


def h_eval(a, b, R):
    R = _f64(np.atleast_1d(R))
    out = np.empty_like(R)
    lib().orc_h(_dp(_f64(a)), _dp(_f64(b)), len(a), _dp(R), R.size, _dp(out))
    return out


def table(a, b, r_max, n):
    out = np.empty(n)
    lib().orc_table(_dp(_f64(a)), _dp(_f64(b)), len(a), float(r_max), int(n), _dp(out))
    return out


def kernel_points(xs, xr, c0, a, b, r_max, pts):
    pts = _f64(pts).reshape(-1, 3)
    out = np.empty(pts.shape[0])
    lib().orc_kernel_points(_dp(_f64(xs)), _dp(_f64(xr)), float(c0), _dp(_f64(a)),
                            _dp(_f64(b)), len(a), float(r_max), _dp(pts),
                            pts.shape[0], _dp(out))
    return out


# ---------------------------------------------------------------- operator
class Oracle:
    """Dense FP64 operator for one geometry and one set of bands.

    bands: list of (a, b) quadrature coefficient pairs, one per band (all of
    the same length), and r_max per band.  With ``tables`` given (list of
    arrays of equal length) the kernel is evaluated from the tables by linear
    interpolation instead.
    """

    def __init__(self, c0, tx, pairs, origin, spacing, dims, mask, r_max,
                 quads=None, tables=None):
        self.tx = _f64(tx).reshape(-1, 3)
        self.pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        self.mask = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        self.r_max = [float(r) for r in r_max]
        B = len(self.r_max)
        assert 1 <= B <= MAX_BANDS
        g = _Geom()
        g.c0 = float(c0)
        g.tx = _dp(self.tx)
        g.n_tx = self.tx.shape[0]
        g.pairs = self.pairs.ctypes.data_as(C.POINTER(C.c_int32))
        g.n_pairs = self.pairs.shape[0]
        for k in range(3):
            g.origin[k] = float(origin[k])
            g.spacing[k] = float(spacing[k])
            g.dims[k] = int(dims[k])
        g.mask = (self.mask.ctypes.data_as(C.POINTER(C.c_uint8))
                  if self.mask is not None else C.POINTER(C.c_uint8)())
        g.n_bands = B
        for k in range(B):
            g.r_max[k] = self.r_max[k]
        if tables is not None:
            self.tab = _f64(np.stack([np.asarray(t, dtype=np.float64) for t in tables]))
            g.use_table = 1
            g.n_tab = self.tab.shape[1]
            g.tab = _dp(self.tab)
            g.nw = 0
        else:
            self.qa = _f64(np.stack([q[0] for q in quads]))
            self.qb = _f64(np.stack([q[1] for q in quads]))
            g.use_table = 0
            g.nw = self.qa.shape[1]
            g.qa = _dp(self.qa)
            g.qb = _dp(self.qb)
        self.g = g
        self.M = self.pairs.shape[0]
        self.N = int(np.prod(dims))
        self.B = B

    @classmethod
    def from_workload(cls, w, table_mode=False, n_table=None, quad_kw=None):
        kw = dict(quad_kw or {})
        if "nw" not in kw:   # one node count for every band (max of the per-band rules)
            kw["nw"] = max(auto_nodes(p.samples, p.dt, w.c0, r)[1]
                           for p, r in zip(w.pulses, w.r_max))
        quads = [quad_coeffs(p.samples, p.dt, w.c0, r_max=r, **kw)
                 for p, r in zip(w.pulses, w.r_max)]
        tables = None
        if table_mode:
            n = n_table or w.n_table
            tables = [table(a, b, r, n) for (a, b), r in zip(quads, w.r_max)]
        o = cls(w.c0, w.tx, w.pairs, w.grid.origin, w.grid.spacing, w.grid.dims,
                w.mask, w.r_max, quads=quads, tables=tables)
        o.quads = quads
        return o

    def apply_J(self, x):
        x = _f64(x)
        y = np.empty(self.B * self.M)
        lib().orc_apply_J(C.byref(self.g), _dp(x), _dp(y))
        return y.reshape(self.B, self.M) if self.B > 1 else y

    def apply_JT(self, y):
        y = _f64(y).ravel()
        x = np.empty(self.N)
        lib().orc_apply_JT(C.byref(self.g), _dp(y), _dp(x))
        return x

    def rows(self, idx, x):
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        x = _f64(x)
        y = np.empty(self.B * idx.size)
        lib().orc_rows(C.byref(self.g), idx.ctypes.data_as(C.POINTER(C.c_int64)),
                       idx.size, _dp(x), _dp(y))
        return y.reshape(self.B, idx.size) if self.B > 1 else y

    def cols(self, idx, y):
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        y = _f64(y).ravel()
        x = np.empty(idx.size)
        lib().orc_cols(C.byref(self.g), idx.ctypes.data_as(C.POINTER(C.c_int64)),
                       idx.size, _dp(y), _dp(x))
        return x

    def block(self, rows=None, cols=None, band=0):
        rows = np.arange(self.M) if rows is None else rows
        cols = np.arange(self.N) if cols is None else cols
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.empty((rows.size, cols.size))
        lib().orc_block(C.byref(self.g), int(band),
                        rows.ctypes.data_as(C.POINTER(C.c_int64)), rows.size,
                        cols.ctypes.data_as(C.POINTER(C.c_int64)), cols.size, _dp(out))
        return out

    def count_pv(self):
        return int(lib().orc_count_pv(C.byref(self.g)))


# ---------------------------------------------------------------- 2D approximation
def prism(w2):
    """The prism of eq. forward_2D's z integral by the midpoint rule: nz
    layers of thickness dz = (z1 - z0) / nz centred at z0 + (k + 1/2) dz over
    the in-plane grid; returns (origin, spacing, dims, mask) of that 3D grid."""
    g = w2.grid
    nz = int(w2.nz)
    dz = (w2.z1 - w2.z0) / nz
    origin = (g.origin[0], g.origin[1], w2.z0 + 0.5 * dz)
    spacing = (g.spacing[0], g.spacing[1], dz)
    dims = (g.dims[0], g.dims[1], nz)
    mask = np.tile(np.asarray(w2.mask, dtype=np.uint8), nz)
    return origin, spacing, dims, mask


class Oracle2D:
    """Eq. forward_2D: J2D_ij = sum over the layers of the 3D operator's
    entries (midpoint rule in z, voxel volume dA dz), i.e. the prism operator
    applied to dc(x, y) repeated in every layer; its transpose sums the
    layers."""

    def __init__(self, w2, table_mode=False, n_table=None):
        origin, spacing, dims, mask = prism(w2)
        kw = dict(nw=max(auto_nodes(p.samples, p.dt, w2.c0, r)[1]
                         for p, r in zip(w2.pulses, w2.r_max)))
        quads = [quad_coeffs(p.samples, p.dt, w2.c0, r_max=r, **kw)
                 for p, r in zip(w2.pulses, w2.r_max)]
        tables = None
        if table_mode:
            n = n_table or w2.n_table
            tables = [table(a, b, r, n) for (a, b), r in zip(quads, w2.r_max)]
        self.o3 = Oracle(w2.c0, w2.tx, w2.pairs, origin, spacing, dims, mask, w2.r_max,
                         quads=quads, tables=tables)
        self.quads = quads
        self.nxy = int(w2.grid.dims[0] * w2.grid.dims[1])
        self.nz = int(w2.nz)
        self.M, self.N, self.B = self.o3.M, self.nxy, self.o3.B

    def apply_J(self, x):
        return self.o3.apply_J(np.tile(np.asarray(x, dtype=np.float64), self.nz))

    def apply_JT(self, y):
        return self.o3.apply_JT(y).reshape(self.nz, self.nxy).sum(axis=0)

    def block(self, rows=None, cols=None, band=0):
        cols = np.arange(self.nxy) if cols is None else np.asarray(cols)
        out = 0.0
        for k in range(self.nz):
            out = out + self.o3.block(rows=rows, cols=cols + k * self.nxy, band=band)
        return out


def kernel_z_integral(xs, xr, c0, a, b, r_max, pts2, z0, z1, n_nodes):
    """int_{z0}^{z1} K0(x, y, z) dz at in-plane points (x, y) by the composite
    Simpson rule on n_nodes (odd) nodes, K0 from kernel_points."""
    pts2 = _f64(pts2).reshape(-1, 2)
    z = np.linspace(z0, z1, n_nodes)
    wgt = np.ones(n_nodes)
    wgt[1:-1:2] = 4.0
    wgt[2:-1:2] = 2.0
    wgt *= (z[1] - z[0]) / 3.0
    P = np.concatenate([np.repeat(pts2, n_nodes, axis=0),
                        np.tile(z, pts2.shape[0])[:, None]], axis=1)
    K = kernel_points(xs, xr, c0, a, b, r_max, P).reshape(pts2.shape[0], n_nodes)
    return K @ wgt
