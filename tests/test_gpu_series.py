"""The sine-series evaluation of the detour function (the paper's stored
representation of eq. Kernel_freq, Sec. II-C) in the FP32 operators, through
the C ABI, against the CPU FP64 oracle.

The series (library builder, ~25 uniform frequency nodes) and the oracle's
quadrature (its own ~100 nodes) are two converged sums of the same integral
(they agree to ~1e-11 of max|h|), so in series mode the FP32 operators are
compared with the quadrature oracle directly: the bar is the FP32 one, 1e-5
norm-wise, and the series path must also beat the table path's own error
(which carries the table's interpolation error) by a factor of four.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1908_03302_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fftt():
    from paper_1908_03302_amd import fftt
    return fftt


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(x, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype or torch.float32).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ragged_bands(fcs):
    """Masked grid that is not a multiple of the 4^3 tile, one band per pulse."""
    g = I.centred_grid((37, 29, 11), 1.0e-3)
    tx = I.ring(24, 0.03, 0.0005, phase=0.1)
    return I.Workload(
        name="ragged%d" % len(fcs), c0=1500.0, tx=tx, pairs=I.all_ordered_pairs(24), grid=g,
        mask=I.cylinder_mask(g, 0.02), pulses=[I.sampled_pulse(f, 1.0) for f in fcs],
        r_max=[I.R_MAX[f] for f in fcs], n_table=4096)


def both_modes(ctx, w, x, yt):
    """(J x, J^T yt) with the table, then with the series."""
    f = _fftt()
    out = []
    for mode in (0, 1):
        ctx.set_tuning(kernel_eval=mode)
        try:
            y = host(ctx.apply_J(dev(x), prec=f.FP32))
            xt = host(ctx.apply_JT(dev(yt), prec=f.FP32))
        finally:
            ctx.set_tuning(kernel_eval=0)
        out.append((y, xt))
    return out


@pytest.fixture(scope="module")
def small():
    w = I.small_fp64()
    say("fixture small:", w.name)
    ctx = _fftt().context_for_workload(w, series=True)
    ctx.prepare()
    return w, oracle.Oracle.from_workload(w), ctx


def test_small_series_J_JT(small):
    """32-element ring, 0.5 MHz / 50 % pulse (31 terms)."""
    w, o, ctx = small
    x = w.model
    yt = I.random_vector(w.m, 71) * 1e-7
    y_ref, x_ref = o.apply_J(x), o.apply_JT(yt)
    (yt_tab, xt_tab), (ys, xs) = both_modes(ctx, w, x, yt)
    e_tab = (rel(yt_tab, y_ref), rel(xt_tab, x_ref))
    e_ser = (rel(ys, y_ref), rel(xs, x_ref))
    say("small J / J^T rel err vs quadrature: table %.2e %.2e, series %.2e %.2e"
        % (e_tab + e_ser))
    for es, et in zip(e_ser, e_tab):
        assert es < 1e-5
        assert es < 0.25 * et


@pytest.mark.parametrize("fcs", [(1e6, 2e6), (0.5e6, 1e6, 1.5e6, 2e6)])
def test_ragged_series_bands(fcs):
    """Two and four bands (one series each) on a masked ragged grid; the
    inactive voxels of J^T are written as zero."""
    w = ragged_bands(fcs)
    f = _fftt()
    o = oracle.Oracle.from_workload(w)
    ctx = f.context_for_workload(w, series=True)
    x = I.random_vector(w.n, 72) * 10.0
    yt = I.random_vector(len(fcs) * w.m, 73) * 1e-7
    y_ref, x_ref = o.apply_J(x), o.apply_JT(yt)
    (ytab, xtab), (ys, xs) = both_modes(ctx, w, x, yt)
    es, et = (rel(ys, y_ref), rel(xs, x_ref)), (rel(ytab, y_ref), rel(xtab, x_ref))
    say("ragged", len(fcs), "bands: series J %.2e J^T %.2e, table J %.2e J^T %.2e" % (es + et))
    assert es[0] < 1e-5 and es[1] < 1e-5
    assert np.all(xs[w.mask == 0] == 0.0)
    # per band, J rows in series mode
    ys2, yr2 = ys.reshape(len(fcs), -1), np.asarray(y_ref).reshape(len(fcs), -1)
    for b in range(len(fcs)):
        assert rel(ys2[b], yr2[b]) < 1e-5


@pytest.mark.parametrize("unroll", [1, 2, 4, 8])
@pytest.mark.parametrize("wpb", [4, 16])
def test_series_launch_shapes_agree(small, unroll, wpb):
    """Results do not depend on the launch shape (unroll 8 runs as 4)."""
    w, o, ctx = small
    f = _fftt()
    x = w.model
    yt = I.random_vector(w.m, 74) * 1e-7
    ctx.set_tuning(kernel_eval=1)
    try:
        ref = (host(ctx.apply_J(dev(x), prec=f.FP32)), host(ctx.apply_JT(dev(yt), prec=f.FP32)))
        ctx.set_tuning(waves_per_block=wpb, unroll_j_staged=unroll, unroll_jt_staged=unroll)
        got = (host(ctx.apply_J(dev(x), prec=f.FP32)), host(ctx.apply_JT(dev(yt), prec=f.FP32)))
    finally:
        ctx.set_tuning(kernel_eval=0, waves_per_block=16, unroll_j_staged=8, unroll_jt_staged=8)
    assert rel(got[0], ref[0]) < 1e-6 and rel(got[1], ref[1]) < 1e-6


def test_series_solve_cgls(small):
    """Twenty CGLS iterations in series mode (FP32 operators and vectors,
    FP64 inner products) track the oracle's FP64 CGLS on its quadrature J."""
    from oracle import solvers
    w, o, ctx = small
    f = _fftt()
    J = o.block()
    sig, alpha = w.noise_sigma, w.extra["alpha"]
    d = J @ w.model + I.noise(w.m, sig, w.noise_seed)
    x_ref, hist = solvers.cgls(lambda v: J @ v, lambda v: J.T @ v, d, sig, alpha, 20)
    errs = []
    for mode in (0, 1):
        ctx.set_tuning(kernel_eval=mode)
        try:
            x = torch.zeros(w.n, dtype=torch.float32, device="cuda:0")
            rep = ctx.solve(dev(d), x, method=0, prec=f.FP32, alpha=alpha, noise_sigma=sig,
                            max_iter=20)
            errs.append(rel(host(x), x_ref))
        finally:
            ctx.set_tuning(kernel_eval=0)
        assert rep["iters"] == 20
    say("CGLS 20 its rel err vs oracle CGLS: table %.2e, series %.2e" % tuple(errs))
    assert errs[1] < 1e-3


def test_ring2d_series_sampled_rows_and_columns():
    """Full-size 128-element ring on the 256x256x64 grid: sampled rows of
    J dc and columns of J^T dT in series mode against the oracle."""
    w = I.ring2d()
    f = _fftt()
    say("ring2d series: set-up")
    ctx = f.context_for_workload(w, series=True)
    ctx.prepare()
    o = oracle.Oracle.from_workload(w)
    rng = np.random.default_rng(19)
    rows = np.sort(rng.choice(w.m, 16, replace=False))
    act = np.flatnonzero(w.mask)
    cols = np.sort(rng.choice(act, 1024, replace=False))
    yt = I.random_vector(w.m, 20) * 1e-7
    ctx.set_tuning(kernel_eval=1)
    y = host(ctx.apply_J(dev(w.model), prec=f.FP32))
    xg = host(ctx.apply_JT(dev(yt), prec=f.FP32))
    ej, et = rel(y[rows], o.rows(rows, w.model)), rel(xg[cols], o.cols(cols, yt))
    say("ring2d series sampled rows %.2e cols %.2e" % (ej, et))
    assert ej < 1e-5 and et < 1e-5


def test_series_errors():
    """Status codes: series mode without a series, outside the staged
    kernels, and bad series arguments."""
    f = _fftt()
    w = ragged_bands((1e6,))
    ctx = f.context_for_workload(w)
    x = dev(np.ones(w.n))
    p = w.pulses[0]
    rm = w.r_max[0]
    a, beta = f.build_series_from_pulse(w.c0, p.samples, p.dt, rm)
    ctx.set_tuning(kernel_eval=1)
    with pytest.raises(f.FFTTError) as e:
        ctx.apply_J(x, prec=f.FP32)
    assert e.value.status == -4                         # FFTT_E_STATE
    with pytest.raises(f.FFTTError):
        ctx.set_kernel_series(0, a, beta, rm * 1.01)    # r_max differs from the table's
    with pytest.raises(f.FFTTError):
        ctx.set_kernel_series(1, a, beta, rm)           # band without a table
    with pytest.raises(f.FFTTError):
        ctx.set_kernel_series(0, a, 1.01 * np.pi / rm, rm)
    with pytest.raises(f.FFTTError):
        ctx.set_kernel_series(0, np.zeros(65), beta, rm)
    ctx.set_kernel_series(0, a, beta, rm)
    ctx.apply_J(x, prec=f.FP32)
    ctx.set_tuning(staged=0)
    with pytest.raises(f.FFTTError) as e:
        ctx.apply_J(x, prec=f.FP32)
    assert e.value.status == -5                         # FFTT_E_UNSUPPORTED
    ctx.set_tuning(staged=1)
    # FP64 keeps the table in series mode
    ctx.apply_J(dev(np.ones(w.n), torch.float64), prec=f.FP64)
    torch.cuda.synchronize()
