"""Parity of the HIP operators with the CPU FP64 oracle (through the C ABI).

Tolerances (norm-wise relative, |y - y_ref|_2 / |y_ref|_2):
  FP32 path vs oracle quadrature ........ 1e-5
  BF16-table path vs oracle quadrature .. 1e-3
  FP64 path vs oracle with the same linear table ... 1e-11
  FP64 path vs oracle quadrature: the table's own interpolation error (the
  oracle's table-vs-quadrature difference) plus 1e-11.
"""
import math
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


def emax(a, b):
    """Largest element error over the largest reference element."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.abs(a - b).max() / np.abs(b).max())


# Element-wise bars, as a multiple of the norm-wise ones (1e-5 FP32, 1e-3
# BF16 table): the largest error of a sample of outputs over the largest
# output may exceed the norm-wise ratio by the spread of the error over the
# sample, which a factor of 5 covers for these smooth kernels.
ELEM = {"FP32": 5e-5, "BF16": 5e-3}


def dev(x, prec):
    f = _fftt()
    dt = torch.float64 if prec == f.FP64 else torch.float32
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dt).to("cuda:0").contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# ------------------------------------------------------------ workloads

def ragged_workload():
    """Grid that is not a multiple of the 4^3 tile, masked, two bands."""
    g = I.centred_grid((37, 29, 11), 1.0e-3)
    tx = I.ring(24, 0.03, 0.0005, phase=0.1)
    return I.Workload(
        name="ragged", c0=1500.0, tx=tx, pairs=I.all_ordered_pairs(24), grid=g,
        mask=I.cylinder_mask(g, 0.02),
        pulses=[I.sampled_pulse(1e6, 1.0), I.sampled_pulse(2e6, 1.0)],
        r_max=[I.R_MAX[1e6], I.R_MAX[2e6]], n_table=4096)


@pytest.fixture(scope="module")
def small():
    w = I.small_fp64()
    say("fixture small:", w.name)
    o = oracle.Oracle.from_workload(w)
    ot = oracle.Oracle.from_workload(w, table_mode=True)
    ctx = _fftt().context_for_workload(w)
    ctx.prepare()
    return w, o, ot, ctx


@pytest.fixture(scope="module")
def ragged():
    w = ragged_workload()
    say("fixture ragged:", w.name)
    o = oracle.Oracle.from_workload(w)
    ot = oracle.Oracle.from_workload(w, table_mode=True)
    ctx = _fftt().context_for_workload(w)
    ctx.prepare()
    return w, o, ot, ctx


# ------------------------------------------------------------ small (config 1)

def test_small_work_count_exact(small):
    """The operator's pv equals the oracle's brute-force count; with every
    pair's reverse present, the kernels evaluate exactly half of it."""
    w, o, ot, ctx = small
    pv, pv_eval, lanes = ctx.work_count()
    assert pv == o.count_pv()
    assert 2 * pv_eval == pv
    assert lanes >= pv_eval


@pytest.mark.parametrize("prec_name", ["FP64", "FP32", "FP32_BF16TABLE"])
def test_small_apply_J(small, prec_name):
    w, o, ot, ctx = small
    f = _fftt()
    prec = getattr(f, prec_name)
    x = w.model
    y_ref = o.apply_J(x)
    y = host(ctx.apply_J(dev(x, prec), prec=prec))
    e = rel(y, y_ref)
    say("small J", prec_name, "rel err vs quadrature oracle", e)
    if prec == f.FP64:
        y_tab = ot.apply_J(x)
        assert rel(y, y_tab) < 1e-11
        assert e <= rel(y_tab, y_ref) + 1e-11
    elif prec == f.FP32:
        assert e < 1e-5
    else:
        assert e < 1e-3


@pytest.mark.parametrize("prec_name", ["FP64", "FP32", "FP32_BF16TABLE"])
def test_small_apply_JT(small, prec_name):
    w, o, ot, ctx = small
    f = _fftt()
    prec = getattr(f, prec_name)
    y = I.random_vector(w.m, 7) * 1e-7
    x_ref = o.apply_JT(y)
    x = host(ctx.apply_JT(dev(y, prec), prec=prec))
    e = rel(x, x_ref)
    say("small JT", prec_name, "rel err vs quadrature oracle", e)
    if prec == f.FP64:
        x_tab = ot.apply_JT(y)
        assert rel(x, x_tab) < 1e-11
        assert e <= rel(x_tab, x_ref) + 1e-11
    elif prec == f.FP32:
        assert e < 1e-5
    else:
        assert e < 1e-3


@pytest.mark.parametrize("prec_name", ["FP64", "FP32"])
def test_small_adjoint_identity(small, prec_name):
    w, o, ot, ctx = small
    f = _fftt()
    prec = getattr(f, prec_name)
    x = I.random_vector(w.n, 21)
    y = I.random_vector(w.m, 22)
    Jx = host(ctx.apply_J(dev(x, prec), prec=prec))
    JTy = host(ctx.apply_JT(dev(y, prec), prec=prec))
    lhs, rhs = float(Jx @ y), float(x @ JTy)
    tol = 1e-12 if prec == f.FP64 else 1e-5
    assert abs(lhs - rhs) <= tol * max(abs(lhs), np.linalg.norm(Jx) * np.linalg.norm(y))


def test_small_determinism(small):
    w, o, ot, ctx = small
    f = _fftt()
    x = dev(I.random_vector(w.n, 3), f.FP32)
    y = dev(I.random_vector(w.m, 4), f.FP32)
    a1 = host(ctx.apply_J(x, prec=f.FP32))
    a2 = host(ctx.apply_J(x, prec=f.FP32))
    b1 = host(ctx.apply_JT(y, prec=f.FP32))
    b2 = host(ctx.apply_JT(y, prec=f.FP32))
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)


def test_small_reciprocity(small):
    w, o, ot, ctx = small
    f = _fftt()
    idx = {tuple(p): i for i, p in enumerate(w.pairs)}
    rec = np.array([idx[(p[1], p[0])] for p in w.pairs])
    y = host(ctx.apply_J(dev(I.random_vector(w.n, 8), f.FP32), prec=f.FP32))
    assert rel(y[rec], y) < 1e-6


def test_small_columns_elementwise(small):
    """J e_j (one column) for a few voxels: element-wise kernel values."""
    w, o, ot, ctx = small
    f = _fftt()
    for j in (0, 1234, 3456, 6911):
        e = np.zeros(w.n)
        e[j] = 1.0
        col_ref = o.block(cols=np.array([j]))[:, 0]
        col = host(ctx.apply_J(dev(e, f.FP32), prec=f.FP32))
        assert np.abs(col - col_ref).max() <= 2e-5 * np.abs(col_ref).max()


def test_small_multi_rhs(small):
    w, o, ot, ctx = small
    f = _fftt()
    X = np.stack([I.random_vector(w.n, 30 + k) for k in range(3)])
    Y = host(ctx.apply_J(dev(X.ravel(), f.FP32), prec=f.FP32, n_rhs=3)).reshape(3, -1)
    for k in range(3):
        yk = host(ctx.apply_J(dev(X[k], f.FP32), prec=f.FP32))
        assert np.array_equal(Y[k], yk)
    Z = np.stack([I.random_vector(w.m, 40 + k) for k in range(2)])
    XT = host(ctx.apply_JT(dev(Z.ravel(), f.FP32), prec=f.FP32, n_rhs=2)).reshape(2, -1)
    for k in range(2):
        assert np.array_equal(XT[k], host(ctx.apply_JT(dev(Z[k], f.FP32), prec=f.FP32)))


# ------------------------------------------------------------ ragged, two bands

@pytest.mark.parametrize("prec_name", ["FP64", "FP32", "FP32_BF16TABLE"])
def test_ragged_two_bands(ragged, prec_name):
    w, o, ot, ctx = ragged
    f = _fftt()
    prec = getattr(f, prec_name)
    x = I.random_vector(w.n, 50) * 10.0
    y_ref = o.apply_J(x)            # [2][M]
    y = host(ctx.apply_J(dev(x, prec), prec=prec)).reshape(2, -1)
    yt = I.random_vector(2 * w.m, 51) * 1e-7
    x_ref = o.apply_JT(yt)
    xg = host(ctx.apply_JT(dev(yt, prec), prec=prec))
    ej, et = rel(y, y_ref), rel(xg, x_ref)
    say("ragged", prec_name, "J", ej, "JT", et)
    # inactive voxels are written as zero
    assert np.all(xg[w.mask == 0] == 0.0)
    if prec == f.FP64:
        assert rel(y, ot.apply_J(x)) < 1e-11 and rel(xg, ot.apply_JT(yt)) < 1e-11
    elif prec == f.FP32:
        assert ej < 1e-5 and et < 1e-5
    else:
        assert ej < 1e-3 and et < 1e-3
    pv, _, _ = ctx.work_count()
    assert pv == o.count_pv()


# ------------------------------------------------------------ on-ray zero

def test_zero_on_the_ray_fp32():
    """A voxel centre on the straight path between a source and a receiver
    has zero sensitivity (R = 0); the FP32 kernel must not lose that to
    cancellation in R_xs + R_xr - L."""
    f = _fftt()
    g = I.centred_grid((41, 21, 9), 0.8e-3)
    tx = np.array([[-0.11, 0.0, 0.0], [0.11, 0.0, 0.0]])
    pairs = np.array([[0, 1]], dtype=np.int32)
    p = I.sampled_pulse(1e6, 1.0)
    ctx = f.Context(0)
    ctx.set_geometry(1500.0, tx, pairs, g.origin, g.spacing, g.dims, None)
    h, rm = f.build_table_from_pulse(1500.0, p.samples, p.dt, 4096, I.R_MAX[1e6])
    ctx.set_kernel_table(0, h, rm)
    y = I.random_vector(1, 1) * 0 + 1.0
    col = host(ctx.apply_JT(dev(y, f.FP32), prec=f.FP32)).reshape(9, 21, 41)
    on = np.abs(col[4, 10, :])            # y = z = 0: on the ray
    say("on-ray max", on.max(), "column max", np.abs(col).max())
    # cancellation-free detour: ~1e-6 of the peak; a plain FP32 sum of the
    # two 0.1 m distances would leave ~1e-4
    assert on.max() <= 2e-5 * np.abs(col).max()


# ------------------------------------------------------------ lab-like ring (config 2)

@pytest.fixture(scope="module")
def ring2d():
    w = I.ring2d()
    say("fixture ring2d:", w.name)
    ctx = _fftt().context_for_workload(w)
    ctx.prepare()
    o = oracle.Oracle.from_workload(w)
    return w, o, ctx


def test_ring2d_sampled_rows_and_columns(ring2d):
    """Full-size 128-element ring on the 256x256x64 grid, FP32: sampled rows
    of J dc (the phantom) and sampled columns of J^T dT against the oracle."""
    w, o, ctx = ring2d
    f = _fftt()
    rng = np.random.default_rng(9)
    rows = np.sort(rng.choice(w.m, 24, replace=False))
    x = w.model
    y = host(ctx.apply_J(dev(x, f.FP32), prec=f.FP32))
    y_ref = o.rows(rows, x)
    ej = rel(y[rows], y_ref)
    act = np.flatnonzero(w.mask)
    cols = np.sort(rng.choice(act, 2048, replace=False))
    yt = I.random_vector(w.m, 10) * 1e-7
    xg = host(ctx.apply_JT(dev(yt, f.FP32), prec=f.FP32))
    x_ref = o.cols(cols, yt)
    et = rel(xg[cols], x_ref)
    mj, mt = emax(y[rows], y_ref), emax(xg[cols], x_ref)
    say("ring2d FP32 sampled rows %.2e (max-elem %.2e) cols %.2e (max-elem %.2e)"
        % (ej, mj, et, mt))
    assert ej < 1e-5 and et < 1e-5
    assert mj < ELEM["FP32"] and mt < ELEM["FP32"]
    yb = host(ctx.apply_J(dev(x, f.FP32_BF16TABLE), prec=f.FP32_BF16TABLE))
    xb = host(ctx.apply_JT(dev(yt, f.FP32_BF16TABLE), prec=f.FP32_BF16TABLE))
    ebj, ebt = rel(yb[rows], y_ref), rel(xb[cols], x_ref)
    mbj, mbt = emax(yb[rows], y_ref), emax(xb[cols], x_ref)
    say("ring2d BF16 table sampled rows %.2e (max-elem %.2e) cols %.2e (max-elem %.2e)"
        % (ebj, mbj, ebt, mbt))
    assert ebj < 1e-3 and ebt < 1e-3
    assert mbj < ELEM["BF16"] and mbt < ELEM["BF16"]


def test_ring2d_fp64_sampled_rows_and_columns(ring2d):
    """Full-size 128-element ring, FP64 path: sampled rows of J dc and
    sampled columns of J^T dT against the oracle with the same linear table
    (1e-11 norm-wise, 1e-10 of the largest element), and against quadrature
    within the table's own interpolation error (the FP32 bar)."""
    w, o, ctx = ring2d
    f = _fftt()
    ot = oracle.Oracle.from_workload(w, table_mode=True)
    rng = np.random.default_rng(19)
    rows = np.sort(rng.choice(w.m, 16, replace=False))
    x = w.model
    y = host(ctx.apply_J(dev(x, f.FP64), prec=f.FP64))
    y_tab, y_q = ot.rows(rows, x), o.rows(rows, x)
    act = np.flatnonzero(w.mask)
    cols = np.sort(rng.choice(act, 512, replace=False))
    yt = I.random_vector(w.m, 20) * 1e-7
    xg = host(ctx.apply_JT(dev(yt, f.FP64), prec=f.FP64))
    x_tab, x_q = ot.cols(cols, yt), o.cols(cols, yt)
    ej, et = rel(y[rows], y_tab), rel(xg[cols], x_tab)
    mj, mt = emax(y[rows], y_tab), emax(xg[cols], x_tab)
    qj, qt = rel(y[rows], y_q), rel(xg[cols], x_q)
    say("ring2d FP64 sampled rows %.2e (max-elem %.2e) cols %.2e (max-elem %.2e) vs table; "
        "%.2e / %.2e vs quadrature" % (ej, mj, et, mt, qj, qt))
    assert ej < 1e-11 and et < 1e-11
    assert mj < 1e-10 and mt < 1e-10
    assert qj < 1e-5 and qt < 1e-5


def test_ring2d_adjoint_fp32(ring2d):
    w, o, ctx = ring2d
    f = _fftt()
    x = I.random_vector(w.n, 61) * w.mask
    y = I.random_vector(w.m, 62)
    Jx = host(ctx.apply_J(dev(x, f.FP32), prec=f.FP32))
    JTy = host(ctx.apply_JT(dev(y, f.FP32), prec=f.FP32))
    lhs, rhs = float(Jx @ y), float(x @ JTy)
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(Jx) * np.linalg.norm(y)


def test_multiband_full_size_sampled_rows_and_columns():
    """Four bands (0.5, 1, 1.5, 2 MHz) on the full 256x256x64 grid of the
    128-element ring, in the shape the bench times (the context's default:
    staged kernels, FP32 node table, J and J^T without the truncation
    select): sampled rows of J dc for every band and sampled columns of
    J^T dT summed over the bands, against the oracle's table mode (1e-5) and
    its quadrature (the tables' own error plus 1e-5)."""
    w = I.multiband()
    f = _fftt()
    say("multiband full size: set-up")
    ctx = f.context_for_workload(w)
    ctx.prepare()
    o = oracle.Oracle.from_workload(w)
    ot = oracle.Oracle.from_workload(w, table_mode=True)
    rng = np.random.default_rng(19)
    rows = np.sort(rng.choice(w.m, 16, replace=False))
    x = w.model
    y = host(ctx.apply_J(dev(x, f.FP32), prec=f.FP32)).reshape(4, w.m)
    yq, yt_ = o.rows(rows, x), ot.rows(rows, x)
    act = np.flatnonzero(w.mask)
    cols = np.sort(rng.choice(act, 1024, replace=False))
    dT = I.random_vector(4 * w.m, 20) * 1e-7
    xg = host(ctx.apply_JT(dev(dT, f.FP32), prec=f.FP32))
    xq, xt = o.cols(cols, dT), ot.cols(cols, dT)
    ej, ejq, ejtab = rel(y[:, rows], yt_), rel(y[:, rows], yq), rel(yt_, yq)
    et, etq, ettab = rel(xg[cols], xt), rel(xg[cols], xq), rel(xt, xq)
    mj, mt = emax(y[:, rows], yt_), emax(xg[cols], xt)
    say("multiband rows: vs table %.2e, vs quadrature %.2e (table's own %.2e); cols: vs table "
        "%.2e, vs quadrature %.2e (table's own %.2e); max-elem vs table: rows %.2e cols %.2e"
        % (ej, ejq, ejtab, et, etq, ettab, mj, mt))
    assert ej < 1e-5 and et < 1e-5
    assert ejq < ejtab + 1e-5 and etq < ettab + 1e-5
    assert mj < ELEM["FP32"] and mt < ELEM["FP32"]
    # the FP64 path (per-wavefront kernels, four bands in one launch) against
    # the same table oracle
    y64 = host(ctx.apply_J(dev(x, f.FP64), prec=f.FP64)).reshape(4, w.m)
    x64 = host(ctx.apply_JT(dev(dT, f.FP64), prec=f.FP64))
    e64j, e64t = rel(y64[:, rows], yt_), rel(x64[cols], xt)
    say("multiband FP64 vs table: rows %.2e cols %.2e" % (e64j, e64t))
    assert e64j < 1e-11 and e64t < 1e-11


# ------------------------------------------------------------ launch shapes

@pytest.mark.parametrize("wpb,unroll,split,staged,stab", [
    (1, 1, 0, 0, 0), (4, 2, 0, 0, 0), (8, 4, 0, 0, 0), (16, 4, 0, 0, 0), (4, 1, 1, 0, 0),
    (8, 2, 1, 0, 0), (16, 4, 1, 0, 0), (1, 1, 1, 1, 0), (4, 2, 1, 1, 0), (16, 4, 1, 1, 0),
    (8, 1, 1, 1, 0), (16, 4, 1, 1, 1), (4, 2, 1, 1, 1), (1, 1, 1, 1, 1), (16, 8, 1, 1, 0),
    (2, 8, 1, 1, 1)])
def test_launch_shapes_agree(ragged, wpb, unroll, split, staged, stab):
    """Every tuning (tiles per workgroup, unroll, split of a tile's pairs over
    a workgroup, LDS-staged distances, staged table layout) computes the same
    operator, within the FP32/FP64 bars."""
    w, o, ot, ctx = ragged
    f = _fftt()
    u_ns = min(unroll, 4)   # the per-wavefront kernels take 1, 2 or 4
    ctx.set_tuning(waves_per_block=wpb, unroll_jt=u_ns, unroll_j=u_ns, split_jt=split,
                   split_j=split, staged=staged, unroll_jt_staged=unroll, unroll_j_staged=unroll,
                   staged_table=stab)
    try:
        x = I.random_vector(w.n, 70) * 5.0
        yt = I.random_vector(2 * w.m, 71) * 1e-7
        y_ref, x_ref = o.apply_J(x), o.apply_JT(yt)
        for prec in (f.FP32, f.FP64):
            y = host(ctx.apply_J(dev(x, prec), prec=prec)).reshape(2, -1)
            xg = host(ctx.apply_JT(dev(yt, prec), prec=prec))
            if prec == f.FP64:
                assert rel(y, ot.apply_J(x)) < 1e-11 and rel(xg, ot.apply_JT(yt)) < 1e-11
            else:
                assert rel(y, y_ref) < 1e-5 and rel(xg, x_ref) < 1e-5
    finally:
        ctx.set_tuning(waves_per_block=16, unroll_jt=2, unroll_j=4, split_jt=0, split_j=1,
                       staged=1, unroll_jt_staged=8, unroll_j_staged=4, staged_table=0)


# ------------------------------------------------ slice-by-slice (full size)

@pytest.fixture(scope="module")
def slices3d():
    w = I.slices3d()
    say("fixture slices3d:", w.name, "M", w.m, "N", w.n)
    ctx = _fftt().context_for_workload(w)
    ctx.prepare()
    o = oracle.Oracle.from_workload(w)
    return w, o, ctx


def test_slices3d_sampled_rows_and_columns(slices3d):
    """256 transducers at 16 heights (1 044 480 pairs) on the 256x256x160
    grid, FP32 (staged by ring-sized transducer blocks) and BF16 table:
    sampled rows of J dc (the blob phantom) and sampled columns of J^T dT
    against the oracle; the operator's work count against the oracle's."""
    w, o, ctx = slices3d
    f = _fftt()
    rng = np.random.default_rng(19)
    rows = np.sort(rng.choice(w.m, 24, replace=False))
    act = np.flatnonzero(w.mask)
    cols = np.sort(rng.choice(act, 256, replace=False))
    yt = I.random_vector(w.m, 20) * 1e-7
    y_ref = o.rows(rows, w.model)
    x_ref = o.cols(cols, yt)
    for prec, bar, ebar in ((f.FP32, 1e-5, ELEM["FP32"]), (f.FP32_BF16TABLE, 1e-3, ELEM["BF16"])):
        y = host(ctx.apply_J(dev(w.model, f.FP32), prec=prec))
        xg = host(ctx.apply_JT(dev(yt, f.FP32), prec=prec))
        ej, et = rel(y[rows], y_ref), rel(xg[cols], x_ref)
        mj, mt = emax(y[rows], y_ref), emax(xg[cols], x_ref)
        say("slices3d", prec, "sampled rows %.2e (max-elem %.2e) cols %.2e (max-elem %.2e)"
            % (ej, mj, et, mt))
        assert ej < bar and et < bar
        assert mj < ebar and mt < ebar
    # FP64 path (per-wavefront kernels over all 4096 transducers) against the
    # oracle with the same linear table
    ot = oracle.Oracle.from_workload(w, table_mode=True)
    y64 = host(ctx.apply_J(dev(w.model, f.FP64), prec=f.FP64))
    x64 = host(ctx.apply_JT(dev(yt, f.FP64), prec=f.FP64))
    e64j, e64t = rel(y64[rows], ot.rows(rows, w.model)), rel(x64[cols], ot.cols(cols, yt))
    say("slices3d FP64 vs table: rows %.2e cols %.2e" % (e64j, e64t))
    assert e64j < 1e-11 and e64t < 1e-11


# ------------------------------------------------------------ autotuner

@pytest.mark.parametrize("prec_name", ["FP32", "FP64"])
def test_autotune_keeps_results(ragged, prec_name):
    """The autotuner picks a valid launch shape; the operators still agree
    with the oracle afterwards."""
    w, o, ot, ctx = ragged
    f = _fftt()
    prec = getattr(f, prec_name)
    before = ctx.get_tuning()
    try:
        chosen = ctx.autotune(prec=prec, max_seconds=3.0)
        say("autotune", prec_name, chosen)
        assert chosen["waves_per_block"] in (4, 8, 16)
        x = I.random_vector(w.n, 70) * 5.0
        yt = I.random_vector(2 * w.m, 71) * 1e-7
        y = host(ctx.apply_J(dev(x, prec), prec=prec)).reshape(2, -1)
        xg = host(ctx.apply_JT(dev(yt, prec), prec=prec))
        if prec == f.FP64:
            assert rel(y, ot.apply_J(x)) < 1e-11 and rel(xg, ot.apply_JT(yt)) < 1e-11
        else:
            assert rel(y, o.apply_J(x)) < 1e-5 and rel(xg, o.apply_JT(yt)) < 1e-5
    finally:
        ctx.set_tuning(**before)
