"""Edge cases of the operators through the C ABI, against the CPU FP64
oracle: no active voxel, pairs whose sensitivity never reaches the grid,
grids of one to a few voxels (every tile ragged), a single pair and
repeated pairs, the shortest and the longest table, and the error statuses
of invalid input.

Bars: FP64 path = oracle's linear-table mode to 1e-11 (norm-wise); FP32
path = oracle's table mode to 1e-5; exact zeros where no pair reaches.
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
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def workload(dims, spacing, tx, pairs, mask=None, fc=1e6, n_table=4096):
    g = I.centred_grid(dims, spacing)
    return I.Workload(name="edge", c0=1500.0, tx=tx, pairs=np.asarray(pairs, dtype=np.int32),
                      grid=g, mask=I.cylinder_mask(g, None) if mask is None else mask,
                      pulses=[I.sampled_pulse(fc, 1.0)], r_max=[I.R_MAX[fc]], n_table=n_table)


def both_precisions(w, seed=0):
    """J x and J^T y in FP64 and FP32 against the oracle's table mode."""
    f = _fftt()
    ot = oracle.Oracle.from_workload(w, table_mode=True)
    ctx = f.context_for_workload(w)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(w.n) * 10.0
    y = rng.standard_normal(w.m) * 1e-7
    yr, xr = ot.apply_J(x), ot.apply_JT(y)
    out = {}
    for name, prec, dt in (("FP64", f.FP64, torch.float64), ("FP32", f.FP32, torch.float32)):
        yg = host(ctx.apply_J(dev(x, dt), prec=prec))
        xg = host(ctx.apply_JT(dev(y, dt), prec=prec))
        out[name] = (yg, xg)
        ej, et = rel(yg, yr), rel(xg, xr)
        say(w.grid.dims, name, "J %.2e J^T %.2e" % (ej, et))
        bar = 1e-11 if prec == f.FP64 else 1e-5
        assert ej <= bar and et <= bar
    return ctx, ot, yr, xr, out


def test_no_active_voxel():
    """A mask with no active voxel: J = 0, J^T = 0, zero work, zero
    coverage; CGLS leaves x = 0 with the data misfit |d|^2 / sigma^2."""
    f = _fftt()
    tx = I.ring(16, 0.03)
    g = I.centred_grid((9, 7, 5), 1e-3)
    w = workload((9, 7, 5), 1e-3, tx, I.all_ordered_pairs(16), mask=np.zeros(g.n, np.uint8))
    ctx = f.context_for_workload(w)
    ctx.prepare()
    assert ctx.work_count() == (0, 0, 0)
    x = torch.ones(w.n, dtype=torch.float32, device="cuda:0")
    assert host(ctx.apply_J(x, prec=f.FP32)).max() == 0.0
    y = torch.ones(w.m, dtype=torch.float32, device="cuda:0")
    assert np.abs(host(ctx.apply_JT(y, prec=f.FP32))).max() == 0.0
    assert np.abs(host(ctx.coverage(1))).max() == 0.0
    d = torch.full((w.m,), 1e-8, dtype=torch.float64, device="cuda:0")
    xs = torch.zeros(w.n, dtype=torch.float64, device="cuda:0")
    rep = ctx.solve(d, xs, method=0, prec=f.FP64, alpha=1e-3, noise_sigma=5e-9, max_iter=3)
    assert np.abs(host(xs)).max() == 0.0
    assert abs(rep["misfit"] - w.m * 4.0) < 1e-9 * w.m * 4.0


def test_pairs_missing_the_grid():
    """A 6 mm cube at the centre of a 3 cm ring: pairs of neighbouring
    transducers pass far from it (no voxel within R_max of their ray), so
    their rows are exactly zero; the other rows match the oracle."""
    tx = I.ring(12, 0.03)
    w = workload((6, 6, 6), 1e-3, tx, I.all_ordered_pairs(12))
    ctx, ot, yr, xr, out = both_precisions(w, seed=1)
    zero = np.flatnonzero(np.abs(yr) == 0.0)
    assert 0 < zero.size < w.m
    for name in ("FP64", "FP32"):
        assert np.all(out[name][0][zero] == 0.0)
    _, pve, _ = ctx.work_count()
    assert 0 < pve


@pytest.mark.parametrize("dims", [(1, 1, 1), (5, 1, 1), (1, 3, 2), (4, 4, 4), (3, 7, 5)])
def test_tiny_grids(dims):
    """Grids smaller than one tile or not a multiple of it in any direction:
    the lanes outside the grid take no part."""
    tx = I.ring(10, 0.004)
    w = workload(dims, 0.5e-3, tx, I.all_ordered_pairs(10))
    both_precisions(w, seed=2)


def test_single_pair_and_repeats():
    tx = I.ring(8, 0.004)
    w1 = workload((6, 5, 4), 0.5e-3, tx, [[0, 3]])
    both_precisions(w1, seed=3)
    # a pair, its reverse and a repeat: three equal rows
    w3 = workload((6, 5, 4), 0.5e-3, tx, [[0, 3], [3, 0], [0, 3]])
    ctx, ot, yr, xr, out = both_precisions(w3, seed=4)
    y64 = out["FP64"][0]
    assert y64[0] == y64[2]
    assert abs(y64[1] - y64[0]) <= 1e-14 * abs(y64[0])


@pytest.mark.parametrize("n_table", [2, 3, 16384])
def test_shortest_and_longest_table(n_table):
    """Two nodes (h interpolated linearly over [0, R_max]) up to the largest
    table accepted, with the same seeded table given to the library and the
    oracle (so only the operator's arithmetic is compared; the staged kernels
    may or may not fit, results may not change)."""
    f = _fftt()
    tx = I.ring(10, 0.004)
    w = workload((7, 6, 5), 0.5e-3, tx, I.all_ordered_pairs(10), n_table=n_table)
    # smooth, like the detour function (a few periods over [0, R_max]): the
    # FP32 table coordinate carries ~1e-3 of a node at 16384 nodes, harmless
    # unless neighbouring nodes differ by O(1) of the table's scale
    t = np.linspace(0.0, 1.0, n_table)
    c = I.random_vector(8, 40)
    h = 1e6 * sum(c[j] * np.sin(2 * np.pi * (j + 1) * t + c[4 + j]) for j in range(4))
    r = w.r_max[0]
    o = oracle.Oracle(w.c0, w.tx, w.pairs, w.grid.origin, w.grid.spacing, w.grid.dims, w.mask,
                      [r], tables=[h])
    ctx = f.Context(0)
    ctx.set_geometry(w.c0, w.tx, w.pairs, w.grid.origin, w.grid.spacing, w.grid.dims, w.mask)
    ctx.set_kernel_table(0, h, r)
    x = I.random_vector(w.n, 41) * 10.0
    y = I.random_vector(w.m, 42) * 1e-7
    yr, xr = o.apply_J(x), o.apply_JT(y)
    for prec, dt, bar in ((f.FP64, torch.float64, 1e-11), (f.FP32, torch.float32, 1e-5)):
        ej = rel(host(ctx.apply_J(dev(x, dt), prec=prec)), yr)
        et = rel(host(ctx.apply_JT(dev(y, dt), prec=prec)), xr)
        say("table", n_table, prec, "J %.2e J^T %.2e" % (ej, et))
        assert ej <= bar and et <= bar


@pytest.mark.parametrize("tail", ["built", "raised"])
def test_table_tail_forms(tail):
    """Two bands from the library's table builder (top node ~1e-7 of max|h|:
    the FP32 node table stores it as 0 and the J / multi-band J^T lookups
    drop the truncation select), and the same tables with the top node
    raised to 1e-3 of max|h| (kept as given, truncation by the select).
    Both match the oracle given the same tables to the FP32 bar."""
    f = _fftt()
    tx = I.ring(16, 0.006)
    g = I.centred_grid((13, 11, 6), 0.5e-3)
    fcs = (1e6, 2e6)
    w = I.Workload(name="tail", c0=1500.0, tx=tx, pairs=I.all_ordered_pairs(16), grid=g,
                   mask=I.cylinder_mask(g, None), pulses=[I.sampled_pulse(fc, 1.0) for fc in fcs],
                   r_max=[I.R_MAX[fc] for fc in fcs], n_table=4096)
    tabs = []
    for p in w.pulses:
        h, rm = f.build_table_from_pulse(w.c0, p.samples, p.dt, w.n_table, w.r_max[len(tabs)])
        h = np.array(h, dtype=np.float64)
        if tail == "raised":
            h[-1] = 1e-3 * np.abs(h).max()
        tabs.append((h, rm))
    o = oracle.Oracle(w.c0, w.tx, w.pairs, w.grid.origin, w.grid.spacing, w.grid.dims, w.mask,
                      [rm for _, rm in tabs], tables=[h for h, _ in tabs])
    ctx = f.Context(0)
    ctx.set_geometry(w.c0, w.tx, w.pairs, w.grid.origin, w.grid.spacing, w.grid.dims, w.mask)
    for b, (h, rm) in enumerate(tabs):
        ctx.set_kernel_table(b, h, rm)
    x = I.random_vector(w.n, 43) * 10.0
    y = I.random_vector(w.m * 2, 44) * 1e-7
    yr = np.asarray(o.apply_J(x)).ravel()          # [band][pair]
    xr = o.apply_JT(y)                              # summed over bands
    yg = host(ctx.apply_J(dev(x, torch.float32), prec=f.FP32))
    xg = host(ctx.apply_JT(dev(y, torch.float32), prec=f.FP32))
    ej, et = rel(yg, yr), rel(xg, xr)
    say("tail", tail, "J %.2e J^T %.2e" % (ej, et))
    assert ej <= 1e-5 and et <= 1e-5
    zero = np.flatnonzero(yr == 0.0)
    assert np.all(yg[zero] == 0.0)


def test_invalid_input_statuses():
    f = _fftt()
    ctx = f.Context(0)
    g = I.centred_grid((4, 4, 4), 1e-3)
    tx = I.ring(4, 0.03)
    ok_pairs = np.array([[0, 1]], dtype=np.int32)

    def geom(tx_=tx, pairs=ok_pairs, dims=g.dims, spacing=g.spacing, mask=None, c0=1500.0):
        ctx.set_geometry(c0, tx_, pairs, g.origin, spacing, dims, mask)

    x = torch.zeros(g.n, dtype=torch.float32, device="cuda:0")
    with pytest.raises(f.FFTTError) as e:          # nothing set yet
        ctx.prepare()
    assert e.value.status == -4
    for bad in (dict(tx_=tx[:1]), dict(pairs=np.array([[1, 1]], np.int32)),
                dict(pairs=np.array([[0, 9]], np.int32)), dict(dims=(4, 0, 4)),
                dict(spacing=(1e-3, -1e-3, 1e-3)), dict(c0=0.0),
                dict(tx_=np.array([[0.0, 0.0, np.nan], [0.03, 0, 0], [0, 0.03, 0]])),
                # transducer on an active voxel centre
                dict(tx_=np.array([g.origin, [0.03, 0.0, 0.0]]))):
        with pytest.raises(f.FFTTError) as e:
            geom(**bad)
        assert e.value.status == -1, bad
    geom()
    with pytest.raises(f.FFTTError) as e:          # geometry but no table
        ctx.prepare()
    assert e.value.status == -4
    h = np.linspace(0.0, 1.0, 64)
    for band, hh, rm in ((4, h, 1e-3), (0, h[:1], 1e-3), (0, h, 0.0), (0, h * np.nan, 1e-3)):
        with pytest.raises(f.FFTTError) as e:
            ctx.set_kernel_table(band, hh, rm)
        assert e.value.status == -1
    ctx.set_kernel_table(0, h, 1e-3)
    with pytest.raises(f.FFTTError):               # a second band of another length
        ctx.set_kernel_table(1, h[:32], 1e-3)
    with pytest.raises(TypeError):                 # buffer dtype must match the precision
        ctx.apply_J(torch.zeros(g.n, dtype=torch.float64, device="cuda:0"), prec=f.FP32)
    with pytest.raises(ValueError):                # and its size the grid
        ctx.apply_J(torch.zeros(g.n + 1, dtype=torch.float32, device="cuda:0"), prec=f.FP32)
    with pytest.raises(f.FFTTError):
        ctx.psf(np.array([g.n]), 5e-9)
    ctx.apply_J(x, prec=f.FP32)
    torch.cuda.synchronize()
