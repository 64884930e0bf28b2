"""Sensitivity coverage sum_i |J_ij| (Sec. III), diag(J^T J) and the
Jacobi-preconditioned CGLS built on it, through the C ABI, against the CPU
FP64 oracle's dense operator.

Bars, norm-wise over the active voxels: with the table, 1e-5 against the
oracle's own linear-table mode and, against quadrature, the table's own
interpolation error (table oracle vs quadrature oracle) plus 1e-5; with the
sine series, 1e-5 against quadrature directly.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import solvers
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


def dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def reductions(blocks):
    """(sum |J|, sum J^2) over rows and bands of the dense blocks."""
    return (sum(np.abs(B).sum(axis=0) for B in blocks),
            sum((B ** 2).sum(axis=0) for B in blocks))


def check(got, ref_q, ref_t, what):
    e_t, e_q, e_tab = rel(got, ref_t), rel(got, ref_q), rel(ref_t, ref_q)
    say("%s: rel err vs table oracle %.2e, vs quadrature %.2e (table's own %.2e)"
        % (what, e_t, e_q, e_tab))
    assert e_t < 1e-5
    assert e_q < e_tab + 1e-5


@pytest.fixture(scope="module")
def small():
    w = I.small_fp64()
    say("fixture small:", w.name)
    o = oracle.Oracle.from_workload(w)
    ot = oracle.Oracle.from_workload(w, table_mode=True)
    ctx = _fftt().context_for_workload(w, series=True)
    ctx.prepare()
    return w, o.block(), ot.block(), ctx


@pytest.mark.parametrize("kind", [0, 1])
def test_small_coverage_and_diag(small, kind):
    w, Jq, Jt, ctx = small
    got = host(ctx.coverage(kind))
    check(got, reductions([Jq])[kind], reductions([Jt])[kind], "small kind %d" % kind)
    ctx.set_tuning(kernel_eval=1)
    try:
        gs = host(ctx.coverage(kind))
    finally:
        ctx.set_tuning(kernel_eval=0)
    es = rel(gs, reductions([Jq])[kind])
    say("small kind %d series: rel err vs quadrature %.2e" % (kind, es))
    assert es < 1e-5
    # BF16 table
    gb = host(ctx.coverage(kind, prec=_fftt().FP32_BF16TABLE))
    assert rel(gb, reductions([Jq])[kind]) < 1e-3


def test_ragged_two_bands_with_repeats_and_missing_reverses():
    """Caller pairs with repeats and pairs without their reverse: every
    caller pair counts once per band; inactive voxels are 0."""
    f = _fftt()
    g = I.centred_grid((37, 29, 11), 1.0e-3)
    tx = I.ring(24, 0.03, 0.0005, phase=0.1)
    pairs = I.all_ordered_pairs(24)
    rng = np.random.default_rng(8)
    keep = rng.random(len(pairs)) < 0.6
    pairs = np.concatenate([pairs[keep], pairs[rng.choice(len(pairs), 40)]]).astype(np.int32)
    w = I.Workload(name="ragged_rep", c0=1500.0, tx=tx, pairs=pairs, grid=g,
                   mask=I.cylinder_mask(g, 0.02),
                   pulses=[I.sampled_pulse(1e6, 1.0), I.sampled_pulse(2e6, 1.0)],
                   r_max=[I.R_MAX[1e6], I.R_MAX[2e6]], n_table=4096)
    o = oracle.Oracle.from_workload(w)
    ot = oracle.Oracle.from_workload(w, table_mode=True)
    ctx = f.context_for_workload(w)
    for kind in (0, 1):
        got = host(ctx.coverage(kind))
        assert np.all(got[w.mask == 0] == 0.0)
        check(got, reductions([o.block(band=b) for b in range(2)])[kind],
              reductions([ot.block(band=b) for b in range(2)])[kind], "ragged kind %d" % kind)


def test_ring2d_coverage_sampled_columns():
    """Full-size 128-element ring: coverage and diag at 256 sampled active
    voxels against the oracle's columns (quadrature; the 1 MHz table's own
    error is below 1e-6 here)."""
    w = I.ring2d()
    f = _fftt()
    say("ring2d coverage: set-up")
    ctx = f.context_for_workload(w)
    ctx.prepare()
    o = oracle.Oracle.from_workload(w)
    act = np.flatnonzero(w.mask)
    cols = np.sort(np.random.default_rng(31).choice(act, 256, replace=False))
    B = o.block(cols=cols)
    cov, dia = host(ctx.coverage(0)), host(ctx.coverage(1))
    e0, e1 = rel(cov[cols], np.abs(B).sum(axis=0)), rel(dia[cols], (B ** 2).sum(axis=0))
    say("ring2d sampled coverage %.2e diag %.2e" % (e0, e1))
    assert e0 < 1e-5 and e1 < 1e-5


# ------------------------------------------------------------ Jacobi PCG

ALPHA = I.ALPHA_SMALL


@pytest.fixture(scope="module")
def solve_case(small):
    w, Jq, Jt, ctx = small
    sig = w.noise_sigma
    d = Jt @ w.model + I.noise(w.m, sig, w.noise_seed)
    minv = 1.0 / ((Jt ** 2).sum(axis=0) / sig ** 2 + ALPHA)
    return w, Jt, ctx, d, sig, minv


# Relative accuracy of the FP32 coverage pass's diag(J^T J) on the small
# ring: the table-oracle comparison above measures ~1.2e-7 norm-wise.
DIAG_FP32 = 3e-7


def test_pcgls_fp64_tracks_oracle_pcgls(solve_case):
    """FP64 operators and vectors; the diagonal comes from the FP32 coverage
    pass, the oracle's from its dense table-mode matrix.  Twenty iterations
    are far from convergence, where the iterate amplifies a change of the
    Jacobi diagonal several hundred times: the bar is 1e-5 plus what the
    oracle's own PCGLS moves when its diagonal is perturbed at the FP32
    pass's accuracy (random relative perturbations of size DIAG_FP32, the
    largest of four draws); likewise for the final misfit."""
    w, Jt, ctx, d, sig, minv = solve_case
    f = _fftt()
    x = dev(np.zeros(w.n), torch.float64)
    rep = ctx.solve(dev(d, torch.float64), x, method=0, prec=f.FP64, alpha=ALPHA,
                    noise_sigma=sig, max_iter=20, precond=True)
    A, At = (lambda v: Jt @ v), (lambda v: Jt.T @ v)
    xr, hist = solvers.pcgls(A, At, d, sig, ALPHA, minv, 20)
    dg = (Jt ** 2).sum(axis=0) / sig ** 2
    dx = dm = 0.0
    for k in range(4):
        z = np.random.default_rng(100 + k).standard_normal(dg.size)
        xk, hk = solvers.pcgls(A, At, d, sig, ALPHA, 1.0 / (dg * (1 + DIAG_FP32 * z) + ALPHA), 20)
        dx, dm = max(dx, rel(xk, xr)), max(dm, abs(hk[-1] / hist[-1] - 1))
    e = rel(host(x), xr)
    say("PCGLS fp64 20 its rel err vs oracle %.2e (oracle's own spread %.2e), misfit %.6e vs "
        "%.6e (spread %.2e)" % (e, dx, rep["misfit"], hist[-1], dm))
    assert rep["iters"] == 20
    assert e < 1e-5 + dx
    assert abs(rep["misfit"] / hist[-1] - 1) < 1e-6 + dm


def test_pcgls_converges_to_direct_solution(solve_case):
    w, Jt, ctx, d, sig, minv = solve_case
    f = _fftt()
    x = dev(np.zeros(w.n), torch.float64)
    rep = ctx.solve(dev(d, torch.float64), x, method=0, prec=f.FP64, alpha=ALPHA,
                    noise_sigma=sig, max_iter=600, rel_tol=1e-11, precond=True)
    A = Jt.T @ Jt / sig ** 2 + ALPHA * np.eye(w.n)
    xd = np.linalg.solve(A, Jt.T @ d / sig ** 2)
    e = rel(host(x), xd)
    say("PCGLS long: iters", rep["iters"], "rel err vs direct %.2e" % e)
    assert rep["rel_resid"] <= 1e-11
    assert e < 1e-7


@pytest.mark.parametrize("prec_name", ["FP64", "FP32"])
def test_pcgls_graph_replays_match_eager(solve_case, prec_name):
    w, Jt, ctx, d, sig, minv = solve_case
    f = _fftt()
    prec = getattr(f, prec_name)
    dt = torch.float64 if prec == f.FP64 else torch.float32
    out = []
    for graph in (False, True, True):
        x = dev(np.zeros(w.n), dt)
        ctx.solve(dev(d, dt), x, method=0, prec=prec, alpha=ALPHA, noise_sigma=sig,
                  max_iter=12, precond=True, graph=graph)
        out.append(host(x))
        ctx.apply_J(dev(w.model), prec=f.FP32)     # eager work between the solves
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_mixed_pcgls_tracks_fp64(solve_case):
    w, Jt, ctx, d, sig, minv = solve_case
    f = _fftt()
    xs = []
    for prec, dt in ((f.FP64, torch.float64), (f.FP32, torch.float32)):
        x = dev(np.zeros(w.n), dt)
        ctx.solve(dev(d, dt), x, method=0, prec=prec, alpha=ALPHA, noise_sigma=sig,
                  max_iter=20, precond=True)
        xs.append(host(x))
    assert rel(xs[1], xs[0]) < 1e-3


def test_coverage_and_precond_errors(solve_case):
    w, Jt, ctx, d, sig, minv = solve_case
    f = _fftt()
    with pytest.raises(f.FFTTError) as e:
        ctx.coverage(0, out=torch.empty(w.n, dtype=torch.float32, device="cuda:0"), prec=f.FP64)
    assert e.value.status == -5
    with pytest.raises(f.FFTTError):
        ctx.coverage(2)
    with pytest.raises(f.FFTTError):       # Jacobi is for CGLS only
        ctx.solve(dev(d), dev(np.zeros(w.n)), method=1, prec=f.FP32, alpha=ALPHA,
                  noise_sigma=sig, max_iter=2, precond=True)
    ctx.set_tuning(staged=0)
    try:
        with pytest.raises(f.FFTTError) as e:
            ctx.coverage(0)
        assert e.value.status == -5
    finally:
        ctx.set_tuning(staged=1)
    torch.cuda.synchronize()
