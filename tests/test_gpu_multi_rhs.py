"""Several right-hand sides in one call (eq. forward_compact and its
transpose for a block of vectors): fftt_apply_J / fftt_apply_JT with
n_rhs >= 8 run as batches on the matrix cores (split-BF16 contractions per
tile).  Against the one-vector launches (FFTT_TUNE_RHS_BATCHED = 0) within
1e-5 norm-wise per vector, and against the oracle's table mode within the
FP32 bar (BF16 table: within 1e-5 of the one-vector path's own error, which
on sign-random vectors sits at that mode's 1e-3), on a ragged, masked two-band grid (partial
tiles, inactive voxels) for 8 and 40 vectors (one and two 32-column
blocks, the second partial), and on the lab-like ring for 32 vectors
(sampled rows and columns)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1908_03302_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def F():
    from paper_1908_03302_amd import fftt
    return fftt


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def ragged():
    g = I.centred_grid((37, 29, 11), 1.0e-3)
    return I.Workload(
        name="ragged", c0=1500.0, tx=I.ring(24, 0.03, 0.0005, phase=0.1),
        pairs=I.all_ordered_pairs(24), grid=g, mask=I.cylinder_mask(g, 0.02),
        pulses=[I.sampled_pulse(1e6, 1.0), I.sampled_pulse(2e6, 1.0)],
        r_max=[I.R_MAX[1e6], I.R_MAX[2e6]], n_table=4096)


@pytest.fixture(scope="module")
def ragged_ctx():
    w = ragged()
    say("fixture ragged multi-RHS")
    ctx = F().context_for_workload(w)
    ctx.prepare()
    ot = oracle.Oracle.from_workload(w, table_mode=True)
    Jt = [ot.block(band=b) for b in range(2)]
    return w, ctx, Jt


@pytest.mark.parametrize("prec_name", ["FP32", "FP32_BF16TABLE"])
@pytest.mark.parametrize("r", [8, 40])
def test_batched_J_and_JT(ragged_ctx, prec_name, r):
    w, ctx, Jt = ragged_ctx
    f = F()
    prec = getattr(f, prec_name)
    bar = 1e-5 if prec == f.FP32 else 1e-3
    X = np.stack([I.random_vector(w.n, 200 + k) for k in range(r)]) * w.mask
    Y = np.stack([I.random_vector(2 * w.m, 300 + k) for k in range(r)]) * 1e-7
    yb = host(ctx.apply_J(dev(X.ravel()), prec=prec, n_rhs=r)).reshape(r, 2, w.m)
    xb = host(ctx.apply_JT(dev(Y.ravel()), prec=prec, n_rhs=r)).reshape(r, w.n)
    ctx.set_tuning(rhs_batched=0)
    try:
        yl = host(ctx.apply_J(dev(X.ravel()), prec=prec, n_rhs=r)).reshape(r, 2, w.m)
        xl = host(ctx.apply_JT(dev(Y.ravel()), prec=prec, n_rhs=r)).reshape(r, w.n)
    finally:
        ctx.set_tuning(rhs_batched=1)
    ej = max(rel(yb[k], yl[k]) for k in range(r))
    et = max(rel(xb[k], xl[k]) for k in range(r))
    refj = [np.stack([Jt[b] @ X[k] for b in range(2)]) for k in range(r)]
    reft = [sum(Jt[b].T @ Y[k].reshape(2, w.m)[b] for b in range(2)) for k in range(r)]
    oj = [rel(yb[k], refj[k]) for k in range(r)]
    ot = [rel(xb[k], reft[k]) for k in range(r)]
    lj = [rel(yl[k], refj[k]) for k in range(r)]
    lt = [rel(xl[k], reft[k]) for k in range(r)]
    say("multi-RHS %s r=%d: batched vs one-vector J %.2e J^T %.2e; vs table oracle J %.2e "
        "J^T %.2e (one-vector path %.2e / %.2e)"
        % (prec_name, r, ej, et, max(oj), max(ot), max(lj), max(lt)))
    assert ej < 1e-5 and et < 1e-5
    if prec == f.FP32:
        assert max(oj) < bar and max(ot) < bar
    else:
        # the BF16 table's own error on sign-random vectors sits at its 1e-3
        # bar (one-vector path alike); batching adds at most 1e-5 to it
        assert all(o <= l + 1e-5 for o, l in zip(oj, lj))
        assert all(o <= l + 1e-5 for o, l in zip(ot, lt))
    assert np.all(xb[:, w.mask == 0] == 0.0)


def test_few_rhs_and_unsupported_modes_loop(ragged_ctx):
    """Fewer than eight vectors, and FP64, take the one-vector launches
    (bitwise equal to separate calls)."""
    w, ctx, Jt = ragged_ctx
    f = F()
    X = np.stack([I.random_vector(w.n, 400 + k) for k in range(3)]) * w.mask
    Y3 = host(ctx.apply_J(dev(X.ravel()), prec=f.FP32, n_rhs=3)).reshape(3, -1)
    for k in range(3):
        assert np.array_equal(Y3[k], host(ctx.apply_J(dev(X[k]), prec=f.FP32)))
    X8 = np.stack([I.random_vector(w.n, 500 + k) for k in range(8)]) * w.mask
    x64 = torch.as_tensor(X8.ravel(), dtype=torch.float64).to("cuda:0")
    Y8 = ctx.apply_J(x64, prec=f.FP64, n_rhs=8).cpu().numpy().reshape(8, -1)
    for k in range(8):
        one = ctx.apply_J(torch.as_tensor(X8[k], dtype=torch.float64).to("cuda:0"),
                          prec=f.FP64).cpu().numpy()
        assert np.array_equal(Y8[k], one)


def test_batched_lab_ring_sampled():
    """32 vectors on the 128-element ring (256x256x64): sampled rows and
    columns against the quadrature oracle (the table's own error plus the
    FP32 bar), and the batched call's time against 32 single calls."""
    import time
    w = I.ring2d()
    f = F()
    say("multi-RHS lab-like ring: set-up")
    ctx = f.context_for_workload(w)
    ctx.prepare()
    o = oracle.Oracle.from_workload(w)
    r = 32
    X = np.stack([w.model * (1.0 + 0.1 * k) + 5.0 * I.random_vector(w.n, 600 + k) * w.mask
                  for k in range(r)])
    Y = np.stack([I.random_vector(w.m, 700 + k) for k in range(r)]) * 1e-7
    xd, yd = dev(X.ravel()), dev(Y.ravel())
    outJ = torch.empty(r * w.m, dtype=torch.float32, device="cuda:0")
    outT = torch.empty(r * w.n, dtype=torch.float32, device="cuda:0")
    times = {}
    for batched in (1, 0):
        ctx.set_tuning(rhs_batched=batched)
        ctx.apply_J(xd, outJ, n_rhs=r)
        ctx.apply_JT(yd, outT, n_rhs=r)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.apply_J(xd, outJ, n_rhs=r)
        ctx.apply_JT(yd, outT, n_rhs=r)
        torch.cuda.synchronize()
        times[batched] = 1e3 * (time.perf_counter() - t0)
        if batched:
            yb, xb = host(outJ).reshape(r, w.m), host(outT).reshape(r, w.n)
    ctx.set_tuning(rhs_batched=1)
    rng = np.random.default_rng(8)
    rows = np.sort(rng.choice(w.m, 6, replace=False))
    cols = np.sort(rng.choice(np.flatnonzero(w.mask), 256, replace=False))
    worst_j = worst_t = 0.0
    for k in (0, 17, 31):
        worst_j = max(worst_j, rel(yb[k][rows], o.rows(rows, X[k])))
        worst_t = max(worst_t, rel(xb[k][cols], o.cols(cols, Y[k])))
    say("multi-RHS lab ring r=32: J+J^T batched %.1f ms, one at a time %.1f ms; sampled rows "
        "%.2e, columns %.2e vs quadrature" % (times[1], times[0], worst_j, worst_t))
    assert worst_j < 2e-5 and worst_t < 2e-5
