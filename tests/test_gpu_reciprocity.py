"""Source-receiver reciprocity in the operators (through the C ABI).

The detour R_xs + R_xr - L and L are symmetric in source and receiver, so
rows (s, r) and (r, s) of J are equal (Sec. II, the reciprocity of the
Green's function).  The library evaluates each unordered pair once by
default; these tests check that the outputs
match the oracle either way, that reversed rows come out identical, and
that pair sets with missing reverses or repeated pairs are handled.
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


def workload(pairs):
    g = I.centred_grid((29, 23, 9), 1.0e-3)
    tx = I.ring(20, 0.025, 0.0004, phase=0.2)
    return I.Workload(
        name="recip", c0=1500.0, tx=tx, pairs=pairs, grid=g, mask=I.cylinder_mask(g, 0.016),
        pulses=[I.sampled_pulse(1e6, 1.0), I.sampled_pulse(1.5e6, 1.0)],
        r_max=[I.R_MAX[1e6], I.R_MAX[1.5e6]], n_table=4096)


def mixed_pairs():
    """All ordered pairs of 20, then: drop the reverse of every third
    unordered pair and repeat a few pairs (some twice)."""
    P = I.all_ordered_pairs(20)
    keep = [i for i, (s, r) in enumerate(P) if not (s > r and (r + 7 * s) % 3 == 0)]
    P = P[keep]
    return np.concatenate([P, P[[5, 40, 40, 123]]])


@pytest.mark.parametrize("which", ["all", "mixed"])
def test_reciprocity_on_off_agree_with_oracle(which):
    f = _fftt()
    pairs = I.all_ordered_pairs(20) if which == "all" else mixed_pairs()
    w = workload(pairs)
    o = oracle.Oracle.from_workload(w)
    ot = oracle.Oracle.from_workload(w, table_mode=True)
    ctx = f.context_for_workload(w)
    x = I.random_vector(w.n, 80) * 4.0 * w.mask
    y = I.random_vector(2 * w.m, 81) * 1e-7
    yq, xq = o.apply_J(x), o.apply_JT(y)
    yt, xt = ot.apply_J(x), ot.apply_JT(y)
    res = {}
    for rec in (1, 0):
        ctx.set_tuning(reciprocity=rec)
        ctx.prepare()
        pv, pve, _ = ctx.work_count()
        assert pv == o.count_pv()
        if which == "all":   # no repeats: every pair's reverse is present
            assert pve == (pv // 2 if rec else pv)
        else:                # exact repeats always share one evaluation
            assert pve < pv
        for prec in (f.FP32, f.FP64):
            Jx = host(ctx.apply_J(dev(x, prec), prec=prec)).reshape(2, -1)
            JTy = host(ctx.apply_JT(dev(y, prec), prec=prec))
            if prec == f.FP64:
                assert rel(Jx, yt) < 1e-11 and rel(JTy, xt) < 1e-11
            else:
                assert rel(Jx, yq) < 1e-5 and rel(JTy, xq) < 1e-5
            res[(rec, prec)] = (Jx, JTy)
        say(which, "reciprocity", rec, "pv", pv, "evaluated", pve)
    for prec, tol in ((f.FP32, 1e-6), (f.FP64, 1e-13)):
        a, b = res[(1, prec)], res[(0, prec)]
        assert rel(a[0], b[0]) < tol and rel(a[1], b[1]) < tol
    # rows of reversed pairs are identical (bitwise: one evaluation feeds both)
    Jx = res[(1, f.FP32)][0]
    idx = {tuple(p): i for i, p in enumerate(pairs)}
    n_rev = 0
    for i, (s_, r_) in enumerate(pairs):
        j = idx.get((r_, s_))
        if j is not None:
            assert np.array_equal(Jx[:, i], Jx[:, j])
            n_rev += 1
    assert n_rev > 0
    ctx.set_tuning(reciprocity=1)


@pytest.mark.parametrize("psf_math,tol", [(1, 1e-6), (0, 1e-5)])
def test_reciprocity_psf_batch(psf_math, tol):
    """Batched PSFs with and without merging reversed pairs agree: to FP32
    rounding with FP32 matrix cores, and to the three-way BF16 split's
    rounding (~4e-6, the groupings round differently) with the default."""
    f = _fftt()
    w = workload(mixed_pairs())
    ctx = f.context_for_workload(w)
    ctx.set_tuning(psf_math=psf_math)
    vox = np.flatnonzero(w.mask)[::97][:40]
    out = {}
    for rec in (1, 0):
        ctx.set_tuning(reciprocity=rec)
        ctx.prepare()
        out[rec] = host(ctx.psf(vox, 5e-9, prec=f.FP32)).reshape(len(vox), w.n)
    for k in range(len(vox)):
        assert rel(out[1][k], out[0][k]) < tol
    ctx.set_tuning(reciprocity=1, psf_math=0)
