"""Staged kernels over several transducer blocks (through the C ABI).

A stack of rings with pairs inside each ring, as in the slice-by-slice
workload: with the staged block capped below the transducer count, a tile's
entries are processed one block (ring) at a time.  Every block size gives
the same operator as the oracle within the FP32 / FP64 bars.
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


def ring_stack(n_per_ring=32, zs=(-0.006, -0.002, 0.002, 0.006)):
    g = I.centred_grid((37, 31, 17), 1.0e-3)
    tx = np.concatenate([I.ring(n_per_ring, 0.03, z, phase=0.05 * k) for k, z in enumerate(zs)])
    pairs = np.concatenate([I.all_ordered_pairs(n_per_ring, k * n_per_ring)
                            for k in range(len(zs))])
    return I.Workload(
        name="ringstack", c0=1500.0, tx=tx, pairs=pairs, grid=g, mask=I.cylinder_mask(g, 0.022),
        pulses=[I.sampled_pulse(1e6, 1.0)], r_max=[I.R_MAX[1e6]], n_table=4096)


@pytest.fixture(scope="module")
def stack():
    w = ring_stack()
    o = oracle.Oracle.from_workload(w)
    ot = oracle.Oracle.from_workload(w, table_mode=True)
    ctx = _fftt().context_for_workload(w)
    ctx.prepare()
    x = I.random_vector(w.n, 90) * 3.0 * w.mask
    y = I.random_vector(w.m, 91) * 1e-7
    return w, ctx, x, y, (o.apply_J(x), o.apply_JT(y)), (ot.apply_J(x), ot.apply_JT(y))


@pytest.mark.parametrize("block,staged,unroll", [(32, 1, 8), (64, 1, 4), (0, 1, 8), (32, 1, 1),
                                                 (0, 0, 4)])
def test_block_sizes_agree_with_oracle(stack, block, staged, unroll):
    w, ctx, x, y, (yq, xq), (yt, xt) = stack
    f = _fftt()
    ctx.set_tuning(staged=staged, staged_block=block, unroll_jt_staged=unroll,
                   unroll_j_staged=unroll)
    try:
        for prec in (f.FP32, f.FP32_BF16TABLE, f.FP64):
            Jx = host(ctx.apply_J(dev(x, prec), prec=prec))
            JTy = host(ctx.apply_JT(dev(y, prec), prec=prec))
            if prec == f.FP64:
                assert rel(Jx, yt) < 1e-11 and rel(JTy, xt) < 1e-11
            else:
                bar = 1e-5 if prec == f.FP32 else 1e-3
                ej, et = rel(Jx, yq), rel(JTy, xq)
                say("blocks", block, "staged", staged, "prec", prec, "J", ej, "J^T", et)
                assert ej < bar and et < bar
    finally:
        ctx.set_tuning(staged=1, staged_block=0, unroll_jt_staged=8, unroll_j_staged=4)
