"""More transducers than the staged kernels take (Sec. II: any set of
transducer pairs): 16 400 ring elements, of which a few dozen pairs are
used, indices on both sides of 16 384.  The staged kernels' entry copies
hold 14-bit transducer indices, so such a geometry must run on the
per-wavefront kernels: J and J^T are checked against the CPU FP64 oracle
(table mode; FP64 path to 1e-11, FP32 to 1e-5), and the staged-only
coverage pass must refuse with FFTT_E_UNSUPPORTED rather than run.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1908_03302_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_more_transducers_than_staged_indices():
    from paper_1908_03302_amd import fftt
    n_tx = 16400
    tx = I.ring(n_tx, 0.04)
    # nearly opposite elements: chords through the small central grid, with
    # sources and receivers below and above index 16 384
    s = np.array([3, 100, 4000, 8150, 8195, 8199, 16383, 16384, 16390, 16399, 7000, 12000])
    pairs = np.stack([s, (s + n_tx // 2 + np.arange(len(s)) % 5 - 2) % n_tx], 1).astype(np.int32)
    pairs = np.concatenate([pairs, pairs[:, ::-1]])
    g = I.centred_grid((9, 8, 5), 1.5e-3)
    w = I.Workload(name="many_tx", c0=1500.0, tx=tx, pairs=pairs, grid=g,
                   mask=I.cylinder_mask(g, None), pulses=[I.sampled_pulse(1e6, 1.0)],
                   r_max=[I.R_MAX[1e6]], n_table=4096)
    ot = oracle.Oracle.from_workload(w, table_mode=True)
    ctx = fftt.context_for_workload(w)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(w.n)
    y = rng.standard_normal(w.m) * 1e-7
    yr, xr = ot.apply_J(x), ot.apply_JT(y)
    assert np.linalg.norm(yr) > 0 and np.linalg.norm(xr) > 0
    for name, prec, dt in (("FP64", fftt.FP64, torch.float64), ("FP32", fftt.FP32, torch.float32)):
        yg = ctx.apply_J(torch.tensor(x, dtype=dt, device="cuda:0"), prec=prec)
        xg = ctx.apply_JT(torch.tensor(y, dtype=dt, device="cuda:0"), prec=prec)
        torch.cuda.synchronize()
        ej = rel(yg.cpu().numpy(), yr)
        et = rel(xg.cpu().numpy(), xr)
        print(name, "J %.2e J^T %.2e" % (ej, et), flush=True)
        sys.stdout.flush()
        bar = 1e-11 if prec == fftt.FP64 else 1e-5
        assert ej <= bar and et <= bar
    with pytest.raises(fftt.FFTTError) as exc:
        ctx.coverage(0)
    assert "UNSUPPORTED" in str(exc.value)
