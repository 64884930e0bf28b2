"""The J^T entry point that allocates nothing (fftt_apply_JT_noalloc),
through the C ABI, against fftt_apply_JT on the same inputs: two calls in a
row on the same device, the second with a smaller input (so the scratch
array still holds the first call's larger contents), then the 2D mode (its
prism buffer also in the scratch array), the size limit and the state
check.  Both entry points run the same kernels on the same weights, so the
outputs must be bitwise equal; the first is also held to the FP32 bar
against the oracle."""
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


def dev(x, dt):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dt).to("cuda:0").contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _pair(ctx, prec, dt, y, n):
    a = torch.full((n,), float("nan"), dtype=dt, device="cuda:0")
    b = torch.full((n,), float("nan"), dtype=dt, device="cuda:0")
    ctx.apply_JT(dev(y, dt), a, prec=prec)
    ctx.apply_JT_noalloc(dev(y, dt), b, prec=prec)
    return host(a), host(b)


def test_noalloc_two_calls_second_smaller():
    f = F()
    # call 1: the lab-like ring (128 elements, 256x256x64 grid), FP32
    w1 = I.ring2d()
    say("no-alloc call 1:", w1.name)
    c1 = f.context_for_workload(w1)
    c1.prepare()
    y1 = I.random_vector(w1.m, 71) * 1e-7
    a1, b1 = _pair(c1, f.FP32, torch.float32, y1, w1.n)
    assert np.array_equal(a1, b1)
    o1 = oracle.Oracle.from_workload(w1)
    cols = np.sort(np.random.default_rng(72).choice(np.flatnonzero(w1.mask), 512, replace=False))
    ref = o1.cols(cols, y1)
    e1 = float(np.linalg.norm(b1[cols] - ref) / np.linalg.norm(ref))
    say("no-alloc call 1: bitwise equal to apply_JT; sampled columns vs oracle %.2e" % e1)
    assert e1 < 1e-5
    # call 2: a smaller input on the same device (ragged grid, two bands, FP64)
    g = I.centred_grid((37, 29, 11), 1.0e-3)
    w2 = I.Workload(name="ragged", c0=1500.0, tx=I.ring(24, 0.03, 0.0005, phase=0.1),
                    pairs=I.all_ordered_pairs(24), grid=g, mask=I.cylinder_mask(g, 0.02),
                    pulses=[I.sampled_pulse(1e6, 1.0), I.sampled_pulse(2e6, 1.0)],
                    r_max=[I.R_MAX[1e6], I.R_MAX[2e6]], n_table=4096)
    say("no-alloc call 2:", w2.name, "FP64")
    c2 = f.context_for_workload(w2)
    c2.prepare()
    y2 = I.random_vector(2 * w2.m, 73) * 1e-7
    a2, b2 = _pair(c2, f.FP64, torch.float64, y2, w2.n)
    assert np.array_equal(a2, b2)
    ot = oracle.Oracle.from_workload(w2, table_mode=True)
    e2 = float(np.linalg.norm(b2 - ot.apply_JT(y2)) / np.linalg.norm(b2))
    say("no-alloc call 2: bitwise equal to apply_JT; vs table oracle %.2e" % e2)
    assert e2 < 1e-11
    # and the larger context once more, after the smaller call
    a3, b3 = _pair(c1, f.FP32, torch.float32, y1, w1.n)
    assert np.array_equal(b3, b1) and np.array_equal(a3, b3)


def test_noalloc_plane_and_limits():
    f = F()
    w = I.plane128()
    say("no-alloc 2D:", w.name)
    ctx = f.context_for_workload(w)
    ctx.prepare()
    y = I.random_vector(w.m, 74) * 1e-7
    a, b = _pair(ctx, f.FP32, torch.float32, y, w.n)
    assert np.array_equal(a, b)
    # FP64 needs the prism's 3.9 M doubles: more than the scratch array holds
    out = torch.empty(w.n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(f.FFTTError) as e:
        ctx.apply_JT_noalloc(dev(y, torch.float64), out, prec=f.FP64)
    assert e.value.status == -1
    # a context whose tables were never prepared is refused, not prepared
    w2 = I.small_fp64()
    c2 = f.Context(0)
    c2.set_geometry(w2.c0, w2.tx, w2.pairs, w2.grid.origin, w2.grid.spacing, w2.grid.dims,
                    w2.mask)
    p = w2.pulses[0]
    h, rm = f.build_table_from_pulse(w2.c0, p.samples, p.dt, w2.n_table, w2.r_max[0])
    c2.set_kernel_table(0, h, rm)
    out2 = torch.empty(w2.n, dtype=torch.float32, device="cuda:0")
    with pytest.raises(f.FFTTError) as e:
        c2.apply_JT_noalloc(dev(np.zeros(w2.m), torch.float32), out2, prec=f.FP32)
    assert e.value.status == -4
    c2.prepare()
    y2 = I.random_vector(w2.m, 75) * 1e-7
    a2, b2 = _pair(c2, f.FP32, torch.float32, y2, w2.n)
    assert np.array_equal(a2, b2)
