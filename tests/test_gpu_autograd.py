"""torch.autograd wrapper of J (backward = the J^T kernel), TV and L-BFGS."""
import numpy as np
import pytest

import oracle
from oracle import solvers
from paper_1908_03302_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def F():
    from paper_1908_03302_amd import fftt
    return fftt


def tiny_workload():
    g = I.centred_grid((10, 9, 6), 1.5e-3)
    return I.Workload(name="tiny", c0=1500.0, tx=I.ring(8, 0.03), pairs=I.all_ordered_pairs(8),
                      grid=g, mask=I.cylinder_mask(g, 0.02), pulses=[I.sampled_pulse(1e6, 1.0)],
                      r_max=[I.R_MAX[1e6]], n_table=4096)


def test_gradcheck_fp64_tiny():
    from paper_1908_03302_amd.autograd import apply_J
    w = tiny_workload()
    ctx = F().context_for_workload(w)
    x = torch.tensor(I.random_vector(w.n, 3), dtype=torch.float64, device="cuda:0",
                     requires_grad=True)
    assert torch.autograd.gradcheck(lambda v: apply_J(ctx, v, F().FP64) * 1e6, (x,),
                                    eps=1e-3, atol=1e-9, rtol=1e-7)


@pytest.fixture(scope="module")
def multiband():
    w = I.multiband()
    print("fixture multiband:", w.name, flush=True)
    ctx = F().context_for_workload(w)
    ctx.prepare()
    return w, ctx


def _objective(w, ctx, x, d, prec, alpha_tv=2e-12, beta=0.1):
    from paper_1908_03302_amd.autograd import misfit_tv
    return misfit_tv(ctx, x, d, w.noise_sigma, alpha_tv, beta, w.grid.dims, w.grid.spacing, prec)


def test_multiband_gradient_fd_on_central_subgrid(multiband):
    """Config-4 objective (4 bands, TV): directional derivatives along 32
    seeded directions supported on the central 32x32x16 subgrid, autograd
    (J^T kernel) vs central differences, FP64; FP32 gradient vs FP64."""
    w, ctx = multiband
    f = F()
    dev = "cuda:0"
    d = ctx.apply_J(torch.tensor(w.model, dtype=torch.float64, device=dev), prec=f.FP64)
    d = d + torch.tensor(I.noise(d.numel(), w.noise_sigma, w.noise_seed), dtype=torch.float64,
                         device=dev)
    x0 = torch.tensor(0.5 * w.model, dtype=torch.float64, device=dev)
    x = x0.clone().requires_grad_(True)
    fx = _objective(w, ctx, x, d, f.FP64)
    fx.backward()
    g = x.grad.detach().cpu().numpy()
    nx, ny, nz = w.grid.dims
    sub = np.zeros((nz, ny, nx), dtype=bool)
    sub[nz // 2 - 8:nz // 2 + 8, ny // 2 - 16:ny // 2 + 16, nx // 2 - 16:nx // 2 + 16] = True
    sub = sub.ravel()
    rng = np.random.default_rng(17)
    worst = 0.0
    for k in range(32):
        dirn = np.zeros(w.n)
        dirn[sub] = rng.standard_normal(sub.sum())
        eps = 1e-2
        dd = torch.tensor(dirn, dtype=torch.float64, device=dev)
        with torch.no_grad():
            fp = _objective(w, ctx, x0 + eps * dd, d, f.FP64)
            fm = _objective(w, ctx, x0 - eps * dd, d, f.FP64)
        fd = float((fp - fm) / (2 * eps))
        an = float(g @ dirn)
        worst = max(worst, abs(fd - an) / abs(an))
    print("FD worst rel", worst, flush=True)
    assert worst < 1e-6
    x32 = x0.float().clone().requires_grad_(True)
    _objective(w, ctx, x32, d.float(), f.FP32).backward()
    g32 = x32.grad.detach().cpu().double().numpy()
    e = np.linalg.norm(g32[sub] - g[sub]) / np.linalg.norm(g[sub])
    print("FP32 vs FP64 gradient on subgrid", e, flush=True)
    assert e < 1e-4


def test_tv_lbfgs_reduces_objective():
    from paper_1908_03302_amd.autograd import invert_tv
    w = I.small_fp64()
    f = F()
    ctx = f.context_for_workload(w)
    d = ctx.apply_J(torch.tensor(w.model, dtype=torch.float32, device="cuda:0"), prec=f.FP32)
    x, hist = invert_tv(ctx, d, w.noise_sigma, 1e-12, 0.1, w.grid.dims, w.grid.spacing, iters=15,
                        prec=f.FP32)
    print("lbfgs objective", hist[0], "->", hist[-1], flush=True)
    assert hist[-1] < 0.05 * hist[0]
    assert torch.isfinite(x).all()


@pytest.fixture(scope="module")
def multiband_subgrid():
    """The four-band workload (0.5 / 1 / 1.5 / 2 MHz, the 128-element ring)
    on the central 32x32x16 block of its 256x256x64 grid (the same voxel
    lattice), a model with structure in every direction, data from the
    table oracle plus 5 ns noise, and the oracle's objective of eq.
    leastSquare_misfit1 with the TV term (value and gradient)."""
    w = I.multiband(dims=(32, 32, 16))
    print("fixture multiband subgrid: oracle objective", flush=True)
    ot = oracle.Oracle.from_workload(w, table_mode=True)
    x_true = w.model + 8.0 * I.random_vector(w.n, 51)
    x = 0.5 * x_true + 3.0 * I.random_vector(w.n, 52)
    B, M = w.n_bands, w.m
    d = ot.apply_J(x_true).reshape(B, M) + I.noise(B * M, w.noise_sigma, 53).reshape(B, M)
    cache = {}

    def J_all(v):
        key = id(v)
        if key not in cache:
            cache.clear()
            cache[key] = ot.apply_J(v).reshape(B, M)
        return cache[key]

    def JT_band(b):
        def f(r):
            y = np.zeros((B, M))
            y[b] = r
            return ot.apply_JT(y)
        return f

    ops = [(lambda v, b=b: J_all(v)[b], JT_band(b)) for b in range(B)]
    beta = 0.1
    mis0, _ = solvers.tv_objective(ops, list(d), w.noise_sigma, 0.0, beta, w.grid.dims,
                                   w.grid.spacing, x)
    tv0, _ = solvers.tv(x, w.grid.dims, w.grid.spacing, beta)
    alpha = 0.3 * mis0 / tv0        # both terms of the objective matter
    chi, grad = solvers.tv_objective(ops, list(d), w.noise_sigma, alpha, beta, w.grid.dims,
                                     w.grid.spacing, x)
    return w, x, d, alpha, beta, chi, grad


@pytest.mark.parametrize("prec_name,tol", [("FP64", 1e-10), ("FP32", 1e-5)])
def test_multiband_objective_and_gradient_match_oracle(multiband_subgrid, prec_name, tol):
    """misfit_tv (four bands in one launch, TV) and its autograd gradient
    (J^T kernel) against the oracle's tv_objective on the same inputs:
    relative error of the value and norm-wise error of the gradient within
    1e-10 (FP64) / 1e-5 (FP32)."""
    from paper_1908_03302_amd.autograd import misfit_tv
    w, x, d, alpha, beta, chi, grad = multiband_subgrid
    f = F()
    prec = getattr(f, prec_name)
    dt = torch.float64 if prec == f.FP64 else torch.float32
    ctx = F().context_for_workload(w)
    xt = torch.tensor(x, dtype=dt, device="cuda:0", requires_grad=True)
    dd = torch.tensor(d.ravel(), dtype=dt, device="cuda:0")
    val = misfit_tv(ctx, xt, dd, w.noise_sigma, alpha, beta, w.grid.dims, w.grid.spacing, prec)
    val.backward()
    g = xt.grad.detach().cpu().double().numpy()
    ev = abs(float(val.detach()) - chi) / abs(chi)
    eg = np.linalg.norm(g - grad) / np.linalg.norm(grad)
    print("multiband subgrid", prec_name, "objective rel err %.2e, gradient %.2e" % (ev, eg),
          flush=True)
    assert ev < tol and eg < tol
