"""Solvers and point-spread functions through the C ABI vs the oracle.

The references use the oracle's own linear-table operator (dense, FP64) so
that only the solver arithmetic is compared; tolerances are stated per test.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import solvers
from paper_1908_03302_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ALPHA = 5e-3          # Tikhonov weight of the small ring workload (discrepancy principle)


def F():
    from paper_1908_03302_amd import fftt
    return fftt


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def dev(x, prec):
    dt = torch.float64 if prec == F().FP64 else torch.float32
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dt).to("cuda:0").contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def small():
    w = I.small_fp64()
    print("fixture small solver:", w.name, flush=True)
    ot = oracle.Oracle.from_workload(w, table_mode=True)
    Jd = ot.block()
    ctx = F().context_for_workload(w)
    d = Jd @ w.model + I.noise(w.m, w.noise_sigma, w.noise_seed)
    return w, Jd, ctx, d


def gpu_solve(ctx, d, prec, n, **kw):
    x = dev(np.zeros(n), prec)
    rep = ctx.solve(dev(d, prec), x, prec=prec, **kw)
    return host(x), rep


def test_cgls_fp64_matches_oracle_cgls(small):
    w, Jd, ctx, d = small
    sig = w.noise_sigma
    x, rep = gpu_solve(ctx, d, F().FP64, w.n, method=0, alpha=ALPHA, noise_sigma=sig, max_iter=20)
    xr, hist = solvers.cgls(lambda v: Jd @ v, lambda v: Jd.T @ v, d, sig, ALPHA, 20)
    print("cgls fp64 rel", rel(x, xr), "misfit", rep["misfit"], hist[-1], flush=True)
    assert rep["iters"] == 20
    assert rel(x, xr) < 1e-8
    assert abs(rep["misfit"] / hist[-1] - 1) < 1e-8


def test_cgls_mixed_precision_tracks_fp64(small):
    w, Jd, ctx, d = small
    sig = w.noise_sigma
    x64, r64 = gpu_solve(ctx, d, F().FP64, w.n, method=0, alpha=ALPHA, noise_sigma=sig, max_iter=20)
    x32, r32 = gpu_solve(ctx, d, F().FP32, w.n, method=0, alpha=ALPHA, noise_sigma=sig, max_iter=20)
    print("cgls fp32 vs fp64 rel", rel(x32, x64), "misfits", r32["misfit"], r64["misfit"], flush=True)
    assert rel(x32, x64) < 1e-3
    assert abs(r32["misfit"] / r64["misfit"] - 1) < 1e-3


def test_cgls_converges_to_direct_solution(small):
    w, Jd, ctx, d = small
    sig = w.noise_sigma
    x, rep = gpu_solve(ctx, d, F().FP64, w.n, method=0, alpha=ALPHA, noise_sigma=sig,
                       max_iter=600, rel_tol=1e-11)
    A = Jd.T @ Jd / sig ** 2 + ALPHA * np.eye(w.n)
    xd = np.linalg.solve(A, Jd.T @ d / sig ** 2)
    print("cgls long: iters", rep["iters"], "rel", rel(x, xd), flush=True)
    assert rel(x, xd) < 1e-7


def test_cgls_stops_at_target_misfit(small):
    w, Jd, ctx, d = small
    sig = w.noise_sigma
    _, hist = solvers.cgls(lambda v: Jd @ v, lambda v: Jd.T @ v, d, sig, ALPHA, 20)
    target = hist[8] * (1 + 1e-9)
    x, rep = gpu_solve(ctx, d, F().FP64, w.n, method=0, alpha=ALPHA, noise_sigma=sig,
                       max_iter=50, target_misfit=target)
    assert rep["iters"] <= 9 and rep["misfit"] <= target and rep["converged"]


def test_lsqr_fp64_matches_oracle_lsqr(small):
    w, Jd, ctx, d = small
    sig = w.noise_sigma
    A = Jd / sig
    # early iterates agree to rounding; later ones drift apart through the
    # loss of orthogonality of the bidiagonalisation, and so does LSQR's
    # recurrence estimate of the misfit
    for iters, tol, mtol in ((5, 1e-10, 1e-9), (30, 1e-4, 1e-2)):
        x, rep = gpu_solve(ctx, d, F().FP64, w.n, method=1, alpha=ALPHA, noise_sigma=sig,
                           max_iter=iters)
        xr = solvers.lsqr(lambda v: A @ v, lambda v: A.T @ v, d / sig, math.sqrt(ALPHA), iters, w.n)
        mis = float(np.sum((Jd @ x - d) ** 2) / sig ** 2)
        print("lsqr", iters, "rel", rel(x, xr), "misfit est", rep["misfit"], "true", mis, flush=True)
        assert rel(x, xr) < tol
        assert abs(rep["misfit"] / mis - 1) < mtol


@pytest.mark.parametrize("prec_name,tol", [("FP64", 1e-10), ("FP32", 1e-5),
                                           ("FP32_BF16TABLE", 1e-3)])
def test_psf_is_hessian_column(small, prec_name, tol):
    w, Jd, ctx, d = small
    f = F()
    prec = getattr(f, prec_name)
    sig = w.noise_sigma
    vox = np.array([100, 3000, 5555])
    out = host(ctx.psf(vox, sig, prec=prec)).reshape(len(vox), w.n)
    for k, v in enumerate(vox):
        ref = Jd.T @ Jd[:, v] / sig ** 2
        e = rel(out[k], ref)
        print("psf", prec_name, v, e, flush=True)
        assert e < tol


def test_solver_argument_errors(small):
    w, Jd, ctx, d = small
    f = F()
    with pytest.raises(f.FFTTError):
        gpu_solve(ctx, d, f.FP64, w.n, method=7, alpha=ALPHA, noise_sigma=1.0)
    with pytest.raises(f.FFTTError):
        gpu_solve(ctx, d, f.FP64, w.n, method=0, alpha=ALPHA, noise_sigma=0.0)
    with pytest.raises(f.FFTTError):
        ctx.psf(np.array([w.n + 5]), 1.0, prec=f.FP64)


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("prec_name", ["FP32", "FP64"])
def test_solve_graph_replays_match_eager(small, method, prec_name):
    """With use_graph, iteration 2 is captured once and replayed; solves of
    1, 2, 3 and 6 iterations (0 to 4 replays), with eager operator work and
    synchronisations in between, give bit-identical iterates to the eager
    solver.  A target-misfit stop (one host check per replay) too."""
    w, Jd, ctx, d = small
    f = F()
    prec = getattr(f, prec_name)
    sig = w.noise_sigma
    probe = dev(w.model, prec)
    for k in (1, 2, 3, 6):
        xe, re_ = gpu_solve(ctx, d, prec, w.n, method=method, alpha=ALPHA, noise_sigma=sig,
                            max_iter=k)
        ctx.apply_J(probe, prec=prec)          # unrelated eager work on the stream
        torch.cuda.synchronize()
        xg, rg = gpu_solve(ctx, d, prec, w.n, method=method, alpha=ALPHA, noise_sigma=sig,
                           max_iter=k, graph=True)
        assert re_["iters"] == rg["iters"] == k
        assert np.array_equal(xe, xg), (k, rel(xg, xe))
        assert re_["misfit"] == rg["misfit"]
    # early stop at a target misfit: same iteration count and iterate
    _, r20 = gpu_solve(ctx, d, prec, w.n, method=method, alpha=ALPHA, noise_sigma=sig,
                       max_iter=20)
    target = r20["misfit"] * 1.05
    xe, re_ = gpu_solve(ctx, d, prec, w.n, method=method, alpha=ALPHA, noise_sigma=sig,
                        max_iter=40, target_misfit=target)
    xg, rg = gpu_solve(ctx, d, prec, w.n, method=method, alpha=ALPHA, noise_sigma=sig,
                       max_iter=40, target_misfit=target, graph=True)
    assert re_["iters"] == rg["iters"] and np.array_equal(xe, xg)
