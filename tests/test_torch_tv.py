"""The torch TV used with L-BFGS equals the oracle's TV and gradient (CPU)."""
import numpy as np
import torch

from oracle import solvers
from paper_1908_03302_amd.autograd import tv


def test_torch_tv_matches_oracle():
    rng = np.random.default_rng(8)
    dims, sp = (7, 5, 4), (1e-3, 0.8e-3, 1.3e-3)
    x = rng.standard_normal(140)
    xt = torch.tensor(x, requires_grad=True)
    v = tv(xt, dims, sp, 0.1)
    v.backward()
    vo, go = solvers.tv(x, dims, sp, 0.1)
    assert abs(float(v) - vo) <= 1e-12 * abs(vo)
    assert np.allclose(xt.grad.numpy(), go, rtol=1e-12, atol=1e-12 * np.abs(go).max())
