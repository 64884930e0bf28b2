"""Closed forms used to pin the oracle (test-side mathematics, written from
the definitions, independent of the oracle's quadrature code).

For the Gaussian-windowed sine f(t) = exp(-t^2/2s^2) sin(wc t) the energy
spectrum is a sum of three Gaussians in w,
    S(w) ~ g(w - wc) + g(w + wc) - 2 exp(-s^2 wc^2) g(w),  g(v) = exp(-s^2 v^2),
so every moment integral of the kernel formula of Sec. II-C extends to the
whole real line and reduces to derivatives of the Gaussian's characteristic
function  Phi_mu(tau) = int exp(-s^2 (w-mu)^2) exp(i w tau) dw
                      = (sqrt(pi)/s) exp(i mu tau - tau^2 / (4 s^2)).
"""
import math

import numpy as np


def _terms(sigma, wc):
    return ((1.0, wc), (1.0, -wc), (-2.0 * math.exp(-(sigma * wc) ** 2), 0.0))


def h_closed(R, c0, sigma, wc):
    """int_0^inf w^3 S sin(w R/c0) dw / int_0^inf w^2 S dw for the Gaussian pulse."""
    tau = np.asarray(R, dtype=np.float64) / c0
    num = np.zeros_like(tau)
    den = 0.0
    s2 = sigma * sigma
    for c, mu in _terms(sigma, wc):
        psi1 = 1j * mu - tau / (2.0 * s2)          # d/dtau of the exponent
        psi2 = -1.0 / (2.0 * s2)
        phi = (math.sqrt(math.pi) / sigma) * np.exp(1j * mu * tau - tau * tau / (4.0 * s2))
        # int w^3 e^{-s^2(w-mu)^2} e^{i w tau} dw = i (3 psi1 psi2 + psi1^3) Phi
        num += c * np.real((3.0 * psi1 * psi2 + psi1 ** 3) * phi)
        den += c * (math.sqrt(math.pi) / sigma) * (mu * mu + 1.0 / (2.0 * s2))
    return num / den


def moment_ratio_4_2(sigma, wc):
    """int w^4 S / int w^2 S for the Gaussian pulse (Gaussian moments)."""
    s2 = sigma * sigma
    m4 = m2 = 0.0
    for c, mu in _terms(sigma, wc):
        m4 += c * (mu ** 4 + 3.0 * mu * mu / s2 + 3.0 / (4.0 * s2 * s2))
        m2 += c * (mu * mu + 1.0 / (2.0 * s2))
    return m4 / m2
