"""Host-side checks of libfftt that need no GPU: the shared library loads,
exports every entry point declared in include/fftt.h, and its host table
builder agrees with the oracle's quadrature."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1908_03302_amd import fftt
from paper_1908_03302_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fftt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fftt_[a-z_A-Z0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = fftt.load()
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(fftt.EXPORTS)


@pytest.mark.parametrize("fc,bw,r_max", [(0.5e6, 0.5, I.R_MAX_HALF_MHZ_BW50),
                                         (1e6, 1.0, I.R_MAX[1e6]), (2e6, 1.0, I.R_MAX[2e6])])
def test_table_builder_matches_oracle(fc, bw, r_max):
    p = I.sampled_pulse(fc, bw)
    h, r = fftt.build_table_from_pulse(1500.0, p.samples, p.dt, 4096, r_max)
    assert r == r_max
    a, b = oracle.quad_coeffs(p.samples, p.dt, 1500.0, r_max=r_max)
    ho = oracle.table(a, b, r_max, 4096)
    assert np.abs(h - ho).max() <= 1e-12 * np.abs(ho).max()


def test_table_builder_auto_radius():
    p = I.sampled_pulse(1e6, 1.0)
    h, r = fftt.build_table_from_pulse(1500.0, p.samples, p.dt, 1024, 0.0)
    a, b = oracle.quad_coeffs(p.samples, p.dt, 1500.0, r_max=3 * I.R_MAX[1e6])
    R = np.linspace(0, 3 * I.R_MAX[1e6], 30001)
    ho = oracle.h_eval(a, b, R)
    big = R[np.abs(ho) >= 1e-7 * np.abs(ho).max()].max()
    assert big <= r <= big + 1e-5


def test_table_builder_rejects_bad_input():
    with pytest.raises(fftt.FFTTError):
        fftt.build_table_from_pulse(1500.0, np.zeros(100), 1e-8, 512, 0.0)
    with pytest.raises(fftt.FFTTError):
        fftt.build_table_from_pulse(-1.0, np.ones(100), 1e-8, 512, 0.0)
    with pytest.raises(fftt.FFTTError):
        fftt.build_table_from_pulse(1500.0, np.ones(100), 1e-8, 1, 0.0)


@pytest.mark.parametrize("fc,bw,r_max", [(0.5e6, 0.5, I.R_MAX_HALF_MHZ_BW50),
                                         (0.5e6, 1.0, I.R_MAX[0.5e6]),
                                         (1e6, 1.0, I.R_MAX[1e6]), (2e6, 1.0, I.R_MAX[2e6])])
def test_series_builder_matches_oracle(fc, bw, r_max):
    """The library's sine series (few uniform nodes) reproduces the oracle's
    quadrature of eq. Kernel_freq on [0, r_max] to 1e-8 of max|h|; its
    argument spacing keeps beta r_max = 0.8 pi (period 2.5 r_max)."""
    p = I.sampled_pulse(fc, bw)
    a, beta = fftt.build_series_from_pulse(1500.0, p.samples, p.dt, r_max)
    assert 8 <= a.size <= 40
    assert abs(beta * r_max - 0.8 * np.pi) < 1e-12
    qa, qb = oracle.quad_coeffs(p.samples, p.dt, 1500.0, r_max=r_max)
    R = np.linspace(0.0, r_max, 20001)
    ho = oracle.h_eval(qa, qb, R)
    hs = np.sin(np.outer(R, beta * np.arange(1, a.size + 1))) @ a
    assert np.abs(hs - ho).max() <= 1e-8 * np.abs(ho).max()


def test_series_builder_rejects_bad_input():
    p = I.sampled_pulse(1e6, 1.0)
    with pytest.raises(fftt.FFTTError):   # needs ~24 terms
        fftt.build_series_from_pulse(1500.0, p.samples, p.dt, I.R_MAX[1e6], max_terms=8)
    with pytest.raises(fftt.FFTTError):
        fftt.build_series_from_pulse(1500.0, p.samples, p.dt, 0.0)
    with pytest.raises(fftt.FFTTError):
        fftt.build_series_from_pulse(1500.0, np.zeros(100), 1e-8, 1e-3)
    with pytest.raises(fftt.FFTTError):
        fftt.build_series_from_pulse(1500.0, p.samples, p.dt, I.R_MAX[1e6], tol=0.0)
