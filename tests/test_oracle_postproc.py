"""Pins of the post-processing oracle (Savitzky-Golay smoothing, Keys cubic
up-sampling) against library routines and exact polynomial properties; the
library's fp32 Savitzky-Golay weights against the oracle's."""
import numpy as np
import pytest
from scipy import signal

from oracle import postproc as pp
from paper_2201_13191_amd import mcx


@pytest.mark.parametrize("window,order", [(5, 3), (7, 3), (11, 3), (21, 3), (9, 2), (31, 5)])
def test_savgol_coefficients_match_scipy(window, order):
    ref = signal.savgol_coeffs(window, order, use="dot")
    assert np.allclose(pp.savgol_coefficients(window, order), ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("window,order", [(7, 3), (15, 3)])
def test_savgol_1d_matches_scipy_mirror(window, order):
    x = np.random.default_rng(0).normal(size=57)
    ref = signal.savgol_filter(x, window, order, mode="mirror")
    assert np.allclose(pp.savgol_1d(x, window, order), ref, rtol=0, atol=1e-12)


def test_savgol_reproduces_cubics_inside():
    t = np.arange(40, dtype=np.float64)
    x = 0.3 - 1.2 * t + 0.05 * t ** 2 - 0.002 * t ** 3
    y = pp.savgol_1d(x, 9, 3)
    assert np.allclose(y[4:-4], x[4:-4], rtol=0, atol=1e-9)
    img = np.add.outer(0.01 * t ** 3, -0.2 * t ** 2)       # cubic in each variable
    sm = pp.savgol_2d(img, 7, 3)
    assert np.allclose(sm[3:-3, 3:-3], img[3:-3, 3:-3], rtol=0, atol=1e-8)


def test_keys_kernel_properties():
    assert pp.keys_kernel(0.0) == 1.0
    for v in (1.0, -1.0, 2.0, -2.0, 2.5):
        assert pp.keys_kernel(v) == 0.0
    for u in np.linspace(-1.0, 1.0, 17):
        ms = np.arange(-3, 5)
        w = np.array([pp.keys_kernel(u - m) for m in ms])
        assert abs(w.sum() - 1.0) < 1e-12                  # partition of unity
        assert abs((w * ms).sum() - u) < 1e-12              # reproduces linear
        assert abs((w * ms ** 2).sum() - u * u) < 1e-12     # and quadratic functions


def test_upsample_reproduces_quadratics_inside():
    t = np.arange(30, dtype=np.float64)
    x = 2.0 + 0.5 * t - 0.03 * t ** 2
    y = pp.upsample_1d(x, 2)
    u = (np.arange(60) + 0.5) / 2 - 0.5
    ref = 2.0 + 0.5 * u - 0.03 * u ** 2
    assert np.allclose(y[4:-4], ref[4:-4], rtol=0, atol=1e-10)
    # constant images stay constant everywhere (edges clamped)
    assert np.allclose(pp.upsample_2d(np.full((5, 7), 3.25), 4), 3.25, atol=1e-12)


@pytest.mark.parametrize("window,order", [(5, 3), (11, 3), (31, 3), (9, 4)])
def test_library_weights_match_oracle(window, order):
    w = mcx.mc_savgol_weights(window, order)
    ref = pp.savgol_coefficients(window, order)
    assert np.allclose(w.astype(np.float64), ref, rtol=0, atol=2e-7)
