"""Pins of the SSIM used by the phase-awareness study (Wang et al. 2004, with K1 = 0.01,
K2 = 0.03 and the reference's maximum as the dynamic range) against closed forms:

- an image against itself gives 1 everywhere;
- constant images alpha and beta give the luminance term alone,
  (2 alpha beta + C1) / (alpha^2 + beta^2 + C1), which pins C1;
- checkerboards mu + delta c and mu + eps c (c = +-1 alternating) have equal local means up to
  the window's response at the Nyquist frequency (about 1e-5 for sigma 1.5), local variances
  delta^2 and eps^2 and covariance delta eps, so that away from the reflected borders the map
  equals the contrast-structure term (2 delta eps + C2) / (delta^2 + eps^2 + C2), which pins C2
  and the covariance."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _rgb(a):
    return np.repeat(np.asarray(a, dtype=np.float64)[..., None], 3, axis=-1)


def test_identical_images():
    rng = np.random.default_rng(0)
    a = _rgb(rng.uniform(0, 2, (40, 52)))
    assert bench.ssim(a, a) == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("alpha,beta", [(0.2, 0.7), (1.3, 0.4), (0.0, 1.0), (0.5, 0.5)])
def test_constant_images(alpha, beta):
    a = _rgb(np.full((24, 30), alpha))
    b = _rgb(np.full((24, 30), beta))
    c1 = (0.01 * beta) ** 2
    expect = (2 * alpha * beta + c1) / (alpha ** 2 + beta ** 2 + c1)
    # the filtered variances cancel to rounding (about 1e-16 of alpha^2) against C2
    np.testing.assert_allclose(bench.ssim_map(a, b), expect, rtol=1e-10)
    assert bench.ssim(a, b) == pytest.approx(expect, rel=1e-10)


@pytest.mark.parametrize("delta,eps", [(0.1, 0.1), (0.1, 0.05), (0.02, 0.3), (0.1, -0.1),
                                       (0.004, 0.01)])
def test_checkerboard_contrast_structure(delta, eps):
    mu = 0.5
    n = 48
    c = np.where((np.add.outer(np.arange(n), np.arange(n)) % 2) == 0, 1.0, -1.0)
    a = _rgb(mu + delta * c)
    b = _rgb(mu + eps * c)
    L = mu + abs(eps)
    c2 = (0.03 * L) ** 2
    expect = (2 * delta * eps + c2) / (delta ** 2 + eps ** 2 + c2)
    m = bench.ssim_map(a, b)
    inner = m[8:-8, 8:-8]  # beyond the window's reach (truncated at 3.5 sigma = 6 pixels)
    np.testing.assert_allclose(inner, expect, rtol=1e-8, atol=1e-10)
