"""Pins for oracle/analytic.py, the closed-form smoothed sky of the App. A.2
accuracy study: the zero-width limit, flux conservation, and the FP64
gridding oracle itself converging to it on densely sampled data."""
import math

import numpy as np

import oracle
from oracle.analytic import smoothed_point_sources
from oracle import grid as og


def test_zero_width_kernel_is_the_input_sky():
    sl, sb, A, sp = np.array([10.0, 10.3]), np.array([0.1, -0.2]), np.array([1.0, 0.4]), 0.05
    lon = np.array([10.0, 10.1, 10.25]); lat = np.array([0.1, 0.0, -0.15])
    got = smoothed_point_sources(sl, sb, A, sp, 0.0, lon, lat)
    want = [sum(a * math.exp(-(((x - l) * math.cos(math.radians(b))) ** 2 + (y - b) ** 2) / (2 * sp * sp))
                for l, b, a in zip(sl, sb, A)) for x, y in zip(lon, lat)]
    np.testing.assert_allclose(got, want, rtol=1e-14)


def test_flux_is_conserved():
    # integral over the plane of one smoothed source = 2 pi sigma_p^2 A
    sp, sk, A = 0.04, 0.03, 0.7
    h = 0.002
    x = np.arange(-0.5, 0.5 + h / 2, h)
    X, Y = np.meshgrid(x, x)
    v = smoothed_point_sources([0.0], [0.0], [A], sp, sk, X.ravel(), Y.ravel())
    assert v.sum() * h * h == __import__("pytest").approx(2 * math.pi * sp * sp * A, rel=1e-9)


def test_gridding_oracle_converges_to_it():
    # Eq. (1)-(3) with a Gaussian kernel on a dense, uniform sampling of one
    # PSF-convolved source tends to the closed form (sampling 0.2 sigma)
    sp, sk, A = 0.04, 0.03, 1.0
    h = 0.2 * sk
    x = np.arange(-0.35, 0.35 + h / 2, h)
    X, Y = np.meshgrid(180.0 + x, x)
    lon, lat = X.ravel(), Y.ravel()
    data = A * np.exp(-(((lon - 180.0) * 1.0) ** 2 + lat ** 2) / (2 * sp * sp))
    tl = np.array([180.0, 180.03, 179.95]); tb = np.array([0.0, 0.02, -0.04])
    out = og.grid_kdtree(lon, lat, data[:, None], tl, tb, ("gauss1d", (sk,)), 5 * sk)
    want = smoothed_point_sources([180.0], [0.0], [A], sp, sk, tl, tb)
    np.testing.assert_allclose(out["R"][0], want, rtol=2e-3)
