"""Closed-form smoothed skies for the accuracy study (test infrastructure;
see package header).

App. A.2 measures the gridded map against the input signal convolved with
the gridding kernel.  For a sky of Gaussian point sources (PSF sigma_p, peak
amplitudes A) and a normalised Gaussian kernel of sigma_k, that convolution
is again a sum of Gaussians: each source keeps its flux 2 pi sigma^2 A, so
its peak becomes A sigma_p^2 / (sigma_p^2 + sigma_k^2) and its width
sqrt(sigma_p^2 + sigma_k^2).  Offsets are taken on the flat sky around each
source (east offsets scaled by cos of the source latitude), as the sky was
built; the study fields are 1.5 deg wide on the equator.
"""
from __future__ import annotations

import math

import numpy as np


def smoothed_point_sources(src_lon, src_lat, amp, psf_sigma, kernel_sigma, lon, lat):
    """Point sources through the PSF, then the normalised kernel: values at
    (lon, lat), degrees in."""
    lon = np.asarray(lon, dtype=np.float64)
    lat = np.asarray(lat, dtype=np.float64)
    s2 = psf_sigma ** 2 + kernel_sigma ** 2
    scale = psf_sigma ** 2 / s2
    out = np.zeros(lon.shape)
    for a, b, A in zip(src_lon, src_lat, amp):
        dx = (lon - a) * math.cos(math.radians(b))
        dy = lat - b
        out += A * scale * np.exp(-(dx * dx + dy * dy) / (2.0 * s2))
    return out
