"""FITS-WCS pixel -> world for the oracle (test infrastructure).

Written from the FITS WCS papers cited in the paper's introduction
(Greisen & Calabretta 2002; Calabretta & Greisen 2002), for the
projections the benchmark grids use and two more the paper names (SFL in
Listing 1, ZEA in Fig. 1):

* CAR, the plate carree: native phi = x, theta = y with intermediate
  coordinates x = CDELT1 (i - CRPIX1), y = CDELT2 (j - CRPIX2).  With
  CRVAL2 = 0, lon = CRVAL1 + x and lat = y (a field away from the equator is
  placed with CRPIX2).  With CRVAL2 != 0 the projection is oblique: the
  native frame has its reference point (phi, theta) = (0, 0) at CRVAL and
  its pole at the point 90 deg from CRVAL that is nearest the celestial
  pole, which is what the default LONPOLE (0 for CRVAL2 > 0, 180 deg below)
  and LATPOLE (+90 deg) select.  The frame is built here as three unit
  vectors (reference point, native pole, their cross product) and a native
  direction is carried to the sky as a linear combination of them.
* SIN (orthographic zenithal, LONPOLE = 180 deg): R = sqrt(x^2 + y^2),
  native phi = atan2(x, -y), native theta = acos(R) (R in radians); the
  native-to-celestial rotation with (alpha_p, delta_p) = (CRVAL1, CRVAL2)
  and phi_p = 180 deg.  Pixels with R > 1 lie outside the projection and
  have no world coordinate (NaN).
* ZEA (zenithal equal-area): as SIN but R = 2 sin((90 deg - theta) / 2)
  (radians), i.e. theta = 90 deg - 2 asin(R / 2); R > 2 has no world
  coordinate.
* SFL (Sanson-Flamsteed): x = phi cos theta, y = theta, so theta = y and
  phi = x / cos(y); points with |y| > 90 deg or |x / cos y| > 180 deg lie
  outside the projection.  Oblique for CRVAL2 != 0 exactly as CAR.

(i, j) are FITS 1-based pixel indices along NAXIS1 / NAXIS2.
"""
from __future__ import annotations

import numpy as np


def _unit(lon_deg, lat_deg):
    a, d = np.radians(lon_deg), np.radians(lat_deg)
    return np.array([np.cos(d) * np.cos(a), np.cos(d) * np.sin(a), np.sin(d)])


def _oblique_cylindrical(crval1, crval2, phi_deg, theta_deg):
    """Native (phi, theta) of a cylindrical projection with its reference
    point at CRVAL -> world (lon, lat) in degrees."""
    ex = _unit(crval1, crval2)                     # native (0, 0)
    north = np.array([0.0, 0.0, 1.0])
    ez = north - np.dot(north, ex) * ex            # native pole: 90 deg from ex, towards north
    ez /= np.linalg.norm(ez)
    ey = np.cross(ez, ex)                          # native (90 deg, 0)
    p, t = np.radians(phi_deg), np.radians(theta_deg)
    v = (np.cos(t) * np.cos(p))[..., None] * ex + (np.cos(t) * np.sin(p))[..., None] * ey \
        + np.sin(t)[..., None] * ez
    lon = np.mod(np.degrees(np.arctan2(v[..., 1], v[..., 0])), 360.0)
    lat = np.degrees(np.arcsin(np.clip(v[..., 2], -1.0, 1.0)))
    return lon, lat


def wcs_world(wcs: dict, i, j):
    """World (lon, lat) in degrees for 1-based pixel coordinates (i, j)."""
    i = np.asarray(i, dtype=np.float64)
    j = np.asarray(j, dtype=np.float64)
    x = wcs["cdelt1"] * (i - wcs["crpix1"])
    y = wcs["cdelt2"] * (j - wcs["crpix2"])
    proj = wcs["proj"].upper()
    crval2 = wcs.get("crval2", 0.0)
    if abs(crval2) > 90.0:
        raise ValueError("|CRVAL2| > 90")
    if proj == "CAR":
        if crval2 != 0.0:
            bad = np.abs(y) > 90.0
            lon, lat = _oblique_cylindrical(wcs["crval1"], crval2, x, np.where(bad, 0.0, y))
            return np.where(bad, np.nan, lon), np.where(bad, np.nan, lat)
        lon = np.mod(wcs["crval1"] + x, 360.0)
        lat = y.copy()
        bad = np.abs(lat) > 90.0
        lon = np.where(bad, np.nan, lon)
        lat = np.where(bad, np.nan, lat)
        return lon, lat
    if proj == "SFL":
        lat = y.copy()
        with np.errstate(invalid="ignore", divide="ignore"):
            dlon = x / np.cos(np.radians(lat))
        dlon = np.where(x == 0.0, 0.0, dlon)
        bad = (np.abs(lat) > 90.0) | ~(np.abs(dlon) <= 180.0)
        if crval2 != 0.0:
            lon, lat = _oblique_cylindrical(wcs["crval1"], crval2, np.where(bad, 0.0, dlon),
                                            np.where(bad, 0.0, lat))
            return np.where(bad, np.nan, lon), np.where(bad, np.nan, lat)
        lon = np.mod(wcs["crval1"] + dlon, 360.0)
        return np.where(bad, np.nan, lon), np.where(bad, np.nan, lat)
    if proj in ("SIN", "ZEA"):
        r = np.radians(np.hypot(x, y))
        phi = np.arctan2(np.radians(x), -np.radians(y))
        with np.errstate(invalid="ignore"):
            if proj == "SIN":
                theta = np.arccos(r)          # NaN outside the disc R > 1
            else:
                theta = np.pi / 2 - 2.0 * np.arcsin(r / 2.0)   # NaN for R > 2
        ap = np.radians(wcs["crval1"])
        dp = np.radians(wcs["crval2"])
        php = np.pi                           # LONPOLE = 180 deg for zenithal
        dphi = phi - php
        st, ct = np.sin(theta), np.cos(theta)
        lat = np.arcsin(np.clip(st * np.sin(dp) + ct * np.cos(dp) * np.cos(dphi), -1.0, 1.0))
        lon = ap + np.arctan2(-ct * np.sin(dphi), st * np.cos(dp) - ct * np.sin(dp) * np.cos(dphi))
        lon = np.mod(np.degrees(lon), 360.0)
        lat = np.degrees(lat)
        bad = ~np.isfinite(theta)
        return np.where(bad, np.nan, lon), np.where(bad, np.nan, lat)
    raise ValueError(f"unsupported projection {proj!r}")


def wcs_targets(wcs: dict):
    """World coordinates of every pixel centre, flattened in FITS order.

    Target t = (j-1) * NAXIS1 + (i-1), i.e. numpy [NAXIS2][NAXIS1] order,
    which is the layout the paper writes with ``fits.writeto`` (Listing 1).
    """
    nx, ny = int(wcs["naxis1"]), int(wcs["naxis2"])
    jj, ii = np.meshgrid(np.arange(1, ny + 1), np.arange(1, nx + 1), indexing="ij")
    lon, lat = wcs_world(wcs, ii.ravel(), jj.ravel())
    return lon, lat
