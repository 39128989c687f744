"""HEALPix pixel centres for the oracle (test infrastructure; see package header).

The paper grids onto a full HEALPix map through its sight-line gridder
(Sect. 5; App. A.1 uses the nside = 512 pixel centres).  The pixel layout is
that of Gorski et al. (2005), the HEALPix reference the paper cites.  Two
routes are written here, deliberately different, so that each checks the
other:

* ``ring_centres``: RING order, ring by ring.  Ring i (1 .. 4 nside - 1)
  holds 4 i pixels in the north cap (i < nside), 4 nside in the belt and
  mirrors the cap in the south.  Centres: cap z = 1 - i^2/(3 nside^2),
  phi = (j + 1/2) pi / (2 i); belt z = (4/3) - 2 i / (3 nside),
  phi = (j + s/2) pi / (2 nside) with s = 1 on rings with i - nside even,
  else 0 (j = 0, 1, ... along the ring).
* ``nest_centres``: NESTED order through the HEALPix projection plane
  (Calabretta & Roukema 2007).  Pixel p lies in base face f = p // nside^2
  at (ix, iy) = (even bits, odd bits) of p mod nside^2.  Face f (row
  f // 4 = north, equator, south; column f % 4) is a square standing on a
  vertex, centred at x_f = (2 col + [row != 1]) pi/4, y_f = (1 - row) pi/4;
  ix runs north-east, iy north-west from its south vertex, so the centre is
      x = x_f + (pi/4)(ix - iy)/nside,
      y = y_f - pi/4 + (pi/4)(ix + iy + 1)/nside.
  The projection is inverted as: |y| <= pi/4 -> z = 8 y / (3 pi), phi = x;
  otherwise sigma = 2 - 4|y|/pi, z = +-(1 - sigma^2/3) and
  phi = x_c + (x - x_c)/sigma with x_c the centre of the polar facet
  holding x (x_c = -pi + (2 floor((x + pi)/(pi/2)) + 1) pi/4).

Outputs are degrees, longitude in [0, 360).
"""
from __future__ import annotations

import numpy as np


def _lonlat(z, phi):
    lat = np.degrees(np.arctan2(z, np.sqrt(np.maximum(0.0, (1.0 - z) * (1.0 + z)))))
    lon = np.mod(np.degrees(phi), 360.0)
    return lon, lat


def ring_centres(nside: int):
    """Centres of all 12 nside^2 pixels in RING order: (lon_deg, lat_deg)."""
    nside = int(nside)
    z_all, phi_all = [], []
    for i in range(1, 4 * nside):
        if i < nside or i > 3 * nside:
            ic = i if i < nside else 4 * nside - i
            j = np.arange(4 * ic, dtype=np.float64)
            zc = 1.0 - ic * ic / (3.0 * nside * nside)
            z = np.full(4 * ic, zc if i < nside else -zc)
            phi = (j + 0.5) * np.pi / (2.0 * ic)
        else:
            j = np.arange(4 * nside, dtype=np.float64)
            z = np.full(4 * nside, 4.0 / 3.0 - 2.0 * i / (3.0 * nside))
            s = 1.0 if (i - nside) % 2 == 0 else 0.0
            phi = (j + 0.5 * s) * np.pi / (2.0 * nside)
        z_all.append(z)
        phi_all.append(phi)
    return _lonlat(np.concatenate(z_all), np.concatenate(phi_all))


def _even_bits(v):
    out = np.zeros_like(v)
    for b in range(32):
        out |= ((v >> (2 * b)) & 1) << b
    return out


def nest_centres(nside: int):
    """Centres of all 12 nside^2 pixels in NESTED order: (lon_deg, lat_deg)."""
    nside = int(nside)
    p = np.arange(12 * nside * nside, dtype=np.int64)
    f = p // (nside * nside)
    loc = p % (nside * nside)
    ix = _even_bits(loc).astype(np.float64)
    iy = _even_bits(loc >> 1).astype(np.float64)
    row, col = f // 4, f % 4
    xf = (2 * col + (row != 1)) * (np.pi / 4)
    yf = (1 - row) * (np.pi / 4)
    x = xf + (np.pi / 4) * (ix - iy) / nside
    y = yf - np.pi / 4 + (np.pi / 4) * (ix + iy + 1) / nside
    z = np.empty_like(y)
    phi = np.empty_like(x)
    eq = np.abs(y) <= np.pi / 4
    z[eq] = 8.0 * y[eq] / (3.0 * np.pi)
    phi[eq] = x[eq]
    pol = ~eq
    sig = 2.0 - 4.0 * np.abs(y[pol]) / np.pi
    z[pol] = np.sign(y[pol]) * (1.0 - sig * sig / 3.0)
    xp = x[pol]
    xc = -np.pi + (2.0 * np.floor((xp + np.pi) / (np.pi / 2)) + 1.0) * np.pi / 4
    phi[pol] = xc + (xp - xc) / sig
    return _lonlat(z, phi)


def centres(nside: int, order: str = "ring"):
    """Pixel centres of an nside map in ``order`` ('ring' or 'nested')."""
    if order == "ring":
        return ring_centres(nside)
    if order == "nested":
        return nest_centres(nside)
    raise ValueError(f"unknown order {order!r}")
