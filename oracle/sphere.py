"""Spherical geometry for the oracle (test infrastructure; see package header).

Plain FP64 NumPy.  Angles in radians unless a name says ``_deg``.
"""
from __future__ import annotations

import numpy as np


def unit_vectors(lon_deg, lat_deg) -> np.ndarray:
    """(cos d cos a, cos d sin a, sin d) for each (a, d) in degrees -> [N][3]."""
    a = np.radians(np.asarray(lon_deg, dtype=np.float64))
    d = np.radians(np.asarray(lat_deg, dtype=np.float64))
    cd = np.cos(d)
    return np.stack([cd * np.cos(a), cd * np.sin(a), np.sin(d)], axis=-1)


def vincenty(lon1, lat1, lon2, lat2):
    """True angular distance by Vincenty's formula (radians in, radians out).

    Sect. 2.1 names the Haversine and the Vincenty formula for the true
    angular distance d; the oracle takes Vincenty (the better-conditioned
    one at every separation):

        d = atan2( sqrt((cos d2 sin da)^2 + (cos d1 sin d2 - sin d1 cos d2 cos da)^2),
                   sin d1 sin d2 + cos d1 cos d2 cos da ),   da = a2 - a1.
    """
    da = lon2 - lon1
    s1, c1 = np.sin(lat1), np.cos(lat1)
    s2, c2 = np.sin(lat2), np.cos(lat2)
    cda = np.cos(da)
    num = np.hypot(c2 * np.sin(da), c1 * s2 - s1 * c2 * cda)
    den = s1 * s2 + c1 * c2 * cda
    return np.arctan2(num, den)


def bearing(lon1, lat1, lon2, lat2):
    """Initial bearing at point 1 towards point 2, from north through east.

    beta = atan2(sin da cos d2, cos d1 sin d2 - sin d1 cos d2 cos da).  Used
    for the elliptical kernel of Sect. 2.1 / Fig. 1, with point 1 the target
    and point 2 the sample.  At a pole the formula uses the longitude given
    for that point, i.e. north is the limit along its own meridian.
    """
    da = lon2 - lon1
    s1, c1 = np.sin(lat1), np.cos(lat1)
    s2, c2 = np.sin(lat2), np.cos(lat2)
    return np.arctan2(np.sin(da) * c2, c1 * s2 - s1 * c2 * np.cos(da))


_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x) -> np.ndarray:
    """Output function of Steele, Lea & Flood's SplitMix64 for state ``x``.

    z = x + 0x9E3779B97F4A7C15; z = (z ^ z>>30) * 0xBF58476D1CE4E5B9;
    z = (z ^ z>>27) * 0x94D049BB133111EB; return z ^ z>>31   (mod 2^64).
    Used only to hash neighbour sets order-independently (sum mod 2^64).
    """
    z = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))
