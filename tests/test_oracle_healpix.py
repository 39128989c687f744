"""Pins for the oracle's HEALPix pixel centres (oracle/healpix.py).

The two orders are computed by different routes (ring formulas for RING,
the HEALPix projection plane for NESTED), and each is pinned by facts of the
HEALPix grid (Gorski et al. 2005) that neither route restates: the twelve
base-pixel centres, equal pixel areas, the nested numbering inside a base
face, and the hierarchy of the nested scheme.  Each pin takes the module it
checks, so that the planted mistakes at the end (each a one-line slip in a
copy of the module) can be shown to fail at least one of them.
"""
import math

import numpy as np
import pytest

from oracle import healpix as oh
from oracle.sphere import vincenty

from mutate import mutated


def _z(lat_deg):
    return np.sin(np.radians(lat_deg))


def pin_base_pixels(h):
    # nside = 1: the twelve base pixels (Gorski et al. 2005, Sect. 4): four
    # centred on z = 2/3 at phi = 45, 135, 225, 315 deg, four on the equator
    # at phi = 0, 90, 180, 270 deg, four on z = -2/3 at 45 .. 315 deg; for
    # nside = 1 both orders number them north to south, eastwards.
    lon = [45, 135, 225, 315, 0, 90, 180, 270, 45, 135, 225, 315]
    z = [2 / 3] * 4 + [0.0] * 4 + [-2 / 3] * 4
    for f in (h.ring_centres, h.nest_centres):
        lo, la = f(1)
        np.testing.assert_allclose(lo, lon, atol=1e-12)
        np.testing.assert_allclose(_z(la), z, atol=1e-14)


def pin_same_pixels(h, nside):
    a = np.stack(h.ring_centres(nside), axis=1)
    b = np.stack(h.nest_centres(nside), axis=1)
    assert a.shape == b.shape == (12 * nside * nside, 2)
    ka = np.lexsort((np.round(a[:, 0], 7), np.round(a[:, 1], 7)))
    kb = np.lexsort((np.round(b[:, 0], 7), np.round(b[:, 1], 7)))
    d = vincenty(np.radians(a[ka, 0]), np.radians(a[ka, 1]),
                 np.radians(b[kb, 0]), np.radians(b[kb, 1]))
    assert d.max() < 1e-12


def pin_equal_areas(h, nside):
    # equal-area pixels: the number of centres above any z0 is Npix (1 - z0)/2
    # up to the pixels of one ring
    for f in (h.ring_centres, h.nest_centres):
        lo, la = f(nside)
        z = _z(la)
        npix = 12 * nside * nside
        for z0 in np.linspace(-0.99, 0.99, 23):
            assert abs(np.sum(z > z0) - npix * (1 - z0) / 2) <= 4 * nside


def pin_nested_numbering(h):
    # nside = 2: pixels 0..3 of base face 0 are its south, east, west and
    # north quarters (the nested Z order, Gorski et al. 2005, Fig. 4)
    lo, la = h.nest_centres(2)
    assert la[3] > la[1] > la[0]
    assert abs(la[1] - la[2]) < 1e-9
    assert lo[1] > lo[0] > lo[2]
    assert abs(lo[0] - lo[3]) < 1e-9


def pin_nested_hierarchy(h, nside):
    # the four children 4p .. 4p + 3 (at 2 nside) of nested pixel p lie inside it
    plo, pla = h.nest_centres(nside)
    clo, cla = h.nest_centres(2 * nside)
    size = math.sqrt(4 * math.pi / (12 * nside * nside))
    parent = np.repeat(np.arange(plo.shape[0]), 4)
    d = vincenty(np.radians(clo), np.radians(cla), np.radians(plo[parent]), np.radians(pla[parent]))
    assert d.max() < 0.75 * size


def pin_ring_order(h, nside):
    lo, la = h.ring_centres(nside)
    z = _z(la)
    assert np.all(np.diff(z) <= 1e-15)
    start = 0
    for i in range(1, 4 * nside):
        n = 4 * min(i, nside, 4 * nside - i)
        ring = slice(start, start + n)
        assert np.ptp(z[ring]) < 1e-15
        assert np.all(np.diff(lo[ring]) > 0)
        assert lo[start] < 360.0 / n
        start += n
    assert start == 12 * nside * nside


def test_base_pixels():
    pin_base_pixels(oh)


@pytest.mark.parametrize("nside", [2, 4, 8, 32])
def test_ring_and_nested_are_the_same_pixels(nside):
    pin_same_pixels(oh, nside)


@pytest.mark.parametrize("nside", [4, 16, 64])
def test_equal_areas(nside):
    pin_equal_areas(oh, nside)


def test_nested_numbering_in_a_face():
    pin_nested_numbering(oh)


@pytest.mark.parametrize("nside", [1, 4, 16])
def test_nested_hierarchy(nside):
    pin_nested_hierarchy(oh, nside)


@pytest.mark.parametrize("nside", [1, 2, 8])
def test_ring_order(nside):
    pin_ring_order(oh, nside)


def _all_pins_pass(h):
    try:
        pin_base_pixels(h)
        pin_nested_numbering(h)
        for ns in (2, 4, 8):
            pin_same_pixels(h, ns)
            pin_equal_areas(h, ns)
            pin_ring_order(h, ns)
        for ns in (1, 4):
            pin_nested_hierarchy(h, ns)
    except AssertionError:
        return False
    return True


MUTATIONS = {
    "face_axes_swapped": ("x = xf + (np.pi / 4) * (ix - iy) / nside",
                          "x = xf + (np.pi / 4) * (iy - ix) / nside"),
    "ring_phase_wrong": ("s = 1.0 if (i - nside) % 2 == 0 else 0.0",
                         "s = 1.0 if (i - nside) % 2 == 1 else 0.0"),
    "cap_latitude_wrong": ("zc = 1.0 - ic * ic / (3.0 * nside * nside)",
                           "zc = 1.0 - ic / (3.0 * nside)"),
    "polar_stretch_wrong": ("phi[pol] = xc + (xp - xc) / sig",
                            "phi[pol] = xc + (xp - xc) * sig"),
    "face_longitude_wrong": ("xf = (2 * col + (row != 1)) * (np.pi / 4)",
                             "xf = (2 * col + (row == 1)) * (np.pi / 4)"),
    "nested_bits_swapped": ("iy = _even_bits(loc >> 1).astype(np.float64)",
                            "iy = _even_bits(loc).astype(np.float64)"),
    "cap_phase_wrong": ("phi = (j + 0.5) * np.pi / (2.0 * ic)",
                        "phi = j * np.pi / (2.0 * ic)"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_healpix_mistakes_fail_a_pin(name):
    old, new = MUTATIONS[name]
    assert _all_pins_pass(oh)
    assert not _all_pins_pass(mutated(oh, old, new)), f"planted mistake {name} passed every pin"
