"""Pins for the CPU oracle: closed forms, invariants, hand cases, brute force.

Each test checks the oracle against something other than itself: values
worked out by hand (tests/golden/hand_cases.json), closed forms of
spherical trigonometry and of Gaussian convolution (Eq. 6), invariants of
Eq. (1)-(3), and a library special case (cKDTree ball query).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import grid as og
from oracle.sphere import vincenty, bearing, splitmix64, unit_vectors
from oracle.wcs import wcs_world, wcs_targets

HERE = os.path.dirname(os.path.abspath(__file__))
ARC = 1.0 / 60.0


def _load_cases():
    with open(os.path.join(HERE, "golden", "hand_cases.json")) as f:
        return json.load(f)


def _run(case, fn=None):
    s = np.array(case["samples"], dtype=np.float64)
    t = np.array(case["targets"], dtype=np.float64)
    fn = fn or og.grid_bruteforce
    return fn(s[:, 0], s[:, 1], s[:, 2:3], t[:, 0], t[:, 1],
              (case["kernel"][0], tuple(case["kernel"][1])), case["support"])


def _dest(lon_deg, lat_deg, brg_deg, d_rad):
    """Spherical destination point (textbook direct formula), degrees out."""
    a1, d1, b = math.radians(lon_deg), math.radians(lat_deg), math.radians(brg_deg)
    d2 = math.asin(math.sin(d1) * math.cos(d_rad) + math.cos(d1) * math.sin(d_rad) * math.cos(b))
    a2 = a1 + math.atan2(math.sin(b) * math.sin(d_rad) * math.cos(d1),
                         math.cos(d_rad) - math.sin(d1) * math.sin(d2))
    return math.degrees(a2) % 360.0, math.degrees(d2)


# --------------------------------------------------------------- hand cases

@pytest.mark.parametrize("case", _load_cases()["cases"], ids=lambda c: c["id"])
def test_hand_cases(case):
    r = _run(case)
    for got, exp in zip(r["R"][0], case["expect_R"]):
        if exp is None:
            assert np.isnan(got)
        else:
            assert got == pytest.approx(exp, rel=1e-11)
    np.testing.assert_allclose(r["W"], case["expect_W"], rtol=1e-11, atol=0)


@pytest.mark.parametrize("case", _load_cases()["cases"], ids=lambda c: c["id"])
def test_hand_cases_kdtree(case):
    r = _run(case, og.grid_kdtree)
    np.testing.assert_allclose(r["W"], case["expect_W"], rtol=1e-11, atol=0)


@pytest.mark.parametrize("row", _load_cases()["ellipse"]["rows"], ids=lambda r: str(r["bearing"]))
def test_ellipse_axes(row):
    e = _load_cases()["ellipse"]
    tl, tb = e["target"]
    lon, lat = _dest(tl, tb, row["bearing"], math.radians(e["d_arcmin"] / 60.0))
    r = og.grid_bruteforce([lon], [lat], [[1.0]], [tl], [tb],
                           (e["kernel"][0], tuple(e["kernel"][1])), e["support"])
    assert r["W"][0] == pytest.approx(row["expect_W"], rel=1e-10)


# ------------------------------------------------------- spherical closed forms

def test_vincenty_closed_forms():
    rng = np.random.default_rng(0)
    lat = np.radians(rng.uniform(-89, 89, 200))
    dl = np.radians(rng.uniform(-5, 5, 200))
    # along a meridian the distance is the latitude difference
    np.testing.assert_allclose(vincenty(0.3, lat, 0.3, lat + 0.01), 0.01, rtol=1e-12)
    # along the equator it is the longitude difference
    np.testing.assert_allclose(vincenty(0.0, 0.0, dl, 0.0), np.abs(dl), rtol=1e-12, atol=1e-18)
    # antipodes and coincident points
    assert vincenty(0.1, 0.2, 0.1 + math.pi, -0.2) == pytest.approx(math.pi, rel=1e-14)
    assert vincenty(1.0, -0.4, 1.0, -0.4) == 0.0
    # against the dot-product form at moderate separations
    a1, d1 = rng.uniform(0, 6.28, 500), rng.uniform(-1.5, 1.5, 500)
    a2, d2 = rng.uniform(0, 6.28, 500), rng.uniform(-1.5, 1.5, 500)
    p = np.stack([np.cos(d1) * np.cos(a1), np.cos(d1) * np.sin(a1), np.sin(d1)], 1)
    q = np.stack([np.cos(d2) * np.cos(a2), np.cos(d2) * np.sin(a2), np.sin(d2)], 1)
    ref = np.arccos(np.clip((p * q).sum(1), -1, 1))
    ok = (ref > 0.1) & (ref < 3.0)
    np.testing.assert_allclose(vincenty(a1, d1, a2, d2)[ok], ref[ok], rtol=1e-11)
    # against haversine at arc-second separations
    d2s = d1 + 1e-5
    hav = 2 * np.arcsin(np.sqrt(np.sin((d2s - d1) / 2) ** 2 +
                                np.cos(d1) * np.cos(d2s) * np.sin(1e-5 / 2) ** 2))
    np.testing.assert_allclose(vincenty(a1, d1, a1 + 1e-5, d2s), hav, rtol=1e-9)


def test_bearing_cardinal():
    assert bearing(0.0, 0.0, 0.0, 0.01) == pytest.approx(0.0, abs=1e-15)
    assert bearing(0.0, 0.0, 0.01, 0.0) == pytest.approx(math.pi / 2, rel=1e-15)
    assert abs(bearing(0.0, 0.0, 0.0, -0.01)) == pytest.approx(math.pi, rel=1e-15)
    assert bearing(0.0, 0.0, -0.01, 0.0) == pytest.approx(-math.pi / 2, rel=1e-15)
    # bearing of a destination point is the bearing used to make it
    for b in (10.0, 75.0, 160.0, 250.0, 340.0):
        lon, lat = _dest(33.0, -41.0, b, 0.002)
        got = math.degrees(bearing(math.radians(33.0), math.radians(-41.0),
                                   math.radians(lon), math.radians(lat))) % 360
        assert got == pytest.approx(b, abs=1e-7)


def test_splitmix64_published_vector():
    # first output of SplitMix64 started from state 0
    assert int(splitmix64(np.array([0], dtype=np.uint64))[0]) == 0xE220A8397B1DCDAF


# ----------------------------------------------------------------------- WCS

def test_car_closed_form():
    w = {"proj": "CAR", "naxis1": 96, "naxis2": 96, "crpix1": 48.5, "crpix2": -851.5,
         "crval1": 120.0, "crval2": 0.0, "cdelt1": -1 / 30, "cdelt2": 1 / 30}
    lon, lat = wcs_world(w, [1, 96, 48.5], [1, 96, 1])
    np.testing.assert_allclose(lat, [852.5 / 30, 947.5 / 30, 852.5 / 30], rtol=1e-15)
    np.testing.assert_allclose(lon, [120 + 47.5 / 30, 120 - 47.5 / 30, 120.0], rtol=1e-15)
    lon, lat = wcs_targets(w)
    assert lon.shape == (96 * 96,)
    # FITS order: x fastest
    assert lat[0] == lat[95] and lat[96] > lat[0] and lon[1] < lon[0]


def _sin_hdr(crval2):
    return {"proj": "SIN", "naxis1": 101, "naxis2": 101, "crpix1": 51.0, "crpix2": 51.0,
            "crval1": 120.0, "crval2": crval2, "cdelt1": -0.1, "cdelt2": 0.1}


@pytest.mark.parametrize("crval2", [0.0, 30.0, -63.0, 89.0])
def test_sin_closed_forms(crval2):
    w = _sin_hdr(crval2)
    lon, lat = wcs_world(w, [51.0], [51.0])
    assert lon[0] == pytest.approx(120.0, abs=1e-12) and lat[0] == pytest.approx(crval2, abs=1e-12)
    # distance from the reference point is asin(R) for every pixel
    ii, jj = np.meshgrid(np.arange(1, 102, 7), np.arange(1, 102, 7))
    lon, lat = wcs_world(w, ii.ravel(), jj.ravel())
    x = -0.1 * (ii.ravel() - 51.0)
    y = 0.1 * (jj.ravel() - 51.0)
    R = np.radians(np.hypot(x, y))
    p = unit_vectors(lon, lat)
    c = unit_vectors([120.0], [crval2])[0]
    dist = np.arctan2(np.linalg.norm(np.cross(p, c), axis=1), p @ c)
    np.testing.assert_allclose(dist, np.arcsin(R), rtol=1e-12, atol=1e-15)
    # position angle (east of north) seen from the reference is atan2(x, y)
    e = np.array([-math.sin(math.radians(120)), math.cos(math.radians(120)), 0.0])
    nvec = np.cross(c, e)
    pa = np.arctan2(p @ e, p @ nvec)
    ok = R > 1e-6
    np.testing.assert_allclose(np.angle(np.exp(1j * (pa[ok] - np.arctan2(x[ok], y[ok])))), 0, atol=1e-10)


@pytest.mark.parametrize("crval2", [0.0, 41.0, -80.0])
def test_zea_closed_forms(crval2):
    # zenithal equal-area: a pixel at projection radius R (radians) lies
    # 2 asin(R/2) from the reference point, in position angle atan2(x, y);
    # the cell spacing 1.2 deg reaches 84 deg from the reference
    w = dict(_sin_hdr(crval2), proj="ZEA", cdelt1=-1.2, cdelt2=1.2)
    lon, lat = wcs_world(w, [51.0], [51.0])
    assert lon[0] == pytest.approx(120.0, abs=1e-12) and lat[0] == pytest.approx(crval2, abs=1e-12)
    ii, jj = np.meshgrid(np.arange(1, 102, 5), np.arange(1, 102, 5))
    lon, lat = wcs_world(w, ii.ravel(), jj.ravel())
    x = -1.2 * (ii.ravel() - 51.0)
    y = 1.2 * (jj.ravel() - 51.0)
    R = np.radians(np.hypot(x, y))
    ok = R <= 2.0
    assert np.all(np.isfinite(lat[ok])) and np.all(np.isnan(lat[~ok]))
    p = unit_vectors(lon[ok], lat[ok])
    c = unit_vectors([120.0], [crval2])[0]
    dist = np.arctan2(np.linalg.norm(np.cross(p, c), axis=1), p @ c)
    np.testing.assert_allclose(dist, 2 * np.arcsin(R[ok] / 2), rtol=1e-12, atol=1e-14)
    e = np.array([-math.sin(math.radians(120)), math.cos(math.radians(120)), 0.0])
    nvec = np.cross(c, e)
    pa = np.arctan2(p @ e, p @ nvec)
    m = (R[ok] > 1e-6) & (R[ok] < 1.9)
    d = np.angle(np.exp(1j * (pa[m] - np.arctan2(x[ok][m], y[ok][m]))))
    np.testing.assert_allclose(d, 0, atol=1e-9)


def test_zea_equal_area():
    # equal-area: the share of a large uniform pixel grid inside a cap of
    # angular radius rho around the reference is the cap's solid angle over
    # the projected area per pixel (2 pi (1 - cos rho) / cdelt^2)
    w = {"proj": "ZEA", "naxis1": 801, "naxis2": 801, "crpix1": 401.0, "crpix2": 401.0,
         "crval1": 10.0, "crval2": 20.0, "cdelt1": -0.05, "cdelt2": 0.05}
    lon, lat = wcs_targets(w)
    p = unit_vectors(lon, lat)
    c = unit_vectors([10.0], [20.0])[0]
    for rho in (5.0, 15.0):
        n = np.sum(p @ c >= math.cos(math.radians(rho)))
        expect = 2 * math.pi * (1 - math.cos(math.radians(rho))) / math.radians(0.05) ** 2
        assert abs(n - expect) < 4 * math.sqrt(expect) + 0.02 * expect


def test_sfl_closed_forms():
    # Sanson-Flamsteed: parallels are straight and true to scale, the
    # central meridian and the equator are true to scale
    w = {"proj": "SFL", "naxis1": 361, "naxis2": 181, "crpix1": 181.0, "crpix2": 91.0,
         "crval1": 30.0, "crval2": 0.0, "cdelt1": -1.0, "cdelt2": 1.0}
    lon, lat = wcs_world(w, [181.0, 181.0, 151.0, 151.0, 181.0], [91.0, 151.0, 91.0, 151.0, 181.0])
    np.testing.assert_allclose(lat, [0.0, 60.0, 0.0, 60.0, 90.0], atol=1e-12)
    # x = +30 deg (east) on the equator is 30 deg east; at lat 60 it is 60 deg east
    np.testing.assert_allclose(lon[:4], [30.0, 30.0, 60.0, 90.0], atol=1e-12)
    # outside the projection: beyond 180 deg of longitude at lat 60
    lo, la = wcs_world(w, [181.0 - 100.0], [151.0])
    assert np.isnan(lo[0]) and np.isnan(la[0])


def _ddeg(lo1, la1, lo2, la2):
    return np.degrees(vincenty(np.radians(lo1), np.radians(la1), np.radians(lo2), np.radians(la2)))


def _world(w, x, y):
    # pixel increments of one degree about pixel (0, 0): (i, j) = (x, y)
    return wcs_world(w, np.atleast_1d(np.asarray(x, dtype=float)),
                     np.atleast_1d(np.asarray(y, dtype=float)))


@pytest.mark.parametrize("proj", ["CAR", "SFL"])
@pytest.mark.parametrize("crval2", [35.0, -50.0, 0.5, 90.0])
def test_oblique_cylindrical_geometry(proj, crval2):
    # An oblique cylindrical projection is the plain one in a rotated native
    # frame: the reference pixel is CRVAL, the native meridian and (CAR) the
    # native equator through it are great circles true to scale, every row
    # lies at 90 deg - y from the native pole, and the default LONPOLE puts
    # the celestial pole on native longitude 0 (CRVAL2 > 0) or 180 deg.
    w = {"proj": proj, "crpix1": 0.0, "crpix2": 0.0, "cdelt1": 1.0, "cdelt2": 1.0,
         "crval1": 100.0, "crval2": crval2}
    lo, la = _world(w, 0.0, 0.0)
    assert _ddeg(lo[0], la[0], 100.0, crval2) < 1e-10
    ys = np.array([-80.0, -33.0, -1.0, 2.0, 45.0, 89.0])
    lo, la = _world(w, np.zeros_like(ys), ys)
    np.testing.assert_allclose(_ddeg(lo, la, 100.0, crval2), np.abs(ys), atol=1e-9)
    plo, pla = _world(dict(w, proj="CAR"), 0.0, 90.0)         # the native pole
    for y in (-60.0, 0.0, 30.0, 75.0):
        xs = np.linspace(-170.0, 170.0, 9) * (math.cos(math.radians(y)) if proj == "SFL" else 1.0)
        lo, la = _world(w, xs, np.full_like(xs, y))
        np.testing.assert_allclose(_ddeg(lo, la, plo[0], pla[0]), 90.0 - y, atol=1e-9)
    if proj == "CAR":
        xs = np.array([-150.0, -20.0, 5.0, 120.0])
        lo, la = _world(w, xs, np.zeros_like(xs))
        np.testing.assert_allclose(_ddeg(lo, la, 100.0, crval2), np.abs(xs), atol=1e-9)
    # the celestial pole: native (0 or 180 deg, 90 - |CRVAL2|)
    t = 90.0 - abs(crval2)
    p = 0.0 if crval2 > 0 else 180.0
    x = p * (math.cos(math.radians(t)) if proj == "SFL" else 1.0)
    lo, la = _world(w, x, t)
    assert la[0] == pytest.approx(90.0, abs=1e-9)
    # east is east: a small step along +x near CRVAL increases the longitude
    lo, la = _world(w, 0.01, 0.0)
    dl = (lo[0] - 100.0 + 180.0) % 360.0 - 180.0
    assert dl > 0 or abs(crval2) == 90.0


def test_oblique_cylindrical_continuity():
    # CRVAL2 -> 0 joins the non-oblique form
    for proj in ("CAR", "SFL"):
        w = {"proj": proj, "crpix1": 0.0, "crpix2": 0.0, "cdelt1": 1.0, "cdelt2": 1.0,
             "crval1": 100.0, "crval2": 0.0}
        x = np.array([-120.0, -3.0, 0.0, 17.0, 100.0])
        y = np.array([-50.0, 10.0, 0.0, 44.0, 70.0])
        lo0, la0 = _world(w, x, y)
        lo1, la1 = _world(dict(w, crval2=1e-9), x, y)
        ok = np.isfinite(lo0)               # SFL: two of the points lie outside its outline
        assert np.array_equal(ok, np.isfinite(lo1)) and ok.sum() >= 3
        np.testing.assert_allclose(la1[ok], la0[ok], atol=1e-8)
        np.testing.assert_allclose((lo1[ok] - lo0[ok] + 180.0) % 360.0 - 180.0, 0.0, atol=1e-8)


def _one_pair(kernel, d_deg, support):
    # one sample d_deg north of the target, value 1: R = 1 and W = w(d)
    out = og.grid_bruteforce(np.array([30.0]), np.array([10.0 + d_deg]), np.ones((1, 1)),
                             np.array([30.0]), np.array([10.0]), kernel, support)
    return out["W"][0]


def test_tapered_sinc_values():
    # sinc zeros at d = b, 2b; sin(pi/2)/(pi/2) = 2/pi at d = b/2; taper exp(-1/2) at d = sigma
    k = ("tapered_sinc", (1e6, 0.3))
    assert _one_pair(k, 0.0, 1.0) == pytest.approx(1.0, abs=1e-15)
    assert abs(_one_pair(k, 0.3, 1.0)) < 1e-12 and abs(_one_pair(k, 0.6, 1.0)) < 1e-12
    assert _one_pair(k, 0.15, 1.0) == pytest.approx(2 / math.pi, rel=1e-12)
    assert _one_pair(("tapered_sinc", (0.2, 1e6)), 0.2, 1.0) == pytest.approx(math.exp(-0.5), rel=1e-9)


def test_table_values():
    # a two-entry table is the linear ramp 1 - d/dmax; zero beyond dmax
    k = ("table", (0.5, 1.0, 0.0))
    assert _one_pair(k, 0.125, 1.0) == pytest.approx(0.75, rel=1e-12)
    assert _one_pair(k, 0.6, 1.0) == 0.0
    # a finely tabulated Gaussian grids like the Gaussian itself (linear
    # interpolation error <= h^2 max|w''| / 8 = h^2 / (8 sigma^2))
    sigma, n = 0.1, 4001
    dk = np.linspace(0.0, 0.5, n)
    tab = ("table", tuple([0.5] + list(np.exp(-dk ** 2 / (2 * sigma ** 2)))))
    for d in (0.0123, 0.0777, 0.1999, 0.31):
        assert _one_pair(tab, d, 0.5) == pytest.approx(math.exp(-d * d / (2 * sigma * sigma)),
                                                       abs=((0.5 / (n - 1)) / sigma) ** 2 / 8 + 1e-12)


def test_sin_equatorial_row_and_column():
    w = _sin_hdr(0.0)
    k = np.arange(1, 40)
    lon, lat = wcs_world(w, 51.0 - k, 51.0 + 0 * k)      # east along the equator
    np.testing.assert_allclose(lat, 0.0, atol=1e-12)
    np.testing.assert_allclose(lon, 120.0 + np.degrees(np.arcsin(np.radians(0.1 * k))), rtol=1e-13)
    lon, lat = wcs_world(w, 51.0 + 0 * k, 51.0 + k)      # north along the meridian
    np.testing.assert_allclose(lon, 120.0, atol=1e-12)
    np.testing.assert_allclose(lat, np.degrees(np.arcsin(np.radians(0.1 * k))), rtol=1e-13)


def test_sin_outside_projection_is_nan():
    w = dict(_sin_hdr(0.0), cdelt1=-2.0, cdelt2=2.0)
    lon, lat = wcs_world(w, [1.0, 51.0], [1.0, 51.0])
    assert np.isnan(lon[0]) and np.isnan(lat[0]) and np.isfinite(lon[1])


# ---------------------------------------------------------------- invariants

def _field(seed, n, lon0=45.0, lat0=-20.0, half=0.3):
    g = np.random.default_rng(seed)
    lon = lon0 + g.uniform(-half, half, n) / math.cos(math.radians(lat0))
    lat = lat0 + g.uniform(-half, half, n)
    return lon, lat, g


def _tgrid(lon0, lat0, half, m):
    tl, tb = np.meshgrid(np.linspace(lon0 - half, lon0 + half, m),
                         np.linspace(lat0 - half, lat0 + half, m))
    return tl.ravel(), tb.ravel()


K1 = ("gauss1d", (1.5 * ARC,))
RS = 4.5 * ARC


def test_constant_field():
    lon, lat, g = _field(1, 1500)
    tl, tb = _tgrid(45.0, -20.0, 0.25, 12)
    r = og.grid_bruteforce(lon, lat, np.full((1500, 1), 3.0), tl, tb, K1, RS)
    m = r["W"] > 0
    assert m.sum() > 100
    np.testing.assert_allclose(r["R"][0][m], 3.0, rtol=1e-14)


def test_linearity_and_channels():
    lon, lat, g = _field(2, 900)
    tl, tb = _tgrid(45.0, -20.0, 0.25, 9)
    x = g.normal(size=(900, 1))
    y = g.normal(size=(900, 1))
    rx = og.grid_bruteforce(lon, lat, x, tl, tb, K1, RS)
    ry = og.grid_bruteforce(lon, lat, y, tl, tb, K1, RS)
    rc = og.grid_bruteforce(lon, lat, np.hstack([x, y, 2 * x - 3 * y]), tl, tb, K1, RS)
    m = rx["W"] > 0
    np.testing.assert_allclose(rc["R"][0][m], rx["R"][0][m], rtol=1e-13)
    np.testing.assert_allclose(rc["R"][1][m], ry["R"][0][m], rtol=1e-13)
    np.testing.assert_allclose(rc["R"][2][m], 2 * rx["R"][0][m] - 3 * ry["R"][0][m],
                               rtol=1e-10, atol=1e-12)


def test_permutation_duplication_chunking():
    lon, lat, g = _field(3, 800)
    x = g.normal(size=(800, 2))
    tl, tb = _tgrid(45.0, -20.0, 0.25, 8)
    r = og.grid_bruteforce(lon, lat, x, tl, tb, K1, RS)
    m = r["W"] > 0
    p = g.permutation(800)
    rp = og.grid_bruteforce(lon[p], lat[p], x[p], tl, tb, K1, RS)
    np.testing.assert_allclose(rp["R"][:, m], r["R"][:, m], rtol=1e-12)
    assert np.array_equal(rp["count"], r["count"])
    rd = og.grid_bruteforce(np.r_[lon, lon], np.r_[lat, lat], np.r_[x, x], tl, tb, K1, RS)
    np.testing.assert_allclose(rd["W"], 2 * r["W"], rtol=1e-13)
    np.testing.assert_allclose(rd["R"][:, m], r["R"][:, m], rtol=1e-12)
    a = og.grid_bruteforce(lon[:300], lat[:300], x[:300], tl, tb, K1, RS)
    b = og.grid_bruteforce(lon[300:], lat[300:], x[300:], tl, tb, K1, RS)
    np.testing.assert_allclose(a["W"] + b["W"], r["W"], rtol=1e-13)
    np.testing.assert_allclose(a["S"] + b["S"], r["S"], rtol=1e-12, atol=1e-14)


def test_seam_and_rotation():
    g = np.random.default_rng(4)
    lon = g.uniform(-0.3, 0.3, 700) % 360.0
    lat = g.uniform(-0.3, 0.3, 700)
    x = g.normal(size=(700, 1))
    tl, tb = _tgrid(0.0, 0.0, 0.2, 8)
    tl = tl % 360.0
    r = og.grid_bruteforce(lon, lat, x, tl, tb, K1, RS)
    r2 = og.grid_bruteforce(lon + 360.0, lat, x, tl - 360.0, tb, K1, RS)
    np.testing.assert_allclose(r2["R"], r["R"], rtol=1e-9, atol=1e-12)
    # random rotation of samples and targets together
    q, _ = np.linalg.qr(g.normal(size=(3, 3)))
    def rot(lo, la):
        v = unit_vectors(lo, la) @ q.T
        return np.degrees(np.arctan2(v[:, 1], v[:, 0])) % 360, np.degrees(np.arcsin(np.clip(v[:, 2], -1, 1)))
    lr, br = rot(lon, lat)
    tlr, tbr = rot(tl, tb)
    r3 = og.grid_bruteforce(lr, br, x, tlr, tbr, K1, RS)
    assert np.array_equal(r3["count"], r["count"])
    m = r["W"] > 0
    np.testing.assert_allclose(r3["R"][0][m], r["R"][0][m], rtol=1e-9, atol=1e-12)


def test_kernel_symmetry():
    g = np.random.default_rng(5)
    a = (g.uniform(10, 11, 30), g.uniform(5, 6, 30))
    b = (a[0] + g.uniform(-0.05, 0.05, 30), a[1] + g.uniform(-0.05, 0.05, 30))
    for k in range(30):
        w_ab = og.grid_bruteforce([a[0][k]], [a[1][k]], [[1.0]], [b[0][k]], [b[1][k]], K1, RS)["W"]
        w_ba = og.grid_bruteforce([b[0][k]], [b[1][k]], [[1.0]], [a[0][k]], [a[1][k]], K1, RS)["W"]
        assert w_ab[0] == pytest.approx(w_ba[0], rel=1e-12)
    lon, lat, g = _field(6, 600)
    tl, tb = _tgrid(45.0, -20.0, 0.25, 8)
    x = g.normal(size=(600, 1))
    base = og.grid_bruteforce(lon, lat, x, tl, tb, ("gauss2d", (2 * ARC, 1 * ARC, 25.0)), 6 * ARC)
    flip = og.grid_bruteforce(lon, lat, x, tl, tb, ("gauss2d", (2 * ARC, 1 * ARC, 205.0)), 6 * ARC)
    swap = og.grid_bruteforce(lon, lat, x, tl, tb, ("gauss2d", (1 * ARC, 2 * ARC, 115.0)), 6 * ARC)
    np.testing.assert_allclose(flip["W"], base["W"], rtol=1e-12)
    np.testing.assert_allclose(swap["W"], base["W"], rtol=1e-12)
    circ = og.grid_bruteforce(lon, lat, x, tl, tb, ("gauss2d", (1.5 * ARC, 1.5 * ARC, 70.0)), RS)
    one = og.grid_bruteforce(lon, lat, x, tl, tb, K1, RS)
    np.testing.assert_allclose(circ["W"], one["W"], rtol=1e-13)


def test_point_source_flux_and_eq6():
    """Isolated Gaussian source, dense regular sampling (Sect. 3.5 Eq. 6, App. A.1).

    Gridding with a Gaussian kernel convolves the source: peak
    A s^2/(s^2+k^2), second moment s^2 + k^2 per axis, total flux 2 pi s^2 A
    conserved (the flux-conservation property of Eq. 3).
    """
    A = 3.0
    ss = 4.0 / math.sqrt(8 * math.log(2))      # arcmin
    sk = 1.5
    h = sk / 4.0
    ax = np.arange(-30.0, 30.0 + 1e-9, h)
    sl, sb = np.meshgrid(ax, ax)
    sl, sb = sl.ravel() * ARC, sb.ravel() * ARC
    # source value by haversine distance from (0, 0), written here independently
    hv = np.sin(np.radians(sb) / 2) ** 2 + np.cos(np.radians(sb)) * np.sin(np.radians(sl) / 2) ** 2
    dsrc = np.degrees(2 * np.arcsin(np.sqrt(hv))) * 60.0
    val = A * np.exp(-dsrc ** 2 / (2 * ss * ss))
    tx = np.arange(-15.0, 15.0 + 1e-9, 0.5)
    tl, tb = np.meshgrid(tx, tx)
    r = og.grid_kdtree(np.mod(sl, 360), sb, val[:, None], np.mod(tl.ravel() * ARC, 360),
                       tb.ravel() * ARC, ("gauss1d", (sk * ARC,)), 5 * sk * ARC)
    R = r["R"][0].reshape(tl.shape)
    omega = 0.5 * 0.5 * np.cos(np.radians(tb * ARC))
    flux = (R * omega).sum()
    assert flux == pytest.approx(2 * math.pi * ss * ss * A, rel=1e-4)
    c = R.shape[0] // 2
    assert R[c, c] == pytest.approx(A * ss * ss / (ss * ss + sk * sk), rel=1e-3)
    var_x = (R * tl ** 2).sum() / R.sum()
    var_y = (R * tb ** 2).sum() / R.sum()
    assert var_x == pytest.approx(ss * ss + sk * sk, rel=1e-3)
    assert var_y == pytest.approx(ss * ss + sk * sk, rel=1e-3)


# ------------------------------------------------ library special case + cross

@pytest.mark.parametrize("where", ["pole", "seam", "midlat"])
def test_kdtree_equals_bruteforce(where):
    g = np.random.default_rng(7)
    if where == "pole":
        lon = g.uniform(0, 360, 1500)
        lat = 90 - np.degrees(np.arccos(g.uniform(math.cos(math.radians(0.6)), 1, 1500)))
        tl, tb = np.meshgrid(np.linspace(0, 359, 12), np.linspace(89.5, 90, 6))
    elif where == "seam":
        lon = g.uniform(-0.4, 0.4, 1500) % 360
        lat = g.uniform(-0.4, 0.4, 1500)
        tl, tb = np.meshgrid(np.linspace(-0.3, 0.3, 9) % 360, np.linspace(-0.3, 0.3, 9))
    else:
        lon = g.uniform(200, 201, 1500)
        lat = g.uniform(50, 50.7, 1500)
        tl, tb = np.meshgrid(np.linspace(200.1, 200.9, 9), np.linspace(50.1, 50.6, 9))
    x = g.normal(size=(1500, 3))
    k2 = ("gauss2d", (3 * ARC, 2 * ARC, 40.0))
    for kern, rs in ((K1, RS), (k2, 9 * ARC)):
        a = og.grid_bruteforce(lon, lat, x, tl.ravel(), tb.ravel(), kern, rs)
        b = og.grid_kdtree(lon, lat, x, tl.ravel(), tb.ravel(), kern, rs, block=17)
        assert np.array_equal(a["count"], b["count"])
        assert np.array_equal(a["hash"], b["hash"])
        np.testing.assert_allclose(b["W"], a["W"], rtol=1e-12)
        m = a["W"] > 0
        np.testing.assert_allclose(b["R"][:, m], a["R"][:, m], rtol=1e-10, atol=1e-13)
        ns = og.neighbour_sets(lon, lat, tl.ravel(), tb.ravel(), rs, block=23)
        assert np.array_equal(ns["count"], a["count"])
        assert np.array_equal(ns["hash"], a["hash"])


def test_validation_rejects_bad_coordinates():
    with pytest.raises(ValueError):
        og.grid_bruteforce([0.0], [91.0], [[1.0]], [0.0], [0.0], K1, RS)
    with pytest.raises(ValueError):
        og.grid_bruteforce([np.nan], [0.0], [[1.0]], [0.0], [0.0], K1, RS)


# ----------------------------------------- planted mistakes must fail a pin

def _pins_pass():
    cases = _load_cases()
    try:
        for c in cases["cases"]:
            test_hand_cases(c)
        for row in cases["ellipse"]["rows"]:
            test_ellipse_axes(row)
        test_kernel_symmetry()
    except AssertionError:
        return False
    return True


MUTATIONS = {
    "vincenty_sign": lambda l1, b1, l2, b2: np.arctan2(
        np.hypot(np.cos(b2) * np.sin(l2 - l1),
                 np.cos(b1) * np.sin(b2) + np.sin(b1) * np.cos(b2) * np.cos(l2 - l1)),
        np.sin(b1) * np.sin(b2) + np.cos(b1) * np.cos(b2) * np.cos(l2 - l1)),
    "bearing_swapped": lambda l1, b1, l2, b2: bearing(l2, b2, l1, b1) + 0.3,
}


@pytest.mark.parametrize("name", ["vincenty_sign", "bearing_swapped", "sigma_not_squared",
                                  "weight_sum_counts", "axes_swapped"])
def test_planted_mistakes_are_caught(monkeypatch, name):
    if name == "vincenty_sign":
        monkeypatch.setattr(og, "vincenty", MUTATIONS[name])
    elif name == "bearing_swapped":
        monkeypatch.setattr(og, "bearing", MUTATIONS[name])
    elif name == "sigma_not_squared":
        orig = og.kernel_weight
        monkeypatch.setattr(og, "kernel_weight",
                            lambda k, d, *a: np.exp(-d / (2 * np.radians(k[1][0]) ** 2)) if k[0] == "gauss1d" else orig(k, d, *a))
    elif name == "weight_sum_counts":
        orig = og.kernel_weight
        calls = {"n": 0}
        def w(k, d, *a):
            calls["n"] += 1
            return orig(k, d, *a) if calls["n"] % 2 else np.ones_like(d)
        monkeypatch.setattr(og, "kernel_weight", w)
    elif name == "axes_swapped":
        orig = og.kernel_weight
        monkeypatch.setattr(og, "kernel_weight",
                            lambda k, d, *a: orig((k[0], (k[1][1], k[1][0], k[1][2])), d, *a) if k[0] == "gauss2d" else orig(k, d, *a))
    assert not _pins_pass(), f"planted mistake {name} slipped through the pins"
