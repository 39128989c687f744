"""Host build of the library's HEALPix RING code (the code the kernels run).

Pinned to the definitions of Gorski et al. (2005), cited by the paper for
the HEALPix grid (Sect. 2.2, 3.2): ring counts, start indices and centre
latitudes in closed form, exact pix -> ang -> pix round trips, equal pixel
areas, and the two geometric facts the ring lookup relies on (latitude
extent of a ring, longitude extent of a pixel), then the lookup's superset
property against brute-force distances.
"""
import math

import numpy as np
import pytest

import paper_1604_06667_amd as cgp


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 64, 1024, 8192])
def test_ring_table_closed_forms(nside):
    total = 0
    for i in [1, 2, nside - 1, nside, nside + 1, 2 * nside, 3 * nside, 3 * nside + 1, 4 * nside - 1]:
        if i < 1 or i > 4 * nside - 1:
            continue
        s, n, z = cgp.hpx_ring_info(nside, i)
        if i < nside:
            assert n == 4 * i and s == 2 * i * (i - 1)
            assert z == pytest.approx(1 - i * i / (3 * nside * nside), abs=1e-15)
        elif i <= 3 * nside:
            assert n == 4 * nside and s == 2 * nside * (nside - 1) + 4 * nside * (i - nside)
            assert z == pytest.approx(4 / 3 - 2 * i / (3 * nside), abs=1e-15)
        else:
            k = 4 * nside - i
            assert n == 4 * k and s == 12 * nside * nside - 2 * k * (k + 1)
            assert z == pytest.approx(-(1 - k * k / (3 * nside * nside)), abs=1e-15)
    if nside <= 64:
        for i in range(1, 4 * nside):
            s, n, _ = cgp.hpx_ring_info(nside, i)
            assert s == total
            total += n
        assert total == 12 * nside * nside


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16, 32, 64])
def test_round_trip_every_pixel(nside):
    pix = np.arange(12 * nside * nside)
    lon, lat = cgp.hpx_pix2ang_ring(nside, pix)
    assert np.array_equal(cgp.hpx_ang2pix_ring(nside, lon, lat), pix)
    ring, j = cgp.hpx_pix2ring(nside, pix)
    # pixel centres: ring centre z, evenly spaced longitudes with the belt shift
    for i in np.unique(ring):
        m = ring == i
        s, n, z = cgp.hpx_ring_info(nside, int(i))
        assert m.sum() == n
        np.testing.assert_allclose(np.sin(np.radians(lat[m])), z, atol=1e-13)
        shift = 0.5 if (i < nside or i > 3 * nside or (i - nside) % 2 == 0) else 0.0
        np.testing.assert_allclose(lon[m], (j[m] + shift) * 360.0 / n, atol=1e-10)


@pytest.mark.parametrize("nside", [4, 16])
def test_equal_area(nside):
    g = np.random.default_rng(nside)
    n = 2_000_000
    lon = g.uniform(0, 360, n)
    lat = np.degrees(np.arcsin(g.uniform(-1, 1, n)))
    pix = cgp.hpx_ang2pix_ring(nside, lon, lat)
    cnt = np.bincount(pix, minlength=12 * nside * nside)
    e = n / cnt.size
    chi2 = ((cnt - e) ** 2 / e).sum()
    dof = cnt.size - 1
    assert abs(chi2 - dof) < 6 * math.sqrt(2 * dof)


def _random_points(g, n):
    lon = g.uniform(0, 360, n)
    lat = np.degrees(np.arcsin(g.uniform(-1, 1, n)))
    return lon, lat


@pytest.mark.parametrize("nside", [1, 2, 4, 16, 256])
def test_ring_latitude_and_pixel_longitude_extent(nside):
    g = np.random.default_rng(100 + nside)
    lon, lat = _random_points(g, 400_000)
    # include the poles and points on ring-centre latitudes
    lon = np.r_[lon, 17.0, 203.0]
    lat = np.r_[lat, 90.0, -90.0]
    pix = cgp.hpx_ang2pix_ring(nside, lon, lat)
    ring, j = cgp.hpx_pix2ring(nside, pix)
    zc = np.array([1.0] + [cgp.hpx_ring_info(nside, i)[2] for i in range(1, 4 * nside)] + [-1.0])
    z = np.sin(np.radians(lat))
    assert np.all(z <= zc[ring - 1] + 1e-12) and np.all(z >= zc[ring + 1] - 1e-12)
    n = np.array([cgp.hpx_ring_info(nside, int(i))[1] for i in ring])
    x = np.radians(lon) * n / (2 * math.pi)          # longitude in units of pixels
    # pixel j covers longitudes within [j - 1/2, j + 1] (mod n)
    d = (x - j + n / 2.0) % n - n / 2.0
    assert np.all(d >= -0.5 - 1e-9) and np.all(d <= 1.0 + 1e-9)
    # ... and, tighter, within half a pixel of its centre longitude, whose
    # phase is 1/2 in the caps and alternates 1/2, 0 along the belt
    clon, _ = cgp.hpx_pix2ang_ring(nside, pix)
    c = np.radians(clon) * n / (2 * math.pi)
    ph = np.where((ring < nside) | (ring > 3 * nside), 0.5,
                  np.where((ring - nside) % 2 == 0, 0.5, 0.0))
    assert np.allclose((c - j), ph, atol=1e-9)
    dc = (x - c + n / 2.0) % n - n / 2.0
    assert np.all(np.abs(dc) <= 0.5 + 1e-9)


def _brute_pix_within(nside, lon0, lat0, rho, g, n=60_000):
    """Pixels of random points inside the cap (rejection sampling near it)."""
    c = np.array([math.cos(math.radians(lat0)) * math.cos(math.radians(lon0)),
                  math.cos(math.radians(lat0)) * math.sin(math.radians(lon0)),
                  math.sin(math.radians(lat0))])
    zmin = math.cos(min(math.pi, math.radians(90 - lat0) + rho))
    zmax = math.cos(max(0.0, math.radians(90 - lat0) - rho))
    z = g.uniform(zmin, zmax, n)
    lon = g.uniform(0, 360, n)
    lat = np.degrees(np.arcsin(z))
    p = np.stack([np.sqrt(1 - z * z) * np.cos(np.radians(lon)),
                  np.sqrt(1 - z * z) * np.sin(np.radians(lon)), z], 1)
    ang = np.arctan2(np.linalg.norm(np.cross(p, c), axis=1), p @ c)
    m = ang <= rho
    return cgp.hpx_ang2pix_ring(nside, lon[m], lat[m])


CAPS = [(10.0, 20.0, 1.0), (0.05, -3.0, 0.5), (359.9, 41.0, 0.2), (123.0, 89.7, 0.5),
        (250.0, -89.95, 0.1), (45.0, 0.0, 0.01), (300.0, 41.8, 2.0), (180.0, -41.8, 3.0),
        (77.0, 60.0, 30.0), (5.0, 10.0, 100.0), (200.0, 90.0, 0.3), (33.0, -90.0, 1.0)]


@pytest.mark.parametrize("nside", [1, 4, 64, 1024, 8192])
@pytest.mark.parametrize("cap", CAPS, ids=lambda c: f"{c[0]}_{c[1]}_{c[2]}")
def test_cap_ranges_superset(nside, cap):
    lon0, lat0, rho_deg = cap
    g = np.random.default_rng(int(nside + 7 * rho_deg * 100 + lat0 * 10) & 0xFFFF)
    rng = cgp.hpx_cap_ranges(nside, lon0, lat0, rho_deg)
    pix = _brute_pix_within(nside, lon0, lat0, math.radians(rho_deg), g)
    assert pix.size > 0
    lo, hi = rng[:, 0], rng[:, 1]
    assert np.all(hi >= lo)
    order = np.argsort(lo)
    lo, hi = lo[order], hi[order]
    k = np.searchsorted(lo, pix, side="right") - 1
    inside = (k >= 0) & (pix <= hi[np.maximum(k, 0)])
    assert inside.all(), f"{(~inside).sum()} pixels of in-cap points missed"


def _coverage(rng, pix):
    lo, hi = rng[:, 0], rng[:, 1]
    order = np.argsort(lo)
    lo, hi = lo[order], hi[order]
    k = np.searchsorted(lo, pix, side="right") - 1
    return (k >= 0) & (pix <= hi[np.maximum(k, 0)])


# 8x8 target patches: (centre lon, centre lat, spacing deg, support deg)
PATCHES = [(10.0, 20.0, 0.02, 0.075), (359.95, -5.0, 0.02, 0.075), (120.0, 89.9, 0.01, 0.05),
           (200.0, -89.93, 0.005, 0.04), (45.0, 41.81, 0.05, 0.2), (300.0, 0.0, 1.0, 3.0),
           (0.0, 60.0, 5.0, 20.0)]


@pytest.mark.parametrize("nside", [4, 256, 8192])
@pytest.mark.parametrize("patch", PATCHES, ids=lambda c: f"{c[0]}_{c[1]}_{c[2]}")
def test_targets_ranges_superset(nside, patch):
    """Union of per-target disks (the tile lookup) covers every pixel of every
    in-support point of every target, and is no wider than the cap lookup."""
    lon0, lat0, dx, rho_deg = patch
    g = np.random.default_rng(int(nside * 3 + lat0 * 7 + dx * 1000) & 0xFFFF)
    ii, jj = np.meshgrid(np.arange(8) - 3.5, np.arange(8) - 3.5)
    lat = np.clip(lat0 + jj.ravel() * dx, -90.0, 90.0)
    lon = (lon0 + ii.ravel() * dx / max(np.cos(np.radians(lat0)), 0.05)) % 360.0
    rng = cgp.hpx_targets_ranges(nside, lon, lat, rho_deg)
    assert np.all(rng[:, 1] >= rng[:, 0])
    for k in range(0, 64, 9):
        pix = _brute_pix_within(nside, lon[k], lat[k], math.radians(rho_deg), g, n=20_000)
        assert pix.size > 0
        inside = _coverage(rng, pix)
        assert inside.all(), f"target {k}: {(~inside).sum()} pixels missed"
    # no wider than one cap around all targets
    c = np.stack([np.cos(np.radians(lat)) * np.cos(np.radians(lon)),
                  np.cos(np.radians(lat)) * np.sin(np.radians(lon)), np.sin(np.radians(lat))], 1)
    m = c.mean(0)
    m /= np.linalg.norm(m)
    r = np.degrees(np.max(np.arccos(np.clip(c @ m, -1, 1))))
    cap = cgp.hpx_cap_ranges(nside, math.degrees(math.atan2(m[1], m[0])) % 360.0,
                             math.degrees(math.asin(m[2])), r + rho_deg + 1e-9)
    npix_t = int((rng[:, 1] - rng[:, 0] + 1).sum())
    npix_c = int((cap[:, 1] - cap[:, 0] + 1).sum())
    assert npix_t <= npix_c


# ---- HEALPix map targets (cg_hpx_centres: the code cg_create_healpix runs) ----

@pytest.mark.parametrize("nside", [1, 2, 16, 256])
@pytest.mark.parametrize("order", ["ring", "nested"])
def test_map_centres_match_oracle(nside, order):
    from oracle.healpix import centres
    lo, la = cgp.hpx_centres(nside, order)
    rlo, rla = centres(nside, order)
    dl = np.abs((lo - rlo + 180.0) % 360.0 - 180.0)
    assert dl.max() < 1e-9 and np.abs(la - rla).max() < 1e-9
    assert lo.min() >= 0.0 and lo.max() < 360.0


def test_map_centres_round_trip_and_ranges():
    # RING centres map back to their own pixel; a sub-range equals the slice
    nside = 64
    lo, la = cgp.hpx_centres(nside, "ring")
    assert np.array_equal(cgp.hpx_ang2pix_ring(nside, lo, la), np.arange(12 * nside * nside))
    slo, sla = cgp.hpx_centres(nside, "nested", first=1000, count=77)
    flo, fla = cgp.hpx_centres(nside, "nested")
    assert np.array_equal(slo, flo[1000:1077]) and np.array_equal(sla, fla[1000:1077])


@pytest.mark.parametrize("args", [(3, "ring"), (0, "ring"), (16384, "nested")])
def test_map_centres_rejects_bad_nside(args):
    with pytest.raises(cgp.CgError):
        cgp.hpx_centres(*args, count=1)


def test_map_centres_rejects_range_outside_map():
    with pytest.raises(cgp.CgError):
        cgp.hpx_centres(2, "ring", first=40, count=9)
