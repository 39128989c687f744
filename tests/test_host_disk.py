"""Host checks of the sample-centric lookup's query disks (Sect. 3.3, Eq.
4-5): the RING pixel ranges that cg_hpx_query_disk returns run the same
code as the disk-lookup kernels.

* Superset: every target within the support of a sample has its nearest
  pixel inside the shifted disk of the sample's pixel (random pairs at every
  latitude, at distances up to the support, with plain spherical geometry in
  NumPy deciding the distance).
* Symmetry: HEALPix is invariant under rotations by 90 deg in longitude.  For
  the pixels a whole number of quarter rings from the reference pixel the
  shift of Eq. 4 is exact on every ring (no rounding), so the disk of the
  pixel a quarter ring east of such a pixel is its disk moved by a quarter of
  every ring.
* Size: the disk is no larger than a few times the cap it must cover.
"""
import math

import numpy as np
import pytest

cgp = pytest.importorskip("paper_1604_06667_amd")


def _ranges_to_set(r):
    out = set()
    for lo, hi in r:
        out.update(range(int(lo), int(hi) + 1))
    return out


def _offset_points(lon, lat, dist, bearing):
    """Points at angular distance dist (rad) and bearing (rad, east of north)
    from (lon, lat) in degrees: the spherical direct problem."""
    la, lo = np.radians(lat), np.radians(lon)
    la2 = np.arcsin(np.sin(la) * np.cos(dist) + np.cos(la) * np.sin(dist) * np.cos(bearing))
    lo2 = lo + np.arctan2(np.sin(bearing) * np.sin(dist) * np.cos(la),
                          np.cos(dist) - np.sin(la) * np.sin(la2))
    return np.degrees(lo2) % 360.0, np.degrees(la2)


def _dist(lo1, la1, lo2, la2):
    a1, b1, a2, b2 = map(np.radians, (lo1, la1, lo2, la2))
    v1 = np.stack([np.cos(b1) * np.cos(a1), np.cos(b1) * np.sin(a1), np.sin(b1)], -1)
    v2 = np.stack([np.cos(b2) * np.cos(a2), np.cos(b2) * np.sin(a2), np.sin(b2)], -1)
    return 2.0 * np.arcsin(np.clip(0.5 * np.linalg.norm(v1 - v2, axis=-1), 0.0, 1.0))


@pytest.mark.parametrize("nside,support_px", [(1, 0.3), (2, 1.0), (8, 2.5), (64, 0.5),
                                              (64, 6.0), (1024, 3.0), (8192, 10.0)])
def test_query_disk_is_superset(nside, support_px):
    pix_deg = math.degrees(math.sqrt(math.pi / 3.0) / nside)
    rs_deg = support_px * pix_deg
    g = np.random.default_rng(nside * 7 + int(10 * support_px))
    m = 300
    # samples: uniform on the sphere plus bands at the poles and at |z| = 2/3
    z = np.concatenate([g.uniform(-1, 1, m), g.uniform(0.995, 1.0, 50) * g.choice([-1, 1], 50),
                        2.0 / 3.0 + g.uniform(-0.01, 0.01, 50) * g.choice([-1, 1], 50)])
    lat = np.degrees(np.arcsin(z))
    lon = g.uniform(0.0, 360.0, lat.size)
    spix = cgp.hpx_ang2pix_ring(nside, lon, lat)
    for k in range(lat.size):
        disk = _ranges_to_set(cgp.hpx_query_disk(nside, int(spix[k]), rs_deg))
        d = math.radians(rs_deg) * np.sqrt(g.uniform(0.0, 1.0, 40))
        d[:8] = math.radians(rs_deg) * (1.0 - 1e-9)      # on the support edge
        tlo, tla = _offset_points(np.full(40, lon[k]), np.full(40, lat[k]), d,
                                  g.uniform(0.0, 2 * math.pi, 40))
        inside = _dist(lon[k], lat[k], tlo, tla) <= math.radians(rs_deg)
        tpix = cgp.hpx_ang2pix_ring(nside, tlo[inside], tla[inside])
        missing = [int(p) for p in tpix if int(p) not in disk]
        assert not missing, (k, int(spix[k]), missing[:5])


@pytest.mark.parametrize("nside,support_px", [(4, 1.5), (64, 3.0), (1024, 8.0)])
def test_query_disk_quarter_turn(nside, support_px):
    rs_deg = support_px * math.degrees(math.sqrt(math.pi / 3.0) / nside)
    rng = np.random.default_rng(nside)
    for ring in rng.integers(1, 4 * nside, 12):
        s, n, _ = cgp.hpx_ring_info(nside, int(ring))
        j = int(rng.integers(0, 4)) * (n // 4)
        a = cgp.hpx_query_disk(nside, s + j, rs_deg)
        b = cgp.hpx_query_disk(nside, s + (j + n // 4) % n, rs_deg)
        moved = set()
        for p in _ranges_to_set(a):
            r2, j2 = cgp.hpx_pix2ring(nside, np.array([p], dtype=np.int64))
            s2, n2, _ = cgp.hpx_ring_info(nside, int(r2[0]))
            moved.add(s2 + (int(j2[0]) + n2 // 4) % n2)
        assert moved == _ranges_to_set(b), (int(ring), j)


@pytest.mark.parametrize("nside,support_px", [(64, 2.0), (1024, 5.0), (8192, 12.0)])
def test_query_disk_size(nside, support_px):
    px = math.sqrt(math.pi / 3.0) / nside                 # pixel side (rad)
    rs = support_px * px
    for lat in (0.0, 30.0, 41.8, 60.0, 89.0):
        p = int(cgp.hpx_ang2pix_ring(nside, np.array([10.0]), np.array([lat]))[0])
        cnt = len(_ranges_to_set(cgp.hpx_query_disk(nside, p, math.degrees(rs))))
        cap = math.pi * (rs + 2.0 * px) ** 2 / px ** 2     # pixels of the cap to cover
        assert cap / 2 <= cnt <= 3.0 * cap + 8 * (support_px + 3), (lat, cnt, cap)


def test_query_disk_rejects_bad_arguments():
    with pytest.raises(cgp.CgError):
        cgp.hpx_query_disk(3, 0, 1.0)
    with pytest.raises(cgp.CgError):
        cgp.hpx_query_disk(4, 12 * 16, 1.0)
    with pytest.raises(cgp.CgError):
        cgp.hpx_query_disk(4, 0, 0.0)
    with pytest.raises(cgp.CgError):
        cgp.hpx_query_disk(8192, 0, 5.0, max_ranges=1)
