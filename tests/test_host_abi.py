"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before any device work (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_1604_06667_amd as cgp
from paper_1604_06667_amd import _cg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "cg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cg_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 20
    L = cgp.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_cg.SIGNATURES), "binding and header disagree"
    assert "gfx950" in cgp.version()


def test_host_argument_errors():
    L = cgp.lib()
    h = C.c_void_p()
    assert L.cg_create_wcs(None, None, 1) == _cg.E_INVALID
    w = _cg.CgWcs(7, 0, 10, 10, 1, 1, 0, 0, 1, 1)
    assert L.cg_create_wcs(C.byref(h), C.byref(w), 1) == _cg.E_UNSUPPORTED
    w = _cg.CgWcs(0, 0, 0, 10, 1, 1, 0, 0, 1, 1)
    assert L.cg_create_wcs(C.byref(h), C.byref(w), 1) == _cg.E_INVALID
    w = _cg.CgWcs(0, 0, 10, 10, 1, 1, 0, 0, 1, 1)
    assert L.cg_create_wcs(C.byref(h), C.byref(w), 0) == _cg.E_INVALID
    w = _cg.CgWcs(0, 0, 10, 10, 1, 1, 0, 95.0, 1, 1)     # |CRVAL2| > 90
    assert L.cg_create_wcs(C.byref(h), C.byref(w), 1) == _cg.E_INVALID
    w = _cg.CgWcs(1, 0, 10, 10, 1, 1, 0, 0, 0.0, 1)      # zero CDELT
    assert L.cg_create_wcs(C.byref(h), C.byref(w), 1) == _cg.E_INVALID
    assert L.cg_create_sightlines(C.byref(h), None, None, 5, 1, None) == _cg.E_INVALID
    p = (C.c_double * 1)(1.0)
    assert L.cg_set_kernel(None, 0, p, 1, 1.0, 1.0) == _cg.E_INVALID
    assert L.cg_grid(None, None, None, None, 1, 1, 1, None, 0, None) == _cg.E_INVALID
    assert L.cg_grid_datacube(None, None, None, None, 1, 1, 1, None, None, None, 0,
                              None) == _cg.E_INVALID
    sz = C.c_size_t()
    assert L.cg_workspace_size(None, 10, C.byref(sz)) == _cg.E_INVALID
    # an allocator needs both functions (or neither)
    keep = _cg.ALLOC_FN(lambda n, d, s, c: None)
    assert L.cg_set_allocator(keep, _cg.FREE_FN(), None) == _cg.E_INVALID
    assert L.cg_set_nside(None, 64) == _cg.E_INVALID
    assert L.cg_set_lookup(None, 1) == _cg.E_INVALID
    a, b = C.c_int64(), C.c_int64()
    assert L.cg_disk_stats(None, C.byref(a), C.byref(b)) == _cg.E_INVALID
    assert L.cg_sync(None, None) == _cg.E_INVALID
    v = C.c_int64()
    assert L.cg_query(None, 0, C.byref(v)) == _cg.E_INVALID
    with pytest.raises(cgp.CgError):
        cgp.hpx_ang2pix_ring(0, [0.0], [0.0])
    with pytest.raises(cgp.CgError):
        cgp.hpx_cap_ranges(64, 0, 0, 30.0, max_ranges=2)
    with pytest.raises(cgp.CgError):
        cgp.wcs_pix2world({"NAXIS1": 4, "NAXIS2": 4, "CTYPE1": "RA---TAN", "CDELT1": 1, "CDELT2": 1},
                          [1.0], [1.0])
    with pytest.raises(cgp.CgError):
        cgp.wcs_pix2world({"NAXIS1": 4, "NAXIS2": 4, "CTYPE1": "RA---SFL", "CDELT1": 1, "CDELT2": 1,
                           "CRVAL2": 91.0}, [1.0], [1.0])


@pytest.mark.parametrize("hdr", [
    {"NAXIS": 2, "NAXIS1": 96, "NAXIS2": 96, "CTYPE1": "RA---CAR", "CTYPE2": "DEC--CAR",
     "CRPIX1": 48.5, "CRPIX2": -851.5, "CRVAL1": 120.0, "CRVAL2": 0.0,
     "CDELT1": -1 / 30, "CDELT2": 1 / 30},
    {"NAXIS": 2, "NAXIS1": 600, "NAXIS2": 600, "CTYPE1": "RA---SIN", "CTYPE2": "DEC--SIN",
     "CRPIX1": 300.5, "CRPIX2": 300.5, "CRVAL1": 120.0, "CRVAL2": 30.0,
     "CDELT1": -1 / 60, "CDELT2": 1 / 60},
    {"NAXIS": 2, "NAXIS1": 101, "NAXIS2": 101, "CTYPE1": "GLON-SIN", "CTYPE2": "GLAT-SIN",
     "CRPIX1": 51, "CRPIX2": 51, "CRVAL1": 12.345, "CRVAL2": 87.0, "CDELT1": -1.0, "CDELT2": 1.0},
    {"NAXIS": 2, "NAXIS1": 4320, "NAXIS2": 2160, "CTYPE1": "RA---CAR", "CTYPE2": "DEC--CAR",
     "CRPIX1": 2160.5, "CRPIX2": 1080.5, "CRVAL1": 0.0, "CRVAL2": 0.0,
     "CDELT1": -1 / 12, "CDELT2": 1 / 12},
    {"NAXIS": 2, "NAXIS1": 400, "NAXIS2": 200, "CTYPE1": "RA---SFL", "CTYPE2": "DEC--SFL",
     "CRPIX1": 200.5, "CRPIX2": 100.5, "CRVAL1": 30.0, "CRVAL2": 0.0,
     "CDELT1": -1.0, "CDELT2": 1.0},
    {"NAXIS": 2, "NAXIS1": 300, "NAXIS2": 300, "CTYPE1": "RA---ZEA", "CTYPE2": "DEC--ZEA",
     "CRPIX1": 150.5, "CRPIX2": 150.5, "CRVAL1": 200.0, "CRVAL2": -35.0,
     "CDELT1": -0.8, "CDELT2": 0.8},
    {"NAXIS": 2, "NAXIS1": 120, "NAXIS2": 120, "CTYPE1": "GLON-ZEA", "CTYPE2": "GLAT-ZEA",
     "CRPIX1": 60.5, "CRPIX2": 60.5, "CRVAL1": 0.0, "CRVAL2": 90.0,
     "CDELT1": -0.05, "CDELT2": 0.05},
    # oblique cylindrical: north and south reference points, a pole, whole-sky planes
    {"NAXIS": 2, "NAXIS1": 200, "NAXIS2": 150, "CTYPE1": "RA---CAR", "CTYPE2": "DEC--CAR",
     "CRPIX1": 100.5, "CRPIX2": 75.5, "CRVAL1": 150.0, "CRVAL2": 40.0,
     "CDELT1": -0.1, "CDELT2": 0.1},
    {"NAXIS": 2, "NAXIS1": 361, "NAXIS2": 181, "CTYPE1": "GLON-CAR", "CTYPE2": "GLAT-CAR",
     "CRPIX1": 181.0, "CRPIX2": 91.0, "CRVAL1": 266.4, "CRVAL2": -28.9,
     "CDELT1": -1.0, "CDELT2": 1.0},
    {"NAXIS": 2, "NAXIS1": 100, "NAXIS2": 100, "CTYPE1": "RA---CAR", "CTYPE2": "DEC--CAR",
     "CRPIX1": 50.5, "CRPIX2": 50.5, "CRVAL1": 10.0, "CRVAL2": 90.0,
     "CDELT1": -0.2, "CDELT2": 0.2},
    {"NAXIS": 2, "NAXIS1": 361, "NAXIS2": 181, "CTYPE1": "RA---SFL", "CTYPE2": "DEC--SFL",
     "CRPIX1": 181.0, "CRPIX2": 91.0, "CRVAL1": 300.0, "CRVAL2": 62.0,
     "CDELT1": -1.0, "CDELT2": 1.0},
    {"NAXIS": 2, "NAXIS1": 120, "NAXIS2": 90, "CTYPE1": "RA---SFL", "CTYPE2": "DEC--SFL",
     "CRPIX1": 60.5, "CRPIX2": 45.5, "CRVAL1": 45.0, "CRVAL2": -70.0,
     "CDELT1": -0.25, "CDELT2": 0.25},
])
def test_library_wcs_matches_oracle(hdr):
    g = np.random.default_rng(0)
    n = 5000
    i = g.uniform(0.5, hdr["NAXIS1"] + 0.5, n)
    j = g.uniform(0.5, hdr["NAXIS2"] + 0.5, n)
    lo, la = cgp.wcs_pix2world(hdr, i, j)
    w = {"proj": hdr["CTYPE1"][-3:], "naxis1": hdr["NAXIS1"], "naxis2": hdr["NAXIS2"],
         "crpix1": hdr["CRPIX1"], "crpix2": hdr["CRPIX2"], "crval1": hdr["CRVAL1"],
         "crval2": hdr["CRVAL2"], "cdelt1": hdr["CDELT1"], "cdelt2": hdr["CDELT2"]}
    olo, ola = oracle.wcs_world(w, i, j)
    assert np.array_equal(np.isnan(lo), np.isnan(olo))
    ok = ~np.isnan(lo)
    np.testing.assert_allclose(la[ok], ola[ok], atol=1e-10)
    dl = (lo[ok] - olo[ok] + 180.0) % 360.0 - 180.0
    assert np.abs(dl * np.cos(np.radians(ola[ok]))).max() < 1e-10
