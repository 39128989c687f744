"""Seeded synthetic workloads for the gridding tests and the benchmark.

This module only *places* samples and targets and draws the synthetic sky
signal (point sources, spectral-line cubes, noise).  It holds none of the
gridding arithmetic: no great-circle distances, no kernel weights, no
HEALPix and no WCS deprojection.  Both the CPU oracle and the GPU path consume
what it returns, so it is the one module they share.

Every generator is driven by ``numpy.random.default_rng(SeedSequence([1604,
6667, k]))`` for a workload number ``k``; the per-element noise of the big
spectral cubes is drawn with a seeded ``torch.Generator`` on the device the
cube is built on (CPU for tests, the GPU for full-size benchmarks), so a
given (workload, device) pair always yields the same arrays.

Angles are in degrees everywhere; data arrays are ``[N][C]`` row-major
(one spectrum contiguous).  BF16 workloads hold float32 values that are
exactly representable in bfloat16 (rounded once here), so an upcast is exact.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ARCMIN = 1.0 / 60.0
FWHM_TO_SIGMA = 1.0 / math.sqrt(8.0 * math.log(2.0))


def rng(k: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([1604, 6667, int(k)]))


@dataclass
class Workload:
    """One gridding job: samples, data, target description and kernel."""

    name: str
    lon: np.ndarray            # float64 [N], degrees
    lat: np.ndarray            # float64 [N], degrees
    data: object               # [N][C]: numpy array or torch tensor
    dtype: str                 # 'f64' | 'f32' | 'bf16' | 'f16' (delivered dtype)
    target: dict               # {'kind': 'wcs', 'wcs': {...}} or {'kind': 'sightlines', 'lon', 'lat'}
    kernel: tuple              # ('gauss1d', (sigma,)) | ('gauss2d', (smaj, smin, pa))
    support: float             # degrees
    nside: int | None = None   # explicit HEALPix nside (None: hpx_maxres rule)
    hpx_maxres: float | None = None
    meta: dict = field(default_factory=dict)

    @property
    def nsamples(self) -> int:
        return int(self.lon.shape[0])

    @property
    def nchan(self) -> int:
        return int(self.data.shape[1])

    def ntargets(self) -> int:
        t = self.target
        if t["kind"] == "wcs":
            return int(t["wcs"]["naxis1"]) * int(t["wcs"]["naxis2"])
        if t["kind"] == "healpix":
            return 12 * int(t["nside"]) ** 2
        return int(np.asarray(t["lon"]).shape[0])


# ---------------------------------------------------------------------------
# placement helpers (no gridding arithmetic)
# ---------------------------------------------------------------------------

def uniform_box(g: np.random.Generator, n: int, lon0: float, lon1: float,
                lat0: float, lat1: float) -> tuple[np.ndarray, np.ndarray]:
    """Area-uniform points in a lon/lat box (lon uniform, sin(lat) uniform)."""
    lon = g.uniform(lon0, lon1, n)
    s0, s1 = math.sin(math.radians(lat0)), math.sin(math.radians(lat1))
    lat = np.degrees(np.arcsin(g.uniform(s0, s1, n)))
    return np.mod(lon, 360.0), lat


def uniform_sphere(g: np.random.Generator, n: int) -> tuple[np.ndarray, np.ndarray]:
    lon = g.uniform(0.0, 360.0, n)
    lat = np.degrees(np.arcsin(g.uniform(-1.0, 1.0, n)))
    return lon, lat


def tangent_place(lon0: float, lat0: float, x_deg: np.ndarray,
                  y_deg: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Place local offsets (x east, y north, degrees) around (lon0, lat0).

    Uses the gnomonic mapping p = normalise(c + x e + y n); it is only a way
    to lay a scan pattern on the sky, not one of the gridder's projections.
    """
    a, d = math.radians(lon0), math.radians(lat0)
    c = np.array([math.cos(d) * math.cos(a), math.cos(d) * math.sin(a), math.sin(d)])
    e = np.array([-math.sin(a), math.cos(a), 0.0])
    nn = np.array([-math.sin(d) * math.cos(a), -math.sin(d) * math.sin(a), math.cos(d)])
    x = np.tan(np.radians(np.asarray(x_deg, dtype=np.float64)))
    y = np.tan(np.radians(np.asarray(y_deg, dtype=np.float64)))
    p = c[None, :] + x[:, None] * e[None, :] + y[:, None] * nn[None, :]
    p /= np.linalg.norm(p, axis=1)[:, None]
    lon = np.mod(np.degrees(np.arctan2(p[:, 1], p[:, 0])), 360.0)
    lat = np.degrees(np.arcsin(np.clip(p[:, 2], -1.0, 1.0)))
    return lon, lat


def raster_scan(g: np.random.Generator, lon0: float, lat0: float, nrows: int,
                row_spacing: float, half_width: float, per_row: int,
                jitter: float, limit: int | None = None):
    """Jittered raster: rows of constant y, evenly spaced x, Gaussian jitter."""
    y = -0.5 * (nrows - 1) * row_spacing + np.arange(nrows) * row_spacing
    x = np.linspace(-half_width, half_width, per_row)
    X = np.tile(x, nrows)
    Y = np.repeat(y, per_row)
    if limit is not None:
        X, Y = X[:limit], Y[:limit]
    X = X + g.normal(0.0, jitter, X.shape[0])
    Y = Y + g.normal(0.0, jitter, Y.shape[0])
    return tangent_place(lon0, lat0, X, Y)


def _to_bf16_exact(t):
    import torch
    return t.to(torch.bfloat16).to(torch.float32)


# ---------------------------------------------------------------------------
# synthetic skies
# ---------------------------------------------------------------------------

def point_source_values(g: np.random.Generator, lon: np.ndarray, lat: np.ndarray,
                        nsrc: int, box: tuple, fwhm: float, amp: tuple,
                        noise: float) -> np.ndarray:
    """Gaussian point sources (flat-sky offsets around each source) + noise."""
    slon = g.uniform(box[0], box[1], nsrc)
    slat = g.uniform(box[2], box[3], nsrc)
    sa = g.uniform(amp[0], amp[1], nsrc)
    sig = fwhm * FWHM_TO_SIGMA
    v = np.zeros(lon.shape[0])
    for k in range(nsrc):
        dx = (np.mod(lon - slon[k] + 180.0, 360.0) - 180.0) * math.cos(math.radians(slat[k]))
        dy = lat - slat[k]
        v += sa[k] * np.exp(-(dx * dx + dy * dy) / (2.0 * sig * sig))
    return v + g.normal(0.0, noise, lon.shape[0])


def line_cube(g: np.random.Generator, lon: np.ndarray, lat: np.ndarray, nchan: int,
              centre: tuple, half_size: float, noise: float, device="cpu",
              seed: int = 0, out_dtype="f32", chunk: int = 1 << 16):
    """Spectral-line cube [N][nchan]: <=3 Gaussian lines per spectrum.

    Line amplitude, centre channel and FWHM (uniform 5..50 channels) vary
    smoothly with position: amplitudes are sums of 2D Gaussian "clouds" of
    scale 5'..60', centres follow a smooth velocity field.  Offsets are flat
    around ``centre`` (degrees), which is all a synthetic sky needs.
    """
    import torch

    dev = torch.device(device)
    ncl = 24
    cx = g.uniform(-half_size, half_size, (3, ncl))
    cy = g.uniform(-half_size, half_size, (3, ncl))
    cs = g.uniform(5.0, 60.0, (3, ncl)) * ARCMIN
    ca = g.uniform(0.2, 2.0, (3, ncl))
    vgrad = g.uniform(-1.0, 1.0, (3, 2))
    vphase = g.uniform(0.0, 2 * math.pi, (3, 2))
    wbase = g.uniform(5.0, 50.0, 3)
    cos0 = math.cos(math.radians(centre[1]))
    x = (np.mod(lon - centre[0] + 180.0, 360.0) - 180.0) * cos0
    y = lat - centre[1]
    n = lon.shape[0]
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16,
           "f64": torch.float64}[out_dtype]
    out = torch.empty((n, nchan), dtype=tdt, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed) * 7919 + 17)
    ch = torch.arange(nchan, dtype=torch.float32, device=dev)[None, :]
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        xs = x[s:e]
        ys = y[s:e]
        spec = torch.zeros((e - s, nchan), dtype=torch.float32, device=dev)
        for k in range(3):
            amp = np.zeros(e - s)
            for j in range(ncl):
                r2 = (xs - cx[k, j]) ** 2 + (ys - cy[k, j]) ** 2
                amp += ca[k, j] * np.exp(-r2 / (2.0 * cs[k, j] ** 2))
            u = xs / max(half_size, 1e-9)
            v = ys / max(half_size, 1e-9)
            c0 = 512.0 + 200.0 * np.sin(vgrad[k, 0] * 2.5 * u + vphase[k, 0]) \
                + 150.0 * np.cos(vgrad[k, 1] * 2.5 * v + vphase[k, 1]) + 60.0 * (k - 1)
            c0 = np.clip(c0 * (nchan / 1024.0), 0.1 * nchan, 0.9 * nchan)
            fw = np.clip(wbase[k] * (1.0 + 0.3 * np.sin(3.0 * u + k)), 5.0, 50.0) * min(1.0, nchan / 1024.0 * 4)
            fw = np.maximum(fw, 1.0)
            sg = fw * FWHM_TO_SIGMA
            a_t = torch.as_tensor(amp, dtype=torch.float32, device=dev)[:, None]
            c_t = torch.as_tensor(c0, dtype=torch.float32, device=dev)[:, None]
            s_t = torch.as_tensor(sg, dtype=torch.float32, device=dev)[:, None]
            spec += a_t * torch.exp(-((ch - c_t) ** 2) / (2.0 * s_t * s_t))
        spec += noise * torch.randn((e - s, nchan), generator=gen, device=dev,
                                    dtype=torch.float32)
        out[s:e] = spec.to(tdt)
    return out


def allsky_field(g: np.random.Generator, lon: np.ndarray, lat: np.ndarray, nchan: int,
                 nsrc: int, fwhm: float, device="cpu", chunk: int = 1 << 18):
    """All-sky [N][nchan] float32: smooth low-order field + point sources."""
    import torch

    dev = torch.device(device)
    a = np.radians(lon)
    s = np.sin(np.radians(lat))
    coef = g.normal(0.0, 1.0, (nchan, 6))
    base = np.stack([np.ones_like(a), np.cos(a), np.sin(a), s, s * s,
                     np.cos(2 * a) * (1 - s * s)], axis=1)
    out = torch.as_tensor(base @ coef.T, dtype=torch.float32, device=dev)
    slon, slat = uniform_sphere(g, nsrc)
    amp = g.uniform(1.0, 10.0, nsrc)
    sidx = g.uniform(-1.0, 1.0, nsrc)
    sig = math.radians(fwhm * FWHM_TO_SIGMA)
    # sources: flat evaluation via chord distance on unit vectors (synthetic sky only)
    sv = np.stack([np.cos(np.radians(slat)) * np.cos(np.radians(slon)),
                   np.cos(np.radians(slat)) * np.sin(np.radians(slon)),
                   np.sin(np.radians(slat))], axis=1)
    sv_t = torch.as_tensor(sv, dtype=torch.float32, device=dev)
    scale = torch.as_tensor(amp[:, None] * (np.arange(1, nchan + 1)[None, :] / nchan) ** sidx[:, None],
                            dtype=torch.float32, device=dev)      # [nsrc][nchan]
    cl = np.cos(np.radians(lat))
    pv = np.stack([cl * np.cos(a), cl * np.sin(a), np.sin(np.radians(lat))], axis=1)
    for st in range(0, lon.shape[0], chunk):
        e = min(lon.shape[0], st + chunk)
        p = torch.as_tensor(pv[st:e], dtype=torch.float32, device=dev)
        c2 = torch.clamp(2.0 - 2.0 * (p @ sv_t.T), min=0.0)           # chord^2 ~ d^2
        prof = torch.exp(-c2 / (2.0 * sig * sig))
        prof = torch.where(c2 < (5.0 * sig) ** 2, prof, torch.zeros_like(prof))
        out[st:e] += prof @ scale
    return out


# ---------------------------------------------------------------------------
# the benchmark workloads (C1..C5) and scaled-down variants for tests
# ---------------------------------------------------------------------------

def wcs_car(naxis1, naxis2, crpix1, crpix2, crval1, cdelt1, cdelt2, crval2=0.0):
    return {"proj": "CAR", "naxis1": int(naxis1), "naxis2": int(naxis2),
            "crpix1": float(crpix1), "crpix2": float(crpix2),
            "crval1": float(crval1), "crval2": float(crval2),
            "cdelt1": float(cdelt1), "cdelt2": float(cdelt2)}


def wcs_sin(naxis1, naxis2, crpix1, crpix2, crval1, crval2, cdelt1, cdelt2):
    return {"proj": "SIN", "naxis1": int(naxis1), "naxis2": int(naxis2),
            "crpix1": float(crpix1), "crpix2": float(crpix2),
            "crval1": float(crval1), "crval2": float(crval2),
            "cdelt1": float(cdelt1), "cdelt2": float(cdelt2)}


def config1() -> Workload:
    """Plain 2D map: 20,000 samples, 1 FP64 channel, 96x96 CAR at 2'."""
    g = rng(1)
    lon0, lon1 = 120.0 - 1.6, 120.0 + 1.6
    lat0, lat1 = 30.0 - 1.6, 30.0 + 1.6
    lon, lat = uniform_box(g, 20000, lon0, lon1, lat0, lat1)
    v = point_source_values(g, lon, lat, 10, (120 - 1.4, 120 + 1.4, 30 - 1.4, 30 + 1.4),
                            4.0 * ARCMIN, (1.0, 10.0), 0.1)
    wcs = wcs_car(96, 96, 48.5, -851.5, 120.0, -1.0 / 30.0, 1.0 / 30.0)
    return Workload("C1 plain map 20k x 96x96 CAR", lon, lat, v[:, None].astype(np.float64),
                    "f64", {"kind": "wcs", "wcs": wcs}, ("gauss1d", (1.5 * ARCMIN,)),
                    4.5 * ARCMIN, nside=4096)


def config2(scale: float = 1.0, nchan: int = 1024, device="cpu", dtype="f32") -> Workload:
    """Spectral cube: jittered raster (1' rows) over 10x10 deg, SIN 600x600 at 1'.

    ``scale`` < 1 shrinks the field linearly (same density, same kernel) for
    oracle-sized parity tests.
    """
    g = rng(2)
    side = 600.0 * scale                          # arcmin
    nrows = max(2, int(round(600 * scale)))
    per_row = max(2, int(round(1667 * scale)))
    limit = int(round(1_000_000 * scale * scale))
    lon, lat = raster_scan(g, 120.0, 30.0, nrows, 1.0 * ARCMIN, 0.5 * side * ARCMIN,
                           per_row, 0.2 * ARCMIN, limit=min(limit, nrows * per_row))
    data = line_cube(g, lon, lat, nchan, (120.0, 30.0), 0.5 * side * ARCMIN, 0.05,
                     device=device, seed=2, out_dtype=dtype)
    npx = max(2, int(round(600 * scale)))
    wcs = wcs_sin(npx, npx, 0.5 * (npx + 1), 0.5 * (npx + 1), 120.0, 30.0, -ARCMIN, ARCMIN)
    return Workload(f"C2 spectral cube {lon.shape[0]} x {npx}x{npx} SIN x {nchan}ch",
                    lon, lat, data, dtype, {"kind": "wcs", "wcs": wcs},
                    ("gauss1d", (1.5 * ARCMIN,)), 4.5 * ARCMIN,
                    hpx_maxres=0.75 * ARCMIN)


def config3(nsamples: int = 12_000_000, naxis1: int = 4320, nchan: int = 8,
            device="cpu") -> Workload:
    """All-sky map: uniform samples on the sphere, CAR over the whole sky.

    The full-size pixel is 5' (4320x2160); smaller ``naxis1`` keeps the
    kernel-to-pixel ratio and the sample density per kernel area by scaling
    sigma with the pixel.
    """
    g = rng(3)
    lon, lat = uniform_sphere(g, nsamples)
    data = allsky_field(g, lon, lat, nchan, 1000, 15.0 * ARCMIN * (4320 / naxis1), device=device)
    naxis2 = naxis1 // 2
    pix = 360.0 / naxis1
    wcs = wcs_car(naxis1, naxis2, 0.5 * naxis1 + 0.5, 0.5 * naxis2 + 0.5, 0.0, -pix, pix)
    sigma = 6.0 * ARCMIN * (4320 / naxis1)
    return Workload(f"C3 all-sky {nsamples} x {naxis1}x{naxis2} CAR x {nchan}ch",
                    lon, lat, data, "f32", {"kind": "wcs", "wcs": wcs},
                    ("gauss1d", (sigma,)), 3.0 * sigma,
                    nside=max(16, 1 << int(math.floor(math.log2(1024 * naxis1 / 4320)))))


def config4(njobs: int = 64, scale: float = 1.0, device="cpu") -> list[Workload]:
    """Batched uneven cubes: log-uniform sizes, 25 % elliptical kernels, BF16 data."""
    g = rng(4)
    jobs = []
    for j in range(njobs):
        n = int(round(math.exp(g.uniform(math.log(5e3), math.log(5e5))) * scale))
        side = int(round(math.exp(g.uniform(math.log(64), math.log(512))) * math.sqrt(scale)))
        side = max(side, 8)
        pix = g.uniform(0.5, 3.0) * ARCMIN
        nchan = int(round(math.exp(g.uniform(math.log(16), math.log(2048)))))
        sig = g.uniform(1.0, 4.0) * ARCMIN
        ell = g.uniform() < 0.25
        q = g.uniform(0.5, 1.0)
        pa = g.uniform(0.0, 180.0)
        clon = g.uniform(0.0, 360.0)
        clat = math.degrees(math.asin(g.uniform(-0.9, 0.9)))
        half = 0.5 * side * pix
        xs = g.uniform(-half, half, max(n, 1))
        ys = g.uniform(-half, half, max(n, 1))
        lon, lat = tangent_place(clon, clat, xs, ys)
        data = line_cube(g, lon, lat, nchan, (clon, clat), half, 0.05, device=device,
                         seed=400 + j, out_dtype="bf16")
        wcs = wcs_sin(side, side, 0.5 * (side + 1), 0.5 * (side + 1), clon, clat, -pix, pix)
        if ell:
            kern = ("gauss2d", (sig, q * sig, pa))
        else:
            kern = ("gauss1d", (sig,))
        jobs.append(Workload(f"C4 job {j}", lon, lat, data, "bf16",
                             {"kind": "wcs", "wcs": wcs}, kern, 3.0 * sig,
                             hpx_maxres=0.5 * q * sig if ell else 0.5 * sig))
    return jobs


def config_stripes(spacing: float, psf_fwhm: float = 0.1, field: float = 1.5,
                   nsrc: int = 3000, along: float = 0.05) -> Workload:
    """Scan-line sampling of App. A.2: a quasi-continuous field of ``nsrc``
    point sources (amplitudes U[0.1, 1]) seen through a Gaussian PSF of FWHM
    ``psf_fwhm`` deg, sampled densely (every ``along`` x PSF) along horizontal
    stripes ``spacing`` x PSF apart over a ``field`` x ``field`` deg map at
    (180, 0) deg; no noise.  Target: the field as a CAR grid at 0.1 x PSF.
    The same sources for every spacing; their list is in ``meta`` so that
    the smoothed sky can be evaluated analytically.  The kernel set here is
    a placeholder (the study varies it)."""
    g = rng(9)
    half = 0.5 * field
    margin = 3.0 * psf_fwhm
    src_lon = g.uniform(180.0 - half - margin, 180.0 + half + margin, nsrc)
    src_lat = g.uniform(-half - margin, half + margin, nsrc)
    src_amp = g.uniform(0.1, 1.0, nsrc)
    d = spacing * psf_fwhm
    lat_rows = np.arange(-half + 0.5 * d, half, d)
    lon_cols = np.arange(180.0 - half, 180.0 + half + 1e-9, along * psf_fwhm)
    lon = np.tile(lon_cols, lat_rows.size)
    lat = np.repeat(lat_rows, lon_cols.size)
    psf_sigma = psf_fwhm * FWHM_TO_SIGMA
    v = np.zeros(lon.shape[0])
    for k in range(nsrc):
        dx = (lon - src_lon[k]) * math.cos(math.radians(src_lat[k]))
        dy = lat - src_lat[k]
        v += src_amp[k] * np.exp(-(dx * dx + dy * dy) / (2.0 * psf_sigma * psf_sigma))
    pix = 0.1 * psf_fwhm
    n = int(round(field / pix)) + 1
    wcs = wcs_car(n, n, 0.5 * (n + 1), 0.5 * (n + 1), 180.0, -pix, pix)
    sig = 0.5 * psf_fwhm * FWHM_TO_SIGMA
    import torch
    return Workload(f"App.A.2 stripes {spacing:.1f} PSF apart: {lon.shape[0]} samples x {n}x{n} CAR",
                    lon, lat, torch.as_tensor(v[:, None].astype(np.float32)), "f32",
                    {"kind": "wcs", "wcs": wcs},
                    ("gauss1d", (sig,)), 5.0 * sig, hpx_maxres=0.5 * sig,
                    meta={"src_lon": src_lon, "src_lat": src_lat, "src_amp": src_amp,
                          "psf_sigma": psf_sigma, "psf_fwhm": psf_fwhm, "field": field})


def config_proj(proj: str, nchan: int = 2, device="cpu") -> Workload:
    """Small maps in the two extra projections: ZEA over the north polar cap
    (121x121 at 0.5 deg centred on the pole), SFL over the whole band
    |lat| < 30 deg (361x61 at 1 deg centred on lon 180, so that the corners
    fall outside the projection); area-uniform samples over a
    slightly larger region, smooth field + point sources, Gaussian kernel of
    one pixel sigma, support 3 sigma."""
    g = rng(7 if proj == "ZEA" else 8)
    if proj == "ZEA":
        lon, lat = uniform_box(g, 60000, 0.0, 360.0, 55.0, 90.0)
        wcs = wcs_sin(121, 121, 61.0, 61.0, 0.0, 90.0, -0.5, 0.5)
        sigma = 0.5
    else:
        lon, lat = uniform_box(g, 80000, 0.0, 360.0, -35.0, 35.0)
        wcs = wcs_car(361, 61, 181.0, 31.0, 180.0, -1.0, 1.0)
        sigma = 1.0
    wcs["proj"] = proj
    data = allsky_field(g, lon, lat, nchan, 200, 3.0 * sigma, device=device)
    return Workload(f"{proj} map {lon.shape[0]} x {wcs['naxis1']}x{wcs['naxis2']} x {nchan}ch",
                    lon, lat, data, "f32", {"kind": "wcs", "wcs": wcs},
                    ("gauss1d", (sigma,)), 3.0 * sigma, hpx_maxres=0.5 * sigma)


def config_oblique(proj: str, nchan: int = 2, device="cpu") -> Workload:
    """Oblique cylindrical maps, 121x81 at 0.5 deg: CAR centred at
    (250, +70) deg, whose rows reach the north celestial pole, and SFL
    centred at (40, -60) deg; area-uniform samples over the polar cap beyond
    |lat| = 30 deg on the map's side, smooth field + point sources, Gaussian
    kernel sigma 0.5 deg, support 1.5 deg."""
    g = rng(9 if proj == "CAR" else 10)
    if proj == "CAR":
        lon, lat = uniform_box(g, 90000, 0.0, 360.0, 30.0, 90.0)
        wcs = wcs_car(121, 81, 61.0, 41.0, 250.0, -0.5, 0.5)
        wcs["crval2"] = 70.0
    else:
        lon, lat = uniform_box(g, 90000, 0.0, 360.0, -90.0, -30.0)
        wcs = wcs_car(121, 81, 61.0, 41.0, 40.0, -0.5, 0.5)
        wcs["crval2"] = -60.0
    wcs["proj"] = proj
    sigma = 0.5
    data = allsky_field(g, lon, lat, nchan, 200, 3.0 * sigma, device=device)
    return Workload(f"oblique {proj} map {lon.shape[0]} x 121x81 x {nchan}ch",
                    lon, lat, data, "f32", {"kind": "wcs", "wcs": wcs},
                    ("gauss1d", (sigma,)), 3.0 * sigma, hpx_maxres=0.5 * sigma)


def config_max_channels(nchan: int = 65535, nsamples: int = 400) -> Workload:
    """The largest channel count of the API on a 9x3 SIN grid at 1' at
    (40, -20) deg: samples uniform over the grid plus a 5' margin, FP32 data
    1 + 0.1 N(0, 1) (a flat continuum with noise); sigma 1.5', support 4.5'."""
    g = rng(300)
    wcs = wcs_sin(9, 3, 5.0, 2.0, 40.0, -20.0, -ARCMIN, ARCMIN)
    lon = 40.0 + g.uniform(-0.5, 0.5, nsamples) * 19 * ARCMIN
    lat = -20.0 + g.uniform(-0.5, 0.5, nsamples) * 13 * ARCMIN
    import torch
    gen = torch.Generator()
    gen.manual_seed(300)
    data = 1.0 + 0.1 * torch.randn((nsamples, nchan), generator=gen, dtype=torch.float32)
    return Workload(f"max channels {nsamples} x 9x3 SIN x {nchan}ch", lon, lat, data, "f32",
                    {"kind": "wcs", "wcs": wcs}, ("gauss1d", (1.5 * ARCMIN,)), 4.5 * ARCMIN,
                    hpx_maxres=0.75 * ARCMIN)


def config_wide_support(nsamples: int = 3000) -> Workload:
    """A whole-sky 12x6 CAR grid of 30 deg pixels with a kernel of sigma
    20 deg and a 60 deg support (every disk takes whole rings and covers a
    pole); samples uniform on the sphere, two channels of unit Gaussian
    noise."""
    g = rng(301)
    lon, lat = uniform_sphere(g, nsamples)
    wcs = wcs_car(12, 6, 6.5, 3.5, 180.0, -30.0, 30.0)
    data = g.normal(size=(nsamples, 2))
    return Workload(f"wide support {nsamples} x 12x6 CAR", lon, lat, data, "f64",
                    {"kind": "wcs", "wcs": wcs}, ("gauss1d", (20.0,)), 60.0, hpx_maxres=10.0)


def config_tiny_grid(nx: int, ny: int, nsamples: int = 3000) -> Workload:
    """A SIN grid of nx x ny pixels at 1' (1x1 up to ragged sizes) at
    (40, -20) deg with uniform samples over the grid plus a 5' margin, two
    FP64 channels of unit Gaussian noise; kernel sigma 1.5', support 4.5'."""
    g = rng(200 + nx)
    wcs = wcs_sin(nx, ny, 0.5 * (nx + 1), 0.5 * (ny + 1), 40.0, -20.0, -ARCMIN, ARCMIN)
    lon = 40.0 + g.uniform(-0.5, 0.5, nsamples) * (nx + 10) * ARCMIN
    lat = -20.0 + g.uniform(-0.5, 0.5, nsamples) * (ny + 10) * ARCMIN
    data = g.normal(size=(nsamples, 2))
    return Workload(f"tiny {nx}x{ny} SIN grid", lon, lat, data, "f64", {"kind": "wcs", "wcs": wcs},
                    ("gauss1d", (1.5 * ARCMIN,)), 4.5 * ARCMIN, hpx_maxres=0.75 * ARCMIN)


def config_hpx_tiny(nside: int, order: str = "ring", nsamples: int = 5000) -> Workload:
    """A HEALPix map of 12 nside^2 pixels (nside 1, 2, 4: tiles straddling
    base faces) from area-uniform samples with a smooth channel and a noise
    channel (FP64); Gaussian kernel sigma 10 deg, support 25 deg."""
    g = rng(100 + nside)
    lon, lat = uniform_sphere(g, nsamples)
    data = np.stack([np.cos(np.radians(lat)) * np.sin(np.radians(lon)),
                     g.normal(0.0, 1.0, nsamples)], axis=1)
    return Workload(f"tiny HEALPix map nside {nside} ({order})", lon, lat, data, "f64",
                    {"kind": "healpix", "nside": int(nside), "order": order},
                    ("gauss1d", (10.0,)), 25.0, hpx_maxres=5.0)


def config_hpx(nside: int = 512, oversample: float = 15.0, nchan: int = 2,
               device="cpu") -> Workload:
    """HEALPix-map gridding of App. A.1: samples uniform on the sphere,
    ``oversample`` times as many as map pixels (15: ~47 M at nside 512);
    channel 0 is 1024 random point sources seen through a Gaussian PSF of
    FWHM 4 pixel sizes plus a smooth field, channel 1 unit Gaussian noise
    (the paper grids signal and noise); kernel FWHM = PSF / 2 (13.7' at
    nside 512), support 3 sigma, lookup resolution sigma / 2.  Targets: every
    pixel centre of the nside map in RING order.
    """
    g = rng(6)
    npix = 12 * nside * nside
    n = int(round(oversample * npix))
    lon, lat = uniform_sphere(g, n)
    theta_pix = math.degrees(math.sqrt(4.0 * math.pi / npix))    # 6.87' at nside 512
    fwhm_psf = 4.0 * theta_pix
    sig = allsky_field(g, lon, lat, 1, 1024, fwhm_psf, device=device)
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(1604_6667_06)
    noise = torch.randn((n, max(nchan - 1, 0)), generator=gen, device=device, dtype=torch.float32)
    data = torch.cat([sig, noise], dim=1) if nchan > 1 else sig
    sigma = 0.5 * fwhm_psf * FWHM_TO_SIGMA
    return Workload(f"App.A.1 HEALPix map {n} -> nside {nside} ({npix} pixels) x {nchan}ch",
                    lon, lat, data, "f32",
                    {"kind": "healpix", "nside": int(nside), "order": "ring"},
                    ("gauss1d", (sigma,)), 3.0 * sigma, hpx_maxres=0.5 * sigma)


def config5(nsamples: int = 10_000_000, ntargets: int = 2_000_000, box: float = 30.0,
            nchan: int = 256, device="cpu") -> Workload:
    """Sight lines: samples and targets area-uniform in a 30x30 deg box, gauss2d."""
    g = rng(5)
    lon0, lat0 = 105.0, 15.0
    lon, lat = uniform_box(g, nsamples, lon0, lon0 + box, lat0, lat0 + box)
    tlon, tlat = uniform_box(g, ntargets, lon0, lon0 + box, lat0, lat0 + box)
    data = line_cube(g, lon, lat, nchan, (lon0 + 0.5 * box, lat0 + 0.5 * box), 0.5 * box,
                     0.05, device=device, seed=5, out_dtype="bf16")
    return Workload(f"C5 sight lines {nsamples} x {ntargets} x {nchan}ch",
                    lon, lat, data, "bf16",
                    {"kind": "sightlines", "lon": tlon, "lat": tlat},
                    ("gauss2d", (3.0 * ARCMIN, 2.0 * ARCMIN, 30.0)), 9.0 * ARCMIN,
                    nside=4096)
