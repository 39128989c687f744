#!/usr/bin/env python3
"""Throughput of the gridding hot path on one MI355X.

One step = one pass of the whole path over one workload: HEALPix indexing,
radix sort, ring offsets, per-tile candidate lookup, the contraction of
Eq. (1)-(2) and the normalisation of Eq. (3), producing the normalised cube
and the weight map.  Inputs are resident in device memory before the timed
region starts.

Workloads (``--workload``; all synthetic, seeded):

* ``cube`` (default): 1,000,000 samples on a jittered raster scan (row
  spacing 1', jitter 0.2') over 10x10 deg around (120, 30) deg, 1024 FP32
  channels of Gaussian spectral lines plus noise, onto a 600x600 SIN grid at
  1'; Gaussian kernel sigma 1.5', support 3 sigma.  BF16 matrix-core
  contraction, with the FP32 gather path timed beside it.
* ``allsky``: 12,000,000 samples uniform on the sphere, 8 FP32 channels, onto
  a 4320x2160 CAR grid at 5' (both poles, the 0/360 seam); sigma 6',
  support 18', nside 1024; FP32 path.
* ``batched``: 64 independent jobs of uneven size (5k-500k samples, grids
  64^2-512^2 at 0.5'-3', 16-2048 BF16 channels, 25 % elliptical kernels) in
  one batch: one lookup pass and one persistent matrix-core launch, tuned,
  and replayed from a HIP graph.
* ``sightlines``: 10,000,000 samples x 256 BF16 channels over 30x30 deg onto
  2,000,000 arbitrary target positions, elliptical Gaussian 3'x2' PA 30 deg,
  support 9', nside 4096; BF16, FP16 and FP32 contractions.
* ``healpix``: the paper's App. A.1 simulation: ~47 M samples uniform on the
  sphere (15 per map pixel), point sources through a 27.5' PSF plus noise
  (2 FP32 channels), onto every pixel centre of the nside = 512 HEALPix map;
  kernel FWHM 13.7', support 3 sigma; FP32 path.

Prints one JSON line.  ``value`` = sample-channel contributions per second =
(number of (target, sample) pairs with d <= support) x channels / time per
step.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = ("gridded sample-channel contributions/sec on 1 GPU, BF16-MFMA vs FP32 at "
          "≤2e-3 rel")
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TFLOPS = 78.6   # FP32 (packed FP32 disabled) and FP64: 256 CU x 64 lanes x 2 x 2.4 GHz
PEAK_BF16_TFLOPS = 2500.0
FLOPS_PER_PAIR = 12       # FP64 chord^2, support test, distance series per in-support pair


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def header_of(wcs, nchan):
    p = wcs["proj"]
    return {"NAXIS": 3, "NAXIS1": wcs["naxis1"], "NAXIS2": wcs["naxis2"], "NAXIS3": nchan,
            "CTYPE1": "RA---" + p, "CTYPE2": "DEC--" + p, "CRPIX1": wcs["crpix1"],
            "CRPIX2": wcs["crpix2"], "CRVAL1": wcs["crval1"], "CRVAL2": wcs["crval2"],
            "CDELT1": wcs["cdelt1"], "CDELT2": wcs["cdelt2"]}


def kernel_source_sha():
    src = os.path.join(HERE, "paper_1604_06667_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(src)):
        if f.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(src, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources."""
    p = os.path.join(HERE, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get(kernel_tag)
        if e and e.get("source_sha") == kernel_source_sha():
            return float(e["fetch_bytes"]) + float(e["write_bytes"])
    except Exception:
        return None
    return None


def roof_hbm(alg_bytes, kms, tag):
    ach = alg_bytes / (kms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic_from_profiles(tag),
            "kernel_ms": round(kms, 4), "alg_bytes": int(alg_bytes)}


def roof_alu(flops, kms, tag):
    ach = flops / (kms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_VALU_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach / PEAK_VALU_TFLOPS, 4),
            "traffic": traffic_from_profiles(tag), "kernel_ms": round(kms, 4),
            "alg_flops": float(flops)}


def time_path(g, lon, lat, data, cube, weights, steps, warmup):
    import torch
    for _ in range(warmup):
        g.grid_datacube(lon, lat, data, cube, weights)
    torch.cuda.synchronize()
    g.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        g.grid_datacube(lon, lat, data, cube, weights)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.profile(False)
    nl, kms = g.profile_read()
    return (t1 - t0) * 1e3 / steps, (kms / max(nl, 1)), nl


def oracle_sample(wl, tidx, margin_deg):
    """Samples that can reach the targets tidx (a compact region), and the
    oracle's result for those targets; returns (result, seconds, nsamples)."""
    import oracle
    import torch
    tlon, tlat = oracle.targets_of(wl)
    bl, bb = tlon[tidx], tlat[tidx]
    ok = np.isfinite(bl) & np.isfinite(bb)
    bl, bb, tidx = bl[ok], bb[ok], tidx[ok]
    m = wl.support + margin_deg
    lat_hi = min(90.0, bb.max() + m)
    lat_lo = max(-90.0, bb.min() - m)
    clat = math.cos(math.radians(max(abs(lat_lo), abs(lat_hi))))
    ref_lon = math.degrees(math.atan2(np.sin(np.radians(bl)).mean(), np.cos(np.radians(bl)).mean()))
    dl = ((bl - ref_lon + 180.0) % 360.0) - 180.0
    half = max(abs(dl.min()), abs(dl.max())) + m / max(clat, 1e-6)
    sl = ((wl.lon - ref_lon + 180.0) % 360.0) - 180.0
    sel = (wl.lat >= lat_lo) & (wl.lat <= lat_hi)
    if lat_hi < 89.9 and lat_lo > -89.9 and half < 180.0:
        sel &= np.abs(sl) <= half
    sidx = np.nonzero(sel)[0]
    if isinstance(wl.data, np.ndarray):
        data = wl.data[sidx].astype(np.float64)
    else:
        data = wl.data[torch.as_tensor(sidx, device=wl.data.device)].to("cpu", torch.float64).numpy()
    t0 = time.perf_counter()
    ref = oracle.grid_kdtree(wl.lon[sidx], wl.lat[sidx], data, bl, bb, wl.kernel, wl.support)
    dt = time.perf_counter() - t0
    return ref, tidx, dt, sidx.size


def cpu_baseline(wl, tidx, desc, cubes, margin_deg=0.02):
    """Oracle (FP64, cKDTree candidates + Vincenty, one thread) on a bounded
    sample of the workload's targets; also the e_val of each GPU cube there."""
    import oracle
    import torch
    ref, tidx, dt, ns = oracle_sample(wl, tidx, margin_deg)
    contrib = float(ref["count"].sum()) * wl.nchan
    errs = {}
    for prec, cube in cubes.items():
        R = cube.reshape(wl.nchan, -1)[:, torch.as_tensor(tidx, device=cube.device)]
        errs[prec] = float(f"{oracle.e_val(R.to('cpu', torch.float64).numpy(), ref['R'], ref['W']):.3e}")
    cpu = {"value": contrib / dt, "unit": "contributions/s", "cores": 1, "kind": "oracle",
           "sample": (f"{desc}: {tidx.size} targets with the {ns} samples that can reach "
                      f"them; FP64 NumPy/SciPy (cKDTree ball query + Vincenty), single "
                      f"thread, {dt:.1f} s"),
           "seconds": round(dt, 2)}
    log(f"cpu oracle: {cpu['value']:.3e} contributions/s in {dt:.1f}s; e_val {errs}")
    return cpu, errs


def device_inputs(wl, dev):
    import torch
    lon = torch.as_tensor(wl.lon, dtype=torch.float64, device=dev)
    lat = torch.as_tensor(wl.lat, dtype=torch.float64, device=dev)
    data = wl.data if wl.data.device.type == "cuda" else wl.data.to(dev)
    if wl.dtype == "bf16":
        data = data.to(torch.bfloat16)
    return lon, lat, data.contiguous()


LOOKUP = "tiles"      # --lookup: 'tiles' or the sample-centric 'disk' lookup
_GRIDDERS = []


def make_gridder(wl, dev):
    import torch
    import paper_1604_06667_amd as cgp
    if wl.target["kind"] == "wcs":
        g = cgp.WcsGrid(header_of(wl.target["wcs"], wl.nchan))
    elif wl.target["kind"] == "healpix":
        g = cgp.HpxGrid(wl.target["nside"], wl.target.get("order", "ring"), wl.nchan)
    else:
        tl = torch.as_tensor(np.asarray(wl.target["lon"], dtype=np.float64), device=dev)
        tb = torch.as_tensor(np.asarray(wl.target["lat"], dtype=np.float64), device=dev)
        g = cgp.SlGrid(tl, tb, wl.nchan)
    kind, params = wl.kernel
    if wl.nside is not None:
        g.set_nside(wl.nside)
    res = wl.hpx_maxres or (0.5 * (params[0] if kind == "gauss1d" else params[1]))
    g.set_kernel(kind, params, wl.support, res)
    g.set_lookup(LOOKUP)
    _GRIDDERS.append(g)
    return g


def count_contributions(g, lon, lat, nchan):
    import torch
    counts, _ = g.neighbour_stats(lon, lat)
    pairs = int(counts.to(torch.int64).sum().item())
    return pairs, pairs * nchan


def base_line(a, wl_desc, value, ms, dtype, config, roof, cpu):
    if LOOKUP != "tiles":
        config = dict(config, lookup=LOOKUP)
    return {"metric": METRIC, "value": value, "unit": "contributions/s",
            "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic",
            "config": dict({"workload": wl_desc}, **config),
            "roofline": roof, "cpu_baseline": cpu}


DT = {"fp32": "f32", "bf16": "bf16", "fp16": "f16"}


# ------------------------------------------------------------------ workloads

def run_cube(a, dev):
    import torch
    import synth
    import paper_1604_06667_amd as cgp
    t0 = time.time()
    wl = synth.config2(device=dev)
    lon, lat, data = device_inputs(wl, dev)
    torch.cuda.synchronize()
    log(f"workload built in {time.time() - t0:.1f}s: {wl.name}")
    g = make_gridder(wl, dev)
    pairs, contributions = count_contributions(g, lon, lat, wl.nchan)
    ntarget = wl.ntargets()
    headline = a.prec
    if headline == "auto":
        try:
            g.set_precision("bf16")
            headline = "bf16"
        except cgp.CgError:
            headline = "fp32"
    g.set_precision(headline)
    cube = torch.empty((wl.nchan, 600, 600), dtype=torch.float32, device=dev)
    weights = torch.empty((600, 600), dtype=torch.float32, device=dev)
    ms, kms, nl = time_path(g, lon, lat, data, cube, weights, a.steps, a.warmup)
    log(f"{headline}: {ms:.3f} ms/step, contraction kernel {kms:.3f} ms x {nl}")
    cubes = {headline: cube.clone()}
    extra = {}
    if headline != "fp32" and not a.no_compare:
        g.set_precision("fp32")
        ms32, kms32, _ = time_path(g, lon, lat, data, cube, weights, max(2, a.steps // 2), 1)
        cubes["fp32"] = cube.clone()
        extra["fp32_path"] = {"value": contributions / (ms32 / 1e3), "ms_per_step": round(ms32, 4),
                              "kernel_ms": round(kms32, 4)}
        extra["speedup_vs_fp32"] = round(ms32 / ms, 3)
        log(f"fp32: {ms32:.3f} ms/step, kernel {kms32:.3f} ms")
    alg_bytes = wl.nsamples * (wl.nchan * data.element_size() + 16) + ntarget * (wl.nchan * 4 + 4)
    if headline == "fp32":
        roof = roof_alu(2.0 * contributions + FLOPS_PER_PAIR * pairs, kms, "contraction_fp32")
    else:
        roof = roof_hbm(alg_bytes, kms, f"contraction_{headline}")
    cpu = None
    if not a.no_cpu:
        b = a.cpu_block
        x0 = (600 - b) // 2
        xs, ys = np.meshgrid(np.arange(x0, x0 + b), np.arange(x0, x0 + b))
        cpu, errs = cpu_baseline(wl, (ys * 600 + xs).ravel(),
                                 f"central {b}x{b} targets of the 600x600 grid", cubes)
        extra["e_val"] = errs
    out = base_line(a, ("spectral cube: 1,000,000 jittered-raster samples x 1024 FP32 channels "
                        "-> 600x600 SIN grid at 1', gauss1d sigma 1.5', support 4.5'"),
                    contributions / (ms / 1e3), ms, DT[headline],
                    {"samples": wl.nsamples, "targets": ntarget, "channels": wl.nchan,
                     "nside": g.nside, "pairs": pairs, "contributions": contributions,
                     "contraction": headline}, roof, cpu)
    out.update(extra)
    return out


def run_map(a, dev):
    """The plain map (20,000 samples x 1 FP64 channel onto 96x96 CAR): launch-
    and latency-bound, so its absolute step time is the figure of interest."""
    import torch
    import synth
    wl = synth.config1()
    lon = torch.as_tensor(wl.lon, dtype=torch.float64, device=dev)
    lat = torch.as_tensor(wl.lat, dtype=torch.float64, device=dev)
    data = torch.as_tensor(wl.data, dtype=torch.float64, device=dev).contiguous()
    log(f"workload: {wl.name}")
    g = make_gridder(wl, dev)
    g.set_precision("fp32")
    pairs, contributions = count_contributions(g, lon, lat, wl.nchan)
    nx, ny = wl.target["wcs"]["naxis1"], wl.target["wcs"]["naxis2"]
    cube = torch.empty((wl.nchan, ny, nx), dtype=torch.float32, device=dev)
    weights = torch.empty((ny, nx), dtype=torch.float32, device=dev)
    ms, kms, nl = time_path(g, lon, lat, data, cube, weights, a.steps, a.warmup)
    log(f"fp32: {ms:.4f} ms/step, contraction kernel {kms:.4f} ms x {nl}")
    roof = roof_alu(2.0 * contributions + FLOPS_PER_PAIR * pairs, kms, "contraction_map_fp32")
    roof["alg_bytes"] = int(wl.nsamples * (wl.nchan * 8 + 16) + nx * ny * (wl.nchan * 4 + 4))
    cpu, extra = None, {}
    if not a.no_cpu:
        cpu, errs = cpu_baseline(wl, np.arange(nx * ny), f"all {nx}x{ny} targets", {"fp32": cube})
        extra["e_val"] = errs
    out = base_line(a, ("plain map: 20,000 samples x 1 FP64 channel -> 96x96 CAR at 2', "
                        "gauss1d sigma 1.5', support 4.5', nside 4096"),
                    contributions / (ms / 1e3), ms, "f32",
                    {"samples": wl.nsamples, "targets": nx * ny, "channels": wl.nchan,
                     "nside": g.nside, "pairs": pairs, "contributions": contributions,
                     "contraction": "fp32"}, roof, cpu)
    out.update(extra)
    return out


def run_allsky(a, dev):
    import torch
    import synth
    t0 = time.time()
    wl = synth.config3(device=dev)
    lon, lat, data = device_inputs(wl, dev)
    torch.cuda.synchronize()
    log(f"workload built in {time.time() - t0:.1f}s: {wl.name}")
    g = make_gridder(wl, dev)
    g.set_precision("fp32")
    pairs, contributions = count_contributions(g, lon, lat, wl.nchan)
    nx, ny = wl.target["wcs"]["naxis1"], wl.target["wcs"]["naxis2"]
    cube = torch.empty((wl.nchan, ny, nx), dtype=torch.float32, device=dev)
    weights = torch.empty((ny, nx), dtype=torch.float32, device=dev)
    ms, kms, nl = time_path(g, lon, lat, data, cube, weights, a.steps, a.warmup)
    log(f"fp32: {ms:.3f} ms/step, contraction kernel {kms:.3f} ms x {nl}")
    roof = roof_alu(2.0 * contributions + FLOPS_PER_PAIR * pairs, kms, "contraction_allsky_fp32")
    roof["alg_bytes"] = int(wl.nsamples * (wl.nchan * 4 + 16) + nx * ny * (wl.nchan * 4 + 4))
    cpu, extra = None, {}
    if not a.no_cpu:
        # a block of targets across the 0/360 seam on the equator
        k = 768
        y0, x0 = ny // 2 - k // 2, nx // 2 - k // 2
        xs, ys = np.meshgrid(np.arange(x0, x0 + k), np.arange(y0, y0 + k))
        cpu, errs = cpu_baseline(wl, (ys * nx + xs).ravel(),
                                 f"{k}x{k} targets across the 0/360 seam on the equator",
                                 {"fp32": cube})
        extra["e_val"] = errs
    out = base_line(a, ("all-sky map: 12,000,000 uniform samples x 8 FP32 channels -> 4320x2160 "
                        "CAR at 5', gauss1d sigma 6', support 18', nside 1024"),
                    contributions / (ms / 1e3), ms, "f32",
                    {"samples": wl.nsamples, "targets": nx * ny, "channels": wl.nchan,
                     "nside": g.nside, "pairs": pairs, "contributions": contributions,
                     "contraction": "fp32"}, roof, cpu)
    out.update(extra)
    return out


def run_healpix(a, dev):
    import torch
    import synth
    t0 = time.time()
    wl = synth.config_hpx(device=dev)
    lon, lat, data = device_inputs(wl, dev)
    torch.cuda.synchronize()
    log(f"workload built in {time.time() - t0:.1f}s: {wl.name}")
    g = make_gridder(wl, dev)
    g.set_precision("fp32")
    pairs, contributions = count_contributions(g, lon, lat, wl.nchan)
    nt = wl.ntargets()
    cube = torch.empty((wl.nchan, nt), dtype=torch.float32, device=dev)
    weights = torch.empty((nt,), dtype=torch.float32, device=dev)
    ms, kms, nl = time_path(g, lon, lat, data, cube, weights, a.steps, a.warmup)
    log(f"fp32: {ms:.3f} ms/step, contraction kernel {kms:.3f} ms x {nl}")
    roof = roof_alu(2.0 * contributions + FLOPS_PER_PAIR * pairs, kms, "contraction_healpix_fp32")
    roof["alg_bytes"] = int(wl.nsamples * (wl.nchan * 4 + 16) + nt * (wl.nchan * 4 + 4))
    cpu, extra = None, {}
    if not a.no_cpu:
        import oracle
        tl, tb = oracle.targets_of(wl)
        tidx = np.nonzero((tb > 0.0) & (tb < 40.0) & (tl > 170.0) & (tl < 230.0))[0]
        cpu, errs = cpu_baseline(wl, tidx, "the map pixels with 0 < lat < 40 and 170 < lon < 230 deg",
                                 {"fp32": cube})
        extra["e_val"] = errs
    nside = wl.target["nside"]
    out = base_line(a, (f"HEALPix map (App. A.1): {wl.nsamples:,} uniform samples x {wl.nchan} "
                        f"FP32 channels (point sources + noise) -> the {nt:,} pixel centres of "
                        f"nside {nside} (RING), gauss1d FWHM 13.7', support 3 sigma"),
                    contributions / (ms / 1e3), ms, "f32",
                    {"samples": wl.nsamples, "targets": nt, "channels": wl.nchan,
                     "nside": g.nside, "map_nside": nside, "pairs": pairs,
                     "contributions": contributions, "contraction": "fp32"}, roof, cpu)
    out.update(extra)
    return out


def run_sightlines(a, dev):
    import torch
    import synth
    t0 = time.time()
    wl = synth.config5(device=dev)
    lon, lat, data = device_inputs(wl, dev)
    torch.cuda.synchronize()
    log(f"workload built in {time.time() - t0:.1f}s: {wl.name}")
    g = make_gridder(wl, dev)
    g.set_precision("bf16")
    pairs, contributions = count_contributions(g, lon, lat, wl.nchan)
    nt = wl.ntargets()
    weights = torch.empty((nt,), dtype=torch.float32, device=dev)
    # one spectrum per sight line contiguous ([T][C]); the channel-major
    # ([C][T]) cube is timed beside it for BF16
    g.set_output_layout("target")
    cube = torch.empty((nt, wl.nchan), dtype=torch.float32, device=dev)
    res, cubes = {}, {}
    for prec in ["bf16", "fp16", "fp32"]:
        if prec == "fp32" and a.no_compare:
            continue
        g.set_precision(prec)
        st = a.steps if prec != "fp32" else max(2, a.steps // 2)
        ms, kms, nl = time_path(g, lon, lat, data, cube, weights, st, 1 if prec == "fp32" else a.warmup)
        res[prec] = (ms, kms)
        cubes[prec] = cube.t().contiguous()
        log(f"{prec}: {ms:.3f} ms/step, contraction kernel {kms:.3f} ms x {nl}")
    g.set_precision("bf16")
    g.set_output_layout("channel")
    cube_c = torch.empty((wl.nchan, nt), dtype=torch.float32, device=dev)
    ms_c, kms_c, _ = time_path(g, lon, lat, data, cube_c, weights, a.steps, a.warmup)
    log(f"bf16 channel-major cube: {ms_c:.3f} ms/step, contraction kernel {kms_c:.3f} ms")
    del cube_c
    ms, kms = res["bf16"]
    alg_bytes = (wl.nsamples * (wl.nchan * data.element_size() + 16) + nt * 16 +
                 nt * (wl.nchan * 4 + 4))
    roof = roof_hbm(alg_bytes, kms, "contraction_sightlines_bf16")
    extra = {"paths": {p: {"value": contributions / (m / 1e3), "ms_per_step": round(m, 4),
                           "kernel_ms": round(k, 4)} for p, (m, k) in res.items()}}
    extra["bf16_channel_major"] = {"value": contributions / (ms_c / 1e3),
                                   "ms_per_step": round(ms_c, 4), "kernel_ms": round(kms_c, 4)}
    if "fp32" in res:
        extra["speedup_vs_fp32"] = round(res["fp32"][0] / ms, 3)
    cpu = None
    if not a.no_cpu:
        # targets in a 3.6 x 3.6 deg box at the field centre
        tl, tb = np.asarray(wl.target["lon"]), np.asarray(wl.target["lat"])
        sel = np.nonzero((np.abs(tl - 120.0) < 1.8) & (np.abs(tb - 30.0) < 1.8))[0]
        cpu, errs = cpu_baseline(wl, sel, "sight lines in a 3.6x3.6 deg box at (120, 30)", cubes)
        extra["e_val"] = errs
    out = base_line(a, ("sight lines: 10,000,000 samples x 256 BF16 channels over 30x30 deg -> "
                        "2,000,000 targets, gauss2d 3'x2' PA 30, support 9', nside 4096"),
                    contributions / (ms / 1e3), ms, "bf16",
                    {"samples": wl.nsamples, "targets": nt, "channels": wl.nchan,
                     "nside": g.nside, "pairs": pairs, "contributions": contributions,
                     "contraction": "bf16", "layout": "target-major [T][C]"}, roof, cpu)
    out.update(extra)
    return out


def run_batched(a, dev):
    import torch
    import synth
    import paper_1604_06667_amd as cgp
    t0 = time.time()
    wls = synth.config4(device=dev)
    ins = [device_inputs(wl, dev) for wl in wls]
    torch.cuda.synchronize()
    log(f"workload built in {time.time() - t0:.1f}s: {len(wls)} jobs, "
        f"{sum(w.nsamples for w in wls)} samples")
    gs = []
    pairs = contributions = 0
    alg_bytes = 0
    for wl, (lon, lat, d) in zip(wls, ins):
        g = make_gridder(wl, dev)
        g.set_precision("bf16")
        p, c = count_contributions(g, lon, lat, wl.nchan)
        pairs += p
        contributions += c
        alg_bytes += wl.nsamples * (wl.nchan * 2 + 16) + wl.ntargets() * (wl.nchan * 4 + 4)
        gs.append(g)
    b = cgp.Batch(gs, torch.bfloat16)
    outs = b.outputs()
    t0 = time.time()
    b.tune(ins, outs, reps=2)
    log(f"tuned in {time.time() - t0:.1f}s: rows/workgroup={b.query(5)} half={b.query(6)} "
        f"wg/CU={b.query(7)} items={b.query(3)}")
    # eager passes (one host synchronisation each)
    for _ in range(a.warmup):
        b.grid(ins, outs)
    torch.cuda.synchronize()
    b.profile(True)
    t1 = time.perf_counter()
    for _ in range(a.steps):
        b.grid(ins, outs)
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t1) * 1e3 / a.steps
    nl, ktot = b.profile_read()
    kms = ktot / max(nl, 1)
    b.profile(False)
    # graph replays (no host synchronisation)
    b.capture(ins, outs)
    for _ in range(a.warmup):
        b.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(a.steps):
        b.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1e3 / a.steps
    b.sync()
    log(f"batched: eager {ms_eager:.3f} ms/step (contraction {kms:.3f} ms), graph {ms:.3f} ms/step")
    roof = roof_hbm(alg_bytes, kms, "contraction_batched_bf16")
    extra = {"eager": {"value": contributions / (ms_eager / 1e3), "ms_per_step": round(ms_eager, 4)},
             "tuned": {"rows_per_workgroup": b.query(5), "half_items": b.query(6),
                       "workgroups_per_cu": b.query(7), "shape": b.query(9), "items": b.query(3)}}
    cpu = None
    if not a.no_cpu:
        # the largest job's central 64x64 targets
        j = int(np.argmax([wl.nsamples for wl in wls]))
        wl = wls[j]
        nx = wl.target["wcs"]["naxis1"]
        ny = wl.target["wcs"]["naxis2"]
        k = min(64, nx, ny)
        x0, y0 = (nx - k) // 2, (ny - k) // 2
        xs, ys = np.meshgrid(np.arange(x0, x0 + k), np.arange(y0, y0 + k))
        cpu, errs = cpu_baseline(wl, (ys * nx + xs).ravel(),
                                 f"job {j} (the largest): central {k}x{k} targets",
                                 {"bf16": outs[j][0]})
        extra["e_val"] = errs
    out = base_line(a, ("batched: 64 jobs, 5k-500k samples, 64^2-512^2 SIN grids, 16-2048 BF16 "
                        "channels, 25% elliptical; one lookup pass + one persistent launch, "
                        "graph replay"),
                    contributions / (ms / 1e3), ms, "bf16",
                    {"jobs": len(wls), "samples": int(sum(w.nsamples for w in wls)),
                     "targets": int(sum(w.ntargets() for w in wls)), "pairs": pairs,
                     "contributions": contributions, "contraction": "bf16"}, roof, cpu)
    out.update(extra)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cube",
                    choices=["cube", "allsky", "batched", "sightlines", "healpix", "map"])
    ap.add_argument("--prec", default="auto", choices=["auto", "fp32", "bf16", "fp16"],
                    help="contraction of the cube workload")
    ap.add_argument("--lookup", default="tiles", choices=["tiles", "disk"],
                    help="candidate lookup: per tile of targets, or the sample-centric "
                         "query disks shifted along rings (Sect. 3.3)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP32 comparison run")
    ap.add_argument("--cpu-block", type=int, default=384)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              f"(requested --gpus {a.gpus}); the path would shard by target tiles or "
              "channel blocks with no reduction.", file=sys.stderr)
        sys.exit(2)

    import torch

    if a.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "launches": 3}))
        return

    global LOOKUP
    LOOKUP = a.lookup
    if a.lookup != "tiles" and a.workload == "batched":
        print("batches always use the tile lookup", file=sys.stderr)
        sys.exit(2)
    dev = "cuda:0"
    run = {"cube": run_cube, "allsky": run_allsky, "batched": run_batched,
           "sightlines": run_sightlines, "healpix": run_healpix, "map": run_map}[a.workload]
    out = run(a, dev)
    if LOOKUP == "disk" and _GRIDDERS:
        npix, npairs = _GRIDDERS[-1].disk_stats()
        out["disk_lookup"] = {"sample_pixels": npix, "tile_pixel_pairs": npairs}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
