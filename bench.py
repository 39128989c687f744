#!/usr/bin/env python3
"""Throughput of the gridding hot path on one MI355X.

One step = one pass of the whole path over the spectral-cube workload:
HEALPix indexing, radix sort, ring offsets, per-tile candidate lookup, the
contraction of Eq. (1)-(2) and the normalisation of Eq. (3), producing the
normalised cube and the weight map (``cg_grid_datacube``).  Inputs are
resident in device memory before the timed region starts.

Workload (spectral cube): 1,000,000 samples on a jittered raster scan (row
spacing 1', jitter 0.2') over 10x10 deg around (120, 30) deg, 1024 FP32
channels of Gaussian spectral lines plus noise, gridded onto a 600x600 SIN
grid at 1' with a Gaussian kernel sigma = 1.5', support 3 sigma.

Prints one JSON line.  ``value`` = sample-channel contributions per second =
(number of (target, sample) pairs with d <= support) x channels / time per step.
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
PEAK_FP32_VALU_TFLOPS = 78.6   # 256 CU x 64 lanes x 2 flop x 2.4 GHz, packed FP32 disabled
PEAK_BF16_TFLOPS = 2500.0


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


def cpu_baseline_and_error(wl, cube_by_prec, block):
    """Oracle (FP64, cKDTree candidates + Vincenty) on a central block of
    block x block targets with the samples that can reach them."""
    import oracle
    w = wl.target["wcs"]
    nx, ny = w["naxis1"], w["naxis2"]
    x0, y0 = (nx - block) // 2, (ny - block) // 2
    xs, ys = np.meshgrid(np.arange(x0, x0 + block), np.arange(y0, y0 + block))
    tidx = (ys * nx + xs).ravel()
    tlon, tlat = oracle.targets_of(wl)
    bl, bb = tlon[tidx], tlat[tidx]
    m = wl.support + 0.02
    clat = math.cos(math.radians(max(abs(bb.min()), abs(bb.max())) + m))
    sel = ((wl.lat >= bb.min() - m) & (wl.lat <= bb.max() + m) &
           (np.abs(((wl.lon - bl.mean() + 180) % 360) - 180) <= (bl.max() - bl.min()) / 2 + m / clat))
    sidx = np.nonzero(sel)[0]
    import torch
    data = wl.data[torch.as_tensor(sidx, device=wl.data.device)].to("cpu", torch.float64).numpy()
    t0 = time.perf_counter()
    ref = oracle.grid_kdtree(wl.lon[sidx], wl.lat[sidx], data, bl, bb, wl.kernel, wl.support)
    dt = time.perf_counter() - t0
    contrib = float(ref["count"].sum()) * wl.nchan
    errs = {}
    for prec, cube in cube_by_prec.items():
        R = cube.reshape(wl.nchan, -1)[:, torch.as_tensor(tidx, device=cube.device)]
        R = R.to("cpu", torch.float64).numpy()
        errs[prec] = oracle.e_val(R, ref["R"], ref["W"])
    return {"value": contrib / dt, "unit": "contributions/s", "cores": 1, "kind": "oracle",
            "sample": (f"central {block}x{block} targets of the 600x600 grid with the "
                       f"{sidx.size} samples that can reach them; FP64 NumPy/SciPy "
                       f"(cKDTree ball query + Vincenty), single thread, {dt:.1f} s"),
            "seconds": round(dt, 2)}, errs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="auto", choices=["auto", "fp32", "bf16", "fp16"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP32 comparison run")
    ap.add_argument("--cpu-block", type=int, default=384)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              f"(requested --gpus {a.gpus}); see DESIGN.md for how the path would shard.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_1604_06667_amd as cgp

    if a.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "launches": 3}))
        return

    dev = "cuda:0"
    t0 = time.time()
    wl = synth.config2(device=dev)
    lon = torch.as_tensor(wl.lon, dtype=torch.float64, device=dev)
    lat = torch.as_tensor(wl.lat, dtype=torch.float64, device=dev)
    data = wl.data
    torch.cuda.synchronize()
    log(f"workload built in {time.time() - t0:.1f}s: {wl.name}")

    g = cgp.WcsGrid(header_of(wl.target["wcs"], wl.nchan))
    g.set_kernel(*wl.kernel, wl.support, wl.hpx_maxres)
    counts, _ = g.neighbour_stats(lon, lat)
    pairs = int(counts.to(torch.int64).sum().item())
    contributions = pairs * wl.nchan
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

    # roofline of the contraction kernel
    in_bytes = wl.nsamples * (wl.nchan * data.element_size() + 24)
    out_bytes = ntarget * (wl.nchan * 4 + 4)
    alg_bytes = in_bytes + out_bytes
    if headline == "fp32":
        flops = 2.0 * contributions
        ach = flops / (kms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP32_VALU_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_VALU_TFLOPS, 4)}
    else:
        ach = alg_bytes / (kms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4)}
    roof["traffic"] = traffic_from_profiles(f"contraction_{headline}")
    roof["kernel_ms"] = round(kms, 4)
    roof["alg_bytes"] = alg_bytes

    cpu = None
    if not a.no_cpu:
        cpu, errs = cpu_baseline_and_error(wl, cubes, a.cpu_block)
        extra["e_val"] = {k: float(f"{v:.3e}") for k, v in errs.items()}
        log(f"cpu oracle: {cpu['value']:.3e} contributions/s; e_val {errs}")

    out = {
        "metric": METRIC,
        "value": contributions / (ms / 1e3),
        "unit": "contributions/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp16": "f16"}[headline],
        "data": "synthetic",
        "config": {"workload": ("spectral cube: 1,000,000 jittered-raster samples x 1024 FP32 "
                                "channels -> 600x600 SIN grid at 1', gauss1d sigma 1.5', "
                                "support 4.5'"),
                   "samples": wl.nsamples, "targets": ntarget, "channels": wl.nchan,
                   "nside": g.nside, "pairs": pairs, "contributions": contributions,
                   "contraction": headline},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
