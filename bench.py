#!/usr/bin/env python3
"""Throughput of the gridding hot path on one MI355X.

One step = one pass of the whole path over one workload: HEALPix indexing,
radix sort, ring offsets, per-tile candidate lookup, the contraction of
Eq. (1)-(2) and the normalisation of Eq. (3), producing the normalised cube
and the weight map.  Inputs are resident in device memory before the timed
region starts.

Workloads (``--workload``; all synthetic, seeded):

* ``all`` (default): ``cube`` as the headline line, with ``batched`` and
  ``sightlines`` as objects under ``workloads`` in the same line.
* ``cube``: 1,000,000 samples on a jittered raster scan (row
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
step.  Each workload's ``cpu_baseline`` is the FP64 oracle on forked worker
processes over a stated sample of its targets, which also yields ``e_val``
and ``e_W`` of every GPU result there.
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
PEAK_PACKED_FP32_TFLOPS = 157.3   # FP32 with packed instructions (not used by these builds)
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


# Sources that define each counted kernel (with the headers every kernel
# includes): a change elsewhere in the library leaves its counters valid.
COUNTED_SOURCES = {
    "contraction_bf16": ["cg_mfma.hip", "cg_mfma_tile.hpp"],
    "contraction_sightlines_bf16": ["cg_mfma.hip", "cg_mfma_tile.hpp"],
    "contraction_batched_bf16": ["cg_batch_mfma.hip", "cg_mfma_tile.hpp"],
}
COMMON_SOURCES = ["cg_internal.hpp", "healpix.hpp", "wcs.hpp"]


def kernel_source_sha(kernel_tag=None):
    """Hash of the sources of one counted kernel (of every .hip/.hpp source
    when the tag names none)."""
    src = os.path.join(HERE, "paper_1604_06667_amd", "csrc")
    if kernel_tag in COUNTED_SOURCES:
        files = sorted(COUNTED_SOURCES[kernel_tag] + COMMON_SOURCES)
    else:
        files = sorted(f for f in os.listdir(src) if f.endswith((".hip", ".hpp")))
    h = hashlib.sha256()
    for f in files:
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
        if e and e.get("source_sha") == kernel_source_sha(kernel_tag):
            return float(e["fetch_bytes"]) + float(e["write_bytes"])
    except Exception:
        return None
    return None


def roof_hbm(alg_bytes, kms, tag):
    ach = alg_bytes / (kms * 1e-3) / 1e9
    bw = copy_bandwidth()
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic_from_profiles(tag),
            "kernel_ms": round(kms, 4), "alg_bytes": int(alg_bytes),
            "copy_bw_measured": round(bw, 1), "frac_of_measured_copy_bw": round(ach / bw, 4)}


def roof_alu(flops, kms, tag):
    ach = flops / (kms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_VALU_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach / PEAK_VALU_TFLOPS, 4),
            "frac_of_packed_fp32_peak": round(ach / PEAK_PACKED_FP32_TFLOPS, 4),
            "traffic": traffic_from_profiles(tag), "kernel_ms": round(kms, 4),
            "alg_flops": float(flops)}


STEP_MS = {}   # per-step HIP-event times of the last timed loop, by label


def timed_steps(fn, steps, label):
    """Run fn() steps times between two host synchronisations; returns the
    mean wall time per step (ms) and records each step's HIP-event time
    (events on the current stream, which the library's calls use)."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    STEP_MS[label] = {"median": round(per[len(per) // 2], 4), "min": round(per[0], 4)}
    return (t1 - t0) * 1e3 / steps


def time_path(g, lon, lat, data, cube, weights, steps, warmup, label="step"):
    import torch
    for _ in range(warmup):
        g.grid_datacube(lon, lat, data, cube, weights)
    torch.cuda.synchronize()
    g.profile(True)
    ms = timed_steps(lambda: g.grid_datacube(lon, lat, data, cube, weights), steps, label)
    g.profile(False)
    nl, kms = g.profile_read()
    return ms, (kms / max(nl, 1)), nl


def time_graph(g, lon, lat, data, cube, weights, steps, warmup, label="graph"):
    """The same grid call with a caller workspace, captured into a HIP graph
    and replayed (no host work per step).  Every replay must give the eager
    call's cube bit for bit; returns ms per replayed step, or None (logged)
    if capture is not possible here."""
    import torch
    try:
        ws = g.workspace(lon.shape[0])
        g.grid_datacube(lon, lat, data, cube, weights, ws=ws)
        torch.cuda.synchronize()
        ref = cube.clone()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            g.grid_datacube(lon, lat, data, cube, weights, ws=ws)
            torch.cuda.synchronize()
            with torch.cuda.graph(graph, stream=s, capture_error_mode="thread_local"):
                g.grid_datacube(lon, lat, data, cube, weights, ws=ws)
        torch.cuda.synchronize()
        for _ in range(warmup):
            graph.replay()
        ms = timed_steps(graph.replay, steps, label)
        same = torch.equal(torch.nan_to_num(cube, nan=-1.0), torch.nan_to_num(ref, nan=-1.0))
        g.sync()
        if not same:
            log("graph replay differs from the eager call: not reported")
            return None
        return ms
    except Exception as e:  # capture unavailable: report the eager figure only
        log(f"graph capture skipped: {e}")
        return None


_COPY_BW = None


def copy_bandwidth():
    """Device copy bandwidth measured in this run: a 2 GiB buffer copied 10
    times; GB/s counts bytes read plus bytes written."""
    global _COPY_BW
    if _COPY_BW is None:
        import torch
        src = torch.ones(1 << 29, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        ms = timed_steps(lambda: dst.copy_(src), 10, "copy")
        _COPY_BW = 2.0 * src.numel() * 4 / (ms * 1e-3) / 1e9
        del src, dst
        torch.cuda.empty_cache()
    return _COPY_BW


# ------------------------------------------------------------ CPU baseline
#
# The oracle (FP64 NumPy/SciPy: cKDTree ball query, Vincenty distance, one
# sparse product per block of targets) runs unchanged in forked worker
# processes, one band of targets per task; each task also compares its band of
# every GPU cube with the oracle (block pieces of e_val), so whole cubes are
# checked without gathering the oracle's result in one process.

PAPER_CPU = {"value": 1.7e7, "unit": "contributions/s", "cores": 16,
             "note": ("Sect. 4, Example 1: 1e8 samples gridded in about 67 s on the authors' "
                      "16-core workstation; contributions derived with a 3-sigma support "
                      "(about 11.5 target pixels per sample); other workload, other machine")}

_ORACLE_JOBS = []


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_workers():
    """Worker processes for the oracle: the host's cores, at most 15 (one
    GPU's 16-core share, less the parent process that holds the GPU)."""
    n = os.cpu_count() or 1
    try:
        n = min(n, len(os.sched_getaffinity(0)))
    except AttributeError:
        pass
    return max(1, min(n, 15))


def samples_near(slon, slat, tlon, tlat, reach):
    """Indices of the samples inside a lon/lat box holding every point within
    ``reach`` degrees of the targets (the whole latitude band if the box nears
    a pole or would span the full circle)."""
    lat_hi = min(90.0, float(tlat.max()) + reach)
    lat_lo = max(-90.0, float(tlat.min()) - reach)
    clat = math.cos(math.radians(max(abs(lat_lo), abs(lat_hi))))
    rl = math.degrees(math.atan2(np.sin(np.radians(tlon)).mean(), np.cos(np.radians(tlon)).mean()))
    dl = ((tlon - rl + 180.0) % 360.0) - 180.0
    half = max(abs(dl.min()), abs(dl.max())) + reach / max(clat, 1e-6)
    sel = (slat >= lat_lo) & (slat <= lat_hi)
    if lat_hi < 89.9 and lat_lo > -89.9 and half < 180.0:
        sel &= np.abs(((slon - rl + 180.0) % 360.0) - 180.0) <= half
    return np.nonzero(sel)[0]


def oracle_job(wl, tidx, cubes, weights, tsort=None):
    """Host copies for one workload: the sampled targets (in band order), the
    samples that can reach them (data as FP32; the GPU inputs are FP32 or
    BF16, so this is exact), and each GPU cube's [C][T] values there."""
    import oracle
    import torch
    tlon, tlat = oracle.targets_of(wl)
    tidx = np.asarray(tidx, dtype=np.int64)
    ok = np.isfinite(tlon[tidx]) & np.isfinite(tlat[tidx])
    tidx = tidx[ok]
    if tsort is not None:
        tidx = tidx[np.argsort(tsort(tlon[tidx], tlat[tidx]), kind="stable")]
    bl, bb = tlon[tidx], tlat[tidx]
    sidx = samples_near(wl.lon, wl.lat, bl, bb, wl.support + 0.05)
    if isinstance(wl.data, np.ndarray):
        data = np.ascontiguousarray(wl.data[sidx], dtype=np.float32)
    else:
        data = wl.data[torch.as_tensor(sidx, device=wl.data.device)].to("cpu", torch.float32).numpy()
    ti = None
    hc, hw = {}, {}
    for prec, cube in cubes.items():
        if ti is None or ti.device != cube.device:
            ti = torch.as_tensor(tidx, device=cube.device)
        hc[prec] = cube.reshape(wl.nchan, -1)[:, ti].to("cpu", torch.float32).numpy()
        hw[prec] = weights[prec].reshape(-1)[ti].to("cpu", torch.float32).numpy()
    return {"lon": np.ascontiguousarray(wl.lon[sidx]), "lat": np.ascontiguousarray(wl.lat[sidx]),
            "data": data, "tlon": bl, "tlat": bb, "kernel": wl.kernel, "support": wl.support,
            "nchan": wl.nchan, "cubes": hc, "weights": hw}


def _oracle_task(task):
    import oracle
    wi, a, b = task
    J = _ORACLE_JOBS[wi]
    tl, tb = J["tlon"][a:b], J["tlat"][a:b]
    s = samples_near(J["lon"], J["lat"], tl, tb, J["support"] + 0.02)
    t0 = time.perf_counter()
    ref = oracle.grid_kdtree(J["lon"][s], J["lat"][s], J["data"][s].astype(np.float64), tl, tb,
                             J["kernel"], J["support"])
    dt = time.perf_counter() - t0
    out = {"pairs": int(ref["count"].sum()), "seconds": dt, "parts": {}, "e_W": {}, "err": None}
    for prec, cube in J["cubes"].items():
        try:
            out["parts"][prec] = oracle.e_val_parts(cube[:, a:b], ref["R"], ref["W"])
            out["e_W"][prec] = oracle.e_weights(J["weights"][prec][a:b], ref["W"])
        except AssertionError as e:
            out["err"] = f"{prec}: {e}"
    return wi, out


def cpu_baseline(jobs, desc, tasks_per_worker=3):
    """Time the oracle over the sampled targets of ``jobs`` (a list of
    ``oracle_job`` dicts) on a fork pool; returns the cpu_baseline object and
    e_val / e_W of each GPU cube (max over jobs; each job's channel norms are
    its own)."""
    import multiprocessing as mp
    import oracle
    global _ORACLE_JOBS
    _ORACLE_JOBS = jobs
    P = oracle_workers()
    work = [len(J["tlon"]) * J["nchan"] for J in jobs]
    ntask = P * tasks_per_worker
    tasks = []
    for wi, J in enumerate(jobs):
        T = len(J["tlon"])
        k = max(1, min(T, int(round(ntask * work[wi] / max(sum(work), 1)))))
        cuts = np.linspace(0, T, k + 1).astype(np.int64)
        tasks += [(wi, int(x), int(y)) for x, y in zip(cuts[:-1], cuts[1:]) if y > x]
    tasks.sort(key=lambda t: -(t[2] - t[1]) * jobs[t[0]]["nchan"])
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(P) as pool:
        res = list(pool.imap_unordered(_oracle_task, tasks, chunksize=1))
    wall = time.perf_counter() - t0
    pairs = [0] * len(jobs)
    parts = [dict() for _ in jobs]
    ew, errs = {}, []
    for wi, o in res:
        pairs[wi] += o["pairs"]
        for prec, pt in o["parts"].items():
            parts[wi].setdefault(prec, []).append(pt)
        for prec, v in o["e_W"].items():
            ew[prec] = max(ew.get(prec, 0.0), v)
        if o["err"]:
            errs.append(f"job {wi}: {o['err']}")
    contrib = float(sum(p * J["nchan"] for p, J in zip(pairs, jobs)))
    e_val = {}
    for wi in range(len(jobs)):
        for prec, pts in parts[wi].items():
            e_val[prec] = max(e_val.get(prec, 0.0), oracle.e_val_combine(pts))
    e_val = {p: float(f"{v:.3e}") for p, v in e_val.items()}
    ew = {p: float(f"{v:.3e}") for p, v in ew.items()}
    nt = sum(len(J["tlon"]) for J in jobs)
    worker_s = sum(o["seconds"] for _, o in res)
    cpu = {"value": contrib / wall, "unit": "contributions/s", "cores": P, "kind": "oracle",
           "sample": (f"{desc}: {nt} targets, {int(sum(pairs))} pairs, {len(tasks)} bands of "
                      f"targets on {P} forked workers; FP64 NumPy/SciPy (cKDTree ball query + "
                      f"Vincenty + sparse product), {wall:.1f} s wall, {worker_s:.1f} s in the "
                      f"oracle summed over workers"),
           "seconds": round(wall, 2), "model": cpu_model(), "cpu_count": os.cpu_count(),
           "paper": PAPER_CPU}
    _ORACLE_JOBS = []
    log(f"cpu oracle: {cpu['value']:.3e} contributions/s in {wall:.1f}s on {P} workers; "
        f"e_val {e_val} e_W {ew}")
    if errs:
        log("oracle comparison failures: " + "; ".join(errs[:8]))
    return cpu, {"e_val": e_val, "e_W": ew, **({"mask_errors": errs[:8]} if errs else {})}


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


def base_line(a, wl_desc, value, ms, dtype, config, roof, cpu, step_label="step"):
    import torch
    if LOOKUP != "tiles":
        config = dict(config, lookup=LOOKUP)
    return {"metric": METRIC, "value": value, "unit": "contributions/s",
            "step_ms_events": STEP_MS.get(step_label), "rocm": torch.version.hip,
            "clocks": "default (not pinned)",
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
    ms, kms, nl = time_path(g, lon, lat, data, cube, weights, a.steps, a.warmup, label="cube")
    log(f"{headline}: {ms:.3f} ms/step, contraction kernel {kms:.3f} ms x {nl}")
    cubes, wmaps = {headline: cube.clone()}, {headline: weights.clone()}
    extra = {}
    gms = time_graph(g, lon, lat, data, cube, weights, a.steps, a.warmup, label="cube_graph")
    if gms is not None:
        log(f"{headline} graph replay: {gms:.3f} ms/step")
        extra["graph"] = {"value": contributions / (gms / 1e3), "ms_per_step": round(gms, 4),
                          "how": "the same call with a caller workspace, captured in a HIP graph and replayed"}
    if headline != "fp32" and not a.no_compare:
        g.set_precision("fp32")
        ms32, kms32, _ = time_path(g, lon, lat, data, cube, weights, max(2, a.steps // 2), 1,
                                   label="cube_fp32")
        cubes["fp32"], wmaps["fp32"] = cube.clone(), weights.clone()
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
        b = a.cpu_block if 0 < a.cpu_block < 600 else 600
        x0 = (600 - b) // 2
        xs, ys = np.meshgrid(np.arange(x0, x0 + b), np.arange(x0, x0 + b))
        what = "every target of the 600x600 grid" if b == 600 else f"central {b}x{b} targets"
        job = oracle_job(wl, (ys * 600 + xs).ravel(), cubes, wmaps)
        del cubes, wmaps
        cpu, errs = cpu_baseline([job], what)
        del job
        extra.update(errs)
    out = base_line(a, ("spectral cube: 1,000,000 jittered-raster samples x 1024 FP32 channels "
                        "-> 600x600 SIN grid at 1', gauss1d sigma 1.5', support 4.5'"),
                    contributions / (ms / 1e3), ms, DT[headline],
                    {"samples": wl.nsamples, "targets": ntarget, "channels": wl.nchan,
                     "nside": g.nside, "pairs": pairs, "contributions": contributions,
                     "contraction": headline}, roof, cpu, step_label="cube")
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
    gms = time_graph(g, lon, lat, data, cube, weights, a.steps, a.warmup)
    if gms is not None:
        log(f"fp32 graph replay: {gms:.4f} ms/step")
    roof = roof_alu(2.0 * contributions + FLOPS_PER_PAIR * pairs, kms, "contraction_map_fp32")
    roof["alg_bytes"] = int(wl.nsamples * (wl.nchan * 8 + 16) + nx * ny * (wl.nchan * 4 + 4))
    cpu, extra = None, {}
    if not a.no_cpu:
        cpu, errs = cpu_baseline([oracle_job(wl, np.arange(nx * ny), {"fp32": cube},
                                             {"fp32": weights})], f"all {nx}x{ny} targets")
        extra.update(errs)
    out = base_line(a, ("plain map: 20,000 samples x 1 FP64 channel -> 96x96 CAR at 2', "
                        "gauss1d sigma 1.5', support 4.5', nside 4096"),
                    contributions / (ms / 1e3), ms, "f32",
                    {"samples": wl.nsamples, "targets": nx * ny, "channels": wl.nchan,
                     "nside": g.nside, "pairs": pairs, "contributions": contributions,
                     "contraction": "fp32"}, roof, cpu)
    out.update(extra)
    if gms is not None:
        out["graph"] = {"value": contributions / (gms / 1e3), "ms_per_step": round(gms, 4),
                        "how": "the same call with a caller workspace, captured in a HIP graph and replayed"}
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
        cpu, errs = cpu_baseline([oracle_job(wl, np.arange(nx * ny), {"fp32": cube},
                                             {"fp32": weights})],
                                 f"all {nx}x{ny} targets (both poles, the 0/360 seam)")
        extra.update(errs)
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
        cpu, errs = cpu_baseline([oracle_job(wl, tidx, {"fp32": cube}, {"fp32": weights})],
                                 "the map pixels with 0 < lat < 40 and 170 < lon < 230 deg")
        extra.update(errs)
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
    res, cubes, wmaps = {}, {}, {}
    for prec in ["bf16", "fp16", "fp32"]:
        if prec == "fp32" and a.no_compare:
            continue
        g.set_precision(prec)
        st = a.steps if prec != "fp32" else max(2, a.steps // 2)
        ms, kms, nl = time_path(g, lon, lat, data, cube, weights, st, 1 if prec == "fp32" else a.warmup,
                                label="sightlines_" + prec)
        res[prec] = (ms, kms)
        cubes[prec] = cube.t().contiguous()
        wmaps[prec] = weights.clone()
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
        # the sight lines in a 10 x 10 deg box at the field centre (1/9 of them),
        # in latitude bands
        tl, tb = np.asarray(wl.target["lon"]), np.asarray(wl.target["lat"])
        sel = np.nonzero((np.abs(tl - 120.0) < 5.0) & (np.abs(tb - 30.0) < 5.0))[0]
        job = oracle_job(wl, sel, cubes, wmaps, tsort=lambda l, b: b)
        del cubes, wmaps
        cpu, errs = cpu_baseline([job], "the sight lines in a 10x10 deg box at (120, 30)")
        del job
        extra.update(errs)
    out = base_line(a, ("sight lines: 10,000,000 samples x 256 BF16 channels over 30x30 deg -> "
                        "2,000,000 targets, gauss2d 3'x2' PA 30, support 9', nside 4096"),
                    contributions / (ms / 1e3), ms, "bf16",
                    {"samples": wl.nsamples, "targets": nt, "channels": wl.nchan,
                     "nside": g.nside, "pairs": pairs, "contributions": contributions,
                     "contraction": "bf16", "layout": "target-major [T][C]"}, roof, cpu,
                    step_label="sightlines_bf16")
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
    ms = timed_steps(b.replay, a.steps, "batched")
    b.sync()
    log(f"batched: eager {ms_eager:.3f} ms/step (contraction {kms:.3f} ms), graph {ms:.3f} ms/step")
    roof = roof_hbm(alg_bytes, kms, "contraction_batched_bf16")
    extra = {"eager": {"value": contributions / (ms_eager / 1e3), "ms_per_step": round(ms_eager, 4)},
             "tuned": {"rows_per_workgroup": b.query(5), "half_items": b.query(6),
                       "workgroups_per_cu": b.query(7), "shape": b.query(9), "items": b.query(3)}}
    # the same 64 jobs through 64 separate FP32 gridders, one eager call each
    outs32 = []
    if not a.no_compare:
        g32 = []
        for wl in wls:
            g = make_gridder(wl, dev)
            g.set_precision("fp32")
            g32.append(g)
            nx, ny = wl.target["wcs"]["naxis1"], wl.target["wcs"]["naxis2"]
            outs32.append((torch.empty((wl.nchan, ny, nx), dtype=torch.float32, device=dev),
                           torch.empty((ny, nx), dtype=torch.float32, device=dev)))

        def pass32():
            for g, (lon, lat, d), (c, w) in zip(g32, ins, outs32):
                g.grid_datacube(lon, lat, d, c, w)

        pass32()
        torch.cuda.synchronize()
        for g in g32:
            g.profile(True)
        st32 = max(2, a.steps // 2)
        t1 = time.perf_counter()
        for _ in range(st32):
            pass32()
        torch.cuda.synchronize()
        ms32 = (time.perf_counter() - t1) * 1e3 / st32
        k32 = sum(g.profile_read()[1] for g in g32) / st32
        for g in g32:
            g.profile(False)
        log(f"batched fp32 (64 gridders): {ms32:.3f} ms/pass, contraction kernels {k32:.3f} ms")
        extra["fp32_path"] = {"value": contributions / (ms32 / 1e3), "ms_per_step": round(ms32, 4),
                              "kernel_ms": round(k32, 4),
                              "how": "64 separate FP32 gridders, one eager call per job"}
        extra["speedup_vs_fp32"] = round(ms32 / ms, 3)
    cpu = None
    if not a.no_cpu:
        # every job: its central band of rows (a quarter of the grid, full
        # width, so both side edges are in)
        jobs = []
        for j, wl in enumerate(wls):
            nx, ny = wl.target["wcs"]["naxis1"], wl.target["wcs"]["naxis2"]
            y0, y1 = (3 * ny) // 8, max((5 * ny) // 8, (3 * ny) // 8 + 1)
            tidx = np.arange(y0 * nx, y1 * nx)
            cubes = {"bf16": outs[j][0]}
            wmaps = {"bf16": outs[j][1]}
            if outs32:
                cubes["fp32"], wmaps["fp32"] = outs32[j]
            jobs.append(oracle_job(wl, tidx, cubes, wmaps))
        cpu, errs = cpu_baseline(jobs, "all 64 jobs, the central quarter of each grid's rows")
        del jobs
        extra.update(errs)
    out = base_line(a, ("batched: 64 jobs, 5k-500k samples, 64^2-512^2 SIN grids, 16-2048 BF16 "
                        "channels, 25% elliptical; one lookup pass + one persistent launch, "
                        "graph replay"),
                    contributions / (ms / 1e3), ms, "bf16",
                    {"jobs": len(wls), "samples": int(sum(w.nsamples for w in wls)),
                     "targets": int(sum(w.ntargets() for w in wls)), "pairs": pairs,
                     "contributions": contributions, "contraction": "bf16"}, roof, cpu,
                    step_label="batched")
    out.update(extra)
    return out


COMMON_KEYS = ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data")


def run_all(a, dev):
    """The cube line, with the batched jobs and the sight lines as objects of
    it (each with its own value, roofline, cpu_baseline and e_val)."""
    import torch
    out = run_cube(a, dev)
    subs = {}
    for name, fn in (("batched", run_batched), ("sightlines", run_sightlines)):
        _GRIDDERS.clear()
        torch.cuda.empty_cache()
        sub = fn(a, dev)
        subs[name] = {k: v for k, v in sub.items() if k not in COMMON_KEYS}
    _GRIDDERS.clear()
    out["workloads"] = subs
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="all",
                    choices=["all", "cube", "allsky", "batched", "sightlines", "healpix", "map"],
                    help="'all' (default): the cube as the headline line, with the batched "
                         "jobs and the sight lines as objects of the same line")
    ap.add_argument("--prec", default="auto", choices=["auto", "fp32", "bf16", "fp16"],
                    help="contraction of the cube workload")
    ap.add_argument("--lookup", default="tiles", choices=["tiles", "disk"],
                    help="candidate lookup: per tile of targets, or the sample-centric "
                         "query disks shifted along rings (Sect. 3.3)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP32 comparison run")
    ap.add_argument("--cpu-block", type=int, default=0,
                    help="cube workload: oracle on the central NxN targets (0: all of them)")
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
    if a.lookup != "tiles" and a.workload in ("batched", "all"):
        print("batches always use the tile lookup", file=sys.stderr)
        sys.exit(2)
    dev = "cuda:0"
    if a.workload == "all":
        out = run_all(a, dev)
        print(json.dumps(out), flush=True)
        return
    run = {"cube": run_cube, "allsky": run_allsky, "batched": run_batched,
           "sightlines": run_sightlines, "healpix": run_healpix, "map": run_map}[a.workload]
    out = run(a, dev)
    if LOOKUP == "disk" and _GRIDDERS:
        npix, npairs = _GRIDDERS[-1].disk_stats()
        out["disk_lookup"] = {"sample_pixels": npix, "tile_pixel_pairs": npairs}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
