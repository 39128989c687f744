"""Glue for GPU tests: build library gridders from synth workloads and compare
them with the oracle."""
import math
import sys

import numpy as np

import oracle
import synth


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def header_of(wcs: dict, nchan: int) -> dict:
    p = wcs["proj"]
    return {"NAXIS": 3, "NAXIS1": wcs["naxis1"], "NAXIS2": wcs["naxis2"], "NAXIS3": nchan,
            "CTYPE1": "RA---" + p, "CTYPE2": "DEC--" + p,
            "CRPIX1": wcs["crpix1"], "CRPIX2": wcs["crpix2"],
            "CRVAL1": wcs["crval1"], "CRVAL2": wcs["crval2"],
            "CDELT1": wcs["cdelt1"], "CDELT2": wcs["cdelt2"]}


def torch_dtype(code):
    import torch
    return {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
            "f16": torch.float16}[code]


def to_device(wl: synth.Workload, dev="cuda:0"):
    import torch
    lon = torch.as_tensor(np.ascontiguousarray(wl.lon), dtype=torch.float64, device=dev)
    lat = torch.as_tensor(np.ascontiguousarray(wl.lat), dtype=torch.float64, device=dev)
    d = wl.data
    if isinstance(d, np.ndarray):
        d = torch.as_tensor(d)
    d = d.to(dev).to(torch_dtype(wl.dtype)).contiguous()
    return lon, lat, d


def make_gridder(wl: synth.Workload, prec="fp32", nside=None, dev="cuda:0"):
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
    if nside is not None:
        g.set_nside(nside)
    elif wl.nside is not None:
        g.set_nside(wl.nside)
    g.set_kernel(kind, params, wl.support, wl.hpx_maxres or (params[-1] if kind == "gauss1d" else params[1]) / 2)
    g.set_precision(prec)
    return g


def oracle_data(wl):
    """Data exactly as delivered to the GPU (BF16/FP16 upcasts are exact)."""
    import torch
    d = wl.data
    if isinstance(d, np.ndarray):
        return d.astype(np.float64)
    return d.detach().to("cpu").to(torch.float64).numpy()


def flat(cube, nchan):
    a = cube.detach().to("cpu").numpy().astype(np.float64)
    return a.reshape(nchan, -1)


def compare_neighbours(counts, hashes, ref):
    """Counts and hashes must match except for targets with edge-band pairs."""
    c = counts.detach().cpu().numpy().astype(np.int64)
    h = hashes.detach().cpu().numpy().view(np.uint64)
    band_t = set(int(t) for t in ref["band"][:, 0]) if ref["band"].size else set()
    ok = np.ones(c.shape[0], dtype=bool)
    for t in band_t:
        ok[t] = False
    bad = np.nonzero(ok & ((c != ref["count"]) | (h != ref["hash"])))[0]
    assert bad.size == 0, f"{bad.size} targets differ, first {bad[:5]}: gpu {c[bad[:5]]} oracle {ref['count'][bad[:5]]}"
    for t in band_t:
        nb = int((ref["band"][:, 0] == t).sum())
        assert abs(int(c[t]) - int(ref["count"][t])) <= nb
    return int(c.sum())
