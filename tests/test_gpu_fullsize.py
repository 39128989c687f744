"""GPU parity at the full benchmark sizes, in the launch configurations the
benchmark times, on sampled outputs the FP64 oracle computes one by one.

* spectral cube (1,000,000 x 1024 FP32 -> 600x600 SIN, nside 8192): BF16
  split and FP32 paths on blocks at the centre, a corner and an edge;
* all-sky (12,000,000 x 8 -> 4320x2160 CAR, nside 1024): FP32 path on blocks
  at both poles, across the 0/360 seam and at the +-180 deg grid edges;
* sight lines (10,000,000 x 256 BF16 -> 2,000,000 targets, target-major
  cube): BF16, FP16 and FP32 paths on the targets of a 0.8x0.8 deg box;
* HEALPix map (App. A.1: ~47 M samples x 2 -> the nside = 512 pixel
  centres): FP32 path at both poles and across the seam;
* batched (64 uneven jobs, tuned, replayed from the captured graph): every
  job on a central and an edge block, with neighbour counts;
* the sample-centric lookup (query disks shifted with Eq. 4-5) on the cube
  and the sight lines: neighbour counts and hashes identical to the tile
  lookup's at every target, and the BF16 path on the sampled blocks.

Bars: e_val <= 2e-3 (matrix-core), <= 1e-6 (FP32); neighbour counts equal
except for samples within 1e-12 rad of the support edge.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import say, make_gridder, to_device, flat

pytestmark = pytest.mark.gpu

TOL_MFMA, TOL32 = 2e-3, 1e-6


def _torch():
    import torch
    return torch


def _select_samples(wl, bl, bb, margin):
    """Indices of the samples that can reach targets (bl, bb) (degrees)."""
    lat_hi = min(90.0, bb.max() + margin)
    lat_lo = max(-90.0, bb.min() - margin)
    sel = (wl.lat >= lat_lo) & (wl.lat <= lat_hi)
    if lat_hi < 89.0 and lat_lo > -89.0:
        ref = math.degrees(math.atan2(np.sin(np.radians(bl)).mean(), np.cos(np.radians(bl)).mean()))
        dl = ((bl - ref + 180.0) % 360.0) - 180.0
        clat = math.cos(math.radians(max(abs(lat_lo), abs(lat_hi))))
        half = max(abs(dl.min()), abs(dl.max())) + margin / clat
        if half < 180.0:
            sel &= np.abs(((wl.lon - ref + 180.0) % 360.0) - 180.0) <= half
    return np.nonzero(sel)[0]


def _oracle_on(wl, tidx):
    torch = _torch()
    tlon, tlat = oracle.targets_of(wl)
    bl, bb = tlon[tidx], tlat[tidx]
    sidx = _select_samples(wl, bl, bb, wl.support + 0.05)
    d = wl.data[torch.as_tensor(sidx, device=wl.data.device)].to("cpu", torch.float64).numpy()
    ref = oracle.grid_kdtree(wl.lon[sidx], wl.lat[sidx], d, bl, bb, wl.kernel, wl.support)
    return ref, sidx


def _check_counts(wl, counts, tidx, ref, sidx):
    got = counts.detach().cpu().numpy().astype(np.int64)[tidx]
    bad = np.nonzero(got != ref["count"])[0]
    tlon, tlat = oracle.targets_of(wl)
    rs = math.radians(wl.support)
    for k in bad:
        t = tidx[k]
        d = oracle.vincenty(math.radians(tlon[t]), math.radians(tlat[t]),
                            np.radians(wl.lon[sidx]), np.radians(wl.lat[sidx]))
        nb = int((np.abs(d - rs) < 1e-12).sum())
        assert abs(int(got[k]) - int(ref["count"][k])) <= nb, f"target {t}: {got[k]} vs {ref['count'][k]}"
    say(f"  neighbour counts: {tidx.size} targets, {bad.size} differ only in the 1e-12 band")


def _blocks(nx, ny, starts, k):
    out = []
    for (y0, x0) in starts:
        y0 = min(max(y0, 0), ny - k)
        x0 = min(max(x0, 0), nx - k)
        xs, ys = np.meshgrid(np.arange(x0, x0 + k), np.arange(y0, y0 + k))
        out.append((ys * nx + xs).ravel())
    return np.unique(np.concatenate(out))


def _ev(cube_cn, wl, tidx, ref):
    R = cube_cn.reshape(wl.nchan, -1)[:, _torch().as_tensor(tidx, device=cube_cn.device)]
    return oracle.e_val(R.to("cpu", _torch().float64).numpy(), ref["R"], ref["W"])


def test_fullsize_cube():
    torch = _torch()
    wl = synth.config2(device="cuda:0")
    say(f"full-size {wl.name}")
    g = make_gridder(wl, "bf16")
    lon, lat, d = to_device(wl)
    counts, _ = g.neighbour_stats(lon, lat)
    tidx = _blocks(600, 600, [(276, 276), (0, 0), (0, 560), (580, 300)], 24)
    ref, sidx = _oracle_on(wl, tidx)
    _check_counts(wl, counts, tidx, ref, sidx)
    cube, w = g.grid_datacube(lon, lat, d)
    g.sync()
    ev = _ev(cube, wl, tidx, ref)
    ew = oracle.e_weights(w.reshape(-1)[torch.as_tensor(tidx, device=w.device)].cpu().numpy(), ref["W"])
    say(f"  bf16 e_val={ev:.2e} e_W={ew:.2e}")
    assert ev <= TOL_MFMA and ew <= TOL32
    g.set_precision("fp32")
    cube, w = g.grid_datacube(lon, lat, d, cube, w)
    g.sync()
    ev = _ev(cube, wl, tidx, ref)
    say(f"  fp32 e_val={ev:.2e}")
    assert ev <= TOL32


def test_fullsize_allsky():
    torch = _torch()
    wl = synth.config3(device="cuda:0")
    say(f"full-size {wl.name}")
    g = make_gridder(wl, "fp32")
    lon, lat, d = to_device(wl)
    counts, _ = g.neighbour_stats(lon, lat)
    nx, ny = 4320, 2160
    tidx = _blocks(nx, ny, [(0, 1000), (ny - 16, 3000), (ny // 2 - 8, nx // 2 - 8),
                            (700, 0), (1500, nx - 16)], 16)
    ref, sidx = _oracle_on(wl, tidx)
    _check_counts(wl, counts, tidx, ref, sidx)
    cube, w = g.grid_datacube(lon, lat, d)
    g.sync()
    ev = _ev(cube, wl, tidx, ref)
    ew = oracle.e_weights(w.reshape(-1)[torch.as_tensor(tidx, device=w.device)].cpu().numpy(), ref["W"])
    say(f"  fp32 e_val={ev:.2e} e_W={ew:.2e}")
    assert ev <= TOL32 and ew <= TOL32


def test_fullsize_sightlines():
    torch = _torch()
    wl = synth.config5(device="cuda:0")
    say(f"full-size {wl.name}")
    g = make_gridder(wl, "bf16")
    g.set_output_layout("target")
    lon, lat, d = to_device(wl)
    counts, _ = g.neighbour_stats(lon, lat)
    # the sight lines in a 0.8 x 0.8 deg box (about 1400 targets), so that the
    # oracle needs only the samples around it
    tl, tb = np.asarray(wl.target["lon"]), np.asarray(wl.target["lat"])
    tidx = np.nonzero((np.abs(tl - 112.0) < 0.4) & (np.abs(tb - 40.0) < 0.4))[0]
    ref, sidx = _oracle_on(wl, tidx)
    _check_counts(wl, counts, tidx, ref, sidx)
    cube = torch.empty((wl.ntargets(), wl.nchan), dtype=torch.float32, device="cuda:0")
    for prec, tol in (("bf16", TOL_MFMA), ("fp16", TOL_MFMA), ("fp32", TOL32)):
        g.set_precision(prec)
        cube, w = g.grid_datacube(lon, lat, d, cube)
        g.sync()
        ev = _ev(cube.t(), wl, tidx, ref)
        say(f"  {prec} e_val={ev:.2e}")
        assert ev <= tol


@pytest.mark.parametrize("name", ["cube", "sightlines"])
def test_fullsize_disk_lookup(name):
    torch = _torch()
    if name == "cube":
        wl = synth.config2(device="cuda:0")
        tidx = _blocks(600, 600, [(276, 276), (0, 0), (580, 300)], 24)
    else:
        wl = synth.config5(device="cuda:0")
        tl, tb = np.asarray(wl.target["lon"]), np.asarray(wl.target["lat"])
        tidx = np.nonzero((np.abs(tl - 125.0) < 0.3) & (np.abs(tb - 20.0) < 0.3))[0]
    say(f"full-size disk lookup {wl.name}")
    g = make_gridder(wl, "bf16")
    g.set_output_layout("channel" if name == "cube" else "target")
    lon, lat, d = to_device(wl)
    c_tiles, h_tiles = g.neighbour_stats(lon, lat)
    g.set_lookup("disk")
    c_disk, h_disk = g.neighbour_stats(lon, lat)
    assert torch.equal(c_tiles, c_disk) and torch.equal(h_tiles, h_disk)
    say(f"  neighbour sets equal at all {c_disk.numel()} targets; pixels, pairs = {g.disk_stats()}")
    ref, sidx = _oracle_on(wl, tidx)
    _check_counts(wl, c_disk, tidx, ref, sidx)
    cube, w = g.grid_datacube(lon, lat, d)
    g.sync()
    ev = _ev(cube if name == "cube" else cube.t(), wl, tidx, ref)
    ew = oracle.e_weights(w.reshape(-1)[torch.as_tensor(tidx, device=w.device)].cpu().numpy(), ref["W"])
    say(f"  bf16 e_val={ev:.2e} e_W={ew:.2e}")
    assert ev <= TOL_MFMA and ew <= TOL32


def test_fullsize_healpix_map():
    # App. A.1: ~47 M uniform samples onto the nside = 512 map (FP32 path), at
    # both poles and across the 0/360 seam on the equator
    torch = _torch()
    wl = synth.config_hpx(device="cuda:0")
    say(f"full-size {wl.name}")
    g = make_gridder(wl, "fp32")
    lon, lat, d = to_device(wl)
    counts, _ = g.neighbour_stats(lon, lat)
    tl, tb = oracle.targets_of(wl)
    seam = (np.abs(tb) < 0.5) & ((tl < 1.5) | (tl > 358.5))
    blocks = [np.nonzero(tb > 88.5)[0], np.nonzero(tb < -88.5)[0], np.nonzero(seam)[0]]
    cube, w = g.grid_datacube(lon, lat, d)
    g.sync()
    for tidx in blocks:
        ref, sidx = _oracle_on(wl, tidx)
        _check_counts(wl, counts, tidx, ref, sidx)
        ev = _ev(cube, wl, tidx, ref)
        ew = oracle.e_weights(w.reshape(-1)[torch.as_tensor(tidx, device=w.device)].cpu().numpy(),
                              ref["W"])
        say(f"  {tidx.size} pixels: fp32 e_val={ev:.2e} e_W={ew:.2e}")
        assert ev <= TOL32 and ew <= TOL32


def test_fullsize_batched_graph():
    """Every one of the 64 jobs, replayed from the captured graph after
    tuning: a central 16 x 16 block and a 16 x 16 block at the grid's edge
    against the oracle (e_val, e_W) and the neighbour counts of both blocks
    (from the job's own lookup) against the oracle's; the elliptical jobs
    are among them."""
    torch = _torch()
    import paper_1604_06667_amd as cgp
    wls = synth.config4(device="cuda:0")
    gs = [make_gridder(wl, "bf16") for wl in wls]
    ins = [to_device(wl) for wl in wls]
    b = cgp.Batch(gs, torch.bfloat16)
    outs = b.outputs()
    b.tune(ins, outs, reps=1)
    b.capture(ins, outs)
    for c, w in outs:
        c.fill_(-7.0)
        w.fill_(-7.0)
    b.replay()
    b.sync()
    nell = 0
    worst = (0.0, 0.0)
    for j, wl in enumerate(wls):
        nx, ny = wl.target["wcs"]["naxis1"], wl.target["wcs"]["naxis2"]
        k = min(16, nx, ny)
        tidx = _blocks(nx, ny, [(ny // 2 - k // 2, nx // 2 - k // 2), (ny - k, 0)], k)
        ref, sidx = _oracle_on(wl, tidx)
        counts, _ = gs[j].neighbour_stats(*ins[j][:2])
        _check_counts(wl, counts, tidx, ref, sidx)
        ev = _ev(outs[j][0], wl, tidx, ref)
        ew = oracle.e_weights(outs[j][1].reshape(-1)[torch.as_tensor(tidx, device="cuda:0")]
                              .cpu().numpy(), ref["W"])
        nell += wl.kernel[0] == "gauss2d"
        worst = (max(worst[0], ev), max(worst[1], ew))
        say(f"  job {j} (N={wl.nsamples}, C={wl.nchan}, {wl.kernel[0]}) e_val={ev:.2e} e_W={ew:.2e}")
        assert ev <= TOL_MFMA and ew <= TOL32
    say(f"  64 jobs ({nell} elliptical): worst e_val={worst[0]:.2e} e_W={worst[1]:.2e}")
    assert nell > 0
