"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

FP32 path bar: e_val <= 1e-6 and e_W <= 1e-6 (relative, see oracle.metrics);
neighbour sets: counts and order-independent hashes identical except for
samples within 1e-12 rad of the support edge.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import (say, make_gridder, to_device, oracle_data, flat, compare_neighbours,
                      header_of)

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ARC = 1.0 / 60.0
TOL32 = 1e-6


def _torch():
    import torch
    return torch


def _run_fp32(wl, nside=None, oneshot=False):
    g = make_gridder(wl, "fp32", nside=nside)
    lon, lat, d = to_device(wl)
    if oneshot:
        cube, w = g.grid_datacube(lon, lat, d)
        g.sync()
    else:
        g.grid(lon, lat, d)
        cube = g.get_datacube()
        w = g.get_weights()
    _torch().cuda.synchronize()
    return g, flat(cube, wl.nchan), w.cpu().numpy().astype(np.float64).ravel(), (lon, lat, d)


def _check_values(R, W, ref, tol=TOL32):
    ev = oracle.e_val(R, ref["R"], ref["W"])
    ew = oracle.e_weights(W, ref["W"])
    say(f"  e_val={ev:.3e} e_W={ew:.3e}")
    assert ev <= tol and ew <= tol
    return ev


# ------------------------------------------------------------ hand cases

def _hand_cases():
    with open(os.path.join(HERE, "golden", "hand_cases.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _hand_cases(), ids=lambda c: c["id"])
def test_hand_cases_gpu(case):
    torch = _torch()
    import paper_1604_06667_amd as cgp
    s = np.array(case["samples"], dtype=np.float64)
    t = np.array(case["targets"], dtype=np.float64)
    say(f"hand case {case['id']}")
    dev = "cuda:0"
    g = cgp.SlGrid(torch.tensor(t[:, 0], device=dev), torch.tensor(t[:, 1], device=dev), 1)
    g.set_kernel(case["kernel"][0], case["kernel"][1], case["support"], case["kernel"][1][0] / 2)
    g.grid(torch.tensor(s[:, 0], device=dev), torch.tensor(s[:, 1], device=dev),
           torch.tensor(s[:, 2:3], device=dev))
    R = g.get_datacube().cpu().numpy().ravel()
    W = g.get_weights().cpu().numpy().ravel()
    for got, exp in zip(R, case["expect_R"]):
        if exp is None:
            assert np.isnan(got)
        else:
            assert got == pytest.approx(exp, rel=TOL32)
    np.testing.assert_allclose(W, case["expect_W"], rtol=TOL32, atol=0)


# ------------------------------------------------------------ C1 full size

def test_config1_full_fp32():
    wl = synth.config1()
    say(f"C1 {wl.name}")
    ref = oracle.grid_workload(wl, method="kdtree")
    g, R, W, (lon, lat, d) = _run_fp32(wl)
    _check_values(R, W, ref)
    counts, hashes = g.neighbour_stats(lon, lat)
    ref_ns = oracle.neighbour_sets(wl.lon, wl.lat, *oracle.targets_of(wl), wl.support)
    compare_neighbours(counts, hashes, ref_ns)
    # one-shot entry point equals grid + get_datacube
    _, R1, W1, _ = _run_fp32(wl, oneshot=True)
    _check_values(R1, W1, ref)


# ------------------------------------------------- scaled-down configurations

def _c2_small(nchan, dtype="f32"):
    return synth.config2(scale=0.06, nchan=nchan, dtype=dtype)


@pytest.mark.parametrize("nchan", [1, 5, 16, 40, 100, 300])
def test_cube_sin_fp32(nchan):
    wl = _c2_small(nchan)
    say(f"C2-small nchan={nchan}: {wl.nsamples} samples, {wl.ntargets()} targets")
    ref = oracle.grid_workload(wl)
    g, R, W, (lon, lat, d) = _run_fp32(wl)
    _check_values(R, W, ref)


def test_cube_dtypes_fp32_path():
    torch = _torch()
    base = _c2_small(64)
    for dt in ("f64", "bf16", "f16"):
        wl = synth.Workload(base.name, base.lon, base.lat,
                            base.data.to(torch.float64) if dt == "f64" else base.data.to(
                                {"bf16": torch.bfloat16, "f16": torch.float16}[dt]),
                            dt, base.target, base.kernel, base.support, hpx_maxres=base.hpx_maxres)
        say(f"dtype {dt}")
        ref = oracle.grid_workload(wl)
        _, R, W, _ = _run_fp32(wl)
        _check_values(R, W, ref)


@pytest.mark.parametrize("nchan", [8, 70])
def test_allsky_poles_seam_fp32(nchan):
    wl = synth.config3(nsamples=120_000, naxis1=360, nchan=nchan)
    say(f"C3-small {wl.name}")
    ref = oracle.grid_workload(wl)
    g, R, W, (lon, lat, d) = _run_fp32(wl)
    _check_values(R, W, ref)
    counts, hashes = g.neighbour_stats(lon, lat)
    ref_ns = oracle.neighbour_sets(wl.lon, wl.lat, *oracle.targets_of(wl), wl.support)
    compare_neighbours(counts, hashes, ref_ns)


@pytest.mark.parametrize("nchan", [3, 48])
def test_sightlines_elliptical_fp32(nchan):
    wl = synth.config5(nsamples=60_000, ntargets=20_000, box=3.0, nchan=nchan)
    say(f"C5-small {wl.name}")
    ref = oracle.grid_workload(wl)
    g, R, W, (lon, lat, d) = _run_fp32(wl)
    _check_values(R, W, ref)
    counts, hashes = g.neighbour_stats(lon, lat)
    ref_ns = oracle.neighbour_sets(wl.lon, wl.lat, *oracle.targets_of(wl), wl.support)
    compare_neighbours(counts, hashes, ref_ns)


@pytest.mark.parametrize("proj", ["ZEA", "SFL"])
def test_extra_projections(proj):
    # the pixel centres of a ZEA map over the north pole and of an SFL band
    # (pixels outside SFL's outline stay empty), FP32 and BF16 paths
    wl = synth.config_proj(proj)
    say(wl.name)
    ref = oracle.grid_workload(wl)
    g, R, W, (lon, lat, d) = _run_fp32(wl)
    _check_values(R, W, ref)
    counts, hashes = g.neighbour_stats(lon, lat)
    ref_ns = oracle.neighbour_sets(wl.lon, wl.lat, *oracle.targets_of(wl), wl.support)
    compare_neighbours(counts, hashes, ref_ns)
    g.set_precision("bf16")
    cube, w = g.grid_datacube(lon, lat, d)
    g.sync()
    ev = oracle.e_val(flat(cube, wl.nchan), ref["R"], ref["W"])
    say(f"  bf16 e_val={ev:.2e}")
    assert ev <= 1e-4


@pytest.mark.parametrize("proj", ["CAR", "SFL"])
def test_oblique_projections(proj):
    # oblique cylindrical maps (CRVAL2 = +70 with rows through the north
    # celestial pole, and -60): the pixel centres come from the rotated
    # native frame; FP32 and BF16 paths, neighbour sets
    wl = synth.config_oblique(proj)
    say(wl.name)
    ref = oracle.grid_workload(wl)
    g, R, W, (lon, lat, d) = _run_fp32(wl)
    _check_values(R, W, ref)
    counts, hashes = g.neighbour_stats(lon, lat)
    ref_ns = oracle.neighbour_sets(wl.lon, wl.lat, *oracle.targets_of(wl), wl.support)
    compare_neighbours(counts, hashes, ref_ns)
    g.set_precision("bf16")
    cube, w = g.grid_datacube(lon, lat, d)
    g.sync()
    ev = oracle.e_val(flat(cube, wl.nchan), ref["R"], ref["W"])
    say(f"  bf16 e_val={ev:.2e}")
    assert ev <= 1e-4


def test_max_channels():
    # 65535 channels (the API's maximum): 64 channel passes with a ragged
    # last one, FP32 and BF16-split paths, one-shot and accumulate
    wl = synth.config_max_channels()
    say(wl.name)
    ref = oracle.grid_workload(wl)
    for prec, tol in (("fp32", TOL32), ("bf16", 1e-4)):
        g = make_gridder(wl, prec)
        lon, lat, d = to_device(wl)
        cube, w = g.grid_datacube(lon, lat, d)
        g.sync()
        _check_values(flat(cube, wl.nchan), w.cpu().numpy().astype(np.float64).ravel(), ref, tol)
        g.grid(lon, lat, d)
        _check_values(flat(g.get_datacube(), wl.nchan), g.get_weights().cpu().numpy().astype(np.float64).ravel(), ref, tol)


@pytest.mark.parametrize("lookup", ["tiles", "disk"])
def test_wide_support(lookup):
    # sigma 20 deg, support 60 deg on a whole-sky 30 deg grid: every lookup
    # window is a whole ring and every support disk holds a pole
    wl = synth.config_wide_support()
    say(f"{wl.name}, {lookup} lookup")
    ref = oracle.grid_workload(wl, method="brute")
    g = make_gridder(wl, "fp32")
    g.set_lookup(lookup)
    lon, lat, d = to_device(wl)
    g.grid(lon, lat, d)
    _check_values(flat(g.get_datacube(), wl.nchan), g.get_weights().cpu().numpy().astype(np.float64).ravel(), ref)
    counts, hashes = g.neighbour_stats(lon, lat)
    ref_ns = oracle.neighbour_sets(wl.lon, wl.lat, *oracle.targets_of(wl), wl.support)
    compare_neighbours(counts, hashes, ref_ns)


def _radial_kernels():
    dmax = 4.5 * ARC
    d = np.linspace(0.0, dmax, 64)
    prof = np.exp(-d ** 2 / (2 * (1.5 * ARC) ** 2)) * (1 - (d / dmax) ** 2)
    return [("tapered_sinc", (2.0 * ARC, 1.5 * ARC)),
            ("table", tuple([dmax] + list(prof))),
            ("table", (3.0 * ARC, 1.0, 0.0))]


@pytest.mark.parametrize("kidx", [0, 1, 2])
@pytest.mark.parametrize("nchan", [3, 40])
def test_radial_kernels_of_any_shape(kidx, nchan):
    # the tapered sinc (negative lobes) and tabulated profiles, FP32 paths
    # (narrow and wide) and, for the cube, the BF16 matrix-core path
    wl = synth.config2(scale=0.05, nchan=nchan)
    wl.kernel = _radial_kernels()[kidx]
    say(f"{wl.name} kernel={wl.kernel[0]} n={len(wl.kernel[1])}")
    ref = oracle.grid_workload(wl)
    g, R, W, (lon, lat, d) = _run_fp32(wl)
    m = np.abs(ref["W"]) > 1e-3 * np.abs(ref["W"]).max()   # the sinc's weights can cancel
    ev = oracle.e_val(R[:, m], ref["R"][:, m], ref["W"][m])
    ew = float(np.abs(W - ref["W"]).max() / np.abs(ref["W"]).max())
    say(f"  fp32 e_val={ev:.2e} e_W={ew:.2e}")
    assert ev <= TOL32 and ew <= TOL32
    if nchan >= 32:
        g.set_precision("bf16")
        cube, w = g.grid_datacube(lon, lat, d)
        g.sync()
        Rb = flat(cube, wl.nchan)
        ev = oracle.e_val(Rb[:, m], ref["R"][:, m], ref["W"][m])
        say(f"  bf16 e_val={ev:.2e}")
        assert ev <= 1e-4


def test_radial_kernels_rejected_in_batches():
    import paper_1604_06667_amd as cgp
    torch = _torch()
    wl = synth.config2(scale=0.03, nchan=64)
    wl.kernel = _radial_kernels()[0]
    g = make_gridder(wl, "bf16")
    with pytest.raises(cgp.CgError):
        cgp.Batch([g], torch.bfloat16)


# ------------------------------------------------------------ semantics

def test_nside_independence():
    wl = _c2_small(4)
    outs = []
    for ns in (64, 512, 8192):
        say(f"nside {ns}")
        g, R, W, (lon, lat, d) = _run_fp32(wl, nside=ns)
        c, h = g.neighbour_stats(lon, lat)
        outs.append((R, W, c.cpu().numpy(), h.cpu().numpy()))
    for R, W, c, h in outs[1:]:
        assert np.array_equal(c, outs[0][2]) and np.array_equal(h, outs[0][3])
        m = outs[0][1] > 0
        np.testing.assert_allclose(R[:, m], outs[0][0][:, m], rtol=1e-6, atol=1e-7)


def test_accumulate_chunks_clear_and_determinism():
    torch = _torch()
    wl = _c2_small(24)
    ref = oracle.grid_workload(wl)
    g = make_gridder(wl)
    lon, lat, d = to_device(wl)
    assert torch.isnan(g.get_datacube()).all()
    assert (g.get_weights() == 0).all()
    n = lon.shape[0]
    cuts = [0, n // 3, n // 3 + 1, n]
    for a, b in zip(cuts[:-1], cuts[1:]):
        g.grid(lon[a:b], lat[a:b], d[a:b])
    R = flat(g.get_datacube(), wl.nchan)
    W = g.get_weights().cpu().numpy().astype(np.float64).ravel()
    _check_values(R, W, ref)
    g.clear()
    assert torch.isnan(g.get_datacube()).all()
    g.grid(lon, lat, d)
    c1 = g.get_datacube().clone()
    g.clear()
    g.grid(lon, lat, d)
    c2 = g.get_datacube()
    assert torch.equal(torch.nan_to_num(c1, nan=-7.0), torch.nan_to_num(c2, nan=-7.0))


def test_empty_and_invalid_inputs():
    torch = _torch()
    import paper_1604_06667_amd as cgp
    wl = _c2_small(3)
    g = make_gridder(wl)
    e = torch.empty(0, dtype=torch.float64, device="cuda:0")
    g.grid(e, e, torch.empty((0, 3), device="cuda:0"))
    assert torch.isnan(g.get_datacube()).all()
    # far-away samples only: every target empty
    lon = torch.full((100,), 300.0, dtype=torch.float64, device="cuda:0")
    lat = torch.full((100,), -60.0, dtype=torch.float64, device="cuda:0")
    g.grid(lon, lat, torch.ones((100, 3), device="cuda:0"))
    assert torch.isnan(g.get_datacube()).all() and (g.get_weights() == 0).all()
    # invalid coordinates are skipped and reported by sync
    lon, lat, d = to_device(wl)
    lat_bad = lat.clone()
    lat_bad[::7] = 95.0
    lon_bad = lon.clone()
    lon_bad[3] = float("nan")
    g.clear()
    g.grid(lon_bad, lat_bad, d)
    with pytest.raises(cgp.CgError) as ei:
        g.sync()
    assert ei.value.status == -6
    g.sync()   # flag cleared
    keep = torch.ones(lon.shape[0], dtype=torch.bool)
    keep[::7] = False
    keep[3] = False
    sub = synth.Workload(wl.name, wl.lon[keep.numpy()], wl.lat[keep.numpy()],
                         wl.data[keep], wl.dtype, wl.target, wl.kernel, wl.support,
                         hpx_maxres=wl.hpx_maxres)
    ref = oracle.grid_workload(sub)
    R = flat(g.get_datacube(check_input=False), wl.nchan)
    W = g.get_weights().cpu().numpy().astype(np.float64).ravel()
    _check_values(R, W, ref)
    with pytest.raises(cgp.CgError):
        g2 = cgp.WcsGrid(header_of(wl.target["wcs"], 3))
        g2.grid(lon, lat, d)     # no kernel set


def test_tiny_and_ragged_grids():
    torch = _torch()
    for nx, ny in ((1, 1), (9, 3), (17, 65)):
        wl = synth.config_tiny_grid(nx, ny)
        say(f"grid {nx}x{ny}")
        ref = oracle.grid_workload(wl, method="brute")
        _, R, W, _ = _run_fp32(wl)
        _check_values(R, W, ref)
