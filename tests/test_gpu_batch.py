"""GPU parity of batched gridding (many uneven jobs in one lookup pass and one
persistent contraction launch).

Each job of a batch must produce what the same gridder produces alone with
cg_grid_datacube (same candidates in the same order and the same tile
contraction, so the two agree to FP32 rounding), and both stay within the
matrix-core bar (e_val <= 2e-3) of the FP64 oracle.  Graph replays are
checked against the eager result on every replay, with eager work and
synchronisations between them.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import say, make_gridder, to_device, flat

pytestmark = pytest.mark.gpu

TOL_MFMA = 2e-3


def _torch():
    import torch
    return torch


def _jobs(njobs=8, scale=0.02, seed_cut=None):
    wls = synth.config4(njobs=njobs, scale=scale)
    return wls


def _batch(wls, prec="bf16"):
    import paper_1604_06667_amd as cgp
    torch = _torch()
    gs = [make_gridder(wl, prec) for wl in wls]
    ins = [to_device(wl) for wl in wls]
    b = cgp.Batch(gs, torch.bfloat16)
    return b, gs, ins


def _out_np(cube, w, nchan):
    return flat(cube, nchan), w.detach().cpu().numpy().astype(np.float64).ravel()


def _alone(g, lon, lat, d):
    cube, w = g.grid_datacube(lon, lat, d)
    g.sync()
    return _out_np(cube, w, g.nchan)


def _same(a, b, tol=2e-6):
    Ra, Wa = a
    Rb, Wb = b
    assert np.array_equal(np.isnan(Ra), np.isnan(Rb))
    m = ~np.isnan(Ra)
    if m.any():
        scale = np.maximum(np.abs(Rb[m]).max(), 1e-30)
        assert np.abs(Ra[m] - Rb[m]).max() <= tol * scale
    assert np.allclose(Wa, Wb, rtol=1e-6, atol=1e-30)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_batch_matches_single_and_oracle(prec):
    wls = _jobs(8, 0.02)
    say(f"batch of {len(wls)} jobs {prec}: n={[wl.nsamples for wl in wls]} "
        f"C={[wl.nchan for wl in wls]}")
    b, gs, ins = _batch(wls, prec)
    outs = b.outputs()
    b.grid(ins, outs)
    b.sync()
    for j, (wl, g, (lon, lat, d), (cube, w)) in enumerate(zip(wls, gs, ins, outs)):
        got = _out_np(cube, w, wl.nchan)
        _same(got, _alone(g, lon, lat, d))
        if j % 3 == 0:
            ref = oracle.grid_workload(wl)
            ev = oracle.e_val(got[0], ref["R"], ref["W"])
            ew = oracle.e_weights(got[1], ref["W"])
            say(f"  job {j} {wl.kernel[0]} C={wl.nchan}: e_val={ev:.2e} e_W={ew:.2e}")
            assert ev <= TOL_MFMA and ew <= 1e-6


def test_batch_mixed_targets_and_empty_job():
    """WCS and sight-line jobs, circular and elliptical kernels, an empty job."""
    torch = _torch()
    wls = _jobs(5, 0.02)
    sl = synth.config5(nsamples=30_000, ntargets=3_000, box=2.0, nchan=48)
    wls.append(sl)
    e = wls[1]
    empty = synth.Workload("empty", e.lon[:0], e.lat[:0], e.data[:0], e.dtype, e.target,
                           e.kernel, e.support, hpx_maxres=e.hpx_maxres)
    wls.append(empty)
    b, gs, ins = _batch(wls)
    outs = b.outputs()
    b.grid(ins, outs)
    b.sync()
    for wl, g, (lon, lat, d), (cube, w) in zip(wls, gs, ins, outs):
        got = _out_np(cube, w, wl.nchan)
        if wl.nsamples == 0:
            assert np.isnan(got[0]).all() and (got[1] == 0).all()
            continue
        _same(got, _alone(g, lon, lat, d))
    cols = np.arange(0, 3000, 7)
    ref = oracle.grid_workload(sl, targets=cols)
    R = _out_np(*outs[5], sl.nchan)[0]
    assert oracle.e_val(R, ref["R"], ref["W"], cols=cols) <= TOL_MFMA


def test_batch_invalid_coordinates_flagged():
    import paper_1604_06667_amd as cgp
    wls = _jobs(3, 0.02)
    b, gs, ins = _batch(wls)
    lon, lat, d = ins[2]
    lat = lat.clone()
    lat[5] = 95.0
    ins[2] = (lon, lat, d)
    outs = b.outputs()
    b.grid(ins, outs)
    with pytest.raises(cgp.CgError) as ei:
        b.sync()
    assert ei.value.status == cgp._cg.E_INPUT
    b.sync()   # flag cleared


def test_batch_tune_and_graph_replay():
    torch = _torch()
    wls = _jobs(10, 0.03)
    b, gs, ins = _batch(wls)
    outs = b.outputs()
    b.tune(ins, outs, reps=1)
    say(f"tuned: rows/workgroup={b.query(5)} half={b.query(6)} wg/CU={b.query(7)} "
        f"items={b.query(3)}")
    ref = [_out_np(c, w, g.nchan) for g, (c, w) in zip(gs, outs)]
    for g, (lon, lat, d), r in zip(gs, ins, ref):
        _same(r, _alone(g, lon, lat, d))
    outs2 = b.outputs()
    b.capture(ins, outs2)
    assert b.query(8) == 1
    for rep in range(3):
        for c, w in outs2:
            c.fill_(-7.0)
            w.fill_(-7.0)
        torch.cuda.synchronize()
        b.replay()
        b.sync()
        for g, (c, w), r in zip(gs, outs2, ref):
            _same(_out_np(c, w, g.nchan), r)
        # eager work of the program between replays
        x = torch.randn(1 << 20, device="cuda:0")
        float(x.sum().item())


def test_batch_replay_follows_moved_samples():
    """The graph holds the sample buffers, not their candidates: after the
    samples move (here from mostly outside every job's grid back inside,
    which multiplies the candidates), a replay grids the new positions and
    equals an eager pass and each job gridded alone."""
    torch = _torch()
    wls = _jobs(2, 0.03)
    b, gs, ins = _batch(wls)
    orig, far = [], []
    for j, (lon0, lat0, d0) in enumerate(ins):
        lon_far = lon0.clone()
        keep = lon0.shape[0] // 10
        lon_far[keep:] = (lon_far[keep:] + 180.0) % 360.0
        ins[j] = (lon_far, lat0, d0)
        orig.append(lon0)
        far.append(lon_far)
    outs = b.outputs()
    b.capture(ins, outs)
    b.sync()
    ncand = b.query(4)
    for lon0, lon_far in zip(orig, far):
        lon_far.copy_(lon0)
    for c, w in outs:
        c.fill_(-7.0)
        w.fill_(-7.0)
    torch.cuda.synchronize()
    b.replay()
    b.sync()
    say(f"candidates: captured pass {ncand}, replay with the samples back {b.query(4)}")
    assert b.query(4) > 2 * ncand
    for g, (lon, lat, d), (c, w) in zip(gs, ins, outs):
        _same(_out_np(c, w, g.nchan), _alone(g, lon, lat, d))


@pytest.mark.parametrize("njobs,scale", [(6, 0.002), (2, 0.0004)])
def test_batch_tiny_jobs_and_few_items(njobs, scale):
    # Jobs of 1-9 tiles: each job's tiles are split into one run per XCD,
    # so most XCD queues hold few items or none, and the second batch has
    # fewer work items (and workgroups) than XCDs.  Every item must still be
    # taken exactly once: each job equals the same gridder alone.
    wls = synth.config4(njobs=njobs, scale=scale)
    say(f"tiny batch: n={[wl.nsamples for wl in wls]} C={[wl.nchan for wl in wls]} "
        f"grids={[wl.target['wcs']['naxis1'] for wl in wls]}")
    b, gs, ins = _batch(wls)
    outs = b.outputs()
    for c, w in outs:
        c.fill_(-7.0)
        w.fill_(-7.0)
    b.grid(ins, outs)
    b.sync()
    say(f"  items={b.query(3)}")
    for j, (wl, g, (lon, lat, d), (cube, w)) in enumerate(zip(wls, gs, ins, outs)):
        got = _out_np(cube, w, wl.nchan)
        _same(got, _alone(g, lon, lat, d))
        if j == 0:
            ref = oracle.grid_workload(wl)
            ev = oracle.e_val(got[0], ref["R"], ref["W"])
            say(f"  job 0 {wl.kernel[0]} C={wl.nchan}: e_val={ev:.2e}")
            assert ev <= TOL_MFMA
