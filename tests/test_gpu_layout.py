"""GPU: target-major cubes (cg_set_output_layout) hold exactly the values of
the default channel-major cubes, for every contraction path and both target
kinds, one-shot and accumulate-then-normalise, and in batches."""
import numpy as np
import pytest

import synth
from gpu_util import say, make_gridder, to_device

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _both(wl, prec, oneshot=True):
    torch = _torch()
    outs = []
    for layout in ("channel", "target"):
        g = make_gridder(wl, prec)
        g.set_output_layout(layout)
        lon, lat, d = to_device(wl)
        if oneshot:
            cube, w = g.grid_datacube(lon, lat, d)
        else:
            g.grid(lon, lat, d)
            cube, w = g.get_datacube(), g.get_weights()
        g.sync()
        c = cube.detach().cpu().numpy()
        if layout == "target":
            c = np.moveaxis(c, -1, 0)
        outs.append((c, w.detach().cpu().numpy()))
    torch.cuda.synchronize()
    return outs


def _same(a, b):
    (ca, wa), (cb, wb) = a, b
    assert ca.shape == cb.shape
    assert np.array_equal(np.isnan(ca), np.isnan(cb))
    m = ~np.isnan(ca)
    assert np.array_equal(ca[m], cb[m])
    assert np.array_equal(wa, wb)


@pytest.mark.parametrize("prec,nchan", [("fp32", 5), ("fp32", 40), ("bf16", 100), ("fp16", 64)])
@pytest.mark.parametrize("oneshot", [True, False])
def test_wcs_target_major(prec, nchan, oneshot):
    wl = synth.config2(scale=0.04, nchan=nchan)
    say(f"layout WCS {prec} C={nchan} oneshot={oneshot}")
    a, b = _both(wl, prec, oneshot)
    _same(a, b)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_sightlines_target_major(prec):
    wl = synth.config5(nsamples=40_000, ntargets=5_000, box=2.0, nchan=48)
    a, b = _both(wl, prec)
    _same(a, b)


def test_batch_target_major():
    torch = _torch()
    import paper_1604_06667_amd as cgp
    wls = synth.config4(njobs=4, scale=0.02)
    res = []
    for layout in ("channel", "target"):
        gs = []
        for wl in wls:
            g = make_gridder(wl, "bf16")
            g.set_output_layout(layout)
            gs.append(g)
        ins = [to_device(wl) for wl in wls]
        b = cgp.Batch(gs, torch.bfloat16)
        outs = b.outputs()
        b.grid(ins, outs)
        b.sync()
        cur = []
        for (c, w) in outs:
            c = c.detach().cpu().numpy()
            if layout == "target":
                c = np.moveaxis(c, -1, 0)
            cur.append((c, w.detach().cpu().numpy()))
        res.append(cur)
    for a, b in zip(*res):
        _same(a, b)


def test_layout_rejects_unknown():
    import paper_1604_06667_amd as cgp
    wl = synth.config2(scale=0.02, nchan=4)
    g = make_gridder(wl, "fp32")
    with pytest.raises(cgp.CgError):
        g.set_output_layout("diagonal")
    assert cgp.lib().cg_set_output_layout(g._handle(), 7) == cgp._cg.E_INVALID
