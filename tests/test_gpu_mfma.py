"""GPU parity of the matrix-core (BF16 / FP16 MFMA) contraction.

Bar: e_val <= 2e-3 against the FP64 oracle (channel-normalised max error);
the weight map W (get_weights, Eq. 2) is accumulated from the unrounded
weights and stays within 1e-6; a constant field is reproduced to FP32
accumulation accuracy because the cube is normalised by the sum of the
rounded weights that entered the products.
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


def _run(wl, prec, oneshot=True):
    g = make_gridder(wl, prec)
    lon, lat, d = to_device(wl)
    if oneshot:
        cube, w = g.grid_datacube(lon, lat, d)
    else:
        g.grid(lon, lat, d)
        cube, w = g.get_datacube(), g.get_weights()
    g.sync()
    return g, flat(cube, wl.nchan), w.cpu().numpy().astype(np.float64).ravel()


def _check(R, W, ref, tol=TOL_MFMA, label=""):
    ev = oracle.e_val(R, ref["R"], ref["W"])
    ew = oracle.e_weights(W, ref["W"])
    pr = oracle.pointwise_rel(R, ref["R"], ref["W"])
    say(f"  {label} e_val={ev:.3e} e_W={ew:.3e} p50={np.percentile(pr, 50):.2e} "
        f"p99={np.percentile(pr, 99):.2e}")
    assert ev <= tol
    assert ew <= 1e-6
    return ev


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("nchan", [16, 64, 100, 300, 1100])
def test_cube_mfma(prec, nchan):
    wl = synth.config2(scale=0.06, nchan=nchan)
    say(f"C2-small {prec} nchan={nchan}")
    ref = oracle.grid_workload(wl)
    _, R, W = _run(wl, prec)
    ev = _check(R, W, ref, label=prec)
    # split BF16 is near FP32 accuracy; one FP16 product rounds to 2^-11
    assert ev <= (1e-4 if prec == "bf16" else 1e-3)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_mfma_accumulate_matches_oneshot(prec):
    wl = synth.config2(scale=0.06, nchan=256)
    ref = oracle.grid_workload(wl)
    g = make_gridder(wl, prec)
    lon, lat, d = to_device(wl)
    n = lon.shape[0]
    g.grid(lon[: n // 2], lat[: n // 2], d[: n // 2])
    g.grid(lon[n // 2:], lat[n // 2:], d[n // 2:])
    R = flat(g.get_datacube(), wl.nchan)
    W = g.get_weights().cpu().numpy().astype(np.float64).ravel()
    _check(R, W, ref, label="chunked")


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_constant_field_exact(prec):
    torch = _torch()
    wl = synth.config2(scale=0.06, nchan=128)
    wl = synth.Workload(wl.name, wl.lon, wl.lat, torch.full((wl.nsamples, 128), 3.0),
                        "f32", wl.target, wl.kernel, wl.support, hpx_maxres=wl.hpx_maxres)
    _, R, W = _run(wl, prec)
    m = W > 0
    assert m.sum() > 100
    np.testing.assert_allclose(R[:, m], 3.0, rtol=2e-6)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_sightlines_elliptical_mfma(prec):
    wl = synth.config5(nsamples=60_000, ntargets=20_000, box=3.0, nchan=96)
    say(f"C5-small {prec}")
    ref = oracle.grid_workload(wl)
    _, R, W = _run(wl, prec)
    _check(R, W, ref, label=prec)


def test_allsky_mfma():
    wl = synth.config3(nsamples=120_000, naxis1=360, nchan=40)
    say("C3-small bf16")
    ref = oracle.grid_workload(wl)
    _, R, W = _run(wl, "bf16", oneshot=False)
    _check(R, W, ref, label="bf16")


def test_bf16_input_data():
    """BF16-delivered data (the batched and sight-line workloads): exact on upcast."""
    torch = _torch()
    base = synth.config2(scale=0.06, nchan=200, dtype="bf16")
    ref = oracle.grid_workload(base)
    for prec in ("fp32", "bf16", "fp16"):
        _, R, W = _run(base, prec)
        _check(R, W, ref, tol=1e-6 if prec == "fp32" else TOL_MFMA, label=f"bf16 in, {prec}")
