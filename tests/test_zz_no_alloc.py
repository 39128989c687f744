"""cg_grid_datacube_noalloc (the grid call on the library's static scratch)
through the C ABI: two calls in a row, the second on fewer samples, each
equal to cg_grid_datacube on the same inputs (same lookup and contraction,
so the outputs are identical), for the FP32 and the matrix-core paths; a
request beyond the scratch is refused on the host before any device work.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth
from gpu_util import say, make_gridder, to_device, flat

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _noalloc(g, lon, lat, d, cube, wts):
    from paper_1604_06667_amd import _cg
    torch = _torch()
    L = _cg.lib()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.cg_grid_datacube_noalloc(g._handle(), C.c_void_p(lon.data_ptr()),
                                      C.c_void_p(lat.data_ptr()), C.c_void_p(d.data_ptr()),
                                      _cg._dtype_code(d), int(lon.shape[0]), int(d.stride(0)),
                                      C.c_void_p(cube.data_ptr()), C.c_void_p(wts.data_ptr()), st)


def _same(a, b):
    torch = _torch()
    assert torch.equal(torch.nan_to_num(a, nan=-7.0), torch.nan_to_num(b, nan=-7.0))


@pytest.mark.parametrize("prec,nchan", [("fp32", 3), ("fp32", 40), ("bf16", 96)])
def test_noalloc_matches_grid_datacube(prec, nchan):
    from paper_1604_06667_amd import _cg
    torch = _torch()
    wl = synth.config2(scale=0.06, nchan=nchan)
    say(f"noalloc {prec}: {wl.name}")
    g = make_gridder(wl, prec)
    lon, lat, d = to_device(wl)
    n = lon.shape[0]
    tol = 1e-6 if prec == "fp32" else 2e-3
    for m in (n, n // 3):
        say(f"  call on {m} samples")
        cube_a = torch.full(g._empty_out(nchan).shape, -5.0, device="cuda:0")
        wts_a = torch.full(g._empty_out(0).shape, -5.0, device="cuda:0")
        assert _noalloc(g, lon[:m], lat[:m], d[:m], cube_a, wts_a) == _cg.OK
        cube_b, wts_b = g.grid_datacube(lon[:m], lat[:m], d[:m])
        torch.cuda.synchronize()
        g.sync()
        _same(cube_a, cube_b)
        _same(wts_a, wts_b)
        sub = synth.Workload(wl.name, wl.lon[:m], wl.lat[:m], wl.data[:m], wl.dtype, wl.target,
                             wl.kernel, wl.support, hpx_maxres=wl.hpx_maxres)
        ref = oracle.grid_workload(sub)
        R = flat(cube_a, nchan)
        W = wts_a.cpu().numpy().astype(np.float64).ravel()
        ev, ew = oracle.e_val(R, ref["R"], ref["W"]), oracle.e_weights(W, ref["W"])
        say(f"  e_val={ev:.3e} e_W={ew:.3e}")
        assert ev <= tol and ew <= 1e-6


def test_noalloc_refuses_more_than_the_scratch():
    from paper_1604_06667_amd import _cg
    torch = _torch()
    wl = synth.config2(scale=0.03, nchan=4)
    g = make_gridder(wl, "fp32")
    lon, lat, d = to_device(wl)
    n_big = 4_000_000   # > 128 MiB of workspace; refused on the host before any device work
    assert g.workspace_size(n_big) > 128 << 20
    L = _cg.lib()
    cube = g._empty_out(4)
    wts = g._empty_out(0)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    r = L.cg_grid_datacube_noalloc(g._handle(), C.c_void_p(lon.data_ptr()),
                                   C.c_void_p(lat.data_ptr()), C.c_void_p(d.data_ptr()),
                                   _cg._dtype_code(d), n_big, int(d.stride(0)),
                                   C.c_void_p(cube.data_ptr()), C.c_void_p(wts.data_ptr()), st)
    assert r == _cg.E_WORKSPACE
    assert b"static scratch holds" in L.cg_last_error()
