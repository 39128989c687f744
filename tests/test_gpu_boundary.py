"""The boundary on the GPU: caller workspaces, HIP-graph capture of a grid
call, the allocator hook (including a failing allocator), FP64 accumulation
over many chunks, and regressions for argument handling (a rejected
set_kernel keeps the previous table; ragged channel counts read nothing past
the rows of the caller's buffers).

Every result is compared with the FP64 oracle (FP32 path e_val <= 1e-6,
matrix cores e_val <= 2e-3) or with the same call without the feature under
test (identical outputs: the feature must not change the arithmetic).
"""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth
from gpu_util import say, make_gridder, to_device, flat, header_of

pytestmark = pytest.mark.gpu

TOL32 = 1e-6
TOL_MFMA = 2e-3


def _torch():
    import torch
    return torch


def _cg():
    from paper_1604_06667_amd import _cg
    return _cg


def _np(cube, w, nchan):
    return flat(cube, nchan), w.detach().cpu().numpy().astype(np.float64).ravel()


def _identical(a, b):
    torch = _torch()
    assert torch.equal(torch.nan_to_num(a, nan=-7.0), torch.nan_to_num(b, nan=-7.0))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_caller_workspace(prec):
    """A caller workspace gives the same cube as the handle's own; a short
    or misaligned one is refused before any device work."""
    torch = _torch()
    cgp = pytest.importorskip("paper_1604_06667_amd")
    wl = synth.config2(scale=0.05, nchan=40)
    say(f"workspace {prec}: {wl.name}")
    g = make_gridder(wl, prec)
    lon, lat, d = to_device(wl)
    n = lon.shape[0]
    need = g.workspace_size(n)
    assert need >= 80 * n
    c0, w0 = g.grid_datacube(lon, lat, d)
    ws = g.workspace(n)
    c1, w1 = g.grid_datacube(lon, lat, d, ws=ws)
    torch.cuda.synchronize()
    _identical(c0, c1)
    _identical(w0, w1)
    ref = oracle.grid_workload(wl)
    R, W = _np(c1, w1, wl.nchan)
    ev = oracle.e_val(R, ref["R"], ref["W"])
    say(f"  e_val={ev:.3e} ({need} workspace bytes for {n} samples)")
    assert ev <= (TOL32 if prec == "fp32" else TOL_MFMA)
    with pytest.raises(cgp.CgError) as ei:
        g.grid_datacube(lon, lat, d, ws=ws[: need - 1])
    assert ei.value.status == _cg().E_WORKSPACE
    big = torch.empty(need + 256, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(cgp.CgError) as ei:
        g.grid_datacube(lon, lat, d, ws=big[8:8 + need])
    assert ei.value.status == _cg().E_INVALID
    # accumulate form with a workspace: two chunks equal one call
    g.clear()
    g.grid(lon[: n // 2], lat[: n // 2], d[: n // 2], ws=ws)
    g.grid(lon[n // 2:], lat[n // 2:], d[n // 2:], ws=ws)
    R2, W2 = _np(g.get_datacube(), g.get_weights(), wl.nchan)
    assert oracle.e_val(R2, ref["R"], ref["W"]) <= (TOL32 if prec == "fp32" else TOL_MFMA)


@pytest.mark.parametrize("prec,lookup_nchan", [("fp32", 3), ("fp32", 40), ("bf16", 64)])
def test_graph_capture_of_grid_datacube(prec, lookup_nchan):
    """One cg_grid_datacube (tile lookup, caller workspace) captured into a
    HIP graph: every replay, with the program's own eager work and
    synchronisations in between, equals the eager call; a replay after the
    sample values change grids the new values."""
    torch = _torch()
    wl = synth.config2(scale=0.04, nchan=lookup_nchan)
    say(f"graph capture {prec}: {wl.name}")
    g = make_gridder(wl, prec)
    lon, lat, d = to_device(wl)
    ws = g.workspace(lon.shape[0])
    cube = g._empty_out(wl.nchan)
    wts = g._empty_out(0)
    g.grid_datacube(lon, lat, d, cube, wts, ws=ws)
    torch.cuda.synchronize()
    eager_c, eager_w = cube.clone(), wts.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        g.grid_datacube(lon, lat, d, cube, wts, ws=ws)   # warm up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s, capture_error_mode="thread_local"):
            g.grid_datacube(lon, lat, d, cube, wts, ws=ws)
    torch.cuda.synchronize()
    for rep in range(4):
        cube.fill_(-3.0)
        wts.fill_(-3.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        _identical(cube, eager_c)
        _identical(wts, eager_w)
        x = torch.randn(1 << 18, device="cuda:0")
        float(x.sum().item())
    # new data in the same buffers: the replay grids it
    d.mul_(2.0)
    graph.replay()
    torch.cuda.synchronize()
    m = ~torch.isnan(eager_c)
    assert torch.allclose(cube[m], 2.0 * eager_c[m], rtol=1e-5, atol=1e-6)
    g.sync()


def test_torch_allocator_is_the_default():
    """Gridders of this binding take their device memory from PyTorch's
    caching allocator: creating one raises torch's allocated bytes by at
    least the handle's target tables, and destroying it gives them back."""
    torch = _torch()
    wl = synth.config2(scale=0.05, nchan=8)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    g = make_gridder(wl, "fp32")
    during = torch.cuda.memory_allocated()
    nslots = g.ntiles * 64
    say(f"torch allocated: +{during - before} bytes for {nslots} target slots")
    assert during - before >= 40 * nslots
    g.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= during - 40 * nslots


def test_failing_allocator_reports_oom_and_keeps_the_handle():
    """An allocator that fails makes the call that needs memory return
    CG_E_OOM; the handle stays usable and grids correctly once memory is
    available again."""
    torch = _torch()
    cgp = pytest.importorskip("paper_1604_06667_amd")
    state = {"fail": False, "live": {}}

    def alloc(n, dev, stream):
        if state["fail"]:
            return 0
        p = torch.cuda.caching_allocator_alloc(int(n), device=int(dev))
        state["live"][p] = n
        return p

    def free(p, n, dev):
        assert state["live"].pop(p) == n
        torch.cuda.caching_allocator_delete(p)

    wl = synth.config2(scale=0.05, nchan=24)
    cgp.set_allocator(alloc, free)
    try:
        # creation fails when the first buffer cannot be had
        state["fail"] = True
        with pytest.raises(cgp.CgError) as ei:
            cgp.WcsGrid(header_of(wl.target["wcs"], wl.nchan))
        assert ei.value.status == _cg().E_OOM
        assert not state["live"]
        state["fail"] = False
        g = make_gridder(wl, "fp32")
        lon, lat, d = to_device(wl)
        # the first grid call needs the handle's own workspace: it fails ...
        state["fail"] = True
        with pytest.raises(cgp.CgError) as ei:
            g.grid_datacube(lon, lat, d)
        assert ei.value.status == _cg().E_OOM
        # ... a caller workspace needs nothing from the allocator ...
        ws = torch.empty(g.workspace_size(lon.shape[0]), dtype=torch.uint8, device="cuda:0")
        c1, w1 = g.grid_datacube(lon, lat, d, ws=ws)
        # ... and once memory is back the handle's own workspace works too
        state["fail"] = False
        c2, w2 = g.grid_datacube(lon, lat, d)
        torch.cuda.synchronize()
        _identical(c1, c2)
        ref = oracle.grid_workload(wl)
        R, W = _np(c2, w2, wl.nchan)
        assert oracle.e_val(R, ref["R"], ref["W"]) <= TOL32
        assert state["live"]
        g.close()
        assert not state["live"], "every block went back through the allocator"
    finally:
        cgp.use_torch_allocator()


def test_rejected_set_kernel_keeps_the_table():
    """A table kernel in force, then a rejected set_kernel with a larger
    table (no hpx_maxres and no fixed nside): the handle keeps the first
    table and grids as before."""
    cgp = pytest.importorskip("paper_1604_06667_amd")
    torch = _torch()
    wl = synth.config2(scale=0.05, nchan=5)
    g = cgp.WcsGrid(header_of(wl.target["wcs"], wl.nchan))
    g.set_precision("fp32")
    sig = 1.5 / 60
    dmax = wl.support
    ks = np.linspace(0.0, dmax, 41)
    tab = np.exp(-0.5 * (ks / sig) ** 2)
    g.set_kernel("table", [dmax, *tab], wl.support, wl.hpx_maxres)
    lon, lat, d = to_device(wl)
    c0, w0 = g.grid_datacube(lon, lat, d)
    c0, w0 = c0.clone(), w0.clone()
    big = np.exp(-0.5 * (np.linspace(0.0, dmax, 4001) / (2 * sig)) ** 2)
    with pytest.raises(cgp.CgError) as ei:
        g.set_kernel("table", [dmax, *big], wl.support, 0.0)
    assert ei.value.status == _cg().E_INVALID
    with pytest.raises(cgp.CgError):
        g.set_kernel("table", [dmax, *big], 95.0, wl.hpx_maxres)
    c1, w1 = g.grid_datacube(lon, lat, d)
    torch.cuda.synchronize()
    _identical(c0, c1)
    _identical(w0, w1)
    wlt = synth.Workload(wl.name, wl.lon, wl.lat, wl.data, wl.dtype, wl.target,
                         ("table", (dmax, *tab)), wl.support, hpx_maxres=wl.hpx_maxres)
    ref = oracle.grid_workload(wlt)
    R, W = _np(c1, w1, wl.nchan)
    assert oracle.e_val(R, ref["R"], ref["W"]) <= TOL32


@pytest.mark.parametrize("prec,nchan", [("bf16", 600), ("bf16", 77), ("fp16", 300)])
def test_ragged_channels_at_the_end_of_storage(prec, nchan):
    """BF16 (or FP16) rows read bit for bit, a channel count that is not a
    multiple of the workgroup's channel range, and the data tensor the last
    bytes of its storage: lanes past the last channel must not read past the
    row (they read its last channel instead).  Per grid and batched."""
    torch = _torch()
    cgp = pytest.importorskip("paper_1604_06667_amd")
    wl = synth.config2(scale=0.04, nchan=nchan)
    say(f"ragged {prec} {nchan} channels: {wl.name}")
    tdt = torch.bfloat16 if prec == "bf16" else torch.float16
    lon, lat, d32 = to_device(wl)
    n = lon.shape[0]
    store = torch.zeros(n * nchan + 4096, dtype=tdt, device="cuda:0")
    d = store[store.numel() - n * nchan:].view(n, nchan)
    d.copy_(d32.to(tdt))
    g = make_gridder(wl, prec)
    c1, w1 = g.grid_datacube(lon, lat, d)
    torch.cuda.synchronize()
    wl16 = synth.Workload(wl.name, wl.lon, wl.lat, d.to(torch.float64).cpu().numpy(), "f64",
                          wl.target, wl.kernel, wl.support, hpx_maxres=wl.hpx_maxres)
    ref = oracle.grid_workload(wl16)
    R, W = _np(c1, w1, nchan)
    ev = oracle.e_val(R, ref["R"], ref["W"])
    say(f"  per grid e_val={ev:.3e}")
    assert ev <= TOL_MFMA
    if prec == "bf16":
        b = cgp.Batch([g], torch.bfloat16)
        outs = b.outputs()
        b.grid([(lon, lat, d)], outs)
        b.sync()
        Rb, Wb = _np(outs[0][0], outs[0][1], nchan)
        assert oracle.e_val(Rb, ref["R"], ref["W"]) <= TOL_MFMA


@pytest.mark.parametrize("prec,tol", [("fp32", TOL32), ("bf16", TOL_MFMA)])
def test_accumulate_64_chunks(prec, tol):
    """grid() in 64 chunks of a cancelling field equals one call to the bar:
    the accumulators are FP64 across calls, so chunking adds no error
    beyond the per-call rounding of the contraction."""
    torch = _torch()
    wl = synth.config_tiny_grid(17, 65, nsamples=12000)
    ref = oracle.grid_workload(wl)
    g = make_gridder(wl, prec)
    lon, lat, d = to_device(wl)
    n = lon.shape[0]
    cuts = np.linspace(0, n, 65).astype(int)
    for a, b in zip(cuts[:-1], cuts[1:]):
        g.grid(lon[a:b], lat[a:b], d[a:b])
    R, W = _np(g.get_datacube(), g.get_weights(), wl.nchan)
    ev = oracle.e_val(R, ref["R"], ref["W"])
    ew = oracle.e_weights(W, ref["W"])
    say(f"  64 chunks {prec}: e_val={ev:.3e} e_W={ew:.3e}")
    assert ev <= tol and ew <= TOL32


@pytest.mark.gpu
def test_support_beyond_1000_sigma_is_rejected():
    """A support of more than 1000 sigma (sigma_min for the elliptical
    kernel) is refused, and the kernel in force before stays usable."""
    torch = _torch()
    cgp = pytest.importorskip("paper_1604_06667_amd")
    wl = synth.config_tiny_grid(9, 3)
    g = make_gridder(wl, "fp32")
    sig = wl.kernel[1][0]
    with pytest.raises(cgp.CgError):
        g.set_kernel("gauss1d", (sig,), 1001.0 * sig, wl.hpx_maxres or 0.5 * sig)
    with pytest.raises(cgp.CgError):
        g.set_kernel("gauss2d", (sig, sig / 2000.0, 30.0), 1.0 * sig, wl.hpx_maxres or 0.5 * sig)
    lon, lat, d = to_device(wl)
    c, w = g.grid_datacube(lon, lat, d)
    torch.cuda.synchronize()
    ref = oracle.grid_workload(wl)
    R, W = _np(c, w, wl.nchan)
    assert oracle.e_val(R, ref["R"], ref["W"]) <= TOL32
