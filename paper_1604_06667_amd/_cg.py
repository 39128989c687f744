"""ctypes binding of libcg (include/cg.h): argument marshalling only.

Every step of the gridding runs in the HIP library; this module converts
torch tensors and Python values into the pointers and sizes of the C ABI
and turns status codes into exceptions.  There is no fallback: if
``libcg.so`` is missing the import of the library fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcg.so")

OK, E_INVALID, E_STATE, E_OOM, E_UNSUPPORTED, E_DEVICE, E_INPUT, E_WORKSPACE = (
    0, -1, -2, -3, -4, -5, -6, -7)
F64, F32, F16, BF16 = 0, 1, 2, 3
PREC = {"fp32": 0, "bf16": 1, "fp16": 2}
KERNEL = {"gauss1d": 0, "gauss2d": 1, "tapered_sinc": 2, "table": 3}
LOOKUP = {"tiles": 0, "disk": 1}
PROJ = {"CAR": 0, "SIN": 1, "SFL": 2, "ZEA": 3}
LAYOUT = {"channel": 0, "target": 1}


class CgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"cg status {status}: {msg}")
        self.status = status


class CgWcs(C.Structure):
    _fields_ = [("proj", C.c_int32), ("reserved", C.c_int32),
                ("naxis1", C.c_int64), ("naxis2", C.c_int64),
                ("crpix1", C.c_double), ("crpix2", C.c_double),
                ("crval1", C.c_double), ("crval2", C.c_double),
                ("cdelt1", C.c_double), ("cdelt2", C.c_double)]


class CgBatchJob(C.Structure):
    _fields_ = [("lon_deg", C.c_void_p), ("lat_deg", C.c_void_p), ("data", C.c_void_p),
                ("nsamples", C.c_int64), ("ld_data", C.c_int64),
                ("cube_out", C.c_void_p), ("weights_out", C.c_void_p)]


_vp, _i32, _i64, _d, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
_P = C.POINTER

# cg_alloc_fn / cg_free_fn (include/cg.h)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_int, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)

SIGNATURES = {
    "cg_create_wcs": (_i32, [_P(_vp), _P(CgWcs), _i64]),
    "cg_create_sightlines": (_i32, [_P(_vp), _vp, _vp, _i64, _i64, _vp]),
    "cg_create_healpix": (_i32, [_P(_vp), _i64, _i32, _i64, _vp]),
    "cg_hpx_centres": (_i32, [_i64, _i32, _i64, _i64, _vp, _vp]),
    "cg_set_kernel": (_i32, [_vp, _i32, _P(_d), _i32, _d, _d]),
    "cg_set_nside": (_i32, [_vp, _i64]),
    "cg_set_precision": (_i32, [_vp, _i32]),
    "cg_set_lookup": (_i32, [_vp, _i32]),
    "cg_disk_stats": (_i32, [_vp, _P(_i64), _P(_i64)]),
    "cg_set_output_layout": (_i32, [_vp, _i32]),
    "cg_set_allocator": (_i32, [ALLOC_FN, FREE_FN, _vp]),
    "cg_workspace_size": (_i32, [_vp, _i64, _P(_sz)]),
    "cg_grid": (_i32, [_vp, _vp, _vp, _vp, _i32, _i64, _i64, _vp, _sz, _vp]),
    "cg_get_datacube": (_i32, [_vp, _vp, _vp]),
    "cg_get_weights": (_i32, [_vp, _vp, _vp]),
    "cg_grid_datacube": (_i32, [_vp, _vp, _vp, _vp, _i32, _i64, _i64, _vp, _vp, _vp, _sz, _vp]),
    "cg_grid_datacube_noalloc": (_i32, [_vp, _vp, _vp, _vp, _i32, _i64, _i64, _vp, _vp, _vp]),
    "cg_clear": (_i32, [_vp, _vp]),
    "cg_sync": (_i32, [_vp, _vp]),
    "cg_neighbour_stats": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "cg_query": (_i32, [_vp, _i32, _P(_i64)]),
    "cg_profile_enable": (_i32, [_vp, _i32]),
    "cg_profile_read": (_i32, [_vp, _P(_i64), _P(_d)]),
    "cg_destroy": (None, [_vp]),
    "cg_batch_create": (_i32, [_P(_vp), _P(_vp), _i32, _i32]),
    "cg_batch_grid": (_i32, [_vp, _P(CgBatchJob), _vp]),
    "cg_batch_tune": (_i32, [_vp, _P(CgBatchJob), _i32, _vp]),
    "cg_batch_capture": (_i32, [_vp, _P(CgBatchJob), _vp]),
    "cg_batch_replay": (_i32, [_vp, _vp]),
    "cg_batch_sync": (_i32, [_vp, _vp]),
    "cg_batch_query": (_i32, [_vp, _i32, _P(_i64)]),
    "cg_batch_profile_enable": (_i32, [_vp, _i32]),
    "cg_batch_profile_read": (_i32, [_vp, _P(_i64), _P(_d)]),
    "cg_batch_destroy": (None, [_vp]),
    "cg_last_error": (C.c_char_p, []),
    "cg_version": (C.c_char_p, []),
    "cg_hpx_ang2pix_ring": (_i32, [_i64, _i64, _vp, _vp, _vp]),
    "cg_hpx_pix2ang_ring": (_i32, [_i64, _i64, _vp, _vp, _vp]),
    "cg_hpx_pix2ring": (_i32, [_i64, _i64, _vp, _vp, _vp]),
    "cg_hpx_ring_info": (_i32, [_i64, _i64, _P(_i64), _P(_i64), _P(_d)]),
    "cg_hpx_cap_ranges": (_i32, [_i64, _d, _d, _d, _vp, _i64, _P(_i64)]),
    "cg_hpx_query_disk": (_i32, [_i64, _i64, _d, _vp, _i64, _P(_i64)]),
    "cg_hpx_targets_ranges": (_i32, [_i64, _i64, _vp, _vp, _d, _vp, _i64, _P(_i64)]),
    "cg_wcs_pix2world": (_i32, [_P(CgWcs), _i64, _vp, _vp, _vp, _vp]),
}

_LIB = None


def lib():
    """Load libcg.so (built in-tree by paper_1604_06667_amd.build)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1604_06667_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def check(status: int):
    if status != OK:
        msg = lib().cg_last_error().decode(errors="replace")
        raise CgError(status, msg)


def version() -> str:
    return lib().cg_version().decode()


# ------------------------------------------------------------- allocator

_ALLOC = {"mode": None}
# Every callback pair ever handed to the library stays alive for the life of
# the process: a handle keeps the allocator it was created with, so its
# functions must outlive any later change of the allocator.
_KEEPALIVE = []


def _torch_alloc(nbytes, device, stream, ctx):
    try:
        torch = _torch()
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=int(device),
                                                  stream=int(stream) if stream else None)
    except Exception:   # out of memory: the library reports CG_E_OOM
        return None


def _torch_free(ptr, nbytes, device, ctx):
    try:
        _torch().cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


_TORCH_FNS = (ALLOC_FN(_torch_alloc), FREE_FN(_torch_free))
_KEEPALIVE.append(_TORCH_FNS)


def set_allocator(alloc=None, free=None):
    """Device memory of gridders and batches created from now on
    (cg_set_allocator): ``alloc(nbytes, device, stream) -> int`` (a device
    address, 0 when out of memory) and ``free(ptr, nbytes, device)``, or
    ``None`` for both to use hipMalloc/hipFree.  Gridders created earlier
    keep the allocator they were created with."""
    if (alloc is None) != (free is None):
        raise ValueError("give both alloc and free, or neither")
    if alloc is None:
        fns = (ALLOC_FN(), FREE_FN())
        mode = "hip"
    else:
        fns = (ALLOC_FN(lambda n, d, s, c: alloc(n, d, s) or None),
               FREE_FN(lambda p, n, d, c: free(p, n, d)))
        mode = "custom"
    _KEEPALIVE.append(fns)
    check(lib().cg_set_allocator(fns[0], fns[1], None))
    _ALLOC["mode"] = mode


def use_torch_allocator():
    """Give gridders and batches created from now on PyTorch's caching
    allocator (the default of this binding)."""
    check(lib().cg_set_allocator(_TORCH_FNS[0], _TORCH_FNS[1], None))
    _ALLOC["mode"] = "torch"


def _default_allocator():
    if _ALLOC["mode"] is None:
        use_torch_allocator()


# ------------------------------------------------------------------- helpers

def _torch():
    import torch
    return torch


def _dev_ptr(t, dtype=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dtype_code(t):
    torch = _torch()
    m = {torch.float64: F64, torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}
    if t.dtype not in m:
        raise TypeError(f"unsupported data dtype {t.dtype}")
    return m[t.dtype]


def _ws_arg(ws):
    """(pointer, bytes) of a caller workspace tensor, or (NULL, 0)."""
    if ws is None:
        return None, 0
    torch = _torch()
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or not ws.is_contiguous():
        raise TypeError("ws must be a contiguous CUDA (HIP) tensor")
    return C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()


def _data2d(signal, nchan):
    if signal.dim() == 1:
        signal = signal[:, None]
    if signal.dim() != 2 or signal.shape[1] != nchan:
        raise ValueError(f"signal must be [N][{nchan}]")
    if signal.stride(1) != 1:
        signal = signal.contiguous()
    return signal


def parse_header(header: dict):
    """FITS-like header dict (Listing 1 keys) -> (CgWcs, nchan)."""
    h = {str(k).upper(): v for k, v in header.items()}
    ctype = str(h.get("CTYPE1", "RA---CAR")).upper()
    proj = ctype[-3:]
    if proj not in PROJ:
        raise CgError(E_UNSUPPORTED, f"projection {proj!r} is not supported (CAR, SIN, SFL, ZEA)")
    w = CgWcs(PROJ[proj], 0, int(h["NAXIS1"]), int(h["NAXIS2"]),
              float(h.get("CRPIX1", 1.0)), float(h.get("CRPIX2", 1.0)),
              float(h.get("CRVAL1", 0.0)), float(h.get("CRVAL2", 0.0)),
              float(h["CDELT1"]), float(h["CDELT2"]))
    nchan = int(h.get("NAXIS3", 1)) if int(h.get("NAXIS", 2)) >= 3 else 1
    return w, nchan


class _Gridder:
    """Common part of WcsGrid and SlGrid (the paper's Cygrid base class)."""

    def __init__(self):
        self._h = None
        self.nchan = 0
        self.out_shape = ()

    def _handle(self):
        if self._h is None:
            raise CgError(E_STATE, "gridder destroyed")
        return self._h

    def __del__(self):
        try:
            if self._h is not None and _LIB is not None:
                _LIB.cg_destroy(self._h)
        except Exception:
            pass
        self._h = None

    def close(self):
        if self._h is not None:
            lib().cg_destroy(self._h)
            self._h = None

    # Listing 1: set_kernel(kernel_type, kernel_params, kernel_support, hpx_maxres)
    def set_kernel(self, kernel_type, kernel_params, kernel_support, hpx_maxres=0.0):
        if kernel_type not in KERNEL:
            raise CgError(E_INVALID, f"unknown kernel type {kernel_type!r}")
        params = [float(p) for p in kernel_params]
        arr = (C.c_double * max(1, len(params)))(*params)
        check(lib().cg_set_kernel(self._handle(), KERNEL[kernel_type], arr, len(params),
                                  float(kernel_support), float(hpx_maxres)))

    def set_nside(self, nside):
        check(lib().cg_set_nside(self._handle(), int(nside)))

    def set_lookup(self, lookup):
        """'tiles' (default) or 'disk': the sample-centric lookup of Sect. 3.3
        (query disks shifted along rings, Eq. 4-5, then inverted)."""
        if lookup not in LOOKUP:
            raise CgError(E_INVALID, f"unknown lookup {lookup!r}")
        check(lib().cg_set_lookup(self._handle(), LOOKUP[lookup]))

    def disk_stats(self):
        """(distinct sample pixels, (tile, pixel) pairs) of the last grid call
        with the 'disk' lookup."""
        a, b = C.c_int64(), C.c_int64()
        check(lib().cg_disk_stats(self._handle(), C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_precision(self, prec):
        if prec not in PREC:
            raise CgError(E_INVALID, f"unknown precision {prec!r}")
        check(lib().cg_set_precision(self._handle(), PREC[prec]))

    def set_output_layout(self, layout):
        """'channel' ([C][...], default) or 'target' ([...][C]) cubes."""
        if layout not in LAYOUT:
            raise CgError(E_INVALID, f"unknown layout {layout!r}")
        check(lib().cg_set_output_layout(self._handle(), LAYOUT[layout]))
        self.layout = layout

    def _coords(self, lon, lat):
        torch = _torch()
        if lon.shape != lat.shape or lon.dim() != 1:
            raise ValueError("lon/lat must be 1-D of equal length")
        return _dev_ptr(lon, torch.float64, "lon"), _dev_ptr(lat, torch.float64, "lat")

    def workspace_size(self, nsamples):
        """Bytes of workspace a grid call on ``nsamples`` samples needs."""
        v = C.c_size_t()
        check(lib().cg_workspace_size(self._handle(), int(nsamples), C.byref(v)))
        return v.value

    def workspace(self, nsamples):
        """A device workspace (uint8 tensor) for grid calls on up to
        ``nsamples`` samples."""
        torch = _torch()
        return torch.empty(self.workspace_size(nsamples), dtype=torch.uint8,
                           device=f"cuda:{self.device}")

    # Listing 1: grid(lon, lat, signal); accumulates
    def grid(self, lon, lat, signal, ws=None, stream=None):
        pl, pb = self._coords(lon, lat)
        sig = _data2d(signal, self.nchan)
        wp, wn = _ws_arg(ws)
        check(lib().cg_grid(self._handle(), pl, pb, C.c_void_p(sig.data_ptr()), _dtype_code(sig),
                            int(lon.shape[0]), int(sig.stride(0)), wp, wn, _stream(stream)))

    def _empty_out(self, nch):
        torch = _torch()
        if not nch:
            shape = self.out_shape
        elif getattr(self, "layout", "channel") == "target":
            shape = self.out_shape + (nch,)
        else:
            shape = (nch,) + self.out_shape
        return torch.empty(shape, dtype=torch.float32, device=f"cuda:{self.device}")

    # Listing 1: get_datacube()
    def get_datacube(self, out=None, stream=None, check_input=True):
        out = self._empty_out(self.nchan) if out is None else out
        check(lib().cg_get_datacube(self._handle(), _dev_ptr(out, name="out"), _stream(stream)))
        if check_input:
            self.sync(stream)
        return out

    def get_weights(self, out=None, stream=None):
        out = self._empty_out(0) if out is None else out
        check(lib().cg_get_weights(self._handle(), _dev_ptr(out, name="out"), _stream(stream)))
        return out

    def grid_datacube(self, lon, lat, signal, cube=None, weights=None, ws=None, stream=None):
        """clear + grid + get_datacube + get_weights in one pass."""
        pl, pb = self._coords(lon, lat)
        sig = _data2d(signal, self.nchan)
        cube = self._empty_out(self.nchan) if cube is None else cube
        wp = None
        if weights is not False:
            weights = self._empty_out(0) if weights is None else weights
            wp = _dev_ptr(weights, name="weights")
        sp, sn = _ws_arg(ws)
        check(lib().cg_grid_datacube(self._handle(), pl, pb, C.c_void_p(sig.data_ptr()),
                                     _dtype_code(sig), int(lon.shape[0]), int(sig.stride(0)),
                                     _dev_ptr(cube, name="cube"), wp, sp, sn, _stream(stream)))
        return cube, (weights if weights is not False else None)

    def grid_datacube_noalloc(self, lon, lat, signal, cube, weights=None, stream=None):
        """grid_datacube into caller buffers with the library's static
        scratch as workspace (cg_grid_datacube_noalloc): no allocation."""
        pl, pb = self._coords(lon, lat)
        sig = _data2d(signal, self.nchan)
        wp = _dev_ptr(weights, name="weights") if weights is not None else None
        check(lib().cg_grid_datacube_noalloc(self._handle(), pl, pb, C.c_void_p(sig.data_ptr()),
                                             _dtype_code(sig), int(lon.shape[0]),
                                             int(sig.stride(0)), _dev_ptr(cube, name="cube"), wp,
                                             _stream(stream)))
        return cube, weights

    def clear(self, stream=None):
        check(lib().cg_clear(self._handle(), _stream(stream)))

    def sync(self, stream=None):
        check(lib().cg_sync(self._handle(), _stream(stream)))

    def neighbour_stats(self, lon, lat, stream=None):
        torch = _torch()
        pl, pb = self._coords(lon, lat)
        n = int(self.query(0))
        counts = torch.empty(n, dtype=torch.int32, device=f"cuda:{self.device}")
        hashes = torch.empty(n, dtype=torch.int64, device=f"cuda:{self.device}")
        check(lib().cg_neighbour_stats(self._handle(), pl, pb, int(lon.shape[0]),
                                       _dev_ptr(counts), _dev_ptr(hashes), _stream(stream)))
        return counts, hashes

    def query(self, what):
        v = C.c_int64()
        check(lib().cg_query(self._handle(), int(what), C.byref(v)))
        return v.value

    def profile(self, enable=True):
        check(lib().cg_profile_enable(self._handle(), 1 if enable else 0))

    def profile_read(self):
        n, ms = C.c_int64(), C.c_double()
        check(lib().cg_profile_read(self._handle(), C.byref(n), C.byref(ms)))
        return n.value, ms.value

    @property
    def nside(self):
        return self.query(2)

    @property
    def ntiles(self):
        return self.query(3)

    @property
    def last_candidates(self):
        return self.query(4)


class WcsGrid(_Gridder):
    """Gridder onto the pixel centres of a FITS/WCS header (CAR, SIN, SFL or ZEA)."""

    def __init__(self, header: dict, nchan: int | None = None):
        super().__init__()
        _default_allocator()
        w, n = parse_header(header)
        self.nchan = int(nchan) if nchan is not None else n
        h = C.c_void_p()
        check(lib().cg_create_wcs(C.byref(h), C.byref(w), self.nchan))
        self._h = h
        self.out_shape = (int(w.naxis2), int(w.naxis1))
        self.device = self.query(6)


class SlGrid(_Gridder):
    """Gridder onto an arbitrary list of sight lines (target coordinates)."""

    def __init__(self, lon, lat, nchan: int = 1, stream=None):
        super().__init__()
        torch = _torch()
        _default_allocator()
        pl = _dev_ptr(lon, torch.float64, "lon")
        pb = _dev_ptr(lat, torch.float64, "lat")
        self.nchan = int(nchan)
        h = C.c_void_p()
        check(lib().cg_create_sightlines(C.byref(h), pl, pb, int(lon.shape[0]), self.nchan,
                                         _stream(stream)))
        self._h = h
        self.out_shape = (int(lon.shape[0]),)
        self.device = self.query(6)


HPX_ORDER = {"ring": 0, "nested": 1}


class HpxGrid(_Gridder):
    """Gridder onto every pixel centre of a HEALPix map (cg_create_healpix):
    12 nside^2 targets, target p being pixel p in ``order`` ("ring" or
    "nested")."""

    def __init__(self, nside: int, order: str = "ring", nchan: int = 1, stream=None):
        super().__init__()
        if order not in HPX_ORDER:
            raise ValueError(f"order must be one of {sorted(HPX_ORDER)}")
        _default_allocator()
        self.nchan = int(nchan)
        self.map_nside = int(nside)     # (nside is the lookup resolution)
        self.map_order = order
        h = C.c_void_p()
        check(lib().cg_create_healpix(C.byref(h), self.map_nside, HPX_ORDER[order], self.nchan,
                                      _stream(stream)))
        self._h = h
        self.out_shape = (12 * self.map_nside * self.map_nside,)
        self.device = self.query(6)


class Batch:
    """Many gridding jobs evaluated in one lookup pass and one persistent
    contraction launch (cg_batch_* of the C ABI).  ``gridders`` are WcsGrid /
    SlGrid objects with their kernel and matrix-core precision set; every
    job's data has the same dtype."""

    def __init__(self, gridders, dtype):
        torch = _torch()
        codes = {torch.float64: F64, torch.float32: F32, torch.float16: F16,
                 torch.bfloat16: BF16}
        if dtype not in codes:
            raise TypeError(f"unsupported data dtype {dtype}")
        _default_allocator()
        self.gridders = list(gridders)
        self.dtype = dtype
        arr = (C.c_void_p * len(self.gridders))(*[g._handle().value for g in self.gridders])
        h = C.c_void_p()
        check(lib().cg_batch_create(C.byref(h), arr, len(self.gridders), codes[dtype]))
        self._h = h
        self._keep = None

    def __del__(self):
        try:
            if self._h is not None and _LIB is not None:
                _LIB.cg_batch_destroy(self._h)
        except Exception:
            pass
        self._h = None

    def close(self):
        if self._h is not None:
            lib().cg_batch_destroy(self._h)
            self._h = None

    def _jobs(self, inputs, outputs):
        """inputs: [(lon, lat, data)], outputs: [(cube, weights or None)]."""
        torch = _torch()
        if len(inputs) != len(self.gridders) or len(outputs) != len(self.gridders):
            raise ValueError("one (lon, lat, data) and one (cube, weights) per job")
        arr = (CgBatchJob * len(self.gridders))()
        keep = []
        for j, (g, (lon, lat, data), (cube, wts)) in enumerate(zip(self.gridders, inputs, outputs)):
            if data.dtype != self.dtype:
                raise TypeError(f"job {j}: data dtype {data.dtype} != batch dtype {self.dtype}")
            n = int(lon.shape[0])
            sig = _data2d(data, g.nchan)
            pl, pb = g._coords(lon, lat)
            arr[j].lon_deg = pl.value
            arr[j].lat_deg = pb.value
            arr[j].data = sig.data_ptr() if n else None
            arr[j].nsamples = n
            arr[j].ld_data = int(sig.stride(0)) if n else g.nchan
            arr[j].cube_out = _dev_ptr(cube, torch.float32, "cube").value
            arr[j].weights_out = (_dev_ptr(wts, torch.float32, "weights").value
                                  if wts is not None else None)
            keep.append((lon, lat, sig, cube, wts))
        return arr, keep

    def outputs(self):
        return [(g._empty_out(g.nchan), g._empty_out(0)) for g in self.gridders]

    def grid(self, inputs, outputs, stream=None):
        arr, keep = self._jobs(inputs, outputs)
        check(lib().cg_batch_grid(self._h, arr, _stream(stream)))
        self._keep = keep

    def tune(self, inputs, outputs, reps=3, stream=None):
        arr, keep = self._jobs(inputs, outputs)
        check(lib().cg_batch_tune(self._h, arr, int(reps), _stream(stream)))
        self._keep = keep

    def capture(self, inputs, outputs, stream=None):
        arr, keep = self._jobs(inputs, outputs)
        check(lib().cg_batch_capture(self._h, arr, _stream(stream)))
        self._keep = keep   # the graph holds these pointers

    def replay(self, stream=None):
        check(lib().cg_batch_replay(self._h, _stream(stream)))

    def sync(self, stream=None):
        check(lib().cg_batch_sync(self._h, _stream(stream)))

    def query(self, what):
        v = C.c_int64()
        check(lib().cg_batch_query(self._h, int(what), C.byref(v)))
        return v.value

    def profile(self, enable=True):
        check(lib().cg_batch_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        n, ms = C.c_int64(), C.c_double()
        check(lib().cg_batch_profile_read(self._h, C.byref(n), C.byref(ms)))
        return n.value, ms.value


# ------------------------------------------------------- host-side helpers

def _np_ptr(a):
    return C.c_void_p(a.ctypes.data)


def hpx_ang2pix_ring(nside, lon_deg, lat_deg):
    import numpy as np
    lon = np.ascontiguousarray(lon_deg, dtype=np.float64)
    lat = np.ascontiguousarray(lat_deg, dtype=np.float64)
    out = np.empty(lon.shape[0], dtype=np.int64)
    check(lib().cg_hpx_ang2pix_ring(int(nside), lon.shape[0], _np_ptr(lon), _np_ptr(lat), _np_ptr(out)))
    return out


def hpx_pix2ang_ring(nside, pix):
    import numpy as np
    p = np.ascontiguousarray(pix, dtype=np.int64)
    lo = np.empty(p.shape[0])
    la = np.empty(p.shape[0])
    check(lib().cg_hpx_pix2ang_ring(int(nside), p.shape[0], _np_ptr(p), _np_ptr(lo), _np_ptr(la)))
    return lo, la


def hpx_centres(nside, order="ring", first=0, count=None):
    """Pixel centres (degrees) of an nside map in ``order``, as the HpxGrid
    targets get them (host code)."""
    import numpy as np
    if order not in HPX_ORDER:
        raise ValueError(f"order must be one of {sorted(HPX_ORDER)}")
    if count is None:
        count = 12 * int(nside) ** 2 - int(first)
    lo = np.empty(int(count))
    la = np.empty(int(count))
    check(lib().cg_hpx_centres(int(nside), HPX_ORDER[order], int(first), int(count),
                               _np_ptr(lo), _np_ptr(la)))
    return lo, la


def hpx_pix2ring(nside, pix):
    import numpy as np
    p = np.ascontiguousarray(pix, dtype=np.int64)
    r = np.empty(p.shape[0], dtype=np.int64)
    j = np.empty(p.shape[0], dtype=np.int64)
    check(lib().cg_hpx_pix2ring(int(nside), p.shape[0], _np_ptr(p), _np_ptr(r), _np_ptr(j)))
    return r, j


def hpx_ring_info(nside, i):
    s, n, z = C.c_int64(), C.c_int64(), C.c_double()
    check(lib().cg_hpx_ring_info(int(nside), int(i), C.byref(s), C.byref(n), C.byref(z)))
    return s.value, n.value, z.value


def hpx_cap_ranges(nside, lon_deg, lat_deg, rho_deg, max_ranges=1 << 16):
    import numpy as np
    buf = np.empty(2 * max_ranges, dtype=np.int64)
    n = C.c_int64()
    check(lib().cg_hpx_cap_ranges(int(nside), float(lon_deg), float(lat_deg), float(rho_deg),
                                  _np_ptr(buf), int(max_ranges), C.byref(n)))
    return buf[: 2 * n.value].reshape(-1, 2)


def hpx_query_disk(nside, pix, support_deg, max_ranges=1 << 16):
    """RING pixel ranges [lo, hi] of the shifted query disk that the 'disk'
    lookup uses for sample pixel ``pix``."""
    import numpy as np
    buf = np.empty(2 * max_ranges, dtype=np.int64)
    n = C.c_int64()
    check(lib().cg_hpx_query_disk(int(nside), int(pix), float(support_deg), _np_ptr(buf),
                                  int(max_ranges), C.byref(n)))
    return buf[: 2 * n.value].reshape(-1, 2)


def hpx_targets_ranges(nside, lon_deg, lat_deg, rho_deg, max_ranges=1 << 16):
    import numpy as np
    lo = np.ascontiguousarray(lon_deg, dtype=np.float64)
    la = np.ascontiguousarray(lat_deg, dtype=np.float64)
    buf = np.empty(2 * max_ranges, dtype=np.int64)
    n = C.c_int64()
    check(lib().cg_hpx_targets_ranges(int(nside), lo.shape[0], _np_ptr(lo), _np_ptr(la),
                                      float(rho_deg), _np_ptr(buf), int(max_ranges), C.byref(n)))
    return buf[: 2 * n.value].reshape(-1, 2)


def wcs_pix2world(header: dict, i, j):
    import numpy as np
    w, _ = parse_header(header)
    i = np.ascontiguousarray(i, dtype=np.float64)
    j = np.ascontiguousarray(j, dtype=np.float64)
    lo = np.empty(i.shape[0])
    la = np.empty(i.shape[0])
    check(lib().cg_wcs_pix2world(C.byref(w), i.shape[0], _np_ptr(i), _np_ptr(j), _np_ptr(lo), _np_ptr(la)))
    return lo, la
