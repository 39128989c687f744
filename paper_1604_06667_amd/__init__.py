"""Convolution-based gridding on AMD MI355X (gfx950).

Python face of libcg (C ABI in include/cg.h), following the API of the
paper's Listing 1: ``WcsGrid(header)`` / ``SlGrid(lon, lat)``,
``set_kernel(kernel_type, kernel_params, kernel_support, hpx_maxres)``,
``grid(lon, lat, signal)``, ``get_datacube()``, ``get_weights()``.
Torch supplies device memory and streams; every step runs in the HIP
library.
"""
from ._cg import (WcsGrid, SlGrid, HpxGrid, Batch, CgError, lib, version, parse_header,  # noqa: F401
                  hpx_ang2pix_ring, hpx_pix2ang_ring, hpx_pix2ring, hpx_ring_info,
                  hpx_cap_ranges, hpx_targets_ranges, hpx_query_disk, hpx_centres,
                  wcs_pix2world, set_allocator, use_torch_allocator, PREC, KERNEL, HPX_ORDER,
                  LOOKUP)
