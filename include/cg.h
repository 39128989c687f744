/*
 * cg.h - convolution-based gridding on AMD Instinct MI355X (gfx950), C ABI.
 *
 * Method: Winkel, Floeer & Lenz (2016), "Cygrid: A fast Cython-powered
 * convolution-based gridding module for Python", Sect. 2 and 3.
 *
 *   S_t[c] = sum_n R_n[c] w(t, n)    Eq. (1)   weighted data sum per channel
 *   W_t    = sum_n w(t, n)           Eq. (2)   weight map
 *   R_t[c] = S_t[c] / W_t            Eq. (3)   normalised cube
 *
 * for every target t (the pixel centres of a FITS/WCS grid, or a list of
 * "sight lines"), over the input samples n within the kernel support of t.
 * Candidate samples are found through a HEALPix RING lookup table (Sect. 2.2,
 * 3.3); the support test is exact (d <= support, inclusive) and is made in
 * FP64 on unit vectors, so the result does not depend on the HEALPix
 * resolution.
 *
 * The call sequence mirrors the paper's Python API (Listing 1, Sect. 3.5):
 *   cg_create_wcs / cg_create_sightlines   (WcsGrid(header) / SlGrid(lon, lat))
 *   cg_set_kernel                          (set_kernel(type, params, support, hpx_maxres))
 *   cg_grid                                (grid(lon, lat, signal); accumulates)
 *   cg_get_datacube / cg_get_weights       (get_datacube(); weight map of Eq. 2)
 *
 * Conventions for every entry point:
 *   - Angles are degrees (Listing 1 passes degrees); longitudes any real
 *     value (reduced mod 360), latitudes in [-90, 90].
 *   - "device" pointers are HIP device memory on the handle's device;
 *     "host" pointers are ordinary host memory.  No pointer is retained
 *     after the call returns except where stated (sight-line coordinates are
 *     copied at creation).  Input device buffers must stay valid and
 *     unmodified until the work queued on `stream` has completed.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All device work is queued on it; calls return without waiting for the
 *     GPU except where stated.
 *   - Every call returns a cg_status; nothing throws across the ABI.
 *     Argument and call-order errors are detected on the host before any
 *     device work is queued and leave the handle unchanged and usable.
 *     cg_last_error() returns a thread-local message for the last failure.
 *   - A handle is used from one host thread at a time and one stream at a
 *     time; different handles are independent.
 */
#ifndef CG_H_
#define CG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cg_status {
  CG_OK = 0,
  CG_E_INVALID = -1,      /* bad argument (null pointer, size, kernel parameter) */
  CG_E_STATE = -2,        /* call out of order (e.g. grid before set_kernel) */
  CG_E_OOM = -3,          /* device allocation failed */
  CG_E_UNSUPPORTED = -4,  /* valid request this build does not implement */
  CG_E_DEVICE = -5,       /* a HIP runtime call failed */
  CG_E_INPUT = -6,        /* device-side input error: non-finite or |lat| > 90 */
  CG_E_WORKSPACE = -7     /* caller workspace smaller than cg_workspace_size */
} cg_status;

/* Device memory of the library (cg_set_allocator).  alloc returns `bytes`
 * of device memory on HIP device `device`, at least 256-byte aligned, or
 * NULL when it has none; `stream` (a hipStream_t as void*, NULL = the null
 * stream) is the stream of the call that needs it.  free gives back a block
 * that alloc returned, with its size; the library calls it only after the
 * device has finished the work it queued on that block. */
typedef void* (*cg_alloc_fn)(size_t bytes, int device, void* stream, void* ctx);
typedef void (*cg_free_fn)(void* ptr, size_t bytes, int device, void* ctx);

/* element type of the sample data handed to cg_grid */
typedef enum cg_dtype { CG_F64 = 0, CG_F32 = 1, CG_F16 = 2, CG_BF16 = 3 } cg_dtype;

/* arithmetic of the channel contraction (Eq. 1); distances and the support
 * test are FP64 and the weight map W is accumulated in FP64 in every mode */
typedef enum cg_prec {
  CG_PREC_FP32 = 0,   /* FP32 weights and FP32 data on the vector ALUs, products and sums in
                         FP64 (exact products, so the sums do not depend on candidate order) */
  CG_PREC_BF16 = 1,   /* matrix cores (MFMA), BF16 operands, FP32 accumulate: data and weights
                         are split into BF16 high and residual parts and each block is the sum
                         of three products (hi*hi + lo*hi + hi*lo) */
  CG_PREC_FP16 = 2    /* matrix cores (MFMA), one FP16 product per block, FP32 accumulate;
                         data must lie within the FP16 range */
} cg_prec;

/* memory layout of the cubes a handle writes (cg_get_datacube,
 * cg_grid_datacube, batches) */
typedef enum cg_layout {
  CG_LAYOUT_CHANNEL_MAJOR = 0,  /* [nchan][naxis2][naxis1] or [nchan][ntarget] (FITS order) */
  CG_LAYOUT_TARGET_MAJOR = 1    /* [naxis2][naxis1][nchan] or [ntarget][nchan]: one spectrum per
                                   target contiguous (sight-line lists, spectral analysis) */
} cg_layout;

typedef enum cg_kernel_type {
  CG_GAUSS1D = 0,  /* params = {sigma}: w = exp(-d^2 / (2 sigma^2))            (Listing 1) */
  CG_GAUSS2D = 1,  /* params = {sigma_maj, sigma_min, pa}: elliptical Gaussian in world
                      coordinates (Sect. 2.1, Fig. 1); pa = position angle of the major
                      axis, east of north, at the target */
  CG_TAPERED_SINC = 2, /* params = {sigma, b}: w = exp(-d^2 / (2 sigma^2)) sin(pi d/b) / (pi d/b),
                          the sin(ax)/ax kernel of Sect. 5 (a = pi/b) under a Gaussian taper */
  CG_TABLE = 3     /* params = {dmax, w_0, ..., w_{n-1}} (n >= 2): radial profile of arbitrary
                      shape (abstract), w_k at d = k dmax/(n-1), linear in between, 0 beyond
                      dmax */
} cg_kernel_type;

/* How a grid call finds the samples near each target (cg_set_lookup).  Both
 * give the same result: the lookup only proposes candidates, and the
 * contraction keeps exactly the samples within the support. */
typedef enum cg_lookup {
  CG_LOOKUP_TILES = 0,  /* per tile of targets: the RING pixel windows of the union of the
                           targets' support disks, turned into runs of sorted samples */
  CG_LOOKUP_DISK = 1    /* sample-centric (Sect. 2.2 step 3, Sect. 3.3-3.4): one query disk
                           per HEALPix ring around the pixel nearest longitude 180 deg, moved to
                           every sample pixel by the integer shifts of Eq. 4-5, matched against
                           targets hashed by their nearest pixel, then inverted into per-tile
                           sample lists */
} cg_lookup;

/* FITS/WCS projections (Calabretta & Greisen 2002): CAR and SFL
 * (Sanson-Flamsteed, Listing 1) cylindrical, also oblique; SIN and ZEA
 * (zenithal equal-area, Fig. 1) zenithal with LONPOLE = 180 deg. */
typedef enum cg_proj { CG_PROJ_CAR = 0, CG_PROJ_SIN = 1, CG_PROJ_SFL = 2, CG_PROJ_ZEA = 3 } cg_proj;

/* Target grid of a WcsGrid: the subset of a FITS/WCS header that defines the
 * pixel centres (Listing 1).  CAR and SFL have their reference point at
 * native (0, 0); with crval2 != 0 they are oblique, with the default LONPOLE
 * (0 for crval2 > 0, 180 deg for crval2 < 0) and LATPOLE = +90 deg.  SIN and
 * ZEA use LONPOLE = 180 deg.  |crval2| <= 90.  Pixel (i, j) is 1-based along
 * NAXIS1/NAXIS2. */
typedef struct cg_wcs {
  int32_t proj;          /* cg_proj */
  int32_t reserved;      /* must be 0 */
  int64_t naxis1, naxis2;
  double crpix1, crpix2; /* reference pixel (1-based) */
  double crval1, crval2; /* reference world coordinate, degrees */
  double cdelt1, cdelt2; /* pixel increments, degrees */
} cg_wcs;

typedef struct cg_gridder cg_gridder;   /* opaque handle */

/* Where handles and batches created from now on take their device memory
 * (PyTorch's caching allocator, a pool, ...): every buffer a handle or batch
 * owns comes from alloc_fn and goes back through free_fn, with `ctx` passed
 * through.  A handle keeps the allocator that was in force when it was
 * created until it is destroyed.  NULL for both restores hipMalloc/hipFree.
 * Grid calls allocate nothing once a handle is set up, apart from growing
 * the handle's own workspace when no caller workspace is passed, the
 * accumulators of the first cg_grid, and the pair lists of the
 * sample-centric lookup.  A failing alloc_fn makes the call that needed the
 * memory return CG_E_OOM and leaves the handle usable.  Errors:
 * CG_E_INVALID (only one of the two functions given). */
cg_status cg_set_allocator(cg_alloc_fn alloc_fn, cg_free_fn free_fn, void* ctx);

/* WcsGrid(header) (Sect. 3.5): a gridder whose targets are the pixel
 * centres of `wcs`, with `nchan` >= 1 channels per target, on the current
 * HIP device.  The handle owns its accumulators (S: nchan x targets FP32,
 * W: FP64); they start empty.  Errors: CG_E_INVALID (null pointer, naxis <
 * 1, nchan < 1, zero cdelt, |crval2| > 90), CG_E_UNSUPPORTED (unknown
 * projection), CG_E_OOM, CG_E_DEVICE.  Pixels without a world coordinate
 * (outside the projection) are empty targets.  Synchronises the null stream
 * once. */
cg_status cg_create_wcs(cg_gridder** out, const cg_wcs* wcs, int64_t nchan);

/* SlGrid(lon, lat) (Sect. 3.5, 5): a gridder whose targets are `ntarget`
 * arbitrary coordinates ("sight lines").  lon_deg/lat_deg: device FP64
 * [ntarget], copied into the handle (the caller may free them after the
 * call returns).  Output order of get_datacube/get_weights is the order
 * given here.  Targets with non-finite or |lat| > 90 coordinates stay empty
 * (NaN) and set the sticky input flag.  Synchronises `stream`. */
cg_status cg_create_sightlines(cg_gridder** out, const double* lon_deg, const double* lat_deg,
                               int64_t ntarget, int64_t nchan, void* stream);

/* Pixel order of a HEALPix map (Gorski et al. 2005, the HEALPix paper the
 * cited method builds on). */
typedef enum cg_hpx_order { CG_HPX_RING = 0, CG_HPX_NESTED = 1 } cg_hpx_order;

/* A full HEALPix map as the targets (Sect. 5: sight-line gridding onto the
 * HEALPix pixel centres; App. A.1 grids to the nside = 512 map): a sight-line
 * gridder whose 12 nside^2 targets are the pixel centres, target p being
 * pixel p in `order` (cg_hpx_order).  The centres are computed on the device;
 * internally 64 NESTED-consecutive pixels (an 8 x 8 block of one base face)
 * form a tile.  Output order of get_datacube/get_weights is the pixel index
 * in `order`.  nside: a power of two in [1, 8192].  Errors: CG_E_INVALID
 * (bad order, nside or nchan), CG_E_OOM, CG_E_DEVICE.  Synchronises
 * `stream`. */
cg_status cg_create_healpix(cg_gridder** out, int64_t nside, int32_t order, int64_t nchan,
                            void* stream);

/* set_kernel(kernel_type, kernel_params, kernel_support, hpx_maxres)
 * (Listing 1, Sect. 3.5).  params: host double[nparams] (1 for GAUSS1D, 3
 * for GAUSS2D, 2 for TAPERED_SINC, 3 to 65537 for TABLE; sigmas, b and dmax
 * in degrees and > 0, 0 < sigma_min <= sigma_maj, pa in degrees, table
 * values finite; the table is copied into the handle, after the device has
 * finished earlier work).  The batch API takes
 * GAUSS1D and GAUSS2D gridders only.  support_deg: radius beyond which samples are ignored (0 <
 * support < 90, and at most 1000 times the Gaussian's sigma, sigma_min for
 * GAUSS2D, the taper's sigma for TAPERED_SINC).  hpx_maxres_deg: resolution of the internal HEALPix grid;
 * nside = smallest power of two with sqrt(pi/3)/nside <= hpx_maxres (a
 * speed knob only: the support test is exact), unless cg_set_nside fixed
 * it.  Builds the handle's lookup tables for this support (the HEALPix
 * pixel windows of every tile of targets) on the null stream and waits for
 * them.  May be called again; changing the kernel discards nothing already
 * accumulated.  Every argument is checked before anything changes: a
 * rejected call leaves the previous kernel in force.  Errors:
 * CG_E_INVALID, CG_E_OOM, CG_E_DEVICE. */
cg_status cg_set_kernel(cg_gridder* g, int32_t kernel_type, const double* params, int32_t nparams,
                        double support_deg, double hpx_maxres_deg);

/* Fix the internal HEALPix nside (power of two, 1 <= nside <= 8192) instead of
 * deriving it from hpx_maxres.  After cg_set_kernel it rebuilds the lookup
 * tables as cg_set_kernel does.  Errors: CG_E_INVALID, CG_E_OOM,
 * CG_E_DEVICE. */
cg_status cg_set_nside(cg_gridder* g, int64_t nside);

/* Select the lookup (cg_lookup) of this handle's grid, grid_datacube and
 * neighbour_stats calls.  Default CG_LOOKUP_TILES.  CG_LOOKUP_DISK widens
 * each query disk by the largest pixel radius of the sample's ring and of
 * the target's ring, plus one pixel for the rounding of Eq. 4, so that it
 * still finds every sample within the support; it waits for the device
 * three times per call (to size its pair lists) and needs
 * 4 nside (2 reach + 1) table entries, reach ~ 1.5 (support + 2 pixel radii)
 * nside.  Batches always use the tile lookup.  Errors: CG_E_INVALID;
 * grid calls in disk mode also CG_E_UNSUPPORTED (table above 2^28 entries
 * or 2^32 - 1 pairs). */
cg_status cg_set_lookup(cg_gridder* g, int32_t lookup);

/* Statistics of the last grid call in CG_LOOKUP_DISK mode: distinct sample
 * pixels and (tile, sample pixel) pairs before the inversion.  Errors:
 * CG_E_INVALID. */
cg_status cg_disk_stats(const cg_gridder* g, int64_t* pixels, int64_t* pairs);

/* Select the contraction arithmetic (cg_prec).  Default CG_PREC_FP32.
 * Errors: CG_E_INVALID. */
cg_status cg_set_precision(cg_gridder* g, int32_t prec);

/* Select the layout of the cubes this handle writes (cg_layout).  Default
 * CG_LAYOUT_CHANNEL_MAJOR, the order of get_datacube in Listing 1 (Sect.
 * 3.5); the weight map is [naxis2][naxis1] / [ntarget] in both.  Errors:
 * CG_E_INVALID. */
cg_status cg_set_output_layout(cg_gridder* g, int32_t layout);

/* Bytes of device workspace a grid call (cg_grid, cg_grid_datacube) on
 * `nsamples` samples needs with the handle's current kernel, nside and
 * precision: the HEALPix keys with their sort buffers, the ring offsets, the
 * sorted unit vectors and sample records, and for FP32 grids of at most 16
 * channels the sorted data rows.  About 80 bytes per sample plus 4 * nchan
 * per sample in that last case.  Errors: CG_E_INVALID, CG_E_STATE (no
 * kernel set). */
cg_status cg_workspace_size(const cg_gridder* g, int64_t nsamples, size_t* bytes);

/* grid(lon, lat, signal) (Listing 1; Sect. 2.1 Eq. 1-2): add the
 * contributions of `nsamples` samples to S and W.  lon_deg, lat_deg: device
 * FP64 [nsamples].  data: device, `dtype` elements, row n at data + n*ld_data
 * elements, channel c at column c (one spectrum contiguous); ld_data >=
 * nchan.  Repeated calls accumulate in FP64 (chunked input equals one call
 * to rounding of the sums).  Samples with non-finite or |lat| > 90
 * coordinates are skipped and set the sticky input flag reported by
 * cg_sync.  nsamples == 0 is a no-op.
 * ws, ws_bytes: device workspace of at least cg_workspace_size bytes,
 * 256-byte aligned, owned by the caller and not touched after the queued
 * work completes (it may be reused for the next call on the same stream);
 * NULL: the handle uses (and if needed grows) a workspace of its own.
 * With the tile lookup the call only queues device work: it neither waits
 * for the device nor (given a workspace) allocates, except for the
 * accumulators (FP64 [nchan][targets]) on the first cg_grid of a handle.
 * Errors: CG_E_STATE (no kernel set), CG_E_INVALID, CG_E_WORKSPACE,
 * CG_E_OOM, CG_E_DEVICE. */
cg_status cg_grid(cg_gridder* g, const double* lon_deg, const double* lat_deg, const void* data,
                  int32_t dtype, int64_t nsamples, int64_t ld_data, void* ws, size_t ws_bytes,
                  void* stream);

/* get_datacube() (Listing 1; Eq. 3): out = device FP32 [nchan][naxis2][naxis1]
 * for a WCS grid (FITS/numpy order) or [nchan][ntarget] for sight lines;
 * R = S / W where W > 0, NaN elsewhere.  Does not reset the accumulators.
 * Errors: CG_E_INVALID (null out). */
cg_status cg_get_datacube(cg_gridder* g, float* out, void* stream);

/* Weight map W of Eq. (2): out = device FP32 [naxis2][naxis1] or [ntarget];
 * 0 where no sample lies within the support. */
cg_status cg_get_weights(cg_gridder* g, float* out, void* stream);

/* clear + grid + get_datacube + get_weights in one pass: the accumulators are
 * left empty and the normalised cube and weight map are written straight to
 * cube_out / weights_out (layouts as above; weights_out may be NULL).  Same
 * argument rules, workspace and errors as cg_grid; with the tile lookup and
 * a caller workspace it queues device work only (no allocation, no wait),
 * so it can be captured into a HIP graph. */
cg_status cg_grid_datacube(cg_gridder* g, const double* lon_deg, const double* lat_deg,
                           const void* data, int32_t dtype, int64_t nsamples, int64_t ld_data,
                           float* cube_out, float* weights_out, void* ws, size_t ws_bytes,
                           void* stream);

/* cg_grid_datacube for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, hosts that forbid
 * allocation) and have no workspace of their own to pass: the same lookup
 * and contraction, with the per-call workspace taken from a scratch array
 * of 128 MiB (134,217,728 bytes) that the library holds in static device
 * memory on every device it runs on, for the life of the process.  The
 * caller passes inputs and outputs as for cg_grid_datacube.  The call
 * allocates nothing and does not wait for the device; it takes the address
 * of its device's scratch on its first call there.  Nothing in the scratch
 * has to start at zero.  All calls on one device share that device's
 * scratch and each overwrites it: calls whose work overlaps on one device
 * (different streams, or different host threads) race; calls queued on one
 * stream do not.  Errors: those of cg_grid_datacube; CG_E_WORKSPACE when
 * the samples need more scratch than 128 MiB (cg_workspace_size tells; about
 * 1.6 million samples, fewer for FP32 grids of up to 16 channels);
 * CG_E_UNSUPPORTED with the sample-centric lookup (it sizes its lists per
 * call); CG_E_STATE if the handle's lookup tables were not built. */
cg_status cg_grid_datacube_noalloc(cg_gridder* g, const double* lon_deg, const double* lat_deg,
                                   const void* data, int32_t dtype, int64_t nsamples,
                                   int64_t ld_data, float* cube_out, float* weights_out,
                                   void* stream);

/* Reset S and W to empty (Sect. 2.1 step 1). */
cg_status cg_clear(cg_gridder* g, void* stream);

/* Wait for `stream` and report the sticky device input flag: CG_E_INPUT if
 * any sample or sight line passed since the last cg_sync had a non-finite
 * coordinate or |lat| > 90 (the flag is then cleared), CG_E_DEVICE on a HIP
 * failure, else CG_OK. */
cg_status cg_sync(cg_gridder* g, void* stream);

/* Neighbour-set statistics for verification: for each target, the number of
 * samples with d <= support (counts: device int32 [ntarget]) and the sum mod
 * 2^64 of splitmix64(n) over their input indices n (hashes: device uint64
 * [ntarget]; may be NULL), found through the same lookup as cg_grid.
 * Target order as get_weights.  Does not touch the accumulators. */
cg_status cg_neighbour_stats(cg_gridder* g, const double* lon_deg, const double* lat_deg,
                             int64_t nsamples, int32_t* counts, uint64_t* hashes, void* stream);

/* Handle queries (host):  what = 0 ntargets, 1 nchan, 2 nside, 3 ntiles,
 * 4 candidates of the last lookup (waits for the device), 5 precision,
 * 6 device, 7 layout. */
cg_status cg_query(const cg_gridder* g, int32_t what, int64_t* value);

/* Measurement: while enabled, every launch of the contraction kernel (the
 * step that evaluates Eq. 1-2) made by this handle is bracketed by two HIP
 * events recorded on the stream it is launched on; at most 4096 launches are
 * kept after enabling.  enable = 0 stops recording.  Errors: CG_E_DEVICE. */
cg_status cg_profile_enable(cg_gridder* g, int32_t enable);

/* Number of bracketed contraction launches since the last enable and their
 * summed duration in milliseconds.  Waits for the last recorded launch. */
cg_status cg_profile_read(cg_gridder* g, int64_t* launches, double* total_ms);

void cg_destroy(cg_gridder* g);

/* ---------------------------------------------------------------- batches
 * Many independent gridding jobs of uneven size (sample counts, grids,
 * channel counts, circular or elliptical kernels) evaluated in one pass:
 * one concatenated HEALPix index + sort + ring-offset + lookup pass over the
 * samples of all jobs, and one persistent matrix-core launch over a queue of
 * (job, tile, channel range) items ordered by estimated cost, largest first.
 * Each job computes exactly what cg_grid_datacube computes for its gridder
 * (Eq. 1-3, the same exact support test and the same precision mode).  The
 * paper grids one data set per call (Sect. 3.5); batching is this library's
 * addition for throughput. */
typedef struct cg_batch cg_batch;

/* Inputs and outputs of one job (all device pointers; see cg_grid_datacube
 * for layouts).  data rows are of the batch's dtype; weights_out may be NULL. */
typedef struct cg_batch_job {
  const double* lon_deg;   /* [nsamples] */
  const double* lat_deg;   /* [nsamples] */
  const void* data;        /* [nsamples][ld_data] */
  int64_t nsamples;        /* >= 0 */
  int64_t ld_data;         /* >= the job's nchan */
  float* cube_out;         /* [nchan][naxis2][naxis1] or [nchan][ntarget] */
  float* weights_out;      /* [naxis2][naxis1] or [ntarget], or NULL */
} cg_batch_job;

/* Create a batch over njobs (1..256) gridders, borrowed: they must outlive
 * the batch, must not be used for other calls while it runs, and must not be
 * reconfigured (cg_set_kernel, cg_set_nside) while it exists (a pass or
 * replay that finds a changed gridder returns CG_E_STATE).  Every gridder
 * needs set_kernel and the same matrix-core precision (CG_PREC_BF16 or
 * CG_PREC_FP16, set with cg_set_precision); dtype is the data type of every
 * job's rows.  Waits for the device once (tile tables).  Errors:
 * CG_E_INVALID, CG_E_STATE (a gridder without kernel), CG_E_UNSUPPORTED
 * (CG_PREC_FP32 or mixed precisions or devices), CG_E_OOM, CG_E_DEVICE. */
cg_status cg_batch_create(cg_batch** out, cg_gridder* const* jobs, int32_t njobs, int32_t dtype);

/* One pass over all jobs: in[njobs] (host array of device pointers).  Writes
 * every job's cube and weights.  Buffers are sized from the sample counts;
 * the call waits for the device only before it reuses its pinned staging of
 * the job table.  Invalid sample coordinates are skipped and reported by
 * cg_batch_sync.  Errors: CG_E_INVALID, CG_E_OOM, CG_E_DEVICE. */
cg_status cg_batch_grid(cg_batch* b, const cg_batch_job* in, void* stream);

/* Autotuner: runs one cg_batch_grid on `in`, then times each configuration
 * of the persistent launch (workgroup shape: 8 or 4 wavefronts with one or
 * two 32-channel blocks each, i.e. 128-512 matrix rows; items of full or half
 * width; one or all resident workgroups per compute unit) `reps` times on the
 * same lookup and keeps the fastest for later calls.  The outputs hold a valid result afterwards.  Waits for the
 * device.  Errors as cg_batch_grid. */
cg_status cg_batch_tune(cg_batch* b, const cg_batch_job* in, int32_t reps, void* stream);

/* Record one cg_batch_grid step on `in` as a HIP graph (after running it
 * once eagerly to size every buffer), for replay by cg_batch_replay without
 * host synchronisation.  The graph keeps the device pointers and sample
 * counts of `in`: a replay grids whatever those buffers hold when it runs.
 * A later cg_batch_grid that must enlarge a buffer, or cg_batch_tune, drops
 * the graph.  Waits for the device.  Errors as cg_batch_grid. */
cg_status cg_batch_capture(cg_batch* b, const cg_batch_job* in, void* stream);

/* Launch the captured graph on `stream`.  Errors: CG_E_STATE (no graph),
 * CG_E_DEVICE. */
cg_status cg_batch_replay(cg_batch* b, void* stream);

/* Wait for `stream`; CG_E_INPUT if an invalid sample coordinate was seen
 * (the flag is then cleared), CG_E_DEVICE on a HIP failure, else CG_OK. */
cg_status cg_batch_sync(cg_batch* b, void* stream);

/* Batch queries (host): what = 0 njobs, 1 samples of the last pass,
 * 2 tiles, 3 work items, 4 candidates of the last pass (waits for the
 * device), 5 matrix rows
 * per workgroup (128-512), 6 half-width items (0/1), 7 workgroups per
 * compute unit, 8 graph captured (0/1), 9 workgroup shape (0-3). */
cg_status cg_batch_query(const cg_batch* b, int32_t what, int64_t* value);

/* Measurement as cg_profile_enable / cg_profile_read: events bracket the
 * persistent contraction launch of each eager pass, and the whole step of
 * each replay. */
cg_status cg_batch_profile_enable(cg_batch* b, int32_t enable);
cg_status cg_batch_profile_read(cg_batch* b, int64_t* launches, double* total_ms);

void cg_batch_destroy(cg_batch* b);

const char* cg_last_error(void);
const char* cg_version(void);

/* ---- host-side helpers (the same code the kernels run; for verification) ----
 * HEALPix RING functions re-implemented after Gorski et al. 2005 (Sect. 3.2). */

/* RING index of each (lon, lat) in degrees: host arrays [n] -> out[n]. */
cg_status cg_hpx_ang2pix_ring(int64_t nside, int64_t n, const double* lon_deg, const double* lat_deg,
                              int64_t* out);
/* Pixel centres: out_lon/out_lat degrees [n] of RING pixels pix[n]. */
cg_status cg_hpx_pix2ang_ring(int64_t nside, int64_t n, const int64_t* pix, double* out_lon,
                              double* out_lat);
/* Centres of pixels first .. first + count - 1 of an nside map in `order`
 * (cg_hpx_order), the coordinates cg_create_healpix gives its targets:
 * degrees into host arrays lon_deg/lat_deg [count].  nside a power of two in
 * [1, 8192]; CG_E_INVALID for a range outside the map. */
cg_status cg_hpx_centres(int64_t nside, int32_t order, int64_t first, int64_t count,
                         double* lon_deg, double* lat_deg);
/* Ring of each RING pixel: ring number (1-based) and position in the ring. */
cg_status cg_hpx_pix2ring(int64_t nside, int64_t n, const int64_t* pix, int64_t* ring, int64_t* j);
/* Ring table: for ring i (1..4 nside - 1): first index, pixel count, centre z. */
cg_status cg_hpx_ring_info(int64_t nside, int64_t i, int64_t* start, int64_t* npix, double* z);
/* Pixel ranges that may hold points within rho_deg of (lon, lat): inclusive
 * RING ranges written as pairs into ranges[2*k], ranges[2*k+1] (host, at most
 * max_ranges pairs); *nranges receives the count.  CG_E_INVALID if
 * max_ranges is too small. */
cg_status cg_hpx_cap_ranges(int64_t nside, double lon_deg, double lat_deg, double rho_deg,
                            int64_t* ranges, int64_t max_ranges, int64_t* nranges);
/* Pixel ranges that may hold points within rho_deg of ANY of n points (the
 * union of their disks, ring by ring: the lookup a tile of n targets uses;
 * 1 <= n <= 4096); output as for cg_hpx_cap_ranges. */
cg_status cg_hpx_targets_ranges(int64_t nside, int64_t n, const double* lon_deg,
                                const double* lat_deg, double rho_deg, int64_t* ranges,
                                int64_t max_ranges, int64_t* nranges);
/* The shifted query disk of CG_LOOKUP_DISK for one sample pixel (host):
 * the RING pixel ranges of targets the lookup matches with RING pixel pix
 * for support_deg, as inclusive pairs in ranges[2*k], ranges[2*k+1] (at
 * most max_ranges pairs); *nranges receives the count.  Errors:
 * CG_E_INVALID (bad arguments, or max_ranges too small). */
cg_status cg_hpx_query_disk(int64_t nside, int64_t pix, double support_deg, int64_t* ranges,
                            int64_t max_ranges, int64_t* nranges);
/* WCS pixel centres (host): world coordinates of 1-based pixels (i, j);
 * NaN where the pixel has none. */
cg_status cg_wcs_pix2world(const cg_wcs* wcs, int64_t n, const double* i, const double* j,
                           double* lon_deg, double* lat_deg);

#ifdef __cplusplus
}
#endif

#endif /* CG_H_ */
