// C ABI of libcg: handles, argument checks, workspace and launch sequence.
#include "cg_handle.hpp"

namespace {

using namespace cgh;

bool small_c(const cg_gridder* g) { return g->nchan <= cg::kSmallC && g->prec == CG_PREC_FP32; }

// Set-up of the sample-centric lookup: targets sorted by their nearest
// RING pixel with per-ring offsets (the hash table of Sect. 2.2), and the
// reference query disk of every ring (Sect. 3.3).  Depends only on the
// targets, the support and nside.
cg_status ensure_disk(cg_gridder* g, hipStream_t st) {
  if (g->disk_valid) return CG_OK;
  const int64_t nside = g->nside, nsl = g->nslots;
  const int64_t reach = cg::hpx::disk_ring_reach(nside, g->support_rad);
  const int64_t entries = 4 * nside * (2 * reach + 1);
  if (entries > (int64_t(1) << 28))
    return fail(CG_E_UNSUPPORTED, "query-disk table of %lld entries (support too wide for nside)",
                (long long)entries);
  CG_HIP(ensure(g->alloc, g->dk_tkeys, sizeof(uint32_t) * nsl), "alloc disk lookup");
  CG_HIP(ensure(g->alloc, g->dk_tvals, sizeof(uint32_t) * nsl), "alloc disk lookup");
  CG_HIP(ensure(g->alloc, g->dk_tkeys2, sizeof(uint32_t) * nsl), "alloc disk lookup");
  CG_HIP(ensure(g->alloc, g->dk_tvals2, sizeof(uint32_t) * nsl), "alloc disk lookup");
  CG_HIP(ensure(g->alloc, g->dk_thist, sizeof(uint32_t) * cg::radix_hist_elems(nsl)), "alloc disk lookup");
  CG_HIP(ensure(g->alloc, g->dk_troff, sizeof(uint32_t) * (4 * nside + 1)), "alloc disk lookup");
  CG_HIP(ensure(g->alloc, g->dk_tab, sizeof(int2) * entries), "alloc disk lookup");
  CG_HIP(cg::launch_target_keys(g->txyz.as<double>(), nsl, nside, g->dk_tkeys.as<uint32_t>(),
                                g->dk_tvals.as<uint32_t>(), st),
         "target keys");
  bool in_tmp = false;
  CG_HIP(cg::radix_sort(g->dk_tkeys.as<uint32_t>(), g->dk_tvals.as<uint32_t>(),
                        g->dk_tkeys2.as<uint32_t>(), g->dk_tvals2.as<uint32_t>(),
                        g->dk_thist.as<uint32_t>(), nsl, bits_for((uint64_t)cg::hpx::npix(nside)),
                        &in_tmp, st),
         "sort targets");
  g->dk_tk = in_tmp ? g->dk_tkeys2.as<uint32_t>() : g->dk_tkeys.as<uint32_t>();
  g->dk_ts = in_tmp ? g->dk_tvals2.as<uint32_t>() : g->dk_tvals.as<uint32_t>();
  CG_HIP(cg::launch_ring_offsets(g->dk_tk, nsl, nside, g->dk_troff.as<uint32_t>(), st),
         "target ring offsets");
  CG_HIP(cg::launch_ref_disks(nside, reach, g->support_rad, g->dk_tab.as<int2>(), st),
         "reference disks");
  g->disk_reach = reach;
  g->disk_valid = true;
  return CG_OK;
}

// Sample-centric candidate ranges of a grid call (after the samples are
// sorted): distinct sample pixels, their shifted query disks matched with
// the targets as (tile, pixel) pairs, the pairs sorted by tile, and per tile
// the merged ranges of sorted samples with their candidate counts.  The pair
// lists are sized on the host, so this lookup waits for the device twice.
cg_status run_disk_lookup(cg_gridder* g, int64_t n, hipStream_t st) {
  cg_status s = ensure_disk(g, st);
  if (s != CG_OK) return s;
  const int64_t nside = g->nside;
  const uint32_t* nvalid = g->ws.ring_off + 4 * nside;
  CG_HIP(ensure(g->alloc, g->dk_flag, sizeof(uint64_t) * n), "alloc disk lookup");
  CG_HIP(ensure(g->alloc, g->dk_uoff, sizeof(uint64_t) * (n + 1)), "alloc disk lookup");
  CG_HIP(ensure(g->alloc, g->dk_upix, sizeof(uint32_t) * n), "alloc disk lookup");
  CG_HIP(ensure(g->alloc, g->dk_ustart, sizeof(uint32_t) * (n + 1)), "alloc disk lookup");
  CG_HIP(cg::launch_run_flags(g->sorted_keys, nvalid, n, g->dk_flag.as<uint64_t>(), st),
         "pixel runs");
  CG_HIP(ensure(g->alloc, g->dk_scan, sizeof(uint64_t) * cg::scan_u64_wide_scratch(n)), "alloc disk lookup");
  CG_HIP(cg::scan_u64_wide(g->dk_flag.as<uint64_t>(), g->dk_uoff.as<uint64_t>(), n,
                           g->dk_scan.as<uint64_t>(), st),
         "scan runs");
  CG_HIP(cg::launch_run_compact(g->sorted_keys, nvalid, n, g->dk_uoff.as<uint64_t>(),
                                g->dk_upix.as<uint32_t>(), g->dk_ustart.as<uint32_t>(), st),
         "pixel runs");
  CG_HIP(hipMemcpyAsync(g->h_word, g->dk_uoff.as<uint64_t>() + n, sizeof(uint64_t),
                        hipMemcpyDeviceToHost, st),
         "read runs");
  CG_HIP(hipStreamSynchronize(st), "sync runs");
  const int64_t nu = (int64_t)g->h_word[0];
  CG_HIP(ensure(g->alloc, g->dk_cnt, sizeof(uint64_t) * nu), "alloc disk lookup");
  CG_HIP(ensure(g->alloc, g->dk_off, sizeof(uint64_t) * (nu + 1)), "alloc disk lookup");
  CG_HIP(cg::launch_disk_pairs(true, g->dk_upix.as<uint32_t>(), nu, nside, g->disk_reach,
                               g->dk_tab.as<int2>(), g->dk_tk, g->dk_ts,
                               g->dk_troff.as<uint32_t>(), nullptr, g->dk_cnt.as<uint64_t>(),
                               nullptr, nullptr, st),
         "count pairs");
  CG_HIP(cg::scan_u64_wide(g->dk_cnt.as<uint64_t>(), g->dk_off.as<uint64_t>(), nu,
                           g->dk_scan.as<uint64_t>(), st),
         "scan pairs");
  CG_HIP(hipMemcpyAsync(g->h_word, g->dk_off.as<uint64_t>() + nu, sizeof(uint64_t),
                        hipMemcpyDeviceToHost, st),
         "read pairs");
  CG_HIP(hipStreamSynchronize(st), "sync pairs");
  const int64_t np = (int64_t)g->h_word[0];
  if (np >= 0xFFFFFFFFll)
    return fail(CG_E_UNSUPPORTED, "%lld (tile, pixel) pairs (split the samples)", (long long)np);
  g->last_upix = nu;
  g->last_pairs = np;
  const int64_t nt = g->ntiles;
  CG_HIP(ensure(g->alloc, g->dk_pk, sizeof(uint32_t) * np), "alloc pairs");
  CG_HIP(ensure(g->alloc, g->dk_pv, sizeof(uint32_t) * np), "alloc pairs");
  CG_HIP(ensure(g->alloc, g->dk_pk2, sizeof(uint32_t) * np), "alloc pairs");
  CG_HIP(ensure(g->alloc, g->dk_pv2, sizeof(uint32_t) * np), "alloc pairs");
  CG_HIP(ensure(g->alloc, g->dk_phist, sizeof(uint32_t) * cg::radix_hist_elems(np)), "alloc pairs");
  CG_HIP(ensure(g->alloc, g->dk_flag, sizeof(uint64_t) * np), "alloc pairs");
  CG_HIP(ensure(g->alloc, g->dk_rsx, sizeof(uint64_t) * (np + 1)), "alloc pairs");
  CG_HIP(ensure(g->alloc, g->dk_scan, sizeof(uint64_t) * cg::scan_u64_wide_scratch(np)), "alloc pairs");
  CG_HIP(ensure(g->alloc, g->dk_ranges, sizeof(uint32_t) * 2 * np), "alloc pairs");
  CG_HIP(ensure(g->alloc, g->dk_range_off, sizeof(uint64_t) * (nt + 1)), "alloc pairs");
  CG_HIP(cg::launch_disk_pairs(false, g->dk_upix.as<uint32_t>(), nu, nside, g->disk_reach,
                               g->dk_tab.as<int2>(), g->dk_tk, g->dk_ts,
                               g->dk_troff.as<uint32_t>(), g->dk_off.as<uint64_t>(), nullptr,
                               g->dk_pk.as<uint32_t>(), g->dk_pv.as<uint32_t>(), st),
         "write pairs");
  bool in_tmp = false;
  CG_HIP(cg::radix_sort(g->dk_pk.as<uint32_t>(), g->dk_pv.as<uint32_t>(), g->dk_pk2.as<uint32_t>(),
                        g->dk_pv2.as<uint32_t>(), g->dk_phist.as<uint32_t>(), np,
                        bits_for((uint64_t)nt), &in_tmp, st),
         "sort pairs");
  const uint32_t* pk = in_tmp ? g->dk_pk2.as<uint32_t>() : g->dk_pk.as<uint32_t>();
  const uint32_t* pv = in_tmp ? g->dk_pv2.as<uint32_t>() : g->dk_pv.as<uint32_t>();
  CG_HIP(cg::launch_disk_ranges(pk, pv, np, g->dk_ustart.as<uint32_t>(), g->dk_flag.as<uint64_t>(),
                                g->dk_rsx.as<uint64_t>(), g->dk_scan.as<uint64_t>(), nt,
                                g->dk_ranges.as<uint32_t>(),
                                g->dk_range_off.as<uint64_t>(), g->nranges.as<uint32_t>(),
                                g->ncand.as<uint64_t>(), st),
         "disk ranges");
  return CG_OK;
}

// HEALPix index, sort, ring offsets and permutation of n samples, then the
// ranges of sorted samples that each tile's lookup finds.  Uses the
// workspace at `base` (workspace_layout for n samples) and the handle's
// set-up tables, and only queues device work: with the tile lookup nothing
// here waits for the device or allocates (the sample-centric lookup sizes
// and allocates its pair lists per call).
cg_status run_lookup(cg_gridder* g, const double* lon, const double* lat, int64_t n,
                     const void* data, int32_t dtype, int64_t ld, bool with_data, char* base,
                     hipStream_t st) {
  cg_status s = ensure_span(g, st);
  if (s != CG_OK) return s;
  const int64_t nside = g->nside;
  workspace_layout(n, nside, with_data ? g->nchan : 0, base, &g->ws);
  Workspace& w = g->ws;
  const int npack = with_data && g->nchan <= 2 ? (int)g->nchan : 0;
  CG_HIP(cg::launch_prep(lon, lat, n, nside, w.keys, w.vals, g->flag.as<int>(), w.rec, data,
                         dtype, ld, npack, st),
         "prep");
  bool in_tmp = false;
  const int bits = bits_for((uint64_t)cg::hpx::npix(nside));
  CG_HIP(cg::radix_sort(w.keys, w.vals, w.keys2, w.vals2, w.hist, n, bits, &in_tmp, st),
         "radix sort");
  g->sorted_keys = in_tmp ? w.keys2 : w.keys;
  g->sorted_vals = in_tmp ? w.vals2 : w.vals;
  CG_HIP(cg::launch_ring_offsets(g->sorted_keys, n, nside, w.ring_off, st), "ring offsets");
  CG_HIP(cg::launch_permute(g->sorted_vals, w.ring_off + 4 * nside, n, w.rec, data, dtype, ld,
                            g->nchan, with_data, npack, w.srec, w.sdata, st),
         "permute");
  g->last_n = n;
  g->have_ranges = false;
  if (g->lookup == CG_LOOKUP_DISK) {
    s = run_disk_lookup(g, n, st);
    if (s != CG_OK) return s;
  } else {
    CG_HIP(cg::launch_tile_ranges(g->ntiles, g->ring_first.as<int32_t>(),
                                  g->range_off.as<uint64_t>(), g->win.as<uint32_t>(),
                                  g->sorted_keys, w.ring_off, g->ranges.as<uint32_t>(),
                                  g->nranges.as<uint32_t>(), g->ncand.as<uint64_t>(), st),
           "tile ranges");
  }
  g->have_ranges = true;
  return CG_OK;
}

cg::TileView tile_view(const cg_gridder* g) {
  cg::TileView tv;
  tv.txyz = g->txyz.as<double>();
  tv.tll = g->tll.as<double>();
  const bool disk = g->lookup == CG_LOOKUP_DISK;
  tv.rng = disk ? g->dk_ranges.as<uint32_t>() : g->ranges.as<uint32_t>();
  tv.roff = disk ? g->dk_range_off.as<uint64_t>() : g->range_off.as<uint64_t>();
  tv.nr = g->nranges.as<uint32_t>();
  tv.ntot = g->ncand.as<uint64_t>();
  tv.nslots = g->nslots;
  // the sorted samples of the last lookup
  tv.srec = reinterpret_cast<const double4*>(g->ws.srec);
  tv.ntiles = g->ntiles;
  tv.ntx = g->kind == 0 ? g->ntx : 0;
  return tv;
}

// Workspace bytes of a grid call on n samples with the handle's settings.
size_t ws_bytes_for(const cg_gridder* g, int64_t n) {
  return workspace_layout(n, g->nside, small_c(g) ? g->nchan : 0, nullptr, nullptr);
}

// The workspace of a grid call: the caller's (checked for size and
// alignment), or the handle's own, grown through the handle's allocator.
cg_status call_workspace(cg_gridder* g, int64_t n, void* ws, size_t ws_bytes, hipStream_t st,
                         char** base) {
  const size_t need = ws_bytes_for(g, n);
  if (ws) {
    if (ws_bytes < need)
      return fail(CG_E_WORKSPACE, "workspace of %zu bytes, %zu needed (cg_workspace_size)",
                  ws_bytes, need);
    if (((uintptr_t)ws & 255) != 0) return fail(CG_E_INVALID, "workspace not 256-byte aligned");
    *base = (char*)ws;
    return CG_OK;
  }
  CG_HIP(ensure(g->alloc, g->own_ws, need, st), "alloc workspace");
  *base = g->own_ws.as<char>();
  return CG_OK;
}

cg_status check_grid_args(const cg_gridder* g, const double* lon, const double* lat,
                          const void* data, int32_t dtype, int64_t n, int64_t ld) {
  if (!g) return fail(CG_E_INVALID, "null handle");
  if (!g->kernel_set) return fail(CG_E_STATE, "set_kernel must be called before grid");
  if (n < 0) return fail(CG_E_INVALID, "nsamples < 0");
  if (n > 0xFFFFFFFFll - 1) return fail(CG_E_UNSUPPORTED, "nsamples >= 2^32 (split into chunks)");
  if (n == 0) return CG_OK;
  if (!lon || !lat || !data) return fail(CG_E_INVALID, "null coordinate or data pointer");
  if (dtype < CG_F64 || dtype > CG_BF16) return fail(CG_E_INVALID, "unknown dtype %d", dtype);
  if (ld < g->nchan) return fail(CG_E_INVALID, "ld_data (%lld) < nchan (%lld)", (long long)ld,
                                 (long long)g->nchan);
  return CG_OK;
}

constexpr size_t kMaxProfiled = 4096;

// may_allocate false: events are recorded only into pairs created earlier
cg_status contract(cg_gridder* g, const void* data, int32_t dtype, int64_t ld,
                   const cg::OutView& ov, hipStream_t st, bool may_allocate = true) {
  const cg::TileView tv = tile_view(g);
  std::pair<hipEvent_t, hipEvent_t>* pe = nullptr;
  if (g->prof && g->nev < kMaxProfiled && (may_allocate || g->nev < g->ev.size())) {
    if (g->nev == g->ev.size()) {
      hipEvent_t a, b;
      CG_HIP(hipEventCreate(&a), "event");
      CG_HIP(hipEventCreate(&b), "event");
      g->ev.emplace_back(a, b);
    }
    pe = &g->ev[g->nev++];
    CG_HIP(hipEventRecord(pe->first, st), "event record");
  }
  if (g->prec == CG_PREC_FP32) {
    CG_HIP(cg::launch_gather_fp32(tv, g->kp, data, dtype, ld, g->ws.sdata, g->nchan, ov, st),
           "gather");
  } else {
    CG_HIP(cg::launch_gather_mfma(tv, g->kp, data, g->zrow.p, dtype, ld, g->nchan, g->prec, ov, st),
           "gather (mfma)");
  }
  if (pe) CG_HIP(hipEventRecord(pe->second, st), "event record");
  return CG_OK;
}

// grid + normalise into the caller's cube (the body of cg_grid_datacube and
// of its variant on the library's static scratch), with the workspace at base
cg_status grid_datacube_ws(cg_gridder* g, const double* lon_deg, const double* lat_deg,
                           const void* data, int32_t dtype, int64_t nsamples, int64_t ld_data,
                           float* cube_out, float* weights_out, char* base, hipStream_t st,
                           bool may_allocate = true) {
  cg_status s = run_lookup(g, lon_deg, lat_deg, nsamples, data, dtype, ld_data, small_c(g), base,
                           st);
  if (s != CG_OK) return s;
  cg::OutView ov{};
  ov.cube = cube_out;
  ov.wout = weights_out;
  cube_strides(g, &ov.cst, &ov.tst);
  ov.slot_target = g->slot_target.as<int32_t>();
  ov.ntarget = g->ntarget;
  ov.mode = cg::ACC_FINAL;
  return contract(g, data, dtype, ld_data, ov, st, may_allocate);
}

cg_status empty_datacube(cg_gridder* g, float* cube_out, float* weights_out, hipStream_t st) {
  CG_HIP(cg::launch_fill(cube_out, g->nchan * g->ntarget, __builtin_nanf(""), st), "fill");
  if (weights_out) CG_HIP(cg::launch_fill(weights_out, g->ntarget, 0.0f, st), "fill");
  return CG_OK;
}

void destroy_buffers(cg_gridder* g) {
  DevBuf* bufs[] = {&g->txyz, &g->tll, &g->slot_target, &g->target_slot, &g->caps,
                    &g->ring_first, &g->span_bound, &g->range_off, &g->win, &g->ranges,
                    &g->nranges, &g->ncand, &g->S, &g->W, &g->Wn, &g->flag, &g->zrow, &g->ktab,
                    &g->own_ws, &g->dk_tkeys, &g->dk_tvals, &g->dk_tkeys2, &g->dk_tvals2,
                    &g->dk_thist, &g->dk_troff, &g->dk_tab, &g->dk_flag, &g->dk_uoff,
                    &g->dk_upix, &g->dk_ustart, &g->dk_cnt, &g->dk_off, &g->dk_pk, &g->dk_pv,
                    &g->dk_pk2, &g->dk_pv2, &g->dk_phist, &g->dk_rsx, &g->dk_ranges,
                    &g->dk_range_off, &g->dk_scan};
  for (DevBuf* b : bufs) b->release();
}

cg_gridder* new_gridder() {
  cg_gridder* g = new cg_gridder();
  (void)hipGetDevice(&g->device);
  g->alloc = current_allocator(g->device);
  return g;
}

// ---- the static scratch of cg_grid_datacube_noalloc
// Every device the library runs on holds one copy of this array for the
// life of the process.  In host code its name only stands for the symbol:
// the device address of the current device's copy comes from
// hipGetSymbolAddress, taken once per device and kept in scratch_ptr.
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxScratchDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxScratchDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of `device`'s copy of the scratch array (that device must
// be current).
cg_status scratch_of(int device, char** out) {
  if (device < 0 || device >= kMaxScratchDevices)
    return fail(CG_E_UNSUPPORTED, "device %d: the static scratch serves devices 0-%d", device,
                kMaxScratchDevices - 1);
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "address of the static scratch");
    if (!p) return fail(CG_E_DEVICE, "address of the static scratch: null");
    scratch_ptr[device] = p;
  }
  *out = static_cast<char*>(scratch_ptr[device]);
  return CG_OK;
}

}  // namespace

extern "C" {

const char* cg_last_error(void) { return g_err.c_str(); }
const char* cg_version(void) { return "cg 0.2 (gfx950)"; }

cg_status cg_set_allocator(cg_alloc_fn alloc_fn, cg_free_fn free_fn, void* ctx) {
  if ((alloc_fn == nullptr) != (free_fn == nullptr))
    return fail(CG_E_INVALID, "give both an allocation and a free function, or neither");
  GlobalAllocator& a = global_allocator();
  std::lock_guard<std::mutex> lk(a.mu);
  a.fa = alloc_fn;
  a.ff = free_fn;
  a.ctx = alloc_fn ? ctx : nullptr;
  return CG_OK;
}

cg_status cg_create_wcs(cg_gridder** out, const cg_wcs* wcs, int64_t nchan) {
  if (!out || !wcs) return fail(CG_E_INVALID, "null pointer");
  *out = nullptr;
  if (wcs->proj != CG_PROJ_CAR && wcs->proj != CG_PROJ_SIN && wcs->proj != CG_PROJ_SFL &&
      wcs->proj != CG_PROJ_ZEA)
    return fail(CG_E_UNSUPPORTED, "unknown projection %d", wcs->proj);
  if (wcs->reserved != 0) return fail(CG_E_INVALID, "reserved field must be 0");
  if (wcs->naxis1 < 1 || wcs->naxis2 < 1) return fail(CG_E_INVALID, "naxis must be >= 1");
  if (nchan < 1 || nchan > 65535) return fail(CG_E_INVALID, "nchan must be in [1, 65535]");
  if (!(wcs->cdelt1 != 0.0 && wcs->cdelt2 != 0.0 && isfinite(wcs->cdelt1) &&
        isfinite(wcs->cdelt2) && isfinite(wcs->crpix1) && isfinite(wcs->crpix2) &&
        isfinite(wcs->crval1) && isfinite(wcs->crval2)))
    return fail(CG_E_INVALID, "WCS keywords must be finite with non-zero CDELT");
  if (fabs(wcs->crval2) > 90.0) return fail(CG_E_INVALID, "|CRVAL2| > 90");
  const int64_t nt = wcs->naxis1 * wcs->naxis2;
  if (nt >= (1ll << 31) - 64) return fail(CG_E_UNSUPPORTED, "grid too large");
  cg_gridder* g = new_gridder();
  g->kind = 0;
  g->wcs.proj = wcs->proj;
  g->wcs.naxis1 = wcs->naxis1;
  g->wcs.naxis2 = wcs->naxis2;
  g->wcs.crpix1 = wcs->crpix1;
  g->wcs.crpix2 = wcs->crpix2;
  g->wcs.crval1 = wcs->crval1;
  g->wcs.crval2 = wcs->crval2;
  g->wcs.cdelt1 = wcs->cdelt1;
  g->wcs.cdelt2 = wcs->cdelt2;
  cg::wcs_set_pole(&g->wcs);
  g->ntarget = nt;
  g->nchan = nchan;
  g->ntx = (wcs->naxis1 + g->tile_w - 1) / g->tile_w;
  g->nty = (wcs->naxis2 + g->tile_h - 1) / g->tile_h;
  g->ntiles = g->ntx * g->nty;
  g->nslots = g->ntiles * cg::kTile;
  cg_status s = alloc_targets(g);
  if (s == CG_OK) {
    hipError_t e = cg::launch_wcs_targets(g->wcs, g->tile_w, g->tile_h, g->ntx, g->nslots,
                                          g->txyz.as<double>(), g->tll.as<double>(),
                                          g->slot_target.as<int32_t>(),
                                          g->target_slot.as<int32_t>(), nullptr);
    if (e == hipSuccess)
      e = cg::launch_tile_caps(g->txyz.as<double>(), g->nslots, g->ntiles, g->caps.as<double>(),
                               nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) s = hip_fail(e, "target setup");
  }
  if (s != CG_OK) {
    cg_destroy(g);
    return s;
  }
  *out = g;
  return CG_OK;
}

cg_status cg_create_sightlines(cg_gridder** out, const double* lon_deg, const double* lat_deg,
                               int64_t ntarget, int64_t nchan, void* stream) {
  if (!out) return fail(CG_E_INVALID, "null pointer");
  *out = nullptr;
  if (ntarget < 1) return fail(CG_E_INVALID, "ntarget must be >= 1");
  if (!lon_deg || !lat_deg) return fail(CG_E_INVALID, "null coordinate pointer");
  if (nchan < 1 || nchan > 65535) return fail(CG_E_INVALID, "nchan must be in [1, 65535]");
  if (ntarget >= (1ll << 31) - 64) return fail(CG_E_UNSUPPORTED, "too many targets");
  hipStream_t st = (hipStream_t)stream;
  cg_gridder* g = new_gridder();
  g->kind = 1;
  g->ntarget = ntarget;
  g->nchan = nchan;
  g->ntiles = (ntarget + cg::kTile - 1) / cg::kTile;
  g->nslots = g->ntiles * cg::kTile;
  cg_status s = alloc_targets(g);
  DevBuf k1, v1, k2, v2, h;
  if (s == CG_OK) {
    const Allocator& al = g->alloc;
    hipError_t e = ensure(al, k1, 4 * ntarget, st);
    if (e == hipSuccess) e = ensure(al, v1, 4 * ntarget, st);
    if (e == hipSuccess) e = ensure(al, k2, 4 * ntarget, st);
    if (e == hipSuccess) e = ensure(al, v2, 4 * ntarget, st);
    if (e == hipSuccess) e = ensure(al, h, 4 * cg::radix_hist_elems(ntarget), st);
    if (e == hipSuccess)
      e = cg::launch_sl_keys(lon_deg, lat_deg, ntarget, k1.as<uint32_t>(), v1.as<uint32_t>(),
                             g->flag.as<int>(), st);
    bool in_tmp = false;
    if (e == hipSuccess)
      e = cg::radix_sort(k1.as<uint32_t>(), v1.as<uint32_t>(), k2.as<uint32_t>(),
                         v2.as<uint32_t>(), h.as<uint32_t>(), ntarget,
                         bits_for((uint64_t)cg::hpx::npix(8192)), &in_tmp, st);
    if (e == hipSuccess)
      e = cg::launch_sl_targets(lon_deg, lat_deg, in_tmp ? v2.as<uint32_t>() : v1.as<uint32_t>(),
                                ntarget, g->nslots, g->txyz.as<double>(), g->tll.as<double>(),
                                g->slot_target.as<int32_t>(), g->target_slot.as<int32_t>(), st);
    if (e == hipSuccess)
      e = cg::launch_tile_caps(g->txyz.as<double>(), g->nslots, g->ntiles, g->caps.as<double>(),
                               st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) s = hip_fail(e, "sight-line setup");
  }
  k1.release(); v1.release(); k2.release(); v2.release(); h.release();
  if (s != CG_OK) {
    cg_destroy(g);
    return s;
  }
  *out = g;
  return CG_OK;
}

cg_status cg_create_healpix(cg_gridder** out, int64_t nside, int32_t order, int64_t nchan,
                            void* stream) {
  if (!out) return fail(CG_E_INVALID, "null pointer");
  *out = nullptr;
  if (order != CG_HPX_RING && order != CG_HPX_NESTED)
    return fail(CG_E_INVALID, "unknown pixel order %d", order);
  if (nside < 1 || nside > 8192 || (nside & (nside - 1)) != 0)
    return fail(CG_E_INVALID, "nside must be a power of two in [1, 8192]");
  if (nchan < 1 || nchan > 65535) return fail(CG_E_INVALID, "nchan must be in [1, 65535]");
  hipStream_t st = (hipStream_t)stream;
  const int64_t ntarget = cg::hpx::npix(nside);
  cg_gridder* g = new_gridder();
  g->kind = 1;
  g->ntarget = ntarget;
  g->nchan = nchan;
  g->ntiles = (ntarget + cg::kTile - 1) / cg::kTile;
  g->nslots = g->ntiles * cg::kTile;
  cg_status s = alloc_targets(g);
  DevBuf lon, lat, ord;
  if (s == CG_OK) {
    const Allocator& al = g->alloc;
    hipError_t e = ensure(al, lon, sizeof(double) * ntarget, st);
    if (e == hipSuccess) e = ensure(al, lat, sizeof(double) * ntarget, st);
    if (e == hipSuccess) e = ensure(al, ord, sizeof(uint32_t) * ntarget, st);
    if (e == hipSuccess)
      e = cg::launch_hpx_centres(nside, order == CG_HPX_NESTED, lon.as<double>(), lat.as<double>(),
                                 ord.as<uint32_t>(), st);
    if (e == hipSuccess)
      e = cg::launch_sl_targets(lon.as<double>(), lat.as<double>(), ord.as<uint32_t>(), ntarget,
                                g->nslots, g->txyz.as<double>(), g->tll.as<double>(),
                                g->slot_target.as<int32_t>(), g->target_slot.as<int32_t>(), st);
    if (e == hipSuccess)
      e = cg::launch_tile_caps(g->txyz.as<double>(), g->nslots, g->ntiles, g->caps.as<double>(),
                               st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) s = hip_fail(e, "HEALPix target setup");
  }
  lon.release(); lat.release(); ord.release();
  if (s != CG_OK) {
    cg_destroy(g);
    return s;
  }
  *out = g;
  return CG_OK;
}

cg_status cg_hpx_centres(int64_t nside, int32_t order, int64_t first, int64_t count,
                         double* lon_deg, double* lat_deg) {
  if (order != CG_HPX_RING && order != CG_HPX_NESTED)
    return fail(CG_E_INVALID, "unknown pixel order %d", order);
  if (nside < 1 || nside > 8192 || (nside & (nside - 1)) != 0)
    return fail(CG_E_INVALID, "nside must be a power of two in [1, 8192]");
  if (count < 0 || first < 0 || first + count > cg::hpx::npix(nside))
    return fail(CG_E_INVALID, "pixel range outside the map");
  if (count > 0 && (!lon_deg || !lat_deg)) return fail(CG_E_INVALID, "null output pointer");
  for (int64_t k = 0; k < count; ++k)
    cg::hpx::pix_centre(nside, first + k, order == CG_HPX_NESTED, lon_deg + k, lat_deg + k);
  return CG_OK;
}


cg_status cg_set_kernel(cg_gridder* g, int32_t kernel_type, const double* params, int32_t nparams,
                        double support_deg, double hpx_maxres_deg) {
  if (!g) return fail(CG_E_INVALID, "null handle");
  if (!params) return fail(CG_E_INVALID, "null params");
  // every argument is checked before the handle changes, so a rejected call
  // leaves the previous kernel (and its table) in force
  cg::KernelParams kp{};
  double smin = 0.0;   // narrowest Gaussian width (rad), 0 for a table
  if (kernel_type == CG_GAUSS1D) {
    if (nparams != 1) return fail(CG_E_INVALID, "gauss1d takes 1 parameter (sigma)");
    const double s = params[0] * kDeg;
    if (!(s > 0.0) || !isfinite(s)) return fail(CG_E_INVALID, "sigma must be > 0");
    smin = s;
    kp.type = 0;
    kp.k1 = kLog2e / (2.0 * s * s);
  } else if (kernel_type == CG_GAUSS2D) {
    if (nparams != 3) return fail(CG_E_INVALID, "gauss2d takes 3 parameters (sigma_maj, sigma_min, pa)");
    const double a = params[0] * kDeg, b = params[1] * kDeg, pa = params[2] * kDeg;
    if (!(a > 0.0 && b > 0.0) || !isfinite(a) || !isfinite(b) || !isfinite(pa))
      return fail(CG_E_INVALID, "sigmas must be > 0 and pa finite");
    if (b > a) return fail(CG_E_INVALID, "sigma_min must not exceed sigma_maj");
    smin = b;
    kp.type = 1;
    kp.kmaj = kLog2e / (2.0 * a * a);
    kp.kmin = kLog2e / (2.0 * b * b);
    kp.cospa = cos(pa);
    kp.sinpa = sin(pa);
  } else if (kernel_type == CG_TAPERED_SINC) {
    if (nparams != 2) return fail(CG_E_INVALID, "tapered sinc takes 2 parameters (sigma, b)");
    const double s = params[0] * kDeg, b = params[1] * kDeg;
    if (!(s > 0.0 && b > 0.0) || !isfinite(s) || !isfinite(b))
      return fail(CG_E_INVALID, "sigma and b must be > 0");
    smin = s;
    kp.type = 2;
    kp.k1 = kLog2e / (2.0 * s * s);
    kp.ks = cg::hpx::kPi / b;
  } else if (kernel_type == CG_TABLE) {
    if (nparams < 3 || nparams > 65537)
      return fail(CG_E_INVALID, "table takes dmax and 2 to 65536 values");
    const double dmax = params[0] * kDeg;
    if (!(dmax > 0.0) || !isfinite(dmax)) return fail(CG_E_INVALID, "dmax must be > 0");
    for (int32_t k = 1; k < nparams; ++k)
      if (!isfinite(params[k])) return fail(CG_E_INVALID, "table values must be finite");
    kp.type = 3;
    kp.ntab = nparams - 1;
    kp.tinv = (double)(nparams - 2) / dmax;
  } else {
    return fail(CG_E_INVALID, "unknown kernel type %d", kernel_type);
  }
  if (!(support_deg > 0.0 && support_deg < 90.0))
    return fail(CG_E_INVALID, "support must be in (0, 90) degrees");
  const double rs = support_deg * kDeg;
  // the base-2 exponent of a Gaussian weight inside the support then stays
  // below 1000^2 / 2 * log2(e), about 7.2e5, so its integer part fits an int
  if (smin > 0.0 && rs > 1000.0 * smin)
    return fail(CG_E_INVALID, "support must not exceed 1000 sigma (sigma_min for gauss2d)");
  const double c = 2.0 * sin(0.5 * rs);
  kp.cs2 = c * c;
  int64_t nside = g->nside;
  if (!g->nside_fixed) {
    if (!(hpx_maxres_deg > 0.0) || !isfinite(hpx_maxres_deg))
      return fail(CG_E_INVALID, "hpx_maxres must be > 0 (or fix nside with cg_set_nside)");
    const double res = hpx_maxres_deg * kDeg;
    nside = 1;
    while (nside < 8192 && sqrt(cg::hpx::kPi / 3.0) / (double)nside > res) nside *= 2;
  }
  if (kp.type == 3) {
    const cg_status sd = set_dev(g);
    if (sd != CG_OK) return sd;
    // the new table goes into a buffer of its own; the old one stays in
    // force (earlier grid calls may still read it) until the upload worked
    DevBuf tab;
    const size_t bytes = sizeof(double) * (size_t)kp.ntab;
    hipError_t e = g->alloc.get(tab, bytes);
    if (e == hipSuccess) e = hipMemcpy(tab.p, params + 1, bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();   // earlier grid calls are done with the old table
    if (e != hipSuccess) {
      tab.release();
      return hip_fail(e, "kernel table");
    }
    g->ktab.release();
    g->ktab = tab;
    kp.tab = g->ktab.as<double>();
  }
  g->kp = kp;
  g->support_rad = rs;
  g->nside = nside;
  g->kernel_set = true;
  g->span_valid = false;
  g->disk_valid = false;
  // the lookup tables of the targets for this support and nside
  const cg_status sd = set_dev(g);
  if (sd != CG_OK) return sd;
  return ensure_span(g, nullptr);
}


cg_status cg_set_lookup(cg_gridder* g, int32_t lookup) {
  if (!g) return fail(CG_E_INVALID, "null handle");
  if (lookup != CG_LOOKUP_TILES && lookup != CG_LOOKUP_DISK)
    return fail(CG_E_INVALID, "unknown lookup %d", lookup);
  g->lookup = lookup;
  g->have_ranges = false;
  return CG_OK;
}

cg_status cg_disk_stats(const cg_gridder* g, int64_t* pixels, int64_t* pairs) {
  if (!g || !pixels || !pairs) return fail(CG_E_INVALID, "null argument");
  *pixels = g->last_upix;
  *pairs = g->last_pairs;
  return CG_OK;
}

cg_status cg_set_nside(cg_gridder* g, int64_t nside) {
  if (!g) return fail(CG_E_INVALID, "null handle");
  if (nside < 1 || nside > 8192 || (nside & (nside - 1)) != 0)
    return fail(CG_E_INVALID, "nside must be a power of two in [1, 8192]");
  g->nside = nside;
  g->nside_fixed = true;
  g->span_valid = false;
  g->disk_valid = false;
  if (!g->kernel_set) return CG_OK;
  const cg_status s = set_dev(g);
  if (s != CG_OK) return s;
  return ensure_span(g, nullptr);
}

cg_status cg_set_output_layout(cg_gridder* g, int32_t layout) {
  if (!g) return fail(CG_E_INVALID, "null handle");
  if (layout != CG_LAYOUT_CHANNEL_MAJOR && layout != CG_LAYOUT_TARGET_MAJOR)
    return fail(CG_E_INVALID, "unknown layout %d", layout);
  g->layout = layout;
  return CG_OK;
}

cg_status cg_set_precision(cg_gridder* g, int32_t prec) {
  if (!g) return fail(CG_E_INVALID, "null handle");
  if (prec < CG_PREC_FP32 || prec > CG_PREC_FP16) return fail(CG_E_INVALID, "unknown precision %d", prec);
  if (prec != CG_PREC_FP32 && !cg::mfma_available())
    return fail(CG_E_UNSUPPORTED, "matrix-core contraction not built");
  g->prec = prec;
  return CG_OK;
}

cg_status cg_workspace_size(const cg_gridder* g, int64_t nsamples, size_t* bytes) {
  if (!g || !bytes) return fail(CG_E_INVALID, "null pointer");
  if (!g->kernel_set) return fail(CG_E_STATE, "set_kernel must be called first");
  if (nsamples < 0 || nsamples > 0xFFFFFFFFll - 1) return fail(CG_E_INVALID, "bad nsamples");
  *bytes = ws_bytes_for(g, nsamples);
  return CG_OK;
}

cg_status cg_grid(cg_gridder* g, const double* lon_deg, const double* lat_deg, const void* data,
                  int32_t dtype, int64_t nsamples, int64_t ld_data, void* ws, size_t ws_bytes,
                  void* stream) {
  cg_status s = check_grid_args(g, lon_deg, lat_deg, data, dtype, nsamples, ld_data);
  if (s != CG_OK || nsamples == 0) return s;
  if ((s = set_dev(g)) != CG_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char* base = nullptr;
  if ((s = call_workspace(g, nsamples, ws, ws_bytes, st, &base)) != CG_OK) return s;
  CG_HIP(ensure(g->alloc, g->S, sizeof(double) * g->nchan * g->nslots, st), "alloc accumulators");
  s = run_lookup(g, lon_deg, lat_deg, nsamples, data, dtype, ld_data, small_c(g), base, st);
  if (s != CG_OK) return s;
  cg::OutView ov{};
  ov.S = g->S.as<double>();
  ov.W = g->W.as<double>();
  ov.Wn = g->Wn.as<double>();
  ov.slot_target = g->slot_target.as<int32_t>();
  ov.ntarget = g->ntarget;
  ov.mode = g->fresh ? cg::ACC_OVERWRITE : cg::ACC_ADD;
  s = contract(g, data, dtype, ld_data, ov, st);
  if (s == CG_OK) g->fresh = false;
  return s;
}

cg_status cg_grid_datacube(cg_gridder* g, const double* lon_deg, const double* lat_deg,
                           const void* data, int32_t dtype, int64_t nsamples, int64_t ld_data,
                           float* cube_out, float* weights_out, void* ws, size_t ws_bytes,
                           void* stream) {
  cg_status s = check_grid_args(g, lon_deg, lat_deg, data, dtype, nsamples, ld_data);
  if (s != CG_OK) return s;
  if (!cube_out) return fail(CG_E_INVALID, "null cube_out");
  if ((s = set_dev(g)) != CG_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  g->fresh = true;
  if (nsamples == 0) return empty_datacube(g, cube_out, weights_out, st);
  char* base = nullptr;
  if ((s = call_workspace(g, nsamples, ws, ws_bytes, st, &base)) != CG_OK) return s;
  return grid_datacube_ws(g, lon_deg, lat_deg, data, dtype, nsamples, ld_data, cube_out,
                          weights_out, base, st);
}

cg_status cg_grid_datacube_noalloc(cg_gridder* g, const double* lon_deg, const double* lat_deg,
                                   const void* data, int32_t dtype, int64_t nsamples,
                                   int64_t ld_data, float* cube_out, float* weights_out,
                                   void* stream) {
  cg_status s = check_grid_args(g, lon_deg, lat_deg, data, dtype, nsamples, ld_data);
  if (s != CG_OK) return s;
  if (!cube_out) return fail(CG_E_INVALID, "null cube_out");
  if (g->lookup == CG_LOOKUP_DISK)
    return fail(CG_E_UNSUPPORTED, "the sample-centric lookup sizes its lists per call");
  if (!g->span_valid) return fail(CG_E_STATE, "lookup tables not built (set_kernel failed)");
  const size_t need = ws_bytes_for(g, nsamples);
  if (need > kScratchBytes)
    return fail(CG_E_WORKSPACE,
                "%lld samples need %zu bytes of scratch, the static scratch holds %zu "
                "(pass a workspace to cg_grid_datacube instead)",
                (long long)nsamples, need, kScratchBytes);
  if ((s = set_dev(g)) != CG_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  g->fresh = true;
  if (nsamples == 0) return empty_datacube(g, cube_out, weights_out, st);
  char* base = nullptr;
  if ((s = scratch_of(g->device, &base)) != CG_OK) return s;
  return grid_datacube_ws(g, lon_deg, lat_deg, data, dtype, nsamples, ld_data, cube_out,
                          weights_out, base, st, false);
}

cg_status cg_get_datacube(cg_gridder* g, float* out, void* stream) {
  if (!g) return fail(CG_E_INVALID, "null handle");
  if (!out) return fail(CG_E_INVALID, "null output");
  cg_status s = set_dev(g);
  if (s != CG_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (g->fresh) {
    CG_HIP(cg::launch_fill(out, g->nchan * g->ntarget, __builtin_nanf(""), st), "fill");
    return CG_OK;
  }
  int64_t cst, tst;
  cube_strides(g, &cst, &tst);
  CG_HIP(cg::launch_normalize(g->S.as<double>(), g->W.as<double>(), g->Wn.as<double>(),
                              g->target_slot.as<int32_t>(), g->nslots, g->nchan, g->ntarget, cst,
                              tst, out, nullptr, st),
         "normalize");
  return CG_OK;
}

cg_status cg_get_weights(cg_gridder* g, float* out, void* stream) {
  if (!g) return fail(CG_E_INVALID, "null handle");
  if (!out) return fail(CG_E_INVALID, "null output");
  cg_status s = set_dev(g);
  if (s != CG_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (g->fresh) {
    CG_HIP(cg::launch_fill(out, g->ntarget, 0.0f, st), "fill");
    return CG_OK;
  }
  CG_HIP(cg::launch_normalize(nullptr, g->W.as<double>(), g->Wn.as<double>(),
                              g->target_slot.as<int32_t>(), g->nslots, g->nchan, g->ntarget, 0, 1,
                              nullptr, out, st),
         "weights");
  return CG_OK;
}

cg_status cg_clear(cg_gridder* g, void* stream) {
  (void)stream;
  if (!g) return fail(CG_E_INVALID, "null handle");
  g->fresh = true;
  return CG_OK;
}

cg_status cg_sync(cg_gridder* g, void* stream) {
  if (!g) return fail(CG_E_INVALID, "null handle");
  cg_status s = set_dev(g);
  if (s != CG_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  CG_HIP(hipStreamSynchronize(st), "sync");
  int f = 0;
  CG_HIP(hipMemcpy(&f, g->flag.p, sizeof(int), hipMemcpyDeviceToHost), "read flag");
  if (f) {
    CG_HIP(hipMemset(g->flag.p, 0, sizeof(int)), "clear flag");
    return fail(CG_E_INPUT, "input contained non-finite coordinates or |lat| > 90 (skipped)");
  }
  return CG_OK;
}

cg_status cg_neighbour_stats(cg_gridder* g, const double* lon_deg, const double* lat_deg,
                             int64_t nsamples, int32_t* counts, uint64_t* hashes, void* stream) {
  if (!g) return fail(CG_E_INVALID, "null handle");
  if (!g->kernel_set) return fail(CG_E_STATE, "set_kernel must be called first");
  if (!counts) return fail(CG_E_INVALID, "null counts");
  if (nsamples < 0 || nsamples > 0xFFFFFFFFll - 1) return fail(CG_E_INVALID, "bad nsamples");
  cg_status s = set_dev(g);
  if (s != CG_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (nsamples == 0) {
    CG_HIP(cg::launch_fill(reinterpret_cast<float*>(counts), g->ntarget, 0.0f, st), "clear counts");
    if (hashes)
      CG_HIP(cg::launch_fill(reinterpret_cast<float*>(hashes), 2 * g->ntarget, 0.0f, st),
             "clear hashes");
    return CG_OK;
  }
  if (!lon_deg || !lat_deg) return fail(CG_E_INVALID, "null coordinate pointer");
  const size_t need = workspace_layout(nsamples, g->nside, 0, nullptr, nullptr);
  CG_HIP(ensure(g->alloc, g->own_ws, need, st), "alloc workspace");
  s = run_lookup(g, lon_deg, lat_deg, nsamples, nullptr, CG_F32, g->nchan, false,
                 g->own_ws.as<char>(), st);
  if (s != CG_OK) return s;
  CG_HIP(cg::launch_stats(tile_view(g), g->kp, g->slot_target.as<int32_t>(), counts, hashes, st),
         "stats");
  return CG_OK;
}

cg_status cg_query(const cg_gridder* g, int32_t what, int64_t* value) {
  if (!g || !value) return fail(CG_E_INVALID, "null pointer");
  switch (what) {
    case 0: *value = g->ntarget; break;
    case 1: *value = g->nchan; break;
    case 2: *value = g->nside; break;
    case 3: *value = g->ntiles; break;
    case 4: {
      // candidates of the last lookup: waits for the device and sums the
      // per-tile counts
      *value = 0;
      if (!g->have_ranges || g->ntiles <= 0) break;
      CG_HIP(hipSetDevice(g->device), "hipSetDevice");
      std::vector<uint64_t> c((size_t)g->ntiles);
      CG_HIP(hipDeviceSynchronize(), "sync");
      CG_HIP(hipMemcpy(c.data(), g->ncand.p, sizeof(uint64_t) * c.size(), hipMemcpyDeviceToHost),
             "read candidates");
      uint64_t t = 0;
      for (uint64_t v : c) t += v;
      *value = (int64_t)t;
      break;
    }
    case 5: *value = g->prec; break;
    case 6: *value = g->device; break;
    case 7: *value = g->layout; break;
    default: return fail(CG_E_INVALID, "unknown query %d", what);
  }
  return CG_OK;
}

cg_status cg_profile_enable(cg_gridder* g, int32_t enable) {
  if (!g) return fail(CG_E_INVALID, "null handle");
  g->prof = enable != 0;
  if (g->prof) g->nev = 0;
  return CG_OK;
}

cg_status cg_profile_read(cg_gridder* g, int64_t* launches, double* total_ms) {
  if (!g || !launches || !total_ms) return fail(CG_E_INVALID, "null pointer");
  cg_status s = set_dev(g);
  if (s != CG_OK) return s;
  double tot = 0.0;
  for (size_t i = 0; i < g->nev; ++i) {
    CG_HIP(hipEventSynchronize(g->ev[i].second), "event sync");
    float ms = 0.0f;
    CG_HIP(hipEventElapsedTime(&ms, g->ev[i].first, g->ev[i].second), "event time");
    tot += ms;
  }
  *launches = (int64_t)g->nev;
  *total_ms = tot;
  return CG_OK;
}

void cg_destroy(cg_gridder* g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  for (auto& e : g->ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  destroy_buffers(g);
  if (g->h_word) (void)hipHostFree(g->h_word);
  delete g;
}

// ------------------------------------------------------------ host helpers

cg_status cg_hpx_ang2pix_ring(int64_t nside, int64_t n, const double* lon_deg,
                              const double* lat_deg, int64_t* out) {
  if (nside < 1 || nside > 8192 || n < 0 || (n > 0 && (!lon_deg || !lat_deg || !out)))
    return fail(CG_E_INVALID, "bad arguments");
  for (int64_t i = 0; i < n; ++i) {
    double am = fmod(lon_deg[i], 360.0);
    if (am < 0.0) am += 360.0;
    const double d = lat_deg[i] * kDeg;
    out[i] = cg::hpx::ang2pix_ring(nside, sin(d), cos(d), am * kDeg);
  }
  return CG_OK;
}

cg_status cg_hpx_pix2ang_ring(int64_t nside, int64_t n, const int64_t* pix, double* out_lon,
                              double* out_lat) {
  if (nside < 1 || nside > 8192 || n < 0 || (n > 0 && (!pix || !out_lon || !out_lat)))
    return fail(CG_E_INVALID, "bad arguments");
  for (int64_t i = 0; i < n; ++i) {
    if (pix[i] < 0 || pix[i] >= cg::hpx::npix(nside)) return fail(CG_E_INVALID, "pixel out of range");
    double z, phi;
    cg::hpx::pix2ang_ring(nside, pix[i], &z, &phi);
    out_lon[i] = phi / kDeg;
    out_lat[i] = asin(z) / kDeg;
  }
  return CG_OK;
}

cg_status cg_hpx_pix2ring(int64_t nside, int64_t n, const int64_t* pix, int64_t* ring,
                          int64_t* j) {
  if (nside < 1 || nside > 8192 || n < 0 || (n > 0 && (!pix || !ring || !j)))
    return fail(CG_E_INVALID, "bad arguments");
  for (int64_t i = 0; i < n; ++i) {
    if (pix[i] < 0 || pix[i] >= cg::hpx::npix(nside)) return fail(CG_E_INVALID, "pixel out of range");
    cg::hpx::pix2ring(nside, pix[i], &ring[i], &j[i]);
  }
  return CG_OK;
}

cg_status cg_hpx_ring_info(int64_t nside, int64_t i, int64_t* start, int64_t* npix, double* z) {
  if (nside < 1 || nside > 8192 || i < 1 || i > 4 * nside - 1 || !start || !npix || !z)
    return fail(CG_E_INVALID, "bad arguments");
  *start = cg::hpx::ring_start(nside, i);
  *npix = cg::hpx::ring_npix(nside, i);
  *z = cg::hpx::ring_z(nside, i);
  return CG_OK;
}

cg_status cg_hpx_cap_ranges(int64_t nside, double lon_deg, double lat_deg, double rho_deg,
                            int64_t* ranges, int64_t max_ranges, int64_t* nranges) {
  if (nside < 1 || nside > 8192 || !ranges || !nranges || !(rho_deg >= 0.0))
    return fail(CG_E_INVALID, "bad arguments");
  const double d = lat_deg * kDeg;
  double am = fmod(lon_deg, 360.0);
  if (am < 0.0) am += 360.0;
  const double cz = sin(d), cs = cos(d), cphi = am * kDeg, rho = rho_deg * kDeg;
  int64_t f, l;
  cg::hpx::cap_ring_span(nside, cz, cs, rho, &f, &l);
  int64_t k = 0;
  for (int64_t i = f; i <= l; ++i) {
    int64_t lo[2], hi[2];
    const int nr = cg::hpx::ring_cap_ranges(nside, i, cz, cs, cphi, rho, lo, hi);
    for (int q = 0; q < nr; ++q) {
      if (k >= max_ranges) return fail(CG_E_INVALID, "max_ranges too small");
      ranges[2 * k] = lo[q];
      ranges[2 * k + 1] = hi[q];
      ++k;
    }
  }
  *nranges = k;
  return CG_OK;
}

cg_status cg_hpx_query_disk(int64_t nside, int64_t pix, double support_deg, int64_t* ranges,
                            int64_t max_ranges, int64_t* nranges) {
  if (nside < 1 || nside > 8192 || (nside & (nside - 1)) != 0 || pix < 0 ||
      pix >= cg::hpx::npix(nside) || !ranges || !nranges || !(support_deg > 0.0) ||
      !(support_deg < 90.0))
    return fail(CG_E_INVALID, "bad arguments");
  const double rs = support_deg * kDeg;
  const int64_t reach = cg::hpx::disk_ring_reach(nside, rs);
  int64_t i, j;
  cg::hpx::pix2ring(nside, pix, &i, &j);
  const int64_t n1 = cg::hpx::ring_npix(nside, i);
  const int64_t k = j - cg::hpx::ring_ref_pixel(nside, i);
  int64_t m = 0;
  for (int64_t i2 = i - reach; i2 <= i + reach; ++i2) {
    if (i2 < 1 || i2 >= 4 * nside) continue;
    const int64_t n2 = cg::hpx::ring_npix(nside, i2);
    int64_t lo = 0, hi = 0, a[2], b[2];
    const int r = cg::hpx::ref_disk_window(nside, i, i2, rs, &lo, &hi);
    if (r == 0) continue;
    int nr = 1;
    if (r == 2) {
      a[0] = cg::hpx::ring_start(nside, i2);
      b[0] = a[0] + n2 - 1;
    } else {
      nr = cg::hpx::shifted_window(nside, i2, lo, hi, cg::hpx::disk_shift(k, n2, n1), a, b);
    }
    for (int q = 0; q < nr; ++q) {
      if (m >= max_ranges) return fail(CG_E_INVALID, "max_ranges too small");
      ranges[2 * m] = a[q];
      ranges[2 * m + 1] = b[q];
      ++m;
    }
  }
  *nranges = m;
  return CG_OK;
}

cg_status cg_hpx_targets_ranges(int64_t nside, int64_t n, const double* lon_deg,
                                const double* lat_deg, double rho_deg, int64_t* ranges,
                                int64_t max_ranges, int64_t* nranges) {
  if (nside < 1 || nside > 8192 || n < 1 || n > 4096 || !lon_deg || !lat_deg || !ranges ||
      !nranges || !(rho_deg >= 0.0))
    return fail(CG_E_INVALID, "bad arguments");
  const double rho = rho_deg * kDeg;
  std::vector<cg::hpx::DiskPrep> d((size_t)n);
  std::vector<double> rel((size_t)n);
  // reference longitude: the first point's
  double ref = 0.0;
  int64_t f = 4 * nside, l = 0;
  for (int64_t k = 0; k < n; ++k) {
    double am = fmod(lon_deg[k], 360.0);
    if (am < 0.0) am += 360.0;
    const double phi = am * kDeg, la = lat_deg[k] * kDeg;
    if (k == 0) ref = phi;
    cg::hpx::disk_prepare(sin(la), cos(la), rho, &d[(size_t)k]);
    rel[(size_t)k] = cg::hpx::rel_lon(phi, ref);
    int64_t a, b;
    cg::hpx::cap_ring_span(nside, sin(la), cos(la), rho, &a, &b);
    if (a < f) f = a;
    if (b > l) l = b;
  }
  int64_t k = 0;
  for (int64_t i = f; i <= l; ++i) {
    double plo, phi;
    int full;
    if (!cg::hpx::ring_union_window(nside, i, d.data(), rel.data(), (int)n, ref, &plo, &phi, &full))
      continue;
    int64_t lo[2], hi[2];
    const int nr = cg::hpx::ring_window_ranges(nside, i, plo, phi, full, lo, hi);
    for (int q = 0; q < nr; ++q) {
      if (k >= max_ranges) return fail(CG_E_INVALID, "max_ranges too small");
      ranges[2 * k] = lo[q];
      ranges[2 * k + 1] = hi[q];
      ++k;
    }
  }
  *nranges = k;
  return CG_OK;
}

cg_status cg_wcs_pix2world(const cg_wcs* wcs, int64_t n, const double* i, const double* j,
                           double* lon_deg, double* lat_deg) {
  if (!wcs || n < 0 || (n > 0 && (!i || !j || !lon_deg || !lat_deg)))
    return fail(CG_E_INVALID, "bad arguments");
  if (wcs->proj != CG_PROJ_CAR && wcs->proj != CG_PROJ_SIN && wcs->proj != CG_PROJ_SFL &&
      wcs->proj != CG_PROJ_ZEA)
    return fail(CG_E_UNSUPPORTED, "unknown projection");
  if (!(fabs(wcs->crval2) <= 90.0)) return fail(CG_E_INVALID, "|CRVAL2| > 90");
  cg::WcsDev w;
  w.proj = wcs->proj;
  w.naxis1 = wcs->naxis1;
  w.naxis2 = wcs->naxis2;
  w.crpix1 = wcs->crpix1;
  w.crpix2 = wcs->crpix2;
  w.crval1 = wcs->crval1;
  w.crval2 = wcs->crval2;
  w.cdelt1 = wcs->cdelt1;
  w.cdelt2 = wcs->cdelt2;
  cg::wcs_set_pole(&w);
  for (int64_t k = 0; k < n; ++k) {
    double lo, la;
    if (cg::wcs_pix2world(w, i[k], j[k], &lo, &la)) {
      lon_deg[k] = lo;
      lat_deg[k] = la;
    } else {
      lon_deg[k] = lat_deg[k] = __builtin_nan("");
    }
  }
  return CG_OK;
}

}  // extern "C"
