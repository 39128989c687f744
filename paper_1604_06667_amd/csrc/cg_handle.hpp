// Host-side state of a gridder handle and the helpers shared by the C ABI
// translation units (argument errors, device buffers, set-up launches).
#pragma once
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/cg.h"
#include "cg_internal.hpp"

namespace cgh {

inline thread_local std::string g_err;

inline cg_status fail(cg_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

inline cg_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(CG_E_OOM, "%s: out of device memory", what);
  return fail(CG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define CG_HIP(call, what)                          \
  do {                                              \
    hipError_t e_ = (call);                         \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

inline hipError_t ensure(DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 1;
  if (b.bytes >= bytes) return hipSuccess;
  b.release();
  // grow geometrically so that slowly growing inputs do not reallocate every call
  const size_t want = bytes + bytes / 8;
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return e;
  }
  b.bytes = want;
  return hipSuccess;
}

constexpr double kDeg = cg::hpx::kPi / 180.0;
constexpr double kLog2e = 1.44269504088896340736;

inline int bits_for(uint64_t v) {
  int b = 0;
  while (b < 32 && (1ull << b) <= v) ++b;
  return b;
}

}  // namespace cgh

struct cg_gridder {
  int device = 0;
  int kind = 0;  // 0 WCS grid, 1 sight lines
  cg::WcsDev wcs{};
  int64_t ntarget = 0, nchan = 0;
  int64_t tile_w = 8, tile_h = 8, ntx = 0, nty = 0, ntiles = 0, nslots = 0;
  cgh::DevBuf txyz, tll, slot_target, target_slot, caps;
  bool kernel_set = false;
  cg::KernelParams kp{};
  double support_rad = 0.0;
  int64_t nside = 0;
  bool nside_fixed = false;
  int prec = CG_PREC_FP32;
  int layout = CG_LAYOUT_CHANNEL_MAJOR;   // of the cubes written by this handle
  bool span_valid = false;
  cgh::DevBuf ring_first, span_bound, range_off, win;
  int64_t total_ranges = 0;
  cgh::DevBuf S, W, Wn;
  bool fresh = true;
  cgh::DevBuf flag;
  cgh::DevBuf zrow;   // nchan zeros of the widest data type
  cgh::DevBuf rec;   // per-sample record in input order (unit vector, narrow data)
  cgh::DevBuf ktab;  // tabulated kernel profile (CG_TABLE)
  cgh::DevBuf keys, vals, keys2, vals2, hist, ring_off, sx, sdata, ranges, nranges, ncand, cand_off,
      cand, crow, cxyz;
  const uint32_t* sorted_keys = nullptr;
  const uint32_t* sorted_vals = nullptr;
  int64_t last_n = 0;
  int64_t last_ncand = 0;
  int64_t ncap = 1;
  // sample-centric lookup (query disks shifted along rings)
  int lookup = CG_LOOKUP_TILES;
  bool disk_valid = false;
  int64_t disk_reach = 0;
  cgh::DevBuf dk_tkeys, dk_tvals, dk_tkeys2, dk_tvals2, dk_thist, dk_troff, dk_tab;
  const uint32_t* dk_tk = nullptr;   // targets sorted by pixel: keys, slots
  const uint32_t* dk_ts = nullptr;
  cgh::DevBuf dk_flag, dk_uoff, dk_upix, dk_ustart, dk_cnt, dk_off, dk_pk, dk_pv, dk_pk2, dk_pv2,
      dk_phist, dk_rsx, dk_ranges, dk_range_off, dk_scan;
  int64_t last_pairs = 0, last_upix = 0;
  uint64_t* h_word = nullptr;  // pinned host word
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t nev = 0;
};

namespace cgh {

inline cg_status set_dev(const cg_gridder* g) {
  CG_HIP(hipSetDevice(g->device), "hipSetDevice");
  return CG_OK;
}

inline cg_status alloc_targets(cg_gridder* g) {
  CG_HIP(ensure(g->txyz, sizeof(double) * 3 * g->nslots), "alloc targets");
  CG_HIP(ensure(g->tll, sizeof(double) * 2 * g->nslots), "alloc targets");
  CG_HIP(ensure(g->slot_target, sizeof(int32_t) * g->nslots), "alloc targets");
  CG_HIP(ensure(g->target_slot, sizeof(int32_t) * (g->ntarget > 0 ? g->ntarget : 1)),
         "alloc targets");
  CG_HIP(ensure(g->caps, sizeof(double) * 4 * (g->ntiles > 0 ? g->ntiles : 1)), "alloc caps");
  CG_HIP(ensure(g->W, sizeof(double) * g->nslots), "alloc weights");
  CG_HIP(ensure(g->Wn, sizeof(double) * g->nslots), "alloc weights");
  CG_HIP(ensure(g->flag, sizeof(int)), "alloc flag");
  CG_HIP(hipMemset(g->flag.p, 0, sizeof(int)), "clear flag");
  CG_HIP(ensure(g->zrow, sizeof(double) * g->nchan), "alloc zero row");
  CG_HIP(hipMemset(g->zrow.p, 0, sizeof(double) * g->nchan), "clear zero row");
  CG_HIP(hipHostMalloc((void**)&g->h_word, sizeof(uint64_t) * 2, hipHostMallocDefault),
         "pinned word");
  return CG_OK;
}

// Ring spans and range-slot offsets of the tiles: depend on targets, support
// and nside only, so they are computed once per set_kernel.
inline cg_status ensure_span(cg_gridder* g, hipStream_t st) {
  if (g->span_valid) return CG_OK;
  const int64_t nt = g->ntiles;
  CG_HIP(ensure(g->ring_first, sizeof(int32_t) * (nt > 0 ? nt : 1)), "alloc span");
  CG_HIP(ensure(g->span_bound, sizeof(uint64_t) * (nt > 0 ? nt : 1)), "alloc span");
  CG_HIP(ensure(g->range_off, sizeof(uint64_t) * (nt + 1)), "alloc span");
  const double rho_extra = g->support_rad + 1e-9;
  CG_HIP(cg::launch_tile_span(g->caps.as<double>(), nt, g->nside, rho_extra,
                              g->ring_first.as<int32_t>(), g->span_bound.as<uint64_t>(), st),
         "tile span");
  CG_HIP(cg::scan_u64(g->span_bound.as<uint64_t>(), g->range_off.as<uint64_t>(), nt, st),
         "scan span");
  CG_HIP(hipMemcpyAsync(g->h_word, g->range_off.as<uint64_t>() + nt, sizeof(uint64_t),
                        hipMemcpyDeviceToHost, st),
         "read span");
  CG_HIP(hipStreamSynchronize(st), "sync span");
  g->total_ranges = (int64_t)g->h_word[0];
  CG_HIP(ensure(g->ranges, sizeof(uint32_t) * 2 * (g->total_ranges > 0 ? g->total_ranges : 1)),
         "alloc ranges");
  CG_HIP(ensure(g->nranges, sizeof(uint32_t) * (nt > 0 ? nt : 1)), "alloc ranges");
  CG_HIP(ensure(g->ncand, sizeof(uint64_t) * (nt > 0 ? nt : 1)), "alloc ranges");
  CG_HIP(ensure(g->cand_off, sizeof(uint64_t) * (nt + 1)), "alloc ranges");
  CG_HIP(ensure(g->win, sizeof(uint32_t) * 2 * (g->total_ranges > 0 ? g->total_ranges : 1)),
         "alloc windows");
  CG_HIP(cg::launch_tile_windows(g->caps.as<double>(), g->txyz.as<double>(), g->nslots, nt,
                                 g->nside, g->support_rad + 1e-9, g->ring_first.as<int32_t>(),
                                 g->range_off.as<uint64_t>(), g->win.as<uint32_t>(), st),
         "tile windows");
  g->span_valid = true;
  return CG_OK;
}

// element strides (channel, target) of a cube in the handle's layout
inline void cube_strides(const cg_gridder* g, int64_t* cst, int64_t* tst) {
  if (g->layout == CG_LAYOUT_TARGET_MAJOR) {
    *cst = 1;
    *tst = g->nchan;
  } else {
    *cst = g->ntarget;
    *tst = 1;
  }
}
}  // namespace cgh
