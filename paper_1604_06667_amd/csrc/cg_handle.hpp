// Host-side state of a gridder handle and the helpers shared by the C ABI
// translation units (argument errors, device memory, workspace layout,
// set-up launches).
#pragma once
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
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

struct Allocator;

// Device memory owned by a handle.  It remembers the allocator that gave it
// (the handle's), so release() returns it there.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  const Allocator* al = nullptr;
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
  void release();
};

// Where a handle's device memory comes from: the caller's functions set with
// cg_set_allocator (captured when the handle is created), else hipMalloc /
// hipFree.  Memory is handed back only after the device has finished the
// work queued so far (hipFree waits by itself; a caller's free function is
// preceded by a device synchronisation), so an allocator that reuses memory
// at once (a caching allocator) never sees it while a kernel still reads it.
struct Allocator {
  cg_alloc_fn fa = nullptr;
  cg_free_fn ff = nullptr;
  void* ctx = nullptr;
  int device = 0;

  hipError_t get(DevBuf& b, size_t bytes, hipStream_t st = nullptr) const {
    b.p = nullptr;
    b.bytes = 0;
    b.al = this;
    if (bytes == 0) bytes = 1;
    if (fa) {
      void* p = fa(bytes, device, (void*)st, ctx);
      if (!p) return hipErrorOutOfMemory;
      b.p = p;
    } else {
      hipError_t e = hipMalloc(&b.p, bytes);
      if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return e;
      }
    }
    b.bytes = bytes;
    return hipSuccess;
  }
  void put(DevBuf& b) const {
    if (b.p) {
      if (ff) {
        (void)hipDeviceSynchronize();
        ff(b.p, b.bytes, device, ctx);
      } else {
        (void)hipFree(b.p);
      }
    }
    b.p = nullptr;
    b.bytes = 0;
  }
};

inline void DevBuf::release() {
  if (p && al) al->put(*this);
  p = nullptr;
  bytes = 0;
}

// Grow a buffer to at least `bytes` (geometrically, so that slowly growing
// inputs do not reallocate every call); its contents are not kept.
inline hipError_t ensure(const Allocator& al, DevBuf& b, size_t bytes, hipStream_t st = nullptr) {
  if (bytes == 0) bytes = 1;
  if (b.p && b.bytes >= bytes) return hipSuccess;
  b.release();
  return al.get(b, bytes + bytes / 8, st);
}

// The process-wide allocator of cg_set_allocator (NULL functions: hipMalloc).
struct GlobalAllocator {
  std::mutex mu;
  cg_alloc_fn fa = nullptr;
  cg_free_fn ff = nullptr;
  void* ctx = nullptr;
};
inline GlobalAllocator& global_allocator() {
  static GlobalAllocator a;
  return a;
}
inline Allocator current_allocator(int device) {
  GlobalAllocator& g = global_allocator();
  std::lock_guard<std::mutex> lk(g.mu);
  Allocator a;
  a.fa = g.fa;
  a.ff = g.ff;
  a.ctx = g.ctx;
  a.device = device;
  return a;
}

constexpr double kDeg = cg::hpx::kPi / 180.0;
constexpr double kLog2e = 1.44269504088896340736;

inline int bits_for(uint64_t v) {
  int b = 0;
  while (b < 32 && (1ull << b) <= v) ++b;
  return b;
}

// The per-call scratch of a grid call, carved from one workspace (the
// caller's or the handle's own): HEALPix keys and sample indices with their
// sort buffers and histogram, the ring offsets, the per-sample records of
// the prep step (input order) and of the sorted samples (unit vector and
// input row) and, for narrow FP32 grids, the sorted data rows.  Every piece
// starts on a 256-byte boundary.
struct Workspace {
  uint32_t *keys = nullptr, *vals = nullptr, *keys2 = nullptr, *vals2 = nullptr;
  uint32_t *hist = nullptr, *ring_off = nullptr;
  double *srec = nullptr, *rec = nullptr;
  float* sdata = nullptr;
};

// Bytes of the workspace for n samples; with base != NULL also the pieces.
inline size_t workspace_layout(int64_t n, int64_t nside, int64_t sdata_chan, char* base,
                               Workspace* w) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return p;
  };
  const size_t un = (size_t)(n > 0 ? n : 1);
  Workspace ws;
  ws.keys = (uint32_t*)take(4 * un);
  ws.vals = (uint32_t*)take(4 * un);
  ws.keys2 = (uint32_t*)take(4 * un);
  ws.vals2 = (uint32_t*)take(4 * un);
  ws.hist = (uint32_t*)take(4 * cg::radix_hist_elems((int64_t)un));
  ws.ring_off = (uint32_t*)take(4 * (size_t)(4 * nside + 1));
  ws.srec = (double*)take(32 * un);
  ws.rec = (double*)take(32 * un);
  if (sdata_chan > 0) ws.sdata = (float*)take(4 * un * (size_t)sdata_chan);
  if (w) *w = ws;
  return off;
}

}  // namespace cgh

struct cg_gridder {
  int device = 0;
  cgh::Allocator alloc;   // where every buffer of this handle comes from
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
  // lookup tables of the targets (set-up): ring spans and pixel windows per
  // tile, and room for the ranges a grid call finds in them
  bool span_valid = false;
  cgh::DevBuf ring_first, span_bound, range_off, win, ranges, nranges, ncand;
  int64_t total_ranges = 0;
  // accumulators of cg_grid: S (FP64, [nchan][nslots]), W, W' (FP64)
  cgh::DevBuf S, W, Wn;
  bool fresh = true;
  cgh::DevBuf flag;
  cgh::DevBuf zrow;   // nchan zeros of the widest data type
  cgh::DevBuf ktab;   // tabulated kernel profile (CG_TABLE)
  cgh::DevBuf own_ws; // the handle's own workspace (calls without a caller workspace)
  cgh::Workspace ws;  // pieces of the workspace of the current call
  const uint32_t* sorted_keys = nullptr;
  const uint32_t* sorted_vals = nullptr;
  int64_t last_n = 0;
  bool have_ranges = false;   // ncand holds the counts of a finished lookup
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
  const Allocator& al = g->alloc;
  CG_HIP(ensure(al, g->txyz, sizeof(double) * 3 * g->nslots), "alloc targets");
  CG_HIP(ensure(al, g->tll, sizeof(double) * 2 * g->nslots), "alloc targets");
  CG_HIP(ensure(al, g->slot_target, sizeof(int32_t) * g->nslots), "alloc targets");
  CG_HIP(ensure(al, g->target_slot, sizeof(int32_t) * (g->ntarget > 0 ? g->ntarget : 1)),
         "alloc targets");
  CG_HIP(ensure(al, g->caps, sizeof(double) * 4 * (g->ntiles > 0 ? g->ntiles : 1)), "alloc caps");
  CG_HIP(ensure(al, g->W, sizeof(double) * g->nslots), "alloc weights");
  CG_HIP(ensure(al, g->Wn, sizeof(double) * g->nslots), "alloc weights");
  CG_HIP(ensure(al, g->flag, sizeof(int)), "alloc flag");
  CG_HIP(hipMemset(g->flag.p, 0, sizeof(int)), "clear flag");
  CG_HIP(ensure(al, g->zrow, sizeof(double) * g->nchan), "alloc zero row");
  CG_HIP(hipMemset(g->zrow.p, 0, sizeof(double) * g->nchan), "clear zero row");
  const int64_t nt = g->ntiles > 0 ? g->ntiles : 1;
  CG_HIP(ensure(al, g->nranges, sizeof(uint32_t) * nt), "alloc ranges");
  CG_HIP(ensure(al, g->ncand, sizeof(uint64_t) * nt), "alloc ranges");
  CG_HIP(hipHostMalloc((void**)&g->h_word, sizeof(uint64_t) * 2, hipHostMallocDefault),
         "pinned word");
  return CG_OK;
}

// Ring spans, range-slot offsets and pixel windows of the tiles: they depend
// on the targets, the support and nside only, so they are computed once per
// set_kernel / set_nside (and waited for here), and every grid call after
// that reuses them without allocating.
inline cg_status ensure_span(cg_gridder* g, hipStream_t st) {
  if (g->span_valid) return CG_OK;
  const Allocator& al = g->alloc;
  const int64_t nt = g->ntiles;
  CG_HIP(ensure(al, g->ring_first, sizeof(int32_t) * (nt > 0 ? nt : 1)), "alloc span");
  CG_HIP(ensure(al, g->span_bound, sizeof(uint64_t) * (nt > 0 ? nt : 1)), "alloc span");
  CG_HIP(ensure(al, g->range_off, sizeof(uint64_t) * (nt + 1)), "alloc span");
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
  const size_t nr = (size_t)(g->total_ranges > 0 ? g->total_ranges : 1);
  CG_HIP(ensure(al, g->ranges, sizeof(uint32_t) * 2 * nr), "alloc ranges");
  CG_HIP(ensure(al, g->win, sizeof(uint32_t) * 2 * nr), "alloc windows");
  CG_HIP(cg::launch_tile_windows(g->caps.as<double>(), g->txyz.as<double>(), g->nslots, nt,
                                 g->nside, g->support_rad + 1e-9, g->ring_first.as<int32_t>(),
                                 g->range_off.as<uint64_t>(), g->win.as<uint32_t>(), st),
         "tile windows");
  CG_HIP(hipStreamSynchronize(st), "sync windows");
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
