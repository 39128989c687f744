// Internal declarations shared by the HIP translation units of libcg.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "healpix.hpp"
#include "wcs.hpp"

namespace cg {

constexpr int kTile = 64;              // targets per tile (one wavefront of target slots)
constexpr int kSmallC = 16;            // up to this many channels the FP32 path stages sorted rows
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;         // keys per thread per radix block
constexpr int kSortTile = kSortThreads * kSortItems;

// Kernel constants derived on the host by set_kernel.
struct KernelParams {
  int type;          // 0 gauss1d, 1 gauss2d, 2 tapered sinc, 3 tabulated radial profile
  double cs2;        // squared chord of the support radius: d <= r_s  <=>  c^2 <= cs2
  double k1;         // gauss1d, tapered sinc: log2(e) / (2 sigma^2)   (base-2 exponent per rad^2)
  double kmaj, kmin; // gauss2d: log2(e) / (2 sigma_maj^2), log2(e) / (2 sigma_min^2)
  double cospa, sinpa;
  double ks;         // tapered sinc: pi / b (per rad)
  const double* tab; // tabulated profile: ntab values at d = k / tinv (device memory)
  int ntab;
  double tinv;       // (ntab - 1) / dmax (per rad)
};

// Device-side description of the tiles' candidates and target slots.  The
// candidates of tile t are the concatenation of its nr[t] ranges of sorted
// samples: range k (0 <= k < nr[t]) sits at rng[2 (roff[t] + k)] = first
// sorted position and rng[2 (roff[t] + k) + 1] = its first candidate index
// within the tile (the exclusive prefix of the range lengths); the tile
// holds ntot[t] candidates.  Kernels walk the ranges directly (RangeWindow),
// so no per-candidate list is materialised and nothing about a grid call's
// memory depends on the data.
struct TileView {
  const double* txyz;          // [3][nslots] target unit vectors (NaN: no target)
  const double* tll;           // [2][nslots] target lon, lat in radians (gauss2d axes)
  const uint32_t* rng;         // ranges (first position, first candidate index)
  const uint64_t* roff;        // [ntiles] offset of each tile's ranges in rng (in ranges)
  const uint32_t* nr;          // [ntiles] ranges per tile
  const uint64_t* ntot;        // [ntiles] candidates per tile
  int64_t nslots;
  int64_t ntiles;
  int64_t ntx;                 // tiles per row of a WCS grid (0: sight lines)
  // the sorted samples the ranges point into: one 32-byte record each, the
  // unit vector and (as the bits of the fourth double) the sample's row,
  // i.e. its index in the caller's input (in a batch, the job's input)
  const double4* srec;
};

// input row of a sorted sample record
__device__ __forceinline__ int64_t rec_row(const double4& r) { return __double_as_longlong(r.w); }

// Block -> tile map that keeps consecutive tiles on one XCD: workgroups are
// dispatched to the 8 XCDs round robin, so block b runs on XCD b % 8; XCD k
// is given the k-th contiguous run of tiles, walked in order, so that tiles
// sharing candidate samples are resident together in that XCD's L2.
constexpr int kNumXcd = 8;

// Accesses through a pointer that addresses device global memory.  With GL
// set the pointer is cast to the global address space first: pointers read
// from memory (a job table) have no known address space, and the compiler
// would otherwise issue flat accesses, which also wait on the LDS counter.
template <bool GL, typename T>
__device__ __forceinline__ T ldg(const T* p, int64_t i) {
  if constexpr (GL) return ((const T __attribute__((address_space(1)))*)p)[i];
  else return p[i];
}
template <bool GL, typename T>
__device__ __forceinline__ void stg(T* p, int64_t i, T v) {
  if constexpr (GL) ((T __attribute__((address_space(1)))*)p)[i] = v;
  else p[i] = v;
}
// sorted sample record i (one 32-byte load)
template <bool GL>
__device__ __forceinline__ double4 ld_rec(const double4* p, int64_t i) {
  if constexpr (GL) {
    typedef double d2g_t __attribute__((ext_vector_type(2)));
    const d2g_t __attribute__((address_space(1)))* q =
        (const d2g_t __attribute__((address_space(1)))*)(p + i);
    const d2g_t a = q[0], b = q[1];
    return make_double4(a.x, a.y, b.x, b.y);
  } else {
    return p[i];
  }
}

__device__ __forceinline__ uint32_t lane_u32(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// One wavefront's view of a tile's ranges: lane l holds range w0 + l (its
// first sorted position b and candidate indices [s, e); past the last range
// s = e = total).  The 64 ranges cover candidates [s of lane 0, e of lane
// 63).  cover() moves the window (monotonically, in the direction of the
// walk) until it holds a span of candidates; pos() then maps a candidate
// index of that span to its sorted position.  Every lane of the wavefront
// must take part in both calls.
template <bool GL>
struct RangeWindow {
  const uint32_t* rng;
  uint32_t nr, total, w0;
  uint32_t b, s, e;

  __device__ __forceinline__ void load(uint32_t first) {
    w0 = first;
    const uint32_t k = first + (uint32_t)(threadIdx.x & 63);
    if (k < nr) {
      b = ldg<GL>(rng, 2 * (int64_t)k);
      s = ldg<GL>(rng, 2 * (int64_t)k + 1);
      e = k + 1 < nr ? ldg<GL>(rng, 2 * (int64_t)k + 3) : total;
    } else {
      b = 0;
      s = e = total;
    }
  }
  // tile of `tv`; fwd: the walk visits candidates in increasing order
  __device__ __forceinline__ void init(const uint32_t* ranges, uint32_t n_ranges, uint32_t n_cand,
                                       bool fwd) {
    rng = ranges;
    nr = n_ranges;
    total = n_cand;
    load(fwd || nr <= 64 ? 0u : nr - 64);
  }
  // make the window hold candidates [qlo, qhi] (qlo <= qhi < total)
  __device__ __forceinline__ void cover(uint32_t qlo, uint32_t qhi, bool fwd) {
    for (;;) {
      const uint32_t wlo = lane_u32(s, 0), whi = lane_u32(e, 63);
      if (wlo <= qlo && qhi < whi) return;
      uint32_t nw;
      if (fwd) {
        // the range holding qlo becomes the first of the window: at least 63
        // more non-empty ranges follow it, which cover any span of 64
        nw = w0 + (uint32_t)__popcll(__ballot(e <= qlo));
      } else if (qhi < wlo) {
        nw = w0 >= 64 ? w0 - 64 : 0;
      } else {
        // the range holding qhi becomes the last of the window
        const uint32_t r = w0 + (uint32_t)__popcll(__ballot(e <= qhi));
        nw = r >= 63 ? r - 63 : 0;
      }
      load(nw);
    }
  }
  // sorted position of candidate q, where [qlo, qhi] (the same on every
  // lane) is the covered span: the range holding qlo is found by one
  // ballot, then each lane steps over the few ranges that start inside the
  // span (scalar reads of their starts), and two independent shuffles fetch
  // its range's first position and first candidate index
  __device__ __forceinline__ uint32_t pos(uint32_t q, uint32_t qlo, uint32_t qhi) const {
    int r = __popcll(__ballot(e <= qlo));
    int mine = r;
    for (int k = r + 1; k < 64; ++k) {
      const uint32_t sk = lane_u32(s, k);
      if (sk > qhi) break;
      if (sk <= q) mine = k;
    }
    const uint32_t br = (uint32_t)__shfl((int)b, mine, 64);
    const uint32_t sr = (uint32_t)__shfl((int)s, mine, 64);
    return br + (q - sr);
  }
};

__device__ __forceinline__ int64_t tile_of_block(int64_t b, int64_t ntiles) {
  const int64_t k = b % kNumXcd;
  const int64_t j = b / kNumXcd;
  int64_t start = 0;
  for (int64_t q = 0; q < k; ++q) start += (ntiles - q + kNumXcd - 1) / kNumXcd;
  return start + j;
}
// Same for a 1-D grid of ntiles * npass work items (channel passes of a
// tile are adjacent, so they run on the same XCD).
__device__ __forceinline__ void work_of_block(int64_t b, int64_t ntiles, int64_t npass,
                                              int64_t* tile, int64_t* pass) {
  const int64_t v = tile_of_block(b, ntiles * npass);
  *tile = v / npass;
  *pass = v % npass;
}
// Visit order of the tiles of a WCS grid (ntx tiles per row): strips of
// kStrip tile rows, each walked column by column, so that the tiles running
// together on one XCD form a compact block that shares candidate samples
// both across and along the columns.  v is the position in the visit order.
constexpr int64_t kStrip = 4;
__host__ __device__ __forceinline__ int64_t strip_tile(int64_t v, int64_t ntiles, int64_t ntx) {
  const int64_t nty = ntiles / ntx;
  const int64_t s = v / (kStrip * ntx);
  const int64_t h = (nty - s * kStrip) < kStrip ? (nty - s * kStrip) : kStrip;
  const int64_t w = v - s * kStrip * ntx;
  return (s * kStrip + w % h) * ntx + w / h;
}

// ---------------------------------------------------------------- device math

// (2 asin(c/2))^2 from the squared chord c^2: the true angular distance
// squared, from the series
//   d^2 = c^2 (1 + c^2/12 + c^4/90 + c^6/560 + c^8/3150 + c^10/16632 + ...)
// (4 asin^2(x/2) = sum_n 2 x^(2n) / (n^2 C(2n, n))), whose truncation error is
// below 1e-10 relative for chords up to 0.35 rad (about 20 deg).  The
// correction c^2 (c^2/12 + ...) is at most 1.1 % of c^2, so it is evaluated
// in FP32 (its rounding moves d^2 by < 1e-9 relative) and added to c^2 with
// one FP64 fma: no FP64 constants, which keeps the hot loops' registers
// free.  Longer chords take the exact form in a separate (not inlined)
// function.
__device__ __noinline__ inline double chord2_to_d2_exact(double c2) {
  const double d = 2.0 * asin(0.5 * sqrt(c2));
  return d * d;
}
__device__ __forceinline__ double chord2_to_d2(double c2) {
  if (c2 <= 0.1225) {
    const float c = (float)c2;
    const float corr =
        c * (1.0f / 12.0f + c * (1.0f / 90.0f + c * (1.0f / 560.0f +
             c * (1.0f / 3150.0f + c * (1.0f / 16632.0f)))));
    return fma(c2, (double)corr, c2);
  }
  return chord2_to_d2_exact(c2);
}

// The same for the pairs of one launch: supports up to ~0.57 deg (c^2 <=
// 1e-4, uniform over the launch) keep d^2 = c^2 (1 + c^2/12), whose next term
// is below 1.1e-10 relative, in two FP64 operations.
__device__ __forceinline__ double chord2_to_d2_for(const KernelParams& kp, double c2) {
  return kp.cs2 <= 1e-4 ? fma(c2 * c2, 1.0 / 12.0, c2) : chord2_to_d2(c2);
}

// 2^(-x) for x >= 0 given in FP64, evaluated as 2^-frac (FP32) * 2^-int so
// that rounding x to FP32 does not cost accuracy at large x.
__device__ __forceinline__ float exp2_neg(double x) {
  const double xi = floor(x);
  if (xi > 126.0) return 0.0f;   // before the conversion: no int overflow
  // 2^-f for f in [0, 1) lies in (0.5, 1], where the hardware exp2 needs no
  // range handling
  return ldexpf(__builtin_amdgcn_exp2f(-(float)(x - xi)), (int)(-xi));
}

// Kernel weight for a pair with chord vector (dx, dy, dz) = p_n - p_t and
// c2 = |p_n - p_t|^2 <= cs2.  Elliptical: the bearing of the great circle
// from the target towards the sample is the direction of the chord's
// projection on the tangent plane at the target; with a, b the unit
// vectors of the major and minor axis there, u = d.a, v = d.b and
// cos^2(beta - pa) = u^2 / (u^2 + v^2).
// Radial kernels of arbitrary shape at distance d (rad): the tapered sinc
// exp(-d^2 / 2 sigma^2) sin(pi d / b) / (pi d / b), or the tabulated profile
// interpolated linearly (zero beyond its last point).
__device__ __forceinline__ double radial_weight(const KernelParams& kp, double d2) {
  const double d = sqrt(d2);
  if (kp.type == 2) {
    const double a = kp.ks * d;
    return (double)exp2_neg(d2 * kp.k1) * (a > 0.0 ? sin(a) / a : 1.0);
  }
  const double u = d * kp.tinv;
  const int last = kp.ntab - 1;
  if (!(u < (double)last)) return u == (double)last ? kp.tab[last] : 0.0;
  const int i = (int)u;
  const double f = u - (double)i;
  return kp.tab[i] + f * (kp.tab[i + 1] - kp.tab[i]);
}

// RADIAL: the kernel is one of the radial shapes (types 2, 3); otherwise a
// Gaussian (types 0, 1).  Separate instantiations keep the Gaussian loops
// free of the radial code's registers.
template <bool RADIAL>
__device__ __forceinline__ float pair_weight(const KernelParams& kp, double c2, double dx, double dy,
                                             double dz, double ax, double ay, double az, double bx,
                                             double by, double bz) {
  const double d2 = chord2_to_d2_for(kp, c2);
  if constexpr (RADIAL) return (float)radial_weight(kp, d2);
  if (kp.type == 0) return exp2_neg(d2 * kp.k1);
  const double u = dx * ax + dy * ay + dz * az;
  if (kp.cs2 <= 1e-4) {
    // u^2 + v^2 is the chord's tangential part c^2 (1 - c^2/4) exactly, so
    // the exponent is d^2 kmin + (kmaj - kmin) u^2 d^2 / (c^2 (1 - c^2/4)),
    // and for these supports d^2 / (c^2 (1 - c^2/4)) = 1 + c^2/3 to 1e-9
    return exp2_neg(fma((kp.kmaj - kp.kmin) * u * u, fma(c2, 1.0 / 3.0, 1.0), d2 * kp.kmin));
  }
  const double v = dx * bx + dy * by + dz * bz;
  const double uv = u * u + v * v;
  if (uv <= 0.0) return 1.0f;
  const double q = (u * u * kp.kmaj + v * v * kp.kmin) / uv;
  return exp2_neg(d2 * q);
}

// ---------------------------------------------------------------- launchers
// All launches are asynchronous on `st`; return hipSuccess or the launch error.

// rec: 4 doubles per sample (unit vector; channels 0-1 as FP32 when npack > 0)
hipError_t launch_prep(const double* lon, const double* lat, int64_t n, int64_t nside,
                       uint32_t* keys, uint32_t* vals, int* flag, double* rec, const void* data,
                       int dtype, int64_t ld, int npack, hipStream_t st);
hipError_t radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp,
                      uint32_t* hist, int64_t n, int bits, bool* result_in_tmp, hipStream_t st);
size_t radix_hist_elems(int64_t n);   // includes 256 digit totals
hipError_t launch_ring_offsets(const uint32_t* keys, int64_t n, int64_t nside, uint32_t* ring_off,
                               hipStream_t st);
// srec: one record per sorted sample (unit vector, input row as int64 bits)
hipError_t launch_permute(const uint32_t* vals, const uint32_t* nvalid_dev, int64_t n,
                          const double* rec, const void* data, int dtype, int64_t ld,
                          int64_t nchan, bool with_data, int npack, double* srec,
                          float* sdata, hipStream_t st);
hipError_t scan_u64(const uint64_t* in, uint64_t* out, int64_t n, hipStream_t st);
// the same over many blocks; scratch holds scan_u64_wide_scratch(n) values
size_t scan_u64_wide_scratch(int64_t n);
hipError_t scan_u64_wide(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* scratch,
                         hipStream_t st);

hipError_t launch_wcs_targets(const WcsDev& w, int64_t tile_w, int64_t tile_h, int64_t ntx,
                              int64_t nslots, double* txyz, double* tll, int32_t* slot_target,
                              int32_t* target_slot, hipStream_t st);
hipError_t launch_hpx_centres(int64_t nside, int nested, double* lon, double* lat,
                              uint32_t* order, hipStream_t st);
hipError_t launch_sl_keys(const double* lon, const double* lat, int64_t n, uint32_t* keys,
                          uint32_t* vals, int* flag, hipStream_t st);
hipError_t launch_sl_targets(const double* lon, const double* lat, const uint32_t* order,
                             int64_t ntarget, int64_t nslots, double* txyz, double* tll,
                             int32_t* slot_target, int32_t* target_slot, hipStream_t st);
hipError_t launch_tile_caps(const double* txyz, int64_t nslots, int64_t ntiles, double* caps,
                            hipStream_t st);
hipError_t launch_tile_span(const double* caps, int64_t ntiles, int64_t nside, double rho_extra,
                            int32_t* ring_first, uint64_t* span_bound, hipStream_t st);
// Pixel windows of every tile's rings (set-up): win[2 * s] = lo, win[2 * s + 1]
// = hi (RING pixel indices, lo > hi when empty) for the range slots s of
// range_off, two per ring.
hipError_t launch_tile_windows(const double* caps, const double* txyz, int64_t nslots,
                               int64_t ntiles, int64_t nside, double rho,
                               const int32_t* ring_first, const uint64_t* range_off,
                               uint32_t* win, hipStream_t st);
// sample-centric lookup (cg_disk.hip)
hipError_t launch_target_keys(const double* txyz, int64_t nslots, int64_t nside, uint32_t* keys,
                              uint32_t* vals, hipStream_t st);
hipError_t launch_ref_disks(int64_t nside, int64_t reach, double rs, int2* tab, hipStream_t st);
hipError_t launch_run_flags(const uint32_t* keys, const uint32_t* nvalid, int64_t n,
                            uint64_t* flag, hipStream_t st);
hipError_t launch_run_compact(const uint32_t* keys, const uint32_t* nvalid, int64_t n,
                              const uint64_t* uoff, uint32_t* upix, uint32_t* ustart,
                              hipStream_t st);
hipError_t launch_disk_pairs(bool count, const uint32_t* upix, int64_t nu, int64_t nside,
                             int64_t reach, const int2* tab, const uint32_t* tkeys,
                             const uint32_t* tslot, const uint32_t* troff, const uint64_t* off,
                             uint64_t* cnt, uint32_t* pk, uint32_t* pv, hipStream_t st);
hipError_t launch_disk_ranges(const uint32_t* pk, const uint32_t* pv, int64_t np,
                              const uint32_t* ustart, uint64_t* flag, uint64_t* rsx,
                              uint64_t* scan_scratch,
                              int64_t ntiles, uint32_t* ranges, uint64_t* range_off,
                              uint32_t* nranges, uint64_t* ncand, hipStream_t st);

hipError_t launch_tile_ranges(int64_t ntiles, const int32_t* ring_first,
                              const uint64_t* range_off, const uint32_t* win,
                              const uint32_t* keys, const uint32_t* ring_off, uint32_t* ranges,
                              uint32_t* nranges, uint64_t* ncand, hipStream_t st);
// contraction kernels
enum AccMode { ACC_OVERWRITE = 0, ACC_ADD = 1, ACC_FINAL = 2 };
struct OutView {
  double* S;           // [nchan][nslots] accumulator (ACC_OVERWRITE / ACC_ADD)
  double* W;           // [nslots] weight map (Eq. 2)
  double* Wn;          // [nslots] normaliser: sum of the weights as they entered the products
  float* cube;         // ACC_FINAL: normalised output in user layout
  float* wout;         // ACC_FINAL: weights in user layout (may be null)
  const int32_t* slot_target;
  int64_t ntarget;
  int64_t cst, tst;    // element strides of the cube: channel, target (layout)
  int mode;
};
hipError_t launch_gather_fp32(const TileView& tv, const KernelParams& kp, const void* data,
                              int dtype, int64_t ld, const float* sdata, int64_t nchan,
                              const OutView& ov, hipStream_t st);
// zrow: device row of at least nchan zeros of the data type (8 * nchan bytes)
hipError_t launch_gather_mfma(const TileView& tv, const KernelParams& kp, const void* data,
                              const void* zrow, int dtype, int64_t ld, int64_t nchan, int prec,
                              const OutView& ov, hipStream_t st);
bool mfma_available();

// ---------------------------------------------------------------- batches
// One job of a batch: its samples, its gridder's targets and tiles, where
// its pieces sit in the batch's concatenated arrays, and its outputs.
struct BatchJob {
  const double* lon;           // [n] sample longitudes (deg)
  const double* lat;           // [n] sample latitudes (deg)
  const void* data;            // [n][ld] sample rows
  int64_t n, noff;             // samples; offset in the concatenated sample order
  int64_t ld, nchan, nside;
  int64_t ro_off;              // offset of the ring offsets [4 nside + 1]
  int64_t toff, ntiles, nslots;  // first global tile; tiles; target slots
  int64_t ntx;                 // tiles per row (WCS grids), 0 for sight lines
  int64_t rbase;               // offset (in ranges) of the job's range slots
  int64_t ntarget;
  const double* txyz;
  const double* tll;
  const double* caps;
  const int32_t* ring_first;
  const uint64_t* range_off;   // [ntiles + 1] job-local range-slot offsets
  const uint32_t* win;         // pixel windows of the range slots
  const int32_t* slot_target;
  float* cube;                 // normalised output (strides cst per channel, tst per target)
  float* wout;                 // [ntarget] weight map (may be null)
  int64_t cst, tst;
  KernelParams kp;
  double rho;                  // support radius + margin (rad)
};
// One work item of the persistent contraction: a tile of a job and a channel
// range [c0, cend).
struct BatchItem {
  int32_t job, tile, c0, cend;
};

// Largest j in [0, n) with off[j] <= x (off ascending, off[0] = 0): the job
// whose range [off[j], off[j + 1]) holds x (empty jobs are skipped).
__device__ __forceinline__ int job_of(const int64_t* __restrict__ off, int n, int64_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

hipError_t launch_batch_prep(const BatchJob* jobs, const int64_t* noff, int njobs, int64_t ntot,
                             uint32_t* keys, uint32_t* vals, int* flag, hipStream_t st);
// Stable LSD sort by the low `bits` of the keys, then one more stable pass by
// the job of each value (values are positions in the concatenated order), so
// the result is job-major and sorted by key within each job.
hipError_t radix_sort_jobs(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp,
                           uint32_t* hist, int64_t n, int bits, const int64_t* noff, int njobs,
                           bool* result_in_tmp, hipStream_t st);
hipError_t launch_batch_ring_offsets(const BatchJob* jobs, const int64_t* rooff, int njobs,
                                     int64_t nentries, const uint32_t* keys, uint32_t* ring_off,
                                     hipStream_t st);
hipError_t launch_batch_permute(const BatchJob* jobs, const int64_t* noff, int njobs, int64_t ntot,
                                const uint32_t* vals, const uint32_t* ring_off, double* srec,
                                hipStream_t st);
hipError_t launch_batch_tile_ranges(const BatchJob* jobs, const int64_t* toff, int njobs,
                                    int64_t ntiles, const uint32_t* keys, const uint32_t* ring_off,
                                    uint32_t* ranges, uint32_t* nranges, uint64_t* ncand,
                                    hipStream_t st);
// The ranges of a batch lookup pass, over the concatenated jobs: per job at
// ranges + 2 rbase (job-local range offsets range_off), counts at toff.
struct BatchRanges {
  const uint32_t* ranges;
  const uint32_t* nranges;
  const uint64_t* ncand;
  const double4* srec;         // sorted records (rows local to each job)
};
// The work queue in one segment per XCD: items [off[k], off[k + 1]) are
// the home queue of the workgroups on XCD k (each job's tiles split into
// kNumXcd runs of neighbouring tiles, one per XCD).
struct BatchQueues {
  int64_t off[kNumXcd + 1];
};
// Persistent contraction over the queues; shape 0..3 selects the workgroup
// (8 or 4 wavefronts, 1 or 2 channel blocks each: at most
// batch_shape_rows(shape) channels per item); counter holds kNumXcd ints,
// zero at launch.
constexpr int kBatchShapes = 4;
hipError_t launch_batch_mfma(const BatchJob* jobs, const BatchItem* items, const BatchQueues& q,
                             int* counter, const BatchRanges& br, const void* zrow, int dtype,
                             int prec, int shape, int blocks_per_cu, hipStream_t st);
int batch_max_blocks_per_cu(int dtype, int prec, int shape);
int batch_shape_rows(int shape);
hipError_t launch_stats(const TileView& tv, const KernelParams& kp, const int32_t* slot_target,
                        int32_t* counts, uint64_t* hashes, hipStream_t st);
hipError_t launch_normalize(const double* S, const double* W, const double* Wn,
                            const int32_t* target_slot, int64_t nslots, int64_t nchan,
                            int64_t ntarget, int64_t cst, int64_t tst, float* cube, float* wout,
                            hipStream_t st);
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t st);

}  // namespace cg
