// Targets, target tiles and the HEALPix ring lookup of candidate samples.
//
// The paper associates every target with a HEALPix pixel and matches the
// per-sample disks queried once per ring and shifted in longitude against
// them (Sect. 2.2 steps 2-3, Sect. 3.3 Eq. 4-5, Sect. 3.4).  Here the lookup
// runs from the target side, so that each thread owns its outputs (the
// race-free ownership of Sect. 2.2): targets are grouped into tiles of 64,
// each tile gets a bounding cap, and for every ring crossing the cap widened
// by the support radius the longitude window of the cap on that ring gives
// a pixel range, i.e. one contiguous run of the RING-sorted samples.
#include "cg_internal.hpp"

namespace cg {

__device__ __forceinline__ void lonlat_to_xyz(double lon_deg, double lat_deg, double* x, double* y,
                                              double* z) {
  double am = fmod(lon_deg, 360.0);
  if (am < 0.0) am += 360.0;
  double sa, ca, sd, cd;
  sincos(am * (hpx::kPi / 180.0), &sa, &ca);
  sincos(lat_deg * (hpx::kPi / 180.0), &sd, &cd);
  *x = cd * ca;
  *y = cd * sa;
  *z = sd;
}

// ---------------------------------------------------------------------------
// WCS grid targets: slot s = tile * 64 + ly * tile_w + lx.

__global__ void __launch_bounds__(256) k_wcs_targets(WcsDev w, int64_t tile_w, int64_t tile_h,
                                                     int64_t ntx, int64_t nslots,
                                                     double* __restrict__ txyz,
                                                     double* __restrict__ tll,
                                                     int32_t* __restrict__ slot_target,
                                                     int32_t* __restrict__ target_slot) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  const int64_t tile = s / kTile;
  const int64_t l = s % kTile;
  const int64_t x = (tile % ntx) * tile_w + l % tile_w;
  const int64_t y = (tile / ntx) * tile_h + l / tile_w;
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  double px = nan, py = nan, pz = nan, lo = nan, la = nan;
  int32_t t = -1;
  if (x < w.naxis1 && y < w.naxis2) {
    t = (int32_t)(y * w.naxis1 + x);
    target_slot[t] = (int32_t)s;
    if (wcs_pix2world(w, (double)(x + 1), (double)(y + 1), &lo, &la)) {
      lonlat_to_xyz(lo, la, &px, &py, &pz);
    } else {
      lo = nan;
      la = nan;
    }
  }
  slot_target[s] = t;
  txyz[s] = px;
  txyz[nslots + s] = py;
  txyz[2 * nslots + s] = pz;
  tll[s] = lo * (hpx::kPi / 180.0);
  tll[nslots + s] = la * (hpx::kPi / 180.0);
}

hipError_t launch_wcs_targets(const WcsDev& w, int64_t tile_w, int64_t tile_h, int64_t ntx,
                              int64_t nslots, double* txyz, double* tll, int32_t* slot_target,
                              int32_t* target_slot, hipStream_t st) {
  hipLaunchKernelGGL(k_wcs_targets, dim3((unsigned)((nslots + 255) / 256)), dim3(256), 0, st, w,
                     tile_w, tile_h, ntx, nslots, txyz, tll, slot_target, target_slot);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sight lines: ordered along a space-filling curve (a Hilbert curve in each
// HEALPix base face) so that runs of 64 consecutive targets are compact
// tiles.

constexpr int64_t kSlNside = 8192;

__global__ void __launch_bounds__(256) k_sl_keys(const double* __restrict__ lon,
                                                 const double* __restrict__ lat, int64_t n,
                                                 uint32_t* __restrict__ keys,
                                                 uint32_t* __restrict__ vals, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = lon[i], d = lat[i];
  uint32_t key;
  if (!(isfinite(a) && isfinite(d) && fabs(d) <= 90.0)) {
    key = (uint32_t)hpx::npix(kSlNside);
    atomicOr(flag, 1);
  } else {
    double am = fmod(a, 360.0);
    if (am < 0.0) am += 360.0;
    double sd, cd;
    sincos(d * (hpx::kPi / 180.0), &sd, &cd);
    key = (uint32_t)hpx::ang2hilbert(kSlNside, sd, cd, am * (hpx::kPi / 180.0));
  }
  keys[i] = key;
  vals[i] = (uint32_t)i;
}

hipError_t launch_sl_keys(const double* lon, const double* lat, int64_t n, uint32_t* keys,
                          uint32_t* vals, int* flag, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sl_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, lon, lat, n,
                     keys, vals, flag);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_sl_targets(const double* __restrict__ lon,
                                                    const double* __restrict__ lat,
                                                    const uint32_t* __restrict__ order,
                                                    int64_t ntarget, int64_t nslots,
                                                    double* __restrict__ txyz,
                                                    double* __restrict__ tll,
                                                    int32_t* __restrict__ slot_target,
                                                    int32_t* __restrict__ target_slot) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  double px = nan, py = nan, pz = nan, lo = nan, la = nan;
  int32_t t = -1;
  if (s < ntarget) {
    t = (int32_t)order[s];
    target_slot[t] = (int32_t)s;
    const double a = lon[t], d = lat[t];
    if (isfinite(a) && isfinite(d) && fabs(d) <= 90.0) {
      lonlat_to_xyz(a, d, &px, &py, &pz);
      double am = fmod(a, 360.0);
      if (am < 0.0) am += 360.0;
      lo = am * (hpx::kPi / 180.0);
      la = d * (hpx::kPi / 180.0);
    }
  }
  slot_target[s] = t;
  txyz[s] = px;
  txyz[nslots + s] = py;
  txyz[2 * nslots + s] = pz;
  tll[s] = lo;
  tll[nslots + s] = la;
}

hipError_t launch_sl_targets(const double* lon, const double* lat, const uint32_t* order,
                             int64_t ntarget, int64_t nslots, double* txyz, double* tll,
                             int32_t* slot_target, int32_t* target_slot, hipStream_t st) {
  hipLaunchKernelGGL(k_sl_targets, dim3((unsigned)((nslots + 255) / 256)), dim3(256), 0, st, lon,
                     lat, order, ntarget, nslots, txyz, tll, slot_target, target_slot);
  return hipGetLastError();
}

// Targets of a HEALPix map: target p is pixel p of the map's own order
// (RING or NESTED), at its centre.  Slot s holds NESTED pixel s, so a tile
// is 64 NESTED-consecutive pixels: an 8 x 8 block of one base face.
// order[s] is the target index of slot s.
__global__ void __launch_bounds__(256) k_hpx_centres(int64_t nside, int nested, int64_t n,
                                                     double* __restrict__ lon,
                                                     double* __restrict__ lat,
                                                     uint32_t* __restrict__ order) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double a, d;
  hpx::pix_centre(nside, p, nested != 0, &a, &d);
  lon[p] = a;
  lat[p] = d;
  int64_t i, j;
  hpx::nest2ring_ij(nside, p, &i, &j);
  order[p] = (uint32_t)(nested ? p : hpx::ring_start(nside, i) + j);
}

hipError_t launch_hpx_centres(int64_t nside, int nested, double* lon, double* lat,
                              uint32_t* order, hipStream_t st) {
  const int64_t n = hpx::npix(nside);
  hipLaunchKernelGGL(k_hpx_centres, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, nside,
                     nested, n, lon, lat, order);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tile caps: centre = normalised sum of the tile's target vectors, radius =
// largest angle from the centre to a target.  One wavefront per tile.

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__global__ void __launch_bounds__(64) k_tile_caps(const double* __restrict__ txyz, int64_t nslots,
                                                  double* __restrict__ caps) {
  const int64_t tile = blockIdx.x;
  const int64_t s = tile * kTile + threadIdx.x;
  const double x = txyz[s], y = txyz[nslots + s], z = txyz[2 * nslots + s];
  const bool ok = isfinite(x);
  const double sx = wave_sum(ok ? x : 0.0);
  const double sy = wave_sum(ok ? y : 0.0);
  const double sz = wave_sum(ok ? z : 0.0);
  const double cnt = wave_sum(ok ? 1.0 : 0.0);
  double cx = 0.0, cy = 0.0, cz = 1.0, r = -1.0;
  if (cnt > 0.0) {
    const double nrm = sqrt(sx * sx + sy * sy + sz * sz);
    if (nrm > 1e-6 * cnt) {
      cx = sx / nrm;
      cy = sy / nrm;
      cz = sz / nrm;
      double a = 0.0;
      if (ok) {
        const double qx = cy * z - cz * y, qy = cz * x - cx * z, qz = cx * y - cy * x;
        a = atan2(sqrt(qx * qx + qy * qy + qz * qz), cx * x + cy * y + cz * z);
      }
      r = wave_max(a) * (1.0 + 1e-12) + 1e-15;
    } else {
      r = hpx::kPi;   // targets spread over the whole sphere: the cap is everything
    }
  }
  if (threadIdx.x == 0) {
    caps[4 * tile + 0] = cx;
    caps[4 * tile + 1] = cy;
    caps[4 * tile + 2] = cz;
    caps[4 * tile + 3] = r;
  }
}

hipError_t launch_tile_caps(const double* txyz, int64_t nslots, int64_t ntiles, double* caps,
                            hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_caps, dim3((unsigned)ntiles), dim3(64), 0, st, txyz, nslots, caps);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ring span of each tile's widened cap and an upper bound of its range count
// (two per ring).

__device__ __forceinline__ void cap_angles(const double* caps, int64_t tile, double* cz, double* cs,
                                           double* cphi, double* r) {
  const double x = caps[4 * tile], y = caps[4 * tile + 1], z = caps[4 * tile + 2];
  *r = caps[4 * tile + 3];
  *cz = z;
  *cs = sqrt(x * x + y * y);
  double p = atan2(y, x);
  if (p < 0.0) p += hpx::kTwoPi;
  if (p >= hpx::kTwoPi) p -= hpx::kTwoPi;
  *cphi = p;
}

__global__ void __launch_bounds__(256) k_tile_span(const double* __restrict__ caps, int64_t ntiles,
                                                   int64_t nside, double rho_extra,
                                                   int32_t* __restrict__ ring_first,
                                                   uint64_t* __restrict__ bound) {
  const int64_t tile = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tile >= ntiles) return;
  double cz, cs, cphi, r;
  cap_angles(caps, tile, &cz, &cs, &cphi, &r);
  if (r < 0.0) {
    ring_first[tile] = 1;
    bound[tile] = 0;
    return;
  }
  int64_t f, l;
  hpx::cap_ring_span(nside, cz, cs, r + rho_extra, &f, &l);
  ring_first[tile] = (int32_t)f;
  bound[tile] = (l >= f) ? (uint64_t)(2 * (l - f + 1)) : 0ull;
}

hipError_t launch_tile_span(const double* caps, int64_t ntiles, int64_t nside, double rho_extra,
                            int32_t* ring_first, uint64_t* span_bound, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_span, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, st, caps,
                     ntiles, nside, rho_extra, ring_first, span_bound);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pixel windows of the tiles (set-up: they depend only on the targets, the
// support and nside).  For each ring crossing a tile's widened cap, the
// longitude window is the union over the tile's targets of the window of
// each target's own support disk, which is tighter than the window of the
// cap around the whole tile.  One 256-thread block per tile: the targets'
// disks are prepared into LDS; rings are taken 256 at a time, each wavefront
// forms for every ring the union over its quarter of the targets, then one
// thread per ring merges the four partial windows and stores up to two RING
// pixel ranges in the ring's two slots (an empty slot holds lo > hi).

constexpr int kRangeThreads = 256;
constexpr int kRangeWaves = kRangeThreads / 64;

__device__ __forceinline__ void tile_windows_body(
    int64_t tile, const double* __restrict__ caps, const double* __restrict__ txyz,
    int64_t nslots, int64_t nside, double rho, const int32_t* __restrict__ ring_first,
    const uint64_t* __restrict__ range_off, uint32_t* __restrict__ win) {
  __shared__ hpx::DiskPrep s_dp[kTile];
  __shared__ double s_rel[kTile];
  __shared__ double s_lo[kRangeWaves][kRangeThreads], s_hi[kRangeWaves][kRangeThreads];
  __shared__ int s_fl[kRangeWaves][kRangeThreads];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t off = range_off[tile];
  const int64_t nring = (int64_t)((range_off[tile + 1] - off) / 2);
  double cz, cs, cphi, r;
  cap_angles(caps, tile, &cz, &cs, &cphi, &r);
  if (tid < kTile) {
    const int64_t slot = tile * kTile + tid;
    const double x = txyz[slot], y = txyz[nslots + slot], z = txyz[2 * nslots + slot];
    hpx::DiskPrep dp;
    double rel = 0.0;
    if (isfinite(x)) {
      hpx::disk_prepare(z, sqrt(x * x + y * y), rho, &dp);
      double p = atan2(y, x);
      if (p < 0.0) p += hpx::kTwoPi;
      rel = hpx::rel_lon(p, cphi);
    } else {
      // padding slot: an empty latitude band meets no ring
      dp.tz = 1.0; dp.ts = 0.0; dp.zmin = 2.0; dp.zmax = -2.0;
      dp.crho = 1.0; dp.zstar = 0.0; dp.all = 0;
    }
    s_dp[tid] = dp;
    s_rel[tid] = rel;
  }
  __syncthreads();
  const int64_t f = ring_first[tile];
  constexpr int kPer = kTile / kRangeWaves;
  for (int64_t q0 = 0; q0 < nring; q0 += kRangeThreads) {
    const int nb = (int)((nring - q0) < kRangeThreads ? (nring - q0) : kRangeThreads);
    // partial unions: wavefront `wave` covers targets [wave*kPer, (wave+1)*kPer)
    for (int q = lane; q < nb; q += 64) {
      double zl, zh;
      hpx::ring_band(nside, f + q0 + q, &zl, &zh);
      double lo = 1e300, hi = -1e300;
      int fl = 0;
      for (int t = wave * kPer; t < (wave + 1) * kPer; ++t) {
        const hpx::DiskPrep dp = s_dp[t];
        double w;
        const int st = hpx::band_disk_halfwidth(zl, zh, dp, &w);
        if (st == 2) fl |= 2;
        if (st == 1) {
          fl |= 1;
          lo = fmin(lo, s_rel[t] - w);
          hi = fmax(hi, s_rel[t] + w);
        }
      }
      s_lo[wave][q] = lo;
      s_hi[wave][q] = hi;
      s_fl[wave][q] = fl;
    }
    __syncthreads();
    if (tid < nb) {
      const int64_t q = q0 + tid;
      const int64_t i = f + q;
      double lo = 1e300, hi = -1e300;
      int fl = 0;
#pragma unroll
      for (int w = 0; w < kRangeWaves; ++w) {
        lo = fmin(lo, s_lo[w][tid]);
        hi = fmax(hi, s_hi[w][tid]);
        fl |= s_fl[w][tid];
      }
      const int full = (fl & 2) || ((fl & 1) && hi - lo >= hpx::kTwoPi);
      int64_t plo[2] = {1, 1}, phi[2] = {0, 0};
      if (fl) hpx::ring_window_ranges(nside, i, cphi + lo, cphi + hi, full, plo, phi);
      uint32_t* wq = win + 2 * (off + 2 * q);
      wq[0] = (uint32_t)plo[0];
      wq[1] = (uint32_t)phi[0];
      wq[2] = (uint32_t)plo[1];
      wq[3] = (uint32_t)phi[1];
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kRangeThreads) k_tile_windows(
    const double* __restrict__ caps, const double* __restrict__ txyz, int64_t nslots,
    int64_t nside, double rho, const int32_t* __restrict__ ring_first,
    const uint64_t* __restrict__ range_off, uint32_t* __restrict__ win) {
  tile_windows_body(blockIdx.x, caps, txyz, nslots, nside, rho, ring_first, range_off, win);
}

hipError_t launch_tile_windows(const double* caps, const double* txyz, int64_t nslots,
                               int64_t ntiles, int64_t nside, double rho,
                               const int32_t* ring_first, const uint64_t* range_off,
                               uint32_t* win, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_windows, dim3((unsigned)ntiles), dim3(kRangeThreads), 0, st, caps,
                     txyz, nslots, nside, rho, ring_first, range_off, win);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Candidate ranges of a grid call: one wavefront per tile, one window slot
// per lane.  Two binary searches in the ring's sorted segment turn a pixel
// range into a range of sorted samples; the non-empty ones are compacted in
// slot (ring) order as (first sorted position, first candidate index of the
// range within the tile), and the tile's candidate count is written.

// First positions in keys[lo, hi) (sorted) whose key is >= v1 and >= v2:
// the two bisections run in step, so that each step's two loads are in
// flight together instead of one search waiting for the other.
__device__ __forceinline__ void lower_bounds_u32(const uint32_t* __restrict__ keys, uint32_t lo,
                                                 uint32_t hi, uint64_t v1, uint64_t v2,
                                                 uint32_t* b, uint32_t* e) {
  uint32_t l1 = lo, h1 = hi, l2 = lo, h2 = hi;
  while (l1 < h1 || l2 < h2) {
    const bool a1 = l1 < h1, a2 = l2 < h2;
    const uint32_t m1 = l1 + ((h1 - l1) >> 1), m2 = l2 + ((h2 - l2) >> 1);
    const uint32_t k1 = a1 ? keys[m1] : 0u, k2 = a2 ? keys[m2] : 0u;
    if (a1) {
      if ((uint64_t)k1 < v1) l1 = m1 + 1;
      else h1 = m1;
    }
    if (a2) {
      if ((uint64_t)k2 < v2) l2 = m2 + 1;
      else h2 = m2;
    }
  }
  *b = l1;
  *e = l2;
}

__device__ __forceinline__ void tile_ranges_body(
    int64_t tile, const int32_t* __restrict__ ring_first, const uint64_t* __restrict__ range_off,
    const uint32_t* __restrict__ win, const uint32_t* __restrict__ keys,
    const uint32_t* __restrict__ ring_off, uint32_t* __restrict__ ranges,
    uint32_t* __restrict__ nranges, uint64_t* __restrict__ ncand) {
  const int lane = threadIdx.x;
  const uint64_t off = range_off[tile];
  const int64_t ns = (int64_t)(range_off[tile + 1] - off);
  const int64_t f = ring_first[tile];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t written = 0;
  uint64_t total = 0;
  for (int64_t s0 = 0; s0 < ns; s0 += 64) {
    const int64_t s = s0 + lane;
    uint32_t b = 0, e = 0;
    if (s < ns) {
      const uint32_t lo = win[2 * (off + s)], hi = win[2 * (off + s) + 1];
      if (lo <= hi) {
        const int64_t i = f + (s >> 1);
        const uint32_t rb = ring_off[i], re = ring_off[i + 1];
        lower_bounds_u32(keys, rb, re, (uint64_t)lo, (uint64_t)hi + 1, &b, &e);
      }
    }
    const bool h = e > b;
    const uint64_t m = __ballot(h);
    const uint32_t k = written + (uint32_t)__popcll(m & lt);
    const uint32_t len = e - b;
    uint32_t incl = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t v = (uint32_t)__shfl_up((int)incl, o, 64);
      if (lane >= o) incl += v;
    }
    if (h) {
      ranges[2 * (off + k) + 0] = b;
      ranges[2 * (off + k) + 1] = (uint32_t)total + (incl - len);
    }
    written += (uint32_t)__popcll(m);
    total += (uint64_t)(uint32_t)__shfl((int)incl, 63, 64);
  }
  if (lane == 0) {
    nranges[tile] = written;
    ncand[tile] = total;
  }
}

__global__ void __launch_bounds__(64) k_tile_ranges(
    const int32_t* __restrict__ ring_first, const uint64_t* __restrict__ range_off,
    const uint32_t* __restrict__ win, const uint32_t* __restrict__ keys,
    const uint32_t* __restrict__ ring_off, uint32_t* __restrict__ ranges,
    uint32_t* __restrict__ nranges, uint64_t* __restrict__ ncand) {
  tile_ranges_body(blockIdx.x, ring_first, range_off, win, keys, ring_off, ranges, nranges, ncand);
}

// Batches: one wavefront per tile of any job; the job's own window slots,
// its range slots at rbase and its ring offsets at ro_off.
__global__ void __launch_bounds__(64) k_batch_tile_ranges(
    const BatchJob* __restrict__ jobs, const int64_t* __restrict__ toff, int njobs,
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ ring_off,
    uint32_t* __restrict__ ranges, uint32_t* __restrict__ nranges, uint64_t* __restrict__ ncand) {
  const int64_t g = blockIdx.x;
  const int j = job_of(toff, njobs, g);
  const BatchJob& jb = jobs[j];
  tile_ranges_body(g - jb.toff, jb.ring_first, jb.range_off, jb.win, keys, ring_off + jb.ro_off,
                   ranges + 2 * jb.rbase, nranges + jb.toff, ncand + jb.toff);
}

hipError_t launch_batch_tile_ranges(const BatchJob* jobs, const int64_t* toff, int njobs,
                                    int64_t ntiles, const uint32_t* keys, const uint32_t* ring_off,
                                    uint32_t* ranges, uint32_t* nranges, uint64_t* ncand,
                                    hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_tile_ranges, dim3((unsigned)ntiles), dim3(64), 0, st, jobs, toff,
                     njobs, keys, ring_off, ranges, nranges, ncand);
  return hipGetLastError();
}

hipError_t launch_tile_ranges(int64_t ntiles, const int32_t* ring_first,
                              const uint64_t* range_off, const uint32_t* win,
                              const uint32_t* keys, const uint32_t* ring_off, uint32_t* ranges,
                              uint32_t* nranges, uint64_t* ncand, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)ntiles), dim3(64), 0, st, ring_first, range_off,
                     win, keys, ring_off, ranges, nranges, ncand);
  return hipGetLastError();
}

}  // namespace cg
