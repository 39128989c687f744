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
// Sight lines: ordered along the NESTED space-filling curve so that runs of
// 64 consecutive targets are compact tiles.

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
    key = (uint32_t)hpx::ang2pix_nest(kSlNside, sd, cd, am * (hpx::kPi / 180.0));
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
// Candidate ranges: one wavefront per tile.  For each ring crossing the
// tile's widened cap, the longitude window is the union over the tile's
// targets of the window of each target's own support disk (lane = target,
// wavefront min/max), which is tighter than the window of the cap around
// the whole tile.  The windows of a batch of rings are collected in LDS, then
// one ring per lane turns them into pixel ranges and two binary searches in
// the ring's sorted segment give the sample ranges.

__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* __restrict__ keys, uint32_t lo,
                                                    uint32_t hi, uint64_t v) {
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if ((uint64_t)keys[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

constexpr int kRingBatch = 256;

__global__ void __launch_bounds__(64) k_tile_ranges(
    const double* __restrict__ caps, const double* __restrict__ txyz, int64_t nslots,
    int64_t nside, double rho, const int32_t* __restrict__ ring_first,
    const uint64_t* __restrict__ range_off, const uint32_t* __restrict__ keys,
    const uint32_t* __restrict__ ring_off, uint32_t* __restrict__ ranges,
    uint32_t* __restrict__ nranges, uint64_t* __restrict__ ncand) {
  __shared__ double s_lo[kRingBatch], s_hi[kRingBatch];
  __shared__ int s_st[kRingBatch];
  const int64_t tile = blockIdx.x;
  const int lane = threadIdx.x;
  const uint64_t off = range_off[tile];
  const int64_t nring = (int64_t)((range_off[tile + 1] - off) / 2);
  double cz, cs, cphi, r;
  cap_angles(caps, tile, &cz, &cs, &cphi, &r);
  // this lane's target disk
  const int64_t slot = tile * kTile + lane;
  const double x = txyz[slot], y = txyz[nslots + slot], z = txyz[2 * nslots + slot];
  const bool valid = isfinite(x);
  hpx::DiskPrep dp;
  double rel = 0.0;
  if (valid) {
    hpx::disk_prepare(z, sqrt(x * x + y * y), rho, &dp);
    double p = atan2(y, x);
    if (p < 0.0) p += hpx::kTwoPi;
    rel = hpx::rel_lon(p, cphi);
  }
  const int64_t f = ring_first[tile];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t written = 0;
  uint64_t total = 0;
  for (int64_t b0 = 0; b0 < nring; b0 += kRingBatch) {
    const int nb = (int)((nring - b0) < kRingBatch ? (nring - b0) : kRingBatch);
    for (int q = 0; q < nb; ++q) {
      const int64_t i = f + b0 + q;
      int st = 0;
      double lo = 1e300, hi = -1e300;
      if (valid) {
        double w;
        st = hpx::ring_disk_halfwidth(nside, i, dp, &w);
        if (st == 1) {
          lo = rel - w;
          hi = rel + w;
        }
      }
      const bool anyfull = __ballot(st == 2) != 0;
      const bool anywin = __ballot(st == 1) != 0;
      lo = wave_min(lo);
      hi = wave_max(hi);
      if (lane == 0) {
        int code = 0;
        if (anyfull || (anywin && hi - lo >= hpx::kTwoPi)) code = 2;
        else if (anywin) code = 1;
        s_st[q] = code;
        s_lo[q] = cphi + lo;
        s_hi[q] = cphi + hi;
      }
    }
    __syncthreads();
    for (int qb = 0; qb < nb; qb += 64) {
      const int q = qb + lane;
      uint32_t b0r = 0, e0 = 0, b1 = 0, e1 = 0;
      if (q < nb && s_st[q] != 0) {
        const int64_t i = f + b0 + q;
        int64_t plo[2], phi[2];
        const int nr = hpx::ring_window_ranges(nside, i, s_lo[q], s_hi[q], s_st[q] == 2, plo, phi);
        const uint32_t rb = ring_off[i], re = ring_off[i + 1];
        if (re > rb) {
          b0r = lower_bound_u32(keys, rb, re, (uint64_t)plo[0]);
          e0 = lower_bound_u32(keys, b0r, re, (uint64_t)phi[0] + 1);
          if (nr >= 2) {
            b1 = lower_bound_u32(keys, rb, re, (uint64_t)plo[1]);
            e1 = lower_bound_u32(keys, b1, re, (uint64_t)phi[1] + 1);
          }
        }
      }
      const bool h0 = e0 > b0r, h1 = e1 > b1;
      const uint64_t m0 = __ballot(h0), m1 = __ballot(h1);
      const uint32_t pos = (uint32_t)(__popcll(m0 & lt) + __popcll(m1 & lt));
      uint32_t k = written + pos;
      if (h0) {
        ranges[2 * (off + k) + 0] = b0r;
        ranges[2 * (off + k) + 1] = e0 - b0r;
        ++k;
      }
      if (h1) {
        ranges[2 * (off + k) + 0] = b1;
        ranges[2 * (off + k) + 1] = e1 - b1;
      }
      written += (uint32_t)(__popcll(m0) + __popcll(m1));
      total += (uint64_t)wave_sum((double)((h0 ? e0 - b0r : 0u) + (h1 ? e1 - b1 : 0u)));
    }
    __syncthreads();
  }
  if (lane == 0) {
    nranges[tile] = written;
    ncand[tile] = total;
  }
}

hipError_t launch_tile_ranges(const double* caps, const double* txyz, int64_t nslots,
                              int64_t ntiles, int64_t nside, double rho,
                              const int32_t* ring_first, const uint64_t* range_off,
                              const uint32_t* keys, const uint32_t* ring_off, uint32_t* ranges,
                              uint32_t* nranges, uint64_t* ncand, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)ntiles), dim3(64), 0, st, caps, txyz, nslots,
                     nside, rho, ring_first, range_off, keys, ring_off, ranges, nranges, ncand);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Expand each tile's ranges into its list of candidates: sorted position,
// input index and unit vector, so the contraction reads them in one level.

__global__ void __launch_bounds__(64) k_expand(const uint64_t* __restrict__ range_off,
                                               const uint32_t* __restrict__ ranges,
                                               const uint32_t* __restrict__ nranges,
                                               const uint64_t* __restrict__ cand_off,
                                               const uint32_t* __restrict__ vals,
                                               const double* __restrict__ sx, int64_t nsorted,
                                               uint32_t* __restrict__ cand,
                                               uint32_t* __restrict__ crow,
                                               double* __restrict__ cxyz, int64_t ncap) {
  const int64_t tile = blockIdx.x;
  const uint64_t roff = range_off[tile];
  const uint32_t nr = nranges[tile];
  uint64_t out = cand_off[tile];
  for (uint32_t k = 0; k < nr; ++k) {
    const uint32_t b = ranges[2 * (roff + k)];
    const uint32_t len = ranges[2 * (roff + k) + 1];
    for (uint32_t q = threadIdx.x; q < len; q += 64) {
      const uint32_t pos = b + q;
      const uint64_t o = out + q;
      cand[o] = pos;
      crow[o] = vals[pos];
      cxyz[o] = sx[pos];
      cxyz[ncap + o] = sx[nsorted + pos];
      cxyz[2 * ncap + o] = sx[2 * nsorted + pos];
    }
    out += len;
  }
}

hipError_t launch_expand(const uint64_t* range_off, const uint32_t* ranges, const uint32_t* nranges,
                         const uint64_t* cand_off, int64_t ntiles, const uint32_t* vals,
                         const double* sx, int64_t nsorted, uint32_t* cand, uint32_t* crow,
                         double* cxyz, int64_t ncap, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_expand, dim3((unsigned)ntiles), dim3(64), 0, st, range_off, ranges, nranges,
                     cand_off, vals, sx, nsorted, cand, crow, cxyz, ncap);
  return hipGetLastError();
}

}  // namespace cg
