// Sample-centric lookup (Sect. 2.2 steps 2-3, Sect. 3.3-3.4): the paper's
// own route to the lists of samples per target, kept beside the tile lookup
// as an alternative that produces the same per-tile sample ranges.
//
//   * targets are keyed by their nearest HEALPix pixel and sorted, so that a
//     RING pixel range maps to a contiguous run of targets (the hash table
//     from HEALPix index to target pixels, as a sorted array with per-ring
//     offsets);
//   * one query disk per ring, around the ring's reference pixel near
//     longitude pi (set-up: it depends only on nside and the support);
//   * every distinct sample pixel moves its ring's disk to itself with the
//     integer shifts of Eq. 4-5 and, per ring of the disk, looks up the
//     targets of the shifted pixel range: the input-to-output mapping, as
//     (tile, sample pixel) pairs;
//   * the inversion (output-to-input mapping) is a stable sort of the pairs
//     by tile; duplicates are dropped and runs of consecutive sample pixels
//     merged into ranges of sorted samples, in the format the candidate
//     expansion reads.
//
// The contraction then applies the exact support test to every candidate,
// so the result is the same as with the tile lookup.
#include "cg_internal.hpp"

namespace cg {

namespace {

__device__ __forceinline__ uint32_t lower_bound_keys(const uint32_t* __restrict__ keys, uint32_t lo,
                                                     uint32_t hi, uint64_t v) {
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if ((uint64_t)keys[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Target keys: the RING pixel of every target slot (padding slots get Npix,
// which sorts after every pixel).
__global__ void __launch_bounds__(256) k_target_keys(const double* __restrict__ txyz,
                                                     int64_t nslots, int64_t nside,
                                                     uint32_t* __restrict__ keys,
                                                     uint32_t* __restrict__ vals) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  const double x = txyz[s], y = txyz[nslots + s], z = txyz[2 * nslots + s];
  uint32_t key = (uint32_t)hpx::npix(nside);
  if (isfinite(x)) {
    double phi = atan2(y, x);
    if (phi < 0.0) phi += hpx::kTwoPi;
    key = (uint32_t)hpx::ang2pix_ring(nside, z, sqrt(x * x + y * y), phi);
  }
  keys[s] = key;
  vals[s] = (uint32_t)s;
}

// Reference disks: entry (i, o) holds the window of ring i + o, for
// o in [-reach, reach]; an empty window has lo > hi, a whole ring lo = 0 and
// hi = its pixel count - 1.
__global__ void __launch_bounds__(256) k_ref_disks(int64_t nside, int64_t reach, double rs,
                                                   int2* __restrict__ tab) {
  const int64_t w = 2 * reach + 1;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 4 * nside * w) return;
  const int64_t i = idx / w, i2 = i + (idx - i * w) - reach;
  int2 e = make_int2(1, 0);
  if (i >= 1 && i < 4 * nside && i2 >= 1 && i2 < 4 * nside) {
    int64_t lo = 0, hi = 0;
    const int r = hpx::ref_disk_window(nside, i, i2, rs, &lo, &hi);
    if (r == 1) e = make_int2((int)lo, (int)hi);
    else if (r == 2) e = make_int2(0, (int)(hpx::ring_npix(nside, i2) - 1));
  }
  tab[idx] = e;
}

// Distinct sample pixels: the first position of every run of equal keys.
__global__ void __launch_bounds__(256) k_run_flags(const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ nvalid_p,
                                                   int64_t n, uint64_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t nv = (int64_t)(*nvalid_p);
  flag[i] = (i < nv && (i == 0 || keys[i] != keys[i - 1])) ? 1ull : 0ull;
}

// upix[u], ustart[u]: pixel and first sorted position of distinct pixel u;
// ustart[U] = number of valid samples closes the last run.
__global__ void __launch_bounds__(256) k_run_compact(const uint32_t* __restrict__ keys,
                                                     const uint32_t* __restrict__ nvalid_p,
                                                     int64_t n, const uint64_t* __restrict__ uoff,
                                                     uint32_t* __restrict__ upix,
                                                     uint32_t* __restrict__ ustart) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t nv = (int64_t)(*nvalid_p);
  if (i == 0) ustart[uoff[n]] = (uint32_t)nv;
  if (i < nv && (i == 0 || keys[i] != keys[i - 1])) {
    const uint64_t u = uoff[i];
    upix[u] = keys[i];
    ustart[u] = (uint32_t)i;
  }
}

// One thread per distinct sample pixel: walk the rings of its shifted query
// disk, look up the targets of each pixel range and emit (tile, u) for every
// change of tile along them.  COUNT stores the number of pairs; otherwise
// they are written at off[u], never past off[u + 1].
template <bool COUNT>
__global__ void __launch_bounds__(256) k_disk_pairs(
    const uint32_t* __restrict__ upix, int64_t nu, int64_t nside, int64_t reach,
    const int2* __restrict__ tab, const uint32_t* __restrict__ tkeys,
    const uint32_t* __restrict__ tslot, const uint32_t* __restrict__ troff,
    const uint64_t* __restrict__ off, uint64_t* __restrict__ cnt, uint32_t* __restrict__ pk,
    uint32_t* __restrict__ pv) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nu) return;
  int64_t i, j;
  hpx::pix2ring(nside, (int64_t)upix[u], &i, &j);
  const int64_t n1 = hpx::ring_npix(nside, i);
  const int64_t k = j - hpx::ring_ref_pixel(nside, i);
  const int64_t w = 2 * reach + 1;
  uint64_t c = 0, o0 = 0, lim = 0;
  if (!COUNT) {
    o0 = off[u];
    lim = off[u + 1];
  }
  uint32_t last = 0xFFFFFFFFu;
  for (int64_t o = -reach; o <= reach; ++o) {
    const int64_t i2 = i + o;
    if (i2 < 1 || i2 >= 4 * nside) continue;
    const int2 e = tab[i * w + o + reach];
    if (e.x > e.y) continue;
    const uint32_t tb = troff[i2], te = troff[i2 + 1];
    if (tb == te) continue;
    const int64_t n2 = hpx::ring_npix(nside, i2);
    int64_t a[2], b[2];
    int nr;
    if ((int64_t)e.y - e.x + 1 >= n2) {
      a[0] = hpx::ring_start(nside, i2);
      b[0] = a[0] + n2 - 1;
      nr = 1;
    } else {
      nr = hpx::shifted_window(nside, i2, e.x, e.y, hpx::disk_shift(k, n2, n1), a, b);
    }
    for (int q = 0; q < nr; ++q) {
      const uint32_t x = lower_bound_keys(tkeys, tb, te, (uint64_t)a[q]);
      const uint32_t y = lower_bound_keys(tkeys, x, te, (uint64_t)b[q] + 1);
      for (uint32_t t = x; t < y; ++t) {
        const uint32_t tile = tslot[t] / (uint32_t)kTile;
        if (tile == last) continue;
        last = tile;
        if (!COUNT && o0 + c < lim) {
          pk[o0 + c] = tile;
          pv[o0 + c] = (uint32_t)u;
        }
        ++c;
      }
    }
  }
  if (COUNT) cnt[u] = c;
}

// Pair p starts a range of its tile's list unless it repeats the previous
// pixel or follows it directly (consecutive distinct pixels are adjacent
// runs of sorted samples).
__device__ __forceinline__ bool starts_range(const uint32_t* __restrict__ pk,
                                             const uint32_t* __restrict__ pv, int64_t p) {
  if (p == 0 || pk[p] != pk[p - 1]) return true;
  return pv[p] != pv[p - 1] && pv[p] != pv[p - 1] + 1u;
}

__global__ void __launch_bounds__(256) k_range_flags(const uint32_t* __restrict__ pk,
                                                     const uint32_t* __restrict__ pv, int64_t np,
                                                     uint64_t* __restrict__ flag) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  flag[p] = starts_range(pk, pv, p) ? 1ull : 0ull;
}

// Range r of all tiles: ranges[2 r] = first sorted position, ranges[2 r + 1]
// = end position (turned into a length by k_tile_disk_ranges).  rsx is the
// exclusive scan of the start flags, so pair p belongs to range rsx[p + 1] - 1.
__global__ void __launch_bounds__(256) k_range_write(const uint32_t* __restrict__ pk,
                                                     const uint32_t* __restrict__ pv, int64_t np,
                                                     const uint64_t* __restrict__ rsx,
                                                     const uint32_t* __restrict__ ustart,
                                                     uint32_t* __restrict__ ranges) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const uint32_t u = pv[p];
  if (starts_range(pk, pv, p)) ranges[2 * rsx[p]] = ustart[u];
  if (p == np - 1 || starts_range(pk, pv, p + 1)) ranges[2 * (rsx[p + 1] - 1) + 1] = ustart[u + 1];
}

// One wavefront per tile: its pairs [p0, p1) by binary search over the
// sorted tiles, its ranges [rsx[p0], rsx[p1]); each range's end becomes its
// first candidate index within the tile (the exclusive prefix of the
// lengths), and the lengths sum to the tile's candidate count.
__global__ void __launch_bounds__(64) k_tile_disk_ranges(
    const uint32_t* __restrict__ pk, int64_t np, const uint64_t* __restrict__ rsx,
    int64_t ntiles, uint32_t* __restrict__ ranges, uint64_t* __restrict__ range_off,
    uint32_t* __restrict__ nranges, uint64_t* __restrict__ ncand) {
  const int64_t tile = blockIdx.x;
  const int lane = threadIdx.x;
  const uint32_t p0 = lower_bound_keys(pk, 0, (uint32_t)np, (uint64_t)tile);
  const uint32_t p1 = lower_bound_keys(pk, p0, (uint32_t)np, (uint64_t)tile + 1);
  const uint64_t r0 = rsx[p0], r1 = rsx[p1];
  uint32_t sum = 0;
  for (uint64_t q0 = r0; q0 < r1; q0 += 64) {
    const uint64_t q = q0 + lane;
    const uint32_t len = q < r1 ? ranges[2 * q + 1] - ranges[2 * q] : 0u;
    uint32_t incl = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t v = (uint32_t)__shfl_up((int)incl, o, 64);
      if (lane >= o) incl += v;
    }
    if (q < r1) ranges[2 * q + 1] = sum + (incl - len);
    sum += (uint32_t)__shfl((int)incl, 63, 64);
  }
  if (lane == 0) {
    range_off[tile] = r0;
    nranges[tile] = (uint32_t)(r1 - r0);
    ncand[tile] = (uint64_t)sum;
    if (tile == ntiles - 1) range_off[ntiles] = r1;
  }
}

inline unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_target_keys(const double* txyz, int64_t nslots, int64_t nside, uint32_t* keys,
                              uint32_t* vals, hipStream_t st) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_target_keys, dim3(blocks(nslots, 256)), dim3(256), 0, st, txyz, nslots,
                     nside, keys, vals);
  return hipGetLastError();
}

hipError_t launch_ref_disks(int64_t nside, int64_t reach, double rs, int2* tab, hipStream_t st) {
  const int64_t n = 4 * nside * (2 * reach + 1);
  hipLaunchKernelGGL(k_ref_disks, dim3(blocks(n, 256)), dim3(256), 0, st, nside, reach, rs, tab);
  return hipGetLastError();
}

hipError_t launch_run_flags(const uint32_t* keys, const uint32_t* nvalid, int64_t n,
                            uint64_t* flag, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_run_flags, dim3(blocks(n, 256)), dim3(256), 0, st, keys, nvalid, n, flag);
  return hipGetLastError();
}

hipError_t launch_run_compact(const uint32_t* keys, const uint32_t* nvalid, int64_t n,
                              const uint64_t* uoff, uint32_t* upix, uint32_t* ustart,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_run_compact, dim3(blocks(n, 256)), dim3(256), 0, st, keys, nvalid, n, uoff,
                     upix, ustart);
  return hipGetLastError();
}

hipError_t launch_disk_pairs(bool count, const uint32_t* upix, int64_t nu, int64_t nside,
                             int64_t reach, const int2* tab, const uint32_t* tkeys,
                             const uint32_t* tslot, const uint32_t* troff, const uint64_t* off,
                             uint64_t* cnt, uint32_t* pk, uint32_t* pv, hipStream_t st) {
  if (nu <= 0) return hipSuccess;
  if (count)
    hipLaunchKernelGGL(k_disk_pairs<true>, dim3(blocks(nu, 256)), dim3(256), 0, st, upix, nu,
                       nside, reach, tab, tkeys, tslot, troff, off, cnt, pk, pv);
  else
    hipLaunchKernelGGL(k_disk_pairs<false>, dim3(blocks(nu, 256)), dim3(256), 0, st, upix, nu,
                       nside, reach, tab, tkeys, tslot, troff, off, cnt, pk, pv);
  return hipGetLastError();
}

hipError_t launch_disk_ranges(const uint32_t* pk, const uint32_t* pv, int64_t np,
                              const uint32_t* ustart, uint64_t* flag, uint64_t* rsx,
                              uint64_t* scan_scratch,
                              int64_t ntiles, uint32_t* ranges, uint64_t* range_off,
                              uint32_t* nranges, uint64_t* ncand, hipStream_t st) {
  if (np > 0) {
    hipLaunchKernelGGL(k_range_flags, dim3(blocks(np, 256)), dim3(256), 0, st, pk, pv, np, flag);
  }
  hipError_t e = scan_u64_wide(flag, rsx, np, scan_scratch, st);
  if (e != hipSuccess) return e;
  if (np > 0) {
    hipLaunchKernelGGL(k_range_write, dim3(blocks(np, 256)), dim3(256), 0, st, pk, pv, np, rsx,
                       ustart, ranges);
  }
  if (ntiles > 0) {
    hipLaunchKernelGGL(k_tile_disk_ranges, dim3((unsigned)ntiles), dim3(64), 0, st, pk, np, rsx,
                       ntiles, ranges, range_off, nranges, ncand);
  }
  return hipGetLastError();
}

}  // namespace cg
