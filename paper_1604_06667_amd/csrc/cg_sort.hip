// Sample preparation, device radix sort and HEALPix ring offsets.
//
// Sect. 2.2 step 3a / Sect. 3.4 (1): every input sample gets its HEALPix
// index.  Sect. 3.4 inverts the sample -> target mapping into a target ->
// sample mapping; here the inversion is a stable sort of the samples by
// RING index, after which the samples of any pixel range of a ring form one
// contiguous run that two binary searches find.
#include "cg_internal.hpp"

namespace cg {

// ---------------------------------------------------------------------------
// prep: RING key per sample; invalid coordinates get the sentinel key Npix
// (sorted past every ring) and raise the sticky input flag.

template <typename T>
__device__ __forceinline__ float to_f32(const T* p, int64_t i);
template <>
__device__ __forceinline__ float to_f32<double>(const double* p, int64_t i) { return (float)p[i]; }
template <>
__device__ __forceinline__ float to_f32<float>(const float* p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ float to_f32<uint16_t>(const uint16_t* p, int64_t i) {
  return __uint_as_float(((uint32_t)p[i]) << 16);   // bfloat16 -> float (exact)
}
template <>
__device__ __forceinline__ float to_f32<_Float16>(const _Float16* p, int64_t i) { return (float)p[i]; }

// HEALPix RING key and value (the sample's own index) of every sample, and
// its record in input order: the unit vector and, when the cube has at most
// two channels, the channels as FP32 in the fourth word.  The permutation
// after the sort then reads one 32-byte record per sample instead of the
// separate longitude, latitude and data rows.
template <typename T>
__global__ void __launch_bounds__(256) k_prep(const double* __restrict__ lon,
                                              const double* __restrict__ lat, int64_t n,
                                              int64_t nside, uint32_t* __restrict__ keys,
                                              uint32_t* __restrict__ vals, int* flag,
                                              double4* __restrict__ rec,
                                              const T* __restrict__ data, int64_t ld, int npack) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = lon[i];
  const double d = lat[i];
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  uint32_t key;
  double4 r = make_double4(nan, nan, nan, 0.0);
  if (!(isfinite(a) && isfinite(d) && fabs(d) <= 90.0)) {
    key = (uint32_t)hpx::npix(nside);
    atomicOr(flag, 1);
  } else {
    double am = fmod(a, 360.0);
    if (am < 0.0) am += 360.0;
    const double phi = am * (hpx::kPi / 180.0);
    double sd, cd, sa, ca;
    sincos(d * (hpx::kPi / 180.0), &sd, &cd);
    sincos(phi, &sa, &ca);
    key = (uint32_t)hpx::ang2pix_ring(nside, sd, cd, phi);
    r.x = cd * ca;
    r.y = cd * sa;
    r.z = sd;
  }
  if (npack > 0) {
    const float d0 = to_f32<T>(data, i * ld);
    const float d1 = npack > 1 ? to_f32<T>(data, i * ld + 1) : 0.0f;
    r.w = __longlong_as_double((long long)(((uint64_t)__float_as_uint(d1) << 32) |
                                           (uint64_t)__float_as_uint(d0)));
  }
  keys[i] = key;
  vals[i] = (uint32_t)i;
  rec[i] = r;
}

hipError_t launch_prep(const double* lon, const double* lat, int64_t n, int64_t nside,
                       uint32_t* keys, uint32_t* vals, int* flag, double* rec, const void* data,
                       int dtype, int64_t ld, int npack, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 255) / 256)), blk(256);
  double4* r = reinterpret_cast<double4*>(rec);
  switch (dtype) {
    case 0:
      hipLaunchKernelGGL(k_prep<double>, grid, blk, 0, st, lon, lat, n, nside, keys, vals, flag, r,
                         (const double*)data, ld, npack);
      break;
    case 1:
      hipLaunchKernelGGL(k_prep<float>, grid, blk, 0, st, lon, lat, n, nside, keys, vals, flag, r,
                         (const float*)data, ld, npack);
      break;
    case 2:
      hipLaunchKernelGGL(k_prep<_Float16>, grid, blk, 0, st, lon, lat, n, nside, keys, vals, flag,
                         r, (const _Float16*)data, ld, npack);
      break;
    default:
      hipLaunchKernelGGL(k_prep<uint16_t>, grid, blk, 0, st, lon, lat, n, nside, keys, vals, flag,
                         r, (const uint16_t*)data, ld, npack);
      break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// LSD radix sort of (key, value) uint32 pairs, 8-bit digits.
// Per pass: block histograms (digit-major), one exclusive scan, and a
// stable scatter that ranks keys inside each wavefront with ballots.

constexpr int kMaxJobs = 256;   // the job pass sorts by one 8-bit digit

// Digit of element i: 8 key bits at `shift`, or (JOB) the job holding the
// value, i.e. its position in the concatenated order (job offsets in LDS).
template <bool JOB>
__device__ __forceinline__ uint32_t sort_digit(uint32_t key, uint32_t val, int shift,
                                               const int64_t* s_off, int njobs) {
  if constexpr (JOB) return (uint32_t)job_of(s_off, njobs, (int64_t)val);
  else return (key >> shift) & 255u;
}

template <bool JOB>
__device__ __forceinline__ void stage_job_offsets(int64_t* s_off, const int64_t* joff, int njobs) {
  if constexpr (JOB) {
    for (int k = threadIdx.x; k <= njobs; k += blockDim.x) s_off[k] = joff[k];
    __syncthreads();
  }
}

template <bool JOB>
__global__ void __launch_bounds__(kSortThreads) k_hist(const uint32_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ vals, int64_t n,
                                                       int shift, uint32_t* __restrict__ hist,
                                                       int64_t nblocks, const int64_t* joff,
                                                       int njobs) {
  __shared__ uint32_t h[256];
  __shared__ int64_t s_off[JOB ? kMaxJobs + 1 : 1];
  const int t = threadIdx.x;
  h[t] = 0;
  stage_job_offsets<JOB>(s_off, joff, njobs);
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + t;
    if (i < n) {
      const uint32_t d = sort_digit<JOB>(JOB ? 0u : keys[i], JOB ? vals[i] : 0u, shift, s_off, njobs);
      atomicAdd(&h[d], 1u);
    }
  }
  __syncthreads();
  hist[(int64_t)t * nblocks + blockIdx.x] = h[t];
}

// Exclusive scan of each digit's per-block counts (one workgroup per digit,
// coalesced), leaving the digit totals in totals[256].  Each pass over 1024
// counts gives every thread four consecutive ones; the threads' sums are
// scanned by shuffles within each wavefront and the four wavefront sums
// are combined through LDS, one barrier per pass.
__global__ void __launch_bounds__(256) k_digit_scan(uint32_t* __restrict__ hist, int64_t nblocks,
                                                    uint32_t* __restrict__ totals) {
  __shared__ uint32_t s_w[2][4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  uint32_t* h = hist + (int64_t)blockIdx.x * nblocks;
  uint32_t carry = 0;
  int buf = 0;
  for (int64_t b0 = 0; b0 < nblocks; b0 += 1024, buf ^= 1) {
    const int64_t i0 = b0 + 4 * (int64_t)t;
    uint32_t v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = i0 + q < nblocks ? h[i0 + q] : 0u;
    const uint32_t local = v[0] + v[1] + v[2] + v[3];
    uint32_t incl = local;   // inclusive scan of the threads' sums in the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) s_w[buf][w] = incl;
    __syncthreads();   // (double-buffered sums: the next pass writes the other half)
    uint32_t wbase = 0;
    for (int k = 0; k < w; ++k) wbase += s_w[buf][k];
    uint32_t run = carry + wbase + (incl - local);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (i0 + q < nblocks) h[i0 + q] = run;
      run += v[q];
    }
    carry += s_w[buf][0] + s_w[buf][1] + s_w[buf][2] + s_w[buf][3];
  }
  if (t == 0) totals[blockIdx.x] = carry;
}

// Scatter of one block of kSortTile pairs.  The pairs are first ranked
// stably by digit (ballots inside each wavefront, a prefix over wavefronts
// per round) and placed in LDS in block-sorted order; the block then writes
// them out in that order, so that each digit's run of the block goes to
// consecutive global positions (whole segments instead of one scattered
// 4-byte store per pair).
template <bool JOB>
__global__ void __launch_bounds__(kSortThreads) k_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, int64_t n, int shift,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ totals, int64_t nblocks,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, const int64_t* joff, int njobs) {
  constexpr int NW = kSortThreads / 64;
  __shared__ uint32_t gbase[256];     // global position of the block's first pair of digit d
  __shared__ uint32_t lrun[256];      // pairs of digit d ranked so far, then local offsets
  __shared__ uint32_t wcnt[NW][256];
  __shared__ uint32_t sk[kSortTile], sv[kSortTile];
  __shared__ int64_t s_off[JOB ? kMaxJobs + 1 : 1];
  const int t = threadIdx.x;
  stage_job_offsets<JOB>(s_off, joff, njobs);
  const int lane = t & 63;
  const int w = t >> 6;
  {
    // digit bases: exclusive scan of the 256 digit totals
    const uint32_t v = totals[t];
    gbase[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const uint32_t u = t >= off ? gbase[t - off] : 0u;
      __syncthreads();
      gbase[t] += u;
      __syncthreads();
    }
    const uint32_t excl = gbase[t] - v;
    __syncthreads();
    gbase[t] = excl + hist[(int64_t)t * nblocks + blockIdx.x];
    lrun[t] = 0u;
  }
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t blk = (int64_t)blockIdx.x * kSortTile;
  uint32_t key[kSortItems], val[kSortItems], dig[kSortItems], lpos[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = blk + (int64_t)r * kSortThreads + t;
    const bool valid = i < n;
    key[r] = valid ? kin[i] : 0u;
    val[r] = valid ? vin[i] : 0u;
  }
  // ranking: round r holds the pairs blk + r * kSortThreads + (0 .. kSortThreads - 1)
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const bool valid = blk + (int64_t)r * kSortThreads + t < n;
    const uint32_t d = valid ? sort_digit<JOB>(key[r], val[r], shift, s_off, njobs) : 0u;
    dig[r] = d;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
    for (int k = t; k < NW * 256; k += kSortThreads) (&wcnt[0][0])[k] = 0u;
    __syncthreads();
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    {
      uint32_t run = lrun[t];
#pragma unroll
      for (int q = 0; q < NW; ++q) {
        const uint32_t c = wcnt[q][t];
        wcnt[q][t] = run;
        run += c;
      }
      lrun[t] = run;
    }
    __syncthreads();
    lpos[r] = wcnt[w][d] + rank;
    __syncthreads();
  }
  // local offsets: exclusive scan of the block's digit counts
  {
    const uint32_t v = lrun[t];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const uint32_t u = t >= off ? lrun[t - off] : 0u;
      __syncthreads();
      lrun[t] += u;
      __syncthreads();
    }
    const uint32_t excl = lrun[t] - v;
    __syncthreads();
    lrun[t] = excl;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    if (blk + (int64_t)r * kSortThreads + t < n) {
      const uint32_t p = lrun[dig[r]] + lpos[r];
      sk[p] = key[r];
      sv[p] = val[r];
    }
  }
  __syncthreads();
  const int nb = (int)((n - blk) < (int64_t)kSortTile ? (n - blk) : (int64_t)kSortTile);
  for (int j = t; j < nb; j += kSortThreads) {
    const uint32_t k = sk[j], v = sv[j];
    const uint32_t d = sort_digit<JOB>(k, v, shift, s_off, njobs);
    const uint32_t pos = gbase[d] + ((uint32_t)j - lrun[d]);
    kout[pos] = k;
    vout[pos] = v;
  }
}

size_t radix_hist_elems(int64_t n) {
  const int64_t nb = (n + kSortTile - 1) / kSortTile;
  return (size_t)(nb < 1 ? 1 : nb) * 256 + 256;
}

static void sort_pass(bool job, uint32_t*& ki, uint32_t*& vi, uint32_t*& ko, uint32_t*& vo,
                      uint32_t* hist, int64_t n, int64_t nb, int shift, const int64_t* joff,
                      int njobs, hipStream_t st) {
  uint32_t* totals = hist + nb * 256;
  if (job) {
    hipLaunchKernelGGL(k_hist<true>, dim3((unsigned)nb), dim3(kSortThreads), 0, st, ki, vi, n,
                       shift, hist, nb, joff, njobs);
  } else {
    hipLaunchKernelGGL(k_hist<false>, dim3((unsigned)nb), dim3(kSortThreads), 0, st, ki, vi, n,
                       shift, hist, nb, joff, njobs);
  }
  hipLaunchKernelGGL(k_digit_scan, dim3(256), dim3(256), 0, st, hist, nb, totals);
  if (job) {
    hipLaunchKernelGGL(k_scatter<true>, dim3((unsigned)nb), dim3(kSortThreads), 0, st, ki, vi, n,
                       shift, hist, totals, nb, ko, vo, joff, njobs);
  } else {
    hipLaunchKernelGGL(k_scatter<false>, dim3((unsigned)nb), dim3(kSortThreads), 0, st, ki, vi, n,
                       shift, hist, totals, nb, ko, vo, joff, njobs);
  }
  uint32_t* tk = ki; ki = ko; ko = tk;
  uint32_t* tv = vi; vi = vo; vo = tv;
}

hipError_t radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp,
                      uint32_t* hist, int64_t n, int bits, bool* result_in_tmp, hipStream_t st) {
  return radix_sort_jobs(keys, vals, keys_tmp, vals_tmp, hist, n, bits, nullptr, 0, result_in_tmp,
                         st);
}

hipError_t radix_sort_jobs(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp,
                           uint32_t* hist, int64_t n, int bits, const int64_t* noff, int njobs,
                           bool* result_in_tmp, hipStream_t st) {
  *result_in_tmp = false;
  if (n <= 1) return hipSuccess;
  if (njobs > kMaxJobs) return hipErrorInvalidValue;
  const int64_t nb = (n + kSortTile - 1) / kSortTile;
  uint32_t *ki = keys, *vi = vals, *ko = keys_tmp, *vo = vals_tmp;
  bool in_tmp = false;
  for (int shift = 0; shift < bits; shift += 8) {
    sort_pass(false, ki, vi, ko, vo, hist, n, nb, shift, noff, njobs, st);
    in_tmp = !in_tmp;
  }
  if (njobs > 1) {
    sort_pass(true, ki, vi, ko, vo, hist, n, nb, 0, noff, njobs, st);
    in_tmp = !in_tmp;
  }
  *result_in_tmp = in_tmp;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batches: the samples of all jobs in one concatenated order (job j at
// [noff[j], noff[j + 1])), each keyed with its own job's nside.

__global__ void __launch_bounds__(256) k_batch_prep(const BatchJob* __restrict__ jobs,
                                                    const int64_t* __restrict__ noff, int njobs,
                                                    int64_t ntot, uint32_t* __restrict__ keys,
                                                    uint32_t* __restrict__ vals, int* flag) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ntot) return;
  const int j = job_of(noff, njobs, g);
  const BatchJob& jb = jobs[j];
  const int64_t i = g - jb.noff;
  const double a = jb.lon[i];
  const double d = jb.lat[i];
  uint32_t key;
  if (!(isfinite(a) && isfinite(d) && fabs(d) <= 90.0)) {
    key = (uint32_t)hpx::npix(jb.nside);
    atomicOr(flag, 1);
  } else {
    double am = fmod(a, 360.0);
    if (am < 0.0) am += 360.0;
    double sd, cd;
    sincos(d * (hpx::kPi / 180.0), &sd, &cd);
    key = (uint32_t)hpx::ang2pix_ring(jb.nside, sd, cd, am * (hpx::kPi / 180.0));
  }
  keys[g] = key;
  vals[g] = (uint32_t)g;
}

hipError_t launch_batch_prep(const BatchJob* jobs, const int64_t* noff, int njobs, int64_t ntot,
                             uint32_t* keys, uint32_t* vals, int* flag, hipStream_t st) {
  if (ntot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_prep, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, st, jobs,
                     noff, njobs, ntot, keys, vals, flag);
  return hipGetLastError();
}

// ring offsets of every job: entry e of job j (ring i = e - rooff[j]) is the
// first position of the job's sorted run whose key is >= ring_start(i); entry
// 4 nside is the end of its valid samples.
__global__ void __launch_bounds__(256) k_batch_ring_offsets(const BatchJob* __restrict__ jobs,
                                                            const int64_t* __restrict__ rooff,
                                                            int njobs,
                                                            const uint32_t* __restrict__ keys,
                                                            uint32_t* __restrict__ ring_off) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rooff[njobs]) return;
  const int j = job_of(rooff, njobs, e);
  const BatchJob& jb = jobs[j];
  const int64_t i = e - rooff[j];
  int64_t lo = jb.noff, hi = jb.noff + jb.n;
  if (i > 0) {
    const uint64_t target = (uint64_t)hpx::ring_start(jb.nside, i);
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((uint64_t)keys[mid] < target) lo = mid + 1;
      else hi = mid;
    }
  }
  ring_off[e] = (uint32_t)lo;
}

hipError_t launch_batch_ring_offsets(const BatchJob* jobs, const int64_t* rooff, int njobs,
                                     int64_t nentries, const uint32_t* keys, uint32_t* ring_off,
                                     hipStream_t st) {
  if (nentries <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_ring_offsets, dim3((unsigned)((nentries + 255) / 256)), dim3(256), 0,
                     st, jobs, rooff, njobs, keys, ring_off);
  return hipGetLastError();
}

// sorted unit vectors of every job's valid samples
__global__ void __launch_bounds__(256) k_batch_permute(const BatchJob* __restrict__ jobs,
                                                       const int64_t* __restrict__ noff, int njobs,
                                                       int64_t ntot,
                                                       const uint32_t* __restrict__ vals,
                                                       const uint32_t* __restrict__ ring_off,
                                                       double4* __restrict__ srec) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ntot) return;
  const int j = job_of(noff, njobs, p);
  const BatchJob& jb = jobs[j];
  if (p >= (int64_t)ring_off[jb.ro_off + 4 * jb.nside]) return;   // invalid samples sort last
  const int64_t src = (int64_t)vals[p] - jb.noff;
  double am = fmod(jb.lon[src], 360.0);
  if (am < 0.0) am += 360.0;
  double sa, ca, sd, cd;
  sincos(am * (hpx::kPi / 180.0), &sa, &ca);
  sincos(jb.lat[src] * (hpx::kPi / 180.0), &sd, &cd);
  // the row is the job's own input index
  srec[p] = make_double4(cd * ca, cd * sa, sd, __longlong_as_double(src));
}

hipError_t launch_batch_permute(const BatchJob* jobs, const int64_t* noff, int njobs, int64_t ntot,
                                const uint32_t* vals, const uint32_t* ring_off, double* srec,
                                hipStream_t st) {
  if (ntot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_permute, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, st,
                     jobs, noff, njobs, ntot, vals, ring_off, reinterpret_cast<double4*>(srec));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ring_off[i] = first sorted position whose key is >= ring_start(i), for
// i = 1 .. 4 nside; ring_off[4 nside] is the number of valid samples.

__global__ void __launch_bounds__(256) k_ring_offsets(const uint32_t* __restrict__ keys, int64_t n,
                                                      int64_t nside, uint32_t* __restrict__ ring_off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
  if (i > 4 * nside) return;
  const uint64_t target = (uint64_t)hpx::ring_start(nside, i);
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((uint64_t)keys[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  ring_off[i] = (uint32_t)lo;
  if (i == 1) ring_off[0] = 0;
}

hipError_t launch_ring_offsets(const uint32_t* keys, int64_t n, int64_t nside, uint32_t* ring_off,
                               hipStream_t st) {
  const int64_t cnt = 4 * nside;
  hipLaunchKernelGGL(k_ring_offsets, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, keys, n,
                     nside, ring_off);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// permute: sorted unit vectors (SoA) and, for narrow cubes, the data rows in
// sorted order converted to FP32 (so the gather streams contiguous rows).

template <typename T, bool VEC4>
__global__ void __launch_bounds__(256) k_permute(const uint32_t* __restrict__ vals,
                                                 const uint32_t* __restrict__ nvalid_p,
                                                 const double4* __restrict__ rec,
                                                 const T* __restrict__ data, int64_t ld,
                                                 int64_t nchan, int with_data, int npack,
                                                 double4* __restrict__ srec,
                                                 float* __restrict__ sdata) {
  const int64_t nvalid = (int64_t)(*nvalid_p);
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nvalid) return;
  const int64_t src = vals[p];
  const double4 r = rec[src];
  srec[p] = make_double4(r.x, r.y, r.z, __longlong_as_double(src));
  if (with_data) {
    if (npack > 0) {
      // channels carried in the record
      const uint64_t b = (uint64_t)__double_as_longlong(r.w);
      sdata[p * nchan] = __uint_as_float((uint32_t)b);
      if (npack > 1) sdata[p * nchan + 1] = __uint_as_float((uint32_t)(b >> 32));
    } else if constexpr (VEC4) {
      // FP32 rows with nchan and ld multiples of 4 and 16-byte aligned: whole
      // 16-byte pieces per load and store
      const float4* in = reinterpret_cast<const float4*>(data + src * ld);
      float4* out = reinterpret_cast<float4*>(sdata + p * nchan);
      for (int64_t c = 0; c < nchan / 4; ++c) out[c] = in[c];
    } else {
      for (int64_t c = 0; c < nchan; ++c) sdata[p * nchan + c] = to_f32<T>(data, src * ld + c);
    }
  }
}

hipError_t launch_permute(const uint32_t* vals, const uint32_t* nvalid_dev, int64_t n,
                          const double* rec, const void* data, int dtype, int64_t ld,
                          int64_t nchan, bool with_data, int npack, double* srec,
                          float* sdata, hipStream_t st) {
  // nvalid_dev points at the number of valid samples (ring_off[4 nside]);
  // the grid covers all n sorted entries and threads past it return.
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 255) / 256)), blk(256);
  const int wd = with_data ? 1 : 0;
  const double4* r = reinterpret_cast<const double4*>(rec);
  double4* sr = reinterpret_cast<double4*>(srec);
  switch (dtype) {
    case 0:
      hipLaunchKernelGGL((k_permute<double, false>), grid, blk, 0, st, vals, nvalid_dev, r,
                         (const double*)data, ld, nchan, wd, npack, sr, sdata);
      break;
    case 1:
      if (wd && nchan % 4 == 0 && ld % 4 == 0 && ((uintptr_t)data & 15) == 0)
        hipLaunchKernelGGL((k_permute<float, true>), grid, blk, 0, st, vals, nvalid_dev, r,
                           (const float*)data, ld, nchan, wd, npack, sr, sdata);
      else
        hipLaunchKernelGGL((k_permute<float, false>), grid, blk, 0, st, vals, nvalid_dev, r,
                           (const float*)data, ld, nchan, wd, npack, sr, sdata);
      break;
    case 2:
      hipLaunchKernelGGL((k_permute<_Float16, false>), grid, blk, 0, st, vals, nvalid_dev, r,
                         (const _Float16*)data, ld, nchan, wd, npack, sr, sdata);
      break;
    default:
      hipLaunchKernelGGL((k_permute<uint16_t, false>), grid, blk, 0, st, vals, nvalid_dev, r,
                         (const uint16_t*)data, ld, nchan, wd, npack, sr, sdata);
      break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exclusive scan of uint64 counts (tile candidate offsets); out has n + 1
// entries, out[n] = total.

__global__ void __launch_bounds__(1024) k_scan_u64(const uint64_t* __restrict__ in,
                                                   uint64_t* __restrict__ out, int64_t n) {
  // one workgroup walks the array in coalesced rounds of 1024 x 4 values,
  // each round a block scan on top of the running total
  __shared__ uint64_t part[1024];
  const int t = threadIdx.x;
  uint64_t carry = 0;
  for (int64_t r0 = 0; r0 < n; r0 += 4096) {
    uint64_t v[4];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t i = r0 + 4 * (int64_t)t + k;
      v[k] = i < n ? in[i] : 0ull;
      s += v[k];
    }
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const uint64_t u = t >= off ? part[t - off] : 0ull;
      __syncthreads();
      part[t] += u;
      __syncthreads();
    }
    uint64_t run = carry + part[t] - s;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t i = r0 + 4 * (int64_t)t + k;
      if (i < n) out[i] = run;
      run += v[k];
    }
    carry += part[1023];
    __syncthreads();
  }
  if (t == 0) out[n] = carry;
}

hipError_t scan_u64(const uint64_t* in, uint64_t* out, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_u64, dim3(1), dim3(1024), 0, st, in, out, n);
  return hipGetLastError();
}

// Device-wide exclusive scan for long arrays: blocks of kScanBlock values
// are summed, the block sums scanned by k_scan_u64, then every block scans
// its own values on top of its offset.
constexpr int kScanBlock = 4096;

__global__ void __launch_bounds__(1024) k_scan_partials(const uint64_t* __restrict__ in, int64_t n,
                                                        uint64_t* __restrict__ part) {
  __shared__ uint64_t red[1024];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + 4 * (int64_t)t + k;
    if (i < n) s += in[i];
  }
  red[t] = s;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  if (t == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(1024) k_scan_apply(const uint64_t* __restrict__ in,
                                                     uint64_t* __restrict__ out, int64_t n,
                                                     const uint64_t* __restrict__ poff,
                                                     int64_t nb) {
  __shared__ uint64_t part[1024];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  uint64_t v[4];
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + 4 * (int64_t)t + k;
    v[k] = i < n ? in[i] : 0ull;
    s += v[k];
  }
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint64_t u = t >= off ? part[t - off] : 0ull;
    __syncthreads();
    part[t] += u;
    __syncthreads();
  }
  uint64_t run = poff[blockIdx.x] + part[t] - s;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + 4 * (int64_t)t + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (blockIdx.x == 0 && t == 0) out[n] = poff[nb];
}

size_t scan_u64_wide_scratch(int64_t n) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  return (size_t)(2 * nb + 1);
}

hipError_t scan_u64_wide(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* scratch,
                         hipStream_t st) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb <= 1) return scan_u64(in, out, n, st);
  uint64_t* part = scratch;
  uint64_t* poff = scratch + nb;
  hipLaunchKernelGGL(k_scan_partials, dim3((unsigned)nb), dim3(1024), 0, st, in, n, part);
  hipLaunchKernelGGL(k_scan_u64, dim3(1), dim3(1024), 0, st, part, poff, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(1024), 0, st, in, out, n, poff, nb);
  return hipGetLastError();
}

}  // namespace cg
