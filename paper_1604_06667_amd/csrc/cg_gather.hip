// FP32 gather contraction, neighbour statistics and normalisation.
//
// Eq. (1)-(2): for every target t of a tile, S_t[c] += R_n[c] w and
// W_t += w over the tile's candidate samples n with d <= r_s.  Each tile's
// outputs are owned by one workgroup, so no atomics are needed (the
// ownership argument of Sect. 2.2).  The support test is FP64 on unit
// vectors; weights are FP32; products and sums are FP64 (an FP32 weight
// times an FP32 value is exact in FP64), so the result does not depend on
// the order in which candidates arrive, even where the sums cancel.
#include "cg_internal.hpp"

namespace cg {

constexpr int kChunk = 64;   // candidates staged per step

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Target-frame axes for the elliptical kernel: east e = (-sin a, cos a, 0),
// north n = (-sin d cos a, -sin d sin a, cos d); major axis along
// cos(pa) n + sin(pa) e, minor axis along cos(pa) e - sin(pa) n.
__device__ __forceinline__ void target_axes(const KernelParams& kp, double lon, double lat,
                                            double* a, double* b) {
  double sa, ca, sd, cd;
  sincos(lon, &sa, &ca);
  sincos(lat, &sd, &cd);
  const double ex = -sa, ey = ca, ez = 0.0;
  const double nx = -sd * ca, ny = -sd * sa, nz = cd;
  a[0] = kp.cospa * nx + kp.sinpa * ex;
  a[1] = kp.cospa * ny + kp.sinpa * ey;
  a[2] = kp.cospa * nz + kp.sinpa * ez;
  b[0] = kp.cospa * ex - kp.sinpa * nx;
  b[1] = kp.cospa * ey - kp.sinpa * ny;
  b[2] = kp.cospa * ez - kp.sinpa * nz;
}

__device__ __forceinline__ float qnan_f() { return __int_as_float(0x7fc00000); }

// ---------------------------------------------------------------------------
// Narrow data (nchan <= CMAX <= 16): one lane per target.  A chunk of
// candidates and their (sorted, FP32) data rows is staged in LDS; each lane
// first marks, in a 64-bit mask, the candidates within the support of its
// target (FP64 test), then walks only its own marked candidates: weight and
// channel products for those pairs alone, with no lane idling on the pairs
// of other targets.  Sums per lane run in the tile's visit order (see the
// loop), the same on every call.

template <int CMAX, bool RADIAL>
__global__ void __launch_bounds__(64) k_gather_tl(TileView tv, KernelParams kp,
                                                  const float* __restrict__ sdata, int64_t nchan,
                                                  OutView ov) {
  const int64_t tile = tile_of_block(blockIdx.x, tv.ntiles);
  const int lane = threadIdx.x;
  const int64_t slot = tile * kTile + lane;
  __shared__ double s_x[kChunk], s_y[kChunk], s_z[kChunk];
  __shared__ double s_d[kChunk * CMAX];
  const int64_t ns = tv.nslots;
  const double tx = tv.txyz[slot], ty = tv.txyz[ns + slot], tz = tv.txyz[2 * ns + slot];
  double ax[3] = {0.0, 0.0, 0.0}, bx[3] = {0.0, 0.0, 0.0};
  if (kp.type == 1 && isfinite(tx)) target_axes(kp, tv.tll[slot], tv.tll[ns + slot], ax, bx);
  double acc[CMAX];
#pragma unroll
  for (int c = 0; c < CMAX; ++c) acc[c] = 0.0;
  double wacc = 0.0;
  const uint32_t total = (uint32_t)tv.ntot[tile];
  const uint32_t nr = tv.nr[tile];
  const uint32_t* rng = tv.rng + 2 * tv.roff[tile];   // per range: first sorted position, first candidate index
  const double thr = 1.0 - 0.5 * kp.cs2 - 2e-15;
  // Visit order.  The candidates are sorted ring by ring, and only the
  // lanes whose target lies near a ring have pairs in its stretch, so a
  // chunk of consecutive candidates would leave most lanes idle while a few
  // walk their marked pairs.  The tile is therefore visited interleaved:
  // chunk ci takes candidates ci, nch + ci, 2 nch + ci, ..., one from each
  // 64th of the list, so every lane finds about its average share of pairs
  // in every chunk.  Lane j loads the candidates of its 64th in order,
  // following the ranges with a cursor of its own: it finds the range of
  // its first candidate by a binary search and, ranges being non-empty,
  // steps to the next range at most once per chunk.
  const uint32_t nch = (total + kChunk - 1) / kChunk;
  const uint64_t q0 = (uint64_t)lane * nch;
  uint32_t rb = 0, rs = 0, re = 0, ri = 0;   // cursor: range ri = positions rb.. for candidates [rs, re)
  if (q0 < total) {
    uint32_t lo = 0, hi = nr - 1;   // last range whose first candidate index is <= q0
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (rng[2 * mid + 1] <= q0) lo = mid;
      else hi = mid - 1;
    }
    ri = lo;
    rb = rng[2 * ri];
    rs = rng[2 * ri + 1];
    re = ri + 1 < nr ? rng[2 * ri + 3] : total;
  }
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  for (uint32_t ci = 0; ci < nch; ++ci) {
    const uint64_t q = q0 + ci;
    if (q < total) {
      while (q >= re) {   // re < total here, so range ri + 1 exists
        ++ri;
        rb = rng[2 * ri];
        rs = re;
        re = ri + 1 < nr ? rng[2 * ri + 3] : total;
      }
      const int64_t pos = (int64_t)rb + (int64_t)(q - rs);
      const double4 r = tv.srec[pos];
      s_x[lane] = r.x;
      s_y[lane] = r.y;
      s_z[lane] = r.z;
      // every slot of the row is written (zeros past nchan), so the walk
      // reads and multiplies all CMAX slots without a branch per channel
#pragma unroll
      for (int c = 0; c < CMAX; ++c)
        s_d[lane * CMAX + c] = c < nchan ? (double)sdata[pos * nchan + c] : 0.0;
    } else {
      s_x[lane] = s_y[lane] = s_z[lane] = nan;   // no candidate: no test marks it
    }
    __syncthreads();
    // candidates of the chunk that may lie within the support of this lane's
    // target: p_n . p_t >= 1 - cs2/2 (the same cut, as |p_n - p_t|^2 =
    // 2 - 2 p_n . p_t for unit vectors) loosened by 2e-15, which covers the
    // few-ulp deviation of the rounded vectors from unit length and the
    // rounding of the dot product, so the marked set is a superset.  The
    // exact FP64 chord test below decides every marked pair.
    uint64_t inside = 0;
#pragma unroll
    for (int k = kChunk - 1; k >= 0; --k) {
      const double dot = fma(s_x[k], tx, fma(s_y[k], ty, s_z[k] * tz));
      inside = (inside << 1) | (uint64_t)(dot >= thr);
    }
    while (inside) {
      const int k = __builtin_ctzll(inside);
      inside &= inside - 1;
      const double dx = s_x[k] - tx, dy = s_y[k] - ty, dz = s_z[k] - tz;
      const double c2 = dx * dx + dy * dy + dz * dz;
      const double w = c2 <= kp.cs2 ? (double)pair_weight<RADIAL>(kp, c2, dx, dy, dz, ax[0], ax[1],
                                                                   ax[2], bx[0], bx[1], bx[2])
                                    : 0.0;
      wacc += w;
#pragma unroll
      for (int c = 0; c < CMAX; ++c) acc[c] = fma(w, s_d[k * CMAX + c], acc[c]);
    }
    __syncthreads();
  }
  if (ov.mode == ACC_FINAL) {
    const int32_t t = ov.slot_target[slot];
    if (t >= 0) {
      for (int c = 0; c < CMAX && c < nchan; ++c)
        ov.cube[(int64_t)c * ov.cst + (int64_t)t * ov.tst] =
            wacc > 0.0 ? (float)(acc[c] / wacc) : qnan_f();
      if (ov.wout) ov.wout[t] = (float)wacc;
    }
  } else {
    const bool add = ov.mode == ACC_ADD;
    for (int c = 0; c < CMAX && c < nchan; ++c) {
      double* s = ov.S + (int64_t)c * ns + slot;
      *s = add ? *s + acc[c] : acc[c];
    }
    ov.W[slot] = add ? ov.W[slot] + wacc : wacc;
    ov.Wn[slot] = add ? ov.Wn[slot] + wacc : wacc;
  }
}

// ---------------------------------------------------------------------------
// Wide data: 8 wavefronts x 8 targets per tile, lanes own VEC consecutive
// channels of a 64*VEC channel block (grid.y).  A chunk of 64 candidates
// and their data rows (read through the sort permutation) are staged in
// LDS; for each target the lanes evaluate the 64 weights in parallel and the
// wavefront then walks only the candidates inside the support.

template <typename T>
__device__ __forceinline__ float ld_f32(const T* p);
template <>
__device__ __forceinline__ float ld_f32<float>(const float* p) { return *p; }
template <>
__device__ __forceinline__ float ld_f32<double>(const double* p) { return (float)*p; }
template <>
__device__ __forceinline__ float ld_f32<uint16_t>(const uint16_t* p) {
  return __uint_as_float(((uint32_t)*p) << 16);
}
template <>
__device__ __forceinline__ float ld_f32<_Float16>(const _Float16* p) { return (float)*p; }

template <int VEC, typename T>
__device__ __forceinline__ void load_row_vec(const T* __restrict__ p, int nvalid, bool vec_ok,
                                             float* out) {
  if (vec_ok && nvalid >= VEC) {
    if constexpr (sizeof(T) == 4 && VEC == 4) {
      const float4 v = *reinterpret_cast<const float4*>(p);
      out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
      return;
    } else if constexpr (sizeof(T) == 2 && VEC == 4) {
      const uint2 v = *reinterpret_cast<const uint2*>(p);
      const uint16_t h[4] = {(uint16_t)(v.x & 0xffff), (uint16_t)(v.x >> 16),
                             (uint16_t)(v.y & 0xffff), (uint16_t)(v.y >> 16)};
#pragma unroll
      for (int i = 0; i < 4; ++i) out[i] = ld_f32<T>(reinterpret_cast<const T*>(&h[i]));
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < VEC; ++i) out[i] = (i < nvalid) ? ld_f32<T>(p + i) : 0.0f;
}

template <int VEC, int KT, typename T>
__global__ void __launch_bounds__(512) k_gather_cl(TileView tv, KernelParams kp,
                                                   const T* __restrict__ data, int64_t ld,
                                                   int64_t nchan, int vec_ok_in, OutView ov) {
  constexpr int CB = 64 * VEC;
  constexpr int NWV = 8;    // wavefronts per workgroup
  constexpr int TPW = kTile / NWV;   // targets per wavefront
  __shared__ double s_x[kChunk], s_y[kChunk], s_z[kChunk];
  __shared__ int64_t s_row[kChunk];
  __shared__ __attribute__((aligned(16))) float s_d[kChunk * CB];
  __shared__ double s_t[kTile][9];   // target xyz, major axis, minor axis
  __shared__ double s_w[kTile];
  int64_t tile, pass;
  work_of_block(blockIdx.x, tv.ntiles, (nchan + CB - 1) / CB, &tile, &pass);
  const int64_t c0 = pass * CB;
  const int t = threadIdx.x, lane = t & 63, wv_id = t >> 6;
  const int64_t ns = tv.nslots;
  if (t < kTile) {
    const int64_t slot = tile * kTile + t;
    const double x = tv.txyz[slot];
    s_t[t][0] = x;
    s_t[t][1] = tv.txyz[ns + slot];
    s_t[t][2] = tv.txyz[2 * ns + slot];
    double a[3] = {0.0, 0.0, 0.0}, b[3] = {0.0, 0.0, 0.0};
    if (KT == 1 && isfinite(x)) target_axes(kp, tv.tll[slot], tv.tll[ns + slot], a, b);
    s_t[t][3] = a[0]; s_t[t][4] = a[1]; s_t[t][5] = a[2];
    s_t[t][6] = b[0]; s_t[t][7] = b[1]; s_t[t][8] = b[2];
  }
  const int col = lane * VEC;
  const int nvalid_c = (int)((nchan - c0 - col) < VEC ? (nchan - c0 - col) : VEC);
  const bool vec_ok = vec_ok_in != 0;
  double acc[TPW][VEC];
  double wl[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    wl[i] = 0.0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[i][v] = 0.0;
  }
  const uint32_t total = (uint32_t)tv.ntot[tile];
  RangeWindow<false> rw;   // used by wavefront 0, which stages the candidates
  if (wv_id == 0) rw.init(tv.rng + 2 * tv.roff[tile], tv.nr[tile], total, true);
  for (uint32_t base = 0; base < total; base += kChunk) {
    const int kmax = (int)(total - base < (uint32_t)kChunk ? total - base : (uint32_t)kChunk);
    if (wv_id == 0) {
      rw.cover(base, base + kmax - 1, true);
      const int64_t pos = rw.pos(base + (t < kmax ? t : kmax - 1), base, base + kmax - 1);
      if (t < kmax) {
        const double4 r = tv.srec[pos];
        s_x[t] = r.x;
        s_y[t] = r.y;
        s_z[t] = r.z;
        s_row[t] = rec_row(r) * ld;
      }
    }
    __syncthreads();
    for (int r = wv_id; r < kmax; r += NWV) {
      float v[VEC];
      if (nvalid_c > 0) load_row_vec<VEC, T>(data + s_row[r] + c0 + col, nvalid_c, vec_ok, v);
      else {
#pragma unroll
        for (int i = 0; i < VEC; ++i) v[i] = 0.0f;
      }
#pragma unroll
      for (int i = 0; i < VEC; ++i) s_d[r * CB + col + i] = v[i];
    }
    __syncthreads();
    double cxv = 0.0, cyv = 0.0, czv = 0.0;
    if (lane < kmax) { cxv = s_x[lane]; cyv = s_y[lane]; czv = s_z[lane]; }
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int tt = wv_id * TPW + i;
      // keep the per-target LDS reads inside the loop (no hoisting of all 16 targets)
      __asm__ volatile("" ::: "memory");
      float w = 0.0f;
      if (lane < kmax) {
        const double dx = cxv - s_t[tt][0], dy = cyv - s_t[tt][1], dz = czv - s_t[tt][2];
        const double c2 = dx * dx + dy * dy + dz * dz;
        if (c2 <= kp.cs2) {
          if (KT == 0)
            w = exp2_neg(chord2_to_d2_for(kp, c2) * kp.k1);
          else
            w = pair_weight<KT == 3>(kp, c2, dx, dy, dz, s_t[tt][3], s_t[tt][4], s_t[tt][5], s_t[tt][6],
                            s_t[tt][7], s_t[tt][8]);
        }
      }
      wl[i] += (double)w;
      uint64_t m = __ballot(w != 0.0f);
      while (m) {
        const int k = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const double wk = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(w), k));
        const float* dp = &s_d[k * CB + col];
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[i][v] = fma(wk, (double)dp[v], acc[i][v]);
      }
    }
    __syncthreads();
  }
  // weight sums: lanes held one candidate each
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const double s = wsum(wl[i]);
    if (lane == 0) s_w[wv_id * TPW + i] = s;
  }
  __syncthreads();
  // transpose the tile's [target][channel] block through LDS (as FP64, in
  // two halves of 32 targets): s_dd[c][target]
  const bool fin = ov.mode == ACC_FINAL;
  const bool tmaj = fin && ov.tst != 1;
  double* s_dd = reinterpret_cast<double*>(s_d);
  static_assert(sizeof(s_d) >= sizeof(double) * CB * (kTile / 2), "transpose buffer");
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    if (half) __syncthreads();
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int tt = wv_id * TPW + i;
      if ((tt >> 5) != half) continue;
      const double wt = s_w[tt];
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        double o;
        if (fin) o = wt > 0.0 ? acc[i][v] / wt : (double)qnan_f();
        else o = acc[i][v];
        s_dd[(col + v) * (kTile / 2) + (tt & 31)] = o;
      }
    }
    __syncthreads();
    // consecutive threads write consecutive targets of a channel, or (target-
    // major cubes) consecutive channels of a target
    for (int idx = t; idx < CB * (kTile / 2); idx += 64 * NWV) {
      const int c = tmaj ? idx % CB : idx / (kTile / 2);
      const int l = tmaj ? idx / CB : idx % (kTile / 2);
      if (c0 + c >= nchan) continue;
      const int64_t slot = tile * kTile + half * (kTile / 2) + l;
      const double o = s_dd[c * (kTile / 2) + l];
      if (fin) {
        const int32_t tg = ov.slot_target[slot];
        if (tg >= 0) ov.cube[(c0 + c) * ov.cst + (int64_t)tg * ov.tst] = (float)o;
      } else if (ov.mode == ACC_ADD) {
        ov.S[(c0 + c) * ns + slot] += o;
      } else {
        ov.S[(c0 + c) * ns + slot] = o;
      }
    }
  }
  if (pass == 0 && t < kTile) {
    const int64_t slot = tile * kTile + t;
    if (fin) {
      const int32_t tg = ov.slot_target[slot];
      if (tg >= 0 && ov.wout) ov.wout[tg] = (float)s_w[t];
    } else {
      ov.W[slot] = ov.mode == ACC_ADD ? ov.W[slot] + s_w[t] : s_w[t];
      ov.Wn[slot] = ov.mode == ACC_ADD ? ov.Wn[slot] + s_w[t] : s_w[t];
    }
  }
}

template <int VEC, typename T>
static void launch_cl(const TileView& tv, const KernelParams& kp, const void* data, int64_t ld,
                      int64_t nchan, const OutView& ov, hipStream_t st) {
  const int64_t ncb = (nchan + 64 * VEC - 1) / (64 * VEC);
  const dim3 g((unsigned)(tv.ntiles * ncb)), b(512);
  // vector loads need every row start aligned to VEC elements
  const int vec_ok = (ld % VEC == 0) && ((uintptr_t)data % (VEC * sizeof(T)) == 0) ? 1 : 0;
  if (kp.type == 0)
    hipLaunchKernelGGL((k_gather_cl<VEC, 0, T>), g, b, 0, st, tv, kp, (const T*)data, ld, nchan,
                       vec_ok, ov);
  else if (kp.type == 1)
    hipLaunchKernelGGL((k_gather_cl<VEC, 1, T>), g, b, 0, st, tv, kp, (const T*)data, ld, nchan,
                       vec_ok, ov);
  else
    hipLaunchKernelGGL((k_gather_cl<VEC, 3, T>), g, b, 0, st, tv, kp, (const T*)data, ld, nchan,
                       vec_ok, ov);
}

template <int VEC>
static void launch_cl_dt(const TileView& tv, const KernelParams& kp, const void* data, int dtype,
                         int64_t ld, int64_t nchan, const OutView& ov, hipStream_t st) {
  switch (dtype) {
    case 0: launch_cl<VEC, double>(tv, kp, data, ld, nchan, ov, st); break;
    case 1: launch_cl<VEC, float>(tv, kp, data, ld, nchan, ov, st); break;
    case 2: launch_cl<VEC, _Float16>(tv, kp, data, ld, nchan, ov, st); break;
    default: launch_cl<VEC, uint16_t>(tv, kp, data, ld, nchan, ov, st); break;
  }
}

hipError_t launch_gather_fp32(const TileView& tv, const KernelParams& kp, const void* data,
                              int dtype, int64_t ld, const float* sdata, int64_t nchan,
                              const OutView& ov, hipStream_t st) {
  if (tv.ntiles <= 0) return hipSuccess;
  if (nchan <= kSmallC) {
    const dim3 g((unsigned)tv.ntiles), b(64);
#define CG_TL(C)                                                                      \
  do {                                                                                \
    if (kp.type >= 2)                                                                 \
      hipLaunchKernelGGL((k_gather_tl<C, true>), g, b, 0, st, tv, kp, sdata, nchan, ov);  \
    else                                                                              \
      hipLaunchKernelGGL((k_gather_tl<C, false>), g, b, 0, st, tv, kp, sdata, nchan, ov); \
  } while (0)
    if (nchan <= 1) CG_TL(1);
    else if (nchan <= 2) CG_TL(2);
    else if (nchan <= 4) CG_TL(4);
    else if (nchan <= 8) CG_TL(8);
    else CG_TL(16);
#undef CG_TL
  } else if (nchan <= 64) {
    launch_cl_dt<1>(tv, kp, data, dtype, ld, nchan, ov, st);
  } else if (nchan <= 128) {
    launch_cl_dt<2>(tv, kp, data, dtype, ld, nchan, ov, st);
  } else {
    launch_cl_dt<4>(tv, kp, data, dtype, ld, nchan, ov, st);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Neighbour statistics: per target, count of samples with d <= r_s and
// sum mod 2^64 of splitmix64(input index).

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(64) k_stats(TileView tv, KernelParams kp,
                                              const int32_t* __restrict__ slot_target,
                                              int32_t* __restrict__ counts,
                                              uint64_t* __restrict__ hashes) {
  const int64_t tile = tile_of_block(blockIdx.x, tv.ntiles);
  const int lane = threadIdx.x;
  const int64_t slot = tile * kTile + lane;
  __shared__ double s_x[kChunk], s_y[kChunk], s_z[kChunk];
  __shared__ uint32_t s_n[kChunk];
  const int64_t ns = tv.nslots;
  const double tx = tv.txyz[slot], ty = tv.txyz[ns + slot], tz = tv.txyz[2 * ns + slot];
  int32_t cnt = 0;
  uint64_t h = 0;
  const uint32_t total = (uint32_t)tv.ntot[tile];
  RangeWindow<false> rw;
  rw.init(tv.rng + 2 * tv.roff[tile], tv.nr[tile], total, true);
  for (uint32_t base = 0; base < total; base += kChunk) {
    const int kmax = (int)(total - base < (uint32_t)kChunk ? total - base : (uint32_t)kChunk);
    rw.cover(base, base + kmax - 1, true);
    const int64_t pos = rw.pos(base + (lane < kmax ? lane : kmax - 1), base, base + kmax - 1);
    if (lane < kmax) {
      const double4 r = tv.srec[pos];
      s_x[lane] = r.x;
      s_y[lane] = r.y;
      s_z[lane] = r.z;
      s_n[lane] = (uint32_t)rec_row(r);
    }
    __syncthreads();
    for (int k = 0; k < kmax; ++k) {
      const double dx = s_x[k] - tx, dy = s_y[k] - ty, dz = s_z[k] - tz;
      if (dx * dx + dy * dy + dz * dz <= kp.cs2) {
        ++cnt;
        h += splitmix64((uint64_t)s_n[k]);
      }
    }
    __syncthreads();
  }
  const int32_t t = slot_target[slot];
  if (t >= 0) {
    counts[t] = cnt;
    if (hashes) hashes[t] = h;
  }
}

hipError_t launch_stats(const TileView& tv, const KernelParams& kp, const int32_t* slot_target,
                        int32_t* counts, uint64_t* hashes, hipStream_t st) {
  if (tv.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stats, dim3((unsigned)tv.ntiles), dim3(64), 0, st, tv, kp, slot_target,
                     counts, hashes);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Eq. (3): R = S / W (NaN where W = 0) into the caller's layout.

__global__ void __launch_bounds__(256) k_normalize(const double* __restrict__ S,
                                                   const double* __restrict__ W,
                                                   const double* __restrict__ Wn,
                                                   const int32_t* __restrict__ target_slot,
                                                   int64_t nslots, int64_t nchan, int64_t ntarget,
                                                   int64_t cst, int64_t tst,
                                                   float* __restrict__ cube, float* __restrict__ wout) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntarget) return;
  const int64_t c = blockIdx.y;
  const int64_t s = target_slot[t];
  if (cube) {
    const double wn = Wn[s];
    cube[c * cst + t * tst] = wn > 0.0 ? (float)(S[c * nslots + s] / wn) : qnan_f();
  }
  if (wout && c == 0) wout[t] = (float)W[s];
}

hipError_t launch_normalize(const double* S, const double* W, const double* Wn,
                            const int32_t* target_slot, int64_t nslots, int64_t nchan,
                            int64_t ntarget, int64_t cst, int64_t tst, float* cube, float* wout,
                            hipStream_t st) {
  if (ntarget <= 0) return hipSuccess;
  const int64_t gy = cube ? nchan : 1;
  hipLaunchKernelGGL(k_normalize, dim3((unsigned)((ntarget + 255) / 256), (unsigned)gy), dim3(256),
                     0, st, S, W, Wn, target_slot, nslots, nchan, ntarget, cst, tst, cube, wout);
  return hipGetLastError();
}

__global__ void k_fill(float* __restrict__ p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace cg
