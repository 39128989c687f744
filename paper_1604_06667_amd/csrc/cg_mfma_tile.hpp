// Matrix-core contraction of one tile of 64 targets over a channel range:
// the device code shared by the per-grid kernel and the persistent batch
// kernel.  Description of the method and data flow: cg_mfma.hip.
#pragma once
#include <type_traits>

#include "cg_internal.hpp"

namespace cg {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

template <bool F16>
__device__ __forceinline__ uint16_t to_bits(float x) {
  if constexpr (F16) {
    const _Float16 h = (_Float16)x;
    return __builtin_bit_cast(uint16_t, h);
  } else {
    const __bf16 h = (__bf16)x;
    return __builtin_bit_cast(uint16_t, h);
  }
}

template <bool F16>
__device__ __forceinline__ float from_bits(uint16_t b) {
  if constexpr (F16) return (float)__builtin_bit_cast(_Float16, b);
  else return __uint_as_float((uint32_t)b << 16);
}

// Two floats -> two packed 16-bit values (round to nearest even), element a
// in the low half.
template <bool F16>
__device__ __forceinline__ uint32_t cvt_pk(float a, float b) {
  if constexpr (F16) {
    return (uint32_t)to_bits<true>(a) | ((uint32_t)to_bits<true>(b) << 16);
  } else {
    const f32x2_t v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
  }
}

// The two packed values as floats.
template <bool F16>
__device__ __forceinline__ float unpk_lo(uint32_t p) {
  if constexpr (F16) return from_bits<true>((uint16_t)(p & 0xffffu));
  else return __uint_as_float(p << 16);
}
template <bool F16>
__device__ __forceinline__ float unpk_hi(uint32_t p) {
  if constexpr (F16) return from_bits<true>((uint16_t)(p >> 16));
  else return __uint_as_float(p & 0xffff0000u);
}

template <typename T>
__device__ __forceinline__ float in_f32(const T* p);
template <>
__device__ __forceinline__ float in_f32<float>(const float* p) { return *p; }
template <>
__device__ __forceinline__ float in_f32<double>(const double* p) { return (float)*p; }
template <>
__device__ __forceinline__ float in_f32<uint16_t>(const uint16_t* p) {
  return __uint_as_float(((uint32_t)*p) << 16);
}
template <>
__device__ __forceinline__ float in_f32<_Float16>(const _Float16* p) { return (float)*p; }

// 4 consecutive channels of one row as floats (zeros past nvalid).
template <typename T>
__device__ __forceinline__ void load4(const T* __restrict__ p, int nvalid, bool vec_ok, float* o) {
  if (vec_ok && nvalid >= 4) {
    if constexpr (sizeof(T) == 4) {
      const float4 v = *reinterpret_cast<const float4*>(p);
      o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
      return;
    } else if constexpr (sizeof(T) == 2) {
      const uint2 v = *reinterpret_cast<const uint2*>(p);
      const uint16_t h[4] = {(uint16_t)(v.x & 0xffff), (uint16_t)(v.x >> 16),
                             (uint16_t)(v.y & 0xffff), (uint16_t)(v.y >> 16)};
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] = in_f32<T>(reinterpret_cast<const T*>(&h[i]));
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) o[i] = (i < nvalid) ? in_f32<T>(p + i) : 0.0f;
}

// MODE 0: BF16 with hi/lo split of data and weights, three products per
//         block (hi*hi + lo*hi + hi*lo);
// MODE 1: FP16, one product per block.
//
// Work of one workgroup: one tile (64 targets) x CP channels.  Wavefront w
// owns channel blocks [w*BPW, (w+1)*BPW) of 32 channels; lane l holds
// channel l%32 of a block and the 8 samples 8*(l/32) .. +7 of a 16-sample
// chunk, i.e. exactly its MFMA A operand, so the data never passes through
// LDS: each lane loads its 8 values straight from the sample rows (one
// 128-byte segment per row and half-wave) and converts them in registers.
// Only the 64 x MK weight block is shared through LDS (double buffered).
// A chunk is KS consecutive 16-sample MFMA steps (MK = 16 KS candidates): a
// larger chunk puts more loads in flight per barrier, which is what bounds
// narrow channel ranges, at KS x 8 data registers per block.
// Software pipeline, one barrier per chunk: while chunk i is on the matrix
// cores, the same wavefront computes the weight block of chunk i+1 and
// reloads its data registers with chunk i+1; candidate records run two
// chunks ahead through a three-deep LDS ring; wavefront 0 loads them from the
// tile's list of sorted positions.  Past-the-end candidates point at a row
// of zeros, so the loads need no bounds selects.  FULL: the channel
// count is a multiple of CP (no channel bounds checks).
constexpr int kListCands = 4096;    // candidates of a tile listed in LDS
constexpr int kListRanges = 512;    // ranges of a tile listed in LDS

template <int NW, int BPW, int KT, int MODE, bool FULL, typename T, int KS = 1, bool GL = false>
__device__ __forceinline__ void mfma_tile(const TileView tv, const KernelParams kp,
                                          const T* __restrict__ data, const T* __restrict__ zrow,
                                          int64_t ld, int64_t nchan, const OutView ov,
                                          int64_t tile, int64_t c0, int64_t cend) {
  // (by value: a reference to a kernel argument would place it in scratch)
  constexpr bool F16 = MODE == 1;
  constexpr bool SPLIT = MODE == 0;
  constexpr bool BF16IN = std::is_same<T, uint16_t>::value;
  constexpr int NS = SPLIT ? 2 : 1;              // hi (+ lo) parts
  constexpr int MK = 16 * KS;                    // candidate samples per chunk
  static_assert(MK <= NW * 64, "one candidate record per thread");
  constexpr int KP = MK + 8;                     // padded LDS row of the weight block
  constexpr int CP = NW * BPW * 32;              // channels per pass
  using opv_t = typename std::conditional<F16, f16x8_t, bf16x8_t>::type;
  __shared__ __attribute__((aligned(16))) uint16_t s_wt[2][NS][kTile * KP];  // [buf][part][target][sample]
  __shared__ double s_c[3][MK][3];
  __shared__ int64_t s_row[3][MK];   // element offset of each candidate's row from data
  __shared__ double s_red[2][NW][kTile];
  __shared__ double s_wfin[2][kTile];
  __shared__ double s_tg[kTile][3];                    // target unit vectors
  __shared__ double s_ax[(KT == 1 || KT == 2) ? kTile : 1][3];  // major axis at the target (elliptical)
  __shared__ uint32_t s_pos[kListCands];               // sorted positions of the tile's candidates
  __shared__ uint32_t s_rb[kListRanges], s_rs[kListRanges];

  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t ns = tv.nslots;
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  const int cl = lane & 31;      // channel within a 32-channel block / target within a 32-target block
  const int kh = lane >> 5;      // which 8 samples of the chunk this lane holds
  const int64_t cbase = c0 + wv * BPW * 32 + cl;   // this lane's channel in block 0
  // KT: 0 gauss1d, 1 gauss2d, 2 either, chosen at run time (batched jobs of
  // both types), 3 a radial kernel of arbitrary shape (tapered sinc or
  // tabulated profile, chosen at run time)
  const bool ell = KT == 1 || (KT == 2 && kp.type == 1);
  bool bvalid[BPW];    // this lane's channel of block b exists
  bool bany[BPW];      // block b has any channel (uniform over the wavefront)
#pragma unroll
  for (int b = 0; b < BPW; ++b) {
    bvalid[b] = FULL || (cbase + 32 * b < cend);
    bany[b] = FULL || (c0 + (wv * BPW + b) * 32 < cend);
  }

  if (t < kTile) {
    const int64_t wslot = tile * kTile + t;
    const double x = ldg<GL>(tv.txyz, wslot);
    s_tg[t][0] = x;
    s_tg[t][1] = ldg<GL>(tv.txyz, ns + wslot);
    s_tg[t][2] = ldg<GL>(tv.txyz, 2 * ns + wslot);
    if constexpr (KT == 1 || KT == 2) {
      // major axis: north turned towards east by the position angle
      double a[3] = {0.0, 0.0, 0.0};
      if (ell && isfinite(x)) {
        double sa, ca, sd, cd;
        sincos(ldg<GL>(tv.tll, wslot), &sa, &ca);
        sincos(ldg<GL>(tv.tll, ns + wslot), &sd, &cd);
        const double ex = -sa, ey = ca, nx = -sd * ca, ny = -sd * sa, nz = cd;
        a[0] = kp.cospa * nx + kp.sinpa * ex;
        a[1] = kp.cospa * ny + kp.sinpa * ey;
        a[2] = kp.cospa * nz;
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) s_ax[t][q] = a[q];
    }
  }
  // this thread's target in the weight block and its candidates kg, kg + NW, ...
  const int nw = t & 63;
  const int kg = t >> 6;
  double wsum = 0.0, wsum_r = 0.0;

  f32x16_t acc[BPW][2];
#pragma unroll
  for (int b = 0; b < BPW; ++b)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[b][nb][j] = 0.0f;

  const uint32_t total = (uint32_t)ldg<GL>(tv.ntot, tile);
  const int64_t nchunks = (int64_t)((total + MK - 1) / MK);
  const uint32_t nr = ldg<GL>(tv.nr, tile);
  const uint32_t* rng = tv.rng + 2 * (int64_t)ldg<GL>(tv.roff, tile);

  // The tile's candidates in walk order: a tile of at most kListCands
  // candidates in kListRanges ranges has its sorted positions listed in LDS
  // at the start (all threads, one binary search over the ranges' starts per
  // candidate), so the loader reads them with one LDS access; a longer tile
  // is walked by wavefront 0 through a window of 64 ranges.
  const bool listed = total <= (uint32_t)kListCands && nr <= (uint32_t)kListRanges;
  if (listed) {
    for (uint32_t i = t; i < nr; i += NW * 64) {
      s_rb[i] = ldg<GL>(rng, 2 * (int64_t)i);
      s_rs[i] = ldg<GL>(rng, 2 * (int64_t)i + 1);
    }
    __syncthreads();
    for (uint32_t q = t; q < total; q += NW * 64) {
      uint32_t lo = 0, hi = nr - 1;   // last range whose first candidate index is <= q
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (s_rs[mid] <= q) lo = mid;
        else hi = mid - 1;
      }
      s_pos[q] = s_rb[lo] + (q - s_rs[lo]);
    }
    __syncthreads();
  }

  // candidate record of chunk ch for thread t < MK (NaN / zero row past the
  // end).  The record stays raw in registers until it is published one
  // chunk later, so that nothing waits for its load in the meantime.
  const int64_t zoff = (int64_t)(zrow - data) - c0;   // offset that lands on the zero row
  double rx = nan, ry = nan, rz = nan;
  int64_t rrow = 0;       // input row of the record (valid when rok)
  bool rok = false;
  // Odd tile rows of a WCS grid walk their candidates backwards (bottom ring
  // first): a tile and the one below it then reach the rings they share at
  // the same time, while those samples are in L2.
  const bool rev = tv.ntx > 0 && ((tile / tv.ntx) & 1);
  RangeWindow<GL> rwin;
  if (wv == 0 && !listed) rwin.init(rng, nr, total, !rev);
  auto load_rec = [&](int64_t ch) {   // every lane of wavefront 0
    rx = ry = rz = nan;
    rok = false;   // the zero row: + channel offsets stays inside it
    if (ch < nchunks) {
      const uint32_t i0 = (uint32_t)ch * MK;
      const uint32_t cnt = total - i0 < (uint32_t)MK ? total - i0 : (uint32_t)MK;
      const uint32_t idx = i0 + ((uint32_t)t < cnt ? (uint32_t)t : cnt - 1);
      const uint32_t q = rev ? total - 1 - idx : idx;
      int64_t p;
      if (listed) {
        p = s_pos[q];
      } else {
        const uint32_t qlo = rev ? total - i0 - cnt : i0, qhi = rev ? total - 1 - i0 : i0 + cnt - 1;
        rwin.cover(qlo, qhi, !rev);
        p = rwin.pos(q, qlo, qhi);
      }
      if ((uint32_t)t < cnt) {
        const double4 r = ld_rec<GL>(tv.srec, p);
        rx = r.x;
        ry = r.y;
        rz = r.z;
        rrow = rec_row(r);
        rok = true;
      }
    }
  };
  auto put_rec = [&](int buf) {
    s_c[buf][t][0] = rx;
    s_c[buf][t][1] = ry;
    s_c[buf][t][2] = rz;
    s_row[buf][t] = rok ? rrow * ld : zoff;
  };
  // weight of candidate k of the chunk in record buffer rb -> weight buffer wb
  // Kernel value of a pair.  The support test is FP64 on the chord.  The
  // value is rounded to 16-bit operand parts, but the weight map sums it
  // unrounded, so it is held to about 2e-7 relative: the base-2 exponent's
  // leading term (k c^2 for the circular Gaussian, kmin c^2 + (kmaj - kmin)
  // u^2 for the elliptical one) is formed in FP64, its integer part split
  // off exactly, and only the fraction, the small series corrections and
  // the exponential are FP32.
  //
  // Elliptical kernel: with u, v the components of the chord along the
  // major and minor axes at the target (both tangent there), u^2 + v^2 is
  // the chord's tangential part c^2 (1 - c^2/4) exactly, so the exponent
  //   d^2 (u^2 kmaj + v^2 kmin) / (u^2 + v^2)
  // equals d^2 kmin + (kmaj - kmin) u^2 rq with rq = d^2 / (c^2 (1 - c^2/4)),
  // which needs only u.  With d^2 = c^2 (1 + s), s = c^2/12 + c^4/90 + ...,
  // and rq = 1 + (s + c^2/4) / (1 - c^2/4), the exponent is the leading term
  // plus kmin c^2 s + (kmaj - kmin) u^2 (rq - 1).  Supports below ~0.57 deg
  // (c^2 <= 1e-4, uniform over the launch) keep s = c^2/12 and rq - 1 =
  // c^2/3, whose next terms are below 1e-8 relative.
  const float k1f = (float)kp.k1, kminf = (float)kp.kmin, kdf = (float)(kp.kmaj - kp.kmin);
  const float ksf = (float)kp.ks, tinvf = (float)kp.tinv;
  const double kdd = kp.kmaj - kp.kmin;
  const bool short_support = kp.cs2 <= 1e-4;
  auto weight = [&](int rb, int wb, int k) {
    const double dx = s_c[rb][k][0] - s_tg[nw][0];
    const double dy = s_c[rb][k][1] - s_tg[nw][1];
    const double dz = s_c[rb][k][2] - s_tg[nw][2];
    const double c2 = dx * dx + dy * dy + dz * dz;
    const float c = (float)c2;
    // s = d^2 / c^2 - 1 (series, or exact for chords beyond ~20 deg)
    auto series = [&]() -> float {
      if (short_support) return c * (1.0f / 12.0f);
      if (c2 > 0.1225) return (float)(chord2_to_d2_exact(c2) / c2 - 1.0);
      return c * (1.0f / 12.0f + c * (1.0f / 90.0f + c * (1.0f / 560.0f +
             c * (1.0f / 3150.0f + c * (1.0f / 16632.0f)))));
    };
    float w;
    if constexpr (KT == 3) {
      // radial kernels of arbitrary shape: the tapered sinc, or the
      // tabulated profile interpolated linearly (zero past its last point)
      const float d2 = c * (1.0f + series());
      const float d = sqrtf(d2);
      float v;
      if (kp.type == 2) {
        const float a = ksf * d;
        v = __builtin_amdgcn_exp2f(-(d2 * k1f)) * (a > 0.0f ? sinf(a) / a : 1.0f);
      } else {
        const float u = d * tinvf;
        const int last = kp.ntab - 1;
        if (u < (float)last) {
          const int i = (int)u;
          const float f = u - (float)i;
          const float t0 = (float)kp.tab[i], t1 = (float)kp.tab[i + 1];
          v = t0 + f * (t1 - t0);
        } else {
          v = u == (float)last ? (float)kp.tab[last] : 0.0f;
        }
      }
      w = c2 <= kp.cs2 ? v : 0.0f;
    } else {
      const float sr = series();
      double xl = c2 * kp.k1;        // leading term of the exponent
      float corr = (float)xl * sr;   // the rest
      if constexpr (KT == 1 || KT == 2) {
        if (ell) {
          const double u = dx * s_ax[nw][0] + dy * s_ax[nw][1] + dz * s_ax[nw][2];
          const double u2 = u * u;
          const float den = 1.0f - 0.25f * c;   // zero only for an antipodal sample (u = 0)
          const float rq1 = short_support ? c * (1.0f / 3.0f)
                            : den > 0.0f ? (sr + 0.25f * c) * __builtin_amdgcn_rcpf(den) : 0.0f;
          xl = fma(kdd, u2, c2 * kp.kmin);
          corr = kminf * c * sr + kdf * (float)u2 * rq1;
        }
      }
      // 2^-(xl + corr) with the integer part of xl split off exactly, so
      // that rounding to FP32 costs < 6e-8 absolute in the exponent however
      // far out the sample is (exponents reach ~26 at the edge of a 3-sigma
      // support along the minor axis of a 2:1 ellipse)
      const double fl = floor(xl);
      const float v = ldexpf(__builtin_amdgcn_exp2f(-((float)(xl - fl) + corr)), (int)(-fl));
      w = c2 <= kp.cs2 ? v : 0.0f;
    }
    const uint16_t whi = to_bits<F16>(w);
    float wr = from_bits<F16>(whi);
    s_wt[wb][0][nw * KP + k] = whi;
    if constexpr (SPLIT) {
      const uint16_t wlo = to_bits<F16>(w - wr);
      s_wt[wb][NS - 1][nw * KP + k] = wlo;
      wr += from_bits<F16>(wlo);
    }
    wsum += (double)w;
    wsum_r += (double)wr;
  };
  // this lane's A-operand values (raw input) of one chunk
  // 16-bit input of the operand's own type is used bit for bit (two values
  // packed per register); any other input is converted through FP32.
  constexpr bool DIRECT = (BF16IN && !F16) || (std::is_same<T, _Float16>::value && F16);
  float raw[BPW][KS][DIRECT ? 1 : 8];
  uint32_t rawp[BPW][KS][4];
  // Lanes whose channel lies past cend read the last valid channel of the
  // same row instead (and discard it), so that every address stays inside
  // the caller's row (or the zero row) whatever the channel count.
  auto load_block = [&](int rb, int b) {
    const int64_t cofs = bvalid[b] ? cbase + 32 * b : cend - 1;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int64_t* rw = &s_row[rb][16 * s + 8 * kh];
      if constexpr (DIRECT) {
        const uint16_t* d16 = reinterpret_cast<const uint16_t*>(data);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t lo = ldg<GL>(d16, rw[2 * q] + cofs), hi = ldg<GL>(d16, rw[2 * q + 1] + cofs);
          rawp[b][s][q] = bvalid[b] ? __builtin_amdgcn_perm(hi, lo, 0x05040100u) : 0u;
        }
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const T v = ldg<GL>(data, rw[i] + cofs);
          raw[b][s][i] = bvalid[b] ? in_f32<T>(&v) : 0.0f;
        }
      }
    }
  };

  // prologue: records of chunks 0, 1 in LDS, of chunk 2 in registers; the
  // weights and data of chunk 0
  if (wv == 0) {
    load_rec(0);
    if (t < MK) put_rec(0);
    load_rec(1);
    if (t < MK) put_rec(1);
    load_rec(2);
  }
  __syncthreads();
  if (nchunks > 0) {
#pragma unroll
    for (int k = kg; k < MK; k += NW) weight(0, 0, k);
#pragma unroll
    for (int b = 0; b < BPW; ++b) load_block(0, b);
  }

  int r1 = 1, r2 = 2;   // record buffers of chunks ch+1, ch+2 (ring of three)
  for (int64_t ch = 0; ch < nchunks; ++ch) {
    const int wc = (int)(ch & 1);                 // weight buffer of chunk ch
    __syncthreads();
    // records: publish chunk ch+2, fetch chunk ch+3
    if (wv == 0) {
      if (t < MK) put_rec(r2);
      load_rec(ch + 3);
    }
    const int kofs = 8 * kh;
    // weight operands of MFMA step s (step 0 read once and shared by the blocks)
    auto load_bop = [&](int s, opv_t (&bo)[NS][2]) {
#pragma unroll
      for (int sp = 0; sp < NS; ++sp)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          bo[sp][nb] = *reinterpret_cast<const opv_t*>(&s_wt[wc][sp][(nb * 32 + cl) * KP + 16 * s + kofs]);
    };
    opv_t bop0[NS][2];
    load_bop(0, bop0);
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
      // this lane's data of chunk ch -> MFMA operands (hi, lo); refill with chunk ch+1
      opv_t aop[KS][NS];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        uint32_t hp[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if constexpr (DIRECT) hp[q] = rawp[b][s][q];
          else hp[q] = cvt_pk<F16>(raw[b][s][2 * q], raw[b][s][2 * q + 1]);
        }
        aop[s][0] = __builtin_bit_cast(opv_t, hp);
        if constexpr (SPLIT && !BF16IN) {
          uint32_t lp[4];
#pragma unroll
          for (int q = 0; q < 4; ++q)
            lp[q] = cvt_pk<F16>(raw[b][s][2 * q] - unpk_lo<F16>(hp[q]),
                                raw[b][s][2 * q + 1] - unpk_hi<F16>(hp[q]));
          aop[s][NS - 1] = __builtin_bit_cast(opv_t, lp);
        }
      }
      load_block(r1, b);   // past the last chunk this reads the zero row
      // independent accumulators back to back; the residual products last
      if (bany[b]) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          opv_t bop[NS][2];
          if (s == 0) {
#pragma unroll
            for (int sp = 0; sp < NS; ++sp)
#pragma unroll
              for (int nb = 0; nb < 2; ++nb) bop[sp][nb] = bop0[sp][nb];
          } else {
            load_bop(s, bop);
          }
          if constexpr (F16) {
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
              acc[b][nb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(aop[s][0], bop[0][nb], acc[b][nb], 0, 0, 0);
          } else {
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
              acc[b][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aop[s][0], bop[0][nb], acc[b][nb], 0, 0, 0);
            if constexpr (SPLIT) {
#pragma unroll
              for (int nb = 0; nb < 2; ++nb)
                acc[b][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aop[s][0], bop[1][nb], acc[b][nb], 0, 0, 0);
              if constexpr (!BF16IN) {
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
                  acc[b][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aop[s][1], bop[0][nb], acc[b][nb], 0, 0, 0);
              }
            }
          }
        }
      }
      // weight block of chunk ch+1 (all zero past the last chunk), spread over
      // the channel blocks
#pragma unroll
      for (int k = kg + b * NW; k < MK; k += BPW * NW) weight(r1, wc ^ 1, k);
    }
    r1 = r2;
    r2 = r2 == 2 ? 0 : r2 + 1;
  }
  __syncthreads();

  // weight sums of each target (8 partial sums per target)
  s_red[0][kg][nw] = wsum;
  s_red[1][kg][nw] = wsum_r;
  __syncthreads();
  if (t < kTile) {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      a += s_red[0][q][t];
      b += s_red[1][q][t];
    }
    s_wfin[0][t] = a;
    s_wfin[1][t] = b;
  }
  __syncthreads();

  // outputs: lane holds target n = nb*32 + lane%32, channels m = 8(j/4) + 4(lane/32) + j%4;
  // one loop nest per (uniform) output mode, one lane test per target
  const bool fin = ov.mode == ACC_FINAL;
  if (fin) {
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const int n = nb * 32 + (lane & 31);
      const int32_t tg = ldg<GL>(ov.slot_target, tile * kTile + n);
      if (tg >= 0) {
        const double wr = s_wfin[1][n];
        const float inv = wr > 0.0 ? (float)(1.0 / wr) : 0.0f;
        const bool filled = wr > 0.0;
        float* __restrict__ dst = ov.cube + (int64_t)tg * ov.tst;
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            const int m = 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
            const int64_t c = c0 + (wv * BPW + b) * 32 + m;
            if (!FULL && c >= cend) continue;
            stg<GL>(dst, c * ov.cst, filled ? acc[b][nb][j] * inv : __int_as_float(0x7fc00000));
          }
        }
      }
    }
  } else {
    const bool add = ov.mode == ACC_ADD;
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const int64_t slot = tile * kTile + nb * 32 + (lane & 31);
      double* __restrict__ dst = ov.S + slot;
#pragma unroll
      for (int b = 0; b < BPW; ++b) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int m = 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
          const int64_t c = c0 + (wv * BPW + b) * 32 + m;
          if (!FULL && c >= cend) continue;
          if (add) dst[c * ns] += (double)acc[b][nb][j];
          else dst[c * ns] = (double)acc[b][nb][j];
        }
      }
    }
  }
  if (c0 == 0 && t < kTile) {
    const int64_t slot = tile * kTile + t;
    if (fin) {
      const int32_t tg = ldg<GL>(ov.slot_target, slot);
      if (tg >= 0 && ov.wout) stg<GL>(ov.wout, tg, (float)s_wfin[0][t]);
    } else if (ov.mode == ACC_ADD) {
      ov.W[slot] += s_wfin[0][t];
      ov.Wn[slot] += s_wfin[1][t];
    } else {
      ov.W[slot] = s_wfin[0][t];
      ov.Wn[slot] = s_wfin[1][t];
    }
  }
}

}  // namespace cg
