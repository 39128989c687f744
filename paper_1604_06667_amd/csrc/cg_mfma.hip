// Matrix-core (MFMA) contraction for many-channel cubes.
//
// For one tile of 64 targets, Eq. (1) over a chunk of candidate samples
// is a dense product S[c][t] += sum_k R[k][c] w[t][k] (the paper's remark
// that all channels of a spectrum share one weight, Sect. 5, is what makes
// it a GEMM).  The weight block w[64][32] is computed once per chunk (FP64
// support test and distance, FP32 kernel value, rounded to BF16/FP16) and
// shared by all channel blocks; the data rows are converted to BF16/FP16
// while being staged through LDS in the operand layout of
// v_mfma_f32_32x32x16_{bf16,f16} (channels as M, targets as N, samples as
// K).  Accumulation is FP32 in the matrix cores.  In BF16 mode data and
// weights are each split into a BF16 high part and a BF16 residual and the
// block is formed from three products (hi*hi + lo*hi + hi*lo); a single
// BF16 product would round data and weights to 2^-9, which is too coarse
// for the 2e-3 bound on noise-dominated channels.  Two weight sums are kept
// in FP64: W of the unrounded weights (the weight map) and W' of the weights
// as they entered the products, which normalises the cube so that a
// constant field stays exactly constant.
#include <type_traits>

#include "cg_internal.hpp"

namespace cg {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

bool mfma_available() { return true; }

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
//         block (hi*hi + lo*hi + hi*lo), 16 samples per chunk;
// MODE 1: FP16, one product per block, 32 samples per chunk.
template <int NW, int BPW, int KT, int MODE, typename T>
__global__ void __launch_bounds__(NW * 64) k_gather_mfma(TileView tv, KernelParams kp,
                                                         const uint32_t* __restrict__ vals,
                                                         const T* __restrict__ data, int64_t ld,
                                                         int64_t nchan, int vec_ok_in,
                                                         OutView ov) {
  constexpr bool F16 = MODE == 1;
  constexpr bool SPLIT = MODE == 0;
  constexpr int NS = SPLIT ? 2 : 1;              // hi (+ lo) planes
  constexpr int MK = SPLIT ? 16 : 32;            // candidate samples per chunk
  constexpr int KP = MK + 8;                     // padded LDS row, multiple of 8 elements
  constexpr int NT = NW * 64;
  constexpr int CP = NW * BPW * 32;              // channels per pass (grid.y)
  constexpr int NITEMS = (MK / 4) * (CP / 4);    // 4 samples x 4 channels per item
  using opv_t = typename std::conditional<F16, f16x8_t, bf16x8_t>::type;
  __shared__ __attribute__((aligned(16))) uint16_t s_dt[NS][CP * KP];    // data^T  [channel][sample]
  __shared__ __attribute__((aligned(16))) uint16_t s_wt[NS][kTile * KP]; // weights [target][sample]
  __shared__ double s_c[MK][3];
  __shared__ int64_t s_row[MK];
  __shared__ double s_red[2][NW][kTile];
  __shared__ double s_wfin[2][kTile];

  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t tile = blockIdx.x;
  const int64_t c0 = (int64_t)blockIdx.y * CP;
  const int64_t ns = tv.nslots;
  const int64_t cap = tv.nsorted;
  const bool vec_ok = vec_ok_in != 0;

  // this thread's target for the weight block
  const int nw = t & 63;
  const int kg = t >> 6;
  const int64_t wslot = tile * kTile + nw;
  const double tx = tv.txyz[wslot], ty = tv.txyz[ns + wslot], tz = tv.txyz[2 * ns + wslot];
  double ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
  if (KT == 1 && isfinite(tx)) {
    double sa, ca, sd, cd;
    sincos(tv.tll[wslot], &sa, &ca);
    sincos(tv.tll[ns + wslot], &sd, &cd);
    const double ex = -sa, ey = ca, nx = -sd * ca, ny = -sd * sa, nz = cd;
    ax = kp.cospa * nx + kp.sinpa * ex;
    ay = kp.cospa * ny + kp.sinpa * ey;
    az = kp.cospa * nz;
    bx = kp.cospa * ex - kp.sinpa * nx;
    by = kp.cospa * ey - kp.sinpa * ny;
    bz = -kp.sinpa * nz;
  }
  double wsum = 0.0, wsum_r = 0.0;

  f32x16_t acc[BPW][2];
#pragma unroll
  for (int b = 0; b < BPW; ++b)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[b][nb][j] = 0.0f;

  const uint64_t cb0 = tv.cand_off[tile], cb1 = tv.cand_off[tile + 1];
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  for (uint64_t base = cb0; base < cb1; base += MK) {
    const int kmax = (int)((cb1 - base) < (uint64_t)MK ? (cb1 - base) : (uint64_t)MK);
    if (t < MK) {
      if (t < kmax) {
        const int64_t pos = tv.cand[base + t];
        s_c[t][0] = tv.sx[pos];
        s_c[t][1] = tv.sx[cap + pos];
        s_c[t][2] = tv.sx[2 * cap + pos];
        s_row[t] = (int64_t)vals[pos] * ld;
      } else {
        s_c[t][0] = nan;
        s_c[t][1] = nan;
        s_c[t][2] = nan;
        s_row[t] = -1;
      }
    }
    __syncthreads();
    // weight block: target nw, candidates kg, kg + NW, ...
#pragma unroll
    for (int k = kg; k < MK; k += NW) {
      const double dx = s_c[k][0] - tx, dy = s_c[k][1] - ty, dz = s_c[k][2] - tz;
      const double c2 = dx * dx + dy * dy + dz * dz;
      float w = 0.0f;
      if (c2 <= kp.cs2) {
        if (KT == 0) w = exp2_neg(chord2_to_d2(c2) * kp.k1);
        else w = pair_weight(kp, c2, dx, dy, dz, ax, ay, az, bx, by, bz);
      }
      const uint16_t whi = to_bits<F16>(w);
      float wr = from_bits<F16>(whi);
      s_wt[0][nw * KP + k] = whi;
      if constexpr (SPLIT) {
        const uint16_t wlo = to_bits<F16>(w - wr);
        s_wt[NS - 1][nw * KP + k] = wlo;
        wr += from_bits<F16>(wlo);
      }
      wsum += (double)w;
      wsum_r += (double)wr;
    }
    // data block: items of 4 samples x 4 channels, stored transposed (hi and lo planes)
    for (int item = t; item < NITEMS; item += NT) {
      const int rg = item / (CP / 4);
      const int cc = (item % (CP / 4)) * 4;
      const int nvalid = (int)((nchan - c0 - cc) < 4 ? (nchan - c0 - cc) : 4);
      float v[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = s_row[rg * 4 + r];
        if (row >= 0 && nvalid > 0) load4<T>(data + row + c0 + cc, nvalid, vec_ok, v[r]);
        else {
#pragma unroll
          for (int q = 0; q < 4; ++q) v[r][q] = 0.0f;
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint16_t h[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) h[r] = to_bits<F16>(v[r][j]);
        uint2 pk;
        pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
        pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
        *reinterpret_cast<uint2*>(&s_dt[0][(cc + j) * KP + rg * 4]) = pk;
        if constexpr (SPLIT) {
          uint16_t l[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) l[r] = to_bits<F16>(v[r][j] - from_bits<F16>(h[r]));
          pk.x = (uint32_t)l[0] | ((uint32_t)l[1] << 16);
          pk.y = (uint32_t)l[2] | ((uint32_t)l[3] << 16);
          *reinterpret_cast<uint2*>(&s_dt[NS - 1][(cc + j) * KP + rg * 4]) = pk;
        }
      }
    }
    __syncthreads();
    // matrix cores: acc[b][nb] (32 channels x 32 targets) += A (32 x 16) * B (16 x 32)
#pragma unroll
    for (int ks = 0; ks < MK / 16; ++ks) {
      const int kofs = ks * 16 + 8 * (lane >> 5);
      opv_t bop[NS][2];
#pragma unroll
      for (int sp = 0; sp < NS; ++sp)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          bop[sp][nb] =
              *reinterpret_cast<const opv_t*>(&s_wt[sp][(nb * 32 + (lane & 31)) * KP + kofs]);
#pragma unroll
      for (int b = 0; b < BPW; ++b) {
        const int cb = (wv * BPW + b) * 32;
        opv_t aop[NS];
#pragma unroll
        for (int sp = 0; sp < NS; ++sp)
          aop[sp] = *reinterpret_cast<const opv_t*>(&s_dt[sp][(cb + (lane & 31)) * KP + kofs]);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          if constexpr (F16) {
            acc[b][nb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(aop[0], bop[0][nb], acc[b][nb], 0, 0, 0);
          } else {
            acc[b][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aop[0], bop[0][nb], acc[b][nb], 0, 0, 0);
            if constexpr (SPLIT) {
              acc[b][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aop[1], bop[0][nb], acc[b][nb], 0, 0, 0);
              acc[b][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aop[0], bop[1][nb], acc[b][nb], 0, 0, 0);
            }
          }
        }
      }
    }
    __syncthreads();
  }

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

  // outputs: lane holds target n = nb*32 + lane%32, channels m = 8(j/4) + 4(lane/32) + j%4
  const bool fin = ov.mode == ACC_FINAL;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int n = nb * 32 + (lane & 31);
    const int64_t slot = tile * kTile + n;
    const double wr = s_wfin[1][n];
    const int32_t tg = fin ? ov.slot_target[slot] : 0;
    const float inv = wr > 0.0 ? (float)(1.0 / wr) : 0.0f;
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int m = 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
        const int64_t c = c0 + (wv * BPW + b) * 32 + m;
        if (c >= nchan) continue;
        const float val = acc[b][nb][j];
        if (fin) {
          if (tg >= 0)
            ov.cube[c * ov.ntarget + tg] = wr > 0.0 ? val * inv : __int_as_float(0x7fc00000);
        } else if (ov.mode == ACC_ADD) {
          ov.S[c * ns + slot] += val;
        } else {
          ov.S[c * ns + slot] = val;
        }
      }
    }
  }
  if (blockIdx.y == 0 && t < kTile) {
    const int64_t slot = tile * kTile + t;
    if (fin) {
      const int32_t tg = ov.slot_target[slot];
      if (tg >= 0 && ov.wout) ov.wout[tg] = (float)s_wfin[0][t];
    } else if (ov.mode == ACC_ADD) {
      ov.W[slot] += s_wfin[0][t];
      ov.Wn[slot] += s_wfin[1][t];
    } else {
      ov.W[slot] = s_wfin[0][t];
      ov.Wn[slot] = s_wfin[1][t];
    }
  }
}

template <int NW, int BPW, int MODE, typename T>
static void launch_cfg(const TileView& tv, const KernelParams& kp, int64_t ntiles,
                       const uint32_t* vals, const void* data, int64_t ld, int64_t nchan,
                       const OutView& ov, hipStream_t st) {
  constexpr int CP = NW * BPW * 32;
  const int64_t npass = (nchan + CP - 1) / CP;
  const dim3 g((unsigned)ntiles, (unsigned)npass), b(NW * 64);
  const int vec_ok = (ld % 4 == 0) && ((uintptr_t)data % (4 * sizeof(T)) == 0) ? 1 : 0;
  if (kp.type == 0)
    hipLaunchKernelGGL((k_gather_mfma<NW, BPW, 0, MODE, T>), g, b, 0, st, tv, kp, vals,
                       (const T*)data, ld, nchan, vec_ok, ov);
  else
    hipLaunchKernelGGL((k_gather_mfma<NW, BPW, 1, MODE, T>), g, b, 0, st, tv, kp, vals,
                       (const T*)data, ld, nchan, vec_ok, ov);
}

template <int MODE, typename T>
static void launch_dt(const TileView& tv, const KernelParams& kp, int64_t ntiles,
                      const uint32_t* vals, const void* data, int64_t ld, int64_t nchan,
                      const OutView& ov, hipStream_t st) {
  if (nchan <= 64) launch_cfg<2, 1, MODE, T>(tv, kp, ntiles, vals, data, ld, nchan, ov, st);
  else if (nchan <= 128) launch_cfg<4, 1, MODE, T>(tv, kp, ntiles, vals, data, ld, nchan, ov, st);
  else if (nchan <= 256) launch_cfg<8, 1, MODE, T>(tv, kp, ntiles, vals, data, ld, nchan, ov, st);
  else if (nchan <= 512) launch_cfg<8, 2, MODE, T>(tv, kp, ntiles, vals, data, ld, nchan, ov, st);
  else launch_cfg<8, 4, MODE, T>(tv, kp, ntiles, vals, data, ld, nchan, ov, st);
}

template <int MODE>
static void launch_prec(const TileView& tv, const KernelParams& kp, int64_t ntiles,
                        const uint32_t* vals, const void* data, int dtype, int64_t ld,
                        int64_t nchan, const OutView& ov, hipStream_t st) {
  switch (dtype) {
    case 0: launch_dt<MODE, double>(tv, kp, ntiles, vals, data, ld, nchan, ov, st); break;
    case 1: launch_dt<MODE, float>(tv, kp, ntiles, vals, data, ld, nchan, ov, st); break;
    case 2: launch_dt<MODE, _Float16>(tv, kp, ntiles, vals, data, ld, nchan, ov, st); break;
    default: launch_dt<MODE, uint16_t>(tv, kp, ntiles, vals, data, ld, nchan, ov, st); break;
  }
}

hipError_t launch_gather_mfma(const TileView& tv, const KernelParams& kp, int64_t ntiles,
                              const uint32_t* vals, const void* data, int dtype, int64_t ld,
                              int64_t nchan, int prec, const OutView& ov, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (prec == 2) launch_prec<1>(tv, kp, ntiles, vals, data, dtype, ld, nchan, ov, st);
  else launch_prec<0>(tv, kp, ntiles, vals, data, dtype, ld, nchan, ov, st);
  return hipGetLastError();
}

}  // namespace cg
