// Matrix-core (MFMA) contraction for many-channel cubes.
//
// For one tile of 64 targets, Eq. (1) over a chunk of candidate samples
// is a dense product S[c][t] += sum_k R[k][c] w[t][k] (the paper's remark
// that all channels of a spectrum share one weight, Sect. 5, is what makes
// it a GEMM).  The weight block w[64][32] is computed once per chunk (FP64
// support test and distance, FP32 kernel value, rounded to BF16/FP16) and
// shared by all channel blocks; each lane loads the data values of its own
// operand of v_mfma_f32_32x32x16_{bf16,f16} (channels as M, targets as N,
// samples as K) and converts them to BF16/FP16 in registers.  Accumulation is FP32 in the matrix cores.  In BF16 mode data and
// weights are each split into a BF16 high part and a BF16 residual and the
// block is formed from three products (hi*hi + lo*hi + hi*lo); a single
// BF16 product would round data and weights to 2^-9, which is too coarse
// for the 2e-3 bound on noise-dominated channels.  Two weight sums are kept
// in FP64: W of the unrounded weights (the weight map) and W' of the weights
// as they entered the products, which normalises the cube so that a
// constant field stays exactly constant.
#include "cg_mfma_tile.hpp"

namespace cg {

bool mfma_available() { return true; }

template <int NW, int BPW, int KT, int MODE, bool FULL, typename T, int KS>
__global__ void __launch_bounds__(NW * 64) k_gather_mfma(TileView tv, KernelParams kp,
                                                         const T* __restrict__ data,
                                                         const T* __restrict__ zrow, int64_t ld,
                                                         int64_t nchan, OutView ov) {
  constexpr int CP = NW * BPW * 32;
  int64_t tile, pass;
  work_of_block(blockIdx.x, tv.ntiles, (nchan + CP - 1) / CP, &tile, &pass);
  if (tv.ntx > 0) tile = strip_tile(tile, tv.ntiles, tv.ntx);
  const int64_t c0 = pass * CP;
  const int64_t cend = c0 + CP < nchan ? c0 + CP : nchan;
  mfma_tile<NW, BPW, KT, MODE, FULL, T, KS>(tv, kp, data, zrow, ld, nchan, ov, tile, c0, cend);
}

template <int NW, int BPW, int MODE, typename T, int KS>
static void launch_cfg(const TileView& tv, const KernelParams& kp, const void* data,
                       const void* zrow, int64_t ld, int64_t nchan, const OutView& ov,
                       hipStream_t st) {
  constexpr int CP = NW * BPW * 32;
  const int64_t npass = (nchan + CP - 1) / CP;
  const dim3 g((unsigned)(tv.ntiles * npass)), b(NW * 64);
  const bool full = nchan % CP == 0;
  const T* d = (const T*)data;
  const T* z = (const T*)zrow;
#define CG_MFMA_LAUNCH(KT_, FULL_)                                                              \
  hipLaunchKernelGGL((k_gather_mfma<NW, BPW, KT_, MODE, FULL_, T, KS>), g, b, 0, st, tv, kp, d, z, \
                     ld, nchan, ov)
  if (kp.type == 0) {
    if (full) CG_MFMA_LAUNCH(0, true);
    else CG_MFMA_LAUNCH(0, false);
  } else if (kp.type == 1) {
    if (full) CG_MFMA_LAUNCH(1, true);
    else CG_MFMA_LAUNCH(1, false);
  } else {
    if (full) CG_MFMA_LAUNCH(3, true);
    else CG_MFMA_LAUNCH(3, false);
  }
#undef CG_MFMA_LAUNCH
}

template <int MODE, typename T>
static void launch_dt(const TileView& tv, const KernelParams& kp, const void* data,
                      const void* zrow, int64_t ld, int64_t nchan, const OutView& ov,
                      hipStream_t st) {
  // KS: 16-sample MFMA steps per pipeline stage.  Two per stage pay off at
  // 512 channels per workgroup (more loads in flight per barrier); wider
  // stages cost occupancy elsewhere.
  if (nchan <= 64) launch_cfg<2, 1, MODE, T, 1>(tv, kp, data, zrow, ld, nchan, ov, st);
  else if (nchan <= 128) launch_cfg<4, 1, MODE, T, 1>(tv, kp, data, zrow, ld, nchan, ov, st);
  else if (nchan <= 256) launch_cfg<8, 1, MODE, T, 1>(tv, kp, data, zrow, ld, nchan, ov, st);
  else if (nchan <= 512) launch_cfg<8, 2, MODE, T, 2>(tv, kp, data, zrow, ld, nchan, ov, st);
  else launch_cfg<8, 4, MODE, T, 1>(tv, kp, data, zrow, ld, nchan, ov, st);
}

template <int MODE>
static void launch_prec(const TileView& tv, const KernelParams& kp, const void* data,
                        const void* zrow, int dtype, int64_t ld, int64_t nchan,
                        const OutView& ov, hipStream_t st) {
  switch (dtype) {
    case 0: launch_dt<MODE, double>(tv, kp, data, zrow, ld, nchan, ov, st); break;
    case 1: launch_dt<MODE, float>(tv, kp, data, zrow, ld, nchan, ov, st); break;
    case 2: launch_dt<MODE, _Float16>(tv, kp, data, zrow, ld, nchan, ov, st); break;
    default: launch_dt<MODE, uint16_t>(tv, kp, data, zrow, ld, nchan, ov, st); break;
  }
}

hipError_t launch_gather_mfma(const TileView& tv, const KernelParams& kp, const void* data,
                              const void* zrow, int dtype, int64_t ld, int64_t nchan, int prec,
                              const OutView& ov, hipStream_t st) {
  if (tv.ntiles <= 0) return hipSuccess;
  if (prec == 2) launch_prec<1>(tv, kp, data, zrow, dtype, ld, nchan, ov, st);
  else launch_prec<0>(tv, kp, data, zrow, dtype, ld, nchan, ov, st);
  return hipGetLastError();
}

}  // namespace cg
