// Persistent matrix-core contraction for a batch of gridding jobs.
//
// Every (job, tile, channel range) of the batch is one work item.  The
// items sit in one queue per XCD: each job's tiles are split into one run
// of neighbouring tiles per XCD, and every queue lists its runs of all jobs
// in order of estimated item cost, largest first (longest processing time
// first).  A grid sized to the resident capacity of the chip takes items
// one at a time from atomic counters: a workgroup drains the queue of its
// own XCD (block b runs on XCD b % 8), so tiles that share candidate rows
// and output lines meet in that XCD's L2, then takes what is left in the
// other queues in turn.  Jobs of very different sizes thus share one launch
// without a tail of idle compute units.
// Each item runs the same tile contraction as the per-grid kernel, with the
// kernel type (circular or elliptical) taken from the job at run time, and
// writes the normalised cube and weights of its job directly.
#include "cg_mfma_tile.hpp"

namespace cg {

// Launch shapes of the persistent kernel (chosen by the autotuner):
// wavefronts per workgroup and 32-channel blocks per wavefront.
//   shape 0: 8 x 1 (256 channels per item)    shape 1: 8 x 2 (512)
//   shape 2: 4 x 1 (128)                      shape 3: 4 x 2 (256, two workgroups per CU)
// (4-wavefront workgroups are held to two wavefronts per SIMD, so that two
// of them share a compute unit and cover each other's barrier waits)
template <int NW, int BPW, int MODE, typename T>
__global__ void __launch_bounds__(NW * 64, NW == 4 ? 2 : 1) k_batch_mfma(
    const BatchJob* __restrict__ jobs, const BatchItem* __restrict__ items, BatchQueues q,
    int* counter, BatchRanges br, const T* __restrict__ zrow) {
  __shared__ int64_t s_item;
  const int home = (int)(blockIdx.x % kNumXcd);
  int visited = 0;   // queues found empty so far (thread 0): home, home + 1, ...
  for (;;) {
    __syncthreads();  // the previous item is done with LDS
    if (threadIdx.x == 0) {
      int64_t next = -1;
      while (visited < kNumXcd) {
        const int k = (home + visited) % kNumXcd;
        const int64_t i = atomicAdd(&counter[k], 1);
        if (i < q.off[k + 1] - q.off[k]) {
          next = q.off[k] + i;
          break;
        }
        ++visited;   // every counter only grows, so an exhausted queue stays so
      }
      s_item = next;
    }
    __syncthreads();
    const int64_t it = s_item;
    if (it < 0) break;
    const BatchItem item = items[it];
    const BatchJob& jb = jobs[item.job];   // global memory, not a kernel argument
    TileView tv;
    tv.txyz = jb.txyz;
    tv.tll = jb.tll;
    tv.rng = br.ranges + 2 * jb.rbase;
    tv.roff = jb.range_off;
    tv.nr = br.nranges + jb.toff;
    tv.ntot = br.ncand + jb.toff;
    tv.nslots = jb.nslots;
    tv.ntiles = jb.ntiles;
    tv.ntx = jb.ntx;   // same candidate order as the per-grid kernel
    tv.srec = br.srec;
    OutView ov;
    ov.S = nullptr;
    ov.W = nullptr;
    ov.Wn = nullptr;
    ov.cube = jb.cube;
    ov.wout = jb.wout;
    ov.slot_target = jb.slot_target;
    ov.ntarget = jb.ntarget;
    ov.cst = jb.cst;
    ov.tst = jb.tst;
    ov.mode = ACC_FINAL;
    mfma_tile<NW, BPW, 2, MODE, false, T, 1, true>(tv, jb.kp, (const T*)jb.data, zrow, jb.ld, jb.nchan, ov,
                                          item.tile, item.c0, item.cend);
  }
}

template <int NW, int BPW, int MODE, typename T>
static int occ_of() {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_mfma<NW, BPW, MODE, T>, NW * 64,
                                                   0) != hipSuccess)
    return 0;
  return occ;
}

template <int NW, int BPW, int MODE, typename T>
static hipError_t launch_bt(const BatchJob* jobs, const BatchItem* items, const BatchQueues& q,
                            int* counter, const BatchRanges& br, const void* zrow,
                            int blocks_per_cu, hipStream_t st) {
  const int64_t nitems = q.off[kNumXcd];
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int occ = occ_of<NW, BPW, MODE, T>();
  int per = blocks_per_cu > 0 && blocks_per_cu < occ ? blocks_per_cu : occ;
  if (per < 1) per = 1;
  int64_t grid = (int64_t)ncu * per;
  if (grid > nitems) grid = nitems;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((k_batch_mfma<NW, BPW, MODE, T>), dim3((unsigned)grid), dim3(NW * 64), 0, st,
                     jobs, items, q, counter, br, (const T*)zrow);
  return hipGetLastError();
}

template <int MODE, typename T>
static hipError_t launch_bs(int shape, const BatchJob* jobs, const BatchItem* items,
                            const BatchQueues& q, int* counter, const BatchRanges& br,
                            const void* zrow, int blocks_per_cu, hipStream_t st) {
#define CG_BT(NW_, BPW_) \
  launch_bt<NW_, BPW_, MODE, T>(jobs, items, q, counter, br, zrow, blocks_per_cu, st)
  switch (shape) {
    case 0: return CG_BT(8, 1);
    case 1: return CG_BT(8, 2);
    case 2: return CG_BT(4, 1);
    case 3: return CG_BT(4, 2);
    default: return hipErrorInvalidValue;
  }
#undef CG_BT
}

template <int MODE>
static hipError_t launch_bm(int dtype, int shape, const BatchJob* jobs, const BatchItem* items,
                            const BatchQueues& q, int* counter, const BatchRanges& br,
                            const void* zrow, int blocks_per_cu, hipStream_t st) {
#define CG_BS(T_) \
  launch_bs<MODE, T_>(shape, jobs, items, q, counter, br, zrow, blocks_per_cu, st)
  switch (dtype) {
    case 0: return CG_BS(double);
    case 1: return CG_BS(float);
    case 2: return CG_BS(_Float16);
    default: return CG_BS(uint16_t);
  }
#undef CG_BS
}

hipError_t launch_batch_mfma(const BatchJob* jobs, const BatchItem* items, const BatchQueues& q,
                             int* counter, const BatchRanges& br, const void* zrow, int dtype,
                             int prec, int shape, int blocks_per_cu, hipStream_t st) {
  if (q.off[kNumXcd] <= 0) return hipSuccess;
  if (prec == 2)
    return launch_bm<1>(dtype, shape, jobs, items, q, counter, br, zrow, blocks_per_cu, st);
  return launch_bm<0>(dtype, shape, jobs, items, q, counter, br, zrow, blocks_per_cu, st);
}

template <int MODE, typename T>
static int occ_s(int shape) {
  switch (shape) {
    case 0: return occ_of<8, 1, MODE, T>();
    case 1: return occ_of<8, 2, MODE, T>();
    case 2: return occ_of<4, 1, MODE, T>();
    case 3: return occ_of<4, 2, MODE, T>();
    default: return 0;
  }
}

template <int MODE>
static int occ_m(int dtype, int shape) {
  switch (dtype) {
    case 0: return occ_s<MODE, double>(shape);
    case 1: return occ_s<MODE, float>(shape);
    case 2: return occ_s<MODE, _Float16>(shape);
    default: return occ_s<MODE, uint16_t>(shape);
  }
}

int batch_max_blocks_per_cu(int dtype, int prec, int shape) {
  return prec == 2 ? occ_m<1>(dtype, shape) : occ_m<0>(dtype, shape);
}

int batch_shape_rows(int shape) {
  static const int rows[4] = {256, 512, 128, 256};
  return shape >= 0 && shape < 4 ? rows[shape] : 0;
}

}  // namespace cg
