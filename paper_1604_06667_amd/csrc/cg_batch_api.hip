// C ABI of batched gridding: many jobs in one lookup pass and one persistent
// contraction launch, with autotuning and HIP graph capture.
#include <algorithm>
#include <numeric>

#include "cg_handle.hpp"

using namespace cgh;

struct cg_batch {
  int device = 0;
  Allocator alloc;   // where the batch's buffers come from (captured at creation)
  int32_t dtype = CG_BF16;
  int32_t prec = CG_PREC_BF16;
  std::vector<cg_gridder*> jobs;
  // static per job (set at creation)
  std::vector<int64_t> toff, rooff, rbase;   // prefix offsets, size njobs + 1
  std::vector<int64_t> snap_nside, snap_ranges;  // per job, as laid out at creation
  int64_t ntiles = 0, nro = 0, nranges_tot = 0;
  int bits = 0;
  // per pass
  std::vector<int64_t> noff;                 // sample offsets, size njobs + 1
  int64_t ntot = 0;
  std::vector<cg::BatchJob> hjobs;           // host copy of the job table
  cg::BatchJob* pin_jobs = nullptr;          // pinned staging of the job table
  int64_t* pin_off = nullptr;                // pinned staging of noff | toff | rooff
  uint64_t* pin_word = nullptr;
  DevBuf d_jobs, d_off, keys, vals, keys2, vals2, hist, ring_off, sx, ranges, nranges, ncand,
      zrow, items, counter, flags;
  bool sorted_in_tmp = false;               // which key/value buffers hold the sorted run
  // work queue
  std::vector<cg::BatchItem> hitems;
  cg::BatchItem* pin_items = nullptr;
  size_t pin_items_cap = 0;
  int64_t nitems = 0;
  cg::BatchQueues queues{};                  // the items' segment of each XCD
  bool items_valid = false;
  std::vector<int64_t> items_for_n;          // sample counts the queue was ordered for
  // tuned launch shape (cg::launch_batch_mfma), item width, workgroups per CU
  int shape = 1, split = 0, bpc = 0;
  // graph
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // measurement
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t nev = 0;
};

namespace {

constexpr size_t kMaxBatchEvents = 4096;

void drop_graph(cg_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// grow a buffer; a captured graph holds the old addresses, so it is dropped
cg_status grow(cg_batch* b, DevBuf& buf, size_t bytes, const char* what) {
  if (bytes == 0) bytes = 1;
  if (buf.bytes >= bytes) return CG_OK;
  drop_graph(b);
  CG_HIP(ensure(b->alloc, buf, bytes), what);
  return CG_OK;
}

cg_status batch_event(cg_batch* b, std::pair<hipEvent_t, hipEvent_t>** pe) {
  *pe = nullptr;
  if (!b->prof || b->nev >= kMaxBatchEvents) return CG_OK;
  if (b->nev == b->ev.size()) {
    hipEvent_t x, y;
    CG_HIP(hipEventCreate(&x), "event");
    CG_HIP(hipEventCreate(&y), "event");
    b->ev.emplace_back(x, y);
  }
  *pe = &b->ev[b->nev++];
  return CG_OK;
}

cg_status check_inputs(const cg_batch* b, const cg_batch_job* in) {
  if (!b) return fail(CG_E_INVALID, "null batch");
  if (!in) return fail(CG_E_INVALID, "null job array");
  for (size_t j = 0; j < b->jobs.size(); ++j) {
    const cg_batch_job& q = in[j];
    const cg_gridder* g = b->jobs[j];
    if (q.nsamples < 0) return fail(CG_E_INVALID, "job %zu: nsamples < 0", j);
    if (!q.cube_out) return fail(CG_E_INVALID, "job %zu: null cube_out", j);
    if (q.nsamples > 0 && (!q.lon_deg || !q.lat_deg || !q.data))
      return fail(CG_E_INVALID, "job %zu: null coordinate or data pointer", j);
    if (q.ld_data < g->nchan) return fail(CG_E_INVALID, "job %zu: ld_data < nchan", j);
  }
  return CG_OK;
}

// Estimated cost of one work item of job j: candidates per tile (sample
// density times the area a tile's lookup covers) times (channels + weights).
double item_cost(const cg_gridder* g, int64_t n, int64_t cw) {
  double cand;
  const double rs = g->support_rad;
  if (g->kind == 0) {
    const double dx = fabs(g->wcs.cdelt1) * kDeg, dy = fabs(g->wcs.cdelt2) * kDeg;
    const double area = (double)g->wcs.naxis1 * dx * (double)g->wcs.naxis2 * dy;
    const double tile = (8.0 * dx + 2.0 * rs) * (8.0 * dy + 2.0 * rs);
    cand = area > 0.0 ? (double)n * std::min(1.0, tile / area) : (double)n;
  } else {
    cand = (double)n / (double)std::max<int64_t>(1, g->ntiles) * 4.0;
  }
  return cand * (double)(cw + 64);
}

// (Re)build the work queues for the current launch shape and sample
// counts: one segment per XCD, holding for every job (in order of
// decreasing estimated item cost) the items of one run of its tiles.  A
// WCS job's tiles are taken in the per-grid kernel's strip order, so each
// XCD gets a compact patch of the grid, as a single grid call gives it.
cg_status build_items(cg_batch* b, const cg_batch_job* in, hipStream_t st) {
  const int njobs = (int)b->jobs.size();
  const int64_t cp = cg::batch_shape_rows(b->shape);
  struct JobOrder { int j; int64_t cw, npass; double cost; };
  std::vector<JobOrder> ord;
  int64_t total = 0;
  for (int j = 0; j < njobs; ++j) {
    const cg_gridder* g = b->jobs[j];
    int64_t npass = (g->nchan + cp - 1) / cp;
    if (b->split) npass *= 2;
    int64_t cw = (g->nchan + npass - 1) / npass;
    cw = (cw + 31) / 32 * 32;
    npass = (g->nchan + cw - 1) / cw;
    ord.push_back({j, cw, npass, item_cost(g, in[j].nsamples, cw)});
    total += g->ntiles * npass;
  }
  if (total >= (1ll << 31)) return fail(CG_E_UNSUPPORTED, "too many work items");
  std::stable_sort(ord.begin(), ord.end(),
                   [](const JobOrder& a, const JobOrder& c) { return a.cost > c.cost; });
  b->hitems.clear();
  b->hitems.reserve((size_t)total);
  for (int k = 0; k < cg::kNumXcd; ++k) {
    b->queues.off[k] = (int64_t)b->hitems.size();
    for (const JobOrder& o : ord) {
      const cg_gridder* g = b->jobs[o.j];
      const int64_t v0 = g->ntiles * k / cg::kNumXcd, v1 = g->ntiles * (k + 1) / cg::kNumXcd;
      for (int64_t v = v0; v < v1; ++v) {
        const int64_t t = g->ntx > 0 ? cg::strip_tile(v, g->ntiles, g->ntx) : v;
        for (int64_t p = 0; p < o.npass; ++p) {
          const int64_t c0 = p * o.cw;
          const int64_t ce = std::min(c0 + o.cw, g->nchan);
          b->hitems.push_back({o.j, (int32_t)t, (int32_t)c0, (int32_t)ce});
        }
      }
    }
  }
  b->nitems = (int64_t)b->hitems.size();
  b->queues.off[cg::kNumXcd] = b->nitems;
  const size_t bytes = sizeof(cg::BatchItem) * std::max<size_t>(1, b->hitems.size());
  cg_status s = grow(b, b->items, bytes, "alloc work items");
  if (s != CG_OK) return s;
  if (b->pin_items_cap < bytes) {
    if (b->pin_items) (void)hipHostFree(b->pin_items);
    b->pin_items = nullptr;
    CG_HIP(hipHostMalloc((void**)&b->pin_items, bytes, hipHostMallocDefault), "pinned items");
    b->pin_items_cap = bytes;
  }
  // the previous upload from the staging buffer must be complete
  CG_HIP(hipStreamSynchronize(st), "sync items");
  memcpy(b->pin_items, b->hitems.data(), sizeof(cg::BatchItem) * b->hitems.size());
  CG_HIP(hipMemcpyAsync(b->items.p, b->pin_items, sizeof(cg::BatchItem) * b->hitems.size(),
                        hipMemcpyHostToDevice, st),
         "upload items");
  b->items_for_n.assign((size_t)njobs, 0);
  for (int j = 0; j < njobs; ++j) b->items_for_n[(size_t)j] = in[j].nsamples;
  b->items_valid = true;
  return CG_OK;
}

// Job table and offsets for the inputs `in`; uploads them on `st`.
cg_status upload_tables(cg_batch* b, const cg_batch_job* in, hipStream_t st) {
  const int njobs = (int)b->jobs.size();
  for (int j = 0; j < njobs; ++j) {
    // the batch's offsets were laid out for each gridder's kernel and nside
    const cg_gridder* g = b->jobs[j];
    if (!g->span_valid || g->nside != b->snap_nside[(size_t)j] ||
        g->total_ranges != b->snap_ranges[(size_t)j])
      return fail(CG_E_STATE, "job %d: gridder kernel or nside changed since cg_batch_create", j);
  }
  b->noff.assign((size_t)njobs + 1, 0);
  for (int j = 0; j < njobs; ++j) b->noff[(size_t)j + 1] = b->noff[(size_t)j] + in[j].nsamples;
  b->ntot = b->noff[(size_t)njobs];
  if (b->ntot > 0xFFFFFFFFll - 1) return fail(CG_E_UNSUPPORTED, "batch has >= 2^32 samples");
  b->hjobs.resize((size_t)njobs);
  for (int j = 0; j < njobs; ++j) {
    const cg_gridder* g = b->jobs[j];
    cg::BatchJob& q = b->hjobs[(size_t)j];
    q.lon = in[j].lon_deg;
    q.lat = in[j].lat_deg;
    q.data = in[j].data;
    q.n = in[j].nsamples;
    q.noff = b->noff[(size_t)j];
    q.ld = in[j].ld_data;
    q.nchan = g->nchan;
    q.nside = g->nside;
    q.ro_off = b->rooff[(size_t)j];
    q.toff = b->toff[(size_t)j];
    q.ntiles = g->ntiles;
    q.nslots = g->nslots;
    q.ntx = g->kind == 0 ? g->ntx : 0;
    q.rbase = b->rbase[(size_t)j];
    q.ntarget = g->ntarget;
    q.txyz = g->txyz.as<double>();
    q.tll = g->tll.as<double>();
    q.caps = g->caps.as<double>();
    q.ring_first = g->ring_first.as<int32_t>();
    q.range_off = g->range_off.as<uint64_t>();
    q.win = g->win.as<uint32_t>();
    q.slot_target = g->slot_target.as<int32_t>();
    q.cube = in[j].cube_out;
    cube_strides(g, &q.cst, &q.tst);
    q.wout = in[j].weights_out;
    if (g->kp.type > 1)
      return fail(CG_E_UNSUPPORTED, "job %d: batches take gauss1d and gauss2d kernels", j);
    q.kp = g->kp;
    q.rho = g->support_rad + 1e-9;
  }
  // staging buffers are reused: the previous upload must be complete
  CG_HIP(hipStreamSynchronize(st), "sync tables");
  memcpy(b->pin_jobs, b->hjobs.data(), sizeof(cg::BatchJob) * (size_t)njobs);
  int64_t* o = b->pin_off;
  for (int j = 0; j <= njobs; ++j) {
    o[j] = b->noff[(size_t)j];
    o[njobs + 1 + j] = b->toff[(size_t)j];
    o[2 * (njobs + 1) + j] = b->rooff[(size_t)j];
  }
  CG_HIP(hipMemcpyAsync(b->d_jobs.p, b->pin_jobs, sizeof(cg::BatchJob) * (size_t)njobs,
                        hipMemcpyHostToDevice, st),
         "upload jobs");
  CG_HIP(hipMemcpyAsync(b->d_off.p, b->pin_off, sizeof(int64_t) * 3 * ((size_t)njobs + 1),
                        hipMemcpyHostToDevice, st),
         "upload offsets");
  return CG_OK;
}

const int64_t* dev_noff(const cg_batch* b) { return b->d_off.as<int64_t>(); }
const int64_t* dev_toff(const cg_batch* b) { return b->d_off.as<int64_t>() + b->jobs.size() + 1; }
const int64_t* dev_rooff(const cg_batch* b) {
  return b->d_off.as<int64_t>() + 2 * (b->jobs.size() + 1);
}

// Device work of one pass up to the candidate scan (no host synchronisation).
cg_status lookup_part(cg_batch* b, hipStream_t st) {
  const int njobs = (int)b->jobs.size();
  const cg::BatchJob* dj = b->d_jobs.as<cg::BatchJob>();
  int* flags = b->flags.as<int>();
  CG_HIP(cg::launch_batch_prep(dj, dev_noff(b), njobs, b->ntot, b->keys.as<uint32_t>(),
                               b->vals.as<uint32_t>(), flags, st),
         "batch prep");
  bool in_tmp = false;
  CG_HIP(cg::radix_sort_jobs(b->keys.as<uint32_t>(), b->vals.as<uint32_t>(),
                             b->keys2.as<uint32_t>(), b->vals2.as<uint32_t>(),
                             b->hist.as<uint32_t>(), b->ntot, b->bits, dev_noff(b), njobs,
                             &in_tmp, st),
         "batch sort");
  b->sorted_in_tmp = in_tmp;
  const uint32_t* skeys = in_tmp ? b->keys2.as<uint32_t>() : b->keys.as<uint32_t>();
  const uint32_t* svals = in_tmp ? b->vals2.as<uint32_t>() : b->vals.as<uint32_t>();
  CG_HIP(cg::launch_batch_ring_offsets(dj, dev_rooff(b), njobs, b->nro, skeys,
                                       b->ring_off.as<uint32_t>(), st),
         "batch ring offsets");
  CG_HIP(cg::launch_batch_permute(dj, dev_noff(b), njobs, b->ntot, svals,
                                  b->ring_off.as<uint32_t>(), b->sx.as<double>(), st),
         "batch permute");
  CG_HIP(cg::launch_batch_tile_ranges(dj, dev_toff(b), njobs, b->ntiles, skeys,
                                      b->ring_off.as<uint32_t>(), b->ranges.as<uint32_t>(),
                                      b->nranges.as<uint32_t>(), b->ncand.as<uint64_t>(), st),
         "batch tile ranges");
  return CG_OK;
}

const uint32_t* sorted_vals(const cg_batch* b) {
  return b->sorted_in_tmp ? b->vals2.as<uint32_t>() : b->vals.as<uint32_t>();
}

// Device work after the lookup: the persistent contraction over the queue.
cg_status contract_part(cg_batch* b, hipStream_t st, bool events) {
  const cg::BatchJob* dj = b->d_jobs.as<cg::BatchJob>();
  CG_HIP(cg::launch_fill(b->counter.as<float>(), cg::kNumXcd, 0.0f, st), "clear counters");
  std::pair<hipEvent_t, hipEvent_t>* pe = nullptr;
  if (events) {
    cg_status s = batch_event(b, &pe);
    if (s != CG_OK) return s;
    if (pe) CG_HIP(hipEventRecord(pe->first, st), "event record");
  }
  cg::BatchRanges br;
  br.ranges = b->ranges.as<uint32_t>();
  br.nranges = b->nranges.as<uint32_t>();
  br.ncand = b->ncand.as<uint64_t>();
  br.srec = reinterpret_cast<const double4*>(b->sx.as<double>());
  CG_HIP(cg::launch_batch_mfma(dj, b->items.as<cg::BatchItem>(), b->queues, b->counter.as<int>(),
                               br, b->zrow.p, b->dtype, b->prec, b->shape, b->bpc, st),
         "batch contraction");
  if (pe) CG_HIP(hipEventRecord(pe->second, st), "event record");
  return CG_OK;
}

cg_status size_pass(cg_batch* b) {
  const int64_t n = std::max<int64_t>(b->ntot, 1);
  cg_status s;
  if ((s = grow(b, b->keys, 4 * n, "alloc keys")) != CG_OK) return s;
  if ((s = grow(b, b->vals, 4 * n, "alloc keys")) != CG_OK) return s;
  if ((s = grow(b, b->keys2, 4 * n, "alloc keys")) != CG_OK) return s;
  if ((s = grow(b, b->vals2, 4 * n, "alloc keys")) != CG_OK) return s;
  if ((s = grow(b, b->hist, 4 * cg::radix_hist_elems(n), "alloc hist")) != CG_OK) return s;
  if ((s = grow(b, b->sx, 32 * n, "alloc sorted records")) != CG_OK) return s;
  return CG_OK;
}

bool need_items(const cg_batch* b, const cg_batch_job* in) {
  if (!b->items_valid) return true;
  for (size_t j = 0; j < b->jobs.size(); ++j) {
    // re-order the queue when a job's sample count changes by more than 2x
    const int64_t a = b->items_for_n[j], c = in[j].nsamples;
    if ((a == 0) != (c == 0) || c > 2 * a || a > 2 * c) return true;
  }
  return false;
}

// One eager pass: tables, lookup and contraction.  Every buffer is sized
// from the sample counts (known on the host), so the pass does not wait for
// the device except to reuse the pinned staging buffers of the tables.
cg_status eager_pass(cg_batch* b, const cg_batch_job* in, hipStream_t st) {
  cg_status s = upload_tables(b, in, st);
  if (s != CG_OK) return s;
  if ((s = size_pass(b)) != CG_OK) return s;
  if (need_items(b, in) && (s = build_items(b, in, st)) != CG_OK) return s;
  if ((s = lookup_part(b, st)) != CG_OK) return s;
  return contract_part(b, st, true);
}

}  // namespace

extern "C" {

cg_status cg_batch_create(cg_batch** out, cg_gridder* const* jobs, int32_t njobs, int32_t dtype) {
  if (!out || !jobs) return fail(CG_E_INVALID, "null pointer");
  *out = nullptr;
  if (njobs < 1 || njobs > 256) return fail(CG_E_INVALID, "njobs must be in [1, 256]");
  if (dtype < CG_F64 || dtype > CG_BF16) return fail(CG_E_INVALID, "unknown dtype %d", dtype);
  for (int j = 0; j < njobs; ++j) {
    const cg_gridder* g = jobs[j];
    if (!g) return fail(CG_E_INVALID, "job %d: null gridder", j);
    if (!g->kernel_set) return fail(CG_E_STATE, "job %d: set_kernel must be called first", j);
    if (g->prec == CG_PREC_FP32)
      return fail(CG_E_UNSUPPORTED, "job %d: batches use the matrix-core precisions", j);
    if (g->prec != jobs[0]->prec) return fail(CG_E_UNSUPPORTED, "mixed precisions in one batch");
    if (g->kp.type > 1)
      return fail(CG_E_UNSUPPORTED, "job %d: batches take gauss1d and gauss2d kernels", j);
    if (g->device != jobs[0]->device) return fail(CG_E_UNSUPPORTED, "mixed devices in one batch");
    for (int k = 0; k < j; ++k)
      if (jobs[k] == g) return fail(CG_E_INVALID, "job %d repeats gridder of job %d", j, k);
  }
  cg_batch* b = new cg_batch();
  b->device = jobs[0]->device;
  b->alloc = current_allocator(b->device);
  b->dtype = dtype;
  b->prec = jobs[0]->prec;
  b->jobs.assign(jobs, jobs + njobs);
  cg_status s = CG_OK;
  auto done = [&](cg_status r) {
    if (r != CG_OK) cg_batch_destroy(b);
    else *out = b;
    return r;
  };
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return done(hip_fail(e, "hipSetDevice"));
  b->toff.assign((size_t)njobs + 1, 0);
  b->rooff.assign((size_t)njobs + 1, 0);
  b->rbase.assign((size_t)njobs + 1, 0);
  int64_t maxside = 1;
  for (int j = 0; j < njobs; ++j) {
    cg_gridder* g = jobs[j];
    if ((s = ensure_span(g, nullptr)) != CG_OK) return done(s);
    b->toff[(size_t)j + 1] = b->toff[(size_t)j] + g->ntiles;
    b->rooff[(size_t)j + 1] = b->rooff[(size_t)j] + 4 * g->nside + 1;
    b->rbase[(size_t)j + 1] = b->rbase[(size_t)j] + g->total_ranges;
    b->snap_nside.push_back(g->nside);
    b->snap_ranges.push_back(g->total_ranges);
    maxside = std::max(maxside, g->nside);
  }
  b->ntiles = b->toff[(size_t)njobs];
  b->nro = b->rooff[(size_t)njobs];
  b->nranges_tot = b->rbase[(size_t)njobs];
  b->bits = bits_for((uint64_t)cg::hpx::npix(maxside));
  if (b->ntiles >= (1ll << 31)) return done(fail(CG_E_UNSUPPORTED, "too many tiles"));
  const int64_t nt = std::max<int64_t>(b->ntiles, 1);
  const Allocator& al = b->alloc;
  if ((e = ensure(al, b->d_jobs, sizeof(cg::BatchJob) * njobs)) != hipSuccess ||
      (e = ensure(al, b->d_off, sizeof(int64_t) * 3 * (njobs + 1))) != hipSuccess ||
      (e = ensure(al, b->ring_off, 4 * std::max<int64_t>(b->nro, 1))) != hipSuccess ||
      (e = ensure(al, b->ranges, 8 * std::max<int64_t>(b->nranges_tot, 1))) != hipSuccess ||
      (e = ensure(al, b->nranges, 4 * nt)) != hipSuccess ||
      (e = ensure(al, b->ncand, 8 * nt)) != hipSuccess ||
      (e = ensure(al, b->zrow, 8 * 512)) != hipSuccess ||
      (e = ensure(al, b->counter, 64)) != hipSuccess || (e = ensure(al, b->flags, 64)) != hipSuccess)
    return done(hip_fail(e, "alloc batch"));
  if ((e = hipMemset(b->zrow.p, 0, 8 * 512)) != hipSuccess ||
      (e = hipMemset(b->flags.p, 0, 64)) != hipSuccess)
    return done(hip_fail(e, "clear batch"));
  if ((e = hipHostMalloc((void**)&b->pin_jobs, sizeof(cg::BatchJob) * njobs,
                         hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc((void**)&b->pin_off, sizeof(int64_t) * 3 * (njobs + 1),
                         hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc((void**)&b->pin_word, sizeof(uint64_t) * 2, hipHostMallocDefault)) !=
          hipSuccess)
    return done(hip_fail(e, "pinned staging"));
  if ((e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess)
    return done(hip_fail(e, "capture stream"));
  return done(CG_OK);
}

cg_status cg_batch_grid(cg_batch* b, const cg_batch_job* in, void* stream) {
  cg_status s = check_inputs(b, in);
  if (s != CG_OK) return s;
  CG_HIP(hipSetDevice(b->device), "hipSetDevice");
  return eager_pass(b, in, (hipStream_t)stream);
}

cg_status cg_batch_tune(cg_batch* b, const cg_batch_job* in, int32_t reps, void* stream) {
  cg_status s = check_inputs(b, in);
  if (s != CG_OK) return s;
  if (reps < 1 || reps > 100) return fail(CG_E_INVALID, "reps must be in [1, 100]");
  CG_HIP(hipSetDevice(b->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  drop_graph(b);
  if ((s = eager_pass(b, in, st)) != CG_OK) return s;
  hipEvent_t e0, e1;
  CG_HIP(hipEventCreate(&e0), "event");
  CG_HIP(hipEventCreate(&e1), "event");
  const bool prof = b->prof;
  b->prof = false;
  float best = 1e30f;
  int bb = b->shape, bs = b->split, bc = b->bpc;
  for (int shape = 0; shape < cg::kBatchShapes; ++shape) {
    const int occ = cg::batch_max_blocks_per_cu(b->dtype, b->prec, shape);
    std::vector<int> shapes = {occ};
    if (occ > 1) shapes.push_back(1);
    for (int split : {0, 1}) {
      for (int bpc : shapes) {
        b->shape = shape;
        b->split = split;
        b->bpc = bpc;
        if ((s = build_items(b, in, st)) != CG_OK) break;
        // one untimed run, then reps timed
        if ((s = contract_part(b, st, false)) != CG_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) {
          s = fail(CG_E_DEVICE, "event");
          break;
        }
        for (int r = 0; r < reps && s == CG_OK; ++r) s = contract_part(b, st, false);
        if (s != CG_OK) break;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          s = fail(CG_E_DEVICE, "event");
          break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
          best = ms;
          bb = shape;
          bs = split;
          bc = bpc;
        }
      }
      if (s != CG_OK) break;
    }
    if (s != CG_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->prof = prof;
  b->shape = bb;
  b->split = bs;
  b->bpc = bc;
  if (s != CG_OK) return s;
  if ((s = build_items(b, in, st)) != CG_OK) return s;
  // leave the outputs from the chosen shape
  if ((s = contract_part(b, st, false)) != CG_OK) return s;
  CG_HIP(hipStreamSynchronize(st), "sync tune");
  return CG_OK;
}

cg_status cg_batch_capture(cg_batch* b, const cg_batch_job* in, void* stream) {
  cg_status s = check_inputs(b, in);
  if (s != CG_OK) return s;
  CG_HIP(hipSetDevice(b->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  drop_graph(b);
  if ((s = eager_pass(b, in, st)) != CG_OK) return s;
  CG_HIP(hipStreamSynchronize(st), "sync before capture");
  // every buffer is sized for `in`; record the device work of one pass
  hipStream_t cs = b->cap_stream;
  CG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
  cg_status s1 = lookup_part(b, cs);
  if (s1 == CG_OK) s1 = contract_part(b, cs, false);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(cs, &graph);
  if (s1 != CG_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s1;
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(e, "instantiate graph");
  }
  b->graph = graph;
  b->exec = exec;
  return CG_OK;
}

cg_status cg_batch_replay(cg_batch* b, void* stream) {
  if (!b) return fail(CG_E_INVALID, "null batch");
  if (!b->exec) return fail(CG_E_STATE, "no captured graph (cg_batch_capture)");
  for (size_t j = 0; j < b->jobs.size(); ++j) {
    const cg_gridder* g = b->jobs[j];
    if (!g->span_valid || g->nside != b->snap_nside[j] || g->total_ranges != b->snap_ranges[j]) {
      drop_graph(b);
      return fail(CG_E_STATE, "job %zu: gridder changed since capture", j);
    }
  }
  CG_HIP(hipSetDevice(b->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  std::pair<hipEvent_t, hipEvent_t>* pe = nullptr;
  cg_status s = batch_event(b, &pe);
  if (s != CG_OK) return s;
  if (pe) CG_HIP(hipEventRecord(pe->first, st), "event record");
  CG_HIP(hipGraphLaunch(b->exec, st), "graph launch");
  if (pe) CG_HIP(hipEventRecord(pe->second, st), "event record");
  return CG_OK;
}

cg_status cg_batch_sync(cg_batch* b, void* stream) {
  if (!b) return fail(CG_E_INVALID, "null batch");
  CG_HIP(hipSetDevice(b->device), "hipSetDevice");
  CG_HIP(hipStreamSynchronize((hipStream_t)stream), "sync");
  int f = 0;
  CG_HIP(hipMemcpy(&f, b->flags.p, sizeof f, hipMemcpyDeviceToHost), "read flags");
  if (f) {
    CG_HIP(hipMemset(b->flags.p, 0, sizeof f), "clear flags");
    return fail(CG_E_INPUT, "input contained non-finite coordinates or |lat| > 90 (skipped)");
  }
  return CG_OK;
}

cg_status cg_batch_query(const cg_batch* b, int32_t what, int64_t* value) {
  if (!b || !value) return fail(CG_E_INVALID, "null pointer");
  switch (what) {
    case 0: *value = (int64_t)b->jobs.size(); break;
    case 1: *value = b->ntot; break;
    case 2: *value = b->ntiles; break;
    case 3: *value = b->nitems; break;
    case 4: {
      // candidates of the last pass: waits for the device, sums the tile counts
      *value = 0;
      if (b->ntiles <= 0 || b->ntot <= 0) break;
      CG_HIP(hipSetDevice(b->device), "hipSetDevice");
      std::vector<uint64_t> c((size_t)b->ntiles);
      CG_HIP(hipDeviceSynchronize(), "sync");
      CG_HIP(hipMemcpy(c.data(), b->ncand.p, sizeof(uint64_t) * c.size(), hipMemcpyDeviceToHost),
             "read candidates");
      uint64_t t = 0;
      for (uint64_t v : c) t += v;
      *value = (int64_t)t;
      break;
    }
    case 5: *value = cg::batch_shape_rows(b->shape); break;
    case 6: *value = b->split; break;
    case 7: *value = b->bpc > 0 ? b->bpc : cg::batch_max_blocks_per_cu(b->dtype, b->prec, b->shape); break;
    case 9: *value = b->shape; break;
    case 8: *value = b->exec ? 1 : 0; break;
    default: return fail(CG_E_INVALID, "unknown query %d", what);
  }
  return CG_OK;
}

cg_status cg_batch_profile_enable(cg_batch* b, int32_t enable) {
  if (!b) return fail(CG_E_INVALID, "null batch");
  b->prof = enable != 0;
  if (b->prof) b->nev = 0;
  return CG_OK;
}

cg_status cg_batch_profile_read(cg_batch* b, int64_t* launches, double* total_ms) {
  if (!b || !launches || !total_ms) return fail(CG_E_INVALID, "null pointer");
  CG_HIP(hipSetDevice(b->device), "hipSetDevice");
  double tot = 0.0;
  for (size_t i = 0; i < b->nev; ++i) {
    CG_HIP(hipEventSynchronize(b->ev[i].second), "event sync");
    float ms = 0.0f;
    CG_HIP(hipEventElapsedTime(&ms, b->ev[i].first, b->ev[i].second), "event time");
    tot += ms;
  }
  *launches = (int64_t)b->nev;
  *total_ms = tot;
  return CG_OK;
}

void cg_batch_destroy(cg_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (auto& e : b->ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  DevBuf* bufs[] = {&b->d_jobs, &b->d_off, &b->keys, &b->vals, &b->keys2, &b->vals2, &b->hist,
                    &b->ring_off, &b->sx, &b->ranges, &b->nranges, &b->ncand, &b->zrow,
                    &b->items, &b->counter, &b->flags};
  for (DevBuf* d : bufs) d->release();
  if (b->pin_jobs) (void)hipHostFree(b->pin_jobs);
  if (b->pin_off) (void)hipHostFree(b->pin_off);
  if (b->pin_word) (void)hipHostFree(b->pin_word);
  if (b->pin_items) (void)hipHostFree(b->pin_items);
  delete b;
}

}  // extern "C"
