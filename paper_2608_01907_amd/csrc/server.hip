// Continuous-batching layout server (the layout_server_* entry points of
// include/snaplayout.h).
//
// Threads: callers submit, poll, wait and take under one mutex; a single
// scheduler thread owns every HIP call after creation.  Jobs fall into three
// classes by size (LDS, one XCD's L2, all CUs), and each class has a stream
// and launches of its own.  In a loop the scheduler
//   1. notes the launches that have ended (an event per class), advances
//      their jobs' epoch counters and retires finished jobs (positions to
//      host, device memory freed, latency recorded) and cancelled ones;
//   2. admits queued jobs in arrival order while a slot is free and the job's
//      device footprint fits the budget (device copy, validation, chunk
//      table, alias table of weighted negatives, initial positions: the
//      caller's, seeded uniform or Pivot MDS);
//   3. starts the next launch of every class whose last one has ended: up to
//      ten epochs of every LDS job, one workgroup each; a slice of the
//      current epoch of every XCD-class job on XCD-local bins; a slice of the
//      current epoch of the oldest all-CU jobs that fit the device's lanes.
// No class waits for another, so a long launch of one class holds up no job
// of the others.  In JACOBI mode (the synchronous test mode) every job runs
// on the global engine with its own accumulator D; the epoch's slices add
// into D and the job's positions move (Y += D) once its last slice of the
// epoch has run.  While the server is held (layout_server_hold) jobs are
// still admitted and set up, but no launch starts; per-job debug requests
// (the negatives a job draws) are answered by the scheduler between
// launches, on the job's own device state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "snaplayout.h"

using namespace snap;

namespace {

double now_s() {
  using clock = std::chrono::steady_clock;
  return std::chrono::duration<double>(clock::now().time_since_epoch()).count();
}

constexpr int64_t kDefaultRoundEdges = 32ll << 20;
constexpr int kCancelled = 1;  // finish_job code of a cancelled job (not an error)
constexpr int64_t kMinSliceEdges = 1ll << 18;
constexpr int32_t kLdsLaunchEpochs = 10;  // LDS class: epochs of a job per launch

struct Job {
  int64_t id = 0;
  int32_t n = 0, k = 0, epochs = 0;
  uint64_t seed = 0;
  int64_t nnz = 0;
  std::vector<int32_t> row, col;  // host copy, dropped once on the device
  std::vector<uint32_t> weights;  // caller's negative weights (LAYOUT_NEG_CUSTOM)
  std::vector<float> init;        // caller's initial positions (n*2) or empty
  std::vector<float> result;
  std::atomic<bool> cancel{false};  // set by layout_server_cancel while running
  int state = LAYOUT_JOB_QUEUED;
  int err_code = LAYOUT_OK;
  std::string error;
  double t_submit = 0, t_done = 0;
  // device side (scheduler thread only)
  DeviceBuffers buf;
  int64_t footprint = 0;
  bool lds = false;
  int cls = 0;             // kClassLds, kClassXcd or kClassWide
  bool in_flight = false;  // part of a launch that has not ended
  int32_t bundle = kDefaultBundle, hub = kDefaultBundle * kHubFactor;
  int32_t lanes = 0;  // LDS engine: working lanes of the workgroup
  int64_t chunk_cap = 0, n_chunks = 0;
  GraphDesc desc{};
  float2* D = nullptr;    // JACOBI: the epoch's accumulated displacement
  int32_t t = 0;          // epochs completed
  int64_t chunk_pos = 0;  // chunks of the current epoch already processed
};

// The three classes of job.  Each has launches of its own, on a stream of its
// own: jobs whose positions fit one workgroup's LDS, jobs whose positions fit
// one XCD's L2, and the rest, which run on all CUs.
enum { kClassLds = 0, kClassXcd = 1, kClassWide = 2, kClasses = 3 };

// A class's launch: the jobs it advances, the chunks of its current epoch
// each runs, and the host tables its uploads read (kept until it has ended).
struct ClassLaunch {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<Job*> jobs;
  std::vector<int64_t> slice;
  std::vector<GraphDesc> table;
  std::vector<int32_t> ids;
  std::vector<XcdSeg> segs;
  XcdBin bins[kXcds];
};

// A caller's request for the negatives a running job draws in one epoch,
// answered by the scheduler thread.
struct DrawRequest {
  int64_t job = 0;
  int32_t epoch = 0;
  int32_t* out = nullptr;  // host, nnz * k
  bool done = false;
  int rc = LAYOUT_OK;
  std::string msg;
};

}  // namespace

struct layout_server {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> queue;
  std::unordered_map<int64_t, Job*> jobs;
  std::vector<Job*> active;  // scheduler thread only
  bool stop = false;
  bool hold = false;  // admit and set up jobs, but start no launch
  std::deque<DrawRequest*> draw_requests;
  bool dead = false;  // a device error stopped the scheduler
  std::string dead_msg;
  std::thread thr;
  layout_opts opts{};
  int32_t mode_global = LAYOUT_HOGWILD_STORE, mode_lds = LAYOUT_ATOMIC;
  int64_t budget = 0, in_use = 0, round_edges = kDefaultRoundEdges;
  int32_t max_slots = 1;
  int64_t next_id = 1;
  int dev = 0;
  hipStream_t stream = nullptr;  // job setup, readout and debug requests
  ClassLaunch cls[kClasses];
  GraphDesc* d_table = nullptr;
  GraphDesc* d_table_lds = nullptr;
  int32_t* d_ids = nullptr;
  uint32_t* d_err = nullptr;
  // XCD-local engine for global jobs whose positions fit one XCD's L2
  bool xcd_ok = false;
  GraphDesc* d_table_xcd = nullptr;
  XcdSeg* d_segs = nullptr;
  XcdBin* d_bins = nullptr;
  int32_t* d_xcd_ctr = nullptr;
  int lds_cap = 0;
  // stats (under mu)
  int64_t submitted = 0, completed = 0, failed = 0, rejected = 0, cancelled = 0, rounds = 0;
  double edge_updates = 0, busy_seconds = 0;
  std::vector<double> latencies;
};

namespace {

int64_t footprint_of(const layout_server_t* S, const Job& j, int32_t bundle, int32_t hub) {
  const int64_t cap = j.nnz > 0 ? chunk_bound(j.nnz, bundle, hub) : 0;
  // row_ptr (64-bit), col, positions, chunk table (64-bit begin + 32-bit source),
  // alias table (weighted negatives)
  int64_t b = 8 * (int64_t(j.n) + 1) + 4 * j.nnz + 8 * int64_t(j.n) + 12 * cap + 8;
  if (S->opts.neg_weights != LAYOUT_NEG_UNIFORM) b += 8 * int64_t(j.n);
  if (S->mode_global == LAYOUT_JACOBI) b += 8 * int64_t(j.n);  // accumulator D
  return b;
}

void plan_job(const layout_server_t* S, Job& j) {
  j.lds = S->opts.engine != LAYOUT_ENGINE_GLOBAL && lds_bytes_for(j.n) <= S->lds_cap;
  const int32_t nz = static_cast<int32_t>(j.nnz);
  if (j.lds) {
    const int block =
        S->opts.block_threads ? S->opts.block_threads : lds_lanes_for(j.n, S->opts.nodes_per_lane);
    j.lanes = block;
    j.bundle = S->opts.bundle_edges ? S->opts.bundle_edges : std::max(1, std::min(16, nz / (4 * block)));
    j.hub = S->opts.hub_split_edges ? S->opts.hub_split_edges : kLdsHub;
  } else {
    j.bundle = S->opts.bundle_edges ? S->opts.bundle_edges : kDefaultBundle;
    j.hub = S->opts.hub_split_edges ? S->opts.hub_split_edges : kHubFactor * j.bundle;
  }
  j.cls = j.lds ? kClassLds
          : (S->xcd_ok && int64_t(j.n) * 8 <= kXcdMaxPositionBytes) ? kClassXcd
                                                                    : kClassWide;
  j.footprint = footprint_of(S, j, j.bundle, j.hub);
}

int jalloc(layout_server_t* S, Job& j, void** p, size_t bytes, const char* what) {
  if (bytes == 0) bytes = 8;
  // stream-ordered: a plain hipMalloc/hipFree pair would make every
  // admission and retirement wait for all classes' launches to end
  hipError_t e = hipMallocAsync(p, bytes, S->stream);
  if (e != hipSuccess) return hip_fail(e, what);
  j.buf.add(*p, bytes);
  return LAYOUT_OK;
}

// Device setup of an admitted job (scheduler thread).
int setup_job(layout_server_t* S, Job& j) {
  int64_t *row = nullptr, *cb = nullptr;
  int32_t *col = nullptr, *cs = nullptr;
  float2* Y = nullptr;
  uint32_t *thr = nullptr, *alias = nullptr;
  j.chunk_cap = j.nnz > 0 ? chunk_bound(j.nnz, j.bundle, j.hub) : 0;
  int rc;
  if ((rc = jalloc(S, j, reinterpret_cast<void**>(&row), 8 * (size_t(j.n) + 1), "row_ptr")) ||
      (rc = jalloc(S, j, reinterpret_cast<void**>(&col), 4 * size_t(j.nnz), "col")) ||
      (rc = jalloc(S, j, reinterpret_cast<void**>(&Y), 8 * size_t(j.n), "positions")) ||
      (rc = jalloc(S, j, reinterpret_cast<void**>(&cb), 8 * size_t(j.chunk_cap + 1), "chunk begin")) ||
      (rc = jalloc(S, j, reinterpret_cast<void**>(&cs), 4 * size_t(j.chunk_cap), "chunk src")))
    return rc;
  if ((rc = upload_row_ptr(S->stream, j.row.data(), j.n, false, row)) != LAYOUT_OK) return rc;
  hipError_t e = hipSuccess;
  if (j.nnz > 0)
    e = hipMemcpyAsync(col, j.col.data(), 4 * size_t(j.nnz), hipMemcpyHostToDevice, S->stream);
  if (e != hipSuccess) return hip_fail(e, "copying a job");
  if ((rc = validate_csr(S->stream, row, col, j.n, j.nnz, S->d_err)) != LAYOUT_OK) return rc;
  if (j.nnz > 0 && (rc = build_chunk_table(S->stream, row, j.n, j.nnz, j.bundle, j.hub, cb, cs,
                                           &j.n_chunks)) != LAYOUT_OK)
    return rc;
  if (S->opts.neg_weights != LAYOUT_NEG_UNIFORM && j.nnz > 0) {
    if ((rc = jalloc(S, j, reinterpret_cast<void**>(&thr), 4 * size_t(j.n), "alias thr")) ||
        (rc = jalloc(S, j, reinterpret_cast<void**>(&alias), 4 * size_t(j.n), "alias")))
      return rc;
    rc = S->opts.neg_weights == LAYOUT_NEG_CUSTOM
             ? upload_weights_and_build_alias(S->stream, row, j.weights.data(), j.n, false, thr,
                                              alias)
             : build_alias_table(S->stream, row, nullptr, j.n, j.nnz, thr, alias);
    if (rc != LAYOUT_OK) return rc;
  }
  if (S->mode_global == LAYOUT_JACOBI) {
    if ((rc = jalloc(S, j, reinterpret_cast<void**>(&j.D), 8 * size_t(j.n), "jacobi delta")))
      return rc;
    launch_fill_zero(S->stream, j.D, j.n);
  }
  if (!j.init.empty()) {
    e = hipMemcpyAsync(Y, j.init.data(), 8 * size_t(j.n), hipMemcpyHostToDevice, S->stream);
    if (e != hipSuccess) return hip_fail(e, "copying init_pos");
  } else if (S->opts.init_mode == LAYOUT_INIT_PMDS && j.n > 0) {
    // blocks the scheduler for the job's Pivot MDS (synchronises the stream)
    if ((rc = pmds_positions(S->stream, row, col, j.n,
                             S->opts.pmds_pivots ? S->opts.pmds_pivots : kDefaultPivots, j.seed,
                             Y, nullptr, nullptr, nullptr)) != LAYOUT_OK)
      return rc;
  } else {
    launch_init_positions(S->stream, Y, j.n, j.seed);
  }
  GraphDesc& d = j.desc;
  d = GraphDesc{};
  d.row_ptr = row;
  d.col = col;
  d.chunk_begin = cb;
  d.chunk_src = cs;
  d.Y = Y;
  d.D = j.D;
  d.thr = thr;
  d.alias = alias;
  d.nnz = j.nnz;
  d.n = j.n;
  d.hub = j.hub;
  d.T = j.epochs;
  d.seed = j.seed;
  d.eta0 = S->opts.eta0;
  d.alpha = S->opts.alpha;
  d.beta = S->opts.beta;
  d.gamma = S->opts.gamma;
  d.force = S->opts.force_kernel;
  d.sc = sampler_consts(j.n);
  d.lanes = j.lds ? j.lanes : 0;
  e = hipStreamSynchronize(S->stream);
  if (e != hipSuccess) return hip_fail(e, "job setup");
  // the host copies are no longer needed
  std::vector<int32_t>().swap(j.row);
  std::vector<int32_t>().swap(j.col);
  std::vector<uint32_t>().swap(j.weights);
  std::vector<float>().swap(j.init);
  return LAYOUT_OK;
}

void finish_job(layout_server_t* S, Job* j, int code, const std::string& msg) {
  j->buf.free_all_async(S->stream);
  std::lock_guard<std::mutex> lk(S->mu);
  S->in_use -= j->footprint;
  j->t_done = now_s();
  if (code == LAYOUT_OK) {
    j->state = LAYOUT_JOB_DONE;
    S->completed += 1;
    S->edge_updates += double(j->nnz / 2) * (1 + j->k) * j->epochs;
    S->latencies.push_back(j->t_done - j->t_submit);
  } else if (code == kCancelled) {
    j->state = LAYOUT_JOB_CANCELLED;
    S->cancelled += 1;
  } else {
    j->state = LAYOUT_JOB_FAILED;
    j->err_code = code;
    j->error = msg;
    S->failed += 1;
  }
  S->cv_done.notify_all();
}

// Jobs of class c that can join its next launch: admitted, in no launch,
// not cancelled and not done.  Arrival order (the order of `active`).
std::vector<Job*> ready_jobs(layout_server_t* S, int c) {
  std::vector<Job*> v;
  for (Job* j : S->active)
    if (j->cls == c && !j->in_flight && !j->cancel.load() && j->nnz > 0 && j->t < j->epochs)
      v.push_back(j);
  return v;
}

// LDS class: every job runs up to kLdsLaunchEpochs of its remaining epochs in
// one workgroup, so that a job arriving meanwhile waits for at most that many
// epochs of the largest LDS job, not for all of them.
int start_lds(layout_server_t* S, ClassLaunch& L, const std::vector<Job*>& jobs) {
  const int k = jobs.front()->k;
  L.table.clear();
  L.ids.clear();
  int max_lds = 8, block = 64;
  for (Job* j : jobs) {
    GraphDesc d = j->desc;
    d.n_chunks = j->n_chunks;
    d.t0 = j->t;
    L.ids.push_back(static_cast<int32_t>(L.table.size()));
    L.table.push_back(d);
    max_lds = std::max(max_lds, lds_bytes_for(j->n));
    block = std::max(block, j->lanes);
  }
  hipError_t e = hipMemcpyAsync(S->d_table_lds, L.table.data(), sizeof(GraphDesc) * L.table.size(),
                                hipMemcpyHostToDevice, L.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(S->d_ids, L.ids.data(), sizeof(int32_t) * L.ids.size(),
                       hipMemcpyHostToDevice, L.stream);
  if (e != hipSuccess) return hip_fail(e, "uploading the LDS table");
  int rc = allow_lds(k, max_lds);
  if (rc != LAYOUT_OK) return rc;
  LdsGroup lg;
  lg.d_table = S->d_table_lds;
  lg.d_ids = S->d_ids;
  lg.blocks = static_cast<int>(L.table.size());
  lg.lds_bytes = max_lds;
  lg.k = k;
  lg.mode = S->mode_lds;
  lg.degree = S->opts.neg_weights != LAYOUT_NEG_UNIFORM;
  lg.block = block;
  // one launch for all: each workgroup stops at its own job's last epoch
  int32_t count = 0;
  L.slice.clear();
  for (Job* j : jobs) {
    const int32_t c = std::min<int32_t>(kLdsLaunchEpochs, j->epochs - j->t);
    L.slice.push_back(c);
    count = std::max(count, c);
  }
  rc = launch_lds_epochs(L.stream, lg, 0, count);
  L.jobs = jobs;
  return rc;
}

// A slice of the current epoch for each job: the launch's edge budget shared
// in proportion to the jobs' sizes, so that every job advances the same
// fraction of an epoch per launch (large jobs are not starved by many small
// ones).
void take_slices(layout_server_t* S, ClassLaunch& L, const std::vector<Job*>& jobs,
                 std::vector<GraphDesc>& out) {
  double total_nnz = 0.0;
  for (Job* j : jobs) total_nnz += double(j->nnz);
  L.jobs = jobs;
  L.slice.clear();
  out.clear();
  for (Job* j : jobs) {
    const int64_t share = std::max<int64_t>(
        kMinSliceEdges,
        int64_t(double(S->round_edges) * double(j->nnz) / std::max(1.0, total_nnz)));
    const double edges_per_chunk = double(j->nnz) / double(std::max<int64_t>(1, j->n_chunks));
    const int64_t want = std::max<int64_t>(1, int64_t(double(share) / edges_per_chunk));
    const int64_t slice = std::min(want, j->n_chunks - j->chunk_pos);
    L.slice.push_back(slice);
    GraphDesc d = j->desc;
    d.t0 = j->t;
    d.chunk_offset = j->chunk_pos;
    d.n_chunks = slice;
    out.push_back(d);
  }
}

// XCD class: the jobs' slices on XCD-local bins, one launch.
int start_xcd(layout_server_t* S, ClassLaunch& L, const std::vector<Job*>& jobs) {
  std::vector<GraphDesc> gx;
  take_slices(S, L, jobs, gx);
  L.table.clear();
  L.segs.clear();
  XcdGroup xg;
  xg.grid = plan_xcd_bins(gx, S->opts.nodes_per_lane, L.table, L.segs, L.bins);
  xg.d_table = S->d_table_xcd;
  xg.d_segs = S->d_segs;
  xg.d_bins = S->d_bins;
  xg.d_counters = S->d_xcd_ctr;
  xg.n_segs = static_cast<int32_t>(L.segs.size());
  xg.k = jobs.front()->k;
  xg.degree = S->opts.neg_weights != LAYOUT_NEG_UNIFORM;
  for (const GraphDesc& d : gx) xg.total_chunks += d.n_chunks;
  hipError_t e = hipMemcpyAsync(S->d_table_xcd, L.table.data(), sizeof(GraphDesc) * L.table.size(),
                                hipMemcpyHostToDevice, L.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(S->d_segs, L.segs.data(), sizeof(XcdSeg) * L.segs.size(),
                       hipMemcpyHostToDevice, L.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(S->d_bins, L.bins, sizeof(XcdBin) * kXcds, hipMemcpyHostToDevice, L.stream);
  if (e != hipSuccess) return hip_fail(e, "uploading the XCD bins");
  launch_fill_i32(L.stream, S->d_xcd_ctr, xg.n_segs, 0);
  return launch_xcd_group_epochs(L.stream, xg, 0, 1);
}

// All-CU class.  The jobs take turns in arrival order: a launch runs the
// oldest ones whose lane caps (n / nodes_per_lane each, the concurrency a job
// has alone) fit the device's lanes together, plus any later one that still
// fits, so that each runs at the speed it has alone instead of all of them
// sharing the device and all finishing late.  The others keep their device
// state and wait.
int start_wide(layout_server_t* S, ClassLaunch& L, const std::vector<Job*>& ready) {
  const int npl = S->opts.nodes_per_lane > 0 ? S->opts.nodes_per_lane : kNodesPerLane;
  const int64_t device_lanes = int64_t(device_props().cus) * kLanesPerCU;
  std::vector<Job*> jobs;
  int64_t used = 0;
  for (Job* j : ready) {
    const int64_t cap = std::max<int64_t>(64, j->n / npl);
    if (!jobs.empty() && used + cap > device_lanes) continue;
    used += cap;
    jobs.push_back(j);
  }
  std::vector<GraphDesc>& gt = L.table;
  take_slices(S, L, jobs, gt);
  GlobalGroup gg;
  gg.d_table = S->d_table;
  gg.G = static_cast<int>(gt.size());
  for (const GraphDesc& d : gt) gg.total_chunks += d.n_chunks;
  gg.k = jobs.front()->k;
  gg.mode = S->mode_global;
  gg.degree = S->opts.neg_weights != LAYOUT_NEG_UNIFORM;
  gg.block = S->opts.block_threads && S->opts.block_threads <= 256 ? S->opts.block_threads : 256;
  gg.grid = S->opts.grid_blocks;
  gg.max_lanes = lane_caps(gt, S->opts.nodes_per_lane);
  if (!S->opts.block_threads)  // small lane caps get small workgroups
    gg.block = static_cast<int>(std::min<int64_t>(
        256, std::max<int64_t>(64, div_up(std::max<int64_t>(1, gg.max_lanes), 64) * 64)));
  const int grid = global_grid(gg);
  plan_lanes(gt, gg, int64_t(grid) * gg.block, S->opts.nodes_per_lane);
  gg.grid = static_cast<int>(std::max<int64_t>(grid, div_up(gg.total_index, gg.block)));
  hipError_t e = hipMemcpyAsync(S->d_table, gt.data(), sizeof(GraphDesc) * gt.size(),
                                hipMemcpyHostToDevice, L.stream);
  if (e != hipSuccess) return hip_fail(e, "uploading the launch table");
  const int rc = launch_global_epochs(L.stream, gg, 0, 1);
  if (rc != LAYOUT_OK) return rc;
  // JACOBI: a job whose epoch ends in this launch moves by its summed D
  if (S->mode_global == LAYOUT_JACOBI)
    for (size_t q = 0; q < jobs.size(); ++q)
      if (jobs[q]->chunk_pos + L.slice[q] >= jobs[q]->n_chunks)
        launch_jacobi_apply(L.stream, jobs[q]->desc.Y, jobs[q]->D, jobs[q]->n);
  return LAYOUT_OK;
}

int start_class(layout_server_t* S, int c, const std::vector<Job*>& jobs) {
  ClassLaunch& L = S->cls[c];
  const int rc = c == kClassLds   ? start_lds(S, L, jobs)
                 : c == kClassXcd ? start_xcd(S, L, jobs)
                                  : start_wide(S, L, jobs);
  if (rc != LAYOUT_OK) return rc;
  const hipError_t e = hipEventRecord(L.done, L.stream);
  if (e != hipSuccess) return hip_fail(e, "recording a launch");
  for (Job* j : L.jobs) j->in_flight = true;
  L.busy = true;
  return LAYOUT_OK;
}

// Book-keeping once a class's launch has ended: epoch counters advance.
void end_class(layout_server_t* S, ClassLaunch& L) {
  for (size_t q = 0; q < L.jobs.size(); ++q) {
    Job* j = L.jobs[q];
    j->in_flight = false;
    if (j->cls == kClassLds) {
      j->t += static_cast<int32_t>(L.slice[q]);  // epochs run in this launch
      continue;
    }
    j->chunk_pos += L.slice[q];
    if (j->chunk_pos >= j->n_chunks) {
      j->chunk_pos = 0;
      j->t += 1;
    }
  }
  L.jobs.clear();
  L.busy = false;
  std::lock_guard<std::mutex> lk(S->mu);
  S->rounds += 1;
}

// Retires the jobs in no launch that are done (positions to host, device
// memory freed) or cancelled.
int retire_jobs(layout_server_t* S) {
  std::vector<Job*> still;
  int rc = LAYOUT_OK;
  for (Job* j : S->active) {
    if (j->in_flight || rc != LAYOUT_OK) {
      still.push_back(j);
      continue;
    }
    if (j->cancel.load()) {
      finish_job(S, j, kCancelled, "cancelled");
      continue;
    }
    if (j->t < j->epochs && j->nnz > 0) {
      still.push_back(j);
      continue;
    }
    j->result.resize(size_t(j->n) * 2);
    hipError_t e = hipSuccess;
    if (j->n > 0) {
      e = hipMemcpyAsync(j->result.data(), j->desc.Y, sizeof(float2) * size_t(j->n),
                         hipMemcpyDeviceToHost, S->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    }
    if (e != hipSuccess) {
      rc = hip_fail(e, "reading positions");
      still.push_back(j);
      continue;
    }
    finish_job(S, j, LAYOUT_OK, "");
  }
  S->active.swap(still);
  return rc;
}

// Answers the pending draw requests of jobs whose device state is set up
// (scheduler thread); requests of queued jobs wait for their admission, and
// those of jobs that ended before it are refused.
void serve_draw_requests(layout_server_t* S) {
  std::vector<DrawRequest*> todo;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    for (DrawRequest* r : S->draw_requests) todo.push_back(r);
  }
  if (todo.empty()) return;
  std::vector<DrawRequest*> answered;
  for (DrawRequest* r : todo) {
    Job* j = nullptr;
    for (Job* a : S->active)
      if (a->id == r->job) j = a;
    if (!j) {
      std::lock_guard<std::mutex> lk(S->mu);
      auto it = S->jobs.find(r->job);
      const bool waiting = it != S->jobs.end() && it->second->state == LAYOUT_JOB_QUEUED;
      if (waiting) continue;
      r->rc = LAYOUT_E_DONE;
      r->msg = "the job is no longer on the device";
      answered.push_back(r);
      continue;
    }
    g_last_error.clear();
    const size_t count = size_t(j->nnz) * size_t(j->k);
    int32_t* d_out = nullptr;
    int rc = LAYOUT_OK;
    if (count > 0) {
      hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&d_out), sizeof(int32_t) * count,
                                    S->stream);
      if (e != hipSuccess) rc = hip_fail(e, "debug draws buffer");
      if (rc == LAYOUT_OK)
        rc = launch_dump_draws(S->stream, j->k, S->opts.neg_weights != LAYOUT_NEG_UNIFORM,
                               j->desc, r->epoch, d_out);
      if (rc == LAYOUT_OK) {
        e = hipMemcpyAsync(r->out, d_out, sizeof(int32_t) * count, hipMemcpyDeviceToHost,
                           S->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
        if (e != hipSuccess) rc = hip_fail(e, "reading debug draws");
      }
      if (d_out) (void)hipFreeAsync(d_out, S->stream);
    }
    r->rc = rc;
    r->msg = g_last_error;
    answered.push_back(r);
  }
  std::lock_guard<std::mutex> lk(S->mu);
  for (DrawRequest* r : answered) {
    r->done = true;
    S->draw_requests.erase(std::find(S->draw_requests.begin(), S->draw_requests.end(), r));
  }
  if (!answered.empty()) S->cv_done.notify_all();
}

bool admissible(const layout_server_t* S) {  // under mu
  return !S->queue.empty() && int64_t(S->active.size()) < int64_t(S->max_slots) &&
         S->in_use + S->queue.front()->footprint <= S->budget;
}

void scheduler(layout_server_t* S) {
  (void)hipSetDevice(S->dev);
  double t_last = now_s();
  for (;;) {
    // launches that have ended, then the jobs that are done
    int rc = LAYOUT_OK;
    for (ClassLaunch& L : S->cls) {
      if (!L.busy || rc != LAYOUT_OK) continue;
      const hipError_t e = hipEventQuery(L.done);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) {
        rc = hip_fail(e, "running a launch");
        continue;
      }
      end_class(S, L);
    }
    if (rc == LAYOUT_OK) rc = retire_jobs(S);
    // admission in arrival order while a slot is free and the job's footprint
    // fits the budget
    std::vector<Job*> admit;
    bool held = false, busy = false;
    for (const ClassLaunch& L : S->cls) busy = busy || L.busy;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (S->stop || rc != LAYOUT_OK) {
        if (rc != LAYOUT_OK) {
          S->dead = true;
          S->dead_msg = g_last_error;
        }
        break;
      }
      while (!S->queue.empty() &&
             int64_t(S->active.size() + admit.size()) < int64_t(S->max_slots)) {
        Job* j = S->queue.front();
        if (S->in_use + j->footprint > S->budget) break;  // arrival order: wait for memory
        S->queue.pop_front();
        S->in_use += j->footprint;
        j->state = LAYOUT_JOB_RUNNING;
        admit.push_back(j);
      }
      held = S->hold;
      const double now = now_s();
      if (!S->active.empty() || busy) S->busy_seconds += now - t_last;
      t_last = now;
    }
    for (Job* j : admit) {
      if (j->cancel.load()) {
        finish_job(S, j, kCancelled, "cancelled");
        continue;
      }
      g_last_error.clear();
      rc = setup_job(S, *j);
      if (rc != LAYOUT_OK) {
        finish_job(S, j, rc, g_last_error);
        if (rc == LAYOUT_E_DEVICE) {
          std::lock_guard<std::mutex> lk(S->mu);
          S->dead = true;
          S->dead_msg = g_last_error;
        }
        continue;
      }
      S->active.push_back(j);
    }
    if (S->dead) break;
    serve_draw_requests(S);
    // every class whose last launch has ended starts its next one, whatever
    // the other classes are doing
    g_last_error.clear();
    rc = LAYOUT_OK;
    for (int c = 0; c < kClasses && !held && rc == LAYOUT_OK; ++c) {
      if (S->cls[c].busy) continue;
      const std::vector<Job*> jobs = ready_jobs(S, c);
      if (!jobs.empty()) rc = start_class(S, c, jobs);
    }
    if (rc != LAYOUT_OK) {
      std::lock_guard<std::mutex> lk(S->mu);
      S->dead = true;
      S->dead_msg = g_last_error;
      break;
    }
    busy = false;
    for (const ClassLaunch& L : S->cls) busy = busy || L.busy;
    if (busy) {
      // a launch is running: look again shortly (its end, new arrivals)
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      continue;
    }
    // nothing running: sleep until a submission, a request, the release or
    // the stop (polling slowly while held, since a request may wait for a
    // job queued behind full slots)
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_work.wait_for(lk, std::chrono::milliseconds(50), [&] {
      return S->stop || !S->draw_requests.empty() || admissible(S) ||
             (!S->hold && !S->active.empty());
    });
  }
  // drain: let every launch end (also those of a class whose start failed
  // part way), then fail whatever is left
  for (ClassLaunch& L : S->cls) (void)hipStreamSynchronize(L.stream);
  for (Job* j : S->active) finish_job(S, j, LAYOUT_E_DEVICE, S->dead ? S->dead_msg : "server stopped");
  S->active.clear();
  std::lock_guard<std::mutex> lk(S->mu);
  for (DrawRequest* r : S->draw_requests) {
    r->rc = LAYOUT_E_DEVICE;
    r->msg = S->dead ? S->dead_msg : "server stopped";
    r->done = true;
  }
  S->draw_requests.clear();
  for (Job* j : S->queue) {
    j->state = LAYOUT_JOB_FAILED;
    j->err_code = LAYOUT_E_DEVICE;
    j->error = S->dead ? S->dead_msg : "server stopped";
  }
  S->queue.clear();
  S->cv_done.notify_all();
}

}  // namespace

extern "C" {

int layout_server_create(int64_t hbm_budget_bytes, int32_t max_slots, int64_t round_edges,
                         const layout_opts* opts, layout_server_t** out) {
  g_last_error.clear();
  if (!out) return fail(LAYOUT_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || hbm_budget_bytes < 0 || round_edges < 0)
    return fail(LAYOUT_E_INVALID_ARG, "max_slots >= 1, budget >= 0, round_edges >= 0");
  layout_opts o;
  if (opts)
    o = *opts;
  else
    layout_opts_init(&o);
  if (o.update_mode < 0 || o.update_mode > 3)
    return fail(LAYOUT_E_INVALID_ARG, "update_mode = %d", o.update_mode);
  if (o.update_mode == LAYOUT_JACOBI && o.engine != LAYOUT_ENGINE_AUTO &&
      o.engine != LAYOUT_ENGINE_GLOBAL)
    return fail(LAYOUT_E_UNSUPPORTED, "JACOBI jobs run on the global engine only");
  if (o.neg_weights != LAYOUT_NEG_UNIFORM && o.neg_weights != LAYOUT_NEG_DEGREE &&
      o.neg_weights != LAYOUT_NEG_CUSTOM)
    return fail(LAYOUT_E_INVALID_ARG, "neg_weights = %d", o.neg_weights);
  if (o.engine < 0 || o.engine > 3) return fail(LAYOUT_E_INVALID_ARG, "engine = %d", o.engine);
  if (o.force_kernel != LAYOUT_FORCE_T && o.force_kernel != LAYOUT_FORCE_GAUSSIAN)
    return fail(LAYOUT_E_INVALID_ARG, "force_kernel = %d", o.force_kernel);
  if (!(o.gamma > (o.force_kernel == LAYOUT_FORCE_T ? 1.0f : 0.0f)))
    return fail(LAYOUT_E_INVALID_ARG, "gamma = %g", o.gamma);
  if (o.init_mode != LAYOUT_INIT_UNIFORM && o.init_mode != LAYOUT_INIT_PMDS)
    return fail(LAYOUT_E_INVALID_ARG, "init_mode = %d", o.init_mode);
  if (o.pmds_pivots < 0 || o.pmds_pivots > 64)
    return fail(LAYOUT_E_INVALID_ARG, "pmds_pivots = %d (1..64, 0 = default)", o.pmds_pivots);
  if (o.block_threads < 0 || o.block_threads > 1024 || (o.block_threads % 64) != 0 ||
      o.bundle_edges < 0 || o.hub_split_edges < 0 || o.grid_blocks < 0 || o.nodes_per_lane < 0)
    return fail(LAYOUT_E_INVALID_ARG, "bad launch option");
  layout_server_t* S = new (std::nothrow) layout_server_t();
  if (!S) return fail(LAYOUT_E_OOM, "host allocation");
  S->opts = o;
  S->mode_global = o.update_mode == LAYOUT_UPDATE_AUTO ? LAYOUT_HOGWILD_STORE : o.update_mode;
  S->xcd_ok = S->mode_global == LAYOUT_HOGWILD_STORE &&
              (o.engine == LAYOUT_ENGINE_AUTO || o.engine == LAYOUT_ENGINE_XCD) &&
              o.grid_blocks == 0 && o.block_threads == 0;
  S->mode_lds = o.update_mode == LAYOUT_UPDATE_AUTO ? LAYOUT_ATOMIC : o.update_mode;
  S->max_slots = max_slots;
  S->round_edges = round_edges ? round_edges : kDefaultRoundEdges;
  (void)hipGetDevice(&S->dev);
  // the LDS engine has no Jacobi mode: JACOBI servers run every job globally
  S->lds_cap = (o.engine == LAYOUT_ENGINE_GLOBAL || o.update_mode == LAYOUT_JACOBI)
                   ? 0
                   : device_props().lds_per_block;
  hipError_t e = hipSuccess;
  if (hbm_budget_bytes == 0) {
    size_t free_b = 0, total_b = 0;
    e = hipMemGetInfo(&free_b, &total_b);
    S->budget = int64_t(double(free_b) * 0.9);
  } else {
    S->budget = hbm_budget_bytes;
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
  for (ClassLaunch& L : S->cls) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipMalloc(&S->d_table, sizeof(GraphDesc) * size_t(max_slots));
  if (e == hipSuccess) e = hipMalloc(&S->d_table_lds, sizeof(GraphDesc) * size_t(max_slots));
  if (e == hipSuccess) e = hipMalloc(&S->d_ids, sizeof(int32_t) * size_t(max_slots));
  if (e == hipSuccess) e = hipMalloc(&S->d_table_xcd, sizeof(GraphDesc) * size_t(max_slots));
  if (e == hipSuccess) e = hipMalloc(&S->d_segs, sizeof(XcdSeg) * size_t(max_slots));
  if (e == hipSuccess) e = hipMalloc(&S->d_bins, sizeof(XcdBin) * kXcds);
  if (e == hipSuccess) e = hipMalloc(&S->d_xcd_ctr, sizeof(int32_t) * size_t(max_slots));
  if (e == hipSuccess) e = hipMalloc(&S->d_err, sizeof(uint32_t));
  if (e != hipSuccess) {
    const int rc = hip_fail(e, "server setup");
    layout_server_destroy(S);
    return rc;
  }
  S->thr = std::thread(scheduler, S);
  *out = S;
  return LAYOUT_OK;
}

int layout_server_submit_ex(layout_server_t* S, const int32_t* row_ptr, const int32_t* col_idx,
                            int32_t n, int32_t k, int32_t epochs, uint64_t seed,
                            const uint32_t* neg_weight_values, const float* init_pos,
                            int64_t* job_id) {
  g_last_error.clear();
  if (!S || !job_id || !row_ptr || n < 0)
    return fail(LAYOUT_E_INVALID_ARG, "NULL server/job_id/row_ptr or n < 0");
  if (k < 0 || k > 8) return fail(k < 0 ? LAYOUT_E_INVALID_ARG : LAYOUT_E_UNSUPPORTED, "k = %d", k);
  if (epochs < 1) return fail(LAYOUT_E_INVALID_ARG, "epochs = %d", epochs);
  const int32_t nnz = row_ptr[n];
  if (nnz < 0 || (nnz > 0 && !col_idx)) return fail(LAYOUT_E_INVALID_ARG, "bad row_ptr[n] or col");
  const bool custom = S->opts.neg_weights == LAYOUT_NEG_CUSTOM;
  if ((neg_weight_values != nullptr) != (custom && n > 0))
    return fail(LAYOUT_E_INVALID_ARG,
                "neg_weight_values must be given exactly when the server uses LAYOUT_NEG_CUSTOM");
  if (custom && n > 0) {
    int64_t W = 0;
    for (int32_t v = 0; v < n; ++v) W += neg_weight_values[v];
    if (W <= 0 || W >= (int64_t(1) << 32))
      return fail(LAYOUT_E_INVALID_ARG, "negative weights sum to %lld (need 0 < W < 2^32)",
                  (long long)W);
  }
  Job* j = new (std::nothrow) Job();
  if (!j) return fail(LAYOUT_E_OOM, "host allocation");
  j->n = n;
  j->k = k;
  j->epochs = epochs;
  j->seed = seed;
  j->nnz = nnz;
  j->row.assign(row_ptr, row_ptr + n + 1);
  if (nnz > 0) j->col.assign(col_idx, col_idx + nnz);
  if (custom && n > 0) j->weights.assign(neg_weight_values, neg_weight_values + n);
  if (init_pos && n > 0) j->init.assign(init_pos, init_pos + 2 * size_t(n));
  j->t_submit = now_s();
  plan_job(S, *j);
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->dead) {
    delete j;
    return fail(LAYOUT_E_DEVICE, "server stopped: %s", S->dead_msg.c_str());
  }
  if (j->footprint > S->budget) {
    S->rejected += 1;
    const int64_t fp = j->footprint;
    delete j;
    return fail(LAYOUT_E_OOM, "job needs %lld bytes, budget is %lld", (long long)fp,
                (long long)S->budget);
  }
  // the jobs of one server share k (one kernel instantiation per launch)
  for (auto& kv : S->jobs)
    if (kv.second->k != k && kv.second->state <= LAYOUT_JOB_RUNNING) {
      delete j;
      return fail(LAYOUT_E_UNSUPPORTED, "jobs in flight use k = %d", kv.second->k);
    }
  j->id = S->next_id++;
  S->jobs[j->id] = j;
  S->queue.push_back(j);
  S->submitted += 1;
  *job_id = j->id;
  S->cv_work.notify_one();
  return LAYOUT_OK;
}

int layout_server_submit(layout_server_t* S, const int32_t* row_ptr, const int32_t* col_idx,
                         int32_t n, int32_t k, int32_t epochs, uint64_t seed, int64_t* job_id) {
  return layout_server_submit_ex(S, row_ptr, col_idx, n, k, epochs, seed, nullptr, nullptr,
                                 job_id);
}

int layout_server_cancel(layout_server_t* S, int64_t job_id) {
  if (!S) return fail(LAYOUT_E_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(job_id);
  if (it == S->jobs.end()) return fail(LAYOUT_E_INVALID_ARG, "unknown job %lld", (long long)job_id);
  Job* j = it->second;
  if (j->state == LAYOUT_JOB_QUEUED) {
    auto q = std::find(S->queue.begin(), S->queue.end(), j);
    if (q != S->queue.end()) S->queue.erase(q);
    j->state = LAYOUT_JOB_CANCELLED;
    j->t_done = now_s();
    S->cancelled += 1;
    S->cv_done.notify_all();
    S->cv_work.notify_one();  // a slot may admit the next job
    return LAYOUT_OK;
  }
  if (j->state == LAYOUT_JOB_RUNNING) {
    j->cancel.store(true);  // retired once its launch in flight has ended
    return LAYOUT_OK;
  }
  return fail(LAYOUT_E_INVALID_ARG, "job %lld has already ended", (long long)job_id);
}

int layout_server_hold(layout_server_t* S, int32_t hold) {
  if (!S) return fail(LAYOUT_E_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(S->mu);
  S->hold = hold != 0;
  S->cv_work.notify_all();
  return LAYOUT_OK;
}

int layout_server_debug_draws(layout_server_t* S, int64_t job_id, int32_t epoch,
                              int32_t* host_out) {
  if (!S) return fail(LAYOUT_E_INVALID_ARG, "NULL server");
  if (epoch < 0) return fail(LAYOUT_E_INVALID_ARG, "epoch = %d", epoch);
  DrawRequest r;
  r.job = job_id;
  r.epoch = epoch;
  r.out = host_out;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->jobs.find(job_id);
  if (it == S->jobs.end()) return fail(LAYOUT_E_INVALID_ARG, "unknown job %lld", (long long)job_id);
  Job* j = it->second;
  if (j->state != LAYOUT_JOB_QUEUED && j->state != LAYOUT_JOB_RUNNING)
    return fail(LAYOUT_E_DONE, "job %lld is no longer on the device", (long long)job_id);
  if (j->nnz > 0 && j->k > 0 && !host_out) return fail(LAYOUT_E_INVALID_ARG, "host_out is NULL");
  if (S->dead) return fail(LAYOUT_E_DEVICE, "server stopped: %s", S->dead_msg.c_str());
  S->draw_requests.push_back(&r);
  S->cv_work.notify_all();
  S->cv_done.wait(lk, [&] { return r.done; });
  if (r.rc != LAYOUT_OK) return fail(r.rc, "%s", r.msg.c_str());
  return LAYOUT_OK;
}

int layout_server_poll(layout_server_t* S, int64_t job_id, int32_t* state) {
  if (!S || !state) return fail(LAYOUT_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(job_id);
  if (it == S->jobs.end()) return fail(LAYOUT_E_INVALID_ARG, "unknown job %lld", (long long)job_id);
  *state = it->second->state;
  return LAYOUT_OK;
}

int layout_server_wait(layout_server_t* S, int64_t job_id, double timeout_s) {
  if (!S) return fail(LAYOUT_E_INVALID_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->jobs.find(job_id);
  if (it == S->jobs.end()) return fail(LAYOUT_E_INVALID_ARG, "unknown job %lld", (long long)job_id);
  Job* j = it->second;
  auto done = [&] {
    return j->state == LAYOUT_JOB_DONE || j->state == LAYOUT_JOB_FAILED ||
           j->state == LAYOUT_JOB_CANCELLED;
  };
  if (timeout_s < 0) {
    S->cv_done.wait(lk, done);
  } else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
    return fail(LAYOUT_E_INVALID_ARG, "timeout waiting for job %lld", (long long)job_id);
  }
  if (j->state == LAYOUT_JOB_FAILED) return fail(j->err_code, "%s", j->error.c_str());
  if (j->state == LAYOUT_JOB_CANCELLED)
    return fail(LAYOUT_E_INVALID_ARG, "job %lld was cancelled", (long long)job_id);
  return LAYOUT_OK;
}

int layout_server_take(layout_server_t* S, int64_t job_id, float* host_out, double* latency_s) {
  if (!S) return fail(LAYOUT_E_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(job_id);
  if (it == S->jobs.end()) return fail(LAYOUT_E_INVALID_ARG, "unknown job %lld", (long long)job_id);
  Job* j = it->second;
  if (j->state == LAYOUT_JOB_FAILED) {
    const int code = j->err_code;
    const std::string msg = j->error;
    S->jobs.erase(it);
    delete j;
    return fail(code, "%s", msg.c_str());
  }
  if (j->state == LAYOUT_JOB_CANCELLED) {
    S->jobs.erase(it);
    delete j;
    return fail(LAYOUT_E_INVALID_ARG, "job %lld was cancelled", (long long)job_id);
  }
  if (j->state != LAYOUT_JOB_DONE) return fail(LAYOUT_E_INVALID_ARG, "job not done");
  if (host_out && !j->result.empty())
    std::memcpy(host_out, j->result.data(), sizeof(float) * j->result.size());
  if (latency_s) *latency_s = j->t_done - j->t_submit;
  S->jobs.erase(it);
  delete j;
  return LAYOUT_OK;
}

int layout_server_get_stats(layout_server_t* S, layout_server_stats* st) {
  if (!S || !st) return fail(LAYOUT_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  std::memset(st, 0, sizeof *st);
  st->submitted = S->submitted;
  st->completed = S->completed;
  st->failed = S->failed;
  st->rejected = S->rejected;
  st->cancelled = S->cancelled;
  st->queued = int64_t(S->queue.size());
  int64_t running = 0;
  for (auto& kv : S->jobs) running += kv.second->state == LAYOUT_JOB_RUNNING ? 1 : 0;
  st->running = running;
  st->hbm_in_use = S->in_use;
  st->hbm_budget = S->budget;
  st->rounds = S->rounds;
  st->edge_updates = S->edge_updates;
  st->busy_seconds = S->busy_seconds;
  if (!S->latencies.empty()) {
    std::vector<double> l = S->latencies;
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {
      const double pos = p * double(l.size() - 1);
      const size_t lo = size_t(std::floor(pos)), hi = size_t(std::ceil(pos));
      return l[lo] + (l[hi] - l[lo]) * (pos - double(lo));
    };
    st->p50_latency_s = pct(0.50);
    st->p99_latency_s = pct(0.99);
    double sum = 0;
    for (double x : l) sum += x;
    st->mean_latency_s = sum / double(l.size());
  }
  return LAYOUT_OK;
}

int layout_server_destroy(layout_server_t* S) {
  if (!S) return LAYOUT_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->thr.joinable()) S->thr.join();
  for (auto& kv : S->jobs) {
    kv.second->buf.free_all_async(S->stream);
    delete kv.second;
  }
  S->jobs.clear();
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  if (S->d_table) (void)hipFree(S->d_table);
  if (S->d_table_lds) (void)hipFree(S->d_table_lds);
  if (S->d_ids) (void)hipFree(S->d_ids);
  if (S->d_table_xcd) (void)hipFree(S->d_table_xcd);
  if (S->d_segs) (void)hipFree(S->d_segs);
  if (S->d_bins) (void)hipFree(S->d_bins);
  if (S->d_xcd_ctr) (void)hipFree(S->d_xcd_ctr);
  if (S->d_err) (void)hipFree(S->d_err);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  for (ClassLaunch& L : S->cls) {
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.stream) (void)hipStreamDestroy(L.stream);
  }
  delete S;
  return LAYOUT_OK;
}

}  // extern "C"
