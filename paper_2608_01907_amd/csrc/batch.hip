// Batched layout of many graphs (the layout_batch_* entry points of
// include/snaplayout.h).
//
// Memory: one packed allocation per array kind -- row pointers (each graph's
// n_g + 1 entries, local indices), columns, positions, chunk tables -- and
// one GraphDesc per graph pointing into it.  Graphs are split into two groups:
//   LDS group:    n_g * 8 B fits one workgroup's LDS; one workgroup per graph
//                 runs every epoch (epoch_lds_kernel).
//   global group: one launch per epoch over the chunks of all its graphs
//                 (epoch_global_kernel with a multi-graph table), or, when
//                 every such graph's positions fit one XCD's L2, the
//                 XCD-local engine: the graphs are split into one bin per XCD
//                 and each XCD runs its bin with plain loads and stores
//                 (epoch_xcd_group_kernel).
// Both groups' epochs are captured once in a HIP graph (two branches forked
// from the batch stream) and replayed by layout_batch_run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "common.hpp"
#include "snaplayout.h"

using namespace snap;

struct layout_batch {
  int32_t count = 0, k = 0, epochs = 0;
  bool ran = false;
  layout_opts opts{};
  int32_t mode_global = LAYOUT_HOGWILD_STORE, mode_lds = LAYOUT_ATOMIC;
  int32_t bundle = kDefaultBundle, hub = kDefaultBundle * kHubFactor;
  int32_t blocks_per_cu = 0;  // 0 = occupancy limit
  hipStream_t stream = nullptr, side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  DeviceBuffers buf;
  // per graph
  std::vector<int32_t> n, lds_block, lds_bundle, lds_hub;
  std::vector<int64_t> nnz, node_off, edge_off, row_off, chunk_off, chunk_cap;
  std::vector<uint8_t> in_lds;
  std::vector<GraphDesc> desc;  // by graph index
  // packed device arrays
  int64_t* d_row = nullptr;
  int32_t* d_col = nullptr;
  float2* d_Y = nullptr;
  float2* d_D = nullptr;
  int64_t* d_chunk_begin = nullptr;
  int32_t* d_chunk_src = nullptr;
  uint32_t* d_thr = nullptr;
  uint32_t* d_alias = nullptr;
  uint32_t* d_err = nullptr;
  // groups
  GraphDesc* d_table_global = nullptr;
  GraphDesc* d_table_lds = nullptr;
  int32_t* d_lds_ids = nullptr;
  std::vector<int32_t> global_ids, lds_ids;
  GlobalGroup gg;
  LdsGroup lg;
  // XCD-local engine for the global group
  bool xcd_mode = false;
  XcdGroup xg;
  GraphDesc* d_table_xcd = nullptr;
  XcdSeg* d_segs = nullptr;
  XcdBin* d_bins = nullptr;
  int32_t* d_xcd_counters = nullptr;  // [epochs][segments], segments <= graphs
  XcdBin bins[kXcds] = {};
  int64_t nodes = 0, total_nnz = 0;
};

namespace {

int balloc(layout_batch_t* B, void** p, size_t bytes, const char* what) {
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return hip_fail(e, what);
  B->buf.add(*p, bytes);
  return LAYOUT_OK;
}

bool check_batch(const layout_batch_t* B) {
  if (!B) {
    fail(LAYOUT_E_INVALID_ARG, "null batch handle");
    return false;
  }
  return true;
}

// Chunk tables of the global group for the batch's (bundle, hub).
int build_global_chunks(layout_batch_t* B) {
  int64_t total = 0;
  for (int32_t g : B->global_ids) {
    if (B->nnz[g] == 0) continue;  // nothing moves; keeps chunk_base strictly useful
    GraphDesc& d = B->desc[g];
    const int64_t cap = chunk_bound(B->nnz[g], B->bundle, B->hub);
    if (cap > B->chunk_cap[g])
      return fail(LAYOUT_E_UNSUPPORTED, "chunk table capacity (internal)");
    int64_t nc = 0;
    if (B->nnz[g] > 0) {
      const int rc = build_chunk_table(B->stream, d.row_ptr, B->n[g], B->nnz[g], B->bundle, B->hub,
                                       const_cast<int64_t*>(d.chunk_begin),
                                       const_cast<int32_t*>(d.chunk_src), &nc);
      if (rc != LAYOUT_OK) return rc;
    }
    d.n_chunks = nc;
    d.hub = B->hub;
    total += nc;
  }
  B->gg.total_chunks = total;
  std::vector<GraphDesc> table;
  for (int32_t g : B->global_ids)
    if (B->nnz[g] > 0) table.push_back(B->desc[g]);
  B->gg.max_lanes = table.empty() ? 0 : lane_caps(table, B->opts.nodes_per_lane);
  // small lane caps get small workgroups (whole wavefronts), as on one graph
  if (!B->opts.block_threads)
    B->gg.block = static_cast<int>(
        std::min<int64_t>(256, std::max<int64_t>(64, div_up(std::max<int64_t>(1, B->gg.max_lanes), 64) * 64)));
  return LAYOUT_OK;
}

// Round plan of the global group for a launch of `grid` workgroups, uploaded
// to the device table.
int upload_global_table(layout_batch_t* B, int grid) {
  std::vector<GraphDesc> table;
  for (int32_t g : B->global_ids)
    if (B->nnz[g] > 0) table.push_back(B->desc[g]);
  if (table.empty()) return LAYOUT_OK;
  plan_lanes(table, B->gg, int64_t(grid) * B->gg.block, B->opts.nodes_per_lane);
  // every graph keeps at least one lane: a launch too small for that grows
  if (B->gg.total_index > int64_t(grid) * B->gg.block)
    B->gg.grid = static_cast<int>(div_up(B->gg.total_index, B->gg.block));
  hipError_t e = hipMemcpyAsync(B->d_table_global, table.data(), sizeof(GraphDesc) * table.size(),
                                hipMemcpyHostToDevice, B->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
  if (e != hipSuccess) return hip_fail(e, "uploading the global table");
  return LAYOUT_OK;
}

// Bins and segments of the XCD-local engine for the current chunk tables,
// uploaded to the device.
int upload_xcd_table(layout_batch_t* B) {
  std::vector<GraphDesc> graphs, table;
  std::vector<XcdSeg> segs;
  for (int32_t g : B->global_ids)
    if (B->nnz[g] > 0) graphs.push_back(B->desc[g]);
  B->xg.total_chunks = B->gg.total_chunks;
  if (graphs.empty()) {
    B->xg.grid = 0;
    return LAYOUT_OK;
  }
  B->xg.grid = plan_xcd_bins(graphs, B->opts.nodes_per_lane, table, segs, B->bins);
  B->xg.n_segs = static_cast<int32_t>(segs.size());
  hipError_t e = hipMemcpyAsync(B->d_table_xcd, table.data(), sizeof(GraphDesc) * table.size(),
                                hipMemcpyHostToDevice, B->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(B->d_segs, segs.data(), sizeof(XcdSeg) * segs.size(),
                       hipMemcpyHostToDevice, B->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(B->d_bins, B->bins, sizeof(XcdBin) * kXcds, hipMemcpyHostToDevice,
                       B->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
  if (e != hipSuccess) return hip_fail(e, "uploading the XCD bins");
  return LAYOUT_OK;
}

int capture(layout_batch_t* B) {
  if (B->exec) {
    (void)hipGraphExecDestroy(B->exec);
    B->exec = nullptr;
  }
  if (B->graph) {
    (void)hipGraphDestroy(B->graph);
    B->graph = nullptr;
  }
  B->gg.grid = B->blocks_per_cu > 0 ? 0 : B->opts.grid_blocks;
  if (B->blocks_per_cu > 0) {
    GlobalGroup probe = B->gg;
    probe.grid = 0;
    const int occ_grid = global_grid(probe);
    B->gg.grid = std::min<int>(occ_grid, B->blocks_per_cu * device_props().cus);
  }
  if (B->gg.total_chunks > 0) {
    GlobalGroup probe = B->gg;
    const int rc = B->xcd_mode ? upload_xcd_table(B) : upload_global_table(B, global_grid(probe));
    if (rc != LAYOUT_OK) return rc;
  }
  hipError_t e = hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  int rc = LAYOUT_OK;
  e = hipEventRecord(B->fork, B->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(B->side, B->fork, 0);
  if (e == hipSuccess) rc = launch_lds_epochs(B->side, B->lg, 0, B->epochs);
  if (e == hipSuccess && rc == LAYOUT_OK) {
    if (B->xcd_mode) {
      // counters start at zero on every replay (a fill kernel: no memset node)
      launch_fill_i32(B->stream, B->d_xcd_counters, int64_t(B->epochs) * B->count, 0);
      rc = launch_xcd_group_epochs(B->stream, B->xg, 0, B->epochs);
    } else {
      rc = launch_global_epochs(B->stream, B->gg, 0, B->epochs);
    }
  }
  if (e == hipSuccess) e = hipEventRecord(B->join, B->side);
  if (e == hipSuccess) e = hipStreamWaitEvent(B->stream, B->join, 0);
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(B->stream, &graph);
  if (e == hipSuccess) e = e2;
  if (rc != LAYOUT_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "capturing the batch epochs");
  B->graph = graph;
  e = hipGraphInstantiate(&B->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  return LAYOUT_OK;
}

// Size class of the global group for the tuning cache: log2 of the directed
// edges and of the mean degree.
std::string tune_key(const layout_batch_t* B) {
  int64_t nodes = 0, nnz = 0;
  for (int32_t g : B->global_ids) {
    nodes += B->n[g];
    nnz += B->nnz[g];
  }
  hipDeviceProp_t prop{};
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipGetDeviceProperties(&prop, dev);
  const int le = nnz > 0 ? static_cast<int>(std::log2(static_cast<double>(nnz))) : 0;
  const int ld = nodes > 0 ? static_cast<int>(std::log2(std::max(1.0, double(nnz) / double(nodes))))
                           : 0;
  char key[256];
  snprintf(key, sizeof key, "%s|k%d|m%d|e%d|d%d|x%d", prop.gcnArchName, B->k, B->mode_global, le,
           ld, B->xcd_mode ? 1 : 0);
  for (char* c = key; *c; ++c)
    if (*c == ' ') *c = '_';
  return key;
}

bool cache_lookup(const char* path, const std::string& key, int* bundle, int* bpc, float* ms) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string k;
    int b = 0, p = 0;
    float t = 0.f;
    if (is >> k >> b >> p >> t && k == key && b > 0) {
      *bundle = b;
      *bpc = p;
      *ms = t;
      found = true;  // the last entry wins
    }
  }
  return found;
}

void cache_store(const char* path, const std::string& key, int bundle, int bpc, float ms) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << bundle << " " << bpc << " " << ms << "\n";
}

}  // namespace

namespace {

// Balance the two halves of a replay.  An LDS graph runs all its epochs on
// one CU, while the other graphs share the whole device epoch by epoch, so
// the LDS half lasts as long as its largest graph.  The largest LDS graphs
// move to the device-wide group while one of them alone would outlast it:
// nnz_g > X / kLdsBalance, with X the device-wide group's directed edges.
// kLdsBalance is the measured ratio of the device's edge rate on the XCD
// bins to one CU's on the LDS engine for the graphs the rule weighs (about
// 250 on MI355X at k = 5: 1.07e10 against 3.8e7 to 5.2e7 directed edges per
// second for 10k- to 18k-node power-law graphs, n / 32 lanes, hub rows
// split).  Graphs below kLdsKeepEdges stay
// in LDS, so a batch of small graphs keeps its one-launch replay.  Then, at
// most one LDS graph per CU: a second LDS workgroup on a CU waits for the
// first when their positions do not fit its LDS together, so the largest
// graphs beyond the CU count move as well.
constexpr double kLdsBalance = 250.0;
constexpr int64_t kLdsKeepEdges = 100000;

void balance_lds(const std::vector<int64_t>& nnz, std::vector<uint8_t>& in_lds, int cus) {
  std::vector<int32_t> cand;
  int64_t X = 0;
  for (size_t g = 0; g < nnz.size(); ++g) {
    if (in_lds[g])
      cand.push_back(static_cast<int32_t>(g));
    else
      X += nnz[g];
  }
  if (X == 0) return;
  std::sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) {
    return nnz[a] != nnz[b] ? nnz[a] > nnz[b] : a < b;
  });
  size_t moved = 0;
  for (int32_t g : cand) {
    if (nnz[g] < kLdsKeepEdges || double(nnz[g]) * kLdsBalance <= double(X)) break;
    in_lds[g] = 0;
    X += nnz[g];
    ++moved;
  }
  for (size_t q = moved; cus > 0 && cand.size() - q > size_t(cus); ++q) in_lds[cand[q]] = 0;
}

}  // namespace

extern "C" {

int layout_batch_create(const layout_graph* graphs, int32_t count, int32_t k, int32_t epochs,
                        const layout_opts* opts, int32_t inputs_on_device, layout_batch_t** out) {
  g_last_error.clear();
  if (!out) return fail(LAYOUT_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!graphs || count < 1) return fail(LAYOUT_E_INVALID_ARG, "need at least one graph");
  if (k < 0 || k > 8)
    return fail(k < 0 ? LAYOUT_E_INVALID_ARG : LAYOUT_E_UNSUPPORTED, "k = %d (0..8)", k);
  if (epochs < 1) return fail(LAYOUT_E_INVALID_ARG, "epochs = %d", epochs);
  layout_opts o;
  if (opts)
    o = *opts;
  else
    layout_opts_init(&o);
  if (o.update_mode < 0 || o.update_mode > 3)
    return fail(LAYOUT_E_INVALID_ARG, "update_mode = %d", o.update_mode);
  if (o.neg_weights != LAYOUT_NEG_UNIFORM && o.neg_weights != LAYOUT_NEG_DEGREE &&
      o.neg_weights != LAYOUT_NEG_CUSTOM)
    return fail(LAYOUT_E_INVALID_ARG, "neg_weights = %d", o.neg_weights);
  for (int32_t g = 0; g < count; ++g) {
    const bool has_w = graphs[g].neg_weight_values != nullptr;
    if (has_w != (o.neg_weights == LAYOUT_NEG_CUSTOM && graphs[g].n > 0))
      return fail(LAYOUT_E_INVALID_ARG,
                  "graph %d: neg_weight_values must be given exactly with LAYOUT_NEG_CUSTOM", g);
  }
  if (o.engine < 0 || o.engine > 3) return fail(LAYOUT_E_INVALID_ARG, "engine = %d", o.engine);
  if (o.bundle_edges < 0 || o.block_threads < 0 || o.grid_blocks < 0 || o.hub_split_edges < 0 ||
      o.nodes_per_lane < 0 || o.block_threads > 1024 || (o.block_threads % 64) != 0)
    return fail(LAYOUT_E_INVALID_ARG, "bad launch option");
  if (o.force_kernel != LAYOUT_FORCE_T && o.force_kernel != LAYOUT_FORCE_GAUSSIAN)
    return fail(LAYOUT_E_INVALID_ARG, "force_kernel = %d", o.force_kernel);
  if (!(o.gamma > (o.force_kernel == LAYOUT_FORCE_T ? 1.0f : 0.0f)))
    return fail(LAYOUT_E_INVALID_ARG, "gamma = %g (must be > 1, > 0 for Gaussian forces)",
                o.gamma);
  if (o.init_mode != LAYOUT_INIT_UNIFORM && o.init_mode != LAYOUT_INIT_PMDS)
    return fail(LAYOUT_E_INVALID_ARG, "init_mode = %d", o.init_mode);
  if (o.pmds_pivots < 0 || o.pmds_pivots > 64)
    return fail(LAYOUT_E_INVALID_ARG, "pmds_pivots = %d (1..64, 0 = default)", o.pmds_pivots);

  layout_batch_t* B = new (std::nothrow) layout_batch_t();
  if (!B) return fail(LAYOUT_E_OOM, "host allocation");
  auto bail = [&](int rc) {
    layout_batch_destroy(B);
    return rc;
  };
  B->count = count;
  B->k = k;
  B->epochs = epochs;
  B->opts = o;
  const bool jacobi = o.update_mode == LAYOUT_JACOBI;
  B->mode_global = o.update_mode == LAYOUT_UPDATE_AUTO ? LAYOUT_HOGWILD_STORE : o.update_mode;
  B->mode_lds = o.update_mode == LAYOUT_UPDATE_AUTO ? LAYOUT_ATOMIC : o.update_mode;
  B->bundle = o.bundle_edges ? o.bundle_edges : kDefaultBundle;
  B->hub = o.hub_split_edges ? o.hub_split_edges : kHubFactor * B->bundle;

  hipError_t e = hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&B->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&B->join, hipEventDisableTiming);
  if (e != hipSuccess) return bail(hip_fail(e, "creating streams"));

  // sizes and group membership
  const DeviceProps& dp = device_props();
  B->n.resize(count);
  B->nnz.resize(count);
  B->node_off.resize(count);
  B->edge_off.resize(count);
  B->row_off.resize(count);
  B->chunk_off.resize(count);
  B->chunk_cap.resize(count);
  B->in_lds.resize(count);
  B->lds_block.resize(count);
  B->lds_bundle.resize(count);
  B->lds_hub.resize(count);
  int64_t rows = 0, chunks = 0;
  int max_lds = 8;
  // sizes first, then the engine of every graph
  for (int32_t g = 0; g < count; ++g) {
    const layout_graph& gr = graphs[g];
    if (gr.n < 0 || !gr.row_ptr) return bail(fail(LAYOUT_E_INVALID_ARG, "graph %d: bad n/row_ptr", g));
    int32_t nnz = 0;
    if (inputs_on_device) {
      e = hipMemcpy(&nnz, gr.row_ptr + gr.n, sizeof nnz, hipMemcpyDeviceToHost);
      if (e != hipSuccess) return bail(hip_fail(e, "reading row_ptr[n]"));
    } else {
      nnz = gr.row_ptr[gr.n];
    }
    if (nnz < 0) return bail(fail(LAYOUT_E_BAD_GRAPH, "graph %d: row_ptr[n] = %d", g, nnz));
    if (nnz > 0 && !gr.col_idx) return bail(fail(LAYOUT_E_INVALID_ARG, "graph %d: col NULL", g));
    B->n[g] = gr.n;
    B->nnz[g] = nnz;
    const bool fits = lds_bytes_for(gr.n) <= dp.lds_per_block;
    bool lds = false;
    if (!jacobi) {
      if (o.engine == LAYOUT_ENGINE_LDS) {
        if (!fits) return bail(fail(LAYOUT_E_UNSUPPORTED, "graph %d does not fit LDS", g));
        lds = true;
      } else if (o.engine == LAYOUT_ENGINE_AUTO) {
        lds = fits;
      }
    }
    B->in_lds[g] = lds;
  }
  if (o.engine == LAYOUT_ENGINE_AUTO && !jacobi) balance_lds(B->nnz, B->in_lds, dp.cus);
  for (int32_t g = 0; g < count; ++g) {
    const layout_graph& gr = graphs[g];
    const int32_t nnz = static_cast<int32_t>(B->nnz[g]);
    B->node_off[g] = B->nodes;
    B->edge_off[g] = B->total_nnz;
    B->row_off[g] = rows;
    const bool lds = B->in_lds[g];
    int64_t cap;
    if (lds) {
      const int block = o.block_threads ? o.block_threads : lds_lanes_for(gr.n, o.nodes_per_lane);
      B->lds_block[g] = block;
      // one workgroup per graph: enough chunks for every lane, hub rows split
      B->lds_bundle[g] = o.bundle_edges ? o.bundle_edges
                                        : std::max(1, std::min(16, nnz / (4 * block)));
      B->lds_hub[g] = o.hub_split_edges ? o.hub_split_edges : kLdsHub;
      cap = nnz > 0 ? chunk_bound(nnz, B->lds_bundle[g], B->lds_hub[g]) : 0;
      max_lds = std::max(max_lds, lds_bytes_for(gr.n));
      B->lds_ids.push_back(g);
    } else {
      // room for every bundle size the autotuner may pick (8 is the smallest)
      cap = nnz > 0 ? std::max(chunk_bound(nnz, std::min(8, B->bundle), B->hub),
                               chunk_bound(nnz, 8, 8 * kHubFactor))
                    : 0;
      B->global_ids.push_back(g);
    }
    B->chunk_off[g] = chunks;
    B->chunk_cap[g] = cap;
    chunks += cap + 1;
    B->nodes += gr.n;
    B->total_nnz += nnz;
    rows += int64_t(gr.n) + 1;
  }
  if (!B->global_ids.empty() && o.block_threads > 256)
    return bail(fail(LAYOUT_E_UNSUPPORTED, "global engine runs at most 256-thread workgroups"));
  {
    bool all_fit = !B->global_ids.empty();
    for (int32_t g : B->global_ids) all_fit = all_fit && int64_t(B->n[g]) * 8 <= kXcdMaxPositionBytes;
    const bool store = B->mode_global == LAYOUT_HOGWILD_STORE;
    const bool plain = !jacobi && store && o.block_threads <= 256 &&
                       o.grid_blocks == 0;
    if (o.engine == LAYOUT_ENGINE_XCD) {
      if (!plain || !all_fit)
        return bail(fail(LAYOUT_E_UNSUPPORTED,
                         "XCD-local engine: HOGWILD_STORE, automatic launch shape and graphs of at most "
                         "%lld B of positions", (long long)kXcdMaxPositionBytes));
      B->xcd_mode = true;
    } else if (o.engine == LAYOUT_ENGINE_AUTO) {
      B->xcd_mode = plain && all_fit;
    }
  }

  // packed allocations
  int rc;
  if ((rc = balloc(B, reinterpret_cast<void**>(&B->d_row), sizeof(int64_t) * size_t(rows), "row_ptr")) ||
      (rc = balloc(B, reinterpret_cast<void**>(&B->d_col), sizeof(int32_t) * size_t(B->total_nnz), "col")) ||
      (rc = balloc(B, reinterpret_cast<void**>(&B->d_Y), sizeof(float2) * size_t(B->nodes), "positions")) ||
      (rc = balloc(B, reinterpret_cast<void**>(&B->d_chunk_begin), sizeof(int64_t) * size_t(chunks), "chunk begin")) ||
      (rc = balloc(B, reinterpret_cast<void**>(&B->d_chunk_src), sizeof(int32_t) * size_t(chunks), "chunk src")) ||
      (rc = balloc(B, reinterpret_cast<void**>(&B->d_err), sizeof(uint32_t), "flag")) ||
      (rc = balloc(B, reinterpret_cast<void**>(&B->d_table_global), sizeof(GraphDesc) * size_t(count), "table")) ||
      (rc = balloc(B, reinterpret_cast<void**>(&B->d_table_lds), sizeof(GraphDesc) * size_t(count), "table")) ||
      (rc = balloc(B, reinterpret_cast<void**>(&B->d_lds_ids), sizeof(int32_t) * size_t(count), "ids")))
    return bail(rc);
  if (B->xcd_mode &&
      ((rc = balloc(B, reinterpret_cast<void**>(&B->d_table_xcd), sizeof(GraphDesc) * size_t(count), "xcd table")) ||
       (rc = balloc(B, reinterpret_cast<void**>(&B->d_segs), sizeof(XcdSeg) * size_t(count), "xcd segments")) ||
       (rc = balloc(B, reinterpret_cast<void**>(&B->d_bins), sizeof(XcdBin) * kXcds, "xcd bins")) ||
       (rc = balloc(B, reinterpret_cast<void**>(&B->d_xcd_counters),
                    sizeof(int32_t) * size_t(epochs) * size_t(count), "xcd counters"))))
    return bail(rc);
  if (jacobi && (rc = balloc(B, reinterpret_cast<void**>(&B->d_D), sizeof(float2) * size_t(B->nodes), "delta")))
    return bail(rc);
  // weighted negatives (degrees or the caller's weights): one alias table per graph
  const bool degree = o.neg_weights != LAYOUT_NEG_UNIFORM;
  if (degree &&
      ((rc = balloc(B, reinterpret_cast<void**>(&B->d_thr), sizeof(uint32_t) * size_t(B->nodes), "alias thr")) ||
       (rc = balloc(B, reinterpret_cast<void**>(&B->d_alias), sizeof(uint32_t) * size_t(B->nodes), "alias"))))
    return bail(rc);

  // per graph: copy, validate, chunk table (LDS group), alias, init
  const hipMemcpyKind kind = inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  B->desc.resize(count);
  for (int32_t g = 0; g < count; ++g) {
    const layout_graph& gr = graphs[g];
    int64_t* row = B->d_row + B->row_off[g];
    int32_t* col = B->d_col + B->edge_off[g];
    float2* Y = B->d_Y + B->node_off[g];
    if ((rc = upload_row_ptr(B->stream, gr.row_ptr, gr.n, inputs_on_device != 0, row)) != LAYOUT_OK)
      return bail(rc);
    if (B->nnz[g] > 0)
      e = hipMemcpyAsync(col, gr.col_idx, sizeof(int32_t) * size_t(B->nnz[g]), kind, B->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "copying a graph"));
    if ((rc = validate_csr(B->stream, row, col, gr.n, B->nnz[g], B->d_err)) != LAYOUT_OK) {
      std::string m = g_last_error;
      return bail(fail(rc, "graph %d: %s", g, m.c_str()));
    }
    GraphDesc d{};
    d.row_ptr = row;
    d.col = col;
    d.chunk_begin = B->d_chunk_begin + B->chunk_off[g];
    d.chunk_src = B->d_chunk_src + B->chunk_off[g];
    d.Y = Y;
    d.D = B->d_D ? B->d_D + B->node_off[g] : nullptr;
    d.nnz = B->nnz[g];
    d.n = gr.n;
    d.t0 = 0;
    d.T = epochs;
    d.seed = gr.seed;
    d.eta0 = o.eta0;
    d.alpha = o.alpha;
    d.beta = o.beta;
    d.gamma = o.gamma;
    d.force = o.force_kernel;
    d.sc = sampler_consts(gr.n);
    d.lanes = B->in_lds[g] ? B->lds_block[g] : 0;
    if (B->in_lds[g] && B->nnz[g] > 0) {
      d.hub = B->lds_hub[g];
      int64_t nc = 0;
      if ((rc = build_chunk_table(B->stream, row, gr.n, B->nnz[g], B->lds_bundle[g], d.hub,
                                  const_cast<int64_t*>(d.chunk_begin),
                                  const_cast<int32_t*>(d.chunk_src), &nc)) != LAYOUT_OK)
        return bail(rc);
      d.n_chunks = nc;
    }
    if (degree && B->nnz[g] > 0) {
      d.thr = B->d_thr + B->node_off[g];
      d.alias = B->d_alias + B->node_off[g];
      if (o.neg_weights == LAYOUT_NEG_CUSTOM) {
        if ((rc = upload_weights_and_build_alias(B->stream, row, gr.neg_weight_values, gr.n,
                                                 inputs_on_device != 0,
                                                 const_cast<uint32_t*>(d.thr),
                                                 const_cast<uint32_t*>(d.alias))) != LAYOUT_OK) {
          std::string m = g_last_error;
          return bail(fail(rc, "graph %d: %s", g, m.c_str()));
        }
      } else if ((rc = build_alias_table(B->stream, row, nullptr, gr.n, B->nnz[g],
                                         const_cast<uint32_t*>(d.thr),
                                         const_cast<uint32_t*>(d.alias))) != LAYOUT_OK) {
        return bail(rc);
      }
    }
    if (gr.init_pos) {
      e = hipMemcpyAsync(Y, gr.init_pos, sizeof(float2) * size_t(gr.n), kind, B->stream);
      if (e != hipSuccess) return bail(hip_fail(e, "copying init_pos"));
    } else if (o.init_mode == LAYOUT_INIT_PMDS && gr.n > 0) {
      if ((rc = pmds_positions(B->stream, row, col, gr.n,
                               o.pmds_pivots ? o.pmds_pivots : kDefaultPivots, gr.seed, Y,
                               nullptr, nullptr, nullptr)) != LAYOUT_OK)
        return bail(rc);
    } else {
      launch_init_positions(B->stream, Y, gr.n, gr.seed);
    }
    B->desc[g] = d;
  }
  if (B->d_D) launch_fill_zero(B->stream, B->d_D, B->nodes);

  // groups
  B->gg.d_table = B->d_table_global;
  B->gg.G = 0;
  for (int32_t g : B->global_ids) B->gg.G += B->nnz[g] > 0 ? 1 : 0;
  B->gg.k = k;
  B->gg.mode = B->mode_global;
  B->gg.degree = degree;
  B->gg.block = o.block_threads ? o.block_threads : 256;
  B->gg.jacobi_Y = B->d_Y;
  B->gg.jacobi_D = B->d_D;
  B->gg.jacobi_nodes = B->nodes;
  B->xg.d_table = B->d_table_xcd;
  B->xg.d_segs = B->d_segs;
  B->xg.d_bins = B->d_bins;
  B->xg.d_counters = B->d_xcd_counters;
  B->xg.k = k;
  B->xg.degree = degree;
  if ((rc = build_global_chunks(B)) != LAYOUT_OK) return bail(rc);
  {
    std::vector<GraphDesc> lt;
    std::vector<int32_t> ids;
    for (size_t q = 0; q < B->lds_ids.size(); ++q) {
      lt.push_back(B->desc[B->lds_ids[q]]);
      ids.push_back(static_cast<int32_t>(q));
    }
    if (!lt.empty()) {
      e = hipMemcpyAsync(B->d_table_lds, lt.data(), sizeof(GraphDesc) * lt.size(),
                         hipMemcpyHostToDevice, B->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(B->d_lds_ids, ids.data(), sizeof(int32_t) * ids.size(),
                           hipMemcpyHostToDevice, B->stream);
      if (e != hipSuccess) return bail(hip_fail(e, "uploading the LDS table"));
    }
    B->lg.d_table = B->d_table_lds;
    B->lg.d_ids = B->d_lds_ids;
    B->lg.blocks = static_cast<int>(lt.size());
    B->lg.lds_bytes = max_lds;
    B->lg.k = k;
    B->lg.mode = B->mode_lds;
    B->lg.degree = degree;
    int lds_block = 64;
    for (int32_t g : B->lds_ids) lds_block = std::max(lds_block, B->lds_block[g]);
    B->lg.block = lds_block;
    if (!lt.empty() && (rc = allow_lds(k, max_lds)) != LAYOUT_OK) return bail(rc);
  }
  e = hipStreamSynchronize(B->stream);
  if (e != hipSuccess) return bail(hip_fail(e, "finishing batch create"));
  if ((rc = capture(B)) != LAYOUT_OK) return bail(rc);
  *out = B;
  return LAYOUT_OK;
}

int layout_batch_run(layout_batch_t* B) {
  if (!check_batch(B)) return LAYOUT_E_INVALID_ARG;
  if (B->ran) return fail(LAYOUT_E_DONE, "the batch already ran its %d epochs", B->epochs);
  hipError_t e = hipGraphLaunch(B->exec, B->stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  B->ran = true;
  return LAYOUT_OK;
}

int layout_batch_run_timed(layout_batch_t* B, float* ms) {
  if (!check_batch(B)) return LAYOUT_E_INVALID_ARG;
  if (!ms) return fail(LAYOUT_E_INVALID_ARG, "ms is NULL");
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  int rc = LAYOUT_OK;
  if (e == hipSuccess) e = hipEventRecord(a, B->stream);
  if (e == hipSuccess) {
    rc = layout_batch_run(B);
    if (rc == LAYOUT_OK) {
      e = hipEventRecord(b, B->stream);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (rc != LAYOUT_OK) return rc;
  if (e != hipSuccess) return hip_fail(e, "timing the batch");
  return LAYOUT_OK;
}

int layout_batch_get_positions(const layout_batch_t* B, int32_t g, float* host_out) {
  if (!check_batch(B)) return LAYOUT_E_INVALID_ARG;
  if (g < 0 || g >= B->count || !host_out) return fail(LAYOUT_E_INVALID_ARG, "graph %d", g);
  if (B->n[g] == 0) return LAYOUT_OK;
  hipError_t e = hipMemcpyAsync(host_out, B->d_Y + B->node_off[g], sizeof(float2) * size_t(B->n[g]),
                                hipMemcpyDeviceToHost, B->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
  if (e != hipSuccess) return hip_fail(e, "reading positions");
  return LAYOUT_OK;
}

int layout_batch_get_positions_device(const layout_batch_t* B, float* dev_out) {
  if (!check_batch(B)) return LAYOUT_E_INVALID_ARG;
  if (!dev_out) return fail(LAYOUT_E_INVALID_ARG, "dev_out is NULL");
  if (B->nodes == 0) return LAYOUT_OK;
  hipError_t e = hipMemcpyAsync(dev_out, B->d_Y, sizeof(float2) * size_t(B->nodes),
                                hipMemcpyDeviceToDevice, B->stream);
  if (e != hipSuccess) return hip_fail(e, "copying positions");
  return LAYOUT_OK;
}

int layout_batch_sync(const layout_batch_t* B) {
  if (!check_batch(B)) return LAYOUT_E_INVALID_ARG;
  hipError_t e = hipStreamSynchronize(B->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return LAYOUT_OK;
}

int layout_batch_debug_draws(const layout_batch_t* B, int32_t g, int32_t epoch, int32_t* host_out) {
  if (!check_batch(B)) return LAYOUT_E_INVALID_ARG;
  if (g < 0 || g >= B->count || !host_out) return fail(LAYOUT_E_INVALID_ARG, "graph %d", g);
  if (B->nnz[g] == 0 || B->k == 0) return LAYOUT_OK;
  const size_t bytes = sizeof(int32_t) * size_t(B->nnz[g]) * size_t(B->k);
  int32_t* d_out = nullptr;
  hipError_t e = hipMalloc(&d_out, bytes);
  if (e != hipSuccess) return hip_fail(e, "debug draws buffer");
  int rc = launch_dump_draws(B->stream, B->k, B->opts.neg_weights != LAYOUT_NEG_UNIFORM, B->desc[g],
                             epoch, d_out);
  if (rc == LAYOUT_OK) {
    e = hipMemcpyAsync(host_out, d_out, bytes, hipMemcpyDeviceToHost, B->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) rc = hip_fail(e, "reading debug draws");
  }
  (void)hipFree(d_out);
  return rc;
}

int layout_batch_get_info(const layout_batch_t* B, layout_batch_info* info) {
  if (!check_batch(B)) return LAYOUT_E_INVALID_ARG;
  if (!info) return fail(LAYOUT_E_INVALID_ARG, "info is NULL");
  std::memset(info, 0, sizeof *info);
  info->graphs = B->count;
  info->lds_graphs = static_cast<int32_t>(B->lds_ids.size());
  info->global_graphs = static_cast<int32_t>(B->global_ids.size());
  info->epochs = B->epochs;
  info->nodes = B->nodes;
  info->nnz = B->total_nnz;
  info->global_chunks = B->gg.total_chunks;
  info->device_bytes = static_cast<int64_t>(B->buf.bytes());
  info->bundle_edges = B->bundle;
  info->hub_split_edges = B->hub;
  info->grid_blocks = B->gg.total_chunks > 0 ? global_grid(B->gg) : 0;
  info->block_threads = B->gg.block;
  info->lds_block_threads = B->lg.block;
  info->update_mode_global = B->mode_global;
  info->update_mode_lds = B->mode_lds;
  info->epochs_done = B->ran ? B->epochs : 0;
  info->xcd_engine = B->xcd_mode ? 1 : 0;
  info->xcd_grid_blocks = B->xcd_mode ? B->xg.grid : 0;
  if (B->xcd_mode) info->grid_blocks = B->xg.grid;
  return LAYOUT_OK;
}

int layout_batch_autotune(layout_batch_t* B, int32_t trial_epochs, const char* cache_path,
                          int32_t* bundle_out, int32_t* blocks_per_cu_out, float* ms_out) {
  if (!check_batch(B)) return LAYOUT_E_INVALID_ARG;
  if (B->ran) return fail(LAYOUT_E_DONE, "tune before running the batch");
  if (trial_epochs < 1) return fail(LAYOUT_E_INVALID_ARG, "trial_epochs = %d", trial_epochs);
  int best_b = B->bundle, best_p = B->blocks_per_cu;
  float best_ms = -1.f;
  const std::string key = tune_key(B);
  bool cached = false;
  if (B->gg.total_chunks > 0 && !cache_lookup(cache_path, key, &best_b, &best_p, &best_ms)) {
    // scratch copy of the positions: the trials must not change the layout
    float2* saved = nullptr;
    hipError_t e = hipMalloc(&saved, sizeof(float2) * size_t(std::max<int64_t>(1, B->nodes)));
    if (e != hipSuccess) return hip_fail(e, "autotune scratch");
    e = hipMemcpyAsync(saved, B->d_Y, sizeof(float2) * size_t(B->nodes), hipMemcpyDeviceToDevice,
                       B->stream);
    hipEvent_t a = nullptr, b = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    int rc = LAYOUT_OK;
    const int bundles[] = {8, 16, 32};
    const int per_cu[] = {2, 4, 8, 0};
    const int32_t keep_b = B->bundle, keep_h = B->hub;
    for (int bi = 0; bi < 3 && e == hipSuccess && rc == LAYOUT_OK; ++bi) {
      B->bundle = bundles[bi];
      B->hub = kHubFactor * bundles[bi];
      if ((rc = build_global_chunks(B)) != LAYOUT_OK) break;
      if (B->xcd_mode) {
        // the XCD-local engine's workers follow from the lane caps: only the
        // chunk size is searched
        if ((rc = upload_xcd_table(B)) != LAYOUT_OK) break;
        const int64_t nctr = int64_t(B->epochs) * B->count;
        launch_fill_i32(B->stream, B->d_xcd_counters, nctr, 0);
        rc = launch_xcd_group_epochs(B->stream, B->xg, 0, 1);  // warm-up
        if (rc == LAYOUT_OK) {
          launch_fill_i32(B->stream, B->d_xcd_counters, nctr, 0);
          e = hipEventRecord(a, B->stream);
        }
        const int32_t trials = std::min(trial_epochs, B->epochs);
        if (rc == LAYOUT_OK && e == hipSuccess) rc = launch_xcd_group_epochs(B->stream, B->xg, 0, trials);
        if (rc == LAYOUT_OK && e == hipSuccess) e = hipEventRecord(b, B->stream);
        if (rc == LAYOUT_OK && e == hipSuccess) e = hipEventSynchronize(b);
        float t = 0.f;
        if (rc == LAYOUT_OK && e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
        const float tt = t * float(trial_epochs) / float(trials);
        if (rc == LAYOUT_OK && e == hipSuccess && (best_ms < 0 || tt < best_ms)) {
          best_ms = tt;
          best_b = bundles[bi];
          best_p = 0;
        }
        if (e == hipSuccess)
          e = hipMemcpyAsync(B->d_Y, saved, sizeof(float2) * size_t(B->nodes),
                             hipMemcpyDeviceToDevice, B->stream);
        continue;
      }
      for (int pi = 0; pi < 4 && e == hipSuccess && rc == LAYOUT_OK; ++pi) {
        GlobalGroup g = B->gg;
        g.grid = 0;
        if (per_cu[pi] > 0) g.grid = std::min(global_grid(g), per_cu[pi] * device_props().cus);
        if ((rc = upload_global_table(B, global_grid(g))) != LAYOUT_OK) break;
        g = B->gg;
        g.grid = 0;
        if (per_cu[pi] > 0) g.grid = std::min(global_grid(g), per_cu[pi] * device_props().cus);
        // warm-up epoch, then the timed ones (epoch index 0.. of the schedule)
        rc = launch_global_epochs(B->stream, g, 0, 1);
        if (rc == LAYOUT_OK) e = hipEventRecord(a, B->stream);
        if (rc == LAYOUT_OK && e == hipSuccess) rc = launch_global_epochs(B->stream, g, 0, trial_epochs);
        if (rc == LAYOUT_OK && e == hipSuccess) e = hipEventRecord(b, B->stream);
        if (rc == LAYOUT_OK && e == hipSuccess) e = hipEventSynchronize(b);
        float t = 0.f;
        if (rc == LAYOUT_OK && e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
        if (rc == LAYOUT_OK && e == hipSuccess && (best_ms < 0 || t < best_ms)) {
          best_ms = t;
          best_b = bundles[bi];
          best_p = per_cu[pi];
        }
        // restore the positions for the next trial
        if (e == hipSuccess)
          e = hipMemcpyAsync(B->d_Y, saved, sizeof(float2) * size_t(B->nodes),
                             hipMemcpyDeviceToDevice, B->stream);
      }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(saved);
    B->bundle = keep_b;
    B->hub = keep_h;
    if (rc != LAYOUT_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "autotune");
    if (best_ms >= 0.f) best_ms /= trial_epochs;
    cache_store(cache_path, key, best_b, best_p, best_ms);
  } else {
    cached = true;
  }
  (void)cached;
  B->bundle = best_b;
  B->hub = kHubFactor * best_b;
  B->blocks_per_cu = best_p;
  int rc = build_global_chunks(B);
  if (rc == LAYOUT_OK) rc = capture(B);
  if (rc != LAYOUT_OK) return rc;
  if (bundle_out) *bundle_out = best_b;
  if (blocks_per_cu_out) *blocks_per_cu_out = best_p;
  if (ms_out) *ms_out = best_ms;
  return LAYOUT_OK;
}

void layout_batch_destroy(layout_batch_t* B) {
  if (!B) return;
  if (B->stream) (void)hipStreamSynchronize(B->stream);
  if (B->side) (void)hipStreamSynchronize(B->side);
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->buf.free_all();
  if (B->fork) (void)hipEventDestroy(B->fork);
  if (B->join) (void)hipEventDestroy(B->join);
  if (B->stream) (void)hipStreamDestroy(B->stream);
  if (B->side) (void)hipStreamDestroy(B->side);
  delete B;
}

}  // extern "C"
