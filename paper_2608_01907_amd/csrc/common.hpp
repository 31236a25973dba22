// Host helpers shared by the plain, batched and served entry points.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>
#include <vector>

#include "desc.hpp"
#include "snaplayout.h"
#include "rng.hpp"

namespace snap {

// Defaults of the launch shape (overridable per handle, tuned by the batch
// autotuner).
constexpr int kDefaultBundle = 16;           // target directed edges per lane chunk (global engine)
constexpr int kHubFactor = 4;                // global engine: rows above 4 * B edges are split
constexpr int kNodesPerLane = 32;            // lanes in flight <= n / 32 (both engines)
constexpr int kLanesPerCU = 256;             // global engine: at most 256 lanes per CU in flight
                                             // (the random-access throughput saturates there)

// Active lanes of the LDS engine for an n-node graph: n / nodes_per_lane
// rounded up to whole wavefronts, as on the other engines (at most 1024, one
// workgroup; a 2D graph that fits LDS has at most 640).
inline int lds_lanes_for(int32_t n, int nodes_per_lane) {
  const int npl = nodes_per_lane > 0 ? nodes_per_lane : kNodesPerLane;
  const int want = (((n / npl) > 1 ? (n / npl) : 1) + 63) / 64 * 64;
  return want > 1024 ? 1024 : want;
}
// LDS engine: rows above this many edges are split into segments, as on the
// other engines.  A wavefront runs its lanes' chunks in step, so one lane on
// a whole hub row would hold its 63 neighbours idle for the row's length;
// on one CU the engine is bound by issue, so segments of at most twice the
// bundle keep the chunks of a wavefront close in length.
constexpr int kLdsHub = 2 * kDefaultBundle;
constexpr long long kLdsAutoMaxEdges = 400000;  // AUTO picks LDS below this many directed edges
constexpr long long kXcdMaxPositionBytes = 3 << 20;  // XCD-local engine: positions within 3 MiB
                                                     // of the 4 MiB L2 of one XCD

extern thread_local std::string g_last_error;
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char* what);

struct DeviceProps {
  bool valid = false;
  int cus = 0;
  int lds_per_block = 0;
};
const DeviceProps& device_props();

SamplerConsts sampler_consts(int32_t n);

inline int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Upper bound of the chunk count, for allocation before the exact count is
// known: one chunk per B-bucket, one per hub segment, one after each hub.
// Most chunks one table may hold: chunk indices and work counters are 32-bit.
constexpr int64_t kMaxChunks = INT32_MAX - (int64_t(1) << 24);

inline int64_t chunk_bound(int64_t nnz, int32_t bundle, int32_t hub) {
  return (nnz + bundle - 1) / bundle + 2 * ((nnz + hub - 1) / hub) + 2;
}

// Preprocessing shared by every entry point (snaplayout.hip).
int build_chunk_table(hipStream_t stream, const int64_t* d_row, int32_t n, int64_t nnz,
                      int32_t bundle, int32_t hub, int64_t* d_chunk_begin, int32_t* d_chunk_src,
                      int64_t* n_chunks);
// Integer alias table for the weights d_weights[0..n) (nullable: degrees from
// d_row), W = their sum, 0 < W < 2^32.
int build_alias_table(hipStream_t stream, const int64_t* d_row, const uint32_t* d_weights,
                      int32_t n, int64_t W, uint32_t* d_thr, uint32_t* d_alias);
// Copies an int32 row_ptr[n + 1] (host, or device when on_device) into the
// 64-bit device row pointers every kernel reads.  Synchronises the stream.
int upload_row_ptr(hipStream_t stream, const int32_t* row_ptr, int32_t n, bool on_device,
                   int64_t* d_row);
// The alias table of caller weights (host, or device when on_device; n
// entries whose sum W must satisfy 0 < W < 2^32, else LAYOUT_E_INVALID_ARG).
// Synchronises the stream.
int upload_weights_and_build_alias(hipStream_t stream, const int64_t* d_row,
                                   const uint32_t* weights, int32_t n, bool on_device,
                                   uint32_t* d_thr, uint32_t* d_alias);
// Device validation of one CSR (LAYOUT_E_BAD_GRAPH with a message on failure);
// err is a device word of scratch.
int validate_csr(hipStream_t stream, const int64_t* d_row, const int32_t* d_col, int32_t n,
                 int64_t nnz, uint32_t* d_err);
// Seeded uniform initial positions; dim 3 writes float4 positions through the
// float2 pointer (n float4 = 2n float2 of storage).
void launch_init_positions(hipStream_t stream, float2* d_Y, int32_t n, uint64_t seed,
                           int dim = 2);
// Pivot MDS positions of a validated CSR (pmds.hip).  d_pivots_out (nullable,
// device, [pivots]) receives the pivots, d_dist_out (nullable, device,
// pivots x n) the hop distances; *pivots_used the pivots taken.  Synchronises
// the stream (the scratch it allocates is freed on return).
constexpr int32_t kDefaultPivots = 50;
int pmds_positions(hipStream_t stream, const int64_t* d_row, const int32_t* d_col, int32_t n,
                   int32_t pivots, uint64_t seed, float2* d_Y, int32_t* d_pivots_out,
                   int32_t* d_dist_out, int32_t* pivots_used);
void launch_fill_zero(hipStream_t stream, float2* d_p, int64_t n);
// Silhouette monitor (the SI metric of Sec. 4.1, exact): host side (clusters
// 0..C-1 in order of label value, nodes counting-sorted by cluster) ...
struct SilhouetteInput {
  int32_t C = 0;
  std::vector<int32_t> order, cs, cstart;
};
int silhouette_input(const int32_t* labels, int32_t n, const double* si_out,
                     SilhouetteInput& in);
// ... and device side: node order (n), cluster of each sorted node (n),
// cluster starts (C + 1), sorted positions (n), two FP64 sums.
struct SilhouetteBuffers {
  int32_t *order = nullptr, *cs = nullptr, *cstart = nullptr;
  float2* Ys = nullptr;
  double* acc = nullptr;
};
// Copies the inputs into b, runs the gather and the exact silhouette kernel on
// the positions d_Y and writes the mean to *si_out (synchronises stream).
int silhouette_run(hipStream_t stream, const float2* d_Y, int32_t n, const SilhouetteInput& in,
                   const SilhouetteBuffers& b, double* si_out);
// What other translation units may read of a layout handle: its size,
// device, stream and device positions.  LAYOUT_E_INVALID_ARG for NULL.
struct HandleView {
  int32_t n = 0, dim = 2;
  int dev = 0;
  hipStream_t stream = nullptr;
  float2* Y = nullptr;
};
int handle_view(const layout_t* L, HandleView* v);
// Jacobi apply of one 2D graph: Y += D, then D = 0.
void launch_jacobi_apply(hipStream_t stream, float2* d_Y, float2* d_D, int32_t n);
// CQ of the positions (cluster.hip): k-means (k-means++ start from seed, or
// init_centers, host K x 2) and the ARI against host labels[n].  Outputs
// (nullable but ari_out) on the host.  Synchronises the stream.
int kmeans_cq(hipStream_t stream, const float2* d_Y, int32_t n, const int32_t* labels,
              int32_t K, uint64_t seed, int32_t max_iter, const float* init_centers,
              double* ari_out, int32_t* assign_out, int32_t* iters_out,
              int32_t* centers_idx_out);
// Epochs [t, t + count) of one single-graph table with the conflict counter
// (probes.hip): writes, writes that followed a concurrent write of the same
// node since their load, and writes whose load the counter no longer held.
int run_conflict_epochs(hipStream_t stream, const GraphDesc* d_table, int32_t n, int k,
                        int mode, bool degree, int grid, int block, int32_t t, int32_t count,
                        int64_t* stores, int64_t* conflicts, int64_t* untracked);
// k_i and |R_i ∩ K_i| of the NP metric for host query nodes (neighbours.hip;
// host outputs, count entries).  Synchronises the stream.
int neighbourhood_counts(hipStream_t stream, const int64_t* d_row, const int32_t* d_col,
                         const float2* d_Y, int32_t n, const int32_t* nodes, int32_t count,
                         int32_t radius, int32_t* k_out, int32_t* inter_out);

// Graphs whose epochs run on the global engine, one launch per epoch for all
// of them (table entries carry chunk_base prefixes over the group).
struct GlobalGroup {
  const GraphDesc* d_table = nullptr;
  int G = 0;
  int64_t total_chunks = 0;  // chunks of all graphs
  int64_t round_size = 0;    // unused by the global engine (lanes, not rounds)
  int64_t total_index = 0;   // G > 1: lanes handed out by plan_lanes
  int k = 5, mode = kStore;
  bool degree = false;
  int block = 256;
  int grid = 0;    // 0 = fill the device, capped by max_lanes
  int64_t max_lanes = 0;  // 0 = no cap
  int dim = 2;            // positions: float2 (2) or float4 (3)
  float2* jacobi_Y = nullptr;  // JACOBI: Y and D of every graph, contiguous
  float2* jacobi_D = nullptr;
  int64_t jacobi_nodes = 0;
};
// Graphs run whole by one workgroup each, positions in LDS.
struct LdsGroup {
  const GraphDesc* d_table = nullptr;
  const int32_t* d_ids = nullptr;  // table index of each workgroup's graph
  int blocks = 0;
  int lds_bytes = 0;
  int k = 5, mode = kAtomic;
  bool degree = false;
  int block = 256;
  int dim = 2;
};
// Global-group graphs on the XCD-local engine (see desc.hpp).
struct XcdGroup {
  const GraphDesc* d_table = nullptr;
  const XcdSeg* d_segs = nullptr;
  const XcdBin* d_bins = nullptr;
  int32_t* d_counters = nullptr;  // [epoch][segment] chunk counters, zero before the epochs run
  int32_t n_segs = 0;
  int k = 5;
  bool degree = false;
  int grid = 0;  // kXcds x the largest bin's workers
  int64_t total_chunks = 0;
};
// Bins, segments and rounds for the graphs of `graphs` (n_chunks set); fills
// the launch table (slice/chunk_base per segment), segs and bins; returns the
// launch grid.
int plan_xcd_bins(const std::vector<GraphDesc>& graphs, int nodes_per_lane,
                  std::vector<GraphDesc>& table, std::vector<XcdSeg>& segs, XcdBin* bins);
int launch_xcd_group_epochs(hipStream_t stream, const XcdGroup& g, int32_t dt, int32_t count);
void launch_fill_i32(hipStream_t stream, int32_t* p, int64_t n, int32_t v);
int lds_bytes_for(int32_t n, int dim = 2);  // LDS of one graph's positions
// Lanes of a multi-graph launch of the global engine (table: host copy,
// n_chunks set): graph g gets the lanes [chunk_base, chunk_base + slice),
// chunk_base on a wavefront boundary, slice its cap n_g / nodes_per_lane (at
// least 1, at most its chunks) when the caps fit `lanes`, else lanes in
// proportion to its chunks up to that cap.  Sets the group's total_index
// (the lanes handed out, which a launch must cover) and total_chunks.
void plan_lanes(std::vector<GraphDesc>& table, GlobalGroup& g, int64_t lanes, int nodes_per_lane);
// The sum of those caps, each padded to whole wavefronts (the lanes such a
// launch wants).
int64_t lane_caps(const std::vector<GraphDesc>& table, int nodes_per_lane);
// Lanes of a multi-graph XCD-local segment such that every graph g, which
// receives lanes in proportion to its chunk count, has at most
// n_g / nodes_per_lane of them.
int64_t fair_lanes(const std::vector<GraphDesc>& table, int nodes_per_lane);
int global_grid(const GlobalGroup& g);  // resolved grid size
int launch_global_epochs(hipStream_t stream, const GlobalGroup& g, int32_t dt, int32_t count);
int launch_lds_epochs(hipStream_t stream, const LdsGroup& g, int32_t dt, int32_t count);
int allow_lds(int k, int bytes, int dim = 2);  // raise the dynamic LDS limit of the LDS kernels
// negatives of every edge of one graph in epoch t (device out[nnz*k])
int launch_dump_draws(hipStream_t stream, int k, bool degree, const GraphDesc& g, int32_t t,
                      int32_t* d_out);

// Device allocations owned by one object, freed together.
struct DeviceBuffers {
  std::vector<void*> ptrs;
  size_t total = 0;
  void add(void* p, size_t bytes) {
    ptrs.push_back(p);
    total += bytes;
  }
  size_t bytes() const { return total; }
  void free_all() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
    total = 0;
  }
  // stream-ordered: for buffers from hipMallocAsync; waits for no other stream
  void free_all_async(hipStream_t stream) {
    for (void* p : ptrs) (void)hipFreeAsync(p, stream);
    ptrs.clear();
    total = 0;
  }
};

}  // namespace snap
