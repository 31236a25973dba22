// Host side of the C ABI declared in include/snaplayout.h.
//
// A handle owns its device copy of the CSR, the chunk table, the positions and
// a one-entry graph table; every kernel of the handle runs on one HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "alias.hpp"
#include "chunks.hpp"
#include "common.hpp"
#include "energy.hpp"
#include "kernels.hpp"
#include "snaplayout.h"

using namespace snap;

// ----------------------------------------------------------------- errors
namespace snap {
thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory)
    return fail(LAYOUT_E_OOM, "%s: out of device memory", what);
  return fail(LAYOUT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

const DeviceProps& device_props() {
  static thread_local DeviceProps cache[64];
  int dev = 0;
  (void)hipGetDevice(&dev);
  DeviceProps& p = cache[dev & 63];
  if (!p.valid) {
    (void)hipDeviceGetAttribute(&p.cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipDeviceGetAttribute(&p.lds_per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (p.cus <= 0) p.cus = 256;
    if (p.lds_per_block <= 0) p.lds_per_block = 65536;
    p.valid = true;
  }
  return p;
}

SamplerConsts sampler_consts(int32_t n) {
  SamplerConsts sc{};
  sc.n = static_cast<uint32_t>(n);
  sc.range = n >= 2 ? static_cast<uint32_t>(n - 1) : 1u;
  sc.reject_range = n >= 2 ? static_cast<uint32_t>((1ull << 32) % static_cast<uint64_t>(n - 1)) : 0u;
  sc.reject_n = n >= 1 ? static_cast<uint32_t>((1ull << 32) % static_cast<uint64_t>(n)) : 0u;
  return sc;
}
}  // namespace snap

// ------------------------------------------------------------- dispatching
namespace {

template <class F>
int with_k(int k, F&& f) {
  switch (k) {
    case 0: return f(std::integral_constant<int, 0>{});
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 7: return f(std::integral_constant<int, 7>{});
    case 8: return f(std::integral_constant<int, 8>{});
    default: return fail(LAYOUT_E_UNSUPPORTED, "k = %d not supported (0..8)", k);
  }
}

template <class F>
int with_mode(int mode, F&& f) {
  switch (mode) {
    case kStore: return f(std::integral_constant<int, kStore>{});
    case kAtomic: return f(std::integral_constant<int, kAtomic>{});
    case kJacobi: return f(std::integral_constant<int, kJacobi>{});
    default: return fail(LAYOUT_E_INVALID_ARG, "update_mode %d", mode);
  }
}

template <class F>
int with_degree(bool degree, F&& f) {
  if (degree) return f(std::true_type{});
  return f(std::false_type{});
}

template <class F>
int with_dim(int dim, F&& f) {
  if (dim == 3) return f(std::integral_constant<int, 3>{});
  return f(std::integral_constant<int, 2>{});
}

}  // namespace

// ------------------------------------------------------------------ handle
struct layout {
  int32_t n = 0, k = 0, epochs = 0, t = 0;
  int32_t dim = 2;  // positions: float2[n] (2) or float4[n] holding x, y, z (3)
  int64_t nnz = 0;
  uint64_t seed = 0;
  layout_opts opts{};
  int32_t engine = LAYOUT_ENGINE_GLOBAL;
  int32_t mode = LAYOUT_ATOMIC;  // resolved update policy
  int32_t bundle = 16;
  int32_t hub = 64;
  int32_t block = 256;
  int32_t grid = 0;
  int32_t hot_degree = 0;  // resolved hot-node threshold (0 = no hot nodes)
  int64_t n_chunks = 0;
  bool own_stream = false;
  hipStream_t stream = nullptr;
  int dev = 0;
  DeviceBuffers buf;
  GraphDesc host_desc{};
  GraphDesc* d_table = nullptr;  // one entry
  int32_t* d_graph_ids = nullptr;
  double* d_energy = nullptr;  // two FP64 accumulators of the energy monitors
  int32_t* d_xcd_owner = nullptr;    // XCD-local engine: owner XCD of each epoch (-1 = none yet)
  int32_t* d_xcd_counter = nullptr;  // XCD-local engine: chunks handed out in each epoch
};

namespace {

int alloc(layout_t* L, void** p, size_t bytes, const char* what) {
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return hip_fail(e, what);
  L->buf.add(*p, bytes);
  return LAYOUT_OK;
}

GlobalGroup global_group_of(const layout_t* L) {
  GlobalGroup g;
  g.d_table = L->d_table;
  g.G = 1;
  g.total_chunks = L->n_chunks;
  g.k = L->k;
  g.mode = L->mode;
  g.degree = L->opts.neg_weights != LAYOUT_NEG_UNIFORM;
  g.block = L->block;
  g.grid = L->opts.grid_blocks;
  g.max_lanes = L->n / (L->opts.nodes_per_lane > 0 ? L->opts.nodes_per_lane : kNodesPerLane);
  g.dim = L->dim;
  g.jacobi_Y = L->host_desc.Y;
  g.jacobi_D = L->host_desc.D;
  g.jacobi_nodes = L->n;
  return g;
}

LdsGroup lds_group_of(const layout_t* L) {
  LdsGroup g;
  g.d_table = L->d_table;
  g.d_ids = L->d_graph_ids;
  g.blocks = 1;
  g.lds_bytes = lds_bytes_for(L->n, L->dim);
  g.dim = L->dim;
  g.k = L->k;
  g.mode = L->mode;
  g.degree = L->opts.neg_weights != LAYOUT_NEG_UNIFORM;
  g.block = L->block;
  return g;
}

// XCD-local engine: workgroups that do the work (at most one per CU of the
// XCD, n / nodes_per_lane lanes), and the launch size that puts about that
// many on the owner XCD when workgroups are spread evenly over the XCDs.
int xcd_workers(const layout_t* L) {
  if (L->opts.grid_blocks > 0) return L->opts.grid_blocks;
  const DeviceProps& dp = device_props();
  const int cus_per_xcd = std::max(1, dp.cus / kXcds);
  const int npl = L->opts.nodes_per_lane > 0 ? L->opts.nodes_per_lane : kNodesPerLane;
  const int64_t lanes = std::max<int64_t>(1, L->n / npl);
  return static_cast<int>(std::min<int64_t>(cus_per_xcd, std::max<int64_t>(1, div_up(lanes, L->block))));
}

int launch_xcd_epochs(layout_t* L, int32_t count) {
  const DeviceProps& dp = device_props();
  const int xcds = dp.cus >= kXcds ? kXcds : 1;
  const int grid = xcd_workers(L) * xcds;
  return with_k(L->k, [&](auto kc) -> int {
    constexpr int K = decltype(kc)::value;
    return with_degree(L->opts.neg_weights != LAYOUT_NEG_UNIFORM, [&](auto dc) -> int {
      constexpr bool DEG = decltype(dc)::value;
      with_dim(L->dim, [&](auto dmc) -> int {
        constexpr int DIM = decltype(dmc)::value;
        for (int32_t ep = 0; ep < count; ++ep) {
          const int32_t t = L->t + ep;
          hipLaunchKernelGGL((epoch_xcd_kernel<K, DEG, DIM>), dim3(grid), dim3(L->block), 0,
                             L->stream, L->d_table, L->d_xcd_owner + t, L->d_xcd_counter + t, t);
        }
        return LAYOUT_OK;
      });
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "epoch_xcd_kernel launch");
      return LAYOUT_OK;
    });
  });
}

int launch_epochs(layout_t* L, int32_t count) {
  if (L->nnz == 0) return LAYOUT_OK;  // no edge, nothing moves
  if (L->engine == LAYOUT_ENGINE_LDS) return launch_lds_epochs(L->stream, lds_group_of(L), L->t, count);
  if (L->engine == LAYOUT_ENGINE_XCD) return launch_xcd_epochs(L, count);
  return launch_global_epochs(L->stream, global_group_of(L), L->t, count);
}

}  // namespace

// Row-aligned chunk table (chunks.hpp), built on the device.  begin/src must
// hold chunk_bound(nnz, bundle, hub) (+1 for begin) entries.
int snap::build_chunk_table(hipStream_t stream, const int64_t* d_row, int32_t n, int64_t nnz,
                            int32_t bundle, int32_t hub, int64_t* d_chunk_begin,
                            int32_t* d_chunk_src, int64_t* n_chunks) {
  // chunk offsets are scanned, and chunk counters advanced, in 32 bits (the
  // margin covers the counters' overshoot past the last chunk)
  if (chunk_bound(nnz, bundle, hub) > kMaxChunks)
    return fail(LAYOUT_E_UNSUPPORTED,
                "%lld edges in chunks of %d (hub rows cut every %d) need more than %lld chunks",
                static_cast<long long>(nnz), bundle, hub, static_cast<long long>(kMaxChunks));
  const int64_t tiles = std::max<int64_t>(1, scan_tiles(n));
  void* tmp = nullptr;
  const size_t b_scan = sizeof(int32_t) * size_t(tiles + 1);
  const size_t bytes = b_scan + size_t(n) + 64;
  // stream-ordered scratch: allocating and freeing it waits for no other
  // stream (a plain free waits for the whole device to go idle)
  hipError_t e = hipMallocAsync(&tmp, bytes, stream);
  if (e != hipSuccess) return hip_fail(e, "chunk scratch");
  auto* scan = static_cast<int32_t*>(tmp);
  auto* flags = reinterpret_cast<uint8_t*>(scan + tiles + 1);
  e = hipMemsetAsync(flags, 0, size_t(n), stream);
  const int64_t buckets = div_up(nnz, bundle);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(chunk_flag_buckets_kernel, dim3(div_up(buckets, 256)), dim3(256), 0,
                       stream, d_row, n, nnz, bundle, flags);
    hipLaunchKernelGGL(chunk_flag_hubs_kernel, dim3(div_up(n, 256)), dim3(256), 0, stream, d_row,
                       n, nnz, hub, flags);
    device_exclusive_scan<int32_t>(stream, n, ChunkCountLoad{d_row, flags, n, hub},
                                   ChunkWrite{d_row, hub, d_chunk_begin, d_chunk_src}, scan);
    hipLaunchKernelGGL(chunk_sentinel_kernel, dim3(1), dim3(1), 0, stream, d_chunk_begin,
                       scan + tiles, nnz);
    int32_t count = 0;
    e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(&count, scan + tiles, sizeof count, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    *n_chunks = count;
  }
  (void)hipFreeAsync(tmp, stream);
  if (e != hipSuccess) return hip_fail(e, "building the chunk table");
  return LAYOUT_OK;
}

// Alias table for weights w_s = degree(s), W = sum w = nnz, built on the
// device (temporary buffers freed before returning).
int snap::build_alias_table(hipStream_t stream, const int64_t* d_row, const uint32_t* d_weights,
                            int32_t n, int64_t W, uint32_t* d_thr, uint32_t* d_alias) {
  // thresholds are own * 2^32 / W with own < W: W must fit 32 bits
  if (W <= 0 || W >= (int64_t(1) << 32))
    return fail(LAYOUT_E_UNSUPPORTED, "alias table: total weight %lld (need 0 < W < 2^32)",
                static_cast<long long>(W));
  const int64_t tiles = std::max<int64_t>(1, scan_tiles(n));
  void* tmp = nullptr;
  const size_t b_sums = sizeof(AliasScanItem) * size_t(tiles + 1);
  const size_t b_items = sizeof(int32_t) * size_t(n);
  const size_t b_inc = sizeof(int64_t) * size_t(n);
  const size_t bytes = b_sums + 2 * b_items + 2 * b_inc + 64;
  hipError_t e = hipMallocAsync(&tmp, bytes, stream);
  if (e != hipSuccess) return hip_fail(e, "alias scratch");
  char* p = static_cast<char*>(tmp);
  auto* sums = reinterpret_cast<AliasScanItem*>(p);
  auto* grand = sums + tiles;
  auto* heavy_inc = reinterpret_cast<int64_t*>(p + b_sums);
  auto* light_inc = heavy_inc + n;
  auto* heavy_item = reinterpret_cast<int32_t*>(light_inc + n);
  auto* light_item = heavy_item + n;
  device_exclusive_scan<AliasScanItem>(stream, n, AliasLoad{d_row, d_weights, n, W},
                                       AliasCompact{heavy_item, heavy_inc, light_item, light_inc},
                                       sums);
  hipLaunchKernelGGL(alias_fill_kernel, dim3(div_up(n, 256)), dim3(256), 0, stream, d_row,
                     d_weights, int64_t(n), W, grand, heavy_item, heavy_inc, light_item, light_inc, d_thr,
                     d_alias);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  (void)hipFreeAsync(tmp, stream);
  if (e != hipSuccess) return hip_fail(e, "building the alias table");
  return LAYOUT_OK;
}

namespace {
__global__ void widen_i32_kernel(const int32_t* __restrict__ src, int64_t* __restrict__ dst,
                                 int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}
}  // namespace

int snap::upload_row_ptr(hipStream_t stream, const int32_t* row_ptr, int32_t n, bool on_device,
                         int64_t* d_row) {
  const size_t count = size_t(n) + 1;
  hipError_t e = hipSuccess;
  if (!on_device) {
    std::vector<int64_t> h(row_ptr, row_ptr + count);
    e = hipMemcpyAsync(d_row, h.data(), sizeof(int64_t) * count, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);  // h is read by the copy
  } else {
    int32_t* tmp = nullptr;
    e = hipMallocAsync(reinterpret_cast<void**>(&tmp), sizeof(int32_t) * count, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(tmp, row_ptr, sizeof(int32_t) * count, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(widen_i32_kernel, dim3(div_up(int64_t(count), 256)), dim3(256), 0, stream,
                         tmp, d_row, int64_t(count));
      e = hipStreamSynchronize(stream);
    }
    if (tmp) (void)hipFreeAsync(tmp, stream);
  }
  if (e != hipSuccess) return hip_fail(e, "copying row_ptr");
  return LAYOUT_OK;
}

int snap::upload_weights_and_build_alias(hipStream_t stream, const int64_t* d_row,
                                         const uint32_t* weights, int32_t n, bool on_device,
                                         uint32_t* d_thr, uint32_t* d_alias) {
  std::vector<uint32_t> w(static_cast<size_t>(n));
  hipError_t e = hipSuccess;
  if (on_device)
    e = hipMemcpy(w.data(), weights, sizeof(uint32_t) * size_t(n), hipMemcpyDeviceToHost);
  else
    std::memcpy(w.data(), weights, sizeof(uint32_t) * size_t(n));
  if (e != hipSuccess) return hip_fail(e, "reading neg_weight_values");
  int64_t W = 0;
  for (uint32_t x : w) W += x;
  if (W <= 0 || W >= (int64_t(1) << 32))
    return fail(LAYOUT_E_INVALID_ARG, "negative weights sum to %lld (need 0 < W < 2^32)",
                (long long)W);
  uint32_t* d_w = nullptr;
  e = hipMallocAsync(reinterpret_cast<void**>(&d_w), sizeof(uint32_t) * size_t(n), stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_w, w.data(), sizeof(uint32_t) * size_t(n), hipMemcpyHostToDevice, stream);
  int rc = LAYOUT_OK;
  if (e == hipSuccess) rc = build_alias_table(stream, d_row, d_w, n, W, d_thr, d_alias);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (d_w) (void)hipFreeAsync(d_w, stream);
  if (e != hipSuccess) return hip_fail(e, "building the weighted alias table");
  return rc;
}

int snap::lds_bytes_for(int32_t n, int dim) { return std::max(16, n * (dim == 3 ? 16 : 8)); }

int snap::global_grid(const GlobalGroup& g) {
  if (g.grid > 0) return g.grid;
  int per_cu = 0;
  with_k(g.k, [&](auto kc) -> int {
    constexpr int K = decltype(kc)::value;
    return with_degree(g.degree, [&](auto dc) -> int {
      constexpr bool DEG = decltype(dc)::value;
      return with_mode(g.mode, [&](auto mc) -> int {
        constexpr int MODE = decltype(mc)::value;
        const void* fn = reinterpret_cast<const void*>(&epoch_global_kernel<K, MODE, DEG>);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, g.block, 0) != hipSuccess)
          per_cu = 0;
        return LAYOUT_OK;
      });
    });
  });
  if (per_cu <= 0) per_cu = 4;
  per_cu = std::min(per_cu, std::max(1, kLanesPerCU / g.block));
  int64_t want = std::max<int64_t>(1, div_up(g.total_chunks, g.block));
  if (g.max_lanes > 0) want = std::min(want, std::max<int64_t>(1, div_up(g.max_lanes, g.block)));
  return static_cast<int>(std::min<int64_t>(want, int64_t(per_cu) * device_props().cus));
}

int64_t snap::lane_caps(const std::vector<GraphDesc>& table, int nodes_per_lane) {
  const int npl = nodes_per_lane > 0 ? nodes_per_lane : kNodesPerLane;
  int64_t total = 0;
  for (const GraphDesc& d : table)
    total += div_up(std::max<int64_t>(1, std::min<int64_t>(d.n / npl, d.n_chunks)), 64) * 64;
  return total;
}

void snap::plan_lanes(std::vector<GraphDesc>& table, GlobalGroup& g, int64_t lanes,
                      int nodes_per_lane) {
  const int npl = nodes_per_lane > 0 ? nodes_per_lane : kNodesPerLane;
  const int64_t G = static_cast<int64_t>(table.size());
  std::vector<int64_t> cap(table.size());
  int64_t chunks = 0, padded = 0;
  for (size_t q = 0; q < table.size(); ++q) {
    cap[q] = std::max<int64_t>(1, std::min<int64_t>(table[q].n / npl, table[q].n_chunks));
    chunks += table[q].n_chunks;
    padded += div_up(cap[q], 64) * 64;
  }
  // Each graph's lanes start on a wavefront boundary, so that no wavefront
  // mixes two graphs (its lanes would run at the pace of the other graph's
  // chunks).  Every graph gets its cap when the caps fit the launch.
  // Otherwise the lanes go in proportion to the graphs' chunks, none beyond
  // its cap (slice = min(cap, lambda * chunks), lambda found by bisection),
  // so that the uncapped graphs end their epochs together and no lane idles
  // while work is left; a wavefront per graph is kept aside for the padding.
  std::vector<int64_t> slice(cap);
  if (padded > lanes) {
    const double target = double(std::max<int64_t>(0, lanes - 64 * G));
    auto used = [&](double lam) {
      double u = 0.0;
      for (size_t q = 0; q < table.size(); ++q)
        u += std::min(double(cap[q]), lam * double(table[q].n_chunks));
      return u;
    };
    double lo = 0.0, hi = 1.0;
    while (used(hi) < target && hi < 1e18) hi *= 2.0;
    for (int it = 0; it < 80; ++it) {
      const double mid = 0.5 * (lo + hi);
      (used(mid) <= target ? lo : hi) = mid;
    }
    for (size_t q = 0; q < table.size(); ++q)
      slice[q] = std::max<int64_t>(
          1, static_cast<int64_t>(std::min(double(cap[q]), lo * double(table[q].n_chunks))));
  }
  int64_t base = 0;
  for (size_t q = 0; q < table.size(); ++q) {
    base = div_up(base, 64) * 64;
    table[q].chunk_base = base;
    table[q].slice = slice[q];
    base += slice[q];
  }
  g.total_chunks = chunks;
  g.total_index = base;  // lanes handed out; a launch must cover them
  g.round_size = 0;
}

int64_t snap::fair_lanes(const std::vector<GraphDesc>& table, int nodes_per_lane) {
  const int npl = nodes_per_lane > 0 ? nodes_per_lane : kNodesPerLane;
  int64_t total = 0;
  for (const GraphDesc& d : table) total += d.n_chunks;
  double best = -1.0;
  for (const GraphDesc& d : table) {
    if (d.n_chunks <= 0) continue;
    const double cap = double(d.n) / npl * double(total) / double(d.n_chunks);
    if (best < 0 || cap < best) best = cap;
  }
  return best < 1.0 ? 1 : static_cast<int64_t>(best);
}

int snap::plan_xcd_bins(const std::vector<GraphDesc>& graphs, int nodes_per_lane,
                        std::vector<GraphDesc>& table, std::vector<XcdSeg>& segs, XcdBin* bins) {
  table.clear();
  segs.clear();
  std::vector<std::vector<int>> members(kXcds);
  {
    // longest-processing-time assignment by edges: biggest graph first, each
    // to the least loaded bin
    std::vector<int> order(graphs.size());
    for (size_t q = 0; q < graphs.size(); ++q) order[q] = static_cast<int>(q);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return graphs[a].nnz > graphs[b].nnz; });
    int64_t load[kXcds] = {0};
    for (int q : order) {
      int x = 0;
      for (int y = 1; y < kXcds; ++y)
        if (load[y] < load[x]) x = y;
      members[x].push_back(q);
      load[x] += graphs[q].nnz;
    }
  }
  const int cus_per_xcd = std::max(1, device_props().cus / kXcds);
  int grid = 0;
  for (int x = 0; x < kXcds; ++x) {
    XcdBin& b = bins[x];
    b = XcdBin{};
    b.seg_begin = static_cast<int32_t>(segs.size());
    // sequence segments whose positions fit the L2 together
    std::vector<std::vector<int>> parts;
    int64_t bytes = 0;
    for (int q : members[x]) {
      const int64_t need = int64_t(graphs[q].n) * 8;
      if (parts.empty() || bytes + need > kXcdMaxPositionBytes) {
        parts.emplace_back();
        bytes = 0;
      }
      parts.back().push_back(q);
      bytes += need;
    }
    for (const auto& part : parts) {
      // workers: the segment's lane cap, at most one workgroup per CU
      std::vector<GraphDesc> sub;
      for (int q : part) sub.push_back(graphs[q]);
      const int64_t cap = fair_lanes(sub, nodes_per_lane);
      XcdSeg sg{};
      sg.workers = static_cast<int32_t>(
          std::min<int64_t>(cus_per_xcd, std::max<int64_t>(1, div_up(cap, 256))));
      sg.table_begin = static_cast<int32_t>(table.size());
      sg.G = static_cast<int32_t>(part.size());
      int64_t total = 0;
      for (int q : part) total += graphs[q].n_chunks;
      const int64_t rounds = std::max<int64_t>(1, div_up(2 * total, int64_t(sg.workers) * 256));
      int64_t base = 0;
      for (int q : part) {
        GraphDesc d = graphs[q];
        d.slice = div_up(d.n_chunks, rounds);
        d.chunk_base = base;
        base += d.slice;
        table.push_back(d);
      }
      sg.round_size = std::max<int64_t>(1, base);
      sg.total_index = rounds * sg.round_size;
      segs.push_back(sg);
      b.workers = std::max(b.workers, sg.workers);
    }
    b.seg_count = static_cast<int32_t>(segs.size()) - b.seg_begin;
    grid = std::max(grid, b.workers);
  }
  return grid * kXcds;
}

void snap::launch_fill_i32(hipStream_t stream, int32_t* p, int64_t n, int32_t v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(div_up(n, 256)), dim3(256), 0, stream, p, n, v);
}

int snap::launch_xcd_group_epochs(hipStream_t stream, const XcdGroup& g, int32_t dt,
                                  int32_t count) {
  if (g.total_chunks == 0 || count <= 0 || g.grid <= 0) return LAYOUT_OK;
  return with_k(g.k, [&](auto kc) -> int {
    constexpr int K = decltype(kc)::value;
    return with_degree(g.degree, [&](auto dc) -> int {
      constexpr bool DEG = decltype(dc)::value;
      for (int32_t ep = 0; ep < count; ++ep) {
        hipLaunchKernelGGL((epoch_xcd_group_kernel<K, DEG, false>), dim3(g.grid), dim3(256), 0,
                           stream, g.d_table, g.d_segs, g.n_segs, g.d_bins, g.d_counters, dt + ep);
        hipLaunchKernelGGL((epoch_xcd_group_kernel<K, DEG, true>), dim3(kXcds), dim3(256), 0,
                           stream, g.d_table, g.d_segs, g.n_segs, g.d_bins, g.d_counters, dt + ep);
      }
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "epoch_xcd_group_kernel launch");
      return LAYOUT_OK;
    });
  });
}

int snap::launch_global_epochs(hipStream_t stream, const GlobalGroup& g, int32_t dt,
                               int32_t count) {
  if (g.total_chunks == 0 || count <= 0) return LAYOUT_OK;
  const int grid = global_grid(g);
  return with_k(g.k, [&](auto kc) -> int {
    constexpr int K = decltype(kc)::value;
    return with_degree(g.degree, [&](auto dc) -> int {
      constexpr bool DEG = decltype(dc)::value;
      return with_mode(g.mode, [&](auto mc) -> int {
        constexpr int MODE = decltype(mc)::value;
        if (g.dim == 3 && g.G != 1)
          return fail(LAYOUT_E_UNSUPPORTED, "3D layouts run one graph per launch");
        return with_dim(g.dim, [&](auto dmc) -> int {
          constexpr int DIM = decltype(dmc)::value;
          using P = Pos<DIM>;
          // several graphs: the lanes their table hands out (plan_lanes);
          // one graph: its table entry bounds its own lanes
          const int64_t lanes_used = g.G > 1 ? g.total_index : int64_t(grid) * g.block;
          for (int32_t ep = 0; ep < count; ++ep) {
            hipLaunchKernelGGL((epoch_global_kernel<K, MODE, DEG, GlobalMem, DIM>), dim3(grid),
                               dim3(g.block), 0, stream, g.d_table, g.G, lanes_used, dt + ep);
            // JACOBI: apply after every epoch when the group owns one contiguous
            // Y/D (a caller that applies per graph itself passes no nodes)
            if constexpr (MODE == kJacobi) {
              if (g.jacobi_nodes > 0)
                hipLaunchKernelGGL(jacobi_apply_kernel<P>, dim3(div_up(g.jacobi_nodes, 256)),
                                   dim3(256), 0, stream, reinterpret_cast<P*>(g.jacobi_Y),
                                   reinterpret_cast<P*>(g.jacobi_D), g.jacobi_nodes);
            }
          }
          hipError_t e = hipGetLastError();
          if (e != hipSuccess) return hip_fail(e, "epoch_global_kernel launch");
          return LAYOUT_OK;
        });
      });
    });
  });
}

int snap::launch_lds_epochs(hipStream_t stream, const LdsGroup& g, int32_t dt, int32_t count) {
  if (g.blocks == 0 || count <= 0) return LAYOUT_OK;
  return with_k(g.k, [&](auto kc) -> int {
    constexpr int K = decltype(kc)::value;
    return with_degree(g.degree, [&](auto dc) -> int {
      constexpr bool DEG = decltype(dc)::value;
      return with_mode(g.mode, [&](auto mc) -> int {
        constexpr int MODE = decltype(mc)::value;
        if constexpr (MODE == kJacobi) {
          return fail(LAYOUT_E_UNSUPPORTED, "LDS engine has no Jacobi mode");
        } else {
          return with_dim(g.dim, [&](auto dmc) -> int {
            constexpr int DIM = decltype(dmc)::value;
            hipLaunchKernelGGL((epoch_lds_kernel<K, MODE, DEG, DIM>), dim3(g.blocks),
                               dim3(g.block), g.lds_bytes, stream, g.d_table, g.d_ids, dt, count);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return hip_fail(e, "epoch_lds_kernel launch");
            return LAYOUT_OK;
          });
        }
      });
    });
  });
}

int snap::allow_lds(int k, int bytes, int dim) {
  if (bytes <= 65536) return LAYOUT_OK;
  return with_k(k, [&](auto kc) -> int {
    constexpr int K = decltype(kc)::value;
    return with_dim(dim, [&](auto dmc) -> int {
      constexpr int D = decltype(dmc)::value;
      const void* fns[] = {
          reinterpret_cast<const void*>(&epoch_lds_kernel<K, kStore, false, D>),
          reinterpret_cast<const void*>(&epoch_lds_kernel<K, kAtomic, false, D>),
          reinterpret_cast<const void*>(&epoch_lds_kernel<K, kStore, true, D>),
          reinterpret_cast<const void*>(&epoch_lds_kernel<K, kAtomic, true, D>)};
      for (const void* fn : fns) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return hip_fail(e, "raising the LDS limit");
      }
      return LAYOUT_OK;
    });
  });
}

int snap::validate_csr(hipStream_t stream, const int64_t* d_row, const int32_t* d_col, int32_t n,
                       int64_t nnz, uint32_t* d_err) {
  hipError_t e = hipMemsetAsync(d_err, 0, sizeof(uint32_t), stream);
  if (e != hipSuccess) return hip_fail(e, "clearing the validation flag");
  hipLaunchKernelGGL(validate_rows_kernel, dim3(div_up(int64_t(n) + 1, 256)), dim3(256), 0,
                     stream, d_row, n, nnz, d_err);
  uint32_t err = 0;
  e = hipMemcpyAsync(&err, d_err, sizeof err, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "validating row_ptr");
  if (err)
    return fail(LAYOUT_E_BAD_GRAPH, "row_ptr invalid (flags 0x%x: %s%s%s)", err,
                (err & kErrRowStart) ? "row_ptr[0] != 0 " : "",
                (err & kErrRowOrder) ? "decreasing " : "",
                (err & kErrRowEnd) ? "row_ptr[n] != nnz" : "");
  if (nnz == 0) return LAYOUT_OK;
  hipLaunchKernelGGL(validate_edges_kernel, dim3(div_up(nnz, 256)), dim3(256), 0, stream, d_row,
                     d_col, n, nnz, d_err);
  e = hipMemcpyAsync(&err, d_err, sizeof err, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "validating col");
  if (err)
    return fail(LAYOUT_E_BAD_GRAPH, "CSR invalid (flags 0x%x: %s%s%s%s)", err,
                (err & kErrColRange) ? "column out of range " : "",
                (err & kErrSelfLoop) ? "self-loop " : "",
                (err & kErrUnsorted) ? "unsorted or duplicate row entries " : "",
                (err & kErrAsymmetric) ? "missing reverse edge" : "");
  return LAYOUT_OK;
}

void snap::launch_init_positions(hipStream_t stream, float2* d_Y, int32_t n, uint64_t seed,
                                 int dim) {
  if (n <= 0) return;
  const float scale = std::sqrt(static_cast<float>(n));
  if (dim == 3)
    hipLaunchKernelGGL(init_positions3_kernel, dim3(div_up(n, 256)), dim3(256), 0, stream,
                       reinterpret_cast<float4*>(d_Y), n, seed, scale);
  else
    hipLaunchKernelGGL(init_positions_kernel, dim3(div_up(n, 256)), dim3(256), 0, stream, d_Y,
                       n, seed, scale);
}

int snap::launch_dump_draws(hipStream_t stream, int k, bool degree, const GraphDesc& g, int32_t t,
                            int32_t* d_out) {
  if (g.nnz == 0 || k == 0) return LAYOUT_OK;
  return with_k(k, [&](auto kc) -> int {
    constexpr int K = decltype(kc)::value;
    return with_degree(degree, [&](auto dc) -> int {
      constexpr bool DEG = decltype(dc)::value;
      hipLaunchKernelGGL((dump_draws_kernel<K, DEG>), dim3(div_up(g.nnz, 256)), dim3(256), 0,
                         stream, g, t, d_out);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "dump_draws_kernel launch");
      return LAYOUT_OK;
    });
  });
}

void snap::launch_fill_zero(hipStream_t stream, float2* d_p, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(div_up(n, 256)), dim3(256), 0, stream, d_p, n);
}

int snap::silhouette_input(const int32_t* labels, int32_t n, const double* si_out,
                           SilhouetteInput& in) {
  if (!labels || !si_out) return fail(LAYOUT_E_INVALID_ARG, "NULL labels or si_out");
  if (n < 2) return fail(LAYOUT_E_INVALID_ARG, "silhouette needs at least 2 nodes");
  std::vector<int32_t> lv(labels, labels + n);
  std::vector<int32_t> uniq(lv);
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  in.C = static_cast<int32_t>(uniq.size());
  if (in.C < 2) return fail(LAYOUT_E_INVALID_ARG, "silhouette needs at least 2 clusters");
  std::vector<int32_t> cid(n);
  in.cstart.assign(size_t(in.C) + 1, 0);
  in.order.resize(n);
  in.cs.resize(n);
  for (int32_t v = 0; v < n; ++v) {
    cid[v] = static_cast<int32_t>(std::lower_bound(uniq.begin(), uniq.end(), lv[v]) - uniq.begin());
    ++in.cstart[size_t(cid[v]) + 1];
  }
  for (int32_t c = 0; c < in.C; ++c) in.cstart[size_t(c) + 1] += in.cstart[c];
  std::vector<int32_t> fill(in.cstart.begin(), in.cstart.end() - 1);
  for (int32_t v = 0; v < n; ++v) {
    const int32_t q = fill[cid[v]]++;
    in.order[q] = v;
    in.cs[q] = cid[v];
  }
  return LAYOUT_OK;
}

namespace {
static __global__ void zero_f64_kernel(double* __restrict__ p, int32_t count) {
  const int32_t i = int32_t(blockIdx.x) * blockDim.x + int32_t(threadIdx.x);
  if (i < count) p[i] = 0.0;
}
}  // namespace

int snap::silhouette_run(hipStream_t stream, const float2* d_Y, int32_t n,
                         const SilhouetteInput& in, const SilhouetteBuffers& b, double* si_out) {
  hipError_t e = hipMemcpyAsync(b.order, in.order.data(), sizeof(int32_t) * size_t(n),
                                hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b.cs, in.cs.data(), sizeof(int32_t) * size_t(n), hipMemcpyHostToDevice,
                       stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b.cstart, in.cstart.data(), sizeof(int32_t) * (size_t(in.C) + 1),
                       hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) {
    // cleared by a kernel rather than a memset node, so that the sequence may
    // sit in a captured graph
    hipLaunchKernelGGL(zero_f64_kernel, dim3(1), dim3(64), 0, stream, b.acc, 2);
    const int grid = static_cast<int>(div_up(n, 256));
    hipLaunchKernelGGL(gather_positions_kernel, dim3(grid), dim3(256), 0, stream, d_Y, b.order, n,
                       b.Ys);
    hipLaunchKernelGGL(silhouette_kernel, dim3(grid), dim3(256), 0, stream, b.Ys, b.cs, b.cstart,
                       n, b.acc);
    e = hipGetLastError();
  }
  double out[2] = {0.0, 0.0};
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, b.acc, 2 * sizeof(double), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "silhouette");
  *si_out = out[0] / double(n);
  return LAYOUT_OK;
}

void snap::launch_jacobi_apply(hipStream_t stream, float2* d_Y, float2* d_D, int32_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(jacobi_apply_kernel<float2>, dim3(div_up(n, 256)), dim3(256), 0, stream, d_Y,
                     d_D, n);
}

namespace {

bool check_handle(const layout_t* L) {
  if (!L) {
    fail(LAYOUT_E_INVALID_ARG, "null layout handle");
    return false;
  }
  return true;
}

}  // namespace

int snap::handle_view(const layout_t* L, HandleView* v) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  v->n = L->n;
  v->dim = L->dim;
  v->dev = L->dev;
  v->stream = L->stream;
  v->Y = L->host_desc.Y;
  return LAYOUT_OK;
}

// --------------------------------------------------------------------- ABI
// ---------------------------------------------------------- energy monitors
namespace {

int energy_buffer(layout_t* L) {
  if (L->d_energy) return LAYOUT_OK;
  return alloc(L, reinterpret_cast<void**>(&L->d_energy), 2 * sizeof(double),
               "energy accumulators");
}

// out[0] = attraction over the directed edges, out[1] = repulsion shape over
// the negatives of epoch t (K = 0 when with_rep is false).
int launch_sampled_energy(layout_t* L, int32_t t, bool with_rep) {
  if (L->n_chunks == 0) return LAYOUT_OK;
  const int64_t want = div_up(L->n_chunks, 256);
  const int grid = static_cast<int>(std::min<int64_t>(want, 4096));
  const int k = with_rep ? L->k : 0;
  return with_k(k, [&](auto kc) -> int {
    constexpr int K = decltype(kc)::value;
    return with_degree(L->opts.neg_weights != LAYOUT_NEG_UNIFORM, [&](auto dc) -> int {
      constexpr bool DEG = decltype(dc)::value;
      hipLaunchKernelGGL((sampled_energy_kernel<K, DEG>), dim3(grid), dim3(256), 0, L->stream,
                         L->d_table, L->n_chunks, t, L->d_energy);
      return LAYOUT_OK;
    });
  });
}

int read_energy(layout_t* L, double* out) {
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, L->d_energy, 2 * sizeof(double), hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "energy monitor");
  return LAYOUT_OK;
}

// 3D positions are 16-byte (x, y, z, w) on the device and rows of 3 floats
// in the caller's host arrays.  A strided copy between device and pageable
// host memory with 12-byte rows moves one row at a time (minutes for
// millions of nodes), so host transfers move whole 16-byte positions
// through a host buffer of n float4 and repack there.
int read_positions3(hipStream_t s, const float2* d_Y, int32_t n, float* host_out) {
  std::unique_ptr<float4[]> tmp(new (std::nothrow) float4[size_t(n)]);
  if (!tmp) return fail(LAYOUT_E_OOM, "host buffer for %d positions", n);
  hipError_t e = hipMemcpyAsync(tmp.get(), d_Y, sizeof(float4) * size_t(n),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "reading positions");
  for (size_t i = 0; i < size_t(n); ++i) {
    host_out[3 * i] = tmp[i].x;
    host_out[3 * i + 1] = tmp[i].y;
    host_out[3 * i + 2] = tmp[i].z;
  }
  return LAYOUT_OK;
}

int write_positions3(hipStream_t s, const float* host_in, int32_t n, float2* d_Y) {
  std::unique_ptr<float4[]> tmp(new (std::nothrow) float4[size_t(n)]);
  if (!tmp) return fail(LAYOUT_E_OOM, "host buffer for %d positions", n);
  for (size_t i = 0; i < size_t(n); ++i)
    tmp[i] = make_float4(host_in[3 * i], host_in[3 * i + 1], host_in[3 * i + 2], 0.0f);
  hipError_t e = hipMemcpyAsync(d_Y, tmp.get(), sizeof(float4) * size_t(n),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "writing positions");
  return LAYOUT_OK;
}

}  // namespace

extern "C" {

const char* layout_last_error(void) { return g_last_error.c_str(); }

void layout_opts_init(layout_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->alpha = 0.1f;
  o->beta = 8.0f;
  o->gamma = 2.0f;
  o->eta0 = 1.0f;
  o->update_mode = LAYOUT_UPDATE_AUTO;
  o->neg_weights = LAYOUT_NEG_UNIFORM;
  o->engine = LAYOUT_ENGINE_AUTO;
}

int layout_create(const int32_t* row_ptr, const int32_t* col_idx, int32_t n, int32_t dim,
                  int32_t k, int32_t epochs, uint64_t seed, layout_t** out) {
  layout_opts o;
  layout_opts_init(&o);
  return layout_create_ex(row_ptr, col_idx, n, dim, k, epochs, seed, &o, 0, out);
}

namespace {

// Both row_ptr widths: row32 (int32 CSR) or row64 (int64 row pointers), one
// of them non-null.
int create_impl(const int32_t* row32, const int64_t* row64, const int32_t* col_idx, int32_t n,
                int32_t dim, int32_t k, int32_t epochs, uint64_t seed, const layout_opts* opts,
                int32_t inputs_on_device, layout_t** out) {
  const void* row_ptr = row32 ? static_cast<const void*>(row32) : static_cast<const void*>(row64);
  g_last_error.clear();
  if (!out) return fail(LAYOUT_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (dim != 2 && dim != 3) return fail(LAYOUT_E_UNSUPPORTED, "dim = %d (2 or 3)", dim);
  if (n < 0) return fail(LAYOUT_E_INVALID_ARG, "n = %d", n);
  if (k < 0 || k > 8) return fail(k < 0 ? LAYOUT_E_INVALID_ARG : LAYOUT_E_UNSUPPORTED,
                                  "k = %d (0..8 supported)", k);
  if (epochs < 1) return fail(LAYOUT_E_INVALID_ARG, "epochs = %d", epochs);
  if (!row_ptr) return fail(LAYOUT_E_INVALID_ARG, "row_ptr is NULL");
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
  if (o.neg_weights == LAYOUT_NEG_CUSTOM && n > 0 && !o.neg_weight_values)
    return fail(LAYOUT_E_INVALID_ARG, "LAYOUT_NEG_CUSTOM needs neg_weight_values");
  if (o.start_epoch < 0 || o.start_epoch > epochs)
    return fail(LAYOUT_E_INVALID_ARG, "start_epoch = %d", o.start_epoch);
  if (o.engine < 0 || o.engine > 3) return fail(LAYOUT_E_INVALID_ARG, "engine = %d", o.engine);
  if (o.init_mode != LAYOUT_INIT_UNIFORM && o.init_mode != LAYOUT_INIT_PMDS)
    return fail(LAYOUT_E_INVALID_ARG, "init_mode = %d", o.init_mode);
  if (dim == 3 && int64_t(n) * 16 > int64_t(0xFFFFFFFF))
    return fail(LAYOUT_E_UNSUPPORTED, "3D layouts address positions by 32-bit offsets: n < 2^28");
  if (dim == 3 && o.init_mode == LAYOUT_INIT_PMDS && !o.init_pos)
    return fail(LAYOUT_E_UNSUPPORTED, "the Pivot MDS start is 2D");
  if (o.pmds_pivots < 0 || o.pmds_pivots > 64)
    return fail(LAYOUT_E_INVALID_ARG, "pmds_pivots = %d (1..64, 0 = default)", o.pmds_pivots);
  if (o.hot_degree < 0) return fail(LAYOUT_E_INVALID_ARG, "hot_degree = %d (>= 0)", o.hot_degree);
  if (o.bundle_edges < 0 || o.block_threads < 0 || o.grid_blocks < 0 || o.hub_split_edges < 0 ||
      o.nodes_per_lane < 0)
    return fail(LAYOUT_E_INVALID_ARG, "negative launch option");
  if (o.block_threads > 1024 || (o.block_threads % 64) != 0)
    return fail(LAYOUT_E_INVALID_ARG, "block_threads = %d (multiple of 64, <= 1024)",
                o.block_threads);
  if (o.force_kernel != LAYOUT_FORCE_T && o.force_kernel != LAYOUT_FORCE_GAUSSIAN)
    return fail(LAYOUT_E_INVALID_ARG, "force_kernel = %d", o.force_kernel);
  if (!(o.gamma > (o.force_kernel == LAYOUT_FORCE_T ? 1.0f : 0.0f)))
    return fail(LAYOUT_E_INVALID_ARG, "gamma = %g (must be > 1, > 0 for Gaussian forces)",
                o.gamma);
  // degree-weighted negatives: the alias table's bin capacity W = nnz must stay
  // below 2^32 (checked here for host inputs, before any device work; device
  // inputs are checked when the table is built)
  if (!inputs_on_device && o.neg_weights == LAYOUT_NEG_DEGREE && n > 0) {
    const int64_t nnz_host = row32 ? int64_t(row32[n]) : row64[n];
    if (nnz_host >= (int64_t(1) << 32))
      return fail(LAYOUT_E_UNSUPPORTED,
                  "degree-weighted negatives need nnz < 2^32 (nnz = %lld)", (long long)nnz_host);
  }

  layout_t* L = new (std::nothrow) layout_t();
  if (!L) return fail(LAYOUT_E_OOM, "host allocation");
  L->n = n;
  L->dim = dim;
  L->k = k;
  L->epochs = epochs;
  L->t = o.start_epoch;
  L->seed = seed;
  L->opts = o;
  (void)hipGetDevice(&L->dev);

  auto bail = [&](int rc) {
    layout_destroy(L);
    return rc;
  };

  if (o.stream) {
    L->stream = static_cast<hipStream_t>(o.stream);
  } else {
    hipError_t e = hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(hip_fail(e, "hipStreamCreate"));
    L->own_stream = true;
  }

  // nnz from row_ptr[n]
  int64_t nnz = 0;
  if (inputs_on_device) {
    int32_t last32 = 0;
    hipError_t e = row32 ? hipMemcpy(&last32, row32 + n, sizeof(int32_t), hipMemcpyDeviceToHost)
                         : hipMemcpy(&nnz, row64 + n, sizeof(int64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return bail(hip_fail(e, "reading row_ptr[n]"));
    if (row32) nnz = last32;
  } else {
    nnz = row32 ? int64_t(row32[n]) : row64[n];
  }
  if (nnz < 0) return bail(fail(LAYOUT_E_BAD_GRAPH, "row_ptr[n] = %lld", (long long)nnz));
  if (nnz > 0 && !col_idx) return bail(fail(LAYOUT_E_INVALID_ARG, "col_idx is NULL"));
  L->nnz = nnz;

  // engine and launch shape
  const DeviceProps& dp = device_props();
  const int64_t pos_bytes = dim == 3 ? 16 : 8;  // one position
  const bool lds_fits = lds_bytes_for(n, dim) <= dp.lds_per_block;
  if (o.engine == LAYOUT_ENGINE_LDS) {
    if (!lds_fits)
      return bail(fail(LAYOUT_E_UNSUPPORTED, "LDS engine: %d nodes need %d B of LDS (> %d)", n,
                       lds_bytes_for(n, dim), dp.lds_per_block));
    if (o.update_mode == LAYOUT_JACOBI)
      return bail(fail(LAYOUT_E_UNSUPPORTED, "LDS engine has no Jacobi mode"));
    L->engine = LAYOUT_ENGINE_LDS;
  } else if (o.engine == LAYOUT_ENGINE_GLOBAL) {
    L->engine = LAYOUT_ENGINE_GLOBAL;
  } else if (o.engine == LAYOUT_ENGINE_XCD) {
    if (int64_t(n) * pos_bytes > kXcdMaxPositionBytes)
      return bail(fail(LAYOUT_E_UNSUPPORTED, "XCD-local engine: %d nodes need %lld B (> %lld)", n,
                       (long long)(n * pos_bytes), (long long)kXcdMaxPositionBytes));
    if (o.update_mode != LAYOUT_UPDATE_AUTO && o.update_mode != LAYOUT_HOGWILD_STORE)
      return bail(fail(LAYOUT_E_UNSUPPORTED, "XCD-local engine runs HOGWILD_STORE only"));
    L->engine = LAYOUT_ENGINE_XCD;
  } else {
    const bool store_ok = o.update_mode == LAYOUT_UPDATE_AUTO || o.update_mode == LAYOUT_HOGWILD_STORE;
    if (lds_fits && L->nnz <= kLdsAutoMaxEdges && o.update_mode != LAYOUT_JACOBI)
      L->engine = LAYOUT_ENGINE_LDS;
    else if (store_ok && int64_t(n) * pos_bytes <= kXcdMaxPositionBytes)
      L->engine = LAYOUT_ENGINE_XCD;
    else
      L->engine = LAYOUT_ENGINE_GLOBAL;
  }
  if (L->engine == LAYOUT_ENGINE_LDS) {
    L->block = o.block_threads ? o.block_threads : lds_lanes_for(n, o.nodes_per_lane);
    // enough chunks to keep every lane busy, each as long as possible
    const int64_t per_lane = std::max<int64_t>(1, L->nnz / (4 * L->block));
    L->bundle = o.bundle_edges ? o.bundle_edges : static_cast<int32_t>(std::min<int64_t>(16, per_lane));
    L->hub = o.hub_split_edges ? o.hub_split_edges : kLdsHub;
  } else {
    // a whole workgroup works on the graph, so small graphs get small
    // workgroups: n / nodes_per_lane lanes rounded up to whole wavefronts
    const int npl = o.nodes_per_lane > 0 ? o.nodes_per_lane : kNodesPerLane;
    const int64_t want = div_up(std::max<int64_t>(1, n / npl), 64) * 64;
    L->block = o.block_threads ? o.block_threads : static_cast<int32_t>(std::min<int64_t>(256, want));
    L->bundle = o.bundle_edges ? o.bundle_edges : kDefaultBundle;
    L->hub = o.hub_split_edges ? o.hub_split_edges : kHubFactor * L->bundle;
  }
  L->mode = o.update_mode != LAYOUT_UPDATE_AUTO
                ? o.update_mode
                : (L->engine == LAYOUT_ENGINE_LDS ? LAYOUT_ATOMIC : LAYOUT_HOGWILD_STORE);
  if ((L->engine == LAYOUT_ENGINE_GLOBAL || L->engine == LAYOUT_ENGINE_XCD) && L->block > 256)
    return bail(fail(LAYOUT_E_UNSUPPORTED, "global engines run at most 256-thread workgroups"));
  const int64_t chunk_cap = L->nnz > 0 ? chunk_bound(L->nnz, L->bundle, L->hub) : 0;
  if (chunk_cap > kMaxChunks)
    return bail(fail(LAYOUT_E_UNSUPPORTED,
                     "%lld edges in chunks of %d (hub rows cut every %d) need more than %lld chunks: "
                     "raise bundle_edges and hub_split_edges",
                     static_cast<long long>(L->nnz), L->bundle, L->hub,
                     static_cast<long long>(kMaxChunks)));

  // device buffers
  int rc;
  int64_t* d_row = nullptr;
  int32_t* d_col = nullptr;
  int32_t* d_chunk = nullptr;
  int64_t* d_chunk_begin = nullptr;
  float2* d_Y = nullptr;
  float2* d_D = nullptr;
  uint32_t* d_err = nullptr;
  if ((rc = alloc(L, reinterpret_cast<void**>(&d_row), sizeof(int64_t) * (size_t(n) + 1), "row_ptr")) ||
      (rc = alloc(L, reinterpret_cast<void**>(&d_col), sizeof(int32_t) * size_t(L->nnz), "col")) ||
      (rc = alloc(L, reinterpret_cast<void**>(&d_chunk), sizeof(int32_t) * size_t(chunk_cap), "chunk src")) ||
      (rc = alloc(L, reinterpret_cast<void**>(&d_chunk_begin), sizeof(int64_t) * size_t(chunk_cap + 1), "chunk begin")) ||
      (rc = alloc(L, reinterpret_cast<void**>(&d_Y), size_t(pos_bytes) * size_t(n), "positions")) ||
      (rc = alloc(L, reinterpret_cast<void**>(&d_err), sizeof(uint32_t), "flag")) ||
      (rc = alloc(L, reinterpret_cast<void**>(&L->d_table), sizeof(GraphDesc), "table")) ||
      (rc = alloc(L, reinterpret_cast<void**>(&L->d_graph_ids), sizeof(int32_t), "ids")))
    return bail(rc);
  if (L->mode == LAYOUT_JACOBI &&
      (rc = alloc(L, reinterpret_cast<void**>(&d_D), size_t(pos_bytes) * size_t(n), "jacobi delta")))
    return bail(rc);

  const hipMemcpyKind kind = inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  hipError_t e = hipSuccess;
  if (row32) {
    if ((rc = upload_row_ptr(L->stream, row32, n, inputs_on_device != 0, d_row)) != LAYOUT_OK)
      return bail(rc);
  } else {
    e = hipMemcpyAsync(d_row, row64, sizeof(int64_t) * (size_t(n) + 1), kind, L->stream);
  }
  if (e == hipSuccess && L->nnz > 0)
    e = hipMemcpyAsync(d_col, col_idx, sizeof(int32_t) * size_t(L->nnz), kind, L->stream);
  if (e != hipSuccess) return bail(hip_fail(e, "copying the graph"));

  // validation on the device, then the chunk table
  if ((rc = validate_csr(L->stream, d_row, d_col, n, L->nnz, d_err)) != LAYOUT_OK) return bail(rc);
  if (L->nnz > 0) {
    if ((rc = build_chunk_table(L->stream, d_row, n, L->nnz, L->bundle, L->hub, d_chunk_begin,
                                d_chunk, &L->n_chunks)) != LAYOUT_OK)
      return bail(rc);
  }

  // alias table of weighted negatives: degrees (W = nnz) or the caller's
  // weights (0 < W < 2^32, summed on the host)
  uint32_t* d_thr = nullptr;
  uint32_t* d_alias = nullptr;
  if (o.neg_weights != LAYOUT_NEG_UNIFORM && L->nnz > 0) {
    if ((rc = alloc(L, reinterpret_cast<void**>(&d_thr), sizeof(uint32_t) * size_t(n), "alias thr")) ||
        (rc = alloc(L, reinterpret_cast<void**>(&d_alias), sizeof(uint32_t) * size_t(n), "alias")))
      return bail(rc);
    if (o.neg_weight_values)
      rc = upload_weights_and_build_alias(L->stream, d_row, o.neg_weight_values, n,
                                          inputs_on_device != 0, d_thr, d_alias);
    else
      rc = build_alias_table(L->stream, d_row, nullptr, n, L->nnz, d_thr, d_alias);
    if (rc != LAYOUT_OK) return bail(rc);
  }

  // initial positions
  if (n > 0) {
    if (o.init_pos && dim == 3 && !inputs_on_device) {
      // n x 3 host rows into 16-byte positions (w = 0)
      if ((rc = write_positions3(L->stream, o.init_pos, n, d_Y)) != LAYOUT_OK) return bail(rc);
    } else if (o.init_pos && dim == 3) {
      e = hipMemsetAsync(d_Y, 0, size_t(pos_bytes) * size_t(n), L->stream);
      if (e == hipSuccess)
        e = hipMemcpy2DAsync(d_Y, 16, o.init_pos, 12, 12, size_t(n), kind, L->stream);
      if (e != hipSuccess) return bail(hip_fail(e, "copying init_pos"));
    } else if (o.init_pos) {
      e = hipMemcpyAsync(d_Y, o.init_pos, sizeof(float2) * size_t(n), kind, L->stream);
      if (e != hipSuccess) return bail(hip_fail(e, "copying init_pos"));
    } else if (o.init_mode == LAYOUT_INIT_PMDS) {
      if ((rc = pmds_positions(L->stream, d_row, d_col, n,
                               o.pmds_pivots ? o.pmds_pivots : kDefaultPivots, seed, d_Y,
                               nullptr, nullptr, nullptr)) != LAYOUT_OK)
        return bail(rc);
    } else {
      launch_init_positions(L->stream, d_Y, n, seed, dim);
    }
  }
  if (d_D) launch_fill_zero(L->stream, d_D, int64_t(n) * (pos_bytes / 8));
  // hot nodes: HOGWILD_STORE on the global engine commits updates of
  // high-degree nodes as the far end of an edge as atomic adds
  uint32_t* d_hot = nullptr;
  L->hot_degree = 0;
  if (L->engine == LAYOUT_ENGINE_GLOBAL && L->mode == LAYOUT_HOGWILD_STORE && L->nnz > 0 &&
      o.hot_degree > 0) {
    L->hot_degree = o.hot_degree;
    const int64_t words = (int64_t(n) + 31) / 32;
    if ((rc = alloc(L, reinterpret_cast<void**>(&d_hot), sizeof(uint32_t) * size_t(words),
                    "hot nodes")) != LAYOUT_OK)
      return bail(rc);
    hipLaunchKernelGGL(hot_bits_kernel, dim3(div_up(words, 256)), dim3(256), 0, L->stream, d_row,
                       n, int64_t(L->hot_degree), d_hot);
    if ((e = hipGetLastError()) != hipSuccess) return bail(hip_fail(e, "hot nodes"));
  }
  if (L->engine == LAYOUT_ENGINE_XCD) {
    const size_t b = sizeof(int32_t) * size_t(epochs);
    if ((rc = alloc(L, reinterpret_cast<void**>(&L->d_xcd_owner), b, "epoch owners")) ||
        (rc = alloc(L, reinterpret_cast<void**>(&L->d_xcd_counter), b, "epoch counters")))
      return bail(rc);
    e = hipMemsetAsync(L->d_xcd_owner, 0xFF, b, L->stream);
    if (e == hipSuccess) e = hipMemsetAsync(L->d_xcd_counter, 0, b, L->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "clearing epoch counters"));
  }

  GraphDesc& g = L->host_desc;
  g.row_ptr = d_row;
  g.col = d_col;
  g.chunk_begin = d_chunk_begin;
  g.chunk_src = d_chunk;
  g.Y = d_Y;
  g.D = d_D;
  g.thr = d_thr;
  g.alias = d_alias;
  g.hot = d_hot;
  // the global engine's lanes for this graph: n / nodes_per_lane, or all of
  // an explicit launch (grid_blocks)
  g.chunk_base = 0;
  g.slice = o.grid_blocks > 0
                ? std::max<int64_t>(1, L->n_chunks)
                : std::max<int64_t>(1, n / (o.nodes_per_lane > 0 ? o.nodes_per_lane : kNodesPerLane));
  g.n_chunks = L->n_chunks;
  g.nnz = L->nnz;
  g.n = n;
  g.hub = L->hub;
  g.t0 = 0;
  g.T = epochs;
  g.seed = seed;
  g.eta0 = o.eta0;
  g.alpha = o.alpha;
  g.beta = o.beta;
  g.gamma = o.gamma;
  g.force = o.force_kernel;
  g.sc = sampler_consts(n);
  const int32_t zero = 0;
  e = hipMemcpyAsync(L->d_table, &g, sizeof g, hipMemcpyHostToDevice, L->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(L->d_graph_ids, &zero, sizeof zero, hipMemcpyHostToDevice, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return bail(hip_fail(e, "finishing create"));
  if (L->engine == LAYOUT_ENGINE_LDS &&
      (rc = allow_lds(k, lds_bytes_for(n, dim), dim)) != LAYOUT_OK)
    return bail(rc);
  *out = L;
  return LAYOUT_OK;
}

}  // namespace

int layout_create_ex(const int32_t* row_ptr, const int32_t* col_idx, int32_t n, int32_t dim,
                     int32_t k, int32_t epochs, uint64_t seed, const layout_opts* opts,
                     int32_t inputs_on_device, layout_t** out) {
  if (!row_ptr) return fail(LAYOUT_E_INVALID_ARG, "row_ptr is NULL");
  return create_impl(row_ptr, nullptr, col_idx, n, dim, k, epochs, seed, opts, inputs_on_device,
                     out);
}

int layout_create64(const int64_t* row_ptr, const int32_t* col_idx, int32_t n, int32_t dim,
                    int32_t k, int32_t epochs, uint64_t seed, const layout_opts* opts,
                    int32_t inputs_on_device, layout_t** out) {
  if (!row_ptr) return fail(LAYOUT_E_INVALID_ARG, "row_ptr is NULL");
  return create_impl(nullptr, row_ptr, col_idx, n, dim, k, epochs, seed, opts, inputs_on_device,
                     out);
}

int layout_epoch(layout_t* L, int32_t count) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (count < 0) return fail(LAYOUT_E_INVALID_ARG, "count = %d", count);
  if (L->t >= L->epochs) return fail(LAYOUT_E_DONE, "all %d epochs done", L->epochs);
  const int32_t run = std::min(count, L->epochs - L->t);
  if (run == 0) return LAYOUT_OK;
  const int rc = launch_epochs(L, run);
  if (rc != LAYOUT_OK) return rc;
  L->t += run;
  return LAYOUT_OK;
}

int layout_epoch_timed(layout_t* L, int32_t count, float* ms) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (!ms) return fail(LAYOUT_E_INVALID_ARG, "ms is NULL");
  hipEvent_t a, b;
  hipError_t e = hipEventCreate(&a);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  e = hipEventCreate(&b);
  if (e != hipSuccess) {
    (void)hipEventDestroy(a);
    return hip_fail(e, "hipEventCreate");
  }
  int rc = LAYOUT_OK;
  e = hipEventRecord(a, L->stream);
  if (e == hipSuccess) {
    rc = layout_epoch(L, count);
    if (rc == LAYOUT_OK) {
      e = hipEventRecord(b, L->stream);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != LAYOUT_OK) return rc;
  if (e != hipSuccess) return hip_fail(e, "timing epochs");
  return LAYOUT_OK;
}

int layout_get_positions(const layout_t* L, float* host_out) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (!host_out) return fail(LAYOUT_E_INVALID_ARG, "host_out is NULL");
  if (L->n == 0) return LAYOUT_OK;
  if (L->dim == 3) return read_positions3(L->stream, L->host_desc.Y, L->n, host_out);
  hipError_t e = hipMemcpyAsync(host_out, L->host_desc.Y, sizeof(float2) * size_t(L->n),
                                hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "reading positions");
  return LAYOUT_OK;
}

int layout_get_positions_device(const layout_t* L, float* dev_out, void* stream) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (!dev_out) return fail(LAYOUT_E_INVALID_ARG, "dev_out is NULL");
  if (L->n == 0) return LAYOUT_OK;
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : L->stream;
  hipError_t e = hipSuccess;
  if (s != L->stream) {
    // order the copy after the handle's work
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, L->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
    (void)hipEventDestroy(ev);
  }
  if (e == hipSuccess)
    e = L->dim == 3 ? hipMemcpy2DAsync(dev_out, 12, L->host_desc.Y, 16, 12, size_t(L->n),
                                       hipMemcpyDeviceToDevice, s)
                    : hipMemcpyAsync(dev_out, L->host_desc.Y, sizeof(float2) * size_t(L->n),
                                     hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "copying positions");
  return LAYOUT_OK;
}

int layout_set_positions(layout_t* L, const float* host_in) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (!host_in) return fail(LAYOUT_E_INVALID_ARG, "host_in is NULL");
  if (L->n == 0) return LAYOUT_OK;
  if (L->dim == 3) return write_positions3(L->stream, host_in, L->n, L->host_desc.Y);
  hipError_t e = hipMemcpyAsync(L->host_desc.Y, host_in, sizeof(float2) * size_t(L->n),
                                hipMemcpyHostToDevice, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "writing positions");
  return LAYOUT_OK;
}

int layout_status(const layout_t* L, int32_t* epochs_done, int64_t* device_bytes) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (epochs_done) *epochs_done = L->t;
  if (device_bytes) *device_bytes = static_cast<int64_t>(L->buf.bytes());
  return LAYOUT_OK;
}

int layout_sync(layout_t* L) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  hipError_t e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return LAYOUT_OK;
}

void layout_destroy(layout_t* L) {
  if (!L) return;
  if (L->stream) (void)hipStreamSynchronize(L->stream);
  L->buf.free_all();
  if (L->own_stream && L->stream) (void)hipStreamDestroy(L->stream);
  delete L;
}


int layout_sampled_energy(layout_t* L, int32_t epoch, double* attr_out, double* rep_out) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (L->dim != 2) return fail(LAYOUT_E_UNSUPPORTED, "energy monitors are 2D");
  if (L->opts.force_kernel != LAYOUT_FORCE_T)
    return fail(LAYOUT_E_UNSUPPORTED, "energy monitors take the t-FDP forces");
  if (!attr_out || !rep_out) return fail(LAYOUT_E_INVALID_ARG, "NULL output");
  if (epoch < 0) return fail(LAYOUT_E_INVALID_ARG, "epoch = %d", epoch);
  int rc = energy_buffer(L);
  if (rc != LAYOUT_OK) return rc;
  hipError_t e = hipMemsetAsync(L->d_energy, 0, 2 * sizeof(double), L->stream);
  if (e != hipSuccess) return hip_fail(e, "clearing energy accumulators");
  rc = launch_sampled_energy(L, epoch, true);
  if (rc != LAYOUT_OK) return rc;
  double out[2] = {0.0, 0.0};
  rc = read_energy(L, out);
  if (rc != LAYOUT_OK) return rc;
  *attr_out = out[0];
  *rep_out = out[1] / (2.0 * (double(L->opts.gamma) - 1.0));
  return LAYOUT_OK;
}

int layout_effective_energy(layout_t* L, double* attr_out, double* rep_out) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (L->dim != 2) return fail(LAYOUT_E_UNSUPPORTED, "energy monitors are 2D");
  if (L->opts.force_kernel != LAYOUT_FORCE_T)
    return fail(LAYOUT_E_UNSUPPORTED, "energy monitors take the t-FDP forces");
  if (!attr_out || !rep_out) return fail(LAYOUT_E_INVALID_ARG, "NULL output");
  int rc = energy_buffer(L);
  if (rc != LAYOUT_OK) return rc;
  hipError_t e = hipMemsetAsync(L->d_energy, 0, 2 * sizeof(double), L->stream);
  if (e != hipSuccess) return hip_fail(e, "clearing energy accumulators");
  rc = launch_sampled_energy(L, 0, false);
  if (rc != LAYOUT_OK) return rc;
  if (L->n > 1 && L->k > 0) {
    const int tiles = static_cast<int>(div_up(L->n, 256));
    // enough workgroups to fill the chip when the row tiles are few
    const int ysplit = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(tiles, div_up(2048, tiles))));
    hipLaunchKernelGGL(pair_energy_kernel, dim3(tiles, ysplit), dim3(256), 0, L->stream,
                       L->host_desc.Y, L->host_desc.row_ptr, L->n, L->opts.gamma,
                       L->d_energy);
  }
  double out[2] = {0.0, 0.0};
  rc = read_energy(L, out);
  if (rc != LAYOUT_OK) return rc;
  *attr_out = out[0];
  // ordered pairs count each unordered pair twice
  const double w = L->n > 1 ? double(L->k) / double(L->n - 1) : 0.0;
  *rep_out = w * 0.5 * out[1] / (2.0 * (double(L->opts.gamma) - 1.0));
  return LAYOUT_OK;
}

int layout_silhouette(layout_t* L, const int32_t* labels, double* si_out) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (L->dim != 2) return fail(LAYOUT_E_UNSUPPORTED, "the silhouette monitor is 2D");
  SilhouetteInput in;
  int rc = silhouette_input(labels, L->n, si_out, in);
  if (rc != LAYOUT_OK) return rc;
  rc = energy_buffer(L);
  if (rc != LAYOUT_OK) return rc;
  const int32_t n = L->n;
  SilhouetteBuffers b;
  b.acc = L->d_energy;
  hipError_t e = hipMalloc(&b.order, sizeof(int32_t) * size_t(n));
  if (e == hipSuccess) e = hipMalloc(&b.cs, sizeof(int32_t) * size_t(n));
  if (e == hipSuccess) e = hipMalloc(&b.cstart, sizeof(int32_t) * (size_t(in.C) + 1));
  if (e == hipSuccess) e = hipMalloc(&b.Ys, sizeof(float2) * size_t(n));
  rc = e == hipSuccess ? silhouette_run(L->stream, L->host_desc.Y, n, in, b, si_out)
                       : hip_fail(e, "silhouette buffers");
  if (b.order) (void)hipFree(b.order);
  if (b.cs) (void)hipFree(b.cs);
  if (b.cstart) (void)hipFree(b.cstart);
  if (b.Ys) (void)hipFree(b.Ys);
  return rc;
}

int layout_neighbourhood(layout_t* L, const int32_t* nodes, int32_t count, int32_t radius,
                         int32_t* k_out, int32_t* inter_out, double* np_out) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (L->dim != 2) return fail(LAYOUT_E_UNSUPPORTED, "the NP monitor is 2D");
  if (count < 0) return fail(LAYOUT_E_INVALID_ARG, "count < 0");
  if (radius != 1 && radius != 2) return fail(LAYOUT_E_INVALID_ARG, "radius must be 1 or 2");
  if (count > 0 && (!nodes || !k_out || !inter_out))
    return fail(LAYOUT_E_INVALID_ARG, "NULL nodes, k_out or inter_out");
  for (int32_t a = 0; a < count; ++a)
    if (nodes[a] < 0 || nodes[a] >= L->n)
      return fail(LAYOUT_E_INVALID_ARG, "query node %d out of range [0, %d)", nodes[a], L->n);
  const int rc = neighbourhood_counts(L->stream, L->host_desc.row_ptr, L->host_desc.col,
                                      L->host_desc.Y, L->n, nodes, count, radius, k_out,
                                      inter_out);
  if (rc != LAYOUT_OK) return rc;
  if (np_out) {
    double sum = 0.0;
    int64_t used = 0;
    for (int32_t a = 0; a < count; ++a) {
      if (k_out[a] == 0) continue;
      sum += double(inter_out[a]) / double(2 * int64_t(k_out[a]) - inter_out[a]);
      ++used;
    }
    *np_out = used ? sum / double(used) : 0.0;
  }
  return LAYOUT_OK;
}

int layout_cluster_quality(layout_t* L, const int32_t* labels, int32_t clusters, uint64_t seed,
                           int32_t max_iter, const float* init_centers, double* cq_out,
                           int32_t* assign_out, int32_t* iters_out, int32_t* centers_out) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (L->dim != 2) return fail(LAYOUT_E_UNSUPPORTED, "the CQ monitor is 2D");
  if (!labels || !cq_out) return fail(LAYOUT_E_INVALID_ARG, "NULL labels or cq_out");
  if (L->n < 1) return fail(LAYOUT_E_INVALID_ARG, "CQ needs at least one node");
  if (clusters < 0 || max_iter < 1)
    return fail(LAYOUT_E_INVALID_ARG, "clusters = %d, max_iter = %d", clusters, max_iter);
  return kmeans_cq(L->stream, L->host_desc.Y, L->n, labels, clusters, seed, max_iter,
                   init_centers, cq_out, assign_out, iters_out, centers_out);
}

int layout_debug_conflicts(layout_t* L, int32_t count, int64_t* stores, int64_t* conflicts,
                           int64_t* untracked) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (!stores || !conflicts || !untracked || count < 0)
    return fail(LAYOUT_E_INVALID_ARG, "NULL output or count < 0");
  if (L->engine != LAYOUT_ENGINE_GLOBAL || L->dim != 2 || L->mode == LAYOUT_JACOBI)
    return fail(LAYOUT_E_UNSUPPORTED,
                "the conflict counter runs 2D lock-free layouts on the global engine");
  if (L->t >= L->epochs) return fail(LAYOUT_E_DONE, "all %d epochs done", L->epochs);
  const int32_t run = std::min(count, L->epochs - L->t);
  *stores = *conflicts = *untracked = 0;
  if (run == 0 || L->nnz == 0) {
    L->t += run;
    return LAYOUT_OK;
  }
  const GlobalGroup g = global_group_of(L);
  const int rc = run_conflict_epochs(L->stream, L->d_table, L->n, L->k, L->mode, g.degree,
                                     global_grid(g), g.block, L->t, run, stores, conflicts,
                                     untracked);
  if (rc == LAYOUT_OK) L->t += run;
  return rc;
}

int layout_get_info(const layout_t* L, layout_info* info) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (!info) return fail(LAYOUT_E_INVALID_ARG, "info is NULL");
  info->engine = L->engine;
  info->bundle_edges = L->bundle;
  info->block_threads = L->block;
  info->grid_blocks = 0;
  if (L->engine == LAYOUT_ENGINE_XCD && L->nnz > 0) {
    info->grid_blocks = xcd_workers(L);  // working workgroups, on one XCD
  } else if (L->engine == LAYOUT_ENGINE_GLOBAL && L->nnz > 0) {
    info->grid_blocks = global_grid(global_group_of(L));
  } else if (L->engine == LAYOUT_ENGINE_LDS) {
    info->grid_blocks = 1;
  }
  info->n_chunks = L->n_chunks;
  info->nnz = L->nnz;
  info->n = L->n;
  info->k = L->k;
  info->epochs = L->epochs;
  info->update_mode = L->mode;
  info->hub_split_edges = L->hub;
  info->hot_degree = L->hot_degree;
  return LAYOUT_OK;
}

int layout_debug_draws(layout_t* L, int32_t epoch, int32_t* host_out) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (!host_out) return fail(LAYOUT_E_INVALID_ARG, "host_out is NULL");
  if (L->nnz == 0 || L->k == 0) return LAYOUT_OK;
  const size_t bytes = sizeof(int32_t) * size_t(L->nnz) * size_t(L->k);
  int32_t* d_out = nullptr;
  hipError_t e = hipMalloc(&d_out, bytes);
  if (e != hipSuccess) return hip_fail(e, "debug draws buffer");
  int rc = launch_dump_draws(L->stream, L->k, L->opts.neg_weights != LAYOUT_NEG_UNIFORM,
                             L->host_desc, epoch, d_out);
  if (rc == LAYOUT_OK) {
    e = hipMemcpyAsync(host_out, d_out, bytes, hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) rc = hip_fail(e, "reading debug draws");
  }
  (void)hipFree(d_out);
  return rc;
}

int layout_debug_draws_at(layout_t* L, int32_t epoch, const int64_t* edges, int64_t count,
                          int32_t* host_out) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (count < 0 || (count > 0 && (!edges || !host_out)))
    return fail(LAYOUT_E_INVALID_ARG, "NULL edges/host_out or count < 0");
  if (count == 0 || L->k == 0) return LAYOUT_OK;
  for (int64_t q = 0; q < count; ++q)
    if (edges[q] < 0 || edges[q] >= L->nnz)
      return fail(LAYOUT_E_INVALID_ARG, "edge %lld out of range [0, %lld)",
                  (long long)edges[q], (long long)L->nnz);
  int64_t* d_e = nullptr;
  int32_t* d_out = nullptr;
  hipError_t e = hipMalloc(&d_e, sizeof(int64_t) * size_t(count));
  if (e == hipSuccess) e = hipMalloc(&d_out, sizeof(int32_t) * size_t(count) * size_t(L->k));
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_e, edges, sizeof(int64_t) * size_t(count), hipMemcpyHostToDevice,
                       L->stream);
  int rc = LAYOUT_OK;
  if (e == hipSuccess) {
    rc = with_k(L->k, [&](auto kc) -> int {
      constexpr int K = decltype(kc)::value;
      return with_degree(L->opts.neg_weights != LAYOUT_NEG_UNIFORM, [&](auto dc) -> int {
        constexpr bool DEG = decltype(dc)::value;
        hipLaunchKernelGGL((dump_draws_at_kernel<K, DEG>), dim3(div_up(count, 256)), dim3(256), 0,
                           L->stream, L->host_desc, epoch, d_e, count, d_out);
        return LAYOUT_OK;
      });
    });
    e = hipGetLastError();
  }
  if (e == hipSuccess && rc == LAYOUT_OK)
    e = hipMemcpyAsync(host_out, d_out, sizeof(int32_t) * size_t(count) * size_t(L->k),
                       hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (d_e) (void)hipFree(d_e);
  if (d_out) (void)hipFree(d_out);
  if (rc != LAYOUT_OK) return rc;
  if (e != hipSuccess) return hip_fail(e, "debug draws of listed edges");
  return LAYOUT_OK;
}

int layout_debug_chunks(const layout_t* L, int64_t* begin_out, int32_t* src_out) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (!begin_out || !src_out) return fail(LAYOUT_E_INVALID_ARG, "NULL output");
  if (L->n_chunks == 0) return LAYOUT_OK;
  hipError_t e = hipMemcpyAsync(begin_out, L->host_desc.chunk_begin,
                                sizeof(int64_t) * size_t(L->n_chunks + 1), hipMemcpyDeviceToHost,
                                L->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(src_out, L->host_desc.chunk_src, sizeof(int32_t) * size_t(L->n_chunks),
                       hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "reading the chunk table");
  return LAYOUT_OK;
}

int layout_debug_alias(const layout_t* L, uint32_t* thr_out, uint32_t* alias_out) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (!thr_out || !alias_out) return fail(LAYOUT_E_INVALID_ARG, "NULL output");
  if (!L->host_desc.thr) return fail(LAYOUT_E_INVALID_ARG, "handle has no alias table");
  hipError_t e = hipMemcpyAsync(thr_out, L->host_desc.thr, sizeof(uint32_t) * size_t(L->n),
                                hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(alias_out, L->host_desc.alias, sizeof(uint32_t) * size_t(L->n),
                       hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "reading alias table");
  return LAYOUT_OK;
}

int layout_bench_gather(layout_t* L, int32_t mode, int32_t reps, float* ms) {
  if (!check_handle(L)) return LAYOUT_E_INVALID_ARG;
  if (L->dim != 2) return fail(LAYOUT_E_UNSUPPORTED, "the gather roofline is 2D");
  if (!ms || reps < 1) return fail(LAYOUT_E_INVALID_ARG, "ms NULL or reps < 1");
  const int32_t kind_bits = mode & 0xF, cache_bits = mode & ~0xF;
  if (kind_bits != LAYOUT_HOGWILD_STORE && kind_bits != LAYOUT_ATOMIC &&
      kind_bits != LAYOUT_GATHER_READ)
    return fail(LAYOUT_E_INVALID_ARG, "mode %d", mode);
  if (cache_bits != 0 && cache_bits != LAYOUT_GATHER_PLAIN && cache_bits != LAYOUT_GATHER_NONTEMPORAL)
    return fail(LAYOUT_E_INVALID_ARG, "mode %d: unknown cache bits", mode);
  if (kind_bits == LAYOUT_ATOMIC && cache_bits != 0)
    return fail(LAYOUT_E_INVALID_ARG, "atomic gathers take the device-scope accesses only");
  if (L->nnz == 0) {
    *ms = 0.f;
    return LAYOUT_OK;
  }
  if (L->engine != LAYOUT_ENGINE_GLOBAL)
    return fail(LAYOUT_E_UNSUPPORTED, "gather roofline runs on the global engine layout");
  const int kind = kind_bits == LAYOUT_ATOMIC ? kGatherAtomic
                   : kind_bits == LAYOUT_GATHER_READ ? kGatherRead
                                                     : kGatherStore;
  const int aux = cache_bits == LAYOUT_GATHER_PLAIN ? 0
                  : cache_bits == LAYOUT_GATHER_NONTEMPORAL ? 2
                                                            : 16;
  hipEvent_t a, b;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  const GlobalGroup gg = global_group_of(L);
  const int grid = global_grid(gg);
  auto launch = [&](auto kernel) -> int {
    hipError_t ee = hipEventRecord(a, L->stream);
    for (int r = 0; r < reps && ee == hipSuccess; ++r) {
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(gg.block), 0, L->stream, L->d_table,
                         L->n_chunks);
      ee = hipGetLastError();
    }
    if (ee == hipSuccess) ee = hipEventRecord(b, L->stream);
    if (ee == hipSuccess) ee = hipEventSynchronize(b);
    float t = 0.f;
    if (ee == hipSuccess) ee = hipEventElapsedTime(&t, a, b);
    if (ee != hipSuccess) return hip_fail(ee, "gather benchmark");
    *ms = t / reps;
    return LAYOUT_OK;
  };
  int rc = with_k(L->k, [&](auto kc) -> int {
    constexpr int K = decltype(kc)::value;
    if (kind == kGatherAtomic) return launch(gather_rmw_kernel<K, kGatherAtomic, GlobalMem, 16>);
    auto by_cache = [&](auto kind_c) -> int {
      constexpr int KIND = decltype(kind_c)::value;
      if (aux == 0) return launch(gather_rmw_kernel<K, KIND, GlobalMem, 0>);
      if (aux == 2) return launch(gather_rmw_kernel<K, KIND, GlobalMem, 2>);
      return launch(gather_rmw_kernel<K, KIND, GlobalMem, 16>);
    };
    if (kind == kGatherRead) return by_cache(std::integral_constant<int, kGatherRead>{});
    return by_cache(std::integral_constant<int, kGatherStore>{});
  });
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

int layout_bench_copy(int64_t bytes, int32_t reps, float* ms) {
  if (!ms || reps < 1 || bytes < 16) return fail(LAYOUT_E_INVALID_ARG, "bad copy benchmark args");
  const int64_t n4 = bytes / 16;
  float4 *src = nullptr, *dst = nullptr;
  hipError_t e = hipMalloc(&src, size_t(n4) * 16);
  if (e != hipSuccess) return hip_fail(e, "copy src");
  e = hipMalloc(&dst, size_t(n4) * 16);
  if (e != hipSuccess) {
    (void)hipFree(src);
    return hip_fail(e, "copy dst");
  }
  hipStream_t s = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = hipMemsetAsync(src, 0, size_t(n4) * 16, s);
  const int grid = device_props().cus * 8;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, s, src, dst, n4);  // warm
    e = hipEventRecord(a, s);
  }
  for (int r = 0; r < reps && e == hipSuccess; ++r)
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, s, src, dst, n4);
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(src);
  (void)hipFree(dst);
  if (e != hipSuccess) return hip_fail(e, "copy benchmark");
  *ms = t / reps;
  return LAYOUT_OK;
}

}  // extern "C"
