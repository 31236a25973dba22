// Race diagnostics of the lock-free epoch (test and measurement support).
//
// Conflict counter.  An epoch runs the real chunk schedule through the same
// process_chunk, with a memory class that keeps one version word per node.
//   * A position load first reads the node's version.
//   * A position write increments that version atomically.  When the old
//     value differs from the one read at the load, another lane wrote the
//     node in between.
//   * Under HOGWILD_STORE such a write overwrites a concurrent update (a
//     lost update); under ATOMIC it adds a change computed from a stale
//     read.  This is the GPU analogue of the conflict rate of Sec. 3.4.
//   * Each lane keeps the (node, version) pairs of its open loads in a small
//     ring; a write looks up the lane's latest load of the node.  A write
//     whose load has left the ring (the source commit of a long run without
//     a reload: a hub segment under HOGWILD_STORE, any long row under
//     ATOMIC) is counted as untracked.
//
// Atomic probe.  Every lane of a launch filling all CUs adds 1 to one FP64
// and one u64 counter at device scope, a given number of times; the totals
// must be exact (cross-XCD atomic visibility, on which the ATOMIC policy
// relies), and the launch time gives the contended atomic rate.  A second
// pass adds to one address per lane (the uncontended rate).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "snaplayout.h"

namespace snap {
namespace {

constexpr int kRing = 16;  // open loads per lane (source, neighbour, k <= 8 negatives, commit)

struct VersionMem {
  float2* base;
  uint32_t* version;
  mutable int32_t node[kRing];
  mutable uint32_t seen[kRing];
  mutable int32_t head;
  mutable unsigned long long stores, conflicts, untracked;

  __device__ VersionMem(float2* Y, uint32_t* v)
      : base(Y), version(v), head(0), stores(0), conflicts(0), untracked(0) {
    for (int q = 0; q < kRing; ++q) node[q] = -1;
  }
  __device__ int32_t idx(const float2* p) const { return static_cast<int32_t>(p - base); }
  __device__ float2 load(const float2* p) const {
    const int32_t v = idx(p);
    const uint32_t ver = __hip_atomic_load(version + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    node[head] = v;
    seen[head] = ver;
    head = (head + 1) % kRing;
    return GlobalMem::load(p);
  }
  __device__ void wrote(const float2* p) const {
    const int32_t v = idx(p);
    const uint32_t old = atomicAdd(version + v, 1u);
    ++stores;
    for (int q = 1; q <= kRing; ++q) {
      const int s = (head - q + kRing) % kRing;
      if (node[s] == v) {
        if (seen[s] != old) ++conflicts;
        seen[s] = old + 1;  // a later write of the same load window starts from here
        return;
      }
    }
    ++untracked;
  }
  __device__ void store(float2* p, float2 x) const {
    GlobalMem::store(p, x);
    wrote(p);
  }
  __device__ void add(float2* p, float2 x) const {
    GlobalMem::add(p, x);
    wrote(p);
  }
};

template <int K, int MODE, bool DEGREE>
__global__ void __launch_bounds__(256)
    conflict_epoch_kernel(const GraphDesc* __restrict__ table, uint32_t* __restrict__ version,
                          int32_t dt, unsigned long long* __restrict__ totals) {
  const GraphDesc& g = table[0];
  const int32_t t = g.t0 + dt;
  const float eta = eta_of(g, t);
  VersionMem mem(g.Y, version);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; c < g.n_chunks;
       c += stride)
    process_chunk<K, MODE, DEGREE>(mem, g, g.Y, g.D, g.chunk_offset + c, t, eta);
  unsigned long long s = mem.stores, x = mem.conflicts, u = mem.untracked;
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_down(s, off, 64);
    x += __shfl_down(x, off, 64);
    u += __shfl_down(u, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (s) atomicAdd(totals, s);
    if (x) atomicAdd(totals + 1, x);
    if (u) atomicAdd(totals + 2, u);
  }
}

__global__ void __launch_bounds__(256)
    atomic_probe_kernel(int32_t reps, int32_t spread, double* __restrict__ fsum,
                        unsigned long long* __restrict__ isum) {
  const int64_t lane = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double* f = spread ? fsum + lane : fsum;
  unsigned long long* u = spread ? isum + lane : isum;
  for (int32_t r = 0; r < reps; ++r) {
    __hip_atomic_fetch_add(f, 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(u, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void zero_u32(uint32_t* p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

}  // namespace

int run_conflict_epochs(hipStream_t stream, const GraphDesc* d_table, int32_t n, int k,
                        int mode, bool degree, int grid, int block, int32_t t, int32_t count,
                        int64_t* stores, int64_t* conflicts, int64_t* untracked) {
  uint32_t* d_ver = nullptr;
  unsigned long long* d_tot = nullptr;
  hipError_t e = hipMalloc(&d_ver, sizeof(uint32_t) * size_t(n > 0 ? n : 1));
  if (e == hipSuccess) e = hipMalloc(&d_tot, 3 * sizeof(unsigned long long));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(zero_u32, dim3(div_up(n, 256) > 0 ? div_up(n, 256) : 1), dim3(256), 0,
                       stream, d_ver, n);
    e = hipMemsetAsync(d_tot, 0, 3 * sizeof(unsigned long long), stream);
  }
  int rc = LAYOUT_OK;
  for (int32_t ep = 0; ep < count && e == hipSuccess && rc == LAYOUT_OK; ++ep) {
    const int32_t dt = t + ep;
#define SNAP_CONFLICT_LAUNCH(KK)                                                                 \
  case KK:                                                                                       \
    if (mode == kAtomic) {                                                                       \
      if (degree)                                                                                \
        hipLaunchKernelGGL((conflict_epoch_kernel<KK, kAtomic, true>), dim3(grid), dim3(block), \
                           0, stream, d_table, d_ver, dt, d_tot);                                \
      else                                                                                       \
        hipLaunchKernelGGL((conflict_epoch_kernel<KK, kAtomic, false>), dim3(grid),             \
                           dim3(block), 0, stream, d_table, d_ver, dt, d_tot);                   \
    } else {                                                                                     \
      if (degree)                                                                                \
        hipLaunchKernelGGL((conflict_epoch_kernel<KK, kStore, true>), dim3(grid), dim3(block),  \
                           0, stream, d_table, d_ver, dt, d_tot);                                \
      else                                                                                       \
        hipLaunchKernelGGL((conflict_epoch_kernel<KK, kStore, false>), dim3(grid), dim3(block), \
                           0, stream, d_table, d_ver, dt, d_tot);                                \
    }                                                                                            \
    break;
    switch (k) {
      SNAP_CONFLICT_LAUNCH(0)
      SNAP_CONFLICT_LAUNCH(1)
      SNAP_CONFLICT_LAUNCH(2)
      SNAP_CONFLICT_LAUNCH(3)
      SNAP_CONFLICT_LAUNCH(4)
      SNAP_CONFLICT_LAUNCH(5)
      SNAP_CONFLICT_LAUNCH(6)
      SNAP_CONFLICT_LAUNCH(7)
      SNAP_CONFLICT_LAUNCH(8)
      default: rc = fail(LAYOUT_E_UNSUPPORTED, "k = %d", k);
    }
#undef SNAP_CONFLICT_LAUNCH
    if (rc == LAYOUT_OK) e = hipGetLastError();
  }
  unsigned long long tot[3] = {0, 0, 0};
  if (e == hipSuccess && rc == LAYOUT_OK)
    e = hipMemcpyAsync(tot, d_tot, sizeof tot, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (d_ver) (void)hipFree(d_ver);
  if (d_tot) (void)hipFree(d_tot);
  if (rc != LAYOUT_OK) return rc;
  if (e != hipSuccess) return hip_fail(e, "conflict counter");
  *stores = static_cast<int64_t>(tot[0]);
  *conflicts = static_cast<int64_t>(tot[1]);
  *untracked = static_cast<int64_t>(tot[2]);
  return LAYOUT_OK;
}

}  // namespace snap

extern "C" int layout_bench_atomics(int32_t reps, int32_t spread, double* fsum_out,
                                    int64_t* isum_out, int64_t* adds_out, float* ms) {
  using namespace snap;
  if (reps < 1 || !fsum_out || !isum_out || !adds_out || !ms)
    return fail(LAYOUT_E_INVALID_ARG, "reps >= 1 and non-NULL outputs");
  const int grid = std::max(1, device_props().cus) * 8;
  const int64_t lanes = int64_t(grid) * 256;
  const int64_t slots = spread ? lanes : 1;
  double* f = nullptr;
  unsigned long long* u = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipMalloc(&f, sizeof(double) * size_t(slots));
  if (e == hipSuccess) e = hipMalloc(&u, sizeof(unsigned long long) * size_t(slots));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = hipMemsetAsync(f, 0, sizeof(double) * size_t(slots), s);
  if (e == hipSuccess) e = hipMemsetAsync(u, 0, sizeof(unsigned long long) * size_t(slots), s);
  if (e == hipSuccess) e = hipEventRecord(a, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(atomic_probe_kernel, dim3(grid), dim3(256), 0, s, reps, spread, f, u);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  std::vector<double> hf(slots);
  std::vector<unsigned long long> hu(slots);
  if (e == hipSuccess)
    e = hipMemcpy(hf.data(), f, sizeof(double) * size_t(slots), hipMemcpyDeviceToHost);
  if (e == hipSuccess)
    e = hipMemcpy(hu.data(), u, sizeof(unsigned long long) * size_t(slots), hipMemcpyDeviceToHost);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (s) (void)hipStreamDestroy(s);
  if (f) (void)hipFree(f);
  if (u) (void)hipFree(u);
  if (e != hipSuccess) return hip_fail(e, "atomic probe");
  double fs = 0.0;
  unsigned long long us = 0;
  for (int64_t q = 0; q < slots; ++q) {
    fs += hf[q];
    us += hu[q];
  }
  *fsum_out = fs;
  *isum_out = static_cast<int64_t>(us);
  *adds_out = lanes * reps;
  *ms = t;
  return LAYOUT_OK;
}
