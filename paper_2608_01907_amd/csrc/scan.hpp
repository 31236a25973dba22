// Device-wide exclusive prefix sum in three launches (tile totals, scan of
// the totals by one workgroup, tile scan + scatter), generic over the item
// type T (needs T + T and a zero value T{}) and two functors:
//   Load:  T operator()(int64_t index) const           -- item at index (T{} past the end)
//   Apply: void operator()(int64_t index, T exclusive, T item) const
// Used by the preprocessing of a layout job (chunk table, alias table).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snap {

constexpr int kScanThreads = 256;
constexpr int kScanItemsPerThread = 4;
constexpr int kScanTile = kScanThreads * kScanItemsPerThread;

// Exclusive scan of one tile held by the workgroup.  On return v[q] holds the
// exclusive prefix of item q of this thread and total the tile's sum.
template <class T>
__device__ void tile_exclusive_scan(T (&v)[kScanItemsPerThread], T* __restrict__ sh, T& total) {
  T run{};
#pragma unroll
  for (int q = 0; q < kScanItemsPerThread; ++q) {
    const T x = v[q];
    v[q] = run;
    run = run + x;
  }
  sh[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    T add{};
    if (threadIdx.x >= static_cast<unsigned>(off)) add = sh[threadIdx.x - off];
    __syncthreads();
    sh[threadIdx.x] = sh[threadIdx.x] + add;
    __syncthreads();
  }
  const T before = threadIdx.x > 0 ? sh[threadIdx.x - 1] : T{};
  total = sh[kScanThreads - 1];
#pragma unroll
  for (int q = 0; q < kScanItemsPerThread; ++q) v[q] = before + v[q];
  __syncthreads();
}

template <class T, class Load>
__global__ void __launch_bounds__(kScanThreads) scan_tile_sums_kernel(Load load,
                                                                      T* __restrict__ sums) {
  __shared__ T sh[kScanThreads];
  T v[kScanItemsPerThread];
  const int64_t base =
      static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItemsPerThread;
#pragma unroll
  for (int q = 0; q < kScanItemsPerThread; ++q) v[q] = load(base + q);
  T total;
  tile_exclusive_scan(v, sh, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One workgroup: each thread scans a contiguous segment of tile totals
// sequentially, the segment totals are scanned in LDS.
template <class T>
__global__ void __launch_bounds__(kScanThreads) scan_tile_totals_kernel(T* __restrict__ sums,
                                                                        int64_t tiles,
                                                                        T* __restrict__ grand) {
  __shared__ T sh[kScanThreads];
  const int64_t per = (tiles + kScanThreads - 1) / kScanThreads;
  const int64_t b0 = threadIdx.x * per;
  const int64_t b1 = b0 + per < tiles ? b0 + per : tiles;
  T run{};
  for (int64_t b = b0; b < b1; ++b) run = run + sums[b];
  T v[kScanItemsPerThread];
  v[0] = run;
#pragma unroll
  for (int q = 1; q < kScanItemsPerThread; ++q) v[q] = T{};
  T total;
  tile_exclusive_scan(v, sh, total);
  T off = v[0];
  for (int64_t b = b0; b < b1; ++b) {
    const T x = sums[b];
    sums[b] = off;
    off = off + x;
  }
  if (threadIdx.x == 0) *grand = total;
}

template <class T, class Load, class Apply>
__global__ void __launch_bounds__(kScanThreads) scan_apply_kernel(Load load, Apply apply,
                                                                  const T* __restrict__ sums,
                                                                  int64_t n) {
  __shared__ T sh[kScanThreads];
  T v[kScanItemsPerThread];
  T raw[kScanItemsPerThread];
  const int64_t base =
      static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItemsPerThread;
#pragma unroll
  for (int q = 0; q < kScanItemsPerThread; ++q) raw[q] = v[q] = load(base + q);
  T total;
  tile_exclusive_scan(v, sh, total);
  const T off = sums[blockIdx.x];
#pragma unroll
  for (int q = 0; q < kScanItemsPerThread; ++q)
    if (base + q < n) apply(base + q, off + v[q], raw[q]);
}

// Host helper: scratch holds tiles(n) + 1 items of T; grand total lands in
// scratch[tiles(n)] (device memory).
inline int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

template <class T, class Load, class Apply>
inline void device_exclusive_scan(hipStream_t stream, int64_t n, Load load, Apply apply,
                                  T* scratch) {
  const int64_t tiles = scan_tiles(n) > 0 ? scan_tiles(n) : 1;
  hipLaunchKernelGGL((scan_tile_sums_kernel<T, Load>), dim3(tiles), dim3(kScanThreads), 0, stream,
                     load, scratch);
  hipLaunchKernelGGL((scan_tile_totals_kernel<T>), dim3(1), dim3(kScanThreads), 0, stream,
                     scratch, tiles, scratch + tiles);
  hipLaunchKernelGGL((scan_apply_kernel<T, Load, Apply>), dim3(tiles), dim3(kScanThreads), 0,
                     stream, load, apply, scratch, n);
}

}  // namespace snap
