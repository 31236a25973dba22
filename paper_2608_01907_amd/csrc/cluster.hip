// Clustering quality CQ (Sec. 4.1) on the device: k-means of the layout and
// the adjusted Rand index against given labels.
//
// k-means++ start (Arthur and Vassilvitskii, SODA 2007).  The draws are word
// x0 of the Philox block (c, 0, 0, tag 4) for center c.
//   * The first center is point floor(x_0 n / 2^64).
//   * Center c >= 1 is the first point whose running sum of D^2 (the FP64
//     squared distance to the nearest chosen center) exceeds
//     u_c * sum(D^2), with u_c = (x_c >> 11) 2^-53.  When every D^2 is 0 it
//     is point floor(x_c n / 2^64).
//   * Each center costs one pass: `kmpp_update_kernel` lowers D^2 and sums
//     it per contiguous block.  The host then finds the block where the
//     running sum crosses the target, and `kmpp_pick_kernel` walks that
//     block in order.
// Lloyd's iterations.
//   * `assign_kernel` moves each point to the nearest center (FP64 squared
//     distances without contraction, lowest index on ties).  It counts the
//     changed assignments and sums points per cluster in LDS, with one
//     global FP64 atomic per cluster and workgroup.
//   * `move_centers_kernel` sets each center to its cluster's mean; an empty
//     cluster keeps its center.
//   * The loop stops when an assignment after the first changes nothing, or
//     after max_iter passes.
// ARI (Hubert and Arabie, 1985): `contingency_kernel` counts (label,
// cluster) pairs; the host evaluates the index from the table.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "snaplayout.h"

namespace snap {
namespace {

constexpr uint64_t kTagKmeans = 4;
constexpr int kPickBlocks = 1024;     // contiguous blocks of the k-means++ sums
constexpr int32_t kMaxClusters = 4096;  // centers, sums and counts in LDS: 36 B each
constexpr int64_t kMaxTable = int64_t(1) << 27;  // labels x clusters

__global__ void kmeans_draws_kernel(uint64_t seed, int32_t K, uint64_t* __restrict__ out) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  out[c] = philox4x64_10(static_cast<uint64_t>(c), 0, 0, kTagKmeans, seed, kKeyDomain).x0;
}

__device__ __forceinline__ double sq_dist(double x, double y, double cx, double cy) {
#pragma clang fp contract(off)
  const double dx = x - cx;
  const double dy = y - cy;
  return dx * dx + dy * dy;
}

__device__ __forceinline__ double block_sum_f64(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) s += red[w];
  return s;  // valid in thread 0
}

// D^2 <- min(D^2, |y - c|^2) over block b's points [b R, min(n, (b+1) R)),
// and the block's sum of D^2.  first: D^2 starts at +inf.
__global__ void __launch_bounds__(256)
    kmpp_update_kernel(const float2* __restrict__ Y, int32_t n, int64_t R, double cx, double cy,
                       int32_t first, double* __restrict__ d2, double* __restrict__ block_sums) {
  __shared__ double red[4];
  const int64_t lo = static_cast<int64_t>(blockIdx.x) * R;
  const int64_t hi = lo + R < n ? lo + R : int64_t(n);
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const float2 p = Y[i];
    const double d = sq_dist(p.x, p.y, cx, cy);
    const double v = first ? d : (d2[i] < d ? d2[i] : d);
    d2[i] = v;
    acc += v;
  }
  acc = block_sum_f64(acc, red);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = acc;
}

// The first point of [lo, hi) at which the running sum of D^2, started at
// `before`, exceeds t (hi - 1 when rounding leaves it short).  One lane,
// points in order.
__global__ void kmpp_pick_kernel(const double* __restrict__ d2, int64_t lo, int64_t hi,
                                 double before, double t, int32_t* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double run = before;
  int64_t pick = hi - 1;
  for (int64_t i = lo; i < hi; ++i) {
    run += d2[i];
    if (run > t) {
      pick = i;
      break;
    }
  }
  *out = static_cast<int32_t>(pick);
}

__global__ void gather_centers_kernel(const float2* __restrict__ Y, const int32_t* __restrict__ idx,
                                      int32_t K, double2* __restrict__ C) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  const float2 p = Y[idx[c]];
  C[c] = make_double2(p.x, p.y);
}

// One assignment pass; sums and counts per cluster accumulate into
// sums[2K] / counts[K] (zero before the pass), *changed counts moved points.
__global__ void __launch_bounds__(256)
    assign_kernel(const float2* __restrict__ Y, int32_t n, const double2* __restrict__ C,
                  int32_t K, int32_t* __restrict__ assign, int32_t* __restrict__ changed,
                  double* __restrict__ sums, unsigned long long* __restrict__ counts) {
  extern __shared__ __align__(16) unsigned char smem[];
  double2* sC = reinterpret_cast<double2*>(smem);
  double* sS = reinterpret_cast<double*>(sC + K);
  unsigned int* sN = reinterpret_cast<unsigned int*>(sS + 2 * K);
  __shared__ int32_t red[4];
  for (int32_t c = threadIdx.x; c < K; c += blockDim.x) {
    sC[c] = C[c];
    sS[2 * c] = 0.0;
    sS[2 * c + 1] = 0.0;
    sN[c] = 0u;
  }
  __syncthreads();
  int32_t moved = 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const float2 p = Y[i];
    const double x = p.x, y = p.y;
    int32_t best = 0;
    double bd = sq_dist(x, y, sC[0].x, sC[0].y);
    for (int32_t c = 1; c < K; ++c) {
      const double d = sq_dist(x, y, sC[c].x, sC[c].y);
      if (d < bd) {
        bd = d;
        best = c;
      }
    }
    if (assign[i] != best) ++moved;
    assign[i] = best;
    atomicAdd(&sS[2 * best], x);
    atomicAdd(&sS[2 * best + 1], y);
    atomicAdd(&sN[best], 1u);
  }
  for (int off = 32; off > 0; off >>= 1) moved += __shfl_down(moved, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = moved;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t m = 0;
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) m += red[w];
    if (m) atomicAdd(changed, m);
  }
  for (int32_t c = threadIdx.x; c < K; c += blockDim.x) {
    if (sN[c] == 0u) continue;
    atomicAdd(&sums[2 * c], sS[2 * c]);
    atomicAdd(&sums[2 * c + 1], sS[2 * c + 1]);
    atomicAdd(&counts[c], static_cast<unsigned long long>(sN[c]));
  }
}

// Centers to their clusters' means (empty clusters keep theirs); clears the
// sums and counts for the next pass.
__global__ void move_centers_kernel(double2* __restrict__ C, int32_t K, double* __restrict__ sums,
                                    unsigned long long* __restrict__ counts) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  const unsigned long long m = counts[c];
  if (m > 0) C[c] = make_double2(sums[2 * c] / double(m), sums[2 * c + 1] / double(m));
  sums[2 * c] = 0.0;
  sums[2 * c + 1] = 0.0;
  counts[c] = 0ull;
}

__global__ void contingency_kernel(const int32_t* __restrict__ lab, const int32_t* __restrict__ assign,
                                   int32_t n, int32_t K, unsigned long long* __restrict__ table) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  atomicAdd(&table[int64_t(lab[i]) * K + assign[i]], 1ull);
}

__global__ void fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_u64(unsigned long long* __restrict__ p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void fill_f64(double* __restrict__ p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

uint64_t mul_hi_n(uint64_t x, int32_t n) {
  return static_cast<uint64_t>((static_cast<unsigned __int128>(x) * uint64_t(n)) >> 64);
}

double c2(double x) { return x * (x - 1.0) / 2.0; }

}  // namespace

int kmeans_cq(hipStream_t stream, const float2* d_Y, int32_t n, const int32_t* labels,
              int32_t K, uint64_t seed, int32_t max_iter, const float* init_centers,
              double* ari_out, int32_t* assign_out, int32_t* iters_out,
              int32_t* centers_idx_out) {
  // labels -> 0..L-1 on the host
  std::vector<int32_t> uniq(labels, labels + n);
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  const int32_t L = static_cast<int32_t>(uniq.size());
  if (K == 0) K = L;
  if (K < 1 || K > n || K > kMaxClusters)
    return fail(LAYOUT_E_INVALID_ARG, "clusters = %d (1..min(n, %d))", K, kMaxClusters);
  if (int64_t(L) * K > kMaxTable)
    return fail(LAYOUT_E_INVALID_ARG, "%d labels x %d clusters exceed the contingency table",
                L, K);
  std::vector<int32_t> lab(n);
  for (int32_t v = 0; v < n; ++v)
    lab[v] = static_cast<int32_t>(std::lower_bound(uniq.begin(), uniq.end(), labels[v]) -
                                  uniq.begin());

  const int64_t R = div_up(n, kPickBlocks);
  const int blocks = static_cast<int>(div_up(n, R));
  double *d_d2 = nullptr, *d_bsum = nullptr, *d_sums = nullptr;
  double2* d_C = nullptr;
  int32_t *d_assign = nullptr, *d_changed = nullptr, *d_idx = nullptr, *d_lab = nullptr;
  uint64_t* d_words = nullptr;
  unsigned long long *d_counts = nullptr, *d_table = nullptr;
  hipError_t e = hipMalloc(&d_d2, sizeof(double) * size_t(n));
  if (e == hipSuccess) e = hipMalloc(&d_bsum, sizeof(double) * size_t(blocks));
  if (e == hipSuccess) e = hipMalloc(&d_sums, sizeof(double) * 2 * size_t(K));
  if (e == hipSuccess) e = hipMalloc(&d_C, sizeof(double2) * size_t(K));
  if (e == hipSuccess) e = hipMalloc(&d_assign, sizeof(int32_t) * size_t(n));
  if (e == hipSuccess) e = hipMalloc(&d_changed, sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&d_idx, sizeof(int32_t) * size_t(K));
  if (e == hipSuccess) e = hipMalloc(&d_lab, sizeof(int32_t) * size_t(n));
  if (e == hipSuccess) e = hipMalloc(&d_words, sizeof(uint64_t) * size_t(K));
  if (e == hipSuccess) e = hipMalloc(&d_counts, sizeof(unsigned long long) * size_t(K));
  if (e == hipSuccess) e = hipMalloc(&d_table, sizeof(unsigned long long) * size_t(L) * size_t(K));
  std::vector<int32_t> idx(K, 0);
  int rc = LAYOUT_OK;
  int32_t iters = 0;
  // --- start: the caller's centers or k-means++
  if (e == hipSuccess && init_centers) {
    std::vector<double2> C(K);
    for (int32_t c = 0; c < K; ++c)
      C[c] = make_double2(init_centers[2 * c], init_centers[2 * c + 1]);
    e = hipMemcpyAsync(d_C, C.data(), sizeof(double2) * size_t(K), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    std::fill(idx.begin(), idx.end(), -1);
  } else if (e == hipSuccess) {
    std::vector<uint64_t> words(K);
    hipLaunchKernelGGL(kmeans_draws_kernel, dim3(div_up(K, 256)), dim3(256), 0, stream, seed, K,
                       d_words);
    e = hipMemcpyAsync(words.data(), d_words, sizeof(uint64_t) * size_t(K), hipMemcpyDeviceToHost,
                       stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    idx[0] = static_cast<int32_t>(mul_hi_n(words[0], n));
    std::vector<float2> hy(1);
    std::vector<double> bsum(blocks);
    for (int32_t c = 1; c < K && e == hipSuccess; ++c) {
      e = hipMemcpyAsync(hy.data(), d_Y + idx[c - 1], sizeof(float2), hipMemcpyDeviceToHost,
                         stream);
      if (e != hipSuccess) break;
      e = hipStreamSynchronize(stream);
      if (e != hipSuccess) break;
      hipLaunchKernelGGL(kmpp_update_kernel, dim3(blocks), dim3(256), 0, stream, d_Y, n, R,
                         double(hy[0].x), double(hy[0].y), c == 1 ? 1 : 0, d_d2, d_bsum);
      e = hipMemcpyAsync(bsum.data(), d_bsum, sizeof(double) * size_t(blocks),
                         hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      if (e != hipSuccess) break;
      double total = 0.0;
      for (double b : bsum) total += b;
      if (!(total > 0.0)) {
        idx[c] = static_cast<int32_t>(mul_hi_n(words[c], n));
        continue;
      }
      const double t = double(words[c] >> 11) * 0x1p-53 * total;
      double before = 0.0;
      int b = 0;
      while (b < blocks - 1 && before + bsum[b] <= t) before += bsum[b++];
      hipLaunchKernelGGL(kmpp_pick_kernel, dim3(1), dim3(64), 0, stream, d_d2, int64_t(b) * R,
                         std::min<int64_t>(n, (int64_t(b) + 1) * R), before, t, d_changed);
      e = hipMemcpyAsync(&idx[c], d_changed, sizeof(int32_t), hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_idx, idx.data(), sizeof(int32_t) * size_t(K), hipMemcpyHostToDevice,
                         stream);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(gather_centers_kernel, dim3(div_up(K, 256)), dim3(256), 0, stream, d_Y,
                         d_idx, K, d_C);
      e = hipGetLastError();
    }
  }
  // --- Lloyd's iterations
  if (e == hipSuccess) {
    const size_t lds = sizeof(double2) * size_t(K) + 2 * sizeof(double) * size_t(K) +
                       sizeof(unsigned int) * size_t(K);
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&assign_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    const int grid = static_cast<int>(
        std::min<int64_t>(div_up(n, 256), int64_t(4) * std::max(1, device_props().cus)));
    if (e == hipSuccess) {
      hipLaunchKernelGGL(fill_i32, dim3(div_up(n, 256)), dim3(256), 0, stream, d_assign, n, -1);
      hipLaunchKernelGGL(fill_f64, dim3(div_up(2 * K, 256)), dim3(256), 0, stream, d_sums,
                         2 * int64_t(K));
      hipLaunchKernelGGL(fill_u64, dim3(div_up(K, 256)), dim3(256), 0, stream, d_counts, K);
    }
    for (int32_t it = 1; it <= std::max(1, max_iter) && e == hipSuccess; ++it) {
      int32_t changed = 0;
      hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, stream, d_changed, 1, 0);
      hipLaunchKernelGGL(assign_kernel, dim3(grid), dim3(256), lds, stream, d_Y, n, d_C, K,
                         d_assign, d_changed, d_sums, d_counts);
      e = hipMemcpyAsync(&changed, d_changed, sizeof(int32_t), hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      iters = it;
      if (e != hipSuccess || (it > 1 && changed == 0)) break;
      hipLaunchKernelGGL(move_centers_kernel, dim3(div_up(K, 256)), dim3(256), 0, stream, d_C, K,
                         d_sums, d_counts);
    }
  }
  // --- ARI from the contingency table
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_lab, lab.data(), sizeof(int32_t) * size_t(n), hipMemcpyHostToDevice,
                       stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(fill_u64, dim3(div_up(int64_t(L) * K, 256)), dim3(256), 0, stream, d_table,
                       int64_t(L) * K);
    hipLaunchKernelGGL(contingency_kernel, dim3(div_up(n, 256)), dim3(256), 0, stream, d_lab,
                       d_assign, n, K, d_table);
  }
  std::vector<unsigned long long> table(size_t(L) * size_t(K));
  if (e == hipSuccess)
    e = hipMemcpyAsync(table.data(), d_table, sizeof(unsigned long long) * table.size(),
                       hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && assign_out)
    e = hipMemcpyAsync(assign_out, d_assign, sizeof(int32_t) * size_t(n), hipMemcpyDeviceToHost,
                       stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  for (void* p : {static_cast<void*>(d_d2), static_cast<void*>(d_bsum), static_cast<void*>(d_sums),
                  static_cast<void*>(d_C), static_cast<void*>(d_assign),
                  static_cast<void*>(d_changed), static_cast<void*>(d_idx),
                  static_cast<void*>(d_lab), static_cast<void*>(d_words),
                  static_cast<void*>(d_counts), static_cast<void*>(d_table)})
    if (p) (void)hipFree(p);
  if (e != hipSuccess) return hip_fail(e, "clustering quality");
  if (rc != LAYOUT_OK) return rc;
  double index = 0.0;
  std::vector<double> rows(L, 0.0), cols(K, 0.0);
  for (int32_t a = 0; a < L; ++a)
    for (int32_t c = 0; c < K; ++c) {
      const double v = double(table[size_t(a) * K + c]);
      index += c2(v);
      rows[a] += v;
      cols[c] += v;
    }
  double sa = 0.0, sb = 0.0;
  for (double v : rows) sa += c2(v);
  for (double v : cols) sb += c2(v);
  const double expected = n > 1 ? sa * sb / c2(double(n)) : 0.0;
  const double mx = 0.5 * (sa + sb);
  *ari_out = mx == expected ? 1.0 : (index - expected) / (mx - expected);
  if (iters_out) *iters_out = iters;
  if (centers_idx_out) std::copy(idx.begin(), idx.end(), centers_idx_out);
  return LAYOUT_OK;
}

}  // namespace snap
