// Exact neighbourhood preservation (the NP metric of Sec. 4.1) on the device.
//
// For a query node i: R_i is the graph r-ring of i (nodes at hop distance
// 1..r, i excluded; r = 1 or 2), k_i = |R_i|, and K_i the k_i nearest nodes
// to y_i in the layout (i excluded), ranked by the squared distance computed
// in FP32 as fl(fl(dx*dx) + fl(dy*dy)) with dx = fl(y_l.x - y_i.x), ties broken
// by node index.  The pass returns k_i and |R_i ∩ K_i|; the node's NP term is
// |R_i ∩ K_i| / |R_i ∪ K_i| = inter / (2 k_i - inter).
//
// Queries run in batches of Q; each query owns a bitmap of n bits in scratch:
//   1. ring_mark: the r-ring is marked into the bitmap (atomic OR), hop 1 by
//      the lanes of each workgroup, hop 2 one neighbour row per wave;
//   2. ring_count: k_i = popcount of the bitmap without bit i;
//   3. radix select of the k_i-th smallest 64-bit key (distance bits << 32 |
//      node id; unique, so the set K_i is exact): eight passes of 8 bits, each
//      a histogram of the digit over the keys that match the prefix so far,
//      then a pick of the bin holding the k_i-th key.  A query is finished as
//      soon as the picked bin holds exactly the keys still needed (usually
//      after the four distance bytes);
//   4. ring_intersect: every marked node whose key is at most the threshold
//      key is counted.
// The histogram pass serves 8 queries per workgroup, so that one load of a
// position feeds 8 distance computations.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "snaplayout.h"

namespace snap {
namespace {

constexpr int kQueriesPerBlock = 8;
constexpr int64_t kScratchBytes = int64_t(256) << 20;  // bitmaps of one batch
constexpr int32_t kMaxBatch = 1024;

struct NpState {
  uint64_t prefix;   // digits picked so far
  uint64_t thr_key;  // largest key of K_i (valid once done)
  int64_t need;      // rank still to find among the keys with this prefix
  int32_t node;
  int32_t k;         // |R_i| (bit i excluded once counted)
  int32_t inter;
  int32_t done;
};

__device__ __forceinline__ uint64_t np_key(float2 yl, float2 yi, int32_t l) {
#pragma clang fp contract(off)
  const float dx = yl.x - yi.x;
  const float dy = yl.y - yi.y;
  const float q = dx * dx + dy * dy;
  return (static_cast<uint64_t>(__float_as_uint(q)) << 32) | static_cast<uint32_t>(l);
}

__device__ __forceinline__ void set_bit(uint32_t* bits, int32_t v) {
  atomicOr(bits + (v >> 5), 1u << (v & 31));
}

__global__ void __launch_bounds__(256)
    ring_mark_kernel(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                     NpState* __restrict__ st, int32_t radius, uint32_t* __restrict__ bits,
                     int64_t words) {
  const int32_t q = blockIdx.y;
  const int32_t i = st[q].node;
  uint32_t* b = bits + static_cast<int64_t>(q) * words;
  const int64_t r0 = row_ptr[i], r1 = row_ptr[i + 1];
  // hop 1
  for (int64_t m = r0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; m < r1;
       m += int64_t(gridDim.x) * blockDim.x)
    set_bit(b, col[m]);
  if (radius < 2) return;
  // hop 2: one neighbour row per wave
  const int32_t waves = blockDim.x >> 6;
  const int32_t lane = threadIdx.x & 63;
  for (int64_t m = r0 + int64_t(blockIdx.x) * waves + (threadIdx.x >> 6); m < r1;
       m += int64_t(gridDim.x) * waves) {
    const int32_t j = col[m];
    const int64_t s0 = row_ptr[j], s1 = row_ptr[j + 1];
    for (int64_t e = s0 + lane; e < s1; e += 64) set_bit(b, col[e]);
  }
}

__device__ __forceinline__ int32_t block_sum_i32(int32_t v, int32_t* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  int32_t s = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) s += red[w];
  return s;  // valid in thread 0
}

__global__ void __launch_bounds__(256)
    ring_count_kernel(const uint32_t* __restrict__ bits, int64_t words, NpState* st) {
  __shared__ int32_t red[4];
  const int32_t q = blockIdx.y;
  const uint32_t* b = bits + static_cast<int64_t>(q) * words;
  int32_t c = 0;
  for (int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < words;
       w += static_cast<int64_t>(gridDim.x) * blockDim.x)
    c += __popc(b[w]);
  c = block_sum_i32(c, red);
  if (threadIdx.x == 0 && c) atomicAdd(&st[q].k, c);
}

// k_i without bit i; the select starts from the full key range
__global__ void select_init_kernel(const uint32_t* __restrict__ bits, int64_t words,
                                   NpState* st, int32_t Q) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q) return;
  NpState s = st[q];
  const int32_t i = s.node;
  if ((bits[static_cast<int64_t>(q) * words + (i >> 5)] >> (i & 31)) & 1u) s.k -= 1;
  s.need = s.k;
  s.prefix = 0;
  s.thr_key = 0;
  s.inter = 0;
  s.done = s.k == 0 ? 1 : 0;
  st[q] = s;
}

// Histogram of digit `pass` (0 = top byte of the key) over the keys that match
// the prefix, for kQueriesPerBlock queries per workgroup.
__global__ void __launch_bounds__(256)
    select_hist_kernel(const float2* __restrict__ Y, int32_t n, const NpState* __restrict__ st,
                       int32_t Q, int32_t pass, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kQueriesPerBlock][256];
  __shared__ int32_t any;
  const int32_t q0 = blockIdx.y * kQueriesPerBlock;
  const int32_t nq = min(kQueriesPerBlock, Q - q0);
  float2 yi[kQueriesPerBlock];
  uint64_t pre[kQueriesPerBlock];
  int32_t node[kQueriesPerBlock];
  bool live[kQueriesPerBlock];
  if (threadIdx.x == 0) any = 0;
  for (int t = threadIdx.x; t < kQueriesPerBlock * 256; t += blockDim.x) (&h[0][0])[t] = 0u;
  __syncthreads();
#pragma unroll
  for (int a = 0; a < kQueriesPerBlock; ++a) {
    live[a] = false;
    node[a] = -1;
    pre[a] = 0;
    yi[a] = make_float2(0.f, 0.f);
    if (a < nq) {
      const NpState& s = st[q0 + a];
      live[a] = !s.done;
      node[a] = s.node;
      pre[a] = s.prefix;
      yi[a] = Y[s.node];
    }
  }
  bool mine = false;
#pragma unroll
  for (int a = 0; a < kQueriesPerBlock; ++a) mine = mine || live[a];
  if (threadIdx.x == 0 && mine) any = 1;
  __syncthreads();
  if (!any) return;
  const int shift_pre = pass > 0 ? 64 - 8 * pass : 0;  // bits above the current digit
  const int shift_dig = 56 - 8 * pass;
  for (int64_t l = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; l < n;
       l += int64_t(gridDim.x) * blockDim.x) {
    const float2 yl = Y[l];
#pragma unroll
    for (int a = 0; a < kQueriesPerBlock; ++a) {
      if (!live[a] || l == node[a]) continue;
      const uint64_t key = np_key(yl, yi[a], l);
      if (pass > 0 && (key >> shift_pre) != pre[a]) continue;
      atomicAdd(&h[a][(key >> shift_dig) & 0xFF], 1u);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nq * 256; t += blockDim.x) {
    const uint32_t v = (&h[0][0])[t];
    if (v) atomicAdd(hist + static_cast<int64_t>(q0) * 256 + t, v);
  }
}

// Pick the bin holding the need-th key (1-based) and clear the histogram.
__global__ void select_pick_kernel(NpState* st, int32_t Q, int32_t pass,
                                   uint32_t* __restrict__ hist) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q) return;
  uint32_t* hq = hist + static_cast<int64_t>(q) * 256;
  NpState s = st[q];
  if (!s.done) {
    int64_t before = 0;
    int bin = 255;
    for (int b = 0; b < 256; ++b) {
      if (before + hq[b] >= s.need) {
        bin = b;
        break;
      }
      before += hq[b];
    }
    const int64_t in_bin = hq[bin];
    s.need -= before;
    s.prefix = (s.prefix << 8) | static_cast<uint64_t>(bin);
    const int low = 56 - 8 * pass;  // bits below this digit
    if (s.need == in_bin || pass == 7) {
      // every key of this prefix is among the k nearest
      const uint64_t low_mask = low > 0 ? ((uint64_t(1) << low) - 1) : 0;
      s.thr_key = (s.prefix << low) | low_mask;
      s.done = 1;
    }
    st[q] = s;
  }
  for (int b = 0; b < 256; ++b) hq[b] = 0u;
}

__global__ void __launch_bounds__(256)
    ring_intersect_kernel(const uint32_t* __restrict__ bits, int64_t words,
                          const float2* __restrict__ Y, NpState* st) {
  __shared__ int32_t red[4];
  const int32_t q = blockIdx.y;
  const uint32_t* b = bits + static_cast<int64_t>(q) * words;
  const int32_t i = st[q].node;
  const uint64_t thr = st[q].thr_key;
  const float2 yi = Y[i];
  int32_t c = 0;
  if (st[q].k > 0) {
    for (int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < words;
         w += static_cast<int64_t>(gridDim.x) * blockDim.x) {
      uint32_t m = b[w];
      while (m) {
        const int bit = __ffs(m) - 1;
        m &= m - 1;
        const int32_t l = static_cast<int32_t>(w * 32 + bit);
        if (l != i && np_key(Y[l], yi, l) <= thr) ++c;
      }
    }
  }
  c = block_sum_i32(c, red);
  if (threadIdx.x == 0 && c) atomicAdd(&st[q].inter, c);
}

}  // namespace

int neighbourhood_counts(hipStream_t stream, const int64_t* d_row, const int32_t* d_col,
                         const float2* d_Y, int32_t n, const int32_t* nodes, int32_t count,
                         int32_t radius, int32_t* k_out, int32_t* inter_out) {
  if (count <= 0) return LAYOUT_OK;
  const int64_t words = div_up(n, 32);
  const int64_t fit = std::max<int64_t>(1, kScratchBytes / (words * 4));
  const int32_t Q = static_cast<int32_t>(std::min<int64_t>({count, kMaxBatch, fit}));
  uint32_t *d_bits = nullptr, *d_hist = nullptr;
  NpState* d_st = nullptr;
  hipError_t e = hipMalloc(&d_bits, sizeof(uint32_t) * size_t(words) * size_t(Q));
  if (e == hipSuccess) e = hipMalloc(&d_hist, sizeof(uint32_t) * 256 * size_t(Q));
  if (e == hipSuccess) e = hipMalloc(&d_st, sizeof(NpState) * size_t(Q));
  std::vector<NpState> hs(Q);
  const int groups = static_cast<int>(div_up(Q, kQueriesPerBlock));
  const int gx_hist = static_cast<int>(
      std::max<int64_t>(1, std::min<int64_t>(div_up(n, 4096), std::max(1, 4096 / groups))));
  const int gx_words = static_cast<int>(
      std::max<int64_t>(1, std::min<int64_t>(div_up(words, 2048), std::max(1, 4096 / Q))));
  if (e == hipSuccess)
    launch_fill_i32(stream, reinterpret_cast<int32_t*>(d_hist), int64_t(256) * Q, 0);
  for (int32_t b0 = 0; b0 < count && e == hipSuccess; b0 += Q) {
    const int32_t nb = std::min(Q, count - b0);
    for (int32_t a = 0; a < nb; ++a) {
      hs[a] = NpState{};
      hs[a].node = nodes[b0 + a];
    }
    e = hipMemcpyAsync(d_st, hs.data(), sizeof(NpState) * size_t(nb), hipMemcpyHostToDevice,
                       stream);
    if (e != hipSuccess) break;
    launch_fill_i32(stream, reinterpret_cast<int32_t*>(d_bits), words * nb, 0);
    // 64 workgroups per query share its row (hop 1) and its neighbours' rows (hop 2)
    hipLaunchKernelGGL(ring_mark_kernel, dim3(64, nb), dim3(256), 0, stream, d_row, d_col, d_st,
                       radius, d_bits, words);
    hipLaunchKernelGGL(ring_count_kernel, dim3(gx_words, nb), dim3(256), 0, stream, d_bits,
                       words, d_st);
    hipLaunchKernelGGL(select_init_kernel, dim3(div_up(nb, 256)), dim3(256), 0, stream, d_bits,
                       words, d_st, nb);
    const int nb_groups = static_cast<int>(div_up(nb, kQueriesPerBlock));
    for (int32_t pass = 0; pass < 8; ++pass) {
      hipLaunchKernelGGL(select_hist_kernel, dim3(gx_hist, nb_groups), dim3(256), 0, stream, d_Y,
                         n, d_st, nb, pass, d_hist);
      hipLaunchKernelGGL(select_pick_kernel, dim3(div_up(nb, 64)), dim3(64), 0, stream, d_st,
                         nb, pass, d_hist);
    }
    hipLaunchKernelGGL(ring_intersect_kernel, dim3(gx_words, nb), dim3(256), 0, stream, d_bits,
                       words, d_Y, d_st);
    e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(hs.data(), d_st, sizeof(NpState) * size_t(nb), hipMemcpyDeviceToHost,
                         stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) break;
    for (int32_t a = 0; a < nb; ++a) {
      k_out[b0 + a] = hs[a].k;
      inter_out[b0 + a] = hs[a].inter;
    }
  }
  if (d_bits) (void)hipFree(d_bits);
  if (d_hist) (void)hipFree(d_hist);
  if (d_st) (void)hipFree(d_st);
  if (e != hipSuccess) return hip_fail(e, "neighbourhood preservation");
  return LAYOUT_OK;
}

}  // namespace snap
