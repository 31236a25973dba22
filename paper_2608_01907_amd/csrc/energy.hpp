// Energy monitors (Sec. 3.3).
//
// The t-forces of Table 1 are the negative gradients (Eq. (2)) of the pair
// potentials
//   U_a(q) = alpha * (q/2 + (beta/2) ln(1 + q))           attraction
//   U_r(q) = (1 + q)^(1 - gamma) / (2 (gamma - 1))        repulsion
// of the squared distance q = |y_i - y_j|^2.  Two totals are monitored:
//   * the sampled energy of epoch t: U_a over every directed edge plus U_r over
//     the k negatives that edge draws in epoch t (the same draws as the epoch
//     kernel);
//   * the degree-weighted objective that the sampling realises in expectation:
//     the same attraction plus k/(n-1) * sum_{i<j} (d_i + d_j) U_r(q_ij).
// The first is a stream over the edges with random gathers; the second is a
// dense all-pairs sweep bound by the vector ALUs.  The exact silhouette index
// of a layout (a quality metric of Sec. 4.1) is the same kind of sweep.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace snap {

__device__ __forceinline__ float energy_attr_f(float q, float alpha, float beta) {
  return alpha * (0.5f * q + 0.5f * beta * log1pf(q));
}

// U_r without its constant factor 1 / (2 (gamma - 1)), applied by the host.
__device__ __forceinline__ float energy_rep_shape(float q, float gamma) {
  const float r = 1.0f / (1.0f + q);
  if (gamma == 2.0f) return r;
  return powf(r, gamma - 1.0f);
}

// Sum of two doubles over the workgroup, then one atomic add per workgroup.
template <int BLOCK>
__device__ __forceinline__ void block_add2(double a, double b, double* out) {
  static_assert(BLOCK % 64 == 0, "whole wavefronts");
  __shared__ double sa[BLOCK / 64], sb[BLOCK / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sa[wave] = a;
    sb[wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) {
      ta += sa[w];
      tb += sb[w];
    }
    atomicAdd(out, ta);
    atomicAdd(out + 1, tb);
  }
}

// out[0] += sum of U_a over the directed edges, out[1] += sum of the repulsion
// shape over the drawn negatives (K = 0: attraction only).  One lane per chunk
// of the chunk table, so every directed edge is visited once.
template <int K, bool DEGREE>
static __global__ void __launch_bounds__(256)
    sampled_energy_kernel(const GraphDesc* __restrict__ table, int64_t n_chunks, int32_t t,
                          double* __restrict__ out) {
  constexpr int KS = K > 0 ? K : 1;
  const GraphDesc& g = table[0];
  const float2* __restrict__ Y = g.Y;
  double ea = 0.0, er = 0.0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < n_chunks; c += stride) {
    const int64_t e0 = g.chunk_begin[c];
    const int64_t e_end = g.chunk_begin[c + 1];
    int32_t i = g.chunk_src[c];
    int64_t row_end = g.row_ptr[i + 1];
    float2 yi = Y[i];
    for (int64_t e = e0; e < e_end; ++e) {
      if (e >= row_end) {
        do {
          ++i;
          row_end = g.row_ptr[i + 1];
        } while (e >= row_end);
        yi = Y[i];
      }
      const int32_t j = g.col[e];
      const float2 yj = Y[j];
      float dx = yi.x - yj.x, dy = yi.y - yj.y;
      ea += energy_attr_f(dx * dx + dy * dy, g.alpha, g.beta);
      if constexpr (K > 0) {
        uint32_t s[KS];
        draw_k<K, DEGREE>(g, e, static_cast<uint32_t>(t), static_cast<uint32_t>(i), s);
#pragma unroll
        for (int m = 0; m < K; ++m) {
          const float2 ys = Y[s[m]];
          dx = yi.x - ys.x;
          dy = yi.y - ys.y;
          er += energy_rep_shape(dx * dx + dy * dy, g.gamma);
        }
      }
    }
  }
  block_add2<256>(ea, er, out);
}

// out[1] += sum over ordered pairs i != j of (d_i + d_j) * shape(q_ij), i.e.
// twice the sum over unordered pairs.  Workgroup (bx, by) owns the 256 rows
// i of tile bx and the column tiles by, by + gridDim.y, ...; each column tile
// is staged in LDS.  A tile's 256 terms are summed in FP32 and then added to
// an FP64 accumulator, which bounds the rounding of any partial sum to 256
// terms.
static __global__ void __launch_bounds__(256)
    pair_energy_kernel(const float2* __restrict__ Y, const int64_t* __restrict__ row_ptr,
                       int32_t n, float gamma, double* __restrict__ out) {
  __shared__ float2 ty[256];
  __shared__ float td[256];
  const int32_t i = int32_t(blockIdx.x) * 256 + int32_t(threadIdx.x);
  const bool live = i < n;
  const float2 yi = live ? Y[i] : make_float2(0.f, 0.f);
  const float di = live ? float(row_ptr[i + 1] - row_ptr[i]) : 0.f;
  const int32_t tiles = (n + 255) / 256;
  double acc = 0.0;
  for (int32_t tj = int32_t(blockIdx.y); tj < tiles; tj += int32_t(gridDim.y)) {
    const int32_t jb = tj * 256;
    const int32_t jl = jb + int32_t(threadIdx.x);
    __syncthreads();  // the previous tile is no longer read
    if (jl < n) {
      ty[threadIdx.x] = Y[jl];
      td[threadIdx.x] = float(row_ptr[jl + 1] - row_ptr[jl]);
    }
    __syncthreads();
    const int32_t cnt = min(256, n - jb);
    float part = 0.f;
    if (gamma == 2.0f) {
      for (int32_t q = 0; q < cnt; ++q) {
        const float dx = yi.x - ty[q].x, dy = yi.y - ty[q].y;
        const float w = (jb + q == i) ? 0.f : di + td[q];
        part += w * __builtin_amdgcn_rcpf(1.0f + dx * dx + dy * dy);
      }
    } else {
      const float ex = gamma - 1.0f;
      for (int32_t q = 0; q < cnt; ++q) {
        const float dx = yi.x - ty[q].x, dy = yi.y - ty[q].y;
        const float w = (jb + q == i) ? 0.f : di + td[q];
        // (1+q)^(1-gamma) = 2^(-(gamma-1) log2(1+q))
        part += w * __builtin_amdgcn_exp2f(-ex * __builtin_amdgcn_logf(1.0f + dx * dx + dy * dy));
      }
    }
    if (live) acc += double(part);
  }
  block_add2<256>(0.0, acc, out);
}

// out[q] = Y[order[q]]
static __global__ void gather_positions_kernel(const float2* __restrict__ Y,
                                               const int32_t* __restrict__ order, int32_t n,
                                               float2* __restrict__ out) {
  const int32_t q = int32_t(blockIdx.x) * blockDim.x + int32_t(threadIdx.x);
  if (q < n) out[q] = Y[order[q]];
}

// Silhouette index (the SI metric of Sec. 4.1) of all nodes for given
// clusters, exactly: s(i) = (b_i - a_i) / max(a_i, b_i) with a_i the mean
// distance from i to the other members of its cluster and b_i the smallest
// mean distance to another cluster (s = 0 for a node alone in its cluster).
// Positions arrive sorted by cluster (Ys, cs; cluster c spans
// [cstart[c], cstart[c+1])).  One lane per node i; every lane sweeps all
// nodes in 256-node LDS tiles, so a cluster boundary inside a tile is the
// same for all lanes (uniform branch).  Distances are summed in FP32 within a
// tile and in FP64 across tiles.  out[0] += sum over the block of s(i).
static __global__ void __launch_bounds__(256)
    silhouette_kernel(const float2* __restrict__ Ys, const int32_t* __restrict__ cs,
                      const int32_t* __restrict__ cstart, int32_t n, double* __restrict__ out) {
  __shared__ float2 ty[256];
  __shared__ int32_t tc[256];
  const int32_t i = int32_t(blockIdx.x) * 256 + int32_t(threadIdx.x);
  const bool live = i < n;
  const float2 yi = live ? Ys[i] : make_float2(0.f, 0.f);
  const int32_t ci = live ? cs[i] : -1;
  double a = 0.0, b = 1.0e300, acc = 0.0;
  int32_t cur = -1;
  float part = 0.f;
  const int32_t tiles = (n + 255) / 256;
  for (int32_t t = 0; t < tiles; ++t) {
    const int32_t jb = t * 256;
    const int32_t jl = jb + int32_t(threadIdx.x);
    __syncthreads();
    if (jl < n) {
      ty[threadIdx.x] = Ys[jl];
      tc[threadIdx.x] = cs[jl];
    }
    __syncthreads();
    const int32_t cnt = min(256, n - jb);
    for (int32_t q = 0; q < cnt; ++q) {
      const int32_t c = tc[q];
      if (c != cur) {  // the same for every lane of the block
        if (cur >= 0) {
          acc += double(part);
          const int32_t size = cstart[cur + 1] - cstart[cur];
          if (cur == ci)
            a = size > 1 ? acc / double(size - 1) : 0.0;
          else
            b = fmin(b, acc / double(size));
        }
        cur = c;
        acc = 0.0;
        part = 0.f;
      }
      const float dx = yi.x - ty[q].x, dy = yi.y - ty[q].y;
      part += sqrtf(dx * dx + dy * dy);
    }
    acc += double(part);
    part = 0.f;
  }
  if (cur >= 0) {
    const int32_t size = cstart[cur + 1] - cstart[cur];
    if (cur == ci)
      a = size > 1 ? acc / double(size - 1) : 0.0;
    else
      b = fmin(b, acc / double(size));
  }
  double si = 0.0;
  if (live) {
    const int32_t own = cstart[ci + 1] - cstart[ci];
    const double m = fmax(a, b);
    si = (own > 1 && m > 0.0) ? (b - a) / m : 0.0;
  }
  block_add2<256>(si, 0.0, out);
}

}  // namespace snap
