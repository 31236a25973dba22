// Device construction of the integer alias table used by degree-weighted
// negatives (Walker's alias method; Vose's light/heavy pairing), reproducing a
// deterministic sequential sweep exactly, in parallel.
//
// Definition (the sweep).  Item s has mass M_s = w_s * n against a bin of
// capacity W = sum_s w_s.  Lights (M < W) are visited in index order; each
// takes its deficit W - M from the current heavy (heavies in index order).  A
// heavy whose residual drops below W turns into a partial bin -- own mass r,
// alias the next heavy -- and the next heavy absorbs its deficit W - r (this can
// chain).  Light bins store thr = floor(M * 2^32 / W), partial heavies
// floor(r * 2^32 / W), untouched heavies thr = 0xFFFFFFFF with alias = self.
//
// Parallel form.  With E_h = M_h - W (heavy excess, heavies in index order),
// D_l = W - M_l (light deficit, lights in index order), and inclusive prefix
// sums SE_h = sum_{h' <= h} E_h', SD_l = sum_{l' <= l} D_l':
//   * light l (exclusive deficit prefix SD_l - D_l = x) is paired with the
//     first heavy h whose SE_h >= x (every earlier heavy is exhausted);
//   * heavy h is exhausted iff SE_h < SD_total, by the first light l with
//     SD_l > SE_h; its residual is r = W + SE_h - SD_l and its alias is the
//     next heavy.
// Both are binary searches over the compacted prefix arrays.  Integer only,
// so the result is bit-identical to the sequential sweep.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scan.hpp"

namespace snap {

struct AliasScanItem {
  int64_t excess;   // heavy: M - W, else 0
  int64_t deficit;  // light: W - M, else 0
  int32_t heavy;    // 1 for heavy
  int32_t pad;
};

__device__ __forceinline__ AliasScanItem operator+(const AliasScanItem& a,
                                                   const AliasScanItem& b) {
  return AliasScanItem{a.excess + b.excess, a.deficit + b.deficit, a.heavy + b.heavy, 0};
}

// Weight of item s: weights[s] when given, else the degree of s.
__device__ __forceinline__ int64_t alias_weight(const int64_t* __restrict__ row_ptr,
                                                const uint32_t* __restrict__ weights, int64_t s) {
  return weights ? static_cast<int64_t>(weights[s])
                 : static_cast<int64_t>(row_ptr[s + 1] - row_ptr[s]);
}

// Item s of the scan: heavy/light classification of M_s = w_s * n against W.
struct AliasLoad {
  const int64_t* row_ptr;
  const uint32_t* weights;  // nullable: degrees
  int64_t n, W;
  __device__ AliasScanItem operator()(int64_t s) const {
    AliasScanItem it{0, 0, 0, 0};
    if (s < n) {
      const int64_t M = alias_weight(row_ptr, weights, s) * n;
      if (M >= W) {
        it.excess = M - W;
        it.heavy = 1;
      } else {
        it.deficit = W - M;
      }
    }
    return it;
  }
};

// Scatter of each item into the compacted heavy or light arrays, with its
// inclusive prefix sum (heavy excess or light deficit).
struct AliasCompact {
  int32_t* heavy_item;
  int64_t* heavy_inc;
  int32_t* light_item;
  int64_t* light_inc;
  __device__ void operator()(int64_t s, AliasScanItem ex, AliasScanItem raw) const {
    if (raw.heavy) {
      heavy_item[ex.heavy] = static_cast<int32_t>(s);
      heavy_inc[ex.heavy] = ex.excess + raw.excess;
    } else {
      const int64_t lrank = s - ex.heavy;
      light_item[lrank] = static_cast<int32_t>(s);
      light_inc[lrank] = ex.deficit + raw.deficit;
    }
  }
};

// first index in [0, len) with a[idx] >= x (len if none)
__device__ __forceinline__ int64_t lower_bound64(const int64_t* __restrict__ a, int64_t len,
                                                 int64_t x) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// first index in [0, len) with a[idx] > x (len if none)
__device__ __forceinline__ int64_t upper_bound64(const int64_t* __restrict__ a, int64_t len,
                                                 int64_t x) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] <= x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint32_t alias_threshold(int64_t own, int64_t W) {
  // own < W < 2^32, so own * 2^32 fits in 64 bits
  return static_cast<uint32_t>((static_cast<uint64_t>(own) << 32) / static_cast<uint64_t>(W));
}

// Phase 4: one thread per item writes thr/alias.
static __global__ void alias_fill_kernel(const int64_t* __restrict__ row_ptr,
                                  const uint32_t* __restrict__ weights, int64_t n, int64_t W,
                                  const AliasScanItem* __restrict__ grand,
                                  const int32_t* __restrict__ heavy_item,
                                  const int64_t* __restrict__ heavy_inc,
                                  const int32_t* __restrict__ light_item,
                                  const int64_t* __restrict__ light_inc,
                                  uint32_t* __restrict__ thr, uint32_t* __restrict__ alias) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nh = grand->heavy;
  const int64_t nl = n - nh;
  const int64_t total_deficit = grand->deficit;
  if (r < nl) {
    // light of rank r
    const int32_t s = light_item[r];
    const int64_t M = alias_weight(row_ptr, weights, s) * n;
    const int64_t x = light_inc[r] - (W - M);  // exclusive deficit prefix
    const int64_t h = lower_bound64(heavy_inc, nh, x);
    thr[s] = alias_threshold(M, W);
    alias[s] = static_cast<uint32_t>(heavy_item[h < nh ? h : nh - 1]);
  }
  if (r < nh) {
    const int32_t s = heavy_item[r];
    const int64_t se = heavy_inc[r];
    if (se < total_deficit && r + 1 < nh) {
      const int64_t l = upper_bound64(light_inc, nl, se);
      const int64_t own = W + se - light_inc[l];
      thr[s] = alias_threshold(own, W);
      alias[s] = static_cast<uint32_t>(heavy_item[r + 1]);
    } else {
      thr[s] = 0xFFFFFFFFu;
      alias[s] = static_cast<uint32_t>(s);
    }
  }
}

}  // namespace snap
