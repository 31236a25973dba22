// Row-aligned chunk table of a layout job (built on the device at create).
//
// A chunk is the unit of work of one lane: a run of whole CSR rows (bundles,
// Sec. 3.4: all out-edges of a source handled by one worker) of about B
// edges, or one segment of at most H edges of a hub row (degree > H), so that
// one long row cannot serialise an epoch.  Boundaries:
//   * the row holding edge b*B starts a chunk, for every b (rows that start in
//     the same B-bucket share a chunk; a chunk ends where the next starts);
//   * a hub row is cut at offsets 0, H, 2H, ... of the row, and the first
//     non-empty row after a hub starts a new chunk.
// chunk_begin[c] (64-bit) is the first edge of chunk c (chunk_begin[n_chunks] = nnz),
// chunk_src[c] the row holding that edge.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "scan.hpp"

namespace snap {

static __global__ void chunk_flag_buckets_kernel(const int64_t* __restrict__ row_ptr, int32_t n,
                                          int64_t nnz, int32_t bundle,
                                          uint8_t* __restrict__ flags) {
  const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b * bundle >= nnz) return;
  flags[row_of(row_ptr, n, b * bundle)] = 1;
}

static __global__ void chunk_flag_hubs_kernel(const int64_t* __restrict__ row_ptr, int32_t n,
                                       int64_t nnz, int32_t hub, uint8_t* __restrict__ flags) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t d = row_ptr[i + 1] - row_ptr[i];
  if (d <= hub) return;
  flags[i] = 1;
  if (row_ptr[i + 1] < nnz) flags[row_of(row_ptr, n, row_ptr[i + 1])] = 1;
}

// chunks starting in row i
struct ChunkCountLoad {
  const int64_t* row_ptr;
  const uint8_t* flags;
  int32_t n, hub;
  __device__ int32_t operator()(int64_t i) const {
    if (i >= n || !flags[i]) return 0;
    const int64_t d = row_ptr[i + 1] - row_ptr[i];
    return d > hub ? static_cast<int32_t>((d + hub - 1) / hub) : 1;
  }
};

struct ChunkWrite {
  const int64_t* row_ptr;
  int32_t hub;
  int64_t* chunk_begin;
  int32_t* chunk_src;
  __device__ void operator()(int64_t i, int32_t off, int32_t cnt) const {
    for (int32_t m = 0; m < cnt; ++m) {
      chunk_begin[off + m] = row_ptr[i] + int64_t(m) * hub;
      chunk_src[off + m] = static_cast<int32_t>(i);
    }
  }
};

static __global__ void chunk_sentinel_kernel(int64_t* __restrict__ chunk_begin,
                                      const int32_t* __restrict__ n_chunks, int64_t nnz) {
  chunk_begin[*n_chunks] = nnz;
}

}  // namespace snap
