// Per-graph descriptor read by the epoch kernels (one entry per graph of a
// launch: a single layout job, a packed batch, or the active jobs of a server
// round).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rng.hpp"

namespace snap {

// Update policies (Sec. 3.4 lock-free scheme; see kernels.hpp).
enum : int { kStore = 0, kAtomic = 1, kJacobi = 2 };

// Kernels of the forces (the values of layout_opts.force_kernel).
enum : int { kForceT = 0, kForceGaussian = 1 };

struct GraphDesc {
  const int64_t* row_ptr;
  const int32_t* col;
  const int64_t* chunk_begin;  // first edge of each chunk; [n_chunks] = nnz
  const int32_t* chunk_src;    // row holding the first edge of each chunk
  float2* Y;
  float2* D;  // Jacobi accumulator (JACOBI only)
  const uint32_t* thr;    // alias table (degree-weighted negatives only)
  const uint32_t* alias;
  // HOGWILD_STORE on the global engine: bitmap of the nodes whose updates as
  // the far end of an edge are committed as atomic adds of the change
  // instead of stores (nodes of high degree, where concurrent updates
  // collide); null = none
  const uint32_t* hot = nullptr;
  int64_t chunk_base;    // offset of this graph's slice inside one round of the launch
  int64_t slice;         // chunks of this graph per round of the launch
  int64_t chunk_offset;  // first chunk of the graph's table processed by the launch
  int64_t n_chunks;      // chunks processed by the launch
  int64_t nnz;
  int32_t n;
  int32_t hub;     // rows longer than this are split into segments of hub edges
  int32_t t0;      // epoch index at launch offset 0
  int32_t T;       // epochs in the step-size schedule
  int32_t lanes;   // LDS engine: lanes of the workgroup that work (0 = all)
  int32_t force;   // kernel of the forces: kForceT (Table 1, t-FDP) or kForceGaussian
  uint64_t seed;
  float eta0, alpha, beta, gamma;
  SamplerConsts sc;
};

// Multi-graph launches on the XCD-local engine.  The graphs are split into
// bins, one per XCD; a bin's graphs run in sequence segments whose positions
// fit the XCD's L2 together, each segment with its own lane cap and chunk
// counter.  Inside a segment the chunk positions are cut into rounds as for
// the global engine (GraphDesc::slice, chunk_base).
constexpr int kXcds = 8;  // accelerator complex dies of the device

struct XcdSeg {
  int64_t total_index;  // positions of the segment (rounds x round_size)
  int64_t round_size;   // positions per round (sum of the slices of its graphs)
  int32_t table_begin;  // first table entry of the segment
  int32_t G;            // table entries of the segment
  int32_t workers;      // workgroups that serve the segment (its graphs' lane cap)
  int32_t pad0;
};

struct XcdBin {
  int32_t seg_begin, seg_count;  // the bin's segments, run in this order
  int32_t workers;               // the most workers any of its segments takes
  int32_t pad0;
};

}  // namespace snap
