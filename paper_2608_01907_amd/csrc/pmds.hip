// Pivot MDS initial layout on the device (Sec. 4.1 initialises every layout
// with Pivot MDS: Brandes and Pich, "Eigensolver methods for progressive
// multidimensional scaling of large data", GD 2006).
//
// The paper fixes neither the pivot count nor the pivot rule.  Definition
// implemented here:
//   1. first pivot: the node of largest degree (smallest index on ties); each
//      further pivot: the node of the first pivot's connected component whose
//      smallest hop distance to the chosen pivots is largest (smallest index
//      on ties); min(p, component size) pivots;
//   2. d_ij: breadth-first hop distance from pivot j to node i;
//   3. c_ij = -1/2 (d_ij^2 - colmean_j - rowmean_i + grandmean) over the
//      component's m nodes (double centring of the squared distances);
//   4. v1, v2: eigenvectors of the two largest eigenvalues mu1 >= mu2 of the
//      p x p matrix C^T C (cyclic Jacobi, FP64, one workgroup);
//   5. x_i = (C v1 / mu1^(1/4), C v2 / mu2^(1/4)): the left singular vectors
//      of C scaled by the square roots of its singular values, which is
//      classical MDS when every node is a pivot; an axis with mu <= 1e-6 mu1
//      is 0 (below the rounding noise of an FP32 C);
//   6. scale s = sum d_ij |x_i - x_pj| / sum |x_i - x_pj|^2 (least-squares
//      fit of the layout distances to the pivot hop distances; 1 if 0/0);
//   7. nodes outside the component: the seeded uniform draws of the plain
//      initial layout in [-R, R]^2, R = largest |coordinate| of the scaled
//      component layout (1 if 0).
//
// Work: one level-synchronous BFS per pivot (frontier rows up to
// kLightDegree edges handled by one lane, longer rows by a whole workgroup),
// then one pass over the p x n distances for C^T C (256-row slabs staged in
// LDS), a single-workgroup eigensolver, and two passes for the coordinates
// and the scale fit.  Distances are stored pivot-major (p x n int32).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "snaplayout.h"

namespace snap {
namespace {

constexpr int kMaxPivots = 64;
constexpr int kLightDegree = 128;
constexpr int kPairsMax = kMaxPivots * (kMaxPivots + 1) / 2;
constexpr int kPairsPerThread = (kPairsMax + 255) / 256;

// larger value first, then smaller index; value >= -1
__device__ __forceinline__ uint64_t argmax_key(int32_t value, int32_t v) {
  return (static_cast<uint64_t>(static_cast<uint32_t>(value + 1)) << 32) |
         static_cast<uint64_t>(0xFFFFFFFFu - static_cast<uint32_t>(v));
}
__device__ __forceinline__ int32_t key_node(uint64_t key) {
  return static_cast<int32_t>(0xFFFFFFFFu - static_cast<uint32_t>(key));
}

template <class T, class Op>
__device__ __forceinline__ T block_reduce(T x, Op op, T* scratch /* [4] */) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = op(x, __shfl_down(x, off, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[wave] = x;
  __syncthreads();
  T r = scratch[0];
  for (int w = 1; w < static_cast<int>(blockDim.x >> 6); ++w) r = op(r, scratch[w]);
  return r;
}

struct MaxU64 {
  __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a > b ? a : b; }
};
struct SumF64 {
  __device__ double operator()(double a, double b) const { return a + b; }
};
struct SumU64 {
  __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a + b; }
};
struct MaxF32 {
  __device__ float operator()(float a, float b) const { return fmaxf(a, b); }
};

// ---------------------------------------------------------------- pivots/BFS
__global__ void __launch_bounds__(256)
    degree_argmax_kernel(const int64_t* __restrict__ row, int32_t n, uint64_t* best) {
  __shared__ uint64_t red[4];
  uint64_t k = 0;
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += int64_t(gridDim.x) * blockDim.x) {
    const uint64_t c = argmax_key(static_cast<int32_t>(row[v + 1] - row[v]), v);
    k = c > k ? c : k;
  }
  k = block_reduce(k, MaxU64{}, red);
  if (threadIdx.x == 0) atomicMax(reinterpret_cast<unsigned long long*>(best), k);
}

__global__ void __launch_bounds__(256)
    bfs_start_kernel(int32_t* __restrict__ dist, int32_t n, const uint64_t* best,
                     int32_t* __restrict__ pivots, int32_t j) {
  const int32_t src = key_node(*best);
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += int64_t(gridDim.x) * blockDim.x)
    dist[v] = v == src ? 0 : -1;
  if (blockIdx.x == 0 && threadIdx.x == 0) pivots[j] = src;
}

// Rows of the frontier (dist == level): short rows by one lane, long rows
// queued for bfs_heavy_kernel.  Concurrent discoverers of a node all write the
// same value, so no atomics are needed on dist.  flags[0]: a node was
// discovered; flags[1]: queued long rows.
__global__ void __launch_bounds__(256)
    bfs_level_kernel(const int64_t* __restrict__ row, const int32_t* __restrict__ col,
                     int32_t* dist, int32_t n, int32_t level, int32_t* flags,
                     int32_t* __restrict__ heavy) {
  bool found = false;
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += int64_t(gridDim.x) * blockDim.x) {
    if (dist[v] != level) continue;
    const int64_t b = row[v], e = row[v + 1];
    if (e - b > kLightDegree) {
      heavy[atomicAdd(&flags[1], 1)] = v;
      continue;
    }
    for (int64_t q = b; q < e; ++q) {
      const int32_t u = col[q];
      if (dist[u] < 0) {
        dist[u] = level + 1;
        found = true;
      }
    }
  }
  if (found) flags[0] = 1;
}

__global__ void __launch_bounds__(256)
    bfs_heavy_kernel(const int64_t* __restrict__ row, const int32_t* __restrict__ col,
                     int32_t* dist, int32_t level, int32_t* flags,
                     const int32_t* __restrict__ heavy) {
  const int32_t count = flags[1];
  bool found = false;
  for (int32_t h = blockIdx.x; h < count; h += gridDim.x) {
    const int32_t v = heavy[h];
    const int64_t e = row[v + 1];
    for (int64_t q = row[v] + threadIdx.x; q < e; q += blockDim.x) {
      const int32_t u = col[q];
      if (dist[u] < 0) {
        dist[u] = level + 1;
        found = true;
      }
    }
  }
  if (found) flags[0] = 1;
}

// After the BFS of pivot j: smallest distance to the pivots so far (-1 marks
// nodes outside the first pivot's component), the column sum of d^2 over the
// component, its size (first pivot only), and the key of the next pivot.
__global__ void __launch_bounds__(256)
    pivot_update_kernel(const int32_t* __restrict__ dist, int32_t* __restrict__ mind, int32_t n,
                        int32_t first, double* colsum, uint64_t* comp_count, uint64_t* best) {
  __shared__ uint64_t redk[4];
  __shared__ double reds[4];
  __shared__ uint64_t redc[4];
  uint64_t k = 0, cnt = 0;
  double s = 0.0;
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += int64_t(gridDim.x) * blockDim.x) {
    const int32_t d = dist[v];
    int32_t m;
    if (first) {
      m = d;
      cnt += d >= 0 ? 1 : 0;
    } else {
      m = mind[v];
      if (m >= 0) m = min(m, d);
    }
    mind[v] = m;
    if (m >= 0) {
      s += static_cast<double>(d) * static_cast<double>(d);
      const uint64_t c = argmax_key(m, v);
      k = c > k ? c : k;
    }
  }
  k = block_reduce(k, MaxU64{}, redk);
  s = block_reduce(s, SumF64{}, reds);
  cnt = block_reduce(cnt, SumU64{}, redc);
  if (threadIdx.x == 0) {
    atomicMax(reinterpret_cast<unsigned long long*>(best), k);
    atomicAdd(colsum, s);
    if (first) atomicAdd(reinterpret_cast<unsigned long long*>(comp_count), cnt);
  }
}

// ------------------------------------------------------------------- C^T C
struct Centring {
  double colmean[kMaxPivots];
  double grand;
};

__device__ __forceinline__ void load_centring(const double* colsum, int32_t p, double inv_m,
                                              Centring& c) {
  if (threadIdx.x < static_cast<unsigned>(p)) c.colmean[threadIdx.x] = colsum[threadIdx.x] * inv_m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double g = 0.0;
    for (int j = 0; j < p; ++j) g += c.colmean[j];
    c.grand = g / p;
  }
  __syncthreads();
}

// Row i of C from the p distances of node v (component node).
__device__ __forceinline__ double row_mean_sq(const int32_t* __restrict__ dist, int64_t n,
                                              int32_t p, int32_t v) {
  double r = 0.0;
  for (int j = 0; j < p; ++j) {
    const double d = dist[j * n + v];
    r += d * d;
  }
  return r / p;
}

// G[a][b] += sum over component rows of c_ia c_ib.  A workgroup stages 256
// rows of C in LDS (FP32), each lane owns up to kPairsPerThread (a, b) pairs
// with a <= b, sums a slab's 256 products in FP32 and adds them to FP64
// accumulators; one FP64 atomic per pair and workgroup at the end.
__global__ void __launch_bounds__(256)
    gram_kernel(const int32_t* __restrict__ dist, const int32_t* __restrict__ mind, int32_t n,
                int32_t p, const double* __restrict__ colsum, double inv_m,
                double* __restrict__ G) {
  __shared__ float slab[256][kMaxPivots + 1];
  __shared__ Centring cen;
  load_centring(colsum, p, inv_m, cen);
  const int npairs = p * (p + 1) / 2;
  int pa[kPairsPerThread], pb[kPairsPerThread];
  double acc[kPairsPerThread];
#pragma unroll
  for (int r = 0; r < kPairsPerThread; ++r) {
    acc[r] = 0.0;
    pa[r] = pb[r] = 0;
    const int q = threadIdx.x + r * 256;
    if (q < npairs) {
      // q -> (a, b), a <= b, row-major over the upper triangle
      int a = 0, rem = q;
      while (rem >= p - a) {
        rem -= p - a;
        ++a;
      }
      pa[r] = a;
      pb[r] = a + rem;
    }
  }
  for (int64_t base = int64_t(blockIdx.x) * 256; base < n; base += int64_t(gridDim.x) * 256) {
    const int64_t v = base + threadIdx.x;
    __syncthreads();  // the previous slab is no longer read
    if (v < n && mind[v] >= 0) {
      const double rmean = row_mean_sq(dist, n, p, static_cast<int32_t>(v));
      for (int j = 0; j < p; ++j) {
        const double d = dist[j * int64_t(n) + v];
        slab[threadIdx.x][j] =
            static_cast<float>(-0.5 * (d * d - cen.colmean[j] - rmean + cen.grand));
      }
    } else {
      for (int j = 0; j < p; ++j) slab[threadIdx.x][j] = 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPairsPerThread; ++r) {
      if (threadIdx.x + r * 256 >= npairs) continue;
      float part = 0.f;
      for (int row = 0; row < 256; ++row) part += slab[row][pa[r]] * slab[row][pb[r]];
      acc[r] += static_cast<double>(part);
    }
  }
#pragma unroll
  for (int r = 0; r < kPairsPerThread; ++r) {
    if (threadIdx.x + r * 256 >= npairs) continue;
    atomicAdd(&G[pa[r] * p + pb[r]], acc[r]);
    if (pa[r] != pb[r]) atomicAdd(&G[pb[r] * p + pa[r]], acc[r]);
  }
}

// ------------------------------------------------------------- eigensolver
// Cyclic Jacobi on the symmetric p x p matrix G (FP64, one 64-lane
// workgroup).  A rotation in the plane (a, b) with t = tan(phi) the smaller
// root of t^2 + 2 theta t - 1 = 0, theta = (G_bb - G_aa) / (2 G_ab), zeroes
// G_ab; lanes update the other rows/columns and the eigenvector matrix.
// out = {v1[p], v2[p], mu1, mu2} for the two largest eigenvalues.
__global__ void __launch_bounds__(64)
    eigen_kernel(const double* __restrict__ Gin, int32_t p, double* __restrict__ out) {
  __shared__ double G[kMaxPivots][kMaxPivots + 1];
  __shared__ double V[kMaxPivots][kMaxPivots + 1];
  __shared__ double rot[4];  // c, s, t, g_ab
  __shared__ int done;
  const int k = threadIdx.x;
  for (int a = 0; a < p; ++a)
    if (k < p) {
      G[a][k] = Gin[a * p + k];
      V[a][k] = a == k ? 1.0 : 0.0;
    }
  __syncthreads();
  for (int sweep = 0; sweep < 50; ++sweep) {
    if (k == 0) {
      double off = 0.0, diag = 0.0;
      for (int a = 0; a < p; ++a) {
        diag += fabs(G[a][a]);
        for (int b = a + 1; b < p; ++b) off += G[a][b] * G[a][b];
      }
      done = (sqrt(off) <= 1e-15 * diag) ? 1 : 0;
    }
    __syncthreads();
    if (done) break;
    for (int a = 0; a < p - 1; ++a)
      for (int b = a + 1; b < p; ++b) {
        if (k == 0) {
          const double gab = G[a][b];
          double t = 0.0;
          if (gab != 0.0) {
            const double th = (G[b][b] - G[a][a]) / (2.0 * gab);
            t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          }
          const double c = 1.0 / sqrt(1.0 + t * t);
          rot[0] = c;
          rot[1] = t * c;
          rot[2] = t;
          rot[3] = gab;
        }
        __syncthreads();
        const double gab = rot[3];
        if (gab != 0.0) {
          const double c = rot[0], s = rot[1];
          if (k < p && k != a && k != b) {
            const double gka = G[k][a], gkb = G[k][b];
            const double na = c * gka - s * gkb, nb = s * gka + c * gkb;
            G[k][a] = na;
            G[a][k] = na;
            G[k][b] = nb;
            G[b][k] = nb;
          }
          if (k < p) {
            const double vka = V[k][a], vkb = V[k][b];
            V[k][a] = c * vka - s * vkb;
            V[k][b] = s * vka + c * vkb;
          }
        }
        __syncthreads();
        if (k == 0 && gab != 0.0) {
          G[a][a] -= rot[2] * gab;
          G[b][b] += rot[2] * gab;
          G[a][b] = 0.0;
          G[b][a] = 0.0;
        }
        __syncthreads();
      }
  }
  __shared__ int top[2];
  if (k == 0) {
    int a1 = 0;
    for (int a = 1; a < p; ++a)
      if (G[a][a] > G[a1][a1]) a1 = a;
    int a2 = -1;
    for (int a = 0; a < p; ++a)
      if (a != a1 && (a2 < 0 || G[a][a] > G[a2][a2])) a2 = a;
    top[0] = a1;
    top[1] = a2;
    out[2 * p] = G[a1][a1];
    out[2 * p + 1] = a2 >= 0 ? G[a2][a2] : 0.0;
  }
  __syncthreads();
  if (k < p) {
    out[k] = V[k][top[0]];
    out[p + k] = top[1] >= 0 ? V[k][top[1]] : 0.0;
  }
}

// ------------------------------------------------------------- coordinates
__global__ void __launch_bounds__(256)
    project_kernel(const int32_t* __restrict__ dist, const int32_t* __restrict__ mind, int32_t n,
                   int32_t p, const double* __restrict__ colsum, double inv_m,
                   const double* __restrict__ eig, float2* __restrict__ X) {
  __shared__ Centring cen;
  __shared__ double w1[kMaxPivots], w2[kMaxPivots];
  load_centring(colsum, p, inv_m, cen);
  if (threadIdx.x < static_cast<unsigned>(p)) {
    const double mu1 = eig[2 * p], mu2 = eig[2 * p + 1];
    // an axis at or below 1e-6 mu1 (sigma <= 1e-3 sigma1) is rounding noise
    w1[threadIdx.x] = mu1 > 0.0 ? eig[threadIdx.x] / sqrt(sqrt(mu1)) : 0.0;
    w2[threadIdx.x] = mu2 > 0.0 && mu2 > 1e-6 * mu1 ? eig[p + threadIdx.x] / sqrt(sqrt(mu2)) : 0.0;
  }
  __syncthreads();
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += int64_t(gridDim.x) * blockDim.x) {
    if (mind[v] < 0) {
      X[v] = make_float2(0.f, 0.f);
      continue;
    }
    const double rmean = row_mean_sq(dist, n, p, v);
    double x = 0.0, y = 0.0;
    for (int j = 0; j < p; ++j) {
      const double d = dist[j * int64_t(n) + v];
      const double c = -0.5 * (d * d - cen.colmean[j] - rmean + cen.grand);
      x += c * w1[j];
      y += c * w2[j];
    }
    X[v] = make_float2(static_cast<float>(x), static_cast<float>(y));
  }
}

// sums[0] += sum d_ij |x_i - x_pj|, sums[1] += sum |x_i - x_pj|^2
__global__ void __launch_bounds__(256)
    scale_fit_kernel(const int32_t* __restrict__ dist, const int32_t* __restrict__ mind,
                     const float2* __restrict__ X, const int32_t* __restrict__ pivots, int32_t n,
                     int32_t p, double* sums) {
  __shared__ float2 xp[kMaxPivots];
  __shared__ double red[4];
  if (threadIdx.x < static_cast<unsigned>(p)) xp[threadIdx.x] = X[pivots[threadIdx.x]];
  __syncthreads();
  double num = 0.0, den = 0.0;
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += int64_t(gridDim.x) * blockDim.x) {
    if (mind[v] < 0) continue;
    const float2 xv = X[v];
    for (int j = 0; j < p; ++j) {
      const double dx = double(xv.x) - double(xp[j].x), dy = double(xv.y) - double(xp[j].y);
      const double q = dx * dx + dy * dy;
      num += double(dist[j * int64_t(n) + v]) * sqrt(q);
      den += q;
    }
  }
  num = block_reduce(num, SumF64{}, red);
  den = block_reduce(den, SumF64{}, red);
  if (threadIdx.x == 0) {
    atomicAdd(&sums[0], num);
    atomicAdd(&sums[1], den);
  }
}

// Component nodes: Y = s X (rounded once to FP32); *maxbits = bits of the
// largest |coordinate| (non-negative floats order like their bit patterns).
__global__ void __launch_bounds__(256)
    place_kernel(const int32_t* __restrict__ mind, const float2* __restrict__ X, int32_t n,
                 const double* __restrict__ sums, float2* __restrict__ Y, unsigned* maxbits) {
  __shared__ float red[4];
  const double s = sums[1] > 0.0 ? sums[0] / sums[1] : 1.0;
  float m = 0.f;
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += int64_t(gridDim.x) * blockDim.x) {
    if (mind[v] < 0) continue;
    const float2 x = X[v];
    const float2 y = make_float2(static_cast<float>(s * double(x.x)), static_cast<float>(s * double(x.y)));
    Y[v] = y;
    m = fmaxf(m, fmaxf(fabsf(y.x), fabsf(y.y)));
  }
  m = block_reduce(m, MaxF32{}, red);
  if (threadIdx.x == 0) atomicMax(maxbits, __float_as_uint(m));
}

// Nodes outside the component: the seeded uniform draws in [-R, R]^2.
__global__ void __launch_bounds__(256)
    place_rest_kernel(const int32_t* __restrict__ mind, int32_t n, uint64_t seed,
                      const unsigned* __restrict__ maxbits, float2* __restrict__ Y) {
  float R = __uint_as_float(*maxbits);
  if (!(R > 0.f)) R = 1.f;
  for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += int64_t(gridDim.x) * blockDim.x)
    if (mind[v] < 0) Y[v] = init_coords(v, seed, R);
}

// ---------------------------------------------------------------- host side
struct Scratch {
  std::vector<void*> ptrs;
  hipError_t err = hipSuccess;
  template <class T>
  T* get(size_t count) {
    void* p = nullptr;
    if (err == hipSuccess) err = hipMalloc(&p, std::max<size_t>(count * sizeof(T), 8));
    if (err != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

int grid_for(int64_t items) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(div_up(items, 256), 2048)));
}

}  // namespace

int pmds_positions(hipStream_t stream, const int64_t* d_row, const int32_t* d_col, int32_t n,
                   int32_t pivots, uint64_t seed, float2* d_Y, int32_t* d_pivots_out,
                   int32_t* d_dist_out, int32_t* pivots_used) {
  if (pivots_used) *pivots_used = 0;
  if (n <= 0) return LAYOUT_OK;
  const int32_t p = std::min(std::max(pivots, 1), kMaxPivots);
  Scratch w;
  int32_t* dist = d_dist_out ? d_dist_out : w.get<int32_t>(size_t(p) * size_t(n));
  int32_t* mind = w.get<int32_t>(n);
  int32_t* heavy = w.get<int32_t>(n);
  int32_t* piv = w.get<int32_t>(kMaxPivots);
  int32_t* flags = w.get<int32_t>(2);
  uint64_t* best = w.get<uint64_t>(1);
  uint64_t* comp = w.get<uint64_t>(1);
  double* colsum = w.get<double>(kMaxPivots);
  double* G = w.get<double>(size_t(kMaxPivots) * kMaxPivots);
  double* eig = w.get<double>(2 * kMaxPivots + 2);
  double* sums = w.get<double>(2);
  unsigned* maxbits = w.get<unsigned>(1);
  float2* X = w.get<float2>(n);
  if (w.err != hipSuccess) return hip_fail(w.err, "PMDS work buffers");

  const int grid = grid_for(n);
  hipError_t e = hipMemsetAsync(best, 0, sizeof(uint64_t), stream);
  if (e == hipSuccess) e = hipMemsetAsync(comp, 0, sizeof(uint64_t), stream);
  if (e == hipSuccess) e = hipMemsetAsync(colsum, 0, sizeof(double) * kMaxPivots, stream);
  if (e != hipSuccess) return hip_fail(e, "PMDS set-up");
  hipLaunchKernelGGL(degree_argmax_kernel, dim3(grid), dim3(256), 0, stream, d_row, n, best);

  int32_t p_eff = p;
  for (int32_t j = 0; j < p_eff; ++j) {
    int32_t* dj = dist + size_t(j) * size_t(n);
    hipLaunchKernelGGL(bfs_start_kernel, dim3(grid), dim3(256), 0, stream, dj, n, best, piv, j);
    for (int32_t level = 0;; ++level) {
      e = hipMemsetAsync(flags, 0, 2 * sizeof(int32_t), stream);
      if (e != hipSuccess) return hip_fail(e, "BFS flags");
      hipLaunchKernelGGL(bfs_level_kernel, dim3(grid), dim3(256), 0, stream, d_row, d_col, dj, n,
                         level, flags, heavy);
      hipLaunchKernelGGL(bfs_heavy_kernel, dim3(256), dim3(256), 0, stream, d_row, d_col, dj,
                         level, flags, heavy);
      int32_t found = 0;
      e = hipMemcpyAsync(&found, flags, sizeof(int32_t), hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      if (e != hipSuccess) return hip_fail(e, "BFS level");
      if (!found) break;
    }
    e = hipMemsetAsync(best, 0, sizeof(uint64_t), stream);
    if (e != hipSuccess) return hip_fail(e, "PMDS pivot key");
    hipLaunchKernelGGL(pivot_update_kernel, dim3(grid), dim3(256), 0, stream, dj, mind, n,
                       j == 0 ? 1 : 0, colsum + j, comp, best);
    if (j == 0) {
      uint64_t m = 0;
      e = hipMemcpyAsync(&m, comp, sizeof(uint64_t), hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      if (e != hipSuccess) return hip_fail(e, "PMDS component size");
      p_eff = static_cast<int32_t>(std::min<uint64_t>(uint64_t(p), m));
    }
  }
  uint64_t m = 0;
  e = hipMemcpyAsync(&m, comp, sizeof(uint64_t), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "PMDS component size");
  const double inv_m = 1.0 / static_cast<double>(m);

  e = hipMemsetAsync(G, 0, sizeof(double) * size_t(p_eff) * size_t(p_eff), stream);
  if (e == hipSuccess) e = hipMemsetAsync(sums, 0, 2 * sizeof(double), stream);
  if (e == hipSuccess) e = hipMemsetAsync(maxbits, 0, sizeof(unsigned), stream);
  if (e != hipSuccess) return hip_fail(e, "PMDS clear");
  hipLaunchKernelGGL(gram_kernel, dim3(std::min(grid, 1024)), dim3(256), 0, stream, dist, mind, n,
                     p_eff, colsum, inv_m, G);
  hipLaunchKernelGGL(eigen_kernel, dim3(1), dim3(64), 0, stream, G, p_eff, eig);
  hipLaunchKernelGGL(project_kernel, dim3(grid), dim3(256), 0, stream, dist, mind, n, p_eff,
                     colsum, inv_m, eig, X);
  hipLaunchKernelGGL(scale_fit_kernel, dim3(grid), dim3(256), 0, stream, dist, mind, X, piv, n,
                     p_eff, sums);
  hipLaunchKernelGGL(place_kernel, dim3(grid), dim3(256), 0, stream, mind, X, n, sums, d_Y,
                     maxbits);
  hipLaunchKernelGGL(place_rest_kernel, dim3(grid), dim3(256), 0, stream, mind, n, seed, maxbits,
                     d_Y);
  e = hipGetLastError();
  if (e == hipSuccess && d_pivots_out)
    e = hipMemcpyAsync(d_pivots_out, piv, sizeof(int32_t) * size_t(p_eff),
                       hipMemcpyDeviceToDevice, stream);
  // the scratch buffers are freed on return: finish their users first
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "PMDS");
  if (pivots_used) *pivots_used = p_eff;
  return LAYOUT_OK;
}

}  // namespace snap

// ------------------------------------------------------------------ C ABI
int layout_pmds(const int32_t* row_ptr, const int32_t* col_idx, int32_t n, int32_t pivots,
                uint64_t seed, int32_t inputs_on_device, float* Y_out, int32_t* pivots_out,
                int32_t* dist_out, int32_t* pivots_used) {
  using namespace snap;
  g_last_error.clear();
  if (n < 0) return fail(LAYOUT_E_INVALID_ARG, "n = %d", n);
  if (pivots < 0 || pivots > kMaxPivots)
    return fail(LAYOUT_E_INVALID_ARG, "pivots = %d (1..%d, 0 = %d)", pivots, kMaxPivots,
                kDefaultPivots);
  if (!Y_out) return fail(LAYOUT_E_INVALID_ARG, "Y_out is NULL");
  if (n > 0 && (!row_ptr || !col_idx)) return fail(LAYOUT_E_INVALID_ARG, "NULL graph arrays");
  if (pivots_used) *pivots_used = 0;
  if (n == 0) return LAYOUT_OK;
  const int32_t p = pivots ? pivots : kDefaultPivots;
  int64_t nnz = 0;
  if (inputs_on_device) {
    int32_t last = 0;
    hipError_t e = hipMemcpy(&last, row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading row_ptr[n]");
    nnz = last;
  } else {
    nnz = row_ptr[n];
  }
  if (nnz < 0) return fail(LAYOUT_E_BAD_GRAPH, "row_ptr[n] = %lld", (long long)nnz);

  hipStream_t stream = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  struct Owned {
    std::vector<void*> ptrs;
    hipStream_t s;
    ~Owned() {
      if (s) (void)hipStreamSynchronize(s);
      for (void* p : ptrs) (void)hipFree(p);
      if (s) (void)hipStreamDestroy(s);
    }
  } own{{}, stream};
  auto dev = [&](size_t bytes, void** p) {
    hipError_t r = hipMalloc(p, std::max<size_t>(bytes, 8));
    if (r == hipSuccess) own.ptrs.push_back(*p);
    return r;
  };
  int64_t* d_row = nullptr;
  int32_t *d_col = nullptr, *d_piv = nullptr, *d_dist = nullptr;
  float2* d_Y = nullptr;
  uint32_t* d_err = nullptr;
  e = dev(sizeof(int64_t) * (size_t(n) + 1), reinterpret_cast<void**>(&d_row));
  if (e == hipSuccess) e = dev(sizeof(int32_t) * size_t(nnz), reinterpret_cast<void**>(&d_col));
  if (e == hipSuccess) e = dev(sizeof(int32_t) * kMaxPivots, reinterpret_cast<void**>(&d_piv));
  if (e == hipSuccess && dist_out)
    e = dev(sizeof(int32_t) * size_t(p) * size_t(n), reinterpret_cast<void**>(&d_dist));
  if (e == hipSuccess) e = dev(sizeof(float2) * size_t(n), reinterpret_cast<void**>(&d_Y));
  if (e == hipSuccess) e = dev(sizeof(uint32_t), reinterpret_cast<void**>(&d_err));
  if (e != hipSuccess) return hip_fail(e, "PMDS buffers");
  const hipMemcpyKind kind = inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  int rc = upload_row_ptr(stream, row_ptr, n, inputs_on_device != 0, d_row);
  if (rc != LAYOUT_OK) return rc;
  if (nnz > 0)
    e = hipMemcpyAsync(d_col, col_idx, sizeof(int32_t) * size_t(nnz), kind, stream);
  if (e != hipSuccess) return hip_fail(e, "copying the graph");
  rc = validate_csr(stream, d_row, d_col, n, nnz, d_err);
  if (rc != LAYOUT_OK) return rc;
  int32_t used = 0;
  rc = pmds_positions(stream, d_row, d_col, n, p, seed, d_Y, d_piv, d_dist, &used);
  if (rc != LAYOUT_OK) return rc;
  e = hipMemcpyAsync(Y_out, d_Y, sizeof(float2) * size_t(n), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && pivots_out)
    e = hipMemcpyAsync(pivots_out, d_piv, sizeof(int32_t) * size_t(used), hipMemcpyDeviceToHost,
                       stream);
  if (e == hipSuccess && dist_out)
    e = hipMemcpyAsync(dist_out, d_dist, sizeof(int32_t) * size_t(used) * size_t(n),
                       hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "reading PMDS results");
  if (pivots_used) *pivots_used = used;
  return LAYOUT_OK;
}
