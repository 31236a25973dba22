// Counter-based random numbers for the layout kernels (device side).
//
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each with two
// 64x64->128-bit products, the key advanced by two Weyl constants between
// rounds.  Every draw is a pure function of (seed, purpose, indices), so any
// thread may draw the samples of any edge in any order, and the same samples
// come out on every run and on the host reference.
//
// Layout of the counters and words:
//   key     = (seed, kKeyDomain)
//   counter = (a, b, block, tag); tag 1 = initial positions, 2 = negatives
//   a block gives u64 x0..x3, read as eight u32 words: lo(x0), hi(x0), lo(x1) ...
//   negatives of directed edge e in epoch t read the word stream of
//   counters (e, t, 0, 2), (e, t, 1, 2), ...
//
// Negative sampling (Algorithm 1: a node drawn uniformly from V \ {i}):
//   uniform: one word u per attempt, p = u * (n-1) as a 64-bit product;
//            the attempt is rejected when lo32(p) < 2^32 mod (n-1) (Lemire's
//            unbiased multiply-shift reduction, ACM TOMACS 2019); otherwise
//            s' = hi32(p) and s = s' + (s' >= i), which skips the source.
//   degree:  two words (u1, u2) per attempt, a bin c = hi32(u1 * n) (same
//            rejection rule with n), then s = u2 < thr[c] ? c : alias[c];
//            the attempt is rejected when s == i.
//   After 64 rejected attempts the draw falls back to (i + 1) mod n; the
//   probability of reaching it is below 2^-64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snap {

constexpr uint64_t kKeyDomain = 0x534E41502D744644ull;  // "SNAP-tFD"
constexpr uint64_t kTagInit = 1;
constexpr uint64_t kTagNeg = 2;
constexpr int kMaxAttempts = 64;

struct U64x4 {
  uint64_t x0, x1, x2, x3;
};

// The 128-bit product m * x as (hi, lo), from four 32 x 32 + 64 -> 64-bit
// multiply-adds (v_mad_u64_u32 on gfx950): with m = mh 2^32 + ml and
// x = xh 2^32 + xl, t = ml xh + (ml xl >> 32) and u = mh xl + lo32(t) cannot
// overflow 64 bits, hi = mh xh + (t >> 32) + (u >> 32), lo = (u << 32) |
// lo32(ml xl).  Exact; a third fewer ALU instructions than the generic
// 64-bit high multiply.
__device__ __forceinline__ void mulhilo64(uint64_t m, uint64_t x, uint64_t& hi, uint64_t& lo) {
  const uint32_t ml = static_cast<uint32_t>(m), mh = static_cast<uint32_t>(m >> 32);
  const uint32_t xl = static_cast<uint32_t>(x), xh = static_cast<uint32_t>(x >> 32);
  const uint64_t p0 = static_cast<uint64_t>(ml) * xl;
  const uint64_t t = static_cast<uint64_t>(ml) * xh + (p0 >> 32);
  const uint64_t u = static_cast<uint64_t>(mh) * xl + static_cast<uint32_t>(t);
  hi = static_cast<uint64_t>(mh) * xh + (t >> 32) + (u >> 32);
  lo = (u << 32) | static_cast<uint32_t>(p0);
}

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                               uint64_t c3, uint64_t k0, uint64_t k1) {
  constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t kMul1 = 0xCA5A826395121157ull;
  constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t p0_hi, p0_lo, p1_hi, p1_lo;
    mulhilo64(kMul0, c0, p0_hi, p0_lo);
    mulhilo64(kMul1, c2, p1_hi, p1_lo);
    const uint64_t n0 = p1_hi ^ c1 ^ k0;
    const uint64_t n2 = p0_hi ^ c3 ^ k1;
    c0 = n0;
    c1 = p1_lo;
    c2 = n2;
    c3 = p0_lo;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  return U64x4{c0, c1, c2, c3};
}

// Sequential u32 words of one counter family (a, b, *, tag): block 0 gives
// words lo(x0), hi(x0), lo(x1), ..., hi(x3), then block 1, and so on.  The
// unread words of the current block sit in a register queue that shifts down
// by one per word, so every register index is a compile-time constant (a
// data-dependent word index would make the compiler keep the block in an
// indexed scratch array).
struct WordStream {
  uint64_t seed, a, b, tag;
  uint64_t block;
  int avail;  // unread words of the current block, 0..8
  uint32_t w0, w1, w2, w3, w4, w5, w6, w7;

  __device__ __forceinline__ void fill() {
    const U64x4 x = philox4x64_10(a, b, block, tag, seed, kKeyDomain);
    w0 = static_cast<uint32_t>(x.x0);
    w1 = static_cast<uint32_t>(x.x0 >> 32);
    w2 = static_cast<uint32_t>(x.x1);
    w3 = static_cast<uint32_t>(x.x1 >> 32);
    w4 = static_cast<uint32_t>(x.x2);
    w5 = static_cast<uint32_t>(x.x2 >> 32);
    w6 = static_cast<uint32_t>(x.x3);
    w7 = static_cast<uint32_t>(x.x3 >> 32);
    avail = 8;
  }

  __device__ __forceinline__ void open(uint64_t seed_, uint64_t a_, uint64_t b_, uint64_t tag_) {
    seed = seed_;
    a = a_;
    b = b_;
    tag = tag_;
    block = 0;
    fill();
  }

  __device__ __forceinline__ uint32_t next() {
    if (avail == 0) {
      ++block;
      fill();
    }
    const uint32_t r = w0;
    w0 = w1;
    w1 = w2;
    w2 = w3;
    w3 = w4;
    w4 = w5;
    w5 = w6;
    w6 = w7;
    --avail;
    return r;
  }
};

// Per-graph constants of the samplers, precomputed on the host.
struct SamplerConsts {
  uint32_t n;             // nodes
  uint32_t range;         // n - 1
  uint32_t reject_range;  // 2^32 mod (n - 1)   (0 when n < 2)
  uint32_t reject_n;      // 2^32 mod n
};

__device__ __forceinline__ uint32_t draw_uniform(WordStream& ws, const SamplerConsts& sc,
                                                 uint32_t i) {
  for (int attempt = 0; attempt < kMaxAttempts; ++attempt) {
    const uint32_t u = ws.next();
    const uint64_t p = static_cast<uint64_t>(u) * sc.range;
    if (static_cast<uint32_t>(p) < sc.reject_range) continue;
    const uint32_t s = static_cast<uint32_t>(p >> 32);
    return s + (s >= i ? 1u : 0u);
  }
  return (i + 1u) % sc.n;
}

__device__ __forceinline__ uint32_t draw_alias(WordStream& ws, const SamplerConsts& sc,
                                               uint32_t i, const uint32_t* __restrict__ thr,
                                               const uint32_t* __restrict__ alias) {
  for (int attempt = 0; attempt < kMaxAttempts; ++attempt) {
    const uint32_t u1 = ws.next();
    const uint32_t u2 = ws.next();
    const uint64_t p = static_cast<uint64_t>(u1) * sc.n;
    if (static_cast<uint32_t>(p) < sc.reject_n) continue;
    const uint32_t c = static_cast<uint32_t>(p >> 32);
    const uint32_t s = u2 < thr[c] ? c : alias[c];
    if (s == i) continue;
    return s;
  }
  return (i + 1u) % sc.n;
}

}  // namespace snap
