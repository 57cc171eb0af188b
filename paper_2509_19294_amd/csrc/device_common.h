// Device helpers shared by the pair kernels (csrc/kernels*.hip).
#pragma once

#include "nbody_internal.h"

namespace nb {

// Hardware reciprocal square root (v_rsq_f32, about 1 ulp).
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Knuth's TwoSum: s + e == a + b exactly (round-to-nearest, no overflow).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Streaming store of a partial sum that only a later kernel reads: marked
// non-temporal, so it does not push reusable data out of the L2.
__device__ __forceinline__ void store_stream(float4 *p, float4 v) {
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  const f32x4 w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, reinterpret_cast<f32x4 *>(p));
}

// Double-single split of an FP64 offset: hi = fp32(d), lo = fp32(d - hi).
__device__ __forceinline__ void ds_split(double d, float &hi, float &lo) {
  hi = static_cast<float>(d);
  lo = static_cast<float>(d - static_cast<double>(hi));
}

// Destination of a block's results.
struct OutArgs {
  double *acc;       // [n][3] or nullptr when writing partials
  double *pot;       // [n] or nullptr
  float4 *part;      // grid j-split partials, nullptr when writing acc/pot
  int64_t n;         // stride of one split in `part`
  int split_index;
  double G;
};

// Self-pair term the kernel adds to the potential sum when eps > 0 (the pair
// j == i contributes m_i * rsq(eps^2) and nothing to the acceleration); it is
// removed again in FP64. The expression matches the in-loop one bit for bit.
__device__ __forceinline__ float self_term(float m, float eps2f) { return m * rsq(eps2f); }

// Target block and grid split of a block launched on a one-dimensional grid
// of nblk x split blocks. Blocks go to the 8 XCDs in turn (block L to XCD
// L % 8), each XCD with its own L2. order 0 takes the splits one after
// another (block L = split * nblk + target block); order 1 (split a multiple
// of 8) gives XCD x the splits x, x + 8, ...; order 2 (8 a multiple of split,
// nblk * split a multiple of 8) gives XCD x split x % split only. With 1 and
// 2 the blocks an XCD runs at a time stage the same split's sources, which
// then stay in that XCD's L2 instead of every XCD streaming every split.
__device__ __forceinline__ void xcd_block(uint32_t L, uint32_t nblk, uint32_t split, int order,
                                          uint32_t &bx, uint32_t &by) {
  if (order == 1) {
    const uint32_t x = L & 7u, r = L >> 3;
    by = x + 8u * (r / nblk);
    bx = r % nblk;
  } else if (order == 2) {
    const uint32_t x = L & 7u, r = L >> 3;
    by = x % split;
    bx = r * (8u / split) + x / split;
  } else {
    by = L / nblk;
    bx = L % nblk;
  }
}

// Four consecutive float4 words, 64-byte aligned: one scalar load.
struct alignas(64) Quad {
  float4 v[4];
};

}  // namespace nb
