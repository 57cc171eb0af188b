// HIP kernels for gfx950 (MI355X): softened all-pairs gravity, FP64
// kick-drift-kick leapfrog and FP64 diagnostics.
//
// Pair sum: the force equation of Section 3 (sum over j != i of
// G m_j (r_j - r_i) / r_ij^3 per unit target mass) with Plummer softening,
// plus the potential. The pair arithmetic is FP32 on the vector ALUs, one
// hardware reciprocal square root per pair; there is no dense contraction, so
// no matrix cores. Layout of the work:
//   * a block covers an i-block; each thread holds K i-particles in VGPRs;
//   * j-particles are streamed through LDS in tiles (double buffered: the
//     global loads of tile t+1 are in flight while tile t is consumed, one
//     barrier per tile); a wave reads a j-entry as an LDS broadcast;
//   * LS lanes may share one i (each takes every LS-th j of a tile) and SW
//     waves may share one i-group (each takes its own slice of a tile); the
//     partial sums are then combined by lane shuffles and through LDS, in a
//     fixed order, so results are bitwise reproducible;
//   * sums are two-level: a plain FP32 partial per tile, merged into the
//     running sum once per tile (plain form) or by TwoSum into a (hi, lo)
//     pair (compensated form).
// The compensated form stages j-particles from the FP64 inputs as
// double-single coordinates relative to an FP64 frame (the first i of the
// block): hi = fp32(x - c), lo = fp32((x - c) - hi); a separation is
// (hi_j - hi_i) + (lo_j - lo_i).
#include "device_common.h"

namespace nb {





template <bool COMP>
struct StageRegs;
template <>
struct StageRegs<false> {
  float4 v;
};
template <>
struct StageRegs<true> {
  double x, y, z, m;
};

template <bool COMP>
__device__ __forceinline__ void stage_load(StageRegs<COMP> &r, const double *__restrict__ pos,
                                           const double *__restrict__ mass,
                                           const float4 *__restrict__ packed, int64_t j, bool valid,
                                           double cx, double cy, double cz) {
  if constexpr (COMP) {
    if (valid) {
      r.x = pos[3 * j];
      r.y = pos[3 * j + 1];
      r.z = pos[3 * j + 2];
      r.m = mass[j];
    } else {
      r.x = cx;
      r.y = cy;
      r.z = cz;
      r.m = 0.0;
    }
  } else {
    r.v = valid ? packed[j] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}


template <bool COMP>
__device__ __forceinline__ void stage_store(float4 *dst, const StageRegs<COMP> &r, double cx,
                                            double cy, double cz) {
  if constexpr (COMP) {
    float hx, hy, hz, lx, ly, lz;
    ds_split(r.x - cx, hx, lx);
    ds_split(r.y - cy, hy, ly);
    ds_split(r.z - cz, hz, lz);
    dst[0] = make_float4(hx, hy, hz, static_cast<float>(r.m));
    dst[1] = make_float4(lx, ly, lz, 0.f);
  } else {
    dst[0] = r.v;
  }
}

// One block computes the i-particles [i0, i1) against the j-particles
// [j0, j1). `lds` holds 2 * TILE * (COMP ? 2 : 1) float4.
template <int BLOCK, int K, int LS, int SW, int TILE, bool COMP, bool EPS0>
__device__ __forceinline__ void pair_block(const double *__restrict__ pos,
                                           const double *__restrict__ mass,
                                           const float4 *__restrict__ packed, int64_t i0,
                                           int64_t i1, int64_t j0, int64_t j1, float eps2f,
                                           float4 *lds, const OutArgs &o) {
  constexpr int NW = BLOCK / 64;
  constexpr int NG = NW / SW;       // i-groups per block
  constexpr int IPW = 64 / LS;      // i's per wave for one k
  constexpr int Q = SW * LS;        // j sub-streams per i
  constexpr int JPT = TILE / Q;     // j's per thread per tile
  constexpr int JW = COMP ? 2 : 1;  // float4 words per staged j
  constexpr int SPT = TILE / BLOCK; // j's each thread stages per tile
  static_assert(BLOCK % 64 == 0 && NW % SW == 0 && 64 % LS == 0, "bad block shape");
  static_assert(TILE % BLOCK == 0 && TILE % Q == 0, "bad tile");
  static_assert((SW - 1) * NG * IPW * K * 4 * JW <= 2 * TILE * JW * 4, "combine does not fit in LDS");

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wj = wave % SW, wg = wave / SW;
  const int lj = lane % LS, li = lane / LS;
  const int q = wj * LS + lj;

  double cx = 0.0, cy = 0.0, cz = 0.0;
  if constexpr (COMP) {
    cx = pos[3 * i0];
    cy = pos[3 * i0 + 1];
    cz = pos[3 * i0 + 2];
  }

  float xh[K], yh[K], zh[K], xl[K], yl[K], zl[K], mi[K];
  int64_t iidx[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t i = i0 + static_cast<int64_t>(k) * (NG * IPW) + wg * IPW + li;
    iidx[k] = i;
    const int64_t ic = i < i1 ? i : i1 - 1;
    if constexpr (COMP) {
      ds_split(pos[3 * ic] - cx, xh[k], xl[k]);
      ds_split(pos[3 * ic + 1] - cy, yh[k], yl[k]);
      ds_split(pos[3 * ic + 2] - cz, zh[k], zl[k]);
    } else {
      xh[k] = static_cast<float>(pos[3 * ic]);
      yh[k] = static_cast<float>(pos[3 * ic + 1]);
      zh[k] = static_cast<float>(pos[3 * ic + 2]);
      xl[k] = yl[k] = zl[k] = 0.f;
    }
    mi[k] = static_cast<float>(mass[ic]);
  }

  float ah[K][4], al[K][4];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) ah[k][c] = al[k][c] = 0.f;

  const int64_t ntiles = j1 > j0 ? (j1 - j0 + TILE - 1) / TILE : 0;
  StageRegs<COMP> sr[SPT];

  if (ntiles > 0) {
#pragma unroll
    for (int r = 0; r < SPT; ++r) {
      const int64_t j = j0 + r * BLOCK + tid;
      stage_load<COMP>(sr[r], pos, mass, packed, j, j < j1, cx, cy, cz);
    }
#pragma unroll
    for (int r = 0; r < SPT; ++r) stage_store<COMP>(lds + (r * BLOCK + tid) * JW, sr[r], cx, cy, cz);
  }
  __syncthreads();

  for (int64_t t = 0; t < ntiles; ++t) {
    const int buf = static_cast<int>(t & 1);
    const bool more = t + 1 < ntiles;
    if (more) {
#pragma unroll
      for (int r = 0; r < SPT; ++r) {
        const int64_t j = j0 + (t + 1) * TILE + r * BLOCK + tid;
        stage_load<COMP>(sr[r], pos, mass, packed, j, j < j1, cx, cy, cz);
      }
    }

    const float4 *T = lds + buf * (TILE * JW);
    float p[K][4];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) p[k][c] = 0.f;

#pragma unroll 8
    for (int jj = 0; jj < JPT; ++jj) {
      const int jl = jj * Q + q;
      const float4 H = T[jl * JW];
      float4 L = make_float4(0.f, 0.f, 0.f, 0.f);
      if constexpr (COMP) L = T[jl * JW + 1];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        float dx, dy, dz;
        if constexpr (COMP) {
          dx = (H.x - xh[k]) + (L.x - xl[k]);
          dy = (H.y - yh[k]) + (L.y - yl[k]);
          dz = (H.z - zh[k]) + (L.z - zl[k]);
        } else {
          dx = H.x - xh[k];
          dy = H.y - yh[k];
          dz = H.z - zh[k];
        }
        float r2 = fmaf(dx, dx, eps2f);
        r2 = fmaf(dy, dy, r2);
        r2 = fmaf(dz, dz, r2);
        float rho = rsq(r2);
        if constexpr (EPS0) rho = r2 > 0.f ? rho : 0.f;
        const float mr = H.w * rho;
        const float s = mr * (rho * rho);
        p[k][0] = fmaf(s, dx, p[k][0]);
        p[k][1] = fmaf(s, dy, p[k][1]);
        p[k][2] = fmaf(s, dz, p[k][2]);
        p[k][3] += mr;
      }
    }

#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if constexpr (COMP) {
          float s, e;
          two_sum(ah[k][c], p[k][c], s, e);
          ah[k][c] = s;
          al[k][c] += e;
        } else {
          ah[k][c] += p[k][c];
        }
      }

    if (more) {
      float4 *D = lds + (buf ^ 1) * (TILE * JW);
#pragma unroll
      for (int r = 0; r < SPT; ++r) stage_store<COMP>(D + (r * BLOCK + tid) * JW, sr[r], cx, cy, cz);
    }
    __syncthreads();
  }

  // Lanes sharing an i: butterfly over the low lane bits (fixed order).
#pragma unroll
  for (int off = 1; off < LS; off <<= 1) {
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float oh = __shfl_xor(ah[k][c], off, 64);
        if constexpr (COMP) {
          const float ol = __shfl_xor(al[k][c], off, 64);
          float s, e;
          two_sum(ah[k][c], oh, s, e);
          ah[k][c] = s;
          al[k][c] = (al[k][c] + ol) + e;
        } else {
          ah[k][c] += oh;
        }
      }
  }

  // Waves sharing an i-group: waves 1..SW-1 park their sums in LDS, wave 0
  // adds them in wave order. The tile buffers are free (last barrier above).
  if constexpr (SW > 1) {
    float *X = reinterpret_cast<float *>(lds);
    constexpr int SLOT = NG * IPW * K * 4 * JW;  // floats per parked wave
    const int base = (wg * IPW + li) * K * 4 * JW;
    if (wj > 0 && lj == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          X[(wj - 1) * SLOT + base + (k * 4 + c) * JW] = ah[k][c];
          if constexpr (COMP) X[(wj - 1) * SLOT + base + (k * 4 + c) * JW + 1] = al[k][c];
        }
    }
    __syncthreads();
    if (wj == 0 && lj == 0) {
      for (int w = 1; w < SW; ++w) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const float oh = X[(w - 1) * SLOT + base + (k * 4 + c) * JW];
            if constexpr (COMP) {
              const float ol = X[(w - 1) * SLOT + base + (k * 4 + c) * JW + 1];
              float s, e;
              two_sum(ah[k][c], oh, s, e);
              ah[k][c] = s;
              al[k][c] = (al[k][c] + ol) + e;
            } else {
              ah[k][c] += oh;
            }
          }
      }
    }
    __syncthreads();
  }

  if (wj != 0 || lj != 0) return;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t i = iidx[k];
    if (i >= i1) continue;
    if (o.part) {
      float4 *P = o.part + (static_cast<int64_t>(o.split_index) * o.n + i) * JW;
      P[0] = make_float4(ah[k][0], ah[k][1], ah[k][2], ah[k][3]);
      if constexpr (COMP) P[1] = make_float4(al[k][0], al[k][1], al[k][2], al[k][3]);
    } else {
      double s[4];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        s[c] = COMP ? static_cast<double>(ah[k][c]) + static_cast<double>(al[k][c])
                    : static_cast<double>(ah[k][c]);
      o.acc[3 * i] = o.G * s[0];
      o.acc[3 * i + 1] = o.G * s[1];
      o.acc[3 * i + 2] = o.G * s[2];
      if (o.pot) {
        const double self = EPS0 ? 0.0 : static_cast<double>(self_term(mi[k], eps2f));
        o.pot[i] = -o.G * (s[3] - self);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Single system.

template <int BLOCK, int K, int LS, int SW, int TILE, bool COMP, bool EPS0>
__global__ __launch_bounds__(BLOCK) void pair_single_kernel(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const float4 *__restrict__ packed, int64_t n, float eps2f, int split, int64_t split_len,
    OutArgs o) {
  constexpr int JW = COMP ? 2 : 1;
  __shared__ float4 lds[2 * TILE * JW];
  constexpr int IB = (BLOCK / 64 / SW) * (64 / LS) * K;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * IB;
  const int64_t i1 = i0 + IB < n ? i0 + IB : n;
  const int s = blockIdx.y;
  const int64_t j0 = static_cast<int64_t>(s) * split_len;
  const int64_t j1 = j0 + split_len < n ? j0 + split_len : n;
  OutArgs oo = o;
  oo.split_index = s;
  pair_block<BLOCK, K, LS, SW, TILE, COMP, EPS0>(pos, mass, packed, i0, i1, j0, j1, eps2f, lds,
                                                  oo);
}

// Sums the grid j-split partials in split order (FP64) and applies G and the
// self-term correction.
template <bool COMP>
__global__ __launch_bounds__(256) void combine_kernel(const float4 *__restrict__ part, int split,
                                                      int64_t n, const double *__restrict__ mass,
                                                      float eps2f, int eps0, double G,
                                                      double *__restrict__ acc,
                                                      double *__restrict__ pot) {
  constexpr int JW = COMP ? 2 : 1;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int s = 0; s < split; ++s) {
    const float4 *P = part + (static_cast<int64_t>(s) * n + i) * JW;
    const float4 h = P[0];
    s0 += h.x;
    s1 += h.y;
    s2 += h.z;
    s3 += h.w;
    if constexpr (COMP) {
      const float4 l = P[1];
      s0 += l.x;
      s1 += l.y;
      s2 += l.z;
      s3 += l.w;
    }
  }
  acc[3 * i] = G * s0;
  acc[3 * i + 1] = G * s1;
  acc[3 * i + 2] = G * s2;
  if (pot) {
    const double self = eps0 ? 0.0 : static_cast<double>(self_term(static_cast<float>(mass[i]), eps2f));
    pot[i] = -G * (s3 - self);
  }
}

__global__ __launch_bounds__(256) void pack_kernel(const double *__restrict__ pos,
                                                   const double *__restrict__ mass, int64_t n,
                                                   int64_t npad, float4 *__restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= npad) return;
  if (i >= n) {
    out[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  out[i] = make_float4(static_cast<float>(pos[3 * i]), static_cast<float>(pos[3 * i + 1]),
                       static_cast<float>(pos[3 * i + 2]), static_cast<float>(mass[i]));
}

// Double-single pack relative to the frame c = pos[0].
__global__ __launch_bounds__(256) void pack_ds_kernel(const double *__restrict__ pos,
                                                      const double *__restrict__ mass, int64_t n,
                                                      int64_t npad, float4 *__restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= npad) return;
  if (i >= n) {
    out[2 * i] = make_float4(0.f, 0.f, 0.f, 0.f);
    out[2 * i + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  float hx, hy, hz, lx, ly, lz;
  ds_split(pos[3 * i] - pos[0], hx, lx);
  ds_split(pos[3 * i + 1] - pos[1], hy, ly);
  ds_split(pos[3 * i + 2] - pos[2], hz, lz);
  out[2 * i] = make_float4(hx, hy, hz, static_cast<float>(mass[i]));
  out[2 * i + 1] = make_float4(lx, ly, lz, 0.f);
}


// Scalar-stream form of the pair kernel. The source index is the same for
// every lane of a wave, so each wave streams its sources straight from the
// packed array with scalar loads (four float4 words per load); coordinates
// and masses arrive in SGPRs and enter the VALU as scalar operands. There is
// no LDS staging and no barrier in the loop, and source operands cost no VGPR
// reads. The packed array is padded with zero-mass entries to a multiple of
// 64, and every split boundary is a multiple of 64, so the loop needs no
// bounds checks. SW waves of a block share an i-group and take interleaved
// groups of sources; their sums are combined through LDS in wave order.
// One block (4 waves) computes targets [i0, i1) (packed index of i0 is ip0)
// against packed sources [J0, J1); J1 - J0 must be a multiple of GS, the
// number of sources a wave loads per group (4 or 8: one or two 64-byte
// scalar loads in the plain form, two or four in the compensated form).
// `X` is LDS scratch of smem_lds_floats<K, SW, COMP>() floats.
template <int K, int SW, bool COMP>
constexpr int smem_lds_floats() {
  return (SW > 1) ? (SW - 1) * (4 / SW) * 64 * K * 4 * (COMP ? 2 : 1) : 1;
}

template <int K, int SW, int TJ, bool COMP, bool EPS0, int GS = 4>
__device__ __forceinline__ void smem_block(const float4 *__restrict__ packed, int64_t i0,
                                           int64_t i1, int64_t ip0, int64_t J0, int64_t J1,
                                           float eps2f, float *X, const OutArgs &o) {
  constexpr int NW = 4;
  constexpr int NG = NW / SW;
  constexpr int JW = COMP ? 2 : 1;
  constexpr int G = GS;                 // sources per group
  constexpr int STEP = SW * G;          // stride between a wave's groups
  static_assert(NW % SW == 0 && TJ % G == 0 && (G == 4 || G == 8), "bad shape");

  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const int wj = wave % SW, wg = wave / SW;

  float xh[K], yh[K], zh[K], xl[K], yl[K], zl[K], mi[K];
  int64_t iidx[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t i = i0 + static_cast<int64_t>(k) * (NG * 64) + wg * 64 + lane;
    iidx[k] = i;
    const int64_t ic = (i < i1 ? i : i1 - 1) - i0 + ip0;
    const float4 P = packed[ic * JW];
    xh[k] = P.x;
    yh[k] = P.y;
    zh[k] = P.z;
    mi[k] = P.w;
    if constexpr (COMP) {
      const float4 L = packed[ic * JW + 1];
      xl[k] = L.x;
      yl[k] = L.y;
      zl[k] = L.z;
    } else {
      xl[k] = yl[k] = zl[k] = 0.f;
    }
  }

  float ah[K][4], al[K][4];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) ah[k][c] = al[k][c] = 0.f;

  const Quad *Qp = reinterpret_cast<const Quad *>(packed);
  for (int64_t t = J0 + wj * G; t < J1; t += static_cast<int64_t>(TJ) * SW) {
    const int64_t tend = t + static_cast<int64_t>(TJ) * SW < J1 ? t + static_cast<int64_t>(TJ) * SW : J1;
    float p[K][4];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) p[k][c] = 0.f;
    // Waves on a SIMD hide each other's scalar-load latency (the loop keeps
    // 8 waves per SIMD resident); group counters are 32-bit so the loop
    // control stays on the scalar unit.
    const uint32_t ngroups = static_cast<uint32_t>((tend - t + STEP - 1) / STEP);
    const Quad *Qt = Qp + ((static_cast<uint64_t>(t) * JW) >> 2);
    // PF: the next group's scalar loads are issued before this group's pairs
    // (one target per lane, and a group of at most 32 scalar registers, so
    // that two of them fit)
    constexpr int NQD = G * JW / 4;
    constexpr bool PF = K == 1 && NQD <= 2;
    Quad cur[NQD];
    if constexpr (PF) {
      if (ngroups > 0) {
#pragma unroll
        for (int q = 0; q < NQD; ++q) cur[q] = Qt[q];
      }
    }
    for (uint32_t gi = 0; gi < ngroups; ++gi) {
      Quad nxt[NQD];
      if constexpr (PF) {
        const uint32_t gn = gi + 1 < ngroups ? gi + 1 : gi;
        const Quad *Qn = Qt + gn * (STEP * JW / 4);
#pragma unroll
        for (int q = 0; q < NQD; ++q) nxt[q] = Qn[q];
      }
      const Quad *Qg = PF ? cur : Qt + gi * (STEP * JW / 4);
      float4 H[G], L[G];
      if constexpr (COMP) {
#pragma unroll
        for (int q = 0; q < G / 2; ++q) {
          const Quad c = Qg[q];
          H[2 * q] = c.v[0];
          L[2 * q] = c.v[1];
          H[2 * q + 1] = c.v[2];
          L[2 * q + 1] = c.v[3];
        }
      } else {
#pragma unroll
        for (int q = 0; q < G / 4; ++q) {
          const Quad c = Qg[q];
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            H[4 * q + g] = c.v[g];
            L[4 * q + g] = make_float4(0.f, 0.f, 0.f, 0.f);
          }
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          float dx, dy, dz;
          if constexpr (COMP) {
            dx = (H[g].x - xh[k]) + (L[g].x - xl[k]);
            dy = (H[g].y - yh[k]) + (L[g].y - yl[k]);
            dz = (H[g].z - zh[k]) + (L[g].z - zl[k]);
          } else {
            dx = H[g].x - xh[k];
            dy = H[g].y - yh[k];
            dz = H[g].z - zh[k];
          }
          float r2 = fmaf(dx, dx, eps2f);
          r2 = fmaf(dy, dy, r2);
          r2 = fmaf(dz, dz, r2);
          float rho = rsq(r2);
          if constexpr (EPS0) rho = r2 > 0.f ? rho : 0.f;
          const float mr = H[g].w * rho;
          const float s = mr * (rho * rho);
          p[k][0] = fmaf(s, dx, p[k][0]);
          p[k][1] = fmaf(s, dy, p[k][1]);
          p[k][2] = fmaf(s, dz, p[k][2]);
          p[k][3] += mr;
        }
      }
      if constexpr (PF) {
#pragma unroll
        for (int q = 0; q < NQD; ++q) cur[q] = nxt[q];
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if constexpr (COMP) {
          float s, e;
          two_sum(ah[k][c], p[k][c], s, e);
          ah[k][c] = s;
          al[k][c] += e;
        } else {
          ah[k][c] += p[k][c];
        }
      }
  }

  if constexpr (SW > 1) {
    constexpr int SLOT = NG * 64 * K * 4 * JW;
    const int base = (wg * 64 + lane) * K * 4 * JW;
    if (wj > 0) {
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          X[(wj - 1) * SLOT + base + (k * 4 + c) * JW] = ah[k][c];
          if constexpr (COMP) X[(wj - 1) * SLOT + base + (k * 4 + c) * JW + 1] = al[k][c];
        }
    }
    __syncthreads();
    if (wj == 0) {
      for (int w = 1; w < SW; ++w) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const float oh = X[(w - 1) * SLOT + base + (k * 4 + c) * JW];
            if constexpr (COMP) {
              const float ol = X[(w - 1) * SLOT + base + (k * 4 + c) * JW + 1];
              float s, e;
              two_sum(ah[k][c], oh, s, e);
              ah[k][c] = s;
              al[k][c] = (al[k][c] + ol) + e;
            } else {
              ah[k][c] += oh;
            }
          }
      }
    }
  }
  if (wj != 0) return;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t i = iidx[k];
    if (i >= i1) continue;
    if (o.part) {
      float4 *P = o.part + (static_cast<int64_t>(o.split_index) * o.n + i) * JW;
      P[0] = make_float4(ah[k][0], ah[k][1], ah[k][2], ah[k][3]);
      if constexpr (COMP) P[1] = make_float4(al[k][0], al[k][1], al[k][2], al[k][3]);
    } else {
      double sum[4];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        sum[c] = COMP ? static_cast<double>(ah[k][c]) + static_cast<double>(al[k][c])
                      : static_cast<double>(ah[k][c]);
      o.acc[3 * i] = o.G * sum[0];
      o.acc[3 * i + 1] = o.G * sum[1];
      o.acc[3 * i + 2] = o.G * sum[2];
      if (o.pot) {
        const double self = EPS0 ? 0.0 : static_cast<double>(self_term(mi[k], eps2f));
        o.pot[i] = -o.G * (sum[3] - self);
      }
    }
  }
}

template <int K, int SW, int TJ, bool COMP, bool EPS0, int GS>
__global__ __launch_bounds__(256) void pair_smem_kernel(const float4 *__restrict__ packed,
                                                        const double *__restrict__ mass,
                                                        int64_t n, float eps2f, int64_t split_len,
                                                        OutArgs o) {
  (void)mass;
  constexpr int IB = (4 / SW) * 64 * K;
  __shared__ float X[smem_lds_floats<K, SW, COMP>()];
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * IB;
  const int64_t i1 = i0 + IB < n ? i0 + IB : n;
  const int64_t np = padded(n);
  const int64_t J0 = static_cast<int64_t>(blockIdx.y) * split_len;
  const int64_t J1 = J0 + split_len < np ? J0 + split_len : np;
  OutArgs oo = o;
  oo.split_index = blockIdx.y;
  smem_block<K, SW, TJ, COMP, EPS0, GS>(packed, i0, i1, i0, J0, J1, eps2f, X, oo);
}

// Compiled single-system configurations: {block, k, ls, sw, tile, smem}
// (smem: 0 = LDS tiles, 1 = scalar stream with 4-source groups, 2 = with
// 8-source groups, 3 = near/far on the spatial order, 4 = near/far with the
// frame stored by the ordering pass, 5 = near/far on half box groups).
static const PairCfg kSingle[] = {
    {256, 1, 1, 1, 256, 0},   // 0
    {256, 2, 1, 1, 256, 0},   // 1
    {256, 4, 1, 1, 256, 0},   // 2
    {256, 2, 1, 2, 512, 0},   // 3
    {256, 1, 1, 4, 1024, 0},  // 4
    {256, 1, 4, 1, 256, 0},   // 5
    {256, 4, 1, 2, 512, 0},   // 6
    {256, 2, 1, 4, 1024, 0},  // 7
    {256, 8, 1, 1, 256, 0},   // 8
    {256, 2, 2, 1, 512, 0},   // 9
    {256, 1, 1, 1, 256, 1},   // 10
    {256, 2, 1, 1, 256, 1},   // 11
    {256, 4, 1, 1, 256, 1},   // 12
    {256, 1, 1, 2, 256, 1},   // 13
    {256, 2, 1, 2, 256, 1},   // 14
    {256, 1, 1, 4, 256, 1},   // 15
    {256, 1, 1, 1, 256, 2},   // 16
    {256, 1, 1, 2, 256, 2},   // 17
    {256, 1, 1, 4, 256, 2},   // 18
    {256, 2, 1, 1, 256, 3},   // 19: near/far on the spatial order, 512 i per block
    {256, 4, 1, 1, 256, 3},   // 20: near/far, 1024 i per block
    {256, 4, 1, 4, 256, 3},   // 21: near/far, 256 i, four waves split the sources
    {256, 4, 1, 2, 256, 3},   // 22: near/far, 512 i, two waves per target group
    {256, 2, 1, 2, 256, 3},   // 23: near/far, 256 i, two waves per target group
    {256, 2, 1, 2, 256, 4},   // 24: as 23, frame stored by the ordering pass, 6 waves per SIMD
    {256, 2, 1, 4, 256, 5},   // 25: near/far, 128 i (half box group), four waves split the sources
};
int single_cfg_count() { return static_cast<int>(sizeof(kSingle) / sizeof(kSingle[0])); }
int single_cfg_count(bool comp) { return comp ? single_cfg_count() : 19; }
const PairCfg &single_cfg(int idx) { return kSingle[idx]; }

template <int BLOCK, int K, int LS, int SW, int TILE>
static hipError_t launch_single_t(bool comp, bool eps0, dim3 grid, const double *pos,
                                  const double *mass, const float4 *packed, int64_t n,
                                  float eps2f, int split, int64_t split_len, const OutArgs &o,
                                  hipStream_t st) {
  if (comp) {
    if (eps0)
      pair_single_kernel<BLOCK, K, LS, SW, TILE, true, true>
          <<<grid, BLOCK, 0, st>>>(pos, mass, packed, n, eps2f, split, split_len, o);
    else
      pair_single_kernel<BLOCK, K, LS, SW, TILE, true, false>
          <<<grid, BLOCK, 0, st>>>(pos, mass, packed, n, eps2f, split, split_len, o);
  } else {
    if (eps0)
      pair_single_kernel<BLOCK, K, LS, SW, TILE, false, true>
          <<<grid, BLOCK, 0, st>>>(pos, mass, packed, n, eps2f, split, split_len, o);
    else
      pair_single_kernel<BLOCK, K, LS, SW, TILE, false, false>
          <<<grid, BLOCK, 0, st>>>(pos, mass, packed, n, eps2f, split, split_len, o);
  }
  return hipGetLastError();
}

template <int K, int SW, int TJ, int GS>
static hipError_t launch_smem_t(bool comp, bool eps0, dim3 grid, const double *mass,
                                const float4 *packed, int64_t n, float eps2f, int64_t split_len,
                                const OutArgs &o, hipStream_t st) {
  if (comp) {
    if (eps0)
      pair_smem_kernel<K, SW, TJ, true, true, GS><<<grid, 256, 0, st>>>(packed, mass, n, eps2f, split_len, o);
    else
      pair_smem_kernel<K, SW, TJ, true, false, GS><<<grid, 256, 0, st>>>(packed, mass, n, eps2f, split_len, o);
  } else {
    if (eps0)
      pair_smem_kernel<K, SW, TJ, false, true, GS><<<grid, 256, 0, st>>>(packed, mass, n, eps2f, split_len, o);
    else
      pair_smem_kernel<K, SW, TJ, false, false, GS><<<grid, 256, 0, st>>>(packed, mass, n, eps2f, split_len, o);
  }
  return hipGetLastError();
}

hipError_t launch_pack(const double *pos, const double *mass, int64_t n, float4 *packed,
                       hipStream_t stream, bool ds) {
  if (n <= 0) return hipSuccess;
  const int64_t np = padded(n);
  const unsigned blocks = static_cast<unsigned>((np + 255) / 256);
  if (ds)
    pack_ds_kernel<<<blocks, 256, 0, stream>>>(pos, mass, n, np, packed);
  else
    pack_kernel<<<blocks, 256, 0, stream>>>(pos, mass, n, np, packed);
  return hipGetLastError();
}

hipError_t launch_pair_single(int cfg, bool comp, const double *pos, const double *mass,
                              const float4 *packed, int64_t n, double eps, double G, int split,
                              double *acc, double *pot, float4 *part, hipStream_t stream,
                              hipEvent_t after_pair) {
  if (n <= 0) return hipSuccess;
  if (cfg < 0 || cfg >= single_cfg_count()) return hipErrorInvalidValue;
  const PairCfg &c = kSingle[cfg];
  if (c.smem >= 3) return hipErrorInvalidValue;  // near/far: launch_order + launch_pair_nf
  const int64_t ib = cfg_iblock(c);
  const int64_t nblk = (n + ib - 1) / ib;
  if (split < 1) split = 1;
  if (split > max_split(n)) split = max_split(n);
  // Each split covers a whole number of tiles (and of kPad for the scalar
  // stream, whose padded source array ends at padded(n)).
  const int64_t unit = c.smem ? kPad : c.tile;
  int64_t split_len = (n + split - 1) / split;
  split_len = (split_len + unit - 1) / unit * unit;
  const float eps2f = static_cast<float>(eps * eps);
  const bool eps0 = eps == 0.0;
  OutArgs o{};
  o.G = G;
  o.n = n;
  if (split > 1) {
    o.part = part;
  } else {
    o.acc = acc;
    o.pot = pot;
  }
  dim3 grid(static_cast<unsigned>(nblk), static_cast<unsigned>(split));
  hipError_t e;
  switch (cfg) {
#define NB_CASE(I, B, K, LS, SW, T) \
  case I: e = launch_single_t<B, K, LS, SW, T>(comp, eps0, grid, pos, mass, packed, n, eps2f, split, split_len, o, stream); break;
#define NB_SMEM(I, K, SW, T, GS) \
  case I: e = launch_smem_t<K, SW, T, GS>(comp, eps0, grid, mass, packed, n, eps2f, split_len, o, stream); break;
    NB_CASE(0, 256, 1, 1, 1, 256)
    NB_CASE(1, 256, 2, 1, 1, 256)
    NB_CASE(2, 256, 4, 1, 1, 256)
    NB_CASE(3, 256, 2, 1, 2, 512)
    NB_CASE(4, 256, 1, 1, 4, 1024)
    NB_CASE(5, 256, 1, 4, 1, 256)
    NB_CASE(6, 256, 4, 1, 2, 512)
    NB_CASE(7, 256, 2, 1, 4, 1024)
    NB_CASE(8, 256, 8, 1, 1, 256)
    NB_CASE(9, 256, 2, 2, 1, 512)
    NB_SMEM(10, 1, 1, 256, 4)
    NB_SMEM(11, 2, 1, 256, 4)
    NB_SMEM(12, 4, 1, 256, 4)
    NB_SMEM(13, 1, 2, 256, 4)
    NB_SMEM(14, 2, 2, 256, 4)
    NB_SMEM(15, 1, 4, 256, 4)
    NB_SMEM(16, 1, 1, 256, 8)
    NB_SMEM(17, 1, 2, 256, 8)
    NB_SMEM(18, 1, 4, 256, 8)
#undef NB_CASE
#undef NB_SMEM
    default:
      return hipErrorInvalidValue;
  }
  if (e == hipSuccess && after_pair) e = hipEventRecord(after_pair, stream);
  if (e != hipSuccess || split == 1) return e;
  const unsigned cb = static_cast<unsigned>((n + 255) / 256);
  if (comp)
    combine_kernel<true><<<cb, 256, 0, stream>>>(part, split, n, mass, eps2f, eps0 ? 1 : 0, G, acc, pot);
  else
    combine_kernel<false><<<cb, 256, 0, stream>>>(part, split, n, mass, eps2f, eps0 ? 1 : 0, G, acc, pot);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched: a persistent grid claims (cluster, i-block) work items, heaviest
// first, from a global counter.

// Modes: LDS-tiled (0-3) and scalar-stream (4-8) block shapes. (Scalar-stream
// modes with 8-source groups were measured and lost to mode 4 at every
// cluster size class: items are too short to amortise the longer groups.) Each mode's
// kernel gets the LDS its shape needs: the double-buffered tile for the LDS
// modes (which also holds their cross-wave combine), the cross-wave combine
// buffer for the scalar-stream ones.
constexpr int kBatchedTile[] = {512, 512, 512, 256, 0, 0, 0, 0, 0};
constexpr int kBatchedK[] = {1, 1, 2, 2, 1, 1, 2, 1, 2};
constexpr int kBatchedSW[] = {4, 2, 2, 1, 4, 2, 2, 1, 1};
constexpr int kBatchedSmem[] = {0, 0, 0, 0, 1, 1, 1, 1, 1};
static_assert(sizeof(kBatchedK) / sizeof(kBatchedK[0]) == kBatchedModes, "mode tables");

template <int MODE, bool COMP>
constexpr int batched_lds_float4() {
  constexpr int tile = kBatchedTile[MODE] * (COMP ? 2 : 1) * 2;
  constexpr int sw = kBatchedSW[MODE];
  constexpr int combine = sw > 1 ? ((sw - 1) * (4 / sw) * 64 * kBatchedK[MODE] * 4 * (COMP ? 2 : 1) + 3) / 4 : 1;
  return tile > combine ? tile : combine;
}
static const PairCfg kBatched[] = {
    {256, 1, 1, 4, 512, 0},  // 0: 64 i per item, j split over 4 waves
    {256, 1, 1, 2, 512, 0},  // 1: 128 i per item
    {256, 2, 1, 2, 512, 0},  // 2: 256 i per item
    {256, 2, 1, 1, 256, 0},  // 3: 512 i per item
    {256, 1, 1, 4, 256, 1},  // 4: 64 i per item, scalar stream, 4-wave j split
    {256, 1, 1, 2, 256, 1},  // 5: 128 i
    {256, 2, 1, 2, 256, 1},  // 6: 256 i
    {256, 1, 1, 1, 256, 1},  // 7: 256 i
    {256, 2, 1, 1, 256, 1},  // 8: 512 i
};
int batched_mode_count() { return static_cast<int>(sizeof(kBatched) / sizeof(kBatched[0])); }
const PairCfg &batched_mode(int idx) { return kBatched[idx]; }

// Item sources in the slot layout: cluster k's sources start at slot
// j0 + delta and are zero-padded to a multiple of kSlotAlign.
template <int MODE, bool COMP, bool EPS0>
__device__ __forceinline__ void batched_item(const Item &d, const double *__restrict__ pos,
                                             const double *__restrict__ mass,
                                             const float4 *__restrict__ packed, float eps2f,
                                             float4 *lds, const OutArgs &o) {
  const int64_t i0 = d.i0, i1 = d.i1, j0 = d.j0, j1 = d.j1, delta = d.delta;
  // LDS modes read the plain sources through a shifted base (slot = j + delta).
  const float4 *pj = COMP ? nullptr : packed + delta;
  const int64_t s0 = j0 + delta;
  const int64_t s1 = s0 + (j1 - j0 + kSlotAlign - 1) / kSlotAlign * kSlotAlign;
  float *X = reinterpret_cast<float *>(lds);
  static_assert(kBatchedSmem[MODE] == 0 ||
                    smem_lds_floats<kBatchedK[MODE], kBatchedSW[MODE], COMP>() <= 4 * batched_lds_float4<MODE, COMP>(),
                "batched LDS too small for the cross-wave combine");
  if constexpr (MODE == 0) pair_block<256, 1, 1, 4, 512, COMP, EPS0>(pos, mass, pj, i0, i1, j0, j1, eps2f, lds, o);
  if constexpr (MODE == 1) pair_block<256, 1, 1, 2, 512, COMP, EPS0>(pos, mass, pj, i0, i1, j0, j1, eps2f, lds, o);
  if constexpr (MODE == 2) pair_block<256, 2, 1, 2, 512, COMP, EPS0>(pos, mass, pj, i0, i1, j0, j1, eps2f, lds, o);
  if constexpr (MODE == 3) pair_block<256, 2, 1, 1, 256, COMP, EPS0>(pos, mass, pj, i0, i1, j0, j1, eps2f, lds, o);
  if constexpr (MODE == 4) smem_block<1, 4, 256, COMP, EPS0>(packed, i0, i1, i0 + delta, s0, s1, eps2f, X, o);
  if constexpr (MODE == 5) smem_block<1, 2, 256, COMP, EPS0>(packed, i0, i1, i0 + delta, s0, s1, eps2f, X, o);
  if constexpr (MODE == 6) smem_block<2, 2, 256, COMP, EPS0>(packed, i0, i1, i0 + delta, s0, s1, eps2f, X, o);
  if constexpr (MODE == 7) smem_block<1, 1, 256, COMP, EPS0>(packed, i0, i1, i0 + delta, s0, s1, eps2f, X, o);
  if constexpr (MODE == 8) smem_block<2, 1, 256, COMP, EPS0>(packed, i0, i1, i0 + delta, s0, s1, eps2f, X, o);
}


// One persistent launch per mode: the grid claims the mode's items (a
// contiguous, heaviest-first segment of the plan's work list) from its own
// counter until none is left.
template <int MODE, bool COMP>
__device__ __forceinline__ void batched_loop(const double *__restrict__ pos,
                                             const double *__restrict__ mass,
                                             const float4 *__restrict__ packed,
                                             const Item *__restrict__ items, int32_t n_items,
                                             const double *__restrict__ eps_k, double G,
                                             int *__restrict__ counter, double *__restrict__ acc,
                                             double *__restrict__ pot) {
  __shared__ float4 lds[batched_lds_float4<MODE, COMP>()];
  __shared__ int s_item;
  OutArgs o{};
  o.acc = acc;
  o.pot = pot;
  o.G = G;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= n_items) break;
    const Item d = items[it];
    const double eps = eps_k[d.cluster];
    const float eps2f = static_cast<float>(eps * eps);
    if (eps == 0.0)
      batched_item<MODE, COMP, true>(d, pos, mass, packed, eps2f, lds, o);
    else
      batched_item<MODE, COMP, false>(d, pos, mass, packed, eps2f, lds, o);
    __syncthreads();
  }
}

// LDS modes: the compiler's own register allocation.
template <int MODE, bool COMP>
__global__ __launch_bounds__(256) void pair_batched_kernel(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const float4 *__restrict__ packed, const Item *__restrict__ items, int32_t n_items,
    const double *__restrict__ eps_k, double G, int *__restrict__ counter,
    double *__restrict__ acc, double *__restrict__ pot) {
  batched_loop<MODE, COMP>(pos, mass, packed, items, n_items, eps_k, G, counter, acc, pot);
}

// Scalar-stream modes: held to 8 waves per SIMD (the compensated form's item
// loop otherwise takes about 100 SGPRs, which leaves room for 7; at 8 it fits
// in 72 with no spills).
template <int MODE, bool COMP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void pair_batched_smem_kernel(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const float4 *__restrict__ packed, const Item *__restrict__ items, int32_t n_items,
    const double *__restrict__ eps_k, double G, int *__restrict__ counter,
    double *__restrict__ acc, double *__restrict__ pot) {
  batched_loop<MODE, COMP>(pos, mass, packed, items, n_items, eps_k, G, counter, acc, pot);
}

// Slot-layout pack of a batched plan: slot s holds source slot_src[s] (or
// zero-mass padding when negative); the compensated form splits x - c with
// the cluster frame c = pos[slot_frame[s]].
__global__ __launch_bounds__(256) void pack_slots_kernel(const double *__restrict__ pos,
                                                         const double *__restrict__ mass,
                                                         const int32_t *__restrict__ slot_src,
                                                         const int32_t *__restrict__ slot_frame,
                                                         int64_t n_slots, int ds,
                                                         float4 *__restrict__ out) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (s >= n_slots) return;
  const int64_t j = slot_src[s];
  if (ds) {
    if (j < 0) {
      out[2 * s] = make_float4(0.f, 0.f, 0.f, 0.f);
      out[2 * s + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
      return;
    }
    const int64_t f = slot_frame[s];
    float hx, hy, hz, lx, ly, lz;
    ds_split(pos[3 * j] - pos[3 * f], hx, lx);
    ds_split(pos[3 * j + 1] - pos[3 * f + 1], hy, ly);
    ds_split(pos[3 * j + 2] - pos[3 * f + 2], hz, lz);
    out[2 * s] = make_float4(hx, hy, hz, static_cast<float>(mass[j]));
    out[2 * s + 1] = make_float4(lx, ly, lz, 0.f);
  } else {
    out[s] = j < 0 ? make_float4(0.f, 0.f, 0.f, 0.f)
                   : make_float4(static_cast<float>(pos[3 * j]), static_cast<float>(pos[3 * j + 1]),
                                 static_cast<float>(pos[3 * j + 2]), static_cast<float>(mass[j]));
  }
}

template <int MODE>
static hipError_t launch_mode(const BatchedArgs &b, int m, const double *pos, const double *mass,
                             const float4 *packed, double G, int *counters, double *acc,
                             double *pot, hipStream_t st) {
  const Item *it = b.items + b.seg_begin[m];
  const int32_t cnt = b.seg_end[m] - b.seg_begin[m];
  if constexpr (kBatchedSmem[MODE] != 0) {
    if (b.comp)
      pair_batched_smem_kernel<MODE, true><<<b.grid[m], 256, 0, st>>>(pos, mass, packed, it, cnt,
                                                                       b.eps_k, G, counters + m, acc, pot);
    else
      pair_batched_smem_kernel<MODE, false><<<b.grid[m], 256, 0, st>>>(pos, mass, packed, it, cnt,
                                                                        b.eps_k, G, counters + m, acc, pot);
  } else {
    if (b.comp)
      pair_batched_kernel<MODE, true><<<b.grid[m], 256, 0, st>>>(pos, mass, packed, it, cnt, b.eps_k,
                                                                  G, counters + m, acc, pot);
    else
      pair_batched_kernel<MODE, false><<<b.grid[m], 256, 0, st>>>(pos, mass, packed, it, cnt, b.eps_k,
                                                                   G, counters + m, acc, pot);
  }
  return hipGetLastError();
}

hipError_t launch_pair_batched(const BatchedArgs &b, const double *pos, const double *mass,
                               float4 *packed, double G, int *counters, double *acc, double *pot,
                               hipStream_t stream) {
  if (b.n_items == 0) return hipSuccess;
  hipError_t e = launch_fill_int(counters, kBatchedModes, 0, stream);
  if (e != hipSuccess) return e;
  if (b.need_pack) {
    const unsigned blocks = static_cast<unsigned>((b.n_slots + 255) / 256);
    pack_slots_kernel<<<blocks, 256, 0, stream>>>(pos, mass, b.slot_src, b.slot_frame, b.n_slots,
                                                  b.comp ? 1 : 0, packed);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  for (int m = 0; m < kBatchedModes && e == hipSuccess; ++m) {
    if (b.seg_end[m] <= b.seg_begin[m]) continue;
    switch (m) {
      case 0: e = launch_mode<0>(b, m, pos, mass, packed, G, counters, acc, pot, stream); break;
      case 1: e = launch_mode<1>(b, m, pos, mass, packed, G, counters, acc, pot, stream); break;
      case 2: e = launch_mode<2>(b, m, pos, mass, packed, G, counters, acc, pot, stream); break;
      case 3: e = launch_mode<3>(b, m, pos, mass, packed, G, counters, acc, pot, stream); break;
      case 4: e = launch_mode<4>(b, m, pos, mass, packed, G, counters, acc, pot, stream); break;
      case 5: e = launch_mode<5>(b, m, pos, mass, packed, G, counters, acc, pot, stream); break;
      case 6: e = launch_mode<6>(b, m, pos, mass, packed, G, counters, acc, pot, stream); break;
      case 7: e = launch_mode<7>(b, m, pos, mass, packed, G, counters, acc, pot, stream); break;
      default: e = launch_mode<8>(b, m, pos, mass, packed, G, counters, acc, pot, stream); break;
    }
  }
  return e;
}

template <int MODE>
static int occupancy(bool comp) {
  int per = 0;
  hipError_t e;
  if constexpr (kBatchedSmem[MODE] != 0)
    e = comp ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pair_batched_smem_kernel<MODE, true>, 256, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pair_batched_smem_kernel<MODE, false>, 256, 0);
  else
    e = comp ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pair_batched_kernel<MODE, true>, 256, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pair_batched_kernel<MODE, false>, 256, 0);
  return e == hipSuccess ? per : 0;
}

int batched_grid(bool comp, int mode) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  int per = 0;
  switch (mode) {
    case 0: per = occupancy<0>(comp); break;
    case 1: per = occupancy<1>(comp); break;
    case 2: per = occupancy<2>(comp); break;
    case 3: per = occupancy<3>(comp); break;
    case 4: per = occupancy<4>(comp); break;
    case 5: per = occupancy<5>(comp); break;
    case 6: per = occupancy<6>(comp); break;
    case 7: per = occupancy<7>(comp); break;
    default: per = occupancy<8>(comp); break;
  }
  if (per < 1) per = 1;
  return cus * per;
}

// ---------------------------------------------------------------------------
// FP64 leapfrog and diagnostics.

__global__ __launch_bounds__(256) void kick_drift_kernel(double *__restrict__ pos,
                                                         double *__restrict__ vel,
                                                         const double *__restrict__ acc,
                                                         int64_t n3, double h, double dt) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; k < n3; k += stride) {
    const double v = vel[k] + h * acc[k];
    vel[k] = v;
    pos[k] = pos[k] + dt * v;
  }
}

__global__ __launch_bounds__(256) void kick_kernel(double *__restrict__ vel,
                                                   const double *__restrict__ acc, int64_t n3,
                                                   double h) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; k < n3; k += stride)
    vel[k] = vel[k] + h * acc[k];
}

static unsigned elementwise_blocks(int64_t n3) {
  int64_t b = (n3 + 255) / 256;
  if (b > 8192) b = 8192;
  return static_cast<unsigned>(b < 1 ? 1 : b);
}

hipError_t launch_kick_drift(double *pos, double *vel, const double *acc, int64_t n, double h,
                             double dt, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  kick_drift_kernel<<<elementwise_blocks(3 * n), 256, 0, stream>>>(pos, vel, acc, 3 * n, h, dt);
  return hipGetLastError();
}

hipError_t launch_kick(double *vel, const double *acc, int64_t n, double h, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  kick_kernel<<<elementwise_blocks(3 * n), 256, 0, stream>>>(vel, acc, 3 * n, h);
  return hipGetLastError();
}

// Quantities reduced for one diagnostics row, before the final pass.
constexpr int kRed = 13;  // K, W, P[3], L[3], sum m x [3], M, non-finite count

__device__ __forceinline__ void block_reduce(double (*sm)[kDiagThreads], double *v) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < kRed; ++q) sm[q][t] = v[q];
  __syncthreads();
  for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int q = 0; q < kRed; ++q) sm[q][t] += sm[q][t + w];
    }
    __syncthreads();
  }
}

// v += h a for every particle, then per-block partial diagnostics of the
// kicked state; one row of kDiagLen doubles per block.
__global__ __launch_bounds__(kDiagThreads) void kick_diag_kernel(
    const double *__restrict__ pos, double *__restrict__ vel, const double *__restrict__ acc,
    const double *__restrict__ pot, const double *__restrict__ mass, int64_t n, double h,
    int do_kick, double *__restrict__ partial) {
  __shared__ double sm[kRed][kDiagThreads];
  double v[kRed];
#pragma unroll
  for (int q = 0; q < kRed; ++q) v[q] = 0.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kDiagThreads;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kDiagThreads + threadIdx.x; i < n;
       i += stride) {
    double vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
    if (do_kick) {
      vx = vx + h * acc[3 * i];
      vy = vy + h * acc[3 * i + 1];
      vz = vz + h * acc[3 * i + 2];
      vel[3 * i] = vx;
      vel[3 * i + 1] = vy;
      vel[3 * i + 2] = vz;
    }
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    const double m = mass[i];
    v[0] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
    v[1] += 0.5 * m * pot[i];
    v[2] += m * vx;
    v[3] += m * vy;
    v[4] += m * vz;
    v[5] += m * (y * vz - z * vy);
    v[6] += m * (z * vx - x * vz);
    v[7] += m * (x * vy - y * vx);
    v[8] += m * x;
    v[9] += m * y;
    v[10] += m * z;
    v[11] += m;
    v[12] += (isfinite(x) ? 0.0 : 1.0) + (isfinite(y) ? 0.0 : 1.0) + (isfinite(z) ? 0.0 : 1.0) +
             (isfinite(vx) ? 0.0 : 1.0) + (isfinite(vy) ? 0.0 : 1.0) + (isfinite(vz) ? 0.0 : 1.0);
  }
  block_reduce(sm, v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kRed; ++q) partial[blockIdx.x * kDiagLen + q] = sm[q][0];
  }
}

__global__ __launch_bounds__(kDiagThreads) void diag_final_kernel(const double *__restrict__ partial,
                                                                  double *__restrict__ diag,
                                                                  int *__restrict__ step_ctr) {
  __shared__ double sm[kRed][kDiagThreads];
  double v[kRed];
#pragma unroll
  for (int q = 0; q < kRed; ++q) v[q] = 0.0;
  for (int b = threadIdx.x; b < kDiagBlocks; b += kDiagThreads) {
#pragma unroll
    for (int q = 0; q < kRed; ++q) v[q] += partial[b * kDiagLen + q];
  }
  block_reduce(sm, v);
  if (threadIdx.x == 0) {
    const int s = *step_ctr;
    double *row = diag + static_cast<int64_t>(s) * kDiagLen;
    const double K = sm[0][0], W = sm[1][0], M = sm[11][0];
    row[0] = K;
    row[1] = W;
    row[2] = K + W;
    for (int q = 0; q < 6; ++q) row[3 + q] = sm[2 + q][0];
    for (int q = 0; q < 3; ++q) row[9 + q] = sm[8 + q][0] / M;
    row[12] = M;
    row[13] = sm[12][0];
    row[14] = static_cast<double>(s + 1);
    row[15] = 0.0;
    *step_ctr = s + 1;
  }
}

hipError_t launch_kick_diag(const double *pos, double *vel, const double *acc, const double *pot,
                            const double *mass, int64_t n, double h, double *partial,
                            hipStream_t stream) {
  kick_diag_kernel<<<kDiagBlocks, kDiagThreads, 0, stream>>>(pos, vel, acc, pot, mass, n, h,
                                                             acc ? 1 : 0, partial);
  return hipGetLastError();
}

hipError_t launch_diag_final(const double *partial, double *diag, int *step_ctr,
                             hipStream_t stream) {
  diag_final_kernel<<<1, kDiagThreads, 0, stream>>>(partial, diag, step_ctr);
  return hipGetLastError();
}

__global__ void fill_int_kernel(int *p, int n, int value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

hipError_t launch_fill_int(int *p, int n, int value, hipStream_t stream) {
  fill_int_kernel<<<(n + 63) / 64, 64, 0, stream>>>(p, n, value);
  return hipGetLastError();
}

}  // namespace nb
