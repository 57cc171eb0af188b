// Acceleration + jerk pair kernel and the FP64 fourth-order Hermite
// predictor-corrector, for gfx950.
//
// The jerk is the time derivative of the softened acceleration (the paper's
// device computes it beside the force, Section 3):
//   jerk_i = G sum_{j != i} m_j [w q^{-3/2} - 3 (d.w) d q^{-5/2}],
//   d = x_j - x_i, w = v_j - v_i, q = |d|^2 + eps^2.
// Per pair, on top of the force's 13 FP32 operations and one v_rsq_f32: the
// relative velocity (3), d.w (3), s beta = s (d.w) rho^2 (2), J1 += s w (3)
// and J2 += s beta d (3), with s = m rho^3; the jerk is J1 - 3 J2, formed
// once per target (two accumulators instead of one keep the factor 3, a
// literal operand, out of the pair loop).
//
// The kernel follows the scalar-stream layout of the force kernel: each wave
// streams its sources from a zero-padded packed array with scalar loads
// (four sources per group), K targets per lane in VGPRs, SW waves of a block
// splitting the sources (combined through LDS in wave order), a grid j-split
// combined in FP64 by a second kernel. Sums are two-level (plain FP32 per
// tile, then a running sum; TwoSum into hi/lo for the compensated form).
// Packed source: plain {x,y,z,m},{v-u,0}; compensated {hi(x-c),m},
// {lo(x-c),0},{v-u,0} with c = pos[0], u = vel[0] (FP64 frames). The jerk
// depends on velocity differences only, so both forms take velocities
// relative to particle 0's: their rounding, and the cancellation of the split
// J1 sum below, then scale with the spread of the velocities, not with a
// bulk motion of the system.
//
// Plain form, one target per lane: J1 is accumulated as sum s v_j and
// sum s, and v_i times the second is subtracted once per tile, so the three
// J1 products take the source velocity straight from the scalar registers
// (two vector-register reads instead of three, which lets more of them
// dual-issue) for one extra add per pair; what v_i sum s cancels is of the
// size of |v_j - u| sum s. The self pair (s = m eps^-3, the
// largest term of all, which the subtraction would then have to cancel)
// never enters those sums: the source groups that overlap the wave's own
// 64 targets use the relative-velocity form, where the self pair's w is 0.
#include <type_traits>

#include "device_common.h"

namespace nb {

namespace {

template <bool COMP>
constexpr int jw_of() {
  return COMP ? 3 : 2;
}

__global__ __launch_bounds__(256) void pack_jerk_kernel(const double *__restrict__ pos,
                                                        const double *__restrict__ vel,
                                                        const double *__restrict__ mass,
                                                        int64_t n, int64_t npad, int comp,
                                                        float4 *__restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= npad) return;
  const int jw = comp ? 3 : 2;
  float4 *o = out + i * jw;
  if (i >= n) {
    for (int c = 0; c < jw; ++c) o[c] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  const float m = static_cast<float>(mass[i]);
  if (comp) {
    float hx, hy, hz, lx, ly, lz;
    ds_split(pos[3 * i] - pos[0], hx, lx);
    ds_split(pos[3 * i + 1] - pos[1], hy, ly);
    ds_split(pos[3 * i + 2] - pos[2], hz, lz);
    o[0] = make_float4(hx, hy, hz, m);
    o[1] = make_float4(lx, ly, lz, 0.f);
    o[2] = make_float4(static_cast<float>(vel[3 * i] - vel[0]), static_cast<float>(vel[3 * i + 1] - vel[1]),
                       static_cast<float>(vel[3 * i + 2] - vel[2]), 0.f);
  } else {
    o[0] = make_float4(static_cast<float>(pos[3 * i]), static_cast<float>(pos[3 * i + 1]),
                       static_cast<float>(pos[3 * i + 2]), m);
    o[1] = make_float4(static_cast<float>(vel[3 * i] - vel[0]), static_cast<float>(vel[3 * i + 1] - vel[1]),
                       static_cast<float>(vel[3 * i + 2] - vel[2]), 0.f);
  }
}

struct JerkOut {
  double *acc, *jerk, *pot;  // direct results (split == 1)
  float4 *part;              // [split][n][2 or 4] partials (split > 1)
  int64_t n;
  double G;
};

// GS: sources a wave loads per group (4, or 8 for the plain form, whose
// eight sources fit the scalar registers: 64 SGPRs).
template <int K, int SW, bool COMP, bool EPS0, int GS>
__global__ __launch_bounds__(256) void pair_jerk_kernel(const float4 *__restrict__ packed,
                                                        int64_t n, float eps2f, int64_t split_len,
                                                        JerkOut o) {
  constexpr int NW = 4, NG = NW / SW, IB = NG * 64 * K;
  constexpr int JW = jw_of<COMP>();
  constexpr int G4 = GS;            // sources per group
  static_assert(GS == 4 || (GS == 8 && !COMP), "group size");
  constexpr int STEP = SW * G4;     // stride between a wave's groups
  constexpr int TJ = 256;           // sources per wave per tile
  // accumulated quantities: a (3), phi, J1 = sum s w (3), J2 = sum s beta d (3)
  constexpr int NQ = 10;
  constexpr int OW = COMP ? 4 : 2;  // float4 words per partial entry
  // J1 as sum s v_j - v_i sum s (plain, one target per lane)
  constexpr bool JS = !COMP && K == 1;
  static_assert(NW % SW == 0, "bad shape");
  __shared__ float X[(SW > 1) ? (SW - 1) * NG * 64 * K * NQ * (COMP ? 2 : 1) : 1];

  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const int wj = wave % SW, wg = wave / SW;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * IB;
  const int64_t i1 = i0 + IB < n ? i0 + IB : n;
  const int64_t np = padded(n);
  const int64_t J0 = static_cast<int64_t>(blockIdx.y) * split_len;
  const int64_t J1 = J0 + split_len < np ? J0 + split_len : np;

  float xh[K], yh[K], zh[K], xl[K], yl[K], zl[K], vx[K], vy[K], vz[K], mi[K];
  int64_t iidx[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t i = i0 + static_cast<int64_t>(k) * (NG * 64) + wg * 64 + lane;
    iidx[k] = i;
    const int64_t ic = i < i1 ? i : i1 - 1;
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
    const float4 V = packed[ic * JW + (COMP ? 2 : 1)];
    vx[k] = V.x;
    vy[k] = V.y;
    vz[k] = V.z;
  }

  float ah[K][NQ], al[K][NQ];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int c = 0; c < NQ; ++c) ah[k][c] = al[k][c] = 0.f;

  const Quad *Qp = reinterpret_cast<const Quad *>(packed);
  for (int64_t t = J0 + wj * G4; t < J1; t += static_cast<int64_t>(TJ) * SW) {
    const int64_t tend = t + static_cast<int64_t>(TJ) * SW < J1 ? t + static_cast<int64_t>(TJ) * SW : J1;
    float p[K][NQ + 1];  // [NQ]: sum s (JS only)
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < NQ + 1; ++c) p[k][c] = 0.f;
    const uint32_t ngroups = static_cast<uint32_t>((tend - t + STEP - 1) / STEP);
    const Quad *Qt = Qp + ((static_cast<uint64_t>(t) * JW) >> 2);
    // SPLIT: J1 into sum s v_j and sum s
    // PF: the next group's scalar loads are issued before this group's pairs
    // (one target per lane, groups of at most 32 scalar registers)
    constexpr int NQD = G4 * JW / 4;
    constexpr bool PF = K == 1 && NQD <= 2;
    auto groups = [&](uint32_t g0, uint32_t g1, auto split_tag) {
      constexpr bool SPLIT = decltype(split_tag)::value;
      Quad cur[NQD];
      if constexpr (PF) {
        if (g0 < g1) {
#pragma unroll
          for (int q = 0; q < NQD; ++q) cur[q] = Qt[g0 * (STEP * JW / 4) + q];
        }
      }
      for (uint32_t gi = g0; gi < g1; ++gi) {
        Quad nxt[NQD];
        if constexpr (PF) {
          const uint32_t gn = gi + 1 < g1 ? gi + 1 : gi;
#pragma unroll
          for (int q = 0; q < NQD; ++q) nxt[q] = Qt[gn * (STEP * JW / 4) + q];
        }
        const Quad *Qg = PF ? cur : Qt + gi * (STEP * JW / 4);
        float4 W[G4 * JW];
#pragma unroll
        for (int w = 0; w < G4 * JW / 4; ++w) {
          const Quad qd = Qg[w];
#pragma unroll
          for (int c = 0; c < 4; ++c) W[w * 4 + c] = qd.v[c];
        }
#pragma unroll
        for (int g = 0; g < G4; ++g) {
          const float4 H = W[g * JW];
          const float4 L = COMP ? W[g * JW + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
          const float4 V = W[g * JW + (COMP ? 2 : 1)];
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
            const float wx = V.x - vx[k], wy = V.y - vy[k], wz = V.z - vz[k];
            float r2 = fmaf(dx, dx, eps2f);
            r2 = fmaf(dy, dy, r2);
            r2 = fmaf(dz, dz, r2);
            float rho = rsq(r2);
            if constexpr (EPS0) rho = r2 > 0.f ? rho : 0.f;
            const float rho2 = rho * rho;
            const float mr = H.w * rho;
            const float s = mr * rho2;
            float rv = dx * wx;
            rv = fmaf(dy, wy, rv);
            rv = fmaf(dz, wz, rv);
            const float sb = s * (rv * rho2);
            p[k][0] = fmaf(s, dx, p[k][0]);
            p[k][1] = fmaf(s, dy, p[k][1]);
            p[k][2] = fmaf(s, dz, p[k][2]);
            p[k][3] += mr;
            if constexpr (SPLIT) {
              p[k][4] = fmaf(s, V.x, p[k][4]);
              p[k][5] = fmaf(s, V.y, p[k][5]);
              p[k][6] = fmaf(s, V.z, p[k][6]);
              p[k][NQ] += s;
            } else {
              p[k][4] = fmaf(s, wx, p[k][4]);
              p[k][5] = fmaf(s, wy, p[k][5]);
              p[k][6] = fmaf(s, wz, p[k][6]);
            }
            p[k][7] = fmaf(sb, dx, p[k][7]);
            p[k][8] = fmaf(sb, dy, p[k][8]);
            p[k][9] = fmaf(sb, dz, p[k][9]);
          }
        }
        if constexpr (PF) {
#pragma unroll
          for (int q = 0; q < NQD; ++q) cur[q] = nxt[q];
        }
      }
    };
    if constexpr (JS) {
      // groups [ga, gb) overlap the wave's own targets [iw, iw + 64): they
      // keep the relative-velocity form, so the self pair adds exactly 0
      const int64_t iw = i0 + wg * 64;
      const int64_t lo = iw - G4 - t, hi = iw + 64 - t;
      int64_t ga = lo < 0 ? 0 : lo / STEP + 1;
      int64_t gb = hi <= 0 ? 0 : (hi + STEP - 1) / STEP;
      ga = ga < ngroups ? ga : ngroups;
      gb = gb < ga ? ga : (gb < ngroups ? gb : ngroups);
      groups(0, static_cast<uint32_t>(ga), std::true_type{});
      groups(static_cast<uint32_t>(ga), static_cast<uint32_t>(gb), std::false_type{});
      groups(static_cast<uint32_t>(gb), ngroups, std::true_type{});
    } else {
      groups(0, ngroups, std::false_type{});
    }
    if constexpr (JS) {
      p[0][4] = fmaf(-vx[0], p[0][NQ], p[0][4]);
      p[0][5] = fmaf(-vy[0], p[0][NQ], p[0][5]);
      p[0][6] = fmaf(-vz[0], p[0][NQ], p[0][6]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        if constexpr (COMP) {
          float hs, he;
          two_sum(ah[k][c], p[k][c], hs, he);
          ah[k][c] = hs;
          al[k][c] += he;
        } else {
          ah[k][c] += p[k][c];
        }
      }
  }

  if constexpr (SW > 1) {
    constexpr int CW = COMP ? 2 : 1;
    constexpr int SLOT = NG * 64 * K * NQ * CW;
    const int base = (wg * 64 + lane) * K * NQ * CW;
    if (wj > 0) {
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < NQ; ++c) {
          X[(wj - 1) * SLOT + base + (k * NQ + c) * CW] = ah[k][c];
          if constexpr (COMP) X[(wj - 1) * SLOT + base + (k * NQ + c) * CW + 1] = al[k][c];
        }
    }
    __syncthreads();
    if (wj == 0) {
      for (int w = 1; w < SW; ++w) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
          for (int c = 0; c < NQ; ++c) {
            const float oh = X[(w - 1) * SLOT + base + (k * NQ + c) * CW];
            if constexpr (COMP) {
              const float ol = X[(w - 1) * SLOT + base + (k * NQ + c) * CW + 1];
              float hs, he;
              two_sum(ah[k][c], oh, hs, he);
              ah[k][c] = hs;
              al[k][c] = (al[k][c] + ol) + he;
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
      // fold jerk = J1 - 3 J2 into one partial (exactly for the hi/lo form:
      // the product's rounding error from an FMA, the sum's from TwoSum)
      float jh[3], jl[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float pr = -3.0f * ah[k][7 + c];
        if constexpr (COMP) {
          const float pe = fmaf(-3.0f, ah[k][7 + c], -pr);
          float hs, he;
          two_sum(ah[k][4 + c], pr, hs, he);
          jh[c] = hs;
          jl[c] = fmaf(-3.0f, al[k][7 + c], al[k][4 + c]) + (pe + he);
        } else {
          jh[c] = fmaf(-3.0f, ah[k][7 + c], ah[k][4 + c]);
          jl[c] = 0.f;
        }
      }
      float4 *P = o.part + (static_cast<int64_t>(blockIdx.y) * o.n + i) * OW;
      P[0] = make_float4(ah[k][0], ah[k][1], ah[k][2], ah[k][3]);
      P[1] = make_float4(jh[0], jh[1], jh[2], 0.f);
      if constexpr (COMP) {
        P[2] = make_float4(al[k][0], al[k][1], al[k][2], al[k][3]);
        P[3] = make_float4(jl[0], jl[1], jl[2], 0.f);
      }
    } else {
      double sum[NQ];
#pragma unroll
      for (int c = 0; c < NQ; ++c)
        sum[c] = COMP ? static_cast<double>(ah[k][c]) + static_cast<double>(al[k][c])
                      : static_cast<double>(ah[k][c]);
      o.acc[3 * i] = o.G * sum[0];
      o.acc[3 * i + 1] = o.G * sum[1];
      o.acc[3 * i + 2] = o.G * sum[2];
      o.jerk[3 * i] = o.G * (sum[4] - 3.0 * sum[7]);
      o.jerk[3 * i + 1] = o.G * (sum[5] - 3.0 * sum[8]);
      o.jerk[3 * i + 2] = o.G * (sum[6] - 3.0 * sum[9]);
      if (o.pot) {
        const double self = EPS0 ? 0.0 : static_cast<double>(self_term(mi[k], eps2f));
        o.pot[i] = -o.G * (sum[3] - self);
      }
    }
  }
}

template <bool COMP>
__global__ __launch_bounds__(256) void combine_jerk_kernel(const float4 *__restrict__ part,
                                                           int split, int64_t n,
                                                           const double *__restrict__ mass,
                                                           float eps2f, int eps0, double G,
                                                           double *__restrict__ acc,
                                                           double *__restrict__ jerk,
                                                           double *__restrict__ pot) {
  constexpr int OW = COMP ? 4 : 2;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int q = 0; q < split; ++q) {
    const float4 *P = part + (static_cast<int64_t>(q) * n + i) * OW;
    for (int w = 0; w < OW; ++w) {
      const float4 v = P[w];
      const int c = (w & 1) * 4;
      s[c] += v.x;
      s[c + 1] += v.y;
      s[c + 2] += v.z;
      s[c + 3] += v.w;
    }
  }
  acc[3 * i] = G * s[0];
  acc[3 * i + 1] = G * s[1];
  acc[3 * i + 2] = G * s[2];
  jerk[3 * i] = G * s[4];
  jerk[3 * i + 1] = G * s[5];
  jerk[3 * i + 2] = G * s[6];
  if (pot) {
    const double self = eps0 ? 0.0 : static_cast<double>(self_term(static_cast<float>(mass[i]), eps2f));
    pot[i] = -G * (s[3] - self);
  }
}

// Hermite predictor: x_p = x + v dt + a dt^2/2 + j dt^3/6, v_p = v + a dt + j dt^2/2.
__global__ __launch_bounds__(256) void hermite_predict_kernel(
    const double *__restrict__ pos, const double *__restrict__ vel, const double *__restrict__ acc,
    const double *__restrict__ jerk, int64_t n3, double dt, double *__restrict__ xp,
    double *__restrict__ vp) {
  const double h2 = 0.5 * dt * dt, h3 = dt * dt * dt / 6.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; k < n3; k += stride) {
    const double v = vel[k], a = acc[k], j = jerk[k];
    xp[k] = pos[k] + dt * v + h2 * a + h3 * j;
    vp[k] = v + dt * a + h2 * j;
  }
}

// Hermite corrector; also moves (a_1, j_1) into (acc, jerk).
__global__ __launch_bounds__(256) void hermite_correct_kernel(
    double *__restrict__ pos, double *__restrict__ vel, double *__restrict__ acc,
    double *__restrict__ jerk, const double *__restrict__ a1, const double *__restrict__ j1,
    int64_t n3, double dt) {
  const double h = 0.5 * dt, h12 = dt * dt / 12.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; k < n3; k += stride) {
    const double v0 = vel[k], a0 = acc[k], jj0 = jerk[k], aa1 = a1[k], jj1 = j1[k];
    const double v1 = v0 + h * (a0 + aa1) + h12 * (jj0 - jj1);
    pos[k] = pos[k] + h * (v0 + v1) + h12 * (a0 - aa1);
    vel[k] = v1;
    acc[k] = aa1;
    jerk[k] = jj1;
  }
}

// GS = 8 applies to the plain form; the compensated form keeps GS = 4.
template <int K, int SW, int GS = 4>
hipError_t launch_jerk_t(bool comp, bool eps0, dim3 grid, const float4 *packed, int64_t n,
                         float eps2f, int64_t split_len, const JerkOut &o, hipStream_t st) {
  if (comp) {
    if (eps0) pair_jerk_kernel<K, SW, true, true, 4><<<grid, 256, 0, st>>>(packed, n, eps2f, split_len, o);
    else pair_jerk_kernel<K, SW, true, false, 4><<<grid, 256, 0, st>>>(packed, n, eps2f, split_len, o);
  } else {
    if (eps0) pair_jerk_kernel<K, SW, false, true, GS><<<grid, 256, 0, st>>>(packed, n, eps2f, split_len, o);
    else pair_jerk_kernel<K, SW, false, false, GS><<<grid, 256, 0, st>>>(packed, n, eps2f, split_len, o);
  }
  return hipGetLastError();
}

// Compiled shapes: K targets per lane, SW of the block's four waves splitting
// the sources of one target group; shapes 8 and 9 load eight sources per
// group in the plain form (four in the compensated form).
struct JerkShape {
  int k, sw;
};
constexpr JerkShape kJerkShapes[] = {{1, 1}, {1, 2}, {1, 4}, {2, 1}, {2, 2}, {2, 4},
                                     {4, 1}, {4, 2}, {1, 4}, {1, 2}, {1, 1}, {2, 2}, {1, 2}};
// shapes 10-12: near/far kernel on the spatial order (compensated form);
// shape 12 takes half a box group (128 targets) per block
constexpr int kJerkFirstNf = 10;
constexpr int kJerkShapeCount = static_cast<int>(sizeof(kJerkShapes) / sizeof(kJerkShapes[0]));

hipError_t launch_jerk_shape(int cfg, bool comp, bool eps0, dim3 grid, const float4 *packed, int64_t n,
                             float eps2f, int64_t split_len, const JerkOut &o, hipStream_t st) {
  switch (cfg) {
    case 0: return launch_jerk_t<1, 1>(comp, eps0, grid, packed, n, eps2f, split_len, o, st);
    case 1: return launch_jerk_t<1, 2>(comp, eps0, grid, packed, n, eps2f, split_len, o, st);
    case 2: return launch_jerk_t<1, 4>(comp, eps0, grid, packed, n, eps2f, split_len, o, st);
    case 3: return launch_jerk_t<2, 1>(comp, eps0, grid, packed, n, eps2f, split_len, o, st);
    case 4: return launch_jerk_t<2, 2>(comp, eps0, grid, packed, n, eps2f, split_len, o, st);
    case 5: return launch_jerk_t<2, 4>(comp, eps0, grid, packed, n, eps2f, split_len, o, st);
    case 6: return launch_jerk_t<4, 1>(comp, eps0, grid, packed, n, eps2f, split_len, o, st);
    case 7: return launch_jerk_t<4, 2>(comp, eps0, grid, packed, n, eps2f, split_len, o, st);
    case 8: return launch_jerk_t<1, 4, 8>(comp, eps0, grid, packed, n, eps2f, split_len, o, st);
    case 9: return launch_jerk_t<1, 2, 8>(comp, eps0, grid, packed, n, eps2f, split_len, o, st);
    // near/far shapes run through launch_pair_nf_jerk
    default: return hipErrorInvalidValue;
  }
}

unsigned elementwise_grid(int64_t n3) {
  int64_t b = (n3 + 255) / 256;
  if (b > 8192) b = 8192;
  return static_cast<unsigned>(b < 1 ? 1 : b);
}

}  // namespace

int jerk_shape_count() { return kJerkShapeCount; }
int jerk_shape_count(bool comp) { return comp ? kJerkShapeCount : kJerkFirstNf; }
bool jerk_shape_nf(int cfg) { return cfg >= kJerkFirstNf && cfg < kJerkShapeCount; }

int jerk_targets_per_block(int cfg) {
  if (cfg < 0 || cfg >= kJerkShapeCount) return 0;
  return (4 / kJerkShapes[cfg].sw) * 64 * kJerkShapes[cfg].k;
}

void jerk_shape(int cfg, int *k, int *sw) {
  *k = kJerkShapes[cfg].k;
  *sw = kJerkShapes[cfg].sw;
}

int jerk_default_split(int64_t n, int cfg) {
  // Aim for about 8192 blocks, each split keeping at least 1024 sources,
  // within the partial buffer's bound.
  const int ib = jerk_targets_per_block(cfg);
  const int64_t blocks = (n + ib - 1) / ib;
  int split = 1;
  while (split < kMaxSplit && blocks * split < 8192 && n / (split * 2) >= 1024 &&
         static_cast<int64_t>(split * 2) * n <= kJerkPartCap)
    split *= 2;
  return split;
}

hipError_t launch_pack_jerk(const double *pos, const double *vel, const double *mass, int64_t n,
                            bool comp, float4 *packed, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int64_t np = padded(n);
  pack_jerk_kernel<<<static_cast<unsigned>((np + 255) / 256), 256, 0, stream>>>(pos, vel, mass, n, np,
                                                                              comp ? 1 : 0, packed);
  return hipGetLastError();
}

hipError_t launch_pair_jerk(int cfg, bool comp, const float4 *packed, const double *mass, int64_t n,
                            double eps, double G, int split, double *acc, double *jerk,
                            double *pot, float4 *part, hipStream_t stream, hipEvent_t after_pair) {
  if (n <= 0) return hipSuccess;
  const int ib = jerk_targets_per_block(cfg);
  if (ib == 0 || split > kMaxSplit || (split > 1 && static_cast<int64_t>(split) * n > kJerkPartCap))
    return hipErrorInvalidValue;
  const int64_t nblk = (n + ib - 1) / ib;
  if (split < 1) split = 1;
  int64_t split_len = (n + split - 1) / split;
  split_len = (split_len + kPad - 1) / kPad * kPad;
  const float eps2f = static_cast<float>(eps * eps);
  const bool eps0 = eps == 0.0;
  JerkOut o{};
  o.G = G;
  o.n = n;
  if (split > 1) {
    o.part = part;
  } else {
    o.acc = acc;
    o.jerk = jerk;
    o.pot = pot;
  }
  dim3 grid(static_cast<unsigned>(nblk), static_cast<unsigned>(split));
  hipError_t e = launch_jerk_shape(cfg, comp, eps0, grid, packed, n, eps2f, split_len, o, stream);
  if (e == hipSuccess && after_pair) e = hipEventRecord(after_pair, stream);
  if (e != hipSuccess || split == 1) return e;
  const unsigned cb = static_cast<unsigned>((n + 255) / 256);
  if (comp)
    combine_jerk_kernel<true><<<cb, 256, 0, stream>>>(part, split, n, mass, eps2f, eps0 ? 1 : 0, G, acc, jerk, pot);
  else
    combine_jerk_kernel<false><<<cb, 256, 0, stream>>>(part, split, n, mass, eps2f, eps0 ? 1 : 0, G, acc, jerk, pot);
  return hipGetLastError();
}

hipError_t launch_hermite_predict(const double *pos, const double *vel, const double *acc,
                                  const double *jerk, int64_t n, double dt, double *xp,
                                  double *vp, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hermite_predict_kernel<<<elementwise_grid(3 * n), 256, 0, stream>>>(pos, vel, acc, jerk, 3 * n, dt, xp, vp);
  return hipGetLastError();
}

hipError_t launch_hermite_correct(double *pos, double *vel, double *acc, double *jerk,
                                  const double *a1, const double *j1, int64_t n, double dt,
                                  hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hermite_correct_kernel<<<elementwise_grid(3 * n), 256, 0, stream>>>(pos, vel, acc, jerk, a1, j1, 3 * n, dt);
  return hipGetLastError();
}

}  // namespace nb
