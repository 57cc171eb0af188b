// Near/far compensated acceleration + jerk kernel (gfx950): the near/far
// scheme of kernels_nf.hip applied to the jerk pair sum of kernels_jerk.hip.
//
// On the spatial order (kernels_order.hip, velocities gathered beside the
// positions), a block of IB = (4 / SW) * 64 * K ordered targets (whole box
// groups, or half of one) takes the centre of its box (diagonal D) as its
// FP64 position frame c and the velocity of its first target as its
// velocity frame u. Each 256-source tile
// is staged in LDS as {hi(x - c), m}, {lo(x - c), 0}, {fp32(v - u), 0};
// source tiles at least D / 4 from the block's box skip the lo parts (the
// separation then carries at most 6 u |d| of error, see kernels_nf.hip).
// The relative velocity is always fp32(v_j - u) - fp32(v_i - u), rounded
// relative to the velocities' spread. Per pair the jerk arithmetic is that of
// kernels_jerk.hip (acceleration, potential, J1 = sum s w, J2 = sum s beta
// d); every sum is TwoSum-merged into (hi, lo) once per tile, in a fixed
// order, and the jerk J1 - 3 J2 is formed once per target.
#include "device_common.h"

namespace nb {

namespace {

constexpr int kNfjTile = kOrderGroup;
constexpr int kNQ = 10;  // a (3), phi, J1 (3), J2 (3)

struct NfjOut {
  double *acc, *jerk, *pot;  // direct results, indexed through perm (split == 1)
  float4 *part;              // [split][n][4] partials in ordered index (split > 1)
  const int32_t *perm;
  int64_t n;
  double G;
};

template <int K, int SW>
constexpr int nfj_lds_float4() {
  constexpr int tiles = 2 * 3 * kNfjTile;
  constexpr int combine = SW > 1 ? ((SW - 1) * (4 / SW) * 64 * K * kNQ * 2 + 3) / 4 : 1;
  return tiles > combine ? tiles : combine;
}

// HG: the block covers half a box group (128 targets) and reads that half's
// box, centre and threshold from the ordering pass; a smaller target box
// makes more source tiles far.
template <int K, int SW, bool HG, bool EPS0>
__global__ __launch_bounds__(256) void pair_nf_jerk_kernel(const double *__restrict__ spos,
                                                           const double *__restrict__ svel,
                                                           const double *__restrict__ smass,
                                                           const double *__restrict__ box,
                                                           const double *__restrict__ bfr,
                                                           const double *__restrict__ hbox, int64_t n,
                                                           float eps2f, int64_t split_len, NfjOut o) {
  constexpr int NG = 4 / SW;
  constexpr int IB = NG * 64 * K;
  static_assert(4 % SW == 0 && (HG ? IB == kOrderGroup / 2 : IB % kOrderGroup == 0),
                "block shape");
  __shared__ float4 smem[nfj_lds_float4<K, SW>()];
  float4 (*lds)[3 * kNfjTile] = reinterpret_cast<float4 (*)[3 * kNfjTile]>(smem);
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int wj = wave % SW, wg = wave / SW;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * IB;
  const int64_t i1 = i0 + IB < n ? i0 + IB : n;
  const int64_t J0 = static_cast<int64_t>(blockIdx.y) * split_len;
  const int64_t J1 = J0 + split_len < n ? J0 + split_len : n;

  // a one-group (half-group) block reads box, centre and threshold as the
  // ordering pass wrote them (uniform loads, held in scalar registers)
  double bl[3], bh[3], cx, cy, cz, D2;
  if constexpr (HG) {
    const int64_t h = i0 / (kOrderGroup / 2);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      bl[c] = hbox[10 * h + c];
      bh[c] = hbox[10 * h + 3 + c];
    }
    cx = hbox[10 * h + 6];
    cy = hbox[10 * h + 7];
    cz = hbox[10 * h + 8];
    D2 = hbox[10 * h + 9];
  } else {
    const int64_t g0 = i0 / kOrderGroup;
    const int64_t g1 = IB == kOrderGroup ? g0 : (i1 - 1) / kOrderGroup;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      bl[c] = box[6 * g0 + c];
      bh[c] = box[6 * g0 + 3 + c];
    }
    for (int64_t g = g0 + 1; g <= g1; ++g) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        bl[c] = fmin(bl[c], box[6 * g + c]);
        bh[c] = fmax(bh[c], box[6 * g + 3 + c]);
      }
    }
    cx = IB == kOrderGroup ? bfr[4 * g0] : 0.5 * (bl[0] + bh[0]);
    cy = IB == kOrderGroup ? bfr[4 * g0 + 1] : 0.5 * (bl[1] + bh[1]);
    cz = IB == kOrderGroup ? bfr[4 * g0 + 2] : 0.5 * (bl[2] + bh[2]);
    D2 = IB == kOrderGroup ? bfr[4 * g0 + 3]
                           : 0.0625 * ((bh[0] - bl[0]) * (bh[0] - bl[0]) +
                                       (bh[1] - bl[1]) * (bh[1] - bl[1]) +
                                       (bh[2] - bl[2]) * (bh[2] - bl[2]));
  }
  const double ux = svel[3 * i0], uy = svel[3 * i0 + 1], uz = svel[3 * i0 + 2];

  float xh[K], yh[K], zh[K], xl[K], yl[K], zl[K], vx[K], vy[K], vz[K], mi[K];
  int64_t iidx[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t i = i0 + static_cast<int64_t>(k) * (NG * 64) + wg * 64 + lane;
    iidx[k] = i;
    const int64_t ic = i < i1 ? i : i1 - 1;
    ds_split(spos[3 * ic] - cx, xh[k], xl[k]);
    ds_split(spos[3 * ic + 1] - cy, yh[k], yl[k]);
    ds_split(spos[3 * ic + 2] - cz, zh[k], zl[k]);
    vx[k] = static_cast<float>(svel[3 * ic] - ux);
    vy[k] = static_cast<float>(svel[3 * ic + 1] - uy);
    vz[k] = static_cast<float>(svel[3 * ic + 2] - uz);
    mi[k] = static_cast<float>(smass[ic]);
  }

  float ah[K][kNQ], al[K][kNQ];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int c = 0; c < kNQ; ++c) ah[k][c] = al[k][c] = 0.f;

  auto is_far = [&](int64_t t) {
    const int64_t g = J0 / kNfjTile + t;
    double d2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double lo = box[6 * g + c], hi = box[6 * g + 3 + c];
      const double gap = lo > bh[c] ? lo - bh[c] : (bl[c] > hi ? bl[c] - hi : 0.0);
      d2 += gap * gap;
    }
    return d2 >= D2;
  };

  const int64_t ntiles = J1 > J0 ? (J1 - J0 + kNfjTile - 1) / kNfjTile : 0;
  double sx = cx, sy = cy, sz = cz, sm = 0.0, svx = ux, svy = uy, svz = uz;
  auto load = [&](int64_t t) {
    const int64_t j = J0 + t * kNfjTile + tid;
    if (j < J1) {
      sx = spos[3 * j];
      sy = spos[3 * j + 1];
      sz = spos[3 * j + 2];
      svx = svel[3 * j];
      svy = svel[3 * j + 1];
      svz = svel[3 * j + 2];
      sm = smass[j];
    } else {
      sx = cx;
      sy = cy;
      sz = cz;
      svx = ux;
      svy = uy;
      svz = uz;
      sm = 0.0;
    }
  };
  auto store = [&](int buf, bool far) {
    float4 *D = lds[buf] + 3 * tid;
    if (far) {
      D[0] = make_float4(static_cast<float>(sx - cx), static_cast<float>(sy - cy),
                         static_cast<float>(sz - cz), static_cast<float>(sm));
    } else {
      float hx, hy, hz, lx, ly, lz;
      ds_split(sx - cx, hx, lx);
      ds_split(sy - cy, hy, ly);
      ds_split(sz - cz, hz, lz);
      D[0] = make_float4(hx, hy, hz, static_cast<float>(sm));
      D[1] = make_float4(lx, ly, lz, 0.f);
    }
    D[2] = make_float4(static_cast<float>(svx - ux), static_cast<float>(svy - uy),
                       static_cast<float>(svz - uz), 0.f);
  };

  bool far_cur = false;
  if (ntiles > 0) {
    far_cur = is_far(0);
    load(0);
    store(0, far_cur);
  }
  __syncthreads();

  for (int64_t t = 0; t < ntiles; ++t) {
    const int buf = static_cast<int>(t & 1);
    const bool more = t + 1 < ntiles;
    bool far_next = false;
    if (more) {
      far_next = is_far(t + 1);
      load(t + 1);
    }
    const float4 *T = lds[buf];
    float p[K][kNQ];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < kNQ; ++c) p[k][c] = 0.f;

    // one pair: d (separation), w (relative velocity), m (source mass)
    // one target per lane: a shallower unroll keeps more waves resident
    constexpr int UNR = K == 1 ? 2 : 4;
    auto pair = [&](int k, float dx, float dy, float dz, const float4 &V, float m) {
      const float wx = V.x - vx[k], wy = V.y - vy[k], wz = V.z - vz[k];
      float r2 = fmaf(dx, dx, eps2f);
      r2 = fmaf(dy, dy, r2);
      r2 = fmaf(dz, dz, r2);
      float rho = rsq(r2);
      if constexpr (EPS0) rho = r2 > 0.f ? rho : 0.f;
      const float rho2 = rho * rho;
      const float mr = m * rho;
      const float s = mr * rho2;
      float rv = dx * wx;
      rv = fmaf(dy, wy, rv);
      rv = fmaf(dz, wz, rv);
      const float sb = s * (rv * rho2);
      p[k][0] = fmaf(s, dx, p[k][0]);
      p[k][1] = fmaf(s, dy, p[k][1]);
      p[k][2] = fmaf(s, dz, p[k][2]);
      p[k][3] += mr;
      p[k][4] = fmaf(s, wx, p[k][4]);
      p[k][5] = fmaf(s, wy, p[k][5]);
      p[k][6] = fmaf(s, wz, p[k][6]);
      p[k][7] = fmaf(sb, dx, p[k][7]);
      p[k][8] = fmaf(sb, dy, p[k][8]);
      p[k][9] = fmaf(sb, dz, p[k][9]);
    };

    if (far_cur) {
#pragma unroll UNR
      for (int jj = wj; jj < kNfjTile; jj += SW) {
        const float4 H = T[3 * jj], V = T[3 * jj + 2];
#pragma unroll
        for (int k = 0; k < K; ++k) pair(k, H.x - xh[k], H.y - yh[k], H.z - zh[k], V, H.w);
      }
    } else {
#pragma unroll UNR
      for (int jj = wj; jj < kNfjTile; jj += SW) {
        const float4 H = T[3 * jj], L = T[3 * jj + 1], V = T[3 * jj + 2];
#pragma unroll
        for (int k = 0; k < K; ++k)
          pair(k, (H.x - xh[k]) + (L.x - xl[k]), (H.y - yh[k]) + (L.y - yl[k]),
               (H.z - zh[k]) + (L.z - zl[k]), V, H.w);
      }
    }

#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < kNQ; ++c) {
        float s, e;
        two_sum(ah[k][c], p[k][c], s, e);
        ah[k][c] = s;
        al[k][c] += e;
      }

    if (more) store(buf ^ 1, far_next);
    far_cur = far_next;
    __syncthreads();
  }

  if constexpr (SW > 1) {
    float *X = reinterpret_cast<float *>(smem);
    constexpr int SLOT = NG * 64 * K * kNQ * 2;
    const int base = (wg * 64 + lane) * K * kNQ * 2;
    if (wj > 0) {
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < kNQ; ++c) {
          X[(wj - 1) * SLOT + base + (k * kNQ + c) * 2] = ah[k][c];
          X[(wj - 1) * SLOT + base + (k * kNQ + c) * 2 + 1] = al[k][c];
        }
    }
    __syncthreads();
    if (wj == 0) {
      for (int w = 1; w < SW; ++w) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
          for (int c = 0; c < kNQ; ++c) {
            const float oh = X[(w - 1) * SLOT + base + (k * kNQ + c) * 2];
            const float ol = X[(w - 1) * SLOT + base + (k * kNQ + c) * 2 + 1];
            float s, e;
            two_sum(ah[k][c], oh, s, e);
            ah[k][c] = s;
            al[k][c] = (al[k][c] + ol) + e;
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
      // jerk = J1 - 3 J2 folded exactly into one (hi, lo) pair per component
      float jh[3], jl[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float pr = -3.0f * ah[k][7 + c];
        const float pe = fmaf(-3.0f, ah[k][7 + c], -pr);
        float hs, he;
        two_sum(ah[k][4 + c], pr, hs, he);
        jh[c] = hs;
        jl[c] = fmaf(-3.0f, al[k][7 + c], al[k][4 + c]) + (pe + he);
      }
      float4 *P = o.part + (static_cast<int64_t>(blockIdx.y) * o.n + i) * 4;
      store_stream(P, make_float4(ah[k][0], ah[k][1], ah[k][2], ah[k][3]));
      store_stream(P + 1, make_float4(jh[0], jh[1], jh[2], 0.f));
      store_stream(P + 2, make_float4(al[k][0], al[k][1], al[k][2], al[k][3]));
      store_stream(P + 3, make_float4(jl[0], jl[1], jl[2], 0.f));
    } else {
      double s[kNQ];
#pragma unroll
      for (int c = 0; c < kNQ; ++c) s[c] = static_cast<double>(ah[k][c]) + static_cast<double>(al[k][c]);
      const int64_t d = o.perm[i];
      o.acc[3 * d] = o.G * s[0];
      o.acc[3 * d + 1] = o.G * s[1];
      o.acc[3 * d + 2] = o.G * s[2];
      o.jerk[3 * d] = o.G * (s[4] - 3.0 * s[7]);
      o.jerk[3 * d + 1] = o.G * (s[5] - 3.0 * s[8]);
      o.jerk[3 * d + 2] = o.G * (s[6] - 3.0 * s[9]);
      if (o.pot) {
        const double self = EPS0 ? 0.0 : static_cast<double>(self_term(mi[k], eps2f));
        o.pot[d] = -o.G * (s[3] - self);
      }
    }
  }
}

__global__ __launch_bounds__(256) void combine_nf_jerk_kernel(const float4 *__restrict__ part, int split,
                                                              int64_t n, const double *__restrict__ smass,
                                                              const int32_t *__restrict__ perm,
                                                              float eps2f, int eps0, double G,
                                                              double *__restrict__ acc,
                                                              double *__restrict__ jerk,
                                                              double *__restrict__ pot) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (k >= n) return;
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int q = 0; q < split; ++q) {
    const float4 *P = part + (static_cast<int64_t>(q) * n + k) * 4;
    for (int w = 0; w < 4; ++w) {
      const float4 v = P[w];
      const int c = (w & 1) * 4;
      s[c] += v.x;
      s[c + 1] += v.y;
      s[c + 2] += v.z;
      s[c + 3] += v.w;
    }
  }
  const int64_t d = perm[k];
  acc[3 * d] = G * s[0];
  acc[3 * d + 1] = G * s[1];
  acc[3 * d + 2] = G * s[2];
  jerk[3 * d] = G * s[4];
  jerk[3 * d + 1] = G * s[5];
  jerk[3 * d + 2] = G * s[6];
  if (pot) {
    const double self = eps0 ? 0.0 : static_cast<double>(self_term(static_cast<float>(smass[k]), eps2f));
    pot[d] = -G * (s[3] - self);
  }
}

// Velocities in the spatial order.
__global__ __launch_bounds__(256) void gather_vel_kernel(const double *__restrict__ vel,
                                                         const int32_t *__restrict__ perm, int64_t n,
                                                         double *__restrict__ svel) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (k >= n) return;
  const int64_t j = perm[k];
  svel[3 * k] = vel[3 * j];
  svel[3 * k + 1] = vel[3 * j + 1];
  svel[3 * k + 2] = vel[3 * j + 2];
}

template <int K, int SW, bool HG = false>
hipError_t launch_nfj_t(bool eps0, dim3 grid, const OrderWs &w, const double *svel, int64_t n,
                        float eps2f, int64_t split_len, const NfjOut &o, hipStream_t st) {
  if (eps0)
    pair_nf_jerk_kernel<K, SW, HG, true><<<grid, 256, 0, st>>>(
        w.spos, svel, w.smass, w.box, w.bfr, w.hbox, n, eps2f, split_len, o);
  else
    pair_nf_jerk_kernel<K, SW, HG, false><<<grid, 256, 0, st>>>(
        w.spos, svel, w.smass, w.box, w.bfr, w.hbox, n, eps2f, split_len, o);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gather_vel(const double *vel, const OrderWs &w, int64_t n, double *svel,
                             hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  gather_vel_kernel<<<static_cast<unsigned>((n + 255) / 256), 256, 0, stream>>>(vel, w.perm, n, svel);
  return hipGetLastError();
}

hipError_t launch_pair_nf_jerk(int k, int sw, const OrderWs &w, const double *svel, int64_t n,
                               double eps, double G, int split, double *acc, double *jerk,
                               double *pot, float4 *part, hipStream_t stream, hipEvent_t after_pair) {
  if (n <= 0) return hipSuccess;
  if (split < 1) split = 1;
  if (split > kMaxSplit || (split > 1 && static_cast<int64_t>(split) * n > kJerkPartCap))
    return hipErrorInvalidValue;
  int64_t split_len = (n + split - 1) / split;
  split_len = (split_len + kNfjTile - 1) / kNfjTile * kNfjTile;
  const int64_t ib = (4 / sw) * 64 * static_cast<int64_t>(k);
  const int64_t nblk = (n + ib - 1) / ib;
  const float eps2f = static_cast<float>(eps * eps);
  const bool eps0 = eps == 0.0;
  NfjOut o{};
  o.G = G;
  o.n = n;
  o.perm = w.perm;
  if (split > 1) {
    o.part = part;
  } else {
    o.acc = acc;
    o.jerk = jerk;
    o.pot = pot;
  }
  dim3 grid(static_cast<unsigned>(nblk), static_cast<unsigned>(split));
  hipError_t e;
  if (k == 1 && sw == 1) e = launch_nfj_t<1, 1>(eps0, grid, w, svel, n, eps2f, split_len, o, stream);
  else if (k == 2 && sw == 2) e = launch_nfj_t<2, 2>(eps0, grid, w, svel, n, eps2f, split_len, o, stream);
  else if (k == 1 && sw == 2)
    e = launch_nfj_t<1, 2, true>(eps0, grid, w, svel, n, eps2f, split_len, o, stream);
  else return hipErrorInvalidValue;
  if (e == hipSuccess && after_pair) e = hipEventRecord(after_pair, stream);
  if (e != hipSuccess || split == 1) return e;
  combine_nf_jerk_kernel<<<static_cast<unsigned>((n + 255) / 256), 256, 0, stream>>>(
      part, split, n, w.smass, w.perm, eps2f, eps0 ? 1 : 0, G, acc, jerk, pot);
  return hipGetLastError();
}

}  // namespace nb
