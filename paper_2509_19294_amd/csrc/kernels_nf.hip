// Near/far compensated pair kernel (gfx950).
//
// Works on the spatially ordered copy of the system (kernels_order.hip). A
// block (four waves) takes IB = (4 / SW) * 64 * K consecutive ordered targets
// (K per lane; SW waves share a target group and split each tile's sources,
// their sums combined through LDS in wave order); the bounding boxes of the
// IB / 256 groups (or of its half group, for IB = 128) give the block's box
// B, diagonal D, and the centre of B is its FP64 frame c. Source tiles of
// 256 ordered particles are staged in LDS relative to c, and each tile takes
// one of two paths, the same for the whole block:
//   * near (the tile's box lies closer to B than D / 4): double-single
//     staging, separation (hi_j - hi_i) + (lo_j - lo_i), as in the
//     compensated form;
//   * far (box distance >= D / 4): hi parts only, separation hi_j - hi_i.
// Far-path error: with |x_i - c| <= D / 2 and |x_j - c| <= |d| + D / 2,
// rounding the two offsets to FP32 and subtracting moves d by at most
// u (|x_i - c| + |x_j - c| + |d|) <= u (2 |d| + D) <= 6 u |d|, since every
// pair of a far tile has |d| >= D / 4 (u = 2^-24): a few units of FP32
// rounding of the separation itself, independent of where the system sits,
// at the plain form's 13 operations per pair. The self pair falls in a near
// tile (its box overlaps B) unless D = 0, where both offsets are exactly 0.
// Tile sums are merged into (hi, lo) accumulators with TwoSum, as in the
// compensated form; the order of every sum is fixed.
#include "device_common.h"

namespace nb {

namespace {

constexpr int kNfTile = kOrderGroup;  // sources per tile = particles per box group

struct NfOut {
  double *acc, *pot;      // direct results, indexed through perm (split == 1)
  float4 *part;           // [split][n][2] partials in ordered index (split > 1)
  const int32_t *perm;    // ordered index -> caller's index
  int64_t n;
  double G;
};

template <int K, int SW>
constexpr int nf_lds_float4() {
  constexpr int tiles = 2 * 2 * kNfTile;
  constexpr int combine = SW > 1 ? ((SW - 1) * (4 / SW) * 64 * K * 8 + 3) / 4 : 1;
  return tiles > combine ? tiles : combine;
}

// Frame modes. FR 0: the block covers whole box groups and computes the
// union of their boxes, its centre and threshold. FR 1: the block covers one
// box group and reads its box, centre and threshold as the ordering pass
// wrote them (uniform loads, which stay in scalar registers), and the
// compiler is held to 6 waves per SIMD, which the two-target shape then
// reaches without spills (94 -> 74 VGPRs). FR 2: the block covers half a box
// group (128 targets) and reads that half's box, centre and threshold: a
// smaller target box makes more source tiles far; the compiler is held to 6
// waves per SIMD as for FR 1.
template <int FR>
constexpr int nf_waves() {
  return FR != 0 ? 6 : 1;
}

template <int K, int SW, int FR, bool EPS0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(nf_waves<FR>()))) void
pair_nf_kernel(const double *__restrict__ spos, const double *__restrict__ smass,
               const double *__restrict__ box, const double *__restrict__ bfr,
               const double *__restrict__ hbox, int64_t n, float eps2f, int64_t split_len,
               uint32_t nblk, uint32_t nsplit, int order, NfOut o) {
  constexpr int NG = 4 / SW;          // target groups of 64 lanes per block
  constexpr int IB = NG * 64 * K;
  constexpr int kHalf = kNfTile / 2;
  static_assert(4 % SW == 0, "block shape");
  static_assert(FR == 0 ? IB % kOrderGroup == 0 : IB == (FR == 1 ? kOrderGroup : kHalf),
                "frame mode and block shape");
  __shared__ float4 smem[nf_lds_float4<K, SW>()];
  float4 (*lds)[2 * kNfTile] = reinterpret_cast<float4 (*)[2 * kNfTile]>(smem);
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int wj = wave % SW, wg = wave / SW;
  uint32_t bx, by;
  xcd_block(blockIdx.x, nblk, nsplit, order, bx, by);
  const int64_t i0 = static_cast<int64_t>(bx) * IB;
  const int64_t i1 = i0 + IB < n ? i0 + IB : n;
  const int64_t J0 = static_cast<int64_t>(by) * split_len;
  const int64_t J1 = J0 + split_len < n ? J0 + split_len : n;

  // the block's box: union of its groups' boxes (or its half group's box);
  // the frame is its centre
  double bl[3], bh[3], cx, cy, cz, D2;  // D2: far threshold (D / 4)^2
  if constexpr (FR == 2) {
    const int64_t h = i0 / kHalf;
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
    const int64_t g1 = FR == 1 ? g0 : (i1 - 1) / kOrderGroup;
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
    if constexpr (FR == 1) {
      cx = bfr[4 * g0];
      cy = bfr[4 * g0 + 1];
      cz = bfr[4 * g0 + 2];
      D2 = bfr[4 * g0 + 3];
    } else {
      cx = 0.5 * (bl[0] + bh[0]);
      cy = 0.5 * (bl[1] + bh[1]);
      cz = 0.5 * (bl[2] + bh[2]);
      D2 = 0.0625 * ((bh[0] - bl[0]) * (bh[0] - bl[0]) + (bh[1] - bl[1]) * (bh[1] - bl[1]) +
                     (bh[2] - bl[2]) * (bh[2] - bl[2]));
    }
  }

  float xh[K], yh[K], zh[K], xl[K], yl[K], zl[K], mi[K];
  int64_t iidx[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t i = i0 + static_cast<int64_t>(k) * (NG * 64) + wg * 64 + lane;
    iidx[k] = i;
    const int64_t ic = i < i1 ? i : i1 - 1;
    ds_split(spos[3 * ic] - cx, xh[k], xl[k]);
    ds_split(spos[3 * ic + 1] - cy, yh[k], yl[k]);
    ds_split(spos[3 * ic + 2] - cz, zh[k], zl[k]);
    mi[k] = static_cast<float>(smass[ic]);
  }

  float ah[K][4], al[K][4];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) ah[k][c] = al[k][c] = 0.f;

  // tile t covers ordered sources [J0 + t * kNfTile, ...): box group
  // (J0 / kNfTile) + t, since split boundaries are multiples of kNfTile
  auto is_far = [&](int64_t t) {
    const int64_t g = J0 / kNfTile + t;
    double d2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double lo = box[6 * g + c], hi = box[6 * g + 3 + c];
      const double gap = lo > bh[c] ? lo - bh[c] : (bl[c] > hi ? bl[c] - hi : 0.0);
      d2 += gap * gap;
    }
    return d2 >= D2;
  };

  const int64_t ntiles = J1 > J0 ? (J1 - J0 + kNfTile - 1) / kNfTile : 0;
  double sx = cx, sy = cy, sz = cz, sm = 0.0;  // staged source (registers)
  auto load = [&](int64_t t) {
    const int64_t j = J0 + t * kNfTile + tid;
    if (j < J1) {
      sx = spos[3 * j];
      sy = spos[3 * j + 1];
      sz = spos[3 * j + 2];
      sm = smass[j];
    } else {
      sx = cx;
      sy = cy;
      sz = cz;
      sm = 0.0;
    }
  };
  auto store = [&](int buf, bool far) {
    if (far) {
      lds[buf][2 * tid] = make_float4(static_cast<float>(sx - cx), static_cast<float>(sy - cy),
                                      static_cast<float>(sz - cz), static_cast<float>(sm));
    } else {
      float hx, hy, hz, lx, ly, lz;
      ds_split(sx - cx, hx, lx);
      ds_split(sy - cy, hy, ly);
      ds_split(sz - cz, hz, lz);
      lds[buf][2 * tid] = make_float4(hx, hy, hz, static_cast<float>(sm));
      lds[buf][2 * tid + 1] = make_float4(lx, ly, lz, 0.f);
    }
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
    float p[K][4];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) p[k][c] = 0.f;

    if (far_cur) {
#pragma unroll 8
      for (int jj = wj; jj < kNfTile; jj += SW) {
        const float4 H = T[2 * jj];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float dx = H.x - xh[k], dy = H.y - yh[k], dz = H.z - zh[k];
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
    } else {
#pragma unroll 8
      for (int jj = wj; jj < kNfTile; jj += SW) {
        const float4 H = T[2 * jj], L = T[2 * jj + 1];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float dx = (H.x - xh[k]) + (L.x - xl[k]);
          const float dy = (H.y - yh[k]) + (L.y - yl[k]);
          const float dz = (H.z - zh[k]) + (L.z - zl[k]);
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
    }

#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        float s, e;
        two_sum(ah[k][c], p[k][c], s, e);
        ah[k][c] = s;
        al[k][c] += e;
      }

    if (more) store(buf ^ 1, far_next);
    far_cur = far_next;
    __syncthreads();
  }

  // waves sharing a target group: waves 1..SW-1 park their sums in LDS (the
  // tile buffers are free after the last barrier), wave 0 adds them in order
  if constexpr (SW > 1) {
    float *X = reinterpret_cast<float *>(smem);
    constexpr int SLOT = NG * 64 * K * 8;
    const int base = (wg * 64 + lane) * K * 8;
    if (wj > 0) {
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          X[(wj - 1) * SLOT + base + k * 8 + 2 * c] = ah[k][c];
          X[(wj - 1) * SLOT + base + k * 8 + 2 * c + 1] = al[k][c];
        }
    }
    __syncthreads();
    if (wj == 0) {
      for (int w = 1; w < SW; ++w) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const float oh = X[(w - 1) * SLOT + base + k * 8 + 2 * c];
            const float ol = X[(w - 1) * SLOT + base + k * 8 + 2 * c + 1];
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
      float4 *P = o.part + (static_cast<int64_t>(by) * o.n + i) * 2;
      store_stream(P, make_float4(ah[k][0], ah[k][1], ah[k][2], ah[k][3]));
      store_stream(P + 1, make_float4(al[k][0], al[k][1], al[k][2], al[k][3]));
    } else {
      double s[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) s[c] = static_cast<double>(ah[k][c]) + static_cast<double>(al[k][c]);
      const int64_t d = o.perm[i];
      o.acc[3 * d] = o.G * s[0];
      o.acc[3 * d + 1] = o.G * s[1];
      o.acc[3 * d + 2] = o.G * s[2];
      if (o.pot) {
        const double self = EPS0 ? 0.0 : static_cast<double>(self_term(mi[k], eps2f));
        o.pot[d] = -o.G * (s[3] - self);
      }
    }
  }
}

// Sums the split partials of ordered particle k in split order (FP64),
// applies G and the self-term correction, and writes to the caller's index.
__global__ __launch_bounds__(256) void combine_nf_kernel(const float4 *__restrict__ part, int split,
                                                         int64_t n, const double *__restrict__ smass,
                                                         const int32_t *__restrict__ perm,
                                                         float eps2f, int eps0, double G,
                                                         double *__restrict__ acc,
                                                         double *__restrict__ pot) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (k >= n) return;
  double s[4] = {0, 0, 0, 0};
  for (int q = 0; q < split; ++q) {
    const float4 *P = part + (static_cast<int64_t>(q) * n + k) * 2;
    const float4 h = P[0], l = P[1];
    s[0] += static_cast<double>(h.x) + static_cast<double>(l.x);
    s[1] += static_cast<double>(h.y) + static_cast<double>(l.y);
    s[2] += static_cast<double>(h.z) + static_cast<double>(l.z);
    s[3] += static_cast<double>(h.w) + static_cast<double>(l.w);
  }
  const int64_t d = perm[k];
  acc[3 * d] = G * s[0];
  acc[3 * d + 1] = G * s[1];
  acc[3 * d + 2] = G * s[2];
  if (pot) {
    const double self = eps0 ? 0.0 : static_cast<double>(self_term(static_cast<float>(smass[k]), eps2f));
    pot[d] = -G * (s[3] - self);
  }
}

template <int K, int SW, int FR = 0>
hipError_t launch_nf_t(bool eps0, uint32_t nblk, uint32_t split, const OrderWs &w, int64_t n,
                       float eps2f, int64_t split_len, const NfOut &o, hipStream_t st) {
  // Block order across the XCDs (xcd_block). A split's sources are staged
  // from 32 B of FP64 position and mass each; once a split holds more than
  // a quarter of an XCD's 4 MB L2, per-XCD splits keep them there (else each
  // XCD's L2 cycles through every split). Below that the plain order is
  // better: it lets each XCD read only its share of the targets per split.
  const uint64_t total = static_cast<uint64_t>(nblk) * split;
  const bool big = static_cast<uint64_t>(n / split) * 32 > (uint64_t{1} << 20);
  const int order = !big ? 0 : (split % 8 == 0 ? 1 : (8 % split == 0 && total % 8 == 0 ? 2 : 0));
  const dim3 grid(static_cast<unsigned>(total));
  if (eps0)
    pair_nf_kernel<K, SW, FR, true><<<grid, 256, 0, st>>>(w.spos, w.smass, w.box, w.bfr, w.hbox, n,
                                                          eps2f, split_len, nblk, split, order, o);
  else
    pair_nf_kernel<K, SW, FR, false><<<grid, 256, 0, st>>>(w.spos, w.smass, w.box, w.bfr, w.hbox, n,
                                                           eps2f, split_len, nblk, split, order, o);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pair_nf(int k, int sw, int fr, const OrderWs &w, int64_t n, double eps,
                          double G, int split, double *acc, double *pot, float4 *part,
                          hipStream_t stream, hipEvent_t after_pair) {
  if (n <= 0) return hipSuccess;
  if (split < 1) split = 1;
  if (split > max_split(n)) split = max_split(n);
  int64_t split_len = (n + split - 1) / split;
  split_len = (split_len + kNfTile - 1) / kNfTile * kNfTile;
  const int64_t ib = (4 / sw) * 64 * static_cast<int64_t>(k);
  const int64_t nblk = (n + ib - 1) / ib;
  const float eps2f = static_cast<float>(eps * eps);
  const bool eps0 = eps == 0.0;
  NfOut o{};
  o.G = G;
  o.n = n;
  o.perm = w.perm;
  if (split > 1) {
    o.part = part;
  } else {
    o.acc = acc;
    o.pot = pot;
  }
  const uint32_t nb = static_cast<uint32_t>(nblk), sp = static_cast<uint32_t>(split);
  hipError_t e;
  if (fr == 1 && k == 2 && sw == 2)
    e = launch_nf_t<2, 2, 1>(eps0, nb, sp, w, n, eps2f, split_len, o, stream);
  else if (fr == 2 && k == 2 && sw == 4)
    e = launch_nf_t<2, 4, 2>(eps0, nb, sp, w, n, eps2f, split_len, o, stream);
  else if (fr != 0) return hipErrorInvalidValue;
  else if (k == 2 && sw == 1) e = launch_nf_t<2, 1>(eps0, nb, sp, w, n, eps2f, split_len, o, stream);
  else if (k == 4 && sw == 1) e = launch_nf_t<4, 1>(eps0, nb, sp, w, n, eps2f, split_len, o, stream);
  else if (k == 4 && sw == 4) e = launch_nf_t<4, 4>(eps0, nb, sp, w, n, eps2f, split_len, o, stream);
  else if (k == 4 && sw == 2) e = launch_nf_t<4, 2>(eps0, nb, sp, w, n, eps2f, split_len, o, stream);
  else if (k == 2 && sw == 2) e = launch_nf_t<2, 2>(eps0, nb, sp, w, n, eps2f, split_len, o, stream);
  else return hipErrorInvalidValue;
  if (e == hipSuccess && after_pair) e = hipEventRecord(after_pair, stream);
  if (e != hipSuccess || split == 1) return e;
  combine_nf_kernel<<<static_cast<unsigned>((n + 255) / 256), 256, 0, stream>>>(
      part, split, n, w.smass, w.perm, eps2f, eps0 ? 1 : 0, G, acc, pot);
  return hipGetLastError();
}

}  // namespace nb
