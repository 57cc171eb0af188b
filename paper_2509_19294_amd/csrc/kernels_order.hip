// Spatial ordering of the particles, for the near/far compensated pair
// kernel (kernels_nf.hip): a deterministic permutation that puts particles
// close in space close in index, the positions and masses gathered in that
// order, and a bounding box for every group of kOrderGroup consecutive
// particles and every half group, with their centres and a quarter of their
// diagonals, squared.
//
// Keys: each coordinate is mapped through u = asinh((x - mean) / s), with s
// the RMS distance from the mean position per axis, so that a Plummer-like
// halo reaching thousands of core radii still leaves most of the resolution to
// the core; u is clamped to [-8, 8] and quantised to 10 bits; the key is the
// 30-bit Morton (Z-order) interleave of the three. Any order is correct for
// the pair kernel (it only decides which source tiles may skip the lo terms);
// a better order only makes more of them eligible.
//
// Sort: least-significant-digit radix sort of (key, index) pairs, four passes
// of 8 bits. Each pass histograms chunks of 256 elements (LDS counters),
// scans the digit-major histogram matrix (digit, chunk) exclusively, and
// scatters every element to its digit's base plus its rank among the earlier
// elements of its chunk with the same digit. The sort is stable and its result
// depends only on the keys, so the permutation is reproducible bit for bit.
#include "device_common.h"

namespace nb {

namespace {

constexpr int kOrdThreads = 256;   // one element per thread in the radix passes
constexpr int kMomentBlocks = 256; // blocks of the moments pass (fixed partition)
constexpr int kScanPer = 1024;     // histogram entries one scan block covers
constexpr double kUClamp = 8.0;    // |asinh| clamp
constexpr int kKeyBits = 10;       // Morton bits per axis

// Per-block partial moments: sum x, y, z and sum x^2, y^2, z^2 (FP64).
__global__ __launch_bounds__(256) void moments_kernel(const double *__restrict__ pos, int64_t n,
                                                      double *__restrict__ part) {
  __shared__ double sm[6][256];
  double v[6] = {0, 0, 0, 0, 0, 0};
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double x = pos[3 * i + c];
      v[c] += x;
      v[3 + c] += x * x;
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) sm[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) {
#pragma unroll
      for (int c = 0; c < 6; ++c) sm[c][threadIdx.x] += sm[c][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sm[threadIdx.x][0];
}

// Spreads the low 10 bits of v to every third bit.
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ __forceinline__ uint32_t quantise(double x, double mean, double inv_s) {
  double u = asinh((x - mean) * inv_s);
  if (!(u == u)) u = 0.0;  // non-finite input: any cell will do
  u = u < -kUClamp ? -kUClamp : (u > kUClamp ? kUClamp : u);
  const double q = (u + kUClamp) * ((1 << kKeyBits) / (2.0 * kUClamp));
  int qi = static_cast<int>(q);
  qi = qi < 0 ? 0 : (qi > (1 << kKeyBits) - 1 ? (1 << kKeyBits) - 1 : qi);
  return static_cast<uint32_t>(qi);
}

// Keys and initial indices. Every block reduces the moment partials itself,
// in the same fixed order, so all blocks use identical means and scales.
__global__ __launch_bounds__(256) void keys_kernel(const double *__restrict__ pos, int64_t n,
                                                   const double *__restrict__ part,
                                                   uint32_t *__restrict__ key,
                                                   int32_t *__restrict__ idx) {
  __shared__ double st[6];
  if (threadIdx.x < 6) {
    double s = 0.0;
    for (int b = 0; b < kMomentBlocks; ++b) s += part[b * 6 + threadIdx.x];
    st[threadIdx.x] = s;
  }
  __syncthreads();
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const double inv_n = 1.0 / static_cast<double>(n);
  uint32_t q[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double mean = st[c] * inv_n;
    double var = st[3 + c] * inv_n - mean * mean;
    const double s = var > 0.0 ? sqrt(var) : 1.0;
    q[c] = quantise(pos[3 * i + c], mean, 1.0 / s);
  }
  key[i] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
  idx[i] = static_cast<int32_t>(i);
}

// Digit histogram of one chunk of 256 elements: H[digit * nchunks + chunk].
__global__ __launch_bounds__(256) void radix_hist_kernel(const uint32_t *__restrict__ key, int64_t n,
                                                         int shift, int64_t nchunks,
                                                         uint32_t *__restrict__ H) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
  __syncthreads();
  H[static_cast<int64_t>(threadIdx.x) * nchunks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of 256 per-thread values in LDS (work-efficient, in place);
// returns the total.
__device__ uint32_t block_exclusive_scan(uint32_t *s) {
  const int t = threadIdx.x;
  for (int d = 1; d < 256; d <<= 1) {  // up-sweep
    __syncthreads();
    const int k = (t + 1) * 2 * d - 1;
    if (k < 256) s[k] += s[k - d];
  }
  __syncthreads();
  const uint32_t total = s[255];
  __syncthreads();
  if (t == 0) s[255] = 0;
  for (int d = 128; d >= 1; d >>= 1) {  // down-sweep
    __syncthreads();
    const int k = (t + 1) * 2 * d - 1;
    if (k < 256) {
      const uint32_t a = s[k - d];
      s[k - d] = s[k];
      s[k] += a;
    }
  }
  __syncthreads();
  return total;
}

// Exclusive scan of kScanPer consecutive entries per block, in place; the
// block's total goes to S[block].
__global__ __launch_bounds__(256) void scan_block_kernel(uint32_t *__restrict__ H, int64_t L,
                                                         uint32_t *__restrict__ S) {
  __shared__ uint32_t s[256];
  constexpr int PER = kScanPer / 256;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanPer + threadIdx.x * PER;
  uint32_t v[PER];
  uint32_t sum = 0;
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    v[r] = base + r < L ? H[base + r] : 0u;
    sum += v[r];
  }
  s[threadIdx.x] = sum;
  const uint32_t total = block_exclusive_scan(s);
  uint32_t run = s[threadIdx.x];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    if (base + r < L) H[base + r] = run;
    run += v[r];
  }
  if (threadIdx.x == 0) S[blockIdx.x] = total;
}

// Exclusive scan of the nb block totals, in place, by one block.
__global__ __launch_bounds__(256) void scan_totals_kernel(uint32_t *__restrict__ S, int64_t nb) {
  __shared__ uint32_t s[256];
  const int64_t per = (nb + 255) / 256;
  const int64_t b0 = static_cast<int64_t>(threadIdx.x) * per;
  uint32_t sum = 0;
  for (int64_t r = 0; r < per && b0 + r < nb; ++r) sum += S[b0 + r];
  s[threadIdx.x] = sum;
  block_exclusive_scan(s);
  uint32_t run = s[threadIdx.x];
  for (int64_t r = 0; r < per && b0 + r < nb; ++r) {
    const uint32_t v = S[b0 + r];
    S[b0 + r] = run;
    run += v;
  }
}

__global__ __launch_bounds__(256) void scan_add_kernel(uint32_t *__restrict__ H, int64_t L,
                                                       const uint32_t *__restrict__ S) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < L) H[i] += S[i / kScanPer];
}

// Stable scatter: base of (digit, chunk) plus the rank among the chunk's
// earlier elements with the same digit.
__global__ __launch_bounds__(256) void radix_scatter_kernel(const uint32_t *__restrict__ kin,
                                                            const int32_t *__restrict__ iin,
                                                            int64_t n, int shift, int64_t nchunks,
                                                            const uint32_t *__restrict__ H,
                                                            uint32_t *__restrict__ kout,
                                                            int32_t *__restrict__ iout) {
  __shared__ int dig[256];
  const int t = threadIdx.x;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + t;
  const bool valid = i < n;
  const uint32_t k = valid ? kin[i] : 0u;
  const int d = valid ? static_cast<int>((k >> shift) & 255u) : -1;
  dig[t] = d;
  __syncthreads();
  if (!valid) return;
  uint32_t r = 0;
  for (int u = 0; u < t; ++u) r += dig[u] == d ? 1u : 0u;
  const uint32_t dest = H[static_cast<int64_t>(d) * nchunks + blockIdx.x] + r;
  kout[dest] = k;
  iout[dest] = iin[i];
}

// Positions and masses in the new order.
__global__ __launch_bounds__(256) void gather_kernel(const double *__restrict__ pos,
                                                     const double *__restrict__ mass,
                                                     const int32_t *__restrict__ perm, int64_t n,
                                                     double *__restrict__ spos,
                                                     double *__restrict__ smass) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (k >= n) return;
  const int64_t j = perm[k];
  spos[3 * k] = pos[3 * j];
  spos[3 * k + 1] = pos[3 * j + 1];
  spos[3 * k + 2] = pos[3 * j + 2];
  smass[k] = mass[j];
}

// Bounding box of every group of kOrderGroup consecutive (ordered)
// particles: box[6 g .. 6 g + 5] = min x, y, z, max x, y, z;
// bfr[4 g .. 4 g + 3] = centre x, y, z and (diagonal / 4)^2, the frame and
// far threshold of a pair-kernel block that covers exactly this group; and
// the same for each half group h = 2 g, 2 g + 1: hbox[10 h .. 10 h + 9] =
// min xyz, max xyz, centre xyz, (diagonal / 4)^2. A half group past the end
// holds min +inf and max -inf (every box is then at infinite distance).
__global__ __launch_bounds__(kOrderGroup) void box_kernel(const double *__restrict__ spos, int64_t n,
                                                          double *__restrict__ box,
                                                          double *__restrict__ bfr,
                                                          double *__restrict__ hbox) {
  constexpr int kHalf = kOrderGroup / 2;
  __shared__ double lo[3][kOrderGroup], hi[3][kOrderGroup];
  const int t = threadIdx.x;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kOrderGroup + t;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double x = k < n ? spos[3 * k + c] : 0.0;
    lo[c][t] = k < n ? x : HUGE_VAL;
    hi[c][t] = k < n ? x : -HUGE_VAL;
  }
  __syncthreads();
  // each half reduced on its own: lo[.][0] and lo[.][kHalf] hold the halves
  for (int w = kHalf / 2; w > 0; w >>= 1) {
    if ((t & (kHalf - 1)) < w) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        lo[c][t] = fmin(lo[c][t], lo[c][t + w]);
        hi[c][t] = fmax(hi[c][t], hi[c][t + w]);
      }
    }
    __syncthreads();
  }
  if (t < 2) {
    const int64_t h = 2 * static_cast<int64_t>(blockIdx.x) + t;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double l = lo[c][t * kHalf], u = hi[c][t * kHalf];
      hbox[10 * h + c] = l;
      hbox[10 * h + 3 + c] = u;
      hbox[10 * h + 6 + c] = 0.5 * (l + u);
    }
    const double ex = hi[0][t * kHalf] - lo[0][t * kHalf];
    const double ey = hi[1][t * kHalf] - lo[1][t * kHalf];
    const double ez = hi[2][t * kHalf] - lo[2][t * kHalf];
    hbox[10 * h + 9] = 0.0625 * (ex * ex + ey * ey + ez * ez);
  }
  if (t < 3) {
    const double l = fmin(lo[t][0], lo[t][kHalf]), u = fmax(hi[t][0], hi[t][kHalf]);
    box[6 * blockIdx.x + t] = l;
    box[6 * blockIdx.x + 3 + t] = u;
    bfr[4 * blockIdx.x + t] = 0.5 * (l + u);
  }
  if (t == 0) {
    // the same expression as the pair kernel's own threshold of a group
    const double ex = fmax(hi[0][0], hi[0][kHalf]) - fmin(lo[0][0], lo[0][kHalf]);
    const double ey = fmax(hi[1][0], hi[1][kHalf]) - fmin(lo[1][0], lo[1][kHalf]);
    const double ez = fmax(hi[2][0], hi[2][kHalf]) - fmin(lo[2][0], lo[2][kHalf]);
    bfr[4 * blockIdx.x + 3] = 0.0625 * (ex * ex + ey * ey + ez * ez);
  }
}

}  // namespace

OrderWs order_ws_at(void *base, int64_t n) {
  OrderWs w{};
  const int64_t nchunks = (n + 255) / 256;
  const int64_t L = 256 * nchunks;
  const int64_t nscan = (L + kScanPer - 1) / kScanPer;
  const int64_t ngroups = (n + kOrderGroup - 1) / kOrderGroup;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~static_cast<size_t>(255);
    return o;
  };
  const size_t o_mom = take(static_cast<size_t>(kMomentBlocks) * 6 * sizeof(double));
  const size_t o_k0 = take(static_cast<size_t>(n) * sizeof(uint32_t));
  const size_t o_k1 = take(static_cast<size_t>(n) * sizeof(uint32_t));
  const size_t o_i0 = take(static_cast<size_t>(n) * sizeof(int32_t));
  const size_t o_i1 = take(static_cast<size_t>(n) * sizeof(int32_t));
  const size_t o_h = take(static_cast<size_t>(L) * sizeof(uint32_t));
  const size_t o_s = take(static_cast<size_t>(nscan) * sizeof(uint32_t));
  const size_t o_pos = take(static_cast<size_t>(n) * 3 * sizeof(double));
  const size_t o_mass = take(static_cast<size_t>(n) * sizeof(double));
  const size_t o_box = take(static_cast<size_t>(ngroups) * 6 * sizeof(double));
  const size_t o_bfr = take(static_cast<size_t>(ngroups) * 4 * sizeof(double));
  const size_t o_hbox = take(static_cast<size_t>(ngroups) * 2 * 10 * sizeof(double));
  w.bytes = off;
  if (base) {
    char *b = static_cast<char *>(base);
    w.moments = reinterpret_cast<double *>(b + o_mom);
    w.key0 = reinterpret_cast<uint32_t *>(b + o_k0);
    w.key1 = reinterpret_cast<uint32_t *>(b + o_k1);
    w.perm = reinterpret_cast<int32_t *>(b + o_i0);
    w.idx1 = reinterpret_cast<int32_t *>(b + o_i1);
    w.hist = reinterpret_cast<uint32_t *>(b + o_h);
    w.scan = reinterpret_cast<uint32_t *>(b + o_s);
    w.spos = reinterpret_cast<double *>(b + o_pos);
    w.smass = reinterpret_cast<double *>(b + o_mass);
    w.box = reinterpret_cast<double *>(b + o_box);
    w.bfr = reinterpret_cast<double *>(b + o_bfr);
    w.hbox = reinterpret_cast<double *>(b + o_hbox);
  }
  return w;
}

hipError_t launch_order(const double *pos, const double *mass, int64_t n, const OrderWs &w,
                        hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n >= (int64_t{1} << 31)) return hipErrorInvalidValue;
  const int64_t nchunks = (n + 255) / 256;
  const int64_t L = 256 * nchunks;
  const int64_t nscan = (L + kScanPer - 1) / kScanPer;
  const unsigned nb = static_cast<unsigned>(nchunks);
  moments_kernel<<<kMomentBlocks, 256, 0, st>>>(pos, n, w.moments);
  keys_kernel<<<nb, 256, 0, st>>>(pos, n, w.moments, w.key0, w.perm);
  // four 8-bit passes: key0/perm -> key1/idx1 -> key0/perm -> ...
  uint32_t *kin = w.key0, *kout = w.key1;
  int32_t *iin = w.perm, *iout = w.idx1;
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 8 * pass;
    radix_hist_kernel<<<nb, 256, 0, st>>>(kin, n, shift, nchunks, w.hist);
    scan_block_kernel<<<static_cast<unsigned>(nscan), 256, 0, st>>>(w.hist, L, w.scan);
    scan_totals_kernel<<<1, 256, 0, st>>>(w.scan, nscan);
    scan_add_kernel<<<static_cast<unsigned>((L + 255) / 256), 256, 0, st>>>(w.hist, L, w.scan);
    radix_scatter_kernel<<<nb, 256, 0, st>>>(kin, iin, n, shift, nchunks, w.hist, kout, iout);
    uint32_t *kt = kin;
    kin = kout;
    kout = kt;
    int32_t *it = iin;
    iin = iout;
    iout = it;
  }
  // after an even number of passes the order is back in key0 / perm
  gather_kernel<<<nb, 256, 0, st>>>(pos, mass, w.perm, n, w.spos, w.smass);
  const unsigned ng = static_cast<unsigned>((n + kOrderGroup - 1) / kOrderGroup);
  box_kernel<<<ng, kOrderGroup, 0, st>>>(w.spos, n, w.box, w.bfr, w.hbox);
  return hipGetLastError();
}

}  // namespace nb
