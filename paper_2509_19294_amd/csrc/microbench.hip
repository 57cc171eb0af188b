// Instruction-rate microbenchmarks for gfx950, used to set the instruction
// budget of the pair kernel. Each kernel runs ILP independent dependency
// chains per lane, so the measurement is issue-bound rather than
// latency-bound; results are stored so nothing is optimised away. Built into
// libnbody_micro.so and driven by paper_2509_19294_amd.microbench; not part
// of libnbody.so.
//
// Operations (OP):
//   0 fma_f32 (VGPR operands)     1 mul_f32            2 add_f32
//   3 rsq_f32                     4 fma_f32 (literal)  5 add_f64
//   6 fma_f64                     7 add_f64 + cvt_f32_f64 + add_f32
//   8 add_f64 + add_f32           9 13 fma_f32 + 1 rsq_f32 (independent)
//  10 the pair arithmetic without memory: per chain and iteration one
//     softened interaction (3 sub, 3 fma, rsq, 3 mul, 4 fma/add) against
//     register-resident source values that change every iteration
//  11 ds_read_b128 broadcast + 4 fma_f32
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

template <int OP, int ILP>
__global__ __launch_bounds__(1024) void mb_kernel(float *out, int iters, float seed) {
  __shared__ float4 tile[256];
  const float tf = 1e-7f * static_cast<float>(threadIdx.x);
  float a[ILP], y[ILP], ax[ILP], ay[ILP], az[ILP], ap[ILP];
  double d[ILP];
#pragma unroll
  for (int k = 0; k < ILP; ++k) {
    a[k] = seed + tf + 0.01f * k;
    y[k] = 1.5f + 0.01f * k + tf;
    d[k] = static_cast<double>(a[k]);
    ax[k] = ay[k] = az[k] = ap[k] = 0.f;
  }
  // Runtime values, so the compiler cannot fold them into literals.
  const float b = 0.9999999f + tf * 1e-3f, c = 1e-7f + tf * 1e-9f;
  if constexpr (OP == 11) {
    tile[threadIdx.x & 255] = make_float4(a[0], b, c, 1.0f);
    __syncthreads();
  }
  float sx = 0.1f + tf, sy = 0.2f, sz = -0.3f, sm = 1e-3f, e2 = 1e-4f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < ILP; ++k) {
      if constexpr (OP == 0) {
        a[k] = fmaf(a[k], b, c);
      } else if constexpr (OP == 1) {
        a[k] = a[k] * b;
      } else if constexpr (OP == 2) {
        a[k] = a[k] + c;
      } else if constexpr (OP == 3) {
        y[k] = rsq(y[k]);
      } else if constexpr (OP == 4) {
        a[k] = fmaf(a[k], 0.9999999f, 1e-7f);
      } else if constexpr (OP == 5) {
        d[k] = d[k] + 1e-12;
      } else if constexpr (OP == 6) {
        d[k] = fma(d[k], 0.99999999999, 1e-12);
      } else if constexpr (OP == 7) {
        d[k] = d[k] + 1e-12;
        a[k] = a[k] + static_cast<float>(d[k]);
      } else if constexpr (OP == 8) {
        d[k] = d[k] + 1e-12;
        a[k] = a[k] + c;
      } else if constexpr (OP == 9) {
        y[k] = rsq(y[k]);
#pragma unroll
        for (int r = 0; r < 13; ++r) a[k] = fmaf(a[k], b, c);
      } else if constexpr (OP == 10) {
        const float dx = sx - a[k], dy = sy - y[k], dz = sz - a[k];
        float r2 = fmaf(dx, dx, e2);
        r2 = fmaf(dy, dy, r2);
        r2 = fmaf(dz, dz, r2);
        const float rho = rsq(r2);
        const float mr = sm * rho;
        const float s = mr * (rho * rho);
        ax[k] = fmaf(s, dx, ax[k]);
        ay[k] = fmaf(s, dy, ay[k]);
        az[k] = fmaf(s, dz, az[k]);
        ap[k] += mr;
      } else if constexpr (OP == 11) {
        const float4 t = tile[(it * ILP + k) & 255];
        a[k] = fmaf(a[k], t.y, t.z);
        a[k] = fmaf(a[k], t.w, t.x);
        a[k] = fmaf(a[k], b, c);
        a[k] = fmaf(a[k], b, c);
      }
    }
    if constexpr (OP == 10) {
      // a new source every iteration (wave-uniform, as an LDS broadcast is)
      sx = sx * 0.999f + 1e-3f;
      sy = sy * 0.999f - 1e-3f;
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < ILP; ++k)
    s += a[k] + y[k] + static_cast<float>(d[k]) + ax[k] + ay[k] + az[k] + ap[k];
  out[static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

template <int OP, int ILP>
hipError_t launch(float *out, int blocks, int threads, int iters) {
  mb_kernel<OP, ILP><<<blocks, threads, 0, nullptr>>>(out, iters, 1.0f);
  return hipGetLastError();
}

template <int ILP>
hipError_t launch_op(int op, float *out, int blocks, int threads, int iters) {
  switch (op) {
    case 0: return launch<0, ILP>(out, blocks, threads, iters);
    case 1: return launch<1, ILP>(out, blocks, threads, iters);
    case 2: return launch<2, ILP>(out, blocks, threads, iters);
    case 3: return launch<3, ILP>(out, blocks, threads, iters);
    case 4: return launch<4, ILP>(out, blocks, threads, iters);
    case 5: return launch<5, ILP>(out, blocks, threads, iters);
    case 6: return launch<6, ILP>(out, blocks, threads, iters);
    case 7: return launch<7, ILP>(out, blocks, threads, iters);
    case 8: return launch<8, ILP>(out, blocks, threads, iters);
    case 9: return launch<9, ILP>(out, blocks, threads, iters);
    case 10: return launch<10, ILP>(out, blocks, threads, iters);
    default: return launch<11, ILP>(out, blocks, threads, iters);
  }
}

}  // namespace

extern "C" {

// Runs operation `op` with `ilp` chains per lane (1, 2, 4, 8 or 16) on
// `blocks` x `threads` (threads a multiple of 64, at most 1024) for `iters`
// iterations; returns the median duration in ms of `reps` timed launches
// after one warm-up. out: device buffer of blocks * threads floats.
// Returns 0 on success, -1 on bad arguments, else the HIP error code.
int mb_run(int op, int ilp, float *out, int blocks, int threads, int iters, int reps,
           double *ms_out) {
  if (op < 0 || op > 11 || reps < 1 || reps > 64 || !out || !ms_out || blocks < 1 ||
      threads < 64 || threads > 1024 || threads % 64 != 0 || iters < 1)
    return -1;
  if (ilp != 1 && ilp != 2 && ilp != 4 && ilp != 8 && ilp != 16) return -1;
  hipEvent_t a, b;
  hipError_t e = hipEventCreate(&a);
  if (e != hipSuccess) return static_cast<int>(e);
  e = hipEventCreate(&b);
  if (e != hipSuccess) return static_cast<int>(e);
  auto go = [&]() -> hipError_t {
    switch (ilp) {
      case 1: return launch_op<1>(op, out, blocks, threads, iters);
      case 2: return launch_op<2>(op, out, blocks, threads, iters);
      case 4: return launch_op<4>(op, out, blocks, threads, iters);
      case 8: return launch_op<8>(op, out, blocks, threads, iters);
      default: return launch_op<16>(op, out, blocks, threads, iters);
    }
  };
  double t[64];
  e = go();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipEventRecord(a, nullptr);
    if (e == hipSuccess) e = go();
    if (e == hipSuccess) e = hipEventRecord(b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    t[r] = ms;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return static_cast<int>(e);
  for (int i = 1; i < reps; ++i)
    for (int j = i; j > 0 && t[j - 1] > t[j]; --j) {
      const double x = t[j];
      t[j] = t[j - 1];
      t[j - 1] = x;
    }
  *ms_out = t[reps / 2];
  return 0;
}

}  // extern "C"
