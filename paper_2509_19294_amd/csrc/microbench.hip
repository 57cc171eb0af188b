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
//  12 symmetric pair arithmetic with lane rotation: each lane holds ILP
//     targets and one source; 16 steps per iteration read the source through
//     a DPP row rotation (free on VOP2 instructions) and add the source-side
//     contribution back through the inverse rotation; one evaluation serves
//     two interactions
//  13 the pair arithmetic with the accumulation moved to the matrix cores:
//     per chain and iteration 3 sub, 3 fma, rsq and 2 mul on the VALU, then
//     two v_mfma_f32_4x4x1_16b_f32 (sixteen 4x4 outer products: the
//     sources' mass-weighted coordinates times r^-3, and masses times r^-1)
//     in place of the 3 fma + 1 add into the accumulators; sources differ
//     per lane, as that lane layout needs
//  14-19 operand placement and co-issue (mb_asm_kernel): sixteen
//     independent accumulations per lane written in inline asm with fixed
//     registers (a VGPR's bank is its index mod 4; every case uses v0-v71, so
//     occupancy is the same):
//     14 v_fmac_f32 acc, a, b with acc, a, b in three different banks
//     15 the same with acc, a, b all in bank 0
//     16 v_fmac_f32 acc, s, b: an SGPR operand in every instruction
//     17 one instruction in four with an SGPR operand, the rest as 14
//     18 v_sub_f32 acc, s, acc: an SGPR operand in every instruction (VOP2)
//     19 two v_rsq_f32 (chains of their own) among sixteen v_fmac_f32 as in 14
//     20 four softened pairs per iteration with hand-placed registers
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

template <int CTRL>
__device__ __forceinline__ float dppf(float x) {
  if constexpr (CTRL == 0) return x;
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, true));
}

// One rotation step r: targets (per lane) against the source r lanes away
// within the row; the source-side sums go back through the inverse rotation.
template <int ILP, int R>
__device__ __forceinline__ void rot_step(float (&tx)[ILP], float (&ty)[ILP], float (&tz)[ILP],
                                         float (&tm)[ILP], float (&ax)[ILP], float (&ay)[ILP],
                                         float (&az)[ILP], float (&ap)[ILP], float sx, float sy,
                                         float sz, float sm, float &bx, float &by, float &bz,
                                         float &bp, float e2) {
  constexpr int FWD = R == 0 ? 0 : 0x120 + R;          // row_ror:R
  constexpr int BWD = R == 0 ? 0 : 0x120 + (16 - R);   // row_ror:16-R
  const float xs = dppf<FWD>(sx), ys = dppf<FWD>(sy), zs = dppf<FWD>(sz), ms = dppf<FWD>(sm);
  float c0 = 0.f, c1 = 0.f, c2 = 0.f, c3 = 0.f;
#pragma unroll
  for (int k = 0; k < ILP; ++k) {
    const float dx = xs - tx[k], dy = ys - ty[k], dz = zs - tz[k];
    float r2 = fmaf(dx, dx, e2);
    r2 = fmaf(dy, dy, r2);
    r2 = fmaf(dz, dz, r2);
    const float rho = rsq(r2);
    const float rho2 = rho * rho;
    const float mr = ms * rho;
    const float si = mr * rho2;
    ax[k] = fmaf(si, dx, ax[k]);
    ay[k] = fmaf(si, dy, ay[k]);
    az[k] = fmaf(si, dz, az[k]);
    ap[k] += mr;
    const float mj = tm[k] * rho;
    const float sj = mj * rho2;
    c0 = fmaf(-sj, dx, c0);
    c1 = fmaf(-sj, dy, c1);
    c2 = fmaf(-sj, dz, c2);
    c3 += mj;
  }
  bx += dppf<BWD>(c0);
  by += dppf<BWD>(c1);
  bz += dppf<BWD>(c2);
  bp += dppf<BWD>(c3);
}

template <int OP, int ILP>
__global__ __launch_bounds__(1024) void mb_kernel(float *out, int iters, float seed) {
  __shared__ float4 tile[256];
  const float tf = 1e-7f * static_cast<float>(threadIdx.x);
  float a[ILP], y[ILP], ax[ILP], ay[ILP], az[ILP], ap[ILP];
  f4 mD[ILP], mP[ILP];
  double d[ILP];
#pragma unroll
  for (int k = 0; k < ILP; ++k) {
    a[k] = seed + tf + 0.01f * k;
    y[k] = 1.5f + 0.01f * k + tf;
    d[k] = static_cast<double>(a[k]);
    ax[k] = ay[k] = az[k] = ap[k] = 0.f;
    mD[k] = f4{0.f, 0.f, 0.f, 0.f};
    mP[k] = f4{0.f, 0.f, 0.f, 0.f};
  }
  // Runtime values, so the compiler cannot fold them into literals.
  const float b = 0.9999999f + tf * 1e-3f, c = 1e-7f + tf * 1e-9f;
  if constexpr (OP == 11) {
    tile[threadIdx.x & 255] = make_float4(a[0], b, c, 1.0f);
    __syncthreads();
  }
  float sx = 0.1f + tf, sy = 0.2f, sz = -0.3f, sm = 1e-3f, e2 = 1e-4f;
  float bq = 0.7f + tf;  // per-lane matrix operand (OP 13)
  float d2[4] = {0.f, 0.f, 0.f, 0.f};
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
      } else if constexpr (OP == 13) {
        const float dx = sx - a[k], dy = sy - y[k], dz = sz - a[k];
        float r2 = fmaf(dx, dx, e2);
        r2 = fmaf(dy, dy, r2);
        r2 = fmaf(dz, dz, r2);
        const float rho = rsq(r2);
        const float r3 = rho * (rho * rho);
        mD[k] = __builtin_amdgcn_mfma_f32_4x4x1f32(r3, bq, mD[k], 0, 0, 0);
        mP[k] = __builtin_amdgcn_mfma_f32_4x4x1f32(rho, sm, mP[k], 0, 0, 0);
      } else if constexpr (OP == 12) {
        // handled below, once per iteration
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
    if constexpr (OP == 13) {
      // a new source every iteration (per lane)
      sx = sx * 0.999f + 1e-3f;
      sy = sy * 0.999f - 1e-3f;
      bq = bq * 0.999f + 1e-4f;
    }
    if constexpr (OP == 12) {
      float tz[ILP], tm[ILP];
#pragma unroll
      for (int k = 0; k < ILP; ++k) {
        tz[k] = a[k] * 0.5f;
        tm[k] = 1e-3f;
      }
      rot_step<ILP, 0>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 1>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 2>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 3>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 4>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 5>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 6>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 7>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 8>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 9>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 10>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 11>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 12>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 13>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 14>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      rot_step<ILP, 15>(a, y, tz, tm, ax, ay, az, ap, sx, sy, sz, sm, d2[0], d2[1], d2[2], d2[3], e2);
      sx = sx * 0.999f + 1e-3f;
      sy = sy * 0.999f - 1e-3f;
      sz = sz * 0.999f + 2e-3f;
      sm = sm * 0.9999f;
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < ILP; ++k)
    s += a[k] + y[k] + static_cast<float>(d[k]) + ax[k] + ay[k] + az[k] + ap[k] + mD[k][0] +
         mD[k][1] + mD[k][2] + mD[k][3] + mP[k][0] + mP[k][1] + mP[k][2] + mP[k][3];
  s += d2[0] + d2[1] + d2[2] + d2[3];
  out[static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

// Operand-placement cases (14-19): ALU-only asm loops, 16 instructions per
// iteration (18 for case 19), on fixed registers v0-v71 and s90-s91.
#define MB_F3(d) "v_fmac_f32_e32 " d ", v65, v70\n"   // banks: d (0), 1, 2
#define MB_F1(d) "v_fmac_f32_e32 " d ", v64, v68\n"   // banks: d (0), 0, 0
#define MB_FS(d) "v_fmac_f32_e32 " d ", s91, v65\n"   // an SGPR operand
#define MB_SS(d) "v_sub_f32_e32 " d ", s91, " d "\n"   // VOP2 with an SGPR
#define MB_RQ(d) "v_rsq_f32_e32 " d ", " d "\n"
#define MB_16(F) F("v0") F("v4") F("v8") F("v12") F("v16") F("v20") F("v24") F("v28") \
  F("v32") F("v36") F("v40") F("v44") F("v48") F("v52") F("v56") F("v60")
#define MB_INIT(F) F("v0") F("v4") F("v8") F("v12") F("v16") F("v20") F("v24") F("v28") \
  F("v32") F("v36") F("v40") F("v44") F("v48") F("v52") F("v56") F("v60")
#define MB_ONE(d) "v_mov_b32 " d ", 1.0\n"
#define MB_LOOP(BODY)                                                                         \
  asm volatile(MB_INIT(MB_ONE) "v_mov_b32 v1, 2.0\n v_mov_b32 v37, 2.0\n"                    \
               "v_mov_b32 v41, 0.25\n v_mov_b32 v42, -0.5\n v_mov_b32 v43, 0.5\n"               \
               "v_mov_b32 v45, -0.25\n v_mov_b32 v46, 0.5\n v_mov_b32 v47, 0.5\n"               \
               "v_mov_b32 v49, 0.5\n v_mov_b32 v50, -1.0\n v_mov_b32 v53, -1.0\n"               \
               "v_mov_b32 v54, 0.5\n v_mov_b32 v57, 0\n v_mov_b32 v58, 0\n v_mov_b32 v59, 0\n" \
               "v_mov_b32 v61, 0\n v_mov_b32 v62, 0\n v_mov_b32 v63, 0\n"                      \
               "v_mov_b32 v64, 0.5\n v_mov_b32 v65, 0.5\n"                                   \
               "v_mov_b32 v68, 0.25\n v_mov_b32 v70, 0.25\n s_mov_b32 s91, 0.5\n"            \
               "s_mov_b32 s90, %1\n"                                                          \
               "1:\n" BODY "s_sub_u32 s90, s90, 1\n s_cmp_lg_u32 s90, 0\n s_cbranch_scc1 1b\n" \
               "v_mov_b32 %0, v0\n"                                                           \
               : "=v"(r)                                                                     \
               : "s"(iters)                                                                  \
               : "s90", "s91", "scc", "v0", "v1", "v2", "v3", "v4", "v5", "v6", "v7", "v8",  \
                 "v9", "v10", "v11", "v12", "v13", "v14", "v15", "v16", "v17", "v18", "v19",   \
                 "v20", "v21", "v22", "v23", "v24", "v25", "v26", "v27", "v28", "v29", "v30",  \
                 "v31", "v32", "v33", "v34", "v35", "v36", "v37", "v38", "v39", "v40", "v41",  \
                 "v42", "v43", "v44", "v45", "v46", "v47", "v48", "v49", "v50", "v51", "v52",  \
                 "v53", "v54", "v55", "v56", "v57", "v58", "v59", "v60", "v61", "v62", "v63",  \
                 "v64", "v65", "v66", "v67", "v68", "v69", "v70", "v71")

// Case 20: four softened pairs (two register-resident sources, two targets,
// the two targets' instruction streams interleaved) with every temporary
// placed by hand: separations in banks 0-2, r^-3 m in bank 3, so no
// instruction reads three operands from one bank; sources v40-v47, targets
// v48-v54, accumulators v56-v63, softening^2 in s91.
#define MB_PAIR4 \
  "v_sub_f32_e32 v0, v40, v48\n" \
  "v_sub_f32_e32 v8, v40, v52\n" \
  "v_sub_f32_e32 v1, v41, v49\n" \
  "v_sub_f32_e32 v9, v41, v53\n" \
  "v_sub_f32_e32 v2, v42, v50\n" \
  "v_sub_f32_e32 v10, v42, v54\n" \
  "v_fma_f32 v4, v0, v0, s91\n" \
  "v_fma_f32 v12, v8, v8, s91\n" \
  "v_fmac_f32_e32 v4, v1, v1\n" \
  "v_fmac_f32_e32 v12, v9, v9\n" \
  "v_fmac_f32_e32 v4, v2, v2\n" \
  "v_fmac_f32_e32 v12, v10, v10\n" \
  "v_rsq_f32_e32 v4, v4\n" \
  "v_rsq_f32_e32 v12, v12\n" \
  "s_nop 0\n" \
  "s_nop 0\n" \
  "v_mul_f32_e32 v5, v43, v4\n" \
  "v_mul_f32_e32 v13, v43, v12\n" \
  "v_mul_f32_e32 v6, v4, v4\n" \
  "v_mul_f32_e32 v14, v12, v12\n" \
  "v_mul_f32_e32 v3, v5, v6\n" \
  "v_mul_f32_e32 v11, v13, v14\n" \
  "v_fmac_f32_e32 v56, v3, v0\n" \
  "v_fmac_f32_e32 v60, v11, v8\n" \
  "v_fmac_f32_e32 v57, v3, v1\n" \
  "v_fmac_f32_e32 v61, v11, v9\n" \
  "v_fmac_f32_e32 v58, v3, v2\n" \
  "v_fmac_f32_e32 v62, v11, v10\n" \
  "v_add_f32_e32 v59, v59, v5\n" \
  "v_add_f32_e32 v63, v63, v13\n" \
  "v_sub_f32_e32 v0, v44, v48\n" \
  "v_sub_f32_e32 v8, v44, v52\n" \
  "v_sub_f32_e32 v1, v45, v49\n" \
  "v_sub_f32_e32 v9, v45, v53\n" \
  "v_sub_f32_e32 v2, v46, v50\n" \
  "v_sub_f32_e32 v10, v46, v54\n" \
  "v_fma_f32 v4, v0, v0, s91\n" \
  "v_fma_f32 v12, v8, v8, s91\n" \
  "v_fmac_f32_e32 v4, v1, v1\n" \
  "v_fmac_f32_e32 v12, v9, v9\n" \
  "v_fmac_f32_e32 v4, v2, v2\n" \
  "v_fmac_f32_e32 v12, v10, v10\n" \
  "v_rsq_f32_e32 v4, v4\n" \
  "v_rsq_f32_e32 v12, v12\n" \
  "s_nop 0\n" \
  "s_nop 0\n" \
  "v_mul_f32_e32 v5, v47, v4\n" \
  "v_mul_f32_e32 v13, v47, v12\n" \
  "v_mul_f32_e32 v6, v4, v4\n" \
  "v_mul_f32_e32 v14, v12, v12\n" \
  "v_mul_f32_e32 v3, v5, v6\n" \
  "v_mul_f32_e32 v11, v13, v14\n" \
  "v_fmac_f32_e32 v56, v3, v0\n" \
  "v_fmac_f32_e32 v60, v11, v8\n" \
  "v_fmac_f32_e32 v57, v3, v1\n" \
  "v_fmac_f32_e32 v61, v11, v9\n" \
  "v_fmac_f32_e32 v58, v3, v2\n" \
  "v_fmac_f32_e32 v62, v11, v10\n" \
  "v_add_f32_e32 v59, v59, v5\n" \
  "v_add_f32_e32 v63, v63, v13\n"

template <int OP>
__global__ __launch_bounds__(256) void mb_asm_kernel(float *out, int iters) {
  float r = 0.f;
  if constexpr (OP == 14) MB_LOOP(MB_16(MB_F3));
  if constexpr (OP == 15) MB_LOOP(MB_16(MB_F1));
  if constexpr (OP == 16) MB_LOOP(MB_16(MB_FS));
  if constexpr (OP == 17)
    MB_LOOP(MB_FS("v0") MB_F3("v4") MB_F3("v8") MB_F3("v12") MB_FS("v16") MB_F3("v20")
                MB_F3("v24") MB_F3("v28") MB_FS("v32") MB_F3("v36") MB_F3("v40") MB_F3("v44")
                    MB_FS("v48") MB_F3("v52") MB_F3("v56") MB_F3("v60"));
  if constexpr (OP == 18) MB_LOOP(MB_16(MB_SS));
  if constexpr (OP == 19)   // the two rsq chains (v1, v37) feed no accumulation
    MB_LOOP(MB_RQ("v1") MB_F3("v0") MB_F3("v4") MB_F3("v8") MB_F3("v12") MB_F3("v16")
                MB_F3("v20") MB_F3("v24") MB_F3("v28") MB_RQ("v37") MB_F3("v32") MB_F3("v36")
                    MB_F3("v40") MB_F3("v44") MB_F3("v48") MB_F3("v52") MB_F3("v56") MB_F3("v60"));
  if constexpr (OP == 20)
    MB_LOOP(MB_PAIR4);
  out[static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = r;
}

template <int OP, int ILP>
hipError_t launch(float *out, int blocks, int threads, int iters) {
  if constexpr (OP >= 14)
    mb_asm_kernel<OP><<<blocks, threads, 0, nullptr>>>(out, iters);
  else
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
    case 11: return launch<11, ILP>(out, blocks, threads, iters);
    case 12: return launch<12, ILP>(out, blocks, threads, iters);
    case 13: return launch<13, ILP>(out, blocks, threads, iters);
    case 14: return launch<14, ILP>(out, blocks, threads, iters);
    case 15: return launch<15, ILP>(out, blocks, threads, iters);
    case 16: return launch<16, ILP>(out, blocks, threads, iters);
    case 17: return launch<17, ILP>(out, blocks, threads, iters);
    case 18: return launch<18, ILP>(out, blocks, threads, iters);
    case 19: return launch<19, ILP>(out, blocks, threads, iters);
    default: return launch<20, ILP>(out, blocks, threads, iters);
  }
}

}  // namespace

extern "C" {

// Runs operation `op` with `ilp` chains per lane (1, 2, 4, 8 or 16; the asm
// cases 14-20 always run 16 and take 256 threads) on
// `blocks` x `threads` (threads a multiple of 64, at most 1024) for `iters`
// iterations; returns the median duration in ms of `reps` timed launches
// after one warm-up. out: device buffer of blocks * threads floats.
// Returns 0 on success, -1 on bad arguments, else the HIP error code.
int mb_run(int op, int ilp, float *out, int blocks, int threads, int iters, int reps,
           double *ms_out) {
  if (op < 0 || op > 20 || (op >= 14 && threads != 256) || reps < 1 || reps > 64 || !out || !ms_out || blocks < 1 ||
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
