// Internal interface between the C ABI (abi.cpp) and the HIP kernels
// (kernels*.hip). Not installed; the public contract is include/nbody.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace nb {

constexpr int kDiagLen = 16;
constexpr int kMaxSplit = 32;         // largest grid-level j-split
constexpr int64_t kPartCap = int64_t{1} << 24;  // most split partial entries kept (force)
constexpr int64_t kJerkPartCap = int64_t{1} << 23;  // the same for acceleration + jerk
constexpr int kPad = 64;              // packed arrays are padded to a multiple of this
constexpr int kDiagBlocks = 512;      // blocks of the first diagnostics pass
constexpr int kDiagThreads = 256;

// One compiled pair-kernel configuration.
struct PairCfg {
  int block;  // threads per block (multiple of 64)
  int k;      // i-particles per thread (register blocking)
  int ls;     // lanes sharing one i (intra-wave j-split, combined by shuffles)
  int sw;     // waves sharing one i-group (inter-wave j-split, combined in LDS)
  int tile;   // j-particles per tile (LDS-staged, or per wave for the scalar stream)
  int smem;   // 0: j-tiles staged in LDS; 1 (2): j streamed by scalar loads into
              // SGPRs in groups of 4 (8); 3: near/far kernel on the spatial order
              // (compensated form only); 4: near/far with the block frame stored
              // by the ordering pass, held to 6 waves per SIMD; 5: near/far on
              // half box groups (128 targets per block), likewise
};

// Largest grid j-split the workspace holds for n particles.
inline int max_split(int64_t n) {
  if (n <= 0) return 1;
  int64_t s = kPartCap / n;
  if (s > kMaxSplit) s = kMaxSplit;
  return s < 1 ? 1 : static_cast<int>(s);
}
__host__ __device__ inline int64_t padded(int64_t n) { return (n + kPad - 1) / kPad * kPad; }

// i-particles one block covers for an item.
inline int cfg_iblock(const PairCfg &c) { return (c.block / 64 / c.sw) * (64 / c.ls) * c.k; }

// Table of compiled single-system configurations. The near/far ones (smem 3
// and 4) come last and exist for the compensated form only.
int single_cfg_count();
int single_cfg_count(bool comp);
const PairCfg &single_cfg(int idx);

// Batched modes compiled into the persistent kernel.
int batched_mode_count();
const PairCfg &batched_mode(int idx);

// Work item of the batched kernel: i in [i0, i1) against j in [j0, j1)
// (particle indices); the cluster's sources sit at slots [j0 + delta, ...) of
// the plan's slot layout, zero-padded to a multiple of kSlotAlign.
struct Item {
  int32_t i0, i1, j0, j1;
  int32_t cluster;  // index into the per-cluster eps array
  int32_t mode;     // batched_mode index
  int32_t delta;    // slot of particle j0 minus j0
  int32_t pad;
};
constexpr int kSlotAlign = 16;
constexpr int kBatchedModes = 9;

// Device arrays of a batched plan used by one force evaluation. Items are
// grouped by mode; mode m owns items [seg_begin[m], seg_end[m]) and runs as
// its own persistent launch of grid[m] blocks.
struct BatchedArgs {
  const Item *items;
  int32_t n_items;
  int32_t seg_begin[kBatchedModes];
  int32_t seg_end[kBatchedModes];
  int grid[kBatchedModes];
  const double *eps_k;
  const int32_t *slot_src;    // [n_slots] particle index of a slot, -1 for padding
  const int32_t *slot_frame;  // [n_slots] particle index of the slot's cluster frame
  int64_t n_slots;
  bool comp;
  bool need_pack;  // plain form, or any scalar-stream mode
};

// Launchers. All enqueue on `stream` and return the launch status.
// Plain pack: packed[j] = {x, y, z, m} in FP32 for j < n, zeros up to
// padded(n). Compensated pack (ds = true): packed[2j] = {hi(x-c), hi(y-c),
// hi(z-c), m}, packed[2j+1] = {lo(x-c), lo(y-c), lo(z-c), 0} with the frame
// c = pos[0], zeros up to padded(n).
hipError_t launch_pack(const double *pos, const double *mass, int64_t n, float4 *packed,
                       hipStream_t stream, bool ds = false);

// Single system: accelerations (and potentials) of all n particles.
// `part` must hold split * n * (comp ? 2 : 1) float4 when split > 1. If
// `after_pair` is non-null it is recorded right after the pair kernel (before
// the split combine), for measurement.
hipError_t launch_pair_single(int cfg, bool comp, const double *pos, const double *mass,
                              const float4 *packed, int64_t n, double eps, double G, int split,
                              double *acc, double *pot, float4 *part, hipStream_t stream,
                              hipEvent_t after_pair = nullptr);

// Batched persistent kernel over a work list. `packed` holds the slot-layout
// sources (n_slots x (comp ? 2 : 1) float4), written here when b.need_pack;
// `counters` holds kBatchedModes ints reset by a fill kernel first.
hipError_t launch_pair_batched(const BatchedArgs &b, const double *pos, const double *mass,
                               float4 *packed, double G, int *counters, double *acc, double *pot,
                               hipStream_t stream);
int batched_grid(bool comp, int mode);  // persistent grid (blocks) for the current device

// Spatial order (kernels_order.hip) and the near/far compensated pair kernel
// (kernels_nf.hip). order_ws_at lays out the ordering buffers in a workspace
// region at `base` (nullptr: sizes only, in .bytes).
constexpr int kOrderGroup = 256;  // particles per bounding-box group (= nf tile)
struct OrderWs {
  size_t bytes;
  double *moments;          // [256][6] partial moments
  uint32_t *key0, *key1;    // [n] Morton keys (ping-pong)
  int32_t *perm, *idx1;     // [n] ordered index -> caller's index (ping-pong)
  uint32_t *hist, *scan;    // digit histograms and their scan's block totals
  double *spos, *smass;     // [n][3], [n] in the order
  double *box;              // [ceil(n / kOrderGroup)][6] min xyz, max xyz
  double *bfr;              // [ceil(n / kOrderGroup)][4] box centre, (diagonal / 4)^2
  double *hbox;             // [2 ceil(n / kOrderGroup)][10] half groups: min, max, centre, (D / 4)^2
};
OrderWs order_ws_at(void *base, int64_t n);
hipError_t launch_order(const double *pos, const double *mass, int64_t n, const OrderWs &w,
                        hipStream_t stream);
// (k targets per lane, sw waves per target group) in {(2,1), (4,1), (4,4),
// (4,2), (2,2)} with the frame computed (fr 0); fr 1 (stored frame of a box
// group, 6 waves per SIMD) for (2,2), fr 2 (stored frame of a half group,
// 6 waves per SIMD) for (2,4). Writes acc/pot at the caller's indices.
hipError_t launch_pair_nf(int k, int sw, int fr, const OrderWs &w, int64_t n, double eps,
                          double G, int split, double *acc, double *pot, float4 *part,
                          hipStream_t stream, hipEvent_t after_pair = nullptr);

// Acceleration + jerk (kernels_jerk.hip). Packed sources hold 2 (plain) or
// 3 (compensated) float4 per particle, padded(n) particles; partials hold
// split x n x (2 or 4) float4.
// Compiled kernel shapes: cfg in [0, jerk_shape_count(comp)); K targets per
// lane and SW waves splitting the sources of a target group. The near/far
// shapes (jerk_shape_nf) exist for the compensated form only and run on the
// spatial order (launch_order, launch_gather_vel, launch_pair_nf_jerk with
// (k, sw) = (1, 1) or (2, 2) on whole box groups, (1, 2) on half groups).
int jerk_shape_count();
int jerk_shape_count(bool comp);
bool jerk_shape_nf(int cfg);
hipError_t launch_gather_vel(const double *vel, const OrderWs &w, int64_t n, double *svel,
                             hipStream_t stream);
hipError_t launch_pair_nf_jerk(int k, int sw, const OrderWs &w, const double *svel, int64_t n,
                               double eps, double G, int split, double *acc, double *jerk,
                               double *pot, float4 *part, hipStream_t stream,
                               hipEvent_t after_pair = nullptr);
void jerk_shape(int cfg, int *k, int *sw);
int jerk_targets_per_block(int cfg);
int jerk_default_split(int64_t n, int cfg);
hipError_t launch_pack_jerk(const double *pos, const double *vel, const double *mass, int64_t n,
                            bool comp, float4 *packed, hipStream_t stream);
hipError_t launch_pair_jerk(int cfg, bool comp, const float4 *packed, const double *mass, int64_t n,
                            double eps, double G, int split, double *acc, double *jerk,
                            double *pot, float4 *part, hipStream_t stream,
                            hipEvent_t after_pair = nullptr);
hipError_t launch_hermite_predict(const double *pos, const double *vel, const double *acc,
                                  const double *jerk, int64_t n, double dt, double *xp,
                                  double *vp, hipStream_t stream);
hipError_t launch_hermite_correct(double *pos, double *vel, double *acc, double *jerk,
                                  const double *a1, const double *j1, int64_t n, double dt,
                                  hipStream_t stream);

// FP64 integrator and diagnostics.
hipError_t launch_kick_drift(double *pos, double *vel, const double *acc, int64_t n, double h,
                             double dt, hipStream_t stream);
hipError_t launch_kick(double *vel, const double *acc, int64_t n, double h, hipStream_t stream);
// Kick fused with the first diagnostics pass (per-block partial rows).
hipError_t launch_kick_diag(const double *pos, double *vel, const double *acc, const double *pot,
                            const double *mass, int64_t n, double h, double *partial,
                            hipStream_t stream);
// Second pass: sums the partial rows in a fixed order into diag[*step_ctr],
// then increments *step_ctr.
hipError_t launch_diag_final(const double *partial, double *diag, int *step_ctr,
                             hipStream_t stream);
hipError_t launch_fill_int(int *p, int n, int value, hipStream_t stream);

// Single-system force evaluation behind nbody_accel (abi.cpp), with the grid
// j-split capped at split_cap (the workspace then needs accel_ws_bytes(n,
// variant, split_cap) bytes). Returns an nbody_status and sets the thread's
// last-error text.
int32_t accel_entry(const double *pos, const double *mass, int64_t n, double eps, double G,
                    int32_t variant, double *acc, double *pot, void *ws, size_t ws_bytes,
                    int split_cap, void *stream);
// Host-only checks of nbody_accel's arguments (everything but the workspace).
int32_t check_accel_args(const double *pos, const double *mass, int64_t n, double eps, double G,
                         int32_t variant, const double *acc, const double *pot);
size_t accel_ws_bytes(int64_t n, int32_t variant, int split_cap);
int accel_tuned_split(int32_t variant, int64_t n);  // the split nbody_accel would use
int32_t set_error(int32_t status, const char *msg);  // records msg, returns status

}  // namespace nb
