// C ABI of libnbody.so (declared in include/nbody.h): host-side validation,
// workspace layout, tuning lookup, kernel dispatch, batched plans and their
// HIP graphs. Every device-side step runs in the kernels of csrc/kernels*.hip.
#include "nbody.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "nbody_internal.h"

namespace {

thread_local std::string g_err;

nbody_status fail(nbody_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

nbody_status hip_fail(hipError_t e, const char *what) {
  return fail(NBODY_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool valid_variant(int32_t v) { return v == NBODY_FP32_PLAIN || v == NBODY_FP32_COMP; }

size_t align_up(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Workspace layout (offsets in bytes from the base, each 256-byte aligned).
struct WsLayout {
  size_t packed, part, pot, diag, ctr, order, total;
};

// Packed sources: padded(n) entries for a single system; a batched plan's
// slot layout pads every cluster to a multiple of kSlotAlign.
int64_t packed_entries(int64_t n, int32_t n_clusters) {
  const int64_t single = nb::padded(n);
  if (n_clusters <= 1) return single;
  const int64_t slots = nb::padded(n + static_cast<int64_t>(nb::kSlotAlign) * n_clusters);
  return slots > single ? slots : single;
}

// `split_cap` bounds the grid j-splits the partial-sum region holds (the
// allocation-free entry point passes what its static scratch can take).
WsLayout ws_layout(int64_t n, int32_t variant, int32_t n_clusters = 1, int split_cap = nb::kMaxSplit) {
  WsLayout L{};
  const size_t un = static_cast<size_t>(n);
  const size_t jw = variant == NBODY_FP32_COMP ? 2 : 1;
  // (a batched plan's kernels write their results directly: no split partials)
  const int splits = n_clusters > 1 ? 0 : std::min(nb::max_split(n), std::max(split_cap, 1));
  size_t off = 0;
  L.packed = off;
  off += align_up(static_cast<size_t>(packed_entries(n, n_clusters)) * jw * sizeof(float4));
  L.part = off;
  off += align_up(static_cast<size_t>(splits) * un * jw * sizeof(float4));
  L.pot = off;
  off += align_up(un * sizeof(double));
  L.diag = off;
  off += align_up(static_cast<size_t>(nb::kDiagBlocks) * nb::kDiagLen * sizeof(double));
  L.ctr = off;
  off += 256;
  // spatial-order buffers of the near/far compensated kernel (single system)
  L.order = off;
  if (variant == NBODY_FP32_COMP && n_clusters <= 1 && n > 0) off += align_up(nb::order_ws_at(nullptr, n).bytes);
  L.total = off;
  return L;
}

template <typename T>
T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

bool overlap(const void *a, size_t na, const void *b, size_t nb_) {
  if (!a || !b || na == 0 || nb_ == 0) return false;
  const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
  return pa < pb + nb_ && pb < pa + na;
}

// ---------------------------------------------------------------------------
// Tuning: per variant and size class (floor(log2(n))), a single-system
// configuration index and grid j-split, and a batched mode.

constexpr int kClasses = 48;

struct SingleTune {
  int cfg;
  int split;
};

std::mutex g_tune_mu;
SingleTune g_single[2][kClasses];
bool g_tune_init = false;
int g_forced[2][kClasses];  // -1 = none

// Batched modes per variant and size class. The process-wide table is what a
// new plan starts from; a plan created with a tuning file keeps its own copy.
struct BatchedTable {
  int mode[2][kClasses];
};
BatchedTable g_batched;

int size_class(int64_t n) {
  int c = 0;
  while (c + 1 < kClasses && (int64_t{1} << (c + 1)) <= n) ++c;
  return c;
}

// Built-in table, measured on MI355X by paper_2509_19294_amd.autotune
// (Plummer spheres of 2^c particles, eps = 0.01): {cfg, split} per size class
// 10..20 for the plain and compensated forms; smaller classes take class 10's
// entry and larger ones class 20's (whose compensated split, 16, times equal
// to 8 and, with the near/far kernel's per-XCD block order, moves about a
// third of the HBM bytes). Batched modes for classes 8..13.
const SingleTune kTuned[2][11] = {
    {{5, 4}, {5, 8}, {5, 8}, {4, 8}, {15, 16}, {15, 16}, {15, 16}, {13, 16}, {13, 32}, {13, 8}, {15, 2}},
    {{5, 4}, {5, 8}, {4, 4}, {0, 16}, {15, 16}, {15, 32}, {15, 32}, {25, 32}, {25, 32}, {25, 8}, {24, 16}},
};
const int kTunedBatched[2][6] = {{8, 4, 4, 4, 4, 4}, {1, 4, 4, 4, 4, 4}};
// Acceleration + jerk kernel: {shape, split} per size class 10..20, measured
// on MI355X by the same autotuner (Plummer spheres of 2^c particles,
// eps = 0.01; split 0 would select the rule of jerk_default_split).
const SingleTune kTunedJerk[2][11] = {
    {{8, 1}, {8, 2}, {8, 4}, {2, 8}, {2, 16}, {2, 32}, {2, 32}, {2, 32}, {1, 32}, {0, 16}, {2, 2}},
    {{2, 1}, {2, 2}, {2, 4}, {2, 8}, {2, 16}, {12, 32}, {12, 32}, {12, 32}, {12, 32}, {12, 16}, {10, 8}},
};
SingleTune g_jerk[2][kClasses];
int g_jerk_forced[2] = {-1, -1};

void tune_defaults() {
  for (int v = 0; v < 2; ++v) {
    for (int c = 0; c < kClasses; ++c) {
      const int tc = c < 10 ? 0 : (c > 20 ? 10 : c - 10);
      g_single[v][c] = kTuned[v][tc];
      const int bc = c < 8 ? 0 : (c > 13 ? 5 : c - 8);
      g_batched.mode[v][c] = kTunedBatched[v][bc];
      g_forced[v][c] = -1;
      g_jerk[v][c] = kTunedJerk[v][tc];
    }
    g_jerk_forced[v] = -1;
  }
}

// Reads a tuning file. Lines: "single v class cfg split", "batched v class
// mode", "jerk v class shape split"; '#' starts a comment. With `only_batched`
// (a plan's own file) the single and jerk lines are checked but not applied.
// Nothing is applied unless the whole file parses.
nbody_status tune_parse(const char *path, BatchedTable &batched, bool only_batched) {
  FILE *f = std::fopen(path, "r");
  if (!f) return fail(NBODY_EINVAL, "cannot open tuning file '%s'", path);
  struct Entry {
    int kind, v, c, a, b;
  };
  std::vector<Entry> entries;
  char line[256];
  int lineno = 0;
  while (std::fgets(line, sizeof(line), f)) {
    ++lineno;
    char kind[32];
    int v, c, a, b = 1;
    if (line[0] == '#' || line[0] == '\n') continue;
    const int got = std::sscanf(line, "%31s %d %d %d %d", kind, &v, &c, &a, &b);
    if (got < 4 || v < 0 || v > 1 || c < 0 || c >= kClasses) {
      std::fclose(f);
      return fail(NBODY_EINVAL, "tuning file '%s' line %d malformed", path, lineno);
    }
    if (std::strcmp(kind, "single") == 0) {
      if (a < 0 || a >= nb::single_cfg_count(v == NBODY_FP32_COMP) || b < 1 || b > nb::kMaxSplit) {
        std::fclose(f);
        return fail(NBODY_EINVAL, "tuning file '%s' line %d: bad single entry", path, lineno);
      }
      entries.push_back({0, v, c, a, b});
    } else if (std::strcmp(kind, "batched") == 0) {
      if (a < 0 || a >= nb::batched_mode_count()) {
        std::fclose(f);
        return fail(NBODY_EINVAL, "tuning file '%s' line %d: bad batched entry", path, lineno);
      }
      entries.push_back({1, v, c, a, 0});
    } else if (std::strcmp(kind, "jerk") == 0) {
      if (a < 0 || a >= nb::jerk_shape_count(v == NBODY_FP32_COMP) || b < 0 || b > nb::kMaxSplit) {
        std::fclose(f);
        return fail(NBODY_EINVAL, "tuning file '%s' line %d: bad jerk entry", path, lineno);
      }
      entries.push_back({2, v, c, a, b});
    } else {
      std::fclose(f);
      return fail(NBODY_EINVAL, "tuning file '%s' line %d: unknown kind", path, lineno);
    }
  }
  std::fclose(f);
  for (const Entry &e : entries) {
    if (e.kind == 1)
      batched.mode[e.v][e.c] = e.a;
    else if (!only_batched && e.kind == 0)
      g_single[e.v][e.c] = SingleTune{e.a, e.b};
    else if (!only_batched && e.kind == 2)
      g_jerk[e.v][e.c] = SingleTune{e.a, e.b};
  }
  return NBODY_OK;
}

nbody_status tune_load_locked(const char *path) { return tune_parse(path, g_batched, false); }

void tune_init_locked() {
  if (g_tune_init) return;
  tune_defaults();
  g_tune_init = true;
  const char *env = std::getenv("NBODY_TUNE");
  if (env && *env) tune_load_locked(env);  // a bad file leaves the defaults
}

SingleTune single_tune(int32_t variant, int64_t n) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_init_locked();
  const int c = size_class(n);
  SingleTune t = g_single[variant][c];
  if (g_forced[variant][c] >= 0) {
    const int f = g_forced[variant][c];
    t = SingleTune{f % 1000, f / 1000 > 0 ? f / 1000 : 1};
  }
  return t;
}

// Shape and split of the acceleration + jerk kernel for n particles.
SingleTune jerk_tune(int32_t variant, int64_t n) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_init_locked();
  SingleTune t = g_jerk[variant][size_class(n)];
  if (g_jerk_forced[variant] >= 0) t = SingleTune{g_jerk_forced[variant] % 1000, g_jerk_forced[variant] / 1000};
  if (t.split <= 0) t.split = nb::jerk_default_split(n, t.cfg);
  // the partial buffer holds at most kJerkPartCap entries
  while (t.split > 1 && static_cast<int64_t>(t.split) * n > nb::kJerkPartCap) t.split /= 2;
  return t;
}

// The process-wide batched table (a new plan's starting point).
BatchedTable batched_table() {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_init_locked();
  return g_batched;
}

// ---------------------------------------------------------------------------
// Optional event brackets around force-kernel launches (measurement only).

struct Timing {
  bool on = false;
  std::vector<hipEvent_t> pool;  // pairs: start at 2k, stop at 2k + 1
  size_t used = 0;               // events recorded since the last read
};
Timing g_timing;
std::mutex g_timing_mu;  // guards g_timing (launches may come from several host threads)

bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
  return cs != hipStreamCaptureStatusNone;
}

hipEvent_t timing_event() {
  if (g_timing.used == g_timing.pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_timing.pool.push_back(e);
  }
  return g_timing.pool[g_timing.used++];
}

// Records the start event; returns the stop event to record after the launch
// (nullptr when timing is off or the stream is being captured).
hipEvent_t timing_begin(hipStream_t st) {
  std::lock_guard<std::mutex> g(g_timing_mu);
  if (!g_timing.on || capturing(st)) return nullptr;
  hipEvent_t a = timing_event();
  if (!a) return nullptr;
  hipEvent_t b = timing_event();
  if (!b) {
    --g_timing.used;
    return nullptr;
  }
  if (hipEventRecord(a, st) != hipSuccess) {
    g_timing.used -= 2;
    return nullptr;
  }
  return b;
}

void timing_end(hipEvent_t stop, hipStream_t st) {
  if (stop) (void)hipEventRecord(stop, st);
}

// ---------------------------------------------------------------------------
// Shared pieces of accel / step.

nbody_status check_scalars(double eps, double G) {
  if (!std::isfinite(eps) || eps < 0.0) return fail(NBODY_EINVAL, "eps must be finite and >= 0 (got %g)", eps);
  if (!std::isfinite(G)) return fail(NBODY_EINVAL, "G must be finite");
  return NBODY_OK;
}

nbody_status check_ws(void *ws, size_t ws_bytes, int64_t n, int32_t variant,
                      int32_t n_clusters = 1, int split_cap = nb::kMaxSplit) {
  const size_t need = ws_layout(n, variant, n_clusters, split_cap).total;
  if (!ws) return fail(NBODY_EWORKSPACE, "workspace is NULL (need %zu bytes)", need);
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(NBODY_EWORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < need) return fail(NBODY_EWORKSPACE, "workspace of %zu bytes < %zu required", ws_bytes, need);
  return NBODY_OK;
}

hipError_t enqueue_accel(const double *pos, const double *mass, int64_t n, double eps, double G,
                         int32_t variant, double *acc, double *pot, void *ws, hipStream_t st,
                         int split_cap = nb::kMaxSplit) {
  if (n <= 0) return hipSuccess;
  const WsLayout L = ws_layout(n, variant, 1, split_cap);
  SingleTune t = single_tune(variant, n);
  t.split = std::min(t.split, std::max(split_cap, 1));
  const bool comp = variant == NBODY_FP32_COMP;
  float4 *packed = at<float4>(ws, L.packed);
  // the spatial order indexes particles with 32-bit integers
  if (nb::single_cfg(t.cfg).smem >= 3 && n >= (int64_t{1} << 31)) t = SingleTune{9, t.split};
  if (nb::single_cfg(t.cfg).smem >= 3) {
    // near/far kernel on the spatial order (compensated form only)
    const nb::OrderWs w = nb::order_ws_at(at<char>(ws, L.order), n);
    const hipError_t e = nb::launch_order(pos, mass, n, w, st);
    if (e != hipSuccess) return e;
    hipEvent_t stop = timing_begin(st);
    const nb::PairCfg &c = nb::single_cfg(t.cfg);
    return nb::launch_pair_nf(c.k, c.sw, c.smem - 3, w, n, eps, G, t.split, acc, pot,
                              at<float4>(ws, L.part), st, stop);
  }
  const bool smem = nb::single_cfg(t.cfg).smem != 0;
  if (!comp || smem) {
    const hipError_t e = nb::launch_pack(pos, mass, n, packed, st, comp);
    if (e != hipSuccess) return e;
  }
  hipEvent_t stop = timing_begin(st);
  return nb::launch_pair_single(t.cfg, comp, pos, mass, packed, n, eps, G, t.split, acc, pot,
                                at<float4>(ws, L.part), st, stop);
}

// Workspace of the jerk / Hermite calls.
struct JerkLayout {
  size_t packed, part, xp, vp, a1, j1, pot, diag, ctr, order, svel, total;
};

// `split` is the grid j-split the call will launch with (resolved once per
// call, so a concurrent change of the tuning cannot outgrow the workspace).
JerkLayout jerk_layout(int64_t n, int32_t variant, int split) {
  JerkLayout L{};
  const size_t un = static_cast<size_t>(n);
  const bool comp = variant == NBODY_FP32_COMP;
  size_t off = 0;
  L.packed = off;
  off += align_up(static_cast<size_t>(nb::padded(n)) * (comp ? 3 : 2) * sizeof(float4));
  L.part = off;
  off += align_up(split > 1 ? static_cast<size_t>(split) * un * (comp ? 4 : 2) * sizeof(float4) : 0);
  L.xp = off;
  off += align_up(un * 3 * sizeof(double));
  L.vp = off;
  off += align_up(un * 3 * sizeof(double));
  L.a1 = off;
  off += align_up(un * 3 * sizeof(double));
  L.j1 = off;
  off += align_up(un * 3 * sizeof(double));
  L.pot = off;
  off += align_up(un * sizeof(double));
  L.diag = off;
  off += align_up(static_cast<size_t>(nb::kDiagBlocks) * nb::kDiagLen * sizeof(double));
  L.ctr = off;
  off += 256;
  // spatial order and ordered velocities of the near/far kernel
  L.order = off;
  L.svel = off;
  if (variant == NBODY_FP32_COMP && n > 0) {
    off += align_up(nb::order_ws_at(nullptr, n).bytes);
    L.svel = off;
    off += align_up(un * 3 * sizeof(double));
  }
  L.total = off;
  return L;
}

hipError_t enqueue_accel_jerk(const double *pos, const double *vel, const double *mass, int64_t n,
                              double eps, double G, int32_t variant, const SingleTune &t,
                              double *acc, double *jerk, double *pot, void *ws, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const JerkLayout L = jerk_layout(n, variant, t.split);
  const bool comp = variant == NBODY_FP32_COMP;
  if (nb::jerk_shape_nf(t.cfg) && comp && n < (int64_t{1} << 31)) {
    const nb::OrderWs w = nb::order_ws_at(at<char>(ws, L.order), n);
    hipError_t e = nb::launch_order(pos, mass, n, w, st);
    double *svel = at<double>(ws, L.svel);
    if (e == hipSuccess) e = nb::launch_gather_vel(vel, w, n, svel, st);
    if (e != hipSuccess) return e;
    int k = 0, sw = 0;
    nb::jerk_shape(t.cfg, &k, &sw);
    hipEvent_t stop = timing_begin(st);
    return nb::launch_pair_nf_jerk(k, sw, w, svel, n, eps, G, t.split, acc, jerk, pot,
                                   at<float4>(ws, L.part), st, stop);
  }
  const int cfg = nb::jerk_shape_nf(t.cfg) ? 2 : t.cfg;  // beyond 2^31 particles
  float4 *packed = at<float4>(ws, L.packed);
  hipError_t e = nb::launch_pack_jerk(pos, vel, mass, n, comp, packed, st);
  if (e != hipSuccess) return e;
  hipEvent_t stop = timing_begin(st);
  return nb::launch_pair_jerk(cfg, comp, packed, mass, n, eps, G, t.split, acc, jerk, pot,
                              at<float4>(ws, L.part), st, stop);
}

}  // namespace

// ---------------------------------------------------------------------------
// Batched plan.

struct nbody_plan {
  int32_t K = 0;
  int32_t variant = 0;
  int64_t n_total = 0;
  std::vector<int64_t> offsets;
  int32_t n_items = 0;
  double pairs = 0.0;
  nb::Item *d_items = nullptr;
  int32_t *d_slot_src = nullptr;    // slot layout of the packed sources
  int32_t *d_slot_frame = nullptr;
  int64_t n_slots = 0;
  bool need_pack = false;
  int32_t seg_begin[nb::kBatchedModes] = {};
  int32_t seg_end[nb::kBatchedModes] = {};
  int grid[nb::kBatchedModes] = {};
  int device = 0;
  // Cache of one captured KDK step and the arguments it was captured with.
  // It changes behind a const plan pointer (a cache, not part of the plan's
  // meaning), which is why calls sharing a plan must be ordered.
  mutable hipStream_t capture = nullptr;
  mutable hipGraphExec_t exec = nullptr;
  mutable const void *key[10] = {};
  mutable double key_g = 0, key_dt = 0;
};

namespace {

hipError_t enqueue_batched(const double *pos, const double *mass, const nbody_plan *p,
                           const double *eps_k, double G, double *acc, double *pot, void *ws,
                           hipStream_t st) {
  const WsLayout L = ws_layout(p->n_total, p->variant, p->K);
  nb::BatchedArgs b{};
  b.items = p->d_items;
  b.n_items = p->n_items;
  b.eps_k = eps_k;
  b.slot_src = p->d_slot_src;
  b.slot_frame = p->d_slot_frame;
  b.n_slots = p->n_slots;
  for (int m = 0; m < nb::kBatchedModes; ++m) {
    b.seg_begin[m] = p->seg_begin[m];
    b.seg_end[m] = p->seg_end[m];
    b.grid[m] = p->grid[m];
  }
  b.comp = p->variant == NBODY_FP32_COMP;
  b.need_pack = p->need_pack;
  hipEvent_t stop = timing_begin(st);
  const hipError_t e = nb::launch_pair_batched(b, pos, mass, at<float4>(ws, L.packed), G,
                                               at<int>(ws, L.ctr) + 4, acc, pot, st);
  timing_end(stop, st);
  return e;
}

// One KDK step: kick-drift, forces, kick (+ diagnostics row). `plan` NULL:
// a single system softened by eps; otherwise the plan's clusters softened by
// eps_k.
hipError_t enqueue_step(double *pos, double *vel, double *acc, double *pot, const double *mass,
                        int64_t n, double eps, double G, double dt, int32_t variant,
                        const nbody_plan *plan, const double *eps_k, double *diag, void *ws,
                        hipStream_t st) {
  const WsLayout L = ws_layout(n, variant, plan ? plan->K : 1);
  const double h = 0.5 * dt;
  hipError_t e = nb::launch_kick_drift(pos, vel, acc, n, h, dt, st);
  if (e != hipSuccess) return e;
  double *potw = pot ? pot : (diag ? at<double>(ws, L.pot) : nullptr);
  if (plan)
    e = enqueue_batched(pos, mass, plan, eps_k, G, acc, potw, ws, st);
  else
    e = enqueue_accel(pos, mass, n, eps, G, variant, acc, potw, ws, st);
  if (e != hipSuccess) return e;
  if (diag) {
    e = nb::launch_kick_diag(pos, vel, acc, potw, mass, n, h, at<double>(ws, L.diag), st);
    if (e != hipSuccess) return e;
    return nb::launch_diag_final(at<double>(ws, L.diag), diag, at<int>(ws, L.ctr), st);
  }
  return nb::launch_kick(vel, acc, n, h, st);
}

// Host checks of a batched call's plan, variant and per-cluster softenings.
nbody_status check_batched(const nbody_plan *plan, int32_t variant, const double *eps_k) {
  if (!plan) return fail(NBODY_EINVAL, "plan is NULL");
  if (!valid_variant(variant)) return fail(NBODY_ENOTSUP, "unknown variant %d", variant);
  if (variant != plan->variant)
    return fail(NBODY_EINVAL, "variant %d does not match the plan's %d", variant, plan->variant);
  if (plan->n_total > 0 && !eps_k) return fail(NBODY_EINVAL, "eps_k must be non-NULL");
  if (reinterpret_cast<uintptr_t>(eps_k) % alignof(double) != 0)
    return fail(NBODY_EINVAL, "eps_k must be 8-byte aligned");
  // the plan's device arrays (work list, slot layout) live on one device
  int dev = -1;
  if (hipGetDevice(&dev) == hipSuccess && dev != plan->device)
    return fail(NBODY_EINVAL, "the plan was created on device %d, the current device is %d", plan->device, dev);
  return NBODY_OK;
}

}  // namespace

namespace nb {

int32_t set_error(int32_t status, const char *msg) { return fail(status, "%s", msg); }

int32_t check_accel_args(const double *pos, const double *mass, int64_t n, double eps, double G,
                         int32_t variant, const double *acc, const double *pot) {
  g_err.clear();
  if (n < 0) return fail(NBODY_EINVAL, "n must be >= 0 (got %lld)", static_cast<long long>(n));
  if (!valid_variant(variant)) return fail(NBODY_ENOTSUP, "unknown variant %d", variant);
  nbody_status st = check_scalars(eps, G);
  if (st != NBODY_OK) return st;
  if (n == 0) return NBODY_OK;
  if (!pos || !mass || !acc) return fail(NBODY_EINVAL, "pos, mass and acc must be non-NULL");
  const size_t b3 = static_cast<size_t>(n) * 3 * sizeof(double), b1 = static_cast<size_t>(n) * sizeof(double);
  if (overlap(acc, b3, pos, b3) || overlap(acc, b3, mass, b1) || overlap(pot, b1, pos, b3) ||
      overlap(pot, b1, mass, b1) || overlap(pot, b1, acc, b3))
    return fail(NBODY_EINVAL, "output arrays overlap inputs or each other");
  return NBODY_OK;
}

size_t accel_ws_bytes(int64_t n, int32_t variant, int split_cap) {
  return ws_layout(n, variant, 1, split_cap).total;
}

int accel_tuned_split(int32_t variant, int64_t n) {
  return std::min(single_tune(variant, n).split, max_split(n));
}

int32_t accel_entry(const double *pos, const double *mass, int64_t n, double eps, double G,
                    int32_t variant, double *acc, double *pot, void *ws, size_t ws_bytes,
                    int split_cap, void *stream) {
  nbody_status st = check_accel_args(pos, mass, n, eps, G, variant, acc, pot);
  if (st != NBODY_OK || n == 0) return st;
  st = check_ws(ws, ws_bytes, n, variant, 1, split_cap);
  if (st != NBODY_OK) return st;
  const hipError_t e = enqueue_accel(pos, mass, n, eps, G, variant, acc, pot, ws,
                                     static_cast<hipStream_t>(stream), split_cap);
  if (e != hipSuccess) return hip_fail(e, "nbody_accel launch");
  return NBODY_OK;
}

}  // namespace nb

extern "C" {

const char *nbody_last_error(void) { return g_err.c_str(); }

const char *nbody_version(void) { return "nbody-mi355x 0.1 (gfx950)"; }

size_t nbody_workspace_bytes(int64_t n_total, int32_t n_clusters, int32_t variant) {
  if (n_total < 0 || n_clusters < 1 || !valid_variant(variant)) return 0;
  return ws_layout(n_total, variant, n_clusters).total;
}

nbody_status nbody_accel(const double *pos, const double *mass, int64_t n, double eps, double G,
                         int32_t variant, double *acc, double *pot, void *ws, size_t ws_bytes,
                         void *stream) {
  return nb::accel_entry(pos, mass, n, eps, G, variant, acc, pot, ws, ws_bytes, nb::kMaxSplit, stream);
}

nbody_plan *nbody_plan_create(const int64_t *offsets_host, int32_t K, int32_t variant,
                              const char *tune_path) {
  g_err.clear();
  if (!offsets_host) {
    fail(NBODY_EINVAL, "offsets must be non-NULL");
    return nullptr;
  }
  if (K < 1) {
    fail(NBODY_EINVAL, "K must be >= 1 (got %d)", K);
    return nullptr;
  }
  if (!valid_variant(variant)) {
    fail(NBODY_ENOTSUP, "unknown variant %d", variant);
    return nullptr;
  }
  if (offsets_host[0] != 0) {
    fail(NBODY_EINVAL, "offsets[0] must be 0");
    return nullptr;
  }
  for (int32_t k = 0; k < K; ++k) {
    if (offsets_host[k + 1] < offsets_host[k]) {
      fail(NBODY_EINVAL, "offsets must be non-decreasing (at %d)", k);
      return nullptr;
    }
  }
  if (offsets_host[K] + static_cast<int64_t>(nb::kSlotAlign) * K >= (int64_t{1} << 31)) {
    fail(NBODY_ENOTSUP, "batched plans hold fewer than 2^31 particles");
    return nullptr;
  }
  // The plan's own modes: the process-wide table, overridden by the batched
  // lines of tune_path (which leaves the process-wide tuning unchanged).
  BatchedTable modes = batched_table();
  if (tune_path && tune_parse(tune_path, modes, true) != NBODY_OK) return nullptr;

  nbody_plan *p = new nbody_plan();
  p->K = K;
  p->variant = variant;
  p->offsets.assign(offsets_host, offsets_host + K + 1);
  p->n_total = offsets_host[K];

  // Slot layout: cluster k's sources start at a multiple of kSlotAlign and
  // are followed by zero-mass padding up to the next multiple.
  std::vector<int64_t> poff(static_cast<size_t>(K) + 1, 0);
  for (int32_t k = 0; k < K; ++k) {
    const int64_t nk = p->offsets[k + 1] - p->offsets[k];
    poff[k + 1] = poff[k] + (nk + nb::kSlotAlign - 1) / nb::kSlotAlign * nb::kSlotAlign;
  }
  p->n_slots = poff[K];
  std::vector<int32_t> slot_src(static_cast<size_t>(p->n_slots), -1), slot_frame(static_cast<size_t>(p->n_slots), 0);
  for (int32_t k = 0; k < K; ++k) {
    const int64_t s = p->offsets[k], nk = p->offsets[k + 1] - s;
    for (int64_t t = 0; t < poff[k + 1] - poff[k]; ++t) {
      slot_src[poff[k] + t] = t < nk ? static_cast<int32_t>(s + t) : -1;
      slot_frame[poff[k] + t] = static_cast<int32_t>(nk > 0 ? s : 0);
    }
  }

  // Work items: every cluster cut into i-blocks of its mode's width; then
  // heaviest first (longest-processing-time order), ties by position.
  std::vector<nb::Item> items;
  p->need_pack = variant == NBODY_FP32_PLAIN;
  for (int32_t k = 0; k < K; ++k) {
    const int64_t s = p->offsets[k], e = p->offsets[k + 1], nk = e - s;
    if (nk == 0) continue;
    const int mode = modes.mode[variant][size_class(nk)];
    if (nb::batched_mode(mode).smem) p->need_pack = true;
    const int ib = nb::cfg_iblock(nb::batched_mode(mode));
    for (int64_t i = s; i < e; i += ib) {
      nb::Item it{};
      it.i0 = static_cast<int32_t>(i);
      it.i1 = static_cast<int32_t>(std::min<int64_t>(i + ib, e));
      it.j0 = static_cast<int32_t>(s);
      it.j1 = static_cast<int32_t>(e);
      it.cluster = k;
      it.mode = mode;
      it.delta = static_cast<int32_t>(poff[k] - s);
      items.push_back(it);
      p->pairs += static_cast<double>(it.i1 - it.i0) * static_cast<double>(nk);
    }
  }
  // Grouped by mode (one persistent launch each), heaviest first within a
  // mode; the stable sort keeps ties in position order.
  std::stable_sort(items.begin(), items.end(), [](const nb::Item &a, const nb::Item &b) {
    if (a.mode != b.mode) return a.mode < b.mode;
    const int64_t ca = int64_t{a.i1 - a.i0} * (a.j1 - a.j0);
    const int64_t cb = int64_t{b.i1 - b.i0} * (b.j1 - b.j0);
    return ca > cb;
  });
  p->n_items = static_cast<int32_t>(items.size());
  for (int32_t t = 0; t < p->n_items; ++t) {
    const int m = items[t].mode;
    if (p->seg_end[m] == p->seg_begin[m]) p->seg_begin[m] = t;
    p->seg_end[m] = t + 1;
  }

  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess && !items.empty()) e = hipMalloc(&p->d_items, items.size() * sizeof(nb::Item));
  if (e == hipSuccess && !items.empty())
    e = hipMemcpy(p->d_items, items.data(), items.size() * sizeof(nb::Item), hipMemcpyHostToDevice);
  if (e == hipSuccess && p->n_slots > 0) e = hipMalloc(&p->d_slot_src, slot_src.size() * sizeof(int32_t));
  if (e == hipSuccess && p->n_slots > 0)
    e = hipMemcpy(p->d_slot_src, slot_src.data(), slot_src.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && p->n_slots > 0) e = hipMalloc(&p->d_slot_frame, slot_frame.size() * sizeof(int32_t));
  if (e == hipSuccess && p->n_slots > 0)
    e = hipMemcpy(p->d_slot_frame, slot_frame.data(), slot_frame.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking);
  for (int m = 0; m < nb::kBatchedModes && e == hipSuccess; ++m) {
    const int32_t cnt = p->seg_end[m] - p->seg_begin[m];
    if (cnt <= 0) continue;
    int g = nb::batched_grid(variant == NBODY_FP32_COMP, m);
    if (g <= 0) {
      e = hipErrorInvalidDeviceFunction;
      break;
    }
    p->grid[m] = g > cnt ? cnt : g;
  }
  if (e != hipSuccess) {
    hip_fail(e, "nbody_plan_create");
    nbody_plan_destroy(p);
    return nullptr;
  }
  return p;
}

void nbody_plan_destroy(nbody_plan *p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->capture) (void)hipStreamDestroy(p->capture);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_slot_src) (void)hipFree(p->d_slot_src);
  if (p->d_slot_frame) (void)hipFree(p->d_slot_frame);
  delete p;
}

int64_t nbody_plan_total(const nbody_plan *p) { return p ? p->n_total : -1; }
int32_t nbody_plan_clusters(const nbody_plan *p) { return p ? p->K : -1; }
int32_t nbody_plan_variant(const nbody_plan *p) { return p ? p->variant : -1; }
int64_t nbody_plan_items(const nbody_plan *p) { return p ? p->n_items : -1; }
double nbody_plan_pairs(const nbody_plan *p) { return p ? p->pairs : -1.0; }

nbody_status nbody_accel_batched(const double *pos, const double *mass, const nbody_plan *plan,
                                 const double *eps_k, double G, int32_t variant, double *acc,
                                 double *pot, void *ws, size_t ws_bytes, void *stream) {
  g_err.clear();
  nbody_status st = check_batched(plan, variant, eps_k);
  if (st != NBODY_OK) return st;
  if (!std::isfinite(G)) return fail(NBODY_EINVAL, "G must be finite");
  const int64_t n = plan->n_total;
  if (n == 0) return NBODY_OK;
  if (!pos || !mass || !acc) return fail(NBODY_EINVAL, "pos, mass and acc must be non-NULL");
  const size_t b3 = static_cast<size_t>(n) * 3 * sizeof(double), b1 = static_cast<size_t>(n) * sizeof(double);
  const size_t bk = static_cast<size_t>(plan->K) * sizeof(double);
  if (overlap(acc, b3, pos, b3) || overlap(acc, b3, mass, b1) || overlap(pot, b1, pos, b3) ||
      overlap(pot, b1, mass, b1) || overlap(pot, b1, acc, b3) || overlap(acc, b3, eps_k, bk) ||
      overlap(pot, b1, eps_k, bk))
    return fail(NBODY_EINVAL, "output arrays overlap inputs or each other");
  st = check_ws(ws, ws_bytes, n, plan->variant, plan->K);
  if (st != NBODY_OK) return st;
  const hipError_t e = enqueue_batched(pos, mass, plan, eps_k, G, acc, pot, ws, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "nbody_accel_batched launch");
  return NBODY_OK;
}

// Checks shared by the KDK entry points: sizes, scalars and overlaps of the
// state arrays (eps_k, when given, is an input that no output may overlap).
static nbody_status check_step_args(double *pos, double *vel, double *acc, double *pot, const double *mass,
                             int64_t n, double dt, int32_t n_steps, double *diag,
                             const double *eps_k, int32_t K) {
  if (n < 0) return fail(NBODY_EINVAL, "n must be >= 0");
  if (n_steps < 0) return fail(NBODY_EINVAL, "n_steps must be >= 0 (got %d)", n_steps);
  if (!std::isfinite(dt)) return fail(NBODY_EINVAL, "dt must be finite");
  if (n == 0 || n_steps == 0) return NBODY_OK;
  if (!pos || !vel || !acc || !mass) return fail(NBODY_EINVAL, "pos, vel, acc and mass must be non-NULL");
  const size_t b3 = static_cast<size_t>(n) * 3 * sizeof(double), b1 = static_cast<size_t>(n) * sizeof(double);
  if (overlap(pos, b3, vel, b3) || overlap(pos, b3, acc, b3) || overlap(vel, b3, acc, b3) ||
      overlap(pos, b3, mass, b1) || overlap(vel, b3, mass, b1) || overlap(acc, b3, mass, b1) ||
      overlap(pot, b1, pos, b3) || overlap(pot, b1, vel, b3) || overlap(pot, b1, acc, b3) ||
      overlap(pot, b1, mass, b1))
    return fail(NBODY_EINVAL, "arrays overlap");
  const size_t db = static_cast<size_t>(n_steps) * nb::kDiagLen * sizeof(double);
  if (diag && (overlap(diag, db, pos, b3) || overlap(diag, db, vel, b3) || overlap(diag, db, acc, b3) ||
               overlap(diag, db, pot, b1) || overlap(diag, db, mass, b1)))
    return fail(NBODY_EINVAL, "diag overlaps the state arrays");
  if (eps_k) {
    const size_t bk = static_cast<size_t>(K) * sizeof(double);
    if (overlap(eps_k, bk, pos, b3) || overlap(eps_k, bk, vel, b3) || overlap(eps_k, bk, acc, b3) ||
        overlap(eps_k, bk, pot, b1) || (diag && overlap(eps_k, bk, diag, db)))
      return fail(NBODY_EINVAL, "eps_k overlaps an output array");
  }
  return NBODY_OK;
}

nbody_status nbody_step(double *pos, double *vel, double *acc, double *pot, const double *mass,
                        int64_t n, double eps, double G, double dt, int32_t n_steps,
                        int32_t variant, const nbody_plan *plan, double *diag, void *ws,
                        size_t ws_bytes, void *stream) {
  g_err.clear();
  if (plan)
    return fail(NBODY_EINVAL,
                "nbody_step steps a single system (plan must be NULL); batched steps take "
                "per-cluster softenings through nbody_step_batched");
  if (!valid_variant(variant)) return fail(NBODY_ENOTSUP, "unknown variant %d", variant);
  nbody_status st = check_scalars(eps, G);
  if (st != NBODY_OK) return st;
  st = check_step_args(pos, vel, acc, pot, mass, n, dt, n_steps, diag, nullptr, 0);
  if (st != NBODY_OK) return st;
  if (n == 0 || n_steps == 0) return NBODY_OK;
  st = check_ws(ws, ws_bytes, n, variant, 1);
  if (st != NBODY_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const WsLayout L = ws_layout(n, variant, 1);
  hipError_t e = hipSuccess;
  if (diag) e = nb::launch_fill_int(at<int>(ws, L.ctr), 1, 0, s);
  for (int32_t k = 0; k < n_steps && e == hipSuccess; ++k)
    e = enqueue_step(pos, vel, acc, pot, mass, n, eps, G, dt, variant, nullptr, nullptr, diag, ws, s);
  if (e != hipSuccess) return hip_fail(e, "nbody_step launch");
  return NBODY_OK;
}

nbody_status nbody_step_batched(double *pos, double *vel, double *acc, double *pot,
                                const double *mass, int64_t n, const nbody_plan *plan,
                                const double *eps_k, double G, double dt, int32_t n_steps,
                                int32_t variant, double *diag, void *ws, size_t ws_bytes,
                                void *stream) {
  g_err.clear();
  nbody_status st = check_batched(plan, variant, eps_k);
  if (st != NBODY_OK) return st;
  if (!std::isfinite(G)) return fail(NBODY_EINVAL, "G must be finite");
  if (n >= 0 && plan->n_total != n)
    return fail(NBODY_EINVAL, "plan covers %lld particles, n = %lld",
                static_cast<long long>(plan->n_total), static_cast<long long>(n));
  st = check_step_args(pos, vel, acc, pot, mass, n, dt, n_steps, diag, eps_k, plan->K);
  if (st != NBODY_OK) return st;
  if (n == 0 || n_steps == 0) return NBODY_OK;
  st = check_ws(ws, ws_bytes, n, variant, plan->K);
  if (st != NBODY_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const WsLayout L = ws_layout(n, variant, plan->K);
  hipError_t e = hipSuccess;

  // Capture one step as a graph (once per argument set), then replay it.
  // eps_k is read from device memory at every replay. The capture comes
  // first, so that a failed capture leaves nothing enqueued on `stream`.
  const void *key[10] = {pos, vel, acc, pot, mass, diag, ws, eps_k, nullptr, nullptr};
  const bool same = plan->exec && std::memcmp(key, plan->key, sizeof(key)) == 0 &&
                    plan->key_g == G && plan->key_dt == dt;
  if (!same) {
    if (plan->exec) {
      (void)hipGraphExecDestroy(plan->exec);
      plan->exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(plan->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    const hipError_t le = enqueue_step(pos, vel, acc, pot, mass, n, 0.0, G, dt, variant, plan, eps_k,
                                       diag, ws, plan->capture);
    e = hipStreamEndCapture(plan->capture, &graph);
    if (le != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(le, "graph capture of a step");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      plan->exec = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
    std::memcpy(plan->key, key, sizeof(key));
    plan->key_g = G;
    plan->key_dt = dt;
  }
  if (diag) e = nb::launch_fill_int(at<int>(ws, L.ctr), 1, 0, s);
  for (int32_t k = 0; k < n_steps && e == hipSuccess; ++k) e = hipGraphLaunch(plan->exec, s);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return NBODY_OK;
}

size_t nbody_workspace_bytes_jerk(int64_t n, int32_t variant) {
  if (n < 0 || !valid_variant(variant)) return 0;
  return jerk_layout(n, variant, jerk_tune(variant, n).split).total;
}

nbody_status nbody_accel_jerk(const double *pos, const double *vel, const double *mass, int64_t n,
                              double eps, double G, int32_t variant, double *acc, double *jerk,
                              double *pot, void *ws, size_t ws_bytes, void *stream) {
  g_err.clear();
  if (n < 0) return fail(NBODY_EINVAL, "n must be >= 0");
  if (!valid_variant(variant)) return fail(NBODY_ENOTSUP, "unknown variant %d", variant);
  nbody_status st = check_scalars(eps, G);
  if (st != NBODY_OK) return st;
  if (n == 0) return NBODY_OK;
  if (!pos || !vel || !mass || !acc || !jerk)
    return fail(NBODY_EINVAL, "pos, vel, mass, acc and jerk must be non-NULL");
  const size_t b3 = static_cast<size_t>(n) * 3 * sizeof(double), b1 = static_cast<size_t>(n) * sizeof(double);
  const void *ins[3] = {pos, vel, mass};
  const size_t inb[3] = {b3, b3, b1};
  void *outs[3] = {acc, jerk, pot};
  const size_t outb[3] = {b3, b3, b1};
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b)
      if (overlap(outs[a], outb[a], ins[b], inb[b])) return fail(NBODY_EINVAL, "outputs overlap inputs");
    for (int b = a + 1; b < 3; ++b)
      if (overlap(outs[a], outb[a], outs[b], outb[b])) return fail(NBODY_EINVAL, "outputs overlap each other");
  }
  const SingleTune t = jerk_tune(variant, n);
  const size_t need = jerk_layout(n, variant, t.split).total;
  if (!ws) return fail(NBODY_EWORKSPACE, "workspace is NULL (need %zu bytes)", need);
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(NBODY_EWORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < need) return fail(NBODY_EWORKSPACE, "workspace of %zu bytes < %zu required", ws_bytes, need);
  const hipError_t e = enqueue_accel_jerk(pos, vel, mass, n, eps, G, variant, t, acc, jerk, pot, ws,
                                          static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "nbody_accel_jerk launch");
  return NBODY_OK;
}

nbody_status nbody_step_hermite(double *pos, double *vel, double *acc, double *jerk, double *pot,
                                const double *mass, int64_t n, double eps, double G, double dt,
                                int32_t n_steps, int32_t variant, double *diag, void *ws,
                                size_t ws_bytes, void *stream) {
  g_err.clear();
  if (n < 0) return fail(NBODY_EINVAL, "n must be >= 0");
  if (n_steps < 0) return fail(NBODY_EINVAL, "n_steps must be >= 0 (got %d)", n_steps);
  if (!valid_variant(variant)) return fail(NBODY_ENOTSUP, "unknown variant %d", variant);
  if (!std::isfinite(dt)) return fail(NBODY_EINVAL, "dt must be finite");
  nbody_status st = check_scalars(eps, G);
  if (st != NBODY_OK) return st;
  if (n == 0 || n_steps == 0) return NBODY_OK;
  if (!pos || !vel || !acc || !jerk || !mass)
    return fail(NBODY_EINVAL, "pos, vel, acc, jerk and mass must be non-NULL");
  const size_t b3 = static_cast<size_t>(n) * 3 * sizeof(double), b1 = static_cast<size_t>(n) * sizeof(double);
  const void *arr[6] = {pos, vel, acc, jerk, mass, pot};
  const size_t ab[6] = {b3, b3, b3, b3, b1, b1};
  for (int a = 0; a < 6; ++a)
    for (int b = a + 1; b < 6; ++b)
      if (overlap(arr[a], ab[a], arr[b], ab[b])) return fail(NBODY_EINVAL, "arrays overlap");
  if (diag) {
    const size_t db = static_cast<size_t>(n_steps) * nb::kDiagLen * sizeof(double);
    for (int a = 0; a < 6; ++a)
      if (overlap(diag, db, arr[a], ab[a])) return fail(NBODY_EINVAL, "diag overlaps the state arrays");
  }
  const SingleTune t = jerk_tune(variant, n);
  const JerkLayout L = jerk_layout(n, variant, t.split);
  if (!ws) return fail(NBODY_EWORKSPACE, "workspace is NULL (need %zu bytes)", L.total);
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(NBODY_EWORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return fail(NBODY_EWORKSPACE, "workspace of %zu bytes < %zu required", ws_bytes, L.total);
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *xp = at<double>(ws, L.xp), *vp = at<double>(ws, L.vp);
  double *a1 = at<double>(ws, L.a1), *j1 = at<double>(ws, L.j1);
  double *potw = pot ? pot : (diag ? at<double>(ws, L.pot) : nullptr);
  hipError_t e = hipSuccess;
  if (diag) e = nb::launch_fill_int(at<int>(ws, L.ctr), 1, 0, s);
  for (int32_t k = 0; k < n_steps && e == hipSuccess; ++k) {
    e = nb::launch_hermite_predict(pos, vel, acc, jerk, n, dt, xp, vp, s);
    if (e == hipSuccess) e = enqueue_accel_jerk(xp, vp, mass, n, eps, G, variant, t, a1, j1, potw, ws, s);
    if (e == hipSuccess) e = nb::launch_hermite_correct(pos, vel, acc, jerk, a1, j1, n, dt, s);
    if (e == hipSuccess && diag) {
      e = nb::launch_kick_diag(pos, vel, nullptr, potw, mass, n, 0.0, at<double>(ws, L.diag), s);
      if (e == hipSuccess) e = nb::launch_diag_final(at<double>(ws, L.diag), diag, at<int>(ws, L.ctr), s);
    }
  }
  if (e != hipSuccess) return hip_fail(e, "nbody_step_hermite launch");
  return NBODY_OK;
}

int32_t nbody_tune_count(int32_t variant) {
  return valid_variant(variant) ? nb::single_cfg_count(variant == NBODY_FP32_COMP) : 0;
}

nbody_status nbody_tune_describe(int32_t variant, int32_t cfg, int32_t *out6) {
  g_err.clear();
  if (!valid_variant(variant)) return fail(NBODY_ENOTSUP, "unknown variant %d", variant);
  if (!out6) return fail(NBODY_EINVAL, "out6 is NULL");
  if (cfg >= 1000) {  // batched modes are described as 1000 + mode
    const int m = cfg - 1000;
    if (m >= nb::batched_mode_count()) return fail(NBODY_EINVAL, "no batched mode %d", m);
    const nb::PairCfg &c = nb::batched_mode(m);
    const int32_t v[6] = {c.block, c.k, c.ls, c.sw, c.tile, nb::cfg_iblock(c)};
    std::memcpy(out6, v, sizeof(v));
    return NBODY_OK;
  }
  if (cfg < 0 || cfg >= nb::single_cfg_count(variant == NBODY_FP32_COMP))
    return fail(NBODY_EINVAL, "no configuration %d", cfg);
  const nb::PairCfg &c = nb::single_cfg(cfg);
  const int32_t v[6] = {c.block, c.k, c.ls, c.sw, c.tile, nb::cfg_iblock(c)};
  std::memcpy(out6, v, sizeof(v));
  return NBODY_OK;
}

// cfg encodes config + 1000 * split; -1 restores the table entry.
nbody_status nbody_tune_set(int32_t variant, int32_t size_class_, int32_t cfg) {
  g_err.clear();
  if (!valid_variant(variant)) return fail(NBODY_ENOTSUP, "unknown variant %d", variant);
  if (size_class_ < 0 || size_class_ >= kClasses) return fail(NBODY_EINVAL, "size class out of range");
  if (cfg != -1) {
    const int c = cfg % 1000, sp = cfg / 1000;
    if (c < 0 || c >= nb::single_cfg_count(variant == NBODY_FP32_COMP) || sp < 0 || sp > nb::kMaxSplit)
      return fail(NBODY_EINVAL, "bad configuration %d", cfg);
  }
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_init_locked();
  g_forced[variant][size_class_] = cfg;
  return NBODY_OK;
}

int32_t nbody_tune_get(int32_t variant, int64_t n) {
  if (!valid_variant(variant) || n < 0) return -1;
  const SingleTune t = single_tune(variant, n);
  return t.cfg + 1000 * t.split;
}

nbody_status nbody_tune_load(const char *path) {
  g_err.clear();
  if (!path) return fail(NBODY_EINVAL, "path is NULL");
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_init_locked();
  return tune_load_locked(path);
}

nbody_status nbody_timing_enable(int32_t on) {
  g_err.clear();
  std::lock_guard<std::mutex> g(g_timing_mu);
  g_timing.on = on != 0;
  g_timing.used = 0;
  return NBODY_OK;
}

nbody_status nbody_timing_read(int64_t *launches, double *total_ms) {
  g_err.clear();
  if (!launches || !total_ms) return fail(NBODY_EINVAL, "launches and total_ms must be non-NULL");
  std::lock_guard<std::mutex> g(g_timing_mu);
  double sum = 0.0;
  int64_t count = 0;
  for (size_t k = 0; k + 1 < g_timing.used; k += 2) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(g_timing.pool[k + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, g_timing.pool[k], g_timing.pool[k + 1]);
    if (e != hipSuccess) {
      g_timing.used = 0;
      return hip_fail(e, "nbody_timing_read");
    }
    sum += ms;
    ++count;
  }
  g_timing.used = 0;
  *launches = count;
  *total_ms = sum;
  return NBODY_OK;
}

int32_t nbody_tune_jerk_count(int32_t variant) {
  return valid_variant(variant) ? nb::jerk_shape_count(variant == NBODY_FP32_COMP) : 0;
}

nbody_status nbody_tune_jerk_describe(int32_t cfg, int32_t *out3) {
  g_err.clear();
  if (!out3) return fail(NBODY_EINVAL, "out3 is NULL");
  if (cfg < 0 || cfg >= nb::jerk_shape_count()) return fail(NBODY_EINVAL, "no jerk shape %d", cfg);
  int k = 0, sw = 0;
  nb::jerk_shape(cfg, &k, &sw);
  out3[0] = k;
  out3[1] = sw;
  out3[2] = nb::jerk_targets_per_block(cfg);
  return NBODY_OK;
}

nbody_status nbody_tune_jerk_set(int32_t variant, int32_t cfg) {
  g_err.clear();
  if (!valid_variant(variant)) return fail(NBODY_ENOTSUP, "unknown variant %d", variant);
  if (cfg != -1) {
    const int c = cfg % 1000, sp = cfg / 1000;
    if (cfg < 0 || c >= nb::jerk_shape_count(variant == NBODY_FP32_COMP) || sp > nb::kMaxSplit)
      return fail(NBODY_EINVAL, "bad jerk configuration %d", cfg);
  }
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_init_locked();
  g_jerk_forced[variant] = cfg;
  return NBODY_OK;
}

int32_t nbody_tune_jerk_get(int32_t variant, int64_t n) {
  if (!valid_variant(variant) || n < 0) return -1;
  const SingleTune t = jerk_tune(variant, n);
  return t.cfg + 1000 * t.split;
}

nbody_status nbody_tune_reset(void) {
  g_err.clear();
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune_init = false;
  tune_init_locked();
  return NBODY_OK;
}

}  // extern "C"
