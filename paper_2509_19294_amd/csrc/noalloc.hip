// Allocation-free force evaluation (nbody_accel_noalloc, declared in
// include/nbody.h), for callers that cannot allocate device memory or hand
// the library a workspace: code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation.
//
// The workspace nbody_accel takes from its caller is here a file-scope device
// array. Each GPU the library runs on holds its own copy for the life of the
// process. Host code never passes the array's name to a kernel (on the host
// that name is only a stand-in, not a device address): the first call on a
// device, with that device current, asks the runtime for the array's device
// address and keeps it per device; every later call on that device passes
// that address as the workspace.
//
// Every call on one GPU shares that GPU's array, which keeps the last call's
// contents (nothing in it needs to start at zero: every region is written
// before it is read within one call). Calls that overlap on one GPU, from two
// streams or two host threads, race on the array; callers must order them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>

#include "nbody.h"
#include "nbody_internal.h"

// 64 MiB: n up to 1,676,064 particles in the plain form and 536,480 in the
// compensated form (with the grid j-split reduced to fit).
constexpr size_t kScratchBytes = size_t{64} << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
hipError_t scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" nbody_status nbody_accel_noalloc(const double *pos, const double *mass, int64_t n,
                                            double eps, double G, int32_t variant, double *acc,
                                            double *pot, void *stream) {
  nbody_status st = nb::check_accel_args(pos, mass, n, eps, G, variant, acc, pot);
  if (st != NBODY_OK || n == 0) return st;
  // The tuned grid split if its partial sums fit, else the largest that does.
  int split = nb::accel_tuned_split(variant, n);
  while (split > 1 && nb::accel_ws_bytes(n, variant, split) > kScratchBytes) --split;
  if (nb::accel_ws_bytes(n, variant, split) > kScratchBytes) {
    char msg[200];
    std::snprintf(msg, sizeof(msg),
                  "n = %lld needs %zu bytes of workspace, more than the %zu-byte no-alloc scratch",
                  static_cast<long long>(n), nb::accel_ws_bytes(n, variant, 1), kScratchBytes);
    return nb::set_error(NBODY_EINVAL, msg);
  }
  void *ws = nullptr;
  const hipError_t e = scratch_address(&ws);
  if (e != hipSuccess) {
    char msg[200];
    std::snprintf(msg, sizeof(msg), "no-alloc scratch address: %s", hipGetErrorString(e));
    return nb::set_error(NBODY_EHIP, msg);
  }
  return nb::accel_entry(pos, mass, n, eps, G, variant, acc, pot, ws, kScratchBytes, split, stream);
}
