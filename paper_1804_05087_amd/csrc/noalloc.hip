// Phi_dt without device allocation: sp_befe_step with its intermediates (the
// y-valued, x-physical and product fields of the transforms) in a fixed,
// file-scope device array instead of the plan's scratch, for callers that
// cannot allocate device memory per call or per plan buffer set.
//
// The array's address is looked up once per device with hipGetSymbolAddress
// (the host-side name of a __device__ array is not a device address) while a
// plan is created on that device; the entry point passes only that address to
// the kernels. Every call on one device shares the array, so calls that
// overlap on one device (different streams or plans) race; the pipeline
// overwrites every intermediate before reading it, so nothing needs clearing
// between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sp_internal.h"

namespace sp {

namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;  // 32 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Bytes of the intermediates of one FP64 or mixed evaluation (the FP32 path
// uses half of each piece).
void pieces(const Dims& d, size_t sz[4]) {
  const size_t cz = sizeof(double2);
  sz[0] = (size_t)6 * d.ny * d.nzm * d.nx * cz;  // yv
  sz[1] = (size_t)6 * d.ny * d.px * d.nzm * cz;  // xp
  sz[2] = (size_t)3 * d.ny * d.px * d.nzm * cz;  // np
  sz[3] = (size_t)3 * d.ny * d.nzm * d.nx * cz;  // nv
}

}  // namespace

// Called by sp_plan_create with the plan's device current: the first call on a
// device looks the array's address up there and keeps it (or the error).
void noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_done[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_err[device] = e;
  g_ptr[device] = (e == hipSuccess) ? ptr : nullptr;
  if (e != hipSuccess) (void)hipGetLastError();
  g_done[device] = true;
}

size_t noalloc_bytes_needed(const Dims& d) {
  size_t sz[4];
  pieces(d, sz);
  return round256(sz[0]) + round256(sz[1]) + round256(sz[2]) + round256(sz[3]);
}

}  // namespace sp

using namespace sp;

extern "C" sp_status sp_befe_step_noalloc(sp_plan* p, const double* u, double* out) {
  if (!p) return SP_ERR_INVALID;
  if (!u || !out) return set_error(p, SP_ERR_INVALID, "null pointer");
  if (p->advect)
    return set_error(p, SP_ERR_INVALID,
                     "sp_befe_step_noalloc: the advected step is not provided");
  const size_t need = noalloc_bytes_needed(p->d);
  if (need > kScratchBytes)
    return set_error(p, SP_ERR_SHAPE,
                     "sp_befe_step_noalloc: the intermediates of this grid (" +
                         std::to_string(need) + " bytes) exceed the 32 MiB scratch");
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (p->device < 0 || p->device >= kMaxDevices || !g_done[p->device])
      return set_error(p, SP_ERR_HIP, "sp_befe_step_noalloc: no scratch address for the device");
    if (!g_ptr[p->device])
      return hip_check(p, g_err[p->device], "hipGetSymbolAddress(scratch)");
    base = g_ptr[p->device];
  }
  size_t sz[4];
  pieces(p->d, sz);
  char* b = static_cast<char*>(base);
  // point the plan's intermediates at the array for the launches of this call
  void* saved[4] = {p->yv, p->xp, p->np, p->nv};
  p->yv = b;
  p->xp = b + round256(sz[0]);
  p->np = b + round256(sz[0]) + round256(sz[1]);
  p->nv = b + round256(sz[0]) + round256(sz[1]) + round256(sz[2]);
  const sp_status s = befe_into(p, (const double2*)u, (double2*)out, p->precision == SP_MIXED);
  p->yv = saved[0];
  p->xp = saved[1];
  p->np = saved[2];
  p->nv = saved[3];
  return s;
}
