// Allocation-free apply (cm_apply_noalloc in include/cmmlfma.h): the same
// kernels as cm_apply, with the apply's workspace (pattern levels and the
// permuted input / near-field output) carved out of one fixed device array
// instead of the handle's own workspace.  For callers that cannot allocate
// device memory.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "cm_device.h"

namespace cm {

cm_status driver_fail(int code, const std::string& msg);

// The fixed workspace: every GPU the library runs on holds its own copy until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: only the address from hipGetSymbolAddress (one per device)
// is passed to kernels.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array; looked up once per device,
// with that device current.
static void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error(CM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

}  // namespace cm

extern "C" cm_status cm_apply_noalloc(cm_handle* h, cm_op op, const void* x, void* y, int64_t ld, int32_t ncols,
                                      cm_dtype dt, void* hip_stream) {
  if (!h || !x || !y) return cm::driver_fail(CM_E_BADARG, "null argument");
  if (!h->has_dev) return cm::driver_fail(CM_E_NOT_BUILT, "handle was built host-only");
  if (ncols < 1 || ncols > h->dev.max_cols) return cm::driver_fail(CM_E_BADARG, "ncols out of range [1, max_cols]");
  if (ld < ncols) return cm::driver_fail(CM_E_BADARG, "ld < ncols");
  if (dt != CM_C64 && dt != CM_C128) return cm::driver_fail(CM_E_BADARG, "bad dtype");
  if ((int)op < 0 || (int)op > 4) return cm::driver_fail(CM_E_BADARG, "bad op");
  if (x == y) return cm::driver_fail(CM_E_BADARG, "x and y must not alias");
  if (op == CM_OP_DZDK && !(h->plan.opt.flags & CM_FLAG_DERIV))
    return cm::driver_fail(CM_E_NOT_BUILT, "dZ/dk needs CM_FLAG_DERIV at create");
  const bool fp64 = dt == CM_C128;
  size_t part[cm::kMaxLevels];
  // each part is followed by a 64 KiB gap inside the array, a margin for any
  // vector load that runs past the last column of a tile
  constexpr size_t kGap = (size_t)64 << 10;
  const size_t need = cm::work_bytes(h->plan, (int)op, ncols, fp64, part) + 2 * (size_t)(h->plan.lf) * kGap;
  if (need > cm::kScratchBytes)
    return cm::driver_fail(CM_E_BADARG, "workspace of " + std::to_string(need) + " bytes exceeds the " +
                                            std::to_string(cm::kScratchBytes) + "-byte fixed scratch array");
  try {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= cm::kMaxDevices)
      return cm::driver_fail(CM_E_HIP, "hipGetDevice failed or device index out of range");
    if (dev != h->dev.device) return cm::driver_fail(CM_E_BADARG, "the current device is not the handle's device");
    unsigned char* base = (unsigned char*)cm::scratch_ptr(dev);
    cm::Work w;
    size_t at = 0;
    w.xi = base + at;
    at += part[0] + kGap;
    w.yi = base + at;
    at += part[0] + kGap;
    for (int l = 2; l <= h->plan.lf; ++l) {
      w.S[l] = base + at;
      at += part[l] + kGap;
      w.G[l] = base + at;
      at += part[l] + kGap;
    }
    cm::dev_apply_ws(h->dev, h->plan, (int)op, x, y, ld, ncols, fp64, w, (hipStream_t)hip_stream);
    return CM_OK;
  } catch (const cm::Error& e) {
    return cm::driver_fail(e.code, e.what());
  } catch (const std::exception& e) {
    return cm::driver_fail(CM_E_BADARG, e.what());
  }
}
