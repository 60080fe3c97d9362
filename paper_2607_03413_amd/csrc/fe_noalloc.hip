// Allocation-free variant of the vertex-patch inverse, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The two-pass patch kernels (k >= 4, k = 1, d = 2, per-patch factors) write
// every patch solution to a scratch buffer and sum the overlaps in a second
// pass.  Here that buffer is a fixed file-scope device array: each GPU the
// library runs on holds one copy of it, at its own address, until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in for the symbol); the device address is looked up once per
// device with hipGetSymbolAddress and kept.
#include <mutex>

#include "fe_internal.h"

namespace fe {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with that device current).
fe_status scratch_ptr(void** out) {
  int dev = -1;
  FE_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FE_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FE_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[dev] = ptr;
  }
  *out = g_ptr[dev];
  return FE_OK;
}

}  // namespace
}  // namespace fe

using namespace fe;

extern "C" {

size_t fe_noalloc_scratch_bytes(void) { return kScratchBytes; }

fe_status patch_fdm_inverse_noalloc(const fe_problem* p, int level, const void* r, void* z, fe_dtype dt, int factors,
                                    void* stream) {
  if (!p) return fail(FE_EINVAL, "null problem");
  if (dt != FE_F64 && dt != FE_F32) return fail(FE_EINVAL, "unknown dtype");
  FE_CHECK(check_level(p, level));
  FE_CHECK(check_ptr(r, "r_cell"));
  FE_CHECK(check_ptr(z, "z_cell"));
  if (r == z) return fail(FE_EINVAL, "r and z must not alias");
  if (factors < 0 || factors > 3) return fail(FE_EINVAL, "factors must be 0, 1, 2 or 3");
  if (factors == 0 && p->desc.geometry != FE_GEOM_CARTESIAN)
    return fail(FE_EINVAL, "exact separable factors need the Cartesian mesh");
  if (factors != 0 && p->desc.geometry != FE_GEOM_DEFORMED)
    return fail(FE_EINVAL, "per-patch factors need the deformed geometry");
  const int li = level < 0 ? (int)p->levels.size() - 1 : level;
  // computing per-patch factors allocates: they must have been set up before
  if (factors != 0 && !p->levels[li].patch_eig_ready[factors])
    return fail(FE_EINVAL, "per-patch factors not set up on this level: call fe_patch_prepare first");
  const bool two_pass = !fused_patch_supported(p, factors != 0);
  const size_t need = two_pass ? patch_scratch_bytes(p, li, dt) : 0;
  if (need > kScratchBytes)
    return fail(FE_EINVAL, "patch scratch of " + std::to_string(need) + " bytes exceeds the fixed " +
                               std::to_string(kScratchBytes) + "-byte buffer of the allocation-free entry point");
  void* ptr = nullptr;
  if (two_pass) FE_CHECK(scratch_ptr(&ptr));
  return launch_patch_inverse(p, li, r, z, ptr, dt, factors, (hipStream_t)stream);
}

}  // extern "C"
