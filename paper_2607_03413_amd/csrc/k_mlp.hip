// Per-patch factor weights: averaged geometry (mode 1) or the learned model (mode 2).
#include "fe_internal.h"
#include "kernel_common.h"

namespace fe {

fe_status averaged_patch_weights(fe_problem* p, int level, DeviceBuf& weights, hipStream_t s);

fe_status patch_weights(fe_problem* p, int level, int mode, DeviceBuf& weights, hipStream_t s) {
  if (mode == 1) return averaged_patch_weights(p, level, weights, s);
  return fail(FE_EUNSUPPORTED, "learned factors need a trained model");
}

}  // namespace fe
