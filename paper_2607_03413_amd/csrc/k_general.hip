// General-geometry operator (deformed mesh, variable coefficient) and its
// setup.  Filled in by the deformed-geometry path.
#include "fe_internal.h"
#include "kernel_common.h"

namespace fe {

fe_status setup_geometry(fe_problem*, hipStream_t) {
  return fail(FE_EUNSUPPORTED, "deformed geometry not built yet");
}
fe_status setup_patch_factors(fe_problem*, int, int, hipStream_t) {
  return fail(FE_EUNSUPPORTED, "per-patch factors not built yet");
}
fe_status launch_apply_general(const fe_problem*, int, const void*, void*, fe_dtype, hipStream_t) {
  return fail(FE_EUNSUPPORTED, "general operator not built yet");
}
fe_status launch_diag_general(const fe_problem*, int, void*, fe_dtype, hipStream_t) {
  return fail(FE_EUNSUPPORTED, "general diagonal not built yet");
}
fe_status launch_rhs_general(const fe_problem*, void*, hipStream_t) {
  return fail(FE_EUNSUPPORTED, "general load vector not built yet");
}

}  // namespace fe
