// Placeholder for the FMM far field; replaced by the multilevel implementation.
#include "state.h"

namespace bem {

struct FmmState {};

void fmm_destroy(FmmState* f) { delete f; }

void fmm_setup_problem(bem_mesh*, hipStream_t) {
  throw Error(BEM_E_STATE, "the FMM far field is not available in this build");
}

void fmm_apply(bem_mesh*, bem_op, bem_precision, const double2*, double2*, hipStream_t) {
  throw Error(BEM_E_STATE, "the FMM far field is not available in this build");
}

size_t fmm_bytes(const bem_mesh*) { return 0; }

}  // namespace bem
