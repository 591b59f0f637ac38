// Layered-medium fast multipole method (Sec. 4.1).
#include "lm_internal.hpp"

struct FmmPlan {
  int dummy;
};

lm_status fmm_build(lm_geom_s* g, hipStream_t s) {
  (void)g;
  (void)s;
  lm_set_error("the FMM method is not available in this build");
  return LM_EINVAL;
}
void fmm_free(FmmPlan* f) { delete f; }
int64_t fmm_bytes(const FmmPlan* f) { return f ? 0 : 0; }
lm_status fmm_matvec(lm_geom_s* g, int precision, int n_rhs, const void* x, void* y, hipStream_t s) {
  (void)g; (void)precision; (void)n_rhs; (void)x; (void)y; (void)s;
  lm_set_error("the FMM method is not available in this build");
  return LM_EINVAL;
}
