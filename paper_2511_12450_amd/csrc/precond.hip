// Overlapping domain-decomposition preconditioner (Sec. 4.2).
#include "lm_internal.hpp"

struct Precond {
  int dummy;
};

lm_status precond_build(lm_geom_s* g, hipStream_t s) {
  (void)g;
  (void)s;
  return LM_OK;
}
void precond_free(Precond* p) { delete p; }
int64_t precond_bytes(const Precond* p) { return p ? 0 : 0; }
lm_status precond_apply(lm_geom_s* g, int n_rhs, const void* x, void* y, hipStream_t s) {
  (void)g; (void)n_rhs; (void)x; (void)y; (void)s;
  lm_set_error("no preconditioner");
  return LM_EINVAL;
}
