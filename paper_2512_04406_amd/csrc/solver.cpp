// Outer loop (Algorithm alg1), RTR + truncated CG, Lanczos: filled in next.
#include "mdsdp_internal.hpp"
extern "C" {
void mdsdp_default_options(mdsdp_options* o) { (void)o; }
mdsdp_status mdsdp_min_eigpair(mdsdp_problem, double, int32_t, uint64_t, double*, double*, double*, int32_t*, void*) {
  return MDSDP_EUNSUPPORTED;
}
mdsdp_status mdsdp_solve(mdsdp_problem, const mdsdp_options*, int32_t, double*, mdsdp_result*, double*, int32_t,
                         void*) {
  return MDSDP_EUNSUPPORTED;
}
}
