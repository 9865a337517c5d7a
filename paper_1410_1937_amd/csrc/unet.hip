// libnfa: learned preconditioner (placeholder until the network lands).
#include "nfa_internal.h"

namespace nfa {
nfa_status unet_precond_apply(void*, Poisson&, const float*, float*, const SolveScalars*, hipStream_t) {
  return fail(NFA_ERR_INVALID, "learned preconditioner not available");
}
}  // namespace nfa
