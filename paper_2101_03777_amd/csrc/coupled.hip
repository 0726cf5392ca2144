// Baseline: FP64 MINRES on the coupled system (filled in below).
#include "internal.h"

namespace crh {
cr_status run_coupled_solve(cr_system*, const cr_solve_opts*, cr_solve_info*, double*, double*) {
  set_error("coupled baseline not built yet");
  return CR_E_INVAL;
}
}  // namespace crh
