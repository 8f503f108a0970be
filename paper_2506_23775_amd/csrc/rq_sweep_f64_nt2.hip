// Sweep-kernel instantiations: double states, tiles of 2 qubits.
#include "rq_sweep.h"

namespace rqk {
int launch_pass_f64_nt2(int mode, int op, int stage, const PassArgs &a, int grid, void *s) {
  return launch_nt<double, 2, true, true, true, true>(mode, op, stage, a, grid, s);
}
}  // namespace rqk
