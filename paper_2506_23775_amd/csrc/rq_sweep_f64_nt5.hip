// Sweep-kernel instantiations: double states, tiles of 5 qubits.
#include "rq_sweep.h"

namespace rqk {
int launch_pass_f64_nt5(int mode, int op, int stage, const PassArgs &a, int grid, void *s) {
  return launch_nt<double, 5, true, false, false, false>(mode, op, stage, a, grid, s);
}
}  // namespace rqk
