// Sweep-kernel instantiations: double states, tiles of 3 qubits.
#include "rq_sweep.h"

namespace rqk {
int launch_pass_f64_nt3(int mode, int op, int stage, const PassArgs &a, int grid, void *s) {
  return launch_nt<double, 3, false, false, true, false>(mode, op, stage, a, grid, s);
}
}  // namespace rqk
