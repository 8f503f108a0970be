// Sweep-kernel instantiations: double states, tiles of 4 qubits.
#include "rq_sweep.h"

namespace rqk {
int launch_pass_f64_nt4(int mode, int op, int stage, const PassArgs &a, int grid, void *s) {
  return launch_nt<double, 4, false, true, false, true>(mode, op, stage, a, grid, s);
}
}  // namespace rqk
