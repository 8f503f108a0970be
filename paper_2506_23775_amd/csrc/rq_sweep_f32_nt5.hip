// Sweep-kernel instantiations: float states, tiles of 5 qubits.
#include "rq_sweep.h"

namespace rqk {
int launch_pass_f32_nt5(int mode, int op, int stage, const PassArgs &a, int grid, void *s) {
  return launch_nt<float, 5, true, true, false, false>(mode, op, stage, a, grid, s);
}
}  // namespace rqk
