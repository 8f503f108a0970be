// Sweep-kernel instantiations: float states, tiles of 4 qubits.
#include "rq_sweep.h"

namespace rqk {
int launch_pass_f32_nt4(int mode, int op, int stage, const PassArgs &a, int grid, void *s) {
  return launch_nt<float, 4, false, false, true, true>(mode, op, stage, a, grid, s);
}
}  // namespace rqk
