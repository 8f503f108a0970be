// Sweep-kernel instantiations: float states, tiles of 2 qubits.
#include "rq_sweep.h"

namespace rqk {
int launch_pass_f32_nt2(int mode, int op, int stage, const PassArgs &a, int grid, void *s) {
  return launch_nt<float, 2, true, true, true, true>(mode, op, stage, a, grid, s);
}
}  // namespace rqk
