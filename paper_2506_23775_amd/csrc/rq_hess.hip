// Hessian blocks (implementation follows).
#include <hip/hip_runtime.h>

#include "../../include/rq.h"

extern "C" int rq_hess_blocks(const rq_circuit *, const rq_target *, const double *,
                              const rq_range *, const rq_exec *, double *, double *, double *,
                              double *, double *) {
  return RQ_EINVAL;
}

extern "C" size_t rq_hess_workspace_bytes(const rq_circuit *, int32_t, int64_t) { return 0; }
