/*
 * rq_static.h -- allocation-free variant of rq_hvp (see rq.h for the
 *                conventions of every argument).
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * workspace (gate coefficients, FP64 partial-sum slots, checkpoint slabs of
 * one chunk of basis columns) lives in a static device array of
 * RQ_STATIC_SCRATCH_BYTES per GPU, which the library holds until the
 * process ends; the call allocates nothing (no hipMalloc / hipFree, no
 * allocating library routine).
 */
#ifndef RQ_STATIC_H
#define RQ_STATIC_H

#include "rq.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Size of the static scratch array on each GPU (256 MiB). */
#define RQ_STATIC_SCRATCH_BYTES ((size_t)256 << 20)

/* rq_hvp with the workspace in the static scratch of the current device:
 * same arguments, outputs and results as rq_hvp (f, egrad, rgrad, ehvp,
 * rhvp; device outputs nullable), the kernels enqueued on `stream` (a
 * hipStream_t of the current device; NULL = default stream), exec_flags as
 * rq_exec.flags (RQ_EXEC_ACCUMULATE or 0).  The chunk of basis columns is
 * the largest multiple of 64 (at most the range's column count rounded up
 * to 64) whose workspace fits RQ_STATIC_SCRATCH_BYTES; it is written to
 * *chunk_used (nullable), and results equal rq_hvp's at that chunk bitwise.
 * Errors: RQ_ESPACE when even a 64-column chunk needs more than the scratch
 * (e.g. k = 16 parity HVP with many passes), the argument errors of rq_hvp,
 * RQ_EHIP if the scratch address cannot be looked up.
 * Concurrency: every call on one GPU shares that GPU's scratch, which keeps
 * the last call's contents (every partial sum is cleared by the call
 * itself); calls that overlap on one GPU -- on different streams, or from
 * different host threads -- race and give wrong results.  Serialise them. */
int rq_hvp_static(const rq_circuit *circuit, const rq_target *target, const double *gates,
                  const double *dir, const rq_range *range, void *stream, uint32_t exec_flags,
                  int64_t *chunk_used, double *d_f, double *d_egrad, double *d_rgrad,
                  double *d_ehvp, double *d_rhvp);

#ifdef __cplusplus
}
#endif

#endif /* RQ_STATIC_H */
