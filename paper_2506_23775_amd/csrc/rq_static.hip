// rq_hvp_static: rq_hvp for callers that cannot allocate device memory.
//
// The workspace of the sweep (gate coefficients, FP64 partial-sum slots and
// the checkpoint slabs of one chunk of basis columns) lives in a file-scope
// device array instead of caller memory.  Host code never passes the array's
// name to a kernel or a copy: on the first call on a device, with that device
// current, its device address is looked up with hipGetSymbolAddress and kept
// per device; every later call on that device uses the stored address.  The
// call itself allocates nothing: it picks the largest chunk whose workspace
// fits the array and runs the same kernels as rq_hvp.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/rq_static.h"
#include "rq_internal.h"

namespace rqk {
int sweep_call(const rq_circuit *c, const rq_target *t, const double *gates, const double *dir,
               const rq_range *range, const rq_exec *ex, int32_t op_pub, double *d_f,
               double *d_egrad, double *d_rgrad, double *d_ehvp, double *d_rhvp);
int api_fail(int code, const char *msg);
}  // namespace rqk

namespace {

__device__ __align__(256) char scratch[RQ_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device).
int scratch_of_current_device(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return rqk::api_fail(RQ_EHIP, "rq_hvp_static: no current HIP device");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return rqk::api_fail(RQ_EHIP, (std::string("rq_hvp_static: hipGetSymbolAddress: ") +
                                     hipGetErrorString(e)).c_str());
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RQ_OK;
}

}  // namespace

extern "C" int rq_hvp_static(const rq_circuit *circuit, const rq_target *target,
                             const double *gates, const double *dir, const rq_range *range,
                             void *stream, uint32_t exec_flags, int64_t *chunk_used,
                             double *d_f, double *d_egrad, double *d_rgrad, double *d_ehvp,
                             double *d_rhvp) {
  if (chunk_used) *chunk_used = 0;
  if (!circuit || !target) return rqk::api_fail(RQ_EINVAL, "rq_hvp_static: circuit or target is NULL");
  if (exec_flags & ~RQ_EXEC_ACCUMULATE) return rqk::api_fail(RQ_EINVAL, "rq_hvp_static: unknown exec flag");
  const bool parity = circuit->flags & RQ_PARITY;
  const int kq = parity ? circuit->n_qubits - 1 : circuit->n_qubits;
  if (kq < 1 || kq > 31) return rqk::api_fail(RQ_EINVAL, "rq_hvp_static: n_qubits out of range");
  // columns of one sweep: the range's count, or a whole sector / the basis
  int64_t ncols = int64_t(1) << kq;
  if (range) ncols = range->count;
  if (ncols < 0) return rqk::api_fail(RQ_EINVAL, "rq_hvp_static: negative basis range count");
  // largest multiple of 64 (at most the padded column count) whose
  // workspace fits the scratch array; the workspace grows with the chunk
  int64_t hi = (ncols + 63) / 64;
  if (hi < 1) hi = 1;
  if (hi > (int64_t(1) << 20)) hi = int64_t(1) << 20;
  const size_t need64 = rq_workspace_bytes(circuit, RQ_OP_HVP, target->dtype, 64);
  if (need64 == 0) return RQ_EINVAL;   // argument error, message already set
  if (need64 > RQ_STATIC_SCRATCH_BYTES)
    return rqk::api_fail(RQ_ESPACE, ("rq_hvp_static: needs " + std::to_string(need64) +
                                     " bytes of scratch at the smallest chunk (64 columns); the "
                                     "static scratch holds " +
                                     std::to_string(size_t(RQ_STATIC_SCRATCH_BYTES)) + " bytes")
                                        .c_str());
  int64_t lo = 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    const size_t need = rq_workspace_bytes(circuit, RQ_OP_HVP, target->dtype, 64 * mid);
    if (need != 0 && need <= RQ_STATIC_SCRATCH_BYTES)
      lo = mid;
    else
      hi = mid - 1;
  }
  void *ws = nullptr;
  int st = scratch_of_current_device(&ws);
  if (st) return st;
  const rq_exec ex{ws, size_t(RQ_STATIC_SCRATCH_BYTES), 64 * lo, stream, exec_flags, 0u};
  st = rqk::sweep_call(circuit, target, gates, dir, range, &ex, RQ_OP_HVP, d_f, d_egrad, d_rgrad,
                       d_ehvp, d_rhvp);
  if (!st && chunk_used) *chunk_used = 64 * lo;
  return st;
}
