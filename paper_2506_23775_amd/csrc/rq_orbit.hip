// Orbit-representative input states and target columns (basis-orbit
// reduction of the trace sum under a translation symmetry; an extension of
// Sec. "Exploiting translational invariance" from hole pairs to the basis
// sum): column r of sector s is sqrt(w_r) |rep_r> on the input side and
// sqrt(w_r) U|rep_r> on the target side, zero beyond the sector's count.
#include <hip/hip_runtime.h>

#include "rq_internal.h"

namespace rqk {

template <typename R>
struct cplx {
  R x, y;
};

// inputs[s][x][r] and ref_out[s][x][r] for s < nsec, x < rows, r < width;
// reps / sw: [nsec][width] representative rows (compressed in parity mode,
// -1 past the sector's count) and square roots of the orbit sizes.
template <typename R>
__global__ void k_orbit_fill(const cplx<R> *__restrict__ ref_in, int64_t ld_in,
                             int64_t sector_stride_in, const int64_t *__restrict__ reps,
                             const double *__restrict__ sw, cplx<R> *__restrict__ inputs,
                             cplx<R> *__restrict__ ref_out, int nsec, int64_t rows,
                             int64_t width) {
  const int64_t total = int64_t(nsec) * rows * width;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = i % width;
    const int64_t x = (i / width) % rows;
    const int s = int(i / (width * rows));
    const int64_t rep = reps[int64_t(s) * width + r];
    cplx<R> vin{R(0), R(0)}, vref{R(0), R(0)};
    if (rep >= 0) {
      const double w = sw[int64_t(s) * width + r];
      if (x == rep) vin.x = R(w);
      const cplx<R> u = ref_in[int64_t(s) * sector_stride_in + x * ld_in + rep];
      vref.x = R(w * double(u.x));
      vref.y = R(w * double(u.y));
    }
    inputs[i] = vin;
    ref_out[i] = vref;
  }
}

int launch_orbit_fill(int is_double, const void *ref_in, int64_t ld_in, int64_t sector_stride_in,
                      const int64_t *reps, const double *sw, void *inputs, void *ref_out,
                      int nsec, int64_t rows, int64_t width, void *s) {
  const int64_t total = int64_t(nsec) * rows * width;
  if (total == 0) return 0;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (is_double)
    hipLaunchKernelGGL(k_orbit_fill<double>, dim3(unsigned(blocks)), dim3(256), 0,
                       (hipStream_t)s, (const cplx<double> *)ref_in, ld_in, sector_stride_in,
                       reps, sw, (cplx<double> *)inputs, (cplx<double> *)ref_out, nsec, rows,
                       width);
  else
    hipLaunchKernelGGL(k_orbit_fill<float>, dim3(unsigned(blocks)), dim3(256), 0,
                       (hipStream_t)s, (const cplx<float> *)ref_in, ld_in, sector_stride_in,
                       reps, sw, (cplx<float> *)inputs, (cplx<float> *)ref_out, nsec, rows,
                       width);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace rqk
