// FP64 reduction of the per-wavefront partial sums, Riemannian
// post-processing, and the dispatcher of the sweep-kernel instantiations.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rq_internal.h"

namespace rqk {

int launch_pass_f32_nt2(int, int, int, const PassArgs &, int, void *);
int launch_pass_f32_nt4(int, int, int, const PassArgs &, int, void *);
int launch_pass_f32_nt5(int, int, int, const PassArgs &, int, void *);
int launch_pass_f64_nt2(int, int, int, const PassArgs &, int, void *);
int launch_pass_f64_nt3(int, int, int, const PassArgs &, int, void *);
int launch_pass_f64_nt4(int, int, int, const PassArgs &, int, void *);
int launch_pass_f64_nt5(int, int, int, const PassArgs &, int, void *);

int launch_pass(int is_double, int nt, int mode, int op, int stage, const PassArgs &a,
                int grid, void *s) {
  if (!is_double) {
    switch (nt) {
      case 2: return launch_pass_f32_nt2(mode, op, stage, a, grid, s);
      case 4: return launch_pass_f32_nt4(mode, op, stage, a, grid, s);
      case 5: return launch_pass_f32_nt5(mode, op, stage, a, grid, s);
    }
  } else {
    switch (nt) {
      case 2: return launch_pass_f64_nt2(mode, op, stage, a, grid, s);
      case 3: return launch_pass_f64_nt3(mode, op, stage, a, grid, s);
      case 4: return launch_pass_f64_nt4(mode, op, stage, a, grid, s);
      case 5: return launch_pass_f64_nt5(mode, op, stage, a, grid, s);
    }
  }
  return -3;
}

// out[r] = sum_s slots[r * nslots + s] for r < rows, summed in a fixed order
// (strided per-thread sums, then a shared-memory tree).
__global__ __launch_bounds__(256) void k_reduce_rows(const double *__restrict__ slots, int nslots,
                                                     double *__restrict__ out) {
  __shared__ double red[256];
  const double *s = slots + int64_t(blockIdx.x) * nslots;
  double v = 0.0;
  for (int i = threadIdx.x; i < nslots; i += 256) v += s[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Binomial coefficients C(n, m), n, m < 32 (C(31, 15) < 2^31).
struct BinomTable {
  int32_t v[32][32];
};
constexpr BinomTable make_binom_table() {
  BinomTable t{};
  for (int n = 0; n < 32; ++n) {
    t.v[n][0] = 1;
    for (int m = 1; m <= n; ++m) t.v[n][m] = t.v[n - 1][m - 1] + (m < n ? t.v[n - 1][m] : 0);
  }
  return t;
}
__constant__ BinomTable kBinom = make_binom_table();

// rank[x] = colex rank of basis index x among the indices of its popcount:
// the number of y < x with popcount(y) = popcount(x), i.e. the sum of
// C(p, j) over the set bits of x (p its position, j = 1, 2, ... its order
// from the least significant set bit).
__global__ void k_rank_table(int32_t *rank, int k) {
  const int64_t n = int64_t(1) << k;
  for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < n;
       x += int64_t(gridDim.x) * blockDim.x) {
    int32_t r = 0;
    int j = 0;
    for (int p = 0; p < k; ++p)
      if ((x >> p) & 1) r += kBinom.v[p][++j];
    rank[x] = r;
  }
}

int launch_rank_table(int32_t *rank, int k, void *s) {
  const int64_t n = int64_t(1) << k;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_rank_table, dim3(blocks), dim3(256), 0, (hipStream_t)s, rank, k);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ void k_zero(double *p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

int launch_reduce(const double *slots, int n_inst, int ne, int nslots, double *out, void *s) {
  const int rows = n_inst * ne;
  if (rows == 0) return 0;
  hipLaunchKernelGGL(k_reduce_rows, dim3(rows), dim3(256), 0, (hipStream_t)s, slots, nslots, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_zero(double *p, int64_t n, void *s) {
  if (n == 0) return 0;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)s, p, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ----------------------------------------------------------------------------
// Streaming device copy (diagnostic: the practical HBM read+write rate the
// sweep kernels are compared with).  Each thread moves UNROLL 16-byte
// vectors per iteration, all loads issued before the stores; the grid
// strides over the buffer.
// ----------------------------------------------------------------------------
template <int UNROLL>
__global__ __launch_bounds__(256) void k_stream_copy(const uint4 *__restrict__ src,
                                                     uint4 *__restrict__ dst, int64_t n16) {
  const int64_t stride = int64_t(gridDim.x) * 256;
  int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  for (; i + (UNROLL - 1) * stride < n16; i += UNROLL * stride) {
    uint4 v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) dst[i + u * stride] = v[u];
  }
  for (; i < n16; i += stride) dst[i] = src[i];
}

int launch_stream_copy(void *dst, const void *src, int64_t bytes, int unroll, int blocks,
                       void *s) {
  const int64_t n16 = bytes / 16;
  const uint4 *a = static_cast<const uint4 *>(src);
  uint4 *b = static_cast<uint4 *>(dst);
  switch (unroll) {
    case 1: hipLaunchKernelGGL(k_stream_copy<1>, dim3(blocks), dim3(256), 0, (hipStream_t)s, a, b, n16); break;
    case 2: hipLaunchKernelGGL(k_stream_copy<2>, dim3(blocks), dim3(256), 0, (hipStream_t)s, a, b, n16); break;
    case 4: hipLaunchKernelGGL(k_stream_copy<4>, dim3(blocks), dim3(256), 0, (hipStream_t)s, a, b, n16); break;
    case 8: hipLaunchKernelGGL(k_stream_copy<8>, dim3(blocks), dim3(256), 0, (hipStream_t)s, a, b, n16); break;
    default: return -2;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ----------------------------------------------------------------------------
// Riemannian post-processing in FP64 (Sec. "Riemannian optimization"):
//   egrad = -conj(T)  (gradient convention d_x f + i d_y f for f = -Re h),
//   rgrad = P_G(egrad),  P_V Y = (Y - V Y^dagger V) / 2,
//   ehvp  = -conj(Tdot),
//   rhvp  = P_G(ehvp - X sym(G^dagger egrad)),  sym(A) = (A + A^dagger) / 2,
// summing instance derivatives per parameter (brick-wall sharing).
// ----------------------------------------------------------------------------
struct c64d {
  double x, y;
};

__device__ inline c64d cadd(c64d a, c64d b) { return {a.x + b.x, a.y + b.y}; }
__device__ inline c64d csub(c64d a, c64d b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline c64d cmulz(c64d a, c64d b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ inline c64d cconj(c64d a) { return {a.x, -a.y}; }

// C = A B (4x4)
__device__ inline void mm4(const c64d *A, const c64d *B, c64d *C) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      c64d s{0, 0};
      for (int k = 0; k < 4; ++k) s = cadd(s, cmulz(A[4 * i + k], B[4 * k + j]));
      C[4 * i + j] = s;
    }
}
__device__ inline void dag4(const c64d *A, c64d *B) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) B[4 * i + j] = cconj(A[4 * j + i]);
}
// P_V Y = (Y - V Y^dagger V) / 2
__device__ inline void proj4(const c64d *V, const c64d *Y, c64d *out) {
  c64d Yd[16], t[16], u[16];
  dag4(Y, Yd);
  mm4(V, Yd, t);
  mm4(t, V, u);
  for (int e = 0; e < 16; ++e) out[e] = {0.5 * (Y[e].x - u[e].x), 0.5 * (Y[e].y - u[e].y)};
}

__device__ const int kParityIdx[8] = {0, 3, 12, 15, 5, 6, 9, 10};

__device__ inline void unpack_T(const double *t, int parity, c64d *M) {
  for (int e = 0; e < 16; ++e) M[e] = {0, 0};
  if (parity) {
    for (int c = 0; c < 8; ++c) M[kParityIdx[c]] = {t[2 * c], t[2 * c + 1]};
  } else {
    for (int e = 0; e < 16; ++e) M[e] = {t[2 * e], t[2 * e + 1]};
  }
}

// parity: 0 U(4), 1 parity pattern, 2 particle-number pattern (the parity
// pattern without (0,3) and (3,0)).
__device__ inline void store4(double *dst, const c64d *M, int parity, int accumulate) {
  for (int e = 0; e < 16; ++e) {
    bool keep = true;
    if (parity) {
      keep = false;
      for (int c = 0; c < 8; ++c) keep |= (kParityIdx[c] == e);
      if (parity == 2 && (e == 3 || e == 12)) keep = false;
    }
    const double re = keep ? M[e].x : 0.0, im = keep ? M[e].y : 0.0;
    dst[2 * e] = accumulate ? dst[2 * e] + re : re;
    dst[2 * e + 1] = accumulate ? dst[2 * e + 1] + im : im;
  }
}

__global__ void k_post(int op, int parity, int accumulate, int P, int N, const int32_t *__restrict__ param_of,
                       const double *__restrict__ tsum, int ne, const double *__restrict__ fsum,
                       const double *__restrict__ gates64, const double *__restrict__ dir64,
                       double *d_f, double *d_egrad, double *d_rgrad, double *d_ehvp,
                       double *d_rhvp) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0 && d_f) d_f[0] = accumulate ? d_f[0] - fsum[0] : -fsum[0];
  if (p >= P || op == OP_COST) return;
  const int nt1 = parity ? 16 : 32;
  double t[32], td[32];
  for (int e = 0; e < 32; ++e) t[e] = td[e] = 0.0;
  for (int l = 0; l < N; ++l) {
    if (param_of[l] != p) continue;
    const double *s = tsum + int64_t(l) * ne;
    for (int e = 0; e < nt1; ++e) t[e] += s[e];
    if (op == OP_HVP)
      for (int e = 0; e < nt1; ++e) td[e] += s[nt1 + e];
  }
  c64d T[16], G[16], eg[16], rg[16];
  unpack_T(t, parity, T);
  for (int e = 0; e < 16; ++e) {
    G[e] = {gates64[(int64_t(p) * 16 + e) * 2], gates64[(int64_t(p) * 16 + e) * 2 + 1]};
    eg[e] = {-T[e].x, T[e].y};  // -conj(T)
  }
  proj4(G, eg, rg);
  if (d_egrad) store4(d_egrad + int64_t(p) * 32, eg, parity, accumulate);
  if (d_rgrad) store4(d_rgrad + int64_t(p) * 32, rg, parity, accumulate);
  if (op != OP_HVP) return;
  c64d Td[16], eh[16], X[16], Gd[16], S[16], sym[16], XS[16], Y[16], rh[16];
  unpack_T(td, parity, Td);
  for (int e = 0; e < 16; ++e) {
    eh[e] = {-Td[e].x, Td[e].y};
    X[e] = {dir64[(int64_t(p) * 16 + e) * 2], dir64[(int64_t(p) * 16 + e) * 2 + 1]};
  }
  dag4(G, Gd);
  mm4(Gd, eg, S);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const c64d a = S[4 * i + j], b = cconj(S[4 * j + i]);
      sym[4 * i + j] = {0.5 * (a.x + b.x), 0.5 * (a.y + b.y)};
    }
  mm4(X, sym, XS);
  for (int e = 0; e < 16; ++e) Y[e] = csub(eh[e], XS[e]);
  proj4(G, Y, rh);
  if (d_ehvp) store4(d_ehvp + int64_t(p) * 32, eh, parity, accumulate);
  if (d_rhvp) store4(d_rhvp + int64_t(p) * 32, rh, parity, accumulate);
}

int launch_post(int op, int parity, int accumulate, int n_params, int n_inst, const int32_t *param_of,
                const double *tsum, int ne, const double *fsum, int, const double *gates64,
                const double *dir64, double *d_f, double *d_egrad, double *d_rgrad,
                double *d_ehvp, double *d_rhvp, void *s) {
  const int threads = 64;
  const int blocks = (n_params + threads - 1) / threads > 0 ? (n_params + threads - 1) / threads : 1;
  hipLaunchKernelGGL(k_post, dim3(blocks), dim3(threads), 0, (hipStream_t)s, op, parity, accumulate, n_params,
                     n_inst, param_of, tsum, ne, fsum, gates64, dir64, d_f, d_egrad, d_rgrad,
                     d_ehvp, d_rhvp);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace rqk
