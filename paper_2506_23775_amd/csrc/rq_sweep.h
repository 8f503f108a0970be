// Sweep-pass kernels: forward gate application, the fused last pass (forward,
// overlap with the target columns, first backward pass) and backward passes
// with gate-hole contractions, for complex64 / complex128 states, dense or
// parity-conserving gates.
//
// Method (arXiv 2506.23775):
//  - forward pass psi_l = G_l psi_{l-1} with cached states (Sec. "Efficient
//    gradient and Hessian computation"), here cached at pass boundaries only;
//  - backward pass phi <- G_l^T phi with the gate hole of G_l contracted
//    between phi (output side) and psi_{l-1} (input side) (same section and
//    Sec. "Gate gradient as a gate hole");
//  - Hessian-vector products by forward-mode tangents (psi-dot, phi-dot) and
//    a second contraction (appendix on Hessian-vector products);
//  - parity-conserving gates act as two 2x2 blocks (Sec. "Parity-conserving
//    gate structure").
//
// GPU design.  State slabs S[x][c] keep the basis column c fastest, so lane c
// of a wavefront owns column c and every row access is a coalesced 64-column
// segment whatever qubits a gate touches.  A pass owns a tile of NT qubits:
// each lane keeps the 2^NT amplitudes of its column on those qubits in
// registers and applies every gate of the pass without data exchange.  In
// parity mode the implied qubit k-1 belongs to every tile for free.  Inside a
// backward pass the states before each gate are recovered by applying G^-1
// (from the checkpoint after the pass), so no per-gate state is stored.
// Contractions are summed per lane in the state precision over the lane's
// 2^(NT-2) groups, converted to FP64, reduced across the wavefront with a
// butterfly reduce-scatter and accumulated per wavefront in LDS; each
// wavefront flushes its FP64 partials to its own slot, and a fixed-order
// tree sums the slots (deterministic results for a given chunking).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "rq_internal.h"

namespace rqk {

template <typename R>
struct alignas(2 * sizeof(R)) cx {
  R x, y;
};

template <int V>
using ic = std::integral_constant<int, V>;

// y = c0 x0 + c1 x1
template <typename R>
__device__ __forceinline__ cx<R> mv2(cx<R> c0, cx<R> x0, cx<R> c1, cx<R> x1) {
  cx<R> y;
  y.x = c0.x * x0.x;
  y.x = fma(-c0.y, x0.y, y.x);
  y.x = fma(c1.x, x1.x, y.x);
  y.x = fma(-c1.y, x1.y, y.x);
  y.y = c0.x * x0.y;
  y.y = fma(c0.y, x0.x, y.y);
  y.y = fma(c1.x, x1.y, y.y);
  y.y = fma(c1.y, x1.x, y.y);
  return y;
}

// y += c x
template <typename R>
__device__ __forceinline__ void cfma(cx<R> &y, cx<R> c, cx<R> x) {
  y.x = fma(c.x, x.x, y.x);
  y.x = fma(-c.y, x.y, y.x);
  y.y = fma(c.x, x.y, y.y);
  y.y = fma(c.y, x.x, y.y);
}

// (re, im) += a b
template <typename R>
__device__ __forceinline__ void cacc(R &re, R &im, cx<R> a, cx<R> b) {
  re = fma(a.x, b.x, re);
  re = fma(-a.y, b.y, re);
  im = fma(a.x, b.y, im);
  im = fma(a.y, b.x, im);
}

template <typename R>
__device__ __forceinline__ cx<R> cld(const cx<R> *p, int64_t off, bool ok) {
  cx<R> z{R(0), R(0)};
  return ok ? p[off] : z;
}

template <typename R>
__device__ __forceinline__ void cst(cx<R> *p, int64_t off, bool ok, cx<R> v) {
  if (ok) p[off] = v;
}

// ----------------------------------------------------------------------------
// Compile-time iteration over the amplitude groups a gate couples.
// ----------------------------------------------------------------------------

// Dense gate on local bits (H, L): groups (i_0, i_1, i_2, i_3), i_a has
// (bit H, bit L) = (a >> 1, a & 1).
template <int NT, int H, int L, typename F>
__device__ __forceinline__ void for_groups(F &&f) {
#pragma unroll
  for (int i = 0; i < (1 << NT); ++i) {
    if (((i >> H) & 1) || ((i >> L) & 1)) continue;
    f(i, i | (1 << L), i | (1 << H), i | (1 << H) | (1 << L));
  }
}

// Parity gate: 2x2 blocks (i0, i1) with compact coefficient indices
// (c00, c01, c10, c11):  y_i0 = C[c00] x_i0 + C[c01] x_i1,
//                       y_i1 = C[c10] x_i0 + C[c11] x_i1.
// KIND 0: both qubits in the tile (local bits H, L).  KIND 1 / 2: the second
// / first qubit of the pair is the implied qubit k-1, whose bit equals
// PI ^ parity(local index) (PI = sector ^ parity of the tile's outer bits).
template <int NT, int KIND, int H, int L, int PI, typename F>
__device__ __forceinline__ void for_blocks(F &&f) {
#pragma unroll
  for (int i = 0; i < (1 << NT); ++i) {
    if constexpr (KIND == 0) {
      if (((i >> H) & 1) || ((i >> L) & 1)) continue;
      f(i, i | (1 << H) | (1 << L), 0, 1, 2, 3);
      f(i | (1 << L), i | (1 << H), 4, 5, 6, 7);
    } else {
      if ((i >> H) & 1) continue;
      const int beta = PI ^ (__builtin_popcount(i) & 1);
      if (beta == 0)
        f(i, i | (1 << H), 0, 1, 2, 3);
      else if (KIND == 1)
        f(i, i | (1 << H), 4, 5, 6, 7);
      else
        f(i, i | (1 << H), 7, 6, 5, 4);
    }
  }
}

template <int C, int NC, typename F>
__device__ __forceinline__ void dispatch(int code, F &&f) {
  if constexpr (C < NC) {
    if (code == C)
      f(ic<C>{});
    else
      dispatch<C + 1, NC>(code, f);
  }
}

template <int MODE, int NT>
struct Codes {
  static constexpr int n = MODE == MODE_DENSE ? NT * NT : NT * NT + 4 * NT;
  template <int C>
  static constexpr int kind() {
    return C < NT * NT ? 0 : 1 + (C - NT * NT) / (2 * NT);
  }
  template <int C>
  static constexpr int h() {
    return C < NT * NT ? C / NT : ((C - NT * NT) % (2 * NT)) / 2;
  }
  template <int C>
  static constexpr int l() {
    return C < NT * NT ? C % NT : 0;
  }
  template <int C>
  static constexpr int pi() {
    return C < NT * NT ? 0 : (C - NT * NT) % 2;
  }
  template <int C>
  static constexpr bool valid() {
    return kind<C>() != 0 || h<C>() != l<C>();
  }
};

__device__ __forceinline__ int gate_code(int mode, int nt, const GateRef &g, int pi) {
  if (mode == MODE_DENSE || g.kind == 0) return g.h * nt + g.l;
  return nt * nt + (g.kind - 1) * 2 * nt + g.h * 2 + pi;
}

// ----------------------------------------------------------------------------
// Gate steps.  coefficient blocks: G at +0, G^-1 at +16, Z at +32, G^-1 Z +48.
// ----------------------------------------------------------------------------

// Forward: psi <- G psi;  (HVP) dpsi <- G dpsi + Z psi.
template <typename R, int NT, int MODE, bool HV, int C>
__device__ __forceinline__ void fwd_gate(cx<R> *ps, cx<R> *dps, const cx<R> *co) {
  using K = Codes<MODE, NT>;
  if constexpr (K::template valid<C>()) {
    constexpr int H = K::template h<C>(), L = K::template l<C>();
    if constexpr (MODE == MODE_DENSE) {
      cx<R> g[16], z[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) g[e] = co[e];
      if constexpr (HV) {
#pragma unroll
        for (int e = 0; e < 16; ++e) z[e] = co[32 + e];
      }
      for_groups<NT, H, L>([&](int i0, int i1, int i2, int i3) {
        const cx<R> x[4] = {ps[i0], ps[i1], ps[i2], ps[i3]};
        const int id[4] = {i0, i1, i2, i3};
        if constexpr (HV) {
          const cx<R> xd[4] = {dps[i0], dps[i1], dps[i2], dps[i3]};
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            cx<R> y = mv2(g[4 * a], xd[0], g[4 * a + 1], xd[1]);
            cfma(y, g[4 * a + 2], xd[2]);
            cfma(y, g[4 * a + 3], xd[3]);
            cfma(y, z[4 * a], x[0]);
            cfma(y, z[4 * a + 1], x[1]);
            cfma(y, z[4 * a + 2], x[2]);
            cfma(y, z[4 * a + 3], x[3]);
            dps[id[a]] = y;
          }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          cx<R> y = mv2(g[4 * a], x[0], g[4 * a + 1], x[1]);
          cfma(y, g[4 * a + 2], x[2]);
          cfma(y, g[4 * a + 3], x[3]);
          ps[id[a]] = y;
        }
      });
    } else {
      constexpr int KD = K::template kind<C>(), PI = K::template pi<C>();
      cx<R> g[8], z[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) g[e] = co[e];
      if constexpr (HV) {
#pragma unroll
        for (int e = 0; e < 8; ++e) z[e] = co[32 + e];
      }
      for_blocks<NT, KD, H, L, PI>([&](int i0, int i1, int c00, int c01, int c10, int c11) {
        const cx<R> x0 = ps[i0], x1 = ps[i1];
        if constexpr (HV) {
          const cx<R> d0 = dps[i0], d1 = dps[i1];
          cx<R> y0 = mv2(g[c00], d0, g[c01], d1);
          cfma(y0, z[c00], x0);
          cfma(y0, z[c01], x1);
          cx<R> y1 = mv2(g[c10], d0, g[c11], d1);
          cfma(y1, z[c10], x0);
          cfma(y1, z[c11], x1);
          dps[i0] = y0;
          dps[i1] = y1;
        }
        ps[i0] = mv2(g[c00], x0, g[c01], x1);
        ps[i1] = mv2(g[c10], x0, g[c11], x1);
      });
    }
  }
}

// Backward through one gate.  On entry ps/dps hold the states after the
// gate and ph/dph the backward states at the gate's output side.  On exit
// ps/dps hold the states before the gate (x = G^-1 psi,
// xd = G^-1 dpsi - G^-1 Z x) and ph/dph the states at its input side
// (phi <- G^T phi, dphi <- G^T dphi + Z^T phi); tp accumulates the hole
// contractions T[a][b] += phi[a] x[b] (and Tdot += dphi[a] x[b] + phi[a] xd[b]).
template <typename R, int NT, int MODE, bool HV, int C, int NE>
__device__ __forceinline__ void bwd_gate(cx<R> *ps, cx<R> *dps, cx<R> *ph, cx<R> *dph,
                                         const cx<R> *co, R *tp) {
  using K = Codes<MODE, NT>;
  constexpr int TD = MODE == MODE_DENSE ? 32 : 16;  // offset of Tdot in tp
  if constexpr (K::template valid<C>()) {
    constexpr int H = K::template h<C>(), L = K::template l<C>();
    if constexpr (MODE == MODE_DENSE) {
      cx<R> g[16], gi[16], z[16], giz[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        g[e] = co[e];
        gi[e] = co[16 + e];
      }
      if constexpr (HV) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          z[e] = co[32 + e];
          giz[e] = co[48 + e];
        }
      }
      for_groups<NT, H, L>([&](int i0, int i1, int i2, int i3) {
        const int id[4] = {i0, i1, i2, i3};
        cx<R> x[4], xd[4], p[4], pd[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          cx<R> y = mv2(gi[4 * a], ps[i0], gi[4 * a + 1], ps[i1]);
          cfma(y, gi[4 * a + 2], ps[i2]);
          cfma(y, gi[4 * a + 3], ps[i3]);
          x[a] = y;
          p[a] = ph[id[a]];
        }
        if constexpr (HV) {
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            cx<R> y = mv2(gi[4 * a], dps[i0], gi[4 * a + 1], dps[i1]);
            cfma(y, gi[4 * a + 2], dps[i2]);
            cfma(y, gi[4 * a + 3], dps[i3]);
            cx<R> m = mv2(giz[4 * a], x[0], giz[4 * a + 1], x[1]);
            cfma(m, giz[4 * a + 2], x[2]);
            cfma(m, giz[4 * a + 3], x[3]);
            y.x -= m.x;
            y.y -= m.y;
            xd[a] = y;
            pd[a] = dph[id[a]];
          }
        }
        // contractions
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int e = 2 * (4 * a + b);
            cacc(tp[e], tp[e + 1], p[a], x[b]);
            if constexpr (HV) {
              cacc(tp[TD + e], tp[TD + e + 1], pd[a], x[b]);
              cacc(tp[TD + e], tp[TD + e + 1], p[a], xd[b]);
            }
          }
        }
        // backward states: phi <- G^T phi ; dphi <- G^T dphi + Z^T phi
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          cx<R> y = mv2(g[a], p[0], g[4 + a], p[1]);
          cfma(y, g[8 + a], p[2]);
          cfma(y, g[12 + a], p[3]);
          ph[id[a]] = y;
          ps[id[a]] = x[a];
          if constexpr (HV) {
            cx<R> yd = mv2(g[a], pd[0], g[4 + a], pd[1]);
            cfma(yd, g[8 + a], pd[2]);
            cfma(yd, g[12 + a], pd[3]);
            cfma(yd, z[a], p[0]);
            cfma(yd, z[4 + a], p[1]);
            cfma(yd, z[8 + a], p[2]);
            cfma(yd, z[12 + a], p[3]);
            dph[id[a]] = yd;
            dps[id[a]] = xd[a];
          }
        }
      });
    } else {
      constexpr int KD = K::template kind<C>(), PI = K::template pi<C>();
      cx<R> g[8], gi[8], z[8], giz[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        g[e] = co[e];
        gi[e] = co[16 + e];
      }
      if constexpr (HV) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          z[e] = co[32 + e];
          giz[e] = co[48 + e];
        }
      }
      for_blocks<NT, KD, H, L, PI>([&](int i0, int i1, int c00, int c01, int c10, int c11) {
        const cx<R> x0 = mv2(gi[c00], ps[i0], gi[c01], ps[i1]);
        const cx<R> x1 = mv2(gi[c10], ps[i0], gi[c11], ps[i1]);
        const cx<R> p0 = ph[i0], p1 = ph[i1];
        cacc(tp[2 * c00], tp[2 * c00 + 1], p0, x0);
        cacc(tp[2 * c01], tp[2 * c01 + 1], p0, x1);
        cacc(tp[2 * c10], tp[2 * c10 + 1], p1, x0);
        cacc(tp[2 * c11], tp[2 * c11 + 1], p1, x1);
        if constexpr (HV) {
          cx<R> xd0 = mv2(gi[c00], dps[i0], gi[c01], dps[i1]);
          cx<R> xd1 = mv2(gi[c10], dps[i0], gi[c11], dps[i1]);
          const cx<R> m0 = mv2(giz[c00], x0, giz[c01], x1);
          const cx<R> m1 = mv2(giz[c10], x0, giz[c11], x1);
          xd0.x -= m0.x;
          xd0.y -= m0.y;
          xd1.x -= m1.x;
          xd1.y -= m1.y;
          const cx<R> q0 = dph[i0], q1 = dph[i1];
          cacc(tp[TD + 2 * c00], tp[TD + 2 * c00 + 1], q0, x0);
          cacc(tp[TD + 2 * c01], tp[TD + 2 * c01 + 1], q0, x1);
          cacc(tp[TD + 2 * c10], tp[TD + 2 * c10 + 1], q1, x0);
          cacc(tp[TD + 2 * c11], tp[TD + 2 * c11 + 1], q1, x1);
          cacc(tp[TD + 2 * c00], tp[TD + 2 * c00 + 1], p0, xd0);
          cacc(tp[TD + 2 * c01], tp[TD + 2 * c01 + 1], p0, xd1);
          cacc(tp[TD + 2 * c10], tp[TD + 2 * c10 + 1], p1, xd0);
          cacc(tp[TD + 2 * c11], tp[TD + 2 * c11 + 1], p1, xd1);
          cx<R> y0 = mv2(g[c00], q0, g[c10], q1);
          cfma(y0, z[c00], p0);
          cfma(y0, z[c10], p1);
          cx<R> y1 = mv2(g[c01], q0, g[c11], q1);
          cfma(y1, z[c01], p0);
          cfma(y1, z[c11], p1);
          dph[i0] = y0;
          dph[i1] = y1;
          dps[i0] = xd0;
          dps[i1] = xd1;
        }
        ph[i0] = mv2(g[c00], p0, g[c10], p1);
        ph[i1] = mv2(g[c01], p0, g[c11], p1);
        ps[i0] = x0;
        ps[i1] = x1;
      });
    }
  }
}

// ----------------------------------------------------------------------------
// FP64 wavefront reduce-scatter of V per-lane values.  After the call, lane L
// (with bits >= log2(V) clear) holds the wavefront sum of entry e(L), where
// e(L) reverses the low log2(V) bits of L.
// ----------------------------------------------------------------------------
template <int V>
__device__ __forceinline__ constexpr int ilog2() {
  return V <= 1 ? 0 : 1 + ilog2<V / 2>();
}

__device__ __forceinline__ int entry_of_lane(int lane, int lv) {
  int e = 0;
  for (int s = 0; s < lv; ++s) e |= ((lane >> s) & 1) << (lv - 1 - s);
  return e;
}

template <typename R, int V>
__device__ __forceinline__ double wave_reduce_scatter(const R *tp, int lane) {
  constexpr int LV = ilog2<V>();
  double v[V / 2];
  {
    const bool hi = lane & 1;
#pragma unroll
    for (int i = 0; i < V / 2; ++i) {
      const double a = (double)tp[i], b = (double)tp[i + V / 2];
      const double keep = hi ? b : a, send = hi ? a : b;
      v[i] = keep + __shfl_xor(send, 1, 64);
    }
  }
#pragma unroll
  for (int s = 1; s < LV; ++s) {
    const int n = V >> s;
    const bool hi = (lane >> s) & 1;
#pragma unroll
    for (int i = 0; i < n / 2; ++i) {
      const double a = v[i], b = v[i + n / 2];
      const double keep = hi ? b : a, send = hi ? a : b;
      v[i] = keep + __shfl_xor(send, 1 << s, 64);
    }
  }
  double r = v[0];
#pragma unroll
  for (int s = LV; s < 6; ++s) r += __shfl_xor(r, 1 << s, 64);
  return r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int s = 0; s < 6; ++s) v += __shfl_xor(v, 1 << s, 64);
  return v;
}

// ----------------------------------------------------------------------------
// The sweep kernel.
// ----------------------------------------------------------------------------
template <typename R, int NT, int MODE, int OP, int STAGE>
__global__ __launch_bounds__(kBlock) void k_pass(const PassArgs A) {
  constexpr int NA = 1 << NT;
  constexpr bool HV = OP == OP_HVP;
  constexpr bool NEEDB = STAGE != ST_FWD && (OP == OP_GRAD || OP == OP_HVP);
  constexpr bool NEEDF = STAGE != ST_BWD;
  constexpr int NT1 = MODE == MODE_DENSE ? 32 : 16;
  constexpr int NE = HV ? 2 * NT1 : NT1;
  constexpr int LV = ilog2<NE>();
  using K = Codes<MODE, NT>;
  extern __shared__ double lds[];

  const int lane = threadIdx.x & 63;
  const int wib = threadIdx.x >> 6;
  const int gwave = blockIdx.x * (kBlock / 64) + wib;
  const int nwaves = gridDim.x * (kBlock / 64);
  double *acc = lds + wib * (kMaxGates * NE);
  const int my_e = entry_of_lane(lane, LV);
  const bool writer = (lane >> LV) == 0;
  if constexpr (NEEDB) {
    for (int g = 0; g < A.ngates; ++g)
      if (writer) acc[g * NE + my_e] = 0.0;
  }
  double facc = 0.0;

  const cx<R> *coef = reinterpret_cast<const cx<R> *>(A.coef);
  int64_t lr[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    int64_t r = 0;
#pragma unroll
    for (int b = 0; b < NT; ++b)
      if ((i >> b) & 1) r |= int64_t(1) << A.pos[b];
    lr[i] = r;
  }

  for (int item = gwave; item < A.n_items; item += nwaves) {
    const int cg = item % A.ncg;
    const int tile = item / A.ncg;
    const int c = cg * 64 + lane;
    const bool ok = c < A.ncols;
    int64_t base = 0;
    {
      int t = tile;
      for (int p = 0; p < A.kq; ++p)
        if (!((A.qmask >> p) & 1)) {
          base |= int64_t(t & 1) << p;
          t >>= 1;
        }
    }
    const int pi = MODE == MODE_PARITY ? ((A.sector ^ __builtin_popcountll(base)) & 1) : 0;
    const int64_t rb = base * A.ld + c;

    cx<R> ps[NA], dps[NA], ph[NA], dph[NA];
    if constexpr (NEEDF) {
      if (A.src_psi) {
        const cx<R> *s = reinterpret_cast<const cx<R> *>(A.src_psi);
#pragma unroll
        for (int i = 0; i < NA; ++i) ps[i] = cld(s, rb + lr[i] * A.ld, ok);
      } else {
        const int64_t tgt = A.col0 + c - base;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
          ps[i].x = (ok && lr[i] == tgt) ? R(1) : R(0);
          ps[i].y = R(0);
        }
      }
      if constexpr (HV) {
        if (A.src_dpsi) {
          const cx<R> *s = reinterpret_cast<const cx<R> *>(A.src_dpsi);
#pragma unroll
          for (int i = 0; i < NA; ++i) dps[i] = cld(s, rb + lr[i] * A.ld, ok);
        } else {
#pragma unroll
          for (int i = 0; i < NA; ++i) dps[i] = cx<R>{R(0), R(0)};
        }
      }
      for (int g = 0; g < A.ngates; ++g) {
        const GateRef gr = A.gates[g];
        const cx<R> *co = coef + int64_t(gr.inst) * kCoefStride;
        dispatch<0, K::n>(gate_code(MODE, NT, gr, pi),
                          [&](auto CC) { fwd_gate<R, NT, MODE, HV, decltype(CC)::value>(ps, dps, co); });
      }
      if constexpr (STAGE == ST_FWD) {
        cx<R> *d = reinterpret_cast<cx<R> *>(A.dst_psi);
#pragma unroll
        for (int i = 0; i < NA; ++i) cst(d, rb + lr[i] * A.ld, ok, ps[i]);
        if constexpr (HV) {
          cx<R> *dd = reinterpret_cast<cx<R> *>(A.dst_dpsi);
#pragma unroll
          for (int i = 0; i < NA; ++i) cst(dd, rb + lr[i] * A.ld, ok, dps[i]);
        }
      }
    } else {
      const cx<R> *s = reinterpret_cast<const cx<R> *>(A.ckpt_psi);
#pragma unroll
      for (int i = 0; i < NA; ++i) ps[i] = cld(s, rb + lr[i] * A.ld, ok);
      if constexpr (HV) {
        const cx<R> *sd = reinterpret_cast<const cx<R> *>(A.ckpt_dpsi);
#pragma unroll
        for (int i = 0; i < NA; ++i) dps[i] = cld(sd, rb + lr[i] * A.ld, ok);
      }
    }

    if constexpr (STAGE == ST_LAST) {
      // phi_0 = conj(U|j>), overlap h_j = sum_x phi_0[x] psi_N[x]
      const cx<R> *u = reinterpret_cast<const cx<R> *>(A.ref);
      const int64_t ub = base * A.ld_ref + A.col0 + c;
      R hre = R(0);
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        cx<R> v = cld(u, ub + lr[i] * A.ld_ref, ok);
        ph[i].x = v.x;
        ph[i].y = -v.y;
        hre = fma(ph[i].x, ps[i].x, hre);
        hre = fma(-ph[i].y, ps[i].y, hre);
        if constexpr (HV) dph[i] = cx<R>{R(0), R(0)};
      }
      facc += (double)hre;
    } else if constexpr (STAGE == ST_BWD) {
      const cx<R> *p = reinterpret_cast<const cx<R> *>(A.phi);
#pragma unroll
      for (int i = 0; i < NA; ++i) ph[i] = cld(p, rb + lr[i] * A.ld, ok);
      if constexpr (HV) {
        const cx<R> *pd = reinterpret_cast<const cx<R> *>(A.dphi);
#pragma unroll
        for (int i = 0; i < NA; ++i) dph[i] = cld(pd, rb + lr[i] * A.ld, ok);
      }
    }

    if constexpr (NEEDB) {
      for (int g = A.ngates - 1; g >= 0; --g) {
        const GateRef gr = A.gates[g];
        const cx<R> *co = coef + int64_t(gr.inst) * kCoefStride;
        R tp[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) tp[e] = R(0);
        dispatch<0, K::n>(gate_code(MODE, NT, gr, pi), [&](auto CC) {
          bwd_gate<R, NT, MODE, HV, decltype(CC)::value, NE>(ps, dps, ph, dph, co, tp);
        });
        const double r = wave_reduce_scatter<R, NE>(tp, lane);
        if (writer) acc[g * NE + my_e] += r;
      }
      if (A.store_phi) {
        cx<R> *p = reinterpret_cast<cx<R> *>(A.phi);
#pragma unroll
        for (int i = 0; i < NA; ++i) cst(p, rb + lr[i] * A.ld, ok, ph[i]);
        if constexpr (HV) {
          cx<R> *pd = reinterpret_cast<cx<R> *>(A.dphi);
#pragma unroll
          for (int i = 0; i < NA; ++i) cst(pd, rb + lr[i] * A.ld, ok, dph[i]);
        }
      }
    }
  }

  if constexpr (NEEDB) {
    if (writer) {
      for (int g = 0; g < A.ngates; ++g) {
        double *s = A.slots + (int64_t(A.gates[g].inst) * A.ne + my_e) * A.nslots + gwave;
        *s += acc[g * NE + my_e];
      }
    }
  }
  if constexpr (STAGE == ST_LAST) {
    const double f = wave_sum(facc);
    if (lane == 0) A.fslots[gwave] += f;
  }
}

// ----------------------------------------------------------------------------
// Host launchers.
// ----------------------------------------------------------------------------
template <typename R, int NT, int MODE, int OP, int STAGE>
static int launch_one(const PassArgs &a, int grid, void *stream) {
  constexpr bool HV = OP == OP_HVP;
  constexpr bool NEEDB = STAGE != ST_FWD && (OP == OP_GRAD || OP == OP_HVP);
  constexpr int NT1 = MODE == MODE_DENSE ? 32 : 16;
  constexpr int NE = HV ? 2 * NT1 : NT1;
  const size_t lds = NEEDB ? size_t(kBlock / 64) * kMaxGates * NE * sizeof(double) : 0;
  hipLaunchKernelGGL((k_pass<R, NT, MODE, OP, STAGE>), dim3(grid), dim3(kBlock), lds,
                     (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Launch every (op, stage) instantiation listed by OPS for one (R, NT, mode).
template <typename R, int NT, int MODE, bool COST, bool GRAD, bool HVP>
static int launch_mode(int op, int stage, const PassArgs &a, int grid, void *s) {
  if (COST && (op == OP_COST || op == OP_APPLY)) {
    if (stage == ST_FWD) return launch_one<R, NT, MODE, OP_COST, ST_FWD>(a, grid, s);
    if (stage == ST_LAST && op == OP_COST) return launch_one<R, NT, MODE, OP_COST, ST_LAST>(a, grid, s);
  }
  if constexpr (GRAD) {
    if (op == OP_GRAD) {
      if (stage == ST_FWD) return launch_one<R, NT, MODE, OP_GRAD, ST_FWD>(a, grid, s);
      if (stage == ST_LAST) return launch_one<R, NT, MODE, OP_GRAD, ST_LAST>(a, grid, s);
      if (stage == ST_BWD) return launch_one<R, NT, MODE, OP_GRAD, ST_BWD>(a, grid, s);
    }
  }
  if constexpr (HVP) {
    if (op == OP_HVP) {
      if (stage == ST_FWD) return launch_one<R, NT, MODE, OP_HVP, ST_FWD>(a, grid, s);
      if (stage == ST_LAST) return launch_one<R, NT, MODE, OP_HVP, ST_LAST>(a, grid, s);
      if (stage == ST_BWD) return launch_one<R, NT, MODE, OP_HVP, ST_BWD>(a, grid, s);
    }
  }
  return -2;
}

template <typename R, int NT, bool COST, bool GRAD, bool HVP>
static int launch_nt(int mode, int op, int stage, const PassArgs &a, int grid, void *s) {
  return mode == MODE_DENSE
             ? launch_mode<R, NT, MODE_DENSE, COST, GRAD, HVP>(op, stage, a, grid, s)
             : launch_mode<R, NT, MODE_PARITY, COST, GRAD, HVP>(op, stage, a, grid, s);
}

}  // namespace rqk
