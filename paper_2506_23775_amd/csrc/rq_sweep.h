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
//
// Every index into a register array is a compile-time constant (static_for
// recursion below), so the tile never leaves the register file.
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

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(ic<B>{});
    static_for<B + 1, E>(f);
  }
}

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

// Gate coefficients are uniform and never written while a sweep kernel runs:
// read them through the constant address space so they become scalar loads
// (SGPR operands) instead of occupying vector registers.
template <typename R>
using ccoef_t = const __attribute__((address_space(4))) cx<R>;

template <typename R>
__device__ __forceinline__ ccoef_t<R> *as_const_coef(const void *p) {
  return (ccoef_t<R> *)(uintptr_t)p;
}

template <typename R>
__device__ __forceinline__ cx<R> ldco(ccoef_t<R> *p, int i) {
  cx<R> v;
  v.x = p[i].x;
  v.y = p[i].y;
  return v;
}

// Row-segment access: `row` points at element (x, 0) of a slab (uniform);
// voff is the lane's byte offset of column c (32-bit, per lane).
template <typename R>
__device__ __forceinline__ cx<R> ldrow(const char *row, uint32_t voff) {
  return *reinterpret_cast<const cx<R> *>(row + voff);
}
template <typename R>
__device__ __forceinline__ void strow(char *row, uint32_t voff, cx<R> v) {
  *reinterpret_cast<cx<R> *>(row + voff) = v;
}

// ----------------------------------------------------------------------------
// Compile-time iteration over the amplitude groups a gate couples.
// ----------------------------------------------------------------------------

// Dense gate on local bits (H, L): groups (i_0, i_1, i_2, i_3), i_a has
// (bit H, bit L) = (a >> 1, a & 1).  f receives integral constants.
template <int NT, int H, int L, typename F>
__device__ __forceinline__ void for_groups(F &&f) {
  static_for<0, (1 << NT)>([&](auto I) __attribute__((always_inline)) {
    constexpr int i = decltype(I)::value;
    if constexpr (!((i >> H) & 1) && !((i >> L) & 1))
      f(ic<i>{}, ic<(i | (1 << L))>{}, ic<(i | (1 << H))>{}, ic<(i | (1 << H) | (1 << L))>{});
  });
}

// Parity gate: 2x2 blocks (i0, i1) with compact coefficient indices
// (c00, c01, c10, c11):  y_i0 = C[c00] x_i0 + C[c01] x_i1,
//                       y_i1 = C[c10] x_i0 + C[c11] x_i1.
// Compact order of the 8 pattern entries: (0,0),(0,3),(3,0),(3,3),
// (1,1),(1,2),(2,1),(2,2).
// KIND 0: both qubits in the tile (local bits H, L).  KIND 1 / 2: the second
// / first qubit of the pair is the implied qubit k-1, whose bit equals
// PI ^ parity(local index) (PI = sector ^ parity of the tile's outer bits).
template <int NT, int KIND, int H, int L, int PI, typename F>
__device__ __forceinline__ void for_blocks(F &&f) {
  static_for<0, (1 << NT)>([&](auto I) __attribute__((always_inline)) {
    constexpr int i = decltype(I)::value;
    if constexpr (KIND == 0) {
      if constexpr (!((i >> H) & 1) && !((i >> L) & 1)) {
        f(ic<i>{}, ic<(i | (1 << H) | (1 << L))>{}, ic<0>{}, ic<1>{}, ic<2>{}, ic<3>{});
        f(ic<(i | (1 << L))>{}, ic<(i | (1 << H))>{}, ic<4>{}, ic<5>{}, ic<6>{}, ic<7>{});
      }
    } else {
      if constexpr (!((i >> H) & 1)) {
        constexpr int beta = PI ^ (__builtin_popcount(i) & 1);
        if constexpr (beta == 0)
          f(ic<i>{}, ic<(i | (1 << H))>{}, ic<0>{}, ic<1>{}, ic<2>{}, ic<3>{});
        else if constexpr (KIND == 1)
          f(ic<i>{}, ic<(i | (1 << H))>{}, ic<4>{}, ic<5>{}, ic<6>{}, ic<7>{});
        else
          f(ic<i>{}, ic<(i | (1 << H))>{}, ic<7>{}, ic<6>{}, ic<5>{}, ic<4>{});
      }
    }
  });
}

// Runtime gate code -> compile-time specialisation.  The empty asm markers
// (distinct per case) keep the compiler from merging the cases' register-
// array accesses into one access with a runtime index, which would move the
// tile out of registers.
template <int C, int NC, typename F>
__device__ __forceinline__ void dispatch(int code, F &&f) {
  if constexpr (C < NC) {
    if (code == C) {
      asm volatile("; gate case begin %0" ::"i"(C));
      f(ic<C>{});
      asm volatile("; gate case end %0" ::"i"(C));
    } else {
      dispatch<C + 1, NC>(code, f);
    }
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

#define CV(x) decltype(x)::value

// ----------------------------------------------------------------------------
// Gate steps.  coefficient blocks: G at +0, G^-1 at +16, Z at +32, G^-1 Z +48.
// ----------------------------------------------------------------------------

// Forward: psi <- G psi;  (HVP) dpsi <- G dpsi + Z psi.
template <typename R, int NT, int MODE, bool HV, int C, int NA>
__device__ __forceinline__ void fwd_gate(cx<R> (&ps)[NA], cx<R> (&dps)[NA], ccoef_t<R> *co) {
  using K = Codes<MODE, NT>;
  if constexpr (K::template valid<C>()) {
    constexpr int H = K::template h<C>(), L = K::template l<C>();
    if constexpr (MODE == MODE_DENSE) {
      cx<R> g[16], z[16];
      static_for<0, 16>([&](auto E) __attribute__((always_inline)) { g[CV(E)] = ldco<R>(co, CV(E)); });
      if constexpr (HV)
        static_for<0, 16>([&](auto E) __attribute__((always_inline)) { z[CV(E)] = ldco<R>(co, 32 + CV(E)); });
      for_groups<NT, H, L>([&](auto I0, auto I1, auto I2, auto I3) __attribute__((always_inline)) {
        constexpr int id[4] = {CV(I0), CV(I1), CV(I2), CV(I3)};
        const cx<R> x[4] = {ps[id[0]], ps[id[1]], ps[id[2]], ps[id[3]]};
        if constexpr (HV) {
          const cx<R> xd[4] = {dps[id[0]], dps[id[1]], dps[id[2]], dps[id[3]]};
          static_for<0, 4>([&](auto A) __attribute__((always_inline)) {
            constexpr int a = CV(A);
            cx<R> y = mv2(g[4 * a], xd[0], g[4 * a + 1], xd[1]);
            cfma(y, g[4 * a + 2], xd[2]);
            cfma(y, g[4 * a + 3], xd[3]);
            cfma(y, z[4 * a], x[0]);
            cfma(y, z[4 * a + 1], x[1]);
            cfma(y, z[4 * a + 2], x[2]);
            cfma(y, z[4 * a + 3], x[3]);
            dps[id[a]] = y;
          });
        }
        static_for<0, 4>([&](auto A) __attribute__((always_inline)) {
          constexpr int a = CV(A);
          cx<R> y = mv2(g[4 * a], x[0], g[4 * a + 1], x[1]);
          cfma(y, g[4 * a + 2], x[2]);
          cfma(y, g[4 * a + 3], x[3]);
          ps[id[a]] = y;
        });
      });
    } else {
      constexpr int KD = K::template kind<C>(), PI = K::template pi<C>();
      cx<R> g[8], z[8];
      static_for<0, 8>([&](auto E) __attribute__((always_inline)) { g[CV(E)] = ldco<R>(co, CV(E)); });
      if constexpr (HV)
        static_for<0, 8>([&](auto E) __attribute__((always_inline)) { z[CV(E)] = ldco<R>(co, 32 + CV(E)); });
      for_blocks<NT, KD, H, L, PI>([&](auto J0, auto J1, auto C00, auto C01, auto C10,
                                       auto C11) __attribute__((always_inline)) {
        constexpr int i0 = CV(J0), i1 = CV(J1);
        constexpr int c00 = CV(C00), c01 = CV(C01), c10 = CV(C10), c11 = CV(C11);
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
template <typename R, int NT, int MODE, bool HV, int C, int NE, int NA>
__device__ __forceinline__ void bwd_gate(cx<R> (&ps)[NA], cx<R> (&dps)[NA], cx<R> (&ph)[NA],
                                         cx<R> (&dph)[NA], ccoef_t<R> *co, R (&tp)[NE]) {
  using K = Codes<MODE, NT>;
  constexpr int TD = MODE == MODE_DENSE ? 32 : 16;  // offset of Tdot in tp
  if constexpr (K::template valid<C>()) {
    constexpr int H = K::template h<C>(), L = K::template l<C>();
    if constexpr (MODE == MODE_DENSE) {
      cx<R> g[16], gi[16], z[16], giz[16];
      static_for<0, 16>([&](auto E) __attribute__((always_inline)) {
        g[CV(E)] = ldco<R>(co, CV(E));
        gi[CV(E)] = ldco<R>(co, 16 + CV(E));
        if constexpr (HV) {
          z[CV(E)] = ldco<R>(co, 32 + CV(E));
          giz[CV(E)] = ldco<R>(co, 48 + CV(E));
        }
      });
      for_groups<NT, H, L>([&](auto I0, auto I1, auto I2, auto I3) __attribute__((always_inline)) {
        constexpr int id[4] = {CV(I0), CV(I1), CV(I2), CV(I3)};
        cx<R> x[4], xd[4], p[4], pd[4];
        static_for<0, 4>([&](auto A) __attribute__((always_inline)) {
          constexpr int a = CV(A);
          cx<R> y = mv2(gi[4 * a], ps[id[0]], gi[4 * a + 1], ps[id[1]]);
          cfma(y, gi[4 * a + 2], ps[id[2]]);
          cfma(y, gi[4 * a + 3], ps[id[3]]);
          x[a] = y;
          p[a] = ph[id[a]];
        });
        if constexpr (HV) {
          static_for<0, 4>([&](auto A) __attribute__((always_inline)) {
            constexpr int a = CV(A);
            cx<R> y = mv2(gi[4 * a], dps[id[0]], gi[4 * a + 1], dps[id[1]]);
            cfma(y, gi[4 * a + 2], dps[id[2]]);
            cfma(y, gi[4 * a + 3], dps[id[3]]);
            cx<R> m = mv2(giz[4 * a], x[0], giz[4 * a + 1], x[1]);
            cfma(m, giz[4 * a + 2], x[2]);
            cfma(m, giz[4 * a + 3], x[3]);
            y.x -= m.x;
            y.y -= m.y;
            xd[a] = y;
            pd[a] = dph[id[a]];
          });
        }
        static_for<0, 16>([&](auto AB) __attribute__((always_inline)) {
          constexpr int a = CV(AB) / 4, b = CV(AB) % 4, e = 2 * CV(AB);
          cacc(tp[e], tp[e + 1], p[a], x[b]);
          if constexpr (HV) {
            cacc(tp[TD + e], tp[TD + e + 1], pd[a], x[b]);
            cacc(tp[TD + e], tp[TD + e + 1], p[a], xd[b]);
          }
        });
        static_for<0, 4>([&](auto A) __attribute__((always_inline)) {
          constexpr int a = CV(A);
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
        });
      });
    } else {
      constexpr int KD = K::template kind<C>(), PI = K::template pi<C>();
      cx<R> g[8], gi[8], z[8], giz[8];
      static_for<0, 8>([&](auto E) __attribute__((always_inline)) {
        g[CV(E)] = ldco<R>(co, CV(E));
        gi[CV(E)] = ldco<R>(co, 16 + CV(E));
        if constexpr (HV) {
          z[CV(E)] = ldco<R>(co, 32 + CV(E));
          giz[CV(E)] = ldco<R>(co, 48 + CV(E));
        }
      });
      for_blocks<NT, KD, H, L, PI>([&](auto J0, auto J1, auto C00, auto C01, auto C10,
                                       auto C11) __attribute__((always_inline)) {
        constexpr int i0 = CV(J0), i1 = CV(J1);
        constexpr int c00 = CV(C00), c01 = CV(C01), c10 = CV(C10), c11 = CV(C11);
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

template <int S, int LV, int V>
__device__ __forceinline__ void rs_steps(double (&v)[V / 2], int lane) {
  if constexpr (S < LV) {
    constexpr int n = V >> S;
    const bool hi = (lane >> S) & 1;
    static_for<0, n / 2>([&](auto I) __attribute__((always_inline)) {
      constexpr int i = CV(I);
      const double a = v[i], b = v[i + n / 2];
      const double keep = hi ? b : a, send = hi ? a : b;
      v[i] = keep + __shfl_xor(send, 1 << S, 64);
    });
    rs_steps<S + 1, LV, V>(v, lane);
  }
}

template <typename R, int V>
__device__ __forceinline__ double wave_reduce_scatter(const R (&tp)[V], int lane) {
  constexpr int LV = ilog2<V>();
  double v[V / 2];
  {
    const bool hi = lane & 1;
    static_for<0, V / 2>([&](auto I) __attribute__((always_inline)) {
      constexpr int i = CV(I);
      const double a = (double)tp[i], b = (double)tp[i + V / 2];
      const double keep = hi ? b : a, send = hi ? a : b;
      v[i] = keep + __shfl_xor(send, 1, 64);
    });
  }
  rs_steps<1, LV, V>(v, lane);
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
// Target wavefronts per SIMD of a sweep instantiation: 512 registers per lane
// divided by the live tile states, the contraction accumulators and a fixed
// allowance for addresses, coefficients in flight and temporaries.
template <typename R, int NT, int MODE, int OP, int STAGE>
struct Occupancy {
  static constexpr int words = sizeof(R) / 4;
  static constexpr int nst = STAGE == ST_FWD ? (OP == OP_HVP ? 2 : 1)
                                              : (OP == OP_HVP ? 4 : (OP == OP_GRAD ? 2 : 1));
  static constexpr int acc = (STAGE != ST_FWD && OP != OP_COST)
                                 ? (MODE == MODE_DENSE ? 32 : 16) * (OP == OP_HVP ? 2 : 1) * words
                                 : 0;
  static constexpr int regs = (1 << NT) * 2 * words * nst + acc + 80;
  static constexpr int w = 512 / (regs + regs / 4);
  // Backward-type kernels keep the compiler's own allocation: at two waves per
  // SIMD they would spill to scratch memory.
  static constexpr int value = STAGE != ST_FWD ? 1 : (w < 1 ? 1 : (w > 8 ? 8 : w));
};

template <typename R, int NT, int MODE, int OP, int STAGE>
__global__ __launch_bounds__(kBlock) __attribute__((
    amdgpu_waves_per_eu(Occupancy<R, NT, MODE, OP, STAGE>::value))) void k_pass(const PassArgs A) {
  constexpr int NA = 1 << NT;
  constexpr bool HV = OP == OP_HVP;
  constexpr bool NEEDB = STAGE != ST_FWD && (OP == OP_GRAD || OP == OP_HVP);
  constexpr bool NEEDF = STAGE != ST_BWD;
  constexpr int NT1 = MODE == MODE_DENSE ? 32 : 16;
  constexpr int NE = HV ? 2 * NT1 : NT1;
  constexpr int LV = ilog2<NE>();
  constexpr uint32_t ES = sizeof(cx<R>);
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

  ccoef_t<R> *coef = as_const_coef<R>(A.coef);
  // byte stride of one tile bit in a slab and in the target
  int64_t bstep[NT], rstep[NT];
  static_for<0, NT>([&](auto B) __attribute__((always_inline)) {
    bstep[CV(B)] = (int64_t(1) << A.pos[CV(B)]) * A.ld * ES;
    rstep[CV(B)] = (int64_t(1) << A.pos[CV(B)]) * A.ld_ref * ES;
  });
  // byte offset of local amplitude I from the tile's first row
  auto boff = [&](auto I) __attribute__((always_inline)) {
    int64_t o = 0;
    static_for<0, NT>([&](auto B) __attribute__((always_inline)) {
      if constexpr ((CV(I) >> CV(B)) & 1) o += bstep[CV(B)];
    });
    return o;
  };
  auto roff = [&](auto I) __attribute__((always_inline)) {
    int64_t o = 0;
    static_for<0, NT>([&](auto B) __attribute__((always_inline)) {
      if constexpr ((CV(I) >> CV(B)) & 1) o += rstep[CV(B)];
    });
    return o;
  };
  auto lrow = [&](auto I) __attribute__((always_inline)) {
    int64_t o = 0;
    static_for<0, NT>([&](auto B) __attribute__((always_inline)) {
      if constexpr ((CV(I) >> CV(B)) & 1) o |= int64_t(1) << A.pos[CV(B)];
    });
    return o;
  };

  for (int item = gwave; item < A.n_items; item += nwaves) {
    const int cg = item % A.ncg;
    const int tile = item / A.ncg;
    const int c = cg * 64 + lane;
    const bool ok = c < A.ncols;
    const int cc = ok ? c : A.ncols - 1;          // clamped: loads stay in bounds
    const uint32_t voff = uint32_t(cc) * ES;
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
    const int64_t rowb = base * A.ld * ES;        // byte offset of the tile's first row
    const cx<R> zero{R(0), R(0)};

    cx<R> ps[NA], dps[NA], ph[NA], dph[NA];
    if constexpr (NEEDF) {
      if (A.src_psi) {
        const char *s = reinterpret_cast<const char *>(A.src_psi) + rowb;
        static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
          const cx<R> v = ldrow<R>(s + boff(I), voff);
          ps[CV(I)] = ok ? v : zero;
        });
      } else {
        const int64_t tgt = A.col0 + c - base;
        static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
          ps[CV(I)].x = (ok && lrow(I) == tgt) ? R(1) : R(0);
          ps[CV(I)].y = R(0);
        });
      }
      if constexpr (HV) {
        if (A.src_dpsi) {
          const char *s = reinterpret_cast<const char *>(A.src_dpsi) + rowb;
          static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
            const cx<R> v = ldrow<R>(s + boff(I), voff);
            dps[CV(I)] = ok ? v : zero;
          });
        } else {
          static_for<0, NA>([&](auto I) __attribute__((always_inline)) { dps[CV(I)] = zero; });
        }
      }
      for (int g = 0; g < A.ngates; ++g) {
        const GateRef gr = A.gates[g];
        ccoef_t<R> *co = coef + int64_t(gr.inst) * kCoefStride;
        dispatch<0, K::n>(gate_code(MODE, NT, gr, pi), [&](auto CC) __attribute__((always_inline)) {
          fwd_gate<R, NT, MODE, HV, CV(CC)>(ps, dps, co);
        });
      }
      if constexpr (STAGE == ST_FWD) {
        if (ok) {
          char *d = reinterpret_cast<char *>(A.dst_psi) + rowb;
          static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
            strow<R>(d + boff(I), voff, ps[CV(I)]);
          });
          if constexpr (HV) {
            char *dd = reinterpret_cast<char *>(A.dst_dpsi) + rowb;
            static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
              strow<R>(dd + boff(I), voff, dps[CV(I)]);
            });
          }
        }
      }
    } else {
      const char *s = reinterpret_cast<const char *>(A.ckpt_psi) + rowb;
      static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
        const cx<R> v = ldrow<R>(s + boff(I), voff);
        ps[CV(I)] = ok ? v : zero;
      });
      if constexpr (HV) {
        const char *sd = reinterpret_cast<const char *>(A.ckpt_dpsi) + rowb;
        static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
          const cx<R> v = ldrow<R>(sd + boff(I), voff);
          dps[CV(I)] = ok ? v : zero;
        });
      }
    }

    if constexpr (STAGE == ST_LAST) {
      // phi_0 = conj(U|j>), overlap h_j = sum_x phi_0[x] psi_N[x]
      const char *u = reinterpret_cast<const char *>(A.ref) + base * A.ld_ref * ES +
                      A.col0 * int64_t(ES);
      R hre = R(0);
      static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = CV(I);
        const cx<R> v = ldrow<R>(u + roff(I), voff);
        ph[i].x = ok ? v.x : R(0);
        ph[i].y = ok ? -v.y : R(0);
        hre = fma(ph[i].x, ps[i].x, hre);
        hre = fma(-ph[i].y, ps[i].y, hre);
        if constexpr (HV) dph[i] = zero;
      });
      facc += (double)hre;
    } else if constexpr (STAGE == ST_BWD) {
      const char *p = reinterpret_cast<const char *>(A.phi) + rowb;
      static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
        const cx<R> v = ldrow<R>(p + boff(I), voff);
        ph[CV(I)] = ok ? v : zero;
      });
      if constexpr (HV) {
        const char *pd = reinterpret_cast<const char *>(A.dphi) + rowb;
        static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
          const cx<R> v = ldrow<R>(pd + boff(I), voff);
          dph[CV(I)] = ok ? v : zero;
        });
      }
    }

    if constexpr (NEEDB) {
      for (int g = A.ngates - 1; g >= 0; --g) {
        const GateRef gr = A.gates[g];
        ccoef_t<R> *co = coef + int64_t(gr.inst) * kCoefStride;
        R tp[NE];
        static_for<0, NE>([&](auto E) __attribute__((always_inline)) { tp[CV(E)] = R(0); });
        dispatch<0, K::n>(gate_code(MODE, NT, gr, pi), [&](auto CC) __attribute__((always_inline)) {
          bwd_gate<R, NT, MODE, HV, CV(CC), NE>(ps, dps, ph, dph, co, tp);
        });
        const double r = wave_reduce_scatter<R, NE>(tp, lane);
        if (writer) acc[g * NE + my_e] += r;
      }
      if (A.store_phi && ok) {
        char *p = reinterpret_cast<char *>(A.phi) + rowb;
        static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
          strow<R>(p + boff(I), voff, ph[CV(I)]);
        });
        if constexpr (HV) {
          char *pd = reinterpret_cast<char *>(A.dphi) + rowb;
          static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
            strow<R>(pd + boff(I), voff, dph[CV(I)]);
          });
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

#undef CV

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

// Launch every (op, stage) instantiation enabled for one (R, NT, mode).
template <typename R, int NT, int MODE, bool COST, bool GRAD, bool HVP>
static int launch_mode(int op, int stage, const PassArgs &a, int grid, void *s) {
  if constexpr (COST) {
    if (op == OP_COST || op == OP_APPLY) {
      if (stage == ST_FWD) return launch_one<R, NT, MODE, OP_COST, ST_FWD>(a, grid, s);
      if (stage == ST_LAST && op == OP_COST) return launch_one<R, NT, MODE, OP_COST, ST_LAST>(a, grid, s);
    }
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
