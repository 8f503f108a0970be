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

// y -= c x (fused: no separate product and subtraction)
template <typename R>
__device__ __forceinline__ void cfms(cx<R> &y, cx<R> c, cx<R> x) {
  y.x = fma(-c.x, x.x, y.x);
  y.x = fma(c.y, x.y, y.x);
  y.y = fma(-c.x, x.y, y.y);
  y.y = fma(-c.y, x.x, y.y);
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

// Direct global->LDS loads (gfx950): each lane of the wavefront writes its
// `size` bytes at lds + lane * size.  Used by the backward sweep to bring
// checkpoint slabs into LDS (the current tile, kept there, or the next one,
// prefetched).  The compiler does not order these against later LDS reads,
// so the kernel waits on vmcnt explicitly (see k_pass).
template <int SIZE>
__device__ __forceinline__ void lds_dma(const char *g, void *lds) {
  if constexpr (SIZE == 4)
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)g,
                                     (__attribute__((address_space(3))) void *)lds, 4, 0, 0);
  else
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)g,
                                     (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
}

// s_waitcnt vmcnt(N) with the other counters unconstrained (gfx9 encoding).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
  asm volatile("" ::: "memory");  // keep LDS reads of the loaded tile after the wait
}
__device__ __forceinline__ void wait_lgkm0() {
  __builtin_amdgcn_s_waitcnt(0xF | (0x3 << 14) | (0x7 << 4) | (0x0 << 8));
  asm volatile("" ::: "memory");  // keep the next direct loads after the wait
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
            static_for<0, 4>([&](auto B) __attribute__((always_inline)) {
              cfms(y, giz[4 * a + CV(B)], x[CV(B)]);
            });
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
          cfms(xd0, giz[c00], x0);
          cfms(xd0, giz[c01], x1);
          cfms(xd1, giz[c10], x0);
          cfms(xd1, giz[c11], x1);
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

// bwd_gate with the forward states psi / dpsi held in LDS ([amplitude][lane],
// this wavefront's tile) instead of registers: each 2x2 block (4-amplitude
// group) reads its amplitudes, un-applies the gate and writes them back, so
// only the backward states stay register resident.
template <typename R, int NT, int MODE, bool HV, int C, int NE, int NA>
__device__ __forceinline__ void bwd_gate_l(cx<R> *sps, cx<R> *sdps, int lane, cx<R> (&ph)[NA],
                                           cx<R> (&dph)[NA], ccoef_t<R> *co, R (&tp)[NE]) {
  auto ps = [&](int i) -> cx<R> & { return sps[i * 64 + lane]; };
  auto dps = [&](int i) -> cx<R> & { return sdps[i * 64 + lane]; };
  using K = Codes<MODE, NT>;
  constexpr int TD = MODE == MODE_DENSE ? 32 : 16;  // offset of Tdot in tp
  if constexpr (K::template valid<C>()) {
    constexpr int H = K::template h<C>(), L = K::template l<C>();
    if constexpr (MODE == MODE_DENSE) {
      // Three phases, each with only its own coefficient blocks live (the
      // four 4x4 blocks of a dense gate do not fit the registers next to the
      // backward states and partials at two wavefronts per SIMD):
      // 1. recover the forward states before the gate, in place in LDS:
      //    x = G^-1 psi, xd = G^-1 dpsi - (G^-1 Z) x;
      {
        cx<R> gi[16], giz[16];
        static_for<0, 16>([&](auto E) __attribute__((always_inline)) {
          gi[CV(E)] = ldco<R>(co, 16 + CV(E));
          if constexpr (HV) giz[CV(E)] = ldco<R>(co, 48 + CV(E));
        });
        for_groups<NT, H, L>([&](auto I0, auto I1, auto I2, auto I3) __attribute__((always_inline)) {
          constexpr int id[4] = {CV(I0), CV(I1), CV(I2), CV(I3)};
          const cx<R> v[4] = {ps(id[0]), ps(id[1]), ps(id[2]), ps(id[3])};
          cx<R> x[4];
          static_for<0, 4>([&](auto A) __attribute__((always_inline)) {
            constexpr int a = CV(A);
            cx<R> y = mv2(gi[4 * a], v[0], gi[4 * a + 1], v[1]);
            cfma(y, gi[4 * a + 2], v[2]);
            cfma(y, gi[4 * a + 3], v[3]);
            x[a] = y;
          });
          if constexpr (HV) {
            const cx<R> d[4] = {dps(id[0]), dps(id[1]), dps(id[2]), dps(id[3])};
            static_for<0, 4>([&](auto A) __attribute__((always_inline)) {
              constexpr int a = CV(A);
              cx<R> y = mv2(gi[4 * a], d[0], gi[4 * a + 1], d[1]);
              cfma(y, gi[4 * a + 2], d[2]);
              cfma(y, gi[4 * a + 3], d[3]);
              static_for<0, 4>([&](auto B) __attribute__((always_inline)) {
                cfms(y, giz[4 * a + CV(B)], x[CV(B)]);
              });
              dps(id[a]) = y;
            });
          }
          static_for<0, 4>([&](auto A) __attribute__((always_inline)) { ps(id[CV(A)]) = x[CV(A)]; });
        });
      }
      // 2. the hole contractions T += phi (x) x, Tdot += dphi (x) x + phi (x) xd;
      for_groups<NT, H, L>([&](auto I0, auto I1, auto I2, auto I3) __attribute__((always_inline)) {
        constexpr int id[4] = {CV(I0), CV(I1), CV(I2), CV(I3)};
        cx<R> x[4], xd[4];
        static_for<0, 4>([&](auto A) __attribute__((always_inline)) {
          x[CV(A)] = ps(id[CV(A)]);
          if constexpr (HV) xd[CV(A)] = dps(id[CV(A)]);
        });
        static_for<0, 16>([&](auto AB) __attribute__((always_inline)) {
          constexpr int a = CV(AB) / 4, b = CV(AB) % 4, e = 2 * CV(AB);
          cacc(tp[e], tp[e + 1], ph[id[a]], x[b]);
          if constexpr (HV) {
            cacc(tp[TD + e], tp[TD + e + 1], dph[id[a]], x[b]);
            cacc(tp[TD + e], tp[TD + e + 1], ph[id[a]], xd[b]);
          }
        });
      });
      // 3. the backward states: phi <- G^T phi, dphi <- G^T dphi + Z^T phi.
      {
        cx<R> g[16], z[16];
        static_for<0, 16>([&](auto E) __attribute__((always_inline)) {
          g[CV(E)] = ldco<R>(co, CV(E));
          if constexpr (HV) z[CV(E)] = ldco<R>(co, 32 + CV(E));
        });
        for_groups<NT, H, L>([&](auto I0, auto I1, auto I2, auto I3) __attribute__((always_inline)) {
          constexpr int id[4] = {CV(I0), CV(I1), CV(I2), CV(I3)};
          const cx<R> p[4] = {ph[id[0]], ph[id[1]], ph[id[2]], ph[id[3]]};
          cx<R> pd[4], y[4], yd[4];
          if constexpr (HV)
            static_for<0, 4>([&](auto A) __attribute__((always_inline)) { pd[CV(A)] = dph[id[CV(A)]]; });
          static_for<0, 4>([&](auto A) __attribute__((always_inline)) {
            constexpr int a = CV(A);
            y[a] = mv2(g[a], p[0], g[4 + a], p[1]);
            cfma(y[a], g[8 + a], p[2]);
            cfma(y[a], g[12 + a], p[3]);
            if constexpr (HV) {
              yd[a] = mv2(g[a], pd[0], g[4 + a], pd[1]);
              cfma(yd[a], g[8 + a], pd[2]);
              cfma(yd[a], g[12 + a], pd[3]);
              cfma(yd[a], z[a], p[0]);
              cfma(yd[a], z[4 + a], p[1]);
              cfma(yd[a], z[8 + a], p[2]);
              cfma(yd[a], z[12 + a], p[3]);
            }
          });
          static_for<0, 4>([&](auto A) __attribute__((always_inline)) {
            ph[id[CV(A)]] = y[CV(A)];
            if constexpr (HV) dph[id[CV(A)]] = yd[CV(A)];
          });
        });
      }
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
        const cx<R> x0 = mv2(gi[c00], ps(i0), gi[c01], ps(i1));
        const cx<R> x1 = mv2(gi[c10], ps(i0), gi[c11], ps(i1));
        const cx<R> p0 = ph[i0], p1 = ph[i1];
        cacc(tp[2 * c00], tp[2 * c00 + 1], p0, x0);
        cacc(tp[2 * c01], tp[2 * c01 + 1], p0, x1);
        cacc(tp[2 * c10], tp[2 * c10 + 1], p1, x0);
        cacc(tp[2 * c11], tp[2 * c11 + 1], p1, x1);
        if constexpr (HV) {
          cx<R> xd0 = mv2(gi[c00], dps(i0), gi[c01], dps(i1));
          cx<R> xd1 = mv2(gi[c10], dps(i0), gi[c11], dps(i1));
          cfms(xd0, giz[c00], x0);
          cfms(xd0, giz[c01], x1);
          cfms(xd1, giz[c10], x0);
          cfms(xd1, giz[c11], x1);
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
          dps(i0) = xd0;
          dps(i1) = xd1;
        }
        ph[i0] = mv2(g[c00], p0, g[c10], p1);
        ph[i1] = mv2(g[c01], p0, g[c11], p1);
        ps(i0) = x0;
        ps(i1) = x1;
      });
    }
  }
}

// ----------------------------------------------------------------------------
// Wavefront reduce-scatter of V = 2^LV per-lane values (LV <= 6).  Step s
// pairs every lane with a partner that differs in lane bit d_s = 5 - s; the
// lane with d_s = 0 keeps the lower half of its values plus the partner's
// lower half, the other the upper halves.  After LV halving steps lane L
// holds the sum of entry L >> (6 - LV) over the lanes that share its bits
// 5 .. 6-LV; the remaining steps add over the low bits, so every lane ends
// with the full wavefront sum of its entry.
//   s = 0: v_permlane32_swap (lanes L, L^32), s = 1: v_permlane16_swap
//   (L, L^16): both exchange whole register halves, so the kept/sent halves
//   need no per-lane select; then DPP inside rows of 16 lanes: row_ror:8
//   (L^8), row_half_mirror (L^7), quad_perm (L^2), quad_perm (L^1).  The
//   masks 32, 16, 8, 7, 2, 1 are linearly independent over GF(2) and none
//   touches an earlier step's bit, so each lane's sum covers all 64 lanes
//   once.
// Complex64 states: the two permlane steps add in FP32 (four lanes' partial
// sums), everything after in FP64.
// ----------------------------------------------------------------------------
template <int V>
__device__ __forceinline__ constexpr int ilog2() {
  return V <= 1 ? 0 : 1 + ilog2<V / 2>();
}

__device__ __forceinline__ int entry_of_lane(int lane, int lv) { return lane >> (6 - lv); }
__device__ __forceinline__ bool entry_writer(int lane, int lv) {
  return (lane & ((1 << (6 - lv)) - 1)) == 0;
}

// (a, b) -> (a', b') with a' = [a.lo32, b.lo32], b' = [a.hi32, b.hi32] over
// lane halves (S = 32) or a' = [a.r0, b.r0, a.r2, b.r2],
// b' = [a.r1, b.r1, a.r3, b.r3] over rows of 16 lanes (S = 16).
template <int S>
__device__ __forceinline__ void lane_swap(uint32_t &a, uint32_t &b) {
  if constexpr (S == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  }
}
template <int S>
__device__ __forceinline__ void lane_swap(float &a, float &b) {
  uint32_t x = __builtin_bit_cast(uint32_t, a), y = __builtin_bit_cast(uint32_t, b);
  lane_swap<S>(x, y);
  a = __builtin_bit_cast(float, x);
  b = __builtin_bit_cast(float, y);
}
template <int S>
__device__ __forceinline__ void lane_swap(double &a, double &b) {
  uint64_t x = __builtin_bit_cast(uint64_t, a), y = __builtin_bit_cast(uint64_t, b);
  uint32_t xl = uint32_t(x), xh = uint32_t(x >> 32), yl = uint32_t(y), yh = uint32_t(y >> 32);
  lane_swap<S>(xl, yl);
  lane_swap<S>(xh, yh);
  a = __builtin_bit_cast(double, uint64_t(xl) | (uint64_t(xh) << 32));
  b = __builtin_bit_cast(double, uint64_t(yl) | (uint64_t(yh) << 32));
}

// value of the partner lane inside a row of 16 lanes (DPP control CTRL)
template <int CTRL>
__device__ __forceinline__ double dpp_partner(double v) {
  const uint64_t x = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_update_dpp(0u, uint32_t(x), CTRL, 0xF, 0xF, false);
  const uint32_t hi = __builtin_amdgcn_update_dpp(0u, uint32_t(x >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, uint64_t(lo) | (uint64_t(hi) << 32));
}
constexpr int kDppRor8 = 0x128, kDppHalfMirror = 0x141, kDppXor2 = 0x4E, kDppXor1 = 0xB1;
template <int S>
struct DppStep;  // steps 2..5
template <> struct DppStep<2> { static constexpr int ctrl = kDppRor8, bit = 3; };
template <> struct DppStep<3> { static constexpr int ctrl = kDppHalfMirror, bit = 2; };
template <> struct DppStep<4> { static constexpr int ctrl = kDppXor2, bit = 1; };
template <> struct DppStep<5> { static constexpr int ctrl = kDppXor1, bit = 0; };

// permlane halving step on n values of type T: v[i] (+) v[i + n/2]
template <int S, int N, typename T>
__device__ __forceinline__ void perm_halve(T (&v)[N]) {
  static_for<0, N / 2>([&](auto I) __attribute__((always_inline)) {
    constexpr int i = CV(I);
    T a = v[i], b = v[i + N / 2];
    lane_swap<S>(a, b);
    v[i] = a + b;
  });
}

// DPP steps STEP.. on the FP64 values (N = values left)
template <int STEP, int N>
__device__ __forceinline__ double dpp_steps(double (&v)[N], int lane) {
  if constexpr (STEP == 6) {
    return v[0];
  } else {
    using D = DppStep<STEP>;
    if constexpr (N > 1) {
      const bool hi = (lane >> D::bit) & 1;
      double w[N / 2];
      static_for<0, N / 2>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = CV(I);
        const double a = v[i], b = v[i + N / 2];
        const double keep = hi ? b : a, send = hi ? a : b;
        w[i] = keep + dpp_partner<D::ctrl>(send);
      });
      return dpp_steps<STEP + 1, N / 2>(w, lane);
    } else {
      double w[1] = {v[0] + dpp_partner<D::ctrl>(v[0])};
      return dpp_steps<STEP + 1, 1>(w, lane);
    }
  }
}

template <typename R, int V>
__device__ __forceinline__ double wave_reduce_scatter(const R (&tp)[V], int lane) {
  static_assert(V >= 4 && V <= 64, "reduce-scatter of 4..64 values");
  R v0[V];
  static_for<0, V>([&](auto I) __attribute__((always_inline)) { v0[CV(I)] = tp[CV(I)]; });
  perm_halve<32, V>(v0);
  R v1[V / 2];
  static_for<0, V / 2>([&](auto I) __attribute__((always_inline)) { v1[CV(I)] = v0[CV(I)]; });
  perm_halve<16, V / 2>(v1);
  double v2[V / 4];
  static_for<0, V / 4>([&](auto I) __attribute__((always_inline)) {
    v2[CV(I)] = (double)v1[CV(I)];
  });
  return dpp_steps<2, V / 4>(v2, lane);
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
// Slabs of a backward tile brought into LDS (bit s: 0 checkpoint psi, 1 phi,
// 2 checkpoint dpsi, 3 dphi): the checkpoints only for complex64 and for
// parity gates (where they stay resident, see Resident), all slabs of the
// next tile for complex128 with dense gates.
template <typename R, int NT, int MODE, int OP>
struct Prefetch {
  static constexpr int mask =
      (sizeof(R) == 4 || MODE != MODE_DENSE) ? (OP == OP_HVP ? 0x5 : 0x1)
                                              : (OP == OP_HVP ? 0xf : 0x3);
};

// Gate cap of a pass: dense complex64 HVP passes keep at most 8 gates, so
// that their FP64 accumulators (one row of entries per gate, in LDS next to
// the resident states) leave room for two wavefronts per SIMD; the scheduler
// applies the same cap.
template <typename R, int MODE, int OP>
struct PassGates {
  static constexpr int value =
      (MODE == MODE_DENSE && OP == OP_HVP && sizeof(R) == 4) ? 8 : kMaxGates;
};

// Backward passes that keep the forward states (checkpoint psi, dpsi) in LDS
// for the whole tile -- loaded there by direct global->LDS loads, un-applied
// block by block in place -- so that only phi (+dphi) and the contraction
// partials occupy registers: two wavefronts per SIMD where the LDS allows it
// (complex64 HVP and gradients, parity and dense gates), else one, which
// still lets complex128 parity HVP run 4-qubit tiles without spills.  Their
// LDS holds exactly the checkpoint slabs of Prefetch (no look-ahead tile).
template <typename R, int NT, int MODE, int OP>
struct Resident {
  static constexpr bool value =
      (MODE != MODE_DENSE || sizeof(R) == 4) && (OP == OP_GRAD || OP == OP_HVP);
  // the fused last pass too, for the HVP (whose backward half holds four
  // states); the gradient's last pass peaks in its forward half
  static constexpr bool last = value && OP == OP_HVP;
  static constexpr int NE = (MODE == MODE_DENSE ? 32 : 16) * (OP == OP_HVP ? 2 : 1);
  // LDS per wavefront: the resident states and the contraction accumulators
  static constexpr int lds_bytes = (OP == OP_HVP ? 2 : 1) * (1 << NT) * 64 * int(2 * sizeof(R)) +
                                   PassGates<R, MODE, OP>::value * NE * 8;
  // two wavefronts per SIMD when 8 of them fit the 160 KB of LDS of a CU
  static constexpr int waves = lds_bytes <= 20480 ? 2 : 1;
};

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
  // Backward-type kernels keep the compiler's own allocation (at two waves per
  // SIMD their register-resident states would spill to scratch memory),
  // except those with LDS-resident forward states.
  static constexpr bool res = STAGE == ST_BWD ? Resident<R, NT, MODE, OP>::value
                              : STAGE == ST_LAST && Resident<R, NT, MODE, OP>::last;
  static constexpr int value = res ? Resident<R, NT, MODE, OP>::waves
                               : STAGE != ST_FWD ? 1 : (w < 1 ? 1 : (w > 8 ? 8 : w));
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
  // particle-number sectors: rows are sector ranks looked up per tile
  constexpr bool NUM = MODE == MODE_NUMBER;
  extern __shared__ double lds[];

  // Backward passes run one wavefront per block and bring the PFMASK slabs
  // (0 checkpoint psi, 1 phi, 2 checkpoint dpsi, 3 dphi) into LDS with direct
  // loads: with LRES the current tile's checkpoints, which stay there while
  // the gates are un-applied in place; otherwise the next tile, prefetched
  // while the current one is computed from registers.  The other slabs are
  // loaded into registers at the top of the tile.
  constexpr bool PF = STAGE == ST_BWD;
  constexpr bool LRES = PF && Resident<R, NT, MODE, OP>::value;   // forward states in LDS
  // the fused last pass of the HVP keeps them in LDS for its backward half
  constexpr bool LRESL = STAGE == ST_LAST && Resident<R, NT, MODE, OP>::last;
  constexpr int DW = int(ES) / 4;                 // dwords per amplitude
  constexpr int PFMASK = Prefetch<R, NT, MODE, OP>::mask;
  constexpr int NPF = __builtin_popcount(PFMASK);
  constexpr int PF_BYTES = (PF || LRESL) ? NPF * NA * 64 * int(ES) : 0;
  static_assert(!(NUM && PF && !LRES), "sector-row tiles are only loaded for the current item");
  const int lane = threadIdx.x & 63;
  const int wib = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int gwave = blockIdx.x * wpb + wib;
  const int nwaves = gridDim.x * wpb;
  char *pf = reinterpret_cast<char *>(lds);       // PF: this wavefront's tile buffer
  double *acc = reinterpret_cast<double *>(reinterpret_cast<char *>(lds) + PF_BYTES) +
                wib * (PassGates<R, MODE, OP>::value * NE);
  const int my_e = entry_of_lane(lane, LV);
  const bool writer = entry_writer(lane, LV);
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
  // byte offset of local amplitude I in the input slab (row stride ld_src)
  auto soff = [&](auto I) __attribute__((always_inline)) {
    int64_t o = 0;
    static_for<0, NT>([&](auto B) __attribute__((always_inline)) {
      if constexpr ((CV(I) >> CV(B)) & 1) o += (int64_t(1) << A.pos[CV(B)]) * A.ld_src * ES;
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
  // NUM: lane i < NA holds the sector row of local amplitude i of the
  // current tile (bit i of vmask: the amplitude belongs to the sector; the
  // others are zero and are neither loaded nor stored)
  int32_t rk_lane = 0;
  uint32_t vmask = ~0u;
  auto rvalid = [&](auto I) __attribute__((always_inline)) -> bool {
    if constexpr (NUM) return (vmask >> CV(I)) & 1u;
    else return true;
  };
  auto nrow = [&](auto I) __attribute__((always_inline)) -> int64_t {
    return int64_t(__builtin_amdgcn_readlane(rk_lane, CV(I)));
  };

  // LDS-DMA prefetch of one tile of the backward sweep
  auto prefetch = [&](int it) __attribute__((always_inline)) {
    const int pcg = it % A.ncg;
    const int ptile = it / A.ncg;
    const int pc = pcg * 64 + lane;
    const int pcc = pc < A.ncols ? pc : A.ncols - 1;
    int64_t pbase = 0;
    {
      int t = ptile;
      for (int p = 0; p < A.kq; ++p)
        if (!((A.qmask >> p) & 1)) {
          pbase |= int64_t(t & 1) << p;
          t >>= 1;
        }
    }
    const int64_t prow = pbase * A.ld * ES;
    const uint32_t pvoff = uint32_t(pcc) * ES;
    const char *src[4] = {reinterpret_cast<const char *>(A.ckpt_psi),
                          reinterpret_cast<const char *>(A.phi),
                          reinterpret_cast<const char *>(A.ckpt_dpsi),
                          reinterpret_cast<const char *>(A.dphi)};
    static_for<0, 4>([&](auto S) __attribute__((always_inline)) {
      constexpr int sl = CV(S);
      if constexpr (((PFMASK >> sl) & 1) && NUM) {
        // sector rows of the current item; rows outside the sector are not
        // loaded (zeroed in LDS once the loads have landed)
        constexpr int li = __builtin_popcount(PFMASK & ((1 << sl) - 1));
        if constexpr (DW == 2) {
          const uint32_t hoff = uint32_t(lane & 31) * 16;
          const int64_t colb = int64_t(pcg) * 64 * ES;
          static_for<0, NA / 2>([&](auto I2) __attribute__((always_inline)) {
            constexpr int i0 = 2 * CV(I2);
            const bool v0 = rvalid(ic<i0>{}), v1 = rvalid(ic<i0 + 1>{});
            const int64_t r0 = nrow(ic<i0>{}), r1 = nrow(ic<i0 + 1>{});
            const int64_t rb = ((lane < 32) ? r0 : r1) * A.ld * ES;
            if ((lane < 32) ? v0 : v1)
              lds_dma<16>(src[sl] + rb + colb + hoff, pf + (li * NA + i0) * 64 * int(ES));
          });
        } else {
          static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
            if (rvalid(I))
              lds_dma<16>(src[sl] + nrow(I) * A.ld * ES + pvoff,
                          pf + (li * NA + CV(I)) * 64 * int(ES));
          });
        }
      } else if constexpr ((PFMASK >> sl) & 1) {
        constexpr int li = __builtin_popcount(PFMASK & ((1 << sl) - 1));
        if constexpr (DW == 2) {
          // complex64: 16 bytes per lane = two columns; lanes 0-31 fetch row
          // I, lanes 32-63 row I+1 of the 64-column segment, so each 16-byte
          // load lands in LDS in the natural [row][column] order (512 bytes
          // per row).  ld is a multiple of 64: whole segments are in bounds.
          const uint32_t hoff = uint32_t(lane & 31) * 16;
          const int64_t colb = int64_t(pcg) * 64 * ES;
          static_for<0, NA / 2>([&](auto I2) __attribute__((always_inline)) {
            constexpr int i0 = 2 * CV(I2);
            const int64_t rb = (lane < 32) ? boff(ic<i0>{}) : boff(ic<i0 + 1>{});
            const char *g = src[sl] + prow + rb + colb + hoff;
            lds_dma<16>(g, pf + (li * NA + i0) * 64 * int(ES));
          });
        } else {
          static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
            const char *g = src[sl] + prow + boff(I) + pvoff;
            lds_dma<16>(g, pf + (li * NA + CV(I)) * 64 * int(ES));
          });
        }
      }
    });
  };
  // tile -> registers: row I of slab S from LDS ([slab][row][column]) if it
  // was prefetched, else straight from the slab
  auto pf_read = [&](auto S, auto I, int64_t rowb, uint32_t voff) __attribute__((always_inline)) {
    constexpr int sl = CV(S);
    if constexpr ((PFMASK >> sl) & 1) {
      constexpr int li = __builtin_popcount(PFMASK & ((1 << sl) - 1));
      const char *l = pf + (li * NA + CV(I)) * 64 * int(ES);
      return reinterpret_cast<const cx<R> *>(l)[lane];
    } else {
      const void *base = sl == 0 ? A.ckpt_psi : sl == 1 ? A.phi : sl == 2 ? A.ckpt_dpsi : A.dphi;
      if constexpr (NUM) {
        cx<R> v{R(0), R(0)};
        if (rvalid(I)) v = ldrow<R>(reinterpret_cast<const char *>(base) + nrow(I) * A.ld * ES, voff);
        return v;
      } else {
        return ldrow<R>(reinterpret_cast<const char *>(base) + rowb + boff(I), voff);
      }
    }
  };
  if constexpr (PF && !LRES) {
    if (gwave < A.n_items) prefetch(gwave);
  }
  cx<R> *sps = reinterpret_cast<cx<R> *>(pf);          // LRES: psi tile [amp][lane]
  cx<R> *sdps = sps + NA * 64;                          // LRES: dpsi tile

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
    // implied bit of local amplitude i: sector ^ parity(base) ^ parity(i); in
    // a particle-number sector it is M - popcount(i), M = n - popcount(base),
    // which has the same parity, so both modes share the gate cases
    const int pi = MODE != MODE_DENSE ? ((A.sector ^ __builtin_popcountll(base)) & 1) : 0;
    if constexpr (NUM) {
      // basis index of local amplitude i: row bits base | lrow(i), then the
      // implied bit M - popcount(i) (0 or 1 inside the sector)
      const int M = A.sector - __builtin_popcountll(base);
      if (M < 0 || M > NT + 1) continue;  // no state of the sector on this tile
      bool vl = false;
      rk_lane = 0;
      if (lane < NA) {
        int64_t lr = 0;
        for (int b = 0; b < NT; ++b)
          if ((lane >> b) & 1) lr |= int64_t(1) << A.pos[b];
        const int imp = M - __builtin_popcount(lane);
        vl = imp == 0 || imp == 1;
        if (vl) rk_lane = A.rank[((base | lr) << 1) | imp];
      }
      vmask = uint32_t(__builtin_amdgcn_ballot_w64(vl));
    }
    const int64_t rowb = base * A.ld * ES;        // byte offset of the tile's first row
    const cx<R> zero{R(0), R(0)};

    cx<R> ps[NA], dps[NA], ph[NA], dph[NA];
    if constexpr (NEEDF) {
      if (A.src_psi && NUM) {
        const char *s = reinterpret_cast<const char *>(A.src_psi);
        static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
          ps[CV(I)] = zero;
          if (rvalid(I)) {
            const cx<R> v = ldrow<R>(s + nrow(I) * A.ld_src * ES, voff);
            ps[CV(I)] = ok ? v : zero;
          }
        });
      } else if (A.src_psi) {
        const char *s = reinterpret_cast<const char *>(A.src_psi) + base * A.ld_src * ES;
        static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
          const cx<R> v = ldrow<R>(s + soff(I), voff);
          ps[CV(I)] = ok ? v : zero;
        });
      } else if constexpr (NUM) {
        const int64_t tgt = A.col0 + c;
        static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
          ps[CV(I)].x = (ok && rvalid(I) && nrow(I) == tgt) ? R(1) : R(0);
          ps[CV(I)].y = R(0);
        });
      } else {
        const int64_t tgt = A.col0 + c - base;
        static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
          ps[CV(I)].x = (ok && lrow(I) == tgt) ? R(1) : R(0);
          ps[CV(I)].y = R(0);
        });
      }
      if constexpr (HV) {
        if (A.src_dpsi && NUM) {
          const char *s = reinterpret_cast<const char *>(A.src_dpsi);
          static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
            dps[CV(I)] = zero;
            if (rvalid(I)) {
              const cx<R> v = ldrow<R>(s + nrow(I) * A.ld * ES, voff);
              dps[CV(I)] = ok ? v : zero;
            }
          });
        } else if (A.src_dpsi) {
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
      if constexpr (STAGE == ST_FWD && NUM) {
        if (ok) {
          static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
            if (rvalid(I)) {
              const int64_t o = nrow(I) * A.ld * ES;
              strow<R>(reinterpret_cast<char *>(A.dst_psi) + o, voff, ps[CV(I)]);
              if constexpr (HV) strow<R>(reinterpret_cast<char *>(A.dst_dpsi) + o, voff, dps[CV(I)]);
            }
          });
        }
      } else if constexpr (STAGE == ST_FWD) {
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
    } else if constexpr (LRES) {
      // this tile's checkpoint slabs straight into LDS (after the previous
      // tile's LDS accesses completed), phi (+dphi) into registers
      wait_lgkm0();
      prefetch(item);
      // padding lanes (ragged chunk) read a clamped copy of a valid column:
      // finite, and every product they enter has a zeroed psi or dpsi factor
      static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
        ph[CV(I)] = pf_read(ic<1>{}, I, rowb, voff);
        if constexpr (HV) dph[CV(I)] = pf_read(ic<3>{}, I, rowb, voff);
      });
      wait_vmcnt<0>();
      if constexpr (NUM) {  // amplitudes outside the sector: zero, not loaded
        static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
          if (!rvalid(I)) {
            sps[CV(I) * 64 + lane] = zero;
            if constexpr (HV) sdps[CV(I) * 64 + lane] = zero;
          }
        });
      }
      if (!ok) {  // padding columns of a ragged chunk: zero states
        static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
          sps[CV(I) * 64 + lane] = zero;
          if constexpr (HV) sdps[CV(I) * 64 + lane] = zero;
        });
      }
    } else {
      // Wait for this tile's prefetch.  Only the previous tile's phi stores
      // (nst * NA vector-memory instructions) were issued after it, so they
      // may stay outstanding.
      if (item != gwave && A.store_phi)
        wait_vmcnt<(HV ? 2 : 1) * NA>();
      else
        wait_vmcnt<0>();
      // direct loads first: the compiler's wait for them then leaves the
      // next tile's prefetch (issued below) outstanding
      static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
        const cx<R> p = pf_read(ic<1>{}, I, rowb, voff);
        ph[CV(I)] = ok ? p : zero;
        if constexpr (HV) {
          const cx<R> pd = pf_read(ic<3>{}, I, rowb, voff);
          dph[CV(I)] = ok ? pd : zero;
        }
      });
      static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
        const cx<R> v = pf_read(ic<0>{}, I, rowb, voff);
        ps[CV(I)] = ok ? v : zero;
        if constexpr (HV) {
          const cx<R> vd = pf_read(ic<2>{}, I, rowb, voff);
          dps[CV(I)] = ok ? vd : zero;
        }
      });
      wait_lgkm0();  // the buffer is read before the next prefetch overwrites it
      if (item + nwaves < A.n_items) prefetch(item + nwaves);
    }

    if constexpr (STAGE == ST_LAST) {
      // phi_0 = conj(U|j>), overlap h_j = sum_x phi_0[x] psi_N[x]
      const char *u = reinterpret_cast<const char *>(A.ref) + (NUM ? 0 : base * A.ld_ref * ES) +
                      A.col0 * int64_t(ES);
      R hre = R(0);
      static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = CV(I);
        cx<R> v = zero;
        if constexpr (NUM) {
          if (rvalid(I)) v = ldrow<R>(u + nrow(I) * A.ld_ref * ES, voff);
        } else {
          v = ldrow<R>(u + roff(I), voff);
        }
        ph[i].x = ok ? v.x : R(0);
        ph[i].y = ok ? -v.y : R(0);
        hre = fma(ph[i].x, ps[i].x, hre);
        hre = fma(-ph[i].y, ps[i].y, hre);
        if constexpr (HV) dph[i] = zero;
      });
      facc += (double)hre;
      if constexpr (LRESL) {  // forward states -> LDS for the backward half
        static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
          sps[CV(I) * 64 + lane] = ps[CV(I)];
          if constexpr (HV) sdps[CV(I) * 64 + lane] = dps[CV(I)];
        });
      }
    }

    if constexpr (NEEDB) {
      for (int g = A.ngates - 1; g >= 0; --g) {
        const GateRef gr = A.gates[g];
        ccoef_t<R> *co = coef + int64_t(gr.inst) * kCoefStride;
        R tp[NE];
        // -0 is the exact additive identity: the first fma into each
        // partial folds into a plain multiply, with no zeroing moves (not in
        // the dense fused last pass, whose allocation then spills)
        constexpr R tp0 = (STAGE == ST_LAST && MODE == MODE_DENSE) ? R(0) : R(-0.0);
        static_for<0, NE>([&](auto E) __attribute__((always_inline)) { tp[CV(E)] = tp0; });
        dispatch<0, K::n>(gate_code(MODE, NT, gr, pi), [&](auto CC) __attribute__((always_inline)) {
          if constexpr (LRES || LRESL)
            bwd_gate_l<R, NT, MODE, HV, CV(CC), NE>(sps, sdps, lane, ph, dph, co, tp);
          else
            bwd_gate<R, NT, MODE, HV, CV(CC), NE>(ps, dps, ph, dph, co, tp);
        });
        const double r = wave_reduce_scatter<R, NE>(tp, lane);
        if (writer) acc[g * NE + my_e] += r;
      }
      if (A.store_phi && ok && NUM) {
        static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
          if (rvalid(I)) {
            const int64_t o = nrow(I) * A.ld * ES;
            strow<R>(reinterpret_cast<char *>(A.phi) + o, voff, ph[CV(I)]);
            if constexpr (HV) strow<R>(reinterpret_cast<char *>(A.dphi) + o, voff, dph[CV(I)]);
          }
        });
      } else if (A.store_phi && ok) {
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
  if (a.ngates > PassGates<R, MODE, OP>::value) return -1;
  constexpr bool HV = OP == OP_HVP;
  constexpr bool NEEDB = STAGE != ST_FWD && (OP == OP_GRAD || OP == OP_HVP);
  constexpr int NT1 = MODE == MODE_DENSE ? 32 : 16;
  constexpr int NE = HV ? 2 * NT1 : NT1;
  constexpr bool LRESL = STAGE == ST_LAST && Resident<R, NT, MODE, OP>::last;
  if constexpr (STAGE == ST_BWD || LRESL) {
    // one wavefront per block: grid * 4 blocks of 64 threads give the same
    // wavefronts (and slot indices) as grid blocks of 256 threads
    constexpr int NPF = __builtin_popcount(Prefetch<R, NT, MODE, OP>::mask);
    const size_t lds = size_t(NPF) * (1 << NT) * 64 * sizeof(cx<R>) +
                       size_t(PassGates<R, MODE, OP>::value) * NE * sizeof(double);
    hipLaunchKernelGGL((k_pass<R, NT, MODE, OP, STAGE>), dim3(grid * (kBlock / 64)), dim3(64),
                       lds, (hipStream_t)stream, a);
  } else {
    const size_t lds =
        NEEDB ? size_t(kBlock / 64) * PassGates<R, MODE, OP>::value * NE * sizeof(double) : 0;
    hipLaunchKernelGGL((k_pass<R, NT, MODE, OP, STAGE>), dim3(grid), dim3(kBlock), lds,
                       (hipStream_t)stream, a);
  }
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

// HVPD / HVPP: HVP instantiations for dense / parity gates (their tile sizes
// differ in complex128).
template <typename R, int NT, bool COST, bool GRAD, bool HVPD, bool HVPP>
static int launch_nt(int mode, int op, int stage, const PassArgs &a, int grid, void *s) {
  return mode == MODE_DENSE
             ? launch_mode<R, NT, MODE_DENSE, COST, GRAD, HVPD>(op, stage, a, grid, s)
         : mode == MODE_PARITY
             ? launch_mode<R, NT, MODE_PARITY, COST, GRAD, HVPP>(op, stage, a, grid, s)
             : launch_mode<R, NT, MODE_NUMBER, COST, GRAD, HVPP>(op, stage, a, grid, s);
}

}  // namespace rqk
