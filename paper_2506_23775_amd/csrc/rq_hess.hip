// Hessian blocks (arXiv 2506.23775, Sec. "Efficient gradient and Hessian
// computation" and Sec. "Gate hole application"):
//   - the gate hole of G_l applied to psi_{l-1} gives a state array with one
//     slice per gate entry (a, b) (16 slices; 8 for parity gates, Sec.
//     "Parity-conserving gate structure"): slice (a,b) holds psi_{l-1} with
//     the pair bits moved from b to a;
//   - the array is propagated through G_{l+1}, G_{l+2}, ... like a state;
//   - at every later gate m the hole of G_m is sandwiched between phi at the
//     output side of m and the array at its input side, giving the block
//     d^2 h / dG_l[a,b] dG_m[a',b'].
// GPU design: a block of four wavefronts owns four slices of one (tile,
// 64-column group) item at a time; each wavefront keeps the 2^NT amplitudes
// of its slice on the tile in registers and fuses every gate of a sweep pass
// (contraction, then application).  The phi tile at each gate output (from
// a stored per-gate backward sweep) is brought into LDS once per block by
// direct global->LDS loads, double-buffered one gate ahead, and read by the
// four slices, so phi crosses HBM once per item instead of once per slice.
// In the first pass after the hole the slices are built in registers from
// the tile of psi before the hole gate (no separate hole-array pass).
// Contractions use the FP64 wavefront reduce-scatter and per-wave slots of
// the gradient.
#include <algorithm>

#include "rq_sweep.h"

#define CV(x) decltype(x)::value

namespace rqk {

// tp[(a', b')] += phi[a'] psi[b'] over the groups of the gate's qubits, phi
// read from the LDS tile ph (amplitude i of this lane at ph[i * 64]).
template <typename R, int NT, int MODE, int C, int NE, int NA>
__device__ __forceinline__ void contract_gate(const cx<R> (&ps)[NA], const cx<R> *ph,
                                              R (&tp)[NE]) {
  using K = Codes<MODE, NT>;
  if constexpr (K::template valid<C>()) {
    constexpr int H = K::template h<C>(), L = K::template l<C>();
    if constexpr (MODE == MODE_DENSE) {
      for_groups<NT, H, L>([&](auto I0, auto I1, auto I2, auto I3) __attribute__((always_inline)) {
        constexpr int id[4] = {CV(I0), CV(I1), CV(I2), CV(I3)};
        cx<R> p[4];
        static_for<0, 4>([&](auto A) __attribute__((always_inline)) { p[CV(A)] = ph[id[CV(A)] * 64]; });
        static_for<0, 16>([&](auto AB) __attribute__((always_inline)) {
          constexpr int a = CV(AB) / 4, b = CV(AB) % 4, e = 2 * CV(AB);
          cacc(tp[e], tp[e + 1], p[a], ps[id[b]]);
        });
      });
    } else {
      constexpr int KD = K::template kind<C>(), PI = K::template pi<C>();
      for_blocks<NT, KD, H, L, PI>([&](auto J0, auto J1, auto C00, auto C01, auto C10,
                                       auto C11) __attribute__((always_inline)) {
        constexpr int i0 = CV(J0), i1 = CV(J1);
        const cx<R> p0 = ph[i0 * 64], p1 = ph[i1 * 64];
        cacc(tp[2 * CV(C00)], tp[2 * CV(C00) + 1], p0, ps[i0]);
        cacc(tp[2 * CV(C01)], tp[2 * CV(C01) + 1], p0, ps[i1]);
        cacc(tp[2 * CV(C10)], tp[2 * CV(C10) + 1], p1, ps[i0]);
        cacc(tp[2 * CV(C11)], tp[2 * CV(C11) + 1], p1, ps[i1]);
      });
    }
  }
}

// Gate-hole application on a register tile: slice (a, b) of the array is the
// state with the gate's pair bits moved from b to a, zero where the pair bits
// of the amplitude differ from a.  ps holds the state before the hole gate on
// entry and the slice on exit.  Pair value of local amplitude i: both bits
// local (kind 0), or one of them the implied qubit k-1 whose bit is
// PI ^ parity(i) (kinds 1, 2; see for_blocks).
template <typename R, int NT, int MODE, int C, int NA>
__device__ __forceinline__ void hole_slice(cx<R> (&ps)[NA], int a, int b) {
  using K = Codes<MODE, NT>;
  if constexpr (K::template valid<C>()) {
    constexpr int H = K::template h<C>(), L = K::template l<C>();
    constexpr int KD = MODE == MODE_DENSE ? 0 : K::template kind<C>();
    constexpr int PI = MODE == MODE_DENSE ? 0 : K::template pi<C>();
    // (component-wise selects: a select of whole structs becomes an indexed
    // stack access)
    auto put = [&](cx<R> &dst, bool keep, R x, R y) __attribute__((always_inline)) {
      dst.x = keep ? x : R(0);
      dst.y = keep ? y : R(0);
    };
    if constexpr (KD == 0) {
      // groups of four amplitudes with pair values 0..3
      for_groups<NT, H, L>([&](auto I0, auto I1, auto I2, auto I3) __attribute__((always_inline)) {
        constexpr int id[4] = {CV(I0), CV(I1), CV(I2), CV(I3)};
        R vx = b == 1 ? ps[id[1]].x : ps[id[0]].x, vy = b == 1 ? ps[id[1]].y : ps[id[0]].y;
        vx = b == 2 ? ps[id[2]].x : vx;
        vy = b == 2 ? ps[id[2]].y : vy;
        vx = b == 3 ? ps[id[3]].x : vx;
        vy = b == 3 ? ps[id[3]].y : vy;
        static_for<0, 4>([&](auto J) __attribute__((always_inline)) {
          put(ps[id[CV(J)]], a == CV(J), vx, vy);
        });
      });
    } else {
      // pairs differing in the explicit bit H; the implied bit is
      // PI ^ parity(local index)
      static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
        constexpr int i0 = CV(I);
        if constexpr (!((i0 >> H) & 1)) {
          constexpr int i1 = i0 | (1 << H);
          constexpr int be0 = PI ^ (__builtin_popcount(i0) & 1), be1 = be0 ^ 1;
          constexpr int pv0 = KD == 1 ? be0 : 2 * be0;
          constexpr int pv1 = KD == 1 ? 2 + be1 : 2 * be1 + 1;
          const R s0x = ps[i0].x, s0y = ps[i0].y, s1x = ps[i1].x, s1y = ps[i1].y;
          const R vx = b == pv0 ? s0x : (b == pv1 ? s1x : R(0));
          const R vy = b == pv0 ? s0y : (b == pv1 ? s1y : R(0));
          ps[i0].x = a == pv0 ? vx : R(0);
          ps[i0].y = a == pv0 ? vy : R(0);
          ps[i1].x = a == pv1 ? vx : R(0);
          ps[i1].y = a == pv1 ? vy : R(0);
        }
      });
    }
  }
}

// Slice mu -> gate entry (a, b): dense 4x4 row-major; parity pattern
// (0,0),(0,3),(3,0),(3,3),(1,1),(1,2),(2,1),(2,2); particle number the same
// without (0,3), (3,0).
__device__ __forceinline__ void slice_entry(int mode, int nd, int mu, int &a, int &b) {
  if (mode == MODE_DENSE) {
    a = mu >> 2;
    b = mu & 3;
  } else if (nd == 6) {
    const int pa = 0x221130, pb = 0x212130;   // nibbles, entry 0 lowest
    a = (pa >> (4 * mu)) & 0xF;
    b = (pb >> (4 * mu)) & 0xF;
  } else {
    const int pa = 0x22113300, pb = 0x21213030;
    a = (pa >> (4 * mu)) & 0xF;
    b = (pb >> (4 * mu)) & 0xF;
  }
}

// Target wavefronts per SIMD of the hole-array sweep: three for complex64
// parity gates on 5-qubit tiles (the compiler's own allocation takes 177
// registers, 9 more than three wavefronts leave; at 168 it spills 44 bytes
// per lane and runs the configuration-3 sweep 4 % faster), otherwise the
// compiler's own allocation.
template <typename R, int NT, int MODE, int W>
struct HessWaves {
  static constexpr int value =
      (sizeof(R) == 4 && NT == 5 && MODE == MODE_PARITY && W == 4) ? 3 : 1;
};

// W wavefronts per block, one slice each (W = 4: the six slices of
// particle-number gates leave two wavefronts of an item's second block
// idle, which at three wavefronts per SIMD runs faster than blocks of three
// at two).
template <typename R, int NT, int MODE, int W>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(
    HessWaves<R, NT, MODE, W>::value))) void k_hess_pass(const HessArgs A) {
  constexpr int NA = 1 << NT;
  constexpr int NE = MODE == MODE_DENSE ? 32 : 16;
  constexpr int LV = ilog2<NE>();
  constexpr uint32_t ES = sizeof(cx<R>);
  constexpr int DW = int(ES) / 4;
  // phi rows loaded by each of the four wavefronts per gate; one direct load
  // moves 16 bytes per lane: two rows of 64 complex64 columns (lanes 0-31 /
  // 32-63), or one row of complex128
  constexpr int ROWS_PER_LOAD = DW == 2 ? 2 : 1;
  constexpr int TOTAL_LOADS = NA / ROWS_PER_LOAD;        // per tile, over the block
  constexpr int LOADS = (TOTAL_LOADS + W - 1) / W;       // per wavefront (at most)
  using K = Codes<MODE, NT>;
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63;
  const int wib = threadIdx.x >> 6;
  const int gwave = blockIdx.x * W + wib;
  cx<R> *phb = reinterpret_cast<cx<R> *>(lds);                       // [2][NA][64]
  double *acc = reinterpret_cast<double *>(phb + 2 * NA * 64) + wib * (kMaxGates * NE);
  const int my_e = entry_of_lane(lane, LV);
  const bool writer = entry_writer(lane, LV);
  // block -> (slice group, first item); the W wavefronts of a block take
  // W consecutive slices of the same items.  Consecutive blocks go to the
  // XCDs in turn, so when the grid is a multiple of kXcds * nquads the
  // nquads blocks of an item are blocks b, b + kXcds, ... of one XCD,
  // started together: the second and later reads of each phi tile hit that
  // XCD's L2 instead of HBM.  Otherwise consecutive blocks share an item.
  const int nq = A.nquads;
  const bool xcd = gridDim.x % (kXcds * nq) == 0;
  const int quad = xcd ? (blockIdx.x / kXcds) % nq : blockIdx.x % nq;
  const int rest0 = xcd ? (blockIdx.x / (kXcds * nq)) * kXcds + blockIdx.x % kXcds
                        : blockIdx.x / nq;
  const int rstride = gridDim.x / nq;
  const int mu = quad * W + wib;
  const bool active = mu < A.nd;           // particle-number mode pads 6 slices to 8
  int ea = 0, eb = 0;
  slice_entry(MODE, A.nd, active ? mu : 0, ea, eb);
  for (int g = 0; g < A.ngates; ++g)
    if (writer) acc[g * NE + my_e] = 0.0;
  ccoef_t<R> *coef = as_const_coef<R>(A.coef);
  int64_t bstep[NT];
  static_for<0, NT>([&](auto B) __attribute__((always_inline)) {
    bstep[CV(B)] = (int64_t(1) << A.pos[CV(B)]) * A.ld * ES;
  });
  auto boff = [&](auto I) __attribute__((always_inline)) {
    int64_t o = 0;
    static_for<0, NT>([&](auto B) __attribute__((always_inline)) {
      if constexpr ((CV(I) >> CV(B)) & 1) o += bstep[CV(B)];
    });
    return o;
  };
  auto tile_base = [&](int rest) {
    int t = rest / A.ncg;
    int64_t base = 0;
    for (int p = 0; p < A.kq; ++p)
      if (!((A.qmask >> p) & 1)) {
        base |= int64_t(t & 1) << p;
        t >>= 1;
      }
    return base;
  };
  const int g0 = A.hole_src ? 1 : 0;       // first gate with a contraction
  const bool any_phi = A.ngates > g0;
  // direct loads of this wavefront's rows of the phi tile of gate g, item rest
  auto prefetch = [&](int rest, int g, int buf) __attribute__((always_inline)) {
    const int cg = rest % A.ncg;
    const int64_t rowb = tile_base(rest) * A.ld * ES;
    const char *src = reinterpret_cast<const char *>(A.phi) +
                      int64_t(A.gates[g].inst) * A.slab * ES + rowb + int64_t(cg) * 64 * ES;
    static_for<0, LOADS>([&](auto Q) __attribute__((always_inline)) {
      const int li = CV(Q) * W + wib;        // load index of this wavefront
      if (TOTAL_LOADS % W == 0 || li < TOTAL_LOADS) {
        const int r0 = li * ROWS_PER_LOAD;
        // byte offset of local row r (runtime: wib varies over the block)
        int64_t ro = 0;
        const int r = DW == 2 ? r0 + (lane >> 5) : r0;
        static_for<0, NT>([&](auto B) __attribute__((always_inline)) {
          if ((r >> CV(B)) & 1) ro += bstep[CV(B)];
        });
        const uint32_t coff = DW == 2 ? uint32_t(lane & 31) * 16 : uint32_t(lane) * 16;
        lds_dma<16>(src + ro + coff, phb + (buf * NA + r0) * 64);
      }
    });
  };

  int buf = 0;
  if (any_phi && rest0 < A.n_rest) prefetch(rest0, g0, 0);
  for (int rest = rest0; rest < A.n_rest; rest += rstride) {
    const int cg = rest % A.ncg;
    const int c = cg * 64 + lane;
    const bool ok = c < A.ncols;
    const int cc = ok ? c : A.ncols - 1;
    const uint32_t voff = uint32_t(cc) * ES;
    const int64_t base = tile_base(rest);
    const int pi = MODE == MODE_PARITY ? ((A.sector ^ __builtin_popcountll(base)) & 1) : 0;
    const int64_t rowb = base * A.ld * ES;
    const cx<R> zero{R(0), R(0)};
    char *sl = reinterpret_cast<char *>(A.psi) + int64_t(active ? mu : 0) * A.slab * ES + rowb;
    const char *ld_src = A.hole_src ? reinterpret_cast<const char *>(A.hole_src) + rowb : sl;
    cx<R> ps[NA];
    // a padding wavefront (no slice: particle-number gates have 6 of 8)
    // reads nothing and computes nothing; it only takes its share of the
    // phi loads and the barriers of its block
    if (active) {
      static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
        const cx<R> v = ldrow<R>(ld_src + boff(I), voff);
        ps[CV(I)] = ok ? v : zero;
      });
    } else {
      static_for<0, NA>([&](auto I) __attribute__((always_inline)) { ps[CV(I)] = zero; });
    }
    if (A.hole_src && active) {
      const GateRef gr = A.gates[0];
      dispatch<0, K::n>(gate_code(MODE, NT, gr, pi), [&](auto CC) __attribute__((always_inline)) {
        hole_slice<R, NT, MODE, CV(CC)>(ps, ea, eb);
      });
    }
    for (int g = g0; g < A.ngates; ++g) {
      // this gate's phi tile is in LDS buffer `buf` once every wavefront's
      // loads completed: only this item's slice loads (NA vector-memory
      // instructions) were issued after it in the first gate, none later,
      // and none at all by a padding wavefront
      if (g == g0 && active)
        wait_vmcnt<NA>();
      else
        wait_vmcnt<0>();
      __syncthreads();
      // the other buffer was last read for the previous gate, which every
      // wavefront finished before the barrier: prefetch the next gate into it
      if (g + 1 < A.ngates)
        prefetch(rest, g + 1, buf ^ 1);
      else if (rest + rstride < A.n_rest)
        prefetch(rest + rstride, g0, buf ^ 1);
      asm volatile("" ::: "memory");
      if (active) {
        const GateRef gr = A.gates[g];
        ccoef_t<R> *co = coef + int64_t(gr.inst) * kCoefStride;
        const cx<R> *ph = phb + buf * NA * 64 + lane;
        R tp[NE];
        // -0: the first fma into each partial folds into a multiply
        static_for<0, NE>([&](auto E) __attribute__((always_inline)) { tp[CV(E)] = R(-0.0); });
        dispatch<0, K::n>(gate_code(MODE, NT, gr, pi), [&](auto CC) __attribute__((always_inline)) {
          contract_gate<R, NT, MODE, CV(CC), NE>(ps, ph, tp);
          fwd_gate<R, NT, MODE, false, CV(CC)>(ps, ps, co);
        });
        const double r = wave_reduce_scatter<R, NE>(tp, lane);
        if (writer) acc[g * NE + my_e] += r;
      }
      buf ^= 1;
    }
    if (ok && active) {
      char *dst = reinterpret_cast<char *>(A.psi) + int64_t(mu) * A.slab * ES + rowb;
      static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
        strow<R>(dst + boff(I), voff, ps[CV(I)]);
      });
    }
  }
  wait_vmcnt<0>();     // no direct load may still target LDS at exit
  if (writer && active)
    for (int g = g0; g < A.ngates; ++g) {
      double *s = A.slots + ((int64_t(A.gates[g].inst) * A.nd + mu) * A.ne + my_e) * A.nslots + gwave;
      *s += acc[g * NE + my_e];
    }
}

// States along the fused gate order: a wavefront carries the 2^NT amplitudes
// of its 64 columns on the pass's tile through the listed gates and stores
// the tile wherever a destination slab is given (before each gate, after the
// last), so a pass reads its input once instead of once per gate.
template <typename R, int NT, int MODE>
__global__ __launch_bounds__(kBlock) void k_state_pass(const StateArgs A) {
  constexpr int NA = 1 << NT;
  constexpr uint32_t ES = sizeof(cx<R>);
  using K = Codes<MODE, NT>;
  const int lane = threadIdx.x & 63;
  const int gwave = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * (kBlock / 64);
  ccoef_t<R> *coef = as_const_coef<R>(A.coef);
  int64_t bstep[NT];
  static_for<0, NT>([&](auto B) __attribute__((always_inline)) {
    bstep[CV(B)] = (int64_t(1) << A.pos[CV(B)]) * A.ld * ES;
  });
  auto boff = [&](auto I) __attribute__((always_inline)) {
    int64_t o = 0;
    static_for<0, NT>([&](auto B) __attribute__((always_inline)) {
      if constexpr ((CV(I) >> CV(B)) & 1) o += bstep[CV(B)];
    });
    return o;
  };
  for (int item = gwave; item < A.n_items; item += nwaves) {
    const int cg = item % A.ncg;
    int t = item / A.ncg;
    const int c = cg * 64 + lane;
    const bool ok = c < A.ncols;
    const uint32_t voff = uint32_t(ok ? c : A.ncols - 1) * ES;
    int64_t base = 0;
    for (int p = 0; p < A.kq; ++p)
      if (!((A.qmask >> p) & 1)) {
        base |= int64_t(t & 1) << p;
        t >>= 1;
      }
    const int pi = MODE == MODE_PARITY ? ((A.sector ^ __builtin_popcountll(base)) & 1) : 0;
    const int64_t rowb = base * A.ld * ES;
    const cx<R> zero{R(0), R(0)};
    cx<R> ps[NA];
    const char *src = reinterpret_cast<const char *>(A.src) + rowb;
    static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
      const cx<R> v = ldrow<R>(src + boff(I), voff);
      ps[CV(I)] = ok ? v : zero;
    });
    auto store = [&](void *dst) __attribute__((always_inline)) {
      if (dst && ok) {
        char *d = reinterpret_cast<char *>(dst) + rowb;
        static_for<0, NA>([&](auto I) __attribute__((always_inline)) {
          strow<R>(d + boff(I), voff, ps[CV(I)]);
        });
      }
    };
    for (int g = 0; g < A.ngates; ++g) {
      store(A.dst[g]);
      const GateRef gr = A.gates[g];
      ccoef_t<R> *co = coef + int64_t(gr.inst) * kCoefStride;
      dispatch<0, K::n>(gate_code(MODE, NT, gr, pi), [&](auto CC) __attribute__((always_inline)) {
        fwd_gate<R, NT, MODE, false, CV(CC)>(ps, ps, co);
      });
    }
    store(A.dst[A.ngates]);
  }
}

// Columns col0..col0+ncols of a slab (row stride ld_src) into a chunk slab,
// conjugated for phi = conj(U|j>) at the output side of the last gate; zero in
// padding columns.
template <typename R>
__global__ void k_copy_cols(const cx<R> *__restrict__ src, int64_t ld_src, int64_t col0,
                            cx<R> *__restrict__ dst, int64_t rows, int64_t ld, int ncols,
                            int conj) {
  const int64_t total = rows * ld;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = i % ld, x = i / ld;
    cx<R> v{R(0), R(0)};
    if (c < ncols) {
      v = src[x * ld_src + col0 + c];
      if (conj) v.y = -v.y;
    }
    dst[i] = v;
  }
}

// Zero columns [c0, c1) of n consecutive slabs of rows x ld elements: the
// padding columns of a ragged chunk's last 64-column group, which the sweep
// passes never write but the Hessian sweep reads (through LDS, unmasked).
template <typename R>
__global__ void k_zero_cols(cx<R> *__restrict__ p, int64_t n, int64_t rows, int64_t ld, int c0,
                            int c1) {
  const int w = c1 - c0;
  const int64_t total = n * rows * w;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = i / w;                   // slab * rows + row
    p[r * ld + c0 + (i % w)] = cx<R>{R(0), R(0)};
  }
}

// |j> for the chunk columns j = col0 + c.
template <typename R>
__global__ void k_onehot(cx<R> *__restrict__ dst, int64_t rows, int64_t ld, int64_t col0,
                         int ncols) {
  const int64_t total = rows * ld;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = i % ld, x = i / ld;
    cx<R> v{R(0), R(0)};
    if (c < ncols && x == col0 + c) v.x = R(1);
    dst[i] = v;
  }
}

// acc[r] += sum_s slots[r * nslots + s] (fixed-order tree).
__global__ __launch_bounds__(256) void k_accum_rows(const double *__restrict__ slots, int nslots,
                                                    double *__restrict__ acc) {
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
  if (threadIdx.x == 0) acc[blockIdx.x] += red[0];
}

// ---------------------------------------------------------------------------
// FP64 assembly per parameter pair (p, q):
//   Hh_pq[e][e'] = sum over instance pairs l in p, m in q, l before m of
//                  hh[l][m][e][e']  +  sum over l in q, m in p, l before m of
//                  hh[l][m][e'][e]           (d^2 h / dG_p[e] dG_q[e'])
// where "before" is the position in the fused gate order of the sweeps.
//   H[(p,r),(q,s)] = -Re sum_{e,e'} X_pr[e] Hh_pq[e][e'] X_qs[e']
//                    - delta_pq Re Tr[A_r^dagger A_s sym(G_p^dagger egrad_p)]
// with X_pr = G_p A_r (orthonormal tangent basis) -- the Riemannian Hessian
// of Sec. "Riemannian optimization" in coordinates; the second term is the
// Weingarten part of P_G(D egrad[X] - X sym(G^dagger egrad)).
// hh layout: [l][m][mu][e'] complex with e' the contraction entry at m (16
// dense, 8 parity) and mu the hole slice at l.
// ---------------------------------------------------------------------------
struct zc {
  double x, y;
};
__device__ inline zc zmul(zc a, zc b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

__global__ __launch_bounds__(256) void k_hess_post(
    int N, int P, int structure, int accumulate, const double *__restrict__ hh, const int32_t *__restrict__ inst_off,
    const int32_t *__restrict__ inst_list, const int32_t *__restrict__ ppos,
    const int32_t *__restrict__ map, const double *__restrict__ gates64,
    const double *__restrict__ egrad, const double *__restrict__ basis, double *hess_holo,
    double *hess_real) {
  const int p = blockIdx.x / P, q = blockIdx.x % P;
  __shared__ zc Hh[256], Xp[256], Xq[256];
  __shared__ zc Sp[16];
  const int t = threadIdx.x;
  // structure 0: U(4), d = 16 entries row-major; 1: parity, d = 8 pattern
  // entries; 2: particle number, d = 6 (the parity order without (0,3),
  // (3,0)).  Stored blocks are [d hole slices][nec contraction entries].
  const int d = structure == 0 ? 16 : structure == 1 ? 8 : 6;
  const int nec = structure == 0 ? 16 : 8;
  const int pidx[8] = {0, 3, 12, 15, 5, 6, 9, 10};
  const int nsel[6] = {0, 3, 4, 5, 6, 7};
  auto cidx = [&](int e) { return structure == 2 ? nsel[e] : e; };   // contraction entry
  auto epos = [&](int e) { return structure == 0 ? e : pidx[cidx(e)]; };  // 4x4 position
  // entry (r, c) of the block of instance pair (l, m), l before m along the
  // sweep order: a stored block, or the transpose of one (translation classes)
  auto blk = [&](int l, int m, int r, int c) -> const double * {
    const int32_t v = map[int64_t(l) * N + m];
    if (v >= 0) return hh + ((int64_t(v) * d + r) * nec + cidx(c)) * 2;
    const int64_t w = -int64_t(v) - 1;
    return hh + ((w * d + c) * nec + cidx(r)) * 2;
  };
  if (t < d * d) {
    const int e = t / d, f = t % d;
    double sx = 0, sy = 0;
    for (int i = inst_off[p]; i < inst_off[p + 1]; ++i)
      for (int j = inst_off[q]; j < inst_off[q + 1]; ++j) {
        const int l = inst_list[i], m = inst_list[j];
        if (ppos[l] < ppos[m]) {
          const double *h = blk(l, m, e, f);
          sx += h[0];
          sy += h[1];
        }
      }
    for (int i = inst_off[q]; i < inst_off[q + 1]; ++i)
      for (int j = inst_off[p]; j < inst_off[p + 1]; ++j) {
        const int l = inst_list[i], m = inst_list[j];
        if (ppos[l] < ppos[m]) {
          const double *h = blk(l, m, f, e);
          sx += h[0];
          sy += h[1];
        }
      }
    Hh[t] = {sx, sy};
    if (hess_holo) {
      double *o = hess_holo + ((((int64_t(p) * d + e) * P + q) * d + f) * 2);
      o[0] = accumulate ? o[0] + sx : sx;
      o[1] = accumulate ? o[1] + sy : sy;
    }
    // X_p[r][e] = (G_p A_r)[pos(e)], X_q likewise
    const int r = e, pe = epos(f);
    const int row = pe / 4, col = pe % 4;
    zc xp{0, 0}, xq{0, 0};
    for (int k2 = 0; k2 < 4; ++k2) {
      const zc a{basis[(r * 16 + k2 * 4 + col) * 2], basis[(r * 16 + k2 * 4 + col) * 2 + 1]};
      const zc gp{gates64[(p * 16 + row * 4 + k2) * 2], gates64[(p * 16 + row * 4 + k2) * 2 + 1]};
      const zc gq{gates64[(q * 16 + row * 4 + k2) * 2], gates64[(q * 16 + row * 4 + k2) * 2 + 1]};
      const zc u = zmul(gp, a), v = zmul(gq, a);
      xp.x += u.x;
      xp.y += u.y;
      xq.x += v.x;
      xq.y += v.y;
    }
    Xp[t] = xp;
    Xq[t] = xq;
  }
  if (t < 16 && p == q) {
    // S = sym(G^dagger egrad)
    const int i = t / 4, j = t % 4;
    zc s1{0, 0}, s2{0, 0};
    for (int k2 = 0; k2 < 4; ++k2) {
      const zc gki{gates64[(p * 16 + k2 * 4 + i) * 2], -gates64[(p * 16 + k2 * 4 + i) * 2 + 1]};
      const zc ekj{egrad[(p * 16 + k2 * 4 + j) * 2], egrad[(p * 16 + k2 * 4 + j) * 2 + 1]};
      const zc gkj{gates64[(p * 16 + k2 * 4 + j) * 2], -gates64[(p * 16 + k2 * 4 + j) * 2 + 1]};
      const zc eki{egrad[(p * 16 + k2 * 4 + i) * 2], egrad[(p * 16 + k2 * 4 + i) * 2 + 1]};
      const zc u = zmul(gki, ekj), v = zmul(gkj, eki);
      s1.x += u.x;
      s1.y += u.y;
      s2.x += v.x;
      s2.y += v.y;
    }
    Sp[t] = {0.5 * (s1.x + s2.x), 0.5 * (s1.y - s2.y)};
  }
  __syncthreads();
  if (t < d * d && hess_real) {
    const int r = t / d, s = t % d;
    double acc = 0.0;
    for (int e = 0; e < d; ++e) {
      zc inner{0, 0};
      for (int f = 0; f < d; ++f) {
        const zc u = zmul(Hh[e * d + f], Xq[s * d + f]);
        inner.x += u.x;
        inner.y += u.y;
      }
      const zc w = zmul(Xp[r * d + e], inner);
      acc -= w.x;
    }
    if (p == q) {
      // Re Tr[A_r^dagger A_s S]
      double tr = 0.0;
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          zc as_s{0, 0};
          for (int k2 = 0; k2 < 4; ++k2) {
            const zc a{basis[(s * 16 + i * 4 + k2) * 2], basis[(s * 16 + i * 4 + k2) * 2 + 1]};
            const zc u = zmul(a, Sp[k2 * 4 + j]);
            as_s.x += u.x;
            as_s.y += u.y;
          }
          // (A_r^dagger)[j][i] = conj(A_r[i][j]) contributes to trace index j
          const zc ar{basis[(r * 16 + i * 4 + j) * 2], -basis[(r * 16 + i * 4 + j) * 2 + 1]};
          tr += zmul(ar, as_s).x;
        }
      acc -= tr;
    }
    double *o = hess_real + (int64_t(p) * d + r) * (int64_t(P) * d) + int64_t(q) * d + s;
    *o = accumulate ? *o + acc : acc;
  }
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
template <typename R, int NT, int MODE, int W>
static size_t hess_lds() {
  constexpr int NE = MODE == MODE_DENSE ? 32 : 16;
  // phi double buffer [2][2^NT][64] and the wavefronts' FP64 accumulators
  return size_t(2) * (1 << NT) * 64 * sizeof(cx<R>) + size_t(W) * kMaxGates * NE * sizeof(double);
}

// grid < 0: return the number of blocks that are resident on the device at
// once (compute units x blocks per compute unit of this instantiation);
// otherwise launch.
template <typename R, int NT, int MODE, int W>
static int launch_hess_w(const HessArgs &a, int grid, void *s) {
  if (grid < 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (k_hess_pass<R, NT, MODE, W>),
                                                     W * 64, hess_lds<R, NT, MODE, W>()) !=
            hipSuccess)
      return -1;
    return cus * per_cu;
  }
  const size_t lds = hess_lds<R, NT, MODE, W>();
  hipLaunchKernelGGL((k_hess_pass<R, NT, MODE, W>), dim3(grid), dim3(W * 64), lds,
                     (hipStream_t)s, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// wavefronts per block of the hole-array sweep (any number of slices)
int hess_block_waves(int) { return 4; }

template <typename R, int NT, int MODE>
static int launch_hess_one(const HessArgs &a, int grid, void *s) {
  return launch_hess_w<R, NT, MODE, 4>(a, grid, s);
}

template <typename R, int NT, int MODE>
static int launch_state_one(const StateArgs &a, int grid, void *s) {
  hipLaunchKernelGGL((k_state_pass<R, NT, MODE>), dim3(grid), dim3(kBlock), 0, (hipStream_t)s, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_state_pass(int is_double, int nt, int mode, const StateArgs &a, int grid, void *s) {
  if (!is_double) {
    if (nt == 5 && mode) return launch_state_one<float, 5, 1>(a, grid, s);
    if (nt == 4) return mode ? launch_state_one<float, 4, 1>(a, grid, s) : launch_state_one<float, 4, 0>(a, grid, s);
    if (nt == 2) return mode ? launch_state_one<float, 2, 1>(a, grid, s) : launch_state_one<float, 2, 0>(a, grid, s);
  } else {
    if (nt == 4) return mode ? launch_state_one<double, 4, 1>(a, grid, s) : launch_state_one<double, 4, 0>(a, grid, s);
    if (nt == 2) return mode ? launch_state_one<double, 2, 1>(a, grid, s) : launch_state_one<double, 2, 0>(a, grid, s);
  }
  return -3;
}

int launch_hess_pass(int is_double, int nt, int mode, const HessArgs &a, int grid, void *s) {
  if (!is_double) {
    if (nt == 5 && mode) return launch_hess_one<float, 5, 1>(a, grid, s);
    if (nt == 4) return mode ? launch_hess_one<float, 4, 1>(a, grid, s) : launch_hess_one<float, 4, 0>(a, grid, s);
    if (nt == 2) return mode ? launch_hess_one<float, 2, 1>(a, grid, s) : launch_hess_one<float, 2, 0>(a, grid, s);
  } else {
    if (nt == 4) return mode ? launch_hess_one<double, 4, 1>(a, grid, s) : launch_hess_one<double, 4, 0>(a, grid, s);
    if (nt == 2) return mode ? launch_hess_one<double, 2, 1>(a, grid, s) : launch_hess_one<double, 2, 0>(a, grid, s);
  }
  return -3;
}

static int grid_of(int64_t total) {
  int64_t b = (total + 255) / 256;
  return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

int launch_copy_cols(int is_double, const void *src, int64_t ld_src, int64_t col0, void *dst,
                     int64_t rows, int64_t ld, int ncols, bool conj, void *s) {
  const int g = grid_of(rows * ld);
  if (is_double)
    hipLaunchKernelGGL(k_copy_cols<double>, dim3(g), dim3(256), 0, (hipStream_t)s,
                       (const cx<double> *)src, ld_src, col0, (cx<double> *)dst, rows, ld, ncols,
                       conj ? 1 : 0);
  else
    hipLaunchKernelGGL(k_copy_cols<float>, dim3(g), dim3(256), 0, (hipStream_t)s,
                       (const cx<float> *)src, ld_src, col0, (cx<float> *)dst, rows, ld, ncols,
                       conj ? 1 : 0);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_onehot(int is_double, void *dst, int64_t rows, int64_t ld, int64_t col0, int ncols,
                  void *s) {
  const int g = grid_of(rows * ld);
  if (is_double)
    hipLaunchKernelGGL(k_onehot<double>, dim3(g), dim3(256), 0, (hipStream_t)s,
                       (cx<double> *)dst, rows, ld, col0, ncols);
  else
    hipLaunchKernelGGL(k_onehot<float>, dim3(g), dim3(256), 0, (hipStream_t)s, (cx<float> *)dst,
                       rows, ld, col0, ncols);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_zero_cols(int is_double, void *p, int64_t n, int64_t rows, int64_t ld, int c0, int c1,
                     void *s) {
  if (c1 <= c0 || n == 0) return 0;
  const int g = grid_of(n * rows * (c1 - c0));
  if (is_double)
    hipLaunchKernelGGL(k_zero_cols<double>, dim3(g), dim3(256), 0, (hipStream_t)s,
                       (cx<double> *)p, n, rows, ld, c0, c1);
  else
    hipLaunchKernelGGL(k_zero_cols<float>, dim3(g), dim3(256), 0, (hipStream_t)s,
                       (cx<float> *)p, n, rows, ld, c0, c1);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_accum_rows(const double *slots, int rows, int nslots, double *acc, void *s) {
  if (rows == 0) return 0;
  hipLaunchKernelGGL(k_accum_rows, dim3(rows), dim3(256), 0, (hipStream_t)s, slots, nslots, acc);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_hess_post(int N, int P, int structure, int accumulate, const double *hh,
                     const int32_t *inst_off, const int32_t *inst_list, const int32_t *ppos,
                     const int32_t *map, const double *gates64, const double *egrad,
                     const double *basis, double *hess_holo, double *hess_real, void *s) {
  hipLaunchKernelGGL(k_hess_post, dim3(P * P), dim3(256), 0, (hipStream_t)s, N, P, structure,
                     accumulate, hh, inst_off, inst_list, ppos, map, gates64, egrad, basis,
                     hess_holo, hess_real);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// dst[i] += src[i] (accumulating Hessian calls: f and the gradients)
__global__ void k_add(double *__restrict__ dst, const double *__restrict__ src, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    dst[i] += src[i];
}

int launch_add(double *dst, const double *src, int64_t n, void *s) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_add, dim3(unsigned(std::min<int64_t>((n + 255) / 256, 1024))), dim3(256),
                     0, (hipStream_t)s, dst, src, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace rqk
