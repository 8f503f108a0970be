// Internal declarations shared by the host side of librq and its kernels.
#pragma once

#include <stdint.h>

namespace rqk {

// Maximum gate instances in one sweep pass.
constexpr int kMaxGates = 16;
// Threads per block of the sweep kernels (4 wavefronts of 64 lanes).
constexpr int kBlock = 256;
// Maximum number of wavefronts of a sweep grid; also the number of FP64
// partial-sum slots per accumulated quantity.
constexpr int kMaxWaves = 2048;
// Largest qubit count with particle-number-sector storage (its rank table
// holds 2^k int32 entries).
constexpr int kMaxSectorQubits = 28;
// Complex coefficients stored per gate instance:
//   [ 0,16) G      [16,32) G^-1      [32,48) Z      [48,64) G^-1 Z
// dense gates row-major 4x4; parity gates the 8 pattern entries in the order
// (0,0),(0,3),(3,0),(3,3),(1,1),(1,2),(2,1),(2,2).
constexpr int kCoefStride = 64;

// MODE_NUMBER: particle-number-conserving gates on states stored per
// particle-number sector (rows = colex rank of the basis state within its
// sector); the gate arithmetic is that of MODE_PARITY.
enum Mode { MODE_DENSE = 0, MODE_PARITY = 1, MODE_NUMBER = 2 };
enum Op { OP_COST = 0, OP_GRAD = 1, OP_HVP = 2, OP_APPLY = 3 };
enum Stage { ST_FWD = 0, ST_LAST = 1, ST_BWD = 2 };

// One gate of a pass.  kind 0: both qubits in the tile (local bits h, l);
// kind 1: parity mode, q_lo is the implied qubit k-1 (h = local bit of q_hi);
// kind 2: parity mode, q_hi is the implied qubit (h = local bit of q_lo).
struct GateRef {
  int16_t inst;
  int16_t kind;
  int16_t h;
  int16_t l;
};

struct PassArgs {
  const void *coef;        // per-instance coefficients (state precision)
  const void *src_psi;     // FWD / LAST input states (NULL: one-hot |j>),
                           // row stride ld_src
  const void *src_dpsi;    // HVP tangent input (NULL: zero)
  void *dst_psi;           // FWD output (checkpoint / in-place apply)
  void *dst_dpsi;
  const void *ckpt_psi;    // BWD: states after this pass
  const void *ckpt_dpsi;
  void *phi;               // BWD in/out, LAST out
  void *dphi;
  const void *ref;         // LAST: target columns U|j> (sector block)
  const int32_t *rank;     // MODE_NUMBER: colex rank of every basis index
                           // within its particle-number sector [2^k]
  double *slots;           // FP64 partials [inst][entry][slot]
  double *fslots;          // FP64 partials of f [slot]
  int64_t ld;              // row stride of the chunk slabs (elements)
  int64_t ld_src;          // row stride of src_psi (elements)
  int64_t ld_ref;          // row stride of ref (elements)
  int64_t col0;            // basis column of chunk column 0
  int32_t ncols;           // valid columns of the chunk
  int32_t ncg;             // column groups of 64
  int32_t kq;              // explicit qubits (k, or k-1 in parity mode)
  int32_t n_items;         // tiles * column groups
  uint32_t qmask;          // bit positions (in the row index) of the tile
  int32_t sector;          // parity sector p (0 in general mode); particle
                           // number n in MODE_NUMBER
  int32_t ngates;
  int32_t nslots;
  int32_t store_phi;
  int32_t ne;              // FP64 entries per instance in slots
  int32_t pos[8];          // row bit position of local tile bit b
  GateRef gates[kMaxGates];
};

// One Hessian hole-array sweep pass (k_hess_pass): the nd slices of the
// array of one hole gate through the gates of one pass, contracted against
// the stored phi after each gate.
struct HessArgs {
  const void *coef;      // per-instance coefficients (state precision)
  void *psi;             // hole-array slices [nd][rows][ld]
  const void *phi;       // phi at the output side of every gate [N][rows][ld]
  const void *hole_src;  // first pass after a hole: psi before the hole gate,
                         // which is gate 0 of the list (no contraction there);
                         // NULL: the slices are read from psi
  double *slots;         // FP64 partials [((inst * nd + mu) * ne + e) * nslots + wave]
  int64_t ld;            // row stride of the slabs (elements)
  int64_t slab;          // rows * ld (elements)
  int32_t ncols, ncg, kq;
  int32_t n_rest;        // tiles * column groups
  int32_t nd;            // slices (16 dense, 8 parity, 6 particle number)
  int32_t nquads;        // blocks per item: ceil(nd / 4)
  int32_t nslots, sector, ngates, ne;
  uint32_t qmask;
  int32_t pos[8];
  GateRef gates[kMaxGates];
};
// One pass of the Hessian's per-gate state sweeps (k_state_pass): the tile
// of src is carried through the gates of the list (coefficients G, or G^T
// for the backward states), storing the tile before gate g to dst[g] and
// after the last gate to dst[ngates] (NULL: not stored).
struct StateArgs {
  const void *coef;
  const void *src;
  void *dst[kMaxGates + 1];
  int64_t ld;
  int32_t ncols, ncg, kq, n_items, sector, ngates;
  uint32_t qmask;
  int32_t pos[8];
  GateRef gates[kMaxGates];
};

// FP64 partial-sum slots (one per wavefront) of the Hessian sweeps: four
// wavefronts per SIMD of 256 compute units.
constexpr int kHessSlots = 4096;
// Accelerator complex dies (XCDs, each with its own L2) over which the
// hardware deals consecutive workgroups of a launch in turn.
constexpr int kXcds = 8;

// Host-side launchers (defined in rq_launch.hip, rq_hess.hip and the sweep
// instantiation units).
int launch_pass(int is_double, int nt, int mode, int op, int stage,
                const PassArgs &a, int grid, void *stream);
int launch_reduce(const double *slots, int n_inst, int ne, int nslots,
                  double *out, void *stream);
int launch_zero(double *p, int64_t n, void *stream);
int launch_rank_table(int32_t *rank, int k, void *stream);
int launch_stream_copy(void *dst, const void *src, int64_t bytes, int unroll, int blocks,
                       void *stream);
int launch_orbit_fill(int is_double, const void *ref_in, int64_t ld_in, int64_t sector_stride_in,
                      const int64_t *reps, const double *sw, void *inputs, void *ref_out,
                      int nsec, int64_t rows, int64_t width, void *stream);
int launch_post(int op, int parity, int accumulate, int n_params, int n_inst, const int32_t *param_of,
                const double *tsum, int ne, const double *fslots, int nslots,
                const double *gates64, const double *dir64, double *d_f,
                double *d_egrad, double *d_rgrad, double *d_ehvp, double *d_rhvp,
                void *stream);

}  // namespace rqk
