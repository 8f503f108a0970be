/*
 * rq.h -- C ABI of librq: matrix-free evaluation of the circuit cost
 *         f(G) = -Re Tr[U^dagger C(G)], its Riemannian gradient, Hessian-vector
 *         products and Hessian blocks on one AMD Instinct MI355X (gfx950).
 *
 * Method: arXiv 2506.23775 ("High-Performance Contraction of Quantum Circuits
 * for Riemannian Optimization").  The trace is a sum over computational basis
 * states |j> (eq. for the basis-vector sum in Sec. "Objective function and
 * matrix-free evaluation"); every entry point below evaluates that sum, or a
 * contiguous range of it, with hand-written HIP kernels.
 *
 * Conventions (all entry points)
 * ------------------------------
 *  - k qubits; qubit q is bit (k-1-q) of a basis index: qubit 0 is the most
 *    significant tensor leg (Sec. "Gate application").
 *  - A gate instance acts on a pair (q_hi, q_lo), q_hi != q_lo, any two
 *    qubits.  Its 4x4 matrix is indexed by 2*bit(q_hi) + bit(q_lo).
 *  - C(G) = G_N ... G_1: instance 0 of the pair list is applied first (Sec.
 *    "Quantum circuits").  Repeated gates (brick-wall translation sharing,
 *    Sec. "Brick wall circuit layout") are instances mapped to one parameter
 *    by param_of; derivatives of a parameter sum over its instances.
 *  - Complex numbers are interleaved (re, im).  Gate arrays are host
 *    double [P][4][4][2], row-major.
 *  - State slabs ("batch-interleaved"): amplitude x of basis column c is at
 *    element x*ld + c; complex128 (RQ_C128) or complex64 (RQ_C64) elements.
 *  - Parity mode (RQ_PARITY, Sec. "Parity-conserving gate structure"): every
 *    gate has the pattern rows/cols {0,3} x {0,3} + {1,2} x {1,2}; entries off
 *    the pattern are ignored (read as zero) and returned as zero.  States live
 *    in one parity sector p and are stored compressed: amplitude x (parity p)
 *    at row x >> 1 (the bit of qubit k-1 is implied).  A sector has 2^(k-1)
 *    basis columns j' = j >> 1.
 *  - Particle-number mode (RQ_PARITY | RQ_NUMBER; the further restriction of
 *    Sec. "Parity-conserving gate structure" that removes two parameters):
 *    gates are U(1) x U(2) x U(1) on {00}, {01,10}, {11}, i.e. the parity
 *    pattern without (0,3) and (3,0); those two entries are also ignored and
 *    returned as zero.  States are stored as in parity mode; the Hessian
 *    propagates 6 hole slices instead of 8 and its blocks have d = 6 entries
 *    in the order (0,0),(3,3),(1,1),(1,2),(2,1),(2,2).
 *  - Particle-number sectors (RQ_PARITY | RQ_NUMBER | RQ_SECTORS): the same
 *    gates, with states stored per particle-number sector (the sectors such
 *    gates keep closed; Sec. "Parity-conserving gate structure"): sector n
 *    (0 <= n <= k) holds the C(k, n) basis states of popcount n, state x at
 *    row rank(x) = number of basis indices y < x of the same popcount.  The
 *    trace then sums C(k, n)^2 amplitudes per sector (sum over n: C(2k, k))
 *    instead of 2 * 4^(k-1).  rq_sector_rows gives the stacked row of every
 *    basis index used by the target layout.  Not available for
 *    rq_hess_blocks, input states or the orbit functions.  This mode is
 *    currently switched off: every entry point returns RQ_EINVAL for a
 *    circuit with RQ_SECTORS (its kernels took a device memory fault whose
 *    cause is not found yet); rq_sector_rows works.
 *  - Precision: states and reference columns are stored and propagated in the
 *    target dtype; every contraction is accumulated in FP64 (per-lane partial
 *    sums of at most 2^(tile-2) products in the state precision, then FP64).
 *    Riemannian post-processing is FP64.
 *
 * Memory, streams, errors
 * -----------------------
 *  - The library allocates no device memory.  The caller owns the reference
 *    columns, the workspace (size from rq_workspace_bytes) and every device
 *    output.  Host inputs are read during the call only.
 *  - Calls are stream-ordered and asynchronous with respect to the host:
 *    they enqueue kernels and small host-to-device copies on exec->stream and
 *    return; device outputs are valid once the stream reaches that point.
 *    Two calls that run concurrently must use distinct workspaces.
 *  - Every call returns RQ_OK (0) or an error code; rq_last_error() returns a
 *    thread-local message for the last failing call of the calling thread.
 *    On an argument error nothing is enqueued and no output is written.
 */
#ifndef RQ_H
#define RQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define RQ_OK         0
#define RQ_EINVAL     1   /* invalid argument (shape, pair, range, flag)      */
#define RQ_EHIP       2   /* HIP runtime error while enqueueing               */
#define RQ_ESPACE     3   /* workspace too small for the requested chunk      */
#define RQ_ESINGULAR  4   /* gate (block) not invertible within tolerance     */

/* ---- state / reference precision ---------------------------------------- */
#define RQ_C128 0         /* complex double states                            */
#define RQ_C64  1         /* complex float states, FP64 accumulation          */

/* ---- circuit flags ------------------------------------------------------ */
#define RQ_PARITY 1u      /* parity-conserving gates, sector-compressed states */
#define RQ_NUMBER 2u      /* with RQ_PARITY: particle-number-conserving gates   */
#define RQ_SECTORS 4u     /* with RQ_PARITY | RQ_NUMBER: states stored per
                             particle-number sector                           */

/* ---- operations (for rq_workspace_bytes) -------------------------------- */
#define RQ_OP_COST  0
#define RQ_OP_GRAD  1
#define RQ_OP_HVP   2
#define RQ_OP_HESS  3
#define RQ_OP_APPLY 4

/* Circuit topology (host memory, read during a call).
 * pairs:    [n_gates][2] (q_hi, q_lo), 0 <= q < n_qubits, q_hi != q_lo.
 * param_of: [n_gates] parameter of each instance in [0, n_params), or NULL
 *           for the identity map (then n_params must equal n_gates).
 * n_qubits: 2..30 (4..31 with RQ_PARITY).
 * shift:    0, or s in [1, n_qubits): the caller states that the circuit and
 *           the target are invariant under the cyclic qubit translation
 *           q -> (q + s) mod n_qubits (Sec. "Exploiting translational
 *           invariance").  The library checks the circuit part -- every
 *           instance maps to an instance of the same parameter on the shifted
 *           pair, in the same order on every qubit -- and rejects the circuit
 *           otherwise (RQ_EINVAL); the target's invariance is the caller's
 *           promise.  rq_hess_blocks then sweeps only the gate holes needed
 *           for one pair of each translation class over the full trace and
 *           fills the others by translation.  Ignored for basis sub-ranges
 *           and input states (their sums are not translation invariant). */
typedef struct rq_circuit {
  int32_t n_qubits;
  int32_t n_gates;
  int32_t n_params;
  uint32_t flags;
  const int32_t *pairs;
  const int32_t *param_of;
  int32_t shift;
  int32_t reserved;
} rq_circuit;

/* Target U given by its columns U|j> on the device (Sec. "Objective function
 * and matrix-free evaluation": the bra side of summand j is (U|j>)^*).
 * General mode: ref[x*ld + j] = U[x][j], x, j < 2^k.
 * Parity mode:  ref[s*sector_stride + x'*ld + j'] = U[x][j] for the sector s
 *               blocks (U conserves parity), x', j' < 2^(k-1).
 * Particle-number sectors (RQ_SECTORS): ref[(first(n) + rank(x))*ld +
 *               rank(j)] = U[x][j] for x, j of popcount n (U conserves
 *               particle number), first(n) = sum of C(k, m) for m < n, i.e.
 *               the sector blocks stacked by n (stacked rows from
 *               rq_sector_rows); ld >= C(k, k/2); sector_stride is ignored.
 * Only the columns of the requested basis range are read, so ref may point
 * (by offset) into a narrower window of columns.
 * dtype is also the state precision of the evaluation.
 *
 * Input states (sampling the trace over random vectors instead of the basis,
 * the follow-up outlined in Sec. "Conclusions"): if inputs is not NULL,
 * summand j starts from the state |psi_j> = inputs column j instead of |j>,
 * laid out like ref (inputs[x*in_ld + j], or
 * inputs[s*in_sector_stride + x'*in_ld + j'] for a sector-s state in parity
 * mode), and ref column j must then hold U|psi_j>.  Every output becomes the
 * same function of the sum over j of <psi_j| U^dagger C(G) |psi_j>; scaling
 * it into a trace estimate is left to the caller.  NULL inputs: in_ld and
 * in_sector_stride are ignored. */
typedef struct rq_target {
  int32_t dtype;
  int32_t reserved;
  const void *ref;
  int64_t ld;
  int64_t sector_stride;
  const void *inputs;
  int64_t in_ld;
  int64_t in_sector_stride;
} rq_target;

/* Range of basis states of the trace sum.  General mode: j in
 * [begin, begin+count) of [0, 2^k), sector must be -1.  Parity mode: sector
 * 0 or 1 and j' in [begin, begin+count) of [0, 2^(k-1)), or sector -1 with
 * begin 0 and count 2^(k-1) for both sectors (with input states: sector -1
 * takes [begin, begin+count) in both sectors).  Particle-number sectors:
 * sector n in [0, k] and rank(j) in [begin, begin+count) of [0, C(k, n)), or
 * sector -1 with begin 0 and count 2^k for every sector in full.  A NULL
 * range is the full trace.  count 0 is allowed (all outputs are then the
 * empty sum, projected). */
typedef struct rq_range {
  int32_t sector;
  int32_t reserved;
  int64_t begin;
  int64_t count;
} rq_range;

/* Execution resources.  workspace: device memory of at least
 * rq_workspace_bytes(circuit, op, dtype, chunk) bytes, 256-byte aligned.
 * chunk: basis columns per sweep (multiple of 64, >= 64).  stream: a
 * hipStream_t (NULL = default stream).  flags: RQ_EXEC_ACCUMULATE makes
 * rq_cost / rq_grad / rq_hvp / rq_hess_blocks add their results to the device
 * outputs instead of overwriting them (at fixed gates every output, the real
 * Riemannian Hessian included, is linear in the basis-state sum, so the
 * partial sums of disjoint ranges add up to the sum over their union). */
#define RQ_EXEC_ACCUMULATE 1u
typedef struct rq_exec {
  void *workspace;
  size_t workspace_bytes;
  int64_t chunk;
  void *stream;
  uint32_t flags;
  uint32_t reserved;
} rq_exec;

/* Bytes of workspace needed for op (RQ_OP_COST, RQ_OP_GRAD, RQ_OP_HVP,
 * RQ_OP_APPLY) with states of dtype and the given chunk.  Returns 0 for
 * invalid arguments (see rq_last_error), including RQ_OP_HESS, whose
 * workspace rq_hess_workspace_bytes gives. */
size_t rq_workspace_bytes(const rq_circuit *circuit, int32_t op, int32_t dtype,
                          int64_t chunk);

/* f = -Re sum_{j in range} <j| U^dagger C(G) |j>   (eq. for the target
 * function and its basis-vector sum).
 * gates: host double [P][4][4][2].  d_f: device double[1]. */
int rq_cost(const rq_circuit *circuit, const rq_target *target,
            const double *gates, const rq_range *range, const rq_exec *exec,
            double *d_f);

/* Gradient (Sec. "Efficient gradient and Hessian computation": forward pass
 * with cached states, backward pass with transposed gates, gate-hole
 * contractions of Sec. "Gate gradient as a gate hole").
 * Outputs (device, each nullable):
 *   d_f      double[1]            f as in rq_cost
 *   d_egrad  double[P][4][4][2]   Euclidean gradient  -conj(dh/dG_p)  (gradient
 *                                 convention d_x f + i d_y f, Sec. "Riemannian
 *                                 optimization"), summed over instances
 *   d_rgrad  double[P][4][4][2]   Riemannian gradient P_G(egrad), with the
 *                                 projection P_V X = V skew(V^dagger X). */
int rq_grad(const rq_circuit *circuit, const rq_target *target,
            const double *gates, const rq_range *range, const rq_exec *exec,
            double *d_f, double *d_egrad, double *d_rgrad);

/* Hessian-vector product along a tangent direction (appendix on
 * Hessian-vector products: forward-mode directed gradient, then
 * backpropagation; Riemannian Hessian Hess f[X] = nabla_X grad f with the
 * Levi-Civita connection of Sec. "Riemannian optimization").
 * dir: host double [P][4][4][2], a tangent vector X_p = G_p A_p (A_p anti-
 * Hermitian); it is used as given (not re-projected).
 * Outputs (device, nullable): f, egrad, rgrad as rq_grad, and
 *   d_ehvp  double[P][4][4][2]   D egrad[X] = -conj(d/deps dh/dG_p)
 *   d_rhvp  double[P][4][4][2]   P_G(D egrad[X] - X sym(G^dagger egrad)). */
int rq_hvp(const rq_circuit *circuit, const rq_target *target,
           const double *gates, const double *dir, const rq_range *range,
           const rq_exec *exec, double *d_f, double *d_egrad, double *d_rgrad,
           double *d_ehvp, double *d_rhvp);

/* All pairwise Hessian blocks (Sec. "Efficient gradient and Hessian
 * computation": gate-hole application to a state, second forward pass of the
 * 16-entry state array (8 in parity mode), contraction at every later gate).
 * Outputs (device, nullable):
 *   d_f, d_egrad, d_rgrad as rq_grad;
 *   d_hess_holo  double[P][d][P][d][2]  holomorphic second derivatives
 *                d^2 h / dG_p[e] dG_q[e'] summed over instances, d = 16 entries
 *                (a,b) row-major, or d = 8 pattern entries in parity mode in
 *                the order (0,0),(0,3),(3,0),(3,3),(1,1),(1,2),(2,1),(2,2),
 *                or d = 6 in particle-number mode (the same order without
 *                (0,3), (3,0));
 *   d_hess_real  double[P*d][P*d]   Riemannian Hessian in the orthonormal
 *                tangent basis X_{p,mu} = G_p A_mu documented in
 *                rq_tangent_basis (d = 16, 8 in parity, 6 in number mode). */
int rq_hess_blocks(const rq_circuit *circuit, const rq_target *target,
                   const double *gates, const rq_range *range,
                   const rq_exec *exec, double *d_f, double *d_egrad,
                   double *d_rgrad, double *d_hess_holo, double *d_hess_real);

/* Bytes of workspace needed by rq_hess_blocks for states of dtype and the
 * given chunk (multiple of 64).  Returns 0 for invalid arguments. */
size_t rq_hess_workspace_bytes(const rq_circuit *circuit, int32_t dtype,
                               int64_t chunk);

/* Apply the circuit to a slab of states in place (Sec. "Gate application"):
 * states[x*ld + c] for c < n_states, x < 2^k (general) or sector-compressed
 * x' < 2^(k-1) of the given sector (parity mode; sector must then be 0/1,
 * otherwise -1), or x' = rank(x) < C(k, n) of particle-number sector n
 * (RQ_SECTORS; sector in [0, k]).  Any number of columns; ld >= n_states.  Used to prepare
 * target columns U|j> from a gate list (e.g. a Trotter circuit).
 * exec: workspace of rq_workspace_bytes(circuit, RQ_OP_APPLY, dtype, 0)
 * bytes (gate coefficients) and the stream; exec->chunk is ignored. */
int rq_apply_circuit(const rq_circuit *circuit, const double *gates,
                     void *d_states, int64_t n_states, int64_t ld,
                     int32_t dtype, int32_t sector, const rq_exec *exec);

/* One trust-region step on the host in FP64 (Sec. "Riemannian optimization":
 * quadratic model, truncated CG of Absil et al. Algorithm 11, polar retraction
 * R_V(xi) = q_polar(V + xi) per gate).  Host inputs: gates [P][4][4][2], the
 * Riemannian gradient g and Hessian H in the basis of rq_tangent_basis
 * (n = P*d), radius delta.  Host outputs: eta[n] (step), cand [P][4][4][2]
 * (retracted gates), model_decrease (m(0) - m(eta)), stop (0 converged,
 * 1 boundary, 2 negative curvature, 3 iteration limit, 4 zero gradient).
 * Constants: theta = 1, kappa = 0.1. */
int rq_tr_step(int32_t n_params, uint32_t flags, const double *gates,
               const double *g, const double *H, double delta, double *eta,
               double *cand, double *model_decrease, int32_t *stop);

/* Coordinates of matrices Y_p (host [P][4][4][2]) in the orthonormal tangent
 * basis of rq_tangent_basis at the gates G_p: out[p*d + mu] =
 * Re Tr[(G_p A_mu)^dagger Y_p] (host double[P*d]).  With Y the Euclidean
 * gradient this is the Riemannian gradient vector taken by rq_tr_step (the
 * projection onto the tangent space is orthogonal). */
int rq_tangent_coords(int32_t n_params, uint32_t flags, const double *gates,
                      const double *Y, double *out);

/* Riemannian trust-region optimisation (Sec. "Riemannian optimization": the
 * trust-region method of Absil et al., Algorithm 10, with the truncated-CG
 * inner solver and the polar retraction of rq_tr_step).  Each iteration
 * evaluates f, the gradient and the real Riemannian Hessian with
 * rq_hess_blocks on the device (skipped after a rejected step, whose point
 * is unchanged), takes rq_tr_step on the host, evaluates f at the candidate
 * with rq_cost and accepts or shrinks with rq_tr_accept.  Radius: starts at
 * delta_bar / 8 with delta_bar = sqrt(P*d) * pi.
 * gates (host [P][4][4][2]): starting point on input, last accepted iterate on
 * output.  Stops after max_iter iterations or when the Riemannian gradient
 * norm is <= gtol.  history (host, nullable): double[max_iter][6] rows
 * (f, |grad f|, delta, rho, accepted, tCG stop code) per iteration;
 * *n_iter receives the number of rows written.
 * exec: workspace of rq_tr_workspace_bytes(circuit, dtype, chunk) bytes; the
 * call synchronizes exec->stream every iteration (host decisions). */
size_t rq_tr_workspace_bytes(const rq_circuit *circuit, int32_t dtype,
                             int64_t chunk);
int rq_tr_solve(const rq_circuit *circuit, const rq_target *target,
                double *gates, const rq_range *range, const rq_exec *exec,
                int32_t max_iter, double gtol, double *history,
                int32_t *n_iter);

/* Trust-region acceptance and radius update after evaluating f at the
 * candidate: rho = (f0 - f1) / model_decrease; accepted = rho > 0.1; radius
 * quartered if rho < 1/4, doubled (capped at delta_bar) if rho > 3/4 and the
 * step norm eta_norm equals delta.  Host scalars only. */
int rq_tr_accept(double f0, double f1, double model_decrease, double delta,
                 double delta_bar, double eta_norm, double *new_delta,
                 int32_t *accepted, double *rho);

/* Orthonormal tangent basis A_mu (host output double[d][4][4][2]) used by
 * rq_hess_blocks / rq_tr_step: X_{p,mu} = G_p A_mu.  Returns d: 16 (U(4)),
 * 8 with RQ_PARITY (U(2) x U(2)), 6 with RQ_PARITY | RQ_NUMBER
 * (U(1) x U(2) x U(1): i E_00, i E_33, i E_11, i E_22, (E_12 - E_21)/sqrt2,
 * i (E_12 + E_21)/sqrt2). */
int rq_tangent_basis(uint32_t flags, double *basis);

/* Basis-orbit reduction of the trace sum (an extension of Sec. "Exploiting
 * translational invariance", which shares Hessian hole pairs between
 * translated gates, to the sum over basis states).  When the circuit and the
 * target are invariant under the cyclic qubit translation by `shift`, the
 * summand of |j> equals that of every translate of |j>, so the trace is the
 * sum over one representative per orbit weighted by the orbit size w.  With
 * input states sqrt(w_r)|rep_r> and target columns sqrt(w_r) U|rep_r>
 * (every output is bilinear in the two), rq_cost / rq_grad / rq_hvp over the
 * representatives return the full-trace results.
 *
 * rq_orbit_reps (host): representatives (the smallest basis index of each
 * orbit under q -> q + shift, ascending) and orbit sizes as doubles, for all
 * 2^k basis states (sector -1) or the states of one popcount parity (sector
 * 0 / 1, representatives as compressed rows j >> 1).  *count: capacity of
 * reps / weights on input, number of representatives on output; with reps
 * and weights both NULL only the count is returned.  RQ_EINVAL for bad
 * arguments or short arrays. */
int rq_orbit_reps(int32_t n_qubits, int32_t shift, int32_t sector, int64_t *count,
                  int64_t *reps, double *weights);

/* Workspace bytes of rq_orbit_target for output slabs of `width` columns
 * (0 on invalid arguments). */
size_t rq_orbit_workspace_bytes(const rq_circuit *circuit, int64_t width);

/* Fill device slabs with the orbit-weighted input states and target
 * columns for circuit->shift (which must be nonzero; the circuit's own
 * invariance is checked as for every call, the target's is the caller's
 * promise).  target: the full basis-state target of rq_target (no inputs;
 * every column j < 2^k, or 2^(k-1) per sector, present: ld >= that count).
 * d_inputs, d_ref: device slabs of the target's dtype, laid out as
 * [rows][width] (general) or [2][rows][width] (parity: sector s at
 * s * rows * width), rows = 2^k or 2^(k-1); column r < count of a sector
 * holds sqrt(w_r)|rep_r> and sqrt(w_r) U|rep_r>, later columns zero.
 * width >= the largest per-sector count (rq_orbit_reps).  Use the result
 * as rq_target{dtype, 0, d_ref, width, rows * width, d_inputs, width,
 * rows * width} with the range (sector -1, 0, width) in parity mode or
 * (-1, 0, width) otherwise.  Workspace: rq_orbit_workspace_bytes.  The call
 * uploads the representatives, synchronizes exec->stream once (set-up
 * call) and enqueues one fill kernel. */
int rq_orbit_target(const rq_circuit *circuit, const rq_target *target, void *d_inputs,
                    void *d_ref, int64_t width, const rq_exec *exec);

/* Diagnostics: gate instances per sweep pass chosen by the scheduler for op
 * and dtype.  pass_of[n_gates] (host) receives the pass index of every
 * instance; returns the number of passes (< 0 on error). */
int rq_plan_passes(const rq_circuit *circuit, int32_t op, int32_t dtype,
                   int32_t *pass_of);

/* Diagnostics: with profiling enabled, every sweep-kernel launch is
 * bracketed by HIP events recorded on the launch's own stream.
 * rq_profile_read synchronizes those events and returns, per kind
 * k = 3*op + stage for k < 12 (op: 0 cost, 1 grad, 2 HVP, 3 apply; stage:
 * 0 forward pass, 1 fused last pass, 2 backward pass), and k = 12 Hessian
 * hole-array sweep, 13 Hessian per-gate state passes, 14 gate-hole
 * application, 15 rq_stream_copy, the summed kernel time in ms, the number
 * of launches, and the algorithmic HBM bytes and flops of those launches
 * (arrays of 16 entries each, any may be NULL); then it resets. */
int rq_profile_enable(int on);
int rq_profile_read(double *ms, int64_t *launches, double *bytes,
                    double *flops);

/* Stacked particle-number-sector row of every basis index (host):
 * row_of[x] = first(popcount(x)) + rank(x) for x < 2^n_qubits (the row of
 * U[x][.] in an RQ_SECTORS target), n_qubits in [1, 28].  row_of: host
 * int64[2^n_qubits].  Returns RQ_EINVAL for bad arguments. */
int rq_sector_rows(int32_t n_qubits, int64_t *row_of);

/* Diagnostics: streaming device-to-device copy of `bytes` bytes (a multiple
 * of 16; both pointers 16-byte aligned) by a hand-written kernel in which
 * every thread moves `unroll` (1, 2, 4 or 8) 16-byte vectors per grid-stride
 * iteration, all loads before the stores; `blocks` workgroups of 256 threads
 * (0: 2048).  The buffers must not overlap.  Measures the practical HBM
 * read+write rate that the streaming sweep kernels are compared with.
 * Stream-ordered like every call; RQ_EINVAL on bad arguments. */
int rq_stream_copy(void *dst, const void *src, size_t bytes, int32_t unroll, int32_t blocks,
                   void *stream);

const char *rq_strerror(int status);
const char *rq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RQ_H */
