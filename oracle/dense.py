"""Dense FP64 definitions of f, its gate derivatives and Hessian blocks.

Conventions (paper Sec. "Problem statement and setup" and Sec. "Details of the
state vector simulation"):

* k qubits, qubit q is bit (k-1-q) of a basis index (leg i0 = most significant);
* a gate acts on a pair (q_hi, q_lo); its row/column index is
  2*bit(q_hi) + bit(q_lo) (general gate-application formula with a 5-leg
  state tensor);
* C(G) = E_N ... E_1 with E_l the embedding of G_l; gate 1 acts first;
* the cost is f(G) = -Re Tr[U^dagger C(G)] (eq. for the target function) and
  the trace is the sum over computational basis states j (eq. for the
  basis-vector sum); every function here takes a subset ``cols`` of basis
  states and returns the partial sum over it (``cols=None``: all 2^k).

Matrices are 2^k x n arrays whose rows are amplitudes and whose columns are
basis states j (a "state slab").
"""

from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Embedding and action of a two-qubit gate
# ---------------------------------------------------------------------------

def embed_kron(k: int, pair, G: np.ndarray) -> np.ndarray:
    """Literal 2^k x 2^k embedding of a two-qubit gate: E = Pi^T (G (x) I) Pi,
    where Pi reorders the qubits to (q_hi, q_lo, remaining qubits ascending).
    The paper's memory discussion (Sec. "Memory considerations") notes this
    matrix is what the matrix-free method avoids; the oracle builds it only for
    small k."""
    qh, ql = pair
    others = [q for q in range(k) if q not in (qh, ql)]
    order = [qh, ql] + others
    x = np.arange(1 << k)
    y = np.zeros_like(x)
    for pos, q in enumerate(order):
        y |= ((x >> (k - 1 - q)) & 1) << (k - 1 - pos)
    K = np.kron(G, np.eye(1 << (k - 2)))
    return K[np.ix_(y, y)]


def circuit_matrix_kron(k: int, pairs, gates) -> np.ndarray:
    """C(G) = E_N ... E_1 from literal Kronecker embeddings (small k)."""
    W = np.eye(1 << k, dtype=np.complex128)
    for pair, G in zip(pairs, gates):
        W = embed_kron(k, pair, G) @ W
    return W


def apply_gate(M: np.ndarray, k: int, pair, G: np.ndarray) -> np.ndarray:
    """E @ M for the embedding E of G on ``pair``, via the tensor contraction
    psi'_{..i1..i3..} = sum_{j1,j3} g_{i1 i3 j1 j3} psi_{..j1..j3..}
    (general gate-application formula).  M has 2^k rows."""
    qh, ql = pair
    n = M.shape[1]
    T = M.reshape([2] * k + [n])
    g = np.asarray(G).reshape(2, 2, 2, 2)      # [out_hi, out_lo, in_hi, in_lo]
    out = np.tensordot(g, T, axes=([2, 3], [qh, ql]))
    out = np.moveaxis(out, [0, 1], [qh, ql])
    return out.reshape(1 << k, n)


def circuit_matrix(k: int, pairs, gates) -> np.ndarray:
    W = np.eye(1 << k, dtype=np.complex128)
    for pair, G in zip(pairs, gates):
        W = apply_gate(W, k, pair, G)
    return W


def _cols(k, cols):
    return np.arange(1 << k) if cols is None else np.asarray(cols, dtype=np.int64)


def reference_columns(U: np.ndarray, cols=None) -> np.ndarray:
    """Columns U|j> of a dense target for the basis states in ``cols``."""
    k = int(np.log2(U.shape[0]))
    return U[:, _cols(k, cols)]


def sector_columns(k: int, parity: int) -> np.ndarray:
    """Basis states whose bit count has the given parity (one parity sector)."""
    x = np.arange(1 << k)
    pc = np.array([bin(v).count("1") & 1 for v in x])
    return x[pc == parity]


def unit_columns(k: int, cols) -> np.ndarray:
    """The basis states |j>, j in cols, as a 2^k x |cols| slab."""
    cols = np.asarray(cols)
    E = np.zeros((1 << k, cols.size), dtype=np.complex128)
    E[cols, np.arange(cols.size)] = 1.0
    return E


def _initial(k, cols, inputs):
    """Starting states of the summands: |j> for j in cols (Sec. "Objective
    function and matrix-free evaluation"), or the given input states psi_j
    (2^k x n) when the sum runs over other vectors (sampling over random
    vectors, Sec. "Conclusions"); Ucols must then hold U psi_j."""
    if inputs is not None:
        return np.asarray(inputs, dtype=np.complex128)
    return unit_columns(k, _cols(k, cols))


# ---------------------------------------------------------------------------
# Cost
# ---------------------------------------------------------------------------

def h_trace(k, pairs, gates, Ucols, cols=None, inputs=None) -> complex:
    """h_S = sum_{j in S} <j| U^dagger C(G) |j>  (complex; holomorphic in the
    gate entries).  ``Ucols`` = U|j> for j in S (2^k x |S|).  With
    ``inputs``: sum over the input states psi_j instead of |j>."""
    Psi = _initial(k, cols, inputs)
    for pair, G in zip(pairs, gates):
        Psi = apply_gate(Psi, k, pair, G)
    return complex(np.sum(np.conj(Ucols) * Psi))


def cost(k, pairs, gates, Ucols, cols=None, inputs=None) -> float:
    """f = -Re Tr[U^dagger C(G)] (eq. for the target function), restricted to
    the basis states in ``cols`` (or summed over input states)."""
    return -h_trace(k, pairs, gates, Ucols, cols, inputs).real


# ---------------------------------------------------------------------------
# Prefix / suffix products and hole contractions
# ---------------------------------------------------------------------------

def forward_states(k, pairs, gates, cols=None, inputs=None):
    """Psi_l = E_l ... E_1 |j>, l = 0..N, for j in cols (prefix products)."""
    Psi = [_initial(k, cols, inputs)]
    for pair, G in zip(pairs, gates):
        Psi.append(apply_gate(Psi[-1], k, pair, G))
    return Psi


def backward_states(k, pairs, gates, Ucols):
    """Lam_l = (U^dagger E_N ... E_{l+1})^T restricted to the columns of
    Ucols, i.e. Lam_N = conj(U|j>) and Lam_{l-1} = E_l^T Lam_l.  Returned as a
    list indexed by l = 0..N."""
    N = len(pairs)
    Lam = [None] * (N + 1)
    Lam[N] = np.conj(Ucols)
    for l in range(N, 0, -1):
        Lam[l - 1] = apply_gate(Lam[l], k, pairs[l - 1], gates[l - 1].T)
    return Lam


def hole_contraction(k, pair, Lam: np.ndarray, Psi: np.ndarray) -> np.ndarray:
    """T[a][b] = sum_j sum_rest Lam[(a, rest), j] Psi[(b, rest), j]: the
    tensor network with one gate removed (gate hole; Sec. "Gate gradient as a
    gate hole"), i.e. d h / d G_ab."""
    qh, ql = pair
    n = Psi.shape[1]

    def legs(M):
        T = M.reshape([2] * k + [n])
        T = np.moveaxis(T, [qh, ql], [0, 1])
        return T.reshape(4, -1)

    return legs(Lam) @ legs(Psi).T


def euclidean_T(k, pairs, gates, Ucols, cols=None, inputs=None) -> np.ndarray:
    """T_l = d h_S / d G_l for every gate instance l (N x 4 x 4 complex).

    With B_l = E_{l-1}...E_1 and A_l = E_N...E_{l+1},
    h = Tr[E_l (B_l U^dagger A_l)] restricted to S, so T_l is the partial trace
    of B_l U^dagger A_l with the two legs of gate l left open (Sec. "Gradient
    and Hessian tensor diagrams")."""
    Psi = forward_states(k, pairs, gates, cols, inputs)
    Lam = backward_states(k, pairs, gates, Ucols)
    N = len(pairs)
    return np.stack([hole_contraction(k, pairs[l], Lam[l + 1], Psi[l]) for l in range(N)])


def tangent_T(k, pairs, gates, Z, Ucols, cols=None, inputs=None):
    """(T, Tdot): T as in euclidean_T and its directional derivative Tdot along
    G_l -> G_l + eps Z_l (all instances), evaluated with dual numbers: every
    prefix/suffix product is carried as a pair (value, derivative).  This is
    the derivative of the directed gradient that the appendix on
    Hessian-vector products differentiates once more."""
    N = len(pairs)
    Psi = [_initial(k, cols, inputs)]
    dPsi = [np.zeros_like(Psi[0])]
    for l in range(N):
        Psi.append(apply_gate(Psi[l], k, pairs[l], gates[l]))
        dPsi.append(apply_gate(dPsi[l], k, pairs[l], gates[l])
                    + apply_gate(Psi[l], k, pairs[l], Z[l]))
    Lam = [None] * (N + 1)
    dLam = [None] * (N + 1)
    Lam[N] = np.conj(Ucols)
    dLam[N] = np.zeros_like(Lam[N])
    for l in range(N, 0, -1):
        Gt, Zt = gates[l - 1].T, Z[l - 1].T
        Lam[l - 1] = apply_gate(Lam[l], k, pairs[l - 1], Gt)
        dLam[l - 1] = (apply_gate(dLam[l], k, pairs[l - 1], Gt)
                       + apply_gate(Lam[l], k, pairs[l - 1], Zt))
    T = np.stack([hole_contraction(k, pairs[l], Lam[l + 1], Psi[l]) for l in range(N)])
    Td = np.stack([hole_contraction(k, pairs[l], dLam[l + 1], Psi[l])
                   + hole_contraction(k, pairs[l], Lam[l + 1], dPsi[l]) for l in range(N)])
    return T, Td


def hessian_holomorphic(k, pairs, gates, Ucols, cols=None, mask=None, inputs=None) -> np.ndarray:
    """All second derivatives d^2 h / dG_l[a,b] dG_m[c,d] (N x 4 x 4 x N x 4 x 4).

    Column (l, a, b) of this matrix is the derivative of every T_m along the
    elementary direction E_ab placed on gate l alone (dual numbers, as in
    tangent_T).  Blocks with l == m vanish because h is linear in each gate
    (Sec. "Gradient and Hessian tensor diagrams").  ``mask`` (4x4 bool)
    restricts the directions to a gate pattern (parity mode)."""
    N = len(pairs)
    H = np.zeros((N, 4, 4, N, 4, 4), dtype=np.complex128)
    Zs = np.zeros((N, 4, 4), dtype=np.complex128)
    for l in range(N):
        for a in range(4):
            for b in range(4):
                if mask is not None and not mask[a, b]:
                    continue
                Zs[:] = 0
                Zs[l, a, b] = 1.0
                _, Td = tangent_T(k, pairs, gates, Zs, Ucols, cols, inputs)
                H[:, :, :, l, a, b] = Td
    return H


def hessian_by_holes(k, pairs, gates, Ucols, cols=None, mask=None, inputs=None) -> np.ndarray:
    """The same second derivatives as hessian_holomorphic (N x 4 x 4 x N x 4 x 4),
    computed by the steps of Sec. "Efficient gradient and Hessian
    computation" and Sec. "Gate hole application": for every gate l, the
    hole of G_l applied to the state before it gives one state per gate
    entry (a, b) -- the embedded elementary matrix |a><b| acting on
    psi_{l-1}; these states run through G_{l+1}, G_{l+2}, ... (the second
    forward pass), and at every later gate m the hole of G_m is contracted
    between the bra-side state after m and the propagated state before m,
    which is d^2 h / dG_m[c,d] dG_l[a,b].  The other triangle follows by
    symmetry of mixed derivatives; blocks with l == m vanish (h is linear in
    each gate).  ``mask`` restricts both entries (a, b) and (c, d) to a
    pattern (parity mode; the other entries are zero).  Memory: 16 propagated
    states of the size of Ucols."""
    N = len(pairs)
    n = np.asarray(Ucols).shape[1]
    Lam = backward_states(k, pairs, gates, Ucols)
    H = np.zeros((N, 4, 4, N, 4, 4), dtype=np.complex128)
    entries = [(a, b) for a in range(4) for b in range(4) if mask is None or mask[a, b]]
    Psi = _initial(k, cols, inputs)
    for l in range(N):
        if l + 1 < N:
            # hole application: one state per entry, stacked as columns
            X = np.concatenate([apply_gate(Psi, k, pairs[l], _elementary(a, b))
                                for a, b in entries], axis=1)
            for m in range(l + 1, N):
                qh, ql = pairs[m]
                lam = np.moveaxis(Lam[m + 1].reshape([2] * k + [n]), [qh, ql], [0, 1])
                xs = np.moveaxis(X.reshape([2] * k + [len(entries), n]), [qh, ql], [0, 1])
                # block[c, d, e] = sum_{rest, j} Lam[(c, rest), j] X_e[(d, rest), j]
                blk = np.tensordot(lam.reshape(4, -1, n), xs.reshape(4, -1, len(entries), n),
                                   axes=([1, 2], [1, 3]))
                if mask is not None:
                    blk = np.where(mask[:, :, None], blk, 0)
                for e, (a, b) in enumerate(entries):
                    H[m, :, :, l, a, b] = blk[:, :, e]
                    H[l, a, b, m, :, :] = blk[:, :, e]
                X = apply_gate(X, k, pairs[m], gates[m])
        Psi = apply_gate(Psi, k, pairs[l], gates[l])
    return H


def _elementary(a, b) -> np.ndarray:
    E = np.zeros((4, 4), dtype=np.complex128)
    E[a, b] = 1.0
    return E
