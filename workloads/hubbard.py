"""Spinful 1D Fermi-Hubbard model on a ring, Jordan-Wigner mapped to qubits.

Conventions (paper: Sec. "Model system and circuit topology", eq. for the
spinful model in Sec. "Comparison with the MPO method"):

* qubit q is bit (k-1-q) of a basis index, i.e. qubit 0 is the most
  significant tensor leg (Sec. "Gate application": leg i0 is slowest);
  operators on several qubits are Kronecker products in qubit order;
* interleaved spin ordering: qubit 2s is site s spin up, qubit 2s+1 is site s
  spin down (the paper enumerates all up-spins first; the interleaved order
  keeps every interaction term on neighbouring qubits);
* local operators c, c^dagger of the Jordan-Wigner section: c|1> = |0>,
  c^dagger|0> = |1>, with the Z-string placed on the qubits *after* the mode;
* the hopping across the periodic wrap bond (L-1, 0) is the bulk bond operator
  translated by 2(L-1) qubits modulo k.  This drops the global Z-string of the
  wrap term, as the paper does for the spinless chain (hard-core boson
  mapping), and makes H commute with the 2-qubit (one-site) translation.

H = -J sum_{s,sigma} (a^dag_{s,sigma} a_{s+1,sigma} + h.c.) + U sum_s n_{s,up} n_{s,dn}.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_I2 = np.eye(2, dtype=np.complex128)
_Z = np.diag([1.0, -1.0]).astype(np.complex128)
# c^dagger |0> = |1>, c |1> = |0>  (basis order |0>, |1>)
_CDAG = np.array([[0, 0], [1, 0]], dtype=np.complex128)
_C = np.array([[0, 1], [0, 0]], dtype=np.complex128)
_N = np.diag([0.0, 1.0]).astype(np.complex128)


def _product_operator(k: int, ops: dict) -> sp.csr_matrix:
    """Kronecker product over qubits 0..k-1 (qubit 0 leftmost) of single-qubit
    operators; qubits absent from ``ops`` carry the identity."""
    out = sp.identity(1, dtype=np.complex128, format="csr")
    for q in range(k):
        out = sp.kron(out, sp.csr_matrix(ops.get(q, _I2)), format="csr")
    return out


def _bond_terms(k: int, s: int):
    """Single-qubit operator dictionaries of the hopping terms of bond (s, s+1)
    for both spins, on qubits 2s .. 2s+3 (mod k).  For the bulk bond these are
    the exact Jordan-Wigner images a^dag_p a_{p+2} = c^dag_p Z_{p+1} c_{p+2};
    the wrap bond uses the same local form translated around the ring."""
    q = [(2 * s + i) % k for i in range(4)]
    terms = []
    for sigma in (0, 1):
        p, mid, r = q[sigma], q[sigma + 1], q[sigma + 2]
        terms.append({p: _CDAG, mid: _Z, r: _C})   # a^dag_p a_r
        terms.append({p: _C, mid: _Z, r: _CDAG})   # a^dag_r a_p  (h.c.)
    return terms


def spinful_fh_hamiltonian(n_sites: int, J: float = 1.0, U: float = 4.0,
                           periodic: bool = True) -> sp.csr_matrix:
    """Sparse 2^k x 2^k Hamiltonian, k = 2 * n_sites (interleaved spins)."""
    k = 2 * n_sites
    dim = 1 << k
    H = sp.csr_matrix((dim, dim), dtype=np.complex128)
    n_bonds = n_sites if periodic else n_sites - 1
    for s in range(n_bonds):
        for t in _bond_terms(k, s):
            H = H - J * _product_operator(k, t)
    for s in range(n_sites):
        H = H + U * _product_operator(k, {2 * s: _N, 2 * s + 1: _N})
    return H.tocsr()


def _spin_counts(k: int):
    """Per basis index: number of up spins (even qubits) and down spins."""
    x = np.arange(1 << k, dtype=np.int64)
    up = np.zeros_like(x)
    dn = np.zeros_like(x)
    for q in range(k):
        bit = (x >> (k - 1 - q)) & 1
        if q % 2 == 0:
            up += bit
        else:
            dn += bit
    return up, dn


def target_unitary(n_sites: int, t: float, J: float = 1.0, U: float = 4.0) -> np.ndarray:
    """Dense exp(-i H t) in complex128 for k = 2*n_sites <= 12.

    H conserves the number of up and of down spins, so the exponential is
    formed block by block over (N_up, N_dn) sectors from a Hermitian
    eigendecomposition, V diag(exp(-i lambda t)) V^dagger.  The result is the
    dense matrix exponential (a test checks it against scipy's expm)."""
    k = 2 * n_sites
    if k > 14:
        raise ValueError("dense target only for k <= 14")
    H = spinful_fh_hamiltonian(n_sites, J, U).toarray()
    up, dn = _spin_counts(k)
    out = np.zeros_like(H)
    for nu in range(n_sites + 1):
        for nd in range(n_sites + 1):
            idx = np.nonzero((up == nu) & (dn == nd))[0]
            if idx.size == 0:
                continue
            block = H[np.ix_(idx, idx)]
            w, v = np.linalg.eigh(block)
            out[np.ix_(idx, idx)] = (v * np.exp(-1j * w * t)) @ v.conj().T
    return out


# ---------------------------------------------------------------------------
# Two-qubit gates of the Trotter circuit.  Matrix rows/columns are indexed by
# 2*bit(first qubit of the pair) + bit(second qubit).
# ---------------------------------------------------------------------------

def hop_gate(tau: float, J: float = 1.0) -> np.ndarray:
    """exp(-i tau h) for h = -J (c^dag c + c c^dag) on two neighbouring modes:
    the paper's closed form of exp(-i t h_loc) with the interaction set to 0."""
    c, s = np.cos(J * tau), np.sin(J * tau)
    return np.array([[1, 0, 0, 0],
                     [0, c, 1j * s, 0],
                     [0, 1j * s, c, 0],
                     [0, 0, 0, 1]], dtype=np.complex128)


def onsite_gate(tau: float, U: float) -> np.ndarray:
    """exp(-i tau U n_up n_dn) on the two spin qubits of one site."""
    return np.diag([1, 1, 1, np.exp(-1j * tau * U)]).astype(np.complex128)


def fswap_gate() -> np.ndarray:
    """Fermionic swap of two neighbouring modes (swap with a sign on |11>)."""
    return np.array([[1, 0, 0, 0],
                     [0, 0, 1, 0],
                     [0, 1, 0, 0],
                     [0, 0, 0, -1]], dtype=np.complex128)


def local_hop_bond_operator(J: float = 1.0) -> np.ndarray:
    """16x16 hopping operator of bond (0,1) on qubits 0..3 (both spins)."""
    H = np.zeros((16, 16), dtype=np.complex128)
    for t in _bond_terms(4, 0):
        H -= J * _product_operator(4, t).toarray()
    return H


def _bond_gates(k: int, s: int, tau: float, J: float):
    q = [(2 * s + i) % k for i in range(4)]
    return [((q[1], q[2]), fswap_gate()),
            ((q[0], q[1]), hop_gate(tau, J)),
            ((q[2], q[3]), hop_gate(tau, J)),
            ((q[1], q[2]), fswap_gate())]


def strang_trotter_gates(n_sites: int, t: float, steps: int, J: float = 1.0,
                         U: float = 4.0):
    """Gate list (application order) of a second-order (Strang) Trotter
    circuit for exp(-i H t).

    H is split into groups of mutually commuting terms: H_int (on-site
    interaction), H_even (hopping of bonds (s, s+1) with s even) and H_odd
    (s odd); for an odd number of sites the wrap bond (L-1, 0) forms a group of
    its own.  With groups A_1..A_m one step is the symmetric product

        e^{-i A_1 dt/2} ... e^{-i A_{m-1} dt/2} e^{-i A_m dt}
        e^{-i A_{m-1} dt/2} ... e^{-i A_1 dt/2},            dt = t / steps,

    i.e. for an even ring  int/2, even/2, odd, even/2, int/2.  Each bond
    exponential is applied as fswap(2s+1, 2s+2) . [hop(2s,2s+1) (x)
    hop(2s+2,2s+3)] . fswap(2s+1, 2s+2), which uses only neighbouring two-qubit
    gates.  The on-site half steps of consecutive Trotter steps are merged into
    one full step (the product is unchanged).

    Returns a list of ((q_hi, q_lo), 4x4 complex128) in application order."""
    k = 2 * n_sites
    dt = t / steps
    if n_sites % 2 == 0:
        groups = [[s for s in range(n_sites) if s % 2 == 0],
                  [s for s in range(n_sites) if s % 2 == 1]]
    else:
        groups = [[s for s in range(n_sites - 1) if s % 2 == 0],
                  [s for s in range(n_sites - 1) if s % 2 == 1],
                  [n_sites - 1]]

    def onsite(tau):
        return [((2 * s, 2 * s + 1), onsite_gate(tau, U)) for s in range(n_sites)]

    def bonds(sel, tau):
        out = []
        for s in sel:
            out += _bond_gates(k, s, tau, J)
        return out

    gates = onsite(dt / 2)
    for step in range(steps):
        for g in groups[:-1]:
            gates += bonds(g, dt / 2)
        gates += bonds(groups[-1], dt)
        for g in reversed(groups[:-1]):
            gates += bonds(g, dt / 2)
        gates += onsite(dt / 2 if step == steps - 1 else dt)
    return gates
