"""Pins of the seeded input generators (CPU)."""

import numpy as np
import scipy.linalg as sl
import pytest

import workloads as w
from workloads.hubbard import _spin_counts

GOLDEN = __file__.replace("test_workloads.py", "golden/")


def _shift2(k):
    """Permutation matrix of the translation by one site (two qubits)."""
    n = 1 << k
    x = np.arange(n)
    y = ((x << 2) | (x >> (k - 2))) & (n - 1)
    T = np.zeros((n, n))
    T[y, x] = 1
    return T


def test_hamiltonian_symmetries():
    for L in (2, 3, 4):
        k = 2 * L
        H = w.spinful_fh_hamiltonian(L, 1.0, 4.0).toarray()
        assert np.abs(H - H.conj().T).max() == 0
        par = np.array([bin(x).count("1") & 1 for x in range(1 << k)])
        P = np.diag(1.0 - 2 * par)
        assert np.abs(H @ P - P @ H).max() < 1e-14
        T = _shift2(k)
        assert np.abs(H @ T - T @ H).max() < 1e-14
        up, dn = _spin_counts(k)
        for cnt in (up, dn):
            Nop = np.diag(cnt.astype(float))
            assert np.abs(H @ Nop - Nop @ H).max() < 1e-14


def test_hubbard_dimer_ground_energy():
    # textbook: open two-site Hubbard at half filling, E0 = (U - sqrt(U^2 + 16 J^2)) / 2
    for U in (0.5, 4.0, 8.0):
        H = w.spinful_fh_hamiltonian(2, 1.0, U, periodic=False).toarray()
        up, dn = _spin_counts(4)
        idx = np.nonzero((up == 1) & (dn == 1))[0]
        e0 = np.linalg.eigvalsh(H[np.ix_(idx, idx)]).min()
        assert abs(e0 - (U - np.sqrt(U * U + 16)) / 2) < 1e-12


def test_target_unitary_vs_expm():
    H = w.spinful_fh_hamiltonian(3, 1.0, 4.0).toarray()
    U = w.target_unitary(3, 0.5, 1.0, 4.0)
    assert np.abs(U - sl.expm(-1j * 0.5 * H)).max() < 1e-12
    assert np.abs(U.conj().T @ U - np.eye(64)).max() < 1e-12


def test_local_gate_closed_form_golden():
    """Paper, Sec. 'Model system and circuit topology': the exponential of the
    local two-site Hamiltonian h_loc has a closed form (fixture)."""
    vals = {}
    for line in open(GOLDEN + "local_trotter_gate.txt"):
        line = line.split("#")[0].strip()
        if line:
            key, val = line.split("=")
            vals[key.strip()] = val.strip()
    J, t, U = float(vals["J"]), float(vals["t"]), float(vals["U"])
    G = np.array([[complex(x) for x in vals[f"row{r}"].split()] for r in range(4)])
    hloc = np.array([[0, 0, 0, 0], [0, 0, -J, 0], [0, -J, 0, 0], [0, 0, 0, U]], dtype=complex)
    assert np.abs(sl.expm(-1j * t * hloc) - G).max() < 1e-12
    # generator: hop and on-site gates commute and multiply to the same matrix
    assert np.abs(w.hop_gate(t, J) @ w.onsite_gate(t, U) - G).max() < 1e-12


def test_fswap_bond_identity():
    hb = w.local_hop_bond_operator(1.0)
    for tau in (0.1, 0.37, 1.3):
        F = np.kron(np.kron(np.eye(2), w.fswap_gate()), np.eye(2))
        P = np.kron(w.hop_gate(tau), w.hop_gate(tau))
        assert np.abs(F @ P @ F - sl.expm(-1j * tau * hb)).max() < 1e-13


def _dense_from_gate_list(k, gl):
    W = np.eye(1 << k, dtype=complex)
    for (qh, ql), G in gl:
        order = [qh, ql] + [q for q in range(k) if q not in (qh, ql)]
        x = np.arange(1 << k)
        y = np.zeros_like(x)
        for pos, q in enumerate(order):
            y |= ((x >> (k - 1 - q)) & 1) << (k - 1 - pos)
        E = np.kron(G, np.eye(1 << (k - 2)))[np.ix_(y, y)]
        W = E @ W
    return W


@pytest.mark.parametrize("L", [3, 4])
def test_strang_trotter_second_order(L):
    t = 0.4
    Uex = w.target_unitary(L, t, 1.0, 4.0)
    errs = []
    for steps in (4, 8):
        Wt = _dense_from_gate_list(2 * L, w.strang_trotter_gates(L, t, steps, 1.0, 4.0))
        errs.append(np.abs(Wt - Uex).max())
    assert errs[1] < 1e-2
    ratio = errs[0] / errs[1]
    assert 3.0 < ratio < 5.0, ratio      # O(dt^2)


def test_haar_and_tangent(rng):
    G = w.haar_gates(rng, 5)
    for g in G:
        assert np.abs(g.conj().T @ g - np.eye(4)).max() < 1e-13
    Gp = w.parity_haar_gates(rng, 5)
    for g in Gp:
        assert np.abs(g.conj().T @ g - np.eye(4)).max() < 1e-13
        assert np.all(g[~w.PARITY_MASK] == 0)
    for gates, par in ((G, False), (Gp, True)):
        X = w.tangent_direction(rng, gates, parity=par)
        assert abs(np.sum(np.abs(X) ** 2) - 1) < 1e-13
        for g, x in zip(gates, X):
            A = g.conj().T @ x
            assert np.abs(A + A.conj().T).max() < 1e-13
            if par:
                assert np.all(x[~w.PARITY_MASK] == 0)


def test_brickwall_pairs():
    pairs, layer = w.brickwall_pairs(8, 3)
    assert pairs[:4] == [(0, 1), (2, 3), (4, 5), (6, 7)]
    assert pairs[4:8] == [(1, 2), (3, 4), (5, 6), (7, 0)]
    assert pairs[8:] == pairs[:4]
    assert list(layer) == [0] * 4 + [1] * 4 + [2] * 4


def test_configs_build():
    p1 = w.make_problem(1)
    assert p1.k == 8 and p1.n_gates == 12 and p1.U_ref.shape == (256, 256)
    p3 = w.make_problem(3, trotter_steps=2)
    assert p3.parity and p3.n_params == 7 and p3.n_gates == 56
    assert np.all(p3.param_of == p3.layer_of)
