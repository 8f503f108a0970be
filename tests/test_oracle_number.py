"""Pins of the particle-number-conserving gate manifold U(1) x U(2) x U(1)
(Sec. "Parity-conserving gate structure": the further restriction that
removes two parameters): tangent basis, Riemannian gradient block by block,
the Riemannian HVP against second differences along the polar retraction,
and trust-region convergence on a representable target."""

import numpy as np

import oracle as O
import workloads as w

NUM = "number"


def _setup(rng, k=6, layers=3):
    pairs, _ = w.brickwall_pairs(k, layers)
    gates = w.number_haar_gates(rng, len(pairs))
    U = O.circuit_matrix(k, pairs, w.number_haar_gates(rng, len(pairs)))
    return pairs, gates, U


def _ip(A, B):
    return np.real(np.sum(np.conj(A) * B))


def test_number_gates_and_basis():
    rng = np.random.default_rng(111)
    G = w.number_haar_gates(rng, 4)
    for g in G:
        assert np.abs(g.conj().T @ g - np.eye(4)).max() < 1e-14
        assert np.all(g[~w.NUMBER_MASK] == 0)
    B = O.real_basis(NUM)
    assert len(B) == 6
    Gm = np.array([[np.real(np.trace(a.conj().T @ b)) for b in B] for a in B])
    assert np.abs(Gm - np.eye(6)).max() < 1e-15
    for a in B:
        assert np.abs(a + a.conj().T).max() == 0
        assert np.all(a[~w.NUMBER_MASK] == 0)


def test_number_rgrad_blockwise(rng=None):
    rng = np.random.default_rng(112)
    k = 6
    pairs, gates, U = _setup(rng, k)
    eg = O.egrad(O.euclidean_T(k, pairs, gates, U))
    g = O.rgrad(gates, eg, NUM)
    for p in range(len(gates)):
        for blk in ([0], [3], [1, 2]):
            V = gates[p][np.ix_(blk, blk)]
            E = eg[p][np.ix_(blk, blk)]
            assert np.abs(g[p][np.ix_(blk, blk)] - 0.5 * (E - V @ E.conj().T @ V)).max() < 1e-13
        assert np.all(g[p][~w.NUMBER_MASK] == 0)
        A = gates[p].conj().T @ g[p]
        assert np.abs(A + A.conj().T).max() < 1e-12


def test_number_hvp_along_retraction():
    rng = np.random.default_rng(113)
    k = 6
    pairs, gates, U = _setup(rng, k)
    X = w.tangent_direction(rng, gates, parity=NUM)
    assert np.all(X[:, ~w.NUMBER_MASK] == 0)
    T, Td = O.tangent_T(k, pairs, gates, X, U)
    eg, eh = O.egrad(T), O.egrad(Td)
    HX = O.rhvp(gates, eg, eh, X, NUM)
    g = O.rgrad(gates, eg, NUM)

    def fR(t):
        Gt = np.stack([O.polar(G + t * x) for G, x in zip(gates, X)])
        assert np.all(np.abs(Gt[:, ~w.NUMBER_MASK]) < 1e-14)
        return O.cost(k, pairs, Gt, U)

    h = 1e-3
    f0 = fR(0.0)
    d1 = (fR(h) - fR(-h)) / (2 * h)
    d2 = (-fR(2 * h) + 16 * fR(h) - 30 * f0 + 16 * fR(-h) - fR(-2 * h)) / (12 * h * h)
    assert abs(d1 - _ip(g, X)) < 1e-6
    assert abs(d2 - _ip(X, HX)) < 1e-6 * max(1.0, abs(d2))


def test_number_trust_region_converges():
    rng = np.random.default_rng(114)
    k = 4
    pairs = [(0, 1), (2, 3), (1, 2)]
    Gs = w.number_haar_gates(rng, 3)
    U = O.circuit_matrix(k, pairs, Gs)
    X = w.tangent_direction(rng, Gs, parity=NUM)
    G0 = np.stack([O.polar(g + 0.8 * x) for g, x in zip(Gs, X)])

    def fgh(G):
        T = np.where(O.riemann.NUMBER_MASK, O.euclidean_T(k, pairs, G, U), 0)
        eg = O.egrad(T)
        Hh = O.hessian_holomorphic(k, pairs, G, U, mask=O.riemann.NUMBER_MASK)
        return (O.cost(k, pairs, G, U), O.gradient_real(G, eg, NUM),
                O.hessian_real(G, eg, Hh, NUM))

    G, hist = O.tr_solve(G0, fgh, lambda G: O.cost(k, pairs, G, U), 40, gtol=1e-10,
                         parity=NUM)
    fs = [h[0] for h in hist]
    assert all(b <= a + 1e-12 for a, b in zip(fs, fs[1:]))
    assert abs(O.cost(k, pairs, G, U) + (1 << k)) <= 1e-9
    assert np.all(np.abs(G[:, ~w.NUMBER_MASK]) < 1e-14)
