"""Pin of the oracle's trust-region loop (Sec. "Riemannian optimization"):
on a target that the circuit represents exactly, U = C(G*), the iteration
started near G* decreases f monotonically to the global minimum -2^k (where
the Riemannian gradient vanishes), converging superlinearly at the end."""

import numpy as np

import oracle as O
import workloads as w


def _fgh(k, pairs, U, parity):
    def fn(G):
        T = O.euclidean_T(k, pairs, G, U)
        if parity:
            T = np.where(O.riemann.PARITY_MASK, T, 0)
        eg = O.egrad(T)
        mask = O.riemann.PARITY_MASK if parity else None
        Hh = O.hessian_holomorphic(k, pairs, G, U, mask=mask)
        return (O.cost(k, pairs, G, U), O.gradient_real(G, eg, parity),
                O.hessian_real(G, eg, Hh, parity))
    return fn


def test_tr_converges_to_global_minimum_on_representable_target():
    rng = np.random.default_rng(71)
    k = 4
    pairs = [(0, 1), (2, 3), (1, 2), (3, 0)]
    Gs = w.haar_gates(rng, len(pairs))
    U = O.circuit_matrix(k, pairs, Gs)
    G0 = np.stack([O.polar(g + 0.15 * (rng.standard_normal((4, 4))
                                       + 1j * rng.standard_normal((4, 4)))) for g in Gs])
    G, hist = O.tr_solve(G0, _fgh(k, pairs, U, False), lambda G: O.cost(k, pairs, G, U), 40,
                         gtol=1e-10)
    fs = [h[0] for h in hist]
    assert all(b <= a + 1e-12 for a, b in zip(fs, fs[1:]))          # monotone
    assert abs(O.cost(k, pairs, G, U) + (1 << k)) <= 1e-9
    assert hist[-1][1] <= 1e-6
    # the circuit equals U up to a phase per gate that cancels in C
    C = O.circuit_matrix(k, pairs, G)
    assert np.abs(C - U).max() <= 1e-5


def test_tr_parity_gates_representable_target():
    rng = np.random.default_rng(72)
    k = 4
    pairs = [(0, 1), (2, 3), (1, 2)]
    Gs = w.parity_haar_gates(rng, len(pairs))
    U = O.circuit_matrix(k, pairs, Gs)
    noise = np.where(O.riemann.PARITY_MASK, rng.standard_normal((3, 4, 4))
                     + 1j * rng.standard_normal((3, 4, 4)), 0)
    G0 = np.stack([O.polar(g + 0.1 * z) for g, z in zip(Gs, noise)])
    G, hist = O.tr_solve(G0, _fgh(k, pairs, U, True), lambda G: O.cost(k, pairs, G, U), 40,
                         gtol=1e-10, parity=True)
    fs = [h[0] for h in hist]
    assert all(b <= a + 1e-12 for a, b in zip(fs, fs[1:]))
    assert abs(O.cost(k, pairs, G, U) + (1 << k)) <= 1e-9
    assert np.all(np.abs(np.where(O.riemann.PARITY_MASK, 0, G)) <= 1e-12)
