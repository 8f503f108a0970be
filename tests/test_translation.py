"""Translation symmetry (Sec. "Exploiting translational invariance"): the
oracle's Hessian blocks of gate-instance pairs related by a cyclic qubit
translation are equal when the circuit (shared gates per brick-wall layer) and
the target are translation invariant and the trace runs over all basis states
-- the premise of sweeping only translation-unique hole pairs; and the C ABI's
check of the declared symmetry."""

import ctypes as C
import os

import numpy as np
import pytest

import oracle as O
import workloads as w


def _tau(pairs, layer, k, s):
    """Instance map of the translation q -> q + s (within each layer)."""
    idx = {(int(layer[i]), tuple(p)): i for i, p in enumerate(pairs)}
    return [idx[(int(layer[i]), ((a + s) % k, (b + s) % k))] for i, (a, b) in enumerate(pairs)]


@pytest.mark.parametrize("parity", [False, True])
def test_translated_pairs_have_equal_hessian_blocks(parity):
    rng = np.random.default_rng([91, parity])
    k, layers = 6, 3
    pairs, layer = w.brickwall_pairs(k, layers)
    P = layers
    gates = (w.parity_haar_gates if parity else w.haar_gates)(rng, P)
    inst = gates[np.asarray(layer)]
    U = w.target_unitary(k // 2, 0.5, 1.0, 4.0)          # one-site (2-qubit) invariant
    mask = O.riemann.PARITY_MASK if parity else None
    H = O.hessian_holomorphic(k, pairs, inst, U, mask=mask)
    tau = _tau(pairs, layer, k, 2)
    N = len(pairs)
    scale = np.abs(H).max()
    for l in range(N):
        for m in range(N):
            assert np.abs(H[tau[l], :, :, tau[m]] - H[l, :, :, m]).max() <= 1e-12 * scale
    # a basis sub-range breaks the symmetry (the optimisation needs the full trace)
    cols = np.arange(5, 29)
    Hs = O.hessian_holomorphic(k, pairs, inst, U[:, cols], cols, mask=mask)
    diff = max(np.abs(Hs[tau[l], :, :, tau[m]] - Hs[l, :, :, m]).max()
               for l in range(N) for m in range(N))
    assert diff > 1e-6 * scale


def test_trotter_target_is_two_site_invariant():
    """The Strang Trotter target is invariant under the two-site (4-qubit)
    translation, not the one-site one (even and odd bond groups swap)."""
    k = 8
    gl = w.strang_trotter_gates(4, 0.5, 3, 1.0, 4.0)
    U = O.circuit_matrix(k, [p for p, _ in gl], np.stack([G for _, G in gl]))
    x = np.arange(1 << k)

    def shift_perm(s):
        bits = (x[:, None] >> (k - 1 - np.arange(k))[None, :]) & 1     # qubit q = bit k-1-q
        rolled = np.roll(bits, s, axis=1)                              # qubit q -> q + s
        return (rolled << (k - 1 - np.arange(k))[None, :]).sum(axis=1)

    p4, p2 = shift_perm(4), shift_perm(2)
    assert np.abs(U[np.ix_(p4, p4)] - U).max() <= 1e-12
    assert np.abs(U[np.ix_(p2, p2)] - U).max() > 1e-3


@pytest.fixture(scope="module")
def rq():
    from paper_2506_23775_amd import rq as _rq
    if not os.path.exists(_rq.LIB_PATH):
        pytest.fail("librq.so not built")
    _rq.lib()
    return _rq


def test_declared_shift_is_checked(rq):
    k = 8
    pairs, layer = w.brickwall_pairs(k, 3)
    L = rq.lib()
    ok = rq.Circuit(k, pairs, param_of=layer, shift=2)
    assert L.rq_workspace_bytes(C.byref(ok._c), rq.RQ_OP_GRAD, rq.RQ_C128, 64) > 0
    ok4 = rq.Circuit(k, pairs, param_of=layer, shift=4, parity=True)
    assert L.rq_hess_workspace_bytes(C.byref(ok4._c), rq.RQ_C128, 64) > 0
    bad = rq.Circuit(k, pairs, shift=2)                      # independent gates
    assert L.rq_workspace_bytes(C.byref(bad._c), rq.RQ_OP_GRAD, rq.RQ_C128, 64) == 0
    assert b"not invariant" in L.rq_last_error()
    odd = rq.Circuit(k, pairs, param_of=layer, shift=1)      # pairs (0,1) -> (1,2): wrong layer
    assert L.rq_workspace_bytes(C.byref(odd._c), rq.RQ_OP_GRAD, rq.RQ_C128, 64) == 0
    rng_bad = rq.Circuit(k, pairs, param_of=layer, shift=k)
    assert L.rq_workspace_bytes(C.byref(rng_bad._c), rq.RQ_OP_GRAD, rq.RQ_C128, 64) == 0


def _orbits_bruteforce(k, s):
    """Orbit representatives and sizes of k-bit strings under the qubit
    translation q -> q + s, by explicit bit lists."""
    seen = {}
    for x in range(1 << k):
        bits = [(x >> (k - 1 - q)) & 1 for q in range(k)]
        orb = set()
        b = bits
        for _ in range(k):
            b = [b[(q - s) % k] for q in range(k)]
            orb.add(sum(v << (k - 1 - q) for q, v in enumerate(b)))
        seen[min(orb)] = len(orb)
    reps = np.array(sorted(seen))
    return reps, np.array([seen[r] for r in reps])


@pytest.mark.parametrize("parity", [False, True])
def test_orbit_weighted_representatives_equal_full_trace(parity):
    """Extension beyond the paper: with a translation-invariant circuit and
    target, the sum over one basis state per translation orbit, weighted by
    the orbit size, equals the full basis sum for f, the per-parameter
    gradients and the HVP (weights folded in as sqrt(w) on both sides)."""
    rng = np.random.default_rng([92, parity])
    k, layers = 6, 3
    pairs, layer = w.brickwall_pairs(k, layers)
    gates = (w.parity_haar_gates if parity else w.haar_gates)(rng, layers)
    direction = w.tangent_direction(rng, gates, parity=parity)
    U = w.target_unitary(k // 2, 0.5, 1.0, 4.0)
    full = O.evaluate(k, pairs, gates, layer, direction, U, None, parity=parity)
    reps, wts = _orbits_bruteforce(k, 2)
    assert wts.sum() == 1 << k and len(reps) < (1 << k) // 2
    Z = np.zeros((1 << k, len(reps)), dtype=complex)
    Z[reps, np.arange(len(reps))] = np.sqrt(wts)
    red = O.evaluate(k, pairs, gates, layer, direction, U @ Z, None, parity=parity, inputs=Z)
    for key in full:
        assert np.abs(np.asarray(red[key]) - np.asarray(full[key])).max() <= 1e-11, key


def test_orbit_helper_matches_bruteforce(rq):
    for k, s in ((8, 2), (8, 4), (6, 2)):
        reps, wts = _orbits_bruteforce(k, s)
        (r2, w2), = rq.translation_orbits(k, s)
        assert np.array_equal(reps, r2) and np.array_equal(wts, w2)
        sec = rq.translation_orbits(k, s, parity=True)
        par = np.array([bin(int(v)).count("1") & 1 for v in reps])
        for p in (0, 1):
            assert np.array_equal(sec[p][0], reps[par == p] >> 1)
            assert np.array_equal(sec[p][1], wts[par == p])
