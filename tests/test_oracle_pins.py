"""Pins of the CPU oracle against closed forms, brute force, exact Taylor
coefficients and finite differences (no GPU)."""

import numpy as np
import pytest

import oracle as O
import workloads as w


def _random_circuit(rng, k, n_layers, parity=False):
    pairs, _ = w.brickwall_pairs(k, n_layers)
    gates = (w.parity_haar_gates if parity else w.haar_gates)(rng, len(pairs))
    return pairs, gates


def _random_unitary(rng, n):
    return w.haar_unitary(rng, n)


# --------------------------------------------------------------------------
# Embedding / application
# --------------------------------------------------------------------------

def test_apply_gate_matches_kron_embedding(rng):
    k = 5
    pairs = [(0, 1), (3, 4), (4, 0), (3, 1), (1, 3), (2, 0)]
    for pair in pairs:
        G = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
        M = rng.standard_normal((32, 3)) + 1j * rng.standard_normal((32, 3))
        assert np.abs(O.embed_kron(k, pair, G) @ M - O.apply_gate(M, k, pair, G)).max() < 1e-13


def test_embed_adjacent_is_plain_kron(rng):
    # textbook: a gate on neighbouring qubits (q, q+1) is I_{2^q} (x) G (x) I
    k = 6
    G = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    for q in range(k - 1):
        ref = np.kron(np.kron(np.eye(1 << q), G), np.eye(1 << (k - q - 2)))
        assert np.abs(O.embed_kron(k, (q, q + 1), G) - ref).max() == 0


def test_swapped_pair_is_conjugated_by_swap(rng):
    # (q_lo, q_hi) order: the gate seen with its two legs exchanged
    k = 3
    G = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    S = np.eye(4)[[0, 2, 1, 3]]
    assert np.abs(O.embed_kron(k, (1, 0), G) - O.embed_kron(k, (0, 1), S @ G @ S)).max() < 1e-15


def test_circuit_matrix_kron_and_unitary(rng):
    k = 6
    pairs, gates = _random_circuit(rng, k, 3)
    W1 = O.circuit_matrix_kron(k, pairs, gates)
    W2 = O.circuit_matrix(k, pairs, gates)
    assert np.abs(W1 - W2).max() < 1e-13
    assert np.abs(W1.conj().T @ W1 - np.eye(1 << k)).max() < 1e-12


# --------------------------------------------------------------------------
# Cost
# --------------------------------------------------------------------------

def test_cost_reproducing_target_is_minus_dim(rng):
    k = 6
    pairs, gates = _random_circuit(rng, k, 4)
    U = O.circuit_matrix(k, pairs, gates)
    assert abs(O.cost(k, pairs, gates, U) + (1 << k)) < 1e-11


def test_cost_frobenius_identity(rng):
    # paper eq. for the Frobenius distance: ||C - U||^2 = 2 Tr I - 2 Re Tr[U^dag C]
    k = 6
    pairs, gates = _random_circuit(rng, k, 3)
    U = _random_unitary(rng, 1 << k)
    W = O.circuit_matrix_kron(k, pairs, gates)
    f = O.cost(k, pairs, gates, U)
    assert abs(np.sum(np.abs(W - U) ** 2) - (2 * (1 << k) + 2 * f)) < 1e-10


def test_cost_single_gate_closed_form(rng):
    U = _random_unitary(rng, 4)
    G = _random_unitary(rng, 4)
    f = O.cost(2, [(0, 1)], G[None], U)
    assert abs(f + np.real(np.trace(U.conj().T @ G))) < 1e-14
    f2 = O.cost(2, [(1, 0)], G[None], U)
    S = np.eye(4)[[0, 2, 1, 3]]
    assert abs(f2 + np.real(np.trace(U.conj().T @ S @ G @ S))) < 1e-14


def test_cost_product_circuit(rng):
    # one brick layer of product gates a (x) b against a product target:
    # f = -Re prod_q Tr[u_q^dag c_q]
    k = 6
    pairs, _ = w.brickwall_pairs(k, 1)
    ones = [_random_unitary(rng, 2) for _ in range(k)]
    us = [_random_unitary(rng, 2) for _ in range(k)]
    gates = np.stack([np.kron(ones[a], ones[b]) for a, b in pairs])
    U = np.eye(1)
    for q in range(k):
        U = np.kron(U, us[q])
    prod = np.prod([np.trace(us[q].conj().T @ ones[q]) for q in range(k)])
    assert abs(O.cost(k, pairs, gates, U) + prod.real) < 1e-12


def test_cost_columns_partition(rng):
    k = 6
    pairs, gates = _random_circuit(rng, k, 3)
    U = _random_unitary(rng, 1 << k)
    cols = np.arange(1 << k)
    f = O.cost(k, pairs, gates, U)
    fa = O.cost(k, pairs, gates, U[:, cols[:20]], cols[:20])
    fb = O.cost(k, pairs, gates, U[:, cols[20:]], cols[20:])
    assert abs(f - fa - fb) < 1e-12


# --------------------------------------------------------------------------
# Gradient
# --------------------------------------------------------------------------

def _taylor(hfun, M, r):
    z = r * np.exp(2j * np.pi * np.arange(M) / M)
    vals = np.array([hfun(zz) for zz in z])
    return np.fft.fft(vals) / M / r ** np.arange(M)


def test_gradient_exact_taylor_and_fd(rng):
    k = 6
    pairs, gates = _random_circuit(rng, k, 3)
    N = len(pairs)
    U = _random_unitary(rng, 1 << k)
    X = rng.standard_normal((N, 4, 4)) + 1j * rng.standard_normal((N, 4, 4))
    T = O.euclidean_T(k, pairs, gates, U)
    c = _taylor(lambda z: O.h_trace(k, pairs, gates + z * X, U), 2 * N + 2, 0.3)
    assert abs(c[0] - O.h_trace(k, pairs, gates, U)) < 1e-11
    assert abs(c[1] - np.sum(T * X)) < 1e-10 * max(1, abs(c[1]))
    # paper's gradient convention: d/deps f(G + eps X) = Re Tr[grad^dag X]
    eg = O.egrad(T)
    eps = 1e-5
    fd = (O.cost(k, pairs, gates + eps * X, U) - O.cost(k, pairs, gates - eps * X, U)) / (2 * eps)
    assert abs(fd - np.real(np.sum(np.conj(eg) * X))) < 1e-7


def test_gradient_single_gate_closed_form(rng):
    U = _random_unitary(rng, 4)
    G = _random_unitary(rng, 4)
    T = O.euclidean_T(2, [(0, 1)], G[None], U)
    assert np.abs(T[0] - np.conj(U)).max() < 1e-14
    rg = O.rgrad(G[None], O.egrad(T))[0]
    assert np.abs(rg - (-0.5 * (U - G @ U.conj().T @ G))).max() < 1e-14


def test_multilinearity(rng):
    k = 6
    pairs, gates = _random_circuit(rng, k, 3)
    U = _random_unitary(rng, 1 << k)
    h = O.h_trace(k, pairs, gates, U)
    T = O.euclidean_T(k, pairs, gates, U)
    for l in range(len(pairs)):
        assert abs(np.sum(gates[l] * T[l]) - h) < 1e-11


def test_gradient_at_exact_target(rng):
    k = 6
    pairs, gates = _random_circuit(rng, k, 3)
    U = O.circuit_matrix(k, pairs, gates)
    eg = O.egrad(O.euclidean_T(k, pairs, gates, U))
    assert np.abs(eg + (1 << (k - 2)) * gates).max() < 1e-11
    assert np.abs(O.rgrad(gates, eg)).max() < 1e-11


def test_gauge_orthogonality(rng):
    # inserting exp(eps K) exp(-eps K) on a wire between two consecutive gates
    # leaves C unchanged, so the gradient is orthogonal to that direction.
    k = 6
    pairs, gates = _random_circuit(rng, k, 2)
    U = _random_unitary(rng, 1 << k)
    eg = O.egrad(O.euclidean_T(k, pairs, gates, U))
    K = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    K = K - K.conj().T
    I2 = np.eye(2)
    checked = 0
    N = len(pairs)
    for l in range(N):
        for q in pairs[l]:
            nxt = [m for m in range(l + 1, N) if q in pairs[m]]
            if not nxt:
                continue
            m = nxt[0]
            Kl = np.kron(K, I2) if pairs[l][0] == q else np.kron(I2, K)
            Km = np.kron(K, I2) if pairs[m][0] == q else np.kron(I2, K)
            X = np.zeros_like(gates)
            X[l] = Kl @ gates[l]
            X[m] = -gates[m] @ Km
            assert abs(np.real(np.sum(np.conj(eg) * X))) < 1e-11
            checked += 1
    assert checked >= 6


def test_shared_gates_sum_instances(rng):
    k = 6
    pairs, layer = w.brickwall_pairs(k, 3)
    P = 3
    G = w.haar_gates(rng, P)
    inst = G[np.asarray(layer)]
    U = _random_unitary(rng, 1 << k)
    T = O.per_param(O.euclidean_T(k, pairs, inst, U), layer, P)
    X = rng.standard_normal((P, 4, 4)) + 1j * rng.standard_normal((P, 4, 4))
    c = _taylor(lambda z: O.h_trace(k, pairs, (G + z * X)[np.asarray(layer)], U),
                len(pairs) + 2, 0.3)
    assert abs(c[1] - np.sum(T * X)) < 1e-10 * max(1, abs(c[1]))


# --------------------------------------------------------------------------
# Hessian-vector products and Hessian blocks
# --------------------------------------------------------------------------

def test_tdot_exact_taylor(rng):
    k = 6
    pairs, gates = _random_circuit(rng, k, 3)
    N = len(pairs)
    U = _random_unitary(rng, 1 << k)
    X = rng.standard_normal((N, 4, 4)) + 1j * rng.standard_normal((N, 4, 4))
    Y = rng.standard_normal((N, 4, 4)) + 1j * rng.standard_normal((N, 4, 4))
    T, Td = O.tangent_T(k, pairs, gates, X, U)
    assert np.abs(T - O.euclidean_T(k, pairs, gates, U)).max() < 1e-12
    c = _taylor(lambda z: O.h_trace(k, pairs, gates + z * X, U), 2 * N + 2, 0.3)
    # sum_l <X_l, Tdot_l> = second Taylor coefficient * 2
    assert abs(np.sum(Td * X) - 2 * c[2]) < 1e-9 * max(1, abs(c[2]))
    # mixed coefficient of h(G + z1 X + z2 Y): sum_l <Y_l, Tdot_l[X]>
    M = 2 * N + 2
    r = 0.3
    zz = r * np.exp(2j * np.pi * np.arange(M) / M)
    vals = np.array([[O.h_trace(k, pairs, gates + a * X + b * Y, U) for b in zz] for a in zz])
    c11 = np.fft.fft2(vals)[1, 1] / M ** 2 / r ** 2
    assert abs(np.sum(Td * Y) - c11) < 1e-9 * max(1, abs(c11))


def test_hessian_holomorphic_blocks(rng):
    k = 4
    pairs, gates = _random_circuit(rng, k, 3)
    N = len(pairs)
    U = _random_unitary(rng, 1 << k)
    H = O.hessian_holomorphic(k, pairs, gates, U)
    Hm = H.reshape(N * 16, N * 16)
    assert np.abs(Hm - Hm.T).max() < 1e-11
    for l in range(N):
        assert np.abs(H[l, :, :, l]).max() < 1e-13      # linear in each gate
    X = rng.standard_normal((N, 4, 4)) + 1j * rng.standard_normal((N, 4, 4))
    _, Td = O.tangent_T(k, pairs, gates, X, U)
    assert np.abs((Hm @ X.reshape(-1)).reshape(N, 4, 4) - Td).max() < 1e-11
    # brute force on sampled entries: bivariate Taylor coefficient
    M = 4
    r = 0.5
    zz = r * np.exp(2j * np.pi * np.arange(M) / M)
    for (l, a, b, m, c, d) in [(0, 1, 2, 3, 0, 3), (2, 3, 3, 5, 1, 0), (1, 0, 0, 4, 2, 2)]:
        Xl = np.zeros_like(gates); Xl[l, a, b] = 1
        Ym = np.zeros_like(gates); Ym[m, c, d] = 1
        vals = np.array([[O.h_trace(k, pairs, gates + s * Xl + t * Ym, U) for t in zz] for s in zz])
        c11 = np.fft.fft2(vals)[1, 1] / M ** 2 / r ** 2
        assert abs(H[l, a, b, m, c, d] - c11) < 1e-11


def test_hessian_by_holes_equals_dual_numbers_and_taylor(rng):
    """The hole-array Hessian (hole application, second forward pass,
    contraction at every later gate) equals the dual-number Hessian
    element by element (general and parity gates, full trace and a column
    subset), and sampled entries equal bivariate Taylor coefficients of h."""
    for k, layers, parity in [(6, 3, False), (4, 4, True), (6, 3, True)]:
        pairs, gates = _random_circuit(rng, k, layers, parity)
        U = _random_unitary(rng, 1 << k)
        mask = O.riemann.PARITY_MASK if parity else None
        for cols in (None, np.array([0, 3, 9, (1 << k) - 1])):
            Uc = U if cols is None else U[:, cols]
            A = O.hessian_holomorphic(k, pairs, gates, Uc, cols, mask=mask)
            B = O.hessian_by_holes(k, pairs, gates, Uc, cols, mask=mask)
            if mask is not None:
                A = np.where(mask[None, :, :, None, None, None] & mask[None, None, None, None],
                             A, 0)
            assert np.abs(A - B).max() < 1e-13 * max(1.0, np.abs(A).max())
    k = 4
    pairs, gates = _random_circuit(rng, k, 3)
    U = _random_unitary(rng, 1 << k)
    H = O.hessian_by_holes(k, pairs, gates, U)
    M, r = 4, 0.5
    zz = r * np.exp(2j * np.pi * np.arange(M) / M)
    for (l, a, b, m, c, d) in [(0, 3, 1, 4, 2, 0), (5, 1, 1, 2, 0, 3)]:
        Xl = np.zeros_like(gates); Xl[l, a, b] = 1
        Ym = np.zeros_like(gates); Ym[m, c, d] = 1
        vals = np.array([[O.h_trace(k, pairs, gates + s * Xl + t * Ym, U) for t in zz] for s in zz])
        c11 = np.fft.fft2(vals)[1, 1] / M ** 2 / r ** 2
        assert abs(H[l, a, b, m, c, d] - c11) < 1e-11


def _retract_cost(k, pairs, gates, U, X, eps):
    cand = np.stack([O.polar(gates[p] + eps * X[p]) for p in range(len(gates))])
    return O.cost(k, pairs, cand, U)


def test_riemannian_hvp_quadratic_form_along_retraction(rng):
    # polar retraction is second order: d^2/deps^2 f(R(eps X)) = <X, Hess X>
    k = 6
    pairs, gates = _random_circuit(rng, k, 3)
    U = _random_unitary(rng, 1 << k)
    X = w.tangent_direction(rng, gates)
    Y = w.tangent_direction(rng, gates)
    T, Td = O.tangent_T(k, pairs, gates, X, U)
    eg, eh = O.egrad(T), O.egrad(Td)
    HX = O.rhvp(gates, eg, eh, X)
    # tangent and self-adjoint
    for p in range(len(gates)):
        A = gates[p].conj().T @ HX[p]
        assert np.abs(A + A.conj().T).max() < 1e-12
    _, TdY = O.tangent_T(k, pairs, gates, Y, U)
    HY = O.rhvp(gates, eg, O.egrad(TdY), Y)
    ip = lambda A, B: np.real(np.sum(np.conj(A) * B))  # noqa: E731
    assert abs(ip(Y, HX) - ip(X, HY)) < 1e-11
    h = 1e-3
    f0 = O.cost(k, pairs, gates, U)
    for D, HD in ((X, HX), (Y, HY)):
        fp = _retract_cost(k, pairs, gates, U, D, h)
        fm = _retract_cost(k, pairs, gates, U, D, -h)
        fp2 = _retract_cost(k, pairs, gates, U, D, 2 * h)
        fm2 = _retract_cost(k, pairs, gates, U, D, -2 * h)
        d2 = (-fp2 + 16 * fp - 30 * f0 + 16 * fm - fm2) / (12 * h * h)
        assert abs(d2 - ip(D, HD)) < 1e-6 * max(1, abs(d2))
    # first derivative along the retraction: <grad, X>
    g = O.rgrad(gates, eg)
    d1 = (_retract_cost(k, pairs, gates, U, X, h) - _retract_cost(k, pairs, gates, U, X, -h)) / (2 * h)
    assert abs(d1 - ip(g, X)) < 1e-6


def test_rhvp_single_gate_closed_form(rng):
    # k=2, N=1: f = -Re Tr[U^dag G], egrad = -U (constant) so
    # Hess[X] = P_G(X sym(G^dag U))
    U = _random_unitary(rng, 4)
    G = _random_unitary(rng, 4)[None]
    X = w.tangent_direction(rng, G)
    T, Td = O.tangent_T(2, [(0, 1)], G, X, U)
    assert np.abs(Td).max() == 0
    S = G[0].conj().T @ U
    ref = O.proj(G[0], X[0] @ (0.5 * (S + S.conj().T)))
    assert np.abs(O.rhvp(G, O.egrad(T), O.egrad(Td), X)[0] - ref).max() < 1e-14


def test_hessian_at_target_psd_and_weingarten(rng):
    k = 4
    pairs, gates = _random_circuit(rng, k, 2)
    N = len(pairs)
    U = O.circuit_matrix(k, pairs, gates)
    T = O.euclidean_T(k, pairs, gates, U)
    Hh = O.hessian_holomorphic(k, pairs, gates, U)
    H = O.hessian_real(gates, O.egrad(T), Hh)
    assert np.abs(H - H.T).max() < 1e-11
    ev = np.linalg.eigvalsh(H)
    assert ev.min() > -1e-10
    # diagonal blocks of unshared gates at C = U: 2^{k-2} I
    for l in range(N):
        blk = H[16 * l:16 * l + 16, 16 * l:16 * l + 16]
        assert np.abs(blk - (1 << (k - 2)) * np.eye(16)).max() < 1e-11


def test_hessian_real_matches_hvp(rng):
    k = 4
    pairs, gates = _random_circuit(rng, k, 3)
    U = _random_unitary(rng, 1 << k)
    T = O.euclidean_T(k, pairs, gates, U)
    eg = O.egrad(T)
    Hh = O.hessian_holomorphic(k, pairs, gates, U)
    H = O.hessian_real(gates, eg, Hh)
    assert np.abs(H - H.T).max() < 1e-11
    x = rng.standard_normal(H.shape[0])
    X = O.tangent_from_real(gates, x)
    _, Td = O.tangent_T(k, pairs, gates, X, U)
    HX = O.rhvp(gates, eg, O.egrad(Td), X)
    assert np.abs(O.gradient_real(gates, HX) - H @ x).max() < 1e-11
    # gradient components <X_mu, grad>
    g = O.gradient_real(gates, eg)
    assert abs(g @ x - np.real(np.sum(np.conj(O.rgrad(gates, eg)) * X))) < 1e-11


def test_real_basis_orthonormal():
    for par in (False, True):
        B = O.real_basis(par)
        G = np.array([[np.real(np.trace(a.conj().T @ b)) for b in B] for a in B])
        assert np.abs(G - np.eye(len(B))).max() < 1e-15
        for a in B:
            assert np.abs(a + a.conj().T).max() == 0
            if par:
                assert np.all(a[~w.PARITY_MASK] == 0)


# --------------------------------------------------------------------------
# Parity sectors
# --------------------------------------------------------------------------

def test_parity_sectors_and_masked_gates(rng):
    k = 6
    pairs, gates = _random_circuit(rng, k, 3, parity=True)
    Uref = O.circuit_matrix(k, pairs, w.parity_haar_gates(rng, len(pairs)))
    s0, s1 = O.sector_columns(k, 0), O.sector_columns(k, 1)
    # parity-conserving U keeps each column in its sector
    par = np.array([bin(x).count("1") & 1 for x in range(1 << k)])
    for s, p in ((s0, 0), (s1, 1)):
        assert np.abs(Uref[np.ix_(par != p, s)]).max() < 1e-14
    f = O.cost(k, pairs, gates, Uref)
    f0 = O.cost(k, pairs, gates, Uref[:, s0], s0)
    f1 = O.cost(k, pairs, gates, Uref[:, s1], s1)
    assert abs(f - f0 - f1) < 1e-12
    T = O.euclidean_T(k, pairs, gates, Uref)
    # off-pattern derivatives are those of the unrestricted f; masking them
    # and projecting equals projecting onto U(2) x U(2)
    eg = O.egrad(T)
    g = O.rgrad(gates, eg, parity=True)
    for p in range(len(gates)):
        ev = [0, 3]; od = [1, 2]
        for blk in (ev, od):
            V = gates[p][np.ix_(blk, blk)]
            E = eg[p][np.ix_(blk, blk)]
            ref = 0.5 * (E - V @ E.conj().T @ V)
            assert np.abs(g[p][np.ix_(blk, blk)] - ref).max() < 1e-13


# --------------------------------------------------------------------------
# Trust region and polar retraction
# --------------------------------------------------------------------------

def test_polar_closed_form(rng):
    V = _random_unitary(rng, 4)
    A = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    xi = V @ (0.5 * (A - A.conj().T))
    Q = O.polar(V + xi)
    assert np.abs(Q.conj().T @ Q - np.eye(4)).max() < 1e-13
    w_, v_ = np.linalg.eigh(np.eye(4) + xi.conj().T @ xi)
    ref = (V + xi) @ (v_ @ np.diag(w_ ** -0.5) @ v_.conj().T)
    assert np.abs(Q - ref).max() < 1e-13


def test_tcg_newton_step_and_boundary(rng):
    n = 12
    A = rng.standard_normal((n, n))
    H = A @ A.T + n * np.eye(n)
    g = rng.standard_normal(n)
    eta, why = O.tcg(g, H, 1e6, kappa=1e-14, theta=1.0)
    assert np.abs(eta + np.linalg.solve(H, g)).max() < 1e-8
    eta, why = O.tcg(g, H, 1e-3)
    assert why == "boundary" and abs(np.linalg.norm(eta) - 1e-3) < 1e-15
    Hn = -np.eye(n)
    eta, why = O.tcg(g, Hn, 0.5)
    assert why == "negative_curvature" and abs(np.linalg.norm(eta) - 0.5) < 1e-14
