"""Riemannian geometry of the product manifold U(4)^P (FP64, dense 4x4).

Paper Sec. "Riemannian optimization":
* tangent space T_V U = {V A : A^dagger = -A}, metric <X, Y> = Re Tr[X^dagger Y];
* projection P_V X = V skew(V^dagger X), skew(A) = (A - A^dagger)/2;
* gradient convention grad f(z) = d_x f + i d_y f, so that
  d/deps f(G + eps X) = Re Tr[(grad f)^dagger X]; for f = -Re h with h
  holomorphic and dh/dG = T this is  grad f = -conj(T);
* Riemannian gradient = P_V(Euclidean gradient);
* Riemannian Hessian Hess f[X] = nabla_X grad f = P_V(D xi(V)[X]) with the
  Levi-Civita connection of the embedded submanifold.  Differentiating the
  extension xi(V) = P_V(egrad(V)) and projecting gives
  Hess f(V)[X] = P_V( D egrad(V)[X] - X sym(V^dagger egrad(V)) ),
  sym(A) = (A + A^dagger)/2;
* product manifold: everything acts per gate parameter; shared (repeated)
  gates sum their instance derivatives (Sec. "Brick wall circuit layout").

Parity mode (Sec. "Parity-conserving gate structure"): gates are restricted to
U(2) x U(2) on the pattern {0,3} x {0,3} + {1,2} x {1,2}; for such V the
projection maps pattern matrices to pattern matrices, so masking after the
U(4) formulas gives the restricted manifold's quantities.

The orthonormal real basis of the tangent space (``real_basis``) is a
convention the paper does not fix: parity unpinned (only basis-invariant
quantities are pinned by tests).
"""

from __future__ import annotations

import numpy as np

PARITY_MASK = np.array([[1, 0, 0, 1],
                        [0, 1, 1, 0],
                        [0, 1, 1, 0],
                        [1, 0, 0, 1]], dtype=bool)


def _dag(A):
    return np.conj(np.swapaxes(A, -1, -2))


# Particle-number-conserving gates (Sec. "Parity-conserving gate structure":
# the further restriction that removes two more parameters): U(1) x U(2) x U(1)
# on {00}, {01, 10}, {11}, i.e. the parity pattern without (0,3) and (3,0).
NUMBER_MASK = np.array([[1, 0, 0, 0],
                        [0, 1, 1, 0],
                        [0, 1, 1, 0],
                        [0, 0, 0, 1]], dtype=bool)


def gate_mask(parity):
    """Entry pattern of the gate manifold: None (U(4)), the parity pattern
    (parity True / "parity") or the particle-number pattern ("number")."""
    if parity == "number":
        return NUMBER_MASK
    return PARITY_MASK if parity else None


def _masked(A, parity):
    m = gate_mask(parity)
    return A if m is None else np.where(m, A, 0)


def per_param(T_inst: np.ndarray, param_of, n_params: int) -> np.ndarray:
    """Sum instance derivatives into parameter derivatives."""
    out = np.zeros((n_params,) + T_inst.shape[1:], dtype=T_inst.dtype)
    for l, p in enumerate(param_of):
        out[p] += T_inst[l]
    return out


def egrad(T: np.ndarray) -> np.ndarray:
    """Euclidean gradient of f = -Re h from T = dh/dG."""
    return -np.conj(T)


def proj(V: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """P_V Y = V skew(V^dagger Y) = (Y - V Y^dagger V)/2 for unitary V."""
    A = _dag(V) @ Y
    return V @ (0.5 * (A - _dag(A)))


def rgrad(V: np.ndarray, eg: np.ndarray, parity=False) -> np.ndarray:
    return _masked(proj(V, eg), parity)


def rhvp(V: np.ndarray, eg: np.ndarray, ehvp: np.ndarray, X: np.ndarray,
         parity: bool = False) -> np.ndarray:
    """Hess f(V)[X] = P_V(D egrad[X] - X sym(V^dagger egrad))."""
    S = _dag(V) @ eg
    sym = 0.5 * (S + _dag(S))
    return _masked(proj(V, ehvp - X @ sym), parity)


def real_basis(parity: bool = False):
    """Orthonormal basis A_mu of the anti-Hermitian 4x4 matrices (u(4), 16
    elements) or of u(2) + u(2) on the parity pattern (8 elements).  Tangent
    basis vectors are X_mu = V A_mu; <V A, V B> = Re Tr[A^dagger B]."""
    E = lambda a, b: np.eye(4, dtype=np.complex128)[:, [a]] @ np.eye(4)[[b], :]  # noqa: E731
    r2 = np.sqrt(0.5)
    if parity == "number":
        return [1j * E(0, 0), 1j * E(3, 3),
                1j * E(1, 1), 1j * E(2, 2), r2 * (E(1, 2) - E(2, 1)), 1j * r2 * (E(1, 2) + E(2, 1))]
    if parity:
        return [1j * E(0, 0), 1j * E(3, 3), r2 * (E(0, 3) - E(3, 0)), 1j * r2 * (E(0, 3) + E(3, 0)),
                1j * E(1, 1), 1j * E(2, 2), r2 * (E(1, 2) - E(2, 1)), 1j * r2 * (E(1, 2) + E(2, 1))]
    offd = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    return ([1j * E(a, a) for a in range(4)]
            + [r2 * (E(a, b) - E(b, a)) for a, b in offd]
            + [1j * r2 * (E(a, b) + E(b, a)) for a, b in offd])


def gradient_real(V: np.ndarray, eg: np.ndarray, parity: bool = False) -> np.ndarray:
    """Components <V_p A_mu, grad f> of the Riemannian gradient."""
    basis = real_basis(parity)
    P = V.shape[0]
    out = np.zeros((P, len(basis)))
    for p in range(P):
        for m, A in enumerate(basis):
            out[p, m] = np.real(np.sum(np.conj(V[p] @ A) * eg[p]))
    return out.reshape(-1)


def tangent_from_real(V: np.ndarray, eta: np.ndarray, parity: bool = False) -> np.ndarray:
    basis = real_basis(parity)
    d = len(basis)
    eta = eta.reshape(V.shape[0], d)
    return np.stack([V[p] @ sum(eta[p, m] * basis[m] for m in range(d))
                     for p in range(V.shape[0])])


def hessian_real(V: np.ndarray, eg: np.ndarray, Hh: np.ndarray,
                 parity: bool = False) -> np.ndarray:
    """Riemannian Hessian in the orthonormal basis X_{p,mu} = V_p A_mu.

    Hh[p, a, b, q, c, d] = d^2 h / dG_p[a,b] dG_q[c,d] summed over instances.
    H[(p,mu),(q,nu)] = <X_{p,mu}, Hess f[X_{q,nu}]>
                     = -Re sum X_{p,mu}[ab] Hh[p,ab,q,cd] X_{q,nu}[cd]
                       - delta_pq Re Tr[A_mu^dagger A_nu sym(V_p^dagger egrad_p)]."""
    basis = real_basis(parity)
    d = len(basis)
    P = V.shape[0]
    X = np.zeros((P, d, 4, 4), dtype=np.complex128)
    for p in range(P):
        for m in range(d):
            X[p, m] = V[p] @ basis[m]
    H = -np.real(np.einsum("pmab,pabqcd,qncd->pmqn", X, Hh, X))
    for p in range(P):
        S = _dag(V[p]) @ eg[p]
        sym = 0.5 * (S + _dag(S))
        for m in range(d):
            for n in range(d):
                H[p, m, p, n] -= np.real(np.trace(_dag(basis[m]) @ basis[n] @ sym))
    return H.reshape(P * d, P * d)


def polar(A: np.ndarray) -> np.ndarray:
    """Unitary factor Q of the polar decomposition A = Q P (paper eq. for the
    retraction), from the SVD A = W S V^dagger as Q = W V^dagger."""
    W, _, Vh = np.linalg.svd(A)
    return W @ Vh
