"""One Riemannian trust-region step (FP64) in an orthonormal tangent basis.

Paper Sec. "Riemannian optimization": the quadratic model
m(X) = f + <grad f, X> + 1/2 <Hess f[X], X>, the Riemannian trust-region
method (Absil et al., Algorithm 10) with the truncated conjugate-gradient
(Steihaug-Toint) inner solver (Algorithm 11), and the polar retraction
R_V(xi) = q_polar(V + xi) applied gate by gate.

The constants are not given by the paper (parity unpinned):
theta = 1, kappa = 0.1 (inner stopping rule), rho' = 0.1 (acceptance),
Delta_bar = sqrt(dim) * pi, Delta_0 = Delta_bar / 8, radius quartered when
rho < 1/4 and doubled (capped at Delta_bar) when rho > 3/4 and the step lies
on the trust-region boundary.
"""

from __future__ import annotations

import numpy as np

from .riemann import polar, tangent_from_real


def tcg(g: np.ndarray, H: np.ndarray, delta: float, theta: float = 1.0,
        kappa: float = 0.1, max_iter: int | None = None):
    """Truncated CG for min <g,eta> + 1/2 <eta, H eta>, ||eta|| <= delta.
    Returns (eta, stop_reason)."""
    n = g.size
    max_iter = n if max_iter is None else max_iter
    eta = np.zeros(n)
    r = g.copy()
    dlt = -r
    r0 = np.linalg.norm(r)
    if r0 == 0.0:
        return eta, "zero_gradient"
    rr = r @ r

    def to_boundary(e, d):
        a, b, c = d @ d, 2 * (e @ d), e @ e - delta * delta
        return e + ((-b + np.sqrt(b * b - 4 * a * c)) / (2 * a)) * d

    for _ in range(max_iter):
        Hd = H @ dlt
        dHd = dlt @ Hd
        if dHd <= 0:
            return to_boundary(eta, dlt), "negative_curvature"
        alpha = rr / dHd
        eta_new = eta + alpha * dlt
        if np.linalg.norm(eta_new) >= delta:
            return to_boundary(eta, dlt), "boundary"
        eta = eta_new
        r = r + alpha * Hd
        rr_new = r @ r
        if np.sqrt(rr_new) <= r0 * min(r0 ** theta, kappa):
            return eta, "converged"
        dlt = -r + (rr_new / rr) * dlt
        rr = rr_new
    return eta, "max_iter"


def tr_step(gates: np.ndarray, f0: float, g: np.ndarray, H: np.ndarray, delta: float,
            cost_fn, parity: bool = False, delta_bar: float | None = None,
            rho_prime: float = 0.1):
    """One trust-region iteration.  ``cost_fn(new_gates) -> f``.
    Returns a dict with the candidate gates, acceptance, rho and new radius."""
    dim = g.size
    delta_bar = np.sqrt(dim) * np.pi if delta_bar is None else delta_bar
    eta, reason = tcg(g, H, delta)
    X = tangent_from_real(gates, eta, parity)
    cand = np.stack([polar(gates[p] + X[p]) for p in range(gates.shape[0])])
    f1 = cost_fn(cand)
    model_dec = -(g @ eta + 0.5 * eta @ (H @ eta))
    rho = (f0 - f1) / model_dec if model_dec > 0 else -np.inf
    on_boundary = abs(np.linalg.norm(eta) - delta) <= 1e-12 * max(1.0, delta)
    if rho < 0.25:
        new_delta = 0.25 * delta
    elif rho > 0.75 and on_boundary:
        new_delta = min(2 * delta, delta_bar)
    else:
        new_delta = delta
    accepted = rho > rho_prime
    return dict(eta=eta, reason=reason, candidate=cand, f_candidate=f1, rho=rho,
                accepted=accepted, new_delta=new_delta, model_decrease=model_dec,
                gates=cand if accepted else gates)


def tr_solve(gates: np.ndarray, evaluate_fn, cost_fn, max_iter: int, gtol: float = 0.0,
             parity: bool = False):
    """Riemannian trust-region method (Sec. "Riemannian optimization": the
    method of Absil et al., Algorithm 10, with tCG as inner solver and the
    polar retraction): repeat tr_step from the current point; the radius
    starts at delta_bar / 8, delta_bar = sqrt(dim) * pi.

    evaluate_fn(G) -> (f, g, H): cost, Riemannian gradient and Hessian in the
    orthonormal tangent basis at G; cost_fn(G) -> f.
    Returns (gates, history) with rows (f, |g|, delta, rho, accepted)."""
    f, g, H = evaluate_fn(gates)
    delta_bar = np.sqrt(g.size) * np.pi
    delta = delta_bar / 8
    hist = []
    for _ in range(max_iter):
        gn = float(np.linalg.norm(g))
        if gn <= gtol:
            hist.append((f, gn, delta, 0.0, False))
            break
        step = tr_step(gates, f, g, H, delta, cost_fn, parity=parity, delta_bar=delta_bar)
        hist.append((f, gn, delta, step["rho"], step["accepted"]))
        delta = step["new_delta"]
        if step["accepted"]:
            gates = step["candidate"]
            f, g, H = evaluate_fn(gates)
    return gates, hist
