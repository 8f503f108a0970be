"""One evaluation of the hot path as the oracle computes it (FP64 CPU):
f, the Euclidean and Riemannian gradient per parameter, and the Euclidean and
Riemannian Hessian-vector product along one tangent direction, summed over a
set of basis states.

TEST INFRASTRUCTURE ONLY (see the package header).

Composition of the steps of Sec. "Riemannian optimization" and Sec.
"Gradient and Hessian tensor diagrams": T_l and its directional derivative
Tdot_l per gate instance (dual numbers), summed per parameter for shared
gates (Sec. "Brick wall circuit layout"), masked to the U(2) x U(2) pattern
in parity mode (Sec. "Parity-conserving gate structure"), then the
Euclidean gradient -conj(T), its projection, and the Riemannian HVP.
"""

from __future__ import annotations

import numpy as np

from .dense import cost, tangent_T
from .riemann import egrad, gate_mask, per_param, rgrad, rhvp


def evaluate(k, pairs, gates, param_of, direction, Ucols, cols=None, parity=False,
             inputs=None) -> dict:
    """Returns dict(f, egrad, rgrad[, ehvp, rhvp]) for gates [P,4,4] with
    instances param_of[l], target columns Ucols = U|j> for j in cols (all
    2^k basis states when cols is None), and an optional direction [P,4,4].
    With ``inputs`` (2^k x n) the sum runs over those states psi_j instead,
    and Ucols holds U psi_j."""
    param_of = np.asarray(param_of)
    inst = gates[param_of]
    Z = direction[param_of] if direction is not None else np.zeros_like(inst)
    T, Td = tangent_T(k, pairs, inst, Z, Ucols, cols, inputs)
    P = gates.shape[0]
    Tp = per_param(T, param_of, P)
    Tdp = per_param(Td, param_of, P)
    mask = gate_mask(parity)
    if mask is not None:
        Tp = np.where(mask, Tp, 0)
        Tdp = np.where(mask, Tdp, 0)
    eg = egrad(Tp)
    out = dict(f=cost(k, pairs, inst, Ucols, cols, inputs), egrad=eg,
               rgrad=rgrad(gates, eg, parity))
    if direction is not None:
        eh = egrad(Tdp)
        out["ehvp"] = eh
        out["rhvp"] = rhvp(gates, eg, eh, direction, parity)
    return out
