"""Shared helpers of the GPU parity tests: oracle evaluation on a set of basis
columns and comparison metrics."""

import numpy as np

import oracle as O


def oracle_eval(k, pairs, gates, param_of, direction, Ucols, cols, parity=False):
    """Oracle f, egrad, rgrad, ehvp, rhvp (per parameter) summed over cols."""
    param_of = np.asarray(param_of)
    inst = gates[param_of]
    Z = direction[param_of] if direction is not None else np.zeros_like(inst)
    T, Td = O.tangent_T(k, pairs, inst, Z, Ucols, cols)
    P = gates.shape[0]
    Tp = O.per_param(T, param_of, P)
    Tdp = O.per_param(Td, param_of, P)
    if parity:
        Tp = np.where(O.riemann.PARITY_MASK, Tp, 0)
        Tdp = np.where(O.riemann.PARITY_MASK, Tdp, 0)
    eg = O.egrad(Tp)
    rg = O.rgrad(gates, eg, parity)
    out = dict(f=O.cost(k, pairs, inst, Ucols, cols), egrad=eg, rgrad=rg)
    if direction is not None:
        eh = O.egrad(Tdp)
        out["ehvp"] = eh
        out["rhvp"] = O.rhvp(gates, eg, eh, direction, parity)
    return out


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def sector_full_index(k, p, jprime):
    """Full basis index of compressed column j' of parity sector p."""
    jprime = np.asarray(jprime, dtype=np.int64)
    par = np.array([bin(int(v)).count("1") & 1 for v in jprime])
    return (jprime << 1) | (par ^ p)
