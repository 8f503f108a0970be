"""Shared helpers of the GPU parity tests: oracle evaluation on a set of basis
columns and comparison metrics."""

import numpy as np

import oracle as O


def oracle_eval(k, pairs, gates, param_of, direction, Ucols, cols, parity=False):
    """Oracle f, egrad, rgrad, ehvp, rhvp (per parameter) summed over cols."""
    return O.evaluate(k, pairs, gates, param_of, direction, Ucols, cols, parity=parity)


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
