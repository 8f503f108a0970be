"""Writes ``config2_eval.json``: the oracle's f, Euclidean and Riemannian
gradient and Hessian-vector product for configuration 2 (k = 12 spinful
Fermi-Hubbard ring of 6 sites, J = 1, U = 4, target exp(-iH/2); brick wall of
5 layers, 30 independent Haar U(4) gates; one seeded tangent direction),
summed over all 4096 basis states.

Calls only ``oracle`` and the seeded input generators of ``workloads``.
Run from the repository root:  python tests/golden/make_config2_golden.py
"""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import workloads as w  # noqa: E402


def _c(a):
    a = np.asarray(a)
    return np.stack([a.real, a.imag], axis=-1).tolist()


def main():
    prob = w.make_problem(2)
    ref = O.evaluate(prob.k, prob.pairs, prob.gates, prob.param_of, prob.direction, prob.U_ref, None)
    out = {"config": "k=12, 5 layers, 30 Haar U(4) gates, target exp(-iH/2), all 4096 basis states",
           "f": float(ref["f"])}
    for key in ("egrad", "rgrad", "ehvp", "rhvp"):
        out[key] = _c(ref[key])
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_eval.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path)


if __name__ == "__main__":
    main()
