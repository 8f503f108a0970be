"""Writes ``config2_hessian.npz``: the oracle's Hessian of configuration 2
(k = 12 spinful Fermi-Hubbard ring of 6 sites, J = 1, U = 4, target
exp(-iH/2); brick wall of 5 layers, 30 independent Haar U(4) gates) summed
over all 4096 basis states:

* ``holo_upper``: the holomorphic blocks d^2 h / dG_l[a,b] dG_m[c,d] for
  l < m, [435, 16, 16] complex (pairs in row-major order of (l, m); entries
  a*4+b, c*4+d) -- the other triangle is their transpose, the diagonal
  blocks vanish;
* ``real_upper``: the upper triangle (row-major, diagonal included) of the
  480 x 480 real Riemannian Hessian in the orthonormal tangent basis of
  ``oracle.real_basis``;
* ``f`` and ``egrad`` at the same gates.

Calls only ``oracle`` (``hessian_by_holes``: hole application, second
forward pass, contraction at every later gate, in FP64) and the seeded input
generators of ``workloads``.  Takes tens of minutes on 8 cores.
Run from the repository root:  python tests/golden/make_config2_hessian.py
"""

import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import workloads as w  # noqa: E402


def main():
    t0 = time.time()
    prob = w.make_problem(2)
    k, pairs, gates, U = prob.k, prob.pairs, prob.gates, prob.U_ref
    inst = prob.instance_gates()
    N = len(pairs)
    H = O.hessian_by_holes(k, pairs, inst, U)
    print(f"holomorphic blocks in {time.time() - t0:.0f} s", flush=True)
    P = gates.shape[0]
    Hp = np.zeros((P, 4, 4, P, 4, 4), dtype=np.complex128)
    for l in range(N):
        for m in range(N):
            Hp[prob.param_of[l], :, :, prob.param_of[m]] += H[l, :, :, m]
    T = O.per_param(O.euclidean_T(k, pairs, inst, U), prob.param_of, P)
    eg = O.egrad(T)
    Hr = O.hessian_real(gates, eg, Hp)
    iu = np.triu_indices(N, 1)
    holo = H.reshape(N, 16, N, 16)[iu[0], :, iu[1], :]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_hessian.npz")
    np.savez_compressed(out, f=O.cost(k, pairs, inst, U), egrad=eg, holo_upper=holo,
                        real_upper=Hr[np.triu_indices(Hr.shape[0])])
    print(f"wrote {out} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
