"""GPU trust-region driver (rq_tr_solve: Hessian, step, candidate cost and
acceptance per iteration) against the oracle's trust-region loop, and its
convergence to the global minimum on a representable target."""

import numpy as np
import pytest

import oracle as O
import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rq():
    import torch
    from paper_2506_23775_amd import rq as _rq
    assert torch.cuda.is_available()
    _rq.lib()
    return _rq


def _oracle_fgh(k, pairs, param_of, U, parity):
    param_of = np.asarray(param_of)
    mask = O.riemann.PARITY_MASK if parity else None

    def fn(G):
        inst = G[param_of]
        P = G.shape[0]
        T = O.per_param(O.euclidean_T(k, pairs, inst, U), param_of, P)
        if parity:
            T = np.where(O.riemann.PARITY_MASK, T, 0)
        eg = O.egrad(T)
        Hi = O.hessian_holomorphic(k, pairs, inst, U, mask=mask)
        Hp = np.zeros((P, 4, 4, P, 4, 4), dtype=complex)
        for l in range(len(pairs)):
            for m in range(len(pairs)):
                Hp[param_of[l], :, :, param_of[m]] += Hi[l, :, :, m]
        return (O.cost(k, pairs, inst, U), O.gradient_real(G, eg, parity),
                O.hessian_real(G, eg, Hp, parity))
    return fn


@pytest.mark.parametrize("parity,shared", [(False, False), (True, True)])
def test_tr_solve_matches_oracle_iterates(rq, parity, shared):
    rng = np.random.default_rng([81, parity])
    k = 6
    pairs, layer = w.brickwall_pairs(k, 3)
    param_of = np.asarray(layer if shared else np.arange(len(pairs)), dtype=np.int32)
    P = int(param_of.max()) + 1
    gates = (w.parity_haar_gates if parity else w.haar_gates)(rng, P)
    U = w.target_unitary(3, 0.4, 1.0, 3.0) if parity else w.haar_unitary(rng, 1 << k)
    circ = rq.Circuit(k, pairs, param_of=param_of, parity=parity)
    tgt = rq.Target.from_dense(U, rq.RQ_C128, parity=parity)
    iters = 5
    G, hist = rq.rq_tr_solve(circ, tgt, gates, max_iter=iters, chunk=64)
    Gr, hr = O.tr_solve(gates, _oracle_fgh(k, pairs, param_of, U, parity),
                        lambda X: O.cost(k, pairs, X[param_of], U), iters, parity=parity)
    assert len(hist) == len(hr) == iters
    for a, b in zip(hist, hr):
        assert abs(a[0] - b[0]) <= 1e-10 * max(1.0, abs(b[0]))        # f
        assert abs(a[1] - b[1]) <= 1e-8 * max(1.0, b[1])              # |grad|
        assert abs(a[2] - b[2]) <= 1e-12 * b[2]                       # radius
        assert bool(a[4]) == bool(b[4])                               # accepted
    assert np.abs(G - Gr).max() <= 1e-8


def test_tr_solve_converges_on_representable_target(rq):
    rng = np.random.default_rng(82)
    k = 8
    pairs, layer = w.brickwall_pairs(k, 3)
    Gs = w.haar_gates(rng, len(pairs))
    U = O.circuit_matrix(k, pairs, Gs)
    G0 = np.stack([O.polar(g + 0.1 * (rng.standard_normal((4, 4))
                                      + 1j * rng.standard_normal((4, 4)))) for g in Gs])
    circ = rq.Circuit(k, pairs)
    tgt = rq.Target.from_dense(U, rq.RQ_C128)
    G, hist = rq.rq_tr_solve(circ, tgt, G0, max_iter=40, gtol=1e-9, chunk=256)
    fs = hist[:, 0]
    assert np.all(np.diff(fs) <= 1e-9)                       # monotone over iterations
    f_end = float(rq.rq_cost(circ, tgt, G))
    assert abs(f_end + (1 << k)) <= 1e-8
    assert hist[-1, 1] <= 1e-6
