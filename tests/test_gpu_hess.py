"""GPU parity of rq_hess_blocks (holomorphic blocks and the real Riemannian
Hessian) and of one trust-region step driven by it, against the oracle."""

import numpy as np
import pytest

import oracle as O
import workloads as w
from gpu_helpers import rel, sector_full_index

pytestmark = pytest.mark.gpu

PIDX = [0, 3, 12, 15, 5, 6, 9, 10]
TOL = {0: 1e-10, 1: 2e-5}


@pytest.fixture(scope="module")
def rq():
    import torch
    from paper_2506_23775_amd import rq as _rq
    assert torch.cuda.is_available()
    _rq.lib()
    return _rq


def _np(t):
    return t.detach().cpu().numpy()


def oracle_hessian(k, pairs, gates, param_of, U, cols=None, parity=False):
    param_of = np.asarray(param_of)
    inst = gates[param_of]
    mask = O.riemann.PARITY_MASK if parity else None
    Ucols = U if cols is None else U[:, cols]
    Hi = O.hessian_holomorphic(k, pairs, inst, Ucols, cols, mask=mask)
    P = gates.shape[0]
    N = len(pairs)
    Hp = np.zeros((P, 4, 4, P, 4, 4), dtype=complex)
    for l in range(N):
        for m in range(N):
            Hp[param_of[l], :, :, param_of[m]] += Hi[l, :, :, m]
    T = O.per_param(O.euclidean_T(k, pairs, inst, Ucols, cols), param_of, P)
    if parity:
        T = np.where(O.riemann.PARITY_MASK, T, 0)
    eg = O.egrad(T)
    Hr = O.hessian_real(gates, eg, Hp, parity)
    d = 8 if parity else 16
    sel = PIDX if parity else list(range(16))
    Hh = Hp.reshape(P, 16, P, 16)[:, sel][:, :, :, sel]
    return Hh, Hr, eg


def _problem(rng, k, layers, shared, parity):
    pairs, layer = w.brickwall_pairs(k, layers)
    param_of = np.asarray(layer if shared else np.arange(len(pairs)), dtype=np.int32)
    P = int(param_of.max()) + 1
    gates = (w.parity_haar_gates if parity else w.haar_gates)(rng, P)
    return pairs, param_of, gates


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("k,layers,shared,parity", [(6, 3, False, False), (6, 4, True, False),
                                                    (6, 3, False, True), (8, 3, True, True)])
def test_hessian_blocks_vs_oracle(rq, dtype, k, layers, shared, parity):
    rng = np.random.default_rng([21, k, layers, dtype, parity])
    pairs, param_of, gates = _problem(rng, k, layers, shared, parity)
    U = w.target_unitary(k // 2, 0.3, 1.0, 2.0) if parity else w.haar_unitary(rng, 1 << k)
    circ = rq.Circuit(k, pairs, param_of=param_of, parity=parity)
    tgt = rq.Target.from_dense(U, dtype, parity=parity)
    f, eg, rg, hh, hr = rq.rq_hess_blocks(circ, tgt, gates, chunk=64)
    Hh, Hr, egr = oracle_hessian(k, pairs, gates, param_of, U, parity=parity)
    assert rel(_np(eg), egr) < TOL[dtype]
    assert rel(_np(hh), Hh) < TOL[dtype], rel(_np(hh), Hh)
    hr = _np(hr)
    assert rel(hr, Hr) < TOL[dtype], rel(hr, Hr)
    assert np.abs(hr - hr.T).max() <= 10 * TOL[dtype] * np.abs(Hr).max()


@pytest.mark.parametrize("dtype", [0, 1])
def test_hessian_times_x_equals_hvp(rq, dtype):
    prob = w.make_problem(1)
    circ = rq.Circuit(prob.k, prob.pairs, param_of=prob.param_of)
    tgt = rq.Target.from_dense(prob.U_ref, dtype)
    _, _, _, _, hr = rq.rq_hess_blocks(circ, tgt, prob.gates, chunk=128)
    hr = _np(hr)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(hr.shape[0])
    X = O.tangent_from_real(prob.gates, x)
    _, _, _, _, rh = rq.rq_hvp(circ, tgt, prob.gates, X)
    hx = O.gradient_real(prob.gates, _np(rh))
    assert rel(hr @ x, hx) < TOL[dtype]


@pytest.mark.parametrize("dtype", [0, 1])
def test_hessian_basis_range_and_sector(rq, dtype):
    rng = np.random.default_rng([22, dtype])
    k = 8
    pairs, param_of, gates = _problem(rng, k, 3, False, True)
    U = w.target_unitary(4, 0.5, 1.0, 4.0)
    circ = rq.Circuit(k, pairs, param_of=param_of, parity=True)
    tgt = rq.Target.from_dense(U, dtype, parity=True)
    cols = sector_full_index(k, 1, np.arange(9, 9 + 70))
    _, _, _, hh, hr = rq.rq_hess_blocks(circ, tgt, gates, range=(1, 9, 70), chunk=64)
    Hh, Hr, _ = oracle_hessian(k, pairs, gates, param_of, U, cols=cols, parity=True)
    assert rel(_np(hh), Hh) < TOL[dtype]
    assert rel(_np(hr), Hr) < TOL[dtype]


def test_trust_region_step_from_gpu_hessian(rq):
    """One trust-region step (truncated CG + polar retraction) from the GPU
    gradient and Hessian matches the oracle's step from its own quantities."""
    prob = w.make_problem(1)
    k, pairs, gates = prob.k, prob.pairs, prob.gates
    circ = rq.Circuit(k, pairs, param_of=prob.param_of)
    tgt = rq.Target.from_dense(prob.U_ref, 0)
    f, eg, rg, _, hr = rq.rq_hess_blocks(circ, tgt, gates, chunk=256)
    g = O.gradient_real(gates, _np(eg))
    H = _np(hr)
    Hh, Hr, egr = oracle_hessian(k, pairs, gates, prob.param_of, prob.U_ref)
    gr = O.gradient_real(gates, egr)
    delta = np.sqrt(H.shape[0]) * np.pi / 8
    eta, cand, md, stop = rq.rq_tr_step(gates, g, H, delta)
    ref = O.tr_step(gates, O.cost(k, pairs, gates, prob.U_ref), gr, Hr, delta,
                    lambda G: O.cost(k, pairs, G, prob.U_ref))
    assert np.abs(eta - ref["eta"]).max() < 1e-8
    assert np.abs(cand - ref["candidate"]).max() < 1e-8
    f1 = float(rq.rq_cost(circ, tgt, cand))
    assert abs(f1 - ref["f_candidate"]) < 1e-10
    nd, acc, rho = rq.rq_tr_accept(float(f), f1, md, delta, np.sqrt(H.shape[0]) * np.pi,
                                   np.linalg.norm(eta))
    assert acc == ref["accepted"] and abs(nd - ref["new_delta"]) < 1e-12
    assert f1 < float(f)


@pytest.mark.parametrize("dtype", [0, 1])
def test_hessian_accumulates_over_basis_ranges(rq, dtype):
    """RQ_EXEC_ACCUMULATE: the Hessian (holomorphic blocks, real Riemannian
    Hessian, f and gradients) over two disjoint basis ranges added into the
    same outputs equals the call over their union (every output is linear
    in the basis-state sum at fixed gates)."""
    import torch
    prob = w.make_problem(1)
    circ = rq.Circuit(prob.k, prob.pairs, param_of=prob.param_of)
    tgt = rq.Target.from_dense(prob.U_ref, dtype)
    ref = [_np(x) for x in rq.rq_hess_blocks(circ, tgt, prob.gates, chunk=64)]
    P = prob.n_params
    outs = [torch.zeros(sh, dtype=torch.float64, device="cuda")
            for sh in ((1,), (P, 4, 4, 2), (P, 4, 4, 2), (P, 16, P, 16, 2), (16 * P, 16 * P))]
    for b, n in ((0, 100), (100, 156)):
        rq.rq_hess_blocks(circ, tgt, prob.gates, range=(-1, b, n), chunk=64, out=outs,
                          accumulate=True)
    got = [o.cpu().numpy() for o in outs]
    got = [got[0][0]] + [g[..., 0] + 1j * g[..., 1] for g in got[1:4]] + [got[4]]
    tol = 1e-12 if dtype == 0 else 1e-6
    assert abs(got[0] - ref[0]) <= tol * max(1.0, abs(ref[0]))
    for a, b in zip(got[1:], ref[1:]):
        assert rel(a, b) <= tol, rel(a, b)
