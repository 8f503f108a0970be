"""GPU parity of the input-state path (trace over random vectors instead of
the basis, Sec. "Conclusions"): rq_cost / rq_grad / rq_hvp / rq_hess_blocks
with input states against the oracle on the same inputs, element by element;
the device-built sampled target (gate-list target applied with
rq_apply_circuit) against the oracle; and the random-vector estimate against
the exact trace within its standard error."""

import numpy as np
import pytest

import oracle as O
import workloads as w
from gpu_helpers import rel, sector_full_index

pytestmark = pytest.mark.gpu

TOL = {0: dict(f=1e-12, v=1e-10), 1: dict(f=1e-5, v=1e-5)}


@pytest.fixture(scope="module")
def rq():
    import torch
    from paper_2506_23775_amd import rq as _rq
    assert torch.cuda.is_available()
    _rq.lib()
    return _rq


def _np(t):
    return t.detach().cpu().numpy()


def _check(res, ref, dtype, name):
    tol = TOL[dtype]
    f, fr = float(res[0]), ref["f"]
    assert abs(f - fr) <= tol["f"] * max(1.0, abs(fr)), (name, f, fr)
    for key, r in zip(["egrad", "rgrad", "ehvp", "rhvp"], res[1:]):
        if key in ref:
            e = rel(_np(r), ref[key])
            assert e <= tol["v"], (name, key, e)


def _problem(rng, k, layers, parity=False):
    pairs, _ = w.brickwall_pairs(k, layers)
    P = len(pairs)
    gates = (w.parity_haar_gates if parity else w.haar_gates)(rng, P)
    direction = w.tangent_direction(rng, gates, parity=parity)
    return pairs, np.arange(P, dtype=np.int32), gates, direction


def _device_target(rq, dtype, parity, Zin, Y):
    """Target with input states Zin and columns Y (sector blocks [2, n, R] in
    parity mode, [2^k, R] otherwise)."""
    import torch
    td = rq.torch_dtype(dtype)
    inp = torch.from_numpy(np.ascontiguousarray(Zin)).to(td).cuda()
    ref = torch.from_numpy(np.ascontiguousarray(Y)).to(td).cuda()
    return rq.Target(ref, dtype, parity, inputs=inp)


@pytest.mark.parametrize("dtype", [0, 1])
def test_inputs_dense_vs_oracle(rq, dtype):
    rng = np.random.default_rng([41, dtype])
    k, R = 8, 77
    pairs, param_of, gates, direction = _problem(rng, k, 4)
    U = w.haar_unitary(rng, 1 << k)
    Z = w.random_states(rng, 1 << k, R) * np.sqrt(1 << k)
    tgt = _device_target(rq, dtype, False, Z, U @ Z)
    circ = rq.Circuit(k, pairs)
    ref = O.evaluate(k, pairs, gates, param_of, direction, U @ Z, None, inputs=Z)
    _check(rq.rq_hvp(circ, tgt, gates, direction, range=(-1, 0, R), chunk=64), ref, dtype, "hvp")
    _check(rq.rq_grad(circ, tgt, gates, range=(-1, 0, R), chunk=64), ref, dtype, "grad")
    f = float(rq.rq_cost(circ, tgt, gates, range=(-1, 0, R), chunk=64))
    assert abs(f - ref["f"]) <= TOL[dtype]["f"] * max(1.0, abs(ref["f"]))
    # a ragged sub-range of the input columns
    sub = O.evaluate(k, pairs, gates, param_of, direction, (U @ Z)[:, 5:70], None,
                     inputs=Z[:, 5:70])
    _check(rq.rq_hvp(circ, tgt, gates, direction, range=(-1, 5, 65), chunk=64), sub, dtype, "sub")


@pytest.mark.parametrize("dtype", [0, 1])
def test_inputs_parity_sectors_vs_oracle(rq, dtype):
    rng = np.random.default_rng([42, dtype])
    k, R = 8, 50
    n = 1 << (k - 1)
    pairs, param_of, gates, direction = _problem(rng, k, 5, parity=True)
    U = w.target_unitary(4, 0.5, 1.0, 4.0)
    Zs = np.stack([w.random_states(rng, n, R) * np.sqrt(n) for _ in (0, 1)])
    Ys = np.stack([U[np.ix_(sector_full_index(k, p, np.arange(n)),
                            sector_full_index(k, p, np.arange(n)))] @ Zs[p] for p in (0, 1)])
    tgt = _device_target(rq, dtype, True, Zs, Ys)
    circ = rq.Circuit(k, pairs, parity=True)
    full = np.zeros((1 << k, 2 * R), dtype=complex)
    for p in (0, 1):
        full[sector_full_index(k, p, np.arange(n)), p * R:(p + 1) * R] = Zs[p]
    ref = O.evaluate(k, pairs, gates, param_of, direction, U @ full, None, parity=True,
                     inputs=full)
    _check(rq.rq_hvp(circ, tgt, gates, direction, range=(-1, 0, R), chunk=64), ref, dtype,
           "both sectors")
    one = O.evaluate(k, pairs, gates, param_of, direction, U @ full[:, R + 3:R + 40], None,
                     parity=True, inputs=full[:, R + 3:R + 40])
    _check(rq.rq_hvp(circ, tgt, gates, direction, range=(1, 3, 37), chunk=64), one, dtype,
           "sector 1")


@pytest.mark.parametrize("dtype", [0, 1])
def test_inputs_hessian_vs_oracle(rq, dtype):
    rng = np.random.default_rng([43, dtype])
    k, R = 6, 20
    pairs, param_of, gates, _ = _problem(rng, k, 3)
    U = w.haar_unitary(rng, 1 << k)
    Z = w.random_states(rng, 1 << k, R)
    tgt = _device_target(rq, dtype, False, Z, U @ Z)
    circ = rq.Circuit(k, pairs)
    _, eg, _, hh, _ = rq.rq_hess_blocks(circ, tgt, gates, range=(-1, 0, R), chunk=64)
    Hi = O.hessian_holomorphic(k, pairs, gates, U @ Z, None, inputs=Z)
    N = len(pairs)
    assert rel(_np(hh), Hi.reshape(N, 16, N, 16)) <= TOL[dtype]["v"] * 10
    T = O.euclidean_T(k, pairs, gates, U @ Z, None, inputs=Z)
    assert rel(_np(eg), O.egrad(T)) <= TOL[dtype]["v"]


def test_sampled_target_from_gate_list(rq):
    """rq.sampled_target builds U z_r on the device from a Trotter gate list;
    the oracle applies the same gate list on the host."""
    rng = np.random.default_rng(44)
    k, R = 8, 40
    pairs, param_of, gates, direction = _problem(rng, k, 3, parity=True)
    gl = w.strang_trotter_gates(4, 0.5, 6, 1.0, 4.0)
    tgt = rq.sampled_target(k, R, np.random.default_rng(45), dtype=rq.RQ_C128, parity=True,
                            gate_list=gl)
    n = 1 << (k - 1)
    Zs = _np(tgt.inputs)
    full = np.zeros((1 << k, 2 * R), dtype=complex)
    for p in (0, 1):
        full[sector_full_index(k, p, np.arange(n)), p * R:(p + 1) * R] = Zs[p]
    Y = full.copy()
    for pair, G in gl:
        Y = O.apply_gate(Y, k, pair, G)
    ref = O.evaluate(k, pairs, gates, param_of, direction, Y, None, parity=True, inputs=full)
    circ = rq.Circuit(k, pairs, parity=True)
    _check(rq.rq_hvp(circ, tgt, gates, direction, range=(-1, 0, R), chunk=64), ref, 0, "sampled")


def test_estimate_unbiased_against_exact_trace(rq):
    """1024 complex-Rademacher vectors per sector at k = 10: the estimate of f
    and of the Riemannian gradient lies within 5 standard errors of the exact
    trace (standard errors from 8 independent batches)."""
    rng = np.random.default_rng(46)
    k = 10
    pairs, param_of, gates, _ = _problem(rng, k, 4, parity=True)
    U = w.target_unitary(5, 0.5, 1.0, 4.0)
    circ = rq.Circuit(k, pairs, parity=True)
    exact = rq.rq_grad(circ, rq.Target.from_dense(U, rq.RQ_C128, parity=True), gates)
    fe, rge = float(exact[0]), _np(exact[2])
    B, R = 8, 128
    fs, rgs = [], []
    for b in range(B):
        tgt = rq.sampled_target(k, R, np.random.default_rng([47, b]), parity=True, U=U)
        res = rq.rq_grad(circ, tgt, gates, range=(-1, 0, R), chunk=64)
        fs.append(float(res[0]) / R)
        rgs.append(_np(res[2]) / R)
    fs, rgs = np.asarray(fs), np.asarray(rgs)
    se = fs.std(ddof=1) / np.sqrt(B)
    assert abs(fs.mean() - fe) <= 5 * se + 1e-9
    m = rgs.mean(axis=0)
    se_g = rgs.std(axis=0, ddof=1) / np.sqrt(B)
    assert np.all(np.abs(m - rge) <= 5 * se_g + 1e-9)
