"""GPU parity of particle-number-sector storage (RQ_SECTORS: states of each
particle-number sector stored compressed, rows = rank of the basis state in
its sector) against the oracle: full traces, single sectors and ranges with
ragged chunks, the device-built Trotter target, and the configuration-3
circuit with particle-number gates at k = 16 in the benchmark's launch
configuration (sparse target: zero except on sampled columns, so the device
sum over every sector equals the oracle's sum over the samples)."""

import math

import numpy as np
import pytest

import oracle as O
import workloads as w
from gpu_helpers import oracle_eval, rel

# The first GPU run of these tests (k = 6, complex128, HVP over every sector)
# took a device memory fault; a host-side replay of every global access of
# that call found none out of bounds, and the cause is not found yet, so the
# library switches RQ_SECTORS off and these tests stay skipped.
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="RQ_SECTORS is switched off: its kernels took a device "
                                      "memory fault whose cause is not found yet")]

TOL = {0: dict(f=1e-12, v=1e-10), 1: dict(f=1e-5, v=1e-5)}


@pytest.fixture(scope="module")
def rq():
    import torch
    from paper_2506_23775_amd import rq as _rq
    assert torch.cuda.is_available()
    _rq.lib()
    return _rq


@pytest.fixture(autouse=True)
def _release_after_each(rq):
    import torch
    yield
    torch.cuda.synchronize()
    rq.release_workspaces()
    torch.cuda.empty_cache()


def _np(t):
    return t.detach().cpu().numpy()


def _sector_states(k, n):
    """Basis indices of popcount n in increasing order (= rank order)."""
    return np.array([x for x in range(1 << k) if bin(x).count("1") == n], dtype=np.int64)


def _problem(rng, k, layers, shared):
    pairs, layer = w.brickwall_pairs(k, layers)
    param_of = np.asarray(layer if shared else np.arange(len(pairs)), dtype=np.int32)
    P = int(param_of.max()) + 1
    gates = w.number_haar_gates(rng, P)
    direction = w.tangent_direction(rng, gates, parity="number")
    return pairs, param_of, gates, direction


def _number_target(rng, k):
    """A particle-number-conserving target: the Hubbard exp(-iHt)."""
    return w.target_unitary(k // 2, 0.5, 1.0, 4.0)


def _check(res, ref, dtype, name):
    tol = TOL[dtype]
    f, fr = float(res[0]), ref["f"]
    assert abs(f - fr) <= tol["f"] * max(1.0, abs(fr)), (name, f, fr)
    for key, r in zip(["egrad", "rgrad", "ehvp", "rhvp"], res[1:]):
        if key in ref:
            e = rel(_np(r), ref[key])
            assert e <= tol["v"], (name, key, e)
            assert np.all(_np(r)[:, ~w.NUMBER_MASK] == 0), (name, key)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("k,shared", [(6, False), (8, True), (10, False)])
def test_sector_full_trace_vs_oracle(rq, dtype, k, shared):
    """f, gradients and HVP over every sector (chunks of 64 columns: the
    sectors of k = 10 hold up to 252 states, so chunks are ragged) against
    the oracle's full trace with particle-number gates."""
    rng = np.random.default_rng([131, dtype, k, shared])
    pairs, param_of, gates, direction = _problem(rng, k, 4, shared)
    U = _number_target(rng, k)
    circ = rq.Circuit(k, pairs, param_of=param_of, number=True, sectors=True)
    tgt = rq.Target.from_dense_sectors(U, dtype)
    ref = oracle_eval(k, pairs, gates, param_of, direction, U, None, parity="number")
    _check(rq.rq_hvp(circ, tgt, gates, direction, chunk=64), ref, dtype, "hvp")
    _check(rq.rq_grad(circ, tgt, gates, chunk=64), ref, dtype, "grad")
    f = float(rq.rq_cost(circ, tgt, gates, chunk=64))
    assert abs(f - ref["f"]) <= TOL[dtype]["f"] * max(1.0, abs(ref["f"]))


@pytest.mark.parametrize("dtype", [0, 1])
def test_sector_ranges_vs_oracle(rq, dtype):
    """Single sectors and column ranges inside them (empty, one state, ragged
    tails across 64-column chunks) against the oracle over those states."""
    rng = np.random.default_rng([132, dtype])
    k = 10
    pairs, param_of, gates, direction = _problem(rng, k, 5, False)
    U = _number_target(rng, k)
    circ = rq.Circuit(k, pairs, param_of=param_of, number=True, sectors=True)
    tgt = rq.Target.from_dense_sectors(U, dtype)
    for n, begin, count in [(0, 0, 1), (1, 3, 7), (5, 30, 200), (9, 0, 10), (10, 0, 1),
                            (4, 0, 210), (6, 100, 0)]:
        res = rq.rq_hvp(circ, tgt, gates, direction, range=(n, begin, count), chunk=64)
        cols = _sector_states(k, n)[begin:begin + count]
        if count == 0:
            assert float(res[0]) == 0.0
            continue
        ref = oracle_eval(k, pairs, gates, param_of, direction, U[:, cols], cols,
                          parity="number")
        _check(res, ref, dtype, f"sector {n} [{begin}, {begin + count})")


def test_sector_sum_equals_parity_storage(rq):
    """At k = 12 the sum over all particle-number sectors equals the same
    circuit on parity-sector storage, and the per-sector results accumulated
    into one output equal the full trace."""
    import torch
    rng = np.random.default_rng(133)
    k = 12
    pairs, param_of, gates, direction = _problem(rng, k, 6, True)
    U = _number_target(rng, k)
    for dtype, tol in ((0, 1e-11), (1, 2e-5)):
        cs = rq.Circuit(k, pairs, param_of=param_of, number=True, sectors=True)
        cp = rq.Circuit(k, pairs, param_of=param_of, number=True)
        rs = rq.rq_hvp(cs, rq.Target.from_dense_sectors(U, dtype), gates, direction, chunk=256)
        rp = rq.rq_hvp(cp, rq.Target.from_dense(U, dtype, parity=True), gates, direction,
                       chunk=256)
        assert abs(float(rs[0]) - float(rp[0])) <= tol * max(1.0, abs(float(rp[0])))
        for a, b in zip(rs[1:], rp[1:]):
            assert rel(_np(a), _np(b)) <= tol
        if dtype == 0:
            tgt = rq.Target.from_dense_sectors(U, dtype)
            out = [torch.zeros((1,), dtype=torch.float64, device="cuda")] + \
                [torch.zeros((len(gates), 4, 4, 2), dtype=torch.float64, device="cuda")
                 for _ in range(4)]
            for n in range(k + 1):
                rq.rq_hvp(cs, tgt, gates, direction, range=(n, 0, math.comb(k, n)), chunk=256,
                          out=out, accumulate=True)
            assert abs(float(out[0][0]) - float(rs[0])) <= 1e-12 * max(1.0, abs(float(rs[0])))
            for a, b in zip(out[1:], rs[1:]):
                assert rel(torch.view_as_complex(a).cpu().numpy(), _np(b)) <= 1e-12


@pytest.mark.parametrize("dtype", [0, 1])
def test_sector_trotter_target_vs_oracle(rq, dtype):
    """rq_apply_circuit per particle-number sector: the device-built Strang
    target equals the sector blocks of the oracle's circuit matrix of the
    same gate list, and evaluating with it matches the oracle."""
    k = 8
    gl = w.strang_trotter_gates(k // 2, 0.5, 4)
    U = np.eye(1 << k, dtype=np.complex128)
    for pair, G in gl:
        U = O.apply_gate(U, k, pair, G)
    tgt = rq.build_trotter_target(k, gl, dtype=dtype, parity=False, sectors=True)
    want = rq.Target.from_dense_sectors(U, dtype).ref
    tol = 1e-12 if dtype == 0 else 2e-6
    assert (tgt.ref - want).abs().max().item() <= tol
    rng = np.random.default_rng([134, dtype])
    pairs, param_of, gates, direction = _problem(rng, k, 4, True)
    circ = rq.Circuit(k, pairs, param_of=param_of, number=True, sectors=True)
    ref = oracle_eval(k, pairs, gates, param_of, direction, U, None, parity="number")
    _check(rq.rq_hvp(circ, tgt, gates, direction, chunk=64), ref, dtype, "trotter")


@pytest.mark.parametrize("dtype", [1, 0])
def test_sector_config3_number_gates_bench_launch(rq, dtype):
    """Configuration 3's circuit (k = 16, 7 shared layers) with
    particle-number gates, all 17 sectors in the benchmark's chunk (4096):
    the target is zero except on sampled columns (first and last state of
    sectors, both sides of a chunk boundary), each a random unit vector of
    its sector, so the device sum equals the oracle's sum over the samples."""
    import torch
    prob = w.make_problem(3)
    k = prob.k
    rng = np.random.default_rng([135, dtype])
    gates = w.number_haar_gates(rng, prob.n_params)
    direction = w.tangent_direction(rng, gates, parity="number")
    circ = rq.Circuit(k, prob.pairs, param_of=prob.param_of, number=True, sectors=True)
    picks = [(0, 0), (1, 15), (8, 0), (8, 4095), (8, 4096), (8, 12869), (7, 11439), (16, 0)]
    td = rq.torch_dtype(dtype)
    width = math.comb(k, k // 2)
    ref = torch.zeros((1 << k, width), dtype=td, device="cuda")
    bounds = rq.sector_bounds(k)
    full = np.zeros((1 << k, len(picks)), dtype=np.complex128)
    cols = []
    for i, (n, r) in enumerate(picks):
        first, size = bounds[n]
        states = _sector_states(k, n)
        v = w.random_states(rng, size, 1)[:, 0]
        ref[first:first + size, r] = torch.from_numpy(v).to(td).cuda()
        full[states, i] = v
        cols.append(int(states[r]))
    tgt = rq.Target(ref, dtype, False)
    res = rq.rq_hvp(circ, tgt, gates, direction, chunk=4096)
    oref = oracle_eval(k, prob.pairs, gates, prob.param_of, direction, full, np.asarray(cols),
                       parity="number")
    _check(res, oref, dtype, f"config 3, number gates, sectors, dtype {dtype}")
