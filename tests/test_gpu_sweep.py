"""GPU parity of rq_cost / rq_grad / rq_hvp / rq_apply_circuit against the
FP64 CPU oracle (element by element on seeded inputs)."""

import numpy as np
import pytest

import oracle as O
import workloads as w
from gpu_helpers import oracle_eval, rel, sector_full_index

pytestmark = pytest.mark.gpu

TOL = {0: dict(f=1e-12, v=1e-10), 1: dict(f=1e-5, v=1e-5)}   # RQ_C128, RQ_C64


@pytest.fixture(scope="module")
def rq():
    import torch
    from paper_2506_23775_amd import rq as _rq
    assert torch.cuda.is_available()
    _rq.lib()
    return _rq


def _np(t):
    return t.detach().cpu().numpy()


def _check(res, ref, dtype, name=""):
    tol = TOL[dtype]
    f, fr = float(res[0]), ref["f"]
    assert abs(f - fr) <= tol["f"] * max(1.0, abs(fr)), (name, f, fr)
    for key, r in zip(["egrad", "rgrad", "ehvp", "rhvp"], res[1:]):
        if key in ref:
            e = rel(_np(r), ref[key])
            assert e <= tol["v"], (name, key, e)


def _dense_problem(rng, k, layers, shared=False, parity=False):
    pairs, layer = w.brickwall_pairs(k, layers)
    param_of = np.asarray(layer if shared else np.arange(len(pairs)), dtype=np.int32)
    P = int(param_of.max()) + 1
    gates = (w.parity_haar_gates if parity else w.haar_gates)(rng, P)
    direction = w.tangent_direction(rng, gates, parity=parity)
    return pairs, param_of, gates, direction


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("k,layers,shared", [(6, 3, False), (8, 3, True), (10, 4, False)])
def test_dense_full_trace(rq, dtype, k, layers, shared):
    rng = np.random.default_rng([7, k, layers, dtype])
    pairs, param_of, gates, direction = _dense_problem(rng, k, layers, shared)
    U = w.haar_unitary(rng, 1 << k)
    circ = rq.Circuit(k, pairs, param_of=param_of)
    tgt = rq.Target.from_dense(U, dtype)
    ref = oracle_eval(k, pairs, gates, param_of, direction, U, None)
    f = rq.rq_cost(circ, tgt, gates)
    assert abs(float(f) - ref["f"]) <= TOL[dtype]["f"] * max(1.0, abs(ref["f"]))
    _check(rq.rq_grad(circ, tgt, gates), ref, dtype, "grad")
    _check(rq.rq_hvp(circ, tgt, gates, direction), ref, dtype, "hvp")


@pytest.mark.parametrize("dtype", [0, 1])
def test_config1_hubbard(rq, dtype):
    prob = w.make_problem(1)
    circ = rq.Circuit(prob.k, prob.pairs, param_of=prob.param_of)
    tgt = rq.Target.from_dense(prob.U_ref, dtype)
    ref = oracle_eval(prob.k, prob.pairs, prob.gates, prob.param_of, prob.direction, prob.U_ref, None)
    _check(rq.rq_hvp(circ, tgt, prob.gates, prob.direction), ref, dtype, "cfg1")
    _check(rq.rq_grad(circ, tgt, prob.gates), ref, dtype, "cfg1")


@pytest.mark.parametrize("dtype", [0, 1])
def test_ragged_ranges_and_chunks(rq, dtype):
    rng = np.random.default_rng([8, dtype])
    k = 8
    pairs, param_of, gates, direction = _dense_problem(rng, k, 3)
    U = w.haar_unitary(rng, 1 << k)
    circ = rq.Circuit(k, pairs)
    tgt = rq.Target.from_dense(U, dtype)
    for begin, count, chunk in [(37, 100, 64), (0, 256, 64), (200, 56, 128), (255, 1, 64), (3, 0, 64)]:
        cols = np.arange(begin, begin + count)
        ref = oracle_eval(k, pairs, gates, param_of, direction, U[:, cols], cols)
        res = rq.rq_hvp(circ, tgt, gates, direction, range=(-1, begin, count), chunk=chunk)
        _check(res, ref, dtype, f"range {begin},{count},{chunk}")
        fc = rq.rq_cost(circ, tgt, gates, range=(-1, begin, count), chunk=chunk)
        assert abs(float(fc) - ref["f"]) <= TOL[dtype]["f"] * max(1.0, abs(ref["f"]))


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("k,layers,shared", [(6, 3, False), (8, 5, True), (10, 4, True)])
def test_parity_sectors(rq, dtype, k, layers, shared):
    rng = np.random.default_rng([9, k, dtype])
    pairs, param_of, gates, direction = _dense_problem(rng, k, layers, shared, parity=True)
    # parity-conserving target: exact Hubbard evolution
    U = w.target_unitary(k // 2, 0.4, 1.0, 3.0)
    circ = rq.Circuit(k, pairs, param_of=param_of, parity=True)
    tgt = rq.Target.from_dense(U, dtype, parity=True)
    ref = oracle_eval(k, pairs, gates, param_of, direction, U, None, parity=True)
    _check(rq.rq_hvp(circ, tgt, gates, direction), ref, dtype, "parity full")
    assert abs(float(rq.rq_cost(circ, tgt, gates)) - ref["f"]) <= TOL[dtype]["f"] * max(1, abs(ref["f"]))
    # one sector, ragged sub-range
    n = 1 << (k - 1)
    for p, b, c in [(1, 5, min(70, n - 5)), (0, 0, n)]:
        cols = sector_full_index(k, p, np.arange(b, b + c))
        ref = oracle_eval(k, pairs, gates, param_of, direction, U[:, cols], cols, parity=True)
        _check(rq.rq_hvp(circ, tgt, gates, direction, range=(p, b, c), chunk=64), ref, dtype,
               f"sector {p}")


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("k", [4, 5])
def test_parity_small_tiles(rq, dtype, k):
    """Parity sectors of 2^3 and 2^4 rows: below the 4-qubit tile (2-qubit
    tiles) and exactly one 4-qubit tile with no tile-index bits, with a
    parity-conserving target made of random parity gates."""
    rng = np.random.default_rng([19, k, dtype])
    # open-chain brick wall (any k): bonds (q, q+1), even bonds then odd ones
    pairs = [(q, q + 1) for layer in range(3) for q in range(layer % 2, k - 1, 2)]
    param_of = np.arange(len(pairs), dtype=np.int32)
    gates = w.parity_haar_gates(rng, len(pairs))
    direction = w.tangent_direction(rng, gates, parity=True)
    U = np.eye(1 << k, dtype=complex)
    for layer in range(6):
        for q in range(layer % 2, k - 1, 2):
            U = O.apply_gate(U, k, (q, q + 1), w.parity_haar_gates(rng, 1)[0])
    circ = rq.Circuit(k, pairs, param_of=param_of, parity=True)
    tgt = rq.Target.from_dense(U, dtype, parity=True)
    ref = oracle_eval(k, pairs, gates, param_of, direction, U, None, parity=True)
    _check(rq.rq_hvp(circ, tgt, gates, direction), ref, dtype, "parity full")
    _check(rq.rq_grad(circ, tgt, gates), ref, dtype, "parity grad")
    n = 1 << (k - 1)
    cols = sector_full_index(k, 1, np.arange(1, n))
    ref = oracle_eval(k, pairs, gates, param_of, direction, U[:, cols], cols, parity=True)
    _check(rq.rq_hvp(circ, tgt, gates, direction, range=(1, 1, n - 1), chunk=64), ref, dtype,
           "sector 1 ragged")


@pytest.mark.parametrize("dtype", [0, 1])
def test_apply_circuit(rq, dtype):
    import torch
    rng = np.random.default_rng([10, dtype])
    tol = 1e-13 if dtype == 0 else 2e-6
    k = 7
    pairs = [(int(a), int(b)) for a, b in (rng.choice(k, 2, replace=False) for _ in range(25))]
    gates = w.haar_gates(rng, len(pairs))
    W = O.circuit_matrix(k, pairs, gates)
    X = rng.standard_normal((1 << k, 77)) + 1j * rng.standard_normal((1 << k, 77))
    st = torch.from_numpy(X).to(rq.torch_dtype(dtype)).cuda()
    rq.rq_apply_circuit(rq.Circuit(k, pairs), gates, st)
    assert np.abs(_np(st) - W @ X).max() <= tol * np.abs(W @ X).max()
    # parity sector-compressed application
    kp = 8
    pp, _ = w.brickwall_pairs(kp, 4)
    gp = w.parity_haar_gates(rng, len(pp))
    Wp = O.circuit_matrix(kp, pp, gp)
    for p in (0, 1):
        rows = sector_full_index(kp, p, np.arange(1 << (kp - 1)))
        st = torch.eye(1 << (kp - 1), dtype=rq.torch_dtype(dtype)).cuda()
        rq.rq_apply_circuit(rq.Circuit(kp, pp, parity=True), gp, st, sector=p)
        assert np.abs(_np(st) - Wp[np.ix_(rows, rows)]).max() <= tol * 4


def test_c64_error_against_c128(rq):
    prob = w.make_problem(1)
    circ = rq.Circuit(prob.k, prob.pairs, param_of=prob.param_of)
    r128 = rq.rq_hvp(circ, rq.Target.from_dense(prob.U_ref, 0), prob.gates, prob.direction)
    r64 = rq.rq_hvp(circ, rq.Target.from_dense(prob.U_ref, 1), prob.gates, prob.direction)
    for a, b in zip(r64[1:], r128[1:]):
        assert rel(_np(a), _np(b)) < 1e-5


def test_deterministic_repeat(rq):
    prob = w.make_problem(1)
    circ = rq.Circuit(prob.k, prob.pairs, param_of=prob.param_of)
    tgt = rq.Target.from_dense(prob.U_ref, 1)
    a = rq.rq_hvp(circ, tgt, prob.gates, prob.direction)
    b = rq.rq_hvp(circ, tgt, prob.gates, prob.direction)
    for x, y in zip(a, b):
        assert np.array_equal(_np(x), _np(y))


@pytest.mark.parametrize("dtype", [0, 1])
def test_large_state_k20_window(rq, dtype):
    """2^20-row states (k = 20 general, k = 21 parity): at chunk 256 a
    complex128 slab is 4 GiB, so row offsets pass 2^31 bytes; the last two
    basis columns against the oracle on the same columns."""
    import torch
    rng = np.random.default_rng([11, dtype])
    for k, parity in ((20, False), (21, True)):
        pairs, layer = w.brickwall_pairs(k if k % 2 == 0 else k - 1, 1)
        gates = (w.parity_haar_gates if parity else w.haar_gates)(rng, 1)
        direction = w.tangent_direction(rng, gates, parity=parity)
        n = 1 << (k - 1) if parity else 1 << k
        width = 2
        j0 = n - width
        V = w.random_states(rng, n, width)
        td = rq.torch_dtype(dtype)
        if parity:
            ref = torch.zeros((2, n, width), dtype=td, device="cuda")
            ref[1] = torch.from_numpy(V).to(td).cuda()
            full = np.zeros((1 << k, width), dtype=complex)
            full[sector_full_index(k, 1, np.arange(n))] = V
            cols = sector_full_index(k, 1, np.arange(j0, j0 + width))
            rng_ = (1, j0, width)
        else:
            ref = torch.from_numpy(V).to(td).cuda()
            full = V
            cols = np.arange(j0, j0 + width)
            rng_ = (-1, j0, width)
        tgt = rq.Target(ref.contiguous(), dtype, parity, col_offset=j0)
        circ = rq.Circuit(k, pairs, param_of=layer, parity=parity)
        refv = oracle_eval(k, pairs, gates, layer, direction, full, cols, parity=parity)
        _check(rq.rq_hvp(circ, tgt, gates, direction, range=rng_, chunk=256), refv, dtype,
               f"k={k} parity={parity}")
        del tgt, ref
        torch.cuda.empty_cache()
