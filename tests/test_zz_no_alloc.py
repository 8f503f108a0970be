"""rq_hvp_static (the allocation-free variant of rq_hvp, workspace in the
library's static device scratch) against rq_hvp at the same chunk, through
the C ABI: two calls in a row, the second on a smaller input, both equal to
rq_hvp bitwise and to the oracle; and the size limit of the scratch."""

import ctypes as C

import numpy as np
import pytest

import workloads as w
from gpu_helpers import oracle_eval, rel, sector_full_index


@pytest.fixture(scope="module")
def rq():
    from paper_2506_23775_amd import rq as _rq
    _rq.lib()
    return _rq


def _static(rq, circ, tgt, gates, direction, rng=None):
    """Direct ctypes call of rq_hvp_static with preallocated outputs."""
    import torch
    L = rq.lib()
    P = circ.n_params
    outs = [torch.full((1,), 7.0, dtype=torch.float64, device="cuda")] + \
        [torch.full((P, 4, 4, 2), 7.0, dtype=torch.float64, device="cuda") for _ in range(4)]
    g = rq._gates_host(gates)
    d = rq._gates_host(direction)
    t = tgt.struct()
    used = C.c_int64(0)
    st = L.rq_hvp_static(C.byref(circ._c), C.byref(t), rq._dptr(g), rq._dptr(d), rq._range(rng),
                         torch.cuda.current_stream().cuda_stream, 0, C.byref(used),
                         *[o.data_ptr() for o in outs])
    assert st == rq.RQ_OK, L.rq_last_error()
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs], used.value


def _ref(rq, circ, tgt, gates, direction, chunk, rng=None):
    import torch
    res = rq.rq_hvp(circ, tgt, gates, direction, range=rng, chunk=chunk)
    torch.cuda.synchronize()
    return [r.detach().cpu().numpy() if r.dim() == 0 else
            torch.view_as_real(r).cpu().numpy() for r in res]


@pytest.mark.gpu
def test_static_equals_hvp_two_calls_second_smaller(rq):
    import torch
    assert torch.cuda.is_available()
    # call 1: configuration 1 (k = 8, 12 Haar gates), all 256 basis states, c128
    prob = w.make_problem(1)
    circ = rq.Circuit(prob.k, prob.pairs, param_of=prob.param_of)
    tgt = rq.Target.from_dense(prob.U_ref, rq.RQ_C128)
    got, chunk = _static(rq, circ, tgt, prob.gates, prob.direction)
    assert chunk == 256
    ref = _ref(rq, circ, tgt, prob.gates, prob.direction, chunk)
    assert float(got[0][0]) == float(ref[0])
    for a, b in zip(got[1:], ref[1:]):
        assert np.array_equal(a, b)
    orc = oracle_eval(prob.k, prob.pairs, prob.gates, prob.param_of, prob.direction,
                      prob.U_ref, None)
    assert abs(float(got[0][0]) - orc["f"]) <= 1e-12 * max(1.0, abs(orc["f"]))
    for key, a in zip(["egrad", "rgrad", "ehvp", "rhvp"], got[1:]):
        assert rel(a[..., 0] + 1j * a[..., 1], orc[key]) <= 1e-10, key
    # call 2, smaller: k = 6 parity circuit, 20 columns of sector 1, c64
    rng_ = np.random.default_rng([w.configs.SEED, 77])
    k = 6
    pairs, _ = w.brickwall_pairs(k, 3)
    gates = w.parity_haar_gates(rng_, len(pairs))
    direction = w.tangent_direction(rng_, gates, parity=True)
    from workloads.hubbard import target_unitary
    Uref = target_unitary(k // 2, 0.4, 1.0, 3.0)
    circ2 = rq.Circuit(k, pairs, parity=True)
    tgt2 = rq.Target.from_dense(Uref, rq.RQ_C64, parity=True)
    rng2 = (1, 5, 20)
    got2, chunk2 = _static(rq, circ2, tgt2, gates, direction, rng2)
    assert chunk2 == 64
    ref2 = _ref(rq, circ2, tgt2, gates, direction, chunk2, rng2)
    assert float(got2[0][0]) == float(ref2[0])
    for a, b in zip(got2[1:], ref2[1:]):
        assert np.array_equal(a, b)
    cols = sector_full_index(k, 1, np.arange(5, 25))
    orc2 = oracle_eval(k, pairs, gates, np.arange(len(pairs)), direction, Uref[:, cols], cols,
                       parity=True)
    assert abs(float(got2[0][0]) - orc2["f"]) <= 1e-5 * max(1.0, abs(orc2["f"]))
    for key, a in zip(["egrad", "rgrad", "ehvp", "rhvp"], got2[1:]):
        assert rel(a[..., 0] + 1j * a[..., 1], orc2[key]) <= 1e-5, key


def test_static_rejects_problems_beyond_the_scratch(rq):
    """Configuration 3 (k = 16 parity HVP) needs more than the 256 MiB scratch
    at the smallest chunk: RQ_ESPACE before any device work (fake pointers,
    never dereferenced)."""
    L = rq.lib()
    prob = w.make_problem(3, trotter_steps=1)
    circ = rq.Circuit(prob.k, prob.pairs, param_of=prob.param_of, parity=True)
    t = rq._Target(rq.RQ_C64, 0, 0x1000, 1 << 15, 1 << 30, None, 0, 0)
    g = rq._gates_host(prob.gates)
    d = rq._gates_host(prob.direction)
    st = L.rq_hvp_static(C.byref(circ._c), C.byref(t), rq._dptr(g), rq._dptr(d), None, None, 0,
                         None, None, None, None, None, None)
    assert st == rq.RQ_ESPACE
    assert b"static scratch" in L.rq_last_error()
