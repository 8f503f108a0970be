"""Continuous batching on the GPU: every request's result is the same alone
and in the mix, and matches the oracle."""

import numpy as np
import pytest

import oracle as O
import workloads as w
from gpu_helpers import oracle_eval, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    from paper_2506_23775_amd import rq, serving
    assert torch.cuda.is_available()
    return torch, rq, serving


def _requests(serving, rq, dtype):
    descs = w.configs.serving_requests(10, rate_hz=400.0, ks=(8, 10, 12), depths=(3, 5))
    return descs, [serving.make_gpu_request(d, dtype) for d in descs]


def test_mix_equals_alone_and_oracle(mods):
    torch, rq, serving = mods
    dtype = rq.RQ_C64
    descs, reqs = _requests(serving, rq, dtype)
    ex = serving.GpuExecutor(dtype, chunk=256)
    b = serving.ContinuousBatcher(ex, hbm_budget=8 << 30, max_active=6)
    done = b.run(reqs)
    assert len(done) == len(reqs)
    admits = [e for e in b.log if e[0] == "admit"]
    # at least one request was admitted while another was still running
    overlap = False
    for r in done:
        for q in done:
            if q.rid != r.rid and r.t_admit < q.t_admit < r.t_done:
                overlap = True
    assert overlap, b.log
    assert len(admits) == len(reqs)
    mixed = {r.rid: r.result for r in done}
    for d in descs:
        alone = serving.ContinuousBatcher(serving.GpuExecutor(dtype, chunk=256),
                                          hbm_budget=8 << 30).run(
            [serving.make_gpu_request({**d, "arrival": 0.0}, dtype)])[0].result
        for key, v in mixed[d["rid"]].items():
            assert np.array_equal(np.asarray(v), np.asarray(alone[key])), (d["rid"], key)
    # oracle on the k=8 requests
    checked = 0
    for d in descs:
        if d["k"] != 8:
            continue
        prob = w.configs.request_problem(d)
        ref = oracle_eval(prob.k, prob.pairs, prob.gates, prob.param_of,
                          prob.direction if d["op"] == "hvp" else None, prob.U_ref, None)
        res = mixed[d["rid"]]
        assert abs(res["f"] - ref["f"]) <= 1e-5 * max(1, abs(ref["f"]))
        for key in ("egrad", "rgrad", "ehvp", "rhvp"):
            if key in res:
                assert rel(res[key], ref[key]) < 1e-5, (d["rid"], key)
        checked += 1
    assert checked >= 1
    st = serving.latency_stats(done)
    assert st["all"]["p99_ms"] >= st["all"]["p50_ms"] > 0


def _trotter_oracle(prob, op):
    """Oracle result of a request whose target is a Trotter gate list: the
    target columns U|j> are the oracle's own gate applications to the
    identity."""
    k = prob.k
    U = np.eye(1 << k, dtype=np.complex128)
    for pair, G in prob.trotter:
        U = O.apply_gate(U, k, pair, G)
    return oracle_eval(k, prob.pairs, prob.gates, prob.param_of,
                       prob.direction if op == "hvp" else None, U, None)


def test_concurrent_trotter_targets_alone_equal_mix_and_oracle(mods):
    """Requests whose targets are built on the device from different Trotter
    gate lists, admitted together on their own streams: each target build
    uses its own apply workspace, so every result equals the request run
    alone (bitwise) and the oracle."""
    torch, rq, serving = mods
    dtype = rq.RQ_C64
    descs = [dict(rid=i, arrival=0.0, k=8, depth=3 + 2 * (i % 2), U=2.0 + 1.5 * i,
                  t=0.3 + 0.4 * i, op=("hvp", "grad", "f", "hvp")[i]) for i in range(4)]
    mk = lambda d: serving.make_gpu_request(d, dtype, trotter_steps=6, dense_max_k=0)
    ex = serving.GpuExecutor(dtype, chunk=64)
    b = serving.ContinuousBatcher(ex, hbm_budget=8 << 30, max_active=4)
    done = b.run([mk(d) for d in descs])
    assert len(done) == 4
    # all four were admitted before the first one finished
    first_done = min(r.t_done for r in done)
    assert all(r.t_admit < first_done for r in done), b.log
    mixed = {r.rid: r.result for r in done}
    for d in descs:
        alone = serving.ContinuousBatcher(serving.GpuExecutor(dtype, chunk=64),
                                          hbm_budget=8 << 30).run([mk(d)])[0].result
        for key, v in mixed[d["rid"]].items():
            assert np.array_equal(np.asarray(v), np.asarray(alone[key])), (d["rid"], key)
        prob = w.configs.request_problem(d, trotter_steps=6, dense_max_k=0)
        ref = _trotter_oracle(prob, d["op"])
        res = mixed[d["rid"]]
        assert abs(res["f"] - ref["f"]) <= 1e-5 * max(1, abs(ref["f"])), (d["rid"], res["f"])
        for key in ("egrad", "rgrad", "ehvp", "rhvp"):
            if key in res:
                assert rel(res[key], ref[key]) < 1e-5, (d["rid"], key)
