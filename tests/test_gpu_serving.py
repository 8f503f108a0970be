"""Continuous batching on the GPU: every request's result is the same alone
and in the mix, and matches the oracle."""

import numpy as np
import pytest

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
    descs = w.configs.serving_requests(10, rate_hz=400.0, ks=(8, 10), depths=(3, 5))
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
