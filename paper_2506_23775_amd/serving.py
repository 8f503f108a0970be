"""Continuous-batching serving loop for f / gradient / HVP requests.

Requests (mixed qubit counts and depths) arrive over time.  Each request is
split into chunks of basis states (disjoint ranges of the trace sum).  The
scheduler keeps a set of active requests, each with its own HIP stream,
device-resident target columns, workspace and output buffers:

* admission: arrivals are admitted in FIFO order while the number of active
  requests is below ``max_active`` and the request's HBM footprint (target
  columns + workspace + outputs) fits the remaining budget; otherwise they
  wait (the loop never allocates beyond the budget);
* interleaving: whenever a request's stream is idle, its next chunk is
  enqueued there, so chunks of different requests -- including ones admitted
  while others run -- execute concurrently on the device;
* accumulation: chunk results are added into the request's outputs by the
  library itself (``RQ_EXEC_ACCUMULATE``), in chunk order, so a request's
  result does not depend on what else is in flight;
* completion frees the request's memory and slot for the next arrival.

Latency of a request = completion time - arrival time (host clock); the
evaluation part (admission -> completion) is reported separately from the
end-to-end time, which includes waiting and target preparation.

The scheduler (``ContinuousBatcher``) only talks to an executor; ``GpuExecutor``
drives librq, and tests drive the same scheduler with a simulated executor.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the start of the run
    op: str                        # "f", "grad" or "hvp"
    k: int
    payload: object = None         # executor-specific description
    # filled by the scheduler
    chunks: List[tuple] = field(default_factory=list)
    next_chunk: int = 0
    footprint: int = 0
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    result: Optional[dict] = None
    state: dict = field(default_factory=dict)


class ContinuousBatcher:
    def __init__(self, executor, hbm_budget: int, max_active: int = 8,
                 clock: Callable[[], float] = time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.clock = clock
        self.sleep = sleep
        self.used = 0
        self.peak_used = 0
        self.log: List[tuple] = []

    def run(self, requests: List[Request]) -> List[Request]:
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        active: List[Request] = []
        done: List[Request] = []
        t0 = self.clock()
        while pending or active:
            now = self.clock() - t0
            # admission (FIFO)
            while pending and pending[0].arrival <= now and len(active) < self.max_active:
                req = pending[0]
                fp = self.ex.footprint(req)
                if fp > self.budget:
                    raise ValueError(f"request {req.rid} needs {fp} bytes > budget {self.budget}")
                if self.used + fp > self.budget:
                    break
                pending.pop(0)
                req.footprint = fp
                self.used += fp
                self.peak_used = max(self.peak_used, self.used)
                req.t_admit = now
                req.chunks = self.ex.admit(req)
                req.next_chunk = 0
                active.append(req)
                self.log.append(("admit", req.rid, now, self.used))
            # issue the next chunk of every request whose stream is idle
            issued = False
            for req in active:
                if req.next_chunk < len(req.chunks) and self.ex.idle(req):
                    self.ex.issue(req, req.chunks[req.next_chunk], first=req.next_chunk == 0)
                    req.next_chunk += 1
                    issued = True
            # completions
            for req in list(active):
                if req.next_chunk == len(req.chunks) and self.ex.idle(req):
                    req.result = self.ex.finish(req)
                    req.t_done = self.clock() - t0
                    self.used -= req.footprint
                    active.remove(req)
                    done.append(req)
                    self.log.append(("done", req.rid, req.t_done, self.used))
            if not issued:
                if not active and pending:
                    wait = pending[0].arrival - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(min(wait, 0.01))
                else:
                    self.ex.wait_any(active)
        return done


def latency_stats(done: List[Request]) -> dict:
    out = {}
    for op in sorted({r.op for r in done}) + ["all"]:
        rs = [r for r in done if op == "all" or r.op == op]
        if not rs:
            continue
        e2e = np.array([r.t_done - r.arrival for r in rs]) * 1e3
        ev = np.array([r.t_done - r.t_admit for r in rs]) * 1e3
        out[op] = dict(n=len(rs), p50_ms=float(np.percentile(e2e, 50)),
                       p99_ms=float(np.percentile(e2e, 99)),
                       eval_p50_ms=float(np.percentile(ev, 50)),
                       eval_p99_ms=float(np.percentile(ev, 99)))
    return out


# ---------------------------------------------------------------------------
# GPU executor (librq)
# ---------------------------------------------------------------------------

@dataclass
class GpuPayload:
    circuit: object                # rq.Circuit
    gates: np.ndarray
    direction: Optional[np.ndarray]
    # (state) -> rq.Target on the device, called at admission on the
    # request's stream; whatever device memory its enqueued work still uses
    # (e.g. an apply workspace) is kept in the request's state dict
    make_target: Callable
    target_bytes: int


class GpuExecutor:
    """Runs requests on one GPU with librq; one HIP stream per active request
    (all at the default priority)."""

    OPS = {"f": 0, "grad": 1, "hvp": 2}

    def __init__(self, dtype: int, chunk: int = 4096, workspace_cap: int = 8 << 30):
        import torch

        from . import rq
        self.torch = torch
        self.rq = rq
        self.dtype = dtype
        self.chunk = chunk
        self.workspace_cap = workspace_cap

    def _chunk_cols(self, req):
        c = req.payload.circuit
        top = min(self.chunk, max(64, 1 << c.kq))
        return min(top, self.rq.default_chunk(c, self.OPS[req.op], self.dtype, c.ncols,
                                              budget_bytes=self.workspace_cap))

    def footprint(self, req) -> int:
        rq = self.rq
        c = req.payload.circuit
        ws = rq.lib().rq_workspace_bytes(rq.C.byref(c._c), self.OPS[req.op], self.dtype,
                                         self._chunk_cols(req))
        return int(req.payload.target_bytes + ws + 256 + 5 * c.n_params * 256)

    def admit(self, req):
        torch, rq = self.torch, self.rq
        pl = req.payload
        st = req.state
        st["stream"] = torch.cuda.Stream()
        with torch.cuda.stream(st["stream"]):
            st["target"] = pl.make_target(st)
            c = pl.circuit
            ws = rq.lib().rq_workspace_bytes(rq.C.byref(c._c), self.OPS[req.op], self.dtype,
                                             self._chunk_cols(req))
            st["ws"] = rq.Workspace(ws)
            n = {"f": 1, "grad": 3, "hvp": 5}[req.op]
            st["out"] = [torch.zeros((1,), dtype=torch.float64, device="cuda")] + \
                [torch.zeros((c.n_params, 4, 4, 2), dtype=torch.float64, device="cuda")
                 for _ in range(n - 1)]
        st["event"] = None
        cols = c.ncols
        chunk = self._chunk_cols(req)
        chunks = []
        sectors = (0, 1) if c.parity else (-1,)
        for s in sectors:
            for b in range(0, cols, chunk):
                chunks.append((s, b, min(chunk, cols - b)))
        return chunks

    def idle(self, req) -> bool:
        ev = req.state.get("event")
        return ev is None or ev.query()

    def issue(self, req, chunk, first=False):
        torch, rq = self.torch, self.rq
        st = req.state
        pl = req.payload
        s = st["stream"]
        kw = dict(range=chunk, chunk=self._chunk_cols(req), workspace=st["ws"], stream=s,
                  out=st["out"], accumulate=True)
        with torch.cuda.stream(s):
            if req.op == "f":
                rq.rq_cost(pl.circuit, st["target"], pl.gates, **{**kw, "out": st["out"][0]})
            elif req.op == "grad":
                rq.rq_grad(pl.circuit, st["target"], pl.gates, **kw)
            else:
                rq.rq_hvp(pl.circuit, st["target"], pl.gates, pl.direction, **kw)
            ev = torch.cuda.Event()
            ev.record(s)
        st["event"] = ev

    def wait_any(self, active, poll_s: float = 1e-4):
        """Return at once if any active request's stream is idle, else after
        a short sleep: the loop then polls again, admits arrivals and feeds
        whichever stream went idle first (blocking on one request's event
        would hold up the others and every new arrival)."""
        for req in active:
            ev = req.state.get("event")
            if ev is None or ev.query():
                return
        time.sleep(poll_s)

    def finish(self, req) -> dict:
        st = req.state
        outs = [o.cpu().numpy() for o in st["out"]]
        names = ["f", "egrad", "rgrad", "ehvp", "rhvp"]
        res = {"f": float(outs[0][0])}
        for n, o in zip(names[1:], outs[1:]):
            res[n] = o[..., 0] + 1j * o[..., 1]
        for key in ("target", "ws", "apply_ws", "out", "event", "stream"):
            st.pop(key, None)
        return res


def make_gpu_request(req_desc: dict, dtype: int, trotter_steps: int = 20,
                     parity: bool = False, dense_max_k: int = 12) -> Request:
    """Request from a configuration-5 descriptor: Hubbard target of k qubits,
    brick wall of the given depth with Haar gates.  Targets are dense
    exp(-iHt) for k <= dense_max_k (uploaded) and a Strang Trotter circuit
    applied on the device for larger k, with an apply workspace of the
    request's own (concurrent target builds never share gate coefficients)."""
    import workloads as w

    from . import rq
    prob = w.configs.request_problem(req_desc, trotter_steps=trotter_steps,
                                     dense_max_k=dense_max_k)
    k = prob.k
    circ = rq.Circuit(k, prob.pairs, param_of=prob.param_of)
    esize = 16 if dtype == rq.RQ_C128 else 8
    tbytes = esize * (1 << (2 * k))

    if prob.U_ref is not None:
        U = prob.U_ref

        def make_target(state):
            return rq.Target.from_dense(U, dtype)
    else:
        gl = prob.trotter

        def make_target(state):
            state["apply_ws"] = rq.apply_workspace(k, gl, dtype)
            return rq.build_trotter_target(k, gl, dtype=dtype, parity=False,
                                           workspace=state["apply_ws"])

    pl = GpuPayload(circ, prob.gates, prob.direction if req_desc["op"] == "hvp" else None,
                    make_target, tbytes)
    return Request(rid=req_desc["rid"], arrival=req_desc["arrival"], op=req_desc["op"], k=k,
                   payload=pl)
