#!/usr/bin/env python3
"""Throughput of the matrix-free f + gradient + HVP hot path on one MI355X.

Workload (default): 16 qubits = 8-site spinful Fermi-Hubbard ring (J=1, U=4,
interleaved spins), target U = Strang Trotter circuit (200 steps, t = 1.0)
built on the GPU with rq_apply_circuit; 7-layer brick wall with one shared
parity-conserving gate per layer (56 instances, 7 parameters); the trace runs
over both parity sectors (2 x 2^15 basis states, sector-compressed states).
One step = one evaluation: f, Riemannian gradient of all gates and one
Hessian-vector product along a seeded tangent direction, summed over all
2^16 basis states, target columns resident in HBM.

Prints one JSON line: the throughput (evaluations per second) and its
per-kernel breakdown, the roofline of the dominant kernel (algorithmic HBM
bytes or flops per launch over its HIP-event time, against the MI355X peaks),
the complex128 run and the c64 error against it, further workloads (Hessian
blocks, configuration 4, orbit-reduced and sampled traces, trust-region
iterations, the serving mix) and the oracle's CPU rate on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0           # MI355X HBM3E, GB/s
PEAK_VALU_TFLOPS = 78.6         # 256 CU x 64 lanes x FMA x 2.4 GHz (FP32 unpacked = FP64)

METRIC = "f+grad+HVP evals/s at n=16 (FP32 vs FP64 states), HBM GB/s, p50/p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_run(rq, torch, circ, target, prob, steps, warmup, chunk, basis_range=None):
    ws_need = rq.lib().rq_workspace_bytes(rq.C.byref(circ._c), rq.RQ_OP_HVP, target.dtype, chunk)
    ws = rq.Workspace(ws_need)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        rq.rq_hvp(circ, target, prob.gates, prob.direction, range=basis_range, chunk=chunk,
                  workspace=ws)
    torch.cuda.synchronize()
    rq.rq_profile_read()                     # drop anything recorded so far
    rq.rq_profile_enable(True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for i in range(steps):
        evs[i][0].record(stream)
        out = rq.rq_hvp(circ, target, prob.gates, prob.direction, range=basis_range, chunk=chunk,
                        workspace=ws)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rq.rq_profile_enable(False)
    prof = rq.rq_profile_read()
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    res = [x.detach().cpu().numpy() for x in out]
    del ws
    return dict(seconds=t1 - t0, lat_ms=lat, prof=prof, result=res, ws_bytes=ws_need)


def copy_bandwidth(torch, rq, nbytes=4 << 30, reps=10):
    """Read+write rate of a plain device copy of nbytes: librq's hand-written
    streaming copy kernel (rq_stream_copy) over a few grid shapes, best of
    them, and torch's copy for comparison -- the practical HBM rate for
    streaming kernels on this GPU, reported next to the 8 TB/s datasheet
    peak.  Returns (best rate of the own kernel, its shape, torch's rate)."""
    x = torch.empty(nbytes // 8, dtype=torch.complex64, device="cuda")
    x.real.fill_(1.0)
    y = torch.empty_like(x)

    def rate(fn):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return 2 * nbytes / (e0.elapsed_time(e1) / reps / 1e3) / 1e9

    best, shape = 0.0, None
    for unroll in (1, 4, 8):
        for blocks in (1024, 4096, 16384):
            r = rate(lambda: rq.rq_stream_copy(y, x, unroll, blocks))
            if r > best:
                best, shape = r, dict(unroll=unroll, blocks=blocks)
    torch_rate = rate(lambda: y.copy_(x))
    del x, y
    torch.cuda.empty_cache()
    return round(best, 1), shape, round(torch_rate, 1)


def _pcts(lat_ms):
    """Per-evaluation latency percentiles (HIP events around each step)."""
    return {f"p{q}": round(float(np.percentile(lat_ms, q)), 3) for q in (10, 50, 90, 99)}


def _kernel_name(key):
    names = {("hess", "sweep"): "k_hess_pass", ("hess", "states"): "k_pass (per-gate states)"}
    return names.get(key, f"k_pass {key[0]}/{key[1]}")


def roofline(prof, key):
    st = prof[key]
    n = st["launches"]
    avg_s = st["ms"] / n / 1e3
    by = st["bytes"] / n
    fl = st["flops"] / n
    gbs = by / avg_s / 1e9
    tfl = fl / avg_s / 1e12
    hbm_frac = gbs / PEAK_HBM_GBS
    alu_frac = tfl / PEAK_VALU_TFLOPS
    if hbm_frac >= alu_frac:
        return dict(bound="hbm", achieved=round(gbs, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(hbm_frac, 4), traffic=None,
                    kernel=_kernel_name(key), avg_launch_ms=round(avg_s * 1e3, 4),
                    alu=dict(achieved=round(tfl, 2), peak=PEAK_VALU_TFLOPS, unit="TFLOP/s",
                             frac=round(alu_frac, 4)))
    return dict(bound="alu", achieved=round(tfl, 2), peak=PEAK_VALU_TFLOPS, unit="TFLOP/s",
                frac=round(alu_frac, 4), traffic=None,
                kernel=_kernel_name(key), avg_launch_ms=round(avg_s * 1e3, 4),
                hbm=dict(achieved=round(gbs, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                         frac=round(hbm_frac, 4)))


def code_hash(path):
    """sha256[:16] of a source file's code with comments and whitespace
    removed, so that edits of comments keep a stored measurement valid."""
    import hashlib
    import re
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    txt = re.sub(r"//[^\n]*", "", txt)
    txt = re.sub(r"\s+", "", txt)
    return hashlib.sha256(txt.encode()).hexdigest()[:16]


# committed rocprofv3 counter summaries: (profile file, kernel source whose
# code hash keys the measurement)
TRAFFIC_PROFILES = {
    "sweep": ("k_pass_hvp_cfg3_c64.txt", "rq_sweep.h"),
    "hess": ("k_hess_pass_cfg3_cfg4.txt", "rq_hess.hip"),
    "cfg4": ("k_pass_hvp_cfg4_c64.txt", "rq_sweep.h"),
}


def measured_traffic(kernel_key, which="sweep"):
    """HBM bytes per launch of a kernel from a committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE runs, calibrated on a copy kernel), or
    None when the kernel code changed since it was taken."""
    pname, sname = TRAFFIC_PROFILES[which]
    prof = os.path.join(ROOT, "profiles", pname)
    src = os.path.join(ROOT, "paper_2506_23775_amd", "csrc", sname)
    if not (os.path.exists(prof) and os.path.exists(src)):
        return None
    sha = code_hash(src)
    import re
    vals = {}
    for line in open(prof):
        m = re.match(r"(traffic_bytes_per_launch\[[^\]]+\]|code_sha256_16):\s*(\S+)", line)
        if m:
            vals[m.group(1)] = m.group(2)
    if vals.get("code_sha256_16") != sha:
        return None
    v = vals.get(f"traffic_bytes_per_launch[{kernel_key}]")
    return float(v) if v else None


def _oracle_batch(args):
    """One batch of the CPU baseline (runs in a worker process): the oracle's
    f, Euclidean gradient T and HVP tangent Tdot summed over the given basis
    columns, with target columns drawn from a seeded generator."""
    k, pairs, inst, Z, cols, seed = args
    import oracle as O
    rng = np.random.default_rng(seed)
    E = rng.standard_normal((1 << k, len(cols))) + 1j * rng.standard_normal((1 << k, len(cols)))
    E /= np.linalg.norm(E, axis=0)
    t0 = time.perf_counter()
    O.tangent_T(k, pairs, inst, Z, E, cols)
    O.cost(k, pairs, inst, E, cols)
    return time.perf_counter() - t0


def cpu_baseline(prob, ncols=512, batch=16):
    """The FP64 oracle timed on the host on a bounded sample: f, gradient and
    HVP contributions (oracle.tangent_T + oracle.cost, dense numpy on full
    2^k-row states -- the oracle has no sector-compressed path) of `ncols`
    basis states of parity sector 0, in batches of `batch` columns spread
    over one single-threaded worker process per host core (at most 16), and
    extrapolated to the full 2^k-term trace: every summand costs the same.
    The target columns of the sample are seeded random unit vectors (the
    oracle's work does not depend on their values; U|j> of the Strang
    target would cost thousands of gate applications per column to build)."""
    import concurrent.futures as cf
    import multiprocessing as mp

    import oracle as O
    k = prob.k
    cols = O.sector_columns(k, 0)[:ncols]
    inst = prob.gates[prob.param_of]
    Z = prob.direction[prob.param_of]
    cores = len(os.sched_getaffinity(0))
    workers = max(1, min(16, cores))
    tasks = [(k, prob.pairs, inst, Z, cols[b:b + batch], [w_seed, b])
             for w_seed in (250623775,) for b in range(0, len(cols), batch)]
    env = {v: os.environ.get(v) for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                          "MKL_NUM_THREADS")}
    for v in env:
        os.environ[v] = "1"               # one thread per worker (inherited at spawn)
    try:
        t0 = time.perf_counter()
        with cf.ProcessPoolExecutor(max_workers=workers,
                                    mp_context=mp.get_context("spawn")) as ex:
            busy = sum(ex.map(_oracle_batch, tasks))
        wall = time.perf_counter() - t0
    finally:
        for v, val in env.items():
            if val is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = val
    rate_cols = len(cols) / wall                     # columns per second, all workers
    return dict(value=rate_cols / (1 << k), unit="evals/s", cores=workers, kind="oracle",
                sample=f"{len(cols)} basis states of parity sector 0 (general-mode 2^{k}-row "
                       f"states), {len(tasks)} batches of {batch} over {workers} single-threaded "
                       f"workers: {wall:.1f} s wall ({busy:.1f} s of worker time), "
                       f"extrapolated x{(1 << k) / len(cols):.0f} to the 2^{k}-state trace",
                seconds_per_column=round(busy / len(cols), 4))


def config4_hessian(rq, torch, circ, target, prob, ncols, chunk=1024):
    """Configuration 4's Hessian step: all 72 x 72 blocks of 16 x 16 complex
    entries (1152 x 1152 real Riemannian Hessian, c64 states + FP64
    accumulation) summed over `ncols` basis states (all 2^16 for the full
    step, else the first ncols, timed and extrapolated: every basis state
    costs the same), then one FP64 trust-region step (truncated CG + polar
    retraction, rq_tr_step) on the resulting gradient and Hessian."""
    full = 1 << prob.k
    ncols = min(int(ncols), full)
    rq.rq_hess_blocks(circ, target, prob.gates, range=(-1, 0, 64), chunk=64)    # warm-up
    P = prob.n_params
    outs = [torch.zeros(shape, dtype=torch.float64, device="cuda")
            for shape in ((1,), (P, 4, 4, 2), (P, 4, 4, 2))] + \
        [None, torch.zeros((16 * P, 16 * P), dtype=torch.float64, device="cuda")]
    torch.cuda.synchronize()
    rq.rq_profile_read()
    rq.rq_profile_enable(True)
    # the basis states in ranges of `part` columns, each added into the same
    # outputs (RQ_EXEC_ACCUMULATE; every output is linear in the basis sum),
    # so that progress is reported between them
    part = min(ncols, 8192)
    t0 = time.perf_counter()
    for b in range(0, ncols, part):
        rq.rq_hess_blocks(circ, target, prob.gates, range=(-1, b, min(part, ncols - b)),
                          chunk=chunk, out=outs, accumulate=True)
        torch.cuda.synchronize()
        log(f"[bench] configuration-4 Hessian: basis states [{b}, {b + part}) done, "
            f"{time.perf_counter() - t0:.1f} s")
    dt = time.perf_counter() - t0
    f, eg, hr = outs[0], torch.view_as_complex(outs[1]), outs[4]
    rq.rq_profile_enable(False)
    prof = rq.rq_profile_read()
    H = hr.cpu().numpy()
    g = rq.rq_tangent_coords(prob.gates, eg.cpu().numpy())
    delta = float(np.sqrt(H.shape[0]) * np.pi / 8)
    t1 = time.perf_counter()
    eta, cand, md, stop = rq.rq_tr_step(prob.gates, g, H, delta)
    dt_tr = time.perf_counter() - t1
    hdom = ("hess", "sweep")
    return {
        "workload": "cfg4 Hessian step: 72 x 72 instance blocks (1152 x 1152 real Riemannian "
                    "Hessian) over basis states [0, ncols) of 2^16, c64 states + FP64 "
                    "accumulation, chunk 1024; then one FP64 trust-region step",
        "ncols": ncols, "seconds": round(dt, 3),
        "seconds_full_trace": round(dt * full / ncols, 1),
        "extrapolated": ncols != full,
        "kernels": {f"{k[0]}/{k[1]}": dict(ms=round(v["ms"], 1), launches=v["launches"],
                                           GBps=round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1),
                                           TFLOPs=round(v["flops"] / (v["ms"] / 1e3) / 1e12, 2))
                    for k, v in prof.items()},
        "roofline": dict(roofline(prof, hdom),
                         traffic=measured_traffic("cfg4:hess/sweep", "hess")),
        "symmetric_rel": float(f"{np.abs(H - H.T).max() / np.abs(H).max():.2e}"),
        "tr_step": {"seconds": round(dt_tr, 3), "delta": round(delta, 4),
                    "grad_norm": float(f"{np.linalg.norm(g):.6e}"),
                    "step_norm": float(f"{np.linalg.norm(eta):.6e}"),
                    "model_decrease": float(f"{md:.6e}"), "tcg_stop": int(stop)}}


def _serve(rq, descs, dtype=None, chunk=4096, max_active=8):
    """Run a list of configuration-5 request descriptors through the
    continuous-batching loop; returns (finished requests, batcher, seconds)."""
    import torch

    from paper_2506_23775_amd import serving
    dtype = rq.RQ_C64 if dtype is None else dtype
    reqs = [serving.make_gpu_request(d, dtype) for d in descs]
    batcher = serving.ContinuousBatcher(serving.GpuExecutor(dtype, chunk=chunk),
                                        hbm_budget=96 << 30, max_active=max_active)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = batcher.run(reqs)
    torch.cuda.synchronize()
    return done, batcher, time.perf_counter() - t0


def _latency(done):
    from paper_2506_23775_amd import serving
    lat = {op: {k: (round(v, 2) if isinstance(v, float) else v) for k, v in st.items()}
           for op, st in serving.latency_stats(done).items()}
    by_k = {}
    for k in sorted({r.k for r in done}):
        e2e = np.array([r.t_done - r.arrival for r in done if r.k == k]) * 1e3
        by_k[str(k)] = dict(n=int(e2e.size), p50_ms=round(float(np.percentile(e2e, 50)), 2),
                            p99_ms=round(float(np.percentile(e2e, 99)), 2))
    return lat, by_k


def _rel_errors(res, ref):
    """|df| / max(1, |f|) and relative Frobenius errors of the arrays."""
    out = {"f_rel": float(f"{abs(res['f'] - ref['f']) / max(1.0, abs(ref['f'])):.3e}")}
    for key in ("egrad", "rgrad", "ehvp", "rhvp"):
        if key in res and key in ref:
            nb = np.linalg.norm(ref[key])
            out[key + "_rel"] = float(f"{np.linalg.norm(res[key] - ref[key]) / (nb or 1.0):.3e}")
    return out


def serving_errors(rq, done, descs, n_sample=4):
    """Error of served (c64, in the mix) results against the FP64 path on a
    sample of the requests: each sampled request is served again alone in
    complex128 (the path the oracle checks in the GPU tests, where the
    served results are also compared with the oracle directly).  The sample
    takes requests of the smallest and the largest qubit counts."""
    by_rid = {r.rid: r for r in done}
    order = sorted(descs, key=lambda d: (d["k"], d["rid"]))
    sample = order[:n_sample // 2] + order[len(order) - (n_sample - n_sample // 2):]
    out = []
    for d in sample:
        alone, _, _ = _serve(rq, [{**d, "arrival": 0.0}], dtype=rq.RQ_C128, max_active=1)
        out.append(dict(rid=d["rid"], k=d["k"], op=d["op"], reference="c128 GPU path, alone",
                        **_rel_errors(by_rid[d["rid"]].result, alone[0].result)))
    return out


def serving_run(rq, n_requests, rate_hz, saturate_requests=32, saturate_rate=1000.0):
    """Configuration 5: Poisson streams of f / f+grad / f+grad+HVP requests
    of mixed size (k = 8..16, depth 3..9), served by the continuous-batching
    loop in complex64 with FP64 accumulation.  Two runs: `n_requests` at
    `rate_hz` (open loop, latency under light load) and `saturate_requests`
    at an arrival rate far above the service rate (all requests queued at
    once: the throughput is the loop's capacity).  Latency = completion -
    arrival (end to end, includes the request's target preparation on the
    device) and completion - admission (evaluation only), per request type
    and per qubit count.  Sampled results are compared with FP64 references."""
    from paper_2506_23775_amd import serving

    import workloads as w
    warm = serving.make_gpu_request(dict(rid=10**6, arrival=0.0, k=8, depth=3, U=4.0, t=0.5,
                                         op="hvp"), rq.RQ_C64)
    serving.ContinuousBatcher(serving.GpuExecutor(rq.RQ_C64), hbm_budget=1 << 30).run([warm])
    res = {"workload": "cfg5: Poisson arrivals of f / f+grad / f+grad+HVP requests, "
                       "k in {8..16}, brick-wall depth in {3,5,7,9}, Hubbard targets "
                       "(dense exp(-iHt) for k <= 12, 20-step Strang Trotter on the device "
                       "beyond), c64 states + FP64 accumulation"}
    for name, n, rate in (("open_loop", n_requests, rate_hz),
                          ("saturated", saturate_requests, saturate_rate)):
        if n <= 0:
            continue
        descs = w.configs.serving_requests(n, rate)
        done, batcher, dt = _serve(rq, descs)
        lat, by_k = _latency(done)
        ks = {}
        for d in descs:
            ks[str(d["k"])] = ks.get(str(d["k"]), 0) + 1
        res[name] = dict(requests=len(done), rate_hz=rate, seconds=round(dt, 3),
                         throughput_req_per_s=round(len(done) / dt, 3), k_mix=ks,
                         peak_hbm_GiB=round(batcher.peak_used / 2**30, 2), latency_ms=lat,
                         latency_ms_by_k=by_k)
        if name == "saturated":
            res["error_vs_fp64"] = serving_errors(rq, done, descs)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--chunk", type=int, default=4096)
    ap.add_argument("--chunk128", type=int, default=4096)
    ap.add_argument("--trotter-steps", type=int, default=200)
    ap.add_argument("--no-c128", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sampled-vectors", type=int, default=256,
                    help="random vectors per parity sector in the sampled-trace leg (0: skip)")
    ap.add_argument("--config4", type=int, default=2,
                    help="timed evaluations of configuration 4 (dense gates; 0: skip)")
    ap.add_argument("--config4-hessian-cols", type=int, default=4096,
                    help="basis states of the timed configuration-4 Hessian + trust-region "
                         "step (65536: the full trace; 0: skip)")
    ap.add_argument("--orbits", type=int, default=1,
                    help="1: time the translation-orbit-reduced evaluation (0: skip)")
    ap.add_argument("--hessian", type=int, default=1,
                    help="1: time the configuration-3 Hessian blocks (0: skip)")
    ap.add_argument("--hessian-c128", type=int, default=1,
                    help="1: also the configuration-3 Hessian with complex128 states (0: skip)")
    ap.add_argument("--hessian-number", type=int, default=1,
                    help="1: also the Hessian with particle-number-conserving gates (0: skip)")
    ap.add_argument("--tr-iters", type=int, default=5,
                    help="trust-region iterations in the configuration-2 leg (0: skip)")
    ap.add_argument("--serving-requests", type=int, default=16,
                    help="requests of the open-loop configuration-5 serving run (0: skip it)")
    ap.add_argument("--serving-rate", type=float, default=1.0, help="Poisson arrival rate, 1/s")
    ap.add_argument("--serving-saturate", type=int, default=32,
                    help="requests of the saturated serving run (arrival rate 1000/s; 0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 2 GiB device copy first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on exactly one GPU (asked for {args.gpus}); sharding the basis "
              "sum over several GPUs is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as w
    from paper_2506_23775_amd import rq

    rq.lib()
    torch.cuda.set_device(0)
    if args.copy_calibration:
        x = torch.ones(1 << 28, dtype=torch.complex64, device="cuda")   # 2 GiB
        y = x.clone()
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {x.numel() * 8} bytes read and written")
        del x, y
    prob = w.make_problem(3, trotter_steps=args.trotter_steps)
    circ = rq.Circuit(prob.k, prob.pairs, param_of=prob.param_of, parity=True)
    log(f"[bench] building target: {len(prob.trotter)} Trotter gates on 2 x 2^15 columns")
    t0 = time.perf_counter()
    tgt128 = rq.build_trotter_target(prob.k, prob.trotter, dtype=rq.RQ_C128, parity=True)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"[bench] target built in {setup_s:.1f} s")
    tgt64 = rq.Target(tgt128.ref.to(torch.complex64), rq.RQ_C64, True)
    if args.no_c128:
        tgt128 = None
        torch.cuda.empty_cache()

    log("[bench] c64 timed run")
    r64 = gpu_run(rq, torch, circ, tgt64, prob, args.steps, args.warmup, args.chunk)
    ms64 = r64["seconds"] / args.steps * 1e3
    log(f"[bench] c64: {ms64:.1f} ms/eval")
    out = {"metric": METRIC, "value": round(args.steps / r64["seconds"], 4), "unit": "evals/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms64, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
           "data": "synthetic (seeded Haar parity gates, Trotter target built on device)",
           "config": {"workload": "cfg3: k=16 spinful Fermi-Hubbard ring (8 sites, J=1, U=4, "
                                  "t=1), Strang-200 target, 7-layer brick wall, 7 shared "
                                  "parity gates (56 instances), 2 x 2^15 parity sectors, "
                                  "c64 states + FP64 accumulation",
                      "k": prob.k, "layers": prob.n_layers, "gates": prob.n_gates,
                      "params": prob.n_params, "basis_states": 1 << prob.k,
                      "chunk": args.chunk, "target_setup_s": round(setup_s, 2)}}
    out["latency_ms"] = _pcts(r64["lat_ms"])
    kern = {f"{k[0]}/{k[1]}": dict(ms=round(v["ms"], 3), launches=v["launches"],
                                   GBps=round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1),
                                   TFLOPs=round(v["flops"] / (v["ms"] / 1e3) / 1e12, 2))
            for k, v in r64["prof"].items()}
    out["kernels_c64"] = kern
    tot_bytes = sum(v["bytes"] for v in r64["prof"].values())
    out["hbm_GBps_algorithmic"] = round(tot_bytes / r64["seconds"] / 1e9, 1)
    dom = max(r64["prof"].items(), key=lambda kv: kv[1]["ms"])[0]
    out["roofline"] = roofline(r64["prof"], dom)
    if args.chunk == 4096:
        out["roofline"]["traffic"] = measured_traffic(f"{dom[0]}/{dom[1]}")
    cref, cshape, ctorch = copy_bandwidth(torch, rq)
    out["roofline"]["copy_ref_GBps"] = cref
    out["roofline"]["copy_ref"] = dict(kernel="rq_stream_copy (4 GiB, read + write)", **cshape)
    out["roofline"]["copy_torch_GBps"] = ctorch

    if args.hessian:
        # all pairwise Hessian blocks of configuration 3 over the full trace,
        # with the two-site translation symmetry of the brick wall and the
        # Strang target (only translation-unique hole pairs swept)
        log("[bench] Hessian leg: configuration 3, shift 4")
        c3s = rq.Circuit(prob.k, prob.pairs, param_of=prob.param_of, parity=True, shift=4)
        torch.cuda.synchronize()
        rq.rq_profile_read()
        rq.rq_profile_enable(True)
        t0 = time.perf_counter()
        hres = rq.rq_hess_blocks(c3s, tgt64, prob.gates, chunk=1024)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rq.rq_profile_enable(False)
        hprof = rq.rq_profile_read()
        hr = hres[4].cpu().numpy()
        hdom = max(hprof.items(), key=lambda kv: kv[1]["ms"])[0]
        out["hessian"] = {
            "workload": "cfg3 Hessian: 56 x 56 instance blocks (7 x 7 parameter blocks of 8 x 8 "
                        "complex entries, 56 x 56 real Riemannian Hessian) over 2 x 2^15 basis "
                        "states, c64 + FP64 accumulation, translation-unique hole pairs (shift 4)",
            "seconds": round(dt, 3),
            "kernels": {f"{k[0]}/{k[1]}": dict(ms=round(v["ms"], 1), launches=v["launches"],
                                               GBps=round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1),
                                               TFLOPs=round(v["flops"] / (v["ms"] / 1e3) / 1e12, 2))
                        for k, v in hprof.items()},
            "roofline": roofline(hprof, hdom),
            "symmetric_rel": float(f"{np.abs(hr - hr.T).max() / np.abs(hr).max():.2e}")}
        out["hessian"]["roofline"]["traffic"] = measured_traffic("cfg3:hess/sweep", "hess")
        log(f"[bench] Hessian: {dt:.2f} s")
        if args.hessian_c128 and tgt128 is not None:
            # the same Hessian with complex128 states (the paper's precision),
            # and the complex64 Hessian's deviation from it
            log("[bench] Hessian leg: configuration 3, complex128")
            rq.release_workspaces()
            torch.cuda.synchronize()
            rq.rq_profile_read()
            rq.rq_profile_enable(True)
            t0 = time.perf_counter()
            h128 = rq.rq_hess_blocks(c3s, tgt128, prob.gates, chunk=1024)
            torch.cuda.synchronize()
            dt128 = time.perf_counter() - t0
            rq.rq_profile_enable(False)
            hprof128 = rq.rq_profile_read()
            hr128 = h128[4].cpu().numpy()
            hh64, hh128 = hres[3].cpu().numpy(), h128[3].cpu().numpy()
            out["hessian_c128"] = {
                "workload": "the cfg3 Hessian leg with complex128 states (FP64 throughout)",
                "seconds": round(dt128, 3),
                "sweep_ms": round(hprof128[("hess", "sweep")]["ms"], 1),
                "sweep_launches": hprof128[("hess", "sweep")]["launches"],
                "roofline": dict(roofline(hprof128, ("hess", "sweep")),
                                 traffic=measured_traffic("cfg3c128:hess/sweep", "hess")),
                "c64_rel_error": {
                    "hess_real": float(f"{np.linalg.norm(hr - hr128) / np.linalg.norm(hr128):.3e}"),
                    "hess_holo": float(f"{np.linalg.norm(hh64 - hh128) / np.linalg.norm(hh128):.3e}")}}
            del h128
            rq.release_workspaces()
            torch.cuda.empty_cache()
            log(f"[bench] Hessian (c128): {dt128:.2f} s")
    if args.hessian and args.hessian_number:
        # the same Hessian with particle-number-conserving gates (6 hole
        # slices instead of 8)
        c3n = rq.Circuit(prob.k, prob.pairs, param_of=prob.param_of, number=True, shift=4)
        gn = w.number_haar_gates(np.random.default_rng([w.configs.SEED, 3, 300]), prob.n_params)
        torch.cuda.synchronize()
        rq.rq_profile_read()
        rq.rq_profile_enable(True)
        t0 = time.perf_counter()
        rq.rq_hess_blocks(c3n, tgt64, gn, chunk=1024)
        torch.cuda.synchronize()
        dtn = time.perf_counter() - t0
        rq.rq_profile_enable(False)
        nprof = rq.rq_profile_read()
        out["hessian_number_gates"] = {
            "workload": "cfg3 circuit with particle-number-conserving gates (U(1) x U(2) x U(1), "
                        "6 x 6 blocks, 6 hole slices), same target and symmetry",
            "seconds": round(dtn, 3),
            "sweep_ms": round(nprof[("hess", "sweep")]["ms"], 1),
            "sweep_launches": nprof[("hess", "sweep")]["launches"],
            "roofline": dict(roofline(nprof, ("hess", "sweep")),
                             traffic=measured_traffic("cfg3num:hess/sweep", "hess")),
            "speedup_vs_parity_gates": round(out["hessian"]["seconds"] / dtn, 3)}
        log(f"[bench] Hessian (number gates): {dtn:.2f} s")

    if args.config4:
        # configuration 4: k = 16 general mode, 9-layer brick wall of 72
        # independent Haar U(4) gates, the same Strang target without parity
        # compression (2^16 x 2^16 columns, c64)
        log("[bench] configuration 4 (dense gates): building the general-mode target")
        p4 = w.make_problem(4, trotter_steps=args.trotter_steps)
        c4 = rq.Circuit(p4.k, p4.pairs, param_of=p4.param_of)
        t4 = rq.build_trotter_target(p4.k, p4.trotter, dtype=rq.RQ_C64, parity=False)
        r4 = gpu_run(rq, torch, c4, t4, p4, args.config4, 1, min(args.chunk, 2048))
        dom4 = max(r4["prof"].items(), key=lambda kv: kv[1]["ms"])[0]
        out["config4"] = {
            "workload": "cfg4: k=16, 9-layer brick wall, 72 independent Haar U(4) gates, "
                        "Strang-200 target, 2^16 basis states, c64 states + FP64 accumulation",
            "evals_per_s": round(args.config4 / r4["seconds"], 4),
            "ms_per_step": round(r4["seconds"] / args.config4 * 1e3, 2),
            "kernels": {f"{k[0]}/{k[1]}": dict(ms=round(v["ms"], 1), launches=v["launches"],
                                               GBps=round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1),
                                               TFLOPs=round(v["flops"] / (v["ms"] / 1e3) / 1e12, 2))
                        for k, v in r4["prof"].items()},
            "roofline": roofline(r4["prof"], dom4)}
        out["config4"]["roofline"]["traffic"] = measured_traffic(f"cfg4:{dom4[0]}/{dom4[1]}",
                                                                 "cfg4")
        log(f"[bench] configuration 4: {out['config4']['ms_per_step']} ms/eval")
        if args.config4_hessian_cols:
            out["config4_hessian"] = config4_hessian(rq, torch, c4, t4, p4,
                                                     args.config4_hessian_cols)
        del t4
        rq.release_workspaces()
        torch.cuda.empty_cache()

    if args.orbits:
        # extension beyond the paper: one basis state per translation orbit
        # (two-site shift of the brick wall and the Strang target), weighted
        # by the orbit size -- the same f, gradient and HVP as the full sum
        log("[bench] orbit-reduced trace (shift 4)")
        c3o = rq.Circuit(prob.k, prob.pairs, param_of=prob.param_of, parity=True, shift=4)
        tgt_o = rq.orbit_target(c3o, tgt64)
        Ro = tgt_o.ref.shape[-1]
        ro = gpu_run(rq, torch, c3o, tgt_o, prob, args.steps, args.warmup, args.chunk,
                     basis_range=(-1, 0, Ro))
        err = {}
        for n, a, b in zip(["f", "egrad", "rgrad", "ehvp", "rhvp"], ro["result"], r64["result"]):
            nb = np.linalg.norm(b)
            err[n] = float(f"{np.linalg.norm(a - b) / (nb if nb else 1.0):.3e}")
        out["orbit_reduced"] = {
            "workload": "cfg3 with one basis state per orbit of the two-site translation "
                        f"({Ro} columns per sector instead of 32768, orbit sizes as weights), c64",
            "evals_per_s": round(args.steps / ro["seconds"], 4),
            "ms_per_step": round(ro["seconds"] / args.steps * 1e3, 3),
            "speedup_vs_full_sum": round(r64["seconds"] / ro["seconds"], 3),
            "rel_diff_vs_full_sum": err}
        del tgt_o
        log(f"[bench] orbit-reduced: {ro['seconds'] / args.steps * 1e3:.1f} ms/eval")

    if args.sampled_vectors > 0:
        # trace over random vectors instead of the 2^16 basis states (same
        # kernels, input states given): time and error against the exact sum
        R = args.sampled_vectors
        log(f"[bench] sampled trace: {R} vectors per sector")
        tgt_s = rq.sampled_target(prob.k, R, np.random.default_rng([w.configs.SEED, 3, 200]),
                                  dtype=rq.RQ_C64, parity=True, gate_list=prob.trotter)
        rs = gpu_run(rq, torch, circ, tgt_s, prob, args.steps, args.warmup,
                     min(args.chunk, max(64, (R + 63) // 64 * 64)), basis_range=(-1, 0, R))
        names = ["f", "egrad", "rgrad", "ehvp", "rhvp"]
        err = {}
        for n, a, b in zip(names[1:], rs["result"][1:], r64["result"][1:]):
            nb = np.linalg.norm(b)
            err[n] = float(f"{np.linalg.norm(a / R - b) / (nb if nb else 1.0):.3e}")
        f_est = float(rs["result"][0]) / R
        f_ex = float(r64["result"][0])
        out["sampled_trace"] = {
            "vectors_per_sector": R, "kind": "complex Rademacher", "dtype": "c64",
            "evals_per_s": round(args.steps / rs["seconds"], 3),
            "ms_per_step": round(rs["seconds"] / args.steps * 1e3, 3),
            "f_exact": round(f_ex, 4), "f_estimate": round(f_est, 4),
            "f_abs_error_over_2k": float(f"{abs(f_est - f_ex) / (1 << prob.k):.3e}"),
            "rel_error_vs_exact_trace": err,
            "note": "estimator noise ~ ||U^dagger C - diag||_F / sqrt(vectors); large relative "
                    "to the exact values at random (far from converged) gates"}
        del tgt_s

    if tgt128 is not None:
        log("[bench] c128 timed run")
        r128 = gpu_run(rq, torch, circ, tgt128, prob, args.steps, args.warmup, args.chunk128)
        ms128 = r128["seconds"] / args.steps * 1e3
        err = {}
        names = ["f", "egrad", "rgrad", "ehvp", "rhvp"]
        for n, a, b in zip(names, r64["result"], r128["result"]):
            nb = np.linalg.norm(b)
            err[n] = float(np.linalg.norm(a - b) / (nb if nb else 1.0))
        err["f_abs_over_2k"] = float(abs(r64["result"][0] - r128["result"][0]) / (1 << prob.k))
        out["c128"] = {"value": round(args.steps / r128["seconds"], 4), "unit": "evals/s",
                       "ms_per_step": round(ms128, 3), "chunk": args.chunk128,
                       "latency_ms": _pcts(r128["lat_ms"])}
        out["fp32_speedup_vs_fp64"] = round(ms128 / ms64, 3)
        out["c64_rel_error_vs_c128"] = {k: float(f"{v:.3e}") for k, v in err.items()}
        dom128 = max(r128["prof"].items(), key=lambda kv: kv[1]["ms"])[0]
        out["roofline_c128"] = roofline(r128["prof"], dom128)
        if args.chunk128 == 4096:
            out["roofline_c128"]["traffic"] = measured_traffic(f"c128:{dom128[0]}/{dom128[1]}")

    if args.tr_iters > 0:
        # configuration 2 (k = 12, 30 gates): full Riemannian trust-region
        # iterations, each with the 480 x 480 Hessian from rq_hess_blocks
        log(f"[bench] trust-region leg: {args.tr_iters} iterations, configuration 2")
        p2 = w.make_problem(2)
        c2 = rq.Circuit(p2.k, p2.pairs, param_of=p2.param_of)
        t2 = rq.Target.from_dense(p2.U_ref, rq.RQ_C128)
        rq.rq_tr_solve(c2, t2, p2.gates, max_iter=1)            # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, hist = rq.rq_tr_solve(c2, t2, p2.gates, max_iter=args.tr_iters)
        dt = time.perf_counter() - t0
        evals = int(1 + hist[:-1, 4].sum()) if len(hist) else 0
        out["trust_region"] = {
            "workload": "cfg2: k=12 Fermi-Hubbard target exp(-iH/2), 5-layer brick wall, "
                        "30 Haar U(4) gates, 480 x 480 real Riemannian Hessian, c128",
            "iterations": int(len(hist)), "seconds": round(dt, 3),
            "ms_per_iteration": round(dt / max(1, len(hist)) * 1e3, 2),
            "hessian_evaluations": evals,
            "f": [round(float(v), 6) for v in hist[:, 0]],
            "grad_norm": [float(f"{v:.4e}") for v in hist[:, 1]],
            "accepted": [int(v) for v in hist[:, 4]]}
        del t2

    if args.serving_requests > 0 or args.serving_saturate > 0:
        del tgt64, tgt128
        rq.release_workspaces()
        torch.cuda.empty_cache()
        log(f"[bench] serving leg: {args.serving_requests} requests at {args.serving_rate}/s, "
            f"{args.serving_saturate} at saturation")
        out["serving"] = serving_run(rq, args.serving_requests, args.serving_rate,
                                     args.serving_saturate)
        log("[bench] serving done")

    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
