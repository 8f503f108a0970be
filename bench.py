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


def copy_bandwidth(torch, nbytes=4 << 30, reps=10):
    """Read+write rate of a plain device copy (torch's copy kernel) of nbytes:
    the practical HBM rate for streaming kernels on this GPU, reported next
    to the 8 TB/s datasheet peak."""
    x = torch.empty(nbytes // 8, dtype=torch.complex64, device="cuda")
    x.real.fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    torch.cuda.empty_cache()
    return round(2 * nbytes / (ms / 1e3) / 1e9, 1)


def _pcts(lat_ms):
    """Per-evaluation latency percentiles (HIP events around each step)."""
    return {f"p{q}": round(float(np.percentile(lat_ms, q)), 3) for q in (10, 50, 90, 99)}


def _kernel_name(key):
    names = {("hess", "sweep"): "k_hess_pass", ("hess", "states"): "k_pass (per-gate states)",
             ("hess", "hole"): "k_hole"}
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


def measured_traffic(kernel_key):
    """HBM bytes per launch of a sweep kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE runs, calibrated on a copy
    kernel), or None when the kernel code changed since it was taken."""
    prof = os.path.join(ROOT, "profiles", "k_pass_hvp_cfg3_c64.txt")
    src = os.path.join(ROOT, "paper_2506_23775_amd", "csrc", "rq_sweep.h")
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


def cpu_baseline(prob, ncols=2, budget_s=15.0):
    """The FP64 oracle timed on the host on a bounded sample: f, gradient and
    HVP contributions of `ncols` basis states of sector 0, extrapolated to the
    full 2^k-term trace (every summand costs the same)."""
    import oracle as O
    k = prob.k
    cols = O.sector_columns(k, 0)[:ncols]
    E = np.zeros((1 << k, ncols), dtype=np.complex128)
    E[cols, np.arange(ncols)] = 1.0
    for pair, G in prob.trotter:             # U|j> for the sample (untimed setup)
        E = O.apply_gate(E, k, pair, G)
    inst = prob.gates[prob.param_of]
    Z = prob.direction[prob.param_of]
    reps = 0
    t0 = time.perf_counter()
    while True:
        O.tangent_T(k, prob.pairs, inst, Z, E, cols)
        O.cost(k, prob.pairs, inst, E, cols)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = (time.perf_counter() - t0) / reps
    per_col = dt / ncols
    cores = len(os.sched_getaffinity(0))
    return dict(value=1.0 / (per_col * (1 << k)), unit="evals/s", cores=cores, kind="oracle",
                sample=f"{ncols} basis states of sector 0 x {reps} repetitions "
                       f"({dt * reps:.1f} s), extrapolated x{(1 << k) // ncols}")


def serving_run(rq, n_requests, rate_hz, seed_requests=None):
    """Configuration 5: a Poisson stream of f / f+grad / f+grad+HVP requests
    of mixed size (k = 8..16, depth 3..9), served by the continuous-batching
    loop in complex64 with FP64 accumulation.  Latency = completion - arrival
    (end to end, includes the request's target preparation on the device) and
    completion - admission (evaluation only)."""
    import torch

    import workloads as w
    from paper_2506_23775_amd import serving
    warm = serving.make_gpu_request(dict(rid=10**6, arrival=0.0, k=8, depth=3, U=4.0, t=0.5,
                                         op="hvp"), rq.RQ_C64)
    serving.ContinuousBatcher(serving.GpuExecutor(rq.RQ_C64), hbm_budget=1 << 30).run([warm])
    descs = w.configs.serving_requests(n_requests, rate_hz)
    reqs = [serving.make_gpu_request(d, rq.RQ_C64) for d in descs]
    ex = serving.GpuExecutor(rq.RQ_C64, chunk=4096)
    batcher = serving.ContinuousBatcher(ex, hbm_budget=96 << 30, max_active=8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = batcher.run(reqs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = serving.latency_stats(done)
    lat = {op: {k: (round(v, 2) if isinstance(v, float) else v) for k, v in st.items()}
           for op, st in stats.items()}
    ks = {}
    for d in descs:
        ks[str(d["k"])] = ks.get(str(d["k"]), 0) + 1
    return dict(workload="cfg5: Poisson arrivals of f / f+grad / f+grad+HVP requests, "
                         "k in {8..16}, brick-wall depth in {3,5,7,9}, Hubbard targets "
                         "(dense exp(-iHt) for k <= 12, 20-step Strang Trotter on the device "
                         "beyond), c64 states + FP64 accumulation",
                requests=len(done), rate_hz=rate_hz, seconds=round(dt, 3),
                throughput_req_per_s=round(len(done) / dt, 3), k_mix=ks,
                peak_hbm_GiB=round(batcher.peak_used / 2**30, 2), latency_ms=lat)


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
    ap.add_argument("--orbits", type=int, default=1,
                    help="1: time the translation-orbit-reduced evaluation (0: skip)")
    ap.add_argument("--hessian", type=int, default=1,
                    help="1: time the configuration-3 Hessian blocks (0: skip)")
    ap.add_argument("--tr-iters", type=int, default=5,
                    help="trust-region iterations in the configuration-2 leg (0: skip)")
    ap.add_argument("--serving-requests", type=int, default=16,
                    help="requests in the configuration-5 serving leg (0: skip it)")
    ap.add_argument("--serving-rate", type=float, default=1.0, help="Poisson arrival rate, 1/s")
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
    out["roofline"]["copy_ref_GBps"] = copy_bandwidth(torch)

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
        log(f"[bench] Hessian: {dt:.2f} s")
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
            "speedup_vs_parity_gates": round(dt / dtn, 3)}
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
        del t4
        torch.cuda.empty_cache()
        log(f"[bench] configuration 4: {out['config4']['ms_per_step']} ms/eval")

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

    if args.serving_requests > 0:
        del tgt64, tgt128
        torch.cuda.empty_cache()
        log(f"[bench] serving leg: {args.serving_requests} requests at {args.serving_rate}/s")
        out["serving"] = serving_run(rq, args.serving_requests, args.serving_rate)
        log(f"[bench] serving: {out['serving']['throughput_req_per_s']} req/s")

    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
