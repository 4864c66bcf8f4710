"""Benchmark of the PRIEST planner on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One step = one batched plan (Alg. 1) of the 3D workload: 64 independent
planning problems with distinct scenes, each N = 2000 samples, M = 128
spherical obstacles, K = 100 steps, 20 CEM iterations of 100 projection
iterations, FP32; every CEM step of all 64 problems runs as one projection
launch and one selection / refit launch, the whole CEM loop captured once in
a hipGraph and replayed, the projection's tile shape picked by the
autotuner.  Every sub-step (draw, project, residual, cost, top-k twice,
refit, Cholesky) runs on the GPU; inputs are resident in HBM before the
timed region.

Prints one JSON line: the metric is projected samples x iterations per
second (64 * N * n_proj_iters * n_cem per step), plus plans/s and per-step
latency percentiles, the roofline position of the projection kernel (its
launches timed by events that each launch stamps, over a second timed region
of the same plans without the graph, since those events need launches
outside capture; the metric comes from the first, graph-replayed region) and
the FP64 CPU oracle timed on a bounded sample of the same workload.  Extra
sections: the plain one-problem-per-launch FP32 form of the same 64 problems,
the single 2D paper-scale plan, 2D batched x64, BF16 mixed precision, the
unfused baseline, D-PRIEST and the continuous-batching server.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X published FP32 vector / MFMA peak
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "project_kernel_c3_traffic.txt")
COUNTER_FILE = os.path.join(ROOT, "profiles", "project_kernel_c3_mfma.txt")
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock: one FP32 op per lane-cycle
KERNEL_SOURCES = ("paper_2309_08235_amd/csrc/project.hip", "paper_2309_08235_amd/csrc/priest_internal.h")


def dense_flops(dims: int, nv: int, K: int) -> float:
    """FLOPs of one projection iteration for one sample outside the obstacle
    pairs: forward rows, velocity / acceleration push-outs, right-hand side,
    multiplier and KKT product (see projection_flops)."""
    return 12 * dims * nv * K + 2 * K * (2 * dims + 2) + dims * (5 * nv + 2 * nv * nv)


def pair_flops(dims: int) -> float:
    """FLOPs of one evaluated (sample, step, obstacle) pair."""
    return 2 * dims + dims + 2 * dims + 1 + 1


def projection_flops(dims: int, nv: int, K: int, M: int) -> float:
    """Algorithmic FLOPs of one projection iteration for one sample (every
    obstacle pair counted at its no-contact cost; pairs the kernel skips by
    culling are still counted).

      forward rows p, v, a      : 3 dims nv K FMA        -> 6 dims nv K
      obstacle pair (t, j)      : centre at t (dims FMA), offset (dims),
                                  scaled squared distance (2 dims + 1), test (1)
      velocity / acceleration   : 2 K (2 dims + 2)
      right-hand side W^T delta : 3 dims nv K FMA        -> 6 dims nv K
      multiplier + KKT product  : dims (2 nv + 2 nv^2 + 3 nv)
    """
    pair = 2 * dims + dims + 2 * dims + 1 + 1
    return (12 * dims * nv * K + pair * K * M + 2 * K * (2 * dims + 2)
            + dims * (5 * nv + 2 * nv * nv))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_values(path):
    """key: value lines of a profiles/ summary, or None when the file is
    missing or the kernel sources changed since its counters were taken."""
    try:
        vals = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    vals[k.strip()] = v.strip()
    except OSError:
        return None
    return vals if vals.get("kernel_source_sha256_16") == kernel_source_hash() else None


def measured_traffic():
    """HBM bytes per projection launch at the headline shape, from the
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary in profiles/ (null when the
    kernel sources changed since the counters were taken)."""
    vals = profile_values(TRAFFIC_FILE)
    try:
        return float(vals["hbm_bytes_per_launch"]) if vals else None
    except (KeyError, ValueError):
        return None


def measured_execution(kernel_ms):
    """What the projection kernel executed per launch at the headline shape,
    from the rocprofv3 SQ counter summary in profiles/ (null when the kernel
    sources changed since): MFMA instructions and their flops (2048 per
    16x16x4 FP32 MFMA), VALU instructions, the MFMA busy share of SIMD
    cycles, the VALU lane operations per second against one FP32 op per
    lane and cycle, and the mean resident waves per CU (of 16)."""
    vals = profile_values(COUNTER_FILE)
    if not vals:
        return None
    try:
        mfma = float(vals["mfma_instructions_per_launch"])
        valu = float(vals["valu_instructions_per_launch"])
        busy = float(vals["mfma_busy_frac"])
    except (KeyError, ValueError):
        return None
    t = kernel_ms * 1e-3
    try:
        waves = float(vals["mean_waves_per_cu"])
    except (KeyError, ValueError):
        waves = None
    return {"mfma_instructions_per_launch": mfma, "mfma_flops_per_launch": mfma * 2048,
            "mean_waves_per_cu": waves,
            "mfma_tflops": round(mfma * 2048 / t / 1e12, 3),
            "mfma_frac": round(mfma * 2048 / t / 1e12 / PEAK_FP32_TFLOPS, 4),
            "mfma_busy_frac": busy, "valu_instructions_per_launch": valu,
            "valu_lane_ops_frac": round(valu * 64 / t / VALU_LANE_OPS_PEAK, 4),
            "source": "profiles/project_kernel_c3_mfma.txt (rocprofv3 SQ counters, same kernel "
                      "sources), per launch over the same plans"}


def cpu_baseline(wl, n_sample: int, gpu_results=None, extra=None):
    """The FP64 oracle on `n_sample` samples of problem 0 of workload `wl`
    (one projection of n_proj_iters iterations), in projected samples x
    iters/s, with the host's math libraries on all their threads and then
    held to one thread (a quarter of the sample).  `gpu_results` maps a label
    to GPU-projected samples of the same inputs (first rows); their error
    against this oracle run is returned.  `extra` maps a label to
    (workload, n, {label: gpu samples}) for further error checks of other
    workloads (not timed)."""
    import oracle as O
    from paper_2309_08235_amd import workloads as W
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = 1

    def oracle_problem(w):
        return O.Problem(w.dims, w.n_coeff, w.n_steps, w.horizon, w.n_obs, w.rho, w.v_max,
                         w.a_max, w.bc_mask)

    def errors_of(pr, results, n):
        errors = {}
        for label, (xb, r) in (results or {}).items():
            xb = np.asarray(xb, np.float64)[:n]
            r = np.asarray(r, np.float64)[:n]
            e = np.abs(xb - pr.xi_bar).max(1) / np.maximum(1.0, np.abs(pr.xi_bar).max(1))
            er = np.abs(r - pr.resid)
            errors[label] = {"coeff_rel_median": float(np.median(e)),
                             "coeff_rel_p99": float(np.quantile(e, 0.99)),
                             "coeff_rel_max": float(e.max()),
                             "samples_above_1e-3": int(np.sum(e > 1e-3)),
                             "resid_abs_median": float(np.median(er)),
                             "resid_abs_max": float(er.max()),
                             "samples": int(n)}
        return errors

    bc, obs = W.scene(wl, 0)
    prob = oracle_problem(wl)
    xi = W.samples(wl, 5, n=n_sample)
    t0 = time.perf_counter()
    pr = O.project(prob, bc, obs, xi, wl.n_proj_iters)
    dt = time.perf_counter() - t0
    # the same oracle with its math libraries held to one thread, on a
    # quarter of the sample
    n1 = max(1, n_sample // 4)
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            O.project(prob, bc, obs, xi[:n1], wl.n_proj_iters)
            dt1 = time.perf_counter() - t1
        one_thread = {"value": n1 * wl.n_proj_iters / dt1, "cores": 1,
                      "sample": f"{n1} samples x {wl.n_proj_iters} projection iterations, {dt1:.1f} s"}
    except ImportError:
        one_thread = None
    errors = {wl.name: errors_of(pr, gpu_results, n_sample)}
    for label, (w2, n2, res2) in (extra or {}).items():
        b2, o2 = W.scene(w2, 0)
        p2 = O.project(oracle_problem(w2), b2, o2, W.samples(w2, 5, n=n2), w2.n_proj_iters)
        errors[label] = errors_of(p2, res2, n2)
    return {"value": n_sample * wl.n_proj_iters / dt, "unit": "projected samples*iters/s",
            "cores": int(threads), "kind": "oracle",
            "sample": f"{n_sample} samples x {wl.n_proj_iters} projection iterations of problem 0 "
                      f"of {wl.name} (part of one CEM iteration's projection; the projection is "
                      f"independent per sample, so the rate extrapolates to the whole batch), "
                      f"FP64 NumPy, {dt:.1f} s",
            "one_thread": one_thread, "host": host_cpu(),
            "gpu_error_vs_oracle": errors}


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}


def mfma_flops(dims: int, nv: int, K: int) -> float:
    """FLOPs of the three dense products of one projection iteration for one
    sample, unpadded: forward rows W xi_bar (3 dims nv K FMA), right-hand
    side W^T delta (the same) and the KKT product (dims nv^2 FMA)."""
    return 12 * dims * nv * K + 2 * dims * nv * nv


def roofline_entry(wl, n_samples_per_launch, avg_ms, launches, tiling, note, pairs_per_launch):
    """Roofline of the fused projection kernel against its algorithmic work:
    per sample and iteration the dense part of the AM iteration (forward
    rows, push-out arithmetic outside the obstacle terms, right-hand side,
    KKT step; plus the forward rows of the final residual pass) and the
    obstacle pairs the kernel evaluated, counted on the device (pairs
    dropped by culling contribute exact zeros and are not work the kernel
    does).  dense_rows_* is the share of the three dense products (their
    unpadded flops) against the FP32 matrix peak.  The kernel does not
    evaluate rows whose push-outs it has proven zero, so it executes fewer
    MFMAs than the dense products hold; the counts it executed are under
    `executed` (from the profile counters)."""
    n, it = n_samples_per_launch, wl.n_proj_iters
    fwd = 6 * wl.dims * wl.n_coeff * wl.n_steps * n
    dense = dense_flops(wl.dims, wl.n_coeff, wl.n_steps) * n * it + fwd
    flops = dense + pair_flops(wl.dims) * pairs_per_launch
    useful = mfma_flops(wl.dims, wl.n_coeff, wl.n_steps) * n * it + fwd
    all_pairs = n * wl.n_steps * wl.n_obs * (it + 1)
    achieved = flops / (avg_ms * 1e-3) / 1e12
    mfma = useful / (avg_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "kernel": f"project_kernel<{wl.dims}D, tiling {tuple(tiling)}>",
            "kernel_ms": round(avg_ms, 4), "launches": launches,
            "flops_per_launch": flops, "pairs_evaluated_per_launch": pairs_per_launch,
            "pairs_evaluated_frac": round(pairs_per_launch / all_pairs, 5) if all_pairs else None,
            "dense_rows_flops_per_launch": useful,
            "dense_rows_tflops": round(mfma, 3),
            "dense_rows_frac": round(mfma / PEAK_FP32_TFLOPS, 4),
            "work": "algorithmic: dense AM-iteration flops per sample-iteration (evaluated or "
                    "proven zero) + evaluated obstacle pairs",
            "frac_note": "the algorithmic work counts the rows the kernel proves zero and does not "
                         "execute, so achieved can pass the peak; what the hardware executed, "
                         "against its own peaks, is in `executed`",
            "timing": note}


def batched(P, W, wl, steps: int, plain_problems: int):
    """n_problems independent problems of workload `wl`: batched = every CEM
    step of all problems in one launch, the whole CEM loop captured in a
    hipGraph and replayed, tile shape from the autotuner; plain = one problem
    per launch, no graph, default tile shape (timed on `plain_problems`
    problems and scaled)."""
    import torch
    dev = "cuda:0"
    prob = P.Problem.from_workload(wl)
    nP = wl.n_problems
    scenes = [W.scene(wl, q) for q in range(nP)]
    bc = torch.tensor(np.stack([s[0] for s in scenes]), dtype=torch.float32, device=dev)
    obs = torch.tensor(np.stack([s[1] for s in scenes]), dtype=torch.float32, device=dev)
    mu0 = torch.tensor(np.stack([W.initial_mean(wl)] * nP), dtype=torch.float32, device=dev)
    cov0 = torch.tensor(np.stack([W.initial_cov(wl)] * nP), dtype=torch.float32, device=dev)
    cem = P.Cem(n_samples=wl.n_samples, n_cem=wl.n_cem, n_proj_iters=wl.n_proj_iters,
                n_proj=wl.n_proj, n_elite=wl.n_elite, sigma=wl.sigma, gamma=wl.gamma,
                cov_jitter=wl.cov_jitter)
    mu, cov = mu0.clone(), cov0.clone()
    out = prob.plan_outputs(cem, nP, full=False)
    ws = prob.workspace(cem, nP)
    s = torch.cuda.Stream()

    def batch_step(graph=True):
        mu.copy_(mu0)
        cov.copy_(cov0)
        prob.plan_batch(nP, bc, obs, cem, mu, cov, seed=77, stream_base=0, out=out, workspace=ws,
                        use_graph=graph, stream=s)

    with torch.cuda.stream(s):
        batch_step()                      # autotune + capture + first replay
        s.synchronize()
        tiling = prob.last_tiling()
        t0 = time.perf_counter()
        for _ in range(steps):
            batch_step()
        s.synchronize()
        t_batch = (time.perf_counter() - t0) / steps
        # projection kernel time of the same launches outside the graph
        P.priest_profile_read()
        P.priest_profile_enable(True)
        batch_step(graph=False)
        s.synchronize()
        P.priest_profile_enable(False)
        n_l, ms = P.priest_profile_read()
        # evaluated pairs of the same launches (same draws: identical work)
        P.priest_profile_count_pairs(True)
        batch_step(graph=False)
        pairs = P.priest_profile_read_pairs()
        P.priest_profile_count_pairs(False)
    assert int(out["status"].abs().sum().item()) == 0
    roof = roofline_entry(wl, nP * wl.n_samples, ms / n_l, n_l, tiling[0],
                          "HIP events around each projection launch of one batched plan (no graph)",
                          pairs / n_l)
    # plain: one problem per launch, no graph, default tile shape
    prob.set_tiling((4, 1, 0))
    out1 = prob.plan_outputs(cem, 1, full=False)
    ws1 = prob.workspace(cem, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in range(plain_problems):
        m, c = mu0[q].clone(), cov0[q].clone()
        prob.plan(bc[q], obs[q], cem, m, c, seed=77, stream_id=q, out=out1, workspace=ws1)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / plain_problems * nP
    work = nP * wl.n_samples * wl.n_proj_iters * wl.n_cem
    prob.close()
    return {"workload": wl.name, "problems": nP, "tiling": list(tiling[0]),
            "tiling_from_autotuner": tiling[1],
            "batched_graph": {"s_per_batch": round(t_batch, 4),
                              "samples_iters_per_s": round(work / t_batch, 1),
                              "plans_per_s": round(nP / t_batch, 2)},
            "plain_per_problem": {"s_per_batch_equivalent": round(t_plain, 4),
                                  "samples_iters_per_s": round(work / t_plain, 1),
                                  "plans_per_s": round(nP / t_plain, 2),
                                  "timed_problems": plain_problems},
            "speedup": round(t_plain / t_batch, 3),
            "roofline": roof}


def dpriest_section(P, W, reps: int, seeds: int = 4):
    """D-PRIEST on the headline scene: G Gaussians fanned out around the
    straight line share N = 1000 samples (N/G each), every CEM step of all
    groups in one launch (one plan_dpriest call), against the plain form of
    G separate priest_plan calls.  Also the mean picked cost over a few
    seeds, the quality side of Sec. III-C."""
    import torch
    dev = "cuda:0"
    base = W.C2
    bc_h, obs_h = W.scene(base, 0)
    bc = torch.tensor(bc_h, dtype=torch.float32, device=dev)
    obs = torch.tensor(obs_h, dtype=torch.float32, device=dev)
    rows = []
    for G in (1, 2, 4, 8):
        n = base.n_samples // G
        wl = W.with_changes(base, n_samples=n, n_proj=W.default_n_proj(n),
                            n_elite=max(4, base.n_elite // G))
        prob = P.Problem.from_workload(wl)
        cem = P.Cem(n_samples=n, n_cem=wl.n_cem, n_proj_iters=wl.n_proj_iters, n_proj=wl.n_proj,
                    n_elite=wl.n_elite, sigma=wl.sigma, gamma=wl.gamma, cov_jitter=wl.cov_jitter)
        mu0 = torch.tensor(W.dpriest_means(wl, G), dtype=torch.float32, device=dev)
        cov0 = torch.tensor(np.stack([W.initial_cov(wl)] * G), dtype=torch.float32, device=dev)
        mu, cov = mu0.clone(), cov0.clone()
        out = prob.plan_outputs(cem, G, full=False)
        ws = prob.workspace(cem, G)
        best = torch.empty(wl.D, device=dev)
        bcost = torch.empty(1, device=dev)
        bg = torch.empty(1, dtype=torch.int32, device=dev)

        def run(seed):
            mu.copy_(mu0)
            cov.copy_(cov0)
            P.priest_plan_dpriest(prob.handle, G, bc, obs, cem.c(), mu, cov, seed, 0, None, out,
                                  best, bcost, bg, ws)

        run(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(reps):
            run(r)
        torch.cuda.synchronize()
        t_d = (time.perf_counter() - t0) / reps
        costs = []
        for sd in range(seeds):
            run(1000 + sd)
            costs.append(float(bcost.item()))
        assert int(out["status"].abs().sum().item()) == 0
        # plain: the G distributions as G separate plans, one launch each
        prob.set_tiling((4, 1, 0))
        out1 = prob.plan_outputs(cem, 1, full=False)
        ws1 = prob.workspace(cem, 1)
        ms = [mu0[g].clone() for g in range(G)]
        cs = [cov0[g].clone() for g in range(G)]
        for g in range(G):
            prob.plan(bc, obs, cem, ms[g], cs[g], seed=0, stream_id=g, out=out1, workspace=ws1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(reps):
            for g in range(G):
                ms[g].copy_(mu0[g])
                cs[g].copy_(cov0[g])
                prob.plan(bc, obs, cem, ms[g], cs[g], seed=r, stream_id=g, out=out1,
                          workspace=ws1)
        torch.cuda.synchronize()
        t_p = (time.perf_counter() - t0) / reps
        prob.close()
        rows.append({"groups": G, "samples_per_group": n,
                     "ms_per_plan": round(t_d * 1e3, 3),
                     "plain_separate_plans_ms": round(t_p * 1e3, 3),
                     "speedup": round(t_p / t_d, 3),
                     "mean_picked_cost": round(float(np.mean(costs)), 4),
                     "seeds": seeds})
    return {"workload": "c2 scene, N=1000 total split over G groups, n_cem=%d" % base.n_cem,
            "rows": rows}


def unfused_baseline(P, W, reps: int):
    """The projection at the headline shape (N=1000) and at N=64000 (the C2
    scene replicated x64) in the fused kernel and in the plain unfused form
    (three kernels per iteration through HBM), HIP-event timed."""
    import torch
    dev = "cuda:0"
    wl = W.C2
    out = {}
    bc_h, obs_h = W.scene(wl, 0)
    bc = torch.tensor(bc_h, dtype=torch.float32, device=dev)
    obs = torch.tensor(obs_h, dtype=torch.float32, device=dev)
    prob = P.Problem.from_workload(wl)
    ka, kb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for N in (wl.n_samples, 64 * wl.n_samples):
        xi = torch.tensor(W.samples(wl, 5, n=N), dtype=torch.float32, device=dev)
        ws = torch.empty(P.priest_project_unfused_workspace_size(prob.handle, N), dtype=torch.uint8,
                         device=dev)
        xo = torch.empty_like(xi)
        r = torch.empty(N, device=dev)
        c1 = torch.empty(N, device=dev)
        times = {}
        for name, fn in (("fused", lambda: P.priest_project(prob.handle, bc, obs, xi, wl.n_proj_iters,
                                                            xo, r, c1)),
                         ("unfused", lambda: P.priest_project_unfused(prob.handle, bc, obs, xi,
                                                                      wl.n_proj_iters, xo, r, c1, ws))):
            fn()
            torch.cuda.synchronize()
            ka.record()
            for _ in range(reps):
                fn()
            kb.record()
            torch.cuda.synchronize()
            times[name] = ka.elapsed_time(kb) / reps
        out[f"n{N}"] = {"fused_ms": round(times["fused"], 4), "unfused_ms": round(times["unfused"], 4),
                        "speedup": round(times["unfused"] / times["fused"], 2),
                        "fused_tiling": list(prob.last_tiling()[0])}
    prob.close()
    out["note"] = ("one projection of 100 iterations of the C2 scene; unfused = forward, push-out "
                   "and update kernels per iteration with p/v/a and push-outs in HBM, no MFMA, no "
                   "culling; per-pass HBM throughput in profiles/unfused_passes_c2x64.md")
    return out


def serving(P, W, n_requests: int, plain_limit_s: float, sweep_requests: int = 2048,
            slo_ms: float = 10.0):
    """Continuous-batching service: the Poisson request stream of many robots
    (mixed N, M, K) replayed in real time through the server, and the same
    stream through one priest_plan call per request (the plain form)."""
    from paper_2309_08235_amd import serve as S
    wl = W.C5
    reqs = W.serving_requests(wl, n_requests=n_requests)
    offered_flop = sum(projection_flops(wl.dims, wl.n_coeff, q.n_steps, q.n_obs) * q.n_samples
                       for q in reqs) * wl.n_proj_iters * wl.n_cem
    span = reqs[-1].arrival
    srv = S.Server.for_workload(wl, max_active=1024, memory_budget=2 << 30)
    S.prepare_shapes(srv, reqs)
    warm = W.serving_requests(wl, n_requests=256)
    S.run_stream(srv, warm, wl, realtime=False)          # warm-up on a throw-away server
    srv.close()
    srv = S.Server.for_workload(wl, max_active=1024, memory_budget=2 << 30)
    S.prepare_shapes(srv, reqs)
    batched_line, done = S.run_stream(srv, reqs, wl, realtime=True)
    bad = sum(1 for c in done if c.status != 0)
    srv.close()
    plain, _ = S.run_plain(reqs, wl, realtime=True, time_limit=plain_limit_s)
    sweep = serving_sweep(P, W, S, wl, sweep_requests, slo_ms)
    return {"workload": wl.name, "robots": wl.n_robots, "requests": n_requests,
            "offered_req_per_s": round(n_requests / span, 1),
            "offered_tflop_per_s": round(offered_flop / span / 1e12, 2),
            "iterations": f"{wl.n_proj_iters} projection x {wl.n_cem} CEM",
            "continuous_batching": batched_line, "nonfinite_results": bad,
            "plain_per_request": plain,
            "plain_note": f"one priest_plan per request, FIFO, synchronised; stopped after "
                          f"{plain_limit_s} s if behind",
            "equal_p99": sweep}


def serving_sweep(P, W, S, wl, n_requests: int, slo_ms: float):
    """The same kind of request stream at several offered rates (the robots'
    Poisson clocks sped up or slowed down), through a fresh server and
    through the plain per-request form.  A form sustains a rate if its p99
    latency (arrival to result) stays within the SLO and it completes every
    request; the comparison is the highest rate each form sustains."""
    server_scales = (1.0, 1.5, 2.0, 2.25, 2.5, 2.75, 3.0, 4.0, 8.0)
    plain_scales = (0.25, 0.5, 0.6, 0.7, 0.8, 1.0, 1.5)
    curve = {"server": [], "plain": []}

    def point(scale, summary):
        return {"rate_scale": scale, "offered_req_per_s": summary.get("offered_req_per_s"),
                "plans_per_s": summary["plans_per_s"], "p50_ms": summary["latency_ms"]["p50"],
                "p99_ms": summary["latency_ms"]["p99"], "completed": summary["requests"],
                "within_slo": bool(summary["latency_ms"]["p99"] <= slo_ms
                                   and summary["requests"] == n_requests)}

    for sc in server_scales:
        reqs = W.serving_requests(wl, n_requests=n_requests, rate_scale=sc)
        srv = S.Server.for_workload(wl, max_active=1024, memory_budget=2 << 30)
        S.prepare_shapes(srv, reqs)
        summ, _ = S.run_stream(srv, reqs, wl, realtime=True)
        srv.close()
        pt = point(sc, summ)
        pt["max_active"] = summ["max_active"]
        curve["server"].append(pt)
    for sc in plain_scales:
        reqs = W.serving_requests(wl, n_requests=n_requests, rate_scale=sc)
        summ, _ = S.run_plain(reqs, wl, realtime=True, time_limit=4.0 * reqs[-1].arrival + 2.0)
        summ["offered_req_per_s"] = round(n_requests / reqs[-1].arrival, 1)
        curve["plain"].append(point(sc, summ))

    def best(points):
        ok = [q for q in points if q["within_slo"]]
        if not ok:
            return None
        q = max(ok, key=lambda q: q["offered_req_per_s"])
        return {"offered_req_per_s": q["offered_req_per_s"], "plans_per_s": q["plans_per_s"],
                "p99_ms": q["p99_ms"]}

    bs, bp = best(curve["server"]), best(curve["plain"])
    return {"slo_p99_ms": slo_ms, "requests_per_point": n_requests, "curve": curve,
            "max_sustained_under_slo": {"server": bs, "plain": bp},
            "server_over_plain": (round(bs["plans_per_s"] / bp["plans_per_s"], 2)
                                  if bs and bp else None),
            "note": "highest offered rate of the sweep at which the form's p99 stays within the "
                    "SLO with every request completed; the server's top rate is a lower bound "
                    "when it still meets the SLO there"}


def headline_c3(P, W, args):
    """The metric: K graph-replayed batched plans of the 3D workload (64
    problems x 2000 samples), then the same plans without the graph with
    every projection launch timed by its own events, then once more with the
    device's pair counter on.  Every step resets (mu, Sigma) and uses the
    same seed, so every step does identical work."""
    import torch
    dev = "cuda:0"
    wl = W.C3
    nP = wl.n_problems
    prob = P.Problem.from_workload(wl)
    if args.tiling:
        prob.set_tiling(tuple(int(v) for v in args.tiling.split(",")))
    scenes = [W.scene(wl, q) for q in range(nP)]
    bc = torch.tensor(np.stack([sc[0] for sc in scenes]), dtype=torch.float32, device=dev)
    obs = torch.tensor(np.stack([sc[1] for sc in scenes]), dtype=torch.float32, device=dev)
    mu0 = torch.tensor(np.stack([W.initial_mean(wl)] * nP), dtype=torch.float32, device=dev)
    cov0 = torch.tensor(np.stack([W.initial_cov(wl)] * nP), dtype=torch.float32, device=dev)
    cem = P.Cem(n_samples=wl.n_samples, n_cem=wl.n_cem, n_proj_iters=wl.n_proj_iters,
                n_proj=wl.n_proj, n_elite=wl.n_elite, sigma=wl.sigma, gamma=wl.gamma,
                cov_jitter=wl.cov_jitter)
    mu, cov = mu0.clone(), cov0.clone()
    out = prob.plan_outputs(cem, nP, full=False)
    ws = prob.workspace(cem, nP)
    s = torch.cuda.Stream()

    def step(graph=True):
        mu.copy_(mu0)
        cov.copy_(cov0)
        prob.plan_batch(nP, bc, obs, cem, mu, cov, seed=77, stream_base=0, out=out, workspace=ws,
                        use_graph=graph, stream=s)

    with torch.cuda.stream(s):
        for _ in range(max(1, args.warmup)):   # the first also tunes the tile shape and captures
            step()
        s.synchronize()
        tiling = prob.last_tiling()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            ev[i][0].record(s)
            step()
            ev[i][1].record(s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = np.array([a.elapsed_time(b) for a, b in ev])
        # the same plans launched outside the graph, each projection launch
        # timed by events that the launch itself stamps
        P.priest_profile_read()
        P.priest_profile_enable(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            step(graph=False)
        torch.cuda.synchronize()
        wall_instr = time.perf_counter() - t1
        P.priest_profile_enable(False)
        n_launch, k_total_ms = P.priest_profile_read()
        # evaluated obstacle pairs of one more identical plan
        P.priest_profile_count_pairs(True)
        step(graph=False)
        pairs = P.priest_profile_read_pairs()
        P.priest_profile_count_pairs(False)
    status = out["status"].cpu().numpy()
    best = out["best_cost"].cpu().numpy()
    assert np.all(status == 0) and np.all(np.isfinite(best)), (status, best)
    assert n_launch == args.steps * wl.n_cem, n_launch
    work = nP * wl.n_samples * wl.n_proj_iters * wl.n_cem
    roof = roofline_entry(wl, nP * wl.n_samples, k_total_ms / n_launch, n_launch, tiling[0],
                          "HIP events stamped by every projection launch (hipExtLaunchKernel) over "
                          "a second timed region of the same batched plans launched without the "
                          "graph; its wall time is instrumented_ms_per_step", pairs / wl.n_cem)
    roof["instrumented_ms_per_step"] = round(wall_instr / args.steps * 1e3, 3)
    roof["traffic"] = measured_traffic()
    roof["executed"] = measured_execution(roof["kernel_ms"])
    roof["traffic_note"] = ("HBM bytes per launch from rocprofv3 FETCH_SIZE + WRITE_SIZE "
                            "(profiles/project_kernel_c3_traffic.txt), null if the kernel sources "
                            "changed since")
    # plain form: one problem per launch, no graph, default tile shape, on
    # plain_problems of the 64 problems (scaled to the batch)
    prob.set_tiling((4, 1, 0))
    out1 = prob.plan_outputs(cem, 1, full=False)
    ws1 = prob.workspace(cem, 1)
    m, c = mu0[0].clone(), cov0[0].clone()
    prob.plan(bc[0], obs[0], cem, m, c, seed=77, stream_id=0, out=out1, workspace=ws1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in range(args.plain_problems):
        m, c = mu0[q].clone(), cov0[q].clone()
        prob.plan(bc[q], obs[q], cem, m, c, seed=77, stream_id=q, out=out1, workspace=ws1)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / args.plain_problems * nP
    # standalone projection of fresh samples of problem 0 (for the oracle's
    # error check in the CPU baseline leg)
    xi = torch.tensor(W.samples(wl, 5), dtype=torch.float32, device=dev)
    xo, r, _ = prob.project(bc[0], obs[0], xi, wl.n_proj_iters)
    torch.cuda.synchronize()
    prob.close()
    return {
        "wall": wall, "lat": lat, "work": work, "roofline": roof, "tiling": tiling,
        "plain": {"s_per_batch_equivalent": round(t_plain, 4),
                  "samples_iters_per_s": round(work / t_plain, 1),
                  "plans_per_s": round(nP / t_plain, 2),
                  "timed_problems": args.plain_problems,
                  "speedup_of_batched_graph": round(t_plain / (wall / args.steps), 3)},
        "gpu_samples": {"fp32": (xo.cpu().numpy(), r.cpu().numpy())},
    }


def single_plan_c2(P, W, args):
    """The 2D paper-scale single plan (N = 1000, M = 50 incl. 20 moving, K =
    100, 100 x 20 iterations), one problem per call: plan time, its
    projection kernel's roofline, a standalone projection of fresh samples,
    and the BF16 mixed-precision projection of the same samples."""
    import torch
    dev = "cuda:0"
    wl = W.C2
    prob = P.Problem.from_workload(wl)
    bc_h, obs_h = W.scene(wl, 0)
    bc = torch.tensor(bc_h, dtype=torch.float32, device=dev)
    obs = torch.tensor(obs_h, dtype=torch.float32, device=dev)
    D = prob.D
    # (mu, Sigma) in one buffer, so that resetting them before a plan is one copy
    state0 = torch.cat([torch.tensor(W.initial_mean(wl), dtype=torch.float32).reshape(-1),
                        torch.tensor(W.initial_cov(wl), dtype=torch.float32).reshape(-1)]).to(dev)
    state = state0.clone()
    mu, cov = state[:D], state[D:].view(D, D)
    cem = P.Cem(n_samples=wl.n_samples, n_cem=wl.n_cem, n_proj_iters=wl.n_proj_iters,
                n_proj=wl.n_proj, n_elite=wl.n_elite, sigma=wl.sigma, gamma=wl.gamma,
                cov_jitter=wl.cov_jitter)
    out = prob.plan_outputs(cem, full=False)
    ws = prob.workspace(cem)
    stream = torch.cuda.current_stream()
    steps = args.c2_steps

    def step(i):
        state.copy_(state0)
        prob.plan(bc, obs, cem, mu, cov, seed=1234 + i, stream_id=0, out=out, workspace=ws)

    for i in range(3):                 # the first plan also runs the autotuner
        step(i)
    torch.cuda.synchronize()
    tiling = prob.last_tiling()

    def timed(kernel_events):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        if kernel_events:
            P.priest_profile_read()
            P.priest_profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            ev[i][0].record(stream)
            step(3 + i)
            ev[i][1].record(stream)
        torch.cuda.synchronize()
        w = time.perf_counter() - t0
        prof = (0, 0.0)
        if kernel_events:
            P.priest_profile_enable(False)
            prof = P.priest_profile_read()
        return w, np.array([a.elapsed_time(b) for a, b in ev]), prof

    wall, lat, _ = timed(False)
    wall_instr, _, (n_launch, k_total_ms) = timed(True)
    P.priest_profile_count_pairs(True)
    for i in range(steps):
        step(3 + i)
    pairs_total = P.priest_profile_read_pairs()
    P.priest_profile_count_pairs(False)
    assert int(out["status"][0].item()) == 0 and np.isfinite(float(out["best_cost"][0].item()))
    assert n_launch == steps * wl.n_cem, n_launch
    per_plan = wl.n_samples * wl.n_proj_iters * wl.n_cem
    roof = roofline_entry(wl, wl.n_samples, k_total_ms / n_launch, n_launch, tiling[0],
                          "HIP events stamped by every projection launch over a second timed "
                          "region of the same plans", pairs_total / n_launch)
    roof["instrumented_ms_per_step"] = round(wall_instr / steps * 1e3, 4)
    # standalone projection of fresh samples at the same shape
    xi = torch.tensor(W.samples(wl, 5), dtype=torch.float32, device=dev)
    xo = torch.empty_like(xi)
    r = torch.empty(wl.n_samples, device=dev)
    c1 = torch.empty(wl.n_samples, device=dev)
    ka, kb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        P.priest_project(prob.handle, bc, obs, xi, wl.n_proj_iters, xo, r, c1)
    torch.cuda.synchronize()
    ka.record(stream)
    for _ in range(args.kernel_reps):
        P.priest_project(prob.handle, bc, obs, xi, wl.n_proj_iters, xo, r, c1)
    kb.record(stream)
    torch.cuda.synchronize()
    k_ms = round(ka.elapsed_time(kb) / args.kernel_reps, 4)
    samples = {"fp32": (xo.cpu().numpy(), r.cpu().numpy())}
    mixed = None
    if not args.no_mixed:
        # BF16 operands for the right-hand side and a BF16 hi/lo KKT product,
        # last 10 iterations in FP32
        prob_bf = P.Problem.from_workload(wl, precision=P.BF16_MIXED, n_refine_fp32=10)
        xo_bf = torch.empty_like(xi)
        r_bf = torch.empty(wl.n_samples, device=dev)
        for _ in range(3):
            P.priest_project(prob_bf.handle, bc, obs, xi, wl.n_proj_iters, xo_bf, r_bf, c1)
        torch.cuda.synchronize()
        ka.record(stream)
        for _ in range(args.kernel_reps):
            P.priest_project(prob_bf.handle, bc, obs, xi, wl.n_proj_iters, xo_bf, r_bf, c1)
        kb.record(stream)
        torch.cuda.synchronize()
        samples["bf16_mixed"] = (xo_bf.cpu().numpy(), r_bf.cpu().numpy())
        mixed = {"kernel_ms_fp32": k_ms,
                 "kernel_ms_bf16_mixed": round(ka.elapsed_time(kb) / args.kernel_reps, 4),
                 "n_refine_fp32": 10,
                 "note": "BF16 operands for W^T(e - F xi) and a BF16 hi/lo split of M11 u, "
                         "FP32 accumulation; errors vs the FP64 oracle in "
                         "cpu_baseline.gpu_error_vs_oracle.c2_fp32_and_bf16"}
        prob_bf.close()
    prob.close()
    return {
        "section": {"workload": wl.name, "samples_iters_per_s": round(per_plan * steps / wall, 1),
                    "ms_per_plan": round(wall * 1e3 / steps, 4),
                    "plans_per_sec": round(steps / wall, 3),
                    "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                                   "p99": round(float(np.percentile(lat, 99)), 4)},
                    "tiling": {"shape": list(tiling[0]), "from_autotuner": tiling[1]},
                    "roofline": roof, "kernel_standalone_ms": k_ms, "plans": steps},
        "mixed": mixed, "samples": samples, "wl": wl,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--c2-steps", type=int, default=20)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--cpu-sample", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary sections")
    ap.add_argument("--no-c2", action="store_true", help="skip the single 2D plan section")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision section")
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--plain-problems", type=int, default=8)
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--serve-plain-limit", type=float, default=20.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-sweep-requests", type=int, default=2048)
    ap.add_argument("--serve-slo-ms", type=float, default=10.0)
    ap.add_argument("--only-serve", action="store_true",
                    help="run only the serving section (profiling runs)")
    ap.add_argument("--only-c2", action="store_true",
                    help="run only the single 2D plan section (profiling runs)")
    ap.add_argument("--only-unfused", action="store_true",
                    help="run only the unfused-baseline section (profiling runs)")
    ap.add_argument("--tiling", type=str, default=None,
                    help="axis_slots,row_tiles,persistent for the headline plans (default: autotuned)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="first run one plain device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): every problem and "
              "request is independent, so N GPUs would run N disjoint copies", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2309_08235_amd import priest as P
    from paper_2309_08235_amd import workloads as W

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.calibration_copy_mib > 0:
        n = args.calibration_copy_mib << 18
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only_unfused:
        print(json.dumps({"unfused_baseline": unfused_baseline(P, W, reps=2)}), flush=True)
        return
    if args.only_c2:
        c2 = single_plan_c2(P, W, args)
        print(json.dumps({"c2_single_plan": c2["section"], "mixed_precision": c2["mixed"]}),
              flush=True)
        return
    if args.only_serve:
        print(json.dumps({"serving": serving(P, W, args.serve_requests, args.serve_plain_limit,
                                             args.serve_sweep_requests, args.serve_slo_ms)}),
              flush=True)
        return

    h = headline_c3(P, W, args)
    wl = W.C3
    print(f"[bench] headline done: {h['wall'] / args.steps * 1e3:.2f} ms per step", file=sys.stderr,
          flush=True)

    c2 = None
    if not args.no_c2:
        c2 = single_plan_c2(P, W, args)
        print("[bench] single 2D plan done", file=sys.stderr, flush=True)

    extra_2d = unfused = dpr = None
    if not args.no_extra:
        extra_2d = batched(P, W, W.with_changes(W.C2, name="c2x64_2d_k100_n1000_m50", n_problems=64),
                           args.batch_steps, args.plain_problems)
        unfused = unfused_baseline(P, W, reps=3)
        dpr = dpriest_section(P, W, reps=5)
        print("[bench] secondary sections done", file=sys.stderr, flush=True)

    serve_line = None
    if not args.no_serve:
        serve_line = serving(P, W, args.serve_requests, args.serve_plain_limit,
                             args.serve_sweep_requests, args.serve_slo_ms)
        print("[bench] serving done", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        extra = None
        if c2 is not None:
            extra = {"c2_fp32_and_bf16": (c2["wl"], 100, c2["samples"])}
        cpu = cpu_baseline(wl, args.cpu_sample, h["gpu_samples"], extra)
        cpu["value"] = round(cpu["value"], 2)

    wall = h["wall"]
    line = {
        "metric": "projected samples*iters/s",
        "value": round(h["work"] * args.steps / wall, 1),
        "unit": "samples*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "dims": wl.dims, "n_problems": wl.n_problems,
                   "n_samples": wl.n_samples, "n_obs": wl.n_obs, "n_steps": wl.n_steps,
                   "n_coeff": wl.n_coeff, "n_proj_iters": wl.n_proj_iters, "n_cem": wl.n_cem,
                   "n_proj": wl.n_proj, "n_elite": wl.n_elite, "hipgraph": True,
                   "parallelism": "single-gpu"},
        "plans_per_sec": round(wl.n_problems * args.steps / wall, 3),
        "latency_ms": {"p50": round(float(np.percentile(h["lat"], 50)), 4),
                       "p99": round(float(np.percentile(h["lat"], 99)), 4),
                       "note": "per step; each step completes all 64 plans together"},
        "tiling": {"shape": list(h["tiling"][0]), "from_autotuner": h["tiling"][1]},
        "roofline": h["roofline"],
        "cpu_baseline": cpu,
        "plain_per_problem": h["plain"],
        "c2_single_plan": c2["section"] if c2 else None,
        "mixed_precision": c2["mixed"] if c2 else None,
        "batched_2d": extra_2d,
        "unfused_baseline": unfused,
        "dpriest": dpr,
        "serving": serve_line,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
