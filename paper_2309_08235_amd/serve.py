"""Continuous-batching planning service on top of the priest_server_* C ABI.

:class:`Server` wraps one server handle.  :func:`run_stream` replays a
request stream in real time (arrivals on the host clock), stepping the
server while requests are in flight, and reports p50/p99 latency (arrival to
observed completion) and plans/s.  :func:`run_plain` replays the same stream
through one ``priest_plan`` call per request (one problem per launch,
sequential), the form without batching, for comparison.

All planning arithmetic runs in libpriest.so; this module only marshals
requests and measures time.
"""
from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import priest as P
from .workloads import C5, ServingWorkload


@dataclass
class Completed:
    request_id: int
    robot: int
    status: int
    arrival: float
    t_admit: float
    t_done: float
    best_cost: float
    best_xi: np.ndarray


class Server:
    """Owns a priest_server handle.  ``stream`` is a torch stream (None: the
    current one); dry-run servers touch no device."""

    def __init__(self, dims=2, n_coeff=11, bc_mask=P.BC_DEFAULT, precision=P.FP32,
                 n_refine_fp32=10, max_active=1024, max_robots=256, max_inflight_steps=2,
                 dry_run=False, rho=1.0, v_max=math.inf, a_max=math.inf, seed=0,
                 memory_budget=1 << 30, sigma=0.5, gamma=1.0, cov_jitter=1e-5, init_std=1.0,
                 stream=None):
        self.cfg = P.ServerConfig(dims, n_coeff, bc_mask, precision, n_refine_fp32, max_active,
                                  max_robots, max_inflight_steps, int(bool(dry_run)), 0, rho,
                                  v_max, a_max, seed, memory_budget, sigma, gamma, cov_jitter,
                                  init_std)
        self.D = dims * n_coeff
        self.dims = dims
        self.handle = P.priest_server_create(self.cfg, stream)

    @classmethod
    def for_workload(cls, wl: ServingWorkload = C5, **kw):
        d = dict(dims=wl.dims, n_coeff=wl.n_coeff, bc_mask=wl.bc_mask, rho=wl.rho,
                 v_max=wl.v_max, a_max=wl.a_max, sigma=wl.sigma, gamma=wl.gamma,
                 cov_jitter=wl.cov_jitter, init_std=wl.init_std, max_robots=wl.n_robots)
        d.update(kw)
        return cls(**d)

    def close(self):
        if self.handle is not None and self.handle.value:
            P.priest_server_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prepare(self, n_steps, n_obs, horizon):
        P.priest_server_prepare(self.handle, n_steps, n_obs, horizon)

    def submit(self, robot, bc, obs, n_samples, n_steps, horizon, n_cem, n_proj_iters, n_proj,
               n_elite, warm_start=P.WARM_KEEP, stream_id=0, arrival=0.0) -> int:
        bc32 = np.ascontiguousarray(bc, dtype=np.float32)
        obs32 = np.ascontiguousarray(obs, dtype=np.float32).reshape(-1, 8)
        if bc32.shape != (self.dims, 6):
            raise ValueError(f"bc must be [{self.dims}, 6]")
        req = P.Request(robot, n_steps, obs32.shape[0], n_samples, n_cem, n_proj_iters, n_proj,
                        n_elite, warm_start, stream_id & 0xFFFFFFFF, horizon, arrival,
                        bc32.ctypes.data, obs32.ctypes.data if obs32.size else None)
        return P.priest_server_submit(self.handle, req)

    def submit_request(self, q, wl: ServingWorkload = C5, t0=0.0, warm_start=P.WARM_KEEP):
        """Submits a workloads.ServingRequest; its stream id is its index."""
        return self.submit(q.robot, q.bc, q.obs, q.n_samples, q.n_steps, q.horizon, wl.n_cem,
                           wl.n_proj_iters, q.n_proj, q.n_elite, warm_start=warm_start,
                           stream_id=q.index, arrival=t0 + q.arrival)

    def step(self) -> int:
        return P.priest_server_step(self.handle)

    def poll(self, max_results=1024):
        out = []
        for r in P.priest_server_poll(self.handle, max_results):
            out.append(Completed(r.request_id, r.robot, r.status, r.arrival, r.t_admit, r.t_done,
                                 r.best_cost, np.ctypeslib.as_array(r.best_xi)[:self.D].copy()))
        return out

    def flush(self):
        P.priest_server_flush(self.handle)

    def counts(self):
        return P.priest_server_counts(self.handle)

    def stats(self) -> dict:
        return P.priest_server_stats_get(self.handle)

    def robot_state(self, robot):
        mu, cov = P.priest_server_robot_state(self.handle, robot, self.D)
        return np.array(mu, dtype=np.float32), np.array(cov, dtype=np.float32).reshape(self.D, self.D)

    def drain(self, max_steps=1_000_000):
        """Steps until nothing is pending or active; returns completions."""
        done = []
        for _ in range(max_steps):
            n = self.step()
            done += self.poll()
            pend, act, _ = self.counts()
            if n == 0 and pend == 0 and act == 0:
                break
        self.flush()
        done += self.poll()
        return done


def _latency_summary(lat_s, wall_s, n):
    lat_ms = np.sort(np.asarray(lat_s) * 1e3)
    return {
        "requests": int(n),
        "wall_s": round(wall_s, 4),
        "plans_per_s": round(n / wall_s, 2) if wall_s > 0 else None,
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                       "p99": round(float(np.percentile(lat_ms, 99)), 3),
                       "max": round(float(lat_ms[-1]), 3)},
    }


def prepare_shapes(server: Server, requests):
    for key in sorted({(q.n_steps, q.n_obs, q.horizon) for q in requests}):
        server.prepare(*key)


def run_stream(server: Server, requests, wl: ServingWorkload = C5, realtime=True):
    """Replays `requests` (ordered by arrival).  realtime=True submits each
    request when the host clock reaches its arrival time; False submits all
    at once (offline throughput).  Returns (summary, completions)."""
    now = P.priest_server_now
    t0 = now() + 0.01
    i, n = 0, len(requests)
    done = []
    while len(done) < n:
        t = now()
        while i < n and (not realtime or t0 + requests[i].arrival <= t):
            server.submit_request(requests[i], wl, t0 if realtime else 0.0)
            i += 1
        stepped = server.step()
        done += server.poll()
        if stepped == 0 and i < n:
            # idle: wait for the next arrival
            wait = t0 + requests[i].arrival - now()
            if wait > 0:
                time.sleep(min(wait, 1e-3))
        elif stepped == 0 and i == n:
            server.flush()
            done += server.poll()
    wall = max(c.t_done for c in done) - (t0 if realtime else min(c.t_admit for c in done))
    lat = [c.t_done - c.arrival for c in done] if realtime else [c.t_done - c.t_admit for c in done]
    summary = _latency_summary(lat, wall, n)
    last_arrival = requests[-1].arrival
    summary["offered_req_per_s"] = round(n / last_arrival, 1) if realtime and last_arrival > 0 else None
    summary["kept_up"] = bool(realtime and summary["latency_ms"]["p99"] < 1e3 * wl.mean_period)
    st = server.stats()
    summary["sample_iters_per_s"] = round(st["sample_iters"] / wall, 1)
    summary["max_active"] = st["max_active_seen"]
    summary["arena_high_water_mb"] = round(st["arena_high_water"] / 2**20, 2)
    summary["steps"] = st["steps"]
    return summary, done


def initial_state(wl: ServingWorkload, bc: np.ndarray):
    """The reset warm start the server uses (straight line start -> goal,
    init_std^2 I), built the same way in float32."""
    nv = wl.n_coeff
    mu = np.zeros(wl.dims * nv, dtype=np.float32)
    for ax in range(wl.dims):
        p0 = np.float32(bc[ax, 0])
        pf = np.float32(bc[ax, 3])
        for c in range(nv):
            mu[ax * nv + c] = p0 + (pf - p0) * np.float32(c) / np.float32(nv - 1)
    cov = np.eye(wl.dims * nv, dtype=np.float32) * np.float32(wl.init_std) ** 2
    return mu, cov


def run_plain(requests, wl: ServingWorkload = C5, realtime=True, seed=0, time_limit=None):
    """One priest_plan call per request, FIFO, synchronised after each (no
    batching across requests, no graph): the plain form of the service.
    Robots keep their (mu, Sigma) between requests as the server does.
    Returns (summary, {index: (best_xi, best_cost)})."""
    dev = torch.device("cuda")
    probs = {}
    D = wl.dims * wl.n_coeff
    state = {}
    results = {}
    for q in requests:
        key = (q.n_steps, q.n_obs, q.horizon)
        if key not in probs:
            probs[key] = P.Problem(wl.dims, wl.n_coeff, q.n_steps, q.horizon, q.n_obs, rho=wl.rho,
                                   v_max=wl.v_max, a_max=wl.a_max, bc_mask=wl.bc_mask)
            probs[key].set_tiling((4, 1, 0))   # the plain form: default shape, no tuning
    torch.cuda.synchronize()
    now = time.perf_counter
    t0 = now() + 0.01
    lat = []
    n_done = 0
    sample_iters = 0
    for q in requests:
        if time_limit is not None and now() - t0 > time_limit:
            break
        if realtime:
            wait = t0 + q.arrival - now()
            if wait > 0:
                time.sleep(wait)
        prob = probs[(q.n_steps, q.n_obs, q.horizon)]
        if q.robot not in state:
            mu, cov = initial_state(wl, q.bc)
            state[q.robot] = (torch.from_numpy(mu).to(dev), torch.from_numpy(cov).to(dev))
        mu_t, cov_t = state[q.robot]
        cem = P.Cem(q.n_samples, wl.n_cem, wl.n_proj_iters, q.n_proj, q.n_elite, wl.sigma,
                    wl.gamma, wl.cov_jitter)
        bc_t = torch.tensor(q.bc, dtype=torch.float32, device=dev)
        obs_t = torch.tensor(q.obs, dtype=torch.float32, device=dev).reshape(-1, 8)
        out = prob.plan_outputs(cem, full=False)
        prob.plan(bc_t, obs_t, cem, mu_t, cov_t, seed=seed, stream_id=q.index, out=out)
        best = out["best_xi"][0].cpu().numpy()
        cost = float(out["best_cost"][0].cpu())
        t_done = now()
        results[q.index] = (best, cost)
        lat.append(t_done - (t0 + q.arrival) if realtime else 0.0)
        n_done += 1
        sample_iters += q.n_samples * wl.n_proj_iters * wl.n_cem
    wall = now() - t0
    summary = _latency_summary(lat, wall, n_done)
    summary["sample_iters_per_s"] = round(sample_iters / wall, 1)
    summary["completed_within_limit"] = n_done
    for p in probs.values():
        p.close()
    return summary, results
