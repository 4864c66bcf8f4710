"""Thin ctypes binding of libpriest.so (include/priest.h).

Functions keep the C names and only marshal arguments: torch tensors become
device pointers, the current torch stream becomes the hipStream_t, and a
non-zero status becomes a :class:`PriestError`.  Every step of the planner
runs in the library's HIP kernels; if the library is not built the first
call raises instead of falling back to anything else.

:class:`Problem` is a convenience wrapper that allocates outputs with torch.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpriest.so")

PRIEST_OK = 0
PRIEST_ERR_INVALID = -1
PRIEST_ERR_SINGULAR = -2
PRIEST_ERR_NOMEM = -3
PRIEST_ERR_DEVICE = -4
PRIEST_ERR_NONFINITE = -5

BC_P0, BC_V0, BC_A0, BC_PF, BC_VF, BC_AF = 1, 2, 4, 8, 16, 32
BC_DEFAULT = BC_P0 | BC_V0 | BC_A0 | BC_PF
BC_REST = BC_DEFAULT | BC_VF | BC_AF
FP32, BF16_MIXED = 0, 1

EXPORTS = (
    "priest_init_problem", "priest_free_problem", "priest_problem_dim", "priest_project",
    "priest_plan_workspace_size", "priest_plan", "priest_plan_batch", "priest_debug_offsets",
    "priest_debug_normals", "priest_debug_constants", "priest_last_error", "priest_version",
    "priest_server_now", "priest_server_create", "priest_server_prepare", "priest_server_submit",
    "priest_server_step", "priest_server_poll", "priest_server_flush", "priest_server_counts",
    "priest_server_stats_get", "priest_server_robot_state", "priest_server_destroy",
    "priest_tiling_candidates", "priest_set_tiling", "priest_last_tiling",
    "priest_profile_enable", "priest_profile_read", "priest_project_unfused_workspace_size",
    "priest_project_unfused", "priest_plan_dpriest", "priest_profile_count_pairs",
    "priest_profile_read_pairs", "priest_project_hist", "priest_project_batch",
    "priest_debug_select", "priest_plan_static",
)

WARM_RESET, WARM_KEEP, WARM_KEEP_MEAN = 0, 1, 2
MAX_D = 48


class ProblemDesc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32), ("n_coeff", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("n_obs", ctypes.c_int32),
                ("horizon", ctypes.c_double), ("rho", ctypes.c_double),
                ("v_max", ctypes.c_double), ("a_max", ctypes.c_double),
                ("bc_mask", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("n_refine_fp32", ctypes.c_int32), ("use_bounds", ctypes.c_int32),
                ("s_min", ctypes.c_double * 3), ("s_max", ctypes.c_double * 3),
                ("obs_model", ctypes.c_int32), ("reserved2", ctypes.c_int32)]


class CostParams(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("w_acc", ctypes.c_float), ("w_curv", ctypes.c_float),
                ("w_path", ctypes.c_float), ("w_steer", ctypes.c_float),
                ("wheelbase", ctypes.c_float), ("eps", ctypes.c_float),
                ("reserved", ctypes.c_int32)]


class CemParams(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int32), ("n_cem", ctypes.c_int32),
                ("n_proj_iters", ctypes.c_int32), ("n_proj", ctypes.c_int32),
                ("n_elite", ctypes.c_int32), ("update", ctypes.c_int32),
                ("sigma", ctypes.c_float), ("gamma", ctypes.c_float),
                ("cov_jitter", ctypes.c_float), ("reserved_f", ctypes.c_float),
                ("cost", CostParams)]


COST_SMOOTH, COST_WEIGHTED = 0, 1
OBS_VELOCITY, OBS_PATH = 0, 1
UPDATE_MPPI, UPDATE_CMA = 0, 1


@dataclass
class Cost:
    """c1 of Alg. 1: kind COST_SMOOTH (sum ||a||^2) or COST_WEIGHTED (the
    weighted navigation terms of priest_cost)."""
    kind: int = COST_SMOOTH
    w_acc: float = 1.0
    w_curv: float = 0.0
    w_path: float = 0.0
    w_steer: float = 0.0
    wheelbase: float = 1.0
    eps: float = 1e-2

    def c(self) -> CostParams:
        return CostParams(self.kind, self.w_acc, self.w_curv, self.w_path, self.w_steer,
                          self.wheelbase, self.eps, 0)


class PlanOut(ctypes.Structure):
    _fields_ = [("best_xi", ctypes.c_void_p), ("best_cost", ctypes.c_void_p),
                ("elite_idx", ctypes.c_void_p), ("proj_idx", ctypes.c_void_p),
                ("xi", ctypes.c_void_p), ("xi_bar", ctypes.c_void_p),
                ("resid", ctypes.c_void_p), ("c1", ctypes.c_void_p),
                ("status", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32), ("n_coeff", ctypes.c_int32),
                ("bc_mask", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("n_refine_fp32", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("max_robots", ctypes.c_int32), ("max_inflight_steps", ctypes.c_int32),
                ("dry_run", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("rho", ctypes.c_double), ("v_max", ctypes.c_double), ("a_max", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("memory_budget", ctypes.c_uint64),
                ("sigma", ctypes.c_float), ("gamma", ctypes.c_float),
                ("cov_jitter", ctypes.c_float), ("init_std", ctypes.c_float)]


class Request(ctypes.Structure):
    _fields_ = [("robot", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("n_obs", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("n_cem", ctypes.c_int32), ("n_proj_iters", ctypes.c_int32),
                ("n_proj", ctypes.c_int32), ("n_elite", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("stream_id", ctypes.c_uint32),
                ("horizon", ctypes.c_double), ("arrival", ctypes.c_double),
                ("bc", ctypes.c_void_p), ("obs", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_int64), ("robot", ctypes.c_int32),
                ("status", ctypes.c_int32), ("arrival", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("best_cost", ctypes.c_float), ("best_xi", ctypes.c_float * MAX_D)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "submitted", "admitted", "completed", "steps", "max_active_seen", "arena_used",
        "arena_budget", "arena_high_water", "sample_iters")]


class Tiling(ctypes.Structure):
    _fields_ = [("axis_slots", ctypes.c_int32), ("row_tiles", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_tuple(self):
        return (self.axis_slots, self.row_tiles, self.persistent)


class PriestError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"priest status {code}: {msg}")
        self.code = code


_LIB = None

_P = ctypes.c_void_p
_I = ctypes.c_int32
_SIGS = {
    "priest_init_problem": (_I, [ctypes.POINTER(ProblemDesc), _P, ctypes.POINTER(_P)]),
    "priest_free_problem": (_I, [_P]),
    "priest_problem_dim": (_I, [_P]),
    "priest_project": (_I, [_P, _P, _P, _P, _I, _I, _P, _P, _P, _P]),
    "priest_plan_workspace_size": (_I, [_P, ctypes.POINTER(CemParams), _I,
                                        ctypes.POINTER(ctypes.c_size_t)]),
    "priest_plan": (_I, [_P, _P, _P, ctypes.POINTER(CemParams), _P, _P, ctypes.c_uint64,
                         ctypes.c_uint32, _P, ctypes.POINTER(PlanOut), _P, ctypes.c_size_t, _P]),
    "priest_plan_static": (_I, [_P, _P, _P, ctypes.POINTER(CemParams), _P, _P, ctypes.c_uint64,
                                ctypes.c_uint32, _P, ctypes.POINTER(PlanOut), _P]),
    "priest_plan_batch": (_I, [_P, _I, _P, _P, ctypes.POINTER(CemParams), _P, _P, ctypes.c_uint64,
                               ctypes.c_uint32, _P, ctypes.POINTER(PlanOut), _P, ctypes.c_size_t,
                               _I, _P]),
    "priest_plan_dpriest": (_I, [_P, _I, _P, _P, ctypes.POINTER(CemParams), _P, _P, ctypes.c_uint64,
                                 ctypes.c_uint32, _P, ctypes.POINTER(PlanOut), _P, _P, _P, _P,
                                 ctypes.c_size_t, _P]),
    "priest_debug_offsets": (_I, [_P, _P, _P, _P, _I, _P, _P]),
    "priest_debug_normals": (_I, [ctypes.c_uint64, ctypes.c_uint32, _I, _I, _I, _P, _P]),
    "priest_debug_select": (_I, [_I, _I, _I, _P, _P, _P, _P, _P]),
    "priest_debug_constants": (_I, [_P, _I, _P, _I]),
    "priest_server_now": (ctypes.c_double, []),
    "priest_server_create": (_I, [ctypes.POINTER(ServerConfig), _P, ctypes.POINTER(_P)]),
    "priest_server_prepare": (_I, [_P, _I, _I, ctypes.c_double]),
    "priest_server_submit": (_I, [_P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_int64)]),
    "priest_server_step": (_I, [_P, ctypes.POINTER(_I)]),
    "priest_server_poll": (_I, [_P, ctypes.POINTER(Result), _I, ctypes.POINTER(_I)]),
    "priest_server_flush": (_I, [_P]),
    "priest_server_counts": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "priest_server_stats_get": (_I, [_P, ctypes.POINTER(ServerStats)]),
    "priest_server_robot_state": (_I, [_P, _I, _P, _P]),
    "priest_server_destroy": (_I, [_P]),
    "priest_tiling_candidates": (_I, [_P, ctypes.POINTER(Tiling), _I, ctypes.POINTER(_I)]),
    "priest_set_tiling": (_I, [_P, ctypes.POINTER(Tiling)]),
    "priest_last_tiling": (_I, [_P, ctypes.POINTER(Tiling), ctypes.POINTER(_I)]),
    "priest_project_unfused_workspace_size": (_I, [_P, _I, ctypes.POINTER(ctypes.c_size_t)]),
    "priest_project_unfused": (_I, [_P, _P, _P, _P, _I, _I, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "priest_profile_enable": (_I, [_I]),
    "priest_profile_read": (_I, [ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_double)]),
    "priest_profile_count_pairs": (_I, [_I]),
    "priest_project_hist": (_I, [_P, _P, _P, _P, _I, _I, _P, _P, _P, _P, _P]),
    "priest_project_batch": (_I, [_P, _I, _P, _P, _P, _I, _I, _P, _P, _P, _P]),
    "priest_profile_read_pairs": (_I, [ctypes.POINTER(ctypes.c_uint64)]),
    "priest_last_error": (ctypes.c_char_p, []),
    "priest_version": (_I, []),
}


def lib():
    """Loads libpriest.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2309_08235_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = handle
    return _LIB


def _check(rc: int):
    if rc != PRIEST_OK:
        raise PriestError(rc, lib().priest_last_error().decode())


def _ptr(t, dtype=torch.float32):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# ---------------------------------------------------------------------------
# C-named functions
# ---------------------------------------------------------------------------
def priest_init_problem(desc: ProblemDesc, stream=None):
    h = ctypes.c_void_p()
    _check(lib().priest_init_problem(ctypes.byref(desc), _stream(stream), ctypes.byref(h)))
    return h


def priest_free_problem(handle):
    _check(lib().priest_free_problem(handle))


def priest_problem_dim(handle) -> int:
    return lib().priest_problem_dim(handle)


def priest_project(handle, bc, obs, xi_in, n_iter, xi_out, resid=None, c1=None, stream=None):
    _check(lib().priest_project(handle, _ptr(bc), _ptr(obs), _ptr(xi_in), xi_in.shape[0], n_iter,
                                _ptr(xi_out), _ptr(resid), _ptr(c1), _stream(stream)))


def priest_project_unfused_workspace_size(handle, N: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().priest_project_unfused_workspace_size(handle, N, ctypes.byref(n)))
    return n.value


def priest_project_unfused(handle, bc, obs, xi_in, n_iter, xi_out, resid, c1, workspace,
                           stream=None):
    _check(lib().priest_project_unfused(handle, _ptr(bc), _ptr(obs), _ptr(xi_in), xi_in.shape[0],
                                        n_iter, _ptr(xi_out), _ptr(resid), _ptr(c1),
                                        _ptr(workspace, torch.uint8), workspace.numel(),
                                        _stream(stream)))


def priest_plan_workspace_size(handle, params: CemParams, n_problems: int = 1) -> int:
    n = ctypes.c_size_t()
    _check(lib().priest_plan_workspace_size(handle, ctypes.byref(params), n_problems, ctypes.byref(n)))
    return n.value


def _plan_out(out: dict) -> PlanOut:
    po = PlanOut()
    for name, dtype in (("best_xi", torch.float32), ("best_cost", torch.float32),
                        ("elite_idx", torch.int32), ("proj_idx", torch.int32),
                        ("xi", torch.float32), ("xi_bar", torch.float32),
                        ("resid", torch.float32), ("c1", torch.float32), ("status", torch.int32)):
        setattr(po, name, _ptr(out.get(name), dtype))
    return po


def priest_plan(handle, bc, obs, params: CemParams, mu, cov, seed, stream_id, noise, out: dict,
                workspace, stream=None):
    po = _plan_out(out)
    _check(lib().priest_plan(handle, _ptr(bc), _ptr(obs), ctypes.byref(params), _ptr(mu), _ptr(cov),
                             seed, stream_id, _ptr(noise), ctypes.byref(po),
                             _ptr(workspace, torch.uint8), workspace.numel(), _stream(stream)))


def priest_plan_static(handle, bc, obs, params: CemParams, mu, cov, seed, stream_id, noise,
                       out: dict, stream=None):
    po = _plan_out(out)
    _check(lib().priest_plan_static(handle, _ptr(bc), _ptr(obs), ctypes.byref(params), _ptr(mu),
                                    _ptr(cov), seed, stream_id, _ptr(noise), ctypes.byref(po),
                                    _stream(stream)))


def priest_plan_batch(handle, n_problems, bc, obs, params: CemParams, mu, cov, seed, stream_base,
                      noise, out: dict, workspace, use_graph=False, stream=None):
    po = _plan_out(out)
    _check(lib().priest_plan_batch(handle, n_problems, _ptr(bc), _ptr(obs), ctypes.byref(params),
                                   _ptr(mu), _ptr(cov), seed, stream_base, _ptr(noise),
                                   ctypes.byref(po), _ptr(workspace, torch.uint8),
                                   workspace.numel(), int(bool(use_graph)), _stream(stream)))


def priest_plan_dpriest(handle, n_groups, bc, obs, params: CemParams, mu, cov, seed, stream_base,
                        noise, out: dict, best_xi, best_cost, best_group, workspace, stream=None):
    po = _plan_out(out)
    _check(lib().priest_plan_dpriest(handle, n_groups, _ptr(bc), _ptr(obs), ctypes.byref(params),
                                     _ptr(mu), _ptr(cov), seed, stream_base, _ptr(noise),
                                     ctypes.byref(po), _ptr(best_xi), _ptr(best_cost),
                                     _ptr(best_group, torch.int32), _ptr(workspace, torch.uint8),
                                     workspace.numel(), _stream(stream)))


def priest_debug_offsets(handle, bc, obs, xi, offsets, stream=None):
    _check(lib().priest_debug_offsets(handle, _ptr(bc), _ptr(obs), _ptr(xi), xi.shape[0],
                                      _ptr(offsets), _stream(stream)))


def priest_debug_normals(seed, stream_id, it, z, stream=None):
    _check(lib().priest_debug_normals(seed, stream_id, it, z.shape[0], z.shape[1], _ptr(z),
                                      _stream(stream)))


def priest_debug_select(n_proj, n_elite, r, c1, elite_idx, proj_idx=None, stream=None):
    """The refit kernel's two selections on r, c1 [N] (device, FP32): fills
    elite_idx [n_elite] and, if given, proj_idx [n_proj] (device, int32)."""
    _check(lib().priest_debug_select(r.shape[0], n_proj, n_elite, _ptr(r), _ptr(c1),
                                     _ptr(elite_idx, torch.int32), _ptr(proj_idx, torch.int32),
                                     _stream(stream)))


def priest_debug_constants(handle, which: int, count: int):
    buf = (ctypes.c_float * count)()
    _check(lib().priest_debug_constants(handle, which, buf, count))
    return list(buf)


def priest_tiling_candidates(handle):
    n = _I()
    _check(lib().priest_tiling_candidates(handle, None, 0, ctypes.byref(n)))
    buf = (Tiling * n.value)()
    _check(lib().priest_tiling_candidates(handle, buf, n.value, ctypes.byref(n)))
    return [buf[i].as_tuple() for i in range(n.value)]


def priest_set_tiling(handle, tiling=None):
    """tiling: (axis_slots, row_tiles, persistent) or None for autotuning."""
    if tiling is None:
        _check(lib().priest_set_tiling(handle, None))
    else:
        t = Tiling(*tiling, 0)
        _check(lib().priest_set_tiling(handle, ctypes.byref(t)))


def priest_last_tiling(handle):
    t = Tiling()
    tuned = _I()
    _check(lib().priest_last_tiling(handle, ctypes.byref(t), ctypes.byref(tuned)))
    return t.as_tuple(), bool(tuned.value)


def priest_profile_enable(on: bool = True):
    _check(lib().priest_profile_enable(int(bool(on))))


def priest_profile_read():
    """(launches, total_ms) of projection launches since the previous read."""
    n = _I()
    ms = ctypes.c_double()
    _check(lib().priest_profile_read(ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def priest_project_batch(handle, bc, obs, xi_in, n_iter, xi_out, resid, c1, stream=None):
    """xi_in [P, N, D]; bc [P, dims, 6]; obs [P, n_obs, row]."""
    P_, N = xi_in.shape[0], xi_in.shape[1]
    _check(lib().priest_project_batch(handle, P_, _ptr(bc), _ptr(obs), _ptr(xi_in), N, n_iter,
                                      _ptr(xi_out), _ptr(resid), _ptr(c1), _stream(stream)))


def priest_project_hist(handle, bc, obs, xi_in, n_iter, xi_out, resid, c1, resid_hist, stream=None):
    N = xi_in.shape[0]
    _check(lib().priest_project_hist(handle, _ptr(bc), _ptr(obs), _ptr(xi_in), N, n_iter,
                                     _ptr(xi_out), _ptr(resid), _ptr(c1), _ptr(resid_hist),
                                     _stream(stream)))


def priest_profile_count_pairs(on: bool):
    _check(lib().priest_profile_count_pairs(1 if on else 0))


def priest_profile_read_pairs() -> int:
    """(sample, step, obstacle) pairs evaluated by fused projection launches
    since the previous read (synchronises the device)."""
    v = ctypes.c_uint64()
    _check(lib().priest_profile_read_pairs(ctypes.byref(v)))
    return v.value


def priest_server_now() -> float:
    return lib().priest_server_now()


def priest_server_create(cfg: ServerConfig, stream=None):
    """`stream`: a torch stream, or None for the current stream (dry-run
    servers take no stream)."""
    h = ctypes.c_void_p()
    st = None if cfg.dry_run else _stream(stream)
    _check(lib().priest_server_create(ctypes.byref(cfg), st, ctypes.byref(h)))
    return h


def priest_server_prepare(server, n_steps, n_obs, horizon):
    _check(lib().priest_server_prepare(server, n_steps, n_obs, horizon))


def priest_server_submit(server, req: Request) -> int:
    rid = ctypes.c_int64()
    _check(lib().priest_server_submit(server, ctypes.byref(req), ctypes.byref(rid)))
    return rid.value


def priest_server_step(server) -> int:
    n = _I()
    _check(lib().priest_server_step(server, ctypes.byref(n)))
    return n.value


def priest_server_poll(server, max_results=256):
    buf = (Result * max_results)()
    n = _I()
    _check(lib().priest_server_poll(server, buf, max_results, ctypes.byref(n)))
    return [buf[i] for i in range(n.value)]


def priest_server_flush(server):
    _check(lib().priest_server_flush(server))


def priest_server_counts(server):
    p, a, f = _I(), _I(), _I()
    _check(lib().priest_server_counts(server, ctypes.byref(p), ctypes.byref(a), ctypes.byref(f)))
    return p.value, a.value, f.value


def priest_server_stats_get(server) -> dict:
    st = ServerStats()
    _check(lib().priest_server_stats_get(server, ctypes.byref(st)))
    return {n: getattr(st, n) for n, _ in ServerStats._fields_}


def priest_server_robot_state(server, robot: int, D: int):
    mu = (ctypes.c_float * D)()
    cov = (ctypes.c_float * (D * D))()
    _check(lib().priest_server_robot_state(server, robot, mu, cov))
    return list(mu), list(cov)


def priest_server_destroy(server):
    _check(lib().priest_server_destroy(server))


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------
@dataclass
class Cem:
    n_samples: int
    n_cem: int
    n_proj_iters: int
    n_proj: int
    n_elite: int
    sigma: float = 0.5
    gamma: float = 1.0
    cov_jitter: float = 1e-5
    cost: Cost = None
    update: int = UPDATE_MPPI

    def c(self) -> CemParams:
        return CemParams(self.n_samples, self.n_cem, self.n_proj_iters, self.n_proj,
                         self.n_elite, self.update, self.sigma, self.gamma, self.cov_jitter,
                         0.0, (self.cost or Cost()).c())


class Problem:
    """Owns a priest_problem handle; methods take/return torch tensors on the GPU."""

    def __init__(self, dims, n_coeff, n_steps, horizon, n_obs, rho=1.0, v_max=math.inf,
                 a_max=math.inf, bc_mask=BC_DEFAULT, precision=FP32, n_refine_fp32=10,
                 s_min=None, s_max=None, obs_model=0, stream=None):
        """s_min / s_max (per axis, both or neither): workspace bounds.
        obs_model OBS_PATH: obstacle rows are paths [K * dims] + (a, b)."""
        if (s_min is None) != (s_max is None):
            raise ValueError("give both s_min and s_max, or neither")
        lo = (ctypes.c_double * 3)(*(list(s_min or ()) + [0.0] * 3)[:3])
        hi = (ctypes.c_double * 3)(*(list(s_max or ()) + [0.0] * 3)[:3])
        self.desc = ProblemDesc(dims, n_coeff, n_steps, n_obs, horizon, rho, v_max, a_max,
                                bc_mask, precision, n_refine_fp32, 0 if s_min is None else 1,
                                lo, hi, obs_model, 0)
        self.dims, self.n_coeff, self.n_steps, self.n_obs = dims, n_coeff, n_steps, n_obs
        self.D = dims * n_coeff
        self.handle = priest_init_problem(self.desc, stream)

    @classmethod
    def from_workload(cls, wl, **kw):
        d = dict(dims=wl.dims, n_coeff=wl.n_coeff, n_steps=wl.n_steps, horizon=wl.horizon,
                 n_obs=wl.n_obs, rho=wl.rho, v_max=wl.v_max, a_max=wl.a_max, bc_mask=wl.bc_mask)
        d.update(kw)
        return cls(**d)

    def close(self):
        if self.handle is not None and self.handle.value:
            priest_free_problem(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tiling_candidates(self):
        return priest_tiling_candidates(self.handle)

    def set_tiling(self, tiling=None):
        priest_set_tiling(self.handle, tiling)

    def last_tiling(self):
        return priest_last_tiling(self.handle)

    def project(self, bc, obs, xi, n_iter, stream=None):
        N = xi.shape[0]
        dev = xi.device
        xo = torch.empty_like(xi)
        r = torch.empty(N, device=dev, dtype=torch.float32)
        c1 = torch.empty(N, device=dev, dtype=torch.float32)
        priest_project(self.handle, bc, obs, xi, n_iter, xo, r, c1, stream)
        return xo, r, c1

    def project_batch(self, bc, obs, xi, n_iter, stream=None):
        """priest_project_batch: xi [P, N, D] -> (xi_out, resid [P, N], c1 [P, N])."""
        P_, N = xi.shape[0], xi.shape[1]
        xo = torch.empty_like(xi)
        r = torch.empty((P_, N), device=xi.device, dtype=torch.float32)
        c1 = torch.empty((P_, N), device=xi.device, dtype=torch.float32)
        priest_project_batch(self.handle, bc, obs, xi, n_iter, xo, r, c1, stream)
        return xo, r, c1

    def project_hist(self, bc, obs, xi, n_iter, stream=None):
        """priest_project_hist: (xi_out, resid, c1, resid_hist [n_iter, N])."""
        N = xi.shape[0]
        xo = torch.empty_like(xi)
        r = torch.empty(N, device=xi.device, dtype=torch.float32)
        c1 = torch.empty(N, device=xi.device, dtype=torch.float32)
        h = torch.empty((max(n_iter, 1), N), device=xi.device, dtype=torch.float32)
        priest_project_hist(self.handle, bc, obs, xi, n_iter, xo, r, c1, h, stream)
        return xo, r, c1, h[:n_iter]

    def project_unfused(self, bc, obs, xi, n_iter, workspace=None, stream=None):
        """The plain unfused form of project() (baseline)."""
        N = xi.shape[0]
        dev = xi.device
        if workspace is None:
            workspace = torch.empty(priest_project_unfused_workspace_size(self.handle, N),
                                    dtype=torch.uint8, device=dev)
        xo = torch.empty_like(xi)
        r = torch.empty(N, device=dev, dtype=torch.float32)
        c1 = torch.empty(N, device=dev, dtype=torch.float32)
        priest_project_unfused(self.handle, bc, obs, xi, n_iter, xo, r, c1, workspace, stream)
        return xo, r, c1

    def offsets(self, bc, obs, xi, stream=None):
        out = torch.empty((xi.shape[0], self.n_obs + 2, self.n_steps, self.dims),
                          device=xi.device, dtype=torch.float32)
        priest_debug_offsets(self.handle, bc, obs, xi, out, stream)
        return out

    def constants(self):
        nv, K = self.n_coeff, self.n_steps
        import numpy as np
        return {
            "M11": np.array(priest_debug_constants(self.handle, 0, nv * nv)).reshape(nv, nv),
            "Pi": np.array(priest_debug_constants(self.handle, 1, nv * nv)).reshape(nv, nv),
            "M12": np.array(priest_debug_constants(self.handle, 2, nv * 6)).reshape(nv, 6),
            "W": np.array(priest_debug_constants(self.handle, 3, K * 3 * nv)).reshape(K, 3, nv),
        }

    def plan_outputs(self, cem: Cem, n_problems=1, full=True, device="cuda"):
        P, N, D = n_problems, cem.n_samples, self.D
        f = dict(device=device, dtype=torch.float32)
        i = dict(device=device, dtype=torch.int32)
        out = {"best_xi": torch.empty((P, D), **f), "best_cost": torch.empty(P, **f),
               "elite_idx": torch.empty((P, cem.n_elite), **i),
               "proj_idx": torch.empty((P, cem.n_proj), **i), "status": torch.empty(P, **i)}
        if full:
            out.update({"xi": torch.empty((P, N, D), **f), "xi_bar": torch.empty((P, N, D), **f),
                        "resid": torch.empty((P, N), **f), "c1": torch.empty((P, N), **f)})
        return out

    def workspace(self, cem: Cem, n_problems=1, device="cuda"):
        n = priest_plan_workspace_size(self.handle, cem.c(), n_problems)
        return torch.empty(n, dtype=torch.uint8, device=device)

    def plan(self, bc, obs, cem: Cem, mu, cov, seed=0, stream_id=0, noise=None, out=None,
             workspace=None, stream=None):
        """Runs Alg. 1 in place on (mu, cov); returns the output dict."""
        out = out if out is not None else self.plan_outputs(cem)
        ws = workspace if workspace is not None else self.workspace(cem)
        priest_plan(self.handle, bc, obs, cem.c(), mu, cov, seed, stream_id, noise, out, ws, stream)
        return out

    def plan_dpriest(self, n_groups, bc, obs, cem: Cem, mu, cov, seed=0, stream_base=0,
                     noise=None, out=None, workspace=None, stream=None, full=False):
        """D-PRIEST on one scene: returns (best_xi [D], best_cost [1],
        best_group [1], per-group outputs)."""
        out = out if out is not None else self.plan_outputs(cem, n_groups, full=full)
        ws = workspace if workspace is not None else self.workspace(cem, n_groups)
        dev = mu.device
        best_xi = torch.empty(self.D, device=dev, dtype=torch.float32)
        best_cost = torch.empty(1, device=dev, dtype=torch.float32)
        best_group = torch.empty(1, device=dev, dtype=torch.int32)
        priest_plan_dpriest(self.handle, n_groups, bc, obs, cem.c(), mu, cov, seed, stream_base,
                            noise, out, best_xi, best_cost, best_group, ws, stream)
        return best_xi, best_cost, best_group, out

    def plan_batch(self, n_problems, bc, obs, cem: Cem, mu, cov, seed=0, stream_base=0,
                   noise=None, out=None, workspace=None, use_graph=False, stream=None):
        out = out if out is not None else self.plan_outputs(cem, n_problems)
        ws = workspace if workspace is not None else self.workspace(cem, n_problems)
        priest_plan_batch(self.handle, n_problems, bc, obs, cem.c(), mu, cov, seed, stream_base,
                          noise, out, ws, use_graph, stream)
        return out
