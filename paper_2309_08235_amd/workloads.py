"""Seeded synthetic planning inputs shaped like the paper's benchmarks.

This module generates inputs only: scenes (boundary values, obstacles),
initial sampling distributions and standard-normal draws.  It holds none of
the method's arithmetic, imports neither the HIP binding nor the oracle, and
is the one piece both sides of a parity test share.

Shapes follow the point-to-point benchmarks of Sec. V-A (random circular /
spherical obstacles between a start and a goal, start and goal at rest) and
the dynamic benchmark (constant-velocity obstacles).  The paper's own scenes
are not published; these seeded generators stand in for them.

Array conventions (float64 here; the binding converts to float32):
  bc  [dims, 6]   per axis (p0, v0, a0, pf, vf, af)
  obs [M, 8]      (cx, cy, cz, vx, vy, vz, a, b): centre at t=0, constant
                  velocity, semi-axes (a, a, b); circles/spheres have a == b
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BC_P0, BC_V0, BC_A0, BC_PF, BC_VF, BC_AF = 1, 2, 4, 8, 16, 32
BC_DEFAULT = BC_P0 | BC_V0 | BC_A0 | BC_PF
BC_REST = BC_DEFAULT | BC_VF | BC_AF


@dataclass
class Workload:
    name: str
    dims: int
    n_coeff: int
    n_steps: int
    horizon: float
    n_obs: int
    v_max: float
    a_max: float
    bc_mask: int
    n_samples: int
    n_proj_iters: int
    n_cem: int
    n_proj: int
    n_elite: int
    rho: float = 1.0
    sigma: float = 0.5
    gamma: float = 1.0
    cov_jitter: float = 1e-5
    init_std: float = 1.0
    n_problems: int = 1
    start: tuple = (0.0, 0.0)
    goal: tuple = (10.0, 10.0)
    extra: dict = field(default_factory=dict)

    @property
    def D(self) -> int:
        return self.dims * self.n_coeff


def default_n_proj(n: int) -> int:
    """N_proj scaled from the paper's setting N_proj = 80 of N_b = 110 (Sec. V-A)."""
    return int(math.floor(n * 80 / 110 + 0.5))


def default_n_elite(n: int) -> int:
    """N_elite scaled from the paper's setting N_elite = 20 of N_b = 110."""
    return int(math.floor(n * 20 / 110 + 0.5))


# Configurations: C1 small parity case, C2 paper-scale single plan, C3 3D batch
C1 = Workload(name="c1_2d_k50_n64_m4", dims=2, n_coeff=11, n_steps=50, horizon=10.0,
              n_obs=4, v_max=1.5, a_max=2.0, bc_mask=BC_REST, n_samples=64,
              n_proj_iters=50, n_cem=1, n_proj=default_n_proj(64),
              n_elite=default_n_elite(64))
C2 = Workload(name="c2_2d_k100_n1000_m50", dims=2, n_coeff=11, n_steps=100, horizon=15.0,
              n_obs=50, v_max=1.5, a_max=2.0, bc_mask=BC_DEFAULT, n_samples=1000,
              n_proj_iters=100, n_cem=20, n_proj=default_n_proj(1000), n_elite=100)
C3 = Workload(name="c3_3d_k100_n2000_m128_x64", dims=3, n_coeff=11, n_steps=100,
              horizon=15.0, n_obs=128, v_max=2.0, a_max=3.0, bc_mask=BC_DEFAULT,
              n_samples=2000, n_proj_iters=100, n_cem=20,
              n_proj=default_n_proj(2000), n_elite=200, n_problems=64,
              start=(4.0, 4.0, 4.0), goal=(16.0, 16.0, 16.0))

CONFIGS = {"c1": C1, "c2": C2, "c3": C3}


def boundary_values(wl: Workload) -> np.ndarray:
    """Start and goal at rest: bc[axis] = (p0, 0, 0, pf, 0, 0)."""
    bc = np.zeros((wl.dims, 6))
    bc[:, 0] = wl.start[:wl.dims]
    bc[:, 3] = wl.goal[:wl.dims]
    return bc


def _far_enough(c, r, pts, margin):
    return all(np.linalg.norm(c - p) >= r + margin for p in pts)


def obstacles(wl: Workload, seed: int) -> np.ndarray:
    """Random obstacles for workload ``wl`` (PCG64 seeded).  Obstacles whose
    disk/ball comes within (radius + 1 m) of the start or goal are re-drawn."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = wl.dims
    start = np.array(wl.start[:d])
    goal = np.array(wl.goal[:d])
    obs = np.zeros((wl.n_obs, 8))
    for j in range(wl.n_obs):
        while True:
            if wl is C1 or wl.name.startswith("c1"):
                c = rng.uniform(2.0, 8.0, size=d)
                r = rng.uniform(0.3, 0.6)
                vel = np.zeros(d)
            elif d == 2:
                c = rng.uniform(0.5, 9.5, size=d)
                r = rng.uniform(0.2, 0.5)
                n_static = int(round(wl.n_obs * 0.6))
                if j >= n_static:
                    head = rng.uniform(0.0, 2.0 * np.pi)
                    speed = rng.uniform(0.0, 1.0)
                    vel = speed * np.array([np.cos(head), np.sin(head)])
                else:
                    vel = np.zeros(d)
            else:
                c = rng.uniform(0.0, 20.0, size=d)
                r = rng.uniform(0.2, 0.8)
                vel = np.zeros(d)
            if _far_enough(c, r, (start, goal), 1.0):
                break
        obs[j, :d] = c
        obs[j, 3:3 + d] = vel
        obs[j, 6] = r
        obs[j, 7] = r
    return obs


def time_stamps(wl: Workload) -> np.ndarray:
    """The planning time stamps of a scene, k T / (K - 1)."""
    return np.arange(wl.n_steps) * (wl.horizon / (wl.n_steps - 1))


def trajectory_obstacles(wl: Workload, obs: np.ndarray, swirl: float = 0.0,
                         seed: int = 0) -> np.ndarray:
    """Obstacles of ``obs`` ([M, 8] rows) given by their positions at every
    time stamp: [M, K * dims + 2] rows (positions step by step, then a, b).
    swirl = 0 reproduces the constant-velocity motion of ``obs``; swirl > 0
    adds a circular motion of that radius (random phase and angular speed
    up to 1 rad/s) on top, a path no constant velocity follows."""
    d, K = wl.dims, wl.n_steps
    t = time_stamps(wl)
    M = obs.shape[0]
    pos = obs[:, None, :d] + obs[:, None, 3:3 + d] * t[None, :, None]
    if swirl > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        ph = rng.uniform(0.0, 2.0 * np.pi, M)
        om = rng.uniform(-1.0, 1.0, M)
        ang = ph[:, None] + om[:, None] * t[None, :]
        pos[:, :, 0] += swirl * (np.cos(ang) - np.cos(ph)[:, None])
        pos[:, :, 1] += swirl * (np.sin(ang) - np.sin(ph)[:, None])
    out = np.zeros((M, K * d + 2))
    out[:, :K * d] = pos.reshape(M, K * d)
    out[:, -2] = obs[:, 6]
    out[:, -1] = obs[:, 7]
    return out


def initial_mean(wl: Workload) -> np.ndarray:
    """mu^0: coefficients spaced evenly on the start-goal segment, per axis."""
    n = wl.n_coeff - 1
    s = np.arange(wl.n_coeff) / n
    start = np.array(wl.start[:wl.dims])
    goal = np.array(wl.goal[:wl.dims])
    return (start[:, None] + (goal - start)[:, None] * s[None, :]).reshape(-1)


def initial_cov(wl: Workload) -> np.ndarray:
    """Sigma^0 = init_std^2 I."""
    return wl.init_std ** 2 * np.eye(wl.D)


def standard_normals(seed: int, shape) -> np.ndarray:
    """Standard-normal draws from PCG64 (used as the sampler's noise input)."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(shape)


def samples(wl: Workload, seed: int, n: int | None = None) -> np.ndarray:
    """Trajectory samples xi = mu^0 + init_std z, [n, D] (projection inputs)."""
    n = wl.n_samples if n is None else n
    z = standard_normals(seed, (n, wl.D))
    return initial_mean(wl)[None, :] + wl.init_std * z


def scene(wl: Workload, index: int = 0):
    """(bc, obs) for problem ``index`` of workload ``wl``: scene seed is
    1000 * config number + index."""
    cfg = {"c1": 1, "c2": 2, "c3": 3}.get(wl.name[:2], 9)
    return boundary_values(wl), obstacles(wl, 1000 * cfg + index)


def with_changes(wl: Workload, **kw) -> Workload:
    d = dict(wl.__dict__)
    d.update(kw)
    return Workload(**d)


# ---------------------------------------------------------------------------
# Serving stream (continuous batching): many robots re-planning on Poisson
# clocks with requests of mixed size.
# ---------------------------------------------------------------------------
@dataclass
class ServingWorkload:
    name: str = "c5_serving_2d_256robots"
    n_robots: int = 256
    n_requests: int = 4096
    mean_period: float = 0.1          # s between a robot's requests (Poisson clock)
    sizes: tuple = (256, 512, 1024, 2048)
    obs_range: tuple = (8, 128)       # M ~ U{lo..hi}
    steps: tuple = (50, 100)          # K fixed per robot
    horizons: tuple = (10.0, 15.0)    # T for K = 50 / 100
    dims: int = 2
    n_coeff: int = 11
    n_proj_iters: int = 20
    n_cem: int = 5
    v_max: float = 1.5
    a_max: float = 2.0
    rho: float = 1.0
    sigma: float = 0.5
    gamma: float = 1.0
    cov_jitter: float = 1e-5
    init_std: float = 1.0
    bc_mask: int = BC_DEFAULT
    seed: int = 5000


C5 = ServingWorkload()


@dataclass
class ServingRequest:
    index: int
    robot: int
    arrival: float      # s after the stream starts
    n_samples: int
    n_obs: int
    n_steps: int
    horizon: float
    n_proj: int
    n_elite: int
    bc: np.ndarray      # [dims, 6]
    obs: np.ndarray     # [n_obs, 8]


def _serving_scene(rng, dims, start, goal, n_obs):
    """Obstacles around the start-goal box; 60% static, 40% moving at
    constant velocity (as in the dynamic benchmark).  Candidates within
    (radius + 1 m) of the start or goal are dropped and re-drawn."""
    lo = np.minimum(start, goal) - 0.5
    hi = np.maximum(start, goal) + 0.5
    cs, rs = [], []
    while len(cs) < n_obs:
        c = rng.uniform(lo, hi, size=(2 * n_obs, dims))
        r = rng.uniform(0.2, 0.5, size=2 * n_obs)
        ok = ((np.linalg.norm(c - start, axis=1) >= r + 1.0) &
              (np.linalg.norm(c - goal, axis=1) >= r + 1.0))
        cs.extend(c[ok])
        rs.extend(r[ok])
    c = np.array(cs[:n_obs])
    r = np.array(rs[:n_obs])
    n_static = int(round(n_obs * 0.6))
    head = rng.uniform(0.0, 2.0 * np.pi, size=n_obs)
    speed = rng.uniform(0.0, 1.0, size=n_obs)
    speed[:n_static] = 0.0
    obs = np.zeros((n_obs, 8))
    obs[:, :dims] = c
    obs[:, 3] = speed * np.cos(head)
    obs[:, 4] = speed * np.sin(head)
    obs[:, 6] = r
    obs[:, 7] = r
    return obs


def serving_requests(wl: ServingWorkload = C5, n_requests: int | None = None,
                     n_robots: int | None = None, rate_scale: float = 1.0):
    """The request stream, ordered by arrival time.  Robot r has a fixed K
    (alternating 50/100), a fixed goal, and exponential inter-arrival times
    with mean mean_period / rate_scale; each request draws N and M
    independently and gets a fresh obstacle scene.  A robot's start moves a
    little toward its goal with every request."""
    n_requests = wl.n_requests if n_requests is None else n_requests
    n_robots = wl.n_robots if n_robots is None else n_robots
    rng = np.random.Generator(np.random.PCG64(wl.seed))
    d = wl.dims
    K = [wl.steps[r % len(wl.steps)] for r in range(n_robots)]
    T = [wl.horizons[r % len(wl.horizons)] for r in range(n_robots)]
    base = rng.uniform(0.0, 2.0, size=(n_robots, d))
    span = np.array([7.0 if k == wl.steps[0] else 10.0 for k in K])
    goal = base + span[:, None]
    # arrival times: per-robot Poisson clocks, merged
    per_robot = max(1, -(-n_requests // n_robots)) + 2
    gaps = rng.exponential(wl.mean_period / rate_scale, size=(n_robots, per_robot))
    times = np.cumsum(gaps, axis=1)
    events = sorted((times[r, j], r, j) for r in range(n_robots) for j in range(per_robot))
    events = events[:n_requests]
    out = []
    for i, (t, r, j) in enumerate(events):
        n = int(rng.choice(wl.sizes))
        m = int(rng.integers(wl.obs_range[0], wl.obs_range[1] + 1))
        frac = min(0.5, 0.02 * j)
        start = base[r] + frac * (goal[r] - base[r])
        bc = np.zeros((d, 6))
        bc[:, 0] = start
        bc[:, 3] = goal[r]
        obs = _serving_scene(rng, d, start, goal[r], m)
        out.append(ServingRequest(index=i, robot=r, arrival=float(t), n_samples=n, n_obs=m,
                                  n_steps=K[r], horizon=T[r], n_proj=default_n_proj(n),
                                  n_elite=default_n_elite(n), bc=bc, obs=obs))
    return out


def dpriest_means(wl: Workload, n_groups: int, spread: float = 1.5) -> np.ndarray:
    """Initial means of D-PRIEST's distributions: the straight control
    polygon of initial_mean() with its interior coefficients shifted
    sideways (perpendicular to start->goal in the x-y plane) by
    spread * (g - (G-1)/2), tapered to zero at both ends, so that the
    distributions start in different homotopy classes.  [G, D]."""
    base = initial_mean(wl).reshape(wl.dims, wl.n_coeff)
    start = np.array(wl.start[:wl.dims], np.float64)
    goal = np.array(wl.goal[:wl.dims], np.float64)
    d = goal - start
    nrm = np.zeros(wl.dims)
    nrm[0], nrm[1] = -d[1], d[0]
    nrm /= max(np.linalg.norm(nrm), 1e-12)
    taper = np.sin(np.pi * np.arange(wl.n_coeff) / (wl.n_coeff - 1))
    out = np.empty((n_groups, wl.D))
    for g in range(n_groups):
        off = spread * (g - (n_groups - 1) / 2.0)
        out[g] = (base + off * nrm[:, None] * taper[None, :]).reshape(-1)
    return out
