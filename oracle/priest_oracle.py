"""Plain FP64 CPU oracle of the PRIEST projection optimizer and its sampling loop.

TEST INFRASTRUCTURE ONLY.  This module exists to check the HIP implementation.
Only the test-suite, the package's smoke check and the CPU-baseline leg of the
benchmark may import it; the product path never calls it and shares no code
with it.  It is deliberately slow and literal:

* the constraint map F and target vector e are formed densely, exactly as the
  paper stacks them (Appendix, eq. (13) and the definition of F, e below
  eq. (14));
* the polar variables alpha, beta, d are computed with trigonometric functions
  and then turned back into targets, in the paper's order (eqs. (15a)-(15c));
* every projection iteration solves the full equality-constrained QP through
  its KKT system with ``numpy.linalg.solve`` (Sec. III-A, eqs. (7a)-(7b)).

Readings of passages that are silent, ambiguous or garbled in the paper:

* basis: Bernstein polynomials of degree n_coeff-1 on tau = t/T (Sec. II-A,
  eq. (2) leaves the basis open); derivative rows scaled by 1/T and 1/T^2;
* time grid: t_k = k T/(K-1), both ends included (Sec. II-A: rows 0 and -1 are
  the first and last planning steps);
* boundary rows: selected by a mask from {P_0, Pdot_0, Pddot_0, P_-1,
  Pdot_-1, Pddot_-1}; default = the paper's four rows (Sec. II-A, eq. (3b));
* sign of the F^T e term in eta: +rho F^T e, which is what the Lagrangian of
  eq. (14) gives; the printed minus sign in eq. (7b) contradicts eq. (14);
* multiplier update (eq. (15e)) uses the targets just computed from the
  current iterate, since eq. (6a) states h depends only on (xi_bar^k, lambda^k);
* xi_bar^0 = xi and lambda^0 = 0 for every projection call;
* alpha/beta/d closed forms: the radial (scaled) forms, which for circles and
  spheres (a = b) are the exact minimisers of eq. (14) over each variable and
  give the Euclidean projection onto the outside of the obstacle; a zero
  offset uses atan2(+0,+0) = 0, i.e. direction +x in 2D and +z in 3D;
* residual r(xi_bar) (Alg. 1, "compute the residuals"): Euclidean norm of
  F xi_bar - e(xi_bar), evaluated with max(0, .) violation terms so that it is
  exactly zero for a trajectory that satisfies every constraint on the grid;
* cost: c1 = sum_k ||a_k||^2 (point-to-point smoothness, Sec. V-A) and
  c_aug = c1 + r (Alg. 1); the optional navigation terms (Sec. V) are a
  curvature |v x a| / (|v|^2 + eps)^(3/2) squared, the Euclidean distance of
  each way-point to the start-goal segment (projection clamped to the
  segment, not squared), and the squared steering angle atan(L kappa) of a
  car-like robot (2D, signed curvature), summed over the grid;
* weight sign in eq. (9c): exp(-(c_aug - delta)/gamma), the MPPI convention
  (with the printed sign the worst elite would get the largest weight);
* CMA-ES-style update (the remark that the update rule is free): eq. (9a)
  for the mean; the covariance by the rank-one and rank-mu updates of CMA-ES
  with the eq. (9c) weights normalised, y about the current mean, Hansen's
  default rates for n = D, an evolution path that starts at zero on every
  plan call, and no step-size adaptation;
* covariance Cholesky jitter: eps = cov_jitter * tr(Sigma)/D added to the
  diagonal before factorising (elites lie on {A xi = b}, so Sigma loses rank);
* selection ties broken by sample index (stable sort), NaN ranked as +inf;
* workspace bounds (Appendix, G xi_bar <= tau): G stacks -P over P for every
  axis and tau stacks -s_min over s_max of that axis; the slack step and the
  bound rows' targets use the same iterate as the other closed forms, so the
  targets of the rows are min(tau, G xi_bar^k); the rows enter F (hence
  I + rho F^T F) whenever bounds are enabled, also for infinite limits.

Parity status: every function below is pinned by tests in tests/ against
closed forms, brute force, invariances or published known answers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# boundary-condition row selectors (bit i selects row i of
# [P_0, Pdot_0, Pddot_0, P_-1, Pdot_-1, Pddot_-1])
BC_P0, BC_V0, BC_A0, BC_PF, BC_VF, BC_AF = 1, 2, 4, 8, 16, 32
BC_DEFAULT = BC_P0 | BC_V0 | BC_A0 | BC_PF
BC_REST = BC_DEFAULT | BC_VF | BC_AF


# ---------------------------------------------------------------------------
# Sec. II-A, eq. (2): polynomial parametrisation
# ---------------------------------------------------------------------------
def time_grid(n_steps: int, horizon: float) -> np.ndarray:
    """Planning instants t_k = k T/(K-1), k = 0..K-1."""
    return np.arange(n_steps, dtype=np.float64) * (horizon / (n_steps - 1))


def _bernstein_values(deg: int, tau: np.ndarray) -> np.ndarray:
    """B_{i,deg}(tau) = C(deg,i) tau^i (1-tau)^(deg-i), shape [len(tau), deg+1]."""
    out = np.empty((tau.size, deg + 1))
    for i in range(deg + 1):
        out[:, i] = math.comb(deg, i) * tau ** i * (1.0 - tau) ** (deg - i)
    return out


def basis_matrices(n_coeff: int, n_steps: int, horizon: float):
    """P, Pdot, Pddot of eq. (2): K x n_coeff matrices mapping coefficients to
    position, velocity and acceleration on the time grid.

    Derivatives follow the textbook Bernstein identity
    d/dtau B_{i,n} = n (B_{i-1,n-1} - B_{i,n-1}), applied twice, with the chain
    rule factor 1/T per derivative."""
    n = n_coeff - 1
    tau = time_grid(n_steps, horizon) / horizon
    P = _bernstein_values(n, tau)
    Pd = np.zeros_like(P)
    Pdd = np.zeros_like(P)
    if n >= 1:
        B1 = _bernstein_values(n - 1, tau)
        for i in range(n + 1):
            lo = B1[:, i - 1] if i >= 1 else 0.0
            hi = B1[:, i] if i <= n - 1 else 0.0
            Pd[:, i] = n * (lo - hi) / horizon
    if n >= 2:
        B2 = _bernstein_values(n - 2, tau)
        for i in range(n + 1):
            t0 = B2[:, i - 2] if i >= 2 else 0.0
            t1 = B2[:, i - 1] if 1 <= i <= n - 1 else 0.0
            t2 = B2[:, i] if i <= n - 2 else 0.0
            Pdd[:, i] = n * (n - 1) * (t0 - 2.0 * t1 + t2) / horizon ** 2
    return P, Pd, Pdd


def _block_diag(block: np.ndarray, copies: int) -> np.ndarray:
    r, c = block.shape
    out = np.zeros((r * copies, c * copies))
    for k in range(copies):
        out[k * r:(k + 1) * r, k * c:(k + 1) * c] = block
    return out


@dataclass
class Problem:
    """Shape of one planning problem: Sec. II-A, eqs. (1)-(3) and Appendix (12).

    ``n_obs`` is the exact obstacle count: the stacked F_o block (eq. (13))
    holds one copy of P per obstacle, so it enters I + rho F^T F."""
    dims: int
    n_coeff: int
    n_steps: int
    horizon: float
    n_obs: int
    rho: float = 1.0
    v_max: float = math.inf
    a_max: float = math.inf
    bc_mask: int = BC_DEFAULT
    s_min: tuple = None     # workspace bounds per axis (Appendix, G xi <= tau); None: off
    s_max: tuple = None
    obs_model: int = 0      # 0: rows (centre, velocity, a, b); 1: per-step positions (traj)
    P: np.ndarray = field(init=False, repr=False)
    Pd: np.ndarray = field(init=False, repr=False)
    Pdd: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        assert self.dims in (2, 3)
        assert (self.s_min is None) == (self.s_max is None)
        self.P, self.Pd, self.Pdd = basis_matrices(self.n_coeff, self.n_steps, self.horizon)

    @property
    def bounded(self) -> bool:
        return self.s_min is not None

    @property
    def n_rows_axis(self) -> int:
        """Rows of F per axis: n_obs position blocks, velocity, acceleration,
        and the two blocks of G when workspace bounds are on."""
        return (self.n_obs + 2 + (2 if self.bounded else 0)) * self.n_steps

    def tau(self, ax: int) -> np.ndarray:
        """tau of G xi <= tau for one axis: [-s_min] * K over [s_max] * K."""
        K = self.n_steps
        return np.concatenate([np.full(K, -float(self.s_min[ax])), np.full(K, float(self.s_max[ax]))])

    @property
    def D(self) -> int:
        return self.dims * self.n_coeff

    # -- eq. (3b): block-diagonal boundary matrix ---------------------------
    def boundary_rows(self) -> list[int]:
        return [i for i in range(6) if self.bc_mask >> i & 1]

    def A_axis(self) -> np.ndarray:
        cand = [self.P[0], self.Pd[0], self.Pdd[0], self.P[-1], self.Pd[-1], self.Pdd[-1]]
        return np.array([cand[i] for i in self.boundary_rows()]).reshape(-1, self.n_coeff)

    def A(self) -> np.ndarray:
        return _block_diag(self.A_axis(), self.dims)

    def b_eq(self, bc: np.ndarray) -> np.ndarray:
        """Stack of b_0 and b_f per axis; ``bc`` is [dims, 6] holding
        (p0, v0, a0, pf, vf, af) for each axis."""
        rows = self.boundary_rows()
        return np.concatenate([np.asarray(bc, np.float64)[ax, rows] for ax in range(self.dims)])

    # -- eq. (13) and the definition below eq. (14): dense F ----------------
    def F_axis(self) -> np.ndarray:
        blocks = [self.P] * self.n_obs + [self.Pd, self.Pdd]
        if self.bounded:
            blocks += [-self.P, self.P]          # G
        return np.vstack(blocks)

    def F(self) -> np.ndarray:
        return _block_diag(self.F_axis(), self.dims)

    def kkt_matrix(self) -> np.ndarray:
        """[[I + rho F^T F, A^T], [A, 0]] of eq. (7b)."""
        F = self.F()
        A = self.A()
        D = self.D
        E = A.shape[0]
        K = np.zeros((D + E, D + E))
        K[:D, :D] = np.eye(D) + self.rho * F.T @ F
        K[:D, D:] = A.T
        K[D:, :D] = A
        return K


# ---------------------------------------------------------------------------
# Appendix, eqs. (10), (11a), (11b), (13), (15a)-(15c), (15f)
# ---------------------------------------------------------------------------
def obstacle_width(prob: Problem) -> int:
    """Floats per obstacle row: 8 (centre at t = 0, velocity, a, b), or
    K * dims + 2 (the position at every planning step, then a, b) when the
    obstacles are given by their trajectories (the stacked x_o, y_o, z_o of
    eq. (13) at every time stamp)."""
    return 8 if prob.obs_model == 0 else prob.n_steps * prob.dims + 2


def semi_axes(prob: Problem, obs: np.ndarray):
    """(a, b) of every obstacle ([n_obs] each)."""
    obs = np.asarray(obs, np.float64).reshape(-1, obstacle_width(prob))
    return obs[:, -2], obs[:, -1]


def obstacle_positions(prob: Problem, obs: np.ndarray) -> np.ndarray:
    """x_o,j(t_k) for constant-velocity obstacles: [n_obs, K, dims].
    ``obs`` rows are (cx, cy, cz, vx, vy, vz, a, b)."""
    if prob.obs_model == 1:
        w = obstacle_width(prob)
        obs = np.asarray(obs, np.float64).reshape(-1, w)
        return obs[:, :prob.n_steps * prob.dims].reshape(-1, prob.n_steps, prob.dims)
    obs = np.asarray(obs, np.float64).reshape(-1, 8)
    t = time_grid(prob.n_steps, prob.horizon)
    c = obs[:, 0:prob.dims]
    v = obs[:, 3:3 + prob.dims]
    return c[:, None, :] + v[:, None, :] * t[None, :, None]


def split_rows(prob: Problem, y: np.ndarray):
    """Split F xi_bar ([..., R]) into per-axis obstacle rows [..., dims, n_obs, K],
    velocity rows [..., dims, K] and acceleration rows [..., dims, K]."""
    K, no = prob.n_steps, prob.n_obs
    y = y.reshape(y.shape[:-1] + (prob.dims, prob.n_rows_axis))
    yo = y[..., :no * K].reshape(y.shape[:-1] + (no, K))
    yv = y[..., no * K:(no + 1) * K]
    ya = y[..., (no + 1) * K:(no + 2) * K]
    return yo, yv, ya


def polar_obstacle(prob: Problem, p: np.ndarray, opos: np.ndarray, obs: np.ndarray):
    """Closed-form alpha, beta, d for every (sample, obstacle, time) (eqs. (15a)-(15c)).

    p: [N, dims, K] robot positions; opos: [n_obs, K, dims].
    Returns alpha, beta, d with shape [N, n_obs, K]."""
    sa, sb = semi_axes(prob, obs)
    a = sa[None, :, None]
    delta = p[:, None, :, :] - np.transpose(opos, (0, 2, 1))[None]  # [N, no, dims, K]
    dx, dy = delta[:, :, 0], delta[:, :, 1]
    alpha = np.arctan2(dy, dx)
    rxy = np.sqrt(dx * dx + dy * dy)
    if prob.dims == 3:
        b = sb[None, :, None]
        dz = delta[:, :, 2]
        beta = np.arctan2(rxy / a, dz / b)
        d = np.maximum(1.0, np.sqrt((dx * dx + dy * dy) / a ** 2 + dz * dz / b ** 2))
    else:
        beta = np.full_like(alpha, np.pi / 2)
        d = np.maximum(1.0, rxy / a)
    return alpha, beta, d


def polar_bound(prob: Problem, w: np.ndarray, wmax: float):
    """Closed-form alpha, beta, d for a norm bound ||w|| <= wmax (eqs. (11a)/(11b)).

    w: [N, dims, K].  d = min(1, ||w||/wmax); with wmax = inf, d = 0 and the
    bound is inactive (the caller keeps the target at w itself)."""
    alpha = np.arctan2(w[:, 1], w[:, 0])
    nxy = np.sqrt(w[:, 0] ** 2 + w[:, 1] ** 2)
    if prob.dims == 3:
        beta = np.arctan2(nxy, w[:, 2])
        nrm = np.sqrt(nxy ** 2 + w[:, 2] ** 2)
    else:
        beta = np.full_like(alpha, np.pi / 2)
        nrm = nxy
    d = np.minimum(1.0, nrm / wmax)
    return alpha, beta, d


def _direction(alpha, beta, dims):
    if dims == 3:
        return [np.cos(alpha) * np.sin(beta), np.sin(alpha) * np.sin(beta), np.cos(beta)]
    return [np.cos(alpha) * np.sin(beta), np.sin(alpha) * np.sin(beta)]


def targets(prob: Problem, obs: np.ndarray, xi_bar: np.ndarray) -> np.ndarray:
    """e~(alpha, beta, d) of eq. (13), stacked in F's row order: [N, R]."""
    F = prob.F()
    y = xi_bar @ F.T
    N = xi_bar.shape[0]
    dims, K, no = prob.dims, prob.n_steps, prob.n_obs
    yo, yv, ya = split_rows(prob, y)
    e = np.zeros((N, dims, prob.n_rows_axis))
    if no > 0:
        p = yo[:, :, 0, :]  # every F_o block row reproduces the position P c
        opos = obstacle_positions(prob, obs)
        alpha, beta, d = polar_obstacle(prob, p, opos, obs)
        u = _direction(alpha, beta, dims)
        sa, sb = semi_axes(prob, obs)
        semi = [sa, sa, sb]
        for ax in range(dims):
            eo = opos[None, :, :, ax] + semi[ax][None, :, None] * d * u[ax]
            e[:, ax, :no * K] = eo.reshape(N, no * K)
    for rows, w, wmax in ((slice(no * K, (no + 1) * K), yv, prob.v_max),
                          (slice((no + 1) * K, (no + 2) * K), ya, prob.a_max)):
        if math.isinf(wmax):
            e[:, :, rows] = w
            continue
        alpha, beta, d = polar_bound(prob, w, wmax)
        u = _direction(alpha, beta, dims)
        for ax in range(dims):
            e[:, ax, rows] = d * wmax * u[ax]
    if prob.bounded:
        # slack s = max(0, tau - G xi_bar) (the minimiser over s >= 0), and the
        # rows' targets tau - s
        yg = y.reshape(N, dims, prob.n_rows_axis)[:, :, (no + 2) * K:]
        for ax in range(dims):
            tau = prob.tau(ax)
            slack = np.maximum(0.0, tau[None, :] - yg[:, ax])
            e[:, ax, (no + 2) * K:] = tau[None, :] - slack
    return e.reshape(N, -1)


# ---------------------------------------------------------------------------
# Sec. III-A eqs. (6)-(7) and Appendix eqs. (14)-(15): the projection
# ---------------------------------------------------------------------------
@dataclass
class ProjectionResult:
    xi_bar: np.ndarray            # [N, D]
    lam: np.ndarray               # [N, D]
    resid: np.ndarray             # [N]  r(xi_bar) of the returned iterate
    resid_hist: np.ndarray        # [n_iter, N] ||F xi_bar^k - e^{k+1}||
    kkt_rel: np.ndarray           # [n_iter] relative KKT residual of each solve
    eq_inf: np.ndarray            # [n_iter] max |A xi_bar - b|
    nu: np.ndarray = None         # [N, E] multipliers of A xi = b of the last solve


def project(prob: Problem, bc: np.ndarray, obs: np.ndarray, xi: np.ndarray,
            n_iter: int) -> ProjectionResult:
    """Project every row of ``xi`` ([N, D]) toward the feasible set with the
    alternating-minimisation / augmented-Lagrangian steps of the Appendix.

    Each iteration k (eqs. (15a)-(15g)):
      1. alpha, beta, d from xi_bar^k (closed forms) -> e^{k+1} (eq. (15f));
      2. lambda^{k+1} = lambda^k - rho F^T (F xi_bar^k - e^{k+1})  (eq. (15e));
      3. xi_bar^{k+1} = argmin of eq. (14) s.t. A xi_bar = b, solved through the
         KKT system of eq. (7b) with eta = [xi + lambda^{k+1} + rho F^T e^{k+1}; b].
    """
    xi = np.asarray(xi, np.float64)
    N, D = xi.shape
    assert D == prob.D
    F = prob.F()
    A = prob.A()
    b = prob.b_eq(bc)
    E = A.shape[0]
    KKT = prob.kkt_matrix()
    xi_bar = xi.copy()
    lam = np.zeros_like(xi)
    hist = np.zeros((n_iter, N))
    kkt_rel = np.zeros(n_iter)
    eq_inf = np.zeros(n_iter)
    nu = np.zeros((N, E))
    for k in range(n_iter):
        e = targets(prob, obs, xi_bar)
        y = xi_bar @ F.T
        hist[k] = np.linalg.norm(y - e, axis=1)
        lam = lam - prob.rho * (y - e) @ F
        rhs = np.zeros((D + E, N))
        rhs[:D] = (xi + lam + prob.rho * e @ F).T
        rhs[D:] = b[:, None]
        sol = np.linalg.solve(KKT, rhs)
        kkt_rel[k] = np.linalg.norm(KKT @ sol - rhs) / max(np.linalg.norm(rhs), 1e-300)
        xi_bar = sol[:D].T.copy()
        nu = sol[D:].T.copy()
        eq_inf[k] = np.max(np.abs(xi_bar @ A.T - b[None, :])) if E else 0.0
    return ProjectionResult(xi_bar=xi_bar, lam=lam, resid=residual(prob, obs, xi_bar),
                            resid_hist=hist, kkt_rel=kkt_rel, eq_inf=eq_inf, nu=nu)


def lagrangian(prob: Problem, xi: np.ndarray, lam: np.ndarray, e: np.ndarray,
               xi_bar: np.ndarray) -> float:
    """Eq. (14) for one sample (vectors of length D, e of length R)."""
    F = prob.F()
    r = F @ xi_bar - e
    return 0.5 * float(np.dot(xi_bar - xi, xi_bar - xi)) - float(np.dot(lam, xi_bar)) \
        + 0.5 * prob.rho * float(np.dot(r, r))


# ---------------------------------------------------------------------------
# Alg. 1: residual and cost
# ---------------------------------------------------------------------------
def residual_dense(prob: Problem, obs: np.ndarray, xi_bar: np.ndarray) -> np.ndarray:
    """||F xi_bar - e(xi_bar)||_2 with the dense F and trigonometric targets."""
    e = targets(prob, obs, xi_bar)
    return np.linalg.norm(xi_bar @ prob.F().T - e, axis=1)


def residual(prob: Problem, obs: np.ndarray, xi_bar: np.ndarray) -> np.ndarray:
    """r(xi_bar) of Alg. 1 written as constraint violations, so that r is exactly
    zero when every constraint of eq. (1) holds on the grid:

      r^2 = sum_{j,k} ||p_k - o_j(t_k)||^2 max(0, 1/n_jk - 1)^2
          + sum_k max(0, ||v_k|| - v_max)^2 + sum_k max(0, ||a_k|| - a_max)^2
          [+ sum_{k,x} max(0, s_min,x - p_k,x)^2 + max(0, p_k,x - s_max,x)^2],

    with n_jk the scaled distance sqrt((dx^2+dy^2)/a^2 + dz^2/b^2).  Each term
    is the squared length of one row block of F xi_bar - e(xi_bar); a zero
    offset (n = 0) contributes the semi-axis along the canonical direction."""
    xi_bar = np.asarray(xi_bar, np.float64)
    N = xi_bar.shape[0]
    dims, nc = prob.dims, prob.n_coeff
    C = xi_bar.reshape(N, dims, nc)
    p = np.einsum('kc,nac->nak', prob.P, C)
    v = np.einsum('kc,nac->nak', prob.Pd, C)
    a = np.einsum('kc,nac->nak', prob.Pdd, C)
    r2 = np.zeros(N)
    if prob.n_obs:
        opos = obstacle_positions(prob, obs)
        sas, sbs = semi_axes(prob, obs)
        for j in range(prob.n_obs):
            delta = p - opos[j].T[None]  # [N, dims, K]
            sa, sb = sas[j], sbs[j]
            n2 = (delta[:, 0] ** 2 + delta[:, 1] ** 2) / sa ** 2
            if dims == 3:
                n2 = n2 + delta[:, 2] ** 2 / sb ** 2
            len2 = np.sum(delta ** 2, axis=1)
            with np.errstate(divide='ignore', invalid='ignore'):
                viol = np.where(n2 > 0, np.maximum(0.0, 1.0 / np.sqrt(n2) - 1.0), 0.0)
            term = len2 * viol ** 2
            zero_semi = sb if dims == 3 else sa
            term = np.where(n2 == 0, zero_semi ** 2, term)
            r2 += term.sum(axis=1)
    for w, wmax in ((v, prob.v_max), (a, prob.a_max)):
        nrm = np.sqrt(np.sum(w ** 2, axis=1))
        r2 += np.sum(np.maximum(0.0, nrm - wmax) ** 2, axis=1)
    if prob.bounded:
        lo = np.asarray(prob.s_min, np.float64)[None, :, None]
        hi = np.asarray(prob.s_max, np.float64)[None, :, None]
        r2 += np.sum(np.maximum(0.0, lo - p) ** 2 + np.maximum(0.0, p - hi) ** 2, axis=(1, 2))
    return np.sqrt(r2)


def smoothness_cost(prob: Problem, xi_bar: np.ndarray) -> np.ndarray:
    """c1 = sum_k ||a_k||^2: the acceleration-norm smoothness cost of the
    point-to-point benchmark (Sec. V-A)."""
    N = xi_bar.shape[0]
    C = np.asarray(xi_bar, np.float64).reshape(N, prob.dims, prob.n_coeff)
    a = np.einsum('kc,nac->nak', prob.Pdd, C)
    return np.sum(a ** 2, axis=(1, 2))


@dataclass
class Cost:
    """Weights of c1 (Sec. II remark that c1 need not be smooth; the navigation
    and steering costs of Sec. V).  kind 0: the smoothness cost sum ||a||^2;
    kind 1: the weighted sum of the terms of trajectory_cost."""
    kind: int = 0
    w_acc: float = 1.0
    w_curv: float = 0.0
    w_path: float = 0.0
    w_steer: float = 0.0
    wheelbase: float = 1.0
    eps: float = 1e-2


def curvature(v: np.ndarray, a: np.ndarray, eps: float, signed: bool = False) -> np.ndarray:
    """kappa_k of a trajectory from its velocity and acceleration rows
    ([N, dims, K]): |v x a| / (|v|^2 + eps)^(3/2), with eps keeping it finite
    at rest.  signed (2D): (v_x a_y - v_y a_x) / (|v|^2 + eps)^(3/2)."""
    s2 = np.sum(v ** 2, axis=1) + eps
    if v.shape[1] == 2:
        cr = v[:, 0] * a[:, 1] - v[:, 1] * a[:, 0]
        num = cr if signed else np.abs(cr)
    else:
        assert not signed
        cr = np.cross(np.moveaxis(v, 1, -1), np.moveaxis(a, 1, -1))
        num = np.linalg.norm(cr, axis=-1)
    return num / s2 ** 1.5


def segment_distance(p: np.ndarray, start: np.ndarray, goal: np.ndarray) -> np.ndarray:
    """Euclidean distance of every way-point p [N, dims, K] to the segment
    start -> goal: the projection onto the line, clamped to the segment."""
    u = goal - start
    uu = float(np.dot(u, u))
    rel = p - start[None, :, None]
    if uu == 0.0:
        return np.sqrt(np.sum(rel ** 2, axis=1))
    lam = np.clip(np.einsum('ndk,d->nk', rel, u) / uu, 0.0, 1.0)
    q = rel - lam[:, None, :] * u[None, :, None]
    return np.sqrt(np.sum(q ** 2, axis=1))


def trajectory_cost(prob: Problem, bc: np.ndarray, xi_bar: np.ndarray, cost: Cost = None) -> np.ndarray:
    """c1 of every projected sample.  kind 0 (or no cost): sum_k ||a_k||^2.
    kind 1: sum_k [w_acc ||a_k||^2 + w_curv kappa_k^2 + w_path dist(p_k, segment)
    + w_steer atan(wheelbase * kappa_signed,k)^2], the last in 2D only (car-like
    steering angle from differential flatness); start and goal of the segment
    are the boundary values p0 and pf of bc."""
    if cost is None or cost.kind == 0:
        return smoothness_cost(prob, xi_bar)
    N = xi_bar.shape[0]
    C = np.asarray(xi_bar, np.float64).reshape(N, prob.dims, prob.n_coeff)
    p = np.einsum('kc,nac->nak', prob.P, C)
    v = np.einsum('kc,nac->nak', prob.Pd, C)
    a = np.einsum('kc,nac->nak', prob.Pdd, C)
    bc = np.asarray(bc, np.float64)
    out = np.zeros(N)
    if cost.w_acc:
        out += cost.w_acc * np.sum(a ** 2, axis=(1, 2))
    if cost.w_curv:
        out += cost.w_curv * np.sum(curvature(v, a, cost.eps) ** 2, axis=1)
    if cost.w_path:
        out += cost.w_path * np.sum(segment_distance(p, bc[:, 0], bc[:, 3]), axis=1)
    if cost.w_steer:
        assert prob.dims == 2
        delta = np.arctan(cost.wheelbase * curvature(v, a, cost.eps, signed=True))
        out += cost.w_steer * np.sum(delta ** 2, axis=1)
    return out


# ---------------------------------------------------------------------------
# Alg. 1 selection and eqs. (9a)-(9c) refit
# ---------------------------------------------------------------------------
def select_lowest(keys: np.ndarray, k: int) -> np.ndarray:
    """Indices of the k smallest keys; ties by index; NaN counts as +inf."""
    keys = np.where(np.isnan(keys), np.inf, np.asarray(keys, np.float64))
    return np.argsort(keys, kind='stable')[:k]


def refit(mu: np.ndarray, Sigma: np.ndarray, elites: np.ndarray, c_aug: np.ndarray,
          sigma: float, gamma: float):
    """Eqs. (9a)-(9c): MPPI-like update of mean and covariance from the elite set.

    c_m = exp(-(c_aug_m - delta)/gamma), delta = min c_aug; the covariance is
    centred on the new mean, as printed."""
    c_aug = np.asarray(c_aug, np.float64)
    delta = np.min(c_aug)
    w = np.exp(-(c_aug - delta) / gamma)
    sw = np.sum(w)
    mu_new = (1.0 - sigma) * mu + sigma * (w @ elites) / sw
    dev = elites - mu_new[None, :]
    cov = (dev * w[:, None]).T @ dev / sw
    Sigma_new = (1.0 - sigma) * Sigma + sigma * cov
    return mu_new, Sigma_new, w


def cma_rates(n: int, mu_eff: float):
    """Learning rates of the covariance adaptation (Hansen's CMA-ES tutorial
    defaults for dimension n and variance-effective selection mass mu_eff):
    c_c of the evolution path, c_1 of the rank-one and c_mu of the rank-mu
    update."""
    cc = (4.0 + mu_eff / n) / (n + 4.0 + 2.0 * mu_eff / n)
    c1 = 2.0 / ((n + 1.3) ** 2 + mu_eff)
    cmu = min(1.0 - c1, 2.0 * (mu_eff - 2.0 + 1.0 / mu_eff) / ((n + 2.0) ** 2 + mu_eff))
    return cc, c1, cmu


def refit_cma(mu: np.ndarray, Sigma: np.ndarray, pc: np.ndarray, elites: np.ndarray,
              c_aug: np.ndarray, sigma: float, gamma: float):
    """A CMA-ES-style covariance update in place of eq. (9b) (the remark after
    eqs. (9a)-(9c) that Alg. 1 is agnostic to the update rule).  The weights
    are those of eq. (9c), normalised; the mean follows eq. (9a); with
    y_m = xi_bar_m - mu (the current mean) and y_w = sum_m w_m y_m:
      p_c'     = (1 - c_c) p_c + sqrt(c_c (2 - c_c) mu_eff) y_w,
      Sigma'   = (1 - c_1 - c_mu) Sigma + c_1 p_c' p_c'^T + c_mu sum_m w_m y_m y_m^T,
    mu_eff = 1 / sum_m w_m^2.  No step-size adaptation: Sigma carries the scale."""
    c_aug = np.asarray(c_aug, np.float64)
    w = np.exp(-(c_aug - np.min(c_aug)) / gamma)
    wn = w / np.sum(w)
    mu_eff = 1.0 / np.sum(wn ** 2)
    mu_new = (1.0 - sigma) * mu + sigma * (wn @ elites)
    y = elites - mu[None, :]
    yw = wn @ y
    cc, c1, cmu = cma_rates(mu.shape[0], mu_eff)
    pc_new = (1.0 - cc) * pc + math.sqrt(cc * (2.0 - cc) * mu_eff) * yw
    rank_mu = (y * wn[:, None]).T @ y
    Sigma_new = (1.0 - c1 - cmu) * Sigma + c1 * np.outer(pc_new, pc_new) + cmu * rank_mu
    return mu_new, Sigma_new, pc_new


def jittered_cholesky(Sigma: np.ndarray, cov_jitter: float) -> np.ndarray:
    D = Sigma.shape[0]
    eps = cov_jitter * np.trace(Sigma) / D
    return np.linalg.cholesky(Sigma + eps * np.eye(D))


@dataclass
class CemParams:
    n_samples: int
    n_proj_iters: int
    n_proj: int
    n_elite: int
    sigma: float = 0.5
    gamma: float = 1.0
    cov_jitter: float = 1e-5
    cost: Cost = None
    update: str = "mppi"    # "mppi": eqs. (9a)-(9c); "cma": refit_cma


@dataclass
class CemStep:
    xi: np.ndarray
    xi_bar: np.ndarray
    resid: np.ndarray
    c1: np.ndarray
    c_aug: np.ndarray       # c1 + r for every sample (used only on proj_idx)
    proj_idx: np.ndarray
    elite_idx: np.ndarray
    mu: np.ndarray
    Sigma: np.ndarray
    best_xi: np.ndarray
    best_cost: float
    pc: np.ndarray = None   # evolution path after the step (update "cma")


def cem_iteration(prob: Problem, bc, obs, mu, Sigma, noise, prm: CemParams, pc=None) -> CemStep:
    """One pass of the loop body of Alg. 1 with the standard-normal draws
    ``noise`` ([N, D]) supplied: xi_i = mu + L z_i with L L^T = Sigma + eps I.
    ``pc``: the evolution path of the "cma" update (zeros when None)."""
    L = jittered_cholesky(np.asarray(Sigma, np.float64), prm.cov_jitter)
    xi = np.asarray(mu, np.float64)[None, :] + np.asarray(noise, np.float64) @ L.T
    pr = project(prob, bc, obs, xi, prm.n_proj_iters)
    r = pr.resid
    c1 = trajectory_cost(prob, bc, pr.xi_bar, prm.cost)
    c_aug = c1 + r
    proj_idx = select_lowest(r, prm.n_proj)
    order = select_lowest(c_aug[proj_idx], prm.n_elite)
    elite_idx = proj_idx[order]
    pc_new = None
    if prm.update == "cma":
        pc0 = np.zeros(prob.D) if pc is None else np.asarray(pc, np.float64)
        mu_new, Sigma_new, pc_new = refit_cma(np.asarray(mu, np.float64),
                                              np.asarray(Sigma, np.float64), pc0,
                                              pr.xi_bar[elite_idx], c_aug[elite_idx],
                                              prm.sigma, prm.gamma)
    else:
        assert prm.update == "mppi"
        mu_new, Sigma_new, _ = refit(np.asarray(mu, np.float64), np.asarray(Sigma, np.float64),
                                     pr.xi_bar[elite_idx], c_aug[elite_idx], prm.sigma, prm.gamma)
    best = elite_idx[0]
    return CemStep(xi=xi, xi_bar=pr.xi_bar, resid=r, c1=c1, c_aug=c_aug, proj_idx=proj_idx,
                   elite_idx=elite_idx, mu=mu_new, Sigma=Sigma_new,
                   best_xi=pr.xi_bar[best].copy(), best_cost=float(c_aug[best]), pc=pc_new)


def plan(prob: Problem, bc, obs, mu, Sigma, prm: CemParams, n_cem: int,
         noise=None, seed: int = 0, stream: int = 0):
    """Alg. 1: n_cem iterations; returns the lowest-c_aug elite of the final
    iteration plus the updated (mu, Sigma).  ``noise`` is [n_cem, N, D] or None,
    in which case draws come from :func:`normals` (Philox4x32-10 + Box-Muller)."""
    steps = []
    pc = None   # the "cma" evolution path starts at zero on every call
    for l in range(n_cem):
        z = noise[l] if noise is not None else normals(seed, stream, l, prm.n_samples, prob.D)
        st = cem_iteration(prob, bc, obs, mu, Sigma, z, prm, pc)
        mu, Sigma, pc = st.mu, st.Sigma, st.pc
        steps.append(st)
    return steps


@dataclass
class DPriestResult:
    groups: list            # per distribution: the list of CemStep of plan()
    best_group: int
    best_xi: np.ndarray
    best_cost: float


def dpriest(prob: Problem, bc, obs, mus, Sigmas, prm: CemParams, n_cem: int,
            noise=None, seed: int = 0, stream_base: int = 0) -> DPriestResult:
    """D-PRIEST (Sec. III-C): M Gaussians, each drawing prm.n_samples samples;
    all samples are projected (per sample, so the row-wise stacking of the
    paper does not change any value), every distribution is refitted on its
    own samples, and the lowest-cost final trajectory over the M instances is
    returned (first index on ties).  Distribution g draws stream
    stream_base + g, or noise[g] ([M, n_cem, N, D]) when given."""
    groups = []
    for g in range(len(mus)):
        z = noise[g] if noise is not None else None
        groups.append(plan(prob, bc, obs, np.asarray(mus[g], np.float64),
                           np.asarray(Sigmas[g], np.float64), prm, n_cem, noise=z, seed=seed,
                           stream=stream_base + g))
    best = pick_group([st[-1].best_cost for st in groups])
    return DPriestResult(groups, best, groups[best][-1].best_xi, float(groups[best][-1].best_cost))


def pick_group(costs) -> int:
    """Index of the lowest final cost over the distributions of D-PRIEST
    (Sec. III-C); NaN ranks last, ties go to the lowest index."""
    c = np.asarray(costs, np.float64)
    c = np.where(np.isnan(c), np.inf, c)
    return int(np.argmin(c))


# ---------------------------------------------------------------------------
# Counter-based normal draws: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
# "Parallel random numbers: as easy as 1, 2, 3", SC'11) + Box-Muller.
# ---------------------------------------------------------------------------
_PHILOX_M0 = 0xD2511F53
_PHILOX_M1 = 0xCD9E8D57
_PHILOX_W0 = 0x9E3779B9
_PHILOX_W1 = 0xBB67AE85
_MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on integer arrays.  ctr: [..., 4], key: [..., 2]
    (uint32 values held in int64/uint64).  Returns [..., 4] uint64 words."""
    c = [np.asarray(ctr, np.uint64)[..., i] & _MASK32 for i in range(4)]
    k0 = np.asarray(key, np.uint64)[..., 0] & _MASK32
    k1 = np.asarray(key, np.uint64)[..., 1] & _MASK32
    m0 = np.uint64(_PHILOX_M0)
    m1 = np.uint64(_PHILOX_M1)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + np.uint64(_PHILOX_W0)) & np.uint64(_MASK32)
            k1 = (k1 + np.uint64(_PHILOX_W1)) & np.uint64(_MASK32)
        p0 = c[0] * m0          # < 2^64, exact in uint64
        p1 = c[2] * m1
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(_MASK32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(_MASK32)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def uniform_open(x):
    """uint32 -> (0,1): ((x >> 9) + 1/2) 2^-23, exactly representable in FP32."""
    return ((np.asarray(x, np.uint64) >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def normals(seed: int, stream: int, it: int, n: int, D: int) -> np.ndarray:
    """Standard normals z[i, d] for CEM iteration ``it``.

    Counter (i, d//4, it, stream), key (seed lo, seed hi); the four words give
    two Box-Muller pairs: z[4q+0,1] from words (0,1), z[4q+2,3] from (2,3)."""
    nq = (D + 3) // 4
    i = np.arange(n, dtype=np.uint64)[:, None]
    q = np.arange(nq, dtype=np.uint64)[None, :]
    ctr = np.stack(np.broadcast_arrays(i, q, np.uint64(it), np.uint64(stream)), axis=-1)
    key = np.array([seed & _MASK32, (seed >> 32) & _MASK32], np.uint64)
    w = philox4x32_10(ctr, np.broadcast_to(key, ctr.shape[:-1] + (2,)))
    z = np.empty((n, nq, 4))
    for pair in range(2):
        u1 = uniform_open(w[..., 2 * pair])
        u2 = uniform_open(w[..., 2 * pair + 1])
        rad = np.sqrt(-2.0 * np.log(u1))
        z[..., 2 * pair] = rad * np.cos(2.0 * np.pi * u2)
        z[..., 2 * pair + 1] = rad * np.sin(2.0 * np.pi * u2)
    return z.reshape(n, nq * 4)[:, :D]
