"""Helpers shared by the GPU parity tests: oracle problem construction and the
comparison rules for FP32 results against the FP64 oracle."""
from __future__ import annotations

import numpy as np

import oracle as O

# FP32 projected coefficients: per sample, max-abs error relative to
# max(1, max |xi_bar|) of the oracle.
XI_TOL = 1e-3
# A sample may exceed XI_TOL only if the FP64 oracle itself moves by more
# than SENS_MOVE when that sample's input is perturbed by SENS_EPS relative
# (the FP32 input rounding is ~6e-8): such samples amplify rounding noise.
SENS_EPS = 1e-7
SENS_MOVE = 1e-4


def oracle_problem(wl, **kw) -> O.Problem:
    d = dict(dims=wl.dims, n_coeff=wl.n_coeff, n_steps=wl.n_steps, horizon=wl.horizon,
             n_obs=wl.n_obs, rho=wl.rho, v_max=wl.v_max, a_max=wl.a_max, bc_mask=wl.bc_mask)
    d.update(kw)
    return O.Problem(**d)


def rel_err(got: np.ndarray, want: np.ndarray) -> np.ndarray:
    """Per-row max |got - want| / max(1, max |want|)."""
    got = np.asarray(got, np.float64).reshape(len(want), -1)
    want = np.asarray(want, np.float64).reshape(len(want), -1)
    return np.abs(got - want).max(1) / np.maximum(1.0, np.abs(want).max(1))


def check_projection(prob, bc, obs, xi32, got, want, n_iter, rng_seed=0, label="",
                     counts=None):
    """Element-wise parity of projected samples with the sensitivity rule.
    Returns the per-sample errors; raises AssertionError on a violation.
    The number of samples above XI_TOL (every one of them shown to be
    sensitive) is printed and, when ``counts`` is a dict, added to
    counts["sensitive"] beside counts["checked"]."""
    err = rel_err(got, want)
    bad = np.nonzero(err > XI_TOL)[0]
    print(f"[parity] {label}: {len(err)} samples checked, {bad.size} above {XI_TOL} "
          f"(median err {np.median(err):.2e}, max {err.max():.2e})", flush=True)
    if counts is not None:
        counts["checked"] = counts.get("checked", 0) + len(err)
        counts["sensitive"] = counts.get("sensitive", 0) + int(bad.size)
    if bad.size:
        rng = np.random.default_rng(rng_seed)
        pert = xi32[bad].astype(np.float64)
        pert = pert * (1.0 + SENS_EPS * rng.choice([-1.0, 1.0], size=pert.shape))
        moved = O.project(prob, bc, obs, pert, n_iter).xi_bar
        sens = rel_err(moved, want[bad])
        unexplained = bad[sens <= SENS_MOVE]
        assert unexplained.size == 0, (
            f"{label}: samples {unexplained.tolist()} exceed {XI_TOL} "
            f"(errors {err[unexplained].tolist()}) without being sensitive")
        assert bad.size <= max(1, int(0.01 * len(err))), f"{label}: {bad.size} sensitive samples"
    return err


def check_selection(keys: np.ndarray, got_idx: np.ndarray, k: int, label=""):
    """The selected k indices must be the k smallest keys, exactly, wherever
    the k-th and (k+1)-th keys (oracle order) are separated by more than
    1e-3 max(1, |key|); inside such a tie band membership may differ."""
    keys = np.where(np.isnan(keys), np.inf, keys)
    order = np.argsort(keys, kind="stable")
    want = set(order[:k].tolist())
    got = set(np.asarray(got_idx).tolist())
    assert len(got) == k, f"{label}: duplicate indices"
    kth = keys[order[k - 1]]
    band = 1e-3 * max(1.0, abs(kth))
    sure_in = {i for i in want if keys[i] < kth - band}
    sure_out = {i for i in range(len(keys)) if keys[i] > kth + band}
    assert sure_in <= got, f"{label}: missing {sorted(sure_in - got)}"
    assert not (sure_out & got), f"{label}: wrongly selected {sorted(sure_out & got)}"
