"""The refit kernel's two selections of Alg. 1 (ConstraintEliteSet, then
EliteSet) on crafted residuals and costs, heavy with ties.  Both device paths
(stable block radix sorts when the ordered first selection is an output;
radix selects and a ranking by counting otherwise) must pick and order
exactly the samples that two stable sorts pick: the n_proj lowest r, ties by
index, then the n_elite lowest c_aug = c1 + r (FP32) among them, ties in the
order of the first selection.  Integer results: compared bit for bit."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2309_08235_amd.priest")


def reference(r, c1, n_proj, n_elite):
    proj = np.argsort(r, kind="stable")[:n_proj]
    c_aug = (c1 + r).astype(np.float32)          # the kernel's FP32 sum
    order = np.argsort(c_aug[proj], kind="stable")[:n_elite]
    return proj, proj[order]


def inputs(kind, n, rng):
    if kind == "distinct":
        r = rng.random(n, dtype=np.float32)
        r[::3] = 0.0
        c1 = (10 * rng.random(n)).astype(np.float32)
    elif kind == "quantised":
        r = (0.25 * rng.integers(0, 4, n)).astype(np.float32)
        c1 = (0.5 * rng.integers(0, 4, n)).astype(np.float32)
    elif kind == "all_equal":
        r = np.ones(n, np.float32)
        c1 = np.full(n, 2.0, np.float32)
    elif kind == "r_zero":
        r = np.zeros(n, np.float32)
        r[1::2] = -0.0                              # -0 ranks with +0
        c1 = (np.arange(n) % 7).astype(np.float32)
    elif kind == "c_aug_ties":
        # equal sums from different (c1, r) pairs: ties broken by r, then index
        r = (0.5 * rng.integers(0, 3, n)).astype(np.float32)
        c1 = (2.0 - r).astype(np.float32)
        c1[::5] = 3.0
    else:
        raise ValueError(kind)
    return r, c1


SIZES = [(7, 5, 1), (64, 40, 10), (1000, 727, 100), (2048, 1500, 300), (1500, 1500, 512),
         (1000, 900, 700), (3000, 2000, 200)]


@pytest.mark.parametrize("kind", ["distinct", "quantised", "all_equal", "r_zero", "c_aug_ties"])
@pytest.mark.parametrize("n,n_proj,n_elite", SIZES)
def test_selection_paths_match_stable_sorts(kind, n, n_proj, n_elite):
    print(f"select {kind} N={n} n_proj={n_proj} n_elite={n_elite}", flush=True)
    rng = np.random.default_rng(n + n_proj + n_elite + len(kind))
    r, c1 = inputs(kind, n, rng)
    proj_ref, elite_ref = reference(r, c1, n_proj, n_elite)
    dr = torch.tensor(r, device="cuda")
    dc = torch.tensor(c1, device="cuda")
    e_sel = torch.full((n_elite,), -1, dtype=torch.int32, device="cuda")
    e_sort = torch.full((n_elite,), -1, dtype=torch.int32, device="cuda")
    proj = torch.full((n_proj,), -1, dtype=torch.int32, device="cuda")
    P.priest_debug_select(n_proj, n_elite, dr, dc, e_sel)
    P.priest_debug_select(n_proj, n_elite, dr, dc, e_sort, proj)
    np.testing.assert_array_equal(proj.cpu().numpy(), proj_ref)
    np.testing.assert_array_equal(e_sort.cpu().numpy(), elite_ref)
    np.testing.assert_array_equal(e_sel.cpu().numpy(), elite_ref)


def test_selection_rejects_bad_sizes():
    d = torch.zeros(8, device="cuda")
    e = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(P.PriestError):
        P.priest_debug_select(9, 4, d, d, e)        # n_proj > N
    with pytest.raises(P.PriestError):
        P.priest_debug_select(3, 4, d, d, e)        # n_elite > n_proj
