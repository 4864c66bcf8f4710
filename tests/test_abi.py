"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/priest.h declares, and rejects invalid arguments on the host
before anything is launched."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "priest.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(priest_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def P():
    from paper_2309_08235_amd import priest
    priest.lib()
    return priest


def test_exports_every_declared_symbol(P):
    names = declared()
    assert "priest_init_problem" in names and "priest_plan" in names
    for n in names:
        assert hasattr(P.lib(), n), n
    assert set(names) == set(P.EXPORTS)
    assert P.lib().priest_version() == 1


def _desc(P, **kw):
    for k in ("s_min", "s_max"):
        if k in kw:
            kw[k] = (ctypes.c_double * 3)(*kw[k])
    d = dict(dims=2, n_coeff=11, n_steps=50, n_obs=4, horizon=10.0, rho=1.0, v_max=1.5,
             a_max=2.0, bc_mask=P.BC_DEFAULT, precision=0, n_refine_fp32=0, use_bounds=0)
    d.update(kw)
    return P.ProblemDesc(**d)


@pytest.mark.parametrize("bad,code", [
    (dict(dims=4), -1), (dict(n_coeff=1), -1), (dict(n_coeff=17), -1), (dict(n_steps=1), -1),
    (dict(n_steps=257), -1), (dict(n_obs=-1), -1), (dict(horizon=0.0), -1),
    (dict(horizon=math.nan), -1), (dict(rho=-1.0), -1), (dict(rho=math.inf), -1),
    (dict(v_max=0.0), -1), (dict(v_max=math.nan), -1), (dict(a_max=-2.0), -1),
    (dict(bc_mask=64), -1), (dict(precision=7), -1), (dict(use_bounds=2), -1),
    (dict(n_coeff=3, bc_mask=63), -2),
    (dict(obs_model=2), -1), (dict(reserved2=1), -1),
    (dict(use_bounds=1, s_min=(1.0, 0.0, 0.0), s_max=(0.0, 1.0, 1.0)), -1),
    (dict(use_bounds=1, s_min=(0.0, math.nan, 0.0), s_max=(1.0, 1.0, 1.0)), -1),
])
def test_init_rejects_invalid_desc_on_host(P, bad, code):
    h = ctypes.c_void_p()
    rc = P.lib().priest_init_problem(ctypes.byref(_desc(P, **bad)), None, ctypes.byref(h))
    assert rc == code
    assert h.value is None
    assert P.lib().priest_last_error()


def test_calls_reject_null_handles(P):
    L = P.lib()
    assert L.priest_project(None, None, None, None, 1, 1, None, None, None, None) == -1
    n = ctypes.c_size_t()
    prm = P.CemParams(64, 1, 10, 47, 12, 0, 0.5, 1.0, 1e-5, 0.0)
    assert L.priest_plan_workspace_size(None, ctypes.byref(prm), 1, ctypes.byref(n)) == -1
    assert L.priest_free_problem(None) == 0
    assert L.priest_debug_normals(0, 0, 0, 4, 0, None, None) == -1
    assert L.priest_problem_dim(None) == 0


def test_plan_static_rejects_on_host(P):
    """The allocation-free plan validates on the host like priest_plan."""
    L = P.lib()
    prm = P.CemParams(64, 1, 10, 47, 12, 0, 0.5, 1.0, 1e-5, 0.0)
    po = P.PlanOut()
    assert L.priest_plan_static(None, None, None, ctypes.byref(prm), None, None, 0, 0, None,
                                ctypes.byref(po), None) == -1
    assert L.priest_last_error()
