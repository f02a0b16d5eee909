"""The Python binding rejects tensors the C-ABI would read or write out of bounds (host
tensors, wrong element types, wrong lengths, non-contiguous views) before any library
call.  The plan handle here is NULL, so a check that let a bad tensor through would reach
the library's own NULL-plan check instead of a kernel."""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1408_3048_amd import _lib as L  # noqa: E402
from paper_1408_3048_amd.autograd import gls_map  # noqa: E402

N_VEC, N_T = 12, 20


@pytest.fixture()
def plan():
    p = object.__new__(L.Plan)
    p._h = ctypes.c_void_p()
    p._lib = L.load()
    p.n_vec, p.n_samples, p.n_intervals, p.lam, p.n_problems = N_VEC, N_T, 2, 4, 1
    p.n_stokes, p.n_obs = 3, N_VEC // 3
    return p


MAP_CALLS = ["apply_P", "apply_A", "precond_bj", "precond_2lvl", "precond_adef2",
             "pcg_solve", "coarse_from_krylov"]


@pytest.mark.parametrize("call", MAP_CALLS)
def test_map_arguments(plan, call):
    fn = getattr(plan, call)
    with pytest.raises(TypeError, match="dtype"):
        fn(torch.zeros(N_VEC, dtype=torch.float32))
    with pytest.raises(ValueError, match="elements"):
        fn(torch.zeros(N_VEC - 1, dtype=torch.float64))
    with pytest.raises(ValueError, match="contiguous"):
        fn(torch.zeros(2 * N_VEC, dtype=torch.float64)[::2])
    with pytest.raises(ValueError, match="GPU"):
        fn(torch.zeros(N_VEC, dtype=torch.float64))
    with pytest.raises(TypeError, match="torch tensor"):
        fn(np.zeros(N_VEC))


@pytest.mark.parametrize("call", ["apply_PT", "rhs"])
def test_tod_arguments(plan, call):
    fn = getattr(plan, call)
    with pytest.raises(TypeError, match="dtype"):
        fn(torch.zeros(N_T, dtype=torch.int32))
    with pytest.raises(ValueError, match="elements"):
        fn(torch.zeros(N_T + 3, dtype=torch.float32))
    with pytest.raises(ValueError, match="GPU"):
        fn(torch.zeros(N_T, dtype=torch.float64))


def test_ninv_precision_dtype(plan):
    with pytest.raises(TypeError, match="dtype"):
        plan.apply_Ninv(torch.zeros(N_T, dtype=torch.float64), precision="mixed")
    with pytest.raises(TypeError, match="dtype"):
        plan.apply_Ninv(torch.zeros(N_T, dtype=torch.float32), precision="fp64")


def test_other_wrappers(plan):
    f64 = torch.float64
    with pytest.raises(ValueError, match="elements"):
        plan.apply_A(torch.zeros(N_VEC, dtype=f64), out=torch.zeros(N_VEC + 1, dtype=f64))
    with pytest.raises(ValueError, match="elements"):
        plan.lag_correlations(torch.zeros(N_T, dtype=f64), torch.zeros(N_T - 1, dtype=f64))
    with pytest.raises(TypeError, match="dtype"):
        plan.lag_correlations(torch.zeros(N_T, dtype=torch.float32), torch.zeros(N_T, dtype=f64))
    with pytest.raises(ValueError, match="elements"):
        plan.adjoint(torch.zeros(N_VEC, dtype=f64), torch.zeros(N_VEC, dtype=f64),
                     torch.zeros(N_T - 1, dtype=f64))
    with pytest.raises(TypeError, match="dtype"):
        plan.adjoint(torch.zeros(N_VEC, dtype=torch.float32), torch.zeros(N_VEC, dtype=f64),
                     torch.zeros(N_T, dtype=f64))
    with pytest.raises(ValueError, match="elements"):
        plan.pcg_solve(torch.zeros(N_VEC, dtype=f64), x0=torch.zeros(3, dtype=f64))


def test_plan_and_gemm_inputs():
    pix = torch.zeros(N_T, dtype=torch.int32)
    with pytest.raises(TypeError, match="dtype"):
        L.Plan(pix.to(torch.int64), None, 10, [0, N_T], [[1.0, 1.0, 1.0]], n_stokes=1)
    with pytest.raises(ValueError, match="GPU"):
        L.Plan(pix, None, 10, [0, N_T], [[1.0, 1.0, 1.0]], n_stokes=1)
    with pytest.raises(ValueError, match="weights: shape"):
        L.Plan(pix, torch.zeros((N_T - 1, 2)), 10, [0, N_T], [[1.0, 1.0, 1.0]])
    with pytest.raises(TypeError, match="weights: dtype"):
        L.Plan(pix, torch.zeros((N_T, 2), dtype=torch.float16), 10, [0, N_T], [[1.0, 1.0, 1.0]])
    with pytest.raises(ValueError, match="required"):
        L.Plan(pix, None, 10, [0, N_T], [[1.0, 1.0, 1.0]], n_stokes=3)
    with pytest.raises(ValueError, match="GPU"):
        L.gemm_tn_f64(torch.zeros((8, 16), dtype=torch.float64),
                      torch.zeros((8, 16), dtype=torch.float64))
    with pytest.raises(TypeError, match="dtype"):
        L.gemm_tn_f64(torch.zeros((8, 16)), torch.zeros((8, 16), dtype=torch.float64))
    with pytest.raises(ValueError, match="2-D"):
        L.gemm_tn_f64(torch.zeros((8, 16), dtype=torch.float64),
                      torch.zeros((4, 16), dtype=torch.float64))


def test_gls_map_checks_tod_before_planning():
    pix = torch.zeros(N_T, dtype=torch.int32)
    with pytest.raises(ValueError, match="elements"):
        gls_map(torch.zeros(N_T + 1, dtype=torch.float64), torch.ones((1, 3)), pix, None, 10,
                [0, N_T], n_stokes=1)
    with pytest.raises(TypeError, match="dtype"):
        gls_map(torch.zeros(N_T, dtype=torch.int64), torch.ones((1, 3)), pix, None, 10,
                [0, N_T], n_stokes=1)
