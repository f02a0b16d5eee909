"""The A-DEF2 two-level preconditioner on the GPU [App. B, eq. ADEF2].

Against the FP64 oracle: the operator M_alt r = R^T M_BD r + Z E^+ Z^T r with Z_S on a
regular and a ragged IQU case and on the I-only case, in FP64 and in mixed plans, and
with the dense a posteriori Z_D; the spectrum shared with A-DEF1 shows up as equal
iteration counts; solves from the A-DEF2 initial guess match the oracle solution; a
batched plan is bitwise equal to standalone plans; captured graphs equal plain launches.
"""

import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
import synth  # noqa: E402
from paper_1408_3048_amd import Plan  # noqa: E402

from gpu_common import TOL_2LVL_AZ16, check, problem, rel  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@functools.lru_cache(maxsize=None)
def coarse_oracle(name):
    sc, pr = problem(name)
    return O.Coarse(pr, O.coarse_zs(pr))


@pytest.mark.parametrize("name,prec", [("small_iqu", "fp64"), ("small_iqu", "mixed"),
                                       ("ragged_iqu", "fp64"), ("ragged_iqu", "mixed"),
                                       ("cfg1", "fp64")])
def test_adef2_operator_zs(name, prec):
    sc, pr = problem(name)
    C = coarse_oracle(name)
    pl = Plan.from_scan(sc, precision=prec, coarse=True)
    rng = np.random.default_rng(15)
    tol = 1e-9 if prec == "fp64" else 1e-4
    for _ in range(2):
        r = rng.standard_normal(pr.n_obs * pr.n_s)
        check(pl.precond_adef2(dev(r)).cpu().numpy(), C.apply_adef2(r), tol, "M_alt")
    # on A z for a column z of Z_S: A-DEF2 against the oracle, while A-DEF1 returns z
    j = int(pl.coarse_columns()[0])
    az = pl.apply_A(dev(C.Z[:, j]))
    a2 = pl.precond_adef2(az).cpu().numpy()
    check(a2, C.apply_adef2(az.cpu().numpy()), tol, "M_alt A z")
    check(pl.precond_2lvl(az).cpu().numpy(), C.Z[:, j],
          1e-9 if prec == "fp64" else TOL_2LVL_AZ16, "M_2lvl A z")
    pl.close()


@pytest.mark.parametrize("name", ["small_iqu", "ragged_iqu"])
def test_adef2_solve_matches_oracle(name):
    sc, pr = problem(name)
    C = coarse_oracle(name)
    b = pr.rhs(pr.signal(sc.sky) + sc.noise)
    xo, ito, st = O.pcg(pr.apply_A, b, C.apply_adef2, tol=1e-13, maxit=3000,
                        x0=C.adef2_start(b))
    assert st == 0
    pl = Plan.from_scan(sc, coarse=True)
    x2, i2 = pl.pcg_solve(dev(b), precond="adef2", tol=1e-13, max_iter=3000)
    assert rel(x2.cpu().numpy(), xo) <= 1e-10
    assert abs(i2["iterations"] - ito) <= 2, (i2["iterations"], ito)
    # same spectrum as A-DEF1: the same number of iterations to a moderate tolerance
    _, i1 = pl.pcg_solve(dev(b), precond="2lvl", tol=1e-8, max_iter=3000)
    _, i2b = pl.pcg_solve(dev(b), precond="adef2", tol=1e-8, max_iter=3000)
    assert abs(i1["iterations"] - i2b["iterations"]) <= 2, (i1["iterations"], i2b["iterations"])
    # from a nonzero initial guess too
    x0 = np.random.default_rng(2).standard_normal(pr.n_obs * pr.n_s)
    x3, i3 = pl.pcg_solve(dev(b), x0=dev(x0), precond="adef2", tol=1e-13, max_iter=3000)
    assert rel(x3.cpu().numpy(), xo) <= 1e-10
    pl.close()


def test_adef2_mixed_solve():
    sc, pr = problem("small_iqu")
    b = pr.rhs(pr.signal(sc.sky) + sc.noise)
    pl = Plan.from_scan(sc, precision="mixed", coarse=True)
    x, info = pl.pcg_solve(dev(b), precond="adef2", precision="mixed", tol=1e-9, max_iter=3000)
    assert info["rel_residual"] <= 1e-9
    xo, _, _ = O.pcg(pr.apply_A, b, pr.bj_apply, tol=1e-13, maxit=3000)
    assert rel(x.cpu().numpy(), xo) <= 1e-7
    xi, ii = pl.pcg_solve(dev(b), precond="adef2", precision="mixed_ir", tol=1e-11,
                          max_iter=3000)
    assert ii["rel_residual"] <= 1e-11 and rel(xi.cpu().numpy(), xo) <= 1e-9
    pl.close()


def test_adef2_with_krylov_coarse_space():
    sc = synth.raster_iqu(side=32, spp=8, n_det=4, interval_len=4096, lam=128,
                          fknee_range=(2.0, 8.0), alpha_range=(2.0, 2.0), seed_key=77,
                          name="raster_iqu_zd")
    pr = O.Problem.from_scan(sc)
    b = pr.rhs(sc.noise + pr.signal(sc.sky))
    pl = Plan.from_scan(sc)
    pl.coarse_from_krylov(dev(b), tol=1e-8, max_iter=3000, eps_tol=0.2)
    (Z,) = pl.dense_columns()
    C = O.Coarse(pr, Z.cpu().numpy().T)
    r = np.random.default_rng(8).standard_normal(pr.n_obs * 3)
    check(pl.precond_adef2(dev(r)).cpu().numpy(), C.apply_adef2(r), 1e-9, "M_alt Z_D")
    b2 = pr.rhs(np.roll(sc.noise, 12345) + pr.signal(sc.sky))
    xo, ito, st = O.pcg(pr.apply_A, b2, C.apply_adef2, tol=1e-12, maxit=3000,
                        x0=C.adef2_start(b2))
    x2, i2 = pl.pcg_solve(dev(b2), precond="adef2", tol=1e-12, max_iter=3000)
    assert st == 0 and rel(x2.cpu().numpy(), xo) <= 1e-9
    assert abs(i2["iterations"] - ito) <= 2
    pl.close()


N_PROB = 5
GEN = dict(n_problems=N_PROB, side=32, n_min=2 ** 13, n_max=2 ** 15, interval_len=2 ** 12,
           lam=128, fknee_range=(0.1, 5.0), seed_key=4400)
FFT = dict(fft_len_f64=4096, fft_len_f32=4096)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adef2_batched_bitwise_equals_standalone(precision):
    sc = synth.cfg4_batched_iqu(**GEN)
    kw = dict(FFT, precision="mixed" if precision == "mixed" else "fp64", coarse=True)
    pb = Plan.from_scan(sc, **kw)
    xb, ib = pb.pcg_solve(pb.rhs(dev(sc.noise)), precond="adef2", precision=precision, tol=1e-9,
                          max_iter=3000)
    off3 = pb.problem_pixels() * 3
    for b in range(N_PROB):
        s1 = synth.cfg4_batched_iqu(problems=[b], **GEN)
        p1 = Plan.from_scan(s1, **kw)
        x1, i1 = p1.pcg_solve(p1.rhs(dev(s1.noise)), precond="adef2", precision=precision,
                              tol=1e-9, max_iter=3000)
        assert i1["iterations"] == ib["problems"][b]["iterations"]
        assert torch.equal(x1, xb[off3[b]:off3[b + 1]]), b
        p1.close()
    pb.close()


def test_adef2_graph_replay_equals_plain_launches():
    sc, pr = problem("small_iqu")
    b = dev(pr.rhs(pr.signal(sc.sky) + sc.noise))
    pg = Plan.from_scan(sc, precision="mixed", coarse=True, graph=True)
    pn = Plan.from_scan(sc, precision="mixed", coarse=True, graph=False)
    xg, ig = pg.pcg_solve(b, precond="adef2", precision="mixed", tol=1e-9, max_iter=3000)
    xg2, _ = pg.pcg_solve(b, precond="adef2", precision="mixed", tol=1e-9, max_iter=3000)
    xn, inn = pn.pcg_solve(b, precond="adef2", precision="mixed", tol=1e-9, max_iter=3000)
    assert torch.equal(xg, xn) and torch.equal(xg2, xn)
    assert ig["iterations"] == inn["iterations"]
    pg.close()
    pn.close()


def test_adef2_fp64_solve_on_a_mixed_plan():
    """A mixed plan stores AZ in FP32; the FP64 A-DEF2 solve recomputes the residual of
    its special start with the FP64 operator and re-applies the coarse correction after a
    residual replacement, so it converges like A-DEF1 to tight tolerances (16x16 IQU, 4
    co-pointed detectors, a rank-3 coarse space from 16 intervals)."""
    sc = synth.raster_iqu(side=16, spp=8, n_det=4, interval_len=1024, lam=64,
                          fknee_range=(0.5, 2.0), alpha_range=(1.0, 2.0), seed_key=99)
    pr = O.Problem.from_scan(sc)
    b = dev(pr.rhs(pr.signal(sc.sky) + sc.noise))
    xo, _, _ = O.pcg(pr.apply_A, b.cpu().numpy(), pr.bj_apply, tol=1e-13, maxit=3000)
    pl = Plan.from_scan(sc, precision="mixed", coarse=True)
    for tol in (1e-8, 1e-12):
        x1, i1 = pl.pcg_solve(b, precond="2lvl", precision="fp64", tol=tol, max_iter=300)
        x2, i2 = pl.pcg_solve(b, precond="adef2", precision="fp64", tol=tol, max_iter=300)
        assert i2["rel_residual"] <= tol and abs(i1["iterations"] - i2["iterations"]) <= 1
    assert rel(x2.cpu().numpy(), xo) <= 1e-10
    pl.close()
