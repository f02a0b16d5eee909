"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle on the
same seeded inputs.  Integer outputs are compared bit-exactly; floating-point
outputs both normwise and element by element (max |gpu - oracle| / max |oracle|),
within tolerances derived in the design notes:

  FP64 operators: N^-1, A, b <= 1e-12 (FFT round-off ~ eps log2 n_r amplified by the
                  cancellation of the 1/f kernel's taps); P 1e-15, P^T 1e-14, M_BD 1e-13.
  FP32 operators: N^-1 and A <= 2e-5 (the same with eps = 6e-8), P^T 1e-6.
  Solves: FP64 <= 1e-10, mixed (FP32 operator + FP64 refinement) <= 1e-6 against the
          oracle's tightly converged map.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import synth  # noqa: E402
from gpu_common import TOL_2LVL_AZ16, check, problem, rel, relmax  # noqa: E402

pytestmark = pytest.mark.gpu

from paper_1408_3048_amd import MMError, Plan, gemm_tn_f64  # noqa: E402
import paper_1408_3048_amd as pkg  # noqa: E402

CASES = ["small_iqu", "ragged_iqu", "cfg1"]


@pytest.fixture(scope="module")
def plans():
    cache = {}

    def get(name, **kw):
        key = (name, tuple(sorted(kw.items())))
        if key not in cache:
            sc, _ = problem(name)
            print(f"[plan] {name} {kw}", flush=True)
            cache[key] = Plan.from_scan(sc, **kw)
        return cache[key]
    yield get
    for p in cache.values():
        p.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("name", CASES)
def test_integer_layout_bit_exact(plans, name):
    sc, pr = problem(name)
    pl = plans(name, precision="mixed")
    assert pl.n_obs == pr.n_obs
    assert np.array_equal(pl.obs_pixels().cpu().numpy(), pr.obs.astype(np.int32))
    assert np.array_equal(pl.hits().cpu().numpy(), pr.s.astype(np.int32))
    perm_or = np.lexsort((np.arange(pr.n_t), pr.cid)).astype(np.int32)
    assert np.array_equal(pl.sorted_samples().cpu().numpy(), perm_or)


@pytest.mark.parametrize("name", CASES + ["long_iqu"])
def test_taps(plans, name):
    sc, pr = problem(name)
    pl = plans(name, precision="mixed")
    for j in range(0, pr.offsets.shape[0] - 1, max(1, (pr.offsets.shape[0] - 1) // 5)):
        t = pl.interval_taps(j)
        assert t.shape == pr.taps[j].shape
        assert np.max(np.abs(t - pr.taps[j])) <= 1e-13 * np.max(np.abs(pr.taps[j]))


@pytest.mark.parametrize("name", CASES)
def test_sub_operators(plans, name):
    sc, pr = problem(name)
    pl = plans(name, precision="mixed")
    rng = np.random.default_rng(1)
    x = rng.standard_normal(pr.n_obs * pr.n_s)
    y = rng.standard_normal(pr.n_t)
    # P
    check(pl.apply_P(dev(x)).cpu().numpy(), pr.depoint(x), 1e-15, "P")
    # N^-1, FP64 and FP32
    zr = pr.ninv(y)
    check(pl.apply_Ninv(dev(y)).cpu().numpy(), zr, 1e-12, "N^-1 fp64")
    z32 = pl.apply_Ninv(dev(y.astype(np.float32)), precision="mixed").cpu().numpy()
    check(z32, pr.ninv(y.astype(np.float32).astype(np.float64)), 2e-5, "N^-1 fp32")
    # P^T, FP64 and FP32
    check(pl.apply_PT(dev(y)).cpu().numpy(), pr.point(y), 1e-14, "P^T fp64")
    y32 = y.astype(np.float32)
    check(pl.apply_PT(dev(y32)).cpu().numpy(), pr.point(y32.astype(np.float64)), 1e-6,
          "P^T fp32")


@pytest.mark.parametrize("name", CASES)
def test_apply_A_rhs_bj(plans, name):
    sc, pr = problem(name)
    pl = plans(name, precision="mixed")
    rng = np.random.default_rng(2)
    x = rng.standard_normal(pr.n_obs * pr.n_s)
    Ax = pr.apply_A(x)
    check(pl.apply_A(dev(x)).cpu().numpy(), Ax, 1e-12, "A fp64")
    check(pl.apply_A(dev(x), precision="mixed").cpu().numpy(), Ax, 2e-5, "A fp32")
    d = rng.standard_normal(pr.n_t)
    check(pl.rhs(dev(d)).cpu().numpy(), pr.rhs(d), 1e-12, "b")
    check(pl.precond_bj(dev(x)).cpu().numpy(), pr.bj_apply(x), 1e-13, "M_BD")


@pytest.mark.parametrize("n_r", [4096, 16384, 32768])
def test_ninv_forced_fft_lengths(n_r):
    # every overlap-save tile size, with spectra from the plan-time FFT (n_r = 16384) or
    # direct sums (other lengths); FP64 operator limited to n_r <= 16384
    sc, pr = problem("long_iqu")
    kw = dict(fft_len_f32=n_r, precision="mixed")
    if n_r <= 16384:
        kw["fft_len_f64"] = n_r
    pl = Plan.from_scan(sc, **kw)
    y = np.random.default_rng(8).standard_normal(pr.n_t)
    zr = pr.ninv(y)
    if n_r <= 16384:
        check(pl.apply_Ninv(dev(y)).cpu().numpy(), zr, 1e-12, "N^-1 fp64")
    y32 = y.astype(np.float32)
    z32 = pl.apply_Ninv(dev(y32), precision="mixed").cpu().numpy()
    check(z32, pr.ninv(y32.astype(np.float64)), 2e-5, "N^-1 fp32")
    pl.close()


def test_determinism_bitwise(plans):
    sc, pr = problem("small_iqu")
    pl = plans("small_iqu", precision="mixed")
    x = dev(np.random.default_rng(3).standard_normal(pr.n_obs * 3))
    for prec in ("fp64", "mixed"):
        a = pl.apply_A(x, precision=prec)
        b = pl.apply_A(x, precision=prec)
        assert torch.equal(a, b)


def test_mfma_gemm_layout():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((1000, 48))
    B = rng.standard_normal((1000, 32))
    C = gemm_tn_f64(dev(A), dev(B)).cpu().numpy()
    assert np.max(np.abs(C - A.T @ B)) <= 1e-12 * np.max(np.abs(A.T @ B))


@pytest.mark.parametrize("name,prec", [("small_iqu", "fp64"), ("small_iqu", "mixed"),
                                       ("small_iqu", "mixed32"),
                                       ("ragged_iqu", "mixed"), ("ragged_iqu", "mixed32"),
                                       ("cfg1", "fp64"),
                                       ("strips_i", "fp64"), ("strips_i", "mixed"),
                                       ("strips_i", "mixed32"),
                                       ("hot_i", "fp64"), ("hot_i", "mixed"),
                                       ("many_i", "fp64"), ("many_i", "mixed"),
                                       ("many_i", "mixed32")])
def test_two_level_operator(plans, name, prec):
    """prec: fp64 plans; mixed plans with the FP16 AZ of the A-DEF1 apply (the default);
    mixed32: mixed plans with FP32 AZ."""
    sc, pr = problem(name)
    pl = plans(name, precision="fp64" if prec == "fp64" else "mixed", coarse=True,
               az_fp16=prec == "mixed")
    Z = O.coarse_zs(pr)
    C = O.Coarse(pr, Z)
    cols = pl.coarse_columns()
    assert pl.coarse_rank() == C.rank
    Ek = C.E[np.ix_(cols, cols)]
    tolE = 1e-11 if prec == "fp64" else 2e-5
    assert np.max(np.abs(pl.coarse_matrix() - Ek)) <= tolE * np.max(np.abs(Ek))
    rng = np.random.default_rng(5)
    r = rng.standard_normal(pr.n_obs * pr.n_s)
    tolM = {"fp64": 1e-9, "mixed32": 1e-4, "mixed": TOL_2LVL_AZ16}[prec]
    e = check(pl.precond_2lvl(dev(r)).cpu().numpy(), C.apply(r), tolM, "M_2lvl")
    print(f"[2lvl] {name} {prec}: M_2lvl r {e}", flush=True)
    # M_2lvl A Z = Z on the kept columns
    for j in cols[:4]:
        az = pl.apply_A(dev(Z[:, j]))
        back = pl.precond_2lvl(az).cpu().numpy()
        assert np.max(np.abs(back - Z[:, j])) <= tolM, (j, np.max(np.abs(back - Z[:, j])))


_REF = {}


def reference_map(name):
    if name not in _REF:
        sc, pr = problem(name)
        d = pr.signal(sc.sky) + sc.noise
        b = pr.rhs(d)
        x, it, st = O.pcg(pr.apply_A, b, pr.bj_apply, tol=1e-14, maxit=5000)
        assert st in (0, 1)
        _REF[name] = (d, b, x)
    return _REF[name]


@pytest.mark.parametrize("name", ["small_iqu", "cfg1"])
@pytest.mark.parametrize("pc", ["bj", "2lvl"])
def test_solve_parity(plans, name, pc):
    sc, pr = problem(name)
    d, b_or, x_ref = reference_map(name)
    pl = plans(name, precision="mixed", coarse=True)
    b = pl.rhs(dev(d))
    x, info = pl.pcg_solve(b, precond=pc, precision="fp64", tol=1e-13, max_iter=3000)
    print(name, pc, "fp64", info["iterations"], info["rel_residual"])
    assert info["rel_residual"] <= 1e-13
    assert rel(x.cpu().numpy(), x_ref) <= 1e-10
    x, info = pl.pcg_solve(b, precond=pc, precision="mixed", tol=1e-10, max_iter=3000)
    print(name, pc, "mixed", info["iterations"], info["outer_iterations"], info["rel_residual"])
    assert info["rel_residual"] <= 1e-10
    assert rel(x.cpu().numpy(), x_ref) <= 1e-6


def test_noiseless_recovers_map_and_white_noise_one_iteration(plans):
    sc = synth.raster_iqu(side=16, spp=8, n_det=4, interval_len=2048, lam=128, seed_key=41)
    pr = O.Problem.from_scan(sc)
    pl = Plan.from_scan(sc)
    m = pr.sky_to_compact(sc.sky)
    d = pl.apply_P(dev(m))
    x, info = pl.pcg_solve(pl.rhs(d), tol=1e-13, max_iter=1000)
    assert rel(x.cpu().numpy(), m) <= 1e-10
    pl.close()
    sc.fknee[:] = 0.0
    pl = Plan.from_scan(sc)
    d = dev(np.random.default_rng(6).standard_normal(sc.n_samples))
    x, info = pl.pcg_solve(pl.rhs(d), tol=1e-12, max_iter=10)
    assert info["iterations"] == 1
    pl.close()


def test_error_paths_on_device():
    # one polariser angle only: every IQU block is singular -> MM_ERR_RANK
    sc = synth.raster_iqu(side=8, spp=4, n_det=1, interval_len=512, lam=16, hwp_hz=0.0,
                          seed_key=43)
    with pytest.raises(MMError) as e:
        Plan.from_scan(sc)
    assert e.value.status == pkg.MM_ERR_RANK
    # steep 1/f with a rectangular band of 4 lags: the symbol dips below zero
    sc = synth.raster_i(side=8, spp=4, n_pass=2, interval_len=256, lam=4, fknee=50.0, alpha=3.0)
    sc.offsets = np.array([0, 512])
    sc.sigma, sc.fknee, sc.alpha = sc.sigma[:1], sc.fknee[:1], sc.alpha[:1]
    with pytest.raises(MMError) as e:
        Plan.from_scan(sc, window="rect")
    assert e.value.status == pkg.MM_ERR_NOT_SPD
    # pixel id out of range -> MM_ERR_ARG
    sc = synth.raster_i(side=8, spp=4, n_pass=2, interval_len=256, lam=16)
    pix = torch.from_numpy(sc.pix).cuda()
    with pytest.raises(MMError) as e:
        Plan(pix, None, 10, sc.offsets, np.stack([sc.sigma, sc.fknee, sc.alpha], 1), n_stokes=1,
             lam=16)
    assert e.value.status == pkg.MM_ERR_ARG
    # maxit too small -> MM_ERR_NOCONV, x holds the last iterate
    pl = Plan.from_scan(sc)
    b = pl.rhs(dev(np.random.default_rng(7).standard_normal(sc.n_samples)))
    x, info = pl.pcg_solve(b, tol=1e-14, max_iter=2, raise_on_error=False)
    assert info["status"] == pkg.MM_ERR_NOCONV and info["iterations"] == 2
    assert torch.isfinite(x).all() and x.abs().sum() > 0
    pl.close()


def test_warm_start_initial_residual_is_fp64(plans):
    """A given x0 is judged by its FP64 true residual in every precision: started at an
    FP64 solution that meets tol, the mixed solve takes no iteration (the FP32 operator's
    residual, ~1e-7 relative, would not have passed) and returns x0 unchanged with MM_OK;
    the reported residual is the FP64 one."""
    sc, pr = problem("small_iqu")
    d, b_or, x_ref = reference_map("small_iqu")
    pl = plans("small_iqu", precision="mixed", coarse=True)
    b = pl.rhs(dev(d))
    x, info = pl.pcg_solve(b, precond="bj", precision="fp64", tol=1e-12, max_iter=3000)
    tol = 2.0 * info["rel_residual"]
    for prec in ("fp64", "mixed"):
        x2, i2 = pl.pcg_solve(b, x0=x, precond="bj", precision=prec, tol=tol, max_iter=3000)
        assert i2["iterations"] == 0 and i2["status"] == pkg.MM_OK, (prec, i2)
        assert i2["rel_residual"] <= tol and torch.equal(x2, x), prec
    # a start just off the solution: the mixed solve iterates until the FP64 residual passes
    x3, i3 = pl.pcg_solve(b, x0=x * (1 + 1e-6), precond="2lvl", precision="mixed", tol=1e-11,
                          max_iter=3000)
    assert i3["iterations"] > 0 and i3["rel_residual"] <= 1e-11
    assert rel(x3.cpu().numpy(), x_ref) <= 1e-9
