"""Bandwidth and apodisation of N^-1 on the GPU [Sect. 5.1.3 (Fig. conv_lambda); App. D].

On a strong-1/f IQU raster (32x32 pixels, 4 detectors, 2^16 samples, 16 intervals of
4096, f_knee 2-8 Hz, alpha = 2; 1/(pi t_samp f_knee) is 8 to 32 samples), for
lambda = 0 .. 256: the operator and the block-Jacobi solution against the FP64 oracle at
every bandwidth and for the three windows; lambda = 0 is white-noise weighting (one PCG
step); the block-Jacobi iteration count grows with the bandwidth while the two-level
count grows less; bandwidths below the knee scale give much noisier maps.
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

from gpu_common import check, rel  # noqa: E402

LAMS = (0, 4, 16, 64, 256)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@functools.lru_cache(maxsize=None)
def case(lam, window="gauss"):
    sc = synth.raster_iqu(side=32, spp=8, n_det=4, interval_len=4096, lam=lam,
                          fknee_range=(2.0, 8.0), alpha_range=(2.0, 2.0), seed_key=77,
                          name="raster_iqu_bw")
    pr = O.Problem.from_scan(sc, window=window)
    return sc, pr


@functools.lru_cache(maxsize=None)
def oracle_solve(lam):
    sc, pr = case(lam)
    b = pr.rhs(sc.noise + pr.signal(sc.sky))
    x, it, st = O.pcg(pr.apply_A, b, pr.bj_apply, tol=1e-8, maxit=3000)
    xt, _, st2 = O.pcg(pr.apply_A, b, pr.bj_apply, tol=1e-13, maxit=5000)
    assert st == 0 and st2 == 0
    return b, it, xt


@pytest.mark.parametrize("lam", LAMS)
def test_operator_and_solution_at_every_bandwidth(lam):
    sc, pr = case(lam)
    b, it_o, xt = oracle_solve(lam)
    x = np.random.default_rng(lam).standard_normal(pr.n_obs * 3)
    for prec, tol in (("fp64", 1e-12), ("mixed", 5e-5)):
        pl = Plan.from_scan(sc, precision=prec)
        check(pl.apply_A(dev(x), precision=prec).cpu().numpy(), pr.apply_A(x), tol,
              f"A {prec} lambda={lam}")
        pl.close()
    pl = Plan.from_scan(sc)
    xs, info = pl.pcg_solve(dev(b), precond="bj", tol=1e-13, max_iter=5000)
    assert rel(xs.cpu().numpy(), xt) <= 1e-9
    _, i8 = pl.pcg_solve(dev(b), precond="bj", tol=1e-8, max_iter=3000)
    assert abs(i8["iterations"] - it_o) <= 1, (i8["iterations"], it_o)
    if lam == 0:  # diagonal N^-1: M_BD = A^-1
        assert info["iterations"] == 1
        assert np.allclose(pl.interval_taps(0), [pr.taps[0][0]], rtol=1e-12, atol=0)
    pl.close()


@pytest.mark.parametrize("window", ["gauss2", "rect"])
@pytest.mark.parametrize("lam", [64, 256])
def test_windows(lam, window):
    sc, _ = case(lam)
    pr = O.Problem.from_scan(sc, window=window)
    pl = Plan.from_scan(sc, window=window)
    x = np.random.default_rng(3).standard_normal(pr.n_obs * 3)
    check(pl.apply_A(dev(x)).cpu().numpy(), pr.apply_A(x), 1e-12, f"A {window} lambda={lam}")
    for j in (0, 7):
        assert np.allclose(pl.interval_taps(j), pr.taps[j], rtol=1e-12, atol=1e-14)
    pl.close()


def test_iterations_and_map_quality_across_bandwidths():
    """Fig. conv_lambda and App. D: the block-Jacobi iteration count grows with the
    bandwidth; the two-level count grows less over the last step; bandwidths at or below
    the knee scale (lambda <= 4 here) give maps at least 1.5 times further from the sky
    than lambda = 256."""
    its_bj, its_2l, err = {}, {}, {}
    for lam in LAMS:
        sc, pr = case(lam)
        b, _, _ = oracle_solve(lam)
        m_true = pr.sky_to_compact(sc.sky)
        pl = Plan.from_scan(sc, coarse=True)
        x, ib = pl.pcg_solve(dev(b), precond="bj", tol=1e-8, max_iter=3000)
        _, i2 = pl.pcg_solve(dev(b), precond="2lvl", tol=1e-8, max_iter=3000)
        its_bj[lam], its_2l[lam] = ib["iterations"], i2["iterations"]
        err[lam] = rel(x.cpu().numpy(), m_true)
        pl.close()
    seq = [its_bj[lam] for lam in LAMS]
    assert all(a < b for a, b in zip(seq, seq[1:])), its_bj
    assert its_2l[256] < 0.8 * its_bj[256], (its_2l, its_bj)
    assert its_2l[256] / its_2l[64] < its_bj[256] / its_bj[64], (its_2l, its_bj)
    assert min(err[0], err[4]) > 1.5 * err[256], err
