"""The a posteriori coarse space Z_D on the GPU [Sect. 3.3.2; App. A].

A 65536-sample IQU raster (32x32 pixels, 4 detectors, 16 intervals of 4096, lambda =
128, strong 1/f noise: f_knee 2-8 Hz, alpha = 2) whose block-Jacobi PCG run leaves 18
Ritz values of M_BD A below eps_tol = 0.2.  Against the FP64 oracle (the same PCG run,
Lanczos matrix and Ritz vectors written from the paper): the Ritz values, the Z_D
columns, the deflation property M_2lvl,D A Z_D = Z_D, and the solution of a second
system with the new preconditioner; then the mixed-precision plan, a batched plan
(bitwise equal to standalone plans per problem), captured-graph replays after the coarse
space is replaced, and the error path.
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
from paper_1408_3048_amd import MMError, MM_ERR_RANK, Plan  # noqa: E402

from gpu_common import rel  # noqa: E402

EPS_TOL = 0.2
TOL = 1e-8


@functools.lru_cache(maxsize=None)
def scan():
    return synth.raster_iqu(side=32, spp=8, n_det=4, interval_len=4096, lam=128,
                            fknee_range=(2.0, 8.0), alpha_range=(2.0, 2.0), seed_key=77,
                            name="raster_iqu_zd")


@functools.lru_cache(maxsize=None)
def oracle_run():
    sc = scan()
    pr = O.Problem.from_scan(sc)
    b = pr.rhs(sc.noise + pr.signal(sc.sky))
    Bk = pr.bj_blocks()
    x, al, rz, Zk = O.pcg_lanczos(pr.apply_A, b, lambda r: pr.bj_apply(r, Bk), TOL, 3000)
    theta, Y, est = O.ritz_pairs(al, rz, Zk)
    keep = theta < EPS_TOL
    return pr, b, x, al.shape[0], theta[keep], Y[:, keep], est[keep]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@functools.lru_cache(maxsize=None)
def fp64_plan():
    pl = Plan.from_scan(scan())
    pr, b, x_o, m, th_o, Y_o, est = oracle_run()
    x, info = pl.coarse_from_krylov(dev(b), tol=TOL, max_iter=3000, eps_tol=EPS_TOL)
    return pl, x, info


def test_recording_solve_and_ritz_values_match_oracle():
    pr, b, x_o, m, th_o, Y_o, est = oracle_run()
    pl, x, info = fp64_plan()
    assert pl.coarse_kind() == 2
    assert info["status"] == 0 and abs(info["iterations"] - m) <= 1
    assert rel(x.cpu().numpy(), x_o) <= 1e-7
    th = pl.ritz_values()
    assert th.shape[0] == th_o.shape[0] == 18
    # every Ritz value of the recorded run, converged or not, follows the oracle's
    assert np.max(np.abs(th - th_o) / th_o) <= 1e-8, np.abs(th - th_o) / th_o
    assert np.array_equal(pl.coarse_columns(), np.arange(18))


def test_zd_columns_are_the_oracle_ritz_vectors():
    pr, b, x_o, m, th_o, Y_o, est = oracle_run()
    pl, x, info = fp64_plan()
    (Z,) = pl.dense_columns()
    Z = Z.cpu().numpy().T
    assert Z.shape == Y_o.shape
    for i in range(Z.shape[1]):
        y = Y_o[:, i]
        err = min(np.linalg.norm(Z[:, i] - y), np.linalg.norm(Z[:, i] + y)) / np.linalg.norm(y)
        assert err <= 1e-6, (i, err)


def test_deflation_property_and_coarse_matrix():
    """M_2lvl,D A z = z for every column z of Z_D (A-DEF1 maps the coarse space onto
    itself), and E_D = Z_D^T A Z_D."""
    pr, b, x_o, m, th_o, Y_o, est = oracle_run()
    pl, x, info = fp64_plan()
    (Z,) = pl.dense_columns()
    for i in range(Z.shape[0]):
        z = Z[i].contiguous()
        w = pl.precond_2lvl(pl.apply_A(z))
        assert rel(w.cpu().numpy(), z.cpu().numpy()) <= 1e-9, i
    Zn = Z.cpu().numpy().T
    E = Zn.T @ np.stack([pr.apply_A(Zn[:, i]) for i in range(Zn.shape[1])], axis=1)
    assert rel(pl.coarse_matrix(), E) <= 1e-11


def test_rank_past_one_transpose_tile():
    """eps_tol above every Ritz value of the recorded run: all 65 Ritz pairs become Z_D,
    one column more than a tile of the column-to-row transposes feeding the Gram product.
    The Ritz values follow the oracle's, E_D = Z_D^T A Z_D, and M_2lvl,D A z = z holds for
    the columns of the second tile."""
    sc = scan()
    pr, b = oracle_run()[:2]
    Bk = pr.bj_blocks()
    _, al, rz, Zk = O.pcg_lanczos(pr.apply_A, b, lambda r: pr.bj_apply(r, Bk), TOL, 3000)
    theta, _, _ = O.ritz_pairs(al, rz, Zk)
    assert theta.shape[0] == 65 and np.max(theta) < 1.5
    pl = Plan.from_scan(sc)
    pl.coarse_from_krylov(dev(b), tol=TOL, max_iter=3000, eps_tol=1.5)
    th = pl.ritz_values()
    assert th.shape == theta.shape
    assert np.max(np.abs(th - theta) / theta) <= 1e-8
    assert pl.coarse_kind() == 2 and pl.coarse_rank() == 65
    (Z,) = pl.dense_columns()
    Zn = Z.cpu().numpy().T
    E = Zn.T @ np.stack([pr.apply_A(Zn[:, i]) for i in range(Zn.shape[1])], axis=1)
    assert rel(pl.coarse_matrix(), E) <= 1e-11
    for i in range(60, 65):
        z = Z[i].contiguous()
        w = pl.precond_2lvl(pl.apply_A(z))
        assert rel(w.cpu().numpy(), z.cpu().numpy()) <= 1e-9, i
    pl.close()


def test_second_system_solve_matches_oracle_with_fewer_iterations():
    sc = scan()
    pr, b, x_o, m, th_o, Y_o, est = oracle_run()
    pl, x, info = fp64_plan()
    b2 = pr.rhs(np.roll(sc.noise, 12345) + pr.signal(sc.sky))
    x2_o, _, st = O.pcg(pr.apply_A, b2, pr.bj_apply, tol=1e-13, maxit=5000)
    assert st == 0
    xd, idd = pl.pcg_solve(dev(b2), precond="2lvl", tol=1e-12, max_iter=3000)
    assert rel(xd.cpu().numpy(), x2_o) <= 1e-9
    _, ib = pl.pcg_solve(dev(b2), precond="bj", tol=1e-12, max_iter=3000)
    _, id8 = pl.pcg_solve(dev(b2), precond="2lvl", tol=TOL, max_iter=3000)
    _, ib8 = pl.pcg_solve(dev(b2), precond="bj", tol=TOL, max_iter=3000)
    assert id8["iterations"] < 0.8 * ib8["iterations"], (id8["iterations"], ib8["iterations"])
    assert idd["iterations"] < ib["iterations"]
    # the oracle's two-level preconditioner on its own Z_D needs as many iterations
    co = O.Coarse(pr, Y_o)
    _, it_o, st = O.pcg(pr.apply_A, b2, co.apply, tol=TOL, maxit=3000)
    assert st == 0 and abs(id8["iterations"] - it_o) <= 2, (id8["iterations"], it_o)


def test_mixed_plan_a_posteriori_solve():
    sc = scan()
    pr, b, x_o, m, th_o, Y_o, est = oracle_run()
    pl = Plan.from_scan(sc, precision="mixed", coarse=True)
    x, info = pl.coarse_from_krylov(dev(b), tol=TOL, max_iter=3000, eps_tol=EPS_TOL)
    assert pl.coarse_kind() == 2 and pl.coarse_rank() == 18
    assert np.max(np.abs(pl.ritz_values() - th_o) / th_o) <= 1e-8
    b2 = pr.rhs(np.roll(sc.noise, 12345) + pr.signal(sc.sky))
    xm, im = pl.pcg_solve(dev(b2), precond="2lvl", precision="mixed", tol=TOL, max_iter=3000)
    _, ibm = pl.pcg_solve(dev(b2), precond="bj", precision="mixed", tol=TOL, max_iter=3000)
    assert im["rel_residual"] <= TOL
    assert im["iterations"] < 0.8 * ibm["iterations"], (im["iterations"], ibm["iterations"])
    x2_o, _, _ = O.pcg(pr.apply_A, b2, pr.bj_apply, tol=1e-13, maxit=5000)
    assert rel(xm.cpu().numpy(), x2_o) <= 1e-6
    pl.close()


N_PROB = 4
GEN = dict(n_problems=N_PROB, side=32, n_min=2 ** 13, n_max=2 ** 15, interval_len=2 ** 12,
           lam=128, fknee_range=(2.0, 8.0), seed_key=4177)
FFT = dict(fft_len_f64=4096, fft_len_f32=4096)


def test_batched_zd_bitwise_equals_standalone():
    sc = synth.cfg4_batched_iqu(**GEN)
    pb = Plan.from_scan(sc, **FFT)
    b_all = pb.rhs(dev(sc.noise))
    x_all, info = pb.coarse_from_krylov(b_all, tol=TOL, max_iter=3000, eps_tol=0.5)
    cols = pb.coarse_problem_columns()
    th_all = pb.ritz_values()
    Zb = pb.dense_columns()
    d2 = dev(np.roll(sc.noise, 999))
    xs, i2 = pb.pcg_solve(pb.rhs(d2), precond="2lvl", tol=TOL, max_iter=3000)
    off3 = pb.problem_pixels() * 3
    assert sum(np.diff(cols) > 0) >= 2
    for b in range(N_PROB):
        s1 = synth.cfg4_batched_iqu(problems=[b], **GEN)
        p1 = Plan.from_scan(s1, **FFT)
        b1 = p1.rhs(dev(s1.noise))
        assert torch.equal(b1, b_all[off3[b]:off3[b + 1]])
        x1, i1 = p1.coarse_from_krylov(b1, tol=TOL, max_iter=3000, eps_tol=0.5,
                                       raise_on_error=False)
        assert torch.equal(x1, x_all[off3[b]:off3[b + 1]])
        r_b = int(cols[b + 1] - cols[b])
        if r_b == 0:
            assert i1["status"] == MM_ERR_RANK
            p1.close()
            continue
        assert np.array_equal(p1.ritz_values(), th_all[cols[b]:cols[b + 1]])
        assert torch.equal(p1.dense_columns()[0], Zb[b])
        y1, j1 = p1.pcg_solve(p1.rhs(dev(np.roll(sc.noise, 999)[sc.offsets[sc.problem_offsets[b]]:
                                                                  sc.offsets[sc.problem_offsets[b + 1]]])),
                              precond="2lvl", tol=TOL, max_iter=3000)
        assert j1["iterations"] == i2["problems"][b]["iterations"]
        assert torch.equal(y1, xs[off3[b]:off3[b + 1]])
        p1.close()
    pb.close()


def test_graph_replay_after_coarse_space_replacement():
    """A plan that captured its two-level iteration with Z_S must not replay it after
    Z_D replaced the coarse space."""
    sc = scan()
    pr, b, x_o, m, th_o, Y_o, est = oracle_run()
    b2 = dev(pr.rhs(np.roll(sc.noise, 4242)))
    pg = Plan.from_scan(sc, coarse=True, graph=True)
    pn = Plan.from_scan(sc, coarse=True, graph=False)
    xs_g, _ = pg.pcg_solve(b2, precond="2lvl", tol=TOL, max_iter=3000)
    xs_n, _ = pn.pcg_solve(b2, precond="2lvl", tol=TOL, max_iter=3000)
    assert torch.equal(xs_g, xs_n)
    for p in (pg, pn):
        p.coarse_from_krylov(dev(b), tol=TOL, max_iter=3000, eps_tol=EPS_TOL)
    xd_g, ig = pg.pcg_solve(b2, precond="2lvl", tol=TOL, max_iter=3000)
    xd_g2, _ = pg.pcg_solve(b2, precond="2lvl", tol=TOL, max_iter=3000)
    xd_n, inn = pn.pcg_solve(b2, precond="2lvl", tol=TOL, max_iter=3000)
    assert torch.equal(xd_g, xd_n) and torch.equal(xd_g2, xd_n)
    assert ig["iterations"] == inn["iterations"]
    assert not torch.equal(xd_g, xs_g)
    pg.close()
    pn.close()


def test_no_ritz_value_below_threshold_keeps_coarse_space():
    sc = scan()
    pr, b, *_ = oracle_run()
    pl = Plan.from_scan(sc, coarse=True)
    r0 = pl.coarse_rank()
    with pytest.raises(MMError) as e:
        pl.coarse_from_krylov(dev(b), tol=TOL, max_iter=3000, eps_tol=1e-6)
    assert e.value.status == MM_ERR_RANK
    assert pl.coarse_kind() == 1 and pl.coarse_rank() == r0
    x, info = pl.pcg_solve(dev(b), precond="2lvl", tol=TOL, max_iter=3000)
    assert info["rel_residual"] <= TOL
    pl.close()


def test_truncated_basis_cap_and_unconverged_recording():
    """krylov_dim keeps the first steps only: the Ritz values are those of the leading
    block of the oracle's Lanczos matrix; max_cols keeps the smallest; a recording solve
    stopped by max_iter reports MM_ERR_NOCONV and still installs Z_D; bad arguments are
    rejected before any device work."""
    from paper_1408_3048_amd import MM_ERR_ARG, MM_ERR_NOCONV
    sc = scan()
    pr, b, x_o, m, th_o, Y_o, est = oracle_run()
    Bk = pr.bj_blocks()
    _, al, rz, _ = O.pcg_lanczos(pr.apply_A, b, lambda r: pr.bj_apply(r, Bk), TOL, 3000)
    k = 20
    T = O.lanczos_tridiagonal(al[:k], rz[:k + 1])
    ev = np.linalg.eigvalsh(T)
    ev = ev[ev < EPS_TOL]
    pl = Plan.from_scan(sc)
    pl.coarse_from_krylov(dev(b), tol=TOL, max_iter=3000, krylov_dim=k, eps_tol=EPS_TOL)
    th = pl.ritz_values()
    assert th.shape == ev.shape and np.max(np.abs(th - ev) / ev) <= 1e-8
    pl.coarse_from_krylov(dev(b), tol=TOL, max_iter=3000, eps_tol=EPS_TOL, max_cols=5)
    assert np.max(np.abs(pl.ritz_values() - th_o[:5]) / th_o[:5]) <= 1e-8
    x, info = pl.coarse_from_krylov(dev(b), tol=TOL, max_iter=k, eps_tol=EPS_TOL,
                                    raise_on_error=False)
    assert info["status"] == MM_ERR_NOCONV and info["iterations"] == k
    assert pl.coarse_kind() == 2 and pl.coarse_rank() == th.shape[0]
    for bad in (dict(tol=0.0), dict(max_iter=0), dict(eps_tol=-1.0), dict(krylov_dim=-1),
                dict(max_cols=-2)):
        kw = dict(tol=TOL, max_iter=100, eps_tol=EPS_TOL)
        kw.update(bad)
        with pytest.raises(MMError) as e:
            pl.coarse_from_krylov(dev(b), **kw)
        assert e.value.status == MM_ERR_ARG, bad
    assert pl.coarse_kind() == 2
    pl.close()
