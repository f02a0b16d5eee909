"""Batched plans (many independent problems in one plan) on the GPU.

Each problem of a batched solve must equal, bit for bit, the solve of a plan
built for that problem alone with the same FFT lengths (the batch changes
which work items share a launch, never the arithmetic of a problem), and the
captured-graph iteration must equal plain launches.  The operator of each
problem block is checked against the FP64 oracle.
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

N_PROB = 6
GEN = dict(n_problems=N_PROB, side=32, n_min=2 ** 13, n_max=2 ** 16, interval_len=2 ** 12,
           lam=128, fknee_range=(0.1, 5.0), seed_key=4100)
FFT = dict(fft_len_f64=4096, fft_len_f32=4096)


@functools.lru_cache(maxsize=None)
def batch_scan():
    return synth.cfg4_batched_iqu(**GEN)


@functools.lru_cache(maxsize=None)
def single_scan(b):
    return synth.cfg4_batched_iqu(problems=[b], **GEN)


def _plan(sc, **kw):
    kw = dict(FFT, **kw)
    return Plan.from_scan(sc, **kw)


def _blocks(pl, v):
    off = pl.problem_pixels() * pl.n_stokes
    return [v[off[b]:off[b + 1]] for b in range(pl.n_problems)]


def test_batched_layout_and_rhs_match_standalone():
    sc = batch_scan()
    pb = _plan(sc, precision="mixed")
    assert pb.n_problems == N_PROB
    off = pb.problem_pixels()
    assert off[0] == 0 and off[-1] == pb.n_obs and np.all(np.diff(off) > 0)
    d = torch.from_numpy(sc.noise).cuda()
    bb = _blocks(pb, pb.rhs(d))
    hits_b = pb.hits().cpu().numpy()
    perm_b = pb.sorted_samples().cpu().numpy()
    s_off = sc.offsets[sc.problem_offsets]
    for b in range(N_PROB):
        s1 = single_scan(b)
        p1 = _plan(s1, precision="mixed")
        assert p1.n_obs == off[b + 1] - off[b]
        assert np.array_equal(p1.hits().cpu().numpy(), hits_b[off[b]:off[b + 1]])
        perm1 = p1.sorted_samples().cpu().numpy()
        assert np.array_equal(perm1 + s_off[b], perm_b[s_off[b]:s_off[b + 1]])
        b1 = p1.rhs(torch.from_numpy(s1.noise).cuda())
        assert torch.equal(b1, bb[b]), f"rhs of problem {b} differs from its standalone plan"
        for prec in ("fp64", "mixed"):
            x = torch.randn(p1.n_vec, dtype=torch.float64, device="cuda",
                            generator=torch.Generator("cuda").manual_seed(b))
            xb = torch.zeros(pb.n_vec, dtype=torch.float64, device="cuda")
            o3 = off * 3
            xb[o3[b]:o3[b + 1]] = x
            yb = pb.apply_A(xb, precision=prec)
            y1 = p1.apply_A(x, precision=prec)
            assert torch.equal(y1, yb[o3[b]:o3[b + 1]]), (b, prec)
        p1.close()
    pb.close()


def test_batched_operator_vs_oracle():
    sc = batch_scan()
    pb = _plan(sc)
    off3 = pb.problem_pixels() * 3
    for b in (0, N_PROB - 1):
        s1 = single_scan(b)
        pr = O.Problem.from_scan(s1)
        x = np.random.default_rng(b).standard_normal(pr.n_obs * pr.n_s)
        xb = torch.zeros(pb.n_vec, dtype=torch.float64, device="cuda")
        xb[off3[b]:off3[b + 1]] = torch.from_numpy(x).cuda()
        y = pb.apply_A(xb).cpu().numpy()
        check(y[off3[b]:off3[b + 1]], pr.apply_A(x), 1e-12, f"A problem {b}")
        # other problems' blocks of A x stay zero
        mask = np.ones(y.shape[0], bool)
        mask[off3[b]:off3[b + 1]] = False
        assert np.all(y[mask] == 0.0)
    pb.close()


@pytest.mark.parametrize("precision,precond", [("fp64", "bj"), ("mixed", "bj"),
                                               ("mixed", "2lvl"), ("fp64", "2lvl")])
def test_batched_solve_bitwise_equals_standalone(precision, precond):
    sc = batch_scan()
    coarse = precond == "2lvl"
    pb = _plan(sc, precision="mixed" if precision == "mixed" else "fp64", coarse=coarse)
    d = torch.from_numpy(sc.noise).cuda()
    b_all = pb.rhs(d)
    x_all, info = pb.pcg_solve(b_all, precond=precond, precision=precision, tol=1e-9,
                               max_iter=2000)
    assert info["status"] == 0
    xs = _blocks(pb, x_all)
    its = []
    for b in range(N_PROB):
        s1 = single_scan(b)
        p1 = _plan(s1, precision="mixed" if precision == "mixed" else "fp64", coarse=coarse)
        b1 = p1.rhs(torch.from_numpy(s1.noise).cuda())
        x1, i1 = p1.pcg_solve(b1, precond=precond, precision=precision, tol=1e-9, max_iter=2000)
        pi = info["problems"][b]
        assert pi["iterations"] == i1["iterations"], (b, pi["iterations"], i1["iterations"])
        assert pi["replacements"] == i1["replacements"]
        assert np.array_equal(pi["history"], i1["history"])
        assert torch.equal(x1, xs[b]), f"problem {b}: batched solution differs from standalone"
        assert pi["rel_residual"] == i1["rel_residual"]
        assert pi["rel_residual"] <= 1e-9
        its.append(i1["iterations"])
        p1.close()
    assert len(set(its)) > 1, "problems should converge at different iterations (masks)"
    pb.close()


@pytest.mark.parametrize("precision,precond", [("mixed", "2lvl"), ("fp64", "bj")])
def test_graph_replay_equals_plain_launches(precision, precond):
    sc = batch_scan()
    coarse = precond == "2lvl"
    kw = dict(precision="mixed" if precision == "mixed" else "fp64", coarse=coarse)
    pg = _plan(sc, graph=True, **kw)
    pn = _plan(sc, graph=False, **kw)
    d = torch.from_numpy(sc.noise).cuda()
    b = pg.rhs(d)
    assert torch.equal(b, pn.rhs(d))
    # two solves in a row on the graph plan (the second replays the cached graph), with
    # eager work between them
    xg1, ig1 = pg.pcg_solve(b, precond=precond, precision=precision, tol=1e-9, max_iter=2000)
    y = pg.apply_A(xg1)
    xg2, ig2 = pg.pcg_solve(b, precond=precond, precision=precision, tol=1e-9, max_iter=2000)
    xn, inn = pn.pcg_solve(b, precond=precond, precision=precision, tol=1e-9, max_iter=2000)
    assert torch.equal(xg1, xn) and torch.equal(xg2, xn)
    assert torch.equal(y, pn.apply_A(xn))
    for a, c in zip(ig1["problems"], inn["problems"]):
        assert a["iterations"] == c["iterations"]
        assert np.array_equal(a["history"], c["history"])
    pg.close()
    pn.close()


def test_batched_solution_vs_oracle_one_problem():
    sc = batch_scan()
    pb = _plan(sc, coarse=True)
    b_all = pb.rhs(torch.from_numpy(sc.noise).cuda())
    x_all, info = pb.pcg_solve(b_all, precond="2lvl", precision="fp64", tol=1e-13,
                               max_iter=3000)
    k = 2
    s1 = single_scan(k)
    pr = O.Problem.from_scan(s1)
    bo = pr.rhs(s1.noise)
    off3 = pb.problem_pixels() * 3
    check(b_all[off3[k]:off3[k + 1]].cpu().numpy(), bo, 1e-12, "b")
    xo, _, st = O.pcg(pr.apply_A, bo, pr.bj_apply, tol=1e-13, maxit=5000)
    assert rel(x_all[off3[k]:off3[k + 1]].cpu().numpy(), xo) <= 1e-10
    pb.close()


def test_batched_rejects_overlapping_pixel_ranges():
    from paper_1408_3048_amd import MMError
    sc = batch_scan()
    pix = sc.pix.copy()
    s_off = sc.offsets[sc.problem_offsets]
    pix[s_off[1]] = sc.pix[s_off[0]]  # a pixel of problem 0 inside problem 1
    bad = synth.Scan(sc.name, pix, sc.weights, 3, sc.n_pix, sc.offsets, sc.sigma, sc.fknee,
                     sc.alpha, sc.lam, sc.f_samp, sc.sky, sc.noise,
                     problem_offsets=sc.problem_offsets)
    with pytest.raises(MMError) as e:
        _plan(bad)
    assert "disjoint" in str(e.value)


@pytest.mark.parametrize("pt_range", [512, 4096])
def test_pt_range_batched_equals_standalone_and_oracle(pt_range):
    """The P^T work range (opts.pt_range) changes only the order of additions within a
    pixel: a batched plan and standalone plans with the same range agree bit for bit (A x,
    the block-Jacobi blocks through M_BD, a mixed two-level solve), and A x stays within the
    oracle's bars; an autotuned batch reports one of the candidate ranges, and standalone
    plans given its range and FFT lengths agree with it bit for bit."""
    sc = batch_scan()
    pb = _plan(sc, precision="mixed", coarse=True, pt_range=pt_range)
    assert pb.pt_range() == pt_range
    off3 = pb.problem_pixels() * 3
    d = torch.from_numpy(sc.noise).cuda()
    xb_sol, _ = pb.pcg_solve(pb.rhs(d), precond="2lvl", precision="mixed", tol=1e-10,
                             max_iter=3000)
    for b in (0, N_PROB - 1):
        s1 = single_scan(b)
        p1 = _plan(s1, precision="mixed", coarse=True, pt_range=pt_range)
        x = torch.randn(p1.n_vec, dtype=torch.float64, device="cuda",
                        generator=torch.Generator("cuda").manual_seed(b))
        xb = torch.zeros(pb.n_vec, dtype=torch.float64, device="cuda")
        xb[off3[b]:off3[b + 1]] = x
        for prec in ("fp64", "mixed"):
            y1 = p1.apply_A(x, precision=prec)
            assert torch.equal(y1, pb.apply_A(xb, precision=prec)[off3[b]:off3[b + 1]]), (b, prec)
        assert torch.equal(p1.precond_bj(x), pb.precond_bj(xb)[off3[b]:off3[b + 1]]), b
        x1, _ = p1.pcg_solve(p1.rhs(torch.from_numpy(s1.noise).cuda()), precond="2lvl",
                             precision="mixed", tol=1e-10, max_iter=3000)
        assert torch.equal(x1, xb_sol[off3[b]:off3[b + 1]]), b
        pr = O.Problem.from_scan(s1)
        xn = x.cpu().numpy()
        check(p1.apply_A(x, precision="mixed").cpu().numpy(), pr.apply_A(xn), 2e-5, "A fp32")
        check(p1.apply_A(x).cpu().numpy(), pr.apply_A(xn), 1e-12, "A fp64")
        p1.close()
    pb.close()
    # an autotuned batch: a standalone plan given the batch's tuned P^T range and FFT
    # lengths computes the same A x bit for bit
    pt = _plan(sc, precision="mixed", autotune=True, fft_len_f64=0, fft_len_f32=0)
    assert pt.pt_range() in (512, 1024, 2048, 4096)
    n64, n32 = pt.fft_lengths()
    for b in (0, N_PROB - 1):
        p1 = _plan(single_scan(b), precision="mixed", pt_range=pt.pt_range(), fft_len_f64=n64,
                   fft_len_f32=n32)
        x = torch.randn(p1.n_vec, dtype=torch.float64, device="cuda",
                        generator=torch.Generator("cuda").manual_seed(7 + b))
        xb = torch.zeros(pt.n_vec, dtype=torch.float64, device="cuda")
        xb[off3[b]:off3[b + 1]] = x
        for prec in ("fp64", "mixed"):
            assert torch.equal(p1.apply_A(x, precision=prec),
                               pt.apply_A(xb, precision=prec)[off3[b]:off3[b + 1]]), (b, prec)
        p1.close()
    pt.close()
