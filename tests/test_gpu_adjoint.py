"""Adjoint of the GLS map on the GPU: lag correlations, tap derivatives, the full
gradient against the FP64 oracle (16x16 IQU sub-case), the autograd Function, and
central finite differences at the full 2^22-sample size."""

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
from paper_1408_3048_amd.autograd import gls_map  # noqa: E402

from gpu_common import long_iqu, ragged_iqu  # noqa: E402


def sub16():
    """The 16x16 IQU sub-case of the 2^22-sample configuration: same generator, 2^14
    samples (4 detectors, two passes), 32 intervals of 512, lambda = 64."""
    return synth.raster_iqu(16, 8, 4, 512, 64, (0.5, 2.0), (1.0, 2.0), seed_key=5000,
                            name="cfg5_sub16")


@functools.lru_cache(maxsize=None)
def sub16_problem():
    sc = sub16()
    return sc, O.Problem.from_scan(sc)


@functools.lru_cache(maxsize=None)
def sub16_oracle():
    """Oracle map and gradients of L = ||m_hat - m_true||^2 on the sub-case."""
    sc, pr = sub16_problem()
    d_np = sc.noise + pr.signal(sc.sky)
    m_true = pr.sky_to_compact(sc.sky)
    m_o = O.map_gradients(pr, d_np, np.zeros(pr.n_obs * pr.n_s))[0]
    _, gd_o, gt_o, mu_o = O.map_gradients(pr, d_np, 2.0 * (m_o - m_true))
    return d_np, m_true, m_o, gd_o, gt_o, mu_o


def _relmax(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("make", [ragged_iqu, sub16])
def test_lag_correlations_vs_oracle(make):
    sc = make()
    pl = Plan.from_scan(sc)
    rng = np.random.default_rng(21)
    u = rng.standard_normal(sc.n_samples)
    v = rng.standard_normal(sc.n_samples)
    c = pl.lag_correlations(torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda()).cpu().numpy()
    for j in range(sc.offsets.shape[0] - 1):
        a, b = sc.offsets[j], sc.offsets[j + 1]
        ref = O.lag_correlations(u[a:b], v[a:b], sc.lam)
        k = ref.shape[0]
        assert np.max(np.abs(c[j, :k] - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))), j
        assert np.all(c[j, k:] == 0.0)
    pl.close()


@pytest.mark.parametrize("make", [ragged_iqu, long_iqu, sub16])
def test_tap_derivatives_vs_oracle(make):
    """Direct cosine-sum path (uneven lengths) and the decimated FFT path (2^16)."""
    sc = make()
    pl = Plan.from_scan(sc)
    dt = pl.tap_derivatives()
    for j in range(sc.offsets.shape[0] - 1):
        n = int(sc.offsets[j + 1] - sc.offsets[j])
        ref = O.tap_derivatives(n, sc.sigma[j], sc.fknee[j], sc.alpha[j], sc.lam, sc.f_samp)
        k = ref.shape[1]
        for i in range(3):
            scale = max(np.max(np.abs(ref[i])), 1e-300)
            assert np.max(np.abs(dt[j, i, :k] - ref[i])) <= 1e-10 * scale, (j, i)
        assert np.all(dt[j, :, k:] == 0.0)
    pl.close()


def test_adjoint_vs_oracle_sub16():
    sc, pr = sub16_problem()
    d_np, m_true, m_o, gd_o, gt_o, mu_o = sub16_oracle()
    for precond in ("bj", "2lvl"):
        pl = Plan.from_scan(sc, coarse=precond == "2lvl")
        d = torch.from_numpy(d_np).cuda()
        m, info = pl.pcg_solve(pl.rhs(d), precond=precond, tol=1e-13, max_iter=3000)
        assert _relmax(m.cpu().numpy(), m_o) <= 1e-9
        g = 2.0 * (m - torch.from_numpy(m_true).cuda())
        gd, gt, mu, ainfo = pl.adjoint(m, g, d, precond=precond, tol=1e-13, max_iter=3000)
        assert _relmax(mu.cpu().numpy(), mu_o) <= 1e-8
        assert _relmax(gd.cpu().numpy(), gd_o) <= 1e-8
        assert _relmax(gt, gt_o) <= 1e-7
        pl.close()


@functools.lru_cache(maxsize=None)
def sub16_oracle_fp32_tod():
    """Oracle map and gradients of the sub-case for the FP32-rounded TOD (its values taken
    exactly in FP64)."""
    sc, pr = sub16_problem()
    d_np = sub16_oracle()[0].astype(np.float32)
    d64 = d_np.astype(np.float64)
    m_true = pr.sky_to_compact(sc.sky)
    m_o = O.map_gradients(pr, d64, np.zeros(pr.n_obs * pr.n_s))[0]
    _, gd_o, gt_o, mu_o = O.map_gradients(pr, d64, 2.0 * (m_o - m_true))
    return d_np, m_true, m_o, gd_o, gt_o, mu_o


def test_adjoint_fp32_tod_and_mixed_solve_sub16():
    """FP32 TOD in, FP32 dL/dd out, and the mu solve in mixed precision (FP32 operator,
    FP64 true residual), against the dense oracle on the FP32-rounded TOD.  Bars: the map
    and mu as the FP64 path (the mixed solve stops on the same FP64 residual; kappa(A) is
    about 4 here); dL/dd in FP32 within 1e-7 of its largest entry (one FP32 rounding)."""
    sc, pr = sub16_problem()
    d_np, m_true, m_o, gd_o, gt_o, mu_o = sub16_oracle_fp32_tod()
    pl = Plan.from_scan(sc, precision="mixed", coarse=True)
    d = torch.from_numpy(d_np).cuda()
    mt = torch.from_numpy(m_true).cuda()
    for precision, tol in (("fp64", 1e-13), ("mixed", 1e-11)):
        m, info = pl.pcg_solve(pl.rhs(d), precond="2lvl", precision=precision, tol=tol,
                               max_iter=3000)
        assert _relmax(m.cpu().numpy(), m_o) <= 1e-9, precision
        g = 2.0 * (m - mt)
        gd, gt, mu, ainfo = pl.adjoint(m, g, d, precond="2lvl", precision=precision, tol=tol,
                                       max_iter=3000, grad_d_dtype=torch.float32)
        assert gd.dtype == torch.float32
        assert ainfo["rel_residual"] <= tol, (precision, ainfo)
        print(f"[adjoint] {precision}: mu {_relmax(mu.cpu().numpy(), mu_o):.2e} "
              f"grad_d {_relmax(gd.cpu().numpy(), gd_o):.2e} "
              f"grad_psd {_relmax(gt, gt_o):.2e}", flush=True)
        assert _relmax(mu.cpu().numpy(), mu_o) <= 1e-8, precision
        assert _relmax(gd.cpu().numpy(), gd_o) <= 1e-7, precision
        assert _relmax(gt, gt_o) <= 1e-7, precision
        gd64, gt64, _, _ = pl.adjoint(m, g, d, precond="2lvl", precision=precision, tol=tol,
                                      max_iter=3000, grad_d_dtype=torch.float64)
        assert _relmax(gd64.cpu().numpy(), gd_o) <= 1e-8, precision
        # the FP32 output is the FP64 gradient rounded once
        assert torch.equal(gd, gd64.to(torch.float32)), precision
    pl.close()


def test_autograd_fp32_tod_mixed_sub16():
    """The autograd Function with an FP32 TOD and mixed-precision solves: d.grad is FP32."""
    sc, pr = sub16_problem()
    d_np, m_true, m_o, gd_o, gt_o, mu_o = sub16_oracle_fp32_tod()
    d = torch.from_numpy(d_np).cuda().requires_grad_(True)
    psd = torch.tensor(np.stack([sc.sigma, sc.fknee, sc.alpha], 1), dtype=torch.float64,
                       requires_grad=True)
    pix = torch.from_numpy(sc.pix).cuda()
    w = torch.from_numpy(sc.weights).cuda()
    m = gls_map(d, psd, pix, w, sc.n_pix, sc.offsets, lam=sc.lam, f_samp=sc.f_samp,
                precond="2lvl", precision="mixed", tol=1e-11)
    assert _relmax(m.detach().cpu().numpy(), m_o) <= 1e-9
    loss = ((m - torch.from_numpy(m_true).cuda()) ** 2).sum()
    loss.backward()
    assert d.grad.dtype == torch.float32
    assert _relmax(d.grad.cpu().numpy(), gd_o) <= 1e-7
    assert _relmax(psd.grad.numpy(), gt_o) <= 1e-7


def test_autograd_function_sub16():
    sc, pr = sub16_problem()
    d_np, m_true, m_o, gd_o, gt_o, mu_o = sub16_oracle()
    d = torch.from_numpy(d_np).cuda().requires_grad_(True)
    psd = torch.tensor(np.stack([sc.sigma, sc.fknee, sc.alpha], 1), dtype=torch.float64,
                       requires_grad=True)
    pix = torch.from_numpy(sc.pix).cuda()
    w = torch.from_numpy(sc.weights).cuda()
    m = gls_map(d, psd, pix, w, sc.n_pix, sc.offsets, lam=sc.lam, f_samp=sc.f_samp,
                precond="2lvl", tol=1e-13)
    loss = ((m - torch.from_numpy(m_true).cuda()) ** 2).sum()
    loss.backward()
    assert _relmax(d.grad.cpu().numpy(), gd_o) <= 1e-8
    assert _relmax(psd.grad.numpy(), gt_o) <= 1e-7


def test_cfg5_gradient_vs_central_differences():
    """2^22 samples, 256x256 IQU, 32 intervals of 2^17, lambda = 2048: the adjoint
    gradient of L = ||m_hat - m_true||^2 against central differences (h = 1e-6 relative,
    FP64 solves to 1e-13) for a few noise parameters and one TOD direction."""
    sc = synth.cfg5_raster_iqu()
    pix = torch.from_numpy(sc.pix).cuda()
    w = torch.from_numpy(sc.weights).cuda()
    psd0 = np.stack([sc.sigma, sc.fknee, sc.alpha], 1)
    kw = dict(n_stokes=3, lam=sc.lam, f_samp=sc.f_samp, coarse=True)
    helper = Plan(pix, w, sc.n_pix, sc.offsets, psd0, **kw)
    obs = helper.obs_pixels().long()
    m_true = torch.from_numpy(sc.sky).cuda()[obs].reshape(-1).contiguous()
    d = helper.apply_P(m_true) + torch.from_numpy(sc.noise).cuda()
    helper.close()

    def loss(psd, dd):
        pl = Plan(pix, w, sc.n_pix, sc.offsets, psd, **kw)
        m, info = pl.pcg_solve(pl.rhs(dd), precond="2lvl", tol=1e-13, max_iter=5000,
                               history=False)
        val = float(((m - m_true) ** 2).sum())
        return val, pl, m

    L0, pl, m = loss(psd0, d)
    gd, gt, _, _ = pl.adjoint(m, 2.0 * (m - m_true), d, precond="2lvl", tol=1e-13,
                              max_iter=5000)
    pl.close()
    for j, i in [(3, 0), (17, 1), (30, 2)]:
        h = 1e-6 * psd0[j, i]
        pp, pm = psd0.copy(), psd0.copy()
        pp[j, i] += h
        pm[j, i] -= h
        Lp, plp, _ = loss(pp, d)
        plp.close()
        Lm, plm, _ = loss(pm, d)
        plm.close()
        fd = (Lp - Lm) / (2 * h)
        assert fd == pytest.approx(gt[j, i], rel=1e-4, abs=1e-7 * np.max(np.abs(gt))), (j, i)
    e = torch.randn(sc.n_samples, dtype=torch.float64, device="cuda",
                    generator=torch.Generator("cuda").manual_seed(5))
    h = 1e-3
    Lp, plp, _ = loss(psd0, d + h * e)
    plp.close()
    Lm, plm, _ = loss(psd0, d - h * e)
    plm.close()
    fd = (Lp - Lm) / (2 * h)
    assert fd == pytest.approx(float(gd @ e), rel=1e-6)


def test_cfg5_fp32_tod_and_mixed_adjoint_vs_central_differences():
    """The 2^22-sample case with the TOD in FP32: the adjoint's FP32 dL/dd and its noise
    gradients, from an FP64 and from a mixed-precision mu solve, against central
    differences of the loss (FP64 solves to 1e-13 on the FP32 data).  The loss is quadratic
    in d, so along the FP32 perturbation actually applied (d32(+) - d32(-)) / 2 the
    difference quotient is exact up to the solves' accuracy."""
    sc = synth.cfg5_raster_iqu()
    pix = torch.from_numpy(sc.pix).cuda()
    w = torch.from_numpy(sc.weights).cuda()
    psd0 = np.stack([sc.sigma, sc.fknee, sc.alpha], 1)
    kw = dict(n_stokes=3, lam=sc.lam, f_samp=sc.f_samp, coarse=True, precision="mixed")
    helper = Plan(pix, w, sc.n_pix, sc.offsets, psd0, **kw)
    obs = helper.obs_pixels().long()
    m_true = torch.from_numpy(sc.sky).cuda()[obs].reshape(-1).contiguous()
    d = (helper.apply_P(m_true) + torch.from_numpy(sc.noise).cuda()).to(torch.float32)
    helper.close()

    def loss(psd, dd):
        pl = Plan(pix, w, sc.n_pix, sc.offsets, psd, **kw)
        m, info = pl.pcg_solve(pl.rhs(dd), precond="2lvl", tol=1e-13, max_iter=5000,
                               history=False)
        return float(((m - m_true) ** 2).sum()), pl, m

    L0, pl, m = loss(psd0, d)
    g = 2.0 * (m - m_true)
    gd, gt, _, _ = pl.adjoint(m, g, d, precond="2lvl", tol=1e-13, max_iter=5000,
                              grad_d_dtype=torch.float32)
    gdm, gtm, _, im = pl.adjoint(m, g, d, precond="2lvl", precision="mixed", tol=1e-11,
                                 max_iter=5000, grad_d_dtype=torch.float32)
    pl.close()
    assert gd.dtype == torch.float32 and gdm.dtype == torch.float32
    print(f"[adjoint 2^22] mixed vs fp64 mu solve: grad_d {_relmax(gdm.cpu().numpy(), gd.cpu().numpy()):.2e}"
          f" grad_psd {_relmax(gtm, gt):.2e} ({im['iterations']} iterations)", flush=True)
    assert _relmax(gdm.cpu().numpy(), gd.cpu().numpy()) <= 1e-6
    assert _relmax(gtm, gt) <= 1e-6
    for j, i in [(5, 0), (20, 1), (9, 2)]:
        h = 1e-6 * psd0[j, i]
        pp, pm = psd0.copy(), psd0.copy()
        pp[j, i] += h
        pm[j, i] -= h
        Lp, plp, _ = loss(pp, d)
        plp.close()
        Lm, plm, _ = loss(pm, d)
        plm.close()
        fd = (Lp - Lm) / (2 * h)
        for grad in (gt, gtm):
            assert fd == pytest.approx(grad[j, i], rel=1e-4, abs=1e-7 * np.max(np.abs(grad))), (j, i)
    e = torch.randn(sc.n_samples, dtype=torch.float64, device="cuda",
                    generator=torch.Generator("cuda").manual_seed(6))
    h = 1e-3
    dp = (d.double() + h * e).to(torch.float32)
    dm = (d.double() - h * e).to(torch.float32)
    Lp, plp, _ = loss(psd0, dp)
    plp.close()
    Lm, plm, _ = loss(psd0, dm)
    plm.close()
    e_eff = (dp.double() - dm.double()) / 2.0  # the perturbation actually applied, times h
    fd = (Lp - Lm) / 2.0
    for grad in (gd, gdm):
        assert fd == pytest.approx(float(grad.double() @ e_eff), rel=1e-5)
