"""The plan's two rejection gates against the oracle's values, on either side of their
thresholds:

- block conditioning [Sect. 3.1, eq. stdPrec]: a pixel's n_s x n_s block of
  P^T diag(N^-1) P with rcond_1 below opts.rcond_min is MM_ERR_RANK.  With rcond_min a
  hair below / above the oracle's smallest rcond (Problem.bj_rcond) the plan is accepted /
  rejected, and the rejection names the oracle's worst pixel and its rcond.
- positive definiteness of N^-1 [Sect. 2.1, eq. N_def; App. D]: a band Toeplitz block
  whose symbol t_0 + 2 sum t_k cos(k theta) is <= 0 somewhere on the FFT grid is
  MM_ERR_NOT_SPD.  For a steep 1/f spectrum with a rectangular band of 4 lags the symbol's
  minimum crosses zero as f_knee grows; on either side of the crossing (found on the
  oracle's symbol on the same grid) the plan is accepted / rejected, and the rejection
  reports the oracle's minimum."""

import re

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
import synth  # noqa: E402
import paper_1408_3048_amd as pkg  # noqa: E402
from paper_1408_3048_amd import MMError, Plan  # noqa: E402


def test_rcond_gate_against_the_oracle():
    sc = synth.raster_iqu(side=16, spp=8, n_det=2, interval_len=1024, lam=32, hwp_hz=0.3,
                          seed_key=61)
    pr = O.Problem.from_scan(sc)
    rc = pr.bj_rcond()
    worst = int(np.argmin(rc))
    r0 = float(rc[worst])
    assert 1e-6 < r0 < 0.5 and np.sum(rc <= r0 * (1 + 1e-5)) == 1
    print(f"[gate] oracle min rcond {r0:.6e} at compact pixel {worst}", flush=True)
    pl = Plan.from_scan(sc, rcond_min=r0 * (1 - 1e-5))
    pl.close()
    with pytest.raises(MMError) as e:
        Plan.from_scan(sc, rcond_min=r0 * (1 + 1e-5))
    assert e.value.status == pkg.MM_ERR_RANK
    msg = str(e.value)
    assert f"compact {worst})" in msg, msg
    rc_dev = float(re.search(r"rcond ([0-9.eE+-]+) <", msg).group(1))
    assert rc_dev == pytest.approx(r0, rel=2e-3)  # printed with 4 significant digits


def _symbol_case(fknee):
    sc = synth.raster_i(side=8, spp=4, n_pass=2, interval_len=256, lam=4, fknee=fknee,
                        alpha=3.0, seed_key=62)
    sc.offsets = np.array([0, sc.n_samples])
    sc.sigma, sc.fknee, sc.alpha = sc.sigma[:1], sc.fknee[:1], sc.alpha[:1]
    return sc


N_R = 4096  # the FP64 tile length forced below: the symbol is checked on its grid


def _oracle_min(fknee):
    sc = _symbol_case(fknee)
    t = O.toeplitz_taps(sc.n_samples, 1.0, fknee, 3.0, 4, sc.f_samp, "rect")
    s = O.taps_symbol(t, N_R // 2 + 1)  # theta_m = 2 pi m / N_R, m = 0 .. N_R / 2
    return float(s.min()), float(s.max())


def test_symbol_gate_against_the_oracle():
    lo, hi = 10.0, 20.0
    assert _oracle_min(lo)[0] > 0 > _oracle_min(hi)[0]
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if _oracle_min(mid)[0] > 0:
            lo = mid
        else:
            hi = mid
    f0 = 0.5 * (lo + hi)
    for fk, positive in ((f0 * (1 - 2e-3), True), (f0 * (1 + 2e-3), False)):
        smin, smax = _oracle_min(fk)
        assert (smin > 0) == positive and abs(smin) >= 1e-5 * smax, (fk, smin)
        print(f"[gate] f_knee {fk:.6f}: oracle symbol min {smin:.4e}", flush=True)
        sc = _symbol_case(fk)
        if positive:
            Plan.from_scan(sc, window="rect", fft_len_f64=N_R).close()
        else:
            with pytest.raises(MMError) as e:
                Plan.from_scan(sc, window="rect", fft_len_f64=N_R)
            assert e.value.status == pkg.MM_ERR_NOT_SPD
            dev_min = float(re.search(r"symbol min ([0-9.eE+-]+)", str(e.value)).group(1))
            assert dev_min == pytest.approx(smin, rel=2e-3), (dev_min, smin)
