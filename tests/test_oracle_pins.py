"""Pins of the FP64 oracle against what the paper and the mathematics fix
(closed forms, explicit matrices, invariants, special cases).  CPU only."""

import numpy as np
import pytest

import oracle as O
import synth


def tiny_iqu(fknee=(0.5, 2.0), alpha=(1.0, 2.0), lam=64, interval_len=1024, seed=7):
    # 8x8 IQU patch, 4 co-pointed detectors, H+V passes, 2^12 samples
    return synth.raster_iqu(side=8, spp=8, n_det=4, interval_len=interval_len, lam=lam,
                            fknee_range=fknee, alpha_range=alpha, seed_key=seed)


def tiny_i(fknee=1.0, lam=32, seed=11):
    return synth.raster_i(side=8, spp=4, n_pass=8, interval_len=256, lam=lam,
                          sigma=1.0, fknee=fknee, alpha=1.0, seed_key=seed)


# ------------------------------------------------------------------ P1: taps

def test_inverse_psd_grid_hand_values():
    # f_m = m * f_samp / n: with n = f_samp = 200 the grid is 1 Hz
    q = O.inverse_psd(200, sigma=1.0, fknee=1.0, alpha=1.0, f_samp=200.0)
    assert q[0] == 0.0
    assert q[1] == pytest.approx(0.5, rel=1e-15)
    assert q[2] == pytest.approx(2.0 / 3.0, rel=1e-15)
    q2 = O.inverse_psd(400, sigma=2.0, fknee=3.0, alpha=2.0, f_samp=200.0)
    # f_2 = 1 Hz: 1 / (4 (1 + 9))
    assert q2[2] == pytest.approx(1.0 / 40.0, rel=1e-15)
    qw = O.inverse_psd(64, sigma=0.5, fknee=0.0, alpha=1.0, f_samp=200.0)
    assert np.all(qw == 4.0)


@pytest.mark.parametrize("n", [512, 513, 1000])
@pytest.mark.parametrize("window", ["gauss", "rect"])
def test_taps_match_explicit_cosine_sum(n, window):
    t = O.toeplitz_taps(n, 1.3, 1.7, 1.4, 48, 200.0, window)
    tc = O.toeplitz_taps_cosine_sum(n, 1.3, 1.7, 1.4, 48, 200.0, window)
    assert t.shape == (49,)
    assert np.max(np.abs(t - tc)) <= 1e-13 * np.max(np.abs(tc))


def test_taps_white_noise_closed_form():
    t = O.toeplitz_taps(4096, 2.0, 0.0, 1.0, 256, 200.0)
    assert t[0] == pytest.approx(0.25, rel=1e-14)
    assert np.max(np.abs(t[1:])) < 1e-16


def test_taps_clipped_to_interval_and_window_values():
    t = O.toeplitz_taps(100, 1.0, 1.0, 1.0, 500, 200.0, "rect")
    assert t.shape == (100,)
    full = np.fft.irfft(O.inverse_psd(1000, 1.0, 1.0, 1.0, 200.0), 1000)
    tg = O.toeplitz_taps(1000, 1.0, 1.0, 1.0, 50, 200.0, "gauss")
    assert tg[50] == pytest.approx(full[50] * np.exp(-1.0), rel=1e-12)
    assert tg[0] == pytest.approx(full[0], rel=1e-15)


def test_unwindowed_row_suppresses_the_mean():
    # q_0 = 0: the full periodic row sums to zero, i.e. N^-1 1_t = 0 for the
    # unbanded circulant (the near-null direction of eq. AsingVect)
    n = 1024
    row = np.fft.irfft(O.inverse_psd(n, 1.0, 1.0, 1.5, 200.0), n)
    assert abs(row.sum()) < 1e-14 * np.abs(row).sum()
    assert row[0] > 0 and row[1] < 0


def test_symbol_positive_and_bounded_gaussian_window():
    for (n, lam, fk, al) in [(2 ** 16, 2048, 2.0, 2.0), (2 ** 14, 1024, 5.0, 1.0),
                             (2 ** 14, 1024, 1.0, 1.0)]:
        t = O.toeplitz_taps(n, 1.0, fk, al, lam, 200.0)
        s = O.taps_symbol(t, 1 << 15)
        assert s.min() > 0.0
        assert s.max() <= 1.0 + 1e-6


# -------------------------------------------------------- P2: Toeplitz apply

def test_banded_sums_equal_explicit_toeplitz_matrices():
    rng = np.random.default_rng(0)
    offsets = np.array([0, 700, 730, 2000, 2100])
    taps = [O.toeplitz_taps(int(offsets[j + 1] - offsets[j]), 1.0, 1.0 + j, 1.5, 64, 200.0)
            for j in range(4)]
    y = rng.standard_normal(2100)
    z = O.toeplitz_apply(y, offsets, taps)
    ref = np.zeros_like(y)
    for j in range(4):
        a, b = offsets[j], offsets[j + 1]
        ref[a:b] = O.toeplitz_dense(taps[j], b - a) @ y[a:b]
    assert np.max(np.abs(z - ref)) <= 1e-13 * np.max(np.abs(ref))
    y2 = rng.standard_normal(2100)
    lhs = O.toeplitz_apply(y, offsets, taps) @ y2
    rhs = y @ O.toeplitz_apply(y2, offsets, taps)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    ts = np.array([0, 5, 699, 700, 729, 1500, 2099])
    assert np.allclose(O.toeplitz_apply_at(y, offsets, taps, ts), ref[ts], rtol=0, atol=1e-13)


# --------------------------------------------------------------- P3: P, P^T

def test_pointing_adjoint_and_hits():
    sc = tiny_iqu()
    pr = O.Problem.from_scan(sc)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(pr.n_obs * 3)
    y = rng.standard_normal(pr.n_t)
    assert pr.depoint(x) @ y == pytest.approx(x @ pr.point(y), rel=1e-12)
    assert np.array_equal(pr.s, np.full(64, 4 * 2 * 8))  # 4 dets x 2 passes x 8 spp


def test_cfg1_geometry_hits_exact():
    sc = synth.cfg1_raster_i()
    obs, cid = O.compact(sc.pix)
    assert obs.shape[0] == 4096
    assert np.array_equal(O.hits(cid, 4096), np.full(4096, 64, dtype=np.int64))


def test_intensity_pointing_of_ones_is_hits():
    pr = O.Problem.from_scan(tiny_i())
    assert np.array_equal(pr.point(np.ones(pr.n_t)), pr.s.astype(np.float64))


# ------------------------------------------------------------------- P4: A

def test_A_symmetric_positive_definite_and_matches_dense():
    pr = O.Problem.from_scan(tiny_iqu())
    A, P, N = O.dense_system(pr)
    assert np.max(np.abs(A - A.T)) <= 1e-13 * np.max(np.abs(A))
    np.linalg.cholesky(A)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(A.shape[0])
    assert np.max(np.abs(pr.apply_A(x) - A @ x)) <= 1e-12 * np.max(np.abs(A @ x))
    d = rng.standard_normal(pr.n_t)
    assert np.max(np.abs(pr.rhs(d) - P.T @ (N @ d))) <= 1e-12 * np.max(np.abs(P.T @ N @ d))


# --------------------------------------------------------- P5: white noise

def test_white_noise_block_jacobi_is_exact_inverse():
    sc = tiny_iqu(fknee=(0.0, 0.0))
    sc.fknee[:] = 0.0
    pr = O.Problem.from_scan(sc)
    A, _, _ = O.dense_system(pr)
    B = pr.bj_blocks()
    Ablk = np.zeros_like(A)
    for p in range(pr.n_obs):
        Ablk[3 * p:3 * p + 3, 3 * p:3 * p + 3] = B[p]
    assert np.max(np.abs(A - Ablk)) <= 1e-13 * np.max(np.abs(A))
    # explicit form: sum W W^T / sigma^2
    Wsum = np.zeros((pr.n_obs, 3, 3))
    np.add.at(Wsum, pr.cid, pr.W[:, :, None] * pr.W[:, None, :])
    assert np.allclose(B, Wsum / sc.sigma[0] ** 2, rtol=1e-13, atol=1e-13)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(pr.n_obs * 3)
    x, it, st = O.pcg(pr.apply_A, b, lambda r: pr.bj_apply(r, B), tol=1e-12, maxit=10)
    assert st == 0 and it == 1
    assert np.allclose(x, pr.bj_apply(b, B), rtol=1e-12, atol=1e-12)


# ------------------------------------------------ P6, P10: solves, noiseless

def test_noiseless_data_returns_input_map():
    sc = tiny_iqu()
    pr = O.Problem.from_scan(sc)
    m = pr.sky_to_compact(sc.sky)
    d = pr.signal(sc.sky)
    b = pr.rhs(d)
    x, it, st = O.pcg(pr.apply_A, b, pr.bj_apply, tol=1e-13, maxit=500)
    assert st == 0
    assert np.linalg.norm(x - m) / np.linalg.norm(m) < 1e-10


def test_pcg_matches_dense_cholesky_solve():
    sc = tiny_iqu()
    pr = O.Problem.from_scan(sc)
    A, P, N = O.dense_system(pr)
    d = pr.signal(sc.sky) + sc.noise
    b = pr.rhs(d)
    L = np.linalg.cholesky(A)
    xd = np.linalg.solve(L.T, np.linalg.solve(L, b))
    x, it, st = O.pcg(pr.apply_A, b, pr.bj_apply, tol=1e-14, maxit=1000)
    assert st == 0
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= 1e-12
    # GLS estimator written out (eq. glsSol)
    xg = np.linalg.solve(P.T @ N @ P, P.T @ N @ d)
    assert np.linalg.norm(xg - xd) / np.linalg.norm(xd) <= 1e-12


def test_pcg_reports_breakdown_and_maxit():
    pr = O.Problem.from_scan(tiny_i())
    b = np.random.default_rng(4).standard_normal(pr.n_obs)
    _, it, st = O.pcg(pr.apply_A, b, lambda r: r, tol=1e-14, maxit=2)
    assert st == 1 and it == 2
    _, it, st = O.pcg(lambda v: -pr.apply_A(v), b, lambda r: r, tol=1e-14, maxit=5)
    assert st == 2


# ------------------------------------------------------ P7, P8: coarse space

def test_zs_structure():
    sc = tiny_iqu(interval_len=256)
    pr = O.Problem.from_scan(sc)
    Z = O.coarse_zs(pr)
    assert Z.shape == (pr.n_obs * 3, 16)
    assert np.allclose(Z[0::3].sum(axis=1), 1.0, rtol=0, atol=1e-15)
    assert np.all(Z[1::3] == 0) and np.all(Z[2::3] == 0)
    sc1 = tiny_i()
    sc1.offsets = np.array([0, sc1.n_samples])
    sc1.sigma, sc1.fknee, sc1.alpha = sc1.sigma[:1], sc1.fknee[:1], sc1.alpha[:1]
    Z1 = O.coarse_zs(O.Problem.from_scan(sc1))
    assert np.array_equal(Z1, np.ones((64, 1)))


def test_two_level_properties():
    sc = tiny_iqu(interval_len=256)
    pr = O.Problem.from_scan(sc)
    Z = O.coarse_zs(pr)
    C = O.Coarse(pr, Z)
    # co-pointed detectors see identical hit patterns: rank deficient Z
    assert C.rank < Z.shape[1]
    MAZ = np.stack([C.apply(C.AZ[:, j]) for j in range(Z.shape[1])], axis=1)
    assert np.max(np.abs(MAZ - Z)) <= 1e-10
    RAZ = np.stack([C.deflation(C.AZ[:, j]) for j in range(Z.shape[1])], axis=1)
    assert np.max(np.abs(RAZ)) <= 1e-10 * np.max(np.abs(C.AZ))
    rng = np.random.default_rng(5)
    X = rng.standard_normal((pr.n_obs * 3, 3))
    Y = X - Z @ (C.Epinv @ (C.AZ.T @ X))     # Y^T A Z = 0
    assert np.max(np.abs(Y.T @ C.AZ)) <= 1e-10 * np.max(np.abs(X.T @ C.AZ))
    AY = np.stack([pr.apply_A(Y[:, i]) for i in range(3)], axis=1)
    lhs = np.stack([C.apply(AY[:, i]) for i in range(3)], axis=1)
    rhs = np.stack([pr.bj_apply(AY[:, i], C.B) for i in range(3)], axis=1)
    assert np.max(np.abs(lhs - rhs)) <= 1e-9 * np.max(np.abs(rhs))


def test_solution_independent_of_preconditioner():
    sc = tiny_iqu(interval_len=256)
    pr = O.Problem.from_scan(sc)
    b = pr.rhs(pr.signal(sc.sky) + sc.noise)
    C = O.Coarse(pr, O.coarse_zs(pr))
    x1, _, s1 = O.pcg(pr.apply_A, b, pr.bj_apply, tol=1e-13, maxit=1000)
    x2, _, s2 = O.pcg(pr.apply_A, b, C.apply, tol=1e-13, maxit=1000)
    assert s1 == 0 and s2 == 0
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-10


def test_adef2_spectrum_and_start():
    """App. B: M_alt A and M_2lvl A share their spectrum (the theorem the paper cites for
    the two deflation variants); from its special initial guess the A-DEF2 PCG reaches
    the dense solution, starting with Z^T r_0 = 0, in about as many iterations as
    A-DEF1."""
    sc = tiny_iqu(interval_len=256)
    pr = O.Problem.from_scan(sc)
    A, _, _ = O.dense_system(pr)
    C = O.Coarse(pr, O.coarse_zs(pr))
    n = A.shape[0]
    eye = np.eye(n)
    M1 = np.stack([C.apply(eye[:, j]) for j in range(n)], axis=1)
    M2 = np.stack([C.apply_adef2(eye[:, j]) for j in range(n)], axis=1)
    assert np.max(np.abs(M1 - M2)) > 1e-2 * np.max(np.abs(M1))  # different operators
    ev1 = np.linalg.eigvals(M1 @ A)
    ev2 = np.linalg.eigvals(M2 @ A)
    assert np.max(np.abs(ev1.imag)) <= 1e-8 and np.max(np.abs(ev2.imag)) <= 1e-8
    e1, e2 = np.sort(ev1.real), np.sort(ev2.real)
    assert np.max(np.abs(e1 - e2)) <= 1e-8 * e1.max()
    # the deflated directions sit at 1: rank(Z) eigenvalues equal to 1
    assert np.sum(np.abs(e1 - 1.0) <= 1e-8) >= C.rank
    b = pr.rhs(pr.signal(sc.sky) + sc.noise)
    x0 = C.adef2_start(b)
    r0 = b - pr.apply_A(x0)
    assert np.max(np.abs(C.Z.T @ r0)) <= 1e-10 * np.max(np.abs(C.Z.T @ b))
    xd = np.linalg.solve(A, b)
    x2, it2, s2 = O.pcg(pr.apply_A, b, C.apply_adef2, tol=1e-12, maxit=1000, x0=x0)
    _, it1, s1 = O.pcg(pr.apply_A, b, C.apply, tol=1e-12, maxit=1000)
    assert s1 == 0 and s2 == 0
    assert np.linalg.norm(x2 - xd) / np.linalg.norm(xd) <= 1e-10
    assert abs(it2 - it1) <= 2, (it1, it2)


# ------------------------------------------------------- P11: near-null mode

def test_ones_in_near_null_space_with_1f_noise():
    ratios = []
    # band wide enough that f_defl = 1/(pi lambda t_samp) ~ 0.25 Hz < f_knee (App. D)
    for fk in (0.0, 5.0):
        sc = tiny_i(fknee=fk, lam=255)
        sc.fknee[:] = fk
        pr = O.Problem.from_scan(sc)
        A, _, _ = O.dense_system(pr)
        one = np.ones(pr.n_obs)
        ratios.append(np.linalg.norm(A @ one) / (np.linalg.norm(A, 2) * np.linalg.norm(one)))
    assert ratios[0] > 0.99          # white noise: 1_p is an eigenvector of the top eigenvalue
    assert ratios[1] < 0.1 * ratios[0]


# ------------------------------------------------ P12: CG bound (sanity only)

def test_cg_error_bound_holds():
    sc = tiny_i()
    pr = O.Problem.from_scan(sc)
    A, _, _ = O.dense_system(pr)
    b = pr.rhs(pr.signal(sc.sky) + sc.noise)
    x = np.linalg.solve(A, b)
    ev = np.linalg.eigvalsh(A)
    kappa = ev[-1] / ev[0]
    rho = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    e0 = np.sqrt(x @ A @ x)
    for j in (1, 3, 6, 10):
        xj, _, _ = O.pcg(pr.apply_A, b, lambda r: r, tol=0.0, maxit=j)
        ej = np.sqrt((x - xj) @ A @ (x - xj))
        assert ej <= 2 * e0 * rho ** j * (1 + 1e-9)


# ----------------------------------------------------- adjoint ingredients

def test_tap_derivatives_match_finite_differences():
    n, lam = 2048, 128
    p = np.array([1.2, 0.8, 1.4])
    D = O.tap_derivatives(n, *p, lam, 200.0)
    for i in range(3):
        h = 1e-6 * p[i]
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (O.toeplitz_taps(n, *pp, lam, 200.0) - O.toeplitz_taps(n, *pm, lam, 200.0)) / (2 * h)
        assert np.max(np.abs(fd - D[i])) <= 1e-6 * np.max(np.abs(D[i]))


def test_lag_correlations_reproduce_bilinear_form():
    rng = np.random.default_rng(6)
    u, v = rng.standard_normal(300), rng.standard_normal(300)
    t = O.toeplitz_taps(300, 1.0, 1.0, 1.0, 40, 200.0)
    c = O.lag_correlations(u, v, 40)
    assert t @ c == pytest.approx(u @ (O.toeplitz_dense(t, 300) @ v), rel=1e-12)


def _tiny_adjoint_problem(seed=7):
    import synth
    sc = synth.raster_iqu(side=8, spp=8, n_det=2, interval_len=256, lam=32,
                          fknee_range=(0.5, 2.0), alpha_range=(1.0, 2.0), seed_key=seed)
    return sc, O.Problem.from_scan(sc)


def test_dense_map_gradients_match_finite_differences():
    """The adjoint formulas against central differences of the dense GLS solve, for the
    linear functional L = g^T m_hat (so dL/dm_hat = g)."""
    sc, pr = _tiny_adjoint_problem()
    rng = np.random.default_rng(11)
    d = sc.noise + pr.signal(sc.sky)
    g = rng.standard_normal(pr.n_obs * pr.n_s)
    m, gd, gt, mu = O.map_gradients_dense(pr, d, g)
    assert np.allclose(m, O.map_dense(pr, d), rtol=0, atol=1e-10 * np.abs(m).max())
    # TOD gradient: L is linear in d, a central difference along a random direction is exact
    e = rng.standard_normal(d.shape[0])
    h = 1e-3
    fd = (g @ O.map_dense(pr, d + h * e) - g @ O.map_dense(pr, d - h * e)) / (2 * h)
    assert fd == pytest.approx(gd @ e, rel=1e-8)
    # noise-parameter gradient of a few (interval, parameter) pairs
    for j, i in [(0, 0), (1, 1), (2, 2), (3, 1)]:
        vals = []
        for s in (+1, -1):
            par = [pr.sigma.copy(), pr.fknee.copy(), pr.alpha.copy()]
            h = 1e-6 * par[i][j]
            par[i][j] += s * h
            pp = O.Problem(sc.pix, sc.weights, 3, sc.offsets, par[0], par[1], par[2], sc.lam,
                           sc.f_samp)
            vals.append(g @ O.map_dense(pp, d))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert fd == pytest.approx(gt[j, i], rel=1e-5, abs=1e-9 * np.abs(gt).max()), (j, i)


def test_banded_map_gradients_equal_dense_ones():
    sc, pr = _tiny_adjoint_problem(seed=8)
    d = sc.noise + pr.signal(sc.sky)
    g = np.random.default_rng(12).standard_normal(pr.n_obs * pr.n_s)
    ref = O.map_gradients_dense(pr, d, g)
    got = O.map_gradients(pr, d, g)
    for a, b in zip(got, ref):
        assert np.max(np.abs(a - b)) <= 1e-9 * np.max(np.abs(b))


# ----------------------------------------------------- a posteriori coarse space

def _small_iqu_problem(seed=9):
    """8x8 IQU, 2 detectors, one 1024-sample interval per detector, strong 1/f noise
    (f_knee 5-10 Hz, alpha 2): M_BD A has 11 eigenvalues below 0.2."""
    import synth
    sc = synth.raster_iqu(side=8, spp=8, n_det=2, interval_len=1024, lam=32,
                          fknee_range=(5.0, 10.0), alpha_range=(2.0, 2.0), seed_key=seed)
    return sc, O.Problem.from_scan(sc)


def test_lanczos_matrix_is_m_a_in_the_krylov_basis():
    """T_m = W^T M^-1 (M A) W = W^T A W for W the normalised preconditioned residuals
    with alternating signs: the CG coefficients reproduce the projected operator."""
    sc, pr = _small_iqu_problem()
    B = pr.bj_blocks()
    b = pr.rhs(sc.noise)
    _, al, rz, Zk = O.pcg_lanczos(pr.apply_A, b, lambda r: pr.bj_apply(r, B), tol=1e-6)
    m = al.shape[0]
    W = Zk[:, :m] * ((-1.0) ** np.arange(m) / np.sqrt(rz[:m]))
    AW = np.stack([pr.apply_A(W[:, k]) for k in range(m)], axis=1)
    T = O.lanczos_tridiagonal(al, rz)
    assert np.max(np.abs(W.T @ AW - T)) <= 1e-8 * np.max(np.abs(T))


def test_ritz_values_converge_to_eigenvalues_of_preconditioned_operator():
    sc, pr = _small_iqu_problem()
    B = pr.bj_blocks()
    b = pr.rhs(sc.noise)
    _, al, rz, Zk = O.pcg_lanczos(pr.apply_A, b, lambda r: pr.bj_apply(r, B), tol=1e-13,
                                  maxit=2000)
    theta, Y, est = O.ritz_pairs(al, rz, Zk)
    A, P, N = O.dense_system(pr)
    n = A.shape[0]
    Mb = np.zeros((n, n))
    for p in range(pr.n_obs):
        Mb[3 * p:3 * p + 3, 3 * p:3 * p + 3] = np.linalg.inv(B[p])
    ev = np.sort(np.linalg.eigvals(Mb @ A).real)
    # the smallest (isolated) Ritz value is a converged eigenvalue of M_BD A; all Ritz
    # values lie inside the spectrum
    assert theta[0] == pytest.approx(ev[0], rel=1e-8)
    assert ev[0] * (1 - 1e-10) <= theta.min() and theta.max() <= ev[-1] * (1 + 1e-10)
    # eq. approxEigen: ||M A y - theta y|| (M^-1 norm) equals the last-term estimate
    i = 0
    res = Mb @ (A @ Y[:, i]) - theta[i] * Y[:, i]
    Minv = np.linalg.inv(Mb)
    assert np.sqrt(res @ Minv @ res) == pytest.approx(est[i], rel=1e-4, abs=1e-10)


def test_deflation_space_two_level_properties():
    sc, pr = _small_iqu_problem()
    b = pr.rhs(sc.noise)
    Zd, theta = O.deflation_space(pr, b, eps_tol=0.2, tol=1e-10, maxit=2000)
    assert Zd.shape[1] >= 1 and np.all(theta[:Zd.shape[1]] < 0.2)
    co = O.Coarse(pr, Zd)
    AZ = np.stack([pr.apply_A(Zd[:, j]) for j in range(Zd.shape[1])], axis=1)
    MAZ = np.stack([co.apply(AZ[:, j]) for j in range(Zd.shape[1])], axis=1)
    assert np.max(np.abs(MAZ - Zd)) <= 1e-8 * np.max(np.abs(Zd))
    # the a posteriori preconditioner needs fewer iterations than block Jacobi on a new RHS
    b2 = pr.rhs(np.roll(sc.noise, 777))
    _, it_bj, _ = O.pcg(pr.apply_A, b2, pr.bj_apply, tol=1e-8, maxit=2000)
    x2, it_d, st = O.pcg(pr.apply_A, b2, co.apply, tol=1e-8, maxit=2000)
    assert st == 0 and it_d < it_bj


# ------------------------------------------- bandwidth and apodisation (App. D)

def _apodised_over_true(taps, f, fs, sigma, fknee, alpha):
    k = np.arange(1, taps.shape[0])
    s = taps[0] + 2.0 * np.sum(taps[1:] * np.cos(2.0 * np.pi * f / fs * k))
    return s / (1.0 / (sigma ** 2 * (1.0 + (fknee / f) ** alpha)))


def test_apodised_inverse_spectrum_deflects_below_f_defl():
    """App. D / Fig. corrPlot: with the Gaussian window the band-limited inverse spectrum
    follows 1/P(f) above a few f_defl = 1/(pi lambda t_samp) and is flattened (lifted far
    above it) below f_defl; a narrower window (exp(-2 (k/lambda)^2)) deflects higher."""
    fs, n = 200.0, 2 ** 16
    for lam in (100, 500, 2000):
        fd = fs / (np.pi * lam)
        taps = O.toeplitz_taps(n, 1.0, 1.0, 2.0, lam, fs)
        for m in (4, 8, 16):
            assert abs(_apodised_over_true(taps, m * fd, fs, 1.0, 1.0, 2.0) - 1.0) <= 0.05
        assert _apodised_over_true(taps, fd / 4, fs, 1.0, 1.0, 2.0) >= 5.0
        assert _apodised_over_true(taps, fd / 8, fs, 1.0, 1.0, 2.0) >= 20.0
        taps2 = O.toeplitz_taps(n, 1.0, 1.0, 2.0, lam, fs, window="gauss2")
        assert (_apodised_over_true(taps2, fd, fs, 1.0, 1.0, 2.0)
                > _apodised_over_true(taps, fd, fs, 1.0, 1.0, 2.0))


def test_bandwidth_below_knee_scale_is_nearly_uniform_weighting():
    """App. D: lambda = 1/(pi t_samp f_knee) is the largest bandwidth that is still about
    as good as uniform (white-noise) weighting: the apodised inverse spectrum varies by
    less than a factor 4 over all frequencies, while 16 times that bandwidth resolves the
    1/f fall-off (a factor above 25)."""
    fs, n = 200.0, 2 ** 16
    for fk, al in ((1.0, 2.0), (5.0, 2.0), (1.0, 1.0), (0.5, 1.5)):
        lam0 = fs / (np.pi * fk)
        narrow = O.taps_symbol(O.toeplitz_taps(n, 1.0, fk, al, int(round(lam0)), fs), 4096)
        wide = O.taps_symbol(O.toeplitz_taps(n, 1.0, fk, al, int(round(16 * lam0)), fs), 4096)
        assert narrow.max() / narrow.min() <= 4.0, (fk, al)
        assert wide.max() / wide.min() >= 25.0, (fk, al)


def test_zero_bandwidth_is_white_noise_weighting():
    """lambda = 0 keeps only t_0 = the mean of the inverse PSD on the interval's grid (the
    window is 1 at lag 0): N^-1 is diagonal, M_BD = A^-1 (one PCG step), and the map is the
    per-pixel noise-weighted least-squares co-addition written out directly."""
    sc = tiny_iqu(fknee=(1.0, 3.0), lam=0)
    pr = O.Problem.from_scan(sc)
    for j, t in enumerate(pr.taps):
        n = int(sc.offsets[j + 1] - sc.offsets[j])
        q = O.inverse_psd(n, sc.sigma[j], sc.fknee[j], sc.alpha[j], sc.f_samp)
        full = np.concatenate([q, q[1:(n + 1) // 2][::-1]])  # the n-point spectrum
        assert t.shape == (1,) and t[0] == pytest.approx(full.mean(), rel=1e-12)
    d = pr.signal(sc.sky) + sc.noise
    b = pr.rhs(d)
    x, it, st = O.pcg(pr.apply_A, b, pr.bj_apply, tol=1e-12, maxit=10)
    assert st == 0 and it == 1
    w_t = np.concatenate([np.full(int(sc.offsets[j + 1] - sc.offsets[j]), pr.taps[j][0])
                          for j in range(len(pr.taps))])
    ref = np.empty((pr.n_obs, 3))
    for p in range(pr.n_obs):
        s = pr.cid == p
        Wp = pr.W[s]
        ref[p] = np.linalg.solve(Wp.T @ (w_t[s, None] * Wp), Wp.T @ (w_t[s] * d[s]))
    assert np.linalg.norm(x - ref.ravel()) / np.linalg.norm(ref) <= 1e-11


# ------------------------------------------- block conditioning and the symbol bound

def test_bj_rcond_closed_forms():
    """rcond_1(B) = 1 / (||B||_1 ||B^-1||_1) on blocks whose inverse is known in closed
    form: diagonal blocks (min/max of the diagonal), and [[a, b, 0], [b, a, 0], [0, 0, a]]
    with a > b > 0, whose inverse has the 2x2 part [[a, -b], [-b, a]] / (a^2 - b^2), so
    ||B||_1 = a + b, ||B^-1||_1 = 1 / (a - b) and rcond = (a - b) / (a + b)."""
    pr = O.Problem.from_scan(tiny_iqu())
    B = np.zeros((4, 3, 3))
    B[0] = np.diag([4.0, 2.0, 1.0])
    B[1] = np.diag([3.0, 3.0, 3.0])
    a, b = 5.0, 3.0
    B[2] = [[a, b, 0], [b, a, 0], [0, 0, a]]
    a2, b2 = 1.0, 1.0 - 1e-6
    B[3] = [[a2, b2, 0], [b2, a2, 0], [0, 0, a2]]
    rc = pr.bj_rcond(B)
    assert rc[0] == pytest.approx(0.25, rel=1e-15)
    assert rc[1] == pytest.approx(1.0, rel=1e-15)
    assert rc[2] == pytest.approx((a - b) / (a + b), rel=1e-14)
    assert rc[3] == pytest.approx((a2 - b2) / (a2 + b2), rel=1e-8)


def test_bj_rcond_of_a_pixel_seen_at_four_angles():
    """A pixel seen once at each of the polariser angles 0, 45, 90, 135 deg (2 phi = 0, 90,
    180, 270 deg) in an interval with diagonal tap t_0: B_p = t_0 sum_t W_t W_t^T =
    t_0 diag(4, 2, 2) (eq. stdPrec), so rcond = 1/2 whatever t_0 is."""
    phi = np.deg2rad([0.0, 45.0, 90.0, 135.0])
    w = np.stack([np.cos(2 * phi), np.sin(2 * phi)], axis=1)
    pr = O.Problem(np.zeros(4, dtype=np.int32), w, 3, np.array([0, 4]), [1.3], [0.0], [1.0],
                   2, 200.0)
    B = pr.bj_blocks()
    t0 = pr.taps[0][0]
    assert t0 == pytest.approx(1.0 / 1.3 ** 2, rel=1e-14)
    assert np.max(np.abs(B[0] - t0 * np.diag([4.0, 2.0, 2.0]))) <= 1e-15 * t0
    assert pr.bj_rcond()[0] == pytest.approx(0.5, rel=1e-14)


@pytest.mark.parametrize("window,fk,al", [("gauss", 2.0, 2.0), ("rect", 1.0, 1.0),
                                          ("gauss2", 5.0, 1.5)])
def test_symbol_bounds_the_spectrum_of_toeplitz_sections(window, fk, al):
    """taps_symbol against the eigenvalues of an explicit n x n section of the band
    Toeplitz matrix (not a restatement of its formula): every eigenvalue lies in
    [min S, max S] and, as n grows, the extreme eigenvalues approach min S and max S
    (Szego); with n = 4096 >> lambda = 32 they are within 1e-3 of the range.  A symbol
    with t_0 + sum t_k cos(k theta) (a lost factor 2) fails both bounds; the pointwise
    values are pinned on the FFT grid by the next test."""
    lam, n = 32, 4096
    t = O.toeplitz_taps(2 ** 14, 1.0, fk, al, lam, 200.0, window)
    s = O.taps_symbol(t, 1 << 16)
    ev = np.linalg.eigvalsh(O.toeplitz_dense(t, n))
    span = s.max() - s.min()
    assert ev.min() >= s.min() - 1e-12 * span
    assert ev.max() <= s.max() + 1e-12 * span
    assert ev.min() - s.min() <= 1e-3 * span
    assert s.max() - ev.max() <= 1e-3 * span


def test_symbol_on_the_fft_grid_is_the_dft_of_the_even_row():
    """On the grid theta_m = 2 pi m / n_r (n_theta = n_r / 2 + 1), taps_symbol equals the
    real DFT of the even sequence h_0 = t_0, h_k = h_{n_r - k} = t_k: the spectrum an
    overlap-save convolution of length n_r multiplies by."""
    t = O.toeplitz_taps(3000, 1.0, 1.5, 1.2, 100, 200.0)
    nr = 1024
    h = np.zeros(nr)
    h[:t.shape[0]] = t
    h[nr - t.shape[0] + 1:] = t[1:][::-1]
    H = np.fft.rfft(h).real
    s = O.taps_symbol(t, nr // 2 + 1)
    assert np.max(np.abs(s - H)) <= 1e-13 * np.max(np.abs(H))
