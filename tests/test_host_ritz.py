"""Host logic of the Z_D construction (no device work): the Ritz pairs that the library
extracts from the PCG step lengths and residual products, against LAPACK's symmetric
eigensolver on the same Lanczos matrix, including a matrix with pairs of eigenvalues
that agree to about 1e-14 (Wilkinson's W21+, shifted to be positive definite), where only
the two-dimensional invariant subspaces are determined."""

import numpy as np
import pytest

import oracle as O
import synth

lib = pytest.importorskip("paper_1408_3048_amd")


def _alpha_rz_from_T(d, e):
    """Step lengths and r^T z products of the PCG run whose Lanczos matrix is the SPD
    tridiagonal (d, e) (e > 0): the LDL^T recurrence of T."""
    m = d.shape[0]
    al = np.empty(m)
    rz = np.empty(m)
    al[0] = 1.0 / d[0]
    rz[0] = 1.0
    for k in range(1, m):
        beta = (e[k - 1] * al[k - 1]) ** 2
        rz[k] = rz[k - 1] * beta
        al[k] = 1.0 / (d[k] - beta / al[k - 1])
    return al, rz


def _tri(d, e):
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


def _check_pairs(T, theta, S, tol_sub=1e-9):
    ev, V = np.linalg.eigh(T)
    r = theta.shape[0]
    scale = np.max(np.abs(ev))
    assert np.max(np.abs(theta - ev[:r])) <= 1e-13 * scale
    assert np.max(np.abs(S.T @ S - np.eye(r))) <= 1e-12
    assert np.max(np.linalg.norm(T @ S - S * theta, axis=0)) <= 1e-12 * scale
    # invariant subspaces of groups of eigenvalues closer than 1e-8 coincide
    i = 0
    while i < r:
        j = i + 1
        while j < r and ev[j] - ev[j - 1] < 1e-8 * scale:
            j += 1
        complete = j == ev.shape[0] or ev[j] - ev[j - 1] >= 1e-8 * scale
        if complete:  # a group cut by the selection is not determined by its members
            Pa = S[:, i:j] @ S[:, i:j].T
            Pb = V[:, i:j] @ V[:, i:j].T
            assert np.max(np.abs(Pa - Pb)) <= tol_sub, (i, j)
        i = j


def test_ritz_pairs_of_pcg_run_match_lapack():
    sc = synth.raster_iqu(side=8, spp=8, n_det=2, interval_len=1024, lam=32,
                          fknee_range=(5.0, 10.0), alpha_range=(2.0, 2.0), seed_key=9)
    pr = O.Problem.from_scan(sc)
    b = pr.rhs(sc.noise)
    Bk = pr.bj_blocks()
    for tol in (1e-8, 1e-14):
        _, al, rz, Zk = O.pcg_lanczos(pr.apply_A, b, lambda r: pr.bj_apply(r, Bk), tol, 3000)
        m = al.shape[0]
        T = O.lanczos_tridiagonal(al, rz)
        theta, S = lib.lanczos_ritz(al, rz[:m], eps_tol=0.2)
        th_o, _, _ = O.ritz_pairs(al, rz, Zk)
        assert theta.shape[0] == np.sum(th_o < 0.2) >= 5
        _check_pairs(T, theta, S)
        # largest-magnitude entry of every vector is positive
        assert np.all(S[np.argmax(np.abs(S), axis=0), np.arange(S.shape[1])] > 0)


def test_wilkinson_close_pairs():
    m = 21
    d = np.abs(np.arange(m) - 10.0) + 2.0  # W21+ shifted by 2: SPD, close pairs near the top
    e = np.ones(m - 1)
    al, rz = _alpha_rz_from_T(d, e)
    T = _tri(d, e)
    assert np.allclose(O.lanczos_tridiagonal(al, np.append(rz, 1.0)), T, rtol=1e-12, atol=0)
    theta, S = lib.lanczos_ritz(al, rz, eps_tol=100.0)
    assert theta.shape[0] == m
    ev = np.linalg.eigvalsh(T)
    assert ev[-1] - ev[-2] < 1e-12 * ev[-1]  # the pair the test is about
    _check_pairs(T, theta, S)


def test_selection_threshold_and_cap():
    rng = np.random.default_rng(3)
    m = 60
    d = rng.uniform(0.5, 3.0, m)
    e = rng.uniform(0.05, 0.5, m - 1)
    al, rz = _alpha_rz_from_T(d, e)
    T = _tri(d, e)
    ev = np.linalg.eigvalsh(T)
    assert ev[0] > 0
    eps = float(ev[6] + ev[7]) / 2  # exactly 7 eigenvalues below
    theta, S = lib.lanczos_ritz(al, rz, eps_tol=eps)
    assert theta.shape[0] == 7
    _check_pairs(T, theta, S)
    theta3, S3 = lib.lanczos_ritz(al, rz, eps_tol=eps, max_cols=3)
    assert np.array_equal(theta3, theta[:3])
    t0, S0 = lib.lanczos_ritz(al, rz, eps_tol=ev[0] * 0.5)
    assert t0.shape[0] == 0 and S0.shape == (m, 0)
    t1, S1 = lib.lanczos_ritz(al[:1], rz[:1], eps_tol=1e9)  # one step: T = [1/alpha_0]
    assert t1 == pytest.approx([1.0 / al[0]], rel=1e-15) and S1[0, 0] == 1.0


def test_invalid_lanczos_data_is_rejected():
    with pytest.raises(lib.MMError) as e:
        lib.lanczos_ritz(np.array([1.0, -2.0]), np.array([1.0, 0.5]), eps_tol=1.0)
    assert e.value.status == lib.MM_ERR_BREAKDOWN
    with pytest.raises(lib.MMError) as e:
        lib.lanczos_ritz(np.array([1.0]), np.array([1.0]), eps_tol=0.0)
    assert e.value.status == lib.MM_ERR_ARG
