"""Plain FP64 oracle for GLS map-making with preconditioned CG.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every routine is the
plain definition of what the method computes, written for readability, not
speed: Toeplitz blocks are applied by direct banded sums, the pointing matrix
by gathers and ``numpy.bincount``, preconditioners by their defining formulas.

Citations refer to the paper's sections and equations (LaTeX labels):
  Sect. 2 (problem definition)        eqs. dataModelGen, signal_with_polarization
  Sect. 2.1 (GLS problem)             eqs. glsSol, N_def, Sdef, linear_system, rhs, a_times_x
  Sect. 3.1 (preconditioning)         eqs. err_bound, stdPrec
  Sect. 3.2 (two-level)               eqs. projection, 2 (A-DEF1)
  App. B (alternative two-level)      eq. ADEF2 (A-DEF2) and its initial guess
  Sect. 3.3.1 (a priori coarse space) eqs. AsingVect, strofZ, strofZ_polar
  Sect. 4.1.4 (noise)                 eq. fknee; band half-width lambda_T
  App. C (implementation)             precomputed AZ and E; 4-step application
  App. D (correlation length)         eqs. glsSolFourier, apodDef

Readings where the paper is silent or garbled (each also listed with the
design notes):
  * PSD per sample: P(f) = sigma^2 (1 + (f_knee/f)^alpha); alpha = 2 and the
    sampling-interval factor of eq. fknee are the paper's special case.
  * Inverse-PSD zero-frequency bin: 0 when f_knee > 0 (limit of 1/P), 1/sigma^2
    for white noise.
  * Toeplitz row of interval j = inverse DFT, on the interval's own length
    n_j, of the inverse PSD sampled at f_m = m f_samp / n_j (App. D: a row is
    the Fourier transform of the inverse spectrum), truncated to lags
    |k| <= lambda and apodised by w(k) = exp(-(k/lambda)^2) (eq. apodDef has a
    garbled sign; this is the Gaussian whose transform falls by e at
    f_defl = 1/(pi lambda t_samp), as the caption of Fig. corrPlot states).
  * diag(N^-1) in eq. stdPrec is t_0 of the sample's interval.
  * Dependent columns of Z: E is replaced by its pseudo-inverse (eigenvalues
    below rank_tol * max dropped); M_2lvl depends only on span(Z).
  * PCG: x0 = 0, Fletcher-Reeves beta, stop when both the recursive and the
    true relative residual ||b - A x|| / ||b|| are <= tol (otherwise the
    recursive residual is replaced by the true one).

Pins (tests marked "not gpu"): taps vs. explicit cosine sums and the white
noise closed form; banded sums vs. explicit dense Toeplitz matrices; P/P^T
adjointness and integer hits; symmetry and positive definiteness of A; white
noise => M_BD = A^-1 and one-iteration convergence; noiseless data => the
input map; M_2lvl A Z = Z and R A Z = 0; M_alt A and M_2lvl A share their
spectrum; PCG vs. dense Cholesky on tiny problems; gradients vs. finite
differences of a dense solve; the CG Lanczos matrix equals W^T A W.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "compact", "hits", "interval_of_sample", "inverse_psd", "toeplitz_taps",
    "toeplitz_taps_cosine_sum", "taps_symbol", "toeplitz_apply", "toeplitz_apply_at",
    "toeplitz_dense", "Problem", "pcg", "dense_system", "coarse_zs", "Coarse",
    "tap_derivatives", "lag_correlations", "map_gradients_dense", "map_dense", "map_gradients",
    "pcg_lanczos", "lanczos_tridiagonal", "ritz_pairs", "deflation_space",
]


# --------------------------------------------------------------------------
# pointing, compaction, hit counts (Sect. 2)
# --------------------------------------------------------------------------

def compact(pix):
    """Observed pixels only (Sect. 2: the pointing matrix is restricted to
    observed pixels and has full column rank).  Returns (obs, cid): sorted
    unique original ids and the compact id of every sample."""
    pix = np.asarray(pix)
    obs = np.unique(pix)
    cid = np.searchsorted(obs, pix)
    return obs, cid


def hits(cid, n_obs):
    """s_p: number of samples falling in each compact pixel (Sect. 3.3.1)."""
    return np.bincount(cid, minlength=n_obs).astype(np.int64)


def interval_of_sample(offsets):
    """j(t): stationary interval of every sample (eq. N_def blocks)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    lens = np.diff(offsets)
    return np.repeat(np.arange(lens.shape[0]), lens)


# --------------------------------------------------------------------------
# noise weighting: band-limited Toeplitz blocks (eq. N_def, eq. fknee, App. D)
# --------------------------------------------------------------------------

def inverse_psd(n, sigma, fknee, alpha, f_samp):
    """q_m = 1 / P(f_m), f_m = m f_samp / n for m = 0..floor(n/2), with the
    per-sample PSD P(f) = sigma^2 (1 + (f_knee / f)^alpha) (eq. fknee);
    q_0 = 0 for f_knee > 0, 1/sigma^2 for white noise."""
    m = np.arange(n // 2 + 1, dtype=np.float64)
    f = m * (f_samp / n)
    q = np.empty_like(f)
    if fknee > 0.0:
        q[0] = 0.0
        q[1:] = 1.0 / (sigma ** 2 * (1.0 + (fknee / f[1:]) ** alpha))
    else:
        q[:] = 1.0 / sigma ** 2
    return q


def _window(k, lam, window):
    """Apodisation window at lags k, |k| <= lam (App. D, eq. apodDef); every window is 1
    at k = 0, so lam = 0 keeps the diagonal alone."""
    k = np.asarray(k, dtype=np.float64)
    if window not in ("gauss", "gauss2", "rect"):
        raise ValueError(window)
    if lam == 0 or window == "rect":
        return np.ones_like(k)
    if window == "gauss":
        return np.exp(-(k / lam) ** 2)
    return np.exp(-2.0 * (k / lam) ** 2)


def toeplitz_taps(n, sigma, fknee, alpha, lam, f_samp, window="gauss"):
    """First row t_0..t_K (K = min(lambda, n-1)) of the band-limited Toeplitz
    block of N^-1 for an interval of n samples: the inverse real DFT of the
    inverse PSD on the interval's own frequency grid (App. D, eq.
    glsSolFourier), apodised by the window (eq. apodDef) and set to zero beyond
    the half bandwidth lambda (Sect. 4.1.4)."""
    q = inverse_psd(n, sigma, fknee, alpha, f_samp)
    row = np.fft.irfft(q, n)
    kmax = min(lam, n - 1)
    k = np.arange(kmax + 1)
    return row[: kmax + 1] * _window(k, lam, window)


def toeplitz_taps_cosine_sum(n, sigma, fknee, alpha, lam, f_samp, window="gauss"):
    """Same taps written as the explicit cosine sum of the inverse DFT of a
    real even spectrum (slow; used to pin toeplitz_taps)."""
    q = inverse_psd(n, sigma, fknee, alpha, f_samp)
    kmax = min(lam, n - 1)
    out = np.empty(kmax + 1)
    half = n // 2
    for k in range(kmax + 1):
        s = q[0]
        for m in range(1, (n + 1) // 2):
            s += 2.0 * q[m] * np.cos(2.0 * np.pi * m * k / n)
        if n % 2 == 0:
            s += q[half] * (-1.0) ** k
        out[k] = s / n * _window(k, lam, window)
    return out


def taps_symbol(taps, n_theta=1 << 16):
    """Symbol S(theta) = t_0 + 2 sum_k t_k cos(k theta) on a uniform grid of
    [0, pi].  min S > 0 implies every finite section of the Toeplitz matrix is
    positive definite (its eigenvalues lie within [min S, max S])."""
    theta = np.linspace(0.0, np.pi, n_theta)
    s = np.full_like(theta, taps[0])
    for k in range(1, taps.shape[0]):
        s += 2.0 * taps[k] * np.cos(k * theta)
    return s


def toeplitz_apply(y, offsets, taps_list):
    """z = N^-1 y by direct banded sums per stationary interval (eq. N_def):
    z_t = t_0 y_t + sum_{k=1..K} t_k (y_{t-k} + y_{t+k}), with t-k and t+k
    restricted to the interval of t (no wrap-around)."""
    y = np.asarray(y, dtype=np.float64)
    z = np.zeros_like(y)
    for j in range(len(offsets) - 1):
        a, b = int(offsets[j]), int(offsets[j + 1])
        ys = y[a:b]
        zs = taps_list[j][0] * ys
        t = taps_list[j]
        n = b - a
        for k in range(1, min(t.shape[0], n)):
            zs[k:] += t[k] * ys[:-k]
            zs[:-k] += t[k] * ys[k:]
        z[a:b] = zs
    return z


def toeplitz_apply_at(y, offsets, taps_list, ts):
    """(N^-1 y)_t only at the sample indices ts (direct banded sums)."""
    y = np.asarray(y, dtype=np.float64)
    offsets = np.asarray(offsets, dtype=np.int64)
    ts = np.asarray(ts, dtype=np.int64)
    js = np.searchsorted(offsets, ts, side="right") - 1
    out = np.empty(ts.shape[0])
    for i, (t, j) in enumerate(zip(ts, js)):
        a, b = offsets[j], offsets[j + 1]
        tp = taps_list[j]
        K = tp.shape[0] - 1
        lo, hi = max(a, t - K), min(b, t + K + 1)
        lags = np.abs(np.arange(lo, hi) - t)
        out[i] = np.dot(tp[lags], y[lo:hi])
    return out


def toeplitz_dense(taps, n):
    """Explicit n x n symmetric banded Toeplitz matrix from its first row."""
    T = np.zeros((n, n))
    for k in range(min(taps.shape[0], n)):
        idx = np.arange(n - k)
        T[idx, idx + k] = taps[k]
        T[idx + k, idx] = taps[k]
    return T


# --------------------------------------------------------------------------
# the GLS problem: A = P^T N^-1 P, b = P^T N^-1 d (eqs. Sdef, rhs, a_times_x)
# --------------------------------------------------------------------------

class Problem:
    """One map-making problem in the compact observed-pixel space.

    Map vectors are flat [n_obs * n_s] with the Stokes parameters of a pixel
    adjacent (I, Q, U); time-domain vectors have one entry per sample."""

    def __init__(self, pix, weights, n_stokes, offsets, sigma, fknee, alpha, lam,
                 f_samp, window="gauss"):
        self.obs, self.cid = compact(pix)
        self.n_obs = int(self.obs.shape[0])
        self.n_s = int(n_stokes)
        self.n_t = int(np.asarray(pix).shape[0])
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.lam = int(lam)
        self.f_samp = float(f_samp)
        self.window = window
        self.sigma = np.asarray(sigma, dtype=np.float64)
        self.fknee = np.asarray(fknee, dtype=np.float64)
        self.alpha = np.asarray(alpha, dtype=np.float64)
        # rows of the pointing matrix (eq. signal_with_polarization)
        if self.n_s == 1:
            self.W = np.ones((self.n_t, 1))
        else:
            w = np.asarray(weights, dtype=np.float64)
            self.W = np.concatenate([np.ones((self.n_t, 1)), w], axis=1)
        self.taps = []
        for j in range(len(self.offsets) - 1):
            n = int(self.offsets[j + 1] - self.offsets[j])
            self.taps.append(toeplitz_taps(n, self.sigma[j], self.fknee[j], self.alpha[j],
                                           self.lam, self.f_samp, window))
        self.iv = interval_of_sample(self.offsets)
        self.s = hits(self.cid, self.n_obs)

    @classmethod
    def from_scan(cls, scan, window="gauss"):
        return cls(scan.pix, scan.weights, scan.n_stokes, scan.offsets, scan.sigma,
                   scan.fknee, scan.alpha, scan.lam, scan.f_samp, window)

    # --- P, N^-1, P^T (Sect. 2, eq. a_times_x)
    def depoint(self, x):
        """y = P x: y_t = sum_s W[t, s] x[c(t), s]."""
        X = np.asarray(x, dtype=np.float64).reshape(self.n_obs, self.n_s)
        return np.einsum("ts,ts->t", self.W, X[self.cid])

    def point(self, z):
        """x = P^T z: x[p, s] = sum_{t: c(t) = p} W[t, s] z_t."""
        z = np.asarray(z, dtype=np.float64)
        out = np.empty((self.n_obs, self.n_s))
        for s in range(self.n_s):
            out[:, s] = np.bincount(self.cid, weights=self.W[:, s] * z, minlength=self.n_obs)
        return out.reshape(-1)

    def ninv(self, y):
        return toeplitz_apply(y, self.offsets, self.taps)

    def apply_A(self, x):
        """A x = P^T [N^-1 [P x]] (eq. a_times_x)."""
        return self.point(self.ninv(self.depoint(x)))

    def rhs(self, d):
        """b = P^T N^-1 d (eq. rhs)."""
        return self.point(self.ninv(d))

    def sky_to_compact(self, sky):
        """Restrict a full-grid map [n_pix, n_s] to the observed pixels."""
        return np.asarray(sky, dtype=np.float64)[self.obs].reshape(-1)

    def signal(self, sky):
        """Noiseless TOD of a full-grid sky (eq. dataModelGen with n = 0)."""
        return self.depoint(self.sky_to_compact(sky))

    # --- sampled outputs for large problems
    def apply_A_at(self, x, pixels):
        """(A x) restricted to some compact pixels: P x everywhere, N^-1 only at
        the samples of those pixels, then their P^T rows."""
        y = self.depoint(x)
        out = np.empty((len(pixels), self.n_s))
        for i, p in enumerate(pixels):
            ts = np.nonzero(self.cid == p)[0]
            z = toeplitz_apply_at(y, self.offsets, self.taps, ts)
            out[i] = self.W[ts].T @ z
        return out

    # --- block-Jacobi preconditioner (eq. stdPrec)
    def bj_blocks(self):
        """B_p = sum_{t in p} t_0^{(j(t))} W_t W_t^T (P^T diag(N^-1) P)."""
        t0 = np.array([tp[0] for tp in self.taps])[self.iv]
        B = np.zeros((self.n_obs, self.n_s, self.n_s))
        for a in range(self.n_s):
            for c in range(self.n_s):
                B[:, a, c] = np.bincount(self.cid, weights=t0 * self.W[:, a] * self.W[:, c],
                                         minlength=self.n_obs)
        return B

    def bj_rcond(self, B=None):
        """Reciprocal 1-norm condition number of every block."""
        B = self.bj_blocks() if B is None else B
        inv = np.linalg.inv(B)
        n1 = np.abs(B).sum(axis=1).max(axis=1)
        ni = np.abs(inv).sum(axis=1).max(axis=1)
        return 1.0 / (n1 * ni)

    def bj_apply(self, r, B=None):
        """z = M_BD r, solving every n_s x n_s block."""
        B = self.bj_blocks() if B is None else B
        R = np.asarray(r, dtype=np.float64).reshape(self.n_obs, self.n_s, 1)
        return np.linalg.solve(B, R).reshape(-1)

    # --- explicit operators for tiny problems
    def dense_P(self):
        P = np.zeros((self.n_t, self.n_obs * self.n_s))
        for s in range(self.n_s):
            P[np.arange(self.n_t), self.cid * self.n_s + s] = self.W[:, s]
        return P

    def dense_Ninv(self):
        N = np.zeros((self.n_t, self.n_t))
        for j in range(len(self.offsets) - 1):
            a, b = int(self.offsets[j]), int(self.offsets[j + 1])
            N[a:b, a:b] = toeplitz_dense(self.taps[j], b - a)
        return N


def dense_system(prob: Problem):
    """A assembled from explicit P and explicit Toeplitz blocks (tiny problems)."""
    P = prob.dense_P()
    N = prob.dense_Ninv()
    return P.T @ N @ P, P, N


# --------------------------------------------------------------------------
# two-level preconditioner with the a priori coarse space (Sect. 3.2, 3.3.1)
# --------------------------------------------------------------------------

def coarse_zs(prob: Problem):
    """Z_S: column j holds, for every observed pixel, the fraction of its hits
    that fall in stationary interval j, s_p^j / s_p, on the I rows; the Q and U
    rows are zero (eqs. strofZ, strofZ_polar).  Dense [n_obs*n_s, n_int]."""
    n_int = len(prob.offsets) - 1
    spj = np.zeros((prob.n_obs, n_int))
    np.add.at(spj, (prob.cid, prob.iv), 1.0)
    Z = np.zeros((prob.n_obs * prob.n_s, n_int))
    Z[0::prob.n_s, :] = spj / prob.s[:, None]
    return Z


class Coarse:
    """Precomputed AZ, E = Z^T A Z and its pseudo-inverse (App. C), and the
    A-DEF1 two-level preconditioner M_2lvl = M_BD (I - A Z E^-1 Z^T) + Z E^-1 Z^T
    (eq. 2)."""

    def __init__(self, prob: Problem, Z, rank_tol=1e-10):
        self.prob = prob
        self.Z = Z
        self.AZ = np.stack([prob.apply_A(Z[:, j]) for j in range(Z.shape[1])], axis=1)
        self.E = Z.T @ self.AZ
        Es = 0.5 * (self.E + self.E.T)
        lam, V = np.linalg.eigh(Es)
        keep = lam > rank_tol * lam.max()
        self.rank = int(keep.sum())
        self.Epinv = (V[:, keep] / lam[keep]) @ V[:, keep].T
        self.B = prob.bj_blocks()

    def apply(self, r):
        v = self.Epinv @ (self.Z.T @ r)
        return self.prob.bj_apply(r - self.AZ @ v, self.B) + self.Z @ v

    def deflation(self, y):
        """R y = (I - A Z E^+ Z^T) y (eq. projection)."""
        return y - self.AZ @ (self.Epinv @ (self.Z.T @ y))

    def apply_adef2(self, r):
        """A-DEF2 (App. B, eq. ADEF2): M_alt r = R^T M_BD r + Z E^+ Z^T r, with
        R^T = I - Z E^+ (A Z)^T since A and E are symmetric."""
        y = self.prob.bj_apply(r, self.B)
        return y - self.Z @ (self.Epinv @ (self.AZ.T @ y)) + self.Z @ (self.Epinv @ (self.Z.T @ r))

    def adef2_start(self, b, x0=None):
        """The initial guess with which A-DEF2 PCG is equivalent to PCG with an SPD
        preconditioner (App. B): x0 + Z E^+ Z^T (b - A x0), i.e. Z E^+ Z^T b + R^T x0;
        its residual R (b - A x0) has Z^T r = 0."""
        x0 = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64)
        return x0 + self.Z @ (self.Epinv @ (self.Z.T @ (b - self.prob.apply_A(x0))))


# --------------------------------------------------------------------------
# preconditioned conjugate gradients (Sect. 3.1)
# --------------------------------------------------------------------------

def pcg(apply_A, b, precond, tol=1e-8, maxit=1000, x0=None, history=None):
    """Preconditioned CG from x0 (default 0).  Returns (x, iterations, status)
    with status 0 = converged, 1 = not converged in maxit, 2 = breakdown
    (p^T A p <= 0).  Convergence: recursive AND true ||b - A x|| / ||b|| <= tol;
    when only the recursive one passes, r is replaced by b - A x."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_A(x) if x0 is not None else b.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, 0
    if np.linalg.norm(r) / bn <= tol:
        return x, 0, 0
    z = precond(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        q = apply_A(p)
        pq = p @ q
        if not pq > 0.0:
            return x, it, 2
        a = rz / pq
        x += a * p
        r -= a * q
        rel = np.linalg.norm(r) / bn
        if history is not None:
            history.append(rel)
        if rel <= tol:
            rt = b - apply_A(x)
            if np.linalg.norm(rt) / bn <= tol:
                return x, it, 0
            r = rt
        z = precond(r)
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, maxit, 1


# --------------------------------------------------------------------------
# adjoint of the map with respect to the noise model
# --------------------------------------------------------------------------

def tap_derivatives(n, sigma, fknee, alpha, lam, f_samp, window="gauss"):
    """d t_k / d(sigma, f_knee, alpha) for k = 0..K: the windowed inverse DFT of
    the derivative of the inverse PSD q_m = 1/(sigma^2 (1 + (f_knee/f_m)^alpha))."""
    m = np.arange(n // 2 + 1, dtype=np.float64)
    f = m * (f_samp / n)
    q = inverse_psd(n, sigma, fknee, alpha, f_samp)
    dq = np.zeros((3, q.shape[0]))
    dq[0] = -2.0 * q / sigma
    if fknee > 0.0:
        ratio = (fknee / f[1:]) ** alpha
        dq[1, 1:] = -q[1:] * (alpha * ratio / fknee) / (1.0 + ratio)
        dq[2, 1:] = -q[1:] * ratio * np.log(fknee / f[1:]) / (1.0 + ratio)
    kmax = min(lam, n - 1)
    w = _window(np.arange(kmax + 1), lam, window)
    return np.stack([np.fft.irfft(dq[i], n)[: kmax + 1] * w for i in range(3)])


def lag_correlations(u, v, K):
    """c(0) = sum u_t v_t; c(k) = sum_t (u_t v_{t+k} + u_{t+k} v_t) for k = 1..K,
    so that u^T T v = sum_k t_k c(k) for a symmetric banded Toeplitz T."""
    n = u.shape[0]
    c = np.zeros(min(K, n - 1) + 1)
    c[0] = u @ v
    for k in range(1, c.shape[0]):
        c[k] = u[:-k] @ v[k:] + u[k:] @ v[:-k]
    return c


def map_gradients_dense(prob: Problem, d, g):
    """Gradients of a loss L(m_hat) of the GLS map m_hat = A^-1 P^T N^-1 d (eq. glsSol),
    given g = dL/dm_hat, from explicit dense matrices (tiny problems):

      mu = A^-1 g                      (A symmetric)
      dL/dd = N^-1 P mu                (m_hat is linear in d)
      dL/dtheta_j = (P mu)_j^T (dT_j/dtheta_j) (d - P m_hat)_j

    the last line from d m_hat = A^-1 P^T dN^-1 (d - P m_hat), dN^-1 being block j's
    Toeplitz derivative (taps from tap_derivatives) and theta_j = (sigma, f_knee, alpha).
    Returns (m_hat, dL/dd, dL/dtheta [n_int, 3], mu)."""
    A, P, N = dense_system(prob)
    d = np.asarray(d, dtype=np.float64)
    L = np.linalg.cholesky(A)

    def solve(rhs):
        return np.linalg.solve(L.T, np.linalg.solve(L, rhs))

    m = solve(P.T @ (N @ d))
    mu = solve(np.asarray(g, dtype=np.float64))
    u = P @ mu
    v = d - P @ m
    grad_d = N @ u
    n_int = len(prob.offsets) - 1
    grad_t = np.zeros((n_int, 3))
    for j in range(n_int):
        a, b = int(prob.offsets[j]), int(prob.offsets[j + 1])
        D = tap_derivatives(b - a, prob.sigma[j], prob.fknee[j], prob.alpha[j], prob.lam,
                            prob.f_samp, prob.window)
        for i in range(3):
            grad_t[j, i] = u[a:b] @ (toeplitz_dense(D[i], b - a) @ v[a:b])
    return m, grad_d, grad_t, mu


def map_dense(prob: Problem, d):
    """m_hat = A^-1 P^T N^-1 d by a dense Cholesky solve (tiny problems)."""
    A, P, N = dense_system(prob)
    return np.linalg.solve(A, P.T @ (N @ np.asarray(d, dtype=np.float64)))


def map_gradients(prob: Problem, d, g):
    """The gradients of map_gradients_dense without dense time-domain matrices, for
    problems with up to a few thousand unknowns: A is assembled column by column from
    the banded operator (apply_A), the noise-parameter gradient is the bilinear form
    (P mu)_j^T (dT_j/dtheta) (d - P m_hat)_j = sum_k dt_k c_j(k) with the lag
    correlations c_j of lag_correlations.  Returns (m_hat, dL/dd, dL/dtheta, mu)."""
    n = prob.n_obs * prob.n_s
    A = np.empty((n, n))
    e = np.zeros(n)
    for i in range(n):
        e[i] = 1.0
        A[:, i] = prob.apply_A(e)
        e[i] = 0.0
    A = 0.5 * (A + A.T)
    L = np.linalg.cholesky(A)

    def solve(rhs):
        return np.linalg.solve(L.T, np.linalg.solve(L, rhs))

    d = np.asarray(d, dtype=np.float64)
    m = solve(prob.rhs(d))
    mu = solve(np.asarray(g, dtype=np.float64))
    u = prob.depoint(mu)
    v = d - prob.depoint(m)
    grad_d = prob.ninv(u)
    n_int = len(prob.offsets) - 1
    grad_t = np.zeros((n_int, 3))
    for j in range(n_int):
        a, b = int(prob.offsets[j]), int(prob.offsets[j + 1])
        D = tap_derivatives(b - a, prob.sigma[j], prob.fknee[j], prob.alpha[j], prob.lam,
                            prob.f_samp, prob.window)
        c = lag_correlations(u[a:b], v[a:b], D.shape[1] - 1)
        grad_t[j] = D @ c
    return m, grad_d, grad_t, mu


# --------------------------------------------------------------------------
# a posteriori coarse space Z_D (Sect. 3.3.2, App. A)
# --------------------------------------------------------------------------

def pcg_lanczos(apply_A, b, precond, tol=1e-8, maxit=1000):
    """PCG from x0 = 0 that keeps what the Krylov process learns about M A: the step
    lengths alpha_k, the residual products rz_k = r_k^T z_k and the preconditioned
    residuals z_k (k = 0 .. m).  Stops on the recursive relative residual.
    Returns (x, alphas [m], rz [m+1], Zk [n, m+1])."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b)
    z = precond(r)
    rz = [r @ z]
    zs = [z.copy()]
    alphas = []
    p = z.copy()
    for _ in range(maxit):
        q = apply_A(p)
        a = rz[-1] / (p @ q)
        alphas.append(a)
        x += a * p
        r -= a * q
        z = precond(r)
        rz.append(r @ z)
        zs.append(z.copy())
        if np.linalg.norm(r) / bn <= tol:
            break
        p = z + (rz[-1] / rz[-2]) * p
    return x, np.array(alphas), np.array(rz), np.stack(zs, axis=1)


def lanczos_tridiagonal(alphas, rz):
    """The Lanczos matrix T_m of M A that CG builds implicitly (M symmetric positive
    definite, the Krylov basis orthonormal in the M^-1 inner product): with
    beta_k = rz_k / rz_{k-1},
      T[k, k]   = 1/alpha_k + beta_k / alpha_{k-1}   (second term absent for k = 0)
      T[k, k+1] = T[k+1, k] = sqrt(beta_{k+1}) / alpha_k,
    in the basis w_k = (-1)^k z_k / sqrt(rz_k) (z_k^T A z_{k+1} = -rz_{k+1} / alpha_k).
    The CG counterpart of the Arnoldi relation of App. A (H_m symmetric tridiagonal)."""
    m = alphas.shape[0]
    beta = rz[1:] / rz[:-1]
    T = np.zeros((m, m))
    for k in range(m):
        T[k, k] = 1.0 / alphas[k] + (beta[k - 1] / alphas[k - 1] if k > 0 else 0.0)
        if k + 1 < m:
            T[k, k + 1] = T[k + 1, k] = np.sqrt(beta[k]) / alphas[k]
    return T


def ritz_pairs(alphas, rz, Zk):
    """Ritz values theta_i and vectors y_i = W_m s_i of M A from one PCG run (eq.
    approxEigen with B = M_BD A): W_m has columns (-1)^k z_k / sqrt(rz_k), T_m s_i =
    theta_i s_i.  Also returns the error estimates |sqrt(beta_m)/alpha_{m-1} s_i[m-1]|,
    the size of the last term of eq. approxEigen in the M^-1 norm."""
    m = alphas.shape[0]
    T = lanczos_tridiagonal(alphas, rz)
    theta, S = np.linalg.eigh(T)
    W = Zk[:, :m] * ((-1.0) ** np.arange(m) / np.sqrt(rz[:m]))
    est = np.abs(np.sqrt(rz[m] / rz[m - 1]) / alphas[m - 1] * S[m - 1, :])
    return theta, W @ S, est


def deflation_space(prob: Problem, b, eps_tol=0.2, tol=1e-8, maxit=1000, max_cols=None):
    """Z_D (Sect. 3.3.2): the Ritz vectors of M_BD A with Ritz values below eps_tol, from
    a block-Jacobi PCG solve of A x' = b'."""
    B = prob.bj_blocks()
    _, al, rz, Zk = pcg_lanczos(prob.apply_A, b, lambda r: prob.bj_apply(r, B), tol, maxit)
    theta, Y, _ = ritz_pairs(al, rz, Zk)
    keep = np.nonzero(theta < eps_tol)[0]
    if max_cols is not None:
        keep = keep[:max_cols]
    return Y[:, keep], theta
