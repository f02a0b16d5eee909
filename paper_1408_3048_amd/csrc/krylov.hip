// Ritz pairs of M_BD A from one block-Jacobi PCG solve [Sect. 3.3.2; App. A, eq.
// approxEigen with B = M_BD A].
//
// PCG on A x = b with an SPD preconditioner M is the Lanczos process on M A in the M^-1
// inner product: with step lengths alpha_k, rz_k = r_k^T z_k and beta_k = rz_k / rz_{k-1},
// the vectors w_k = (-1)^k z_k / sqrt(rz_k) are M^-1-orthonormal and W^T A W is the
// symmetric tridiagonal T with
//   T[k][k]   = 1/alpha_k + beta_k / alpha_{k-1}     (second term absent for k = 0)
//   T[k][k+1] = sqrt(beta_{k+1}) / alpha_k,
// the CG counterpart of the Arnoldi relation (H_m symmetric tridiagonal).  The Ritz pairs
// are (theta_i, y_i = W s_i) with T s_i = theta_i s_i.
//
// Only the Ritz values below eps_tol are wanted (a few of m), so the eigenvalues come from
// Sturm-sequence bisection (exact counts, O(m) per step) and the eigenvectors from inverse
// iteration on T - theta I with a pivoted tridiagonal LU, re-orthogonalised against the
// vectors of the same cluster of close eigenvalues.  Everything here is host code on
// O(m) data.
#include <algorithm>
#include <cmath>
#include <vector>

#include "mm_device.h"

namespace mm {
namespace {

// number of eigenvalues of the tridiagonal (d, e) below x (LDL^T pivot signs)
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x,
                double pivmin) {
    const int m = (int)d.size();
    int cnt = 0;
    double q = d[0] - x;
    if (std::fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
    for (int i = 1; i < m; ++i) {
        q = d[i] - x - e[i - 1] * e[i - 1] / q;
        if (std::fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// solve (T - sigma I) y = rhs in place by Gaussian elimination with partial pivoting on
// the tridiagonal (d, e); zero pivots are replaced by tiny
void tridiag_shift_solve(const std::vector<double>& d, const std::vector<double>& e, double sigma,
                         double tiny, std::vector<double>& y) {
    const int m = (int)d.size();
    std::vector<double> a(m), b(m, 0.0), u2(m, 0.0), l(m, 0.0);
    std::vector<char> sw(m, 0);
    for (int i = 0; i < m; ++i) a[i] = d[i] - sigma;
    for (int i = 0; i + 1 < m; ++i) b[i] = e[i];
    // row i holds (a[i], b[i], u2[i]) at columns i, i+1, i+2 after its elimination step;
    // row i+1 enters step i as (e[i], a[i+1], b[i+1])
    for (int i = 0; i + 1 < m; ++i) {
        const double c = e[i];  // sub-diagonal entry of row i+1 (never modified before step i)
        if (std::fabs(a[i]) >= std::fabs(c)) {
            if (a[i] == 0.0) a[i] = tiny;
            l[i] = c / a[i];
            a[i + 1] -= l[i] * b[i];
            u2[i] = 0.0;
        } else {
            // rows i and i+1 trade places
            const double t = l[i] = a[i] / c;
            const double ai1 = a[i + 1], bi = b[i];
            const double bi1 = i + 2 < m ? b[i + 1] : 0.0;
            a[i] = c;
            b[i] = ai1;
            u2[i] = bi1;
            a[i + 1] = bi - t * ai1;
            if (i + 2 < m) b[i + 1] = -t * bi1;
            sw[i] = 1;
        }
    }
    if (a[m - 1] == 0.0) a[m - 1] = tiny;
    for (int i = 0; i + 1 < m; ++i) {
        if (sw[i]) std::swap(y[i], y[i + 1]);
        y[i + 1] -= l[i] * y[i];
    }
    for (int i = m - 1; i >= 0; --i) {
        double v = y[i];
        if (i + 1 < m) v -= b[i] * y[i + 1];
        if (i + 2 < m) v -= u2[i] * y[i + 2];
        y[i] = v / a[i];
    }
}

double norm2(const std::vector<double>& v) {
    double s = 0.0;
    for (double x : v) s += x * x;
    return std::sqrt(s);
}

}  // namespace

int ritz_select(const double* alpha, const double* rz, int m, double eps_tol, int max_cols,
                std::vector<double>& theta, std::vector<double>& S) {
    theta.clear();
    S.clear();
    if (m <= 0) return MM_OK;
    std::vector<double> d(m), e(std::max(m - 1, 1), 0.0);
    for (int k = 0; k < m; ++k) {
        if (!(alpha[k] > 0.0) || !(rz[k] > 0.0) || !std::isfinite(alpha[k]) ||
            !std::isfinite(rz[k])) {
            set_error("Lanczos matrix undefined: step %d has alpha = %g, r^T z = %g", k,
                      alpha[k], rz[k]);
            return MM_ERR_BREAKDOWN;
        }
        d[k] = 1.0 / alpha[k] + (k > 0 ? (rz[k] / rz[k - 1]) / alpha[k - 1] : 0.0);
        if (k + 1 < m) e[k] = std::sqrt(rz[k + 1] / rz[k]) / alpha[k];
    }
    // Gershgorin interval and scale
    double lo = d[0], hi = d[0];
    for (int k = 0; k < m; ++k) {
        const double rad = (k > 0 ? std::fabs(e[k - 1]) : 0.0) + (k + 1 < m ? std::fabs(e[k]) : 0.0);
        lo = std::min(lo, d[k] - rad);
        hi = std::max(hi, d[k] + rad);
    }
    const double tnorm = std::max(std::fabs(lo), std::fabs(hi));
    const double eps = 2.220446049250313e-16;
    const double pivmin = std::max(tnorm * eps * eps, 1e-300);
    int r = eps_tol > lo ? sturm_count(d, e, std::min(eps_tol, hi + 1.0), pivmin) : 0;
    if (max_cols > 0) r = std::min(r, max_cols);
    if (r == 0) return MM_OK;
    // eigenvalue i (ascending): bisection on the count until the bracket is at rounding level
    theta.resize(r);
    for (int i = 0; i < r; ++i) {
        double a = lo - eps * tnorm, b = hi + eps * tnorm;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (a + b);
            if (mid <= a || mid >= b) break;
            if (b - a <= 2.0 * eps * std::max(std::fabs(a), std::fabs(b)) + pivmin) break;
            if (sturm_count(d, e, mid, pivmin) > i) b = mid;
            else a = mid;
        }
        theta[i] = 0.5 * (a + b);
    }
    // eigenvectors by inverse iteration; members of a cluster (gap below 1e-3 ||T||) are
    // kept orthogonal to the earlier members
    S.assign((size_t)m * r, 0.0);
    std::vector<std::vector<double>> vecs;
    const double tiny = eps * tnorm;
    int cluster0 = 0;
    for (int i = 0; i < r; ++i) {
        if (i > 0 && theta[i] - theta[i - 1] > 1e-3 * tnorm) cluster0 = i;
        std::vector<double> y(m);
        uint64_t s = 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
        for (int k = 0; k < m; ++k) {  // deterministic start vector with every component set
            s ^= s >> 12;
            s ^= s << 25;
            s ^= s >> 27;
            y[k] = 0.5 + (double)((s * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
        }
        for (int it = 0; it < 4; ++it) {
            for (int j = cluster0; j < i; ++j) {
                double dot = 0.0;
                for (int k = 0; k < m; ++k) dot += vecs[j][k] * y[k];
                for (int k = 0; k < m; ++k) y[k] -= dot * vecs[j][k];
            }
            double nrm = norm2(y);
            if (!(nrm > 0.0)) {
                set_error("inverse iteration failed for Ritz value %d", i);
                return MM_ERR_BREAKDOWN;
            }
            for (double& v : y) v /= nrm;
            tridiag_shift_solve(d, e, theta[i], tiny, y);
        }
        for (int j = cluster0; j < i; ++j) {
            double dot = 0.0;
            for (int k = 0; k < m; ++k) dot += vecs[j][k] * y[k];
            for (int k = 0; k < m; ++k) y[k] -= dot * vecs[j][k];
        }
        const double nrm = norm2(y);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) {
            set_error("inverse iteration failed for Ritz value %d", i);
            return MM_ERR_BREAKDOWN;
        }
        for (double& v : y) v /= nrm;
        // sign convention: largest-magnitude component positive
        int kmax = 0;
        for (int k = 1; k < m; ++k)
            if (std::fabs(y[k]) > std::fabs(y[kmax])) kmax = k;
        if (y[kmax] < 0.0)
            for (double& v : y) v = -v;
        for (int k = 0; k < m; ++k) S[(size_t)k * r + i] = y[k];
        vecs.push_back(std::move(y));
    }
    return MM_OK;
}

}  // namespace mm
