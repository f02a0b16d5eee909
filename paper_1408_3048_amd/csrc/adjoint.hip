// Adjoint of the GLS map m_hat = A^-1 P^T N^-1 d [Sect. 2.1, eq. glsSol] with respect to
// the time-ordered data and the noise parameters of every stationary interval.
//
// For a loss L(m_hat) with g = dL/dm_hat, mu = A^-1 g (one more PCG solve, A symmetric):
//   dL/dd        = N^-1 P mu
//   dL/dtheta_j  = (P mu)_j^T (dT_j/dtheta_j) (d - P m_hat)_j
//                = sum_k dt_k^(j)/dtheta_j c_j(k),
// where T_j is interval j's symmetric band Toeplitz block with taps t_k [Sect. 4.1.4,
// App. D] and c_j(0) = sum_t u_t v_t, c_j(k) = sum_t (u_t v_{t+k} + u_{t+k} v_t), u = P mu,
// v = d - P m_hat, t and t+k inside interval j.  The lag correlations are a banded
// product of the same shape as N^-1 itself; the tap derivatives are the windowed inverse
// DFTs of the derivatives of the inverse PSD, computed by the taps transform.
#include <algorithm>
#include <vector>

#include "mm_device.h"

namespace mm {
namespace {

constexpr int kLcThreads = 256;
constexpr int kLcR = 4;                       // lags per thread, 256 apart
constexpr int kLcLags = kLcThreads * kLcR;    // lags per block
constexpr int kLcT = 1024;                    // samples per chunk

__device__ __forceinline__ int find_interval(const int64_t* __restrict__ off, int n, int64_t v) {
    int a = 0, b = n - 1;
    while (a < b) {
        const int m = (a + b + 1) >> 1;
        if (off[m] <= v) a = m; else b = m - 1;
    }
    return a;
}

// Partial lag correlations of one chunk of kLcT samples of one interval for the lags
// [1 + blockIdx.y * kLcLags, ...) into part[chunk][k]; samples past the interval end are
// zeros, so only pairs inside the interval contribute.
__global__ __launch_bounds__(kLcThreads) void k_lag_corr(
    const double* __restrict__ u, const double* __restrict__ v,
    const int64_t* __restrict__ int_lo, const int64_t* __restrict__ int_hi,
    const int64_t* __restrict__ choff, int32_t n_int, int lam, double* __restrict__ part) {
    __shared__ double su[kLcT], sv[kLcT], su2[kLcT + kLcLags], sv2[kLcT + kLcLags];
    const int64_t ch = blockIdx.x;
    const int j = find_interval(choff, n_int, ch);
    const int64_t lo = int_lo[j], hi = int_hi[j];
    const int64_t t0 = lo + (ch - choff[j]) * kLcT;
    const int64_t K = min((int64_t)lam, hi - lo - 1);
    const int64_t k0 = 1 + (int64_t)blockIdx.y * kLcLags;
    if (k0 > K) return;
    for (int i = threadIdx.x; i < kLcT; i += kLcThreads) {
        const int64_t t = t0 + i;
        su[i] = t < hi ? u[t] : 0.0;
        sv[i] = t < hi ? v[t] : 0.0;
    }
    for (int i = threadIdx.x; i < kLcT + kLcLags; i += kLcThreads) {
        const int64_t t = t0 + k0 + i;
        su2[i] = t < hi ? u[t] : 0.0;
        sv2[i] = t < hi ? v[t] : 0.0;
    }
    __syncthreads();
    double acc[kLcR];
#pragma unroll
    for (int r = 0; r < kLcR; ++r) acc[r] = 0.0;
    for (int i = 0; i < kLcT; ++i) {
        const double a = su[i], b = sv[i];
#pragma unroll
        for (int r = 0; r < kLcR; ++r) {
            const int q = i + threadIdx.x + r * kLcThreads;
            acc[r] = fma(a, sv2[q], acc[r]);
            acc[r] = fma(su2[q], b, acc[r]);
        }
    }
    double* out = part + ch * (int64_t)(lam + 1);
#pragma unroll
    for (int r = 0; r < kLcR; ++r) {
        const int64_t k = k0 + threadIdx.x + r * kLcThreads;
        if (k <= K) out[k] = acc[r];
    }
}

// lag 0 of every chunk: sum u_t v_t over the chunk
__global__ __launch_bounds__(kLcThreads) void k_lag0(const double* __restrict__ u,
                                                     const double* __restrict__ v,
                                                     const int64_t* __restrict__ int_lo,
                                                     const int64_t* __restrict__ int_hi,
                                                     const int64_t* __restrict__ choff,
                                                     int32_t n_int, int lam,
                                                     double* __restrict__ part) {
    __shared__ double red[kLcThreads];
    const int64_t ch = blockIdx.x;
    const int j = find_interval(choff, n_int, ch);
    const int64_t hi = int_hi[j];
    const int64_t t0 = int_lo[j] + (ch - choff[j]) * kLcT;
    double s = 0.0;
    for (int i = threadIdx.x; i < kLcT; i += kLcThreads) {
        const int64_t t = t0 + i;
        if (t < hi) s = fma(u[t], v[t], s);
    }
    write_partial_at(s, part + ch * (int64_t)(lam + 1), 0, red);
}

// c[j][k] = sum over the chunks of interval j, in chunk order; 0 for k > K_j
__global__ void k_lag_reduce(const double* __restrict__ part, const int64_t* __restrict__ choff,
                             const int64_t* __restrict__ int_lo, const int64_t* __restrict__ int_hi,
                             int lam, double* __restrict__ c) {
    const int j = blockIdx.y;
    const int64_t K = min((int64_t)lam, int_hi[j] - int_lo[j] - 1);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= lam;
         k += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        if (k <= K)
            for (int64_t ch = choff[j]; ch < choff[j + 1]; ++ch) s += part[ch * (lam + 1) + k];
        c[(int64_t)j * (lam + 1) + k] = s;
    }
}

// v = d - v (d FP32 or FP64)
template <typename TD>
__global__ void k_resid_tod(const TD* __restrict__ d, double* __restrict__ v, int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        v[t] = (double)d[t] - v[t];
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        b[t] = (float)a[t];
}

inline int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

}  // namespace

int lag_correlations(mm_plan_t pl, const double* u, const double* v, double* c) {
    hipStream_t st = pl->stream;
    const int lam = pl->opts.lambda;
    std::vector<int64_t> choff(pl->n_int + 1, 0);
    for (int32_t j = 0; j < pl->n_int; ++j)
        choff[j + 1] = choff[j] + (pl->h_off[j + 1] - pl->h_off[j] + kLcT - 1) / kLcT;
    const int64_t nch = choff[pl->n_int];
    DBuf<int64_t> dch;
    DBuf<double> part;
    MM_TRY(dch.alloc(pl->n_int + 1));
    MM_TRY(part.alloc((size_t)nch * (lam + 1)));
    MM_HIP(hipMemcpyAsync(dch.p, choff.data(), (pl->n_int + 1) * 8, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_lag0, dim3(nch), dim3(kLcThreads), 0, st, u, v, pl->int_lo.p,
                       pl->int_hi.p, dch.p, pl->n_int, lam, part.p);
    MM_HIP(hipGetLastError());
    if (lam > 0) {
        const int ly = (lam + kLcLags - 1) / kLcLags;
        hipLaunchKernelGGL(k_lag_corr, dim3(nch, ly), dim3(kLcThreads), 0, st, u, v, pl->int_lo.p,
                           pl->int_hi.p, dch.p, pl->n_int, lam, part.p);
        MM_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_lag_reduce, dim3((lam + 256) / 256, pl->n_int), dim3(256), 0, st, part.p,
                       dch.p, pl->int_lo.p, pl->int_hi.p, lam, c);
    MM_HIP(hipGetLastError());
    MM_HIP(hipStreamSynchronize(st));  // scratch is released on return
    return MM_OK;
}

// dt[j][i][k] (host, [n_int][3][lambda+1], zero past K_j) for every interval
int tap_derivatives(mm_plan_t pl, std::vector<double>& dt) {
    const int lam = pl->opts.lambda;
    dt.assign((size_t)pl->n_int * 3 * (lam + 1), 0.0);
    for (int i = 0; i < 3; ++i) {
        std::vector<double> t;
        std::vector<int64_t> toff, tcnt;
        MM_TRY(kernel_taps(pl, i + 1, t, toff, tcnt));
        for (int32_t j = 0; j < pl->n_int; ++j) {
            const int g = pl->h_int_kern[j];
            double* o = dt.data() + ((size_t)j * 3 + i) * (lam + 1);
            for (int64_t k = 0; k < tcnt[g]; ++k) o[k] = t[toff[g] + k];
        }
    }
    return MM_OK;
}

int adjoint_tod(mm_plan_t pl, const double* m_hat, const double* mu, const void* d, int d_f64,
                void* grad_d, int grad_d_f64, double* grad_psd) {
    hipStream_t st = pl->stream;
    const int64_t n = pl->n_t;
    const int lam = pl->opts.lambda;
    DBuf<double> u, v, c;
    MM_TRY(u.alloc(n));
    MM_TRY(v.alloc(n));
    MM_TRY(depoint(pl, mu, u.p, 1));  // u = P mu
    if (grad_d) {
        if (grad_d_f64) {
            MM_TRY(toeplitz_tod64(pl, u.p, 1, (double*)grad_d));
        } else {
            MM_TRY(toeplitz_tod64(pl, u.p, 1, v.p));
            hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(256), 0, st, (const double*)v.p,
                               (float*)grad_d, n);
            MM_HIP(hipGetLastError());
        }
    }
    if (!grad_psd) return MM_OK;
    MM_TRY(depoint(pl, m_hat, v.p, 1));  // v = d - P m_hat
    if (d_f64)
        hipLaunchKernelGGL(k_resid_tod<double>, dim3(grid_for(n)), dim3(256), 0, st,
                           (const double*)d, v.p, n);
    else
        hipLaunchKernelGGL(k_resid_tod<float>, dim3(grid_for(n)), dim3(256), 0, st,
                           (const float*)d, v.p, n);
    MM_HIP(hipGetLastError());
    MM_TRY(c.alloc((size_t)pl->n_int * (lam + 1)));
    MM_TRY(lag_correlations(pl, u.p, v.p, c.p));
    std::vector<double> hc((size_t)pl->n_int * (lam + 1));
    MM_HIP(hipMemcpyAsync(hc.data(), c.p, hc.size() * 8, hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    std::vector<double> dt;
    MM_TRY(tap_derivatives(pl, dt));
    for (int32_t j = 0; j < pl->n_int; ++j)
        for (int i = 0; i < 3; ++i) {
            const double* a = dt.data() + ((size_t)j * 3 + i) * (lam + 1);
            const double* b = hc.data() + (size_t)j * (lam + 1);
            double s = 0.0;
            for (int k = 0; k <= lam; ++k) s += a[k] * b[k];
            grad_psd[3 * j + i] = s;
        }
    return MM_OK;
}

}  // namespace mm
