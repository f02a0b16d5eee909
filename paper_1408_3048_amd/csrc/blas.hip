// Pixel-domain vector kernels of PCG [Sect. 3.1]: fused updates with
// deterministic partial sums (fixed grid, fixed reduction trees) and device
// scalars, so the host never waits for a dot product.
#include "mm_device.h"

namespace mm {
namespace {

__global__ __launch_bounds__(kVecThreads) void k_dot(const double* __restrict__ a,
                                                     const double* __restrict__ b, int64_t n,
                                                     double* __restrict__ part,
                                                     const int* __restrict__ done) {
    __shared__ double red[kVecThreads];
    if (done && *done) return;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kVecThreads)
        acc += a[i] * b[i];
    write_partial(acc, part, red);
}

// alpha = r^T z / p^T q; x += alpha p; r -= alpha q; partial ||r||^2
__global__ __launch_bounds__(kVecThreads) void k_update_xr(double* __restrict__ x,
                                                           double* __restrict__ r,
                                                           const double* __restrict__ p,
                                                           const double* __restrict__ q,
                                                           int64_t n, PcgCtl ctl) {
    __shared__ double red[kVecThreads];
    if (ctl.sc->done) return;
    const double pq = reduce_partials(ctl.part + kSlotPQ * kVecBlocks, kVecBlocks, red);
    const double rz = ctl.rz_hist[ctl.iter];
    const bool ok = pq > 0.0 && isfinite(pq) && isfinite(rz);
    if (!ok) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctl.sc->status = 1;
            ctl.sc->done = 1;
            ctl.sc->pq = pq;
        }
        return;
    }
    const double alpha = rz / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl.sc->alpha = alpha;
        ctl.sc->pq = pq;
        ctl.sc->iter = ctl.iter + 1;
    }
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kVecThreads) {
        x[i] += alpha * p[i];
        const double rv = r[i] - alpha * q[i];
        r[i] = rv;
        acc += rv * rv;
    }
    write_partial(acc, ctl.part + kSlotRR * kVecBlocks, red);
}

// beta = r_new^T z_new / r^T z; p = z + beta p (p = z on the first call)
__global__ __launch_bounds__(kVecThreads) void k_update_p(double* __restrict__ p,
                                                          const double* __restrict__ z, int64_t n,
                                                          PcgCtl ctl) {
    __shared__ double red[kVecThreads];
    if (ctl.sc->done) return;
    const double rz_new = reduce_partials(ctl.part + kSlotRZ * kVecBlocks, kVecBlocks, red);
    const double beta = ctl.first ? 0.0 : rz_new / ctl.rz_hist[ctl.iter];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl.rz_hist[ctl.iter + 1] = rz_new;
        ctl.sc->beta = beta;
    }
    if (ctl.rz_only) return;
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kVecThreads)
        p[i] = ctl.first ? z[i] : z[i] + beta * p[i];
}

__global__ __launch_bounds__(kVecThreads) void k_axpby(double a, const double* __restrict__ x,
                                                       double b, const double* __restrict__ y,
                                                       double* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kVecThreads)
        out[i] = a * x[i] + b * y[i];
}

__global__ __launch_bounds__(kVecThreads) void k_set_scalars(PcgCtl ctl, double tol,
                                                             const double* __restrict__ part_bb,
                                                             int iter_base) {
    __shared__ double red[kVecThreads];
    const double bb = reduce_partials(part_bb, kVecBlocks, red);
    if (threadIdx.x == 0) {
        ctl.sc->bnorm = sqrt(bb);
        ctl.sc->tol = tol;
        ctl.sc->done = 0;
        ctl.sc->status = 0;
        ctl.sc->iter = iter_base;
    }
}

}  // namespace

int64_t nvec(mm_plan_t pl) { return pl->n_obs * pl->n_s; }

int vec_dot(mm_plan_t pl, const double* a, const double* b, double* part, const int* done) {
    hipLaunchKernelGGL(k_dot, dim3(kVecBlocks), dim3(kVecThreads), 0, pl->stream, a, b, nvec(pl),
                       part, done);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int pcg_update_xr(mm_plan_t pl, double* x, double* r, const double* p, const double* q,
                  const PcgCtl& ctl) {
    hipLaunchKernelGGL(k_update_xr, dim3(kVecBlocks), dim3(kVecThreads), 0, pl->stream, x, r, p, q,
                       nvec(pl), ctl);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int pcg_update_p(mm_plan_t pl, double* p, const double* z, const PcgCtl& ctl) {
    hipLaunchKernelGGL(k_update_p, dim3(kVecBlocks), dim3(kVecThreads), 0, pl->stream, p, z,
                       nvec(pl), ctl);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int vec_axpby(mm_plan_t pl, double a, const double* x, double b, const double* y, double* out) {
    hipLaunchKernelGGL(k_axpby, dim3(kVecBlocks), dim3(kVecThreads), 0, pl->stream, a, x, b, y, out,
                       nvec(pl));
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int vec_set_scalars(mm_plan_t pl, const PcgCtl& ctl, double tol, const double* part_bb,
                    int iter_base) {
    hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(kVecThreads), 0, pl->stream, ctl, tol, part_bb,
                       iter_base);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

}  // namespace mm
