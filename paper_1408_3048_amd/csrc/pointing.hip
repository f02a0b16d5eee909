// Pointing P^T (deterministic segmented reduction over pixel-sorted samples),
// de-pointing P (time-ordered gather), and the block-Jacobi preconditioner
// M_BD = (P^T diag(N^-1) P)^-1 [Sect. 3.1, eq. stdPrec].
#include <cfloat>

#include "mm_device.h"

namespace mm {
namespace {

// x[p, s] = sum_{t in p} W[t, s] z_t.  Each wave owns a contiguous range of
// whole pixels (about 2048 samples) and walks it in chunks of 64 sorted
// samples: every lane forms W_t z_t for one sample, a segmented inclusive
// scan over the wave (segment starts are flagged by the head bitmask) sums
// the runs of each pixel, and the lane at a segment's end writes the total.
// Segments that straddle chunks carry their partial sum into the next chunk.
// The summation order is fixed by the plan, so results are deterministic.
template <typename T, int NS>
__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ perm,
                                                 const T* __restrict__ ws, const T* __restrict__ z,
                                                 const unsigned long long* __restrict__ heads,
                                                 const int32_t* __restrict__ wave_pix,
                                                 const int64_t* __restrict__ seg, int64_t n_waves,
                                                 double* __restrict__ out,
                                                 const int* __restrict__ done) {
    if (done && *done) return;
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= n_waves) return;
    const int32_t p0 = wave_pix[w], p1 = wave_pix[w + 1];
    if (p0 >= p1) return;
    const int64_t i0 = seg[p0], i1 = seg[p1];
    T carry[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) carry[s] = (T)0;
    int64_t pprev = (int64_t)p0 - 1;
    const unsigned long long le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    for (int64_t c = i0; c < i1; c += 64) {
        const int64_t i = c + lane;
        const bool valid = i < i1;
        T v[NS];
        bool head = false, end = false;
        if (valid) {
            const int64_t t = perm[i];
            const T zt = z[t];
            v[0] = zt;
            if constexpr (NS == 3) {
                v[1] = ws[2 * i] * zt;
                v[2] = ws[2 * i + 1] * zt;
            }
            head = (heads[i >> 6] >> (i & 63)) & 1ull;
            const int64_t i2 = i + 1;
            end = (i2 == i1) || ((heads[i2 >> 6] >> (i2 & 63)) & 1ull);
        } else {
#pragma unroll
            for (int s = 0; s < NS; ++s) v[s] = (T)0;
        }
        const unsigned long long hm = __ballot(head);
        int f = head ? 1 : 0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            T u[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) u[s] = __shfl_up(v[s], d);
            const int fu = __shfl_up(f, d);
            if (lane >= d) {
                if (!f) {
#pragma unroll
                    for (int s = 0; s < NS; ++s) v[s] += u[s];
                }
                f |= fu;
            }
        }
        const bool cont = (hm & le) == 0ull;
        const int64_t pix = pprev + __popcll(hm & le);
        T tot[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) tot[s] = cont ? v[s] + carry[s] : v[s];
        if (valid && end) {
#pragma unroll
            for (int s = 0; s < NS; ++s) out[pix * NS + s] = (double)tot[s];
        }
        const int open63 = __shfl((valid && !end) ? 1 : 0, 63);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const T c63 = __shfl(tot[s], 63);
            carry[s] = open63 ? c63 : (T)0;
        }
        pprev = __shfl(pix, 63);
    }
}

// y_t = sum_s W[t, s] x[c(t), s]
template <typename TO>
__global__ void k_depoint(const int32_t* __restrict__ cid, const double* __restrict__ w,
                          const double* __restrict__ x, int64_t n, int ns, TO* __restrict__ y) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = cid[t];
        double v;
        if (ns == 3)
            v = x[3 * c] + w[2 * t] * x[3 * c + 1] + w[2 * t + 1] * x[3 * c + 2];
        else
            v = x[c];
        y[t] = (TO)v;
    }
}

__device__ __forceinline__ int32_t interval_of(const int64_t* __restrict__ lo, int32_t n_int,
                                               int64_t t) {
    int32_t a = 0, b = n_int - 1;
    while (a < b) {
        const int32_t m = (a + b + 1) >> 1;
        if (lo[m] <= t) a = m; else b = m - 1;
    }
    return a;
}

// B_p = sum_{t in p} t_0^{(j(t))} W_t W_t^T, summed in ascending t; inverse and
// reciprocal 1-norm condition number.  bad[0] receives the smallest failing pixel.
__global__ void k_bj_build(const int32_t* __restrict__ perm, const double* __restrict__ ws,
                           const int64_t* __restrict__ seg, int64_t n_obs, int ns,
                           const int64_t* __restrict__ int_lo, int32_t n_int,
                           const int32_t* __restrict__ int_kern, const double* __restrict__ t0,
                           double rcond_min, double* __restrict__ bj, int* __restrict__ bad,
                           double* __restrict__ rc_out) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_obs;
         c += (int64_t)gridDim.x * blockDim.x) {
        double b00 = 0, b01 = 0, b02 = 0, b11 = 0, b12 = 0, b22 = 0;
        for (int64_t i = seg[c]; i < seg[c + 1]; ++i) {
            const int64_t t = perm[i];
            const double d = t0[int_kern[interval_of(int_lo, n_int, t)]];
            if (ns == 3) {
                const double u = ws[2 * i], v = ws[2 * i + 1];
                b00 += d;
                b01 += d * u;
                b02 += d * v;
                b11 += d * u * u;
                b12 += d * u * v;
                b22 += d * v * v;
            } else {
                b00 += d;
            }
        }
        double rc;
        if (ns == 1) {
            bj[c] = 1.0 / b00;
            rc = b00 > 0.0 ? 1.0 : 0.0;
        } else {
            // inverse of the symmetric block by cofactors
            const double c00 = b11 * b22 - b12 * b12;
            const double c01 = b02 * b12 - b01 * b22;
            const double c02 = b01 * b12 - b02 * b11;
            const double c11 = b00 * b22 - b02 * b02;
            const double c12 = b01 * b02 - b00 * b12;
            const double c22 = b00 * b11 - b01 * b01;
            const double det = b00 * c00 + b01 * c01 + b02 * c02;
            const double id = 1.0 / det;
            const double i00 = c00 * id, i01 = c01 * id, i02 = c02 * id, i11 = c11 * id,
                         i12 = c12 * id, i22 = c22 * id;
            bj[6 * c + 0] = i00;
            bj[6 * c + 1] = i01;
            bj[6 * c + 2] = i02;
            bj[6 * c + 3] = i11;
            bj[6 * c + 4] = i12;
            bj[6 * c + 5] = i22;
            const double n1 = fmax(fabs(b00) + fabs(b01) + fabs(b02),
                                   fmax(fabs(b01) + fabs(b11) + fabs(b12),
                                        fabs(b02) + fabs(b12) + fabs(b22)));
            const double ni = fmax(fabs(i00) + fabs(i01) + fabs(i02),
                                   fmax(fabs(i01) + fabs(i11) + fabs(i12),
                                        fabs(i02) + fabs(i12) + fabs(i22)));
            rc = (det > 0.0 && isfinite(ni)) ? 1.0 / (n1 * ni) : 0.0;
        }
        if (rc_out) rc_out[c] = rc;
        if (!(rc >= rcond_min)) atomicMin(bad, (int)c);
    }
}

// z = M_BD r (+ partial r^T z; optional convergence test on ||r|| in the prologue)
template <int NS>
__global__ __launch_bounds__(kVecThreads) void k_bj_apply(const double* __restrict__ r,
                                                          double* __restrict__ z,
                                                          const double* __restrict__ bj,
                                                          int64_t n_obs, PcgCtl ctl) {
    __shared__ double red[kVecThreads];
    if (ctl.part) {
        if (ctl.sc->done) return;
        if (ctl.check) {
            const double rr = reduce_partials(ctl.part + kSlotRR * kVecBlocks, kVecBlocks, red);
            const double rel = sqrt(rr) / ctl.sc->bnorm;
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                ctl.sc->rr = rr;
                if (ctl.hist) ctl.hist[ctl.iter] = rel;
                if (rel <= ctl.sc->tol) ctl.sc->done = 1;
            }
            if (rel <= ctl.sc->tol) return;
        }
    }
    double acc = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; c < n_obs;
         c += (int64_t)gridDim.x * kVecThreads) {
        if constexpr (NS == 1) {
            const double rv = r[c];
            const double zv = bj[c] * rv;
            z[c] = zv;
            acc += rv * zv;
        } else {
            const double* m = bj + 6 * c;
            const double r0 = r[3 * c], r1 = r[3 * c + 1], r2 = r[3 * c + 2];
            const double z0 = m[0] * r0 + m[1] * r1 + m[2] * r2;
            const double z1 = m[1] * r0 + m[3] * r1 + m[4] * r2;
            const double z2 = m[2] * r0 + m[4] * r1 + m[5] * r2;
            z[3 * c] = z0;
            z[3 * c + 1] = z1;
            z[3 * c + 2] = z2;
            acc += r0 * z0 + r1 * z1 + r2 * z2;
        }
    }
    if (ctl.part) write_partial(acc, ctl.part + kSlotRZ * kVecBlocks, red);
}

inline int grid_for(int64_t n, int threads = 256, int cap = 65536) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

template <typename T>
int scatter_t(mm_plan_t pl, const T* z, const T* ws, double* x, const int* done) {
    const int64_t nb = (pl->n_waves + 3) / 4;
    if (nb == 0) return MM_OK;
    if (pl->n_s == 3)
        hipLaunchKernelGGL((k_scatter<T, 3>), dim3(nb), dim3(256), 0, pl->stream, pl->perm.p, ws, z,
                           (const unsigned long long*)pl->heads.p, pl->wave_pix.p, pl->seg.p,
                           pl->n_waves, x, done);
    else
        hipLaunchKernelGGL((k_scatter<T, 1>), dim3(nb), dim3(256), 0, pl->stream, pl->perm.p, ws, z,
                           (const unsigned long long*)pl->heads.p, pl->wave_pix.p, pl->seg.p,
                           pl->n_waves, x, done);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

}  // namespace

int scatter64(mm_plan_t pl, const double* z, double* x, const int* done) {
    return scatter_t<double>(pl, z, pl->ws64.p, x, done);
}

int scatter32(mm_plan_t pl, const float* z, double* x, const int* done) {
    return scatter_t<float>(pl, z, pl->ws32.p, x, done);
}

int depoint(mm_plan_t pl, const double* x, void* y, int y_f64) {
    if (y_f64)
        hipLaunchKernelGGL(k_depoint<double>, dim3(grid_for(pl->n_t)), dim3(256), 0, pl->stream,
                           pl->cid.p, pl->w64.p, x, pl->n_t, pl->n_s, (double*)y);
    else
        hipLaunchKernelGGL(k_depoint<float>, dim3(grid_for(pl->n_t)), dim3(256), 0, pl->stream,
                           pl->cid.p, pl->w64.p, x, pl->n_t, pl->n_s, (float*)y);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int build_bj(mm_plan_t pl) {
    hipStream_t st = pl->stream;
    MM_TRY(pl->bj.alloc((size_t)pl->n_obs * (pl->n_s == 3 ? 6 : 1)));
    DBuf<int> bad;
    DBuf<double> rc;
    MM_TRY(bad.alloc(1));
    MM_TRY(rc.alloc(pl->n_obs));
    const int big = 0x7fffffff;
    MM_HIP(hipMemcpyAsync(bad.p, &big, sizeof(int), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_bj_build, dim3(grid_for(pl->n_obs, 128)), dim3(128), 0, st, pl->perm.p,
                       pl->ws64.p, pl->seg.p, pl->n_obs, pl->n_s, pl->int_lo.p, pl->n_int,
                       pl->int_kern.p, pl->kern_t0.p, pl->opts.rcond_min, pl->bj.p, bad.p, rc.p);
    MM_HIP(hipGetLastError());
    int h_bad = big;
    MM_HIP(hipMemcpyAsync(&h_bad, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    if (h_bad != big) {
        double rcv = 0.0;
        int32_t orig = -1;
        MM_HIP(hipMemcpy(&rcv, rc.p + h_bad, sizeof(double), hipMemcpyDeviceToHost));
        MM_HIP(hipMemcpy(&orig, pl->obs.p + h_bad, sizeof(int32_t), hipMemcpyDeviceToHost));
        set_error("pixel %d (compact %d): block-Jacobi block rcond %.3e < rcond_min %.3e "
                  "(pointing not full column rank there)",
                  orig, h_bad, rcv, pl->opts.rcond_min);
        return MM_ERR_RANK;
    }
    return MM_OK;
}

int bj_apply(mm_plan_t pl, const double* r, double* z, const PcgCtl& ctl) {
    if (pl->n_s == 3)
        hipLaunchKernelGGL(k_bj_apply<3>, dim3(kVecBlocks), dim3(kVecThreads), 0, pl->stream, r, z,
                           pl->bj.p, pl->n_obs, ctl);
    else
        hipLaunchKernelGGL(k_bj_apply<1>, dim3(kVecBlocks), dim3(kVecThreads), 0, pl->stream, r, z,
                           pl->bj.p, pl->n_obs, ctl);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

}  // namespace mm
