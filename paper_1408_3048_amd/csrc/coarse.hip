// Two-level A-DEF1 preconditioner with the a priori coarse space Z_S
// [Sect. 3.2, eqs. projection and 2; Sect. 3.3.1, eqs. strofZ, strofZ_polar;
// App. C].
//
// Construction (App. C): Z_S has one column per stationary interval holding,
// on the I row of every observed pixel, the fraction s_p^j / s_p of the
// pixel's hits that fall in interval j (Q and U rows are zero).  Identical
// columns (intervals with identical hit patterns, e.g. co-pointed detectors)
// are merged first; AZ is formed by applying A to each remaining column; the
// coarse matrix E = Z^T (AZ) is a tall-skinny FP64 product on the matrix
// cores; a pivoted Cholesky factorisation of E on the host keeps a maximal
// A-independent subset of columns (span(Z), and hence M_2lvl, unchanged) and
// inverts E on it.
//
// Application (App. C, four steps): v = Z^T r; w = E^-1 v; then per pixel
// z = M_BD (r - (AZ) w) + Z w.
#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <unordered_map>

#include "mm_device.h"

namespace mm {
namespace {

inline int grid_for(int64_t n, int threads = 256, int cap = 65536) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
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

// number of distinct intervals among each pixel's samples (ascending in t)
__global__ void k_zs_count(const int32_t* __restrict__ perm, const int64_t* __restrict__ seg,
                           int64_t n_obs, const int64_t* __restrict__ int_lo, int32_t n_int,
                           int64_t* __restrict__ nnz) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_obs;
         c += (int64_t)gridDim.x * blockDim.x) {
        int64_t cnt = 0;
        int32_t last = -1;
        for (int64_t i = seg[c]; i < seg[c + 1]; ++i) {
            const int32_t j = interval_of(int_lo, n_int, perm[i]);
            if (j != last) {
                ++cnt;
                last = j;
            }
        }
        nnz[c] = cnt;
    }
}

__global__ void k_zs_fill(const int32_t* __restrict__ perm, const int64_t* __restrict__ seg,
                          int64_t n_obs, const int64_t* __restrict__ int_lo, int32_t n_int,
                          const int64_t* __restrict__ ptr, int32_t* __restrict__ col,
                          double* __restrict__ val) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_obs;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = seg[c + 1] - seg[c];
        int64_t o = ptr[c];
        int32_t last = -1;
        int64_t run = 0;
        for (int64_t i = seg[c]; i < seg[c + 1]; ++i) {
            const int32_t j = interval_of(int_lo, n_int, perm[i]);
            if (j != last) {
                if (last >= 0) {
                    col[o] = last;
                    val[o] = (double)run / (double)s;
                    ++o;
                }
                last = j;
                run = 0;
            }
            ++run;
        }
        if (last >= 0) {
            col[o] = last;
            val[o] = (double)run / (double)s;
        }
    }
}


__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

// scatter column entries (pixel, value) into a zeroed map vector (I rows)
__global__ void k_col_to_vec(const int32_t* __restrict__ rows, const double* __restrict__ vals,
                             int64_t cnt, int ns, double* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
         i += (int64_t)gridDim.x * blockDim.x)
        out[(int64_t)rows[i] * ns] = vals[i];
}

// Z_S rows restricted to the kept columns: count pass (out == nullptr) or fill pass
__global__ void k_csr_filter(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                             const double* __restrict__ val, int64_t n_obs,
                             const int32_t* __restrict__ colmap, const int64_t* __restrict__ optr,
                             int64_t* __restrict__ cnt, int32_t* __restrict__ ocol,
                             double* __restrict__ oval) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_obs;
         p += (int64_t)gridDim.x * blockDim.x) {
        int64_t o = optr ? optr[p] : 0;
        for (int64_t e = ptr[p]; e < ptr[p + 1]; ++e) {
            const int32_t a = colmap[col[e]];
            if (a < 0) continue;
            if (ocol) {
                ocol[o] = a;
                oval[o] = val[e];
            }
            ++o;
        }
        if (cnt) cnt[p] = o;
    }
}

// dense Z_I, row-major [n_obs_pad][rp] from per-column entry lists
__global__ void k_dense_z(const int64_t* __restrict__ cptr, const int32_t* __restrict__ rows,
                          const double* __restrict__ vals, int32_t r, int32_t rp,
                          double* __restrict__ zd) {
    const int32_t c = blockIdx.y;
    if (c >= r) return;
    for (int64_t i = cptr[c] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cptr[c + 1];
         i += (int64_t)gridDim.x * blockDim.x)
        zd[(int64_t)rows[i] * rp + c] = vals[i];
}

// AZ_I row-major [n_obs_pad][rp] from column-major AZ [r][n_vec] (I rows)
template <typename TA>
__global__ void k_az_rows(const TA* __restrict__ az, int64_t n_vec, int64_t n_obs, int ns,
                          int32_t r, int32_t rp, double* __restrict__ out) {
    const int32_t c = blockIdx.y;
    if (c >= r) return;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_obs;
         p += (int64_t)gridDim.x * blockDim.x)
        out[p * rp + c] = (double)az[(int64_t)c * n_vec + p * ns];
}

// ---------------------------------------------------------------- FP64 MFMA: C = A^T B
// A: row-major [n][ra], B: row-major [n][rb] (n a multiple of 4, ra and rb multiples of
// 16), C partials [ksplit][ra][rb].  One wave per 16x16 output tile and pixel slab;
// v_mfma_f64_16x16x4f64: lane l supplies A(i = l%16, k = l/16) and B(k = l/16, j = l%16)
// and holds D(i = l/16 + 4 v, j = l%16) in accumulator register v (v = 0..3).
typedef double dbl4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_gemm_tn_f64(const double* __restrict__ A,
                                                     const double* __restrict__ B, int64_t n,
                                                     int32_t ra, int32_t rb, int32_t ksplit,
                                                     double* __restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int32_t ta_n = ra / 16, tb_n = rb / 16;
    const int64_t ntile = (int64_t)ta_n * tb_n;
    if (wid >= ntile * ksplit) return;
    const int32_t ks = (int32_t)(wid / ntile);
    const int64_t tile = wid % ntile;
    const int32_t ta = (int32_t)(tile / tb_n), tb = (int32_t)(tile % tb_n);
    const int64_t nq = n / 4;
    const int64_t q0 = nq * ks / ksplit, q1 = nq * (ks + 1) / ksplit;
    const int i = lane & 15, k = lane >> 4;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    const double* Ap = A + (int64_t)16 * ta + i;
    const double* Bp = B + (int64_t)16 * tb + i;
    for (int64_t q = q0; q < q1; ++q) {
        const int64_t row = 4 * q + k;
        const double a = Ap[row * ra];
        const double b = Bp[row * rb];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    double* out = part + (int64_t)ks * ra * rb;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = 16 * ta + k + 4 * v;
        const int col = 16 * tb + i;
        out[(int64_t)row * rb + col] = acc[v];
    }
}

__global__ void k_sum_parts(const double* __restrict__ part, int64_t m, int32_t ksplit,
                            double* __restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int32_t k = 0; k < ksplit; ++k) s += part[(int64_t)k * m + e];
        out[e] = s;
    }
}

// v = Z^T r: each kept column's entries are split over `slices` waves whose partial sums
// go to vpart[column][slice]; optional convergence test in the prologue
__global__ __launch_bounds__(256) void k_ztr(const int64_t* __restrict__ cbeg,
                                             const int64_t* __restrict__ cend,
                                             const int32_t* __restrict__ rows,
                                             const double* __restrict__ vals,
                                             const double* __restrict__ r, int ns, int32_t rk,
                                             int32_t slices, double* __restrict__ vpart,
                                             PcgCtl ctl) {
    __shared__ double red[256];
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
    const int lane = threadIdx.x & 63;
    const int64_t wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wv >= (int64_t)rk * slices) return;
    const int32_t c = (int32_t)(wv / slices), sl = (int32_t)(wv % slices);
    const int64_t e0 = cbeg[c], len = cend[c] - e0;
    const int64_t a = e0 + len * sl / slices, b = e0 + len * (sl + 1) / slices;
    double s = 0.0;
    for (int64_t e = a + lane; e < b; e += 64) s += vals[e] * r[(int64_t)rows[e] * ns];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) vpart[wv] = s;
}

// w = E^-1 v with v[c] = sum of the slice partials of column c (one wave per row)
__global__ __launch_bounds__(256) void k_einv(const double* __restrict__ Einv,
                                              const double* __restrict__ vpart, int32_t rk,
                                              int32_t slices, double* __restrict__ w,
                                              const PcgScalars* sc) {
    if (sc && sc->done) return;
    const int lane = threadIdx.x & 63;
    const int32_t a = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (a >= rk) return;
    double s = 0.0;
    for (int32_t c = lane; c < rk; c += 64) {
        double v = 0.0;
        for (int32_t q = 0; q < slices; ++q) v += vpart[(int64_t)c * slices + q];
        s += Einv[(int64_t)a * rk + c] * v;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) w[a] = s;
}

// z = M_BD (r - AZ w) + Z w, partial r^T z
template <typename TA, int NS>
__global__ __launch_bounds__(kVecThreads) void k_2lvl(
    const double* __restrict__ r, double* __restrict__ z, const double* __restrict__ bj,
    const TA* __restrict__ az, int64_t n_obs, int32_t rk, const double* __restrict__ w,
    const int64_t* __restrict__ zptr, const int32_t* __restrict__ zcol,
    const double* __restrict__ zval, PcgCtl ctl) {
    __shared__ double red[kVecThreads];
    extern __shared__ double sw[];
    if (ctl.part && ctl.sc->done) return;
    for (int c = threadIdx.x; c < rk; c += kVecThreads) sw[c] = w[c];
    __syncthreads();
    const int64_t nv = n_obs * NS;
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; p < n_obs;
         p += (int64_t)gridDim.x * kVecThreads) {
        double u[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) u[s] = r[p * NS + s];
        for (int32_t c = 0; c < rk; ++c) {
            const double wc = sw[c];
            const TA* col = az + (int64_t)c * nv + p * NS;
#pragma unroll
            for (int s = 0; s < NS; ++s) u[s] -= (double)col[s] * wc;
        }
        double zz[NS];
        if constexpr (NS == 1) {
            zz[0] = bj[p] * u[0];
        } else {
            const double* m = bj + 6 * p;
            zz[0] = m[0] * u[0] + m[1] * u[1] + m[2] * u[2];
            zz[1] = m[1] * u[0] + m[3] * u[1] + m[4] * u[2];
            zz[2] = m[2] * u[0] + m[4] * u[1] + m[5] * u[2];
        }
        double zw = 0.0;
        for (int64_t e = zptr[p]; e < zptr[p + 1]; ++e) zw += zval[e] * sw[zcol[e]];
        zz[0] += zw;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            z[p * NS + s] = zz[s];
            acc += r[p * NS + s] * zz[s];
        }
    }
    if (ctl.part) write_partial(acc, ctl.part + kSlotRZ * kVecBlocks, red);
}

// pivoted Cholesky of a symmetric PSD matrix: indices of a maximal set of columns whose
// Schur-complement diagonal stays above tol * max diag
std::vector<int> pivoted_cholesky_select(const std::vector<double>& E, int r, double tol) {
    std::vector<double> A(E);
    std::vector<double> L((size_t)r * r, 0.0);
    std::vector<int> piv(r);
    for (int i = 0; i < r; ++i) piv[i] = i;
    std::vector<double> d(r);
    double dmax0 = 0.0;
    for (int i = 0; i < r; ++i) {
        d[i] = A[(size_t)i * r + i];
        dmax0 = std::max(dmax0, d[i]);
    }
    std::vector<int> sel;
    if (!(dmax0 > 0.0)) return sel;
    // L stored by (original index, step)
    for (int s = 0; s < r; ++s) {
        int jb = -1;
        double db = -1.0;
        for (int q = s; q < r; ++q) {
            if (d[piv[q]] > db) {
                db = d[piv[q]];
                jb = q;
            }
        }
        if (db <= tol * dmax0) break;
        std::swap(piv[s], piv[jb]);
        const int j = piv[s];
        const double ljj = std::sqrt(db);
        L[(size_t)j * r + s] = ljj;
        for (int q = s + 1; q < r; ++q) {
            const int i = piv[q];
            double v = A[(size_t)i * r + j];
            for (int t = 0; t < s; ++t) v -= L[(size_t)i * r + t] * L[(size_t)j * r + t];
            v /= ljj;
            L[(size_t)i * r + s] = v;
            d[i] -= v * v;
        }
        sel.push_back(j);
    }
    std::sort(sel.begin(), sel.end());
    return sel;
}

// inverse of an SPD matrix by Cholesky (row-major, in place result in out); false if not PD
bool spd_inverse(const std::vector<double>& A, int k, std::vector<double>& out) {
    std::vector<double> L((size_t)k * k, 0.0);
    for (int j = 0; j < k; ++j) {
        double s = A[(size_t)j * k + j];
        for (int t = 0; t < j; ++t) s -= L[(size_t)j * k + t] * L[(size_t)j * k + t];
        if (!(s > 0.0)) return false;
        const double ljj = std::sqrt(s);
        L[(size_t)j * k + j] = ljj;
        for (int i = j + 1; i < k; ++i) {
            double v = A[(size_t)i * k + j];
            for (int t = 0; t < j; ++t) v -= L[(size_t)i * k + t] * L[(size_t)j * k + t];
            L[(size_t)i * k + j] = v / ljj;
        }
    }
    // Linv (lower triangular)
    std::vector<double> Li((size_t)k * k, 0.0);
    for (int j = 0; j < k; ++j) {
        Li[(size_t)j * k + j] = 1.0 / L[(size_t)j * k + j];
        for (int i = j + 1; i < k; ++i) {
            double s = 0.0;
            for (int t = j; t < i; ++t) s += L[(size_t)i * k + t] * Li[(size_t)t * k + j];
            Li[(size_t)i * k + j] = -s / L[(size_t)i * k + i];
        }
    }
    out.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = 0.0;
            for (int t = i; t < k; ++t) s += Li[(size_t)t * k + i] * Li[(size_t)t * k + j];
            out[(size_t)i * k + j] = s;
            out[(size_t)j * k + i] = s;
        }
    return true;
}

}  // namespace

// C[ra][rb] (host, row-major) = A^T B for device row-major A [n][ra], B [n][rb]
int gemm_tn_f64(hipStream_t st, const double* A, const double* B, int64_t n, int32_t ra,
                int32_t rb, double* dev_C) {
    const int32_t ntile = (ra / 16) * (rb / 16);
    int32_t ksplit = (int32_t)std::max<int64_t>(1, std::min<int64_t>(n / 4 / 64, 4096 / std::max(1, ntile)));
    DBuf<double> part;
    MM_TRY(part.alloc((size_t)ksplit * ra * rb));
    const int64_t waves = (int64_t)ntile * ksplit;
    hipLaunchKernelGGL(k_gemm_tn_f64, dim3((waves + 3) / 4), dim3(256), 0, st, A, B, n, ra, rb,
                       ksplit, part.p);
    MM_HIP(hipGetLastError());
    const int64_t m = (int64_t)ra * rb;
    hipLaunchKernelGGL(k_sum_parts, dim3(grid_for(m)), dim3(256), 0, st, part.p, m, ksplit, dev_C);
    MM_HIP(hipGetLastError());
    MM_HIP(hipStreamSynchronize(st));
    return MM_OK;
}

int build_coarse(mm_plan_t pl) {
    hipStream_t st = pl->stream;
    const bool verbose = std::getenv("MM_PLAN_TIMING") != nullptr;
    const auto c0 = std::chrono::steady_clock::now();
    auto tick = [&](const char* what) {
        if (!verbose) return;
        (void)hipStreamSynchronize(st);
        std::fprintf(stderr, "[coarse ] %-10s %8.3f ms\n", what,
                     std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - c0).count());
    };
    Coarse& co = pl->co;
    const int64_t n_obs = pl->n_obs, ns = pl->n_s, nv = n_obs * ns;
    // Z_S in CSR form (per pixel, ascending interval)
    DBuf<int64_t> nnz, ptr;
    MM_TRY(nnz.alloc(n_obs));
    MM_TRY(ptr.alloc(n_obs + 1));
    hipLaunchKernelGGL(k_zs_count, dim3(grid_for(n_obs, 128)), dim3(128), 0, st, pl->perm.p,
                       pl->seg.p, n_obs, pl->int_lo.p, pl->n_int, nnz.p);
    MM_HIP(hipGetLastError());
    {
        // exclusive scan on host (n_obs values)
        std::vector<int64_t> h(n_obs), hp(n_obs + 1);
        MM_HIP(hipMemcpyAsync(h.data(), nnz.p, n_obs * 8, hipMemcpyDeviceToHost, st));
        MM_HIP(hipStreamSynchronize(st));
        hp[0] = 0;
        for (int64_t c = 0; c < n_obs; ++c) hp[c + 1] = hp[c] + h[c];
        MM_HIP(hipMemcpyAsync(ptr.p, hp.data(), (n_obs + 1) * 8, hipMemcpyHostToDevice, st));
    }
    int64_t total = 0;
    MM_HIP(hipMemcpyAsync(&total, ptr.p + n_obs, 8, hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    DBuf<int32_t> col;
    DBuf<double> val;
    MM_TRY(col.alloc(total));
    MM_TRY(val.alloc(total));
    hipLaunchKernelGGL(k_zs_fill, dim3(grid_for(n_obs, 128)), dim3(128), 0, st, pl->perm.p,
                       pl->seg.p, n_obs, pl->int_lo.p, pl->n_int, ptr.p, col.p, val.p);
    MM_HIP(hipGetLastError());
    std::vector<int64_t> hptr(n_obs + 1);
    std::vector<int32_t> hcol(total);
    std::vector<double> hval(total);
    MM_HIP(hipMemcpyAsync(hptr.data(), ptr.p, (n_obs + 1) * 8, hipMemcpyDeviceToHost, st));
    MM_HIP(hipMemcpyAsync(hcol.data(), col.p, total * 4, hipMemcpyDeviceToHost, st));
    MM_HIP(hipMemcpyAsync(hval.data(), val.p, total * 8, hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    // per-column entry lists (ascending pixel), duplicate columns merged
    const int32_t K = pl->n_int;
    std::vector<int64_t> ccnt(K + 1, 0);
    for (int64_t e = 0; e < total; ++e) ccnt[hcol[e] + 1]++;
    for (int32_t j = 0; j < K; ++j) ccnt[j + 1] += ccnt[j];
    std::vector<int32_t> crow(total);
    std::vector<double> cval(total);
    {
        std::vector<int64_t> fillp(ccnt.begin(), ccnt.end() - 1);
        for (int64_t p = 0; p < n_obs; ++p)
            for (int64_t e = hptr[p]; e < hptr[p + 1]; ++e) {
                const int64_t d = fillp[hcol[e]]++;
                crow[d] = (int32_t)p;
                cval[d] = hval[e];
            }
    }
    std::vector<int32_t> uniq;  // representative interval of every distinct column
    {
        std::unordered_map<uint64_t, std::vector<int32_t>> buckets;
        for (int32_t j = 0; j < K; ++j) {
            if (ccnt[j + 1] == ccnt[j]) continue;  // empty column (cannot happen: every interval has samples)
            uint64_t h = 1469598103934665603ull;
            for (int64_t e = ccnt[j]; e < ccnt[j + 1]; ++e) {
                uint64_t bits;
                std::memcpy(&bits, &cval[e], 8);
                h = (h ^ (uint64_t)crow[e]) * 1099511628211ull;
                h = (h ^ bits) * 1099511628211ull;
            }
            auto& bk = buckets[h];
            bool dup = false;
            for (int32_t u : bk) {
                if (ccnt[u + 1] - ccnt[u] != ccnt[j + 1] - ccnt[j]) continue;
                bool same = true;
                for (int64_t e = 0; e < ccnt[j + 1] - ccnt[j] && same; ++e)
                    same = crow[ccnt[u] + e] == crow[ccnt[j] + e] &&
                           cval[ccnt[u] + e] == cval[ccnt[j] + e];
                if (same) {
                    dup = true;
                    break;
                }
            }
            if (!dup) {
                bk.push_back(j);
                uniq.push_back(j);
            }
        }
        std::sort(uniq.begin(), uniq.end());
    }
    const int32_t rd = (int32_t)uniq.size();
    co.r_dedup = rd;
    tick("zs+dedup");
    // AZ for the distinct columns
    const bool mixed = pl->opts.precision == MM_MIXED;
    DBuf<double> azd;
    DBuf<float> azf;
    if (mixed) MM_TRY(azf.alloc((size_t)rd * nv));
    else MM_TRY(azd.alloc((size_t)rd * nv));
    DBuf<double> zc, tmp;
    MM_TRY(zc.alloc(nv));
    MM_TRY(tmp.alloc(nv));
    DBuf<int32_t> drow;
    DBuf<double> dval;
    DBuf<int64_t> dptr;
    std::vector<int64_t> uptr(rd + 1, 0);
    std::vector<int32_t> urow;
    std::vector<double> uval;
    for (int32_t u = 0; u < rd; ++u) {
        const int32_t j = uniq[u];
        urow.insert(urow.end(), crow.begin() + ccnt[j], crow.begin() + ccnt[j + 1]);
        uval.insert(uval.end(), cval.begin() + ccnt[j], cval.begin() + ccnt[j + 1]);
        uptr[u + 1] = (int64_t)urow.size();
    }
    MM_TRY(drow.alloc(urow.size()));
    MM_TRY(dval.alloc(uval.size()));
    MM_TRY(dptr.alloc(rd + 1));
    MM_HIP(hipMemcpyAsync(drow.p, urow.data(), urow.size() * 4, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(dval.p, uval.data(), uval.size() * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(dptr.p, uptr.data(), (rd + 1) * 8, hipMemcpyHostToDevice, st));
    for (int32_t u = 0; u < rd; ++u) {
        MM_HIP(hipMemsetAsync(zc.p, 0, nv * 8, st));
        const int64_t cnt = uptr[u + 1] - uptr[u];
        hipLaunchKernelGGL(k_col_to_vec, dim3(grid_for(cnt)), dim3(256), 0, st,
                           drow.p + uptr[u], dval.p + uptr[u], cnt, (int)ns, zc.p);
        MM_HIP(hipGetLastError());
        if (mixed) {
            MM_TRY(apply_A32(pl, zc.p, tmp.p, nullptr));
            hipLaunchKernelGGL(k_to_f32, dim3(grid_for(nv)), dim3(256), 0, st, (const double*)tmp.p,
                               azf.p + (size_t)u * nv, nv);
            MM_HIP(hipGetLastError());
        } else {
            MM_TRY(apply_A64(pl, zc.p, azd.p + (size_t)u * nv, nullptr));
        }
    }
    tick("AZ");
    // E = Z^T (AZ) on the matrix cores
    const int32_t rp = (rd + 15) / 16 * 16;
    const int64_t npad = (n_obs + 3) / 4 * 4;
    DBuf<double> zd, azr, dE;
    MM_TRY(zd.alloc((size_t)npad * rp));
    MM_TRY(azr.alloc((size_t)npad * rp));
    MM_TRY(dE.alloc((size_t)rp * rp));
    MM_HIP(hipMemsetAsync(zd.p, 0, (size_t)npad * rp * 8, st));
    MM_HIP(hipMemsetAsync(azr.p, 0, (size_t)npad * rp * 8, st));
    hipLaunchKernelGGL(k_dense_z, dim3(64, rd), dim3(256), 0, st, dptr.p, drow.p, dval.p, rd, rp, zd.p);
    if (mixed)
        hipLaunchKernelGGL(k_az_rows<float>, dim3(grid_for(n_obs, 256, 4096), rd), dim3(256), 0, st,
                           azf.p, nv, n_obs, (int)ns, rd, rp, azr.p);
    else
        hipLaunchKernelGGL(k_az_rows<double>, dim3(grid_for(n_obs, 256, 4096), rd), dim3(256), 0,
                           st, azd.p, nv, n_obs, (int)ns, rd, rp, azr.p);
    MM_HIP(hipGetLastError());
    MM_TRY(gemm_tn_f64(st, zd.p, azr.p, npad, rp, rp, dE.p));
    std::vector<double> Ep((size_t)rp * rp);
    MM_HIP(hipMemcpy(Ep.data(), dE.p, Ep.size() * 8, hipMemcpyDeviceToHost));
    zd.release();
    azr.release();
    std::vector<double> E((size_t)rd * rd);
    for (int32_t a = 0; a < rd; ++a)
        for (int32_t b = 0; b < rd; ++b)
            E[(size_t)a * rd + b] = 0.5 * (Ep[(size_t)a * rp + b] + Ep[(size_t)b * rp + a]);
    tick("E");
    // independent subset and E^-1 on it
    std::vector<int> sel = pivoted_cholesky_select(E, rd, pl->opts.rank_tol);
    const int32_t k = (int32_t)sel.size();
    if (k == 0) {
        set_error("coarse matrix E is zero");
        return MM_ERR_RANK;
    }
    std::vector<double> Es((size_t)k * k), Einv;
    for (int32_t a = 0; a < k; ++a)
        for (int32_t b = 0; b < k; ++b) Es[(size_t)a * k + b] = E[(size_t)sel[a] * rd + sel[b]];
    if (!spd_inverse(Es, k, Einv)) {
        set_error("coarse matrix E not positive definite on the selected columns");
        return MM_ERR_RANK;
    }
    co.r_eff = k;
    co.E = Es;
    co.cols.resize(k);
    for (int32_t a = 0; a < k; ++a) co.cols[a] = uniq[sel[a]];
    MM_TRY(co.Einv.alloc((size_t)k * k));
    MM_HIP(hipMemcpyAsync(co.Einv.p, Einv.data(), Einv.size() * 8, hipMemcpyHostToDevice, st));
    // kept AZ columns: compact in place (sel is increasing and sel[a] >= a, so a source
    // column is never overwritten before it is copied)
    for (int32_t a = 0; a < k; ++a) {
        if (sel[a] == a) continue;
        if (mixed)
            MM_HIP(hipMemcpyAsync(azf.p + (size_t)a * nv, azf.p + (size_t)sel[a] * nv, nv * 4,
                                  hipMemcpyDeviceToDevice, st));
        else
            MM_HIP(hipMemcpyAsync(azd.p + (size_t)a * nv, azd.p + (size_t)sel[a] * nv, nv * 8,
                                  hipMemcpyDeviceToDevice, st));
    }
    if (mixed) co.AZ32.swap(azf);
    else co.AZ64.swap(azd);
    // kept columns by column: entry ranges into the distinct-column lists
    std::vector<int64_t> kb(k), ke(k);
    int64_t maxlen = 1;
    for (int32_t a = 0; a < k; ++a) {
        kb[a] = uptr[sel[a]];
        ke[a] = uptr[sel[a] + 1];
        maxlen = std::max(maxlen, ke[a] - kb[a]);
    }
    co.csc_row.swap(drow);
    co.csc_val.swap(dval);
    MM_TRY(co.csc_beg.alloc(k));
    MM_TRY(co.csc_end.alloc(k));
    MM_HIP(hipMemcpyAsync(co.csc_beg.p, kb.data(), k * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(co.csc_end.p, ke.data(), k * 8, hipMemcpyHostToDevice, st));
    // kept columns by pixel (CSR), filtered on the device from the full Z_S rows
    std::vector<int32_t> colmap(K, -1);
    for (int32_t a = 0; a < k; ++a) colmap[co.cols[a]] = a;
    DBuf<int32_t> dmap;
    DBuf<int64_t> kcnt;
    MM_TRY(dmap.alloc(K));
    MM_TRY(kcnt.alloc(n_obs));
    MM_HIP(hipMemcpyAsync(dmap.p, colmap.data(), K * 4, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_csr_filter, dim3(grid_for(n_obs)), dim3(256), 0, st, ptr.p, col.p, val.p,
                       n_obs, dmap.p, (const int64_t*)nullptr, kcnt.p, (int32_t*)nullptr,
                       (double*)nullptr);
    MM_HIP(hipGetLastError());
    MM_TRY(co.csr_ptr.alloc(n_obs + 1));
    MM_TRY(scan_exclusive_i64(kcnt.p, co.csr_ptr.p, n_obs, st));
    int64_t kn = 0;
    MM_HIP(hipMemcpy(&kn, co.csr_ptr.p + n_obs, 8, hipMemcpyDeviceToHost));
    MM_TRY(co.csr_col.alloc(std::max<int64_t>(1, kn)));
    MM_TRY(co.csr_val.alloc(std::max<int64_t>(1, kn)));
    hipLaunchKernelGGL(k_csr_filter, dim3(grid_for(n_obs)), dim3(256), 0, st, ptr.p, col.p, val.p,
                       n_obs, dmap.p, (const int64_t*)co.csr_ptr.p, (int64_t*)nullptr,
                       co.csr_col.p, co.csr_val.p);
    MM_HIP(hipGetLastError());
    MM_TRY(co.v.alloc(k));
    MM_TRY(co.w.alloc(k));
    co.zslices = (int)std::min<int64_t>(256, std::max<int64_t>(1, (maxlen + 511) / 512));
    MM_TRY(co.vpart.alloc((size_t)k * co.zslices));
    MM_HIP(hipStreamSynchronize(st));
    pl->has_coarse = true;
    return MM_OK;
}

int twolvl_apply(mm_plan_t pl, const double* r, double* z, const PcgCtl& ctl) {
    Coarse& co = pl->co;
    hipStream_t st = pl->stream;
    const int32_t k = co.r_eff;
    const int64_t nw = (int64_t)k * co.zslices;
    hipLaunchKernelGGL(k_ztr, dim3((nw + 3) / 4), dim3(256), 0, st, co.csc_beg.p, co.csc_end.p,
                       co.csc_row.p, co.csc_val.p, r, pl->n_s, k, co.zslices, co.vpart.p, ctl);
    hipLaunchKernelGGL(k_einv, dim3((k + 3) / 4), dim3(256), 0, st, co.Einv.p, co.vpart.p, k,
                       co.zslices, co.w.p, ctl.part ? ctl.sc : nullptr);
    const size_t shm = (size_t)k * sizeof(double);
    if (pl->n_s == 3) {
        if (co.AZ32.p)
            hipLaunchKernelGGL((k_2lvl<float, 3>), dim3(kVecBlocks), dim3(kVecThreads), shm, st, r,
                               z, pl->bj.p, co.AZ32.p, pl->n_obs, k, co.w.p, co.csr_ptr.p,
                               co.csr_col.p, co.csr_val.p, ctl);
        else
            hipLaunchKernelGGL((k_2lvl<double, 3>), dim3(kVecBlocks), dim3(kVecThreads), shm, st, r,
                               z, pl->bj.p, co.AZ64.p, pl->n_obs, k, co.w.p, co.csr_ptr.p,
                               co.csr_col.p, co.csr_val.p, ctl);
    } else {
        if (co.AZ32.p)
            hipLaunchKernelGGL((k_2lvl<float, 1>), dim3(kVecBlocks), dim3(kVecThreads), shm, st, r,
                               z, pl->bj.p, co.AZ32.p, pl->n_obs, k, co.w.p, co.csr_ptr.p,
                               co.csr_col.p, co.csr_val.p, ctl);
        else
            hipLaunchKernelGGL((k_2lvl<double, 1>), dim3(kVecBlocks), dim3(kVecThreads), shm, st, r,
                               z, pl->bj.p, co.AZ64.p, pl->n_obs, k, co.w.p, co.csr_ptr.p,
                               co.csr_col.p, co.csr_val.p, ctl);
    }
    MM_HIP(hipGetLastError());
    return MM_OK;
}

}  // namespace mm
