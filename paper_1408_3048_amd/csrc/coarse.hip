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
#include <mutex>
#include <unordered_map>

#include <hip/hip_fp16.h>

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

// interval of sample t, searched only when t leaves the last interval found ([lo, hi), kept
// by the caller): a pixel's samples ascend in t, so most lookups cost one comparison
struct IntervalCache {
    int64_t lo = 0, hi = 0;
    int32_t j = 0;
    __device__ __forceinline__ int32_t of(const int64_t* __restrict__ int_lo, int32_t n_int,
                                          int64_t t) {
        if (t < lo || t >= hi) {
            j = interval_of(int_lo, n_int, t);
            lo = int_lo[j];
            hi = j + 1 < n_int ? int_lo[j + 1] : INT64_MAX;
        }
        return j;
    }
};

// number of distinct intervals among each pixel's samples (ascending in t)
__global__ void k_zs_count(const int32_t* __restrict__ perm, const int64_t* __restrict__ seg,
                           const int32_t* __restrict__ hits, int64_t n_obs,
                           const int64_t* __restrict__ int_lo, int32_t n_int,
                           int64_t* __restrict__ nnz) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_obs;
         c += (int64_t)gridDim.x * blockDim.x) {
        int64_t cnt = 0;
        int32_t last = -1;
        IntervalCache ic;
        for (int64_t i = seg[c]; i < seg[c] + hits[c]; ++i) {
            const int32_t j = ic.of(int_lo, n_int, perm[i]);
            if (j != last) {
                ++cnt;
                last = j;
            }
        }
        nnz[c] = cnt;
    }
}

__global__ void k_zs_fill(const int32_t* __restrict__ perm, const int64_t* __restrict__ seg,
                          const int32_t* __restrict__ hits, int64_t n_obs,
                          const int64_t* __restrict__ int_lo, int32_t n_int,
                          const int64_t* __restrict__ ptr, int32_t* __restrict__ col,
                          double* __restrict__ val) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_obs;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = hits[c];
        int64_t o = ptr[c];
        int32_t last = -1;
        int64_t run = 0;
        IntervalCache ic;
        for (int64_t i = seg[c]; i < seg[c] + s; ++i) {
            const int32_t j = ic.of(int_lo, n_int, perm[i]);
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


// entry -> pixel of the Z_S rows (CSR) and the identity permutation
__global__ void k_expand_rows(const int64_t* __restrict__ ptr, int64_t n_obs,
                              int32_t* __restrict__ rowid, int32_t* __restrict__ eidx) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_obs;
         p += (int64_t)gridDim.x * blockDim.x)
        for (int64_t e = ptr[p]; e < ptr[p + 1]; ++e) {
            rowid[e] = (int32_t)p;
            eidx[e] = (int32_t)e;
        }
}

// Z_S by column (CSC) from the entries stably sorted by column: rows ascend within a
// column; [cbeg[j], cend[j]) are column j's entries (every interval has samples, so no
// column is empty)
__global__ void k_csc_fill(const int32_t* __restrict__ skey, const int32_t* __restrict__ sidx,
                           int64_t total, const int32_t* __restrict__ rowid,
                           const double* __restrict__ val, int32_t* __restrict__ crow,
                           double* __restrict__ cval, int64_t* __restrict__ cbeg,
                           int64_t* __restrict__ cend) {
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < total;
         d += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = sidx[d], k = skey[d];
        crow[d] = rowid[e];
        cval[d] = val[e];
        if (d == 0 || skey[d - 1] != k) cbeg[k] = d;
        if (d == total - 1 || skey[d + 1] != k) cend[k] = d + 1;
    }
}

// the SplitMix64 finaliser (Steele, Lea & Flood 2014) as a 64-bit mixing function
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// order-independent hash of every column: wrapping sum over its entries of
// mix(mix(row) ^ bits(value)); equal columns have equal hashes
__global__ __launch_bounds__(256) void k_col_hash(const int64_t* __restrict__ cbeg,
                                                  const int64_t* __restrict__ cend,
                                                  const int32_t* __restrict__ crow,
                                                  const double* __restrict__ cval,
                                                  unsigned long long* __restrict__ hash) {
    __shared__ unsigned long long red[256];
    const int j = blockIdx.x;
    unsigned long long h = 0;
    for (int64_t e = cbeg[j] + threadIdx.x; e < cend[j]; e += 256)
        h += mix64(mix64((uint64_t)crow[e]) ^ (uint64_t)__double_as_longlong(cval[e]));
    red[threadIdx.x] = h;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) hash[j] = red[0];
}

// neq[i] = 1 unless columns ca[i] and cb[i] (same entry count) hold identical entries
__global__ __launch_bounds__(256) void k_cols_equal(const int32_t* __restrict__ ca,
                                                    const int32_t* __restrict__ cb,
                                                    const int64_t* __restrict__ cbeg,
                                                    const int64_t* __restrict__ cend,
                                                    const int32_t* __restrict__ crow,
                                                    const double* __restrict__ cval,
                                                    int* __restrict__ neq) {
    const int i = blockIdx.x;
    const int64_t a0 = cbeg[ca[i]], b0 = cbeg[cb[i]], n = cend[ca[i]] - a0;
    for (int64_t e = threadIdx.x; e < n; e += 256)
        if (crow[a0 + e] != crow[b0 + e] ||
            __double_as_longlong(cval[a0 + e]) != __double_as_longlong(cval[b0 + e]))
            neq[i] = 1;
}

// on[k * K + j] = 1 when layer k's column of interval j's problem has a pixel hit in
// interval j, i.e. when P applied to that column does not vanish on the whole interval
// (an entry of Z_S^T Z_S): row p of Z_S lists the intervals that hit pixel p, and each
// pair of its entries marks one (layer, interval) pair.  A row longer than kPairCap marks
// every layer for its intervals instead (more flags than needed, never fewer).
constexpr int kPairCap = 64;
__global__ void k_az_int_flags(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                               int64_t n_obs, const int32_t* __restrict__ layer, int32_t K,
                               int32_t n_layers, uint8_t* __restrict__ on) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_obs;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a0 = ptr[p], a1 = ptr[p + 1];
        if (a1 - a0 <= kPairCap) {
            for (int64_t a = a0; a < a1; ++a) {
                uint8_t* row = on + (int64_t)layer[col[a]] * K;
                for (int64_t c = a0; c < a1; ++c) {
                    const int32_t j = col[c];
                    if (!row[j]) row[j] = 1;
                }
            }
        } else {
            for (int64_t c = a0; c < a1; ++c) {
                const int32_t j = col[c];
                for (int32_t k = 0; k < n_layers; ++k)
                    if (!on[(int64_t)k * K + j]) on[(int64_t)k * K + j] = 1;
            }
        }
    }
}

// the entries of the columns ucol[0..gridDim.y) into zeroed maps of their I rows (the Q
// and U rows of Z_S are zero), column y into map lay[y] - k0 (x + (lay[y] - k0) xstride)
__global__ void k_cols_to_maps(const int32_t* __restrict__ ucol, const int32_t* __restrict__ lay,
                               int32_t k0, int64_t xstride, const int64_t* __restrict__ ub,
                               const int64_t* __restrict__ ue, const int32_t* __restrict__ rows,
                               const double* __restrict__ vals, double* __restrict__ xm) {
    const int32_t u = ucol[blockIdx.y];
    double* x = xm + (int64_t)(lay[blockIdx.y] - k0) * xstride;
    for (int64_t i = ub[u] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ue[u];
         i += (int64_t)gridDim.x * blockDim.x)
        x[rows[i]] = vals[i];
}

// copy problem lp[y]'s slice of the map vector y into column `col` of its AZ block
template <typename TA>
__global__ void k_store_az(const int32_t* __restrict__ lp, const double* __restrict__ y,
                           const int64_t* __restrict__ ooff, int ns,
                           const int64_t* __restrict__ blk_off, int32_t col,
                           TA* __restrict__ az) {
    const int32_t b = lp[blockIdx.y];
    const int64_t v0 = ooff[b] * ns, n = (ooff[b + 1] - ooff[b]) * ns;
    TA* dst = az + blk_off[b] + (int64_t)col * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (TA)y[v0 + i];
}

// copy n[c] values from src + so[c] to dst + d_o[c] for every column c = blockIdx.y; with
// mx != nullptr also the column's largest |value| into mx[c] as FP32 bits (non-negative
// floats order like their bit patterns; mx starts at zero): one atomic max per block
template <typename TA>
__global__ __launch_bounds__(256) void k_copy_cols(const TA* __restrict__ src,
                                                   TA* __restrict__ dst,
                                                   const int64_t* __restrict__ so,
                                                   const int64_t* __restrict__ d_o,
                                                   const int64_t* __restrict__ n,
                                                   unsigned* __restrict__ mx) {
    __shared__ float red[4];
    const int32_t c = blockIdx.y;
    const int64_t a = so[c], d = d_o[c], m = n[c];
    float am = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * 256) {
        const TA v = src[a + i];
        dst[d + i] = v;
        am = fmaxf(am, fabsf((float)v));
    }
    if (!mx) return;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) am = fmaxf(am, __shfl_xor(am, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = am;
    __syncthreads();
    if (threadIdx.x == 0) {
        am = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        if (am > 0.0f) atomicMax(mx + c, __float_as_uint(am));
    }
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

// ---------------------------------------------------------------- FP64 MFMA: C = A^T B
// A: row-major [n][ra], B: row-major [n][rb] (n a multiple of 4, ra and rb multiples of
// 16), C partials [ksplit][ra][rb].  One wave per 16x16 output tile and pixel slab;
// v_mfma_f64_16x16x4f64: lane l supplies A(i = l%16, k = l/16) and B(k = l/16, j = l%16)
// and holds D(i = l/16 + 4 v, j = l%16) in accumulator register v (v = 0..3).
typedef double dbl4 __attribute__((ext_vector_type(4)));

// one wave's share of C = A^T B: output tile (ta, tb) of the slab ks of the n dimension
__device__ __forceinline__ void gemm_tn_wave(const double* __restrict__ A,
                                             const double* __restrict__ B, int64_t n, int32_t ra,
                                             int32_t rb, int32_t ksplit, int64_t wid,
                                             double* __restrict__ part) {
    const int lane = threadIdx.x & 63;
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
    // eight steps' loads in flight before their products (one step at a time, every step
    // waited for the memory latency); the products keep the order of q
    int64_t q = q0;
    for (; q + 8 <= q1; q += 8) {
        double a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t row = 4 * (q + u) + k;
            a[u] = Ap[row * ra];
            b[u] = Bp[row * rb];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
    }
    for (; q < q1; ++q) {
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

__global__ __launch_bounds__(256) void k_gemm_tn_f64(const double* __restrict__ A,
                                                     const double* __restrict__ B, int64_t n,
                                                     int32_t ra, int32_t rb, int32_t ksplit,
                                                     double* __restrict__ part) {
    gemm_tn_wave(A, B, n, ra, rb, ksplit, (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6), part);
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

// Gram products E_b = Z_b^T (AZ)_b of several problems in one launch: problem b's row
// blocks start at a_off in A and B (row-major [n][rp], rp a multiple of 16), its partials
// at part_off, its E at c_off; its waves are [woff[b], woff[b+1]) and the slab split
// ksplit is the one the single-problem product takes, so every E_b is bitwise the same.
struct GramDesc {
    int64_t a_off, n, part_off, c_off;
    int32_t rp, ksplit;
};

__device__ __forceinline__ int find_off(const int64_t* __restrict__ off, int nb, int64_t v) {
    int a = 0, b = nb - 1;
    while (a < b) {
        const int m = (a + b + 1) >> 1;
        if (off[m] <= v) a = m; else b = m - 1;
    }
    return a;
}

__global__ __launch_bounds__(256) void k_gemm_tn_f64_batch(const double* __restrict__ A,
                                                           const double* __restrict__ B,
                                                           const GramDesc* __restrict__ d,
                                                           const int64_t* __restrict__ woff,
                                                           int nb, double* __restrict__ part) {
    const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wid >= woff[nb]) return;
    const int b = find_off(woff, nb, wid);
    const GramDesc g = d[b];
    gemm_tn_wave(A + g.a_off, B + g.a_off, g.n, g.rp, g.rp, g.ksplit, wid - woff[b],
                 part + g.part_off);
}

// E entries of the problems: [eoff[b], eoff[b+1]) is problem b's rp x rp block
__global__ void k_sum_parts_batch(const double* __restrict__ part, const GramDesc* __restrict__ d,
                                  const int64_t* __restrict__ eoff, int nb,
                                  double* __restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < eoff[nb];
         e += (int64_t)gridDim.x * blockDim.x) {
        const int b = find_off(eoff, nb, e);
        const GramDesc g = d[b];
        const int64_t m = (int64_t)g.rp * g.rp, loc = e - eoff[b];
        double s = 0.0;
        // in slab order; eight loads in flight
#pragma unroll 8
        for (int32_t k = 0; k < g.ksplit; ++k) s += part[g.part_off + (int64_t)k * m + loc];
        out[g.c_off + loc] = s;
    }
}

// dense I rows of the distinct Z_S columns of problems b0 + z (z = blockIdx.z) in the row
// blocks of the Gram products (row p - ooff[b], column c)
__global__ void k_dense_z_batch(const int64_t* __restrict__ cb, const int64_t* __restrict__ ce,
                                const int32_t* __restrict__ rows, const double* __restrict__ vals,
                                const int32_t* __restrict__ ud_off,
                                const int64_t* __restrict__ ooff, const GramDesc* __restrict__ d,
                                int b0, double* __restrict__ zd) {
    const int b = b0 + (int)blockIdx.z;
    const int32_t c = blockIdx.y;
    if (c >= ud_off[b + 1] - ud_off[b]) return;
    const GramDesc g = d[blockIdx.z];
    const int32_t u = ud_off[b] + c;
    for (int64_t i = cb[u] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ce[u];
         i += (int64_t)gridDim.x * blockDim.x)
        zd[g.a_off + ((int64_t)rows[i] - ooff[b]) * g.rp + c] = vals[i];
}

// I rows of problem b0 + z's AZ block (column-major [r_b][n_vec_b] at az_off[b]) in the row
// blocks of the Gram products.  A block moves tiles of 64 pixels x 64 columns (columns
// 64 blockIdx.y + ...) through LDS, so that both the column reads and the row writes are
// coalesced.
template <typename TA>
__global__ __launch_bounds__(256) void k_az_rows_batch(const TA* __restrict__ az,
                                                       const int64_t* __restrict__ az_off,
                                                       const int32_t* __restrict__ ud_off,
                                                       const int64_t* __restrict__ ooff, int ns,
                                                       const GramDesc* __restrict__ d, int b0,
                                                       double* __restrict__ out) {
    __shared__ double tile[64][65];
    const int b = b0 + (int)blockIdx.z;
    const int32_t rb = ud_off[b + 1] - ud_off[b];
    const int32_t c0 = (int32_t)blockIdx.y * 64;
    if (c0 >= rb) return;
    const int32_t nc = rb - c0 < 64 ? rb - c0 : 64;
    const GramDesc g = d[blockIdx.z];
    const int64_t nob = ooff[b + 1] - ooff[b], n_vec = nob * ns;
    const TA* src = az + az_off[b] + (int64_t)c0 * n_vec;
    const int lo = threadIdx.x & 63, hi = threadIdx.x >> 6;
    for (int64_t p0 = (int64_t)blockIdx.x * 64; p0 < nob; p0 += (int64_t)gridDim.x * 64) {
        const int64_t p = p0 + lo;
        for (int c = hi; c < nc; c += 4)
            if (p < nob) tile[c][lo] = (double)src[(int64_t)c * n_vec + p * ns];
        __syncthreads();
        for (int i = hi; i < 64; i += 4)
            if (p0 + i < nob && lo < nc) out[g.a_off + (p0 + i) * g.rp + c0 + lo] = tile[lo][i];
        __syncthreads();
    }
}

// v = Z^T r: kept column c owns the slices [vslice[c], vslice[c+1]) of 512 entries
// (slice_col: the column of every slice); one wave per slice writes its partial sum to
// vpart[slice].  A lane's entries a + lane + 64 k are loaded together (from entry a where
// past the slice end: guarded loads would be waited for one by one) and summed in order.
__global__ __launch_bounds__(256) void k_ztr(const int64_t* __restrict__ cbeg,
                                             const int64_t* __restrict__ cend,
                                             const int32_t* __restrict__ rows,
                                             const double* __restrict__ vals,
                                             const double* __restrict__ r, int ns,
                                             const int32_t* __restrict__ vslice,
                                             const int32_t* __restrict__ slice_col,
                                             int64_t n_slices,
                                             const int32_t* __restrict__ col_prob,
                                             double* __restrict__ vpart,
                                             const int* __restrict__ mask) {
    constexpr int K = 512 / 64;
    const int lane = threadIdx.x & 63;
    const int64_t wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wv >= n_slices) return;
    const int32_t c = slice_col[wv];
    if (mask && !mask[col_prob[c]]) return;
    const int64_t a = cbeg[c] + (wv - vslice[c]) * 512;
    const int64_t b = a + 512 < cend[c] ? a + 512 : cend[c];
    if (a >= b) {  // empty column
        if (lane == 0) vpart[wv] = 0.0;
        return;
    }
    int32_t rw[K];
    double vv[K], rr[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t e = a + lane + 64 * k;
        const int64_t ec = e < b ? e : a;
        rw[k] = rows[ec];
        vv[k] = vals[ec];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) rr[k] = r[(int64_t)rw[k] * ns];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (a + lane + 64 * k < b) s += vv[k] * rr[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) vpart[wv] = s;
}

// w = E^-1 v per problem, with v[c] = sum of the slice partials of column c (one wave per
// kept column a, summing over the columns of a's problem)
__global__ __launch_bounds__(256) void k_einv(const double* __restrict__ Einv,
                                              const int64_t* __restrict__ einv_off,
                                              const int32_t* __restrict__ col_off,
                                              const int32_t* __restrict__ col_prob,
                                              const double* __restrict__ vpart,
                                              const int32_t* __restrict__ vslice, int32_t rk,
                                              double* __restrict__ w,
                                              const int* __restrict__ mask) {
    const int lane = threadIdx.x & 63;
    const int32_t a = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (a >= rk) return;
    const int32_t b = col_prob[a];
    if (mask && !mask[b]) return;
    const int32_t c0 = col_off[b], r = col_off[b + 1] - c0;
    const double* E = Einv + einv_off[b] + (int64_t)(a - c0) * r;
    double s = 0.0;
    for (int32_t q = lane; q < r; q += 64) {
        const int32_t c = c0 + q;
        double v = 0.0;
        for (int32_t t = vslice[c]; t < vslice[c + 1]; ++t) v += vpart[t];
        s += E[q] * v;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) w[a] = s;
}

// FP16 copy of the kept AZ columns for the A-DEF1 apply.  Column a (blockIdx.y) as
// entry / scale[a], scale[a] = 2^(e - 14) for the column's largest |entry| mx[a] < 2^e (1 for
// a zero column): scaled entries stay below 2^14, far from FP16's 65504 limit, the
// power-of-two scaling is exact, and every entry is rounded once.  Entries [len[a], ld[a])
// of the column (the pixel-pair padding) are zero.
__global__ __launch_bounds__(256) void k_az_to_half(const float* __restrict__ az,
                                                    const int64_t* __restrict__ src_off,
                                                    const int64_t* __restrict__ len,
                                                    const int64_t* __restrict__ dst_off,
                                                    const int64_t* __restrict__ ld,
                                                    const unsigned* __restrict__ mx,
                                                    double* __restrict__ scale,
                                                    uint16_t* __restrict__ out) {
    const int a = blockIdx.y;
    const float* col = az + src_off[a];
    uint16_t* dst = out + dst_off[a];
    const float m = __uint_as_float(mx[a]);
    int e = 0;
    if (m > 0.0f) (void)frexpf(m, &e);  // m < 2^e
    const float inv = m > 0.0f ? ldexpf(1.0f, 14 - e) : 1.0f;  // a power of two: exact
    if (blockIdx.x == 0 && threadIdx.x == 0) scale[a] = m > 0.0f ? ldexp(1.0, e - 14) : 1.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < ld[a];
         i += (int64_t)gridDim.x * 256) {
        const float v = i < len[a] ? col[i] * inv : 0.0f;
        dst[i] = __half_as_ushort(__float2half_rn(v));
    }
}

// z = M_BD (r - AZ w) + Z w per pixel of every masked problem, partials of r^T z.
// DZ: Z is dense (Z_D blocks laid out like AZ, every Stokes row); else the sparse Z_S rows
// (I rows only) in CSR form.
template <typename TA, int NS, bool DZ>
__global__ __launch_bounds__(kVecThreads) void k_2lvl(
    const double* __restrict__ r, double* __restrict__ z, const double* __restrict__ bj,
    const TA* __restrict__ az, const int64_t* __restrict__ az_off,
    const int32_t* __restrict__ col_off, const double* __restrict__ w,
    const int64_t* __restrict__ zptr, const int32_t* __restrict__ zcol,
    const double* __restrict__ zval, const TA* __restrict__ zd, PcgCtl ctl) {
    __shared__ double red[kVecThreads];
    extern __shared__ double sw[];
    const VecBlock vb = vec_block(ctl, NS, false);
    if (ctl.mask && !ctl.mask[vb.b]) return;
    const int32_t c0 = col_off[vb.b], rk = col_off[vb.b + 1] - c0;
    for (int c = threadIdx.x; c < rk; c += kVecThreads) sw[c] = w[c0 + c];
    __syncthreads();
    const int64_t nv = vb.n * NS;
    const TA* azb = az + az_off[vb.b];
    double acc = 0.0;
    // sparse Z: a thread's pixels q and q + stride go through the column loop together
    // (twice the loads in flight per column); a missing second pixel reads the first again
    // and is not stored.  Every per-pixel sum and the order of acc are those of one pixel
    // at a time.  Dense Z already streams two blocks per column and takes one pixel.
    constexpr int PX = DZ ? 1 : 2;
    for (int64_t q = (int64_t)vb.k * kVecThreads + threadIdx.x; q < vb.n;
         q += PX * vb.stride) {
        const int64_t q1 = PX == 2 && q + vb.stride < vb.n ? q + vb.stride : q;
        const int64_t qq[2] = {q, q1};
        double u[PX][NS], zw[PX][NS];
#pragma unroll
        for (int j = 0; j < PX; ++j)
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                u[j][s] = r[(vb.base + qq[j]) * NS + s];
                zw[j][s] = 0.0;
            }
        // one column at a time: batches of columns with their loads issued together were
        // slower here (more pages open per wave), unlike the FP16 layout of k_2lvl16
        for (int32_t c = 0; c < rk; ++c) {
            const double wc = sw[c];
            const TA* col = azb + (int64_t)c * nv;
#pragma unroll
            for (int j = 0; j < PX; ++j)
#pragma unroll
                for (int s = 0; s < NS; ++s) u[j][s] -= (double)col[qq[j] * NS + s] * wc;
            if constexpr (DZ) {
                const TA* zc = zd + az_off[vb.b] + (int64_t)c * nv;
#pragma unroll
                for (int j = 0; j < PX; ++j)
#pragma unroll
                    for (int s = 0; s < NS; ++s) zw[j][s] += (double)zc[qq[j] * NS + s] * wc;
            }
        }
#pragma unroll
        for (int j = 0; j < PX; ++j) {
            if (j == 1 && q1 == q) break;
            const int64_t p = vb.base + qq[j];
            double zz[NS];
            if constexpr (NS == 1) {
                zz[0] = bj[p] * u[j][0];
            } else {
                const double* m = bj + 6 * p;
                zz[0] = m[0] * u[j][0] + m[1] * u[j][1] + m[2] * u[j][2];
                zz[1] = m[1] * u[j][0] + m[3] * u[j][1] + m[4] * u[j][2];
                zz[2] = m[2] * u[j][0] + m[4] * u[j][1] + m[5] * u[j][2];
            }
            if constexpr (DZ) {
#pragma unroll
                for (int s = 0; s < NS; ++s) zz[s] += zw[j][s];
            } else {
                double zs = zw[j][0];
                for (int64_t e = zptr[p]; e < zptr[p + 1]; ++e) zs += zval[e] * sw[zcol[e] - c0];
                zz[0] += zs;
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                z[p * NS + s] = zz[s];
                acc += r[p * NS + s] * zz[s];
            }
        }
    }
    if (ctl.part) write_partial_at(acc, slot_part(ctl, kSlotRZ, vb.b), vb.k, red);
}

// k_2lvl for sparse Z_S with AZ in FP16 (the az_fp16 layout): z = M_BD (r - AZ w) + Z w.
// A thread takes two adjacent pixels, whose 2 n_s FP16 entries of a column are one aligned
// 4- or 12-byte load; the column scales are folded into w (exact: powers of two).  Per
// pixel the sums run over the columns in order, in FP64, as in k_2lvl.
template <int NS>
__global__ __launch_bounds__(kVecThreads) void k_2lvl16(
    const double* __restrict__ r, double* __restrict__ z, const double* __restrict__ bj,
    const uint16_t* __restrict__ az16, const int64_t* __restrict__ az16_off,
    const double* __restrict__ az_scale, const int32_t* __restrict__ col_off,
    const double* __restrict__ w, const int64_t* __restrict__ zptr,
    const int32_t* __restrict__ zcol, const double* __restrict__ zval, PcgCtl ctl) {
    __shared__ double red[kVecThreads];
    extern __shared__ double sw[];  // [2 r_max]: w, and w times the column scales
    const VecBlock vb = vec_block(ctl, NS, false);
    if (ctl.mask && !ctl.mask[vb.b]) return;
    const int32_t c0 = col_off[vb.b], rk = col_off[vb.b + 1] - c0;
    double* swa = sw + rk;
    for (int c = threadIdx.x; c < rk; c += kVecThreads) {
        const double wc = w[c0 + c];
        sw[c] = wc;
        swa[c] = wc * az_scale[c0 + c];
    }
    __syncthreads();
    const int64_t ld = rk > 0 ? (az16_off[vb.b + 1] - az16_off[vb.b]) / rk : 0;
    const uint16_t* azb = az16 + az16_off[vb.b];
    const int64_t npair = (vb.n + 1) / 2;
    double acc = 0.0;
    for (int64_t jp = (int64_t)vb.k * kVecThreads + threadIdx.x; jp < npair; jp += vb.stride) {
        const int64_t q0 = 2 * jp;
        const bool two = q0 + 1 < vb.n;
        const int64_t qq[2] = {q0, two ? q0 + 1 : q0};
        // r, the M_BD blocks and the Z_S row ranges of both pixels are loaded before the
        // column loop, so that their latency overlaps it
        double u[2][NS], r0[2][NS], bm[2][NS == 3 ? 6 : 1];
        int64_t e0[2], e1[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t p = vb.base + qq[j];
#pragma unroll
            for (int s = 0; s < NS; ++s) u[j][s] = r0[j][s] = r[p * NS + s];
#pragma unroll
            for (int t = 0; t < (NS == 3 ? 6 : 1); ++t) bm[j][t] = bj[(NS == 3 ? 6 : 1) * p + t];
            e0[j] = zptr[p];
            e1[j] = zptr[p + 1];
        }
        const uint16_t* pe = azb + 2 * NS * jp;
        // the 2 NS FP16 entries of column c as NS 32-bit words
        auto load_col = [&](int32_t c, uint32_t* wd) {
            if constexpr (NS == 3) {
                const uint3 raw = *reinterpret_cast<const uint3*>(pe + (int64_t)c * ld);
                wd[0] = raw.x;
                wd[1] = raw.y;
                wd[2] = raw.z;
            } else {
                wd[0] = *reinterpret_cast<const uint32_t*>(pe + (int64_t)c * ld);
            }
        };
        auto add_col = [&](double wc, const uint32_t* wd) {
            float f[2 * NS];
#pragma unroll
            for (int h = 0; h < NS; ++h) {
                const float2 v = __half22float2(__builtin_bit_cast(__half2, wd[h]));
                f[2 * h] = v.x;
                f[2 * h + 1] = v.y;
            }
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int s = 0; s < NS; ++s) u[j][s] -= (double)f[NS * j + s] * wc;
        };
        // columns in batches of CB: the batch's loads are issued together, then added in
        // column order
        constexpr int CB = 8;
        int32_t c = 0;
        for (; c + CB <= rk; c += CB) {
            uint32_t wd[CB][NS];
#pragma unroll
            for (int t = 0; t < CB; ++t) load_col(c + t, wd[t]);
#pragma unroll
            for (int t = 0; t < CB; ++t) add_col(swa[c + t], wd[t]);
        }
        for (; c < rk; ++c) {
            uint32_t wd[NS];
            load_col(c, wd);
            add_col(swa[c], wd);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (j == 1 && !two) break;
            const int64_t p = vb.base + qq[j];
            double zz[NS];
            if constexpr (NS == 1) {
                zz[0] = bm[j][0] * u[j][0];
            } else {
                const double* m = bm[j];
                zz[0] = m[0] * u[j][0] + m[1] * u[j][1] + m[2] * u[j][2];
                zz[1] = m[1] * u[j][0] + m[3] * u[j][1] + m[4] * u[j][2];
                zz[2] = m[2] * u[j][0] + m[4] * u[j][1] + m[5] * u[j][2];
            }
            double zs = 0.0;
            for (int64_t e = e0[j]; e < e1[j]; ++e) zs += zval[e] * sw[zcol[e] - c0];
            zz[0] += zs;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                z[p * NS + s] = zz[s];
                acc += r0[j][s] * zz[s];
            }
        }
    }
    if (ctl.part) write_partial_at(acc, slot_part(ctl, kSlotRZ, vb.b), vb.k, red);
}

// ---------------------------------------------------------------- dense Z_D
// Z_D columns [c0, c0 + 16) of one problem (c0 = 16 blockIdx.y): out[c][e] =
// sum_k basis[k][v0 + e] G[k][c], k < m, for its n vector entries e
template <typename TA>
__global__ __launch_bounds__(256) void k_ritz_vectors(const double* __restrict__ basis,
                                                      int64_t stride, int64_t v0, int64_t n,
                                                      int32_t m, const double* __restrict__ G,
                                                      int32_t r, TA* __restrict__ out) {
    const int32_t c0 = blockIdx.y * 16;
    const int32_t nc = min(16, r - c0);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        double acc[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = 0.0;
        const double* bp = basis + v0 + e;
        for (int32_t k = 0; k < m; ++k) {
            const double v = bp[(int64_t)k * stride];
            const double* g = G + (int64_t)k * r + c0;
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (j < nc) acc[j] = fma(v, g[j], acc[j]);
        }
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (j < nc) out[(int64_t)(c0 + j) * n + e] = (TA)acc[j];
    }
}

__global__ void k_f32_to_f64(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (double)a[i];
}

// column `col` of the dense block of problem lp[y] into its slice of a zeroed map vector
template <typename TA>
__global__ void k_zd_to_vec(const int32_t* __restrict__ lp, const TA* __restrict__ zd,
                            const int64_t* __restrict__ ooff, int ns,
                            const int64_t* __restrict__ blk_off, int32_t col,
                            double* __restrict__ out) {
    const int32_t b = lp[blockIdx.y];
    const int64_t v0 = ooff[b] * ns, n = (ooff[b + 1] - ooff[b]) * ns;
    const TA* src = zd + blk_off[b] + (int64_t)col * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[v0 + i] = (double)src[i];
}

// column-major [r][n] block -> row-major [npad][rp] FP64 (rows past n and columns past r
// are left as they are: zeroed by the caller); tiles of 64 entries x 64 columns (columns
// 64 blockIdx.y + ...) go through LDS, so that reads and writes are both coalesced
template <typename TA>
__global__ __launch_bounds__(256) void k_cols_to_rows(const TA* __restrict__ src, int64_t n,
                                                      int32_t r, int32_t rp,
                                                      double* __restrict__ dst) {
    __shared__ double tile[64][65];
    const int32_t c0 = (int32_t)blockIdx.y * 64;
    if (c0 >= r) return;
    const int32_t nc = r - c0 < 64 ? r - c0 : 64;
    const TA* s = src + (int64_t)c0 * n;
    const int lo = threadIdx.x & 63, hi = threadIdx.x >> 6;
    for (int64_t e0 = (int64_t)blockIdx.x * 64; e0 < n; e0 += (int64_t)gridDim.x * 64) {
        const int64_t e = e0 + lo;
        for (int c = hi; c < nc; c += 4)
            if (e < n) tile[c][lo] = (double)s[(int64_t)c * n + e];
        __syncthreads();
        for (int i = hi; i < 64; i += 4)
            if (e0 + i < n && lo < nc) dst[(e0 + i) * rp + c0 + lo] = tile[lo][i];
        __syncthreads();
    }
}

// v = Z_D^T r, first stage: block g takes the chunk [ch*kZtChunk, +kZtChunk) of its
// problem's vector (ch = g - ch_off[b]) and writes the chunk's partial sum of every kept
// column i of the problem to cpart[i * n_ch + g] (r and every column read once,
// coalesced; fixed reduction order)
constexpr int kZtChunk = 1024;
constexpr int kZtCols = 32;  // columns per block of the chunk partials (grid y)
template <typename TA>
__global__ __launch_bounds__(256) void k_ztr_chunks(const TA* __restrict__ zd,
                                                    const int64_t* __restrict__ blk_off,
                                                    const int32_t* __restrict__ col_off,
                                                    const int64_t* __restrict__ ch_off, int B,
                                                    const int64_t* __restrict__ ooff, int ns,
                                                    const double* __restrict__ r,
                                                    int64_t n_ch, double* __restrict__ cpart,
                                                    const int* __restrict__ mask) {
    __shared__ double red[4 * kZtCols];
    const int64_t g = blockIdx.x;
    int lo = 0, hi = B - 1;  // problem: largest b with ch_off[b] <= g
    while (lo < hi) {
        const int m = (lo + hi + 1) >> 1;
        if (ch_off[m] <= g) lo = m; else hi = m - 1;
    }
    const int b = lo;
    if (mask && !mask[b]) return;
    const int32_t rb = col_off[b + 1] - col_off[b];
    const int32_t cg0 = (int32_t)blockIdx.y * kZtCols;  // this block's group of columns
    if (cg0 >= rb) return;
    const int32_t cg1 = cg0 + kZtCols < rb ? cg0 + kZtCols : rb;
    const int64_t v0 = ooff[b] * ns, n = (ooff[b + 1] - ooff[b]) * ns;
    const int64_t e0 = (g - ch_off[b]) * kZtChunk;
    constexpr int E = kZtChunk / 256;
    // entries past the vector end read its last entry against r = 0, and columns past
    // the last read the last column (their sums are not stored), so that the loads carry
    // no branches and the eight columns of a step are in flight together
    double rv[E];
    int64_t ee[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int64_t e = e0 + j * 256 + threadIdx.x;
        rv[j] = e < n ? r[v0 + e] : 0.0;
        ee[j] = e < n ? e : n - 1;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const TA* zb = zd + blk_off[b];
    for (int32_t c0 = cg0; c0 < cg1; c0 += 8) {
        double acc[8];
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
            const TA* zc = zb + (int64_t)min(c0 + cc, rb - 1) * n;
            double a = 0.0;
#pragma unroll
            for (int j = 0; j < E; ++j) a = fma((double)zc[ee[j]], rv[j], a);
            acc[cc] = a;
        }
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
            double a = acc[cc];
            for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
            if (lane == 0 && c0 + cc < cg1) red[wv * kZtCols + c0 + cc - cg0] = a;
        }
    }
    __syncthreads();
    for (int32_t c = threadIdx.x; c < cg1 - cg0; c += 256)
        cpart[(cg0 + c) * n_ch + g] =
            ((red[c] + red[kZtCols + c]) + red[2 * kZtCols + c]) + red[3 * kZtCols + c];
}

// sum of n_ch-strided chunk partials ci[g0..g1) over the wave (four independent load
// streams per lane, fixed order)
__device__ __forceinline__ double wave_chunk_sum(const double* __restrict__ ci, int64_t g0,
                                                 int64_t g1, int lane) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t g = g0 + lane;
    for (; g + 192 < g1; g += 256) {
        s0 += ci[g];
        s1 += ci[g + 64];
        s2 += ci[g + 128];
        s3 += ci[g + 192];
    }
    for (; g < g1; g += 64) s0 += ci[g];
    double s = (s0 + s1) + (s2 + s3);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    return s;
}

// v_a = the sum of the chunk partials of column a of Z^T r (Z_D: cz), or of its slice
// partials (Z_S: vpart, vslice), minus that of (AZ)^T y (caz) where given, for every kept
// column a of the masked problems: one wave per column over all problems
__global__ __launch_bounds__(256) void k_coarse_sums(
    const double* __restrict__ cz, const double* __restrict__ vpart,
    const int32_t* __restrict__ vslice, const double* __restrict__ caz,
    const int64_t* __restrict__ ch_off, const int32_t* __restrict__ col_off,
    const int32_t* __restrict__ col_prob, int64_t n_ch, int32_t r_eff,
    double* __restrict__ v, const int* __restrict__ mask) {
    const int lane = threadIdx.x & 63;
    const int32_t a = (int32_t)blockIdx.x * 4 + (int32_t)(threadIdx.x >> 6);
    if (a >= r_eff) return;
    const int b = col_prob[a];
    if (mask && !mask[b]) return;
    const int32_t i = a - col_off[b];
    const int64_t g0 = ch_off[b], g1 = ch_off[b + 1];
    double s;
    if (cz) {
        s = wave_chunk_sum(cz + (int64_t)i * n_ch, g0, g1, lane);
    } else {
        s = 0.0;
        for (int32_t t = vslice[a] + lane; t < vslice[a + 1]; t += 64) s += vpart[t];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    }
    if (caz) s -= wave_chunk_sum(caz + (int64_t)i * n_ch, g0, g1, lane);
    if (lane == 0) v[a] = s;
}

// w = E_b^-1 v_b per masked problem b: one wave per kept column (a row of E_b^-1)
__global__ __launch_bounds__(256) void k_coarse_einv(
    const double* __restrict__ Einv, const int64_t* __restrict__ einv_off,
    const int32_t* __restrict__ col_off, const int32_t* __restrict__ col_prob, int32_t r_eff,
    const double* __restrict__ v, double* __restrict__ w, const int* __restrict__ mask) {
    const int lane = threadIdx.x & 63;
    const int32_t a = (int32_t)blockIdx.x * 4 + (int32_t)(threadIdx.x >> 6);
    if (a >= r_eff) return;
    const int b = col_prob[a];
    if (mask && !mask[b]) return;
    const int32_t c0 = col_off[b], rb = col_off[b + 1] - c0, i = a - c0;
    const double* E = Einv + einv_off[b] + (int64_t)i * rb;
    double s = 0.0;
    for (int32_t q = lane; q < rb; q += 64) s += E[q] * v[c0 + q];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) w[a] = s;
}

// A-DEF2, last step: z = y + Z w per pixel (y = M_BD r already in z), partials of r^T z.
// DZ: dense Z blocks (layout of AZ); else the Z_S rows in CSR form.
template <typename TA, int NS, bool DZ>
__global__ __launch_bounds__(kVecThreads) void k_adef2_finish(
    const double* __restrict__ r, double* __restrict__ z, const TA* __restrict__ zd,
    const int64_t* __restrict__ az_off, const int32_t* __restrict__ col_off,
    const double* __restrict__ w, const int64_t* __restrict__ zptr,
    const int32_t* __restrict__ zcol, const double* __restrict__ zval, PcgCtl ctl) {
    __shared__ double red[kVecThreads];
    extern __shared__ double sw[];
    const VecBlock vb = vec_block(ctl, NS, false);
    if (ctl.mask && !ctl.mask[vb.b]) return;
    const int32_t c0 = col_off[vb.b], rk = col_off[vb.b + 1] - c0;
    for (int c = threadIdx.x; c < rk; c += kVecThreads) sw[c] = w[c0 + c];
    __syncthreads();
    const int64_t nv = vb.n * NS;
    double acc = 0.0;
    for (int64_t q = (int64_t)vb.k * kVecThreads + threadIdx.x; q < vb.n;
         q += vb.stride) {
        const int64_t p = vb.base + q;
        double zz[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) zz[s] = z[p * NS + s];
        if constexpr (DZ) {
            const TA* zb = zd + az_off[vb.b] + q * NS;
            for (int32_t c = 0; c < rk; ++c) {
                const double wc = sw[c];
#pragma unroll
                for (int s = 0; s < NS; ++s) zz[s] += (double)zb[(int64_t)c * nv + s] * wc;
            }
        } else {
            double zw = 0.0;
            for (int64_t e = zptr[p]; e < zptr[p + 1]; ++e) zw += zval[e] * sw[zcol[e] - c0];
            zz[0] += zw;
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            z[p * NS + s] = zz[s];
            acc += r[p * NS + s] * zz[s];
        }
    }
    if (ctl.part) write_partial_at(acc, slot_part(ctl, kSlotRZ, vb.b), vb.k, red);
}

// coarse correction of an initial guess: x += Z w, r -= AZ w per pixel
template <typename TA, int NS, bool DZ>
__global__ __launch_bounds__(kVecThreads) void k_coarse_correct(
    double* __restrict__ x, double* __restrict__ r, const TA* __restrict__ az,
    const TA* __restrict__ zd, const int64_t* __restrict__ az_off,
    const int32_t* __restrict__ col_off, const double* __restrict__ w,
    const int64_t* __restrict__ zptr, const int32_t* __restrict__ zcol,
    const double* __restrict__ zval, PcgCtl ctl) {
    extern __shared__ double sw[];
    const VecBlock vb = vec_block(ctl, NS, false);
    if (ctl.mask && !ctl.mask[vb.b]) return;
    const int32_t c0 = col_off[vb.b], rk = col_off[vb.b + 1] - c0;
    for (int c = threadIdx.x; c < rk; c += kVecThreads) sw[c] = w[c0 + c];
    __syncthreads();
    const int64_t nv = vb.n * NS;
    for (int64_t q = (int64_t)vb.k * kVecThreads + threadIdx.x; q < vb.n;
         q += vb.stride) {
        const int64_t p = vb.base + q;
        double dx[NS], dr[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) dx[s] = dr[s] = 0.0;
        const TA* ab = az + az_off[vb.b] + q * NS;
        for (int32_t c = 0; c < rk; ++c) {
            const double wc = sw[c];
#pragma unroll
            for (int s = 0; s < NS; ++s) dr[s] += (double)ab[(int64_t)c * nv + s] * wc;
            if constexpr (DZ) {
                const TA* zb = zd + az_off[vb.b] + q * NS;
#pragma unroll
                for (int s = 0; s < NS; ++s) dx[s] += (double)zb[(int64_t)c * nv + s] * wc;
            }
        }
        if constexpr (!DZ)
            for (int64_t e = zptr[p]; e < zptr[p + 1]; ++e) dx[0] += zval[e] * sw[zcol[e] - c0];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            x[p * NS + s] += dx[s];
            r[p * NS + s] -= dr[s];
        }
    }
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

// C[ra][rb] (device, row-major) = A^T B for device row-major A [n][ra], B [n][rb], enqueued
// on st (no synchronisation: its scratch is released in stream order)
// slabs of the n dimension: about 64 MFMA steps per wave, at most 4096 waves in all
int32_t gram_ksplit(int64_t n, int32_t ra, int32_t rb) {
    const int32_t ntile = (ra / 16) * (rb / 16);
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(n / 4 / 64, 4096 / std::max(1, ntile)));
}

// layers of the A Z columns per zero-skipping N^-1 launch (mixed plans; even)
constexpr int kAzGroup = 8;

// P^T work range (samples per wave) of the A Z passes, whatever range the plan's P^T
// takes: the eight-column pass holds few waves per SIMD (its registers), and shorter
// ranges only add wave start-up work there (A Z build of the 2^24 raster with ranges of
// 512 / 2048 / 4096 samples: plan 9.76 / 9.16 / 9.06 ms)
constexpr int64_t kAzPtRange = 4096;

// dense row blocks of the batched Gram products, zd and azr together (bytes)
constexpr int64_t kGramBudget = (int64_t)1 << 30;

int gemm_tn_f64(hipStream_t st, const double* A, const double* B, int64_t n, int32_t ra,
                int32_t rb, double* dev_C) {
    const int32_t ntile = (ra / 16) * (rb / 16);
    const int32_t ksplit = gram_ksplit(n, ra, rb);
    DBuf<double> part;
    MM_TRY(part.alloc((size_t)ksplit * ra * rb));
    const int64_t waves = (int64_t)ntile * ksplit;
    hipLaunchKernelGGL(k_gemm_tn_f64, dim3((waves + 3) / 4), dim3(256), 0, st, A, B, n, ra, rb,
                       ksplit, part.p);
    MM_HIP(hipGetLastError());
    const int64_t m = (int64_t)ra * rb;
    hipLaunchKernelGGL(k_sum_parts, dim3(grid_for(m)), dim3(256), 0, st, part.p, m, ksplit, dev_C);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

// ---- the E product without allocation: its slab partials live in a fixed device array.
//
// The array holds kNoAllocDoubles FP64 values (8 MiB) on every device the library runs
// on, until the process ends.  Host code never passes the array's name to a kernel (on
// the host it only stands in for the symbol): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current and kept per
// device.  Every call on a device shares that device's array, so calls that overlap on
// one device race.
constexpr int64_t kNoAllocDoubles = (int64_t)1 << 20;
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[kNoAllocMaxDevices] = {};
}  // namespace

// the device address of the calling thread's current device's array
int scratch_address(double** out) {
    int dev = -1;
    MM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices) {
        set_error("device %d outside the %d devices the fixed scratch supports", dev,
                  kNoAllocMaxDevices);
        return MM_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress of the fixed scratch failed on device %d: %s", dev,
                      hipGetErrorString(e));
            return MM_ERR_DEVICE;
        }
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return MM_OK;
}

int gemm_tn_f64_noalloc(hipStream_t st, const double* A, const double* B, int64_t n,
                        int32_t ra, int32_t rb, double* dev_C) {
    const int32_t ntile = (ra / 16) * (rb / 16);
    const int32_t ksplit = gram_ksplit(n, ra, rb);
    const int64_t need = (int64_t)ksplit * ra * rb;
    if (need > kNoAllocDoubles) {
        set_error("mm_gemm_tn_f64_noalloc: %lld partial values (ra %d, rb %d, %d slabs) exceed "
                  "the fixed scratch of %lld FP64 values (ra * rb <= 2^20 always fits)",
                  (long long)need, ra, rb, ksplit, (long long)kNoAllocDoubles);
        return MM_ERR_ARG;
    }
    if (st) {
        int sdev = -1, dev = -1;
        MM_HIP(hipStreamGetDevice(st, &sdev));
        MM_HIP(hipGetDevice(&dev));
        if (sdev != dev) {
            set_error("mm_gemm_tn_f64_noalloc: the stream belongs to device %d, the current "
                      "device is %d", sdev, dev);
            return MM_ERR_ARG;
        }
    }
    double* part = nullptr;
    MM_TRY(scratch_address(&part));
    const int64_t waves = (int64_t)ntile * ksplit;
    hipLaunchKernelGGL(k_gemm_tn_f64, dim3((waves + 3) / 4), dim3(256), 0, st, A, B, n, ra, rb,
                       ksplit, part);
    MM_HIP(hipGetLastError());
    const int64_t m = (int64_t)ra * rb;
    hipLaunchKernelGGL(k_sum_parts, dim3(grid_for(m)), dim3(256), 0, st, part, m, ksplit, dev_C);
    MM_HIP(hipGetLastError());
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
    const int B = pl->n_prob;
    const int64_t n_obs = pl->n_obs, ns = pl->n_s, nv = n_obs * ns;
    const std::vector<int64_t>& oo = pl->h_ooff;
    // Z_S in CSR form (per pixel, ascending interval)
    DBuf<int64_t> nnz, ptr;
    MM_TRY(nnz.alloc(n_obs));
    MM_TRY(ptr.alloc(n_obs + 1));
    hipLaunchKernelGGL(k_zs_count, dim3(grid_for(n_obs, 128)), dim3(128), 0, st, pl->perm.p,
                       pl->seg.p, pl->hits.p, n_obs, pl->int_lo.p, pl->n_int, nnz.p);
    MM_HIP(hipGetLastError());
    MM_TRY(scan_exclusive_i64(nnz.p, ptr.p, n_obs, st));
    int64_t total = 0;
    MM_HIP(hipMemcpyAsync(&total, ptr.p + n_obs, 8, hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    DBuf<int32_t> col;
    DBuf<double> val;
    MM_TRY(col.alloc(total));
    MM_TRY(val.alloc(total));
    hipLaunchKernelGGL(k_zs_fill, dim3(grid_for(n_obs, 128)), dim3(128), 0, st, pl->perm.p,
                       pl->seg.p, pl->hits.p, n_obs, pl->int_lo.p, pl->n_int, ptr.p, col.p, val.p);
    MM_HIP(hipGetLastError());
    tick("zs");
    // Z_S by column on the device: entries stably sorted by column (rows stay ascending)
    const int32_t K = pl->n_int;
    DBuf<int32_t> rowid, eidx, skey, sidx, crow;
    DBuf<double> cval;
    DBuf<int64_t> cbeg, cend;
    DBuf<unsigned long long> chash;
    MM_TRY(rowid.alloc(total));
    MM_TRY(eidx.alloc(total));
    MM_TRY(skey.alloc(total));
    MM_TRY(sidx.alloc(total));
    MM_TRY(crow.alloc(total));
    MM_TRY(cval.alloc(total));
    MM_TRY(cbeg.alloc(K));
    MM_TRY(cend.alloc(K));
    MM_TRY(chash.alloc(K));
    hipLaunchKernelGGL(k_expand_rows, dim3(grid_for(n_obs)), dim3(256), 0, st, ptr.p, n_obs,
                       rowid.p, eidx.p);
    MM_HIP(hipGetLastError());
    MM_TRY(radix_sort_pairs(col.p, eidx.p, total, K - 1, skey.p, sidx.p, st));
    hipLaunchKernelGGL(k_csc_fill, dim3(grid_for(total)), dim3(256), 0, st, skey.p, sidx.p, total,
                       rowid.p, val.p, crow.p, cval.p, cbeg.p, cend.p);
    hipLaunchKernelGGL(k_col_hash, dim3(K), dim3(256), 0, st, cbeg.p, cend.p, crow.p, cval.p,
                       chash.p);
    MM_HIP(hipGetLastError());
    std::vector<unsigned long long> hh(K);
    std::vector<int64_t> hb(K), he(K);
    MM_HIP(hipMemcpyAsync(hh.data(), chash.p, K * 8, hipMemcpyDeviceToHost, st));
    MM_HIP(hipMemcpyAsync(hb.data(), cbeg.p, K * 8, hipMemcpyDeviceToHost, st));
    MM_HIP(hipMemcpyAsync(he.data(), cend.p, K * 8, hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    rowid.release();
    eidx.release();
    skey.release();
    sidx.release();
    // duplicate columns: proposed by (hash, entry count), confirmed by an exact comparison;
    // a column keeps the first (lowest) interval with the same content as representative
    std::vector<int32_t> cand_a, cand_b;
    {
        std::unordered_map<uint64_t, int32_t> first;
        for (int32_t j = 0; j < K; ++j) {
            const uint64_t key = hh[j] ^ ((uint64_t)(he[j] - hb[j]) * 0x9E3779B97F4A7C15ull);
            auto it = first.find(key);
            if (it == first.end()) {
                first.emplace(key, j);
            } else if (he[it->second] - hb[it->second] == he[j] - hb[j]) {
                cand_a.push_back(j);
                cand_b.push_back(it->second);
            }
        }
    }
    std::vector<char> dup(K, 0);
    std::vector<int32_t> rep(K);  // interval whose column represents interval j's column
    for (int32_t j = 0; j < K; ++j) rep[j] = j;
    if (!cand_a.empty()) {
        const int nc = (int)cand_a.size();
        DBuf<int32_t> da, db;
        DBuf<int> neq;
        MM_TRY(da.alloc(nc));
        MM_TRY(db.alloc(nc));
        MM_TRY(neq.alloc(nc));
        MM_HIP(hipMemcpyAsync(da.p, cand_a.data(), nc * 4, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(db.p, cand_b.data(), nc * 4, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemsetAsync(neq.p, 0, nc * sizeof(int), st));
        hipLaunchKernelGGL(k_cols_equal, dim3(nc), dim3(256), 0, st, da.p, db.p, cbeg.p, cend.p,
                           crow.p, cval.p, neq.p);
        MM_HIP(hipGetLastError());
        std::vector<int> hn(nc);
        MM_HIP(hipMemcpyAsync(hn.data(), neq.p, nc * sizeof(int), hipMemcpyDeviceToHost, st));
        MM_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < nc; ++i)
            if (!hn[i]) {
                dup[cand_a[i]] = 1;
                rep[cand_a[i]] = cand_b[i];
            }
    }
    std::vector<int32_t> uniq;  // representative interval of every distinct column
    for (int32_t j = 0; j < K; ++j)
        if (!dup[j]) uniq.push_back(j);
    const int32_t rd = (int32_t)uniq.size();
    co.r_dedup = rd;
    // distinct columns per problem (columns of distinct problems have disjoint rows, so
    // none is merged across problems; intervals are problem-ordered)
    std::vector<int32_t> ud_off(B + 1, 0);
    {
        int32_t u = 0;
        for (int b = 0; b < B; ++b) {
            ud_off[b] = u;
            while (u < rd && uniq[u] < pl->h_pint[b + 1]) ++u;
        }
        ud_off[B] = rd;
    }
    int32_t rd_max = 0;
    std::vector<int64_t> azd_off(B + 1, 0);
    for (int b = 0; b < B; ++b) {
        const int32_t r_b = ud_off[b + 1] - ud_off[b];
        if (r_b == 0) {
            set_error("problem %d has no coarse-space column", b);
            return MM_ERR_RANK;
        }
        rd_max = std::max(rd_max, r_b);
        azd_off[b + 1] = azd_off[b] + (int64_t)r_b * (oo[b + 1] - oo[b]) * ns;
    }
    tick("dedup");
    // entry ranges of the distinct columns in the CSC arrays
    std::vector<int64_t> ub(rd), ue(rd);
    for (int32_t u = 0; u < rd; ++u) {
        ub[u] = hb[uniq[u]];
        ue[u] = he[uniq[u]];
    }
    DBuf<int64_t> dub, due;
    MM_TRY(dub.alloc(rd));
    MM_TRY(due.alloc(rd));
    MM_HIP(hipMemcpyAsync(dub.p, ub.data(), rd * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(due.p, ue.data(), rd * 8, hipMemcpyHostToDevice, st));
    // AZ of the distinct columns, block per problem: A is block diagonal over the problems,
    // so one application to the sum of every problem's k-th column (layer k) gives all k-th
    // columns.  Layer k's columns reach only the intervals flagged in on[k]; the tiles of the
    // others write zeros without loading.
    const bool mixed = pl->opts.precision == MM_MIXED;
    const int64_t pt_keep = pl->pt_range;  // the plan's P^T range, restored after A Z
    if (pt_keep != kAzPtRange) MM_TRY(build_wave_ranges(pl, kAzPtRange));
    DBuf<double> azd;
    DBuf<float> azf;
    if (mixed) MM_TRY(azf.alloc((size_t)azd_off[B]));
    else MM_TRY(azd.alloc((size_t)azd_off[B]));
    DBuf<int64_t> d_azd_off;
    MM_TRY(d_azd_off.alloc(B + 1));
    MM_HIP(hipMemcpyAsync(d_azd_off.p, azd_off.data(), (B + 1) * 8, hipMemcpyHostToDevice, st));
    // layer of every interval's column within its problem, and the (layer, interval) flags
    std::vector<int32_t> u_of(K, -1), h_layer(K);
    for (int32_t u = 0; u < rd; ++u) u_of[uniq[u]] = u;
    for (int b = 0; b < B; ++b)
        for (int32_t j = pl->h_pint[b]; j < pl->h_pint[b + 1]; ++j) {
            h_layer[j] = u_of[rep[j]] - ud_off[b];
            if (h_layer[j] < 0 || h_layer[j] >= ud_off[b + 1] - ud_off[b]) {  // flags index
                set_error("interval %d: column layer %d outside [0, %d)", j, h_layer[j],
                          ud_off[b + 1] - ud_off[b]);
                return MM_ERR_ARG;
            }
        }
    DBuf<int32_t> d_layer;
    DBuf<uint8_t> on;
    MM_TRY(d_layer.alloc(K));
    MM_TRY(on.alloc((size_t)rd_max * K));
    MM_HIP(hipMemcpyAsync(d_layer.p, h_layer.data(), (size_t)K * 4, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemsetAsync(on.p, 0, (size_t)rd_max * K, st));
    hipLaunchKernelGGL(k_az_int_flags, dim3(grid_for(n_obs)), dim3(256), 0, st, ptr.p, col.p,
                       n_obs, d_layer.p, K, rd_max, on.p);
    MM_HIP(hipGetLastError());
    std::vector<int32_t> h_rb(B);
    for (int b = 0; b < B; ++b) h_rb[b] = ud_off[b + 1] - ud_off[b];
    DBuf<int32_t> d_rb;
    MM_TRY(d_rb.alloc(B));
    MM_HIP(hipMemcpyAsync(d_rb.p, h_rb.data(), B * 4, hipMemcpyHostToDevice, st));
    // the I rows of the columns of a layer (mixed: of a group of layers), the Q and U rows
    // of Z_S being zero: N^-1 P reads no weights
    DBuf<double> zc, tmp;
    MM_TRY(zc.alloc((size_t)(mixed ? kAzGroup : 1) * n_obs));
    if (!mixed) MM_TRY(tmp.alloc(nv));
    DBuf<float> todg;  // mixed: the time streams of a group of layers
    if (mixed) MM_TRY(todg.alloc((size_t)kAzGroup * pl->n_t));
    DBuf<int32_t> lcols, lprob, llay;
    MM_TRY(lcols.alloc((size_t)rd_max * B));
    MM_TRY(lprob.alloc((size_t)rd_max * B));
    MM_TRY(llay.alloc((size_t)rd_max * B));
    {
        // the columns by layer: layer k's are [lo_k, lo_k + lcnt[k]) of lcols (problem in
        // lprob, layer in llay)
        std::vector<int32_t> hc, hp, hl;
        std::vector<int32_t> lcnt(rd_max, 0);
        for (int32_t k = 0; k < rd_max; ++k)
            for (int b = 0; b < B; ++b)
                if (ud_off[b] + k < ud_off[b + 1]) {
                    hc.push_back(ud_off[b] + k);
                    hp.push_back(b);
                    hl.push_back(k);
                    lcnt[k]++;
                }
        MM_HIP(hipMemcpyAsync(lcols.p, hc.data(), hc.size() * 4, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(lprob.p, hp.data(), hp.size() * 4, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(llay.p, hl.data(), hl.size() * 4, hipMemcpyHostToDevice, st));
        int64_t nb_max = 1;  // largest problem vector
        for (int b = 0; b < B; ++b) nb_max = std::max<int64_t>(nb_max, (oo[b + 1] - oo[b]) * ns);
        const int sgx = (int)std::min<int64_t>(1024, (nb_max + 255) / 256);
        int64_t lo = 0;
        // the I rows of layers k0 .. k0 + nc (columns lo .. lo + their count) into zeroed
        // maps of n_obs values side by side, in launches of at most 65535 columns
        auto layer_maps = [&](int32_t k0, int nc) -> int {
            MM_HIP(hipMemsetAsync(zc.p, 0, (size_t)nc * n_obs * 8, st));
            int64_t cnt = 0;
            for (int c = 0; c < nc; ++c) cnt += lcnt[k0 + c];
            for (int64_t c0 = 0; c0 < cnt; c0 += 65535) {
                const unsigned gy = (unsigned)std::min<int64_t>(65535, cnt - c0);
                hipLaunchKernelGGL(k_cols_to_maps, dim3(16, gy), dim3(256), 0, st,
                                   lcols.p + lo + c0, llay.p + lo + c0, k0, n_obs, dub.p, due.p,
                                   crow.p, cval.p, zc.p);
                MM_HIP(hipGetLastError());
            }
            lo += cnt;
            return MM_OK;
        };
        if (mixed) {
            // kAzGroup layers at a time: one N^-1 P launch over their maps, P^T
            // kScatterCols layers per pass
            for (int32_t k0 = 0; k0 < rd_max; k0 += kAzGroup) {
                const int nc = std::min<int32_t>(kAzGroup, rd_max - k0);
                MM_TRY(layer_maps(k0, nc));
                MM_TRY(toeplitz_map32_layers(pl, zc.p, n_obs, nullptr, 0, todg.p, pl->n_t,
                                             on.p + (int64_t)k0 * K, K, nc));
                for (int c = 0; c < nc; c += kScatterCols)
                    MM_TRY(scatter_cols32(pl, todg.p + c * pl->n_t, pl->n_t,
                                          std::min(kScatterCols, nc - c), k0 + c, d_rb.p,
                                          d_azd_off.p, azf.p));
            }
        } else {
            for (int32_t k = 0; k < rd_max; ++k) {
                const int nl = lcnt[k];
                const int64_t lo_k = lo;
                MM_TRY(layer_maps(k, 1));
                MM_TRY(apply_A64_sparse_i(pl, zc.p, tmp.p, on.p + (int64_t)k * K));
                hipLaunchKernelGGL(k_store_az<double>, dim3(sgx, nl), dim3(256), 0, st,
                                   lprob.p + lo_k, (const double*)tmp.p, pl->ooff.p, (int)ns,
                                   (const int64_t*)d_azd_off.p, k, azd.p);
                MM_HIP(hipGetLastError());
            }
        }
    }
    zc.release();
    tmp.release();
    todg.release();
    on.release();
    if (pt_keep != kAzPtRange) MM_TRY(build_wave_ranges(pl, pt_keep));
    tick("AZ");
    // per problem: E_b = Z_b^T (AZ)_b on the matrix cores, independent subset, E_b^-1
    // every problem's E_b = Z_b^T (AZ)_b on the matrix cores into one device array
    // (offsets eoff), in batched launches over groups of problems whose dense row blocks
    // fit kGramBudget bytes, read back once
    std::vector<int64_t> eoff(B + 1, 0);
    for (int b = 0; b < B; ++b) {
        const int64_t rp = (ud_off[b + 1] - ud_off[b] + 15) / 16 * 16;
        eoff[b + 1] = eoff[b] + rp * rp;
    }
    DBuf<double> dE;
    DBuf<int32_t> d_ud_off;
    MM_TRY(dE.alloc((size_t)eoff[B]));
    MM_TRY(d_ud_off.alloc(B + 1));
    MM_HIP(hipMemcpyAsync(d_ud_off.p, ud_off.data(), (B + 1) * 4, hipMemcpyHostToDevice, st));
    for (int b0 = 0; b0 < B;) {
        std::vector<GramDesc> gd;
        std::vector<int64_t> woff(1, 0), leoff(1, 0);
        int64_t rows = 0, parts = 0;
        int32_t rmax = 1;
        int64_t nob_max = 1;
        int b1 = b0;
        for (; b1 < B; ++b1) {
            const int32_t rb = ud_off[b1 + 1] - ud_off[b1];
            const int32_t rp = (rb + 15) / 16 * 16;
            const int64_t nob = oo[b1 + 1] - oo[b1];
            const int64_t npad = (nob + 3) / 4 * 4;
            if (b1 > b0 && ((rows + npad * rp) * 16 > kGramBudget || b1 - b0 == 65535)) break;
            GramDesc g;
            g.a_off = rows;
            g.n = npad;
            g.rp = rp;
            g.ksplit = gram_ksplit(npad, rp, rp);
            g.part_off = parts;
            g.c_off = eoff[b1];
            gd.push_back(g);
            rows += npad * rp;
            parts += (int64_t)g.ksplit * rp * rp;
            woff.push_back(woff.back() + (int64_t)(rp / 16) * (rp / 16) * g.ksplit);
            leoff.push_back(leoff.back() + (int64_t)rp * rp);
            rmax = std::max(rmax, rb);
            nob_max = std::max(nob_max, nob);
        }
        const int nbc = b1 - b0;
        DBuf<GramDesc> d_gd;
        DBuf<int64_t> d_woff, d_leoff;
        DBuf<double> zd, azr, part;
        MM_TRY(d_gd.alloc(nbc));
        MM_TRY(d_woff.alloc(nbc + 1));
        MM_TRY(d_leoff.alloc(nbc + 1));
        MM_TRY(zd.alloc((size_t)rows));
        MM_TRY(azr.alloc((size_t)rows));
        MM_TRY(part.alloc((size_t)parts));
        MM_HIP(hipMemcpyAsync(d_gd.p, gd.data(), nbc * sizeof(GramDesc), hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(d_woff.p, woff.data(), (nbc + 1) * 8, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(d_leoff.p, leoff.data(), (nbc + 1) * 8, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemsetAsync(zd.p, 0, (size_t)rows * 8, st));
        MM_HIP(hipMemsetAsync(azr.p, 0, (size_t)rows * 8, st));
        hipLaunchKernelGGL(k_dense_z_batch, dim3(64, rmax, nbc), dim3(256), 0, st, dub.p, due.p,
                           crow.p, cval.p, d_ud_off.p, pl->ooff.p, d_gd.p, b0, zd.p);
        if (mixed)
            hipLaunchKernelGGL(k_az_rows_batch<float>, dim3(grid_for(nob_max, 64, 2048), (rmax + 63) / 64, nbc),
                               dim3(256), 0, st, azf.p, d_azd_off.p, d_ud_off.p, pl->ooff.p,
                               (int)ns, d_gd.p, b0, azr.p);
        else
            hipLaunchKernelGGL(k_az_rows_batch<double>, dim3(grid_for(nob_max, 64, 2048), (rmax + 63) / 64, nbc),
                               dim3(256), 0, st, azd.p, d_azd_off.p, d_ud_off.p, pl->ooff.p,
                               (int)ns, d_gd.p, b0, azr.p);
        hipLaunchKernelGGL(k_gemm_tn_f64_batch, dim3((woff[nbc] + 3) / 4), dim3(256), 0, st, zd.p,
                           azr.p, d_gd.p, d_woff.p, nbc, part.p);
        hipLaunchKernelGGL(k_sum_parts_batch, dim3(grid_for(leoff[nbc])), dim3(256), 0, st, part.p,
                           d_gd.p, d_leoff.p, nbc, dE.p);
        MM_HIP(hipGetLastError());
        b0 = b1;
    }
    std::vector<double> Eh((size_t)eoff[B]);
    MM_HIP(hipMemcpyAsync(Eh.data(), dE.p, Eh.size() * 8, hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    std::vector<std::vector<int>> sels(B);
    std::vector<double> Eall, Einv_all;
    co.h_col_off.assign(B + 1, 0);
    co.h_einv_off.assign(B + 1, 0);
    co.h_az_off.assign(B + 1, 0);
    co.cols.clear();
    co.r_max = 0;
    for (int b = 0; b < B; ++b) {
        const int32_t rb = ud_off[b + 1] - ud_off[b];
        const int64_t nob = oo[b + 1] - oo[b];
        const int32_t rp = (rb + 15) / 16 * 16;
        const double* Ep = Eh.data() + eoff[b];
        std::vector<double> E((size_t)rb * rb);
        for (int32_t i = 0; i < rb; ++i)
            for (int32_t j = 0; j < rb; ++j)
                E[(size_t)i * rb + j] = 0.5 * (Ep[(size_t)i * rp + j] + Ep[(size_t)j * rp + i]);
        std::vector<int> sel = pivoted_cholesky_select(E, rb, pl->opts.rank_tol);
        const int32_t k = (int32_t)sel.size();
        if (k == 0) {
            set_error("coarse matrix E of problem %d is zero", b);
            return MM_ERR_RANK;
        }
        std::vector<double> Es((size_t)k * k), Einv;
        for (int32_t i = 0; i < k; ++i)
            for (int32_t j = 0; j < k; ++j) Es[(size_t)i * k + j] = E[(size_t)sel[i] * rb + sel[j]];
        if (!spd_inverse(Es, k, Einv)) {
            set_error("coarse matrix E of problem %d not positive definite on the selected columns",
                      b);
            return MM_ERR_RANK;
        }
        Eall.insert(Eall.end(), Es.begin(), Es.end());
        Einv_all.insert(Einv_all.end(), Einv.begin(), Einv.end());
        for (int32_t i = 0; i < k; ++i) co.cols.push_back(uniq[ud_off[b] + sel[i]]);
        co.h_col_off[b + 1] = co.h_col_off[b] + k;
        co.h_einv_off[b + 1] = co.h_einv_off[b] + (int64_t)k * k;
        co.h_az_off[b + 1] = co.h_az_off[b] + (int64_t)k * nob * ns;
        co.r_max = std::max(co.r_max, k);
        sels[b] = std::move(sel);
    }
    dE.release();
    const int32_t keff = co.h_col_off[B];
    co.r_eff = keff;
    co.E = std::move(Eall);
    tick("E");
    MM_TRY(co.Einv.alloc(Einv_all.size()));
    MM_HIP(hipMemcpyAsync(co.Einv.p, Einv_all.data(), Einv_all.size() * 8, hipMemcpyHostToDevice,
                          st));
    tick("Einv");
    // kept AZ columns into the final per-problem blocks
    {
        std::vector<int64_t> so(keff), d_o(keff), cn(keff);
        for (int b = 0; b < B; ++b) {
            const int64_t n_b = (oo[b + 1] - oo[b]) * ns;
            for (size_t i = 0; i < sels[b].size(); ++i) {
                const int32_t a = co.h_col_off[b] + (int32_t)i;
                so[a] = azd_off[b] + (int64_t)sels[b][i] * n_b;
                d_o[a] = co.h_az_off[b] + (int64_t)i * n_b;
                cn[a] = n_b;
            }
        }
        DBuf<int64_t> dso, ddo, dcn;
        MM_TRY(dso.alloc(keff));
        MM_TRY(ddo.alloc(keff));
        MM_TRY(dcn.alloc(keff));
        MM_HIP(hipMemcpyAsync(dso.p, so.data(), keff * 8, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(ddo.p, d_o.data(), keff * 8, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(dcn.p, cn.data(), keff * 8, hipMemcpyHostToDevice, st));
        // the FP16 copy of AZ for the A-DEF1 apply of mixed plans (column maxima taken by the
        // copy into AZ32)
        const bool fp16 = mixed && pl->opts.az_fp16 && keff > 0;
        DBuf<unsigned> dmx;
        if (fp16) {
            MM_TRY(dmx.alloc(keff));
            MM_HIP(hipMemsetAsync(dmx.p, 0, keff * sizeof(unsigned), st));
        }
        if (mixed) {
            MM_TRY(co.AZ32.alloc((size_t)co.h_az_off[B]));
            hipLaunchKernelGGL(k_copy_cols<float>, dim3(64, keff), dim3(256), 0, st,
                               (const float*)azf.p, co.AZ32.p, (const int64_t*)dso.p,
                               (const int64_t*)ddo.p, (const int64_t*)dcn.p, dmx.p);
        } else {
            MM_TRY(co.AZ64.alloc((size_t)co.h_az_off[B]));
            hipLaunchKernelGGL(k_copy_cols<double>, dim3(64, keff), dim3(256), 0, st,
                               (const double*)azd.p, co.AZ64.p, (const int64_t*)dso.p,
                               (const int64_t*)ddo.p, (const int64_t*)dcn.p, nullptr);
        }
        MM_HIP(hipGetLastError());
        if (fp16) {
            // FP16 copy for the A-DEF1 apply: pixel pairs, columns padded to 8 entries
            std::vector<int64_t> h16(B + 1, 0), lenv(keff), dof(keff), ldv(keff);
            for (int b = 0; b < B; ++b) {
                const int64_t pix_b = oo[b + 1] - oo[b];
                const int64_t ld = (ns * 2 * ((pix_b + 1) / 2) + 7) / 8 * 8;
                const int32_t r_b = co.h_col_off[b + 1] - co.h_col_off[b];
                for (int32_t i = 0; i < r_b; ++i) {
                    const int32_t a = co.h_col_off[b] + i;
                    lenv[a] = pix_b * ns;
                    dof[a] = h16[b] + (int64_t)i * ld;
                    ldv[a] = ld;
                }
                h16[b + 1] = h16[b] + (int64_t)r_b * ld;
            }
            DBuf<int64_t> dlen, ddof, dld;
            MM_TRY(dlen.alloc(keff));
            MM_TRY(ddof.alloc(keff));
            MM_TRY(dld.alloc(keff));
            MM_TRY(co.AZ16.alloc((size_t)h16[B]));
            MM_TRY(co.az16_off.alloc(B + 1));
            MM_TRY(co.az16_scale.alloc(keff));
            MM_HIP(hipMemcpyAsync(dlen.p, lenv.data(), keff * 8, hipMemcpyHostToDevice, st));
            MM_HIP(hipMemcpyAsync(ddof.p, dof.data(), keff * 8, hipMemcpyHostToDevice, st));
            MM_HIP(hipMemcpyAsync(dld.p, ldv.data(), keff * 8, hipMemcpyHostToDevice, st));
            MM_HIP(hipMemcpyAsync(co.az16_off.p, h16.data(), (B + 1) * 8, hipMemcpyHostToDevice,
                                  st));
            hipLaunchKernelGGL(k_az_to_half, dim3(64, keff), dim3(256), 0, st,
                               (const float*)co.AZ32.p, (const int64_t*)ddo.p,
                               (const int64_t*)dlen.p, (const int64_t*)ddof.p,
                               (const int64_t*)dld.p, (const unsigned*)dmx.p, co.az16_scale.p,
                               co.AZ16.p);
            MM_HIP(hipGetLastError());
            MM_HIP(hipStreamSynchronize(st));
        }
        MM_HIP(hipStreamSynchronize(st));
    }
    azf.release();
    azd.release();
    tick("AZ kept");
    // kept columns by column: entry ranges into the distinct-column lists; Z^T r slices
    std::vector<int64_t> kb(keff), ke(keff);
    std::vector<int32_t> vs(keff + 1, 0), cprob(keff);
    for (int b = 0; b < B; ++b)
        for (size_t i = 0; i < sels[b].size(); ++i) {
            const int32_t a = co.h_col_off[b] + (int32_t)i;
            const int32_t u = ud_off[b] + sels[b][i];
            kb[a] = ub[u];
            ke[a] = ue[u];
            cprob[a] = b;
        }
    for (int32_t a = 0; a < keff; ++a)
        vs[a + 1] = vs[a] + (int32_t)std::max<int64_t>(1, (ke[a] - kb[a] + 511) / 512);
    co.n_slices = vs[keff];
    std::vector<int32_t> scol((size_t)co.n_slices);
    for (int32_t a = 0; a < keff; ++a)
        for (int32_t t = vs[a]; t < vs[a + 1]; ++t) scol[t] = a;
    MM_TRY(co.slice_col.alloc(co.n_slices));
    MM_HIP(hipMemcpyAsync(co.slice_col.p, scol.data(), co.n_slices * 4, hipMemcpyHostToDevice, st));
    co.csc_row.swap(crow);
    co.csc_val.swap(cval);
    MM_TRY(co.csc_beg.alloc(keff));
    MM_TRY(co.csc_end.alloc(keff));
    MM_TRY(co.vslice.alloc(keff + 1));
    MM_TRY(co.col_prob.alloc(keff));
    MM_TRY(co.col_off.alloc(B + 1));
    MM_TRY(co.az_off.alloc(B + 1));
    MM_TRY(co.einv_off.alloc(B + 1));
    MM_HIP(hipMemcpyAsync(co.csc_beg.p, kb.data(), keff * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(co.csc_end.p, ke.data(), keff * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(co.vslice.p, vs.data(), (keff + 1) * 4, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(co.col_prob.p, cprob.data(), keff * 4, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(co.col_off.p, co.h_col_off.data(), (B + 1) * 4, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(co.az_off.p, co.h_az_off.data(), (B + 1) * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(co.einv_off.p, co.h_einv_off.data(), (B + 1) * 8, hipMemcpyHostToDevice,
                          st));
    tick("csc");
    // kept columns by pixel (CSR), filtered on the device from the full Z_S rows
    std::vector<int32_t> colmap(K, -1);
    for (int32_t a = 0; a < keff; ++a) colmap[co.cols[a]] = a;
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
    MM_HIP(hipMemcpyAsync(&kn, co.csr_ptr.p + n_obs, 8, hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    MM_TRY(co.csr_col.alloc(std::max<int64_t>(1, kn)));
    MM_TRY(co.csr_val.alloc(std::max<int64_t>(1, kn)));
    hipLaunchKernelGGL(k_csr_filter, dim3(grid_for(n_obs)), dim3(256), 0, st, ptr.p, col.p, val.p,
                       n_obs, dmap.p, (const int64_t*)co.csr_ptr.p, (int64_t*)nullptr,
                       co.csr_col.p, co.csr_val.p);
    MM_HIP(hipGetLastError());
    MM_TRY(co.w.alloc(keff));
    MM_TRY(co.v.alloc(keff));
    MM_TRY(co.vpart.alloc(co.n_slices));
    // chunk tables of the dense (AZ)^T y products (A-DEF2)
    {
        std::vector<int64_t> choff(B + 1, 0);
        for (int b = 0; b < B; ++b)
            choff[b + 1] = choff[b] + ((oo[b + 1] - oo[b]) * ns + kZtChunk - 1) / kZtChunk;
        co.n_chunks = choff[B];
        MM_TRY(co.ch_off.alloc(B + 1));
        MM_TRY(co.cpart2.alloc((size_t)co.n_chunks * co.r_max));
        MM_HIP(hipMemcpyAsync(co.ch_off.p, choff.data(), (B + 1) * 8, hipMemcpyHostToDevice, st));
    }
    MM_HIP(hipStreamSynchronize(st));
    tick("csr");
    co.kind = 1;
    pl->has_coarse = true;
    return MM_OK;
}

// Z_D [Sect. 3.3.2]: the selected Ritz vectors y = W s of every problem, stored densely
// (all Stokes rows) in the layout of the AZ blocks, in the precision of AZ.  AZ_D follows
// from one A application per column index (A is block diagonal over the problems), E_D =
// Z_D^T AZ_D per problem on the matrix cores, and the pivoted Cholesky selection keeps an
// independent subset (the Lanczos process in finite precision can return near-copies of a
// converged Ritz vector).  Replaces the plan's coarse space.
int build_coarse_dense(mm_plan_t pl, const double* basis, int64_t basis_stride,
                       const std::vector<std::vector<double>>& G, const std::vector<int>& m,
                       const std::vector<std::vector<double>>& theta) {
    hipStream_t st = pl->stream;
    const int B = pl->n_prob;
    const int64_t ns = pl->n_s, nv = pl->n_obs * pl->n_s;
    const std::vector<int64_t>& oo = pl->h_ooff;
    const bool mixed = pl->opts.precision == MM_MIXED;
    std::vector<int32_t> rb(B);
    std::vector<int64_t> zoff(B + 1, 0), goff(B + 1, 0);
    int32_t r_all = 0, r_max = 0;
    for (int b = 0; b < B; ++b) {
        rb[b] = (int32_t)theta[b].size();
        zoff[b + 1] = zoff[b] + (int64_t)rb[b] * (oo[b + 1] - oo[b]) * ns;
        goff[b + 1] = goff[b] + (int64_t)m[b] * rb[b];
        r_all += rb[b];
        r_max = std::max(r_max, rb[b]);
    }
    if (r_all == 0) {
        set_error("no Ritz value below eps_tol: Z_D would be empty");
        return MM_ERR_RANK;
    }
    DBuf<double> zd64, az64;
    DBuf<float> zd32, az32;
    if (mixed) {
        MM_TRY(zd32.alloc((size_t)zoff[B]));
        MM_TRY(az32.alloc((size_t)zoff[B]));
    } else {
        MM_TRY(zd64.alloc((size_t)zoff[B]));
        MM_TRY(az64.alloc((size_t)zoff[B]));
    }
    {
        std::vector<double> hg((size_t)std::max<int64_t>(1, goff[B]));
        for (int b = 0; b < B; ++b) std::copy(G[b].begin(), G[b].end(), hg.begin() + goff[b]);
        DBuf<double> dG;
        MM_TRY(dG.alloc(hg.size()));
        MM_HIP(hipMemcpyAsync(dG.p, hg.data(), hg.size() * 8, hipMemcpyHostToDevice, st));
        for (int b = 0; b < B; ++b) {
            if (rb[b] == 0) continue;
            const int64_t nb = (oo[b + 1] - oo[b]) * ns;
            const dim3 g(grid_for(nb, 256, 4096), (rb[b] + 15) / 16);
            if (mixed)
                hipLaunchKernelGGL(k_ritz_vectors<float>, g, dim3(256), 0, st, basis, basis_stride,
                                   oo[b] * ns, nb, m[b], (const double*)dG.p + goff[b], rb[b],
                                   zd32.p + zoff[b]);
            else
                hipLaunchKernelGGL(k_ritz_vectors<double>, g, dim3(256), 0, st, basis,
                                   basis_stride, oo[b] * ns, nb, m[b],
                                   (const double*)dG.p + goff[b], rb[b], zd64.p + zoff[b]);
            MM_HIP(hipGetLastError());
        }
        MM_HIP(hipStreamSynchronize(st));
    }
    // AZ_D, one A application per column index over all problems
    {
        DBuf<int64_t> dzoff;
        DBuf<int32_t> lprob;
        DBuf<double> x, y;
        MM_TRY(dzoff.alloc(B + 1));
        MM_TRY(lprob.alloc((size_t)r_max * B));
        MM_TRY(x.alloc(nv));
        MM_TRY(y.alloc(nv));
        MM_HIP(hipMemcpyAsync(dzoff.p, zoff.data(), (B + 1) * 8, hipMemcpyHostToDevice, st));
        std::vector<int32_t> hp;
        std::vector<int32_t> lcnt(r_max, 0);
        for (int32_t k = 0; k < r_max; ++k)
            for (int b = 0; b < B; ++b)
                if (k < rb[b]) {
                    hp.push_back(b);
                    lcnt[k]++;
                }
        MM_HIP(hipMemcpyAsync(lprob.p, hp.data(), hp.size() * 4, hipMemcpyHostToDevice, st));
        int64_t nb_max = 1;
        for (int b = 0; b < B; ++b) nb_max = std::max<int64_t>(nb_max, (oo[b + 1] - oo[b]) * ns);
        const int sgx = (int)std::min<int64_t>(1024, (nb_max + 255) / 256);
        int64_t lo = 0;
        for (int32_t k = 0; k < r_max; ++k) {
            const dim3 g(sgx, lcnt[k]);
            MM_HIP(hipMemsetAsync(x.p, 0, nv * 8, st));
            if (mixed) {
                hipLaunchKernelGGL(k_zd_to_vec<float>, g, dim3(256), 0, st, lprob.p + lo,
                                   (const float*)zd32.p, pl->ooff.p, (int)ns,
                                   (const int64_t*)dzoff.p, k, x.p);
                MM_HIP(hipGetLastError());
                MM_TRY(apply_A32_sparse(pl, x.p, y.p));
                hipLaunchKernelGGL(k_store_az<float>, g, dim3(256), 0, st, lprob.p + lo,
                                   (const double*)y.p, pl->ooff.p, (int)ns,
                                   (const int64_t*)dzoff.p, k, az32.p);
            } else {
                hipLaunchKernelGGL(k_zd_to_vec<double>, g, dim3(256), 0, st, lprob.p + lo,
                                   (const double*)zd64.p, pl->ooff.p, (int)ns,
                                   (const int64_t*)dzoff.p, k, x.p);
                MM_HIP(hipGetLastError());
                MM_TRY(apply_A64_sparse(pl, x.p, y.p));
                hipLaunchKernelGGL(k_store_az<double>, g, dim3(256), 0, st, lprob.p + lo,
                                   (const double*)y.p, pl->ooff.p, (int)ns,
                                   (const int64_t*)dzoff.p, k, az64.p);
            }
            MM_HIP(hipGetLastError());
            lo += lcnt[k];
        }
        MM_HIP(hipStreamSynchronize(st));
    }
    // E_b = Z_b^T AZ_b, independent subset, E_b^-1
    int64_t npad_max = 4;
    for (int b = 0; b < B; ++b)
        npad_max = std::max<int64_t>(npad_max, ((oo[b + 1] - oo[b]) * ns + 3) / 4 * 4);
    const int32_t rp_max = (r_max + 15) / 16 * 16;
    std::vector<std::vector<int>> sels(B);
    std::vector<int32_t> col_off(B + 1, 0), cols;
    std::vector<int64_t> az_off(B + 1, 0), einv_off(B + 1, 0);
    std::vector<double> Eall, Einv_all, ritz;
    int32_t keep_max = 0;
    {
        DBuf<double> zr, azr, dE;
        MM_TRY(zr.alloc((size_t)npad_max * rp_max));
        MM_TRY(azr.alloc((size_t)npad_max * rp_max));
        MM_TRY(dE.alloc((size_t)rp_max * rp_max));
        for (int b = 0; b < B; ++b) {
            const int32_t r = rb[b];
            const int64_t nb = (oo[b + 1] - oo[b]) * ns;
            if (r > 0) {
                const int32_t rp = (r + 15) / 16 * 16;
                const int64_t npad = (nb + 3) / 4 * 4;
                MM_HIP(hipMemsetAsync(zr.p, 0, (size_t)npad * rp * 8, st));
                MM_HIP(hipMemsetAsync(azr.p, 0, (size_t)npad * rp * 8, st));
                const dim3 g(grid_for(nb, 64, 2048), (r + 63) / 64);
                if (mixed) {
                    hipLaunchKernelGGL(k_cols_to_rows<float>, g, dim3(256), 0, st,
                                       (const float*)zd32.p + zoff[b], nb, r, rp, zr.p);
                    hipLaunchKernelGGL(k_cols_to_rows<float>, g, dim3(256), 0, st,
                                       (const float*)az32.p + zoff[b], nb, r, rp, azr.p);
                } else {
                    hipLaunchKernelGGL(k_cols_to_rows<double>, g, dim3(256), 0, st,
                                       (const double*)zd64.p + zoff[b], nb, r, rp, zr.p);
                    hipLaunchKernelGGL(k_cols_to_rows<double>, g, dim3(256), 0, st,
                                       (const double*)az64.p + zoff[b], nb, r, rp, azr.p);
                }
                MM_HIP(hipGetLastError());
                MM_TRY(gemm_tn_f64(st, zr.p, azr.p, npad, rp, rp, dE.p));
                std::vector<double> Ep((size_t)rp * rp);
                MM_HIP(hipMemcpyAsync(Ep.data(), dE.p, Ep.size() * 8, hipMemcpyDeviceToHost, st));
                MM_HIP(hipStreamSynchronize(st));
                std::vector<double> E((size_t)r * r);
                for (int32_t i = 0; i < r; ++i)
                    for (int32_t j = 0; j < r; ++j)
                        E[(size_t)i * r + j] = 0.5 * (Ep[(size_t)i * rp + j] + Ep[(size_t)j * rp + i]);
                sels[b] = pivoted_cholesky_select(E, r, pl->opts.rank_tol);
                const int32_t k = (int32_t)sels[b].size();
                if (k == 0) {
                    set_error("coarse matrix E_D of problem %d is zero", b);
                    return MM_ERR_RANK;
                }
                std::vector<double> Es((size_t)k * k), Einv;
                for (int32_t i = 0; i < k; ++i)
                    for (int32_t j = 0; j < k; ++j)
                        Es[(size_t)i * k + j] = E[(size_t)sels[b][i] * r + sels[b][j]];
                if (!spd_inverse(Es, k, Einv)) {
                    set_error("coarse matrix E_D of problem %d not positive definite on the "
                              "selected columns", b);
                    return MM_ERR_RANK;
                }
                Eall.insert(Eall.end(), Es.begin(), Es.end());
                Einv_all.insert(Einv_all.end(), Einv.begin(), Einv.end());
                for (int32_t i = 0; i < k; ++i) {
                    cols.push_back(sels[b][i]);
                    ritz.push_back(theta[b][sels[b][i]]);
                }
                keep_max = std::max(keep_max, k);
            }
            const int32_t k = (int32_t)sels[b].size();
            col_off[b + 1] = col_off[b] + k;
            einv_off[b + 1] = einv_off[b] + (int64_t)k * k;
            az_off[b + 1] = az_off[b] + (int64_t)k * nb;
        }
    }
    const int32_t keff = col_off[B];
    // kept columns of Z_D and AZ_D into the final blocks
    DBuf<double> fz64, faz64;
    DBuf<float> fz32, faz32;
    {
        std::vector<int64_t> so(keff), d_o(keff), cn(keff);
        for (int b = 0; b < B; ++b) {
            const int64_t nb = (oo[b + 1] - oo[b]) * ns;
            for (size_t i = 0; i < sels[b].size(); ++i) {
                const int32_t a = col_off[b] + (int32_t)i;
                so[a] = zoff[b] + (int64_t)sels[b][i] * nb;
                d_o[a] = az_off[b] + (int64_t)i * nb;
                cn[a] = nb;
            }
        }
        DBuf<int64_t> dso, ddo, dcn;
        MM_TRY(dso.alloc(keff));
        MM_TRY(ddo.alloc(keff));
        MM_TRY(dcn.alloc(keff));
        MM_HIP(hipMemcpyAsync(dso.p, so.data(), keff * 8, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(ddo.p, d_o.data(), keff * 8, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(dcn.p, cn.data(), keff * 8, hipMemcpyHostToDevice, st));
        const dim3 g(64, keff);
        if (mixed) {
            MM_TRY(fz32.alloc((size_t)az_off[B]));
            MM_TRY(faz32.alloc((size_t)az_off[B]));
            hipLaunchKernelGGL(k_copy_cols<float>, g, dim3(256), 0, st, (const float*)zd32.p,
                               fz32.p, (const int64_t*)dso.p, (const int64_t*)ddo.p,
                               (const int64_t*)dcn.p, nullptr);
            hipLaunchKernelGGL(k_copy_cols<float>, g, dim3(256), 0, st, (const float*)az32.p,
                               faz32.p, (const int64_t*)dso.p, (const int64_t*)ddo.p,
                               (const int64_t*)dcn.p, nullptr);
        } else {
            MM_TRY(fz64.alloc((size_t)az_off[B]));
            MM_TRY(faz64.alloc((size_t)az_off[B]));
            hipLaunchKernelGGL(k_copy_cols<double>, g, dim3(256), 0, st, (const double*)zd64.p,
                               fz64.p, (const int64_t*)dso.p, (const int64_t*)ddo.p,
                               (const int64_t*)dcn.p, nullptr);
            hipLaunchKernelGGL(k_copy_cols<double>, g, dim3(256), 0, st, (const double*)az64.p,
                               faz64.p, (const int64_t*)dso.p, (const int64_t*)ddo.p,
                               (const int64_t*)dcn.p, nullptr);
        }
        MM_HIP(hipGetLastError());
        MM_HIP(hipStreamSynchronize(st));
    }
    // per-column tables; Z^T r goes through per-chunk partials (kZtChunk entries each)
    std::vector<int32_t> cprob(keff);
    std::vector<int64_t> choff(B + 1, 0);
    for (int b = 0; b < B; ++b) {
        const int64_t nb = (oo[b + 1] - oo[b]) * ns;
        choff[b + 1] = choff[b] + (nb + kZtChunk - 1) / kZtChunk;
        for (int32_t a = col_off[b]; a < col_off[b + 1]; ++a) cprob[a] = b;
    }
    DBuf<int64_t> d_choff;
    DBuf<double> d_cpart, d_cpart2;
    MM_TRY(d_choff.alloc(B + 1));
    MM_TRY(d_cpart.alloc((size_t)choff[B] * keep_max));
    MM_TRY(d_cpart2.alloc((size_t)choff[B] * keep_max));
    MM_HIP(hipMemcpyAsync(d_choff.p, choff.data(), (B + 1) * 8, hipMemcpyHostToDevice, st));
    DBuf<int32_t> d_cprob, d_coloff;
    DBuf<int64_t> d_azoff, d_einvoff;
    DBuf<double> d_einv, d_w, d_v;
    MM_TRY(d_cprob.alloc(keff));
    MM_TRY(d_coloff.alloc(B + 1));
    MM_TRY(d_azoff.alloc(B + 1));
    MM_TRY(d_einvoff.alloc(B + 1));
    MM_TRY(d_einv.alloc(Einv_all.size()));
    MM_TRY(d_w.alloc(keff));
    MM_TRY(d_v.alloc(keff));
    MM_HIP(hipMemcpyAsync(d_cprob.p, cprob.data(), keff * 4, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(d_coloff.p, col_off.data(), (B + 1) * 4, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(d_azoff.p, az_off.data(), (B + 1) * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(d_einvoff.p, einv_off.data(), (B + 1) * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(d_einv.p, Einv_all.data(), Einv_all.size() * 8, hipMemcpyHostToDevice,
                          st));
    MM_HIP(hipStreamSynchronize(st));
    // install (captured iterations hold the old coarse-space pointers)
    drop_graphs(pl);
    Coarse& co = pl->co;
    co.kind = 2;
    co.r_dedup = r_all;
    co.r_eff = keff;
    co.r_max = keep_max;
    co.cols = std::move(cols);
    co.ritz = std::move(ritz);
    co.h_col_off = col_off;
    co.h_az_off = az_off;
    co.h_einv_off = einv_off;
    co.E = std::move(Eall);
    co.col_off.swap(d_coloff);
    co.col_prob.swap(d_cprob);
    co.az_off.swap(d_azoff);
    co.einv_off.swap(d_einvoff);
    co.Einv.swap(d_einv);
    co.w.swap(d_w);
    co.v.swap(d_v);
    co.vslice.release();
    co.slice_col.release();
    co.vpart.release();
    co.n_slices = 0;
    co.ch_off.swap(d_choff);
    co.cpart.swap(d_cpart);
    co.cpart2.swap(d_cpart2);
    co.n_chunks = choff[B];
    co.AZ64.swap(faz64);
    co.AZ32.swap(faz32);
    co.AZ16.release();
    co.az16_off.release();
    co.az16_scale.release();
    co.ZD64.swap(fz64);
    co.ZD32.swap(fz32);
    co.csr_ptr.release();
    co.csr_col.release();
    co.csr_val.release();
    co.csc_beg.release();
    co.csc_end.release();
    co.csc_row.release();
    co.csc_val.release();
    pl->has_coarse = true;
    return MM_OK;
}

// the kept Z_D blocks in FP64 (the layout of AZ)
int coarse_dense_columns(mm_plan_t pl, double* out) {
    Coarse& co = pl->co;
    const int64_t n = co.h_az_off[pl->n_prob];
    hipStream_t st = pl->stream;
    if (co.ZD64.p) {
        MM_HIP(hipMemcpyAsync(out, co.ZD64.p, n * 8, hipMemcpyDeviceToDevice, st));
    } else {
        hipLaunchKernelGGL(k_f32_to_f64, dim3(grid_for(n)), dim3(256), 0, st,
                           (const float*)co.ZD32.p, out, n);
        MM_HIP(hipGetLastError());
    }
    MM_HIP(hipStreamSynchronize(st));
    return MM_OK;
}

namespace {

// w = E^-1 (Z^T r - (AZ)^T y) of the masked problems from the partials of the first
// stage: cz (Z_D chunk partials) or the Z_S slice partials, and caz ((AZ)^T y chunk
// partials) or none
int coarse_solve(mm_plan_t pl, const double* cz, const double* caz, const int* mask) {
    Coarse& co = pl->co;
    const int32_t k = co.r_eff;
    const dim3 g((unsigned)((k + 3) / 4)), t(256);
    hipLaunchKernelGGL(k_coarse_sums, g, t, 0, pl->stream, cz, (const double*)co.vpart.p,
                       (const int32_t*)co.vslice.p, caz, co.ch_off.p, co.col_off.p,
                       co.col_prob.p, co.n_chunks, k, co.v.p, mask);
    hipLaunchKernelGGL(k_coarse_einv, g, t, 0, pl->stream, co.Einv.p, co.einv_off.p,
                       co.col_off.p, co.col_prob.p, k, (const double*)co.v.p, co.w.p, mask);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int twolvl_apply_dense(mm_plan_t pl, const double* r, double* z, const PcgCtl& ctl) {
    Coarse& co = pl->co;
    hipStream_t st = pl->stream;
    const int ns = pl->n_s;
    const dim3 gc((unsigned)co.n_chunks, (unsigned)((co.r_max + kZtCols - 1) / kZtCols)),
        t256(256);
    if (co.ZD32.p)
        hipLaunchKernelGGL(k_ztr_chunks<float>, gc, t256, 0, st, (const float*)co.ZD32.p,
                           co.az_off.p, co.col_off.p, co.ch_off.p, pl->n_prob, pl->ooff.p, ns,
                           r, co.n_chunks, co.cpart.p, ctl.mask);
    else
        hipLaunchKernelGGL(k_ztr_chunks<double>, gc, t256, 0, st, (const double*)co.ZD64.p,
                           co.az_off.p, co.col_off.p, co.ch_off.p, pl->n_prob, pl->ooff.p, ns,
                           r, co.n_chunks, co.cpart.p, ctl.mask);
    MM_TRY(coarse_solve(pl, (const double*)co.cpart.p, nullptr, ctl.mask));
    const size_t shm = (size_t)co.r_max * sizeof(double);
    const dim3 g(pl->n_pblk), t(kVecThreads);
    const int64_t* np64 = nullptr;
    const int32_t* np32 = nullptr;
    const double* npd = nullptr;
    if (ns == 3) {
        if (co.AZ32.p)
            hipLaunchKernelGGL((k_2lvl<float, 3, true>), g, t, shm, st, r, z, pl->bj.p, co.AZ32.p,
                               co.az_off.p, co.col_off.p, co.w.p, np64, np32, npd,
                               (const float*)co.ZD32.p, ctl);
        else
            hipLaunchKernelGGL((k_2lvl<double, 3, true>), g, t, shm, st, r, z, pl->bj.p,
                               co.AZ64.p, co.az_off.p, co.col_off.p, co.w.p, np64, np32, npd,
                               (const double*)co.ZD64.p, ctl);
    } else {
        if (co.AZ32.p)
            hipLaunchKernelGGL((k_2lvl<float, 1, true>), g, t, shm, st, r, z, pl->bj.p, co.AZ32.p,
                               co.az_off.p, co.col_off.p, co.w.p, np64, np32, npd,
                               (const float*)co.ZD32.p, ctl);
        else
            hipLaunchKernelGGL((k_2lvl<double, 1, true>), g, t, shm, st, r, z, pl->bj.p,
                               co.AZ64.p, co.az_off.p, co.col_off.p, co.w.p, np64, np32, npd,
                               (const double*)co.ZD64.p, ctl);
    }
    MM_HIP(hipGetLastError());
    return MM_OK;
}

}  // namespace

int twolvl_apply(mm_plan_t pl, const double* r, double* z, const PcgCtl& ctl) {
    Coarse& co = pl->co;
    if (co.kind == 2) return twolvl_apply_dense(pl, r, z, ctl);
    hipStream_t st = pl->stream;
    const int32_t k = co.r_eff;
    hipLaunchKernelGGL(k_ztr, dim3((co.n_slices + 3) / 4), dim3(256), 0, st, co.csc_beg.p,
                       co.csc_end.p, co.csc_row.p, co.csc_val.p, r, pl->n_s, co.vslice.p,
                       co.slice_col.p, co.n_slices, co.col_prob.p, co.vpart.p, ctl.mask);
    hipLaunchKernelGGL(k_einv, dim3((k + 3) / 4), dim3(256), 0, st, co.Einv.p, co.einv_off.p,
                       co.col_off.p, co.col_prob.p, co.vpart.p, co.vslice.p, k, co.w.p, ctl.mask);
    const size_t shm = (size_t)co.r_max * sizeof(double);
    const dim3 g(pl->n_pblk), t(kVecThreads);
    if (co.AZ16.p) {
        if (pl->n_s == 3)
            hipLaunchKernelGGL((k_2lvl16<3>), g, t, 2 * shm, st, r, z, pl->bj.p, co.AZ16.p,
                               co.az16_off.p, co.az16_scale.p, co.col_off.p, co.w.p,
                               co.csr_ptr.p, co.csr_col.p, co.csr_val.p, ctl);
        else
            hipLaunchKernelGGL((k_2lvl16<1>), g, t, 2 * shm, st, r, z, pl->bj.p, co.AZ16.p,
                               co.az16_off.p, co.az16_scale.p, co.col_off.p, co.w.p,
                               co.csr_ptr.p, co.csr_col.p, co.csr_val.p, ctl);
        MM_HIP(hipGetLastError());
        return MM_OK;
    }
    if (pl->n_s == 3) {
        if (co.AZ32.p)
            hipLaunchKernelGGL((k_2lvl<float, 3, false>), g, t, shm, st, r, z, pl->bj.p, co.AZ32.p,
                               co.az_off.p, co.col_off.p, co.w.p, co.csr_ptr.p, co.csr_col.p,
                               co.csr_val.p, (const float*)nullptr, ctl);
        else
            hipLaunchKernelGGL((k_2lvl<double, 3, false>), g, t, shm, st, r, z, pl->bj.p, co.AZ64.p,
                               co.az_off.p, co.col_off.p, co.w.p, co.csr_ptr.p, co.csr_col.p,
                               co.csr_val.p, (const double*)nullptr, ctl);
    } else {
        if (co.AZ32.p)
            hipLaunchKernelGGL((k_2lvl<float, 1, false>), g, t, shm, st, r, z, pl->bj.p, co.AZ32.p,
                               co.az_off.p, co.col_off.p, co.w.p, co.csr_ptr.p, co.csr_col.p,
                               co.csr_val.p, (const float*)nullptr, ctl);
        else
            hipLaunchKernelGGL((k_2lvl<double, 1, false>), g, t, shm, st, r, z, pl->bj.p, co.AZ64.p,
                               co.az_off.p, co.col_off.p, co.w.p, co.csr_ptr.p, co.csr_col.p,
                               co.csr_val.p, (const double*)nullptr, ctl);
    }
    MM_HIP(hipGetLastError());
    return MM_OK;
}

namespace {

template <typename TA>
const TA* az_blocks(const Coarse& co);
template <>
const float* az_blocks<float>(const Coarse& co) { return co.AZ32.p; }
template <>
const double* az_blocks<double>(const Coarse& co) { return co.AZ64.p; }
template <typename TA>
const TA* z_blocks(const Coarse& co);
template <>
const float* z_blocks<float>(const Coarse& co) { return co.ZD32.p; }
template <>
const double* z_blocks<double>(const Coarse& co) { return co.ZD64.p; }

// chunk partials of X^T v for dense blocks X laid out like AZ
template <typename TA>
int chunk_partials(mm_plan_t pl, const TA* X, const double* v, double* out, const int* mask) {
    const Coarse& co = pl->co;
    hipLaunchKernelGGL(k_ztr_chunks<TA>,
                       dim3((unsigned)co.n_chunks, (unsigned)((co.r_max + kZtCols - 1) / kZtCols)),
                       dim3(256), 0, pl->stream, X, co.az_off.p, co.col_off.p, co.ch_off.p,
                       pl->n_prob, pl->ooff.p, pl->n_s, v, co.n_chunks, out, mask);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

// w = E^-1 (Z^T r - (AZ)^T y) per masked problem (the second term only when y is given)
int coarse_w(mm_plan_t pl, const double* r, const double* y, const int* mask) {
    Coarse& co = pl->co;
    hipStream_t st = pl->stream;
    const bool f32 = co.AZ32.p != nullptr;
    if (co.kind == 2) {
        MM_TRY(f32 ? chunk_partials<float>(pl, co.ZD32.p, r, co.cpart.p, mask)
                   : chunk_partials<double>(pl, co.ZD64.p, r, co.cpart.p, mask));
    } else {
        hipLaunchKernelGGL(k_ztr, dim3((co.n_slices + 3) / 4), dim3(256), 0, st, co.csc_beg.p,
                           co.csc_end.p, co.csc_row.p, co.csc_val.p, r, pl->n_s, co.vslice.p,
                           co.slice_col.p, co.n_slices, co.col_prob.p, co.vpart.p, mask);
        MM_HIP(hipGetLastError());
    }
    if (y)
        MM_TRY(f32 ? chunk_partials<float>(pl, co.AZ32.p, y, co.cpart2.p, mask)
                   : chunk_partials<double>(pl, co.AZ64.p, y, co.cpart2.p, mask));
    MM_TRY(coarse_solve(pl, co.kind == 2 ? (const double*)co.cpart.p : nullptr,
                        y ? (const double*)co.cpart2.p : nullptr, mask));
    MM_HIP(hipGetLastError());
    return MM_OK;
}

template <typename TA, int NS, bool DZ>
int adef2_finish_t(mm_plan_t pl, const double* r, double* z, const PcgCtl& ctl) {
    const Coarse& co = pl->co;
    const TA* zd = DZ ? z_blocks<TA>(co) : nullptr;
    hipLaunchKernelGGL((k_adef2_finish<TA, NS, DZ>), dim3(pl->n_pblk), dim3(kVecThreads),
                       (size_t)co.r_max * sizeof(double), pl->stream, r, z, zd, co.az_off.p,
                       co.col_off.p, co.w.p, co.csr_ptr.p, co.csr_col.p, co.csr_val.p, ctl);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

template <typename TA, int NS, bool DZ>
int coarse_correct_t(mm_plan_t pl, double* x, double* r, const PcgCtl& ctl) {
    const Coarse& co = pl->co;
    const TA* zd = DZ ? z_blocks<TA>(co) : nullptr;
    hipLaunchKernelGGL((k_coarse_correct<TA, NS, DZ>), dim3(pl->n_pblk), dim3(kVecThreads),
                       (size_t)co.r_max * sizeof(double), pl->stream, x, r, az_blocks<TA>(co), zd,
                       co.az_off.p, co.col_off.p, co.w.p, co.csr_ptr.p, co.csr_col.p,
                       co.csr_val.p, ctl);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

// instantiation for the plan's AZ precision, Stokes count and kind of Z
template <template <typename, int, bool> class K, typename... Args>
int by_layout(mm_plan_t pl, Args... args) {
    const bool f = pl->co.AZ32.p != nullptr, d = pl->co.kind == 2;
    if (pl->n_s == 3) {
        if (f) return d ? K<float, 3, true>::run(pl, args...) : K<float, 3, false>::run(pl, args...);
        return d ? K<double, 3, true>::run(pl, args...) : K<double, 3, false>::run(pl, args...);
    }
    if (f) return d ? K<float, 1, true>::run(pl, args...) : K<float, 1, false>::run(pl, args...);
    return d ? K<double, 1, true>::run(pl, args...) : K<double, 1, false>::run(pl, args...);
}
template <typename TA, int NS, bool DZ>
struct Adef2Finish {
    static int run(mm_plan_t pl, const double* r, double* z, PcgCtl ctl) {
        return adef2_finish_t<TA, NS, DZ>(pl, r, z, ctl);
    }
};
template <typename TA, int NS, bool DZ>
struct CoarseCorrect {
    static int run(mm_plan_t pl, double* x, double* r, PcgCtl ctl) {
        return coarse_correct_t<TA, NS, DZ>(pl, x, r, ctl);
    }
};

}  // namespace

// A-DEF2 [App. B, eq. ADEF2]: z = R^T M_BD r + Z E^-1 Z^T r = y + Z E^-1 (Z^T r - (AZ)^T y),
// y = M_BD r (R^T = I - Z E^-1 (AZ)^T, A and E symmetric); partials of r^T z as ctl asks
int adef2_apply(mm_plan_t pl, const double* r, double* z, const PcgCtl& ctl) {
    PcgCtl c0 = ctl;
    c0.part = nullptr;
    MM_TRY(bj_apply(pl, r, z, c0));  // y in z
    MM_TRY(coarse_w(pl, r, z, ctl.mask));
    return by_layout<Adef2Finish>(pl, r, z, ctl);
}

// the A-DEF2 initial guess [App. B]: w = E^-1 Z^T r, x += Z w, r -= AZ w for the problems
// in mask (nullptr: all; r = b - A x on entry), after which Z^T r = 0
int coarse_start(mm_plan_t pl, double* x, double* r, const int* mask) {
    PcgCtl c = batch_ctl(pl);
    c.part = nullptr;
    c.mask = mask;
    MM_TRY(coarse_w(pl, r, nullptr, mask));
    return by_layout<CoarseCorrect>(pl, x, r, c);
}

}  // namespace mm

extern "C" int mm_gemm_tn_f64_noalloc(void* stream, const double* A, const double* B, int64_t n,
                                      int32_t ra, int32_t rb, double* C) {
    mm::clear_error();
    if (!A || !B || !C || n < 4 || n % 4 || ra < 16 || rb < 16 || ra % 16 || rb % 16) {
        mm::set_error("mm_gemm_tn_f64_noalloc: n must be a positive multiple of 4, ra and rb "
                      "multiples of 16");
        return MM_ERR_ARG;
    }
    return mm::gemm_tn_f64_noalloc((hipStream_t)stream, A, B, n, ra, rb, C);
}
