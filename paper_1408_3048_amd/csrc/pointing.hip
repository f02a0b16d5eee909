// Pointing P^T (deterministic segmented reduction over pixel-sorted samples),
// de-pointing P (time-ordered gather), and the block-Jacobi preconditioner
// M_BD = (P^T diag(N^-1) P)^-1 [Sect. 3.1, eq. stdPrec].
#include <cfloat>
#include <map>
#include <mutex>
#include <vector>

#include "mm_device.h"

namespace mm {
namespace {

// Wave-level segmented reduction over pixel-sorted samples.
//
// A wave owns the sorted samples [i0, i1) of whole pixels p0, p0+1, ... and walks
// them in chunks of 64*E samples aligned to E: lane l holds samples c + E l + e
// (e < E), loaded with aligned vector loads so E gathers are in flight per lane.
// Each lane first sums its own samples segment by segment, then one segmented
// inclusive scan over the 64 lane summaries (flag: the lane holds a segment
// start) gives every lane the partial sum entering it; the sample at a pixel's
// last position emits the pixel total.  A segment left open at the end of a
// chunk carries its sum into the next chunk.  The order of additions is fixed by
// the plan, so results are deterministic; samples outside [i0, i1) are zeros.
// `load(base, valid, v)` fills v[e][.] for the E samples; `emit(pixel, val)`.
template <typename T, int NV, int E, class Load, class Emit>
__device__ __forceinline__ void seg_reduce(int64_t i0, int64_t i1, int64_t p0,
                                           const unsigned long long* __restrict__ heads,
                                           Load&& load, Emit&& emit) {
    static_assert(64 % E == 0, "E must divide 64");
    const int lane = threadIdx.x & 63;
    T carry[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) carry[q] = (T)0;
    int64_t pprev = p0 - 1;
    for (int64_t c = i0 & ~(int64_t)(E - 1); c < i1; c += 64 * E) {
        const int64_t base = c + (int64_t)E * lane;
        bool valid[E];
#pragma unroll
        for (int e = 0; e < E; ++e) valid[e] = base + e >= i0 && base + e < i1;
        // segment-start words of the lane's samples and of the sample after them, loaded
        // unconditionally (a valid word for lanes past the range) ahead of the samples, so
        // that a chunk's loads are in flight together; their bits are read after load()
        const int64_t inext = base + E;
        const unsigned long long hw = heads[(base < i1 ? base : i0) >> 6];
        const unsigned long long hn = heads[(inext < i1 ? inext : i0) >> 6];
        T v[E][NV];
        load(base, valid, v);
        uint32_t hb = base < i1 ? (uint32_t)(hw >> (base & 63)) & ((1u << E) - 1u) : 0u;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (!valid[e]) hb &= ~(1u << e);
        // lane-local segmented prefix sums
        T sl[E][NV];
        T run[NV];
        bool seen[E];
        bool any = false;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const bool h = (hb >> e) & 1u;
#pragma unroll
            for (int q = 0; q < NV; ++q) run[q] = (e == 0 || h) ? v[e][q] : run[q] + v[e][q];
            any = any || h;
            seen[e] = any;
#pragma unroll
            for (int q = 0; q < NV; ++q) sl[e][q] = run[q];
        }
        // segmented inclusive scan over lanes of (any, run)
        T acc[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] = run[q];
        int f = any ? 1 : 0;
        int hc = __popc(hb), hcs = hc;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            T u[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) u[q] = __shfl_up(acc[q], d);
            const int fu = __shfl_up(f, d);
            const int cu = __shfl_up(hcs, d);
            if (lane >= d) {
                if (!f) {
#pragma unroll
                    for (int q = 0; q < NV; ++q) acc[q] += u[q];
                }
                f |= fu;
                hcs += cu;
            }
        }
        // partial sum entering this lane (from earlier lanes and the previous chunk)
        T pre[NV];
        int fex = __shfl_up(f, 1);
#pragma unroll
        for (int q = 0; q < NV; ++q) pre[q] = __shfl_up(acc[q], 1);
        if (lane == 0) {
            fex = 0;
#pragma unroll
            for (int q = 0; q < NV; ++q) pre[q] = (T)0;
        }
        if (!fex) {
#pragma unroll
            for (int q = 0; q < NV; ++q) pre[q] += carry[q];
        }
        // segment ends and totals
        const bool next_head_last =
            valid[E - 1] && inext < i1 && ((hn >> (inext & 63)) & 1ull) != 0;
        int64_t pix = pprev + (hcs - hc);
        T last[NV];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if ((hb >> e) & 1u) ++pix;
            T tot[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) tot[q] = seen[e] ? sl[e][q] : sl[e][q] + pre[q];
            const int64_t i = base + e;
            bool end = false;
            if (valid[e]) {
                if (i + 1 == i1) end = true;
                else if (e < E - 1) end = (hb >> (e + 1)) & 1u;
                else end = next_head_last;
            }
            if (end) emit(pix, tot);
            if (e == E - 1) {
#pragma unroll
                for (int q = 0; q < NV; ++q) last[q] = (valid[e] && !end) ? tot[q] : (T)0;
            }
        }
#pragma unroll
        for (int q = 0; q < NV; ++q) carry[q] = __shfl(last[q], 63);
        pprev += __shfl(hcs, 63);
    }
}

// Loads of the sorted pointing (sample indices and weights), which P^T streams once per
// application, marked non-temporal: they then do not displace from the caches the vectors
// and A Z columns that the next kernels of an iteration read again (P^T of the 2^24-sample
// raster 60.7 -> 58.7 us, its mixed two-level solve 19.25 -> 18.90 ms)
typedef float stream_f4 __attribute__((ext_vector_type(4)));
typedef double stream_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int32_t ld_stream(const int32_t* p) {
    return __builtin_nontemporal_load(p);
}
__device__ __forceinline__ float4 ld_stream4(const float* p) {
    const stream_f4 v = __builtin_nontemporal_load(reinterpret_cast<const stream_f4*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double2 ld_stream2(const double* p) {
    const stream_d2 v = __builtin_nontemporal_load(reinterpret_cast<const stream_d2*>(p));
    return make_double2(v.x, v.y);
}

// LDS exchange among the lanes of one wave: orders the wave's LDS writes before its reads
// (a wave's LDS instructions execute in order; this keeps the compiler from moving them)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// x[p, s] = sum_{t in p} W[t, s] z_t (P^T), E samples per lane (a multiple of 4).  The z
// gather of a chunk of 64 E sorted samples is issued lane-strided (one instruction covers
// 64 consecutive sorted samples, i.e. a few runs of consecutive time samples, so few cache
// lines) and handed to the lane layout of the segmented reduction (E consecutive samples
// per lane) through LDS; the additions are unchanged.
template <typename T, int NS, int E>
__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ perm,
                                                 const T* __restrict__ ws, const T* __restrict__ z,
                                                 const unsigned long long* __restrict__ heads,
                                                 const int32_t* __restrict__ wave_pix,
                                                 const int64_t* __restrict__ seg,
                                                 const int32_t* __restrict__ hits, int64_t n_waves,
                                                 double* __restrict__ out,
                                                 const int* __restrict__ mask,
                                                 const int32_t* __restrict__ wave_prob) {
    static_assert(E % 4 == 0, "E must be a multiple of 4");
    __shared__ __align__(16) T zx[4][64 * E];
    // the blocks of one XCD take a contiguous range of waves (neighbouring pixels share the
    // time samples whose z they gather)
    const int64_t blk = xcd_item(blockIdx.x, (n_waves + 3) / 4);
    if (blk < 0) return;
    const int64_t w = blk * 4 + (threadIdx.x >> 6);
    if (w >= n_waves) return;
    if (mask && !mask[wave_prob[w]]) return;
    const int32_t p0 = wave_pix[w], p1 = wave_pix[w + 1];
    if (p0 >= p1) return;
    const int64_t i0 = seg[p0];
    const int64_t i1 = seg[p1 - 1] + hits[p1 - 1];
    const int lane = threadIdx.x & 63;
    T* zw = zx[threadIdx.x >> 6];
    // sample indices of the next chunk, loaded one chunk ahead (-1 outside [i0, i1)).  The
    // loads here and the z gathers below are unconditional, from a valid address for lanes
    // outside the range (sorted position i0, sample 0), with the value selected afterwards:
    // guarded loads become one branch each, and the compiler then waits for every load
    // before issuing the next.
    int32_t pf[E];
    auto fetch = [&](int64_t c) {
#pragma unroll
        for (int g = 0; g < E; ++g) {
            const int64_t i = c + lane + 64 * g;
            const bool in = i >= i0 && i < i1;
            const int32_t t = ld_stream(perm + (in ? i : i0));
            pf[g] = in ? t : -1;
        }
    };
    fetch(i0 & ~(int64_t)(E - 1));
    auto load = [&](int64_t base, const bool* valid, T (*v)[NS]) {
        // the sorted weights are loaded first, so their latency overlaps the z gather's
        // (loads after the exchange below would wait for it); lanes past the range skip them
        T wv[2 * E];
        if constexpr (NS == 3) {
            if (base < i1) {
                if constexpr (sizeof(T) == 4) {
#pragma unroll
                    for (int g = 0; g < E / 2; ++g) {
                        const float4 a = ld_stream4(ws + 2 * base + 4 * g);
                        wv[4 * g] = a.x;
                        wv[4 * g + 1] = a.y;
                        wv[4 * g + 2] = a.z;
                        wv[4 * g + 3] = a.w;
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const double2 a = ld_stream2(ws + 2 * (base + e));
                        wv[2 * e] = a.x;
                        wv[2 * e + 1] = a.y;
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < 2 * E; ++e) wv[e] = (T)0;
            }
        }
        // every lane takes part in the exchange, also lanes past the range
        const int64_t c = base - (int64_t)E * lane;
        int32_t tc[E];
#pragma unroll
        for (int g = 0; g < E; ++g) tc[g] = pf[g];
        fetch(c + 64 * E);
        T zg[E];
#pragma unroll
        for (int g = 0; g < E; ++g) zg[g] = z[tc[g] >= 0 ? tc[g] : 0];
#pragma unroll
        for (int g = 0; g < E; ++g) zw[lane + 64 * g] = tc[g] >= 0 ? zg[g] : (T)0;
        wave_lds_sync();
        T zz[E];
#pragma unroll
        for (int e = 0; e < E; ++e) zz[e] = zw[E * lane + e];
        wave_lds_sync();  // the next chunk's writes come after these reads
        if (base >= i1) {  // whole lane past the range
#pragma unroll
            for (int e = 0; e < E; ++e)
#pragma unroll
                for (int q = 0; q < NS; ++q) v[e][q] = (T)0;
            return;
        }
#pragma unroll
        for (int e = 0; e < E; ++e) zz[e] = valid[e] ? zz[e] : (T)0;
        if constexpr (NS == 3) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                v[e][0] = zz[e];
                v[e][1] = wv[2 * e] * zz[e];
                v[e][2] = wv[2 * e + 1] * zz[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e][0] = zz[e];
        }
    };
    auto emit = [&](int64_t pix, const T* tot) {
#pragma unroll
        for (int q = 0; q < NS; ++q) out[pix * NS + q] = (double)tot[q];
    };
    seg_reduce<T, NS, E>(i0, i1, p0, heads, load, emit);
}

// P^T of NC FP32 time streams z + k zstride (k < NC), the A Z columns of the coarse space
// several layers at a time: the sorted indices, weights and segment heads of a chunk are
// loaded once for all, the gathers of a sample are issued together, the segmented
// reduction is that of k_scatter (the same additions in the same order for each stream),
// and the pixel sums go to columns k0 + k of the pixel's problem block in az (where the
// problem has them; streams past nc are not read).
template <int NS, int E, int NC>
__global__ __launch_bounds__(256) void k_scatter_cols(
    const int32_t* __restrict__ perm, const float* __restrict__ ws, const float* __restrict__ z,
    int64_t zstride, int nc, const unsigned long long* __restrict__ heads,
    const int32_t* __restrict__ wave_pix, const int64_t* __restrict__ seg,
    const int32_t* __restrict__ hits, int64_t n_waves, const int32_t* __restrict__ wave_prob,
    const int64_t* __restrict__ ooff, const int32_t* __restrict__ ncols,
    const int64_t* __restrict__ blk_off, int k0, float* __restrict__ az) {
    static_assert(E % 4 == 0, "E must be a multiple of 4");
    constexpr int NV = NC * NS;
    __shared__ __align__(16) float zx[4][NC][64 * E];
    const int64_t blk = xcd_item(blockIdx.x, (n_waves + 3) / 4);
    if (blk < 0) return;
    const int64_t w = blk * 4 + (threadIdx.x >> 6);
    if (w >= n_waves) return;
    const int b = wave_prob[w];
    int ncb = ncols[b] - k0;  // columns this problem has in the group
    ncb = ncb < nc ? ncb : nc;
    if (ncb <= 0) return;
    const int32_t p0 = wave_pix[w], p1 = wave_pix[w + 1];
    if (p0 >= p1) return;
    const int64_t q0 = ooff[b], n_vec = (ooff[b + 1] - q0) * NS;
    float* const azb = az + blk_off[b] + (int64_t)k0 * n_vec - q0 * NS;  // pixel q0 at 0
    const int64_t i0 = seg[p0];
    const int64_t i1 = seg[p1 - 1] + hits[p1 - 1];
    const int lane = threadIdx.x & 63;
    float (*zw)[64 * E] = zx[threadIdx.x >> 6];
    int32_t pf[E];
    auto fetch = [&](int64_t c) {
#pragma unroll
        for (int g = 0; g < E; ++g) {
            const int64_t i = c + lane + 64 * g;
            const bool in = i >= i0 && i < i1;
            const int32_t t = ld_stream(perm + (in ? i : i0));
            pf[g] = in ? t : -1;
        }
    };
    fetch(i0 & ~(int64_t)(E - 1));
    auto load = [&](int64_t base, const bool* valid, float (*v)[NV]) {
        float wv[2 * E];
        if constexpr (NS == 3) {
            if (base < i1) {
#pragma unroll
                for (int g = 0; g < E / 2; ++g) {
                    const float4 a = ld_stream4(ws + 2 * base + 4 * g);
                    wv[4 * g] = a.x;
                    wv[4 * g + 1] = a.y;
                    wv[4 * g + 2] = a.z;
                    wv[4 * g + 3] = a.w;
                }
            } else {
#pragma unroll
                for (int e = 0; e < 2 * E; ++e) wv[e] = 0.0f;
            }
        }
        const int64_t c = base - (int64_t)E * lane;
        int32_t tc[E];
#pragma unroll
        for (int g = 0; g < E; ++g) tc[g] = pf[g];
        fetch(c + 64 * E);
        // streams past nc load stream 0 (unconditional loads; never written out)
        float zg[NC][E];
#pragma unroll
        for (int k = 0; k < NC; ++k)
#pragma unroll
            for (int g = 0; g < E; ++g)
                zg[k][g] = z[(k < nc ? k : 0) * zstride + (tc[g] >= 0 ? tc[g] : 0)];
#pragma unroll
        for (int k = 0; k < NC; ++k)
#pragma unroll
            for (int g = 0; g < E; ++g) zw[k][lane + 64 * g] = tc[g] >= 0 ? zg[k][g] : 0.0f;
        wave_lds_sync();
        float zz[NC][E];
#pragma unroll
        for (int k = 0; k < NC; ++k)
#pragma unroll
            for (int e = 0; e < E; ++e) zz[k][e] = zw[k][E * lane + e];
        wave_lds_sync();
        if (base >= i1) {
#pragma unroll
            for (int e = 0; e < E; ++e)
#pragma unroll
                for (int q = 0; q < NV; ++q) v[e][q] = 0.0f;
            return;
        }
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const float zk = valid[e] ? zz[k][e] : 0.0f;
                if constexpr (NS == 3) {
                    v[e][3 * k] = zk;
                    v[e][3 * k + 1] = wv[2 * e] * zk;
                    v[e][3 * k + 2] = wv[2 * e + 1] * zk;
                } else {
                    v[e][k] = zk;
                }
            }
    };
    auto emit = [&](int64_t pix, const float* tot) {
        float* dst = azb + pix * NS;
#pragma unroll
        for (int k = 0; k < NC; ++k)
            if (k < ncb) {
#pragma unroll
                for (int q = 0; q < NS; ++q) dst[k * n_vec + q] = tot[NS * k + q];
            }
    };
    seg_reduce<float, NV, E>(i0, i1, p0, heads, load, emit);
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

// B_p = sum_{t in p} t_0^{(j(t))} W_t W_t^T (P^T diag(N^-1) P), accumulated in FP64 with
// the segmented reduction of P^T; the lane at a pixel's last sample inverts the block
// and tests its reciprocal 1-norm condition number.  bad[0] receives the smallest
// failing pixel.
template <int NV>
__global__ __launch_bounds__(256) void k_bj_build(
    const int32_t* __restrict__ perm, const double* __restrict__ ws,
    const unsigned long long* __restrict__ heads, const int32_t* __restrict__ wave_pix,
    const int64_t* __restrict__ seg, const int32_t* __restrict__ hits, int64_t n_waves,
    const int64_t* __restrict__ int_lo,
    int32_t n_int, const int32_t* __restrict__ int_kern, const double* __restrict__ t0,
    double rcond_min, double* __restrict__ bj, int* __restrict__ bad, double* __restrict__ rc_out) {
    constexpr int E = 4;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= n_waves) return;
    const int32_t p0 = wave_pix[w], p1 = wave_pix[w + 1];
    if (p0 >= p1) return;
    // a pixel's sorted samples come in time-ordered runs within one interval: the lane keeps
    // the interval [jlo, jhi) and t_0 of its last sample and searches only outside it
    int64_t jlo = 0, jhi = 0;
    double dj = 0.0;
    const int64_t s0 = seg[p0];  // a valid sorted position for the unconditional loads
    auto load = [&](int64_t base, const bool* valid, double (*v)[NV]) {
        int64_t tt[E];
        double wa[E], wb[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t ic = valid[e] ? base + e : s0;
            tt[e] = perm[ic];
            if constexpr (NV == 6) {
                wa[e] = ws[2 * ic];
                wb[e] = ws[2 * ic + 1];
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (!valid[e]) {
#pragma unroll
                for (int q = 0; q < NV; ++q) v[e][q] = 0.0;
                continue;
            }
            const int64_t t = tt[e];
            if (t < jlo || t >= jhi) {
                const int32_t j = interval_of(int_lo, n_int, t);
                jlo = int_lo[j];
                jhi = j + 1 < n_int ? int_lo[j + 1] : INT64_MAX;
                dj = t0[int_kern[j]];
            }
            const double d = dj;
            if constexpr (NV == 6) {
                const double a = wa[e], b = wb[e];
                v[e][0] = d;
                v[e][1] = d * a;
                v[e][2] = d * b;
                v[e][3] = d * a * a;
                v[e][4] = d * a * b;
                v[e][5] = d * b * b;
            } else {
                v[e][0] = d;
            }
        }
    };
    auto emit = [&](int64_t c, const double* B) {
        double rc;
        if constexpr (NV == 1) {
            bj[c] = 1.0 / B[0];
            rc = B[0] > 0.0 ? 1.0 : 0.0;
        } else {
            const double b00 = B[0], b01 = B[1], b02 = B[2], b11 = B[3], b12 = B[4], b22 = B[5];
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
    };
    seg_reduce<double, NV, E>(seg[p0], seg[p1 - 1] + hits[p1 - 1], p0, heads, load, emit);
}

// z = M_BD r per pixel of every masked problem (+ partials of r^T z for the PCG)
template <int NS>
__global__ __launch_bounds__(kVecThreads) void k_bj_apply(const double* __restrict__ r,
                                                          double* __restrict__ z,
                                                          const double* __restrict__ bj,
                                                          PcgCtl ctl) {
    __shared__ double red[kVecThreads];
    const VecBlock vb = vec_block(ctl, NS, false);
    if (ctl.mask && !ctl.mask[vb.b]) return;
    double acc = 0.0;
    for (int64_t q = (int64_t)vb.k * kVecThreads + threadIdx.x; q < vb.n;
         q += vb.stride) {
        const int64_t c = vb.base + q;
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
    if (ctl.part) write_partial_at(acc, slot_part(ctl, kSlotRZ, vb.b), vb.k, red);
}

inline int grid_for(int64_t n, int threads = 256, int cap = 65536) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

template <typename T>
int scatter_t(mm_plan_t pl, const T* z, const T* ws, double* x, const int* mask) {
    const int64_t nb = (pl->n_waves + 3) / 4;
    if (nb == 0) return MM_OK;
    // 4 samples per lane: 8 gathers more per lane cost the residency they would add
    constexpr int E = 4;
    if (pl->n_s == 3)
        hipLaunchKernelGGL((k_scatter<T, 3, E>), dim3(xcd_grid(nb)), dim3(256), 0, pl->stream, pl->perm.p, ws,
                           z, (const unsigned long long*)pl->heads.p, pl->wave_pix.p, pl->seg.p,
                           pl->hits.p, pl->n_waves, x, mask, pl->wave_prob.p);
    else
        hipLaunchKernelGGL((k_scatter<T, 1, E>), dim3(xcd_grid(nb)), dim3(256), 0, pl->stream, pl->perm.p, ws,
                           z, (const unsigned long long*)pl->heads.p, pl->wave_pix.p, pl->seg.p,
                           pl->hits.p, pl->n_waves, x, mask, pl->wave_prob.p);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

}  // namespace

int scatter_cols32(mm_plan_t pl, const float* z, int64_t zstride, int nc, int k0,
                   const int32_t* ncols, const int64_t* blk_off, float* az) {
    if (nc < 1 || nc > kScatterCols) {
        set_error("scatter_cols32: %d streams (1..%d)", nc, kScatterCols);
        return MM_ERR_ARG;
    }
    const int64_t nb = (pl->n_waves + 3) / 4;
    if (nb == 0) return MM_OK;
    constexpr int E = 4;  // the lane layout of scatter32: the same additions
    if (pl->n_s == 3)
        hipLaunchKernelGGL((k_scatter_cols<3, E, kScatterCols>), dim3(xcd_grid(nb)), dim3(256), 0,
                           pl->stream, pl->perm.p, pl->ws32.p, z, zstride, nc,
                           (const unsigned long long*)pl->heads.p, pl->wave_pix.p, pl->seg.p,
                           pl->hits.p, pl->n_waves, pl->wave_prob.p, pl->ooff.p, ncols, blk_off,
                           k0, az);
    else
        hipLaunchKernelGGL((k_scatter_cols<1, E, kScatterCols>), dim3(xcd_grid(nb)), dim3(256), 0,
                           pl->stream, pl->perm.p, pl->ws32.p, z, zstride, nc,
                           (const unsigned long long*)pl->heads.p, pl->wave_pix.p, pl->seg.p,
                           pl->hits.p, pl->n_waves, pl->wave_prob.p, pl->ooff.p, ncols, blk_off,
                           k0, az);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int scatter64(mm_plan_t pl, const double* z, double* x, const int* mask) {
    return scatter_t<double>(pl, z, pl->ws64.p, x, mask);
}

int scatter32(mm_plan_t pl, const float* z, double* x, const int* mask) {
    return scatter_t<float>(pl, z, pl->ws32.p, x, mask);
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
    const int64_t nb = (pl->n_waves + 3) / 4;
    if (pl->n_s == 3)
        hipLaunchKernelGGL(k_bj_build<6>, dim3(nb), dim3(256), 0, st, pl->perm.p, pl->ws64.p,
                           (const unsigned long long*)pl->heads.p, pl->wave_pix.p, pl->seg.p,
                           pl->hits.p, pl->n_waves, pl->int_lo.p, pl->n_int, pl->int_kern.p,
                           pl->kern_t0.p,
                           pl->opts.rcond_min, pl->bj.p, bad.p, rc.p);
    else
        hipLaunchKernelGGL(k_bj_build<1>, dim3(nb), dim3(256), 0, st, pl->perm.p, pl->ws64.p,
                           (const unsigned long long*)pl->heads.p, pl->wave_pix.p, pl->seg.p,
                           pl->hits.p, pl->n_waves, pl->int_lo.p, pl->n_int, pl->int_kern.p,
                           pl->kern_t0.p,
                           pl->opts.rcond_min, pl->bj.p, bad.p, rc.p);
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
        hipLaunchKernelGGL(k_bj_apply<3>, dim3(pl->n_pblk), dim3(kVecThreads), 0, pl->stream, r, z,
                           pl->bj.p, ctl);
    else
        hipLaunchKernelGGL(k_bj_apply<1>, dim3(pl->n_pblk), dim3(kVecThreads), 0, pl->stream, r, z,
                           pl->bj.p, ctl);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

namespace {
std::mutex g_pt_mu;
std::map<std::vector<int64_t>, int64_t> g_pt_cache;
}  // namespace

// The P^T work range of the plan's operator (FP32 for mixed plans, else FP64): each of
// 512, 1024, 2048 and 4096 samples per range timed over five launches on a nonzero TOD
// (after one untimed launch), the fastest kept; cached per process for the same scan shape.
int tune_pt_range(mm_plan_t pl) {
    const bool f32 = pl->opts.precision == MM_MIXED;
    std::vector<int64_t> key = {pl->n_t, pl->n_obs, pl->n_s, pl->n_prob, f32 ? 1 : 0};
    for (int32_t j = 0; j < pl->n_int; ++j) key.push_back(pl->h_off[j + 1] - pl->h_off[j]);
    {
        std::lock_guard<std::mutex> lk(g_pt_mu);
        auto it = g_pt_cache.find(key);
        if (it != g_pt_cache.end()) return build_wave_ranges(pl, it->second);
    }
    hipStream_t st = pl->stream;
    DBuf<unsigned char> z;
    DBuf<double> x;
    MM_TRY(z.alloc((size_t)pl->n_t * (f32 ? 4 : 8)));
    MM_TRY(x.alloc((size_t)pl->n_obs * pl->n_s));
    MM_HIP(hipMemsetAsync(z.p, 0x3f, z.n, st));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MM_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        set_error("hipEventCreate failed");
        return MM_ERR_DEVICE;
    }
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{e0, e1};
    auto run = [&]() {
        return f32 ? scatter32(pl, (const float*)z.p, x.p, nullptr)
                   : scatter64(pl, (const double*)z.p, x.p, nullptr);
    };
    int64_t best = 0;
    float best_ms = 0.0f;
    for (const int64_t cand : {512, 1024, 2048, 4096}) {
        MM_TRY(build_wave_ranges(pl, cand));
        MM_TRY(run());
        MM_HIP(hipEventRecord(e0, st));
        for (int k = 0; k < 5; ++k) MM_TRY(run());
        MM_HIP(hipEventRecord(e1, st));
        MM_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        MM_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (best == 0 || ms < best_ms) {
            best = cand;
            best_ms = ms;
        }
    }
    MM_TRY(build_wave_ranges(pl, best));
    std::lock_guard<std::mutex> lk(g_pt_mu);
    g_pt_cache[key] = best;
    return MM_OK;
}

}  // namespace mm
