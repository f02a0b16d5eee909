// Plan-time pointing layout: validation of pixel ids, hit counts, compaction
// to observed pixels, and a stable LSD radix sort of the samples by compact
// pixel (so every pixel's samples are in ascending time order).  Integer work
// only: results are bit-exact and independent of scheduling.
#include <climits>

#include "mm_internal.h"

namespace mm {
namespace {

constexpr int kScanThreads = 256;
constexpr int64_t kSortedPad = 8;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

// exclusive scan of one tile; writes the tile total to sums[block]
template <typename TI>
__global__ void k_scan_tile(const TI* __restrict__ in, int64_t* __restrict__ out, int64_t n,
                            int64_t* __restrict__ sums) {
    __shared__ int64_t s[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        v[i] = idx < n ? (int64_t)in[idx] : 0;
        acc += v[i];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        int64_t t = (int)threadIdx.x >= d ? s[threadIdx.x - d] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t run = s[threadIdx.x] - acc;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
    if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = s[threadIdx.x];
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ offs) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const int64_t add = offs[blockIdx.x];
    for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
        const int64_t idx = base + i;
        if (idx < n) out[idx] += add;
    }
}

// out[0..n] = exclusive scan of in[0..n-1], out[n] = total
template <typename TI>
int scan_exclusive(const TI* in, int64_t* out, int64_t n, hipStream_t st) {
    if (n == 0) {
        MM_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), st));
        return MM_OK;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    DBuf<int64_t> sums, soff;
    MM_TRY(sums.alloc(nb));
    MM_TRY(soff.alloc(nb + 1));
    hipLaunchKernelGGL(k_scan_tile<TI>, dim3(nb), dim3(kScanThreads), 0, st, in, out, n, sums.p);
    MM_HIP(hipGetLastError());
    if (nb == 1) {  // one tile: its total is the total
        MM_HIP(hipMemcpyAsync(out + n, sums.p, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
        return MM_OK;
    }
    MM_TRY(scan_exclusive<int64_t>(sums.p, soff.p, nb, st));
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanThreads), 0, st, out, n, soff.p);
    MM_HIP(hipGetLastError());
    MM_HIP(hipMemcpyAsync(out + n, soff.p + nb, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    return MM_OK;  // the scratch buffers are released in stream order
}

// hit counts: every thread counts runs of equal pixel ids in 8 consecutive samples and
// adds each run once (scans revisit a pixel for several consecutive samples)
__global__ void k_hist(const int32_t* __restrict__ pix, int64_t n, int32_t* __restrict__ h) {
    const int64_t ng = (n + 7) / 8;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t0 = 8 * g, t1 = t0 + 8 < n ? t0 + 8 : n;
        int cur = pix[t0], cnt = 1;
        for (int64_t t = t0 + 1; t < t1; ++t) {
            const int v = pix[t];
            if (v == cur) {
                ++cnt;
            } else {
                atomicAdd(&h[cur], cnt);
                cur = v;
                cnt = 1;
            }
        }
        atomicAdd(&h[cur], cnt);
    }
}

__global__ void k_flags(const int32_t* __restrict__ h, int64_t n, int32_t* __restrict__ f) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        f[p] = h[p] > 0 ? 1 : 0;
}

__global__ void k_compact(const int32_t* __restrict__ h, const int64_t* __restrict__ pos,
                          int64_t n_pix, int32_t* __restrict__ cmap, int32_t* __restrict__ obs,
                          int32_t* __restrict__ hits) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_pix;
         p += (int64_t)gridDim.x * blockDim.x) {
        if (h[p] > 0) {
            const int64_t c = pos[p];
            cmap[p] = (int32_t)c;
            obs[c] = (int32_t)p;
            hits[c] = h[p];
        } else {
            cmap[p] = -1;
        }
    }
}

__global__ void k_cid(const int32_t* __restrict__ pix, int64_t n, const int32_t* __restrict__ cmap,
                      int32_t* __restrict__ cid, int32_t* __restrict__ tidx) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        cid[t] = cmap[pix[t]];
        tidx[t] = (int32_t)t;
    }
}

// ---- stable LSD radix sort of (key = compact pixel, value = sample index)
constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 16;
constexpr int kRadixTile = kRadixThreads * kRadixItems;

__global__ void k_radix_hist(const int32_t* __restrict__ keys, int64_t n, int shift,
                             int64_t* __restrict__ counts, int64_t ntiles) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    for (int it = 0; it < kRadixItems; ++it) {
        const int64_t idx = base + it * kRadixThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[((uint32_t)keys[idx] >> shift) & 255u], 1);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_radix_scatter(const int32_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                int32_t* __restrict__ kout, int32_t* __restrict__ vout, int64_t n,
                                int shift, const int64_t* __restrict__ offs, int64_t ntiles) {
    __shared__ int64_t running[256];
    __shared__ int wcnt[4][256];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    running[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    for (int it = 0; it < kRadixItems; ++it) {
        const int64_t idx = base + it * kRadixThreads + tid;
        const bool valid = idx < n;
        const int32_t key = valid ? kin[idx] : 0;
        const int32_t val = valid ? vin[idx] : 0;
        const int d = (int)(((uint32_t)key >> shift) & 255u);
        for (int q = tid; q < 4 * 256; q += kRadixThreads) (&wcnt[0][0])[q] = 0;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bb : ~bb;
        }
        __syncthreads();
        const int rank = __popcll(peers & lt);
        if (valid && rank == 0) wcnt[wv][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int64_t dst = running[d] + rank;
            for (int w = 0; w < wv; ++w) dst += wcnt[w][d];
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
        running[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        __syncthreads();
    }
}

__global__ void k_heads(const int64_t* __restrict__ seg, int64_t n_obs,
                        unsigned long long* __restrict__ heads) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_obs;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = seg[c];
        atomicOr(&heads[i >> 6], 1ull << (i & 63));
    }
}

// largest b in [0, B) with off[b] <= v (off non-decreasing, off[0] <= v)
__device__ __forceinline__ int find_range(const int64_t* __restrict__ off, int B, int64_t v) {
    int a = 0, b = B - 1;
    while (a < b) {
        const int m = (a + b + 1) >> 1;
        if (off[m] <= v) a = m; else b = m - 1;
    }
    return a;
}

// per-problem pixel id range (samples of problem b: [samp[b], samp[b+1])): every wave reads
// a chunk of 64 kMinmaxRun consecutive samples with coalesced loads and combines its range by
// shuffles (one atomic per wave); a chunk that crosses problem boundaries (at most B - 1 of
// them) does the same for its part in each problem it reaches
constexpr int kMinmaxRun = 64;
__global__ void k_prob_minmax(const int32_t* __restrict__ pix, int64_t n,
                              const int64_t* __restrict__ samp, int B, int* __restrict__ lo,
                              int* __restrict__ hi) {
    constexpr int64_t kChunk = 64 * kMinmaxRun;
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t c0 = w0 * kChunk; c0 < n; c0 += nw * kChunk) {  // wave-uniform
        const int64_t c1 = c0 + kChunk < n ? c0 + kChunk : n;
        const int b = find_range(samp, B, c0);
        if (c1 <= samp[b + 1]) {
            int l = INT_MAX, h = INT_MIN;
#pragma unroll 8
            for (int r = 0; r < kMinmaxRun; ++r) {
                const int64_t t = c0 + (int64_t)r * 64 + lane;
                if (t < c1) {
                    const int v = pix[t];
                    l = min(l, v);
                    h = max(h, v);
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                l = min(l, __shfl_xor(l, o));
                h = max(h, __shfl_xor(h, o));
            }
            if (lane == 0) {
                atomicMin(&lo[b], l);
                atomicMax(&hi[b], h);
            }
        } else {
            // the chunk's part in each problem it reaches, combined by shuffles as above
            for (int bt = b;; ++bt) {
                const int64_t s0 = c0 > samp[bt] ? c0 : samp[bt];
                const int64_t s1 = c1 < samp[bt + 1] ? c1 : samp[bt + 1];
                int l = INT_MAX, h = INT_MIN;
                for (int64_t t = s0 + lane; t < s1; t += 64) {
                    const int v = pix[t];
                    l = min(l, v);
                    h = max(h, v);
                }
                for (int o = 32; o > 0; o >>= 1) {
                    l = min(l, __shfl_xor(l, o));
                    h = max(h, __shfl_xor(h, o));
                }
                if (lane == 0 && s1 > s0) {
                    atomicMin(&lo[bt], l);
                    atomicMax(&hi[bt], h);
                }
                if (samp[bt + 1] >= c1) break;  // c1 <= samp[B]: ends at bt < B
            }
        }
    }
}

// P^T work ranges: the sorted samples of problem b (from its padded start soff[b]) are cut
// at soff[b] + k per_wave, each wave taking whole pixels; wave w belongs to problem wprob[w]
__global__ void k_wave_ranges(const int64_t* __restrict__ seg, const int64_t* __restrict__ ooff,
                              const int64_t* __restrict__ soff, const int64_t* __restrict__ woff,
                              int B, int64_t n_obs, int64_t n_waves, int64_t per_wave,
                              int32_t* __restrict__ wp, int32_t* __restrict__ wprob) {
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w <= n_waves;
         w += (int64_t)gridDim.x * blockDim.x) {
        if (w == n_waves) {
            wp[w] = (int32_t)n_obs;
            continue;
        }
        const int b = find_range(woff, B, w);
        wprob[w] = b;
        const int64_t target = soff[b] + (w - woff[b]) * per_wave;
        int64_t lo = ooff[b], hi = ooff[b + 1];  // first c in [ooff[b], ooff[b+1]] with seg[c] >= target
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (seg[mid] >= target) hi = mid; else lo = mid + 1;
        }
        wp[w] = (int32_t)lo;
    }
}

// contiguous sorted order -> padded layout: sorted position i of problem b moves to
// i - s0[b] + soff[b]; seg shifts with it (pad positions keep perm = -1)
__global__ void k_pad_sorted(const int32_t* __restrict__ vin, int64_t n,
                             const int64_t* __restrict__ s0, const int64_t* __restrict__ soff,
                             int B, int32_t* __restrict__ perm) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int b = find_range(s0, B, i);
        perm[i - s0[b] + soff[b]] = vin[i];
    }
}

__global__ void k_pad_seg(int64_t* __restrict__ seg, int64_t n_obs, const int64_t* __restrict__ ooff,
                          const int64_t* __restrict__ s0, const int64_t* __restrict__ soff, int B,
                          int64_t n_sorted) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= n_obs;
         c += (int64_t)gridDim.x * blockDim.x) {
        if (c == n_obs) {
            seg[c] = n_sorted;
            continue;
        }
        const int b = find_range(ooff, B, c);
        seg[c] = seg[c] - s0[b] + soff[b];
    }
}

template <typename TW>
__global__ void k_weights(const TW* __restrict__ w, const int32_t* __restrict__ perm, int64_t n,
                          int64_t n_sorted, double* __restrict__ w64, float* __restrict__ w32,
                          double* __restrict__ ws64, float* __restrict__ ws32) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_sorted;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (t < n) {
            const double a = (double)w[2 * t], b = (double)w[2 * t + 1];
            w64[2 * t] = a;
            w64[2 * t + 1] = b;
            if (w32) {
                w32[2 * t] = (float)a;
                w32[2 * t + 1] = (float)b;
            }
        }
        if (perm[t] < 0) {  // pad position
            ws64[2 * t] = ws64[2 * t + 1] = 0.0;
            if (ws32) ws32[2 * t] = ws32[2 * t + 1] = 0.0f;
            continue;
        }
        const int64_t s = perm[t];
        const double sa = (double)w[2 * s], sb = (double)w[2 * s + 1];
        ws64[2 * t] = sa;
        ws64[2 * t + 1] = sb;
        if (ws32) {
            ws32[2 * t] = (float)sa;
            ws32[2 * t + 1] = (float)sb;
        }
    }
}

inline int grid_for(int64_t n, int threads = 256, int cap = 65536) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

int scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t st) {
    return scan_exclusive<int64_t>(in, out, n, st);
}

int radix_sort_pairs(const int32_t* keys, const int32_t* vals, int64_t n, int32_t key_max,
                     int32_t* keys_out, int32_t* vals_out, hipStream_t st) {
    if (n == 0) return MM_OK;
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) <= key_max) ++bits;
    const int passes = (bits + 7) / 8;
    const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
    DBuf<int64_t> counts, offs;
    DBuf<int32_t> ka, kb, va, vb;
    MM_TRY(counts.alloc(256 * ntiles));
    MM_TRY(offs.alloc(256 * ntiles + 1));
    MM_TRY(ka.alloc(n));
    MM_TRY(kb.alloc(n));
    MM_TRY(va.alloc(n));
    MM_TRY(vb.alloc(n));
    MM_HIP(hipMemcpyAsync(ka.p, keys, n * 4, hipMemcpyDeviceToDevice, st));
    MM_HIP(hipMemcpyAsync(va.p, vals, n * 4, hipMemcpyDeviceToDevice, st));
    int32_t *kin = ka.p, *kout = kb.p, *vin = va.p, *vout = vb.p;
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = 8 * ps;
        hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(kRadixThreads), 0, st, kin, n, shift,
                           counts.p, ntiles);
        MM_HIP(hipGetLastError());
        MM_TRY(scan_exclusive<int64_t>(counts.p, offs.p, 256 * ntiles, st));
        hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(kRadixThreads), 0, st, kin, vin,
                           kout, vout, n, shift, offs.p, ntiles);
        MM_HIP(hipGetLastError());
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    MM_HIP(hipMemcpyAsync(keys_out, kin, n * 4, hipMemcpyDeviceToDevice, st));
    MM_HIP(hipMemcpyAsync(vals_out, vin, n * 4, hipMemcpyDeviceToDevice, st));
    return MM_OK;
}

// out[b] = src[idx[b]], b < n
template <typename T, typename I>
__global__ void k_gather(const T* __restrict__ src, const I* __restrict__ idx, int n,
                         T* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n) out[b] = src[idx[b]];
}

int build_pointing(mm_plan_t pl, const int32_t* pix, const void* weights, int wdtype) {
    hipStream_t st = pl->stream;
    const int64_t n = pl->n_t;
    const int B = pl->n_prob;
    // pixel range of every problem; problems must use disjoint, increasing id ranges so that
    // the compact pixels of problem b form one block [ooff[b], ooff[b+1])
    DBuf<int> lo, hi;
    DBuf<int64_t> samp;
    MM_TRY(lo.alloc(B));
    MM_TRY(hi.alloc(B));
    MM_TRY(samp.alloc(B + 1));
    {
        std::vector<int> l(B, INT_MAX), h(B, INT_MIN);
        MM_HIP(hipMemcpyAsync(lo.p, l.data(), B * sizeof(int), hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(hi.p, h.data(), B * sizeof(int), hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(samp.p, pl->h_samp.data(), (B + 1) * 8, hipMemcpyHostToDevice, st));
    }
    hipLaunchKernelGGL(k_prob_minmax, dim3(grid_for((n + 4 * 64 * kMinmaxRun - 1) / (4 * 64 * kMinmaxRun), 1, 2048)), dim3(256), 0, st,
                       pix, n, samp.p, B, lo.p, hi.p);
    MM_HIP(hipGetLastError());
    std::vector<int> h_lo(B), h_hi(B);
    MM_HIP(hipMemcpyAsync(h_lo.data(), lo.p, B * sizeof(int), hipMemcpyDeviceToHost, st));
    MM_HIP(hipMemcpyAsync(h_hi.data(), hi.p, B * sizeof(int), hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < B; ++b) {
        if (h_lo[b] < 0 || (int64_t)h_hi[b] >= pl->n_pix) {
            set_error("pixel ids%s span [%d, %d], outside [0, %lld)", B > 1 ? " of a problem" : "",
                      h_lo[b], h_hi[b], (long long)pl->n_pix);
            return MM_ERR_ARG;
        }
        if (b > 0 && h_lo[b] <= h_hi[b - 1]) {
            set_error("pixel ids of problem %d (from %d) do not all exceed those of problem %d "
                      "(up to %d): batched problems need disjoint increasing pixel id ranges",
                      b, h_lo[b], b - 1, h_hi[b - 1]);
            return MM_ERR_ARG;
        }
    }
    // hits on the full grid, compaction
    DBuf<int32_t> hfull, flags, cmap;
    DBuf<int64_t> pos;
    MM_TRY(hfull.alloc(pl->n_pix));
    MM_TRY(flags.alloc(pl->n_pix));
    MM_TRY(cmap.alloc(pl->n_pix));
    MM_TRY(pos.alloc(pl->n_pix + 1));
    MM_HIP(hipMemsetAsync(hfull.p, 0, pl->n_pix * sizeof(int32_t), st));
    hipLaunchKernelGGL(k_hist, dim3(grid_for((n + 7) / 8)), dim3(256), 0, st, pix, n, hfull.p);
    hipLaunchKernelGGL(k_flags, dim3(grid_for(pl->n_pix)), dim3(256), 0, st, hfull.p, pl->n_pix,
                       flags.p);
    MM_HIP(hipGetLastError());
    MM_TRY(scan_exclusive<int32_t>(flags.p, pos.p, pl->n_pix, st));
    int64_t n_obs = 0;
    MM_HIP(hipMemcpyAsync(&n_obs, pos.p + pl->n_pix, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    pl->n_obs = n_obs;
    if (n_obs >= ((int64_t)1 << 27)) {  // the map gathers use 32-bit byte offsets
        set_error("%lld observed pixels: at most 2^27 - 1 supported", (long long)n_obs);
        return MM_ERR_ARG;
    }
    // compact pixel offsets of the problems: observed pixels below each problem's first id
    pl->h_ooff.assign(B + 1, n_obs);
    {
        DBuf<int64_t> g;
        MM_TRY(g.alloc(B));
        hipLaunchKernelGGL((k_gather<int64_t, int>), dim3((B + 255) / 256), dim3(256), 0, st, pos.p,
                           lo.p, B, g.p);
        MM_HIP(hipGetLastError());
        MM_HIP(hipMemcpyAsync(pl->h_ooff.data(), g.p, B * sizeof(int64_t), hipMemcpyDeviceToHost,
                              st));
    }
    MM_TRY(pl->obs.alloc(n_obs));
    MM_TRY(pl->hits.alloc(n_obs));
    hipLaunchKernelGGL(k_compact, dim3(grid_for(pl->n_pix)), dim3(256), 0, st, hfull.p, pos.p,
                       pl->n_pix, cmap.p, pl->obs.p, pl->hits.p);
    MM_HIP(hipGetLastError());
    MM_HIP(hipStreamSynchronize(st));
    hfull.release();
    flags.release();
    pos.release();
    MM_TRY(pl->ooff.alloc(B + 1));
    MM_HIP(hipMemcpyAsync(pl->ooff.p, pl->h_ooff.data(), (B + 1) * 8, hipMemcpyHostToDevice, st));
    // compact id per sample
    MM_TRY(pl->cid.alloc(n));
    DBuf<int32_t> k2, v1, v2;
    MM_TRY(v1.alloc(n));
    hipLaunchKernelGGL(k_cid, dim3(grid_for(n)), dim3(256), 0, st, pix, n, cmap.p, pl->cid.p, v1.p);
    MM_HIP(hipGetLastError());
    cmap.release();
    // segments (contiguous sorted order for now)
    MM_TRY(pl->seg.alloc(n_obs + 1));
    MM_TRY(scan_exclusive<int32_t>(pl->hits.p, pl->seg.p, n_obs, st));
    // stable radix sort by compact pixel
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < n_obs) ++bits;
    const int passes = (bits + 7) / 8;
    const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
    DBuf<int64_t> counts, offs;
    MM_TRY(counts.alloc(256 * ntiles));
    MM_TRY(offs.alloc(256 * ntiles + 1));
    DBuf<int32_t> k1;
    MM_TRY(k1.alloc(n));
    MM_TRY(k2.alloc(n));
    MM_TRY(v2.alloc(n));
    MM_HIP(hipMemcpyAsync(k1.p, pl->cid.p, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    int32_t *kin = k1.p, *kout = k2.p, *vin = v1.p, *vout = v2.p;
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = 8 * ps;
        hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(kRadixThreads), 0, st, kin, n, shift,
                           counts.p, ntiles);
        MM_HIP(hipGetLastError());
        MM_TRY(scan_exclusive<int64_t>(counts.p, offs.p, 256 * ntiles, st));
        hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(kRadixThreads), 0, st, kin, vin,
                           kout, vout, n, shift, offs.p, ntiles);
        MM_HIP(hipGetLastError());
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    // padded layout: every problem's sorted samples start at a multiple of 8, so the
    // P^T lane and wave structure of a problem does not depend on what precedes it
    std::vector<int64_t> s0(B + 1);
    {
        DBuf<int64_t> g;
        MM_TRY(g.alloc(B));
        hipLaunchKernelGGL((k_gather<int64_t, int64_t>), dim3((B + 255) / 256), dim3(256), 0, st,
                           pl->seg.p, pl->ooff.p, B, g.p);
        MM_HIP(hipGetLastError());
        MM_HIP(hipMemcpyAsync(s0.data(), g.p, B * 8, hipMemcpyDeviceToHost, st));
    }
    MM_HIP(hipStreamSynchronize(st));
    s0[B] = n;
    pl->h_soff.assign(B + 1, 0);
    for (int b = 0; b < B; ++b)
        pl->h_soff[b + 1] = (pl->h_soff[b] + (s0[b + 1] - s0[b]) + kSortedPad - 1) / kSortedPad *
                            kSortedPad;
    const int64_t ns_sorted = B == 1 ? n : pl->h_soff[B];
    pl->n_sorted = ns_sorted;
    DBuf<int64_t> ds0, dsoff;
    MM_TRY(ds0.alloc(B + 1));
    MM_TRY(dsoff.alloc(B + 1));
    MM_HIP(hipMemcpyAsync(ds0.p, s0.data(), (B + 1) * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(dsoff.p, pl->h_soff.data(), (B + 1) * 8, hipMemcpyHostToDevice, st));
    // sorted arrays carry a zeroed tail of kSortedPad samples for aligned vector loads
    MM_TRY(pl->perm.alloc(ns_sorted + kSortedPad));
    MM_HIP(hipMemsetAsync(pl->perm.p + ns_sorted, 0, kSortedPad * sizeof(int32_t), st));
    if (B == 1) {
        MM_HIP(hipMemcpyAsync(pl->perm.p, vin, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    } else {
        MM_HIP(hipMemsetAsync(pl->perm.p, 0xff, ns_sorted * sizeof(int32_t), st));
        hipLaunchKernelGGL(k_pad_sorted, dim3(grid_for(n)), dim3(256), 0, st, vin, n, ds0.p,
                           dsoff.p, B, pl->perm.p);
        hipLaunchKernelGGL(k_pad_seg, dim3(grid_for(n_obs + 1)), dim3(256), 0, st, pl->seg.p, n_obs,
                           pl->ooff.p, ds0.p, dsoff.p, B, ns_sorted);
        MM_HIP(hipGetLastError());
    }
    k1.release();  // released in stream order after the kernels that use them
    k2.release();
    v1.release();
    v2.release();
    counts.release();
    offs.release();
    // segment heads and P^T work ranges (per problem)
    const int64_t nwords = (ns_sorted + 63) / 64 + 1;
    MM_TRY(pl->heads.alloc(nwords));
    MM_HIP(hipMemsetAsync(pl->heads.p, 0, nwords * sizeof(uint64_t), st));
    hipLaunchKernelGGL(k_heads, dim3(grid_for(n_obs)), dim3(256), 0, st, pl->seg.p, n_obs,
                       (unsigned long long*)pl->heads.p);
    MM_HIP(hipGetLastError());
    pl->h_pn.assign(B, 0);
    for (int b = 0; b < B; ++b) pl->h_pn[b] = s0[b + 1] - s0[b];
    MM_TRY(pl->soff.alloc(B + 1));
    MM_HIP(hipMemcpyAsync(pl->soff.p, pl->h_soff.data(), (B + 1) * 8, hipMemcpyHostToDevice, st));
    MM_TRY(build_wave_ranges(pl, pl->opts.pt_range > 0 ? pl->opts.pt_range : 2048));
    // weights, time-ordered and pixel-sorted
    if (pl->n_s == 3) {
        const bool mixed = pl->opts.precision == MM_MIXED;
        MM_TRY(pl->w64.alloc(2 * n));
        MM_TRY(pl->ws64.alloc(2 * (ns_sorted + kSortedPad)));
        MM_HIP(hipMemsetAsync(pl->ws64.p + 2 * ns_sorted, 0, 2 * kSortedPad * sizeof(double), st));
        if (mixed) {
            MM_TRY(pl->w32.alloc(2 * n));
            MM_TRY(pl->ws32.alloc(2 * (ns_sorted + kSortedPad)));
            MM_HIP(hipMemsetAsync(pl->ws32.p + 2 * ns_sorted, 0, 2 * kSortedPad * sizeof(float), st));
        }
        if (wdtype == MM_F64)
            hipLaunchKernelGGL(k_weights<double>, dim3(grid_for(ns_sorted)), dim3(256), 0, st,
                               (const double*)weights, pl->perm.p, n, ns_sorted, pl->w64.p,
                               pl->w32.p, pl->ws64.p, pl->ws32.p);
        else
            hipLaunchKernelGGL(k_weights<float>, dim3(grid_for(ns_sorted)), dim3(256), 0, st,
                               (const float*)weights, pl->perm.p, n, ns_sorted, pl->w64.p,
                               pl->w32.p, pl->ws64.p, pl->ws32.p);
        MM_HIP(hipGetLastError());
    }
    MM_HIP(hipStreamSynchronize(st));
    return MM_OK;
}

// P^T work ranges: problem b's sorted samples (from its padded start) are cut every
// per_wave samples; each range's wave takes the whole pixels that start in it
int build_wave_ranges(mm_plan_t pl, int64_t per_wave) {
    hipStream_t st = pl->stream;
    const int B = pl->n_prob;
    std::vector<int64_t> woff(B + 1, 0);
    for (int b = 0; b < B; ++b) woff[b + 1] = woff[b] + (pl->h_pn[b] + per_wave - 1) / per_wave;
    pl->n_waves = woff[B];
    pl->pt_range = per_wave;
    MM_TRY(pl->wave_off.alloc(B + 1));
    MM_HIP(hipMemcpyAsync(pl->wave_off.p, woff.data(), (B + 1) * 8, hipMemcpyHostToDevice, st));
    MM_TRY(pl->wave_pix.alloc(pl->n_waves + 1));
    MM_TRY(pl->wave_prob.alloc(std::max<int64_t>(1, pl->n_waves)));
    hipLaunchKernelGGL(k_wave_ranges, dim3(grid_for(pl->n_waves + 1)), dim3(256), 0, st, pl->seg.p,
                       pl->ooff.p, pl->soff.p, pl->wave_off.p, B, pl->n_obs, pl->n_waves, per_wave,
                       pl->wave_pix.p, pl->wave_prob.p);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

}  // namespace mm
