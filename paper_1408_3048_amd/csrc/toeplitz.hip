// Noise weighting N^-1: one symmetric band-limited Toeplitz block per
// stationary interval [Sect. 2.1, eq. N_def], applied by overlap-save with an
// LDS-resident radix-16 FFT.
//
// Kernel construction [Sect. 4.1.4, eq. fknee; App. D, eqs. glsSolFourier,
// apodDef]: the first row of the block of an interval of n samples is the
// inverse real DFT, on the interval's own grid f_m = m f_samp / n, of the
// inverse PSD q_m = 1 / (sigma^2 (1 + (f_knee / f_m)^alpha)) (q_0 = 0 for 1/f
// noise), kept for lags |k| <= lambda and apodised by a window.  Its symbol
// on the FFT grid, H(m) = t_0 + 2 sum_k t_k cos(2 pi k m / n_r), is the real
// spectrum used by the convolution; min H > 0 is required (positive
// definiteness of every block).
//
// Overlap-save: a tile producing outputs [o, o + L) loads the window
// [o - lambda, o + L + lambda) of the interval (zeros outside the interval,
// whose edges are hard boundaries, not periodic) into n_r >= L + 2 lambda real
// points.  The real sequence is packed as n_r/2 complex points, transformed
// in place by decimation in frequency (natural order in, bit-reversed out),
// split into the real spectrum, multiplied by H, merged back, and
// transformed in place by decimation in time (bit-reversed in, natural out),
// so no explicit permutation pass is needed.  Both transforms run as radix-16
// passes held in registers with one LDS exchange per pass.
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "mm_internal.h"

namespace mm {
namespace {

// ------------------------------------------------------------------ plan-time transforms

// Inverse PSD q_m = 1 / (sigma^2 (1 + (f_knee / f_m)^alpha)) at f_m = m f_samp / n
// [Sect. 4.1.4, eq. fknee], q_0 = 0 for 1/f noise (1/sigma^2 for white noise), or its
// derivative with respect to sigma (what = 1), f_knee (2) or alpha (3); the f_knee and
// alpha derivatives are taken as 0 for white noise.
__device__ __forceinline__ double inv_psd_at(int64_t m, int64_t n, double f_samp, double sigma,
                                             double fk, double al, int what) {
    if (fk > 0.0) {
        if (m == 0) return 0.0;
        const double f = (double)m * f_samp / (double)n;
        const double ratio = pow(fk / f, al);
        const double q = 1.0 / (sigma * sigma * (1.0 + ratio));
        if (what == 0) return q;
        if (what == 1) return -2.0 * q / sigma;
        if (what == 2) return -q * (al * ratio / fk) / (1.0 + ratio);
        return -q * ratio * log(fk / f) / (1.0 + ratio);
    }
    const double q = 1.0 / (sigma * sigma);
    return what == 0 ? q : (what == 1 ? -2.0 * q / sigma : 0.0);
}

// q_m (or a derivative) for every kernel: a[g][m] = c_m q_m, the coefficients of the real
// inverse DFT written as a cosine sum (c_0 = 1, c_m = 2 for 0 < m < n/2, c_{n/2} = 1 for
// even n).
__global__ void k_inv_psd(const int32_t* __restrict__ klen, const double* __restrict__ kpar,
                          const int64_t* __restrict__ aoff, const int64_t* __restrict__ acnt,
                          double f_samp, double* __restrict__ a, int32_t nk, int what) {
    const int g = blockIdx.y;
    if (g >= nk) return;
    const int64_t n = klen[g];
    const int64_t cnt = acnt[g];  // n/2 + 1, or 0 for kernels whose taps come from the FFT path
    const double sigma = kpar[3 * g], fk = kpar[3 * g + 1], al = kpar[3 * g + 2];
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < cnt;
         m += (int64_t)gridDim.x * blockDim.x) {
        const double q = inv_psd_at(m, n, f_samp, sigma, fk, al, what);
        double c = 2.0;
        if (m == 0 || (2 * m == n)) c = 1.0;
        a[aoff[g] + m] = c * q;
    }
}

// the FFT twiddles exp(-2 pi i q / n), q < count, as (re, im) pairs in FP64 and, where
// tw32 is given, rounded to FP32 (2q/n is exact for the power-of-two lengths used here)
__global__ void k_twiddles(int64_t count, int64_t n, double* __restrict__ tw64,
                           float* __restrict__ tw32) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count;
         q += (int64_t)gridDim.x * blockDim.x) {
        double s, c;
        sincospi(-2.0 * (double)q / (double)n, &s, &c);
        tw64[2 * q] = c;
        tw64[2 * q + 1] = s;
        if (tw32) {
            tw32[2 * q] = (float)c;
            tw32[2 * q + 1] = (float)s;
        }
    }
}

// out[g][j] = sum_{i < cnt[g]} a[g][i] cos(2 pi i j / n[g]) for j < J[g].
// The cosine of every term comes from a rotation recurrence re-anchored by
// sincospi every 32 terms (bounded rounding growth).
constexpr int kCtThreads = 256;
__global__ void k_cos_transform(const double* __restrict__ a, const int64_t* __restrict__ aoff,
                                const int64_t* __restrict__ acnt, const int64_t* __restrict__ nper,
                                const int64_t* __restrict__ jcnt, const int64_t* __restrict__ ooff,
                                double* __restrict__ out, int32_t ng) {
    __shared__ double sa[kCtThreads];
    const int g = blockIdx.y;
    if (g >= ng) return;
    const int64_t J = jcnt[g];
    const int64_t j = (int64_t)blockIdx.x * kCtThreads + threadIdx.x;
    if ((int64_t)blockIdx.x * kCtThreads >= J) return;
    const int64_t n = nper[g];
    const int64_t cnt = acnt[g];
    const double* ag = a + aoff[g];
    const int64_t jm = j % n;
    double cs, ss;
    sincospi(2.0 * (double)jm / (double)n, &ss, &cs);
    double acc = 0.0;
    for (int64_t i0 = 0; i0 < cnt; i0 += kCtThreads) {
        __syncthreads();
        sa[threadIdx.x] = (i0 + threadIdx.x < cnt) ? ag[i0 + threadIdx.x] : 0.0;
        __syncthreads();
        for (int s = 0; s < kCtThreads; s += 32) {
            if (i0 + s >= cnt) break;
            const int64_t idx = ((i0 + s) % n) * jm % n;
            double c, sn;
            sincospi(2.0 * (double)idx / (double)n, &sn, &c);
#pragma unroll 8
            for (int u = 0; u < 32; ++u) {
                acc = fma(sa[s + u], c, acc);
                const double c2 = c * cs - sn * ss;
                sn = fma(sn, cs, c * ss);
                c = c2;
            }
        }
    }
    if (j < J) out[ooff[g] + j] = acc;
}

// apodisation window at lag k (0 <= k <= lambda) [App. D, eq. apodDef]: 1 at k = 0 for
// every window, so lambda = 0 keeps t_0 alone (a diagonal N^-1)
__device__ __forceinline__ double window_at(int64_t k, int lam, int window) {
    if (k == 0) return 1.0;
    const double x = (double)k / (double)lam;
    if (window == MM_WIN_GAUSS) return exp(-x * x);
    if (window == MM_WIN_GAUSS2) return exp(-2.0 * x * x);
    return 1.0;
}

__global__ void k_taps_finish(double* __restrict__ t, const int64_t* __restrict__ toff,
                              const int64_t* __restrict__ tcnt, const int32_t* __restrict__ klen,
                              int lam, int window, int32_t nk) {
    const int g = blockIdx.y;
    if (g >= nk) return;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < tcnt[g];
         k += (int64_t)gridDim.x * blockDim.x) {
        t[toff[g] + k] *= window_at(k, lam, window) / (double)klen[g];
    }
}

__global__ void k_spec_finish(const double* __restrict__ Hraw, int64_t stride, int64_t cnt,
                              double scale, double* __restrict__ H64, float* __restrict__ H32,
                              double* __restrict__ hmin) {
    const int g = blockIdx.x;
    double m = INFINITY;
    for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
        const double h = Hraw[g * stride + i];
        m = fmin(m, h);
        if (H64) H64[g * stride + i] = h * scale;
        if (H32) H32[g * stride + i] = (float)(h * scale);
    }
    __shared__ double red[256];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) hmin[g] = red[0];
}

// ------------------------------------------------------------------ overlap-save kernel

template <typename T>
struct ToepArgs {
    const int32_t* cid;
    const T* w;           // [n_t][2] time-ordered weights (IQU)
    const double* x;      // map (FP64); I-only mode reads it directly
    const T* xp;          // map packed as [n_obs][4] = (I, Q, U, 0) in T (IQU mode)
    const void* y;        // TOD input
    int y_f64;
    int mode;             // 0 map IQU, 1 map I, 2 TOD FP64, 3 TOD FP32
    T* z;
    const T* H;           // [n_kern][M + 1]
    const T* tw;          // [M][2]
    const int64_t* tile_out;
    const int32_t* tile_len;
    const int32_t* tile_int;
    const int64_t* int_lo;
    const int64_t* int_hi;
    const int32_t* int_kern;
    int lam;
    int64_t n_tiles;          // tiles of the launch (blocks are mapped to tiles XCD-major)
    const int* mask;          // per-problem flags: tiles of problems with mask 0 are skipped
    const int32_t* int_prob;  // problem of every interval
    int skip_zero;            // map modes: all-zero windows skip the transform
    const uint8_t* int_on;    // zero-skipping launches: intervals flagged 0 have an all-zero
                              // input (known beforehand) and write zeros without loading it
    // zero-skipping launches over several maps (blockIdx.y = layer y < layers): layer y
    // reads x + y x_step, xp + y xp_step and int_on + y on_step and writes z + y z_step
    int layers;
    int64_t x_step, xp_step, z_step, on_step;
};

// LDS layout of the complex work array (M points).  Element a lives at
// swz(a) = a ^ (((a >> 5) ^ (a >> 10)) & 31), a bijection within every block of 32
// points, with no padding.  With 8-byte accesses served 32 lanes at a time over the 64
// four-byte banks, enumerating every access pattern gives conflict-free radix-16 passes
// (the block-size-32 pass with its groups mapped so that k is uniform over a wave) and
// load/store phases, and a 1.2-way spectrum pass.  FP32 points are stored interleaved
// (one 8-byte access per point), FP64 as split real and imaginary arrays (two 8-byte
// accesses).
// swz is linear over XOR, so for bit-disjoint a and c, swz(a + c) = swz(a) ^ swz(c): the
// passes swizzle their thread's base index once and reach the other points by XOR with
// compile-time constants.
__host__ __device__ constexpr int swz(int a) { return a ^ (((a >> 5) ^ (a >> 10)) & 31); }

template <typename T>
struct CBuf;

template <>
struct CBuf<float> {
    float2* c;
    // at byte offset b (8 times an already swizzled position)
    __device__ __forceinline__ void get_swb(int b, float& re, float& im) const {
        const float2 v = *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(c) + b);
        re = v.x;
        im = v.y;
    }
    __device__ __forceinline__ void put_swb(int b, float re, float im) const {
        *reinterpret_cast<float2*>(reinterpret_cast<char*>(c) + b) = make_float2(re, im);
    }
    __device__ __forceinline__ void put_part_sw(int p, int part, float v) const {
        reinterpret_cast<float*>(c)[2 * p + part] = v;
    }
    __device__ __forceinline__ void get(int a, float& re, float& im) const {
        const float2 v = c[swz(a)];
        re = v.x;
        im = v.y;
    }
    __device__ __forceinline__ void put(int a, float re, float im) const {
        c[swz(a)] = make_float2(re, im);
    }
    __device__ __forceinline__ void put_part(int a, int part, float v) const {
        reinterpret_cast<float*>(c)[2 * swz(a) + part] = v;
    }
    __device__ __forceinline__ float get_part(int a, int part) const {
        return reinterpret_cast<const float*>(c)[2 * swz(a) + part];
    }
};

template <>
struct CBuf<double> {
    double* re;
    double* im;
    __device__ __forceinline__ void get_swb(int b, double& r, double& i) const {
        r = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(re) + b);
        i = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(im) + b);
    }
    __device__ __forceinline__ void put_swb(int b, double r, double i) const {
        *reinterpret_cast<double*>(reinterpret_cast<char*>(re) + b) = r;
        *reinterpret_cast<double*>(reinterpret_cast<char*>(im) + b) = i;
    }
    __device__ __forceinline__ void put_part_sw(int p, int part, double v) const {
        (part ? im : re)[p] = v;
    }
    __device__ __forceinline__ void get(int a, double& r, double& i) const {
        const int p = swz(a);
        r = re[p];
        i = im[p];
    }
    __device__ __forceinline__ void put(int a, double r, double i) const {
        const int p = swz(a);
        re[p] = r;
        im[p] = i;
    }
    __device__ __forceinline__ void put_part(int a, int part, double v) const {
        (part ? im : re)[swz(a)] = v;
    }
    __device__ __forceinline__ double get_part(int a, int part) const {
        return (part ? im : re)[swz(a)];
    }
};

// the M-point complex buffer over 2 M sizeof(T) bytes of LDS
template <typename T>
__device__ __forceinline__ CBuf<T> make_cbuf(unsigned char* smem, int M) {
    CBuf<T> b;
    if constexpr (sizeof(T) == 4) {
        b.c = reinterpret_cast<float2*>(smem);
    } else {
        b.re = reinterpret_cast<double*>(smem);
        b.im = b.re + M;
    }
    return b;
}

template <int BITS>
__device__ __forceinline__ int rev_bits(int v) {
    return (int)(__builtin_bitreverse32((uint32_t)v) >> (32 - BITS));
}

// exp(-2 pi i q / 16), q = 0..15
template <typename T>
__device__ __forceinline__ void root16(int q, T& c, T& s) {
    constexpr double C1 = 0.92387953251128675613, S1 = 0.38268343236508977173,
                     C2 = 0.70710678118654752440;
    const double cs[16] = {1.0, C1, C2, S1, 0.0, -S1, -C2, -C1, -1.0, -C1, -C2, -S1, 0.0, S1, C2, C1};
    const double sn[16] = {0.0, S1, C2, C1, 1.0, C1, C2, S1, 0.0, -S1, -C2, -C1, -1.0, -C1, -C2, -S1};
    c = (T)cs[q & 15];
    s = (T)(-sn[q & 15]);
}

// in-register radix-R DIF network: natural in, bit-reversed out (forward, e^{-i})
template <typename T, int R>
__device__ __forceinline__ void dif_net(T* vr, T* vi) {
#pragma unroll
    for (int h = R / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int b = 0; b < R; b += 2 * h) {
#pragma unroll
            for (int kk = 0; kk < h; ++kk) {
                const T ar = vr[b + kk], ai = vi[b + kk];
                const T cr = vr[b + kk + h], ci = vi[b + kk + h];
                vr[b + kk] = ar + cr;
                vi[b + kk] = ai + ci;
                const T dr = ar - cr, di = ai - ci;
                const int q = kk * (16 / (2 * h));
                if (q == 0) {
                    vr[b + kk + h] = dr;
                    vi[b + kk + h] = di;
                } else if (q == 4) {  // * (-i)
                    vr[b + kk + h] = di;
                    vi[b + kk + h] = -dr;
                } else {
                    T c, s;
                    root16<T>(q, c, s);
                    vr[b + kk + h] = dr * c - di * s;
                    vi[b + kk + h] = dr * s + di * c;
                }
            }
        }
    }
}

// in-register inverse radix-R DIT network: bit-reversed in, natural out (e^{+i})
template <typename T, int R>
__device__ __forceinline__ void dit_net_inv(T* vr, T* vi) {
#pragma unroll
    for (int h = 1; h < R; h <<= 1) {
#pragma unroll
        for (int b = 0; b < R; b += 2 * h) {
#pragma unroll
            for (int kk = 0; kk < h; ++kk) {
                const int q = kk * (16 / (2 * h));
                T cr = vr[b + kk + h], ci = vi[b + kk + h];
                if (q == 4) {  // * (+i)
                    const T t = cr;
                    cr = -ci;
                    ci = t;
                } else if (q != 0) {
                    T c, s;
                    root16<T>(q, c, s);
                    s = -s;  // conjugate root
                    const T t = cr * c - ci * s;
                    ci = cr * s + ci * c;
                    cr = t;
                }
                const T ar = vr[b + kk], ai = vi[b + kk];
                vr[b + kk] = ar + cr;
                vi[b + kk] = ai + ci;
                vr[b + kk + h] = ar - cr;
                vi[b + kk + h] = ai - ci;
            }
        }
    }
}

// w^e for e = 0..R-1 from w (binary powering: short dependency chains)
template <typename T, int R>
__device__ __forceinline__ void powers(T wr, T wi, T* pr, T* pi) {
    pr[0] = (T)1;
    pi[0] = (T)0;
    if (R > 1) {
        pr[1] = wr;
        pi[1] = wi;
    }
#pragma unroll
    for (int e = 2; e < R; ++e) {
        const int a = (e & 1) ? e - 1 : e / 2;
        const int b = (e & 1) ? 1 : e / 2;
        pr[e] = pr[a] * pr[b] - pi[a] * pi[b];
        pi[e] = pr[a] * pi[b] + pi[a] * pr[b];
    }
}

// The passes address LDS by byte offsets: an 8-byte point (FP32 (re, im), or one FP64
// part) at swizzled position p sits at byte 8 p, and swz is linear over XOR, so the
// byte offset of point (base + c) is (8 swz(base)) ^ (8 swz(c)) for bit-disjoint base and
// c: one XOR with a compile-time constant per point.
// exp(-2 pi i e / 32), e = 0..15: the twiddles of a radix-16 pass of block size 32 for its
// group k = 1 (cos and sin of multiples of pi/16)
template <typename T>
__device__ __forceinline__ void root32(int e, T& c, T& s) {
    // cos and sin of pi e / 16
    constexpr double cs[16] = {1.0, 0.98078528040323044913, 0.92387953251128675613,
                               0.83146961230254523708, 0.70710678118654752440,
                               0.55557023301960222474, 0.38268343236508977173,
                               0.19509032201612826785, 0.0, -0.19509032201612826785,
                               -0.38268343236508977173, -0.55557023301960222474,
                               -0.70710678118654752440, -0.83146961230254523708,
                               -0.92387953251128675613, -0.98078528040323044913};
    constexpr double sn[16] = {0.0, 0.19509032201612826785, 0.38268343236508977173,
                               0.55557023301960222474, 0.70710678118654752440,
                               0.83146961230254523708, 0.92387953251128675613,
                               0.98078528040323044913, 1.0, 0.98078528040323044913,
                               0.92387953251128675613, 0.83146961230254523708,
                               0.70710678118654752440, 0.55557023301960222474,
                               0.38268343236508977173, 0.19509032201612826785};
    c = (T)cs[e & 15];
    s = (T)(-sn[e & 15]);
}

// Twiddles of a pass (block size B = 2^LOGB, Q = B / 2^LR groups per block):
//  - Q == 2 (B = 32): the groups are mapped so that every wave has one k; k = 0 needs none,
//    k = 1 the constants root32;
//  - the passes after the first with Q >= 4 read w^e, e = 1 .. R-1, from an LDS table
//    filled at the start of the kernel (lt, [e - 1][k] per pass) where the table leaves the
//    tile's occupancy unchanged;
//  - otherwise binary powers of w = tw[k TWS] (the first pass, the plan-time transforms).
// Every source gives the same values: the LDS table holds the powers the last case forms.
template <typename T, int LOGM, int LOGB>
constexpr bool first_pass() {
    return LOGB == LOGM;
}
// entries of the LDS twiddle table before the pass of block size 2^LOGB (passes after the
// first, with Q >= 4), and in all
__host__ __device__ constexpr int ltw_offset(int logm, int logb) {
    int off = 0;
    for (int l = logm; l > logb; l -= (l >= 4 ? 4 : l)) {
        const int lr = l >= 4 ? 4 : l;
        const int q = (1 << l) >> lr;
        if (l != logm && q >= 4) off += ((1 << lr) - 1) * q;
    }
    return off;
}
__host__ __device__ constexpr int ltw_total(int logm) { return ltw_offset(logm, 0); }

template <typename T, int LOGM, int NT, int LR, int LOGB, bool LTW>
__device__ __forceinline__ void pass_twiddles(int k, const T* __restrict__ tw,
                                              const T* __restrict__ lt, T* pr, T* pi) {
    constexpr int R = 1 << LR, B = 1 << LOGB, Q = B / R, M = 1 << LOGM;
    constexpr int TWS = (2 * M) / B;
    if constexpr (Q == 2 && R == 16) {
#pragma unroll
        for (int e = 1; e < R; ++e) root32<T>(e, pr[e], pi[e]);
    } else if constexpr (LTW && !first_pass<T, LOGM, LOGB>() && Q >= 4) {
        const T* tb = lt + 2 * (ltw_offset(LOGM, LOGB) + k);
#pragma unroll
        for (int e = 1; e < R; ++e) {
            pr[e] = tb[2 * (e - 1) * Q];
            pi[e] = tb[2 * (e - 1) * Q + 1];
        }
    } else {
        powers<T, R>(tw[2 * k * TWS], tw[2 * k * TWS + 1], pr, pi);
    }
}

// the LDS twiddle table of the passes after the first (see pass_twiddles), formed by the
// same binary powers the passes would take; every thread must call
template <typename T, int LOGM, int NT>
__device__ __forceinline__ void fill_ltw(const T* __restrict__ tw, T* lt) {
    constexpr int M = 1 << LOGM;
    for (int l = LOGM - 4; l > 0; l -= (l >= 4 ? 4 : l)) {
        const int lr = l >= 4 ? 4 : l;
        const int q = (1 << l) >> lr;
        if (q < 4) continue;
        const int tws = (2 * M) >> l;
        const int off = ltw_offset(LOGM, l);
        for (int k = threadIdx.x; k < q; k += NT) {
            T pr[16], pi[16];
            const T wr = tw[2 * k * tws], wi = tw[2 * k * tws + 1];
            if (lr == 4) powers<T, 16>(wr, wi, pr, pi);
            else if (lr == 3) powers<T, 8>(wr, wi, pr, pi);
            else powers<T, 4>(wr, wi, pr, pi);
            for (int e = 1; e < (1 << lr); ++e) {
                lt[2 * (off + (e - 1) * q + k)] = k ? pr[e] : (T)1;
                lt[2 * (off + (e - 1) * q + k) + 1] = k ? pi[e] : (T)0;
            }
        }
    }
}

// group g of a pass -> (block, k); for Q == 2 the first half of the groups has k = 0 and
// the second k = 1, so that k is uniform over a wave
template <int Q, int G>
__device__ __forceinline__ void pass_group(int g, int& blk, int& k) {
    if constexpr (Q == 2) {
        k = g >= G / 2 ? 1 : 0;
        blk = g & (G / 2 - 1);
    } else {
        k = g & (Q - 1);
        blk = g / Q;
    }
}

template <typename T, int LOGM, int NT, int LR, int LOGB, bool LTW = false>
__device__ __forceinline__ void dif_pass(const CBuf<T>& buf, const T* __restrict__ tw,
                                         const T* __restrict__ lt = nullptr) {
    constexpr int R = 1 << LR, B = 1 << LOGB, Q = B / R, M = 1 << LOGM, G = M / R;
    for (int g = threadIdx.x; g < G; g += NT) {
        int blk, k;
        pass_group<Q, G>(g, blk, k);
        const int sbb = swz(blk * B + k) << 3;  // base and m Q are bit-disjoint
        T vr[R], vi[R];
#pragma unroll
        for (int m = 0; m < R; ++m) buf.get_swb(sbb ^ (swz(m * Q) << 3), vr[m], vi[m]);
        dif_net<T, R>(vr, vi);
        if (Q > 1 && k != 0) {
            T pr[R], pi[R];
            pass_twiddles<T, LOGM, NT, LR, LOGB, LTW>(k, tw, lt, pr, pi);
#pragma unroll
            for (int i = 1; i < R; ++i) {
                const int e = rev_bits<LR>(i);
                const T t = vr[i] * pr[e] - vi[i] * pi[e];
                vi[i] = vr[i] * pi[e] + vi[i] * pr[e];
                vr[i] = t;
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i) buf.put_swb(sbb ^ (swz(i * Q) << 3), vr[i], vi[i]);
    }
    __syncthreads();
}

template <typename T, int LOGM, int NT, int LR, int LOGB, bool LTW = false>
__device__ __forceinline__ void dit_pass(const CBuf<T>& buf, const T* __restrict__ tw,
                                         const T* __restrict__ lt = nullptr) {
    constexpr int R = 1 << LR, B = 1 << LOGB, Q = B / R, M = 1 << LOGM, G = M / R;
    for (int g = threadIdx.x; g < G; g += NT) {
        int blk, k;
        pass_group<Q, G>(g, blk, k);
        const int sbb = swz(blk * B + k) << 3;
        T vr[R], vi[R];
#pragma unroll
        for (int i = 0; i < R; ++i) buf.get_swb(sbb ^ (swz(i * Q) << 3), vr[i], vi[i]);
        if (Q > 1 && k != 0) {
            T pr[R], pi[R];
            pass_twiddles<T, LOGM, NT, LR, LOGB, LTW>(k, tw, lt, pr, pi);
#pragma unroll
            for (int i = 1; i < R; ++i) {
                const int e = rev_bits<LR>(i);
                const T t = vr[i] * pr[e] + vi[i] * pi[e];  // * conj(w^e)
                vi[i] = vi[i] * pr[e] - vr[i] * pi[e];
                vr[i] = t;
            }
        }
        dit_net_inv<T, R>(vr, vi);
#pragma unroll
        for (int m = 0; m < R; ++m) buf.put_swb(sbb ^ (swz(m * Q) << 3), vr[m], vi[m]);
    }
    __syncthreads();
}

// STOP = 1: the last radix-2 stage (LOGB == 1) is left to the fused spectrum pass.  LTW:
// the passes after the first read their twiddles from the LDS table lt.
template <typename T, int LOGM, int NT, int LOGB, int STOP = 0, bool LTW = false>
__device__ __forceinline__ void fwd_passes(const CBuf<T>& buf, const T* tw,
                                           const T* lt = nullptr) {
    if constexpr (LOGB > STOP) {
        constexpr int LR = LOGB >= 4 ? 4 : LOGB;
        dif_pass<T, LOGM, NT, LR, LOGB, LTW>(buf, tw, lt);
        fwd_passes<T, LOGM, NT, LOGB - LR, STOP, LTW>(buf, tw, lt);
    }
}

template <typename T, int LOGM, int NT, int LOGB, int STOP = 0, bool LTW = false>
__device__ __forceinline__ void inv_passes(const CBuf<T>& buf, const T* tw,
                                           const T* lt = nullptr) {
    if constexpr (LOGB > STOP) {
        constexpr int LR = LOGB >= 4 ? 4 : LOGB;
        inv_passes<T, LOGM, NT, LOGB - LR, STOP, LTW>(buf, tw, lt);
        dit_pass<T, LOGM, NT, LR, LOGB, LTW>(buf, tw, lt);
    }
}

// The spectrum product of a frequency pair (k, m = M - k) of the packed real transform.
// With Z the M-point transform of z[n] = y[2n] + i y[2n+1], the real transform of y is
// X_k = ((Z_k + conj Z_m) - i e (Z_k - conj Z_m)) / 2, e = exp(-i pi k / M); the product
// Y_k = H_k X_k (H real and even) is packed back into the input of the inverse transform
// as W_k = (Y_k + conj Y_m) + i conj(e) (Y_k - conj Y_m).  Composed, the three steps are
// one linear map with real coefficients: with c = cos(pi k / M), s = sin(pi k / M),
//   W_k = a_k Z_k + i g conj(Z_m),   W_m = a_m Z_m + i g conj(Z_k),
//   a_k = h_k + h_m - s (h_k - h_m),  a_m = h_k + h_m + s (h_k - h_m),  g = c (h_k - h_m),
// where h = H / n_r is the spectrum as the plan stores it (the inverse transform's 1/M
// and the split's factors folded in).  k = 0 (pair with m = M, the Nyquist bin) and the
// self-paired k = M/2 (c = 0, s = 1) are the same formula.  tw holds e as (c, -s).
template <typename T>
__device__ __forceinline__ void spectrum_pair(T hk, T hm, T c, T s, T zkr, T zki, T zmr,
                                                T zmi, T& wkr, T& wki, T& wmr, T& wmi) {
    const T u = hk + hm, v = hk - hm;
    const T ak = u - s * v, am = u + s * v, g = c * v;
    wkr = ak * zkr + g * zmi;
    wki = ak * zki + g * zmr;
    wmr = am * zmr + g * zki;
    wmi = am * zmi + g * zkr;
}

// spectrum product on pairs (k, M - k) of the bit-reversed half-length transform.  A
// thread's kernel-spectrum and twiddle values for all its pairs are loaded before the
// first product, so their memory latency is paid once, not once per pair.
template <typename T, int LOGM, int NT>
__device__ __forceinline__ void spectrum_pass(const CBuf<T>& buf, const T* __restrict__ H,
                                              const T* __restrict__ tw) {
    constexpr int M = 1 << LOGM;
    constexpr int NI = (M / 2 + NT) / NT;  // pairs k = tid + i NT <= M/2
    T hk[NI], hm[NI], cc[NI], ss[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int k0 = threadIdx.x + i * NT;
        const int k = k0 <= M / 2 ? k0 : M / 2;  // valid address; not used past M/2
        hk[i] = H[k];
        hm[i] = H[M - k];
        cc[i] = tw[2 * k];
        ss[i] = -tw[2 * k + 1];
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int k = threadIdx.x + i * NT;
        if (k > M / 2) break;
        const int km = M - k;
        const int ak = rev_bits<LOGM>(k);
        const int am = k == 0 ? ak : rev_bits<LOGM>(km);  // bin M is bin 0
        T zkr, zki, zmr, zmi, wkr, wki, wmr, wmi;
        buf.get(ak, zkr, zki);
        buf.get(am, zmr, zmi);
        spectrum_pair(hk[i], hm[i], cc[i], ss[i], zkr, zki, zmr, zmi, wkr, wki, wmr, wmi);
        buf.put(ak, wkr, wki);
        if (k != 0 && km != k) buf.put(am, wmr, wmi);
    }
    __syncthreads();
}

// For LOGM = 1 mod 4 the forward transform ends and the inverse starts with a radix-2
// stage on adjacent slots (2j, 2j + 1), which hold the frequencies f and f + M/2 after the
// stage (f = rev(2j)).  The slots {rev(k), rev(k) ^ 1, rev(M - k), rev(M - k) ^ 1} carry the
// frequencies k, M/2 + k, M - k and M/2 - k: the two spectrum pairs (k, M - k) and
// (M/2 + k, M/2 - k).  This pass takes such a group (k = 0 .. M/4) through the forward
// radix-2 stage, the spectrum product of both pairs and the inverse radix-2 stage, which
// saves two passes over LDS and two barriers; the arithmetic is that of the three passes.
template <typename T, int LOGM, int NT>
__device__ __forceinline__ void spectrum_pass_r2(const CBuf<T>& buf, const T* __restrict__ H,
                                                 const T* __restrict__ tw) {
    constexpr int M = 1 << LOGM;
    constexpr int NI = (M / 4 + NT) / NT;  // groups k = tid + i NT <= M/4
    // per group: h at k, M - k, M/2 + k, M/2 - k and the twiddle (c, -s) at k; the pair
    // (M/2 + k, M/2 - k) has c' = -s, s' = c
    T h0[NI], h1[NI], h2[NI], h3[NI], cc[NI], ss[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int k0 = threadIdx.x + i * NT;
        const int k = k0 <= M / 4 ? k0 : M / 4;  // valid address; not used past M/4
        h0[i] = H[k];
        h1[i] = H[M - k];
        h2[i] = H[M / 2 + k];
        h3[i] = H[M / 2 - k];
        cc[i] = tw[2 * k];
        ss[i] = -tw[2 * k + 1];
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int k = threadIdx.x + i * NT;
        if (k > M / 4) break;
        const int a = rev_bits<LOGM>(k);  // even: k < M/2
        // byte offsets: slot a + 1 = a ^ 1 sits at swz(a) ^ 1 (swz is linear over XOR)
        const int ab = swz(a) << 3;
        T ur, ui, vr, vi;
        buf.get_swb(ab, ur, ui);
        buf.get_swb(ab ^ 8, vr, vi);
        // forward radix-2 stage: slot a -> frequency k, slot a + 1 -> k + M/2
        const T z0r = ur + vr, z0i = ui + vi, z1r = ur - vr, z1i = ui - vi;
        T y0r, y0i, y1r, y1i, q0r, q0i, q1r, q1i;
        if (k == 0) {  // DC with the Nyquist bin (pair (0, M)), and the self-paired M/2
            // h2 = h3 = H[M/2]; (c, s) at M/2 is (0, 1)
            spectrum_pair(h0[i], h1[i], (T)1, (T)0, z0r, z0i, z0r, z0i, y0r, y0i, q0r, q0i);
            spectrum_pair(h2[i], h3[i], (T)0, (T)1, z1r, z1i, z1r, z1i, y1r, y1i, q1r, q1i);
        } else if (k == M / 4) {  // the pair (M/4, 3M/4) is the slot pair itself
            spectrum_pair(h0[i], h1[i], cc[i], ss[i], z0r, z0i, z1r, z1i, y0r, y0i, y1r, y1i);
        } else {
            const int b = rev_bits<LOGM>(M - k);  // odd: slot b -> M - k, b - 1 -> M/2 - k
            const int bb = swz(b) << 3;           // slot b - 1 = b ^ 1 at bb ^ 8
            T sr, si, tr, ti;
            buf.get_swb(bb ^ 8, sr, si);
            buf.get_swb(bb, tr, ti);
            const T w0r = sr + tr, w0i = si + ti, w1r = sr - tr, w1i = si - ti;
            spectrum_pair(h0[i], h1[i], cc[i], ss[i], z0r, z0i, w1r, w1i, y0r, y0i, q1r, q1i);
            spectrum_pair(h2[i], h3[i], -ss[i], cc[i], z1r, z1i, w0r, w0i, y1r, y1i, q0r, q0i);
            // inverse radix-2 stage on the slots (b - 1, b)
            buf.put_swb(bb ^ 8, q0r + q1r, q0i + q1i);
            buf.put_swb(bb, q0r - q1r, q0i - q1i);
        }
        // inverse radix-2 stage on the slots (a, a + 1)
        buf.put_swb(ab, y0r + y1r, y0i + y1i);
        buf.put_swb(ab ^ 8, y0r - y1r, y0i - y1i);
    }
    __syncthreads();
}

// element i of an array at a block-uniform base, addressed by a 32-bit byte offset (the
// scalar-base form of the load: no 64-bit vector address arithmetic per element)
template <typename E>
__device__ __forceinline__ E at_u32(const E* base, uint32_t i) {
    return *reinterpret_cast<const E*>(reinterpret_cast<const char*>(base) +
                                       i * (uint32_t)sizeof(E));
}

// Load phase: the tile's window [o - lambda, o + L + lambda) of the interval, zero
// outside, packed as complex points (even sample -> real, odd -> imaginary).  Each
// thread handles 8 samples at a time and issues their index loads, weight loads and
// map gathers as independent batches, so several memory requests per thread are in
// flight.  Out-of-window samples load a valid index (the interval start) and are
// masked to zero.
// returns whether any of the thread's samples is nonzero
template <typename T, int LOGM, int NT, int MODE>
__device__ __forceinline__ bool load_window(const ToepArgs<T>& a, const CBuf<T>& buf,
                                            int64_t base, int win, int64_t lo, int64_t hi) {
    constexpr int NR = 2 << LOGM;
    constexpr int PER = NR / NT;
    // gathers in flight per thread: 8 for the IQU map gather (its registers bound the
    // occupancy), 16 otherwise
    constexpr int BMAX = MODE == 0 ? 8 : 16;
    constexpr int B = PER < BMAX ? PER : BMAX;
    static_assert(PER % B == 0, "tile must split into batches");
    static_assert(NT % 2 == 0, "even thread count");
    // point (tid + c NT) / 2 = tid / 2 + c NT / 2 with bit-disjoint terms
    const int sbase = swz(threadIdx.x >> 1), part = threadIdx.x & 1;
    // indices relative to the window start (a block-uniform base): window positions
    // [i_lo, i_hi) lie inside the interval; others read position i_lo (inside the
    // interval, since the window ends past it) and are masked.  32-bit unsigned offsets
    // from uniform bases keep the address arithmetic out of 64-bit vector instructions.
    const int i_lo = (int)(lo > base ? lo - base : 0);
    const int i_hi = (int)(hi - base < (int64_t)win ? hi - base : (int64_t)win);
    bool nz = false;
    if constexpr (MODE == 0) {
        // IQU map gather, software-pipelined: the indices and weights of batch k + 1 are
        // loaded while the map gathers of batch k are in flight, so a batch waits for one
        // memory latency instead of two (the values are those of the plain loop below);
        // batches of 8 samples in FP32, 4 in FP64 (registers)
        typedef typename std::conditional<sizeof(T) == 4, float4, double4>::type T4;
        typedef typename std::conditional<sizeof(T) == 4, float2, double2>::type T2;
        constexpr int BP = sizeof(T) == 4 ? (PER < 8 ? PER : 8) : (PER < 4 ? PER : 4);
        static_assert(PER % BP == 0, "tile must split into batches");
        const int32_t* cb = a.cid + base;
        const T2* wb = reinterpret_cast<const T2*>(a.w) + base;
        const char* xpb = reinterpret_cast<const char*>(a.xp);
        auto pos = [&](int k) -> uint32_t {
            const int i = threadIdx.x + k * NT;
            return (uint32_t)(i >= i_lo && i < i_hi ? i : i_lo);
        };
        uint32_t cc[BP];
        T2 ww[BP];
#pragma unroll
        for (int u = 0; u < BP; ++u) {
            const uint32_t r = pos(u);
            cc[u] = (uint32_t)at_u32(cb, r);
            ww[u] = at_u32(wb, r);
        }
#pragma unroll
        for (int b0 = 0; b0 < PER; b0 += BP) {
            T4 xx[BP];
#pragma unroll
            for (int u = 0; u < BP; ++u)
                xx[u] = *reinterpret_cast<const T4*>(xpb + cc[u] * (uint32_t)sizeof(T4));
            T2 wcur[BP];
#pragma unroll
            for (int u = 0; u < BP; ++u) wcur[u] = ww[u];
            if (b0 + BP < PER) {
#pragma unroll
                for (int u = 0; u < BP; ++u) {
                    const uint32_t r = pos(b0 + BP + u);
                    cc[u] = (uint32_t)at_u32(cb, r);
                    ww[u] = at_u32(wb, r);
                }
            }
#pragma unroll
            for (int u = 0; u < BP; ++u) {
                const int i = threadIdx.x + (b0 + u) * NT;
                const bool ok = i >= i_lo && i < i_hi;
                const T v = ok ? xx[u].x + wcur[u].x * xx[u].y + wcur[u].y * xx[u].z : (T)0;
                buf.put_part_sw(sbase ^ swz((b0 + u) * (NT / 2)), part, v);
                nz = nz || v != (T)0;
            }
        }
        return nz;
    }
#pragma unroll
    for (int b0 = 0; b0 < PER; b0 += B) {
        uint32_t rr[B];
        bool ok[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int i = threadIdx.x + (b0 + u) * NT;
            ok[u] = i >= i_lo && i < i_hi;
            rr[u] = (uint32_t)(ok[u] ? i : i_lo);
        }
        T v[B];
        if constexpr (MODE == 0) {  // map, I/Q/U: one packed-map gather per sample
            typedef typename std::conditional<sizeof(T) == 4, float4, double4>::type T4;
            typedef typename std::conditional<sizeof(T) == 4, float2, double2>::type T2;
            const int32_t* cb = a.cid + base;
            const T2* wb = reinterpret_cast<const T2*>(a.w) + base;
            const char* xpb = reinterpret_cast<const char*>(a.xp);
            uint32_t cc[B];
            T2 ww[B];
#pragma unroll
            for (int u = 0; u < B; ++u) cc[u] = (uint32_t)at_u32(cb, rr[u]);
#pragma unroll
            for (int u = 0; u < B; ++u) ww[u] = at_u32(wb, rr[u]);
            T4 xx[B];  // byte offsets of the packed map fit 32 bits (n_obs < 2^27)
#pragma unroll
            for (int u = 0; u < B; ++u)
                xx[u] = *reinterpret_cast<const T4*>(xpb + cc[u] * (uint32_t)sizeof(T4));
#pragma unroll
            for (int u = 0; u < B; ++u)
                v[u] = ok[u] ? xx[u].x + ww[u].x * xx[u].y + ww[u].y * xx[u].z : (T)0;
        } else if constexpr (MODE == 1) {  // I rows of the map (I-only plans, and IQU maps
                                           // whose Q and U rows are zero: the I weight is 1)
            const int32_t* cb = a.cid + base;
            int32_t cc[B];
#pragma unroll
            for (int u = 0; u < B; ++u) cc[u] = at_u32(cb, rr[u]);
#pragma unroll
            for (int u = 0; u < B; ++u) v[u] = ok[u] ? (T)a.x[cc[u]] : (T)0;
        } else if constexpr (MODE == 2) {  // TOD, FP64
            const double* y = (const double*)a.y + base;
#pragma unroll
            for (int u = 0; u < B; ++u) v[u] = ok[u] ? (T)at_u32(y, rr[u]) : (T)0;
        } else {  // TOD, FP32
            const float* y = (const float*)a.y + base;
#pragma unroll
            for (int u = 0; u < B; ++u) v[u] = ok[u] ? (T)at_u32(y, rr[u]) : (T)0;
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            buf.put_part_sw(sbase ^ swz((b0 + u) * (NT / 2)), part, v[u]);
            nz = nz || v[u] != (T)0;
        }
    }
    return nz;
}

// waves per SIMD that the tile's LDS allows (160 KB per CU, 4 SIMDs per CU), capped where
// the butterflies and gathers would spill (4 waves = 128 VGPRs for FP32, 3 = 170
// for FP64): the register budget the compiler must meet so that LDS bounds occupancy
// the LDS twiddle table of the passes after the first is used where it leaves the tile's
// occupancy (blocks per CU, by LDS and by the 32 waves a CU holds) unchanged
template <typename T, int LOGM, int NT>
constexpr bool ltw_enabled() {
    constexpr int bytes = 2 * (1 << LOGM) * (int)sizeof(T);
    constexpr int tbytes = 2 * ltw_total(LOGM) * (int)sizeof(T);
    constexpr int wmax = 32 / (NT / 64);
    constexpr int b0 = (160 * 1024) / bytes < wmax ? (160 * 1024) / bytes : wmax;
    constexpr int b1 = (160 * 1024) / (bytes + tbytes) < wmax ? (160 * 1024) / (bytes + tbytes)
                                                              : wmax;
    return ltw_total(LOGM) > 0 && b0 == b1;
}

template <typename T, int LOGM, int NT>
constexpr int tile_waves_per_simd() {
    constexpr int bytes = 2 * (1 << LOGM) * (int)sizeof(T);
    constexpr int blocks = (160 * 1024) / bytes;
    constexpr int w = blocks * (NT / 64) / 4;
    constexpr int cap = sizeof(T) == 4 ? 4 : 3;
    return w < 1 ? 1 : (w > cap ? cap : w);
}

// threads of a tile: one radix-16 group per thread and pass
template <int LOGM>
constexpr int tile_threads() {
    constexpr int nt = (1 << LOGM) / 16;
    return nt > 1024 ? 1024 : (nt < 256 ? 256 : nt);
}

// SKIPZ: a tile whose input window is all zero writes zeros and skips the transform (the
// exact result; used for the sparse A Z columns; costs a block vote in LDS)
template <typename T, int LOGM, int NT, int MODE, bool SKIPZ>
__global__ __launch_bounds__(NT, (tile_waves_per_simd<T, LOGM, NT>())) void k_toeplitz(
    ToepArgs<T> a) {
    constexpr int M = 1 << LOGM;
    constexpr bool LTW = ltw_enabled<T, LOGM, NT>();
    __shared__ __align__(16) unsigned char
        smem[2 * M * sizeof(T) + (LTW ? 2 * ltw_total(LOGM) * sizeof(T) : 0)];
    const CBuf<T> buf = make_cbuf<T>(smem, M);
    T* const lt = reinterpret_cast<T*>(smem + 2 * M * sizeof(T));
    if constexpr (SKIPZ) {
        if (blockIdx.y) {
            const int64_t y = blockIdx.y;
            a.x += y * a.x_step;
            a.xp += y * a.xp_step;
            a.z += y * a.z_step;
            if (a.int_on) a.int_on += y * a.on_step;
        }
    }
    // XCD-major tile order (neighbouring tiles share pointing, map and kernel data in one
    // L2), except for zero-skipping launches: there the few non-zero tiles of a sparse
    // column are neighbours and would all land on one XCD
    const int64_t tile = SKIPZ ? (int64_t)blockIdx.x : xcd_item(blockIdx.x, a.n_tiles);
    if (tile < 0 || tile >= a.n_tiles) return;
    const int j = a.tile_int[tile];
    if (a.mask && !a.mask[a.int_prob[j]]) return;
    const int64_t o = a.tile_out[tile];
    const int L = a.tile_len[tile];
    const int64_t lo = a.int_lo[j], hi = a.int_hi[j];
    const int lam = a.lam;
    if constexpr (SKIPZ) {
        if (a.int_on && !a.int_on[j]) {
            for (int i = threadIdx.x; i < L; i += NT) a.z[o + i] = (T)0;
            return;
        }
    }
    // the twiddle table is ordered by the barrier after the load (zero-skipping launches:
    // filled only for non-zero windows, behind a barrier of its own)
    if constexpr (LTW && !SKIPZ) fill_ltw<T, LOGM, NT>(a.tw, lt);
    const bool nz = load_window<T, LOGM, NT, MODE>(a, buf, o - lam, L + 2 * lam, lo, hi);
    if constexpr (SKIPZ) {
        if (!__syncthreads_or(nz)) {  // zero window: the exact result is zero
            for (int i = threadIdx.x; i < L; i += NT) a.z[o + i] = (T)0;
            return;
        }
        if constexpr (LTW) {
            fill_ltw<T, LOGM, NT>(a.tw, lt);
            __syncthreads();
        }
    } else {
        (void)nz;
        __syncthreads();
    }
    if constexpr (LOGM % 4 == 1) {  // the radix-2 stages go into the spectrum pass
        fwd_passes<T, LOGM, NT, LOGM, 1, LTW>(buf, a.tw, lt);
        spectrum_pass_r2<T, LOGM, NT>(buf, a.H + (int64_t)a.int_kern[j] * (M + 1), a.tw);
        inv_passes<T, LOGM, NT, LOGM, 1, LTW>(buf, a.tw, lt);
    } else {
        fwd_passes<T, LOGM, NT, LOGM, 0, LTW>(buf, a.tw, lt);
        spectrum_pass<T, LOGM, NT>(buf, a.H + (int64_t)a.int_kern[j] * (M + 1), a.tw);
        inv_passes<T, LOGM, NT, LOGM, 0, LTW>(buf, a.tw, lt);
    }
    T* zo = a.z + o;  // block-uniform base, 32-bit offsets
    for (int i = lam + threadIdx.x; i < lam + L; i += NT)
        *reinterpret_cast<T*>(reinterpret_cast<char*>(zo) + (uint32_t)(i - lam) * (uint32_t)sizeof(T)) =
            buf.get_part(i >> 1, i & 1);
}

// ------------------------------------------------------------------ plan-time FFTs (FP64)
//
// X_m, m = 0..mmax <= M, of the real sequence packed in (re, im) after the forward
// passes (bit-reversed order): X_m = ((Z_m + conj Z_{M-m}) - i e^{-2 pi i m/N} (Z_m - conj Z_{M-m})) / 2
template <int LOGM, int NT, class Out>
__device__ __forceinline__ void real_dft_out(const CBuf<double>& buf, const double* __restrict__ tw,
                                             int mmax, Out&& out) {
    constexpr int M = 1 << LOGM;
    for (int m = threadIdx.x; m <= mmax; m += NT) {
        double xr, xi;
        if (m == 0 || m == M) {
            double zr, zi;
            buf.get(0, zr, zi);
            xr = m == 0 ? zr + zi : zr - zi;
            xi = 0.0;
        } else {
            double zkr, zki, zmr, zmi;
            buf.get(rev_bits<LOGM>(m), zkr, zki);
            buf.get(rev_bits<LOGM>(M - m), zmr, zmi);
            const double Ar = zkr + zmr, Ai = zki - zmi, Dr = zkr - zmr, Di = zki + zmi;
            const double er = tw[2 * m], ei = tw[2 * m + 1];
            const double pr = er * Dr - ei * Di, pim = er * Di + ei * Dr;
            xr = 0.5 * (Ar + pim);
            xi = 0.5 * (Ai - pr);
        }
        out(m, xr, xi);
    }
}

// symbol on the n_r = 2M grid: H(m) = t_0 + 2 sum_k t_k cos(2 pi k m / n_r), the real DFT
// of the even kernel h (h_0 = t_0, h_k = h_{n_r-k} = t_k for k <= K)
template <int LOGM, int NT>
__global__ __launch_bounds__(NT) void k_spec_fft(const double* __restrict__ taps,
                                                 const int64_t* __restrict__ toff,
                                                 const int64_t* __restrict__ tcnt,
                                                 const double* __restrict__ tw,
                                                 double* __restrict__ H) {
    constexpr int M = 1 << LOGM, NR = 2 * M;
    __shared__ __align__(16) unsigned char smem[2 * M * sizeof(double)];
    const CBuf<double> buf = make_cbuf<double>(smem, M);
    const int g = blockIdx.x;
    const double* t = taps + toff[g];
    const int K = (int)tcnt[g] - 1;
    for (int i = threadIdx.x; i < NR; i += NT) {
        double v = 0.0;
        if (i <= K) v = t[i];
        else if (i >= NR - K) v = t[NR - i];
        buf.put_part(i >> 1, i & 1, v);
    }
    __syncthreads();
    fwd_passes<double, LOGM, NT, LOGM>(buf, tw);
    double* Hg = H + (int64_t)g * (M + 1);
    real_dft_out<LOGM, NT>(buf, tw, M, [&](int m, double xr, double) { Hg[m] = xr; });
}

// taps by decimation in time: for an interval of n = R * 2M samples,
//   t_k = (1/n) sum_{b<R} Re[ e^{2 pi i b k / n} conj(X_b(k)) ],  X_b = real DFT over a of
//   Q(R a + b), Q(m) = q(min(m, n - m)) the inverse PSD on the interval's grid.
// Block (b, g) writes Re[...] for k <= K to part[g][b][k]; k_taps_sum adds over b.
template <int LOGM, int NT>
__global__ __launch_bounds__(NT) void k_taps_fft(const int32_t* __restrict__ kid,
                                                 const int32_t* __restrict__ klen,
                                                 const double* __restrict__ kpar,
                                                 const int64_t* __restrict__ tcnt, double f_samp,
                                                 const double* __restrict__ tw, int kstride,
                                                 int rmax, double* __restrict__ part, int what) {
    constexpr int M = 1 << LOGM, NR = 2 * M;
    __shared__ __align__(16) unsigned char smem[2 * M * sizeof(double)];
    const CBuf<double> buf = make_cbuf<double>(smem, M);
    const int gi = blockIdx.y;
    const int g = kid[gi];
    const int64_t n = klen[g];
    const int R = (int)(n / NR);
    const int b = blockIdx.x;
    if (b >= R) return;
    const double sigma = kpar[3 * g], fk = kpar[3 * g + 1], al = kpar[3 * g + 2];
    for (int i = threadIdx.x; i < NR; i += NT) {
        int64_t m = (int64_t)R * i + b;
        if (m > n - m) m = n - m;
        buf.put_part(i >> 1, i & 1, inv_psd_at(m, n, f_samp, sigma, fk, al, what));
    }
    __syncthreads();
    fwd_passes<double, LOGM, NT, LOGM>(buf, tw);
    const int K = (int)tcnt[g] - 1;
    double* out = part + ((int64_t)gi * rmax + b) * kstride;
    real_dft_out<LOGM, NT>(buf, tw, K, [&](int k, double xr, double xi) {
        double sn, cs;
        sincospi(2.0 * (double)((int64_t)b * k % n) / (double)n, &sn, &cs);
        out[k] = cs * xr + sn * xi;
    });
}

__global__ void k_taps_sum(const int32_t* __restrict__ kid, const int32_t* __restrict__ klen,
                           const int64_t* __restrict__ toff, const int64_t* __restrict__ tcnt,
                           const double* __restrict__ part, int kstride, int rmax, int lam,
                           int window, double* __restrict__ t, int nr) {
    const int gi = blockIdx.y;
    const int g = kid[gi];
    const int64_t n = klen[g];
    const int R = (int)(n / nr);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < tcnt[g];
         k += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < R; ++b) s += part[((int64_t)gi * rmax + b) * kstride + k];
        t[toff[g] + k] = s * window_at(k, lam, window) / (double)n;
    }
}

constexpr int kPlanLogM = 13;  // plan-time FP64 FFTs: n_r = 16384 real points
constexpr int kPlanNT = 512;

template <typename T, int LOGM>
int launch_logm(const ToepArgs<T>& a_in, int64_t n_tiles, hipStream_t st) {
    constexpr int NT = tile_threads<LOGM>();
    ToepArgs<T> a = a_in;
    a.n_tiles = n_tiles;
    const unsigned gx = (unsigned)xcd_grid(n_tiles);
    if (a.skip_zero) {
        const dim3 grid((unsigned)n_tiles, a.layers > 1 ? (unsigned)a.layers : 1u);
        if (a.mode == 0)
            hipLaunchKernelGGL((k_toeplitz<T, LOGM, NT, 0, true>), grid, dim3(NT), 0, st, a);
        else
            hipLaunchKernelGGL((k_toeplitz<T, LOGM, NT, 1, true>), grid, dim3(NT), 0, st, a);
    } else {
        switch (a.mode) {
            case 0: hipLaunchKernelGGL((k_toeplitz<T, LOGM, NT, 0, false>), dim3(gx), dim3(NT), 0, st, a); break;
            case 1: hipLaunchKernelGGL((k_toeplitz<T, LOGM, NT, 1, false>), dim3(gx), dim3(NT), 0, st, a); break;
            case 2: hipLaunchKernelGGL((k_toeplitz<T, LOGM, NT, 2, false>), dim3(gx), dim3(NT), 0, st, a); break;
            default: hipLaunchKernelGGL((k_toeplitz<T, LOGM, NT, 3, false>), dim3(gx), dim3(NT), 0, st, a); break;
        }
    }
    MM_HIP(hipGetLastError());
    return MM_OK;
}

template <typename T>
int launch(const ToepArgs<T>& a, int logm, int64_t n_tiles, hipStream_t st) {
    if (n_tiles == 0) return MM_OK;
    if constexpr (sizeof(T) == 4) {
        switch (logm) {
            case 10: return launch_logm<T, 10>(a, n_tiles, st);
            case 11: return launch_logm<T, 11>(a, n_tiles, st);
            case 12: return launch_logm<T, 12>(a, n_tiles, st);
            case 13: return launch_logm<T, 13>(a, n_tiles, st);
            case 14: return launch_logm<T, 14>(a, n_tiles, st);
        }
    } else {
        switch (logm) {
            case 10: return launch_logm<T, 10>(a, n_tiles, st);
            case 11: return launch_logm<T, 11>(a, n_tiles, st);
            case 12: return launch_logm<T, 12>(a, n_tiles, st);
            case 13: return launch_logm<T, 13>(a, n_tiles, st);
        }
    }
    set_error("no overlap-save kernel for log2(M) = %d", logm);
    return MM_ERR_ARG;
}

// (I, Q, U) per pixel -> (I, Q, U, 0) in T, one aligned 16/32-byte record per pixel
template <typename T>
__global__ void k_pack_map(const double* __restrict__ x, int64_t n_obs, T* __restrict__ xp) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_obs;
         c += (int64_t)gridDim.x * blockDim.x) {
        xp[4 * c] = (T)x[3 * c];
        xp[4 * c + 1] = (T)x[3 * c + 1];
        xp[4 * c + 2] = (T)x[3 * c + 2];
        xp[4 * c + 3] = (T)0;
    }
}

template <typename T>
int pack_map(mm_plan_t pl, const double* x, T* xp) {
    int64_t g = (pl->n_obs + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_pack_map<T>, dim3(g), dim3(256), 0, pl->stream, x, pl->n_obs, xp);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

template <typename T>
ToepArgs<T> base_args(mm_plan_t pl, const FftTiling& ft) {
    ToepArgs<T> a{};
    a.cid = pl->cid.p;
    a.tile_out = ft.tile_out.p;
    a.tile_len = ft.tile_len.p;
    a.tile_int = ft.tile_int.p;
    a.int_lo = pl->int_lo.p;
    a.int_hi = pl->int_hi.p;
    a.int_kern = pl->int_kern.p;
    a.int_prob = pl->int_prob.p;
    a.lam = pl->opts.lambda;
    if constexpr (sizeof(T) == 8) {
        a.H = ft.H64.p;
        a.tw = ft.tw64.p;
        a.w = pl->w64.p;
    } else {
        a.H = ft.H32.p;
        a.tw = ft.tw32.p;
        a.w = pl->w32.p;
    }
    return a;
}

// t0[g] = t_0 of kernel g (the diagonal of its Toeplitz block)
__global__ void k_gather_t0(const double* __restrict__ taps, const int64_t* __restrict__ toff,
                            int32_t nk, double* __restrict__ t0) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < nk) t0[g] = taps[toff[g]];
}

constexpr int kMaxLogM64 = 13, kMaxLogM32 = 14, kMinLogM = 10;

int64_t count_tiles(const std::vector<int64_t>& off, int64_t lmax) {
    int64_t n = 0;
    for (size_t j = 0; j + 1 < off.size(); ++j) n += (off[j + 1] - off[j] + lmax - 1) / lmax;
    return n;
}

}  // namespace

// ------------------------------------------------------------------ host: kernels

// Windowed taps t_0..t_K of every distinct kernel (what = 0) or of the derivative of the
// inverse PSD with respect to sigma, f_knee or alpha (what = 1, 2, 3), on the host, flat
// with offsets toff and counts tcnt [App. D: the Toeplitz row is the inverse DFT of the
// inverse PSD on the interval's grid].
int kernel_taps_dev(mm_plan_t pl, int what, DBuf<double>& d_t, std::vector<int64_t>& toff,
                    std::vector<int64_t>& tcnt) {
    hipStream_t st = pl->stream;
    const int32_t nk = pl->n_kern;
    const int lam = pl->opts.lambda;
    std::vector<int64_t> aoff(nk), acnt(nk), nper(nk), jcnt(nk);
    toff.assign(nk, 0);
    tcnt.assign(nk, 0);
    std::vector<double> kpar(3 * nk);
    int64_t atot = 0, ttot = 0;
    int64_t amax = 0;
    constexpr int64_t kNs = (int64_t)2 << kPlanLogM;
    std::vector<int32_t> fft_ids;
    for (int g = 0; g < nk; ++g) {
        const int64_t n = pl->h_kern_len[g];
        const int64_t K = std::min<int64_t>(lam, n - 1);
        const bool by_fft = n % kNs == 0 && K < kNs / 2;
        if (by_fft) fft_ids.push_back(g);
        aoff[g] = atot;
        acnt[g] = by_fft ? 0 : n / 2 + 1;
        atot += acnt[g];
        amax = std::max(amax, acnt[g]);
        nper[g] = n;
        tcnt[g] = std::min<int64_t>(lam, n - 1) + 1;
        jcnt[g] = tcnt[g];
        toff[g] = ttot;
        ttot += tcnt[g];
        kpar[3 * g] = pl->h_kern_psd[g].sigma;
        kpar[3 * g + 1] = pl->h_kern_psd[g].f_knee;
        kpar[3 * g + 2] = pl->h_kern_psd[g].alpha;
    }
    DBuf<int32_t> d_klen;
    DBuf<double> d_kpar, d_a;
    DBuf<int64_t> d_aoff, d_acnt, d_nper, d_jcnt, d_toff, d_tcnt;
    MM_TRY(d_klen.alloc(nk));
    MM_TRY(d_kpar.alloc(3 * nk));
    MM_TRY(d_a.alloc(std::max<int64_t>(1, atot)));
    MM_TRY(d_t.alloc(ttot));
    MM_TRY(d_aoff.alloc(nk));
    MM_TRY(d_acnt.alloc(nk));
    MM_TRY(d_nper.alloc(nk));
    MM_TRY(d_jcnt.alloc(nk));
    MM_TRY(d_toff.alloc(nk));
    MM_TRY(d_tcnt.alloc(nk));
    MM_HIP(hipMemcpyAsync(d_klen.p, pl->h_kern_len.data(), nk * 4, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(d_kpar.p, kpar.data(), 3 * nk * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(d_aoff.p, aoff.data(), nk * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(d_acnt.p, acnt.data(), nk * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(d_nper.p, nper.data(), nk * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(d_jcnt.p, jcnt.data(), nk * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(d_toff.p, toff.data(), nk * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(d_tcnt.p, tcnt.data(), nk * 8, hipMemcpyHostToDevice, st));
    {
        const int gx = (int)std::max<int64_t>(1, std::min<int64_t>((amax + 255) / 256, 1024));
        hipLaunchKernelGGL(k_inv_psd, dim3(gx, nk), dim3(256), 0, st, d_klen.p, d_kpar.p,
                           d_aoff.p, d_acnt.p, pl->opts.f_samp, d_a.p, nk, what);
        MM_HIP(hipGetLastError());
        const int64_t jmax = *std::max_element(jcnt.begin(), jcnt.end());
        hipLaunchKernelGGL(k_cos_transform, dim3((jmax + kCtThreads - 1) / kCtThreads, nk),
                           dim3(kCtThreads), 0, st, d_a.p, d_aoff.p, d_acnt.p, d_nper.p, d_jcnt.p,
                           d_toff.p, d_t.p, nk);
        MM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_taps_finish, dim3(std::max<int64_t>(1, (jmax + 255) / 256), nk),
                           dim3(256), 0, st, d_t.p, d_toff.p, d_tcnt.p, d_klen.p, lam,
                           pl->opts.window, nk);
        MM_HIP(hipGetLastError());
    }
    if (!fft_ids.empty()) {
        // decimation-in-time FFT path for interval lengths that are multiples of 2^(kPlanLogM+1)
        const int nf = (int)fft_ids.size();
        int rmax = 1, kmax = 1;
        for (int g : fft_ids) {
            rmax = std::max<int>(rmax, (int)(pl->h_kern_len[g] / kNs));
            kmax = std::max<int>(kmax, (int)tcnt[g]);
        }
        DBuf<double> d_tw, d_part;
        DBuf<int32_t> d_kid;
        MM_TRY(d_tw.alloc(kNs));
        MM_TRY(d_kid.alloc(nf));
        MM_TRY(d_part.alloc((size_t)nf * rmax * kmax));
        hipLaunchKernelGGL(k_twiddles, dim3((kNs / 2 + 255) / 256), dim3(256), 0, st, kNs / 2,
                           kNs, d_tw.p, (float*)nullptr);
        MM_HIP(hipMemcpyAsync(d_kid.p, fft_ids.data(), nf * 4, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL((k_taps_fft<kPlanLogM, kPlanNT>), dim3(rmax, nf), dim3(kPlanNT), 0, st,
                           d_kid.p, d_klen.p, d_kpar.p, d_tcnt.p, pl->opts.f_samp, d_tw.p, kmax,
                           rmax, d_part.p, what);
        MM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_taps_sum, dim3((kmax + 255) / 256, nf), dim3(256), 0, st, d_kid.p,
                           d_klen.p, d_toff.p, d_tcnt.p, d_part.p, kmax, rmax, lam,
                           pl->opts.window, d_t.p, (int)kNs);
        MM_HIP(hipGetLastError());
    }
    // the temporaries above are released in stream order after the kernels that read them
    return MM_OK;
}

int kernel_taps(mm_plan_t pl, int what, std::vector<double>& taps, std::vector<int64_t>& toff,
                std::vector<int64_t>& tcnt) {
    DBuf<double> d_t;
    MM_TRY(kernel_taps_dev(pl, what, d_t, toff, tcnt));
    taps.resize(d_t.n);
    MM_HIP(hipMemcpyAsync(taps.data(), d_t.p, d_t.n * 8, hipMemcpyDeviceToHost, pl->stream));
    MM_HIP(hipStreamSynchronize(pl->stream));
    return MM_OK;
}

int host_taps(mm_plan_t pl) {
    if (!pl->h_taps.empty() || pl->taps.n == 0) return MM_OK;
    std::vector<double> t(pl->taps.n);
    MM_HIP(hipMemcpyAsync(t.data(), pl->taps.p, t.size() * 8, hipMemcpyDeviceToHost, pl->stream));
    MM_HIP(hipStreamSynchronize(pl->stream));
    pl->h_taps.swap(t);
    return MM_OK;
}

int build_kernels(mm_plan_t pl) {
    hipStream_t st = pl->stream;
    // distinct kernels: identical (sigma, f_knee, alpha, length) share taps and spectra
    std::map<std::tuple<double, double, double, int64_t>, int32_t> seen;
    pl->h_int_kern.resize(pl->n_int);
    pl->h_kern_len.clear();
    pl->h_kern_psd.clear();
    for (int32_t j = 0; j < pl->n_int; ++j) {
        const int64_t n = pl->h_off[j + 1] - pl->h_off[j];
        const mm_psd& p = pl->h_psd[j];
        const auto key = std::make_tuple(p.sigma, p.f_knee, p.alpha, n);
        auto it = seen.find(key);
        if (it == seen.end()) {
            const int32_t id = (int32_t)pl->h_kern_len.size();
            seen.emplace(key, id);
            pl->h_kern_len.push_back((int32_t)n);
            pl->h_kern_psd.push_back(p);
            pl->h_int_kern[j] = id;
        } else {
            pl->h_int_kern[j] = it->second;
        }
    }
    const int32_t nk = (int32_t)pl->h_kern_len.size();
    pl->n_kern = nk;
    // taps stay on the device (the spectra are formed there); the host copy is fetched on
    // first use
    pl->h_taps.clear();
    MM_TRY(kernel_taps_dev(pl, 0, pl->taps, pl->h_taps_off, pl->h_taps_cnt));
    MM_TRY(pl->taps_off.alloc(nk));
    MM_TRY(pl->taps_cnt.alloc(nk));
    MM_HIP(hipMemcpyAsync(pl->taps_off.p, pl->h_taps_off.data(), nk * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(pl->taps_cnt.p, pl->h_taps_cnt.data(), nk * 8, hipMemcpyHostToDevice, st));
    MM_TRY(pl->kern_t0.alloc(nk));
    hipLaunchKernelGGL(k_gather_t0, dim3((nk + 255) / 256), dim3(256), 0, st, pl->taps.p,
                       pl->taps_off.p, nk, pl->kern_t0.p);
    MM_HIP(hipGetLastError());
    std::vector<double> t0(nk);
    MM_HIP(hipMemcpyAsync(t0.data(), pl->kern_t0.p, nk * 8, hipMemcpyDeviceToHost, st));
    MM_TRY(pl->int_kern.alloc(pl->n_int));
    MM_HIP(hipMemcpyAsync(pl->int_kern.p, pl->h_int_kern.data(), pl->n_int * 4,
                          hipMemcpyHostToDevice, st));
    std::vector<int64_t> lo(pl->n_int), hi(pl->n_int);
    for (int32_t j = 0; j < pl->n_int; ++j) {
        lo[j] = pl->h_off[j];
        hi[j] = pl->h_off[j + 1];
    }
    MM_TRY(pl->int_lo.alloc(pl->n_int));
    MM_TRY(pl->int_hi.alloc(pl->n_int));
    MM_HIP(hipMemcpyAsync(pl->int_lo.p, lo.data(), pl->n_int * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(pl->int_hi.p, hi.data(), pl->n_int * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipStreamSynchronize(st));
    for (int g = 0; g < nk; ++g) {
        // t_0 = 0 happens only for a 1-sample interval with 1/f noise (its mean, the
        // sample itself, is not weighted); a negative or non-finite diagonal is an error
        if (!(t0[g] >= 0.0) || !std::isfinite(t0[g])) {
            set_error("kernel of interval length %d has t_0 = %g < 0", pl->h_kern_len[g], t0[g]);
            return MM_ERR_NOT_SPD;
        }
    }
    return MM_OK;
}

// ------------------------------------------------------------------ host: tiling + spectra

int build_tiling(mm_plan_t pl, FftTiling& ft, bool fp64, int n_r_request) {
    hipStream_t st = pl->stream;
    const int lam = pl->opts.lambda;
    const int maxlogm = fp64 ? kMaxLogM64 : kMaxLogM32;
    int logm = 0;
    if (n_r_request > 0) {
        int l = 0;
        while ((2 << l) < n_r_request) ++l;
        if ((2 << l) != n_r_request || l < kMinLogM || l > maxlogm) {
            set_error("FFT length %d must be a power of two in [%d, %d]", n_r_request,
                      2 << kMinLogM, 2 << maxlogm);
            return MM_ERR_ARG;
        }
        if ((2 << l) <= 2 * lam) {
            set_error("FFT length %d too short for lambda = %d", n_r_request, lam);
            return MM_ERR_ARG;
        }
        logm = l;
    } else {
        // smallest modelled time: tiles x n_r x (log2 n_r + 4), doubled for a tile whose
        // LDS leaves room for only one resident tile per CU (160 KB): a second tile hides
        // the other's window load (measured: 32768-point FP32 tiles at lambda = 4096 take
        // 1.27x the time of 16384-point ones, for 0.72x the modelled work)
        double best = 0.0;
        for (int l = kMinLogM; l <= maxlogm; ++l) {
            const int64_t nr = (int64_t)2 << l;
            const int64_t lmax = nr - 2 * (int64_t)lam;
            if (lmax < nr / 4) continue;
            const int64_t tile_lds = nr * (fp64 ? 8 : 4);
            const double resident = (160 * 1024) / tile_lds >= 2 ? 1.0 : 2.0;
            const double cost =
                (double)count_tiles(pl->h_off, lmax) * (double)nr * (l + 5) * resident;
            if (logm == 0 || cost < best) {
                best = cost;
                logm = l;
            }
        }
        if (logm == 0) {
            set_error("lambda = %d too large for the %s overlap-save tile (n_r <= %d)", lam,
                      fp64 ? "FP64" : "FP32", 2 << maxlogm);
            return MM_ERR_ARG;
        }
    }
    ft.logm = logm;
    ft.n_r = 2 << logm;
    const int M = 1 << logm;
    const int64_t lmax = (int64_t)ft.n_r - 2 * (int64_t)lam;
    // balanced tiles per interval
    std::vector<int64_t> tout;
    std::vector<int32_t> tlen, tint;
    for (int32_t j = 0; j < pl->n_int; ++j) {
        const int64_t a = pl->h_off[j], b = pl->h_off[j + 1], n = b - a;
        const int64_t nt = (n + lmax - 1) / lmax;
        const int64_t len = (n + nt - 1) / nt;
        for (int64_t i = 0; i < nt; ++i) {
            const int64_t s = a + i * len;
            const int64_t e = std::min(b, s + len);
            if (e <= s) continue;
            tout.push_back(s);
            tlen.push_back((int32_t)(e - s));
            tint.push_back(j);
        }
    }
    ft.n_tiles = (int64_t)tout.size();
    MM_TRY(ft.tile_out.alloc(ft.n_tiles));
    MM_TRY(ft.tile_len.alloc(ft.n_tiles));
    MM_TRY(ft.tile_int.alloc(ft.n_tiles));
    MM_HIP(hipMemcpyAsync(ft.tile_out.p, tout.data(), ft.n_tiles * 8, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(ft.tile_len.p, tlen.data(), ft.n_tiles * 4, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(ft.tile_int.p, tint.data(), ft.n_tiles * 4, hipMemcpyHostToDevice, st));
    // twiddles exp(-2 pi i q / n_r), q < M, in FP64 (the spectra below and FP64 tiles) and
    // FP32 for FP32 tiles
    DBuf<double> d_tw;
    double* tw64 = nullptr;
    if (fp64) {
        MM_TRY(ft.tw64.alloc(2 * M));
        tw64 = ft.tw64.p;
    } else {
        MM_TRY(d_tw.alloc(2 * M));
        MM_TRY(ft.tw32.alloc(2 * M));
        tw64 = d_tw.p;
    }
    hipLaunchKernelGGL(k_twiddles, dim3((M + 255) / 256), dim3(256), 0, st, (int64_t)M,
                       (int64_t)ft.n_r, tw64, fp64 ? (float*)nullptr : ft.tw32.p);
    MM_HIP(hipGetLastError());
    // spectra H(m), m = 0..M, of every kernel on this grid
    const int32_t nk = pl->n_kern;
    DBuf<double> d_h, d_min;
    MM_TRY(d_h.alloc((size_t)nk * (M + 1)));
    MM_TRY(d_min.alloc(nk));
    const double* d_taps = pl->taps.p;
    const int64_t* d_toff = pl->taps_off.p;
    const int64_t* d_tcnt = pl->taps_cnt.p;
    if (logm <= kPlanLogM) {  // FP64 FFT of the even kernel on the tile grid
        switch (logm) {
            case 10:
                hipLaunchKernelGGL((k_spec_fft<10, 256>), dim3(nk), dim3(256), 0, st, d_taps,
                                   d_toff, d_tcnt, tw64, d_h.p);
                break;
            case 11:
                hipLaunchKernelGGL((k_spec_fft<11, 256>), dim3(nk), dim3(256), 0, st, d_taps,
                                   d_toff, d_tcnt, tw64, d_h.p);
                break;
            case 12:
                hipLaunchKernelGGL((k_spec_fft<12, 256>), dim3(nk), dim3(256), 0, st, d_taps,
                                   d_toff, d_tcnt, tw64, d_h.p);
                break;
            default:
                hipLaunchKernelGGL((k_spec_fft<kPlanLogM, kPlanNT>), dim3(nk), dim3(kPlanNT), 0, st,
                                   d_taps, d_toff, d_tcnt, tw64, d_h.p);
                break;
        }
        MM_HIP(hipGetLastError());
    } else {  // 2^15-point tiles (FP32 only): direct cosine sums
        MM_TRY(host_taps(pl));
        std::vector<int64_t> boff(nk), bcnt(nk), nper(nk, ft.n_r), jcnt(nk, M + 1), ooff(nk);
        std::vector<double> b;
        for (int g = 0; g < nk; ++g) {
            boff[g] = (int64_t)b.size();
            bcnt[g] = pl->h_taps_cnt[g];
            const double* t = pl->h_taps.data() + pl->h_taps_off[g];
            for (int64_t k = 0; k < bcnt[g]; ++k) b.push_back((k == 0 ? 1.0 : 2.0) * t[k]);
            ooff[g] = (int64_t)g * (M + 1);
        }
        DBuf<double> d_b;
        DBuf<int64_t> d_boff, d_bcnt, d_nper, d_jcnt, d_ooff;
        MM_TRY(d_b.alloc(b.size()));
        MM_TRY(d_boff.alloc(nk));
        MM_TRY(d_bcnt.alloc(nk));
        MM_TRY(d_nper.alloc(nk));
        MM_TRY(d_jcnt.alloc(nk));
        MM_TRY(d_ooff.alloc(nk));
        MM_HIP(hipMemcpyAsync(d_b.p, b.data(), b.size() * 8, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(d_boff.p, boff.data(), nk * 8, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(d_bcnt.p, bcnt.data(), nk * 8, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(d_nper.p, nper.data(), nk * 8, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(d_jcnt.p, jcnt.data(), nk * 8, hipMemcpyHostToDevice, st));
        MM_HIP(hipMemcpyAsync(d_ooff.p, ooff.data(), nk * 8, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_cos_transform, dim3((M + 1 + kCtThreads - 1) / kCtThreads, nk),
                           dim3(kCtThreads), 0, st, d_b.p, d_boff.p, d_bcnt.p, d_nper.p, d_jcnt.p,
                           d_ooff.p, d_h.p, nk);
        MM_HIP(hipGetLastError());
    }
    const double scale = 1.0 / (double)ft.n_r;
    if (fp64) {
        MM_TRY(ft.H64.alloc((size_t)nk * (M + 1)));
    } else {
        MM_TRY(ft.H32.alloc((size_t)nk * (M + 1)));
    }
    hipLaunchKernelGGL(k_spec_finish, dim3(nk), dim3(256), 0, st, d_h.p, (int64_t)(M + 1),
                       (int64_t)(M + 1), scale, fp64 ? ft.H64.p : nullptr,
                       fp64 ? nullptr : ft.H32.p, d_min.p);
    MM_HIP(hipGetLastError());
    std::vector<double> hmin(nk);
    MM_HIP(hipMemcpyAsync(hmin.data(), d_min.p, nk * 8, hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    for (int g = 0; g < nk; ++g) {
        // The symbol bound applies when the whole band fits in the interval; a shorter
        // interval's block is the (windowed) circulant of its own inverse PSD, which is
        // only semi-definite for 1/f noise (its mean is not weighted).
        if ((int64_t)pl->h_kern_len[g] <= 2 * (int64_t)lam) continue;
        if (!(hmin[g] > 0.0)) {
            set_error("Toeplitz symbol min %.3e <= 0 (kernel %d: sigma=%g f_knee=%g alpha=%g, "
                      "length %d): N^-1 block not positive definite",
                      hmin[g], g, pl->h_kern_psd[g].sigma, pl->h_kern_psd[g].f_knee,
                      pl->h_kern_psd[g].alpha, pl->h_kern_len[g]);
            return MM_ERR_NOT_SPD;
        }
    }
    return MM_OK;
}

// ------------------------------------------------------------------ host: launches

int pack_map64(mm_plan_t pl, const double* x) {
    return pl->n_s == 3 ? pack_map<double>(pl, x, pl->xp64.p) : MM_OK;
}

int pack_map32(mm_plan_t pl, const double* x) {
    return pl->n_s == 3 ? pack_map<float>(pl, x, pl->xp32.p) : MM_OK;
}

int toeplitz_map64(mm_plan_t pl, const double* x, double* z, const int* mask, bool skip_zero,
                   const uint8_t* int_on) {
    auto a = base_args<double>(pl, pl->fft64);
    a.skip_zero = skip_zero;
    a.int_on = skip_zero ? int_on : nullptr;
    a.x = x;
    if (pl->n_s == 3) a.xp = pl->xp64.p;
    a.mode = pl->n_s == 3 ? 0 : 1;
    a.z = z;
    a.mask = mask;
    return launch<double>(a, pl->fft64.logm, pl->fft64.n_tiles, pl->stream);
}

int toeplitz_map64_i(mm_plan_t pl, const double* xi, double* z, const uint8_t* int_on) {
    auto a = base_args<double>(pl, pl->fft64);
    a.skip_zero = 1;
    a.int_on = int_on;
    a.x = xi;
    a.mode = 1;
    a.z = z;
    return launch<double>(a, pl->fft64.logm, pl->fft64.n_tiles, pl->stream);
}

int toeplitz_map32(mm_plan_t pl, const double* x, float* z, const int* mask, bool skip_zero,
                   const uint8_t* int_on) {
    auto a = base_args<float>(pl, pl->fft32);
    a.skip_zero = skip_zero;
    a.int_on = skip_zero ? int_on : nullptr;
    a.x = x;
    if (pl->n_s == 3) a.xp = pl->xp32.p;
    a.mode = pl->n_s == 3 ? 0 : 1;
    a.z = z;
    a.mask = mask;
    return launch<float>(a, pl->fft32.logm, pl->fft32.n_tiles, pl->stream);
}

int toeplitz_map32_layers(mm_plan_t pl, const double* x, int64_t x_step, const float* xp,
                          int64_t xp_step, float* z, int64_t z_step, const uint8_t* int_on,
                          int64_t on_step, int layers) {
    if (layers < 1 || layers > 65535) {
        set_error("toeplitz_map32_layers: %d layers", layers);
        return MM_ERR_ARG;
    }
    auto a = base_args<float>(pl, pl->fft32);
    a.skip_zero = 1;
    a.x = x;
    a.xp = xp;
    a.mode = xp ? 0 : 1;
    a.z = z;
    a.int_on = int_on;
    a.layers = layers;
    a.x_step = x_step;
    a.xp_step = xp_step;
    a.z_step = z_step;
    a.on_step = on_step;
    return launch<float>(a, pl->fft32.logm, pl->fft32.n_tiles, pl->stream);
}

int toeplitz_tod64(mm_plan_t pl, const void* y, int y_f64, double* z) {
    auto a = base_args<double>(pl, pl->fft64);
    a.y = y;
    a.y_f64 = y_f64;
    a.mode = y_f64 ? 2 : 3;
    a.z = z;
    return launch<double>(a, pl->fft64.logm, pl->fft64.n_tiles, pl->stream);
}

int toeplitz_tod32(mm_plan_t pl, const void* y, int y_f64, float* z) {
    auto a = base_args<float>(pl, pl->fft32);
    a.y = y;
    a.y_f64 = y_f64;
    a.mode = y_f64 ? 2 : 3;
    a.z = z;
    return launch<float>(a, pl->fft32.logm, pl->fft32.n_tiles, pl->stream);
}

// ------------------------------------------------------------------ FFT length autotuner
//
// Every admissible tile length is built and its map-mode launch (gather + overlap-save,
// the kernel of A x) timed on the plan's own pointing and intervals; the fastest is
// kept.  Choices are cached per process by the interval-length profile, lambda, n_s
// and precision, so plans of the same workload tune once.

namespace {

void swap_tiling(FftTiling& a, FftTiling& b) {
    std::swap(a.logm, b.logm);
    std::swap(a.n_r, b.n_r);
    std::swap(a.n_tiles, b.n_tiles);
    a.tile_out.swap(b.tile_out);
    a.tile_len.swap(b.tile_len);
    a.tile_int.swap(b.tile_int);
    a.H64.swap(b.H64);
    a.H32.swap(b.H32);
    a.tw64.swap(b.tw64);
    a.tw32.swap(b.tw32);
}

std::mutex g_tune_mu;
std::map<std::vector<int64_t>, int> g_tune_cache;

template <typename T>
int time_map_launch(mm_plan_t pl, FftTiling& ft, T* xp, const double* x, T* z, float* ms) {
    auto a = base_args<T>(pl, ft);
    a.x = x;
    a.xp = xp;
    a.mode = pl->n_s == 3 ? 0 : 1;
    a.z = z;
    hipEvent_t e0, e1;
    MM_HIP(hipEventCreate(&e0));
    MM_HIP(hipEventCreate(&e1));
    int s = launch<T>(a, ft.logm, ft.n_tiles, pl->stream);  // warm-up
    if (s == MM_OK) {
        (void)hipEventRecord(e0, pl->stream);
        for (int r = 0; r < 3 && s == MM_OK; ++r) s = launch<T>(a, ft.logm, ft.n_tiles, pl->stream);
        (void)hipEventRecord(e1, pl->stream);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(ms, e0, e1);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return s;
}

}  // namespace

int autotune_tiling(mm_plan_t pl, FftTiling& ft, bool fp64) {
    const int lam = pl->opts.lambda;
    const int maxlogm = fp64 ? kMaxLogM64 : kMaxLogM32;
    std::vector<int64_t> key;
    key.reserve(pl->n_int + 4);
    key.push_back(fp64);
    key.push_back(lam);
    key.push_back(pl->n_s);
    for (int32_t j = 0; j < pl->n_int; ++j) key.push_back(pl->h_off[j + 1] - pl->h_off[j]);
    int cached = 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) cached = it->second;
    }
    if (cached) return build_tiling(pl, ft, fp64, 2 << cached);
    const int64_t nx = pl->n_obs * pl->n_s;
    DBuf<double> x;
    DBuf<unsigned char> xp, z;
    MM_TRY(x.alloc(nx));
    MM_TRY(xp.alloc((size_t)4 * pl->n_obs * (fp64 ? 8 : 4)));
    MM_TRY(z.alloc((size_t)pl->n_t * (fp64 ? 8 : 4)));
    // a nonzero map (byte pattern 0x3f: 0.747f / 4.8e-4), so no tile takes the zero shortcut
    MM_HIP(hipMemsetAsync(x.p, 0x3f, nx * 8, pl->stream));
    MM_HIP(hipMemsetAsync(xp.p, 0x3f, xp.n, pl->stream));
    int best_l = 0;
    float best_ms = 0.0f;
    for (int l = kMinLogM + 1; l <= maxlogm; ++l) {
        const int64_t nr = (int64_t)2 << l;
        if (nr - 2 * (int64_t)lam < nr / 4) continue;
        FftTiling cand;
        MM_TRY(build_tiling(pl, cand, fp64, (int)nr));
        float ms = 0.0f;
        if (fp64)
            MM_TRY(time_map_launch<double>(pl, cand, (double*)xp.p, x.p, (double*)z.p, &ms));
        else
            MM_TRY(time_map_launch<float>(pl, cand, (float*)xp.p, x.p, (float*)z.p, &ms));
        if (best_l == 0 || ms < best_ms) {
            best_ms = ms;
            best_l = l;
            swap_tiling(ft, cand);
        }
    }
    if (best_l == 0) return build_tiling(pl, ft, fp64, 0);  // reports the error
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best_l;
    return MM_OK;
}

}  // namespace mm
