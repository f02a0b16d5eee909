// Internal declarations shared by the translation units of libmm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mm.h"

namespace mm {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
void clear_error();

#define MM_HIP(call)                                                               \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::mm::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                            __FILE__, __LINE__);                                   \
            return MM_ERR_DEVICE;                                                  \
        }                                                                          \
    } while (0)

#define MM_TRY(expr)               \
    do {                           \
        int s_ = (expr);           \
        if (s_ != MM_OK) return s_; \
    } while (0)

// ---------------------------------------------------------------- device buffers
// Device buffers are stream-ordered allocations (hipMallocAsync) from the device's
// default memory pool, whose release threshold is raised at first use so that memory
// freed by one plan is reused by the next without returning to the driver.  The stream
// is the one current for the calling API entry (set_alloc_stream).
void set_alloc_stream(hipStream_t st);
hipStream_t alloc_stream();
int pool_alloc(void** p, size_t bytes, hipStream_t st);
void pool_free(void* p, hipStream_t st);

template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    hipStream_t st = nullptr;
    int alloc(size_t count) {
        release();
        n = count;
        if (count == 0) return MM_OK;
        st = alloc_stream();
        const int s = pool_alloc(reinterpret_cast<void**>(&p), count * sizeof(T), st);
        if (s != MM_OK) {
            p = nullptr;
            n = 0;
        }
        return s;
    }
    void release() {
        if (p) pool_free(p, st);
        p = nullptr;
        n = 0;
    }
    void swap(DBuf& o) {
        std::swap(p, o.p);
        std::swap(n, o.n);
        std::swap(st, o.st);
    }
    ~DBuf() { release(); }
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
};

// ---------------------------------------------------------------- overlap-save tiling
// One FFT configuration (per precision): tiles of L_max outputs read a window of
// L + 2 lambda samples into a real buffer of n_r = 2^(logm+1) points.
// Workgroups of a launch are dispatched to the chip's kXcds XCDs round-robin by their
// linear index, and each XCD has its own L2.  A launch of n work items (tiles, wave groups)
// over xcd_grid(n) blocks maps block b to item xcd_item(b, n): XCD x (= b mod kXcds) takes
// the contiguous items [x n / kXcds, (x + 1) n / kXcds) (balanced to within one), in order,
// so neighbouring items, which share pointing, map and kernel data, meet in one L2.
// Returns -1 for the blocks of an XCD past its share.
constexpr int kXcds = 8;
__host__ __device__ inline int64_t xcd_grid(int64_t n) { return (n + kXcds - 1) / kXcds * kXcds; }
__host__ __device__ inline int64_t xcd_item(int64_t b, int64_t n) {
    const int64_t x = b % kXcds, j = b / kXcds, q = n / kXcds, r = n % kXcds;
    const int64_t cnt = q + (x < r ? 1 : 0);
    return j < cnt ? x * q + (x < r ? x : r) + j : -1;
}

struct FftTiling {
    int logm = 0;            // complex half-length M = 2^logm, real length n_r = 2M
    int n_r = 0;
    int64_t n_tiles = 0;
    DBuf<int64_t> tile_out;  // first output sample of every tile
    DBuf<int32_t> tile_len;  // outputs of every tile
    DBuf<int32_t> tile_int;  // interval of every tile
    DBuf<double> H64;        // [n_kern][M+1] kernel spectrum / n_r, FP64 operator
    DBuf<float> H32;         // same, FP32 operator
    DBuf<double> tw64;       // [n_r/2][2] exp(-2 pi i q / n_r)
    DBuf<float> tw32;
};

// States of one problem's PCG.  kCheck: the recursive residual met the tolerance or has
// dropped by the replacement ratio since the last true-residual evaluation; the problem
// pauses until the host evaluates b - A x for it.
enum PcgState {
    kActive = 0,
    kCheck = 1,
    kDone = 2,
    kBreakdown = 3,
    kMaxIter = 4,
    kResume = 5,  // true residual evaluated and copied into r; z and p follow
};

// Per-problem PCG scalars.  Every field has one writer per launch: block 0 of the
// problem in the vector kernels, or the problem's block in the one-block-per-problem
// control kernels.
struct PcgScalars {
    double bnorm;     // ||b_b||
    double tol;       // relative tolerance
    double alpha, beta, pq, rr;
    double rel;       // last recursive (or evaluated true) relative residual
    double last_rel;  // true relative residual at the last evaluation (1 at the start)
    int state;        // PcgState
    int status;       // 0 ok, 1 breakdown
    int iter;         // iterations completed
    int iter_next;    // iter + 1 once the current iteration's x, r update ran
    int evals;        // true-residual evaluations that replaced r
    int pad;
};

// Control block of the PCG kernels (passed by value).  A batch of B independent problems
// shares every launch; problem b owns the compact pixels [ooff[b], ooff[b+1]).  Vector
// kernels map block g to (problem b, block k < kVecBlocks of b) through the block offsets
// eblk (elements, n_s per pixel) or pblk (pixels); the partial sums of b go to
// part[(slot * B + b) * kVecBlocks + k], so each problem's reductions follow the same tree
// whatever else is in the batch.
struct PcgCtl {
    double* part = nullptr;      // [kNumSlots][B][kVecBlocks]; nullptr: plain operator call
    PcgScalars* sc = nullptr;    // [B]
    const int* mask = nullptr;   // [B] problems that take part in this launch (nullptr: all)
    int* act = nullptr;          // [B] problems that iterate (cleared when a problem stops)
    double* rz_hist = nullptr;   // [B][hstride] r^T z after every iteration
    double* hist = nullptr;      // [B][hstride] recursive relative residual, or nullptr
    const int32_t* eblk = nullptr;
    const int32_t* pblk = nullptr;
    const int64_t* ooff = nullptr;
    int B = 1;
    int hstride = 0;
    int first = 0;               // update_p: p = z
    int replace = 1;             // recursive convergence triggers a true-residual evaluation
    int max_iter = 0;
    double replace_ratio = 0.0;  // > 0: also evaluate when ||r|| fell by this factor
    // Krylov recording (nullptr: off): z of iteration k of every problem into
    // krylov[k * knv + element] for k < kcap, and the step length of iteration k into
    // alpha_hist[b * hstride + k]
    double* krylov = nullptr;
    double* alpha_hist = nullptr;
    int64_t knv = 0;
    int kcap = 0;
};

// Coarse space, block diagonal over the problems of a batch: problem b keeps the columns
// [col_off[b], col_off[b+1]) (all of them supported on its own pixels), its AZ block is
// [r_b][n_b] column-major at az_off[b] (n_b = n_s * its pixels) and its E^-1 block is
// r_b x r_b row-major at einv_off[b].
struct Coarse {
    int kind = 0;                    // 0 none, 1 Z_S (sparse, I rows), 2 Z_D (dense Ritz vectors)
    int r_dedup = 0;                 // columns after removing duplicates (all problems)
    int r_eff = 0;                   // columns kept (independent), all problems
    int r_max = 0;                   // largest r_b
    std::vector<int32_t> cols;       // Z_S: interval of every kept column; Z_D: index of its
                                     // Ritz value among the problem's ascending Ritz values
    std::vector<double> ritz;        // Z_D: Ritz value of every kept column
    std::vector<int32_t> h_col_off;  // [B+1]
    std::vector<int64_t> h_az_off;   // [B+1]
    std::vector<int64_t> h_einv_off; // [B+1]
    std::vector<double> E;           // E blocks, row-major, concatenated like Einv
    DBuf<int32_t> col_off;           // [B+1]
    DBuf<int32_t> col_prob;          // [r_eff] problem of every kept column
    DBuf<int64_t> az_off, einv_off;  // [B+1]
    DBuf<int64_t> csr_ptr;           // [n_obs+1] kept-column entries per pixel
    DBuf<int32_t> csr_col;           // global kept-column index
    DBuf<double> csr_val;
    DBuf<int64_t> csc_beg, csc_end;  // [r_eff] entry range of every kept column
    DBuf<int32_t> csc_row;           // compact pixel (entries of all distinct columns)
    DBuf<double> csc_val;
    DBuf<double> AZ64;               // AZ blocks (FP64 plans)
    DBuf<float> AZ32;                // same (mixed plans)
    // mixed plans with Z_S (opts.az_fp16): AZ for the A-DEF1 apply in FP16 (raw bits), column
    // c of problem b at az16_off[b] + c * ld_b with ld_b = (az16_off[b+1] - az16_off[b]) / r_b
    // a multiple of 8 covering an even number of pixels (the entries past the problem's
    // pixels are 0); entry value times az16_scale[column] is the FP32 AZ entry rounded
    DBuf<uint16_t> AZ16;
    DBuf<int64_t> az16_off;          // [B+1]
    DBuf<double> az16_scale;         // [r_eff] power of two
    DBuf<double> ZD64;               // Z_D blocks, same layout as AZ (FP64 plans)
    DBuf<float> ZD32;                // same (mixed plans)
    DBuf<double> Einv;               // E^-1 blocks
    DBuf<double> w;                  // coarse solution [r_eff]
    DBuf<double> v;                  // coarse right-hand side Z^T r (- (AZ)^T y) [r_eff]
    DBuf<int32_t> vslice;            // [r_eff+1] first Z^T r slice of every kept column
    DBuf<int32_t> slice_col;         // [n_slices] kept column of every slice
    int64_t n_slices = 0;            // slices of 512 entries over all kept columns
    DBuf<double> vpart;              // [n_slices] partial sums of Z^T r
    DBuf<int64_t> ch_off;            // [B+1] first chunk (kZtChunk vector entries) of every problem
    DBuf<double> cpart;              // Z_D: [r_max][n_chunks] chunk partials of Z^T r
    DBuf<double> cpart2;             // [r_max][n_chunks] chunk partials of (AZ)^T y (A-DEF2)
    int64_t n_chunks = 0;
};

}  // namespace mm

struct mm_plan_s {
    int device = 0;
    hipStream_t stream = nullptr;
    mm_opts opts{};
    int n_s = 1;
    int64_t n_t = 0, n_pix = 0, n_obs = 0;
    int32_t n_int = 0;
    // batch of independent problems (1 for a plain plan): problem b owns the intervals
    // [h_pint[b], h_pint[b+1]), the samples [h_samp[b], h_samp[b+1]) and the compact
    // pixels [h_ooff[b], h_ooff[b+1])
    int32_t n_prob = 1;
    std::vector<int32_t> h_pint;
    std::vector<int64_t> h_samp, h_ooff;
    std::vector<int64_t> h_soff;        // [B+1] first padded sorted position of every problem
    std::vector<int64_t> h_pn;          // [B] samples of every problem
    int64_t pt_range = 2048;            // samples per P^T work range
    int64_t n_sorted = 0;               // padded sorted length (problems start 8-aligned)
    mm::DBuf<int32_t> int_prob;         // [n_int] problem of every interval
    mm::DBuf<int64_t> ooff;             // [B+1] compact pixel offsets
    mm::DBuf<int32_t> eblk, pblk;       // [B+1] vector-kernel block offsets (elements, pixels)
    int32_t n_eblk = 0, n_pblk = 0;     // grid sizes of the vector kernels
    std::vector<int64_t> h_off;         // interval offsets
    std::vector<mm_psd> h_psd;
    std::vector<int32_t> h_int_kern;    // interval -> distinct kernel
    std::vector<int32_t> h_kern_len;    // kernel -> interval length n_j
    std::vector<mm_psd> h_kern_psd;
    mm::DBuf<double> taps;              // t_0..t_K of every kernel, flat (FP64)
    mm::DBuf<int64_t> taps_off, taps_cnt;  // [n_kern] offset and count of its taps
    std::vector<int64_t> h_taps_off, h_taps_cnt;
    std::vector<double> h_taps;         // host copy of taps, fetched on first use (host_taps)
    int32_t n_kern = 0;

    // time-ordered data
    mm::DBuf<int32_t> cid;              // compact pixel of every sample
    mm::DBuf<double> w64;               // [n_t][2] (IQU)
    mm::DBuf<float> w32;
    // pixel-sorted data
    mm::DBuf<int32_t> perm;             // sorted position -> sample
    mm::DBuf<double> ws64;              // [n_t][2] weights in sorted order
    mm::DBuf<float> ws32;
    mm::DBuf<int64_t> seg;              // [n_obs+1] first sorted position of every pixel;
                                        // pixel c holds [seg[c], seg[c] + hits[c])
    mm::DBuf<uint64_t> heads;           // segment-start bit per sorted sample
    mm::DBuf<int32_t> wave_pix;         // [n_waves+1] pixel ranges of the P^T waves
    mm::DBuf<int32_t> wave_prob;        // [n_waves] problem of every wave
    mm::DBuf<int64_t> wave_off;         // [B+1] first P^T wave of every problem
    mm::DBuf<int64_t> soff;             // [B+1] h_soff on the device
    int64_t n_waves = 0;
    mm::DBuf<int32_t> obs;              // compact -> original id
    mm::DBuf<int32_t> hits;             // s_p
    // intervals / kernels
    mm::DBuf<int64_t> int_lo, int_hi;
    mm::DBuf<int32_t> int_kern;
    mm::DBuf<double> kern_t0;           // t_0 of every kernel
    mm::FftTiling fft64, fft32;
    // block-Jacobi inverse blocks: 6 unique entries (a00 a01 a02 a11 a12 a22) or 1
    mm::DBuf<double> bj;
    // coarse space
    bool has_coarse = false;
    mm::Coarse co;
    // work buffers
    mm::DBuf<double> tod64a, tod64b;
    mm::DBuf<double> xp64;              // packed map (I, Q, U, 0) for the fused gather
    mm::DBuf<float> xp32;
    mm::DBuf<float> tod32a, tod32b;
    mm::DBuf<double> vec[8];            // PCG vectors [n_obs*n_s]
    mm::DBuf<double> part;              // reduction partials [kNumSlots][B][kVecBlocks]
    mm::DBuf<mm::PcgScalars> sc;        // [B]
    mm::PcgScalars* h_sc = nullptr;     // pinned host mirror [B]
    mm::DBuf<int> act, sel;             // [B] masks: iterating / in a residual evaluation
    mm::DBuf<double> hist;              // residual history [B][hstride]
    mm::DBuf<double> rz_hist;           // r^T z per iteration [B][hstride]
    int hstride = 0;
    // Krylov recording of a solve (set only while mm_coarse_from_krylov runs)
    struct KrylovRec {
        double* basis = nullptr;        // [cap][n_obs * n_s]
        double* alpha = nullptr;        // [B][hstride]
        int cap = 0;
    } krec;
    // captured PCG iteration (one per operator precision / preconditioner MM_BJ, MM_2LVL,
    // MM_ADEF2)
    hipStream_t gstream = nullptr;      // non-blocking stream the graphs are captured on
    hipGraphExec_t gexec[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    struct GraphKey {          // control arguments baked into a captured iteration
        int replace = -1;
        double ratio = 0.0;
        int max_iter = 0;
    } gkey[2][3];
    double plan_ms = 0.0;
    // optional event timing of the hot kernels
    bool prof_on = false;
    struct ProfRec {
        hipEvent_t a, b;
        int tag;     // PCG iteration index of the launch (-1: not part of an iteration)
        bool valid;  // false for launches of iterations that were skipped after convergence
    };
    std::vector<ProfRec> prof_ev[MM_K_COUNT];
    size_t prof_used[MM_K_COUNT] = {};
    ~mm_plan_s();
};

namespace mm {

constexpr int kVecBlocks = 512;   // fixed grid of the vector kernels (deterministic reductions)
constexpr int kVecThreads = 256;
constexpr int kVecPerThreadE = 8;  // elements per thread of a problem's vector grid (sizing)
constexpr int kVecPerThreadP = 1;  // pixels per thread of the per-pixel kernels (sizing)

// ---- sort.hip
int build_pointing(mm_plan_t pl, const int32_t* pix, const void* weights, int wdtype);
// out[0..n] = exclusive scan of in[0..n-1] (int64), out[n] = total, enqueued on st
int scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t st);
// stable LSD radix sort of (key, value) pairs, keys in [0, key_max]; synchronises st
int radix_sort_pairs(const int32_t* keys, const int32_t* vals, int64_t n, int32_t key_max,
                     int32_t* keys_out, int32_t* vals_out, hipStream_t st);

// ---- toeplitz.hip
int build_kernels(mm_plan_t pl);
int build_tiling(mm_plan_t pl, FftTiling& ft, bool fp64, int n_r_request);
// the admissible tile length whose map-mode launch is fastest on this plan's data
int autotune_tiling(mm_plan_t pl, FftTiling& ft, bool fp64);
// windowed taps of every distinct kernel (what 0) or of the inverse-PSD derivative with
// respect to sigma / f_knee / alpha (what 1 / 2 / 3), host, flat with offsets and counts
// host copy of the plan's taps (pl->h_taps), fetched once
int host_taps(mm_plan_t pl);
int kernel_taps(mm_plan_t pl, int what, std::vector<double>& taps, std::vector<int64_t>& toff,
                std::vector<int64_t>& tcnt);

// ---- adjoint.hip
// c[j][k], k = 0..lambda (device, zero past K_j): lag cross-correlations of u and v per interval
int lag_correlations(mm_plan_t pl, const double* u, const double* v, double* c);
// dt[j][i][k] (host [n_int][3][lambda+1]): tap derivatives of every interval
int tap_derivatives(mm_plan_t pl, std::vector<double>& dt);
// TOD and noise-parameter gradients from m_hat and mu = A^-1 g
int adjoint_tod(mm_plan_t pl, const double* m_hat, const double* mu, const void* d, int d_f64,
                void* grad_d, int grad_d_f64, double* grad_psd);
// map-mode N^-1 P x; mask: per-problem flags (nullptr = all problems); the IQU map must
// have been packed by pack_map64/32 first.  skip_zero: tiles whose input window is all
// zero write zeros without a transform; int_on (with skip_zero, optional): per-interval
// flags, 0 where P x is known to vanish on the whole interval (no load either)
int pack_map64(mm_plan_t pl, const double* x);
int pack_map32(mm_plan_t pl, const double* x);
int toeplitz_map64(mm_plan_t pl, const double* x, double* z, const int* mask,
                   bool skip_zero = false, const uint8_t* int_on = nullptr);
int toeplitz_map32(mm_plan_t pl, const double* x, float* z, const int* mask,
                   bool skip_zero = false, const uint8_t* int_on = nullptr);
// zero-skipping N^-1 P of a map whose Q and U rows are zero (or of an I-only plan's map),
// given by its I rows xi (n_obs values): no weights are read; int_on as above
int toeplitz_map64_i(mm_plan_t pl, const double* xi, double* z, const uint8_t* int_on);
// zero-skipping FP32 N^-1 P of `layers` maps at once (blockIdx.y = layer y): layer y
// reads the I rows x + y x_step (xp null: I-only plans, and IQU maps whose Q and U rows
// are zero; no weights are read) or the packed FP32 IQU map xp + y xp_step, and the
// interval flags int_on + y on_step (or none), and writes z + y z_step
int toeplitz_map32_layers(mm_plan_t pl, const double* x, int64_t x_step, const float* xp,
                          int64_t xp_step, float* z, int64_t z_step, const uint8_t* int_on,
                          int64_t on_step, int layers);
int toeplitz_tod64(mm_plan_t pl, const void* y, int y_f64, double* z);
int toeplitz_tod32(mm_plan_t pl, const void* y, int y_f64, float* z);

// ---- pointing.hip
// P^T work ranges (wave_pix, wave_prob, wave_off) for per_wave samples per range
int build_wave_ranges(mm_plan_t pl, int64_t per_wave);
// the P^T range: opts.pt_range, else the fastest candidate (autotune) or the default
int tune_pt_range(mm_plan_t pl);
// x = P^T z for the problems in mask
int scatter64(mm_plan_t pl, const double* z, double* x, const int* mask);
int scatter32(mm_plan_t pl, const float* z, double* x, const int* mask);
// P^T of nc <= kScatterCols FP32 time streams z + k zstride into columns k0 + k of the
// per-problem FP32 blocks of az (block b at blk_off[b], column-major [ncols[b]][n_vec_b]);
// columns at or past ncols[b] are not written.  Each stream's sums are those of scatter32.
constexpr int kScatterCols = 8;
int scatter_cols32(mm_plan_t pl, const float* z, int64_t zstride, int nc, int k0,
                   const int32_t* ncols, const int64_t* blk_off, float* az);
int depoint(mm_plan_t pl, const double* x, void* y, int y_f64);
int build_bj(mm_plan_t pl);
int bj_apply(mm_plan_t pl, const double* r, double* z, const PcgCtl& ctl);

// ---- coarse.hip
int build_coarse(mm_plan_t pl);
// Z_D [Sect. 3.3.2]: column i of problem b is sum_k basis[k][problem b's slice] G_b[k][i]
// (G_b row-major [m_b][r_b]); replaces the plan's coarse space with Z_D, its AZ and E^-1
int build_coarse_dense(mm_plan_t pl, const double* basis, int64_t basis_stride,
                       const std::vector<std::vector<double>>& G, const std::vector<int>& m,
                       const std::vector<std::vector<double>>& theta);
int twolvl_apply(mm_plan_t pl, const double* r, double* z, const PcgCtl& ctl);
// A-DEF2 preconditioner z = R^T M_BD r + Z E^-1 Z^T r (partials of r^T z as ctl asks)
int adef2_apply(mm_plan_t pl, const double* r, double* z, const PcgCtl& ctl);
// A-DEF2 initial guess: x += Z E^-1 Z^T r, r -= AZ E^-1 Z^T r (r = b - A x on entry) for
// the problems in mask (nullptr: all)
int coarse_start(mm_plan_t pl, double* x, double* r, const int* mask = nullptr);
// the kept Z_D blocks, FP64, into out (h_az_off[B] values)
int coarse_dense_columns(mm_plan_t pl, double* out);

// ---- krylov.hip
// Ritz pairs of the Lanczos matrix that m PCG steps (step lengths alpha[0..m), r^T z
// products rz[0..m)) build implicitly: the eigenvalues theta below eps_tol, ascending (at
// most max_cols of them, max_cols <= 0: no cap), and their unit eigenvectors, S row-major
// [m][r]
int ritz_select(const double* alpha, const double* rz, int m, double eps_tol, int max_cols,
                std::vector<double>& theta, std::vector<double>& S);
void drop_graphs(mm_plan_t pl);

// ---- blas.hip (per-problem vector kernels; ctl supplies the batch layout and mask)
int build_batch_layout(mm_plan_t pl);
PcgCtl batch_ctl(mm_plan_t pl);
// part slot `slot` of every masked problem <- partials of a^T b
int vec_dot(mm_plan_t pl, const double* a, const double* b, int slot, const PcgCtl& ctl);
int pcg_update_xr(mm_plan_t pl, double* x, double* r, const double* p, const double* q,
                  const PcgCtl& ctl);
int pcg_update_p(mm_plan_t pl, double* p, const double* z, const PcgCtl& ctl);
// out = b - y for masked problems, with partials of ||out||^2 in the Aux slot
int vec_residual(mm_plan_t pl, const double* b, const double* y, double* out, const PcgCtl& ctl);
int vec_axpby(mm_plan_t pl, double a, const double* x, double b, const double* y, double* out);
int vec_zero_flagged(mm_plan_t pl, double* x, const int* flag, const PcgCtl& ctl);
// control kernels (one block per problem)
int pcg_init(mm_plan_t pl, const PcgCtl& ctl, double tol, int zero_b_done);
int pcg_check(mm_plan_t pl, const PcgCtl& ctl, int initial);
int pcg_decide(mm_plan_t pl, const PcgCtl& ctl);
int pcg_select(mm_plan_t pl, const PcgCtl& ctl);
int pcg_resume(mm_plan_t pl, const PcgCtl& ctl);
int pcg_final(mm_plan_t pl, const PcgCtl& ctl);

// host helpers
int64_t nvec(mm_plan_t pl);
// event timing around a launch (no-op unless profiling is on)
int prof_begin(mm_plan_t pl, int k, int tag = -1);
int prof_end(mm_plan_t pl, int k);
// mark launches recorded since mark[] with tag >= first_skipped as no-ops
void prof_invalidate(mm_plan_t pl, const size_t* mark, int first_skipped);
int apply_A64(mm_plan_t pl, const double* x, double* y, const int* mask);
int apply_A32(mm_plan_t pl, const double* x, double* y, const int* mask);
// A x for mostly-zero x (the coarse-space columns): all-zero tiles skip the transform;
// int_on (optional): per-interval flags, 0 where P x vanishes on the whole interval
int apply_A64_sparse(mm_plan_t pl, const double* x, double* y, const uint8_t* int_on = nullptr);
int apply_A32_sparse(mm_plan_t pl, const double* x, double* y, const uint8_t* int_on = nullptr);
// the same for a map whose Q and U rows are zero, given by its I rows xi (n_obs values)
int apply_A64_sparse_i(mm_plan_t pl, const double* xi, double* y, const uint8_t* int_on);

}  // namespace mm
