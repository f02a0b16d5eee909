// C-ABI entry points (include/mm.h): argument validation, plan construction,
// operator calls, and the PCG / iterative-refinement driver [Sect. 3].
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "mm_device.h"

namespace mm {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}

void clear_error() { g_err.clear(); }

static thread_local hipStream_t g_alloc_stream = nullptr;
void set_alloc_stream(hipStream_t st) { g_alloc_stream = st; }
hipStream_t alloc_stream() { return g_alloc_stream; }

int pool_alloc(void** p, size_t bytes, hipStream_t st) {
    static thread_local int configured_dev = -1;
    int dev = 0;
    MM_HIP(hipGetDevice(&dev));
    if (configured_dev != dev) {
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
        configured_dev = dev;
    }
    hipError_t e = hipMallocAsync(p, bytes, st);
    if (e != hipSuccess) {
        set_error("hipMallocAsync(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
        return MM_ERR_DEVICE;
    }
    return MM_OK;
}

void pool_free(void* p, hipStream_t st) { (void)hipFreeAsync(p, st); }

// RAII: the stream for allocations made during one API call
struct AllocStream {
    hipStream_t prev;
    explicit AllocStream(hipStream_t st) : prev(g_alloc_stream) { g_alloc_stream = st; }
    ~AllocStream() { g_alloc_stream = prev; }
};

int prof_begin(mm_plan_t pl, int k, int tag) {
    if (!pl->prof_on) return MM_OK;
    auto& v = pl->prof_ev[k];
    if (pl->prof_used[k] == v.size()) {
        mm_plan_s::ProfRec r{};
        MM_HIP(hipEventCreate(&r.a));
        MM_HIP(hipEventCreate(&r.b));
        v.push_back(r);
    }
    auto& r = v[pl->prof_used[k]];
    r.tag = tag;
    r.valid = true;
    MM_HIP(hipEventRecord(r.a, pl->stream));
    return MM_OK;
}

int prof_end(mm_plan_t pl, int k) {
    if (!pl->prof_on) return MM_OK;
    MM_HIP(hipEventRecord(pl->prof_ev[k][pl->prof_used[k]].b, pl->stream));
    pl->prof_used[k]++;
    return MM_OK;
}

void prof_invalidate(mm_plan_t pl, const size_t* mark, int first_skipped) {
    if (!pl->prof_on) return;
    for (int k = 0; k < MM_K_COUNT; ++k)
        for (size_t i = mark[k]; i < pl->prof_used[k]; ++i)
            if (pl->prof_ev[k][i].tag >= first_skipped) pl->prof_ev[k][i].valid = false;
}

static int apply_A64_tag(mm_plan_t pl, const double* x, double* y, const int* done, int tag) {
    MM_TRY(prof_begin(pl, MM_K_NINV64, tag));
    MM_TRY(toeplitz_map64(pl, x, pl->tod64a.p, done));
    MM_TRY(prof_end(pl, MM_K_NINV64));
    MM_TRY(prof_begin(pl, MM_K_PT64, tag));
    MM_TRY(scatter64(pl, pl->tod64a.p, y, done));
    return prof_end(pl, MM_K_PT64);
}

static int apply_A32_tag(mm_plan_t pl, const double* x, double* y, const int* done, int tag) {
    MM_TRY(prof_begin(pl, MM_K_NINV32, tag));
    MM_TRY(toeplitz_map32(pl, x, pl->tod32a.p, done));
    MM_TRY(prof_end(pl, MM_K_NINV32));
    MM_TRY(prof_begin(pl, MM_K_PT32, tag));
    MM_TRY(scatter32(pl, pl->tod32a.p, y, done));
    return prof_end(pl, MM_K_PT32);
}

int apply_A64(mm_plan_t pl, const double* x, double* y, const int* done) {
    return apply_A64_tag(pl, x, y, done, -1);
}

int apply_A32(mm_plan_t pl, const double* x, double* y, const int* done) {
    return apply_A32_tag(pl, x, y, done, -1);
}

int gemm_tn_f64(hipStream_t st, const double* A, const double* B, int64_t n, int32_t ra,
                int32_t rb, double* dev_C);

namespace {

using clk = std::chrono::steady_clock;

// mixed precision: replace the recursive residual each time it has dropped this much
constexpr double kReplaceRatio = 1e-2;

double ms_since(clk::time_point t0) {
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

int precond(mm_plan_t pl, int pc, const double* r, double* z, const PcgCtl& ctl, int tag = -1) {
    MM_TRY(prof_begin(pl, MM_K_PRECOND, tag));
    MM_TRY(pc == MM_2LVL ? twolvl_apply(pl, r, z, ctl) : bj_apply(pl, r, z, ctl));
    return prof_end(pl, MM_K_PRECOND);
}

int ensure_solver_buffers(mm_plan_t pl, int max_iter) {
    if (pl->rz_hist.n < (size_t)max_iter + 2) MM_TRY(pl->rz_hist.alloc((size_t)max_iter + 2));
    if (pl->hist.n < (size_t)max_iter + 1) MM_TRY(pl->hist.alloc((size_t)max_iter + 1));
    return MM_OK;
}

int read_scalars(mm_plan_t pl) {
    MM_HIP(hipMemcpyAsync(pl->h_sc, pl->sc.p, sizeof(PcgScalars), hipMemcpyDeviceToHost,
                          pl->stream));
    MM_HIP(hipStreamSynchronize(pl->stream));
    return MM_OK;
}

// ||v||^2 on the host (deterministic device reduction)
int norm2(mm_plan_t pl, const double* v, double* out) {
    double* part = pl->part.p + kSlotAux * kVecBlocks;
    MM_TRY(vec_dot(pl, v, v, part, nullptr));
    std::vector<double> h(kVecBlocks);
    MM_HIP(hipMemcpyAsync(h.data(), part, kVecBlocks * 8, hipMemcpyDeviceToHost, pl->stream));
    MM_HIP(hipStreamSynchronize(pl->stream));
    // same fixed tree as the device prologue reductions is not needed here: a single
    // sequential host sum is deterministic too
    double s = 0.0;
    for (double v2 : h) s += v2;
    *out = s;
    return MM_OK;
}

struct CoreResult {
    int iters = 0;
    int replacements = 0;
    int status = MM_OK;
    int hist_len = 0;
};

// PCG on A x = b from the x passed in.  op32: FP32 operator.  x_zero: x is zero (r = b).
// replace: on recursive convergence test the FP64 true residual and replace r if needed.
int pcg_core(mm_plan_t pl, const double* b, double* x, int pc, bool op32, bool x_zero, double tol,
             int max_iter, bool replace, CoreResult* res, mm_solve_info* info, int hist_off,
             double replace_ratio = 0.0) {
    const int64_t n = nvec(pl);
    double* r = pl->vec[0].p;
    double* z = pl->vec[1].p;
    double* p = pl->vec[2].p;
    double* q = pl->vec[3].p;
    double* t = pl->vec[4].p;
    hipStream_t st = pl->stream;
    PcgCtl ctl;
    ctl.part = pl->part.p;
    ctl.sc = pl->sc.p;
    ctl.rz_hist = pl->rz_hist.p;
    ctl.hist = pl->hist.p;
    const int* done = &pl->sc.p->done;
    auto A = [&](const double* in, double* out, const int* dn, int tag = -1) {
        return op32 ? apply_A32_tag(pl, in, out, dn, tag) : apply_A64_tag(pl, in, out, dn, tag);
    };
    size_t mark[MM_K_COUNT];
    for (int k = 0; k < MM_K_COUNT; ++k) mark[k] = pl->prof_used[k];
    // r = b - A x
    if (x_zero) {
        MM_HIP(hipMemcpyAsync(r, b, n * 8, hipMemcpyDeviceToDevice, st));
    } else {
        MM_TRY(A(x, q, nullptr));
        MM_TRY(vec_axpby(pl, 1.0, b, -1.0, q, r));
    }
    MM_TRY(vec_dot(pl, b, b, pl->part.p + kSlotAux * kVecBlocks, nullptr));
    MM_TRY(vec_set_scalars(pl, ctl, tol, pl->part.p + kSlotAux * kVecBlocks, 0));
    // initial residual test
    MM_TRY(vec_dot(pl, r, r, pl->part.p + kSlotRR * kVecBlocks, nullptr));
    ctl.iter = 0;
    ctl.check = 1;
    ctl.hist = nullptr;
    MM_TRY(precond(pl, pc, r, z, ctl));
    ctl.check = 0;
    ctl.hist = pl->hist.p;
    ctl.iter = -1;
    ctl.first = 1;
    MM_TRY(pcg_update_p(pl, p, z, ctl));
    ctl.first = 0;
    MM_TRY(read_scalars(pl));
    if (pl->h_sc->done) {  // b - A x0 already small enough
        res->iters = 0;
        res->status = MM_OK;
        return MM_OK;
    }
    int i = 0;
    const int chunk = 4;
    double last_rel = 1.0;
    while (i < max_iter) {
        const int i_end = std::min(max_iter, i + chunk);
        for (int it = i; it < i_end; ++it) {
            ctl.iter = it;
            MM_TRY(A(p, q, done, it));
            MM_TRY(prof_begin(pl, MM_K_VEC, it));
            MM_TRY(vec_dot(pl, p, q, pl->part.p + kSlotPQ * kVecBlocks, done));
            MM_TRY(pcg_update_xr(pl, x, r, p, q, ctl));
            MM_TRY(prof_end(pl, MM_K_VEC));
            ctl.check = 1;
            MM_TRY(precond(pl, pc, r, z, ctl, it));
            ctl.check = 0;
            MM_TRY(prof_begin(pl, MM_K_VEC, it));
            MM_TRY(pcg_update_p(pl, p, z, ctl));
            MM_TRY(prof_end(pl, MM_K_VEC));
        }
        MM_TRY(read_scalars(pl));
        i = i_end;
        if (!pl->h_sc->done) {
            // reliable update: the recursive residual has fallen by replace_ratio since the
            // last replacement -> replace it by the FP64 true residual, keep p
            if (replace_ratio > 0.0) {
                const double rel = std::sqrt(pl->h_sc->rr) / pl->h_sc->bnorm;
                if (rel < replace_ratio * last_rel) {
                    const int ndone = pl->h_sc->iter;
                    MM_TRY(apply_A64(pl, x, q, nullptr));
                    MM_TRY(vec_axpby(pl, 1.0, b, -1.0, q, r));
                    double rr = 0.0;
                    MM_TRY(norm2(pl, r, &rr));
                    last_rel = std::sqrt(rr) / pl->h_sc->bnorm;
                    res->replacements++;
                    if (last_rel <= tol) {
                        res->iters = ndone;
                        res->hist_len = ndone;
                        res->status = MM_OK;
                        return MM_OK;
                    }
                    PcgCtl c2 = ctl;
                    c2.iter = ndone - 1;
                    c2.check = 0;
                    c2.hist = nullptr;
                    MM_TRY(precond(pl, pc, r, z, c2));
                    c2.rz_only = 1;
                    MM_TRY(pcg_update_p(pl, p, z, c2));
                }
            }
            continue;
        }
        const int ndone = pl->h_sc->iter;
        prof_invalidate(pl, mark, ndone);
        res->iters = ndone;
        res->hist_len = ndone;
        if (pl->h_sc->status != 0) {
            res->status = MM_ERR_BREAKDOWN;
            set_error("PCG breakdown at iteration %d (p^T A p = %g)", ndone, pl->h_sc->pq);
            return MM_OK;
        }
        if (!replace) {
            res->status = MM_OK;
            return MM_OK;
        }
        // true residual with the FP64 operator
        MM_TRY(apply_A64(pl, x, q, nullptr));
        MM_TRY(vec_axpby(pl, 1.0, b, -1.0, q, t));
        double rr = 0.0;
        MM_TRY(norm2(pl, t, &rr));
        const double rel = std::sqrt(rr) / pl->h_sc->bnorm;
        last_rel = rel;
        if (rel <= tol) {
            res->status = MM_OK;
            return MM_OK;
        }
        // residual replacement, then continue from iteration ndone
        res->replacements++;
        MM_HIP(hipMemcpyAsync(r, t, n * 8, hipMemcpyDeviceToDevice, st));
        const int zero = 0;
        MM_HIP(hipMemcpyAsync(&pl->sc.p->done, &zero, sizeof(int), hipMemcpyHostToDevice, st));
        ctl.iter = ndone - 1;
        ctl.check = 0;
        PcgCtl c2 = ctl;
        c2.hist = nullptr;
        MM_TRY(precond(pl, pc, r, z, c2));
        MM_TRY(pcg_update_p(pl, p, z, ctl));
        i = ndone;
    }
    MM_TRY(read_scalars(pl));
    res->iters = pl->h_sc->iter;
    res->hist_len = res->iters;
    if (pl->h_sc->done && pl->h_sc->status == 0 && !replace) {
        res->status = MM_OK;
        return MM_OK;
    }
    res->status = pl->h_sc->status ? MM_ERR_BREAKDOWN : MM_ERR_NOCONV;
    if (res->status == MM_ERR_NOCONV)
        set_error("PCG did not converge in %d iterations", max_iter);
    return MM_OK;
}

int check_vec_args(mm_plan_t pl, const void* a, const void* b) {
    if (!pl) {
        set_error("plan is NULL");
        return MM_ERR_ARG;
    }
    if (!a || !b) {
        set_error("NULL vector argument");
        return MM_ERR_ARG;
    }
    return MM_OK;
}

}  // namespace
}  // namespace mm

using namespace mm;

mm_plan_s::~mm_plan_s() {
    if (h_sc) (void)hipHostFree(h_sc);
    for (auto& v : prof_ev)
        for (auto& r : v) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
}

extern "C" {

const char* mm_last_error(void) { return g_err.c_str(); }

void mm_default_opts(mm_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->n_stokes = 3;
    o->lambda = 1024;
    o->f_samp = 200.0;
    o->window = MM_WIN_GAUSS;
    o->precision = MM_FP64;
    o->coarse = MM_COARSE_NONE;
    o->rank_tol = 1e-10;
    o->rcond_min = 1e-8;
    o->fft_len_f64 = 0;
    o->fft_len_f32 = 0;
    o->stream = nullptr;
}

int mm_plan(mm_plan_t* out, int64_t n_samples, const int32_t* pix, const void* weights,
            int weights_dtype, int64_t n_pix, int32_t n_intervals,
            const int64_t* interval_offsets, const mm_psd* psd, const mm_opts* opts) {
    clear_error();
    const auto t0 = clk::now();
    if (!out) {
        set_error("out is NULL");
        return MM_ERR_ARG;
    }
    *out = nullptr;
    if (!opts || !pix || !interval_offsets || !psd) {
        set_error("NULL argument (opts, pix, interval_offsets and psd are required)");
        return MM_ERR_ARG;
    }
    if (n_samples < 1 || n_samples >= ((int64_t)1 << 31)) {
        set_error("n_samples = %lld outside [1, 2^31)", (long long)n_samples);
        return MM_ERR_ARG;
    }
    if (opts->n_stokes != 1 && opts->n_stokes != 3) {
        set_error("n_stokes must be 1 or 3 (got %d)", opts->n_stokes);
        return MM_ERR_ARG;
    }
    if (opts->n_stokes == 3 && !weights) {
        set_error("weights are required for n_stokes = 3");
        return MM_ERR_ARG;
    }
    if (opts->n_stokes == 3 && weights_dtype != MM_F32 && weights_dtype != MM_F64) {
        set_error("weights_dtype must be MM_F32 or MM_F64");
        return MM_ERR_ARG;
    }
    if (n_pix < 1 || n_pix > INT32_MAX) {
        set_error("n_pix = %lld outside [1, 2^31)", (long long)n_pix);
        return MM_ERR_ARG;
    }
    if (n_intervals < 1) {
        set_error("n_intervals must be >= 1");
        return MM_ERR_ARG;
    }
    if (interval_offsets[0] != 0 || interval_offsets[n_intervals] != n_samples) {
        set_error("interval_offsets must start at 0 and end at n_samples");
        return MM_ERR_ARG;
    }
    for (int32_t j = 0; j < n_intervals; ++j) {
        if (interval_offsets[j + 1] <= interval_offsets[j]) {
            set_error("interval_offsets not strictly increasing at %d", j);
            return MM_ERR_ARG;
        }
        const mm_psd& p = psd[j];
        if (!(p.sigma > 0.0) || !std::isfinite(p.sigma) || !(p.f_knee >= 0.0) ||
            !std::isfinite(p.f_knee) || !(p.alpha > 0.0) || !std::isfinite(p.alpha)) {
            set_error("interval %d: invalid PSD (sigma=%g f_knee=%g alpha=%g)", j, p.sigma,
                      p.f_knee, p.alpha);
            return MM_ERR_ARG;
        }
    }
    if (opts->lambda < 0 || !(opts->f_samp > 0.0) || opts->window < 0 || opts->window > 2 ||
        (opts->precision != MM_FP64 && opts->precision != MM_MIXED) ||
        (opts->coarse != MM_COARSE_NONE && opts->coarse != MM_COARSE_ZS) ||
        !(opts->rank_tol > 0.0) || !(opts->rcond_min >= 0.0)) {
        set_error("invalid mm_opts (lambda >= 0, f_samp > 0, window/precision/coarse enums, "
                  "rank_tol > 0, rcond_min >= 0)");
        return MM_ERR_ARG;
    }
    mm_plan_s* pl = new mm_plan_s();
    auto fail = [&](int s) {
        delete pl;
        return s;
    };
    pl->opts = *opts;
    pl->n_s = opts->n_stokes;
    pl->n_t = n_samples;
    pl->n_pix = n_pix;
    pl->n_int = n_intervals;
    pl->h_off.assign(interval_offsets, interval_offsets + n_intervals + 1);
    pl->h_psd.assign(psd, psd + n_intervals);
    pl->stream = (hipStream_t)opts->stream;
    AllocStream alloc_scope(pl->stream);
    if (hipGetDevice(&pl->device) != hipSuccess) {
        set_error("no HIP device available");
        return fail(MM_ERR_DEVICE);
    }
    int s;
    const bool verbose = std::getenv("MM_PLAN_TIMING") != nullptr;
    auto tick = [&](const char* what) {
        if (!verbose) return;
        (void)hipStreamSynchronize(pl->stream);
        std::fprintf(stderr, "[mm_plan] %-10s %8.3f ms\n", what, ms_since(t0));
    };
    if ((s = build_pointing(pl, pix, weights, weights_dtype)) != MM_OK) return fail(s);
    tick("pointing");
    if ((s = build_kernels(pl)) != MM_OK) return fail(s);
    tick("taps");
    if ((s = build_tiling(pl, pl->fft64, true, opts->fft_len_f64)) != MM_OK) return fail(s);
    tick("tiling64");
    const bool mixed = opts->precision == MM_MIXED;
    if (mixed && (s = build_tiling(pl, pl->fft32, false, opts->fft_len_f32)) != MM_OK)
        return fail(s);
    tick("tiling32");
    if ((s = build_bj(pl)) != MM_OK) return fail(s);
    tick("bj");
    const int64_t n = pl->n_obs * pl->n_s;
    if ((s = pl->tod64a.alloc(pl->n_t)) != MM_OK) return fail(s);
    if (pl->n_s == 3 && (s = pl->xp64.alloc(4 * pl->n_obs)) != MM_OK) return fail(s);
    if (pl->n_s == 3 && mixed && (s = pl->xp32.alloc(4 * pl->n_obs)) != MM_OK) return fail(s);
    if (mixed && (s = pl->tod32a.alloc(pl->n_t)) != MM_OK) return fail(s);
    for (auto& v : pl->vec)
        if ((s = v.alloc(n)) != MM_OK) return fail(s);
    if ((s = pl->part.alloc(kNumSlots * kVecBlocks)) != MM_OK) return fail(s);
    if ((s = pl->sc.alloc(1)) != MM_OK) return fail(s);
    if (hipHostMalloc((void**)&pl->h_sc, sizeof(PcgScalars), hipHostMallocDefault) != hipSuccess) {
        pl->h_sc = nullptr;
        set_error("hipHostMalloc failed");
        return fail(MM_ERR_DEVICE);
    }
    if ((s = ensure_solver_buffers(pl, 1000)) != MM_OK) return fail(s);
    tick("buffers");
    if (opts->coarse == MM_COARSE_ZS && (s = build_coarse(pl)) != MM_OK) return fail(s);
    tick("coarse");
    if (hipStreamSynchronize(pl->stream) != hipSuccess) {
        set_error("device error during plan construction");
        return fail(MM_ERR_DEVICE);
    }
    pl->plan_ms = ms_since(t0);
    *out = pl;
    return MM_OK;
}

void mm_destroy(mm_plan_t pl) {
    if (!pl) return;
    (void)hipStreamSynchronize(pl->stream);
    delete pl;  // buffers go back to the stream-ordered pool
}

int64_t mm_n_obs(mm_plan_t pl) { return pl ? pl->n_obs : -1; }
int mm_n_stokes(mm_plan_t pl) { return pl ? pl->n_s : -1; }

int mm_obs_pixels(mm_plan_t pl, int32_t* dev_out) {
    MM_TRY(check_vec_args(pl, dev_out, dev_out));
    MM_HIP(hipMemcpyAsync(dev_out, pl->obs.p, pl->n_obs * 4, hipMemcpyDeviceToDevice, pl->stream));
    return MM_OK;
}

int mm_hits(mm_plan_t pl, int32_t* dev_out) {
    MM_TRY(check_vec_args(pl, dev_out, dev_out));
    MM_HIP(hipMemcpyAsync(dev_out, pl->hits.p, pl->n_obs * 4, hipMemcpyDeviceToDevice, pl->stream));
    return MM_OK;
}

int mm_sorted_samples(mm_plan_t pl, int32_t* dev_out) {
    MM_TRY(check_vec_args(pl, dev_out, dev_out));
    MM_HIP(hipMemcpyAsync(dev_out, pl->perm.p, pl->n_t * 4, hipMemcpyDeviceToDevice, pl->stream));
    return MM_OK;
}

int mm_interval_taps(mm_plan_t pl, int32_t j, double* host_out, int cap) {
    if (!pl || j < 0 || j >= pl->n_int) {
        set_error("bad plan or interval index");
        return MM_ERR_ARG;
    }
    const auto& t = pl->h_taps[pl->h_int_kern[j]];
    if (host_out)
        for (int k = 0; k < cap && k < (int)t.size(); ++k) host_out[k] = t[k];
    return (int)t.size();
}

int mm_coarse_rank(mm_plan_t pl) {
    if (!pl) {
        set_error("plan is NULL");
        return MM_ERR_ARG;
    }
    if (!pl->has_coarse) {
        set_error("plan built without a coarse space");
        return MM_ERR_STATE;
    }
    return pl->co.r_eff;
}

int mm_coarse_columns(mm_plan_t pl, int32_t* host_out, int cap) {
    const int r = mm_coarse_rank(pl);
    if (r < 0) return r;
    for (int a = 0; a < r && a < cap; ++a) host_out[a] = pl->co.cols[a];
    return r;
}

int mm_coarse_matrix(mm_plan_t pl, double* host_out, int64_t cap) {
    const int r = mm_coarse_rank(pl);
    if (r < 0) return r;
    for (int64_t e = 0; e < (int64_t)r * r && e < cap; ++e) host_out[e] = pl->co.E[e];
    return r;
}

int mm_gemm_tn_f64(void* stream, const double* A, const double* B, int64_t n, int32_t ra,
                   int32_t rb, double* C) {
    clear_error();
    AllocStream alloc_scope((hipStream_t)stream);
    if (!A || !B || !C || n < 4 || n % 4 || ra < 16 || rb < 16 || ra % 16 || rb % 16) {
        set_error("mm_gemm_tn_f64: n must be a positive multiple of 4, ra and rb multiples of 16");
        return MM_ERR_ARG;
    }
    return gemm_tn_f64((hipStream_t)stream, A, B, n, ra, rb, C);
}

int mm_apply_P(mm_plan_t pl, const double* x, void* y, int y_dtype) {
    clear_error();
    MM_TRY(check_vec_args(pl, x, y));
    if (y_dtype != MM_F32 && y_dtype != MM_F64) {
        set_error("y_dtype must be MM_F32 or MM_F64");
        return MM_ERR_ARG;
    }
    return depoint(pl, x, y, y_dtype == MM_F64);
}

int mm_apply_Ninv(mm_plan_t pl, const void* y, void* z, int precision) {
    clear_error();
    MM_TRY(check_vec_args(pl, y, z));
    if (y == z) {
        set_error("y and z may not alias");
        return MM_ERR_ARG;
    }
    if (precision == MM_FP64) return toeplitz_tod64(pl, y, 1, (double*)z);
    if (precision == MM_MIXED) {
        if (pl->opts.precision != MM_MIXED) {
            set_error("FP32 operator requested from a plan built with precision MM_FP64");
            return MM_ERR_STATE;
        }
        return toeplitz_tod32(pl, y, 0, (float*)z);
    }
    set_error("precision must be MM_FP64 or MM_MIXED");
    return MM_ERR_ARG;
}

int mm_apply_PT(mm_plan_t pl, const void* z, int z_dtype, double* x) {
    clear_error();
    MM_TRY(check_vec_args(pl, z, x));
    if (z_dtype == MM_F64) return scatter64(pl, (const double*)z, x, nullptr);
    if (z_dtype == MM_F32) {
        if (pl->n_s == 3 && !pl->ws32.p) {
            set_error("FP32 pointing requested from a plan built with precision MM_FP64");
            return MM_ERR_STATE;
        }
        return scatter32(pl, (const float*)z, x, nullptr);
    }
    set_error("z_dtype must be MM_F32 or MM_F64");
    return MM_ERR_ARG;
}

int mm_rhs(mm_plan_t pl, const void* d, int d_dtype, double* b) {
    clear_error();
    MM_TRY(check_vec_args(pl, d, b));
    if (d_dtype != MM_F32 && d_dtype != MM_F64) {
        set_error("d_dtype must be MM_F32 or MM_F64");
        return MM_ERR_ARG;
    }
    MM_TRY(toeplitz_tod64(pl, d, d_dtype == MM_F64, pl->tod64a.p));
    return scatter64(pl, pl->tod64a.p, b, nullptr);
}

int mm_apply_A(mm_plan_t pl, const double* x, double* y, int precision) {
    clear_error();
    MM_TRY(check_vec_args(pl, x, y));
    if (x == y) {
        set_error("x and y may not alias");
        return MM_ERR_ARG;
    }
    if (precision == MM_FP64) return apply_A64(pl, x, y, nullptr);
    if (precision == MM_MIXED) {
        if (pl->opts.precision != MM_MIXED) {
            set_error("FP32 operator requested from a plan built with precision MM_FP64");
            return MM_ERR_STATE;
        }
        return apply_A32(pl, x, y, nullptr);
    }
    set_error("precision must be MM_FP64 or MM_MIXED");
    return MM_ERR_ARG;
}

int mm_precond_bj(mm_plan_t pl, const double* r, double* z) {
    clear_error();
    MM_TRY(check_vec_args(pl, r, z));
    return bj_apply(pl, r, z, PcgCtl{});
}

int mm_precond_2lvl(mm_plan_t pl, const double* r, double* z) {
    clear_error();
    MM_TRY(check_vec_args(pl, r, z));
    if (!pl->has_coarse) {
        set_error("plan built without a coarse space (opts.coarse = MM_COARSE_ZS)");
        return MM_ERR_STATE;
    }
    if (r == z) {
        set_error("r and z may not alias");
        return MM_ERR_ARG;
    }
    return twolvl_apply(pl, r, z, PcgCtl{});
}

int mm_pcg_solve(mm_plan_t pl, const double* b, double* x, int pc, int precision, double tol,
                 int max_iter, mm_solve_info* info) {
    clear_error();
    MM_TRY(check_vec_args(pl, b, x));
    if (pc != MM_BJ && pc != MM_2LVL) {
        set_error("precond must be MM_BJ or MM_2LVL");
        return MM_ERR_ARG;
    }
    if (pc == MM_2LVL && !pl->has_coarse) {
        set_error("MM_2LVL needs a plan built with opts.coarse = MM_COARSE_ZS");
        return MM_ERR_STATE;
    }
    if (precision != MM_FP64 && precision != MM_MIXED && precision != MM_MIXED_IR) {
        set_error("precision must be MM_FP64, MM_MIXED or MM_MIXED_IR");
        return MM_ERR_ARG;
    }
    if (precision != MM_FP64 && pl->opts.precision != MM_MIXED) {
        set_error("mixed solve requested from a plan built with precision MM_FP64");
        return MM_ERR_STATE;
    }
    if (!(tol > 0.0) || max_iter < 1) {
        set_error("tol must be > 0 and max_iter >= 1");
        return MM_ERR_ARG;
    }
    if (b == x) {
        set_error("b and x may not alias");
        return MM_ERR_ARG;
    }
    const auto t0 = clk::now();
    AllocStream alloc_scope(pl->stream);
    MM_TRY(ensure_solver_buffers(pl, max_iter));
    mm_solve_info loc{};
    if (!info) info = &loc;
    info->iterations = 0;
    info->outer_iterations = 0;
    info->replacements = 0;
    info->history_len = 0;
    int status = MM_OK;
    std::vector<double> hist_all;
    if (precision == MM_FP64 || precision == MM_MIXED) {
        const bool op32 = precision == MM_MIXED;
        CoreResult res;
        MM_TRY(pcg_core(pl, b, x, pc, op32, false, tol, max_iter, true, &res, info, 0,
                        op32 ? kReplaceRatio : 0.0));
        info->iterations = res.iters;
        info->outer_iterations = 1;
        info->replacements = res.replacements;
        status = res.status;
        if (res.hist_len > 0) {
            hist_all.resize(res.hist_len);
            MM_HIP(hipMemcpy(hist_all.data(), pl->hist.p, res.hist_len * 8, hipMemcpyDeviceToHost));
        }
    } else {
        // iterative refinement: r = b - A64 x; solve A32 d = r by PCG; x += d
        const int64_t n = nvec(pl);
        double bb = 0.0;
        MM_TRY(norm2(pl, b, &bb));
        const double bn = std::sqrt(bb);
        double* rout = pl->vec[5].p;
        double* d = pl->vec[6].p;
        double* tq = pl->vec[7].p;
        int total = 0;
        status = MM_ERR_NOCONV;
        for (int outer = 0; outer < 30 && total < max_iter; ++outer) {
            MM_TRY(apply_A64(pl, x, tq, nullptr));
            MM_TRY(vec_axpby(pl, 1.0, b, -1.0, tq, rout));
            double rr = 0.0;
            MM_TRY(norm2(pl, rout, &rr));
            const double rel = bn > 0.0 ? std::sqrt(rr) / bn : 0.0;
            info->outer_iterations = outer;
            if (rel <= tol) {
                status = MM_OK;
                break;
            }
            double eta = 0.1 * tol / rel;
            if (eta < 1e-6) eta = 1e-6;
            if (eta > 0.5) eta = 0.5;
            MM_HIP(hipMemsetAsync(d, 0, n * 8, pl->stream));
            CoreResult res;
            MM_TRY(pcg_core(pl, rout, d, pc, true, true, eta, max_iter - total, false, &res, info, 0));
            if (res.hist_len > 0) {
                std::vector<double> h(res.hist_len);
                MM_HIP(hipMemcpy(h.data(), pl->hist.p, res.hist_len * 8, hipMemcpyDeviceToHost));
                for (double v : h) hist_all.push_back(v * rel);  // relative to ||b||
            }
            total += res.iters;
            MM_TRY(vec_axpby(pl, 1.0, x, 1.0, d, x));
            if (res.status == MM_ERR_BREAKDOWN) {
                status = MM_ERR_BREAKDOWN;
                break;
            }
            info->outer_iterations = outer + 1;
        }
        info->iterations = total;
    }
    // final true residual (FP64 operator)
    {
        double bb = 0.0, rr = 0.0;
        MM_TRY(norm2(pl, b, &bb));
        MM_TRY(apply_A64(pl, x, pl->vec[3].p, nullptr));
        MM_TRY(vec_axpby(pl, 1.0, b, -1.0, pl->vec[3].p, pl->vec[4].p));
        MM_TRY(norm2(pl, pl->vec[4].p, &rr));
        info->rel_residual = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
        if (status == MM_ERR_NOCONV && info->rel_residual <= tol) status = MM_OK;
    }
    if (info->history && info->history_cap > 0) {
        const int m = std::min<int>(info->history_cap, (int)hist_all.size());
        for (int k = 0; k < m; ++k) info->history[k] = hist_all[k];
        info->history_len = m;
    }
    MM_HIP(hipStreamSynchronize(pl->stream));
    info->solve_ms = ms_since(t0);
    info->status = status;
    if (status == MM_ERR_NOCONV && g_err.empty())
        set_error("no convergence to %g within %d iterations (relres %g)", tol, max_iter,
                  info->rel_residual);
    return status;
}

double mm_plan_time_ms(mm_plan_t pl) { return pl ? pl->plan_ms : -1.0; }

int mm_profile(mm_plan_t pl, int enable) {
    clear_error();
    if (!pl) {
        set_error("plan is NULL");
        return MM_ERR_ARG;
    }
    if (enable) {
        MM_HIP(hipStreamSynchronize(pl->stream));
        for (int k = 0; k < MM_K_COUNT; ++k) pl->prof_used[k] = 0;
    }
    pl->prof_on = enable != 0;
    return MM_OK;
}

int mm_profile_read(mm_plan_t pl, int k, int64_t* launches, double* total_ms) {
    clear_error();
    if (!pl || k < 0 || k >= MM_K_COUNT || !launches || !total_ms) {
        set_error("bad arguments to mm_profile_read");
        return MM_ERR_ARG;
    }
    MM_HIP(hipStreamSynchronize(pl->stream));
    int64_t n = 0;
    double t = 0.0;
    for (size_t i = 0; i < pl->prof_used[k]; ++i) {
        const auto& r = pl->prof_ev[k][i];
        if (!r.valid) continue;
        float ms = 0.0f;
        MM_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        t += ms;
        ++n;
    }
    *launches = n;
    *total_ms = t;
    return MM_OK;
}

}  // extern "C"
