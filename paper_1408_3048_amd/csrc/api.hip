// C-ABI entry points (include/mm.h): argument validation, plan construction,
// operator calls, and the PCG / iterative-refinement driver [Sect. 3].
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

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

namespace {

// Freed device blocks are kept for reuse: hipMallocAsync and hipFreeAsync take tens to
// hundreds of microseconds of host time each, and building a plan makes about fifty of
// each.  Requests are rounded up to a size class (1/8 of their power of two); a freed block
// is kept per device and class with an event recorded on the freeing stream, and the
// allocation that reuses it makes its own stream wait on that event, so reuse is
// stream-ordered whatever the streams.  At most kCacheCap bytes are kept per device; past
// that, and when the device runs out of memory, blocks go back to the pool.  No allocation
// or release happens inside a captured stream region.
struct CachedBlock {
    void* p;
    hipEvent_t ev;
};
struct LiveBlock {
    int dev;
    size_t cls;
};
constexpr size_t kCacheCap = (size_t)16 << 30;
std::mutex g_cache_mu;
std::map<std::pair<int, size_t>, std::vector<CachedBlock>> g_cache;
std::map<int, size_t> g_cached_bytes;
std::unordered_map<void*, LiveBlock> g_live;
std::map<int, std::vector<hipEvent_t>> g_events;  // idle events per device

size_t size_class(size_t b) {
    if (b <= 4096) return 4096;
    const int l = 63 - __builtin_clzll((unsigned long long)b);
    const size_t q = (size_t)1 << (l - 3);
    return (b + q - 1) / q * q;
}

// hand every cached block of device dev back to the pool (g_cache_mu held)
void flush_cache(int dev, hipStream_t st) {
    for (auto& kv : g_cache) {
        if (kv.first.first != dev) continue;
        for (const CachedBlock& c : kv.second) {
            (void)hipStreamWaitEvent(st, c.ev, 0);
            (void)hipFreeAsync(c.p, st);
            g_events[dev].push_back(c.ev);
        }
        kv.second.clear();
    }
    g_cached_bytes[dev] = 0;
}

}  // namespace

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
    const size_t cls = size_class(bytes);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find({dev, cls});
    if (it != g_cache.end() && !it->second.empty()) {
        const CachedBlock c = it->second.back();
        it->second.pop_back();
        g_cached_bytes[dev] -= cls;
        g_events[dev].push_back(c.ev);
        const hipError_t e = hipStreamWaitEvent(st, c.ev, 0);
        if (e != hipSuccess) {
            (void)hipFreeAsync(c.p, st);
            set_error("hipStreamWaitEvent failed: %s", hipGetErrorString(e));
            return MM_ERR_DEVICE;
        }
        g_live[c.p] = {dev, cls};
        *p = c.p;
        return MM_OK;
    }
    hipError_t e = hipMallocAsync(p, cls, st);
    if (e == hipErrorOutOfMemory && g_cached_bytes[dev] > 0) {
        (void)hipGetLastError();
        flush_cache(dev, st);
        e = hipMallocAsync(p, cls, st);
    }
    if (e != hipSuccess) {
        set_error("hipMallocAsync(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
        return MM_ERR_DEVICE;
    }
    g_live[*p] = {dev, cls};
    return MM_OK;
}

void pool_free(void* p, hipStream_t st) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) {  // not from pool_alloc
        (void)hipFreeAsync(p, st);
        return;
    }
    const LiveBlock b = it->second;
    g_live.erase(it);
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != b.dev || g_cached_bytes[b.dev] + b.cls > kCacheCap) {
        (void)hipFreeAsync(p, st);
        return;
    }
    hipEvent_t ev = nullptr;
    auto& idle = g_events[b.dev];
    if (!idle.empty()) {
        ev = idle.back();
        idle.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipFreeAsync(p, st);
        return;
    }
    if (hipEventRecord(ev, st) != hipSuccess) {
        idle.push_back(ev);
        (void)hipFreeAsync(p, st);
        return;
    }
    g_cache[{b.dev, b.cls}].push_back({p, ev});
    g_cached_bytes[b.dev] += b.cls;
}

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

static int apply_A64_tag(mm_plan_t pl, const double* x, double* y, const int* mask, int tag) {
    MM_TRY(pack_map64(pl, x));
    MM_TRY(prof_begin(pl, MM_K_NINV64, tag));
    MM_TRY(toeplitz_map64(pl, x, pl->tod64a.p, mask));
    MM_TRY(prof_end(pl, MM_K_NINV64));
    MM_TRY(prof_begin(pl, MM_K_PT64, tag));
    MM_TRY(scatter64(pl, pl->tod64a.p, y, mask));
    return prof_end(pl, MM_K_PT64);
}

static int apply_A32_tag(mm_plan_t pl, const double* x, double* y, const int* mask, int tag) {
    MM_TRY(pack_map32(pl, x));
    MM_TRY(prof_begin(pl, MM_K_NINV32, tag));
    MM_TRY(toeplitz_map32(pl, x, pl->tod32a.p, mask));
    MM_TRY(prof_end(pl, MM_K_NINV32));
    MM_TRY(prof_begin(pl, MM_K_PT32, tag));
    MM_TRY(scatter32(pl, pl->tod32a.p, y, mask));
    return prof_end(pl, MM_K_PT32);
}

int apply_A64(mm_plan_t pl, const double* x, double* y, const int* mask) {
    return apply_A64_tag(pl, x, y, mask, -1);
}

int apply_A64_sparse(mm_plan_t pl, const double* x, double* y, const uint8_t* int_on) {
    MM_TRY(pack_map64(pl, x));
    MM_TRY(toeplitz_map64(pl, x, pl->tod64a.p, nullptr, true, int_on));
    return scatter64(pl, pl->tod64a.p, y, nullptr);
}

int apply_A64_sparse_i(mm_plan_t pl, const double* xi, double* y, const uint8_t* int_on) {
    MM_TRY(toeplitz_map64_i(pl, xi, pl->tod64a.p, int_on));
    return scatter64(pl, pl->tod64a.p, y, nullptr);
}

int apply_A32_sparse(mm_plan_t pl, const double* x, double* y, const uint8_t* int_on) {
    MM_TRY(pack_map32(pl, x));
    MM_TRY(toeplitz_map32(pl, x, pl->tod32a.p, nullptr, true, int_on));
    return scatter32(pl, pl->tod32a.p, y, nullptr);
}

int apply_A32(mm_plan_t pl, const double* x, double* y, const int* mask) {
    return apply_A32_tag(pl, x, y, mask, -1);
}

int gemm_tn_f64(hipStream_t st, const double* A, const double* B, int64_t n, int32_t ra,
                int32_t rb, double* dev_C);

void drop_graphs(mm_plan_t pl) {
    for (auto& row : pl->gexec)
        for (auto& g : row)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
}

namespace {

using clk = std::chrono::steady_clock;

// mixed precision: evaluate the true residual each time the recursive one has dropped
// by this factor since the last evaluation
constexpr double kReplaceRatio = 1e-4;
// iterations launched between two reads of the problem states
constexpr int kChunk = 4;

double ms_since(clk::time_point t0) {
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

int precond(mm_plan_t pl, int pc, const double* r, double* z, const PcgCtl& ctl, int tag = -1) {
    MM_TRY(prof_begin(pl, MM_K_PRECOND, tag));
    MM_TRY(pc == MM_2LVL    ? twolvl_apply(pl, r, z, ctl)
           : pc == MM_ADEF2 ? adef2_apply(pl, r, z, ctl)
                            : bj_apply(pl, r, z, ctl));
    return prof_end(pl, MM_K_PRECOND);
}

int ensure_solver_buffers(mm_plan_t pl, int max_iter) {
    const int hs = max_iter + 2;
    if (pl->hstride < hs) {
        drop_graphs(pl);  // captured launches hold the old pointers
        pl->hstride = hs;
        MM_TRY(pl->rz_hist.alloc((size_t)pl->n_prob * hs));
        MM_TRY(pl->hist.alloc((size_t)pl->n_prob * hs));
    }
    return MM_OK;
}

int read_scalars(mm_plan_t pl) {
    MM_HIP(hipMemcpyAsync(pl->h_sc, pl->sc.p, sizeof(PcgScalars) * pl->n_prob,
                          hipMemcpyDeviceToHost, pl->stream));
    MM_HIP(hipStreamSynchronize(pl->stream));
    return MM_OK;
}

// ||v_b||^2 of every problem on the host (partials from the device, summed in order)
int prob_sq_norms(mm_plan_t pl, const double* v, std::vector<double>& out) {
    PcgCtl c = batch_ctl(pl);
    MM_TRY(vec_dot(pl, v, v, kSlotAux, c));
    const int B = pl->n_prob;
    std::vector<double> h((size_t)B * kVecBlocks);
    MM_HIP(hipMemcpyAsync(h.data(), pl->part.p + (size_t)kSlotAux * B * kVecBlocks,
                          h.size() * 8, hipMemcpyDeviceToHost, pl->stream));
    MM_HIP(hipStreamSynchronize(pl->stream));
    out.assign(B, 0.0);
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < kVecBlocks; ++k) out[b] += h[(size_t)b * kVecBlocks + k];
    return MM_OK;
}

// One PCG iteration for every iterating problem (mask act): q = A p, alpha, x and r,
// convergence test, z = M r, beta and p.  Launch arguments do not change between
// iterations, so the sequence can be captured once and replayed.
int pcg_iteration(mm_plan_t pl, bool op32, double* x, double* r, double* p, double* q,
                  int tag) {
    PcgCtl c = batch_ctl(pl);
    c.mask = pl->act.p;
    MM_TRY(op32 ? apply_A32_tag(pl, p, q, c.mask, tag) : apply_A64_tag(pl, p, q, c.mask, tag));
    MM_TRY(prof_begin(pl, MM_K_VEC, tag));
    MM_TRY(vec_dot(pl, p, q, kSlotPQ, c));
    MM_TRY(pcg_update_xr(pl, x, r, p, q, c));
    MM_TRY(prof_end(pl, MM_K_VEC));
    return MM_OK;
}

struct EngineArgs {
    int pc = MM_BJ;
    bool op32 = false;
    bool x_zero = false;
    double tol = 1e-8;
    int max_iter = 1000;
    bool replace = true;
    double replace_ratio = 0.0;
};

// the part of an iteration after the x, r update
int pcg_iteration_tail(mm_plan_t pl, const EngineArgs& ea, double* r, double* z, double* p,
                       int tag) {
    PcgCtl c = batch_ctl(pl);
    c.mask = pl->act.p;
    c.replace = ea.replace;
    c.replace_ratio = ea.replace_ratio;
    c.max_iter = ea.max_iter;
    MM_TRY(pcg_check(pl, c, 0));
    MM_TRY(precond(pl, ea.pc, r, z, c, tag));
    MM_TRY(prof_begin(pl, MM_K_VEC, tag));
    MM_TRY(pcg_update_p(pl, p, z, c));
    return prof_end(pl, MM_K_VEC);
}

int full_iteration(mm_plan_t pl, const EngineArgs& ea, double* x, double* r, double* z, double* p,
                   double* q, int tag) {
    MM_TRY(pcg_iteration(pl, ea.op32, x, r, p, q, tag));
    return pcg_iteration_tail(pl, ea, r, z, p, tag);
}

// PCG on A x_b = b_b for every problem b of the plan, from x (or x = 0 when x_zero).
// Every decision is taken on the device per problem; the host launches iterations in
// chunks, reads the problem states between chunks and runs the true-residual evaluation
// (FP64 operator) for the problems that asked for one.  On return pl->sc holds the
// per-problem results (state, iterations, evaluations).
int pcg_engine(mm_plan_t pl, const double* b, double* x, const EngineArgs& ea) {
    const int B = pl->n_prob;
    double* r = pl->vec[0].p;
    double* z = pl->vec[1].p;
    double* p = pl->vec[2].p;
    double* q = pl->vec[3].p;
    double* xw = pl->vec[4].p;  // iterate (plan-owned, so captured launches stay valid)
    const int64_t n = nvec(pl);
    hipStream_t st = pl->stream;
    PcgCtl all = batch_ctl(pl);
    all.replace = ea.replace;
    all.replace_ratio = ea.replace_ratio;
    all.max_iter = ea.max_iter;
    MM_HIP(hipMemsetAsync(pl->part.p, 0, pl->part.n * sizeof(double), st));
    if (ea.x_zero) {
        MM_HIP(hipMemsetAsync(xw, 0, n * 8, st));
        MM_HIP(hipMemcpyAsync(r, b, n * 8, hipMemcpyDeviceToDevice, st));
    } else {
        // the initial residual of a given x0 is a true residual: FP64 operator for every
        // precision, so that a start already within tol is judged as the final test would
        MM_HIP(hipMemcpyAsync(xw, x, n * 8, hipMemcpyDeviceToDevice, st));
        MM_TRY(apply_A64(pl, xw, q, nullptr));
        MM_TRY(vec_residual(pl, b, q, r, all));
    }
    // A-DEF2 starts from x0 + Z E^-1 Z^T (b - A x0) [App. B].  Its equivalence to an SPD
    // preconditioner needs Z^T r = 0; where AZ is stored in FP32 (mixed plans) the update
    // r -= AZ w is off by its rounding, so the FP64 operator recomputes r = b - A x.
    if (ea.pc == MM_ADEF2) {
        MM_TRY(coarse_start(pl, xw, r));
        if (!ea.op32 && pl->co.AZ32.p) {
            MM_TRY(apply_A64(pl, xw, q, nullptr));
            MM_TRY(vec_residual(pl, b, q, r, all));
        }
    }
    MM_TRY(vec_dot(pl, b, b, kSlotAux, all));
    MM_TRY(pcg_init(pl, all, ea.tol, 1));
    MM_TRY(vec_zero_flagged(pl, xw, pl->sel.p, all));  // b_b = 0: x_b = 0 exactly
    MM_TRY(pcg_resume(pl, all));                          // clears the flags
    PcgCtl ca = all;
    ca.mask = pl->act.p;
    MM_TRY(vec_dot(pl, r, r, kSlotRR, ca));
    MM_TRY(pcg_check(pl, ca, 1));
    MM_TRY(precond(pl, ea.pc, r, z, ca));
    ca.first = 1;
    MM_TRY(pcg_update_p(pl, p, z, ca));
    MM_TRY(read_scalars(pl));
    auto count = [&](int state) {
        int k = 0;
        for (int i = 0; i < B; ++i) k += pl->h_sc[i].state == state;
        return k;
    };
    // graph of one chunk of kChunk iterations for this operator / preconditioner and control
    // arguments (one launch per chunk: the gaps between graph launches are paid once)
    const bool use_graph = pl->opts.graph != 0 && !pl->prof_on && pl->gstream != nullptr &&
                           pl->stream == pl->gstream;
    const int gi = ea.op32 ? 1 : 0, gj = ea.pc;
    hipGraphExec_t& gx = pl->gexec[gi][gj];
    auto& key = pl->gkey[gi][gj];
    if (use_graph && gx &&
        (key.replace != (int)ea.replace || key.ratio != ea.replace_ratio ||
         key.max_iter != ea.max_iter)) {
        (void)hipGraphExecDestroy(gx);
        gx = nullptr;
    }
    if (use_graph && !gx) {
        hipGraph_t g = nullptr;
        MM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        int s1 = MM_OK;
        for (int c = 0; c < kChunk && s1 == MM_OK; ++c)
            s1 = full_iteration(pl, ea, xw, r, z, p, q, -1);
        const hipError_t e1 = hipStreamEndCapture(st, &g);
        if (s1 != MM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s1;
        }
        MM_HIP(e1);
        const hipError_t e2 = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) gx = nullptr;
        MM_HIP(e2);
        key.replace = (int)ea.replace;
        key.ratio = ea.replace_ratio;
        key.max_iter = ea.max_iter;
    }
    const bool graph_ok = use_graph && gx;
    int host_it = 0;
    const int guard = 4 * ea.max_iter + 64;
    for (int loop = 0; count(kActive) > 0; ++loop) {
        if (loop > guard) {
            set_error("PCG driver did not terminate");
            return MM_ERR_DEVICE;
        }
        size_t mark[MM_K_COUNT];
        for (int k = 0; k < MM_K_COUNT; ++k) mark[k] = pl->prof_used[k];
        const int it0 = B == 1 ? pl->h_sc[0].iter : 0;
        const int chunk_start = host_it;
        if (graph_ok) {
            MM_HIP(hipGraphLaunch(gx, st));
            host_it += kChunk;
        } else {
            for (int c = 0; c < kChunk; ++c, ++host_it)
                MM_TRY(full_iteration(pl, ea, xw, r, z, p, q, host_it));
        }
        MM_TRY(read_scalars(pl));
        if (B == 1) prof_invalidate(pl, mark, chunk_start + (pl->h_sc[0].iter - it0));
        if (count(kCheck) > 0) {
            // true residual b - A x (FP64 operator) of the problems that asked for it
            PcgCtl cs = all;
            cs.mask = pl->sel.p;
            MM_TRY(pcg_select(pl, all));
            MM_TRY(apply_A64(pl, xw, q, pl->sel.p));
            MM_TRY(vec_residual(pl, b, q, r, cs));
            MM_TRY(pcg_decide(pl, cs));
            // A-DEF2: the replaced residual gets the coarse correction again (Z^T r = 0)
            if (ea.pc == MM_ADEF2) MM_TRY(coarse_start(pl, xw, r, pl->sel.p));
            MM_TRY(precond(pl, ea.pc, r, z, cs));
            MM_TRY(pcg_update_p(pl, p, z, cs));
            MM_TRY(pcg_resume(pl, all));
            MM_TRY(read_scalars(pl));
        }
    }
    MM_HIP(hipMemcpyAsync(x, xw, n * 8, hipMemcpyDeviceToDevice, st));
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
    for (auto& row : gexec)
        for (auto& g : row)
            if (g) (void)hipGraphExecDestroy(g);
    if (gstream) {
        (void)hipStreamSynchronize(gstream);
        (void)hipStreamDestroy(gstream);
    }
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
    o->graph = 1;
    o->autotune = 0;
    o->az_fp16 = 1;
}

int mm_plan(mm_plan_t* out, int64_t n_samples, const int32_t* pix, const void* weights,
            int weights_dtype, int64_t n_pix, int32_t n_intervals,
            const int64_t* interval_offsets, const mm_psd* psd, const mm_opts* opts) {
    if (n_intervals < 1) {
        clear_error();
        if (out) *out = nullptr;
        set_error("n_intervals must be >= 1");
        return MM_ERR_ARG;
    }
    const int32_t pint[2] = {0, n_intervals};
    return mm_plan_batched(out, 1, pint, n_samples, pix, weights, weights_dtype, n_pix,
                           n_intervals, interval_offsets, psd, opts);
}

int mm_plan_batched(mm_plan_t* out, int32_t n_problems, const int32_t* problem_intervals,
                    int64_t n_samples, const int32_t* pix, const void* weights,
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
    if (n_problems < 1 || !problem_intervals || problem_intervals[0] != 0 ||
        problem_intervals[n_problems] != n_intervals) {
        set_error("problem_intervals must be given for n_problems >= 1 problems, from 0 to "
                  "n_intervals");
        return MM_ERR_ARG;
    }
    for (int32_t b = 0; b < n_problems; ++b)
        if (problem_intervals[b + 1] <= problem_intervals[b]) {
            set_error("problem_intervals not strictly increasing at %d", b);
            return MM_ERR_ARG;
        }
    if (opts->lambda < 0 || !(opts->f_samp > 0.0) || opts->window < 0 || opts->window > 2 ||
        (opts->precision != MM_FP64 && opts->precision != MM_MIXED) ||
        (opts->coarse != MM_COARSE_NONE && opts->coarse != MM_COARSE_ZS) ||
        !(opts->rank_tol > 0.0) || !(opts->rcond_min >= 0.0) ||
        (opts->az_fp16 != 0 && opts->az_fp16 != 1) ||
        (opts->pt_range != 0 && (opts->pt_range < 256 || opts->pt_range > 65536 ||
                                 (opts->pt_range & (opts->pt_range - 1))))) {
        set_error("invalid mm_opts (lambda >= 0, f_samp > 0, window/precision/coarse enums, "
                  "rank_tol > 0, rcond_min >= 0, az_fp16 0 or 1, pt_range 0 or a power of two "
                  "in [256, 65536])");
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
    pl->n_prob = n_problems;
    pl->h_pint.assign(problem_intervals, problem_intervals + n_problems + 1);
    pl->h_samp.resize(n_problems + 1);
    for (int32_t b = 0; b <= n_problems; ++b) pl->h_samp[b] = interval_offsets[problem_intervals[b]];
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
    if ((s = build_batch_layout(pl)) != MM_OK) return fail(s);
    tick("pointing");
    if ((s = build_kernels(pl)) != MM_OK) return fail(s);
    tick("taps");
    const bool tune64 = opts->autotune && opts->fft_len_f64 == 0;
    const bool tune32 = opts->autotune && opts->fft_len_f32 == 0;
    if ((s = tune64 ? autotune_tiling(pl, pl->fft64, true)
                    : build_tiling(pl, pl->fft64, true, opts->fft_len_f64)) != MM_OK)
        return fail(s);
    tick("tiling64");
    const bool mixed = opts->precision == MM_MIXED;
    if (mixed && (s = tune32 ? autotune_tiling(pl, pl->fft32, false)
                             : build_tiling(pl, pl->fft32, false, opts->fft_len_f32)) != MM_OK)
        return fail(s);
    tick("tiling32");
    // the P^T work ranges before anything that sums over them (block-Jacobi blocks, A Z)
    if (opts->autotune && opts->pt_range == 0 && (s = tune_pt_range(pl)) != MM_OK)
        return fail(s);
    tick("pt_range");
    if ((s = build_bj(pl)) != MM_OK) return fail(s);
    tick("bj");
    const int64_t n = pl->n_obs * pl->n_s;
    if ((s = pl->tod64a.alloc(pl->n_t)) != MM_OK) return fail(s);
    if (pl->n_s == 3 && (s = pl->xp64.alloc(4 * pl->n_obs)) != MM_OK) return fail(s);
    if (pl->n_s == 3 && mixed && (s = pl->xp32.alloc(4 * pl->n_obs)) != MM_OK) return fail(s);
    if (mixed && (s = pl->tod32a.alloc(pl->n_t)) != MM_OK) return fail(s);
    for (auto& v : pl->vec)
        if ((s = v.alloc(n)) != MM_OK) return fail(s);
    if ((s = pl->part.alloc((size_t)kNumSlots * pl->n_prob * kVecBlocks)) != MM_OK) return fail(s);
    // slots past a problem's block count are never written and must read as zero
    if (hipError_t e = hipMemsetAsync(pl->part.p, 0, pl->part.n * sizeof(double), pl->stream);
        e != hipSuccess) {
        set_error("hipMemsetAsync failed: %s", hipGetErrorString(e));
        return fail(MM_ERR_DEVICE);
    }
    if ((s = pl->sc.alloc(pl->n_prob)) != MM_OK) return fail(s);
    if ((s = pl->act.alloc(pl->n_prob)) != MM_OK) return fail(s);
    if ((s = pl->sel.alloc(pl->n_prob)) != MM_OK) return fail(s);
    if (hipHostMalloc((void**)&pl->h_sc, sizeof(PcgScalars) * pl->n_prob, hipHostMallocDefault) !=
        hipSuccess) {
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
int mm_n_problems(mm_plan_t pl) { return pl ? pl->n_prob : -1; }

int mm_problem_pixels(mm_plan_t pl, int64_t* host_out) {
    clear_error();
    if (!pl || !host_out) {
        set_error("NULL argument");
        return MM_ERR_ARG;
    }
    for (int b = 0; b <= pl->n_prob; ++b) host_out[b] = pl->h_ooff[b];
    return MM_OK;
}
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
    if (pl->n_prob == 1) {
        MM_HIP(hipMemcpyAsync(dev_out, pl->perm.p, pl->n_t * 4, hipMemcpyDeviceToDevice,
                              pl->stream));
        return MM_OK;
    }
    // without the alignment gaps between problems
    int64_t o = 0;
    for (int b = 0; b < pl->n_prob; ++b) {
        const int64_t len = pl->h_samp[b + 1] - pl->h_samp[b];
        MM_HIP(hipMemcpyAsync(dev_out + o, pl->perm.p + pl->h_soff[b], len * 4,
                              hipMemcpyDeviceToDevice, pl->stream));
        o += len;
    }
    return MM_OK;
}

int mm_interval_taps(mm_plan_t pl, int32_t j, double* host_out, int cap) {
    if (!pl || j < 0 || j >= pl->n_int) {
        set_error("bad plan or interval index");
        return MM_ERR_ARG;
    }
    MM_TRY(host_taps(pl));
    const int32_t g = pl->h_int_kern[j];
    const double* t = pl->h_taps.data() + pl->h_taps_off[g];
    const int n = (int)pl->h_taps_cnt[g];
    if (host_out)
        for (int k = 0; k < cap && k < n; ++k) host_out[k] = t[k];
    return n;
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
    for (int64_t e = 0; e < (int64_t)pl->co.E.size() && e < cap; ++e) host_out[e] = pl->co.E[e];
    return r;
}

int mm_coarse_problem_columns(mm_plan_t pl, int32_t* host_out, int cap) {
    const int r = mm_coarse_rank(pl);
    if (r < 0) return r;
    for (int b = 0; b <= pl->n_prob && b < cap; ++b) host_out[b] = pl->co.h_col_off[b];
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
    MM_TRY(gemm_tn_f64((hipStream_t)stream, A, B, n, ra, rb, C));
    MM_HIP(hipStreamSynchronize((hipStream_t)stream));
    return MM_OK;
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
    PcgCtl c = batch_ctl(pl);
    c.part = nullptr;
    return bj_apply(pl, r, z, c);
}

int mm_precond_2lvl(mm_plan_t pl, const double* r, double* z) {
    clear_error();
    MM_TRY(check_vec_args(pl, r, z));
    if (!pl->has_coarse) {
        set_error("plan without a coarse space (opts.coarse = MM_COARSE_ZS or "
                  "mm_coarse_from_krylov)");
        return MM_ERR_STATE;
    }
    if (r == z) {
        set_error("r and z may not alias");
        return MM_ERR_ARG;
    }
    PcgCtl c = batch_ctl(pl);
    c.part = nullptr;
    return twolvl_apply(pl, r, z, c);
}

int mm_precond_adef2(mm_plan_t pl, const double* r, double* z) {
    clear_error();
    MM_TRY(check_vec_args(pl, r, z));
    if (!pl->has_coarse) {
        set_error("plan without a coarse space (opts.coarse = MM_COARSE_ZS or "
                  "mm_coarse_from_krylov)");
        return MM_ERR_STATE;
    }
    if (r == z) {
        set_error("r and z may not alias");
        return MM_ERR_ARG;
    }
    PcgCtl c = batch_ctl(pl);
    c.part = nullptr;
    return adef2_apply(pl, r, z, c);
}

int mm_pcg_solve(mm_plan_t pl, const double* b, double* x, int pc, int precision, double tol,
                 int max_iter, mm_solve_info* info) {
    clear_error();
    MM_TRY(check_vec_args(pl, b, x));
    if (pc != MM_BJ && pc != MM_2LVL && pc != MM_ADEF2) {
        set_error("precond must be MM_BJ, MM_2LVL or MM_ADEF2");
        return MM_ERR_ARG;
    }
    if (pc != MM_BJ && !pl->has_coarse) {
        set_error("MM_2LVL and MM_ADEF2 need a coarse space (opts.coarse = MM_COARSE_ZS or "
                  "mm_coarse_from_krylov)");
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
    if (precision == MM_MIXED_IR && pl->n_prob > 1) {
        set_error("MM_MIXED_IR is available for single-problem plans only");
        return MM_ERR_ARG;
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
    const int B = pl->n_prob;
    // the solve runs on the plan's own non-blocking stream (graph capture needs one),
    // ordered after the caller's stream and synchronised before returning
    hipStream_t user = pl->stream;
    AllocStream alloc_scope(user);  // plan buffers always live on the caller's stream
    MM_TRY(ensure_solver_buffers(pl, max_iter));
    if (pl->opts.graph && !pl->gstream)
        MM_HIP(hipStreamCreateWithFlags(&pl->gstream, hipStreamNonBlocking));
    if (pl->opts.graph) {
        MM_HIP(hipStreamSynchronize(user));
        pl->stream = pl->gstream;
    }
    struct Restore {
        mm_plan_t pl;
        hipStream_t user;
        ~Restore() {
            (void)hipStreamSynchronize(pl->stream);
            pl->stream = user;
        }
    } restore{pl, user};
    std::vector<mm_solve_info> loc(B);
    mm_solve_info* inf = info ? info : loc.data();
    for (int i = 0; i < B; ++i) {
        inf[i].iterations = 0;
        inf[i].outer_iterations = 0;
        inf[i].replacements = 0;
        inf[i].history_len = 0;
    }
    std::vector<int> status(B, MM_OK);
    std::vector<std::vector<double>> hist_all(B);
    auto fetch_hist = [&](int bprob, int len, double scale) -> int {
        if (len <= 0) return MM_OK;
        std::vector<double> h(len);
        MM_HIP(hipMemcpy(h.data(), pl->hist.p + (size_t)bprob * pl->hstride, len * 8,
                         hipMemcpyDeviceToHost));
        for (double v : h) hist_all[bprob].push_back(v * scale);
        return MM_OK;
    };
    if (precision == MM_FP64 || precision == MM_MIXED) {
        EngineArgs ea;
        ea.pc = pc;
        ea.op32 = precision == MM_MIXED;
        ea.x_zero = false;
        ea.tol = tol;
        ea.max_iter = max_iter;
        ea.replace = true;
        ea.replace_ratio = ea.op32 ? kReplaceRatio : 0.0;
        MM_TRY(pcg_engine(pl, b, x, ea));
        MM_TRY(read_scalars(pl));
        for (int i = 0; i < B; ++i) {
            const PcgScalars& sc = pl->h_sc[i];
            inf[i].iterations = sc.iter;
            inf[i].outer_iterations = 1;
            inf[i].replacements = sc.evals;
            status[i] = sc.state == kDone ? MM_OK
                        : sc.state == kBreakdown ? MM_ERR_BREAKDOWN : MM_ERR_NOCONV;
            MM_TRY(fetch_hist(i, sc.iter, 1.0));
        }
    } else {
        // iterative refinement: r = b - A64 x; solve A32 d = r by PCG from d = 0; x += d
        std::vector<double> bb;
        MM_TRY(prob_sq_norms(pl, b, bb));
        const double bn = std::sqrt(bb[0]);
        double* rout = pl->vec[5].p;
        double* d = pl->vec[6].p;
        double* tq = pl->vec[7].p;
        int total = 0;
        status[0] = MM_ERR_NOCONV;
        for (int outer = 0; outer < 30 && total < max_iter; ++outer) {
            MM_TRY(apply_A64(pl, x, tq, nullptr));
            MM_TRY(vec_axpby(pl, 1.0, b, -1.0, tq, rout));
            std::vector<double> rr;
            MM_TRY(prob_sq_norms(pl, rout, rr));
            const double rel = bn > 0.0 ? std::sqrt(rr[0]) / bn : 0.0;
            inf[0].outer_iterations = outer;
            if (rel <= tol) {
                status[0] = MM_OK;
                break;
            }
            double eta = 0.1 * tol / rel;
            if (eta < 1e-6) eta = 1e-6;
            if (eta > 0.5) eta = 0.5;
            EngineArgs ea;
            ea.pc = pc;
            ea.op32 = true;
            ea.x_zero = true;
            ea.tol = eta;
            ea.max_iter = max_iter - total;
            ea.replace = false;
            MM_TRY(pcg_engine(pl, rout, d, ea));
            MM_TRY(read_scalars(pl));
            const PcgScalars& sc = pl->h_sc[0];
            MM_TRY(fetch_hist(0, sc.iter, rel));  // relative to ||b||
            total += sc.iter;
            MM_TRY(vec_axpby(pl, 1.0, x, 1.0, d, x));
            if (sc.state == kBreakdown) {
                status[0] = MM_ERR_BREAKDOWN;
                break;
            }
            inf[0].outer_iterations = outer + 1;
        }
        inf[0].iterations = total;
    }
    // final true residual of every problem (FP64 operator)
    {
        PcgCtl all = batch_ctl(pl);
        MM_TRY(vec_dot(pl, b, b, kSlotAux, all));
        MM_TRY(pcg_init(pl, all, tol, 0));  // bnorm per problem
        MM_TRY(apply_A64(pl, x, pl->vec[3].p, nullptr));
        MM_TRY(vec_residual(pl, b, pl->vec[3].p, pl->vec[4].p, all));
        MM_TRY(pcg_final(pl, all));
        MM_TRY(read_scalars(pl));
    }
    int ret = MM_OK;
    for (int i = 0; i < B; ++i) {
        inf[i].rel_residual = pl->h_sc[i].rel;
        if (status[i] == MM_ERR_NOCONV && inf[i].rel_residual <= tol) status[i] = MM_OK;
        // the status follows the final FP64 true residual: a problem the engine stopped
        // on a residual that the FP64 operator does not confirm has not converged
        if (status[i] == MM_OK && !(inf[i].rel_residual <= tol)) status[i] = MM_ERR_NOCONV;
        if (inf[i].history && inf[i].history_cap > 0) {
            const int m = std::min<int>(inf[i].history_cap, (int)hist_all[i].size());
            for (int k = 0; k < m; ++k) inf[i].history[k] = hist_all[i][k];
            inf[i].history_len = m;
        }
        inf[i].status = status[i];
        if (status[i] != MM_OK && ret == MM_OK) ret = status[i];
    }
    MM_HIP(hipStreamSynchronize(pl->stream));
    const double ms = ms_since(t0);
    for (int i = 0; i < B; ++i) inf[i].solve_ms = ms;
    if (ret == MM_ERR_NOCONV && g_err.empty())
        set_error("no convergence to %g within %d iterations", tol, max_iter);
    if (ret == MM_ERR_BREAKDOWN && g_err.empty())
        set_error("PCG breakdown (p^T A p <= 0 or not finite)");
    return ret;
}

int mm_coarse_from_krylov(mm_plan_t pl, const double* b, double* x, double tol, int max_iter,
                          int krylov_dim, double eps_tol, int max_cols, mm_solve_info* info) {
    clear_error();
    MM_TRY(check_vec_args(pl, b, x));
    if (!(tol > 0.0) || max_iter < 1 || krylov_dim < 0 || !(eps_tol > 0.0) || max_cols < 0) {
        set_error("tol > 0, max_iter >= 1, krylov_dim >= 0, eps_tol > 0 and max_cols >= 0 "
                  "required");
        return MM_ERR_ARG;
    }
    if (b == x) {
        set_error("b and x may not alias");
        return MM_ERR_ARG;
    }
    const int B = pl->n_prob;
    const int kcap = krylov_dim > 0 ? std::min(krylov_dim, max_iter) : max_iter;
    const int64_t n = nvec(pl);
    AllocStream alloc_scope(pl->stream);
    MM_TRY(ensure_solver_buffers(pl, max_iter));
    DBuf<double> basis, ahist;
    MM_TRY(basis.alloc((size_t)kcap * n));
    MM_TRY(ahist.alloc((size_t)B * pl->hstride));
    // the recording solve: FP64 operator, block Jacobi, plain launches (a captured
    // iteration would keep the recording pointers)
    struct Recording {
        mm_plan_t pl;
        int graph;
        ~Recording() {
            pl->krec = mm_plan_s::KrylovRec{};
            pl->opts.graph = graph;
            drop_graphs(pl);
        }
    } rec{pl, pl->opts.graph};
    drop_graphs(pl);
    pl->opts.graph = 0;
    pl->krec.basis = basis.p;
    pl->krec.alpha = ahist.p;
    pl->krec.cap = kcap;
    std::vector<mm_solve_info> loc(B);
    mm_solve_info* inf = info ? info : loc.data();
    if (!info)
        for (auto& i : loc) std::memset(&i, 0, sizeof(i));
    const int solve_status = mm_pcg_solve(pl, b, x, MM_BJ, MM_FP64, tol, max_iter, inf);
    if (solve_status != MM_OK && solve_status != MM_ERR_NOCONV) return solve_status;
    const std::string solve_err = g_err;
    // Lanczos data of every problem: alpha_k and r^T z_k for the recorded steps
    const int hs = pl->hstride;
    std::vector<double> ha((size_t)B * hs), hr((size_t)B * hs);
    MM_HIP(hipMemcpyAsync(ha.data(), ahist.p, ha.size() * 8, hipMemcpyDeviceToHost, pl->stream));
    MM_HIP(hipMemcpyAsync(hr.data(), pl->rz_hist.p, hr.size() * 8, hipMemcpyDeviceToHost,
                          pl->stream));
    MM_HIP(hipStreamSynchronize(pl->stream));
    std::vector<std::vector<double>> G(B), theta(B);
    std::vector<int> m(B);
    for (int i = 0; i < B; ++i) {
        m[i] = std::min(inf[i].iterations, kcap);
        std::vector<double> S;
        const double* al = ha.data() + (size_t)i * hs;
        const double* rz = hr.data() + (size_t)i * hs;
        MM_TRY(ritz_select(al, rz, m[i], eps_tol, max_cols, theta[i], S));
        const int r = (int)theta[i].size();
        G[i].resize((size_t)m[i] * r);
        for (int k = 0; k < m[i]; ++k) {
            const double sc = ((k & 1) ? -1.0 : 1.0) / std::sqrt(rz[k]);
            for (int c = 0; c < r; ++c) G[i][(size_t)k * r + c] = sc * S[(size_t)k * r + c];
        }
    }
    MM_TRY(build_coarse_dense(pl, basis.p, n, G, m, theta));
    if (solve_status != MM_OK) g_err = solve_err;
    return solve_status;
}

int mm_lanczos_ritz(const double* alpha, const double* rz, int m, double eps_tol, int max_cols,
                    double* theta_out, double* s_out) {
    clear_error();
    if (!alpha || !rz || m < 1 || !(eps_tol > 0.0) || max_cols < 1 || !theta_out) {
        set_error("alpha, rz, theta_out non-NULL, m >= 1, eps_tol > 0, max_cols >= 1 required");
        return MM_ERR_ARG;
    }
    std::vector<double> theta, S;
    MM_TRY(ritz_select(alpha, rz, m, eps_tol, max_cols, theta, S));
    const int r = (int)theta.size();
    for (int i = 0; i < r; ++i) theta_out[i] = theta[i];
    if (s_out)
        for (size_t e = 0; e < S.size(); ++e) s_out[e] = S[e];
    return r;
}

int mm_coarse_kind(mm_plan_t pl) {
    if (!pl) {
        set_error("plan is NULL");
        return MM_ERR_ARG;
    }
    return pl->has_coarse ? pl->co.kind : 0;
}

int mm_coarse_ritz_values(mm_plan_t pl, double* host_out, int cap) {
    const int r = mm_coarse_rank(pl);
    if (r < 0) return r;
    if (pl->co.kind != 2) {
        set_error("the plan's coarse space is not Z_D");
        return MM_ERR_STATE;
    }
    for (int a = 0; a < r && a < cap; ++a) host_out[a] = pl->co.ritz[a];
    return r;
}

int64_t mm_coarse_dense_columns(mm_plan_t pl, double* dev_out) {
    clear_error();
    const int r = mm_coarse_rank(pl);
    if (r < 0) return r;
    if (pl->co.kind != 2) {
        set_error("the plan's coarse space is not Z_D");
        return MM_ERR_STATE;
    }
    const int64_t total = pl->co.h_az_off[pl->n_prob];
    if (dev_out) MM_TRY(coarse_dense_columns(pl, dev_out));
    return total;
}

double mm_plan_time_ms(mm_plan_t pl) { return pl ? pl->plan_ms : -1.0; }

int mm_lag_correlations(mm_plan_t pl, const double* u, const double* v, double* dev_out) {
    clear_error();
    MM_TRY(check_vec_args(pl, u, v));
    if (!dev_out) {
        set_error("NULL output");
        return MM_ERR_ARG;
    }
    AllocStream alloc_scope(pl->stream);
    return lag_correlations(pl, u, v, dev_out);
}

int mm_tap_derivatives(mm_plan_t pl, double* host_out, int64_t cap) {
    clear_error();
    if (!pl || !host_out) {
        set_error("NULL argument");
        return MM_ERR_ARG;
    }
    AllocStream alloc_scope(pl->stream);
    std::vector<double> dt;
    MM_TRY(tap_derivatives(pl, dt));
    for (int64_t e = 0; e < (int64_t)dt.size() && e < cap; ++e) host_out[e] = dt[e];
    return MM_OK;
}

int mm_adjoint(mm_plan_t pl, const double* m_hat, const double* g, const void* d, int d_dtype,
               int pc, int precision, double tol, int max_iter, double* mu_out, void* grad_d,
               int grad_d_dtype, double* grad_psd, mm_solve_info* info) {
    clear_error();
    MM_TRY(check_vec_args(pl, m_hat, g));
    if (!d || (d_dtype != MM_F32 && d_dtype != MM_F64) ||
        (grad_d && grad_d_dtype != MM_F32 && grad_d_dtype != MM_F64)) {
        set_error("d (and grad_d) need a device pointer and dtype MM_F32 or MM_F64");
        return MM_ERR_ARG;
    }
    DBuf<double> mu_tmp;
    double* mu = mu_out;
    {
        AllocStream alloc_scope(pl->stream);
        if (!mu) {
            MM_TRY(mu_tmp.alloc(nvec(pl)));
            mu = mu_tmp.p;
        }
        MM_HIP(hipMemsetAsync(mu, 0, nvec(pl) * 8, pl->stream));
    }
    const int s = mm_pcg_solve(pl, g, mu, pc, precision, tol, max_iter, info);
    if (s != MM_OK) return s;
    AllocStream alloc_scope(pl->stream);
    MM_TRY(adjoint_tod(pl, m_hat, mu, d, d_dtype == MM_F64, grad_d, grad_d_dtype == MM_F64,
                       grad_psd));
    MM_HIP(hipStreamSynchronize(pl->stream));
    return MM_OK;
}

int mm_fft_lengths(mm_plan_t pl, int* n64, int* n32) {
    clear_error();
    if (!pl || !n64 || !n32) {
        set_error("NULL argument");
        return MM_ERR_ARG;
    }
    *n64 = pl->fft64.n_r;
    *n32 = pl->opts.precision == MM_MIXED ? pl->fft32.n_r : 0;
    return MM_OK;
}

int mm_pt_range(mm_plan_t pl) {
    clear_error();
    if (!pl) {
        set_error("plan is NULL");
        return MM_ERR_ARG;
    }
    return (int)pl->pt_range;
}

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
