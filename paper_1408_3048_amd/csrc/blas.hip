// Pixel-domain kernels of PCG [Sect. 3.1] for a batch of independent problems:
// fused updates with deterministic per-problem partial sums and device-resident
// per-problem scalars, so the host never waits for a dot product, and the small
// control kernels (one block per problem) that take every convergence decision
// on the device.  A plain plan is a batch of one.
#include <algorithm>
#include <vector>

#include "mm_device.h"

namespace mm {
namespace {

__device__ __forceinline__ bool first_thread(const VecBlock& v) {
    return v.k == 0 && threadIdx.x == 0;
}

// partials of a^T b (per problem) into `slot`
__global__ __launch_bounds__(kVecThreads) void k_dot(const double* __restrict__ a,
                                                     const double* __restrict__ b, int slot,
                                                     int ns, PcgCtl c) {
    __shared__ double red[kVecThreads];
    const VecBlock v = vec_block(c, ns, true);
    if (c.mask && !c.mask[v.b]) return;
    double acc = 0.0;
    for (int64_t i = (int64_t)v.k * kVecThreads + threadIdx.x; i < v.n;
         i += v.stride)
        acc += a[v.base + i] * b[v.base + i];
    write_partial_at(acc, slot_part(c, slot, v.b), v.k, red);
}

// alpha = r^T z / p^T q; x += alpha p; r -= alpha q; partials of ||r||^2
__global__ __launch_bounds__(kVecThreads) void k_update_xr(double* __restrict__ x,
                                                           double* __restrict__ r,
                                                           const double* __restrict__ p,
                                                           const double* __restrict__ q, int ns,
                                                           PcgCtl c) {
    __shared__ double red[kVecThreads];
    const VecBlock v = vec_block(c, ns, true);
    if (c.mask && !c.mask[v.b]) return;
    PcgScalars& s = c.sc[v.b];
    const double pq = reduce_partials(slot_part(c, kSlotPQ, v.b), kVecBlocks, red);
    const double rz = c.rz_hist[(int64_t)v.b * c.hstride + s.iter];
    const bool ok = pq > 0.0 && isfinite(pq) && isfinite(rz);
    if (!ok) {
        if (first_thread(v)) {
            s.status = 1;
            s.state = kBreakdown;
            s.pq = pq;
            c.act[v.b] = 0;
        }
        return;
    }
    const double alpha = rz / pq;
    if (first_thread(v)) {
        s.alpha = alpha;
        s.pq = pq;
        s.iter_next = s.iter + 1;
        if (c.alpha_hist) c.alpha_hist[(int64_t)v.b * c.hstride + s.iter] = alpha;
    }
    double acc = 0.0;
    for (int64_t i = (int64_t)v.k * kVecThreads + threadIdx.x; i < v.n;
         i += v.stride) {
        const int64_t e = v.base + i;
        x[e] += alpha * p[e];
        const double rv = r[e] - alpha * q[e];
        r[e] = rv;
        acc += rv * rv;
    }
    write_partial_at(acc, slot_part(c, kSlotRR, v.b), v.k, red);
}

// beta = r_new^T z_new / r^T z; p = z + beta p (p = z on the first call).  The
// iteration count it = iter is that of the iteration just completed (or of the last
// completed one when resuming after a residual evaluation): r^T z of the new residual
// is stored at rz_hist[it] and divided by rz_hist[it - 1].
__global__ __launch_bounds__(kVecThreads) void k_update_p(double* __restrict__ p,
                                                          const double* __restrict__ z, int ns,
                                                          PcgCtl c) {
    __shared__ double red[kVecThreads];
    const VecBlock v = vec_block(c, ns, true);
    if (c.mask && !c.mask[v.b]) return;
    PcgScalars& s = c.sc[v.b];
    const double rz_new = reduce_partials(slot_part(c, kSlotRZ, v.b), kVecBlocks, red);
    const int it = s.iter;
    double* rh = c.rz_hist + (int64_t)v.b * c.hstride;
    const double beta = c.first ? 0.0 : rz_new / rh[it - 1];
    if (first_thread(v)) {
        rh[it] = rz_new;
        s.beta = beta;
    }
    // Krylov recording: z of this iteration (rewritten when a residual evaluation resumes
    // the same iteration, together with rz_hist[it])
    double* kz = c.krylov && it < c.kcap ? c.krylov + (int64_t)it * c.knv : nullptr;
    for (int64_t i = (int64_t)v.k * kVecThreads + threadIdx.x; i < v.n;
         i += v.stride) {
        const int64_t e = v.base + i;
        const double zv = z[e];
        p[e] = c.first ? zv : zv + beta * p[e];
        if (kz) kz[e] = zv;
    }
}

// out = b - y; partials of ||out||^2 in the Aux slot
__global__ __launch_bounds__(kVecThreads) void k_residual(const double* __restrict__ b,
                                                          const double* __restrict__ y,
                                                          double* __restrict__ out, int ns,
                                                          PcgCtl c) {
    __shared__ double red[kVecThreads];
    const VecBlock v = vec_block(c, ns, true);
    if (c.mask && !c.mask[v.b]) return;
    double acc = 0.0;
    for (int64_t i = (int64_t)v.k * kVecThreads + threadIdx.x; i < v.n;
         i += v.stride) {
        const int64_t e = v.base + i;
        const double t = b[e] - y[e];
        out[e] = t;
        acc += t * t;
    }
    write_partial_at(acc, slot_part(c, kSlotAux, v.b), v.k, red);
}

__global__ __launch_bounds__(kVecThreads) void k_axpby(double a, const double* __restrict__ x,
                                                       double b, const double* __restrict__ y,
                                                       double* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kVecThreads)
        out[i] = a * x[i] + b * y[i];
}

// x_b = 0 for the problems flagged in `flag`
__global__ __launch_bounds__(kVecThreads) void k_zero_flagged(double* __restrict__ x,
                                                              const int* __restrict__ flag,
                                                              int ns, PcgCtl c) {
    const VecBlock v = vec_block(c, ns, true);
    if (!flag[v.b]) return;
    for (int64_t i = (int64_t)v.k * kVecThreads + threadIdx.x; i < v.n;
         i += v.stride)
        x[v.base + i] = 0.0;
}

// ---------------------------------------------------------------- control kernels
// One block per problem b (gridDim.x = B).

// start of a solve: ||b_b|| from the Aux partials; a problem with b_b = 0 is done at
// once (its solution is 0) and flagged in zero_b when zero_b_done is set
__global__ __launch_bounds__(kVecThreads) void k_pcg_init(PcgCtl c, double tol, int zero_b_done,
                                                          int* __restrict__ sel) {
    __shared__ double red[kVecThreads];
    const int b = blockIdx.x;
    const double bb = reduce_partials(slot_part(c, kSlotAux, b), kVecBlocks, red);
    if (threadIdx.x == 0) {
        PcgScalars& s = c.sc[b];
        s.bnorm = sqrt(bb);
        s.tol = tol;
        s.alpha = s.beta = s.pq = s.rr = 0.0;
        s.rel = 1.0;
        s.last_rel = 1.0;
        s.status = 0;
        s.iter = 0;
        s.iter_next = 0;
        s.evals = 0;
        const bool zero = !(bb > 0.0);
        s.state = (zero && zero_b_done) ? kDone : kActive;
        c.act[b] = s.state == kActive;
        sel[b] = zero && zero_b_done;
    }
}

// convergence test on the recursive residual (RR partials) of every iterating problem;
// after an iteration (initial = 0) it also counts the iteration and records the history
__global__ __launch_bounds__(kVecThreads) void k_pcg_check(PcgCtl c, int initial) {
    __shared__ double red[kVecThreads];
    const int b = blockIdx.x;
    if (!c.act[b]) return;
    const double rr = reduce_partials(slot_part(c, kSlotRR, b), kVecBlocks, red);
    if (threadIdx.x != 0) return;
    PcgScalars& s = c.sc[b];
    if (!initial) s.iter = s.iter_next;
    const double rel = sqrt(rr) / s.bnorm;
    s.rr = rr;
    s.rel = rel;
    if (!initial && c.hist) c.hist[(int64_t)b * c.hstride + s.iter - 1] = rel;
    int st = kActive;
    if (rel <= s.tol) st = (!initial && c.replace) ? kCheck : kDone;
    else if (!initial && c.replace_ratio > 0.0 && rel < c.replace_ratio * s.last_rel) st = kCheck;
    else if (!initial && s.iter >= c.max_iter) st = kMaxIter;
    if (st != kActive) {
        s.state = st;
        c.act[b] = 0;
    }
}

// after b - A x of the problems in c.mask (state kCheck) is in r with its Aux partials:
// done when it meets the tolerance, else resume from it (or stop at max_iter)
__global__ __launch_bounds__(kVecThreads) void k_pcg_decide(PcgCtl c, int* __restrict__ sel) {
    __shared__ double red[kVecThreads];
    const int b = blockIdx.x;
    if (!sel[b]) return;
    const double tt = reduce_partials(slot_part(c, kSlotAux, b), kVecBlocks, red);
    if (threadIdx.x != 0) return;
    PcgScalars& s = c.sc[b];
    const double rel = sqrt(tt) / s.bnorm;
    s.last_rel = rel;
    s.rel = rel;
    if (rel <= s.tol) {
        s.state = kDone;
        sel[b] = 0;
    } else if (s.iter >= c.max_iter) {
        s.state = kMaxIter;
        sel[b] = 0;
    } else {
        s.state = kResume;
        s.evals++;
    }
}

// op 0: sel = (state == kCheck); op 1: resumed problems iterate again, sel cleared
__global__ void k_pcg_states(PcgCtl c, int* __restrict__ sel, int op) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= c.B) return;
    PcgScalars& s = c.sc[b];
    if (op == 0) {
        sel[b] = s.state == kCheck;
    } else {
        if (sel[b] && s.state == kResume) {
            s.state = kActive;
            c.act[b] = 1;
        }
        sel[b] = 0;
    }
}

// final true relative residual of every problem from the Aux partials (stored in rel)
__global__ __launch_bounds__(kVecThreads) void k_pcg_final(PcgCtl c) {
    __shared__ double red[kVecThreads];
    const int b = blockIdx.x;
    const double tt = reduce_partials(slot_part(c, kSlotAux, b), kVecBlocks, red);
    if (threadIdx.x == 0) {
        PcgScalars& s = c.sc[b];
        s.rel = s.bnorm > 0.0 ? sqrt(tt) / s.bnorm : sqrt(tt);
    }
}

}  // namespace

int64_t nvec(mm_plan_t pl) { return pl->n_obs * pl->n_s; }

// interval -> problem map and the block offsets of the per-problem vector kernels
int build_batch_layout(mm_plan_t pl) {
    const int B = pl->n_prob;
    std::vector<int32_t> ip(pl->n_int);
    for (int b = 0; b < B; ++b)
        for (int32_t j = pl->h_pint[b]; j < pl->h_pint[b + 1]; ++j) ip[j] = b;
    std::vector<int32_t> eb(B + 1, 0), pb(B + 1, 0);
    for (int b = 0; b < B; ++b) {
        const int64_t np = pl->h_ooff[b + 1] - pl->h_ooff[b];
        const int64_t ne = np * pl->n_s;
        // several items per thread: the prologue reductions of every block (over the
        // problem's partials) cost as much as a few items, so small problems of a batch
        // get few blocks; the count depends on the problem alone
        auto blocks = [](int64_t m, int per_thread) {
            const int64_t per_block = (int64_t)kVecThreads * per_thread;
            int64_t g = (m + per_block - 1) / per_block;
            return (int32_t)std::min<int64_t>(kVecBlocks, std::max<int64_t>(1, g));
        };
        eb[b + 1] = eb[b] + blocks(ne, kVecPerThreadE);
        pb[b + 1] = pb[b] + blocks(np, kVecPerThreadP);
    }
    pl->n_eblk = eb[B];
    pl->n_pblk = pb[B];
    hipStream_t st = pl->stream;
    MM_TRY(pl->int_prob.alloc(pl->n_int));
    MM_TRY(pl->eblk.alloc(B + 1));
    MM_TRY(pl->pblk.alloc(B + 1));
    MM_HIP(hipMemcpyAsync(pl->int_prob.p, ip.data(), ip.size() * 4, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(pl->eblk.p, eb.data(), (B + 1) * 4, hipMemcpyHostToDevice, st));
    MM_HIP(hipMemcpyAsync(pl->pblk.p, pb.data(), (B + 1) * 4, hipMemcpyHostToDevice, st));
    MM_HIP(hipStreamSynchronize(st));
    return MM_OK;
}

PcgCtl batch_ctl(mm_plan_t pl) {
    PcgCtl c;
    c.part = pl->part.p;
    c.sc = pl->sc.p;
    c.mask = nullptr;
    c.act = pl->act.p;
    c.rz_hist = pl->rz_hist.p;
    c.hist = pl->hist.p;
    c.eblk = pl->eblk.p;
    c.pblk = pl->pblk.p;
    c.ooff = pl->ooff.p;
    c.B = pl->n_prob;
    c.hstride = pl->hstride;
    if (pl->krec.basis) {
        c.krylov = pl->krec.basis;
        c.alpha_hist = pl->krec.alpha;
        c.kcap = pl->krec.cap;
        c.knv = nvec(pl);
    }
    return c;
}

int vec_dot(mm_plan_t pl, const double* a, const double* b, int slot, const PcgCtl& ctl) {
    hipLaunchKernelGGL(k_dot, dim3(pl->n_eblk), dim3(kVecThreads), 0, pl->stream, a, b, slot,
                       pl->n_s, ctl);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int pcg_update_xr(mm_plan_t pl, double* x, double* r, const double* p, const double* q,
                  const PcgCtl& ctl) {
    hipLaunchKernelGGL(k_update_xr, dim3(pl->n_eblk), dim3(kVecThreads), 0, pl->stream, x, r, p,
                       q, pl->n_s, ctl);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int pcg_update_p(mm_plan_t pl, double* p, const double* z, const PcgCtl& ctl) {
    hipLaunchKernelGGL(k_update_p, dim3(pl->n_eblk), dim3(kVecThreads), 0, pl->stream, p, z,
                       pl->n_s, ctl);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int vec_residual(mm_plan_t pl, const double* b, const double* y, double* out,
                 const PcgCtl& ctl) {
    hipLaunchKernelGGL(k_residual, dim3(pl->n_eblk), dim3(kVecThreads), 0, pl->stream, b, y, out,
                       pl->n_s, ctl);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int vec_axpby(mm_plan_t pl, double a, const double* x, double b, const double* y, double* out) {
    hipLaunchKernelGGL(k_axpby, dim3(kVecBlocks), dim3(kVecThreads), 0, pl->stream, a, x, b, y, out,
                       nvec(pl));
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int vec_zero_flagged(mm_plan_t pl, double* x, const int* flag, const PcgCtl& ctl) {
    hipLaunchKernelGGL(k_zero_flagged, dim3(pl->n_eblk), dim3(kVecThreads), 0, pl->stream, x, flag,
                       pl->n_s, ctl);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int pcg_init(mm_plan_t pl, const PcgCtl& ctl, double tol, int zero_b_done) {
    hipLaunchKernelGGL(k_pcg_init, dim3(pl->n_prob), dim3(kVecThreads), 0, pl->stream, ctl, tol,
                       zero_b_done, pl->sel.p);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int pcg_check(mm_plan_t pl, const PcgCtl& ctl, int initial) {
    hipLaunchKernelGGL(k_pcg_check, dim3(pl->n_prob), dim3(kVecThreads), 0, pl->stream, ctl,
                       initial);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int pcg_decide(mm_plan_t pl, const PcgCtl& ctl) {
    hipLaunchKernelGGL(k_pcg_decide, dim3(pl->n_prob), dim3(kVecThreads), 0, pl->stream, ctl,
                       pl->sel.p);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int pcg_select(mm_plan_t pl, const PcgCtl& ctl) {
    hipLaunchKernelGGL(k_pcg_states, dim3((pl->n_prob + 255) / 256), dim3(256), 0, pl->stream, ctl,
                       pl->sel.p, 0);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int pcg_resume(mm_plan_t pl, const PcgCtl& ctl) {
    hipLaunchKernelGGL(k_pcg_states, dim3((pl->n_prob + 255) / 256), dim3(256), 0, pl->stream, ctl,
                       pl->sel.p, 1);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

int pcg_final(mm_plan_t pl, const PcgCtl& ctl) {
    hipLaunchKernelGGL(k_pcg_final, dim3(pl->n_prob), dim3(kVecThreads), 0, pl->stream, ctl);
    MM_HIP(hipGetLastError());
    return MM_OK;
}

}  // namespace mm
