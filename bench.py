#!/usr/bin/env python
"""Time-to-solution benchmark of the GLS map-making hot path on one MI355X.

Workload: the 2^24-sample polarised raster (4 co-pointed detectors at
0/45/90/135 deg + 2 Hz HWP, 512x512 IQU patch = 786,432 unknowns, 256
stationary intervals of 2^16 samples, f_knee ~ U[0.5, 2] Hz, alpha ~ U[1, 2],
lambda = 2048), synthetic and seeded.  Inputs (pointing, weights, TOD) are
resident in HBM before the timed region.

One step = plan construction (pointing sort, Toeplitz kernels, block-Jacobi,
coarse space: AZ and E) + right-hand side + mixed-precision two-level PCG to a
true relative residual <= 1e-8.  The same step with the plain FP64
block-Jacobi PCG (the reference method) is timed beside it.

Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time-to-solution @‖r‖/‖b‖≤1e-8 (2^24-sample IQU); "
          "A·x HBM GB/s vs peak")
HBM_PEAK_GBPS = 8000.0
# algorithmic bytes per sample of the hot kernels (mixed path: FP32 weights/TOD, int32 ids)
BYTES_NINV32 = 4 + 8 + 4     # compact pixel id + (cos, sin) read, z written
BYTES_PT32 = 4 + 8 + 4       # sorted sample index + sorted (cos, sin) + z gathered
BYTES_NINV64 = 4 + 16 + 8
BYTES_PT64 = 4 + 16 + 8
# FP32 vector peak without packed FP32 instructions (the library is built without them):
# 256 CUs x 64 lanes x 2 flops (FMA) x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 78.6


def fft_tile_flops(offsets, lam, n_r):
    """Tiles of the overlap-save N^-1 and its algorithmic flops per launch: per tile a
    forward and an inverse real FFT of n_r points, each a complex FFT of M = n_r/2 points
    (5 M log2 M flops) plus the O(M) real-to-complex split, spectrum product and merge
    (10 M flops in all): 10 M log2 M + 10 M."""
    lmax = n_r - 2 * lam
    lens = np.diff(np.asarray(offsets, dtype=np.int64))
    tiles = int(np.sum((lens + lmax - 1) // lmax))
    M = n_r // 2
    per_tile = 10 * M * np.log2(M) + 10 * M
    return tiles, float(tiles * per_tile)

# HBM traffic of the dominant kernel per launch, from two rocprofv3 --pmc runs of this
# script (FETCH_SIZE, then WRITE_SIZE, median over the kernel's launches in that run), each
# scaled by what the same counter reads for a plain 256 MiB device copy (--copy-calibration):
# FETCH_SIZE reads 128 MiB for the 256 MiB read (factor 2.0), WRITE_SIZE 256 MiB (factor 1.0).
# The factor 2 is that of 128-byte read requests, which FETCH_SIZE counts as 64 bytes; the
# TCC_EA0_RDREQ_{32B,64B,128B} counters show both kernels read with 128-byte requests too.
# The figures hold only for the kernel source they were taken on (sha256 of its code, see
# source_digest); after any change to that code the traffic is reported as null until the
# counters are taken again.
TRAFFIC = {
    # 2^24-sample IQU raster, FP32 tile length 16384 (the autotuner's choice on it)
    "ninv32": dict(source="paper_1408_3048_amd/csrc/toeplitz.hip",
                   sha256="408fad95fc00c24b63e108915c3cbb43e0a643f705bfc51b1553a9e1606836d9",
                   by_cfg={16384: dict(fetch_kib=138176.2, write_kib=65548.3)},
                   fetch_factor=2.0, write_factor=1.0),
    # P^T on the same scan, by work range (samples per wave)
    "pt32": dict(source="paper_1408_3048_amd/csrc/pointing.hip",
                 sha256="d142dab8a229cfbc5bbfb2e3c6a6184bb7bc97440bf9e094fae2d2fbd3755cd7",
                 by_cfg={512: dict(fetch_kib=135697.9, write_kib=6642.4)},
                 fetch_factor=2.0, write_factor=1.0),
    # one GPU's share of the ring scan (2^25 samples), FP32 tile length 16384
    "ring_ninv32": dict(source="paper_1408_3048_amd/csrc/toeplitz.hip",
                        sha256="408fad95fc00c24b63e108915c3cbb43e0a643f705bfc51b1553a9e1606836d9",
                        by_cfg={16384: dict(fetch_kib=247742.8, write_kib=131072.0)},
                        fetch_factor=2.0, write_factor=1.0),
    "ring_pt32": dict(source="paper_1408_3048_amd/csrc/pointing.hip",
                      sha256="d142dab8a229cfbc5bbfb2e3c6a6184bb7bc97440bf9e094fae2d2fbd3755cd7",
                      by_cfg={512: dict(fetch_kib=293624.8, write_kib=41099.8),
                              1024: dict(fetch_kib=296798.5, write_kib=43535.6)},
                      fetch_factor=2.0, write_factor=1.0),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- the FP64 oracle on the host
#
# The oracle's operators are separable by stationary interval in their time-domain part:
# A x = sum over intervals j of P_j^T N_j^-1 P_j x.  A pool of worker processes (forked
# before the GPU is touched, so no worker carries a GPU context) each holds the oracle's
# Problem for a fixed share of the intervals and returns its contribution in the global
# compact pixel numbering; the parent adds the shares in a fixed order.  The oracle's
# functions are called unchanged.

_POOL_SCANS = {}     # name -> (scan, shares), inherited by the forked workers
_POOL_BUFS = {}      # name -> (map buffer, TOD buffer): shared memory written by the parent
_POOL_PROBS = {}     # (name, share) -> (Problem of the share, global compact index, samples)


def _share_problem(name, share):
    import oracle as O
    import synth
    key = (name, share)
    if key not in _POOL_PROBS:
        sc, n_shares = _POOL_SCANS[name]
        idx = np.arange(share, sc.n_intervals, n_shares)
        sub = synth.subset_intervals(sc, idx)
        pr = O.Problem.from_scan(sub)
        gobs = np.unique(sc.pix)
        gidx = np.searchsorted(gobs, pr.obs)
        samples = np.concatenate([np.arange(sc.offsets[j], sc.offsets[j + 1]) for j in idx])
        _POOL_PROBS[key] = (pr, gidx, samples)
    return _POOL_PROBS[key]


def _share_apply(task):
    """One share's part of A x (kind "A", x from the shared map buffer), of b = P^T N^-1 d
    (kind "rhs", d from the shared TOD buffer) or of the block-Jacobi blocks (kind "bj")."""
    name, share, kind = task
    pr, gidx, samples = _share_problem(name, share)
    xb, db = _POOL_BUFS[name]
    if kind == "A":
        y = pr.apply_A(np.frombuffer(xb).reshape(-1, pr.n_s)[gidx].reshape(-1))
    elif kind == "rhs":
        y = pr.rhs(np.frombuffer(db)[samples])
    else:
        y = pr.bj_blocks().reshape(-1)
    return gidx, y


class OraclePool:
    """The oracle's A x, b and block-Jacobi blocks of a scan, computed by the worker pool."""

    def __init__(self, pool, name):
        self.pool, self.name = pool, name
        sc, self.n_shares = _POOL_SCANS[name]
        self.n_obs = int(np.unique(sc.pix).shape[0])
        self.ns = sc.n_stokes

    def _run(self, kind, width):
        out = np.zeros((self.n_obs, width))
        tasks = [(self.name, k, kind) for k in range(self.n_shares)]
        for gidx, y in self.pool.map(_share_apply, tasks):  # shares in order
            np.add.at(out, gidx, y.reshape(-1, width))
        return out.reshape(-1)

    def apply_A(self, x):
        np.frombuffer(_POOL_BUFS[self.name][0])[:] = x
        return self._run("A", self.ns)

    def rhs(self, d):
        np.frombuffer(_POOL_BUFS[self.name][1])[:] = d
        return self._run("rhs", self.ns)

    def bj_apply(self, r):
        if not hasattr(self, "_B"):
            self._B = self._run("bj", self.ns * self.ns).reshape(self.n_obs, self.ns, self.ns)
        R = np.asarray(r).reshape(self.n_obs, self.ns, 1)
        return np.linalg.solve(self._B, R).reshape(-1)


def make_oracle_pool(scans):
    """Fork the worker pool (before any GPU work) with the scans it serves and shared map and
    TOD buffers for the vectors it is applied to."""
    import multiprocessing as mp
    workers = max(1, min(16, os.cpu_count() or 1))
    for name, (sc, n_shares) in scans.items():
        _POOL_SCANS[name] = (sc, n_shares)
        n_obs = int(np.unique(sc.pix).shape[0])
        _POOL_BUFS[name] = (mp.RawArray("d", n_obs * sc.n_stokes), mp.RawArray("d", sc.n_samples))
    return mp.get_context("fork").Pool(workers), workers


def cpu_baseline(pool, workers, n_ax, x_gpu, d_gpu, cfg1_gpu, tol):
    """The FP64 oracle on the host cores (see OraclePool):
    - one full oracle A x of the 2^24-sample workload, timed; times the number of A x
      applications of the timed GPU solve (plan A Z columns + PCG) it is the oracle's
      time to solution at the GPU's iteration count (extrapolated from the measured A x);
    - the GPU map's relative residual in the oracle's system, ||b - A x|| / ||b|| with the
      oracle's b and A (the map's error against the FP64 oracle, as a residual);
    - the 2^18-sample intensity raster solved by the oracle's PCG to tol and to 1e-12
      (timed), and the GPU map's distance from both."""
    import oracle as O
    big = OraclePool(pool, "cfg2")
    b_or = big.rhs(d_gpu)
    big.apply_A(x_gpu)  # warm: the workers build their Problems
    t0 = time.perf_counter()
    ax = big.apply_A(x_gpu)
    t_ax = time.perf_counter() - t0
    relres = float(np.linalg.norm(b_or - ax) / np.linalg.norm(b_or))
    small = OraclePool(pool, "cfg1")
    b1 = small.rhs(cfg1_gpu["d"])
    t0 = time.perf_counter()
    x1, it1, st1 = O.pcg(small.apply_A, b1, small.bj_apply, tol=tol, maxit=2000)
    t_solve = time.perf_counter() - t0
    x1t, it1t, st1t = O.pcg(small.apply_A, b1, small.bj_apply, tol=1e-12, maxit=5000)
    xg = cfg1_gpu["x"]
    return dict(
        value=round(t_ax * n_ax, 3), unit="s", cores=workers, kind="oracle",
        sample=(f"one full oracle A*x of the 2^24-sample IQU raster (all 256 intervals) on "
                f"{workers} worker processes ({t_ax:.2f} s), times the {n_ax} A*x applications "
                f"of the timed GPU solve (plan A Z columns + PCG): extrapolated time to solution"),
        os_cpu_count=os.cpu_count(), workers=workers, oracle_ax_s=round(t_ax, 3),
        gpu_map_oracle_relres=relres,
        small_workload=dict(
            workload="2^18-sample I raster, 64x64, 16 intervals of 2^14, lambda=1024",
            oracle_bj_pcg_s=round(t_solve, 3), oracle_iterations=it1, oracle_status=st1,
            oracle_iterations_tol_1e12=it1t,
            gpu_iterations=cfg1_gpu["iterations"], gpu_solve_ms=cfg1_gpu["solve_ms"],
            gpu_map_rel_err_vs_oracle_same_tol=float(np.linalg.norm(xg - x1) / np.linalg.norm(x1)),
            gpu_map_rel_err_vs_oracle_1e12=float(np.linalg.norm(xg - x1t) / np.linalg.norm(x1t)),
            tol=tol))


def cfg1_gpu_solve(sc, tol):
    """The 2^18-sample intensity raster on the GPU: d = P m + n formed on the device, mixed
    two-level PCG to tol.  Returns the host copies the oracle compares with."""
    import torch
    from paper_1408_3048_amd import Plan
    pix = torch.from_numpy(sc.pix).cuda()
    psd = np.stack([sc.sigma, sc.fknee, sc.alpha], axis=1)
    plan = Plan(pix, None, sc.n_pix, sc.offsets, psd, n_stokes=1, lam=sc.lam, f_samp=sc.f_samp,
                precision="mixed", coarse=True)
    obs = plan.obs_pixels().long()
    m = torch.from_numpy(sc.sky).cuda()[obs].reshape(-1).contiguous()
    d = plan.apply_P(m) + torch.from_numpy(sc.noise).cuda()
    b = plan.rhs(d)
    x, info = plan.pcg_solve(b, precond="2lvl", precision="mixed", tol=tol, max_iter=5000,
                             history=False)
    out = dict(d=d.cpu().numpy(), x=x.cpu().numpy(), iterations=info["iterations"],
               solve_ms=round(info["solve_ms"], 3))
    plan.close()
    return out


def batched_leg(tol, warmup=1, graph=True):
    """The batched Monte Carlo workload: 256 independent noise-only problems of uneven
    length (2^16..2^20 samples before dropping out-of-patch samples) over 128x128 IQU
    patches, one batched plan, mixed-precision two-level PCG to tol for all problems at
    once.  Reported: plan + solve wall time and right-hand sides per second."""
    import torch
    import synth
    from paper_1408_3048_amd import Plan
    t = time.perf_counter()
    sc = synth.cfg4_batched_iqu()
    log(f"batched scans generated in {time.perf_counter() - t:.1f}s: {sc.n_samples} samples, "
        f"{len(sc.problem_offsets) - 1} problems, {sc.offsets.shape[0] - 1} intervals")
    pix = torch.from_numpy(sc.pix).cuda()
    w = torch.from_numpy(sc.weights).cuda()
    d = torch.from_numpy(sc.noise).cuda()
    psd = np.stack([sc.sigma, sc.fknee, sc.alpha], axis=1)
    res = None
    for i in range(warmup + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = Plan(pix, w, sc.n_pix, sc.offsets, psd, n_stokes=3, lam=sc.lam, f_samp=sc.f_samp,
                    precision="mixed", coarse=True, problem_intervals=sc.problem_offsets,
                    graph=graph)
        t1 = time.perf_counter()
        b = plan.rhs(d)
        t2 = time.perf_counter()
        x, info = plan.pcg_solve(b, precond="2lvl", precision="mixed", tol=tol, max_iter=5000,
                                 history=False)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        tt = t3 - t0
        log(f"batched walls: plan {1e3 * (t1 - t0):.1f} ms, rhs {1e3 * (t2 - t1):.1f} ms, "
            f"solve {1e3 * (t3 - t2):.1f} ms")
        its = [p["iterations"] for p in info["problems"]]
        res = dict(problems=plan.n_problems, n_samples=sc.n_samples, unknowns=plan.n_vec,
                   time_s=tt, plan_ms=plan.plan_ms, solve_ms=info["solve_ms"],
                   rhs_per_s=plan.n_problems / tt, samples_per_s=sc.n_samples / tt,
                   iterations_max=max(its), iterations_mean=float(np.mean(its)),
                   rel_residual_max=info["rel_residual_max"], r_eff=plan.coarse_rank(),
                   method="mixed two-level PCG, one batched plan, " +
                   ("graph-captured iterations" if graph else "launches issued one by one"))
        log(f"batched {'warmup' if i < warmup else 'timed'}: {tt * 1e3:.1f} ms {res}")
        plan.close()
        # the outputs are consumed here, so the next iteration's allocations reuse them
        del plan, b, x, info
        torch.cuda.synchronize()
    return res


def multi_rhs_leg(pix, w, sc, psd, m, noise, tol, n_rhs, autotune, krylov_dim=256):
    """One plan, n_rhs right-hand sides (the same sky with the noise timeline rolled by a
    different offset each time): plan time once, then the mean solve time per RHS, for the
    mixed two-level solver with Z_S, the mixed two-level solver with the a posteriori Z_D
    (built from the FP64 block-Jacobi solve of the first RHS, which that solve's time
    includes), the mixed block-Jacobi and the FP64 block-Jacobi solvers."""
    import torch
    from paper_1408_3048_amd import Plan
    out = {}
    kw = dict(n_stokes=3, lam=sc.lam, f_samp=sc.f_samp, autotune=autotune)
    for name, precision, coarse, precond in (("mixed_2lvl", "mixed", True, "2lvl"),
                                             ("mixed_2lvl_zd", "mixed", False, "zd"),
                                             ("mixed_bj", "mixed", False, "bj"),
                                             ("fp64_bj", "fp64", False, "bj")):
        torch.cuda.synchronize()
        plan = Plan(pix, w, sc.n_pix, sc.offsets, psd, precision=precision, coarse=coarse, **kw)
        sig = plan.apply_P(m)
        times, its, extra = [], [], {}
        for k in range(n_rhs):
            d = sig + torch.roll(noise, shifts=1 + 7919 * k)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if precond == "zd" and k == 0:
                x, info = plan.coarse_from_krylov(plan.rhs(d), tol=tol, max_iter=5000,
                                                  krylov_dim=krylov_dim, eps_tol=0.2,
                                                  history=False)
            else:
                x, info = plan.pcg_solve(plan.rhs(d), precond="2lvl" if precond == "zd" else precond,
                                         precision=precision, tol=tol, max_iter=5000, history=False)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            its.append(info["iterations"])
            if precond == "zd" and k == 0:
                extra = dict(first_rhs_fp64_bj_and_zd_build_ms=1e3 * times[0],
                             first_rhs_iterations=info["iterations"], zd_rank=plan.coarse_rank(),
                             ritz_min=float(plan.ritz_values().min()), krylov_dim=krylov_dim)
        rest = its[1:] if precond == "zd" else its
        out[name] = dict(plan_ms=plan.plan_ms, solve_ms_mean=1e3 * float(np.mean(times[1:] or times)),
                         iterations_mean=float(np.mean(rest or its)), n_rhs=n_rhs,
                         ms_per_rhs_incl_plan=(plan.plan_ms + 1e3 * float(np.sum(times))) / n_rhs,
                         **extra)
        log(f"multi-rhs {name}: {out[name]}")
        plan.close()
    return out


def knee_leg(tol, knees, autotune, krylov_dim=2048):
    """Solvers against the knee frequency of the 1/f noise (Sect. 5.1, Fig.
    deflation_iterations; Sect. 5.2, Fig. overall_time): the 2^22-sample IQU raster (4
    co-pointed detectors + 2 Hz HWP, 256x256 patch, 32 intervals of 2^17, lambda = 2048)
    with every interval's f_knee set to each value (alpha = 2).  For each, the mixed
    block-Jacobi solve; the mixed two-level solve with Z_S, whose construction (the plan's
    coarse build) is reported apart; and the mixed two-level solve with Z_D, whose
    construction is a recording block-Jacobi solve plus the Ritz extraction and A Z_D, E_D.
    Iterations and solve times are per right-hand side once the preconditioner exists."""
    import torch
    import synth
    from paper_1408_3048_amd import Plan
    out = []
    for fk in knees:
        sc = synth.raster_iqu(256, 8, 4, 2 ** 17, 2048, (fk, fk), (2.0, 2.0), seed_key=5000,
                              name=f"raster_iqu_2^22_fknee{fk}")
        pix = torch.from_numpy(sc.pix).cuda()
        w = torch.from_numpy(sc.weights).cuda()
        d = torch.from_numpy(sc.noise).cuda()
        psd = np.stack([sc.sigma, sc.fknee, sc.alpha], axis=1)
        kw = dict(n_stokes=3, lam=sc.lam, f_samp=sc.f_samp, precision="mixed", autotune=autotune)
        row = dict(f_knee=fk)

        def solve(plan, b, pc):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = plan.pcg_solve(b, precond=pc, precision="mixed", tol=tol, max_iter=5000,
                                     history=False)
            torch.cuda.synchronize()
            return info["iterations"], round(1e3 * (time.perf_counter() - t0), 2)

        plan = Plan(pix, w, sc.n_pix, sc.offsets, psd, coarse=False, **kw)
        b = plan.rhs(d)
        it, ms = solve(plan, b, "bj")
        row["bj"] = dict(plan_ms=round(plan.plan_ms, 2), iterations=it, solve_ms=ms)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.coarse_from_krylov(b, tol=tol, max_iter=5000, krylov_dim=krylov_dim, eps_tol=0.2,
                                history=False)
        torch.cuda.synchronize()
        build = round(1e3 * (time.perf_counter() - t0), 2)
        it, ms = solve(plan, b, "2lvl")
        row["zd"] = dict(construction_ms=build, rank=plan.coarse_rank(), iterations=it,
                         solve_ms=ms)
        plan.close()
        plan = Plan(pix, w, sc.n_pix, sc.offsets, psd, coarse=True, **kw)
        b = plan.rhs(d)
        it, ms = solve(plan, b, "2lvl")
        row["zs"] = dict(plan_ms=round(plan.plan_ms, 2), rank=plan.coarse_rank(), iterations=it,
                         solve_ms=ms)
        plan.close()
        log(f"knee sweep: {row}")
        out.append(row)
    return out


def bandwidth_leg(pix, w, sc, psd, m, d, tol, lams, autotune):
    """The bandwidth study on the same data (Sect. 5.1.3, Fig. conv_lambda; App. D): for
    every half-bandwidth lambda (0 = white-noise weighting) a mixed plan with Z_S, then the
    mixed block-Jacobi and two-level solves: iterations, solve time, time per iteration and
    the map's distance from the input sky; the same at lambda = 2048 for the narrower
    Gaussian and the rectangular window."""
    import torch
    from paper_1408_3048_amd import Plan
    out = []
    mn = float(m.norm())
    cases = [(lam, "gauss") for lam in lams] + [(2048, "gauss2"), (2048, "rect")]
    for lam, window in cases:
        plan = Plan(pix, w, sc.n_pix, sc.offsets, psd, n_stokes=3, lam=lam, f_samp=sc.f_samp,
                    window=window, precision="mixed", coarse=True, autotune=autotune)
        b = plan.rhs(d)
        row = dict(lam=lam, window=window, plan_ms=round(plan.plan_ms, 2),
                   fft_lengths=plan.fft_lengths(), r_eff=plan.coarse_rank())
        for pc in ("bj", "2lvl"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = plan.pcg_solve(b, precond=pc, precision="mixed", tol=tol, max_iter=5000,
                                     history=False)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            row[pc] = dict(iterations=info["iterations"], solve_ms=round(ms, 2),
                           ms_per_iteration=round(ms / max(info["iterations"], 1), 4),
                           map_err=round(float((x - m).norm()) / mn, 6))
        log(f"bandwidth: {row}")
        out.append(row)
        plan.close()
    return out


def ring_share_leg(tol, autotune, reps=10, fft_len_f32=0, fft_len_f64=0, pt_range=0):
    """One GPU's share of the 2^28-sample ring scan at its real shape (Sect. 4.1.1, Table 1
    big-circle scan, sharded by detectors): 2 of the 16 detectors, 2^25 samples, 128
    intervals of 2^18, lambda = 4096, 2048x1024 equirectangular IQU grid.  Reported: the
    FP32 A x kernels' algorithmic GB/s (16 B/sample each) and a mixed two-level solve to
    tol (plan + solve).  One detector pair leaves some pixels with too few polariser angles
    for an IQU solution; their samples are assigned to one extra pixel (a flagged-sample
    sink, as map-makers do), the pixels with rcond_1 of their block above 1e-6 are solved."""
    import torch
    import synth
    from paper_1408_3048_amd import Plan
    t = time.perf_counter()
    sc = synth.cfg3_ring_iqu(det_subset=[0, 1])
    log(f"ring share generated in {time.perf_counter() - t:.1f}s: {sc.n_samples} samples")
    pix = torch.from_numpy(sc.pix).cuda().long()
    w = torch.from_numpy(sc.weights).cuda()
    # block conditioning of every pixel (input preparation; not part of any timed region)
    W = torch.cat([torch.ones_like(w[:, :1]), w], 1)
    Bp = torch.zeros((sc.n_pix, 3, 3), dtype=torch.float64, device="cuda")
    Bp.view(sc.n_pix, 9).index_add_(0, pix, (W[:, :, None] * W[:, None, :]).reshape(-1, 9))
    hit = torch.zeros(sc.n_pix, dtype=torch.int64, device="cuda").index_add_(
        0, pix, torch.ones_like(pix))
    seen = hit > 0
    Bs = Bp[seen]
    det = torch.linalg.det(Bs)
    okd = det > 1e-12 * Bs.abs().amax(dim=(1, 2)) ** 3
    Binv = torch.zeros_like(Bs)
    Binv[okd] = torch.linalg.inv(Bs[okd])
    rc = torch.where(okd, 1.0 / (Bs.abs().sum(1).amax(1) * Binv.abs().sum(1).amax(1)),
                     torch.zeros_like(det))
    bad = torch.zeros(sc.n_pix, dtype=torch.bool, device="cuda")
    bad[torch.nonzero(seen).squeeze(1)[rc < 1e-6]] = True
    n_bad = int(bad.sum())
    pix2 = torch.where(bad[pix], torch.full_like(pix, sc.n_pix), pix).to(torch.int32).contiguous()
    wf = w.to(torch.float32).contiguous()
    psd = np.stack([sc.sigma, sc.fknee, sc.alpha], axis=1)
    kw = dict(n_stokes=3, lam=sc.lam, f_samp=sc.f_samp, autotune=autotune,
              fft_len_f32=fft_len_f32, fft_len_f64=fft_len_f64, pt_range=pt_range)
    del W, Bp, Bs, Binv, hit, seen
    # A x kernels
    plan = Plan(pix2, wf, sc.n_pix + 1, sc.offsets, psd, precision="mixed", **kw)
    x = torch.randn(plan.n_vec, dtype=torch.float64, device="cuda",
                    generator=torch.Generator("cuda").manual_seed(3))
    for _ in range(2):
        plan.apply_A(x, precision="mixed")
    plan.profile(True)
    for _ in range(reps):
        plan.apply_A(x, precision="mixed")
    pr = plan.profile_read()
    n_ninv, t_ninv = pr["ninv32"]
    n_pt, t_pt = pr["pt32"]
    a_ninv, a_pt = t_ninv / n_ninv, t_pt / n_pt
    res = dict(workload=("one GPU's share of the 2^28-sample ring scan: 2 of 16 detectors, "
                         "2^25 samples, 128 intervals of 2^18, lambda=4096, 2048x1024 IQU"),
               n_samples=sc.n_samples, unknowns=plan.n_vec, sink_pixels=n_bad,
               fft_lengths=plan.fft_lengths(), pt_range=plan.pt_range(),
               ninv32=dict(avg_ms=round(a_ninv, 5),
                           GBps=round(BYTES_NINV32 * sc.n_samples / (a_ninv * 1e-3) / 1e9, 1),
                           traffic=kernel_traffic("ring_ninv32", plan.fft_lengths()[1])),
               pt32=dict(avg_ms=round(a_pt, 5),
                         GBps=round(BYTES_PT32 * sc.n_samples / (a_pt * 1e-3) / 1e9, 1),
                         traffic=kernel_traffic("ring_pt32", plan.pt_range())),
               ax_fp32_GBps=round((BYTES_NINV32 + BYTES_PT32) * sc.n_samples /
                                  ((a_ninv + a_pt) * 1e-3) / 1e9, 1))
    res["ax_fp32_frac_of_peak"] = round(res["ax_fp32_GBps"] / HBM_PEAK_GBPS, 4)
    plan.close()
    # data and the mixed two-level solve (plan + solve)
    helper = Plan(pix2, wf, sc.n_pix + 1, sc.offsets, psd, precision="mixed", **kw)
    obs = helper.obs_pixels().long()
    sky = torch.cat([torch.from_numpy(sc.sky).cuda(), torch.zeros((1, 3), dtype=torch.float64,
                                                                  device="cuda")])
    m = sky[obs].reshape(-1).contiguous()
    d = helper.apply_P(m) + torch.from_numpy(sc.noise).cuda()
    helper.close()
    del helper
    for name, coarse, pc in (("mixed_2lvl", True, "2lvl"), ("mixed_bj", False, "bj")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = Plan(pix2, wf, sc.n_pix + 1, sc.offsets, psd, precision="mixed", coarse=coarse,
                    **kw)
        xs, info = plan.pcg_solve(plan.rhs(d), precond=pc, precision="mixed", tol=tol,
                                  max_iter=5000, history=False, raise_on_error=False)
        torch.cuda.synchronize()
        tt = time.perf_counter() - t0
        res[name] = dict(time_s=round(tt, 4), plan_ms=round(plan.plan_ms, 2),
                         solve_ms=round(info["solve_ms"], 2), iterations=info["iterations"],
                         relres=info["rel_residual"], status=info["status"],
                         r_eff=plan.coarse_rank() if coarse else 0)
        plan.close()
        del xs
    log(f"ring share: {res}")
    return res


def source_digest(rel):
    """sha256 of a source file's code: '//' comments, trailing blanks and empty lines
    removed, so that editing a comment does not void the counter figures taken on it."""
    lines = []
    with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
        for ln in f:
            i = ln.find("//")
            if i >= 0 and '"' not in ln[:i]:
                ln = ln[:i]
            ln = ln.rstrip()
            if ln:
                lines.append(ln)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def kernel_traffic(name, cfg):
    """HBM bytes per launch of a kernel from the stored counter figures for its launch
    configuration cfg (the FFT tile length of N^-1, the work range of P^T), or None when its
    source has changed since they were taken or no figures exist for that configuration."""
    t = TRAFFIC[name]
    c = t["by_cfg"].get(cfg)
    if t["sha256"] is None or c is None:
        return None
    if source_digest(t["source"]) != t["sha256"]:
        return None
    return round(1024 * (c["fetch_kib"] * t["fetch_factor"] + c["write_kib"] * t["write_factor"]))


def copy_calibration():
    """A plain device copy of 256 MiB, three times: the known-size reference for the
    FETCH_SIZE and WRITE_SIZE counters."""
    import torch
    a = torch.ones(2 ** 25, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(3):
        b.copy_(a)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / 3
    print(json.dumps(dict(copy_bytes_read=a.numel() * 8, copy_bytes_written=b.numel() * 8,
                          avg_ms=ms, GBps=2 * a.numel() * 8 / (ms * 1e-3) / 1e9)), flush=True)


def device_copy_rate(gib=2, reps=10):
    """GB/s of a plain device-to-device copy of gib GiB (bytes read + written per second):
    the streaming rate the HBM delivers in practice, far from the 8 TB/s peak; arrays of
    this size do not fit the 256 MB last-level cache."""
    import torch
    a = torch.ones(int(gib * 2 ** 30) // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        b.copy_(a)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    rate = 2 * a.numel() * 8 / (ms * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return round(rate, 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reference", action="store_true", help="skip the FP64 block-Jacobi leg")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 256-problem batched Monte Carlo leg")
    ap.add_argument("--bandwidth", default="0,64,256,1024,2048,4096",
                    help="half-bandwidths of the bandwidth-study leg ('' skips it)")
    ap.add_argument("--knees", default="0.5,2,8",
                    help="f_knee values (Hz) of the knee-frequency leg ('' skips it)")
    ap.add_argument("--no-ring-share", action="store_true",
                    help="skip the one-GPU share of the 2^28-sample ring scan")
    ap.add_argument("--multi-rhs", type=int, default=8,
                    help="right-hand sides of the plan-reuse leg (0 skips it)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: FFT tile lengths picked by timing at plan time (cached per process)")
    ap.add_argument("--fft-len-f32", type=int, default=0,
                    help="fixed FP32 overlap-save length instead of the autotuner (profiling runs)")
    ap.add_argument("--fft-len-f64", type=int, default=0)
    ap.add_argument("--pt-range", type=int, default=0,
                    help="fixed P^T work range (samples per wave) instead of the autotuner "
                         "(profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 256 MiB copy that calibrates the HBM byte counters")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the 256-problem batched leg (profiling runs) and print its "
                         "record")
    ap.add_argument("--graph", type=int, default=1,
                    help="batched leg: 1 captures the PCG iterations in HIP graphs, 0 issues "
                         "every launch from the host (kernel traces of the iterations)")
    ap.add_argument("--ring-only", action="store_true",
                    help="only run the ring-scan share leg (profiling runs) and print its record")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU path "
              "is a design (interval sharding + a map reduce-scatter), not built.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.batched_only:
        print(json.dumps(dict(batched=batched_leg(args.tol, warmup=args.warmup,
                                                  graph=bool(args.graph)))), flush=True)
        return
    if args.ring_only:
        print(json.dumps(dict(ring_share=ring_share_leg(
            args.tol, bool(args.autotune), fft_len_f32=args.fft_len_f32,
            fft_len_f64=args.fft_len_f64, pt_range=args.pt_range))), flush=True)
        return

    import synth

    t = time.perf_counter()
    sc = synth.cfg2_raster_iqu()
    log(f"scan generated in {time.perf_counter() - t:.1f}s: {sc.n_samples} samples, "
        f"{sc.n_intervals} intervals")
    pool = None
    if not args.no_cpu_baseline:
        sc1 = synth.cfg1_raster_i()
        # the oracle's worker pool is forked before anything touches the GPU
        pool, workers = make_oracle_pool({"cfg2": (sc, 64), "cfg1": (sc1, 16)})
        log(f"oracle pool: {workers} workers (os.cpu_count() = {os.cpu_count()})")

    import torch
    from paper_1408_3048_amd import Plan

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    pix = torch.from_numpy(sc.pix).cuda()
    w = torch.from_numpy(sc.weights).cuda()
    psd = np.stack([sc.sigma, sc.fknee, sc.alpha], axis=1)
    kw = dict(n_stokes=3, lam=sc.lam, f_samp=sc.f_samp)
    # TOD d = P m + n, formed on the device (untimed)
    helper = Plan(pix, w, sc.n_pix, sc.offsets, psd, **kw)
    obs = helper.obs_pixels().long()
    m = torch.from_numpy(sc.sky).cuda()[obs].reshape(-1).contiguous()
    d = helper.apply_P(m) + torch.from_numpy(sc.noise).cuda()
    helper.close()
    del helper
    torch.cuda.synchronize()
    log("inputs resident in HBM")
    copy_rate = device_copy_rate()
    log(f"plain 2 GiB device copy: {copy_rate} GB/s")

    def step(precision, coarse, precond, profile=False):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = Plan(pix, w, sc.n_pix, sc.offsets, psd, precision=precision, coarse=coarse,
                    autotune=bool(args.autotune), fft_len_f32=args.fft_len_f32,
                    fft_len_f64=args.fft_len_f64, pt_range=args.pt_range, **kw)
        if profile:
            plan.profile(True)
        b = plan.rhs(d)
        x, info = plan.pcg_solve(b, precond=precond, precision=precision, tol=args.tol,
                                 max_iter=5000)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = plan.profile_read() if profile else None
        extra = dict(plan_ms=plan.plan_ms, solve_ms=info["solve_ms"], iterations=info["iterations"],
                     fft_lengths=plan.fft_lengths(), pt_range=plan.pt_range(),
                     outer=info["outer_iterations"], relres=info["rel_residual"],
                     r_eff=plan.coarse_rank() if coarse else 0, unknowns=plan.n_vec)
        plan.close()
        return t1 - t0, x, extra, prof

    # mixed-precision two-level PCG (the measured method)
    for i in range(args.warmup):
        tt, _, ex, _ = step("mixed", True, "2lvl")
        log(f"warmup {i}: {tt * 1e3:.1f} ms {ex}")
    times, extras, prof = [], [], None
    for i in range(args.steps):
        last = i == args.steps - 1
        tt, x_mixed, ex, pr = step("mixed", True, "2lvl", profile=last)
        times.append(tt)
        extras.append(ex)
        if last:
            prof = pr
        log(f"step {i}: {tt * 1e3:.1f} ms {ex}")
    t_step = float(np.mean(times))

    ref = None
    if not args.no_reference:
        rtimes, rex = [], None
        tt, _, ex, _ = step("fp64", False, "bj")
        log(f"fp64 bj warmup: {tt * 1e3:.1f} ms {ex}")
        for i in range(args.steps):
            last = i == args.steps - 1
            tt, x_ref, ex, pr64 = step("fp64", False, "bj", profile=last)
            rtimes.append(tt)
            rex = ex
            log(f"fp64 bj step {i}: {tt * 1e3:.1f} ms {ex}")
        ax64 = None
        if pr64:
            n64, t64 = pr64["ninv64"]
            np64, tp64 = pr64["pt64"]
            ax64 = dict(ninv64_avg_ms=t64 / max(n64, 1), pt64_avg_ms=tp64 / max(np64, 1),
                        ax_GBps=(BYTES_NINV64 + BYTES_PT64) * sc.n_samples /
                        ((t64 / max(n64, 1) + tp64 / max(np64, 1)) * 1e-3) / 1e9)
        map_diff = float((x_mixed - x_ref).norm() / x_ref.norm())
        ref = dict(method="fp64 block-Jacobi PCG", time_s=float(np.mean(rtimes)), **rex,
                   speedup_of_mixed_2lvl=float(np.mean(rtimes)) / t_step,
                   map_rel_diff_mixed_vs_fp64=map_diff, fp64_kernels=ax64)

    # the other combinations, incl. the A-DEF2 variant (one run each, for context)
    legs = {}
    if not args.no_reference:
        for prec, pc in (("fp64", "2lvl"), ("mixed", "bj"), ("mixed", "adef2")):
            tt, _, ex, _ = step(prec, pc != "bj", pc)
            legs[f"{prec}_{pc}"] = dict(time_s=tt, **ex)
            log(f"{prec} {pc}: {tt * 1e3:.1f} ms {ex}")

    # roofline of the dominant kernel, from the live event timings of the last timed step
    n_ninv, t_ninv = prof["ninv32"]
    n_pt, t_pt = prof["pt32"]
    avg_ninv = t_ninv / max(n_ninv, 1)
    avg_pt = t_pt / max(n_pt, 1)
    n_r32 = extras[-1]["fft_lengths"][1]
    tiles, flops = fft_tile_flops(sc.offsets, sc.lam, n_r32)
    hbm = {
        "ninv32": dict(GBps=round(BYTES_NINV32 * sc.n_samples / (avg_ninv * 1e-3) / 1e9, 1),
                       algorithmic_bytes_per_launch=BYTES_NINV32 * sc.n_samples,
                       traffic=kernel_traffic("ninv32", n_r32), avg_ms=round(avg_ninv, 5)),
        "pt32": dict(GBps=round(BYTES_PT32 * sc.n_samples / (avg_pt * 1e-3) / 1e9, 1),
                     algorithmic_bytes_per_launch=BYTES_PT32 * sc.n_samples,
                     traffic=kernel_traffic("pt32", extras[-1]["pt_range"]), avg_ms=round(avg_pt, 5),
                     frac=round(BYTES_PT32 * sc.n_samples / (avg_pt * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)),
        "ax_fp32_GBps": round((BYTES_NINV32 + BYTES_PT32) * sc.n_samples /
                              ((avg_ninv + avg_pt) * 1e-3) / 1e9, 1),
    }
    # the dominant kernel against the HBM roofline by its algorithmic bytes (16 per sample
    # for each FP32 A x kernel); the overlap-save kernel's FFT flops against the FP32 vector
    # peak beside it
    if t_ninv >= t_pt:
        achieved = BYTES_NINV32 * sc.n_samples / (avg_ninv * 1e-3) / 1e9
        alu = flops / (avg_ninv * 1e-3) / 1e12
        roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBPS, 4), traffic=kernel_traffic("ninv32", n_r32),
                    kernel="k_toeplitz<float> (gather P + overlap-save N^-1)",
                    avg_launch_ms=round(avg_ninv, 5), launches=n_ninv, tiles=tiles, n_r=n_r32,
                    bytes_per_sample=BYTES_NINV32,
                    algorithmic_bytes_per_launch=BYTES_NINV32 * sc.n_samples,
                    alu_view=dict(achieved_TFLOPs=round(alu, 2), peak_TFLOPs=FP32_VALU_PEAK_TFLOPS,
                                  frac=round(alu / FP32_VALU_PEAK_TFLOPS, 4),
                                  flops_per_launch=flops))
    else:
        achieved = BYTES_PT32 * sc.n_samples / (avg_pt * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBPS, 4),
                    traffic=kernel_traffic("pt32", extras[-1]["pt_range"]),
                    kernel="k_scatter<float,3> (P^T segmented reduction)",
                    avg_launch_ms=round(avg_pt, 5), launches=n_pt, bytes_per_sample=BYTES_PT32,
                    algorithmic_bytes_per_launch=BYTES_PT32 * sc.n_samples)
    roof["hbm_view"] = hbm
    # context: what a plain streaming copy reaches on this GPU, and the kernel's measured HBM
    # traffic over its launch time
    roof["device_copy_GBps"] = copy_rate
    if roof.get("traffic"):
        roof["traffic_GBps"] = round(roof["traffic"] / (roof["avg_launch_ms"] * 1e-3) / 1e9, 1)
    roof["other_kernels"] = {k: dict(launches=v[0], avg_ms=v[1] / max(v[0], 1))
                             for k, v in prof.items() if v[0] > 0}

    multi = None
    if args.multi_rhs > 0 and not args.no_reference:
        multi = multi_rhs_leg(pix, w, sc, psd, m, torch.from_numpy(sc.noise).cuda(), args.tol,
                              args.multi_rhs, bool(args.autotune))

    bandwidth = None
    if args.bandwidth and not args.no_reference:
        lams = [int(v) for v in args.bandwidth.split(",")]
        bandwidth = bandwidth_leg(pix, w, sc, psd, m, d, args.tol, lams, bool(args.autotune))

    knee = None
    if args.knees and not args.no_reference:
        knee = knee_leg(args.tol, [float(v) for v in args.knees.split(",")], bool(args.autotune))

    batched = None
    if not args.no_batched:
        batched = batched_leg(args.tol)

    ring = None
    if not args.no_ring_share:
        ring = ring_share_leg(args.tol, bool(args.autotune))

    cpu = None
    if pool is not None:
        ex = extras[-1]
        n_ax = ex["iterations"] + ex["outer"] + 2 + ex["r_eff"]
        cfg1 = cfg1_gpu_solve(sc1, args.tol)
        log("the FP64 oracle on the host cores ...")
        t0 = time.perf_counter()
        cpu = cpu_baseline(pool, workers, n_ax, x_mixed.cpu().numpy(), d.cpu().numpy(), cfg1,
                           args.tol)
        pool.close()
        log(f"cpu baseline ({time.perf_counter() - t0:.1f} s): {cpu}")

    out = dict(
        metric=METRIC, value=round(t_step, 6), unit="s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(t_step * 1e3, 3), higher_is_better=False,
        scaling="weak", vs_baseline=None, dtype="f32+f64", data="synthetic",
        config=dict(workload=("2^24-sample IQU cross-linked raster, 4 detectors + 2 Hz HWP, "
                              "512x512 patch (786432 unknowns), 256 intervals of 2^16, "
                              "lambda=2048, mixed FP32/FP64 two-level PCG to 1e-8 incl. plan"),
                    n_samples=sc.n_samples, unknowns=extras[-1]["unknowns"],
                    tol=args.tol, parallelism="single GPU"),
        breakdown=extras[-1], reference=ref, other_legs=legs, multi_rhs=multi,
        bandwidth=bandwidth, knee_sweep=knee, batched=batched, ring_share=ring,
        roofline=roof,
        cpu_baseline=cpu,
    )
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
