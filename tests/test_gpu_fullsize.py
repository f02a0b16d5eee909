"""Parity at the workloads' full sizes, on outputs the oracle computes one by one.

- 2^24-sample IQU raster in the benchmark's launch configuration (mixed-precision plan
  with the coarse space and autotuned FFT tiles): integer layout bit-exact over the whole
  scan; A x, b and N^-1 y at sampled pixels / samples; the noiseless solve returns the
  input map.
- One detector's share (2^24 samples) of the 2^28-sample ring scan: lambda = 4096,
  2^18-sample intervals, skewed hit counts (1 to 60); A x at sampled pixels including the
  most and least observed ones.
- The 256-problem batched Monte Carlo plan: A x at sampled pixels of several problems.
- The 2^22-sample case of the differentiated solve: A x at sampled pixels.
- The a posteriori coarse space and A-DEF2 on the 2^24-sample raster (properties that hold
  at any size: the deflation property, iteration counts, residuals).
"""

import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
import synth  # noqa: E402
from paper_1408_3048_amd import Plan  # noqa: E402

from gpu_common import check, interval_edge_samples, tile_edges  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _sampled_A(pl, pr, x, pixels, ns, what):
    """A x at some pixels, FP64 and FP32 operators, normwise and element by element."""
    ref = pr.apply_A_at(x, pixels)
    y64 = pl.apply_A(dev(x)).cpu().numpy().reshape(-1, ns)[pixels]
    y32 = pl.apply_A(dev(x), precision="mixed").cpu().numpy().reshape(-1, ns)[pixels]
    e64 = check(y64, ref, 1e-12, f"{what} A fp64")
    e32 = check(y32, ref, 5e-5, f"{what} A fp32")
    print(f"[fullsize] {what}: A at {len(pixels)} pixels, fp64 {e64}, fp32 {e32}", flush=True)


def _edge_samples(pl, pr, rng, n_random=200):
    """Sample indices where N^-1 is most likely to go wrong: the first and last output of
    every overlap-save tile of both operators (tile seams), the samples next to every
    interval edge (hard zero boundaries), plus random ones."""
    n64, n32 = pl.fft_lengths()
    ts = [rng.choice(pr.n_t, n_random, replace=False), interval_edge_samples(pr.offsets, pr.lam)]
    for n_r in (n64, n32):
        if n_r:
            ts.append(tile_edges(pr.offsets, pr.lam, n_r))
    return np.unique(np.concatenate(ts))


def _sampled_ninv(pl, pr, y, ts, what):
    """N^-1 y at the samples ts, FP64 and FP32 operators, element by element."""
    z64 = pl.apply_Ninv(dev(y)).cpu().numpy()[ts]
    e64 = check(z64, O.toeplitz_apply_at(y, pr.offsets, pr.taps, ts), 1e-12, f"{what} N^-1 fp64")
    y32 = y.astype(np.float32)
    z32 = pl.apply_Ninv(dev(y32), precision="mixed").cpu().numpy()[ts]
    ref32 = O.toeplitz_apply_at(y32.astype(np.float64), pr.offsets, pr.taps, ts)
    e32 = check(z32, ref32, 5e-5, f"{what} N^-1 fp32")
    print(f"[fullsize] {what}: N^-1 at {len(ts)} samples, fp64 {e64}, fp32 {e32}", flush=True)


def _seam_pixels(pr, ts, rng, k):
    """k pixels observed at some of the samples ts (so that A x there sums tile seams)."""
    cand = np.unique(pr.cid[ts])
    return rng.choice(cand, min(k, cand.shape[0]), replace=False)


@functools.lru_cache(maxsize=None)
def cfg2():
    sc = synth.cfg2_raster_iqu()
    return sc, O.Problem.from_scan(sc)


def test_cfg2_fullsize_layout_operators_and_solution():
    sc, pr = cfg2()
    pl = Plan.from_scan(sc, precision="mixed", coarse=True, autotune=True)
    # integer layout over all 2^24 samples
    assert np.array_equal(pl.obs_pixels().cpu().numpy(), pr.obs)
    assert np.array_equal(pl.hits().cpu().numpy(), pr.s)
    assert np.array_equal(pl.sorted_samples().cpu().numpy(), np.argsort(pr.cid, kind="stable"))
    rng = np.random.default_rng(40)
    x = rng.standard_normal(pr.n_obs * pr.n_s)
    d = sc.noise
    ts = _edge_samples(pl, pr, rng)
    pixels = np.unique(np.concatenate([rng.choice(pr.n_obs, 30, replace=False),
                                       [0, pr.n_obs - 1], _seam_pixels(pr, ts, rng, 48)]))
    _sampled_A(pl, pr, x, pixels, 3, "2^24 raster")
    # N^-1 (FP64, FP32) at tile seams, interval edges and random samples
    _sampled_ninv(pl, pr, d, ts, "2^24 raster")
    # b = P^T N^-1 d at sampled pixels
    b = pl.rhs(dev(d)).cpu().numpy().reshape(-1, 3)
    bref = np.stack([pr.W[np.nonzero(pr.cid == p)[0]].T @
                     O.toeplitz_apply_at(d, pr.offsets, pr.taps, np.nonzero(pr.cid == p)[0])
                     for p in pixels])
    check(b[pixels], bref, 1e-12, "2^24 raster b")
    # noiseless data: the FP64 two-level solve and the mixed solve return the input map
    m = pr.sky_to_compact(sc.sky)
    dn = pl.apply_P(dev(m))
    xs, info = pl.pcg_solve(pl.rhs(dn), precond="2lvl", precision="fp64", tol=1e-12,
                            max_iter=3000)
    assert _rel(xs.cpu().numpy(), m) <= 1e-7, info["rel_residual"]
    xm, info = pl.pcg_solve(pl.rhs(dn), precond="2lvl", precision="mixed", tol=1e-10,
                            max_iter=3000)
    assert _rel(xm.cpu().numpy(), m) <= 1e-5
    pl.close()


def test_ring_share_fullsize_sampled_operator():
    sc = synth.cfg3_ring_iqu(det_subset=[0])
    pr = O.Problem.from_scan(sc)
    # one detector leaves pixels with fewer than 3 hits: their IQU blocks are singular,
    # which only the block-Jacobi preconditioner (not tested here) cares about
    pl = Plan.from_scan(sc, precision="mixed", rcond_min=0.0, autotune=True)
    assert np.array_equal(pl.hits().cpu().numpy(), pr.s)
    rng = np.random.default_rng(41)
    x = rng.standard_normal(pr.n_obs * pr.n_s)
    ts = _edge_samples(pl, pr, rng)
    pixels = np.unique(np.concatenate([rng.choice(pr.n_obs, 24, replace=False),
                                       [int(np.argmax(pr.s)), int(np.argmin(pr.s))],
                                       _seam_pixels(pr, ts, rng, 24)]))
    _sampled_A(pl, pr, x, pixels, 3, "ring share")
    _sampled_ninv(pl, pr, rng.standard_normal(pr.n_t), ts, "ring share")
    pl.close()


def test_batched_fullsize_sampled_operator():
    sc = synth.cfg4_batched_iqu()
    pl = Plan.from_scan(sc, precision="mixed", coarse=True)
    assert pl.n_problems == 256
    off3 = pl.problem_pixels() * 3
    rng = np.random.default_rng(42)
    x = rng.standard_normal(pl.n_vec)
    y64 = pl.apply_A(dev(x)).cpu().numpy()
    y32 = pl.apply_A(dev(x), precision="mixed").cpu().numpy()
    lengths = np.diff(sc.offsets[sc.problem_offsets])
    for b in (0, int(np.argmax(lengths)), int(np.argmin(lengths)), 255):
        s1 = synth.cfg4_batched_iqu(problems=[b])
        pr = O.Problem.from_scan(s1)
        assert pr.n_obs * 3 == off3[b + 1] - off3[b]
        xb = x[off3[b]:off3[b + 1]]
        pixels = rng.choice(pr.n_obs, 12, replace=False)
        ref = pr.apply_A_at(xb, pixels)
        check(y64[off3[b]:off3[b + 1]].reshape(-1, 3)[pixels], ref, 1e-12, f"problem {b} fp64")
        check(y32[off3[b]:off3[b + 1]].reshape(-1, 3)[pixels], ref, 5e-5, f"problem {b} fp32")
    pl.close()


def test_cfg5_fullsize_sampled_operator():
    sc = synth.cfg5_raster_iqu()
    pr = O.Problem.from_scan(sc)
    pl = Plan.from_scan(sc, precision="mixed", coarse=True, autotune=True)
    rng = np.random.default_rng(43)
    x = rng.standard_normal(pr.n_obs * pr.n_s)
    ts = _edge_samples(pl, pr, rng)
    pixels = np.unique(np.concatenate([rng.choice(pr.n_obs, 24, replace=False),
                                       _seam_pixels(pr, ts, rng, 24)]))
    _sampled_A(pl, pr, x, pixels, 3, "2^22 raster")
    _sampled_ninv(pl, pr, rng.standard_normal(pr.n_t), ts, "2^22 raster")
    pl.close()


def test_cfg2_fullsize_a_posteriori_and_adef2():
    """2^24 samples, mixed plan: Z_D from the FP64 block-Jacobi solve of one right-hand
    side (M_2lvl,D A z = z for sampled columns, a second right-hand side in fewer
    iterations than block Jacobi), and A-DEF2 with Z_S in as many iterations as A-DEF1."""
    sc, pr = cfg2()
    pl = Plan.from_scan(sc, precision="mixed", coarse=True, autotune=True)
    noise = torch.from_numpy(sc.noise).cuda()
    m = torch.from_numpy(pr.sky_to_compact(sc.sky)).cuda()
    sig = pl.apply_P(m)
    b2 = pl.rhs(sig + torch.roll(noise, 7919))
    _, i1 = pl.pcg_solve(b2, precond="2lvl", precision="mixed", tol=1e-8, max_iter=3000)
    _, i2 = pl.pcg_solve(b2, precond="adef2", precision="mixed", tol=1e-8, max_iter=3000)
    assert i2["rel_residual"] <= 1e-8 and abs(i1["iterations"] - i2["iterations"]) <= 2
    _, ib = pl.pcg_solve(b2, precond="bj", precision="mixed", tol=1e-8, max_iter=3000)
    x, info = pl.coarse_from_krylov(pl.rhs(sig + noise), tol=1e-8, max_iter=3000,
                                    krylov_dim=256, eps_tol=0.2)
    assert pl.coarse_kind() == 2 and pl.coarse_rank() >= 5
    assert info["rel_residual"] <= 1e-8
    (Z,) = pl.dense_columns()
    for i in (0, Z.shape[0] - 1):  # FP32 Z_D and AZ_D: deflation property to FP32 accuracy
        z = Z[i].contiguous()
        w = pl.precond_2lvl(pl.apply_A(z, precision="mixed"))
        assert _rel(w.cpu().numpy(), z.cpu().numpy()) <= 1e-4, i
    xd, idd = pl.pcg_solve(b2, precond="2lvl", precision="mixed", tol=1e-8, max_iter=3000)
    assert idd["rel_residual"] <= 1e-8 and idd["iterations"] < ib["iterations"]
    pl.close()
