"""Shared fixtures of the GPU tests: seeded scans, oracle problems, device plans."""

import functools

import numpy as np

import oracle as O
import synth


def small_iqu(seed=31, side=32, interval_len=4096, lam=256):
    # 4 co-pointed detectors, H + V passes, 32x32 patch: 2^16 samples, 16 intervals
    return synth.raster_iqu(side=side, spp=8, n_det=4, interval_len=interval_len, lam=lam,
                            fknee_range=(0.5, 2.0), alpha_range=(1.0, 2.0), seed_key=seed)


def ragged_iqu(seed=33):
    """Uneven interval lengths (some shorter than the band, one of 1 sample,
    lengths not multiples of any tile) on a 24x24 patch."""
    sc = synth.raster_iqu(side=24, spp=8, n_det=2, interval_len=24 * 24 * 8, lam=100,
                          fknee_range=(0.3, 3.0), alpha_range=(1.0, 2.0), seed_key=seed)
    n = sc.n_samples
    rng = np.random.default_rng(seed)
    cuts = np.sort(rng.choice(np.arange(1, n - 1), size=17, replace=False))
    cuts = np.concatenate([cuts, [cuts[3] + 1]]) if cuts[3] + 1 not in cuts else cuts
    off = np.unique(np.concatenate([[0], cuts, [n - 1, n]])).astype(np.int64)
    k = off.shape[0] - 1
    sc.offsets = off
    sc.sigma = rng.uniform(0.5, 2.0, k)
    sc.fknee = rng.uniform(0.1, 3.0, k)
    sc.alpha = rng.uniform(1.0, 2.0, k)
    return sc


@functools.lru_cache(maxsize=None)
def problem(name):
    sc = SCANS[name]()
    return sc, O.Problem.from_scan(sc)


def long_iqu(seed=35):
    # one 2^16-sample interval: taps by the decimated FFT with 4 sub-transforms
    sc = synth.raster_iqu(side=64, spp=8, n_det=1, interval_len=2 ** 16, lam=512,
                          fknee_range=(0.5, 2.0), alpha_range=(1.0, 2.0), seed_key=seed)
    return sc


def strips_i(seed=37):
    # I only, 24x24 patch, two identical passes cut into 9 intervals each: 9 distinct Z_S
    # columns (strips of about 2.7 rows), more than one group of layers in the A Z build
    return synth.raster_i(side=24, spp=4, n_pass=2, interval_len=256, lam=64, seed_key=seed)


def hot_i(seed=39):
    # I only, 8x8 patch, 72 passes cut into halves: every pixel is hit by 72 intervals
    # (rows of Z_S longer than 64 entries), 2 distinct Z_S columns
    return synth.raster_i(side=8, spp=4, n_pass=72, interval_len=128, lam=16, seed_key=seed)


def many_i(seed=43):
    # I only, 48x48 patch, two identical passes cut into intervals of 16 pixels: 144
    # distinct Z_S columns, more than the 64 of one tile of the coarse-build transposes
    # and nine 16-column MFMA tiles per side of E
    return synth.raster_i(side=48, spp=4, n_pass=2, interval_len=64, lam=16, seed_key=seed)


SCANS = {
    "long_iqu": long_iqu,
    "small_iqu": small_iqu,
    "ragged_iqu": ragged_iqu,
    "cfg1": synth.cfg1_raster_i,
    "strips_i": strips_i,
    "hot_i": hot_i,
    "many_i": many_i,
}


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# two-level preconditioner of a mixed plan whose A-DEF1 apply reads AZ in FP16 (the default
# az_fp16 layout): every AZ entry is rounded once to FP16 (relative error <= 2^-11 after the
# exact power-of-two column scaling), so M_2lvl r moves by up to that fraction of the
# coarse correction M_BD AZ w
TOL_2LVL_AZ16 = 1e-3


def relmax(a, b):
    """Element-wise error: max |a - b| / max |b|."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def check(a, b, bar, what=""):
    """Both the normwise and the element-wise relative error of a against b within bar."""
    e_norm, e_max = rel(a, b), relmax(a, b)
    assert e_norm <= bar and e_max <= bar, (what, e_norm, e_max, bar)
    return e_norm, e_max


def tile_edges(offsets, lam, n_r):
    """First and last output sample of every overlap-save tile of length n_r: each interval
    of n samples is cut into ceil(n / (n_r - 2 lam)) tiles of equal length (the last one
    shorter), as the library's plan lays them out."""
    out = []
    lmax = n_r - 2 * lam
    for a, b in zip(offsets[:-1], offsets[1:]):
        n = int(b - a)
        nt = -(-n // lmax)
        ln = -(-n // nt)
        for i in range(nt):
            s, e = int(a) + i * ln, min(int(b), int(a) + (i + 1) * ln)
            if e > s:
                out += [s, e - 1]
    return np.unique(np.asarray(out, dtype=np.int64))


def interval_edge_samples(offsets, lam):
    """Samples next to the hard boundaries of every interval: its first and last sample and
    the samples lam - 1, lam and lam + 1 away from either end (where the band first reaches
    past the edge), clipped to the interval."""
    out = []
    for a, b in zip(offsets[:-1], offsets[1:]):
        a, b = int(a), int(b)
        for d in (0, 1, lam - 1, lam, lam + 1):
            for t in (a + d, b - 1 - d):
                if a <= t < b:
                    out.append(t)
    return np.unique(np.asarray(out, dtype=np.int64))
