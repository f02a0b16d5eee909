"""Seeded synthetic scanning strategies, skies and piece-wise stationary noise.

Stand-ins for the simulated observations of the paper's numerical experiments
(Sect. 4.1: grid-like and circle scans, polariser scenarios, 1/f + white noise
per stationary interval).  The paper's pointing files, CAMB/HEALPix skies and
Planck parameters are not available, so every input here is synthetic and
seeded (``numpy.random.SeedSequence(1000 * cfg)``), spawned into independent
streams: sky | noise (one child per interval) | PSD draws | orientations.

Conventions shared by every scan:
  * ``pix[t]`` is the sky pixel seen at sample ``t`` (int32, original pixel id).
  * For polarised scans ``weights[t] = (cos 2 phi_t, sin 2 phi_t)``; the I
    weight is exactly 1 (eq. signal_with_polarization) and is not stored.
  * The time-ordered data of several detectors is their concatenation; every
    stationary interval lies inside one detector's timeline.
  * Noise PSD per interval, per sample: sigma^2 (1 + (f_knee / f)^alpha), i.e.
    the paper's 1/f + white model (eq. fknee) with a free slope and the
    sampling interval folded into sigma^2 (sigma^2 is the single-sample
    white-noise variance).
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

F_SAMP = 200.0  # Hz, all configurations
HWP_HZ = 2.0    # half-wave-plate mechanical rotation frequency


@dataclasses.dataclass
class Scan:
    name: str
    pix: np.ndarray                 # int32 [N_t], original pixel ids
    weights: Optional[np.ndarray]   # float64 [N_t, 2] (cos 2phi, sin 2phi) or None (I only)
    n_stokes: int
    n_pix: int                      # size of the original pixel grid
    offsets: np.ndarray             # int64 [n_int + 1], interval boundaries in samples
    sigma: np.ndarray               # float64 [n_int]
    fknee: np.ndarray               # float64 [n_int]
    alpha: np.ndarray               # float64 [n_int]
    lam: int                        # Toeplitz half bandwidth
    f_samp: float
    sky: np.ndarray                 # float64 [n_pix, n_stokes], true map on the full grid
    noise: np.ndarray               # float64 [N_t]
    problem_offsets: Optional[np.ndarray] = None  # int64 [n_prob + 1] interval index bounds (batched)
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_samples(self) -> int:
        return int(self.pix.shape[0])

    @property
    def n_intervals(self) -> int:
        return int(self.offsets.shape[0] - 1)


# --------------------------------------------------------------------------
# streams and noise
# --------------------------------------------------------------------------

def _streams(seed_key: int, n_intervals: int):
    ss = np.random.SeedSequence(seed_key)
    sky_ss, noise_ss, psd_ss, orient_ss = ss.spawn(4)
    noise_children = noise_ss.spawn(n_intervals)
    return (np.random.default_rng(sky_ss), noise_children,
            np.random.default_rng(psd_ss), np.random.default_rng(orient_ss))


def noise_realisation(offsets, sigma, fknee, alpha, f_samp, noise_children,
                      dtype=np.float64) -> np.ndarray:
    """Gaussian piece-wise stationary noise: per interval, white N(0,1) samples
    are coloured in Fourier space by sqrt(1 + (f_knee/f)^alpha), the zero
    frequency bin is removed (the 1/f power is unbounded there), and the
    result is scaled by sigma.  The realisation is periodic within each
    interval."""
    n_t = int(offsets[-1])
    out = np.empty(n_t, dtype=dtype)
    for j in range(len(offsets) - 1):
        a, b = int(offsets[j]), int(offsets[j + 1])
        n = b - a
        rng = np.random.default_rng(noise_children[j])
        white = rng.standard_normal(n)
        spec = np.fft.rfft(white)
        f = np.arange(spec.shape[0]) * (f_samp / n)
        amp = np.zeros_like(f)
        if fknee[j] > 0:
            amp[1:] = np.sqrt(1.0 + (fknee[j] / f[1:]) ** alpha[j])
        else:
            amp[1:] = 1.0
        out[a:b] = sigma[j] * np.fft.irfft(spec * amp, n)
    return out


def _sky(rng, n_pix, n_stokes, qu_sigma=0.1):
    sky = rng.standard_normal((n_pix, n_stokes))
    if n_stokes == 3:
        sky[:, 1:] *= qu_sigma
    return sky


# --------------------------------------------------------------------------
# raster scans on flat patches
# --------------------------------------------------------------------------

def _raster_pass(side: int, spp: int, vertical: bool) -> np.ndarray:
    """One boustrophedon pass over a side x side patch, spp samples per pixel.
    Horizontal: rows in turn, alternating direction.  Vertical: columns."""
    lines = np.repeat(np.arange(side, dtype=np.int64), side * spp)
    along = np.tile(np.repeat(np.arange(side, dtype=np.int64), spp), side)
    along = np.where(lines % 2 == 1, side - 1 - along, along)
    if vertical:
        row, col = along, lines
    else:
        row, col = lines, along
    return (row * side + col).astype(np.int32)


def raster_i(side=64, spp=4, n_pass=16, interval_len=2 ** 14, lam=1024,
             sigma=1.0, fknee=1.0, alpha=1.0, seed_key=1000, name="raster_i"):
    """Intensity-only raster: one detector sweeping rows back and forth,
    n_pass identical passes."""
    one = _raster_pass(side, spp, vertical=False)
    pix = np.tile(one, n_pass)
    n_t = pix.shape[0]
    assert n_t % interval_len == 0
    n_int = n_t // interval_len
    offsets = np.arange(n_int + 1, dtype=np.int64) * interval_len
    rng_sky, noise_children, _, _ = _streams(seed_key, n_int)
    sig = np.full(n_int, float(sigma))
    fk = np.full(n_int, float(fknee))
    al = np.full(n_int, float(alpha))
    sky = _sky(rng_sky, side * side, 1)
    noise = noise_realisation(offsets, sig, fk, al, F_SAMP, noise_children)
    return Scan(name, pix, None, 1, side * side, offsets, sig, fk, al, lam, F_SAMP,
                sky, noise, meta=dict(side=side, spp=spp, n_pass=n_pass))


def cfg1_raster_i():
    """1 detector, 2^18 samples, 64x64 patch, 4 samples/pixel per pass, 16
    identical passes (one pass = one 2^14-sample interval), sigma=1,
    f_knee=1 Hz, alpha=1, lambda=1024, I only."""
    return raster_i(64, 4, 16, 2 ** 14, 1024, 1.0, 1.0, 1.0, seed_key=1000,
                    name="cfg1_raster_i_2^18")


def raster_iqu(side=512, spp=8, n_det=4, interval_len=2 ** 16, lam=2048,
               fknee_range=(0.5, 2.0), alpha_range=(1.0, 2.0), sigma=1.0,
               det_angles_deg=(0.0, 45.0, 90.0, 135.0), hwp_hz=HWP_HZ,
               seed_key=2000, name="raster_iqu", qu_sigma=0.1):
    """Polarised cross-linked raster: n_det co-pointed detectors at fixed
    polariser angles, each scanning a horizontal then a vertical boustrophedon
    pass; a half-wave plate at hwp_hz rotates the polariser, so
    phi_t = theta_det + 2 psi_t with psi_t = 2 pi hwp_hz t / f_samp."""
    per_det = np.concatenate([_raster_pass(side, spp, False), _raster_pass(side, spp, True)])
    n_det_samples = per_det.shape[0]
    assert n_det_samples % interval_len == 0
    pix = np.tile(per_det, n_det)
    n_t = pix.shape[0]
    n_int = n_t // interval_len
    offsets = np.arange(n_int + 1, dtype=np.int64) * interval_len
    rng_sky, noise_children, rng_psd, _ = _streams(seed_key, n_int)
    t = np.arange(n_det_samples, dtype=np.float64) / F_SAMP
    psi = 2.0 * np.pi * hwp_hz * t
    weights = np.empty((n_t, 2), dtype=np.float64)
    for d in range(n_det):
        phi = np.deg2rad(det_angles_deg[d % len(det_angles_deg)]) + 2.0 * psi
        sl = slice(d * n_det_samples, (d + 1) * n_det_samples)
        weights[sl, 0] = np.cos(2.0 * phi)
        weights[sl, 1] = np.sin(2.0 * phi)
    fk = rng_psd.uniform(fknee_range[0], fknee_range[1], n_int)
    al = rng_psd.uniform(alpha_range[0], alpha_range[1], n_int)
    sig = np.full(n_int, float(sigma))
    sky = _sky(rng_sky, side * side, 3, qu_sigma)
    noise = noise_realisation(offsets, sig, fk, al, F_SAMP, noise_children)
    return Scan(name, pix, weights, 3, side * side, offsets, sig, fk, al, lam, F_SAMP,
                sky, noise, meta=dict(side=side, spp=spp, n_det=n_det))


def cfg2_raster_iqu():
    """4 co-pointed detectors (0/45/90/135 deg) + 2 Hz HWP, 512x512 patch,
    horizontal then vertical pass of 2^21 samples each (8 samples/pixel),
    2^24 samples in total, 64 intervals of 2^16 per detector,
    f_knee ~ U[0.5, 2] Hz, alpha ~ U[1, 2], lambda = 2048."""
    return raster_iqu(512, 8, 4, 2 ** 16, 2048, (0.5, 2.0), (1.0, 2.0), seed_key=2000,
                      name="cfg2_raster_iqu_2^24")


def cfg5_raster_iqu():
    """As the 2^24 configuration on a 256x256 patch: 4 detectors x 2^20 samples
    (2^22), 32 intervals of 2^17, lambda = 2048."""
    return raster_iqu(256, 8, 4, 2 ** 17, 2048, (0.5, 2.0), (1.0, 2.0), seed_key=5000,
                      name="cfg5_raster_iqu_2^22")


# --------------------------------------------------------------------------
# precessing great-circle ring scan on an equirectangular full-sky grid
# --------------------------------------------------------------------------

def ring_iqu(n_det=16, samples_per_det=2 ** 24, interval_len=2 ** 18, lam=4096,
             n_lon=2048, n_lat=1024, spin_rpm=1.0, precess_deg_per_min=0.1,
             fp_spacing_deg=0.5, sigma=1.0, fknee=1.0, alpha=1.0, hwp_hz=HWP_HZ,
             seed_key=3000, name="ring_iqu", det_subset=None):
    """Satellite-like scan: the spin axis moves along the equator at
    precess_deg_per_min; the boresight sweeps the great circle perpendicular
    to it (through both poles) at spin_rpm.  Detectors sit on a 4x4 focal
    plane grid with fp_spacing_deg spacing (cross- and along-scan) and
    polariser angles d * 11.25 deg; a 2 Hz HWP modulates the angle.
    Pixels: n_lon x n_lat equirectangular grid, id = ilat * n_lon + ilon.

    det_subset restricts the generation to some detectors (their own
    timelines, unchanged), e.g. one GPU's share of the full scan."""
    dets = list(range(n_det)) if det_subset is None else list(det_subset)
    n_int_per_det = samples_per_det // interval_len
    assert samples_per_det % interval_len == 0
    n_int_total = n_det * n_int_per_det
    rng_sky, noise_children_all, _, _ = _streams(seed_key, n_int_total)
    n_t = len(dets) * samples_per_det
    pix = np.empty(n_t, dtype=np.int32)
    weights = np.empty((n_t, 2), dtype=np.float64)
    omega = 2.0 * np.pi * spin_rpm / 60.0
    prec = np.deg2rad(precess_deg_per_min) / 60.0
    chunk = 2 ** 22
    for k, d in enumerate(dets):
        ix, iy = d % 4, d // 4
        cross = np.deg2rad((ix - 1.5) * fp_spacing_deg)
        along = np.deg2rad((iy - 1.5) * fp_spacing_deg)
        theta_det = np.deg2rad(d * 11.25)
        for c0 in range(0, samples_per_det, chunk):
            c1 = min(samples_per_det, c0 + chunk)
            t = np.arange(c0, c1, dtype=np.float64) / F_SAMP
            a = prec * t
            s = np.stack([np.cos(a), np.sin(a), np.zeros_like(a)], -1)       # spin axis
            u1 = np.array([0.0, 0.0, 1.0])
            u2 = np.stack([np.sin(a), -np.cos(a), np.zeros_like(a)], -1)     # s x z
            ph = omega * t + along
            b = np.cos(ph)[:, None] * u1 + np.sin(ph)[:, None] * u2
            v = -np.sin(ph)[:, None] * u1 + np.cos(ph)[:, None] * u2          # scan direction
            b = np.cos(cross) * b + np.sin(cross) * s
            z = np.clip(b[:, 2], -1.0, 1.0)
            colat = np.arccos(z)
            lon = np.mod(np.arctan2(b[:, 1], b[:, 0]), 2.0 * np.pi)
            ilat = np.minimum((colat / np.pi * n_lat).astype(np.int64), n_lat - 1)
            ilon = np.minimum((lon / (2.0 * np.pi) * n_lon).astype(np.int64), n_lon - 1)
            sl = slice(k * samples_per_det + c0, k * samples_per_det + c1)
            pix[sl] = (ilat * n_lon + ilon).astype(np.int32)
            e_north = np.stack([-np.cos(colat) * np.cos(lon), -np.cos(colat) * np.sin(lon),
                                np.sin(colat)], -1)
            e_east = np.stack([-np.sin(lon), np.cos(lon), np.zeros_like(lon)], -1)
            gamma = np.arctan2((v * e_east).sum(-1), (v * e_north).sum(-1))
            phi = theta_det + 2.0 * (2.0 * np.pi * hwp_hz * t) + gamma
            weights[sl, 0] = np.cos(2.0 * phi)
            weights[sl, 1] = np.sin(2.0 * phi)
    offsets = np.arange(len(dets) * n_int_per_det + 1, dtype=np.int64) * interval_len
    int_ids = np.concatenate([np.arange(d * n_int_per_det, (d + 1) * n_int_per_det) for d in dets])
    sig = np.full(len(int_ids), float(sigma))
    fk = np.full(len(int_ids), float(fknee))
    al = np.full(len(int_ids), float(alpha))
    sky = _sky(rng_sky, n_lon * n_lat, 3)
    noise = noise_realisation(offsets, sig, fk, al, F_SAMP,
                              [noise_children_all[i] for i in int_ids])
    return Scan(name, pix, weights, 3, n_lon * n_lat, offsets, sig, fk, al, lam, F_SAMP,
                sky, noise, meta=dict(dets=dets, n_lon=n_lon, n_lat=n_lat))


def cfg3_ring_iqu(det_subset=None):
    """16 detectors x 2^24 samples (2^28), 2048x1024 equirectangular IQU grid,
    1 rpm spin, 0.1 deg/min precession, 1024 intervals of 2^18,
    sigma=1, f_knee=1 Hz, alpha=1, lambda=4096."""
    return ring_iqu(seed_key=3000, name="cfg3_ring_iqu_2^28", det_subset=det_subset)


# --------------------------------------------------------------------------
# batched Monte Carlo: many small rotated rasters of uneven length
# --------------------------------------------------------------------------

def _rotated_raster(n_pass_samples, side, theta, spp_line=2.0):
    """A boustrophedon raster in a frame rotated by theta about the patch
    centre, covering the patch's circumscribed square; n_pass_samples samples
    (before dropping the ones that fall outside the patch).  Returns float
    patch coordinates (x, y) in pixel units."""
    half = side * np.sqrt(2.0) / 2.0
    n_lines = max(2, int(np.sqrt(n_pass_samples / spp_line)))
    per_line = int(np.ceil(n_pass_samples / n_lines))
    k = np.arange(n_lines * per_line)[:n_pass_samples]
    line = k // per_line
    u = (k % per_line + 0.5) / per_line
    u = np.where(line % 2 == 1, 1.0 - u, u)
    xr = -half + 2.0 * half * u
    yr = -half + 2.0 * half * (line + 0.5) / n_lines
    c, s = np.cos(theta), np.sin(theta)
    x = c * xr - s * yr + side / 2.0
    y = s * xr + c * yr + side / 2.0
    return x, y


def cfg4_batched_iqu(n_problems=256, side=128, n_min=2 ** 16, n_max=2 ** 20,
                     interval_len=2 ** 14, lam=1024, fknee_range=(0.1, 5.0), alpha=1.0,
                     sigma=1.0, n_det=4, seed_key=4000, problems=None):
    """Batched Monte Carlo: independent noise-only problems of uneven length
    (N_t log-uniform in [n_min, n_max] before dropping), each a 128x128 IQU
    raster rotated by theta_b ~ U[0, pi), 4 co-pointed detectors + HWP;
    samples outside the patch are dropped, then each detector's timeline is
    cut into intervals of interval_len (last one partial).  All problems are
    concatenated; problem_offsets indexes the interval list, and pixel ids of
    problem b are offset by b * side^2 so the problems are disjoint blocks.

    problems: optional subset of problem indices to generate (same draws)."""
    ss = np.random.SeedSequence(seed_key)
    geo_ss, prob_ss = ss.spawn(2)
    geo = np.random.default_rng(geo_ss)
    lengths = np.exp(geo.uniform(np.log(n_min), np.log(n_max), n_problems)).astype(np.int64)
    thetas = geo.uniform(0.0, np.pi, n_problems)
    fk_all = geo.uniform(fknee_range[0], fknee_range[1], n_problems)
    prob_children = prob_ss.spawn(n_problems)
    sel = list(range(n_problems)) if problems is None else list(problems)
    det_angles = np.deg2rad([0.0, 45.0, 90.0, 135.0])
    pix_l, w_l, off_l, noise_l, fk_l = [], [], [0], [], []
    prob_off = [0]
    base = 0
    npx = side * side
    for bi, b in enumerate(sel):
        per_det = int(lengths[b]) // n_det
        half = per_det // 2
        xh, yh = _rotated_raster(half, side, thetas[b])
        xv, yv = _rotated_raster(per_det - half, side, thetas[b] + np.pi / 2.0)
        x = np.concatenate([xh, xv])
        y = np.concatenate([yh, yv])
        keep = (x >= 0) & (x < side) & (y >= 0) & (y < side)
        ix = np.floor(x[keep]).astype(np.int64)
        iy = np.floor(y[keep]).astype(np.int64)
        p1 = (iy * side + ix).astype(np.int64) + bi * npx
        t = np.nonzero(keep)[0].astype(np.float64) / F_SAMP
        n_keep = p1.shape[0]
        n_int_det = (n_keep + interval_len - 1) // interval_len
        rng_psd_noise = np.random.default_rng(prob_children[b])
        noise_children = np.random.SeedSequence(
            rng_psd_noise.integers(0, 2 ** 63)).spawn(n_det * n_int_det)
        for d in range(n_det):
            pix_l.append(p1.astype(np.int32))
            phi = det_angles[d] + 2.0 * (2.0 * np.pi * HWP_HZ * t)
            w_l.append(np.stack([np.cos(2 * phi), np.sin(2 * phi)], -1))
            bounds = list(range(0, n_keep, interval_len)) + [n_keep]
            for j in range(len(bounds) - 1):
                off_l.append(base + bounds[j + 1])
                fk_l.append(fk_all[b])
            base += n_keep
        prob_off.append(len(off_l) - 1)
        o = np.array(off_l[-(n_det * n_int_det + 1):], dtype=np.int64)
        m = n_det * n_int_det
        noise_l.append(noise_realisation(o - o[0], np.full(m, sigma), np.full(m, fk_all[b]),
                                         np.full(m, alpha), F_SAMP, noise_children))
    pix = np.concatenate(pix_l)
    weights = np.concatenate(w_l)
    offsets = np.array(off_l, dtype=np.int64)
    n_int = offsets.shape[0] - 1
    fk = np.array(fk_l)
    return Scan("cfg4_batched_iqu", pix, weights, 3, npx * len(sel), offsets,
                np.full(n_int, sigma), fk, np.full(n_int, alpha), lam, F_SAMP,
                np.zeros((npx * len(sel), 3)), np.concatenate(noise_l),
                problem_offsets=np.array(prob_off, dtype=np.int64),
                meta=dict(problems=sel, lengths=lengths[sel], side=side))


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------

def subset_intervals(scan: Scan, idx) -> Scan:
    """The scan restricted to some stationary intervals (their samples,
    pointing, PSD parameters and noise), concatenated in the given order.
    The pixel grid and sky are unchanged."""
    idx = np.asarray(idx, dtype=np.int64)
    parts = [np.arange(scan.offsets[j], scan.offsets[j + 1]) for j in idx]
    lens = np.array([p.shape[0] for p in parts], dtype=np.int64)
    sel = np.concatenate(parts)
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return Scan(scan.name + f"[{len(idx)} intervals]", scan.pix[sel],
                None if scan.weights is None else scan.weights[sel],
                scan.n_stokes, scan.n_pix, offsets, scan.sigma[idx], scan.fknee[idx],
                scan.alpha[idx], scan.lam, scan.f_samp, scan.sky, scan.noise[sel],
                meta=dict(scan.meta, parent=scan.name, intervals=idx.tolist()))
