"""Seeded synthetic interferograms shaped like the paper's workloads.

This module is the one piece shared by the HIP path's tests/bench and by the
CPU oracle's tests: it produces inputs only and holds none of the unwrapping
arithmetic (no residues, costs, flows or integration).

Every interferogram is simulated from its L looks (Section II-B, eq. 3): per
pixel, L pairs (a_k, b_k) of independent unit circular complex Gaussians give
z1 = a_k and z2 = (g a_k + sqrt(1 - g^2) b_k) exp(-i phi), so each pair has
correlation g and interferometric phase phi.  The multilooked interferogram is
I = (1/L) sum z1 z2^*, the wrapped phase psi = angle(I) (computed in float64,
stored as float32) and the sample coherence is eq. 3 evaluated on the same
looks.  The true phase and coherence are kept for diagnostics.

Workloads (sizes, phase fields, coherence fields, masks and seeds):

  * ``c0``  256 x 256, ramp 0.3 rad/px along x + Gaussian bump (peak 40 rad,
    sigma 30 px, centred), coherence = uniform noise smoothed with a sigma-16
    Gaussian filter and rescaled to [0.2, 0.95], L = 9, no mask, seed 0.
  * ``c1``  2048 x 2048, the c0 recipe (bump centred) plus 6 low-coherence
    disks (radius U[40,150] px, coherence U[0.05,0.15] each) and a 5 % nodata
    mask of random rectangles (sides U[16,256] px), L = 9, seed 1.
  * ``c2``  6912 x 10752 (74.3 Mpixel), L = 15: a strike-slip-like field,
    sign(s) * 60 * (1 - (2/pi) atan(|s|/200)) rad with s the signed distance
    (px) to the corner-to-corner diagonal through the centre, plus a ramp of
    0.02 rad/px along x; coherence 0.1 within 50 px of the fault and a sigma-16
    smooth field rescaled to [0.3, 0.9] elsewhere; 3 % nodata; seed 2.
  * ``stack``  64 jobs, rows log-uniform in [512, 2048], cols log-uniform in
    [512, 4096], c0 recipe with bump peak U[5, 80] rad, L in {5, 9, 15},
    seed 1000 + k.
  * ``serve``  request pool, rows/cols log-uniform in [256, 8192], c1 recipe,
    seed 2000 + k.  :func:`serve_request_device` draws the same recipe with
    torch's generator on a GPU (a pool of hundreds of requests up to 67
    Mpixel each is far too slow to simulate on the host); its numbers differ
    from :func:`serve_request`'s, and a check against the oracle copies them
    back to the host.

  * ``river`` masks (bridging inputs, :func:`river_mask`): a meandering
    river of width w (centre column n/2 + (n/8) sin(2 pi i / (m/2))) cuts the
    scene in two; a canal of width w/2 runs from the left edge to the river
    at one third of the height; lakes (squares of side U[4w, 8w]) each hold a
    square island of half the lake's side.  Several regions of very
    different sizes, the structure rivers, coastlines and lakes give.

Any other size can be produced with :func:`make` for tests.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = ["Scene", "make", "config", "stack_job", "serve_request", "serve_request_device",
           "make_device", "CONFIGS"]

ROW_BLOCK = 64


@dataclass
class Scene:
    """One synthetic interferogram (all arrays row-major, m rows x n cols)."""
    name: str
    psi: np.ndarray          # float32 wrapped phase in [-pi_f32, pi_f32]
    coh: np.ndarray          # float32 sample coherence (eq. 3)
    valid: np.ndarray        # uint8 validity mask (1 = valid)
    looks: int
    phi_true: np.ndarray = field(repr=False, default=None)    # float64 true phase
    gamma_true: np.ndarray = field(repr=False, default=None)  # float32 true coherence
    igram: Optional[np.ndarray] = field(repr=False, default=None)  # complex64 I

    @property
    def shape(self):
        return self.psi.shape


# ----------------------------------------------------------------------------
# looks simulation
# ----------------------------------------------------------------------------

def _looks_block(args):
    phi, gam, L, seed_seq = args
    rng = np.random.Generator(np.random.PCG64(seed_seq))
    r, c = phi.shape
    shape = (L, r, c)
    # a_k, b_k ~ CN(0, 1): real and imaginary parts N(0, 1/2)
    s = math.sqrt(0.5)
    a = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * s
    b = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * s
    g = gam.astype(np.float64)[None]
    z1 = a
    z2 = (g * a + np.sqrt(1.0 - g * g) * b) * np.exp(-1j * phi)[None]
    prod = z1 * np.conj(z2)
    S = prod.sum(axis=0)
    p1 = (np.abs(z1) ** 2).sum(axis=0)
    p2 = (np.abs(z2) ** 2).sum(axis=0)
    I = S / L
    psi = np.angle(I).astype(np.float32)
    coh = (np.abs(S) / np.sqrt(p1 * p2)).astype(np.float32)
    return I.astype(np.complex64), psi, coh


def simulate_looks(phi: np.ndarray, gamma: np.ndarray, L: int, seed: int,
                   workers: Optional[int] = None):
    """Simulate the L-look interferogram for true phase ``phi`` and coherence
    ``gamma``.  Row blocks of 64 rows draw from ``SeedSequence(seed).spawn``,
    so the result does not depend on the number of worker processes."""
    m, n = phi.shape
    nblk = (m + ROW_BLOCK - 1) // ROW_BLOCK
    seqs = np.random.SeedSequence(seed).spawn(nblk)
    jobs = [(phi[k * ROW_BLOCK:(k + 1) * ROW_BLOCK],
             gamma[k * ROW_BLOCK:(k + 1) * ROW_BLOCK], L, seqs[k])
            for k in range(nblk)]
    if workers is None:
        workers = int(os.environ.get("WW_SYNTH_WORKERS", "0")) or min(16, os.cpu_count() or 1)
    if m * n < (1 << 20) or workers <= 1:
        parts = [_looks_block(j) for j in jobs]
    else:
        import multiprocessing as mp
        ctx = mp.get_context("fork")
        with ctx.Pool(workers) as pool:
            parts = pool.map(_looks_block, jobs, chunksize=1)
    I = np.concatenate([p[0] for p in parts], axis=0)
    psi = np.concatenate([p[1] for p in parts], axis=0)
    coh = np.concatenate([p[2] for p in parts], axis=0)
    return I, psi, coh


# ----------------------------------------------------------------------------
# fields
# ----------------------------------------------------------------------------

def smooth_field(m, n, sigma, lo, hi, rng):
    """Uniform noise, Gaussian-filtered (reflect borders), min-max rescaled."""
    from scipy.ndimage import gaussian_filter
    u = rng.random((m, n))
    f = gaussian_filter(u, sigma, mode="reflect")
    f = (f - f.min()) / max(f.max() - f.min(), 1e-300)
    return (lo + (hi - lo) * f).astype(np.float32)


def rect_mask(m, n, frac, rng, side_lo=16, side_hi=256):
    """Random axis-aligned nodata rectangles until ``frac`` of pixels are
    covered; sides U[side_lo, side_hi], at most a quarter of the image side
    (so that small scenes keep several rectangles).  Returns uint8 valid
    mask (1 = valid)."""
    valid = np.ones((m, n), np.uint8)
    if frac <= 0:
        return valid
    target = int(round(frac * m * n))
    covered = 0
    while covered < target:
        h = int(rng.integers(side_lo, side_hi + 1))
        w = int(rng.integers(side_lo, side_hi + 1))
        h = max(1, min(h, m // 4 if m >= 4 else m))
        w = max(1, min(w, n // 4 if n >= 4 else n))
        i0 = int(rng.integers(0, m - h + 1))
        j0 = int(rng.integers(0, n - w + 1))
        blk = valid[i0:i0 + h, j0:j0 + w]
        covered += int(blk.sum())
        blk[...] = 0
    return valid


def river_mask(m, n, rng, width=6, lakes=6):
    """Mask (uint8, 1 = valid) of a meandering river, a canal and lakes with
    islands: several regions separated by invalid pixels."""
    valid = np.ones((m, n), np.uint8)
    i = np.arange(m)
    centre = n / 2.0 + (n / 8.0) * np.sin(2.0 * np.pi * i / max(m / 2.0, 1.0))
    j = np.arange(n)[None, :]
    valid[np.abs(j - centre[:, None]) < width / 2.0] = 0
    c0 = m // 3
    lim = int(max(0, centre[c0] - width / 2.0))
    valid[c0:c0 + max(1, width // 2), :lim] = 0
    for _ in range(lakes):
        side = int(rng.integers(4 * width, 8 * width + 1))
        side = max(3, min(side, m - 1, n - 1))
        a = int(rng.integers(0, max(1, m - side)))
        b = int(rng.integers(0, max(1, n - side)))
        valid[a:a + side, b:b + side] = 0
        k = side // 4
        valid[a + k:a + side - k, b + k:b + side - k] = 1
    return valid


def ramp_bump_phase(m, n, ramp=0.3, peak=40.0, sigma=30.0, centre=None):
    i = np.arange(m, dtype=np.float64)[:, None]
    j = np.arange(n, dtype=np.float64)[None, :]
    ci, cj = centre if centre is not None else (m / 2.0, n / 2.0)
    return ramp * j + peak * np.exp(-((i - ci) ** 2 + (j - cj) ** 2) / (2 * sigma ** 2))


def fault_phase(m, n, amp=60.0, D=200.0, ramp=0.02):
    """Opposite-sign arctan profiles across the main diagonal through the
    centre; s = signed distance to the line from (0,0) to (m-1,n-1)."""
    i = np.arange(m, dtype=np.float64)[:, None]
    j = np.arange(n, dtype=np.float64)[None, :]
    di, dj = (m - 1), (n - 1)
    norm = math.hypot(di, dj)
    s = (j * di - i * dj) / norm
    phi = np.sign(s) * amp * (1.0 - (2.0 / math.pi) * np.arctan(np.abs(s) / D)) + ramp * j
    return phi, s


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def make(m, n, *, looks=9, seed=0, ramp=0.3, peak=40.0, bump_sigma=30.0,
         coh_lo=0.2, coh_hi=0.95, coh_sigma=16.0, disks=0, disk_coh=(0.05, 0.15),
         disk_radius=(40, 150), mask_frac=0.0, name=None, keep_truth=True,
         workers=None) -> Scene:
    """The c0/c1 recipe at any size (``disks``/``mask_frac`` switch on the c1
    additions)."""
    ss = np.random.SeedSequence(seed)
    s_field, s_disk, s_mask, s_looks = ss.spawn(4)
    phi = ramp_bump_phase(m, n, ramp, peak, bump_sigma)
    gam = smooth_field(m, n, min(coh_sigma, max(1.0, min(m, n) / 4)), coh_lo, coh_hi,
                       np.random.default_rng(s_field))
    if disks:
        rng = np.random.default_rng(s_disk)
        ii = np.arange(m)[:, None]
        jj = np.arange(n)[None, :]
        for _ in range(disks):
            r = rng.uniform(*disk_radius)
            ci = rng.uniform(0, m)
            cj = rng.uniform(0, n)
            g = rng.uniform(*disk_coh)
            gam[(ii - ci) ** 2 + (jj - cj) ** 2 <= r * r] = g
    valid = rect_mask(m, n, mask_frac, np.random.default_rng(s_mask))
    seed_looks = int(s_looks.generate_state(1)[0])
    I, psi, coh = simulate_looks(phi, gam, looks, seed_looks, workers)
    return Scene(name or f"{m}x{n}", psi, coh, valid, looks,
                 phi if keep_truth else None, gam if keep_truth else None,
                 I if keep_truth else None)


def make_fault(m, n, *, looks=15, seed=2, mask_frac=0.03, band=50.0, band_coh=0.1,
               coh_lo=0.3, coh_hi=0.9, name=None, keep_truth=False, workers=None) -> Scene:
    """The c2 recipe at any size."""
    ss = np.random.SeedSequence(seed)
    s_field, s_mask, s_looks = ss.spawn(3)
    phi, s = fault_phase(m, n)
    gam = smooth_field(m, n, 16.0, coh_lo, coh_hi, np.random.default_rng(s_field))
    gam[np.abs(s) <= band] = band_coh
    del s
    valid = rect_mask(m, n, mask_frac, np.random.default_rng(s_mask))
    seed_looks = int(s_looks.generate_state(1)[0])
    I, psi, coh = simulate_looks(phi, gam, looks, seed_looks, workers)
    return Scene(name or f"fault{m}x{n}", psi, coh, valid, looks,
                 phi if keep_truth else None, gam if keep_truth else None,
                 I if keep_truth else None)


CONFIGS = {
    "c0": dict(kind="ramp", m=256, n=256, looks=9, seed=0),
    "c1": dict(kind="ramp", m=2048, n=2048, looks=9, seed=1, disks=6, mask_frac=0.05),
    "c2": dict(kind="fault", m=6912, n=10752, looks=15, seed=2, mask_frac=0.03),
}


def _cache_dir():
    d = os.environ.get("WW_SYNTH_CACHE")
    if d:
        os.makedirs(d, exist_ok=True)
    return d


def config(name: str, keep_truth: bool = False, workers=None) -> Scene:
    """Build workload ``c0``, ``c1`` or ``c2``; cached as .npy files when the
    ``WW_SYNTH_CACHE`` environment variable names a directory."""
    spec = dict(CONFIGS[name])
    cache = _cache_dir()
    if cache and not keep_truth:
        base = os.path.join(cache, name)
        if all(os.path.exists(f"{base}_{k}.npy") for k in ("psi", "coh", "valid")):
            return Scene(name, np.load(f"{base}_psi.npy"), np.load(f"{base}_coh.npy"),
                         np.load(f"{base}_valid.npy"), spec["looks"])
    kind = spec.pop("kind")
    m, n = spec.pop("m"), spec.pop("n")
    if kind == "ramp":
        sc = make(m, n, name=name, keep_truth=keep_truth, workers=workers, **spec)
    else:
        sc = make_fault(m, n, name=name, keep_truth=keep_truth, workers=workers, **spec)
    if cache and not keep_truth:
        base = os.path.join(cache, name)
        np.save(f"{base}_psi.npy", sc.psi)
        np.save(f"{base}_coh.npy", sc.coh)
        np.save(f"{base}_valid.npy", sc.valid)
    return sc


def _logu(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def stack_job(k: int, workers=None) -> Scene:
    """Job k (0..63) of the 64-interferogram stack."""
    rng = np.random.default_rng(1000 + k)
    m = _logu(rng, 512, 2048)
    n = _logu(rng, 512, 4096)
    peak = float(rng.uniform(5, 80))
    L = int(rng.choice([5, 9, 15]))
    return make(m, n, looks=L, seed=1000 + k, peak=peak, name=f"stack{k}",
                keep_truth=False, workers=workers)


def serve_request(k: int, workers=None) -> Scene:
    """Request k of the serving pool (c1 recipe, log-uniform sizes)."""
    rng = np.random.default_rng(2000 + k)
    m = _logu(rng, 256, 8192)
    n = _logu(rng, 256, 8192)
    return make(m, n, looks=9, seed=2000 + k, disks=6, mask_frac=0.05,
                name=f"req{k}", keep_truth=False, workers=workers)


# ----------------------------------------------------------------------------
# the same recipes drawn on a GPU (torch), for large request pools
# ----------------------------------------------------------------------------

def _blur_axis(u, sigma, axis):
    """Gaussian filter (truncated at 4 sigma, half-sample symmetric borders
    like scipy's "reflect") along one axis of a 2-D float tensor."""
    import torch
    r = int(4.0 * sigma + 0.5)
    size = u.shape[axis]
    r = max(1, min(r, size))
    x = torch.arange(-r, r + 1, dtype=torch.float64)
    w = torch.exp(-x * x / (2.0 * sigma * sigma))
    w = (w / w.sum()).tolist()
    lo = u.narrow(axis, 0, r).flip(axis)
    hi = u.narrow(axis, size - r, r).flip(axis)
    pad = torch.cat([lo, u, hi], dim=axis)
    out = torch.zeros_like(u)
    for t in range(2 * r + 1):
        out += w[t] * pad.narrow(axis, t, size)
    return out


def make_device(m, n, *, looks=9, seed=0, ramp=0.3, peak=40.0, bump_sigma=30.0,
                coh_lo=0.2, coh_hi=0.95, coh_sigma=16.0, disks=0, disk_coh=(0.05, 0.15),
                disk_radius=(40, 150), mask_frac=0.0, device="cuda", rows_per_draw=256):
    """The c0/c1 recipe of :func:`make` drawn on ``device`` with a seeded
    torch generator (float64 arithmetic, float32 outputs): returns device
    tensors (psi, coh, valid).  The disks and the nodata rectangles come
    from numpy generators seeded as in :func:`make`; the smooth coherence
    field and the looks from torch's."""
    import torch
    ss = np.random.SeedSequence(seed)
    s_field, s_disk, s_mask, s_looks = ss.spawn(4)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(s_field.generate_state(1)[0]))
    ii = torch.arange(m, dtype=torch.float64, device=device)[:, None]
    jj = torch.arange(n, dtype=torch.float64, device=device)[None, :]
    ci, cj = m / 2.0, n / 2.0
    phi = ramp * jj + peak * torch.exp(-((ii - ci) ** 2 + (jj - cj) ** 2) / (2 * bump_sigma ** 2))
    sig = min(coh_sigma, max(1.0, min(m, n) / 4))
    u = torch.rand((m, n), generator=gen, dtype=torch.float32, device=device)
    f = _blur_axis(_blur_axis(u, sig, 1), sig, 0)
    del u
    f = (f - f.min()) / torch.clamp(f.max() - f.min(), min=1e-30)
    gam = (coh_lo + (coh_hi - coh_lo) * f).to(torch.float64)
    del f
    if disks:
        rng = np.random.default_rng(s_disk)
        for _ in range(disks):
            r = rng.uniform(*disk_radius)
            di = rng.uniform(0, m)
            dj = rng.uniform(0, n)
            g = rng.uniform(*disk_coh)
            gam[(ii - di) ** 2 + (jj - dj) ** 2 <= r * r] = g
    valid = torch.from_numpy(rect_mask(m, n, mask_frac, np.random.default_rng(s_mask))).to(device)
    gen.manual_seed(int(s_looks.generate_state(1)[0]))
    psi = torch.empty((m, n), dtype=torch.float32, device=device)
    coh = torch.empty((m, n), dtype=torch.float32, device=device)
    s2 = math.sqrt(0.5)
    for r0 in range(0, m, rows_per_draw):
        r1 = min(m, r0 + rows_per_draw)
        # a_k, b_k ~ CN(0, 1); z1 = a, z2 = (g a + sqrt(1 - g^2) b) e^{-i phi}
        ar, ai, br, bi = torch.randn((4, looks, r1 - r0, n), generator=gen, dtype=torch.float64,
                                     device=device).mul_(s2).unbind(0)
        g = gam[r0:r1][None]
        h = torch.sqrt(1.0 - g * g)
        xr, xi = g * ar + h * br, g * ai + h * bi
        c, s_ = torch.cos(phi[r0:r1])[None], torch.sin(phi[r0:r1])[None]
        zr, zi = xr * c + xi * s_, xi * c - xr * s_
        Sr = (ar * zr + ai * zi).sum(0)
        Si = (ai * zr - ar * zi).sum(0)
        p1 = (ar * ar + ai * ai).sum(0)
        p2 = (zr * zr + zi * zi).sum(0)
        psi[r0:r1] = torch.atan2(Si, Sr).to(torch.float32)
        coh[r0:r1] = (torch.sqrt(Sr * Sr + Si * Si) / torch.sqrt(p1 * p2)).to(torch.float32)
    return psi, coh, valid


def serve_request_device(k: int, device="cuda"):
    """Request k of the serving pool, drawn on ``device`` (c1 recipe at the
    size :func:`serve_request` gives it): (psi, coh, valid) device tensors."""
    rng = np.random.default_rng(2000 + k)
    m = _logu(rng, 256, 8192)
    n = _logu(rng, 256, 8192)
    return make_device(m, n, looks=9, seed=2000 + k, disks=6, mask_frac=0.05, device=device)
