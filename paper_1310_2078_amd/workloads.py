"""Seeded synthetic workloads for the SL1M operator, solver and server.

This module only builds inputs: pixel positions and scales, interferometer
(u, v, w) coordinates, per-antenna gain constants, a true sky and a noise
realisation.  It holds none of the method's arithmetic (no matrix entries,
no visibilities, no solver steps): the data vector V = M x_true + noise is
formed by whoever consumes a workload, with its own operator.

Every draw comes from ``numpy.random.default_rng(seed)`` and the draws are
taken in the order written below, so a workload is a pure function of its
seed.  Coordinates follow the paper's conventions (Section "Defining the
direct solution"): (u, v, w) in wavelengths, (l, m) direction cosines with
l along u and m along v.

Workloads (sizes as stated in the docstrings of the builders):

* ``config1``  32x32 delta grid over +-0.05, 2,000 visibilities, 5 sources.
* ``config2``  256x256 wide-field delta grid over +-0.3, 128-antenna array,
               97,536 visibilities, 200 power-law sources.
* ``config3``  config 1 plus Stokes Q, U, V per source (4 right-hand sides).
* ``config4``  1024x1024 delta grid plus Gaussian layers (1,392,640 pixels),
               256 antennas, 409,600 visibilities, direction-dependent gains.
* ``config5``  a stream of 256 requests with log-uniform sizes.

Where the paper leaves a recipe choice open (array layout, flux law, noise
level, the uvw transform of a textbook), the choice is the one stated at
each generator below.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Pixel kinds (shared numbering with the C ABI header; plain integers).
PIX_DELTA = 0
PIX_GAUSS_PARAXIAL = 1
PIX_GAUSS_WIDE = 2

SPEED_OF_LIGHT = 299_792_458.0


@dataclasses.dataclass
class Workload:
    """Inputs of one deconvolution problem (all float64 unless noted)."""

    name: str
    # pixels
    l: np.ndarray
    m: np.ndarray
    sigma: np.ndarray          # paper's sigma (exp(-pi r^2 / sigma^2)); 0 for delta
    kind: np.ndarray           # uint8 pixel kind per pixel
    # visibilities
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    # antennas (None => unit gains)
    ant_p: Optional[np.ndarray] = None   # int32 per visibility
    ant_q: Optional[np.ndarray] = None   # int32 per visibility
    ant_gain: Optional[np.ndarray] = None  # complex128 c_p per antenna
    ant_fwhm: Optional[np.ndarray] = None  # power-beam FWHM (rad) per antenna
    # sky and noise
    x_true: Optional[np.ndarray] = None  # float64 [n_pix] (or [R, n_pix])
    noise: Optional[np.ndarray] = None   # complex128 [n_vis]
    # extra sky components that are not on the pixel list (delta sub-pixels
    # sampling extended sources finely); visibilities of these must be added
    # to the data by the consumer.
    extra_l: Optional[np.ndarray] = None
    extra_m: Optional[np.ndarray] = None
    extra_flux: Optional[np.ndarray] = None
    # solver settings
    lam: float = 0.0
    n_iter: int = 100
    power_iters: int = 30
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_pix(self) -> int:
        return int(self.l.shape[0])

    @property
    def n_vis(self) -> int:
        return int(self.u.shape[0])


# --------------------------------------------------------------------------
# pixel lists
# --------------------------------------------------------------------------

def grid_pixels(n_side: int, half_extent: float):
    """Square grid of n_side^2 pixels spanning +-half_extent.

    Spacing Delta = 2*half_extent/n_side, integer offsets -N/2 .. N/2-1, linear
    index j = col + N*row (Section "Delta function pixels"; the row index uses
    N_l, which equals N_m for every square grid here).  The phase-centre pixel
    (0, 0) sits at (col, row) = (N/2, N/2).
    """
    delta = 2.0 * half_extent / n_side
    idx = np.arange(n_side * n_side, dtype=np.int64)
    col = idx % n_side
    row = idx // n_side
    l = (col - n_side // 2) * delta
    m = (row - n_side // 2) * delta
    return l.astype(np.float64), m.astype(np.float64), delta


def inner_pixel_indices(n_side: int, frac: float = 0.8) -> np.ndarray:
    """Linear indices of the grid pixels inside the central `frac` of each axis."""
    lo = int(round(n_side * (1.0 - frac) / 2.0))
    hi = n_side - lo
    cols = np.arange(lo, hi)
    rows = np.arange(lo, hi)
    return (cols[None, :] + n_side * rows[:, None]).ravel()


# --------------------------------------------------------------------------
# visibility coordinates
# --------------------------------------------------------------------------

def disk_uvw(rng: np.random.Generator, n_vis: int, radius: float, w_sigma: float):
    """u, v uniform in a disk of `radius` wavelengths; w ~ N(0, w_sigma^2)."""
    a = rng.random(n_vis)
    b = rng.random(n_vis)
    rad = radius * np.sqrt(a)
    u = rad * np.cos(2.0 * np.pi * b)
    v = rad * np.sin(2.0 * np.pi * b)
    w = w_sigma * rng.standard_normal(n_vis)
    return u, v, w


def random_array_enu(rng: np.random.Generator, n_ant: int, diameter_m: float,
                     height_m: float):
    """Antenna East/North/Up positions: uniform in a disk, heights uniform."""
    a = rng.random(n_ant)
    b = rng.random(n_ant)
    rad = 0.5 * diameter_m * np.sqrt(a)
    east = rad * np.cos(2.0 * np.pi * b)
    north = rad * np.sin(2.0 * np.pi * b)
    up = rng.uniform(-height_m, height_m, n_ant)
    return east, north, up


def baseline_pairs(n_ant: int):
    """All antenna pairs p < q: no autocorrelations and no conjugate copies."""
    p, q = np.triu_indices(n_ant, k=1)
    return p.astype(np.int32), q.astype(np.int32)


def enu_to_uvw(east, north, up, p, q, hour_angles, lat_rad, dec_rad, wavelength_m):
    """Textbook ENU -> equatorial -> (u, v, w) for every (time, baseline).

    Baseline b = x_q - x_p.  Returns arrays ordered time-major (all baselines of
    the first hour angle, then the next), plus the matching antenna indices.
    """
    de = east[q] - east[p]
    dn = north[q] - north[p]
    du = up[q] - up[p]
    X = -math.sin(lat_rad) * dn + math.cos(lat_rad) * du
    Y = de
    Z = math.cos(lat_rad) * dn + math.sin(lat_rad) * du
    us, vs, ws = [], [], []
    sd, cd = math.sin(dec_rad), math.cos(dec_rad)
    for H in hour_angles:
        sh, ch = math.sin(H), math.cos(H)
        us.append(sh * X + ch * Y)
        vs.append(-sd * ch * X + sd * sh * Y + cd * Z)
        ws.append(cd * ch * X - cd * sh * Y + sd * Z)
    u = np.concatenate(us) / wavelength_m
    v = np.concatenate(vs) / wavelength_m
    w = np.concatenate(ws) / wavelength_m
    nt = len(hour_angles)
    return u, v, w, np.tile(p, nt), np.tile(q, nt)


def hour_angles(n: int, span_hours: float = 6.0):
    half = 0.5 * span_hours
    return np.linspace(-half, half, n) * (np.pi / 12.0)


def power_law_flux(rng: np.random.Generator, n: int, lo: float = 0.01, hi: float = 5.0):
    """Fluxes with p(S) ~ S^-1.5 on [lo, hi] by inverse-CDF sampling."""
    a = lo ** -0.5
    b = hi ** -0.5
    return (a + rng.random(n) * (b - a)) ** -2.0


def complex_noise(rng: np.random.Generator, n: int, sigma: float):
    """sigma * (N(0,1) + i N(0,1)): independent noise on both parts."""
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return sigma * (re + 1j * im)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def config1(seed: int = 0) -> Workload:
    """32x32 delta pixels over +-0.05; 2,000 disk visibilities; 5 sources."""
    rng = np.random.default_rng(seed)
    l, m, delta = grid_pixels(32, 0.05)
    u, v, w = disk_uvw(rng, 2000, 500.0, 50.0)
    src = rng.choice(l.shape[0], 5, replace=False)
    flux = rng.uniform(0.5, 2.0, 5)
    x = np.zeros(l.shape[0])
    x[src] = flux
    noise = complex_noise(rng, 2000, 0.01)
    n = l.shape[0]
    return Workload("config1", l, m, np.zeros(n), np.zeros(n, np.uint8), u, v, w,
                    x_true=x, noise=noise, lam=0.01, n_iter=100, power_iters=30,
                    meta={"delta": delta, "n_side": 32, "sources": src})


def config2(seed: int = 1, diameter_m: float = 3000.0) -> Workload:
    """256x256 wide-field delta pixels over +-0.3; 128 antennas, 12 snapshots.

    97,536 visibilities = 8,128 baselines x 12 hour angles; latitude -27 deg,
    declination -30 deg, 150 MHz.  200 power-law sources in the inner 80 %.
    """
    rng = np.random.default_rng(seed)
    l, m, delta = grid_pixels(256, 0.3)
    east, north, up = random_array_enu(rng, 128, diameter_m, 20.0)
    p, q = baseline_pairs(128)
    lam_obs = SPEED_OF_LIGHT / 150e6
    u, v, w, ap, aq = enu_to_uvw(east, north, up, p, q, hour_angles(12),
                                 math.radians(-27.0), math.radians(-30.0), lam_obs)
    inner = inner_pixel_indices(256)
    src = rng.choice(inner, 200, replace=False)
    flux = power_law_flux(rng, 200)
    x = np.zeros(l.shape[0])
    x[src] = flux
    noise = complex_noise(rng, u.shape[0], 0.005)
    n = l.shape[0]
    lam = 3.0 * 0.005 * math.sqrt(u.shape[0])
    return Workload("config2", l, m, np.zeros(n), np.zeros(n, np.uint8), u, v, w,
                    ant_p=ap, ant_q=aq, x_true=x, noise=noise, lam=lam, n_iter=100,
                    power_iters=30,
                    meta={"delta": delta, "n_side": 256, "sources": src,
                          "diameter_m": diameter_m})


def config3(seed: int = 2) -> Workload:
    """Config 1's grid, array and Stokes I, plus Q, U, V = I * U[-0.1, 0.1].

    ``x_true`` has shape [4, n_pix] (I, Q, U, V).
    """
    base = config1(0)
    rng = np.random.default_rng(seed)
    src = base.meta["sources"]
    stokes_i = base.x_true
    x = np.zeros((4, base.n_pix))
    x[0] = stokes_i
    for r in range(1, 4):
        x[r, src] = stokes_i[src] * rng.uniform(-0.1, 0.1, src.shape[0])
    base.name = "config3"
    base.x_true = x
    base.meta = dict(base.meta, n_rhs=4)
    return base


def config4(seed: int = 3) -> Workload:
    """Multiscale Gaussian pixels with direction-dependent gains.

    Pixels: 1024x1024 delta grid over +-0.35 followed by wide-field Gaussian
    layers with sigma = 2, 4 and 8 base spacings, each on its own grid of
    spacing sigma over +-0.35 (512^2, 256^2, 128^2): 1,392,640 pixels.
    Visibilities: 256 antennas, 13 snapshots, 424,320 records of which a
    seeded uniform choice of 14,720 is flagged, leaving 409,600.
    Gains: c_p = (1 + 0.05 a_p) exp(0.05 i phi_p), power-beam FWHM 0.4 rad.
    Sky: 1,000 point sources plus 50 Gaussian sources given as fine delta
    sub-pixels (``extra_*``; step sigma/4 over +-3 sigma).
    """
    rng = np.random.default_rng(seed)
    ls, ms, sig, kinds = [], [], [], []
    l0, m0, delta = grid_pixels(1024, 0.35)
    ls.append(l0), ms.append(m0)
    sig.append(np.zeros(l0.shape[0])), kinds.append(np.full(l0.shape[0], PIX_DELTA, np.uint8))
    for f, n_side in ((2, 512), (4, 256), (8, 128)):
        lg, mg, _ = grid_pixels(n_side, 0.35)
        ls.append(lg), ms.append(mg)
        sig.append(np.full(lg.shape[0], f * delta))
        kinds.append(np.full(lg.shape[0], PIX_GAUSS_WIDE, np.uint8))
    l = np.concatenate(ls)
    m = np.concatenate(ms)
    sigma = np.concatenate(sig)
    kind = np.concatenate(kinds)

    east, north, up = random_array_enu(rng, 256, 3000.0, 20.0)
    p, q = baseline_pairs(256)
    lam_obs = SPEED_OF_LIGHT / 150e6
    u, v, w, ap, aq = enu_to_uvw(east, north, up, p, q, hour_angles(13),
                                 math.radians(-27.0), math.radians(-30.0), lam_obs)
    flagged = rng.choice(u.shape[0], 14_720, replace=False)
    keep = np.ones(u.shape[0], bool)
    keep[flagged] = False
    u, v, w, ap, aq = u[keep], v[keep], w[keep], ap[keep], aq[keep]

    amp = rng.standard_normal(256)
    phs = rng.standard_normal(256)
    gain = (1.0 + 0.05 * amp) * np.exp(1j * 0.05 * phs)
    fwhm = np.full(256, 0.4)

    inner = inner_pixel_indices(1024)
    src = rng.choice(inner, 1000, replace=False)
    flux = power_law_flux(rng, 1000)
    x = np.zeros(l.shape[0])
    x[src] = flux

    centres = rng.choice(inner, 50, replace=False)
    s_src = rng.uniform(2 * delta, 8 * delta, 50)
    f_src = rng.uniform(0.5, 5.0, 50)
    el, em, ef = [], [], []
    for c, s, fl in zip(centres, s_src, f_src):
        step = s / 4.0
        offs = np.arange(-12, 13) * step            # +-3 sigma in steps of sigma/4
        dl, dm = np.meshgrid(offs, offs, indexing="xy")
        prof = np.exp(-np.pi * (dl ** 2 + dm ** 2) / s ** 2)
        el.append((l0[c] + dl).ravel())
        em.append((m0[c] + dm).ravel())
        ef.append((fl * prof / prof.sum()).ravel())

    noise = complex_noise(rng, u.shape[0], 0.005)
    lam = 3.0 * 0.005 * math.sqrt(u.shape[0])
    return Workload("config4", l, m, sigma, kind, u, v, w, ant_p=ap, ant_q=aq,
                    ant_gain=gain, ant_fwhm=fwhm, x_true=x, noise=noise,
                    extra_l=np.concatenate(el), extra_m=np.concatenate(em),
                    extra_flux=np.concatenate(ef), lam=lam, n_iter=100,
                    power_iters=30,
                    meta={"delta": delta, "n_side": 1024, "sources": src,
                          "gauss_centres": centres, "gauss_sigma": s_src,
                          "gauss_flux": f_src})


def config5_arrivals(seed: int = 4, n_req: int = 256, mean_gap_s: float = 0.25):
    """Poisson arrival times (exponential gaps) for the serving stream."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(mean_gap_s, n_req))


def config5_request(r: int, np_range=(4096, 262144), nv_range=(10_000, 200_000)) -> Workload:
    """Request r of the serving stream (seed 10,000 + r).

    Pixel count and visibility count log-uniform in their ranges; pixels
    row-major on a ceil(sqrt(N_p))-wide grid spanning +-0.05 (truncated to
    N_p); pixel kind drawn once per request: delta or wide-field Gaussian with
    sigma = 2 grid spacings.  Visibilities from config 1's disk/w generator,
    sky and noise as config 1, lambda = 0.01, 200 iterations.
    """
    rng = np.random.default_rng(10_000 + r)
    n_pix = int(round(math.exp(rng.uniform(math.log(np_range[0]), math.log(np_range[1])))))
    n_vis = int(round(math.exp(rng.uniform(math.log(nv_range[0]), math.log(nv_range[1])))))
    gaussian = bool(rng.random() < 0.5)
    side = int(math.ceil(math.sqrt(n_pix)))
    lg, mg, delta = grid_pixels(side, 0.05)
    l, m = lg[:n_pix].copy(), mg[:n_pix].copy()
    if gaussian:
        sigma = np.full(n_pix, 2.0 * delta)
        kind = np.full(n_pix, PIX_GAUSS_WIDE, np.uint8)
    else:
        sigma = np.zeros(n_pix)
        kind = np.full(n_pix, PIX_DELTA, np.uint8)
    u, v, w = disk_uvw(rng, n_vis, 500.0, 50.0)
    src = rng.choice(n_pix, 5, replace=False)
    flux = rng.uniform(0.5, 2.0, 5)
    x = np.zeros(n_pix)
    x[src] = flux
    noise = complex_noise(rng, n_vis, 0.01)
    return Workload(f"config5_req{r}", l, m, sigma, kind, u, v, w, x_true=x,
                    noise=noise, lam=0.01, n_iter=200, power_iters=30,
                    meta={"delta": delta, "gaussian": gaussian, "sources": src})


def small_random(seed: int, n_pix: int, n_vis: int, half_extent: float = 0.2,
                 uv_radius: float = 800.0, w_sigma: float = 200.0,
                 kind: int = PIX_DELTA, sigma: float = 0.0,
                 with_gains: bool = False, n_ant: int = 16,
                 distinct_fwhm: bool = False) -> Workload:
    """Irregular (non-grid) pixels and disk visibilities for parity tests.

    Pixels are uniform in a square of +-half_extent; this exercises arbitrary
    pixel placement and ragged sizes.
    """
    rng = np.random.default_rng(seed)
    l = rng.uniform(-half_extent, half_extent, n_pix)
    m = rng.uniform(-half_extent, half_extent, n_pix)
    u, v, w = disk_uvw(rng, n_vis, uv_radius, w_sigma)
    sig = np.full(n_pix, float(sigma))
    kd = np.full(n_pix, kind, np.uint8)
    x = rng.standard_normal(n_pix)
    wl = Workload(f"random{seed}", l, m, sig, kd, u, v, w, x_true=x)
    if with_gains:
        wl.ant_p = rng.integers(0, n_ant, n_vis).astype(np.int32)
        off = rng.integers(1, n_ant, n_vis)
        wl.ant_q = ((wl.ant_p + off) % n_ant).astype(np.int32)
        wl.ant_gain = (1.0 + 0.05 * rng.standard_normal(n_ant)) * np.exp(
            1j * 0.05 * rng.standard_normal(n_ant))
        if distinct_fwhm:
            wl.ant_fwhm = rng.uniform(0.3, 0.6, n_ant)
        else:
            wl.ant_fwhm = np.full(n_ant, 0.4)
    return wl
