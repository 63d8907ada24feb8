"""Seeded synthetic ALMA-shaped visibility data sets.

This module only *simulates observations*: antenna layouts, earth-rotation
(u,v) tracks, a continuous sky made of Gaussian components and point
sources, its visibilities in closed form, thermal noise and flagging.  It
holds none of the imaging method's arithmetic (no discrete forward model,
no chi-squared, entropy, gradients or optimiser): the oracle and the GPU
path both take what this module produces as plain input arrays.

Data model (paper Sec. 2.1): a channel is a list of Z visibilities V^o_k at
(u_k, v_k) in wavelengths with noise sigma_k (weights w_k = 1/sigma_k^2); the
image is an N x N grid with cell Delta x (radians), pixel (i, j) at
x_j = (j - N/2) Delta x, y_i = (i - N/2) Delta x (Alg. 3 with x_c = y_c = N/2).

Closed forms used for the simulated visibilities of the continuous sky
I(x) times the Gaussian primary beam A(x) = exp(-|x|^2 / (2 s_A^2)) (Eq. fft,
Sec. 2.4 item 1: FWHM 21 arcsec at 300 GHz for 12 m dishes, scaling with
wavelength).  Sky brightness is in Jy/pixel, so the visibility of the
continuous sky is (1/Delta x^2) times the integral of Eq. fft:

* point source of flux a at pixel centre x0:   a A(x0) exp(-2 pi i u.x0)
* Gaussian of peak a, std s, centre x0:
      (a/Delta x^2) 2 pi s_e^2 exp(-|x0|^2 / (2 (s^2 + s_A^2)))
      exp(-2 pi^2 s_e^2 |u|^2) exp(-2 pi i u.x0 kappa)
  with s_e^2 = s^2 s_A^2/(s^2 + s_A^2) and kappa = s_A^2/(s^2 + s_A^2)
  (product of two Gaussians is a Gaussian; its Fourier transform is one).

These are the physics of a noiseless observation of a continuous sky, not
the discrete DFT the imaging method evaluates; the two differ by the usual
pixelisation error, as real data would.

RNG: numpy Generator(PCG64(SeedSequence([170302920, c]))) with spawned child
streams for (layout, sky, noise, flagging, images).
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import List, Optional

import numpy as np

ARCSEC = math.pi / (180.0 * 3600.0)
C_LIGHT = 299792458.0
ALMA_LAT_DEG = -23.03
DEC_DEG = -40.0
DISH_M = 12.0
MIN_SPACING_M = 15.0
SEED_ROOT = 170302920


def beam_fwhm(wavelength_m: float) -> float:
    """ALMA 12 m primary-beam FWHM in radians: 21 arcsec at 300 GHz, linear in
    wavelength (Sec. 2.4, item 1)."""
    nu = C_LIGHT / wavelength_m
    return 21.0 * ARCSEC * (300e9 / nu)


def fwhm_to_sigma(fwhm: float) -> float:
    return fwhm / math.sqrt(8.0 * math.log(2.0))


@dataclasses.dataclass
class Channel:
    u: np.ndarray          # float64 [Z], wavelengths
    v: np.ndarray          # float64 [Z]
    vis: np.ndarray        # complex64 [Z], observed V^o
    w: np.ndarray          # float32 [Z], 1/sigma^2 (0 = flagged)
    fwhm: float            # primary beam FWHM, radians
    wavelength: float      # metres
    x0: float = 0.0        # pointing centre (mosaics): beam centre and phase-
    y0: float = 0.0        # tracking centre, radians from the image centre

    @property
    def nvis(self) -> int:
        return int(self.u.shape[0])


@dataclasses.dataclass
class Dataset:
    name: str
    n: int                      # image side N
    cell: float                 # Delta x, radians
    channels: List[Channel]
    sky: np.ndarray             # float64 [C][N][N] true pixel image (Jy/pixel)
    prior_m: float              # M (= G of the paper), the image floor
    lam: float                  # entropy weight lambda
    cg_iters: int
    description: str = ""
    shared: bool = False        # one image for all channels (mosaic pointings)

    @property
    def n_chan(self) -> int:
        return len(self.channels)

    @property
    def total_vis(self) -> int:
        return sum(ch.nvis for ch in self.channels)

    @property
    def pairs(self) -> int:
        """Sum over channels of Z_c N^2: (visibility, pixel) pairs per pass."""
        return self.total_vis * self.n * self.n


# ----------------------------------------------------------------------------
# Array geometry and uv tracks (textbook earth-rotation synthesis)
# ----------------------------------------------------------------------------

def antenna_layout(rng: np.random.Generator, n_ant: int, diameter_m: float) -> np.ndarray:
    """Antennas uniform in a disk of the given diameter in the local East-North
    plane, rejection-sampled so that no two are closer than 15 m."""
    radius = diameter_m / 2.0
    pos: list = []
    tries = 0
    while len(pos) < n_ant:
        tries += 1
        if tries > 1_000_000:
            raise RuntimeError("antenna layout: cannot place antennas")
        e, nn = rng.uniform(-radius, radius, size=2)
        if e * e + nn * nn > radius * radius:
            continue
        if any((e - p[0]) ** 2 + (nn - p[1]) ** 2 < MIN_SPACING_M ** 2 for p in pos):
            continue
        pos.append((e, nn))
    return np.asarray(pos, dtype=np.float64)


def baselines(pos: np.ndarray) -> tuple:
    """One baseline per antenna pair p < q (no conjugate duplicates)."""
    n = pos.shape[0]
    p_idx, q_idx = np.triu_indices(n, k=1)
    d = pos[q_idx] - pos[p_idx]           # (E, N) metres
    return d, p_idx, q_idx


def uv_tracks(bl_en: np.ndarray, n_int: int, wavelength_m: float,
              lat_deg: float = ALMA_LAT_DEG, dec_deg: float = DEC_DEG,
              ha_span_h: float = 2.0) -> tuple:
    """(u, v) in wavelengths for every (integration, baseline), time-major.

    ENU baseline (E, N, U=0) -> equatorial (X, Y, Z), then the usual rotation by
    hour angle H and declination delta (Thompson, Moran & Swenson, ch. 4).
    Hour angles evenly spaced on [-ha_span, +ha_span] inclusive; w ignored.
    """
    lat = math.radians(lat_deg)
    dec = math.radians(dec_deg)
    E = bl_en[:, 0]
    N = bl_en[:, 1]
    X = -math.sin(lat) * N
    Y = E
    Zc = math.cos(lat) * N
    H = np.linspace(-ha_span_h, ha_span_h, n_int) * (math.pi / 12.0)
    sH = np.sin(H)[:, None]
    cH = np.cos(H)[:, None]
    u = (sH * X[None, :] + cH * Y[None, :]) / wavelength_m
    v = (-math.sin(dec) * cH * X[None, :] + math.sin(dec) * sH * Y[None, :]
         + math.cos(dec) * Zc[None, :]) / wavelength_m
    return u.reshape(-1), v.reshape(-1)


# ----------------------------------------------------------------------------
# Continuous sky: list of components (x0, y0 radians; amplitude; sigma radians)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Components:
    x0: np.ndarray
    y0: np.ndarray
    amp: np.ndarray     # Gaussian peak or point flux, Jy/pixel
    sig: np.ndarray     # Gaussian std (radians); 0 for a point source

    @staticmethod
    def empty() -> "Components":
        z = np.zeros(0)
        return Components(z, z.copy(), z.copy(), z.copy())

    def __add__(self, other: "Components") -> "Components":
        return Components(np.concatenate([self.x0, other.x0]),
                          np.concatenate([self.y0, other.y0]),
                          np.concatenate([self.amp, other.amp]),
                          np.concatenate([self.sig, other.sig]))

    def scaled(self, f: float) -> "Components":
        return Components(self.x0, self.y0, self.amp * f, self.sig)


def sample_sky(comp: Components, n: int, cell: float) -> np.ndarray:
    """Pixel image of the continuous sky, sampled at pixel centres."""
    c = (np.arange(n) - n // 2) * cell
    img = np.zeros((n, n))
    for x0, y0, a, s in zip(comp.x0, comp.y0, comp.amp, comp.sig):
        if s == 0.0:
            j = int(round(x0 / cell)) + n // 2
            i = int(round(y0 / cell)) + n // 2
            if 0 <= i < n and 0 <= j < n:
                img[i, j] += a
        else:
            gx = np.exp(-((c - x0) ** 2) / (2 * s * s))
            gy = np.exp(-((c - y0) ** 2) / (2 * s * s))
            img += a * np.outer(gy, gx)
    return img


def sky_visibilities(comp: Components, u: np.ndarray, v: np.ndarray,
                     cell: float, fwhm: float, floor: float = 0.0) -> np.ndarray:
    """Closed-form visibilities of (continuous sky x Gaussian beam), see module
    docstring.  Returns complex128 [Z].  Components are split into contiguous
    groups summed on worker threads; the group sums are added in group order,
    so the result does not depend on the thread count."""
    n_comp = comp.x0.shape[0]
    work = n_comp * u.shape[0]
    groups = 1 if work < 2e7 else min(32, n_comp)
    if groups == 1:
        return _sky_vis_serial(comp, u, v, cell, fwhm, floor)
    from concurrent.futures import ThreadPoolExecutor
    edges = np.linspace(0, n_comp, groups + 1).astype(int)
    parts = [Components(comp.x0[a:b], comp.y0[a:b], comp.amp[a:b], comp.sig[a:b])
             for a, b in zip(edges[:-1], edges[1:])]
    workers = min(groups, max(1, (os.cpu_count() or 1)), 16)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        sums = list(ex.map(lambda cp: _sky_vis_serial(cp, u, v, cell, fwhm, 0.0), parts))
    out = np.zeros(u.shape[0], dtype=np.complex128)
    for part in sums:
        out += part
    if floor:
        out += _sky_vis_serial(Components.empty(), u, v, cell, fwhm, floor)
    return out


def _sky_vis_serial(comp: Components, u: np.ndarray, v: np.ndarray,
                    cell: float, fwhm: float, floor: float = 0.0) -> np.ndarray:
    sA2 = fwhm_to_sigma(fwhm) ** 2
    q2 = u * u + v * v
    out = np.zeros(u.shape[0], dtype=np.complex128)
    two_pi = 2.0 * math.pi
    for x0, y0, a, s in zip(comp.x0, comp.y0, comp.amp, comp.sig):
        r2 = x0 * x0 + y0 * y0
        if s == 0.0:
            amp = a * math.exp(-r2 / (2 * sA2))
            ph = two_pi * (u * x0 + v * y0)
            out += amp * (np.cos(ph) - 1j * np.sin(ph))
        else:
            s2 = s * s
            se2 = s2 * sA2 / (s2 + sA2)
            kap = sA2 / (s2 + sA2)
            amp = (a / (cell * cell)) * two_pi * se2 * math.exp(-r2 / (2 * (s2 + sA2)))
            env = amp * np.exp(-2.0 * math.pi ** 2 * se2 * q2)
            ph = two_pi * kap * (u * x0 + v * y0)
            out += env * (np.cos(ph) - 1j * np.sin(ph))
    if floor:
        # an unbounded constant floor seen through the beam
        out += (floor / (cell * cell)) * two_pi * sA2 * np.exp(-2.0 * math.pi ** 2 * sA2 * q2)
    return out


def add_noise(rng: np.random.Generator, vtrue: np.ndarray, frac: float,
              p_idx: np.ndarray, q_idx: np.ndarray, n_ant: int,
              slot_baseline: np.ndarray) -> tuple:
    """Thermal noise: sigma_k = s max|V_true| sqrt(f_p f_q), per-antenna factors
    f ~ U[0.8, 1.25]; Re and Im independent N(0, sigma_k^2) (Sec. 2.2)."""
    f = rng.uniform(0.8, 1.25, size=n_ant)
    sig0 = frac * float(np.max(np.abs(vtrue))) if vtrue.size else 1.0
    if sig0 == 0.0:
        sig0 = 1.0
    b = slot_baseline
    sigma = sig0 * np.sqrt(f[p_idx[b]] * f[q_idx[b]])
    noise = sigma * (rng.standard_normal(vtrue.shape[0]) + 1j * rng.standard_normal(vtrue.shape[0]))
    vis = (vtrue + noise).astype(np.complex64)
    w = (1.0 / (sigma * sigma)).astype(np.float32)
    return vis, w


# ----------------------------------------------------------------------------
# The five workload configurations
# ----------------------------------------------------------------------------

_CFG = {
    1: dict(n_ant=20, diam=500.0, n_int=27, n=64, noise=0.01, iters=20),
    2: dict(n_ant=40, diam=1500.0, n_int=128, n=256, noise=0.005, iters=20),
    3: dict(n_ant=50, diam=3000.0, n_int=816, n=512, noise=0.005, iters=20),
    4: dict(n_ant=45, diam=1500.0, n_int=304, n=256, noise=0.005, iters=50, n_chan=64),
    5: dict(n_ant=60, diam=8000.0, n_int=2825, n=1024, noise=0.002, iters=30),
    6: dict(n_ant=16, diam=400.0, n_int=54, n=512, noise=0.01, iters=20, n_point=23),
}

DESCRIPTIONS = {
    1: "c1: 64x64, 1 channel, 5,130 vis (20 ant, 500 m), FP64",
    2: "c2: 256x256, 1 channel, 99,840 vis (40 ant, 1.5 km), FP32",
    3: "c3: 512x512, 1 channel, 999,600 vis (50 ant, 3 km), disk+spiral sky",
    4: "c4: 64 channels x 256x256, per-channel Z_c in [2e4, 3e5] (45 ant, 1.5 km)",
    5: "c5: 1024x1024, 1 channel, 5,000,250 vis (60 ant, 8 km)",
    6: "c6: mosaic, one 512x512 image, 23 pointings, 149,040 vis (16 ant, 400 m), lambda 0.1",
}

WAVELENGTH = 1.3e-3
PRIOR_M = 1e-3
LAMBDA = 0.01


def _rngs(c: int):
    ss = np.random.SeedSequence([SEED_ROOT, c])
    kids = ss.spawn(5)
    return [np.random.Generator(np.random.PCG64(k)) for k in kids]


def _gaussians(rng, count, n, cell, sig_px_lo, sig_px_hi, amp_lo, amp_hi, extent, log_sig=False,
               log_amp=False) -> Components:
    off = rng.uniform(-extent, extent, size=(count, 2)) * cell
    if log_sig:
        sig = np.exp(rng.uniform(math.log(sig_px_lo), math.log(sig_px_hi), size=count))
    else:
        sig = rng.uniform(sig_px_lo, sig_px_hi, size=count)
    if log_amp:
        amp = np.exp(rng.uniform(math.log(amp_lo), math.log(amp_hi), size=count))
    else:
        amp = rng.uniform(amp_lo, amp_hi, size=count)
    return Components(off[:, 0], off[:, 1], amp, sig * cell)


def _points(rng, count, n, cell, amp_lo, amp_hi, extent) -> Components:
    pix = rng.integers(-int(extent), int(extent) + 1, size=(count, 2))
    amp = rng.uniform(amp_lo, amp_hi, size=count)
    return Components(pix[:, 0] * cell, pix[:, 1] * cell, amp, np.zeros(count))


def _disk_spiral(n: int, cell: float) -> Components:
    """c3 sky: a faint disk (radius 0.35 N, level 1e-3 of the peak) built from a
    square lattice of Gaussians (std 12 px, spacing 18 px: plateau ripple
    below 1e-3 of its level, edge taper ~12 px), a two-armed logarithmic
    spiral r = 4 exp(0.25 theta) px, theta in [0, 3.5 pi], traced by Gaussians
    of std 1 px every 1.5 px with ridge brightness falling linearly 1 -> 0.05,
    and a central point source of 1.0."""
    comp = Components.empty()
    R = 0.35 * n
    d, s = 18.0, 12.0
    level = 1e-3
    a_disk = level * d * d / (2 * math.pi * s * s)
    m = int(R // d)
    g = np.arange(-m, m + 1) * d
    gx, gy = np.meshgrid(g, g)
    keep = gx ** 2 + gy ** 2 <= (R - 0.5 * s) ** 2
    gx, gy = gx[keep], gy[keep]
    comp = comp + Components(gx * cell, gy * cell, np.full(gx.size, a_disk), np.full(gx.size, s * cell))
    # spiral arms
    b = 0.25
    r0 = 4.0
    th_end = 3.5 * math.pi
    length = math.sqrt(1 + b * b) / b * (r0 * math.exp(b * th_end) - r0)
    h = 1.5
    sig = 1.0
    n_blob = int(length // h) + 1
    s_arc = np.arange(n_blob) * h
    th = np.log(1.0 + s_arc * b / (r0 * math.sqrt(1 + b * b))) / b
    ridge = 1.0 - (1.0 - 0.05) * th / th_end
    amp = ridge * h / (math.sqrt(2 * math.pi) * sig)
    r = r0 * np.exp(b * th)
    for arm in range(2):
        phi = th + arm * math.pi
        comp = comp + Components(r * np.cos(phi) * cell, r * np.sin(phi) * cell, amp,
                                 np.full(n_blob, sig * cell))
    comp = comp + Components(np.zeros(1), np.zeros(1), np.ones(1), np.zeros(1))
    return comp


CACHE_VERSION = 2


def make_config(c: int, channels: Optional[int] = None, cache: bool = True) -> Dataset:
    """Build workload configuration c (1..5).  `channels` truncates c4 to its
    first few channels (for quick tests); the data of the kept channels are
    identical to the full configuration's.  Generated data sets are cached as
    .npz files in $UVMEM_SYNTH_CACHE (default: the system temp directory)."""
    if cache:
        import tempfile
        root = os.environ.get("UVMEM_SYNTH_CACHE", os.path.join(tempfile.gettempdir(), "uvmem_synth"))
        path = os.path.join(root, f"c{c}_{channels or 'all'}_v{CACHE_VERSION}.npz")
        if os.path.exists(path):
            try:
                return _load(path)
            except Exception:
                pass
        ds = _make_config(c, channels)
        try:
            os.makedirs(root, exist_ok=True)
            _save(ds, path)
        except OSError:
            pass
        return ds
    return _make_config(c, channels)


def _save(ds: Dataset, path: str) -> None:
    arrs = dict(n=ds.n, cell=ds.cell, sky=ds.sky, prior_m=ds.prior_m, lam=ds.lam, cg_iters=ds.cg_iters,
                name=ds.name, description=ds.description, n_chan=ds.n_chan, shared=ds.shared)
    for i, ch in enumerate(ds.channels):
        arrs.update({f"u{i}": ch.u, f"v{i}": ch.v, f"vis{i}": ch.vis, f"w{i}": ch.w,
                     f"fwhm{i}": ch.fwhm, f"lam{i}": ch.wavelength, f"x0{i}": ch.x0, f"y0{i}": ch.y0})
    tmp = path + ".tmp%d.npz" % os.getpid()
    np.savez(tmp, **arrs)
    os.replace(tmp, path)


def _load(path: str) -> Dataset:
    z = np.load(path, allow_pickle=False)
    chans = [Channel(z[f"u{i}"], z[f"v{i}"], z[f"vis{i}"], z[f"w{i}"], float(z[f"fwhm{i}"]), float(z[f"lam{i}"]),
                     float(z[f"x0{i}"]), float(z[f"y0{i}"]))
             for i in range(int(z["n_chan"]))]
    return Dataset(str(z["name"]), int(z["n"]), float(z["cell"]), chans, z["sky"], float(z["prior_m"]),
                   float(z["lam"]), int(z["cg_iters"]), str(z["description"]), bool(z["shared"]))


def _make_config(c: int, channels: Optional[int] = None) -> Dataset:
    if c not in _CFG:
        raise ValueError(f"unknown configuration {c}")
    p = _CFG[c]
    if c == 6:
        return _make_mosaic(p)
    r_layout, r_sky, r_noise, r_flag, _ = _rngs(c)
    n = p["n"]
    pos = antenna_layout(r_layout, p["n_ant"], p["diam"])
    bl, p_idx, q_idx = baselines(pos)
    n_bl = bl.shape[0]
    fwhm0 = beam_fwhm(WAVELENGTH)
    cell = 0.5 * fwhm0 / n
    if c == 1:
        comp = (_gaussians(r_sky, 3, n, cell, 1.5, 4.0, 0.3, 1.0, n / 4)
                + _points(r_sky, 2, n, cell, 0.3, 1.0, n / 4))
    elif c == 2:
        comp = _gaussians(r_sky, 20, n, cell, 2.0, 15.0, 0.1, 1.0, 3 * n / 8)
    elif c == 3:
        comp = _disk_spiral(n, cell)
    elif c == 5:
        comp = (_gaussians(r_sky, 200, n, cell, 1.0, 40.0, 1e-3, 1.0, 0.45 * n, log_sig=True, log_amp=True)
                + _points(r_sky, 50, n, cell, 0.05, 1.0, 0.45 * n))
    else:
        comp = None
    if c != 4:
        img = sample_sky(comp, n, cell)
        scale = 1.0 / float(img.max())
        comp = comp.scaled(scale)
        floor = PRIOR_M if c == 2 else 0.0
        sky = img * scale + floor
        u, v = uv_tracks(bl, p["n_int"], WAVELENGTH)
        slot_bl = np.tile(np.arange(n_bl), p["n_int"])
        vt = sky_visibilities(comp, u, v, cell, fwhm0, floor=floor)
        vis, w = add_noise(r_noise, vt, p["noise"], p_idx, q_idx, p["n_ant"], slot_bl)
        ch = Channel(u, v, vis, w, fwhm0, WAVELENGTH)
        ds = Dataset(f"c{c}", n, cell, [ch], sky[None], PRIOR_M, LAMBDA, p["iters"], DESCRIPTIONS[c])
        _check_nyquist(ds)
        return ds
    # c4: spectral cube, 64 channels, wavelength stepping 0.1 % per channel
    n_chan = p["n_chan"]
    keep_chan = n_chan if channels is None else min(channels, n_chan)
    base = _gaussians(r_sky, 10, n, cell, 3.0, 20.0, 0.1, 1.0, 3 * n / 8)
    dshift = r_sky.uniform(-8.0, 8.0, size=10)
    c0 = 32.0
    prof = 0.1 + np.exp(-((np.arange(n_chan)[:, None] - c0 - dshift[None, :]) ** 2) / (2 * 6.0 ** 2))
    cube = np.zeros((n_chan, n, n))
    for ci in range(n_chan):
        cube[ci] = sample_sky(Components(base.x0, base.y0, base.amp * prof[ci], base.sig), n, cell)
    scale = 1.0 / float(cube.max())
    n_slots = n_bl * p["n_int"]
    zc = r_flag.integers(20000, 300001, size=n_chan)
    chans = []
    slot_bl_all = np.tile(np.arange(n_bl), p["n_int"])
    for ci in range(n_chan):
        lam_c = WAVELENGTH * 1.001 ** ci
        keep = np.sort(r_flag.choice(n_slots, size=int(zc[ci]), replace=False))
        if ci >= keep_chan:
            continue
        u, v = uv_tracks(bl, p["n_int"], lam_c)
        u, v = u[keep], v[keep]
        fw = beam_fwhm(lam_c)
        comp_c = Components(base.x0, base.y0, base.amp * prof[ci] * scale, base.sig)
        vt = sky_visibilities(comp_c, u, v, cell, fw)
        rn = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 4, 1000 + ci])))
        vis, w = add_noise(rn, vt, p["noise"], p_idx, q_idx, p["n_ant"], slot_bl_all[keep])
        chans.append(Channel(u, v, vis, w, fw, lam_c))
    ds = Dataset("c4", n, cell, chans, cube[:keep_chan] * scale, PRIOR_M, LAMBDA, p["iters"], DESCRIPTIONS[4])
    _check_nyquist(ds)
    return ds


def hex_pointings(count: int, spacing: float) -> np.ndarray:
    """The `count` points of a hexagonal grid of the given spacing nearest the
    origin (ties broken by angle): a Nyquist-sampled mosaic pattern."""
    pts = []
    r = int(math.ceil(math.sqrt(count))) + 2
    for a in range(-r, r + 1):
        for b in range(-r, r + 1):
            x = spacing * (a + 0.5 * b)
            y = spacing * (math.sqrt(3.0) / 2.0) * b
            pts.append((round(x * x + y * y, 12), round(math.atan2(y, x), 12), x, y))
    pts.sort()
    return np.asarray([(x, y) for _, _, x, y in pts[:count]])


def _make_mosaic(p: dict) -> Dataset:
    """c6: mosaic (Sec. 1, mosaic support; Sec. 2.4 items 1 and 3): one sky
    observed in n_point pointings on a hexagonal grid spaced FWHM/2; pointing
    p has its primary beam and its phase-tracking centre at (x_p, y_p), its
    own hour-angle span and noise stream.  Visibilities of pointing p are
    those of the sky seen through the beam centred at (x_p, y_p), with phases
    relative to (x_p, y_p): the closed forms above with every component
    position taken relative to the pointing centre."""
    r_layout, r_sky, r_noise, _, _ = _rngs(6)
    n = p["n"]
    fwhm0 = beam_fwhm(WAVELENGTH)
    cell = 5.0 * fwhm0 / n
    pos = antenna_layout(r_layout, p["n_ant"], p["diam"])
    bl, p_idx, q_idx = baselines(pos)
    n_bl = bl.shape[0]
    comp = (_gaussians(r_sky, 2, n, cell, 25.0, 40.0, 0.5, 1.0, n / 10)
            + _gaussians(r_sky, 30, n, cell, 3.0, 15.0, 0.1, 1.0, 0.3 * n)
            + _points(r_sky, 10, n, cell, 0.2, 1.0, 0.3 * n))
    img = sample_sky(comp, n, cell)
    scale = 1.0 / float(img.max())
    comp = comp.scaled(scale)
    sky = img * scale
    cen = hex_pointings(p["n_point"], 0.5 * fwhm0)
    slot_bl = np.tile(np.arange(n_bl), p["n_int"])
    chans = []
    for k, (xp, yp) in enumerate(cen):
        u, v = uv_tracks(bl, p["n_int"], WAVELENGTH, ha_span_h=1.5 + 0.5 * k / max(1, len(cen) - 1))
        rel = Components(comp.x0 - xp, comp.y0 - yp, comp.amp, comp.sig)
        vt = sky_visibilities(rel, u, v, cell, fwhm0)
        rn = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 6, 2000 + k])))
        vis, w = add_noise(rn, vt, p["noise"], p_idx, q_idx, p["n_ant"], slot_bl)
        chans.append(Channel(u, v, vis, w, fwhm0, WAVELENGTH, float(xp), float(yp)))
    ds = Dataset("c6", n, cell, chans, sky[None], PRIOR_M, 0.1, p["iters"], DESCRIPTIONS[6], shared=True)
    _check_nyquist(ds)
    return ds


def _check_nyquist(ds: Dataset) -> None:
    """Sec. 2.3: the cell must satisfy 1/Delta x >= 2 u_max."""
    for ch in ds.channels:
        if ch.nvis:
            umax = float(max(np.abs(ch.u).max(), np.abs(ch.v).max()))
            if 1.0 / ds.cell < 2.0 * umax:
                raise AssertionError(f"{ds.name}: cell violates Nyquist")


# ----------------------------------------------------------------------------
# Evaluation images and small random problems
# ----------------------------------------------------------------------------

def eval_images(ds: Dataset, which: str) -> np.ndarray:
    """Images at which a single evaluation is compared:
    P1 = M everywhere; P2 = max(true sky, M); P3 = M + U[0, 1) (seeded)."""
    shape = (1 if ds.shared else ds.n_chan, ds.n, ds.n)
    if which == "P1":
        return np.full(shape, ds.prior_m)
    if which == "P2":
        return np.maximum(ds.sky, ds.prior_m)
    if which == "P3":
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, int(ds.name[1:]), 7])))
        return ds.prior_m + rng.uniform(0.0, 1.0, size=shape)
    raise ValueError(which)


def random_problem(n: int, nvis: int, seed: int, cell: float = 1.0e-6, fill: float = 0.45):
    """Arbitrary small problem: uv uniform in the Nyquist disk |u| cell <= fill,
    complex data, positive weights.  Returns (u, v, vis, w)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 99, seed])))
    rad = fill / cell
    r = rad * np.sqrt(rng.uniform(0, 1, nvis))
    ph = rng.uniform(0, 2 * math.pi, nvis)
    u = r * np.cos(ph)
    v = r * np.sin(ph)
    vis = (rng.standard_normal(nvis) + 1j * rng.standard_normal(nvis)).astype(np.complex64)
    w = rng.uniform(0.5, 2.0, nvis).astype(np.float32)
    return u, v, vis, w


def random_image(n: int, seed: int, lo: float = 1e-3, hi: float = 1.0, n_chan: int = 1) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 98, seed])))
    return rng.uniform(lo, hi, size=(n_chan, n, n))
