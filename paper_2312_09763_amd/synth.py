"""Seeded synthetic inputs for the visibility simulator.

This module produces *inputs only*: antenna layouts, point-source catalogues,
per-channel fluxes, gridded beam models and observation times.  It contains
none of the simulator's own arithmetic (no rotation, horizon cut,
interpolation, phase or visibility product), so both the HIP path and the CPU
reference can take their inputs from here without sharing any of the method.

The paper's own datasets (GLEAM-like catalogues, GSM / EoR maps, the HERA CST
beam) are not available; the generators below are stand-ins with the same
shapes, sizes and value distributions:

* hexagonal arrays with 14.6 m spacing (the paper's HERA-like layouts, App. A);
* point sources uniform on the sphere with a dN/dS ~ S^-2 power law (Sec. 6.1
  draws sources uniformly across the sky);
* an equal-area ring pixelisation equivalent to HEALPix (Sec. 5.3 uses
  HEALPix maps) with a log-normal brightness field;
* analytic beams sampled on a regular az/za grid with the zenith as the pole
  (Sec. 3.4 requires that geometry).

Every generator takes an explicit seed; the default seed of each workload is
231209763 + workload id, drawn through numpy's PCG64.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Optional

import numpy as np

SEED_BASE = 231209763
HERA_LATITUDE_DEG = -30.7
HEX_SPACING_M = 14.6
SIDEREAL_DAY_RAD = 2.0 * math.pi  # LST advances 2*pi rad per sidereal day


def rng_for(workload: int, salt: int = 0) -> np.random.Generator:
    """PCG64 generator seeded with 231209763 + workload id (+ salt)."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + int(workload) + 1000 * int(salt)))


# --------------------------------------------------------------------------
# Arrays
# --------------------------------------------------------------------------
def hex_array(n_ant: int, spacing: float = HEX_SPACING_M) -> np.ndarray:
    """First ``n_ant`` points of a triangular (hexagonal-packed) lattice.

    Points are ordered by (radius, polar angle in [0, 2pi), axial q) so the
    cut at ``n_ant`` is deterministic when several points share the cut
    radius.  Returns ENU metres, shape [n_ant, 3], with z = 0.
    """
    if n_ant <= 0:
        return np.zeros((0, 3))
    rings = 1
    while 1 + 3 * rings * (rings + 1) < n_ant:
        rings += 1
    rings += 1  # one extra ring so every point at the cut radius is a candidate
    cand = []
    for q in range(-rings, rings + 1):
        for r in range(-rings, rings + 1):
            if abs(q + r) > rings:
                continue
            x = spacing * (q + 0.5 * r)
            y = spacing * (r * math.sqrt(3.0) / 2.0)
            rad = round(math.hypot(x, y), 6)
            ang = round(math.atan2(y, x) % (2.0 * math.pi), 9)
            cand.append((rad, ang, q, x, y))
    cand.sort()
    out = np.zeros((n_ant, 3))
    for i in range(n_ant):
        out[i, 0] = cand[i][3]
        out[i, 1] = cand[i][4]
    return out


# --------------------------------------------------------------------------
# Sky models
# --------------------------------------------------------------------------
def uniform_sphere(rng: np.random.Generator, n: int):
    """RA = 2 pi u, Dec = asin(2 v - 1): uniform on the sphere."""
    u = rng.random(n)
    v = rng.random(n)
    ra = 2.0 * math.pi * u
    dec = np.arcsin(2.0 * v - 1.0)
    return ra, dec


def power_law_fluxes(rng: np.random.Generator, n: int, smin: float = 0.1, smax: float = 10.0):
    """Inverse-CDF draw from dN/dS ~ S^-2 on [smin, smax] (Jy)."""
    f = rng.random(n)
    return 1.0 / (1.0 / smin - f * (1.0 / smin - 1.0 / smax))


def spectral_fluxes(s150: np.ndarray, freqs: np.ndarray, alpha: Optional[np.ndarray]) -> np.ndarray:
    """Per-channel flux [n_freq, n_src] = S_150 (nu / 150 MHz)^alpha (flat if alpha is None)."""
    if alpha is None:
        return np.broadcast_to(s150[None, :], (len(freqs), len(s150))).copy()
    return s150[None, :] * (freqs[:, None] / 150e6) ** alpha[None, :]


def polarised_stokes(flux: np.ndarray, freqs: np.ndarray, seed: int = 0, frac_full: float = 0.05,
                     frac_minus_q: float = 0.01) -> np.ndarray:
    """A physical polarised sky [4][n_freq][n_src] (I, Q, U, V) on top of Stokes I.

    Per source: linear polarisation fraction p ~ U(0, 0.6), circular fraction
    v ~ U(-0.05, 0.05), angle chi(nu) = chi0 + RM (c / nu)^2 with chi0 ~ U(0, pi)
    and a rotation measure RM ~ N(0, 20) rad m^-2 (Faraday rotation), so
    Q = I p cos 2 chi, U = I p sin 2 chi, V = I v.  A fraction frac_full of the
    sources is fully polarised (p^2 + v^2 = 1) and a fraction frac_minus_q has
    Q = -I, U = V = 0 exactly (the I + Q = 0 edge of the brightness matrix's
    square root).  Every source satisfies Q^2 + U^2 + V^2 <= I^2.
    """
    flux = np.asarray(flux, dtype=np.float64)
    n_freq, n_src = flux.shape
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    p = rng.uniform(0.0, 0.6, n_src)
    v = rng.uniform(-0.05, 0.05, n_src)
    full = rng.uniform(size=n_src) < frac_full
    p[full] = np.sqrt(1.0 - v[full] ** 2)
    chi0 = rng.uniform(0.0, math.pi, n_src)
    rm = rng.normal(0.0, 20.0, n_src)
    lam2 = (299792458.0 / np.asarray(freqs, dtype=np.float64)) ** 2
    chi = chi0[None, :] + rm[None, :] * lam2[:, None]
    st = np.empty((4, n_freq, n_src))
    st[0] = flux
    st[1] = flux * p[None, :] * np.cos(2.0 * chi)
    st[2] = flux * p[None, :] * np.sin(2.0 * chi)
    st[3] = flux * v[None, :]
    minus_q = rng.uniform(size=n_src) < frac_minus_q
    st[1][:, minus_q] = -flux[:, minus_q]
    st[2][:, minus_q] = 0.0
    st[3][:, minus_q] = 0.0
    return st


def dipole_modulated_sphere(rng: np.random.Generator, n: int, amp: float):
    """Directions drawn by rejection from a density proportional to 1 + amp * x.

    x is the first Cartesian equatorial component (toward RA = 0, Dec = 0).
    """
    ra = np.empty(0)
    dec = np.empty(0)
    while ra.size < n:
        m = int((n - ra.size) * (1.0 + amp) * 1.1) + 16
        r_, d_ = uniform_sphere(rng, m)
        x = np.cos(r_) * np.cos(d_)
        keep = rng.random(m) * (1.0 + amp) < (1.0 + amp * x)
        ra = np.concatenate([ra, r_[keep]])
        dec = np.concatenate([dec, d_[keep]])
    return ra[:n], dec[:n]


def ring_pixel_centres(nside: int):
    """Centres of the 12 nside^2 equal-area pixels of the HEALPix ring scheme.

    Written from the published ring-scheme definition (Gorski et al. 2005):
    polar-cap rings i = 1..nside-1 hold 4 i pixels at z = 1 - i^2/(3 nside^2),
    the 2 nside + 1 equatorial rings hold 4 nside pixels each at
    z = (2 nside - i) * 2/(3 nside) with a half-pixel phi shift on alternate
    rings.  Returns (ra, dec) in radians, in ring (pixel-index) order.
    """
    npix = 12 * nside * nside
    p = np.arange(npix, dtype=np.int64)
    ncap = 2 * nside * (nside - 1)
    z = np.empty(npix)
    phi = np.empty(npix)

    north = p < ncap
    pn = p[north]
    ir = ((1 + np.sqrt(1 + 2 * pn.astype(np.float64))) // 2).astype(np.int64)
    # guard the float sqrt near ring boundaries
    ir = np.where(2 * ir * (ir - 1) > pn, ir - 1, ir)
    ir = np.where(2 * (ir + 1) * ir <= pn, ir + 1, ir)
    iphi = pn + 1 - 2 * ir * (ir - 1)
    z[north] = 1.0 - ir.astype(np.float64) ** 2 / (3.0 * nside * nside)
    phi[north] = (iphi - 0.5) * math.pi / (2.0 * ir)

    eq = (p >= ncap) & (p < npix - ncap)
    pe = p[eq] - ncap
    ir = pe // (4 * nside) + nside
    iphi = pe % (4 * nside) + 1
    fodd = np.where(((ir + nside) & 1) == 1, 1.0, 0.5)
    z[eq] = (2 * nside - ir) * 2.0 / (3.0 * nside)
    phi[eq] = (iphi - fodd) * math.pi / (2.0 * nside)

    south = p >= npix - ncap
    ps = npix - p[south]  # 1-based from the south pole
    ir = ((1 + np.sqrt(2 * ps.astype(np.float64) - 1)) // 2).astype(np.int64)
    ir = np.where(2 * ir * (ir - 1) >= ps, ir - 1, ir)
    ir = np.where(2 * (ir + 1) * ir < ps, ir + 1, ir)
    iphi = 4 * ir + 1 - (ps - 2 * ir * (ir - 1))
    z[south] = -1.0 + ir.astype(np.float64) ** 2 / (3.0 * nside * nside)
    phi[south] = (iphi - 0.5) * math.pi / (2.0 * ir)

    dec = np.arcsin(np.clip(z, -1.0, 1.0))
    ra = np.mod(phi, 2.0 * math.pi)
    return ra, dec


def morton_order(ra: np.ndarray, dec: np.ndarray, bits: int = 16) -> np.ndarray:
    """Permutation that sorts directions along a 3-D Morton (Z-order) curve."""
    xyz = np.stack([np.cos(ra) * np.cos(dec), np.sin(ra) * np.cos(dec), np.sin(dec)])
    q = np.clip(((xyz + 1.0) * 0.5 * ((1 << bits) - 1)).astype(np.uint64), 0, (1 << bits) - 1)
    key = np.zeros(ra.shape, dtype=np.uint64)
    for b in range(bits):
        for c in range(3):
            key |= ((q[c] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + c)
    return np.argsort(key, kind="stable")


def lognormal_field(rng: np.random.Generator, ra: np.ndarray, dec: np.ndarray,
                    n_waves: int = 1024, scale_min_deg: float = 1.0,
                    scale_max_deg: float = 90.0, chunk: int = 1 << 16) -> np.ndarray:
    """Brightness T = exp(g - 1/2) with g a unit-variance random field.

    g is a sum of ``n_waves`` random 3-D plane waves restricted to the unit
    sphere, with isotropic wave vectors whose length is log-uniform between
    the wavenumbers of the given angular scales (a power-law spectrum).
    """
    kmin = 2.0 * math.pi / math.radians(scale_max_deg)
    kmax = 2.0 * math.pi / math.radians(scale_min_deg)
    kmag = np.exp(rng.uniform(math.log(kmin), math.log(kmax), n_waves))
    kr, kd = uniform_sphere(rng, n_waves)
    kvec = kmag[:, None] * np.stack([np.cos(kr) * np.cos(kd), np.sin(kr) * np.cos(kd), np.sin(kd)], axis=1)
    ph = rng.uniform(0.0, 2.0 * math.pi, n_waves)
    amp = math.sqrt(2.0 / n_waves)
    out = np.empty(ra.shape)

    def one(s):
        e = min(ra.size, s + chunk)
        cd = np.cos(dec[s:e])
        xyz = np.stack([np.cos(ra[s:e]) * cd, np.sin(ra[s:e]) * cd, np.sin(dec[s:e])], axis=1)
        # the products one at a time (not a BLAS call), so the values do not depend on threading
        arg = ph[None, :] + xyz[:, 0:1] * kvec[None, :, 0]
        arg += xyz[:, 1:2] * kvec[None, :, 1]
        arg += xyz[:, 2:3] * kvec[None, :, 2]
        g = amp * np.cos(arg).sum(axis=1)
        out[s:e] = np.exp(g - 0.5)

    # chunks are independent: numpy releases the GIL inside each chunk's work
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(one, range(0, ra.size, chunk)))
    return out


# --------------------------------------------------------------------------
# Beams sampled on the az/za grid (zenith is the pole)
# --------------------------------------------------------------------------
def grid_axes(step_deg: float):
    """za rows 0..90 deg inclusive, az columns 0..360 deg exclusive (periodic)."""
    n_za = int(round(90.0 / step_deg)) + 1
    n_az = int(round(360.0 / step_deg))
    dza = math.radians(90.0) / (n_za - 1)
    daz = 2.0 * math.pi / n_az
    return n_za, n_az, dza, daz


def gaussian_beam(za, az, freq, fwhm150_deg: float = 10.0):
    """Scalar E-field Gaussian whose *power* FWHM is fwhm150 * 150 MHz / nu."""
    fwhm = math.radians(fwhm150_deg) * 150e6 / freq
    sig_e = math.sqrt(2.0) * fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    return np.exp(-np.asarray(za) ** 2 / (2.0 * sig_e ** 2)) + 0j * np.asarray(az)


def dipole_beam(za, az, freq, fwhm150_deg: float = 60.0, chrom: float = 0.1):
    """Complex 2x2 Jones beam J[p, k] of a crossed short-dipole pair.

    Returns an array [2 (feed X, Y), 2 (axis theta, phi), *za.shape].  The
    dipole projections onto (theta-hat, phi-hat) use phi = pi/2 - az, a
    Gaussian envelope with a power FWHM of fwhm150 * 150 MHz / nu, a
    frequency-dependent phase 2 pi chrom (nu / 150 MHz)(1 - cos za) and a
    cos(za) horizon roll-off.
    """
    za = np.asarray(za, dtype=np.float64)
    az = np.asarray(az, dtype=np.float64)
    th = za
    ph = math.pi / 2.0 - az
    fwhm = math.radians(fwhm150_deg) * 150e6 / freq
    sig_e = math.sqrt(2.0) * fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    env = np.exp(-th ** 2 / (2.0 * sig_e ** 2)) * np.exp(1j * 2.0 * math.pi * chrom * (freq / 150e6) * (1.0 - np.cos(th)))
    env = env * np.cos(th)
    out = np.empty((2, 2) + za.shape, dtype=np.complex128)
    out[0, 0] = env * np.cos(th) * np.cos(ph)
    out[0, 1] = env * (-np.sin(ph))
    out[1, 0] = env * np.cos(th) * np.sin(ph)
    out[1, 1] = env * np.cos(ph)
    return out


def beam_grid(kind: str, freqs: np.ndarray, step_deg: float, n_feed: int, n_ax: int) -> np.ndarray:
    """Sample an analytic beam on the az/za grid.

    Returns complex128 [1 (unique beam), n_freq, n_feed, n_ax, n_za, n_az].
    """
    n_za, n_az, dza, daz = grid_axes(step_deg)
    za = (np.arange(n_za) * dza)[:, None] * np.ones((1, n_az))
    az = np.ones((n_za, 1)) * (np.arange(n_az) * daz)[None, :]
    g = np.zeros((1, len(freqs), n_feed, n_ax, n_za, n_az), dtype=np.complex128)
    for f, nu in enumerate(freqs):
        if kind == "gaussian":
            if n_feed != 1 or n_ax != 1:
                raise ValueError("gaussian beam is scalar")
            g[0, f, 0, 0] = gaussian_beam(za, az, nu)
        elif kind == "dipole":
            j = dipole_beam(za, az, nu)
            g[0, f] = j[:n_feed, :n_ax]
        else:
            raise ValueError(kind)
    return g


def antenna_beams(freqs: np.ndarray, step_deg: float, n_beam: int, seed: int = 0,
                  dtype=np.complex64) -> np.ndarray:
    """n_beam distinct crossed-dipole Jones beams on the az/za grid, one per antenna
    (Sec. 3.5 allows a beam per antenna: beam index a_i): beam b has its own power
    FWHM 60 deg x (1 + 0.05 g_b) at 150 MHz and chromatic phase 0.1 x (1 + 0.2 h_b),
    g_b, h_b ~ N(0, 1) seeded.  Returns [n_beam, n_freq, 2, 2, n_za, n_az]."""
    n_za, n_az, dza, daz = grid_axes(step_deg)
    za = (np.arange(n_za) * dza)[:, None] * np.ones((1, n_az))
    az = np.ones((n_za, 1)) * (np.arange(n_az) * daz)[None, :]
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 9000 + int(seed)))
    g, h = rng.normal(0.0, 1.0, n_beam), rng.normal(0.0, 1.0, n_beam)
    out = np.empty((n_beam, len(freqs), 2, 2, n_za, n_az), dtype=dtype)
    for b in range(n_beam):
        for f, nu in enumerate(freqs):
            out[b, f] = dipole_beam(za, az, nu, fwhm150_deg=60.0 * (1.0 + 0.05 * g[b]), chrom=0.1 * (1.0 + 0.2 * h[b]))
    return out


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    antpos: np.ndarray        # [n_ant, 3] ENU metres
    freqs: np.ndarray         # [n_freq] Hz
    lsts: np.ndarray          # [n_time] rad
    ra: np.ndarray            # [n_src] rad
    dec: np.ndarray           # [n_src] rad
    flux: np.ndarray          # [n_freq, n_src] Jy
    beam: np.ndarray          # [n_beam, n_freq, n_feed, n_ax, n_za, n_az] complex128
    beam_kind: str
    latitude: float           # rad
    n_feed: int
    n_ax: int
    dza: float
    daz: float
    interp: str               # "bilinear" | "bicubic"

    @property
    def n_ant(self):
        return self.antpos.shape[0]

    @property
    def n_src(self):
        return self.ra.shape[0]

    @property
    def n_time(self):
        return self.lsts.shape[0]

    @property
    def n_freq(self):
        return self.freqs.shape[0]

    @property
    def radec(self):
        """SoA [2, n_src] (row 0 = RA, row 1 = Dec)."""
        return np.ascontiguousarray(np.stack([self.ra, self.dec]))

    def work_units(self) -> float:
        """src * ant-pair * (t, nu): n_src * n_ant (n_ant + 1) / 2 * n_time * n_freq."""
        return float(self.n_src) * self.n_ant * (self.n_ant + 1) / 2.0 * self.n_time * self.n_freq


def workload(cfg: int, n_ant=None, n_src=None, n_time=None, n_freq=None, seed_salt=0) -> Workload:
    """The five synthetic workloads (optionally shrunk for fast tests).

    1: 37-antenna hex, 2000 uniform sources, 4 LSTs 10 sidereal minutes apart,
       150/160 MHz, scalar Gaussian beam on a 1 deg grid, bilinear.
    2: 128-antenna hex, 2 feeds x 2 axes, 50 000 uniform sources with
       power-law fluxes and spectral index ~ N(-0.8, 0.2), 32 LSTs over 24 h,
       16 channels 100-200 MHz, dipole beam on a 0.5 deg grid, bicubic.
    3: 350-antenna hex, scalar, 3 145 728 equal-area pixels (nside 512) with a
       log-normal brightness, 64 LSTs, 128 channels 50-250 MHz, Gaussian
       beam on a 1 deg grid, bilinear.
    4: 128 antennas polarised, 200 000 sources from a dipole-modulated density
       (visible fraction 40-60 % over the day), 16 LSTs x 16 channels.
    5: the array and sky of 3, polarised (2 x 2 dipole beam), channels of 3
       inside 100-200 MHz.
    """
    rng = rng_for(cfg, seed_salt)
    lat = math.radians(HERA_LATITUDE_DEG)
    if cfg == 1:
        na, ns, nt, nf = 37, 2000, 4, 2
        na, ns, nt, nf = (n_ant or na), (n_src or ns), (n_time or nt), (n_freq or nf)
        freqs = np.array([150e6, 160e6])[:nf] if nf <= 2 else np.linspace(150e6, 160e6, nf)
        lsts = np.arange(nt) * (10.0 / 1440.0) * SIDEREAL_DAY_RAD
        ra, dec = uniform_sphere(rng, ns)
        s = power_law_fluxes(rng, ns)
        flux = spectral_fluxes(s, freqs, None)
        n_feed, n_ax, step, kind, interp = 1, 1, 1.0, "gaussian", "bilinear"
    elif cfg in (2, 4):
        na = 128
        ns = 50_000 if cfg == 2 else 200_000
        nt, nf = (32, 16) if cfg == 2 else (16, 16)
        na, ns, nt, nf = (n_ant or na), (n_src or ns), (n_time or nt), (n_freq or nf)
        freqs = np.linspace(100e6, 200e6, nf)
        lsts = np.arange(nt) * (SIDEREAL_DAY_RAD / nt)
        if cfg == 2:
            ra, dec = uniform_sphere(rng, ns)
        else:
            ra, dec = dipole_modulated_sphere(rng, ns, 0.4652)
        s = power_law_fluxes(rng, ns)
        alpha = rng.normal(-0.8, 0.2, ns)
        flux = spectral_fluxes(s, freqs, alpha)
        n_feed, n_ax, step, kind, interp = 2, 2, 0.5, "dipole", "bicubic"
    elif cfg in (3, 5):
        na = 350
        nside = 512
        nt = 64
        na, nt = (n_ant or na), (n_time or nt)
        freqs_all = np.linspace(50e6, 250e6, 128)
        if cfg == 5:
            freqs_all = freqs_all[(freqs_all >= 100e6) & (freqs_all <= 200e6)]
        nf = n_freq or len(freqs_all)
        freqs = freqs_all[np.linspace(0, len(freqs_all) - 1, nf).round().astype(int)] if nf < len(freqs_all) else freqs_all
        lsts = np.arange(nt) * (SIDEREAL_DAY_RAD / nt)
        if n_src is not None:
            # shrunk variant: a coarser equal-area pixelisation of the same kind
            nside = max(1, int(round(math.sqrt(n_src / 12.0))))
        ra, dec = ring_pixel_centres(nside)
        order = morton_order(ra, dec)
        ra, dec = ra[order], dec[order]
        omega = 4.0 * math.pi / ra.size
        t = lognormal_field(rng, ra, dec)
        flux = (t * omega)[None, :] * (freqs[:, None] / 150e6) ** -0.5
        if cfg == 3:
            n_feed, n_ax, step, kind, interp = 1, 1, 1.0, "gaussian", "bilinear"
        else:
            n_feed, n_ax, step, kind, interp = 2, 2, 0.5, "dipole", "bicubic"
    else:
        raise ValueError(f"unknown workload {cfg}")
    antpos = hex_array(na)
    grid = beam_grid(kind, freqs, step, n_feed, n_ax)
    n_za, n_az, dza, daz = grid_axes(step)
    return Workload(name=f"workload{cfg}", antpos=antpos, freqs=np.asarray(freqs, dtype=np.float64),
                    lsts=np.asarray(lsts, dtype=np.float64), ra=ra, dec=dec,
                    flux=np.ascontiguousarray(flux, dtype=np.float64), beam=grid, beam_kind=kind,
                    latitude=lat, n_feed=n_feed, n_ax=n_ax, dza=dza, daz=daz, interp=interp)


# --------------------------------------------------------------------------
# Learned beam: random draws only (initial parameters and sample points)
# --------------------------------------------------------------------------
# Parameter-vector order of the learned beam: (name, shape) in storage order.
SURROGATE_LAYOUT = (("Bff", (128, 2)), ("W1", (128, 256)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)),
                    ("W3", (128, 128)), ("b3", (128,)), ("W4", (128, 128)), ("b4", (128,)), ("W5", (64, 128)),
                    ("b5", (64,)))
SURROGATE_N_PARAMS = sum(int(np.prod(s)) for _, s in SURROGATE_LAYOUT)  # 90944


def surrogate_init(seed: int, az_max: int = 4, sigma_v: float = 2.0) -> np.ndarray:
    """Initial learned-beam parameters (float32 [90944]).

    Fourier matrix rows (az, za columns): integer az frequencies uniform in
    [-az_max, az_max] (features periodic in az) and N(0, sigma_v^2) for the za
    column.  Weights and biases of every layer uniform in +-1 / sqrt(fan_in).
    """
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 7000 + int(seed)))
    parts = []
    for name, shape in SURROGATE_LAYOUT:
        if name == "Bff":
            b = np.empty(shape)
            b[:, 0] = rng.integers(-az_max, az_max + 1, shape[0])
            b[:, 1] = rng.normal(0.0, sigma_v, shape[0])
            parts.append(b.ravel())
        else:
            fan_in = {"W1": 256, "b1": 256, "W5": 128, "b5": 128}.get(name, 128)
            parts.append(rng.uniform(-1.0, 1.0, int(np.prod(shape))) / math.sqrt(fan_in))
    return np.concatenate(parts).astype(np.float32)


def hemisphere_points(rng: np.random.Generator, n: int):
    """(za, az) uniform by solid angle over the visible hemisphere (cos za ~ U(0, 1])."""
    za = np.arccos(1.0 - rng.random(n))
    az = rng.random(n) * 2.0 * math.pi
    return za, az
