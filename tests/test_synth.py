"""Checks on the seeded input generators (CPU only)."""
import json
import math
import os

import numpy as np

from paper_2312_09763_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_hex_array_full_hexagon_and_cut_ties():
    a = synth.hex_array(37)
    r = np.hypot(a[:, 0], a[:, 1])
    assert a.shape == (37, 3) and np.all(a[:, 2] == 0)
    assert abs(r.max() - 3 * 14.6) < 1e-9  # 4 antennas per side
    # nearest-neighbour distance is the spacing
    d = np.hypot(*(a[:, None, :2] - a[None, :, :2]).transpose(2, 0, 1))
    d[d == 0] = np.inf
    assert abs(d.min() - 14.6) < 1e-9
    # 350 cuts through a ring: deterministic and unique positions
    b = synth.hex_array(350)
    assert np.unique(np.round(b, 6), axis=0).shape[0] == 350
    np.testing.assert_array_equal(b, synth.hex_array(350))
    np.testing.assert_array_equal(synth.hex_array(128)[:37], a)


def test_power_law_moments():
    rng = np.random.default_rng(0)
    s = synth.power_law_fluxes(rng, 400_000)
    assert s.min() >= 0.1 and s.max() <= 10.0
    # mean of dN/dS ~ S^-2 on [a, b]: ln(b/a) / (1/a - 1/b)
    want = math.log(100.0) / (10.0 - 0.1)
    assert abs(s.mean() - want) / want < 0.01


def test_uniform_sphere_moments():
    ra, dec = synth.uniform_sphere(np.random.default_rng(1), 200_000)
    z = np.sin(dec)
    assert abs(z.mean()) < 0.01 and abs((z ** 2).mean() - 1 / 3) < 0.01
    assert abs(np.cos(ra).mean()) < 0.01


def test_ring_pixels_nside1_and_area():
    ra, dec = synth.ring_pixel_centres(1)
    np.testing.assert_allclose(np.sort(np.sin(dec)), [-2 / 3] * 4 + [0] * 4 + [2 / 3] * 4, atol=1e-15)
    for nside in (2, 4, 16):
        ra, dec = synth.ring_pixel_centres(nside)
        assert ra.size == 12 * nside * nside
        xyz = np.stack([np.cos(ra) * np.cos(dec), np.sin(ra) * np.cos(dec), np.sin(dec)], 1)
        assert np.abs(xyz.mean(0)).max() < 1e-12  # equal-area, symmetric tessellation
        assert np.unique(np.round(xyz, 9), axis=0).shape[0] == ra.size


def test_ring_pixel_resolution_matches_paper():
    with open(os.path.join(HERE, "golden", "healpix_resolution.json")) as fh:
        gold = json.load(fh)
    for c in gold["cases"]:
        res = math.degrees(math.sqrt(4 * math.pi / (12 * c["nside"] ** 2))) * 60
        assert abs(res - c["resolution_arcmin"]) / c["resolution_arcmin"] < gold["rel_tol"]


def test_dipole_modulated_visible_fraction():
    """Visible fraction of density 1 + A x is 1/2 + (A/4) cos(lat) cos(LST)."""
    rng = np.random.default_rng(3)
    ra, dec = synth.dipole_modulated_sphere(rng, 400_000, 0.4652)
    lat = math.radians(synth.HERA_LATITUDE_DEG)
    for lst in (0.0, math.pi / 2, math.pi):
        h = lst - ra
        up = math.cos(lat) * np.cos(dec) * np.cos(h) + math.sin(lat) * np.sin(dec)
        want = 0.5 + 0.4652 / 4 * math.cos(lat) * math.cos(lst)
        assert abs((up > 0).mean() - want) < 3e-3


def test_grid_axes_and_beams():
    n_za, n_az, dza, daz = synth.grid_axes(0.5)
    assert (n_za, n_az) == (181, 720)
    assert abs((n_za - 1) * dza - math.pi / 2) < 1e-15 and abs(n_az * daz - 2 * math.pi) < 1e-15
    g = synth.beam_grid("gaussian", np.array([150e6]), 1.0, 1, 1)
    assert g.shape == (1, 1, 1, 1, 91, 360)
    # power beam at half the FWHM from the zenith is one half
    fwhm = math.radians(10.0)
    assert abs(abs(synth.gaussian_beam(fwhm / 2, 0.0, 150e6)) ** 2 - 0.5) < 1e-12
    j = synth.dipole_beam(np.array([0.0]), np.array([0.3]), 150e6)
    # at the zenith the X dipole responds along theta/phi according to phi = pi/2 - az
    ph = math.pi / 2 - 0.3
    np.testing.assert_allclose(j[0, :, 0], [math.cos(ph), -math.sin(ph)], atol=1e-15)
    jh = synth.dipole_beam(np.array([math.pi / 2]), np.array([1.0]), 150e6)
    assert np.abs(jh).max() < 1e-15  # rolls off to zero on the horizon


def test_workloads_shapes():
    wl = synth.workload(1)
    assert (wl.n_ant, wl.n_src, wl.n_time, wl.n_freq) == (37, 2000, 4, 2)
    assert wl.beam.shape == (1, 2, 1, 1, 91, 360)
    wl = synth.workload(2, n_src=500, n_time=3, n_freq=2)
    assert wl.n_ant == 128 and wl.beam.shape == (1, 2, 2, 2, 181, 720)
    assert wl.flux.shape == (2, 500) and np.all(wl.flux > 0)
    wl = synth.workload(3, n_ant=20, n_src=12 * 16 * 16, n_time=2, n_freq=3)
    mean_t = wl.flux[0].sum() / (4 * math.pi / 3072) / 3072 / (wl.freqs[0] / 150e6) ** -0.5
    assert wl.n_src == 3072 and abs(mean_t - 1) < 0.3  # log-normal brightness has mean 1


def test_lognormal_field_independent_of_chunking():
    # the chunks run on a thread pool: the field must not depend on how the
    # pixels are cut, and it is log-normal with unit mean in expectation
    ra, dec = synth.ring_pixel_centres(16)
    f1 = synth.lognormal_field(np.random.Generator(np.random.PCG64(3)), ra, dec, chunk=1 << 16)
    f2 = synth.lognormal_field(np.random.Generator(np.random.PCG64(3)), ra, dec, chunk=97)
    np.testing.assert_array_equal(f1, f2)
    assert np.all(f1 > 0) and 0.5 < f1.mean() < 1.5
