"""FP64 CPU reference for the visibility simulator -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The product path (the HIP library and its
Python binding) never does, and shares no code with it.

The arithmetic lives in ``matvis_oracle.c`` (plain C, double precision); this
module compiles it with gcc and wraps it with ctypes and numpy.  The
surrogate-network reference is in ``mlp.py`` (numpy, float64).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "matvis_oracle.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_SO = os.path.join(_OUT_DIR, "liboracle.so")

_lib = None


_SO_LD = os.path.join(_OUT_DIR, "liboracle_ld.so")
_lib_ld = None


def _gcc(out: str, extra) -> None:
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off"] +
                          list(extra) + ["-o", tmp, _SRC, "-lm"])
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the C reference with gcc (plain -O2, IEEE semantics, OpenMP): the
    double build, and the same source with long double arithmetic (used only to
    bound the double build's own rounding on small cases)."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    for so, extra in ((_SO, []), (_SO_LD, ['-DORC_REAL=long double'])):
        if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(_SRC):
            _gcc(so, extra)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_SO)
        _declare(_lib)
    return _lib


def lib_ld():
    """The long double build (same source, ORC_REAL = long double)."""
    global _lib_ld
    if _lib_ld is None:
        if not os.path.exists(_SO_LD) or os.path.getmtime(_SO_LD) < os.path.getmtime(_SRC):
            build(force=True)
        _lib_ld = ctypes.CDLL(_SO_LD)
        _lib_ld.orc_simulate.argtypes = [ctypes.POINTER(GeomLD)] + [_P] * 3 + [ctypes.c_int32, _P, ctypes.c_int64] + \
            [_P] * 4 + [ctypes.c_int32] + [_P] * 3
        _lib_ld.orc_simulate.restype = ctypes.c_int
    return _lib_ld


class Geom(ctypes.Structure):
    _fields_ = [("n_ant", ctypes.c_int32), ("n_feed", ctypes.c_int32), ("n_ax", ctypes.c_int32),
                ("n_beam", ctypes.c_int32), ("n_za", ctypes.c_int32), ("n_az", ctypes.c_int32),
                ("dza", ctypes.c_double), ("daz", ctypes.c_double), ("latitude", ctypes.c_double),
                ("interp", ctypes.c_int32)]


class GeomLD(ctypes.Structure):
    _fields_ = [("n_ant", ctypes.c_int32), ("n_feed", ctypes.c_int32), ("n_ax", ctypes.c_int32),
                ("n_beam", ctypes.c_int32), ("n_za", ctypes.c_int32), ("n_az", ctypes.c_int32),
                ("dza", ctypes.c_longdouble), ("daz", ctypes.c_longdouble), ("latitude", ctypes.c_longdouble),
                ("interp", ctypes.c_int32)]


_P = ctypes.c_void_p


def _declare(L):
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_get_threads.restype = ctypes.c_int
    L.orc_xeq.argtypes = [ctypes.c_int64, _P, _P, _P]
    L.orc_rotation.argtypes = [ctypes.c_double, ctypes.c_double, _P]
    L.orc_topocentric.argtypes = [_P, ctypes.c_int64, _P, _P]
    L.orc_visible.argtypes = [ctypes.c_int64, _P, _P]
    L.orc_visible.restype = ctypes.c_int64
    L.orc_azza.argtypes = [ctypes.c_int64, _P, _P, _P]
    L.orc_interp.argtypes = [ctypes.c_int, _P, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                             ctypes.c_int64, _P, _P, _P]
    L.orc_simulate.argtypes = [ctypes.POINTER(Geom), _P, _P, _P, ctypes.c_int32, _P, ctypes.c_int64, _P, _P, _P,
                               _P, ctypes.c_int32, _P, _P, _P]
    L.orc_simulate.restype = ctypes.c_int
    L.orc_simulate_pairs.argtypes = [ctypes.POINTER(Geom), _P, _P, _P, ctypes.c_int32, _P, ctypes.c_int64, _P, _P,
                                     _P, _P, ctypes.c_int32, _P, _P, ctypes.c_int32, _P, _P, _P]
    L.orc_simulate_pairs.restype = ctypes.c_int
    L.orc_simulate_pol.argtypes = [ctypes.POINTER(Geom), _P, _P, _P, ctypes.c_int32, _P, ctypes.c_int64, _P, _P,
                                   _P, _P, ctypes.c_int32, _P, _P, ctypes.c_int32, _P, _P, _P]
    L.orc_simulate_pol.restype = ctypes.c_int
    L.orc_simulate_given_beam.argtypes = [ctypes.POINTER(Geom), _P, _P, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_int64, _P, _P, _P, _P, _P]
    L.orc_simulate_given_beam.restype = ctypes.c_int64
    L.orc_zmatrix.argtypes = [ctypes.POINTER(Geom), _P, _P, ctypes.c_double, ctypes.c_int64, _P, _P, _P,
                              ctypes.c_int64, _P]
    L.orc_gram.argtypes = [ctypes.c_int64, ctypes.c_int64, _P, _P]
    L.orc_instance_sky.argtypes = [ctypes.POINTER(Geom), ctypes.c_double, ctypes.c_int64, _P, _P, _P, _P, _P, _P]
    L.orc_instance_sky.restype = ctypes.c_int64


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _c128(x):
    return np.ascontiguousarray(x, dtype=np.complex128)


def _i32(x):
    return np.ascontiguousarray(x, dtype=np.int32)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


# ---- step-level functions -------------------------------------------------
def xeq(ra, dec) -> np.ndarray:
    ra, dec = _f64(ra), _f64(dec)
    out = np.empty((ra.size, 3))
    lib().orc_xeq(ra.size, _ptr(ra), _ptr(dec), _ptr(out))
    return out


def rotation(lst: float, latitude: float) -> np.ndarray:
    R = np.empty((3, 3))
    lib().orc_rotation(float(lst), float(latitude), _ptr(R))
    return R


def topocentric(R, x_eq) -> np.ndarray:
    R, x_eq = _f64(R), _f64(x_eq)
    out = np.empty_like(x_eq)
    lib().orc_topocentric(_ptr(R), x_eq.shape[0], _ptr(x_eq), _ptr(out))
    return out


def visible(x_hrz) -> np.ndarray:
    x_hrz = _f64(x_hrz)
    idx = np.empty(x_hrz.shape[0], dtype=np.int32)
    m = lib().orc_visible(x_hrz.shape[0], _ptr(x_hrz), _ptr(idx))
    return idx[:m].copy()


def azza(x_hrz):
    x_hrz = _f64(x_hrz)
    n = x_hrz.shape[0]
    az, za = np.empty(n), np.empty(n)
    lib().orc_azza(n, _ptr(x_hrz), _ptr(az), _ptr(za))
    return az, za


def interp(mode: str, plane, dza: float, daz: float, za, az) -> np.ndarray:
    plane = _c128(plane)
    za, az = _f64(za), _f64(az)
    out = np.empty(za.size, dtype=np.complex128)
    lib().orc_interp(0 if mode == "bilinear" else 1, _ptr(plane), plane.shape[0], plane.shape[1], dza, daz,
                     za.size, _ptr(za), _ptr(az), _ptr(out))
    return out


def _geom(n_ant, n_feed, n_ax, n_beam, n_za, n_az, dza, daz, latitude, interp_mode) -> Geom:
    return Geom(n_ant, n_feed, n_ax, n_beam, n_za, n_az, dza, daz, latitude,
                0 if interp_mode == "bilinear" else 1)


def simulate(antpos, freqs, lsts, ra, dec, flux, beam_grid, latitude: float, dza: float, daz: float,
             interp_mode: str, instances: Optional[Sequence] = None, beam_idx=None) -> np.ndarray:
    """Direct-sum visibilities V[inst][a][b][p][q] (complex128).

    ``instances`` is a list of (t, f) pairs; default: every (t, f) in
    t-major order.  beam_grid is [n_beam][n_freq][n_feed][n_ax][n_za][n_az].
    flux is Stokes I [n_freq][n_src], or a polarised sky [4][n_freq][n_src]
    (I, Q, U, V; needs n_ax = 2).
    """
    antpos, freqs, lsts, ra, dec, flux = map(_f64, (antpos, freqs, lsts, ra, dec, flux))
    if flux.ndim == 3:
        return _simulate_pol(antpos, freqs, lsts, ra, dec, flux, beam_grid, latitude, dza, daz, interp_mode,
                             instances, None, beam_idx)
    beam_grid = _c128(beam_grid)
    nb, nfreq, nf, nx, nza, naz = beam_grid.shape
    na = antpos.shape[0]
    if instances is None:
        instances = [(t, f) for t in range(lsts.size) for f in range(freqs.size)]
    it = _i32([i[0] for i in instances])
    iff = _i32([i[1] for i in instances])
    bi = None if beam_idx is None else _i32(beam_idx)
    G = _geom(na, nf, nx, nb, nza, naz, dza, daz, latitude, interp_mode)
    V = np.zeros((len(instances), na, na, nf, nf), dtype=np.complex128)
    rc = lib().orc_simulate(ctypes.byref(G), _ptr(antpos), _ptr(bi), _ptr(freqs), freqs.size, _ptr(lsts),
                            ra.size, _ptr(ra), _ptr(dec), _ptr(flux), _ptr(beam_grid), len(instances),
                            _ptr(it), _ptr(iff), _ptr(V))
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return V


def simulate_pairs(antpos, freqs, lsts, ra, dec, flux, beam_grid, latitude: float, dza: float, daz: float,
                   interp_mode: str, instances: Sequence, pairs: Sequence, beam_idx=None) -> np.ndarray:
    """Direct sum for selected antenna pairs only: V[inst][pair][p][q] (complex128).
    flux as in simulate (Stokes I, or [4][n_freq][n_src] for a polarised sky)."""
    antpos, freqs, lsts, ra, dec, flux = map(_f64, (antpos, freqs, lsts, ra, dec, flux))
    if flux.ndim == 3:
        return _simulate_pol(antpos, freqs, lsts, ra, dec, flux, beam_grid, latitude, dza, daz, interp_mode,
                             instances, pairs, beam_idx)
    beam_grid = _c128(beam_grid)
    nb, nfreq, nf, nx, nza, naz = beam_grid.shape
    na = antpos.shape[0]
    it = _i32([i[0] for i in instances])
    iff = _i32([i[1] for i in instances])
    pa = _i32([p[0] for p in pairs])
    pb = _i32([p[1] for p in pairs])
    bi = None if beam_idx is None else _i32(beam_idx)
    G = _geom(na, nf, nx, nb, nza, naz, dza, daz, latitude, interp_mode)
    V = np.zeros((len(instances), len(pairs), nf, nf), dtype=np.complex128)
    rc = lib().orc_simulate_pairs(ctypes.byref(G), _ptr(antpos), _ptr(bi), _ptr(freqs), freqs.size, _ptr(lsts),
                                  ra.size, _ptr(ra), _ptr(dec), _ptr(flux), _ptr(beam_grid), len(instances),
                                  _ptr(it), _ptr(iff), len(pairs), _ptr(pa), _ptr(pb), _ptr(V))
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return V


def _simulate_pol(antpos, freqs, lsts, ra, dec, stokes, beam_grid, latitude, dza, daz, interp_mode, instances, pairs,
                  beam_idx):
    """Polarised-sky direct sum (Sec. 2.1 brightness matrix from I, Q, U, V)."""
    beam_grid = _c128(beam_grid)
    nb, nfreq, nf, nx, nza, naz = beam_grid.shape
    if nx != 2 or stokes.shape[0] != 4:
        raise ValueError("a polarised sky needs two E-field axes and stokes [4][n_freq][n_src]")
    na = antpos.shape[0]
    if instances is None:
        instances = [(t, f) for t in range(lsts.size) for f in range(freqs.size)]
    it = _i32([i[0] for i in instances])
    iff = _i32([i[1] for i in instances])
    bi = None if beam_idx is None else _i32(beam_idx)
    G = _geom(na, nf, nx, nb, nza, naz, dza, daz, latitude, interp_mode)
    if pairs is None:
        V = np.zeros((len(instances), na, na, nf, nf), dtype=np.complex128)
        pa = pb = None
        npair = -1
    else:
        V = np.zeros((len(instances), len(pairs), nf, nf), dtype=np.complex128)
        pa = _i32([p[0] for p in pairs])
        pb = _i32([p[1] for p in pairs])
        npair = len(pairs)
    rc = lib().orc_simulate_pol(ctypes.byref(G), _ptr(antpos), _ptr(bi), _ptr(freqs), freqs.size, _ptr(lsts),
                                ra.size, _ptr(ra), _ptr(dec), _ptr(_f64(stokes)), _ptr(beam_grid), len(instances),
                                _ptr(it), _ptr(iff), npair, _ptr(pa), _ptr(pb), _ptr(V))
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return V


def simulate_given_beam(antpos, freq: float, lst: float, ra, dec, flux_f, A_all, latitude: float,
                        beam_idx=None) -> np.ndarray:
    """Direct sum for one instance with the beam given at every source.

    A_all is [n_beam][n_feed][n_ax][n_src].  Returns V[a][b][p][q].
    """
    antpos, ra, dec, flux_f = map(_f64, (antpos, ra, dec, flux_f))
    A_all = _c128(A_all)
    nb, nf, nx, ns = A_all.shape
    na = antpos.shape[0]
    G = _geom(na, nf, nx, nb, 3, 3, 1.0, 1.0, latitude, "bilinear")
    bi = None if beam_idx is None else _i32(beam_idx)
    V = np.zeros((na, na, nf, nf), dtype=np.complex128)
    lib().orc_simulate_given_beam(ctypes.byref(G), _ptr(antpos), _ptr(bi), float(freq), float(lst), ns,
                                  _ptr(ra), _ptr(dec), _ptr(flux_f), _ptr(A_all), _ptr(V))
    return V


def instance_sky(lst: float, ra, dec, beam_f, latitude: float, dza: float, daz: float, interp_mode: str):
    """Visible indices, their X_hrz [m][3] and the beam A [n_beam][n_feed][n_ax][m]."""
    ra, dec = _f64(ra), _f64(dec)
    beam_f = _c128(beam_f)
    nb, nf, nx, nza, naz = beam_f.shape
    G = _geom(0, nf, nx, nb, nza, naz, dza, daz, latitude, interp_mode)
    ns = ra.size
    idx = np.empty(ns, dtype=np.int32)
    xv = np.empty((ns, 3))
    A = np.empty((nb, nf, nx, ns), dtype=np.complex128)
    m = lib().orc_instance_sky(ctypes.byref(G), float(lst), ns, _ptr(ra), _ptr(dec), _ptr(beam_f), _ptr(idx),
                               _ptr(xv), _ptr(A))
    return idx[:m].copy(), xv[:m].copy(), A[..., :m].copy()


def zmatrix(antpos, freq: float, x_hrz_vis, flux_vis, A, beam_idx=None) -> np.ndarray:
    """Z [(a, p)][(n, k)] of Eq. (littlez) for one instance (complex128)."""
    antpos, x_hrz_vis, flux_vis = map(_f64, (antpos, x_hrz_vis, flux_vis))
    A = _c128(A)
    nb, nf, nx, m = A.shape
    na = antpos.shape[0]
    G = _geom(na, nf, nx, nb, 3, 3, 1.0, 1.0, 0.0, "bilinear")
    bi = None if beam_idx is None else _i32(beam_idx)
    Z = np.empty((na * nf, m * nx), dtype=np.complex128)
    lib().orc_zmatrix(ctypes.byref(G), _ptr(antpos), _ptr(bi), float(freq), m, _ptr(x_hrz_vis), _ptr(flux_vis),
                      _ptr(A), m, _ptr(Z))
    return Z


def gram(Z) -> np.ndarray:
    """Z Z^H by definition (Eq. zz), both triangles."""
    Z = _c128(Z)
    V = np.empty((Z.shape[0], Z.shape[0]), dtype=np.complex128)
    lib().orc_gram(Z.shape[0], Z.shape[1], _ptr(Z), _ptr(V))
    return V


def simulate_longdouble(antpos, freqs, lsts, ra, dec, flux, beam_grid, latitude: float, dza: float, daz: float,
                        interp_mode: str, instances: Optional[Sequence] = None) -> np.ndarray:
    """The direct sum of ``simulate`` (Stokes I, one beam or beam_idx = None) in long
    double arithmetic: the same C source built with ORC_REAL = long double.  The
    inputs are the double values, widened exactly; the result is V[inst][a][b][p][q]
    as numpy clongdouble.  Used only to bound the double build's own error."""
    ld, cld = np.longdouble, np.clongdouble
    if np.finfo(ld).nmant <= np.finfo(np.float64).nmant:
        raise RuntimeError("long double is not wider than double on this platform")
    conv = lambda x: np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(ld))
    antpos, freqs, lsts, ra, dec, flux = map(conv, (antpos, freqs, lsts, ra, dec, flux))
    beam_grid = np.ascontiguousarray(np.asarray(beam_grid, dtype=np.complex128).astype(cld))
    nb, nfreq, nf, nx, nza, naz = beam_grid.shape
    na = antpos.shape[0]
    if instances is None:
        instances = [(t, f) for t in range(lsts.size) for f in range(freqs.size)]
    it = _i32([i[0] for i in instances])
    iff = _i32([i[1] for i in instances])
    G = GeomLD(na, nf, nx, nb, nza, naz, dza, daz, latitude, 0 if interp_mode == "bilinear" else 1)
    V = np.zeros((len(instances), na, na, nf, nf), dtype=cld)
    rc = lib_ld().orc_simulate(ctypes.byref(G), _ptr(antpos), None, _ptr(freqs), freqs.size, _ptr(lsts), ra.size,
                               _ptr(ra), _ptr(dec), _ptr(flux), _ptr(beam_grid), len(instances), _ptr(it),
                               _ptr(iff), _ptr(V))
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return V
