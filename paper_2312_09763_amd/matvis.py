"""Python binding of libmatvis (ctypes).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of libmatvis.so.  PyTorch supplies device memory and the stream;
tensors are passed by ``data_ptr()`` and must already live on the GPU in the
dtype and layout the C ABI documents (include/matvis.h).

The library is loaded from ``paper_2312_09763_amd/_lib/libmatvis.so`` (built
in-tree by ``paper_2312_09763_amd/build.py``).  There is no fallback: if the
library is missing or cannot be loaded, every entry point raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libmatvis.so")

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, ESTATE, EDATA = 0, -1, -2, -3, -4, -5, -6
FP64, FP32, BF16X3 = 0, 1, 2
BILINEAR, BICUBIC, SURROGATE = 0, 1, 2
FLAG_NO_GRAPH = 1
FLAG_UNFUSED = 2
FLAG_POLARISED_SKY = 4

STEPS = ("sky", "beam", "zform", "herk", "reduce", "other", "herk_pairs")
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
BEAM_MODES = {"bilinear": BILINEAR, "bicubic": BICUBIC, "surrogate": SURROGATE}
MLP_N_PARAMS = 90944  # learned-beam parameter count (include/matvis.h)
PRODUCT_PATHS = ("z_in_hbm", "fused", "fused_rows", "sources", "fused_blocks")  # matvis_product_path


class MatvisError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_status_name(status)}: {message}")
        self.status = status


class _Config(ctypes.Structure):
    _fields_ = [("n_ant", ctypes.c_int32), ("n_feed", ctypes.c_int32), ("n_ax", ctypes.c_int32),
                ("n_beam", ctypes.c_int32), ("max_src", ctypes.c_int64), ("max_time", ctypes.c_int32),
                ("max_freq", ctypes.c_int32), ("latitude_rad", ctypes.c_double), ("precision", ctypes.c_int32),
                ("beam_mode", ctypes.c_int32), ("n_za", ctypes.c_int32), ("n_az", ctypes.c_int32),
                ("dza_rad", ctypes.c_double), ("daz_rad", ctypes.c_double), ("src_chunk", ctypes.c_int64),
                ("batch_time", ctypes.c_int32), ("batch_freq", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("ksplit", ctypes.c_int64), ("tile", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p


def load_library():
    """Load libmatvis.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libmatvis.so not found at {LIB_PATH}; build it with paper_2312_09763_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    L.matvis_init.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(_P)]
    L.matvis_init.restype = ctypes.c_int
    L.matvis_simulate.argtypes = [_P, _P, _P, _P, ctypes.c_int32, _P, ctypes.c_int32, _P, ctypes.c_int64, _P, _P,
                                  _P, _P]
    L.matvis_simulate.restype = ctypes.c_int
    L.matvis_finish.argtypes = [_P]
    L.matvis_finish.restype = ctypes.c_int
    L.matvis_last_error.argtypes = [_P]
    L.matvis_last_error.restype = ctypes.c_char_p
    L.matvis_status_string.argtypes = [ctypes.c_int32]
    L.matvis_status_string.restype = ctypes.c_char_p
    L.matvis_destroy.argtypes = [_P]
    L.matvis_destroy.restype = None
    L.matvis_step_sky.argtypes = [_P, _P, ctypes.c_int32, _P, ctypes.c_int64, _P, _P, _P, _P, _P]
    L.matvis_step_sky.restype = ctypes.c_int
    L.matvis_step_interp.argtypes = [_P, _P, ctypes.c_int64, _P, _P, _P]
    L.matvis_step_interp.restype = ctypes.c_int
    L.matvis_step_herk.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _P, _P]
    L.matvis_step_herk.restype = ctypes.c_int
    L.matvis_autotune.argtypes = [ctypes.POINTER(_Config), _P, _P, _P, ctypes.c_int32, _P, ctypes.c_int32, _P,
                                  ctypes.c_int64, _P, _P, _P, _P, ctypes.c_char_p, ctypes.POINTER(_Config),
                                  ctypes.POINTER(ctypes.c_double), _P, ctypes.c_double, ctypes.c_double]
    L.matvis_autotune.restype = ctypes.c_int
    L.matvis_profile_enable.argtypes = [_P, ctypes.c_int32]
    L.matvis_profile_enable.restype = ctypes.c_int
    L.matvis_profile_read.argtypes = [_P, _P, _P]
    L.matvis_profile_read.restype = ctypes.c_int
    L.matvis_mlp_forward.argtypes = [_P, _P, ctypes.c_int64, _P, _P]
    L.matvis_mlp_forward.restype = ctypes.c_int
    L.matvis_mlp_loss_grad.argtypes = [_P, _P, _P, ctypes.c_int64, ctypes.c_int32, _P, _P, _P]
    L.matvis_mlp_loss_grad.restype = ctypes.c_int
    L.matvis_mlp_loss_grad_noalloc.argtypes = [_P, _P, _P, ctypes.c_int64, ctypes.c_int32, _P, _P, _P]
    L.matvis_mlp_loss_grad_noalloc.restype = ctypes.c_int
    L.matvis_mlp_adam.argtypes = [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_float, _P]
    L.matvis_mlp_adam.restype = ctypes.c_int
    L.matvis_beam_samples.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32, _P, _P, _P,
                                      ctypes.c_int64, _P, _P, ctypes.c_double, ctypes.c_double, _P, _P]
    L.matvis_beam_samples.restype = ctypes.c_int
    L.matvis_train_surrogate.argtypes = [_P, _P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_uint64, ctypes.c_int32, _P, _P]
    L.matvis_train_surrogate.restype = ctypes.c_int
    L.matvis_set_surrogate.argtypes = [_P, _P, ctypes.c_double, ctypes.c_double]
    L.matvis_set_surrogate.restype = ctypes.c_int
    L.matvis_product_path_of.argtypes = [_P]
    L.matvis_product_path_of.restype = ctypes.c_int32
    L.matvis_redundant_groups.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_double, _P, _P, _P, _P]
    L.matvis_redundant_groups.restype = ctypes.c_int
    L.matvis_submatrix_plan.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P]
    L.matvis_submatrix_plan.restype = ctypes.c_int
    L.matvis_set_pairs.argtypes = [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P]
    L.matvis_set_pairs.restype = ctypes.c_int
    L.matvis_simulate_pairs.argtypes = [_P, _P, _P, _P, ctypes.c_int32, _P, ctypes.c_int32, _P, ctypes.c_int64, _P,
                                        _P, _P, _P]
    L.matvis_simulate_pairs.restype = ctypes.c_int
    _lib = L
    return L


def _status_name(s: int) -> str:
    try:
        return load_library().matvis_status_string(int(s)).decode()
    except Exception:  # library unavailable: still give a readable message
        return f"status {s}"


@dataclasses.dataclass
class Config:
    """Mirror of matvis_config (include/matvis.h)."""
    n_ant: int
    n_feed: int = 1
    n_ax: int = 1
    n_beam: int = 1
    max_src: int = 1
    max_time: int = 1
    max_freq: int = 1
    latitude_rad: float = math.radians(-30.7)
    precision: str = "fp32"
    beam_mode: str = "bilinear"
    n_za: int = 91
    n_az: int = 360
    dza_rad: float = math.radians(1.0)
    daz_rad: float = math.radians(1.0)
    src_chunk: int = 0
    batch_time: int = 0
    batch_freq: int = 0
    use_graph: bool = True
    unfused: bool = False  # FP32 / BF16X3: separate Z-formation step (Z in device memory)
    ksplit: int = 0        # columns per product work item (multiple of 64); 0 = automatic
    polarised_sky: bool = False  # src_flux is [4][n_freq][n_src] (I, Q, U, V); needs n_ax = 2
    tile: int = 0          # product kernel variant (bits 0-3: forming split in 32-antenna units); 0 = automatic

    def _c(self) -> _Config:
        return _Config(self.n_ant, self.n_feed, self.n_ax, self.n_beam, self.max_src, self.max_time, self.max_freq,
                       self.latitude_rad, PRECISIONS[self.precision], BEAM_MODES[self.beam_mode], self.n_za,
                       self.n_az, self.dza_rad, self.daz_rad, self.src_chunk, self.batch_time, self.batch_freq,
                       (0 if self.use_graph else FLAG_NO_GRAPH) | (FLAG_UNFUSED if self.unfused else 0) |
                       (FLAG_POLARISED_SKY if self.polarised_sky else 0),
                       self.ksplit, self.tile)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


def _need(t, dtype, shape, name):
    import torch
    if t is None:
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Context:
    """A libmatvis context: device scratch for the capacities in ``cfg``."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        self._L = load_library()
        h = _P()
        st = self._L.matvis_init(ctypes.byref(cfg._c()), ctypes.byref(h))
        if st != OK:
            raise MatvisError(st, "matvis_init failed (details on stderr)")
        self._h = h

    @property
    def product_path(self) -> str:
        """Which product kernel this context runs (matvis_product_path_of)."""
        v = self._L.matvis_product_path_of(self._h)
        if v < 0:
            self._check(v)
        return PRODUCT_PATHS[v]

    @property
    def complex_dtype(self):
        import torch
        return torch.complex128 if self.cfg.precision == "fp64" else torch.complex64

    def _check(self, st: int):
        if st != OK:
            raise MatvisError(st, self._L.matvis_last_error(self._h).decode())

    def simulate(self, antpos, freqs, lsts, src_radec, src_flux, beam_grid, vis=None, beam_idx=None, stream=None):
        """Enqueue matvis_simulate; returns vis [t][f][a][b][p][q] (allocated if None)."""
        import torch
        c = self.cfg
        n_freq, n_time, n_src = freqs.shape[0], lsts.shape[0], src_radec.shape[1]
        _need(antpos, torch.float64, (c.n_ant, 3), "antpos")
        _need(freqs, torch.float64, (n_freq,), "freqs")
        _need(lsts, torch.float64, (n_time,), "lsts")
        _need(src_radec, torch.float64, (2, n_src), "src_radec")
        _need(src_flux, torch.float64, (4, n_freq, n_src) if c.polarised_sky else (n_freq, n_src), "src_flux")
        if c.beam_mode == "surrogate":
            beam_grid = None  # the learned beam replaces the grid
        else:
            _need(beam_grid, self.complex_dtype, (c.n_beam, n_freq, c.n_feed, c.n_ax, c.n_za, c.n_az), "beam_grid")
        if beam_idx is not None:
            _need(beam_idx, torch.int32, (c.n_ant,), "beam_idx")
        shape = (n_time, n_freq, c.n_ant, c.n_ant, c.n_feed, c.n_feed)
        if vis is None:
            vis = torch.empty(shape, dtype=self.complex_dtype, device=antpos.device)
        _need(vis, self.complex_dtype, shape, "vis")
        self._check(self._L.matvis_simulate(self._h, _ptr(antpos), _ptr(beam_idx), _ptr(freqs), n_freq, _ptr(lsts),
                                            n_time, _ptr(src_radec), n_src, _ptr(src_flux), _ptr(beam_grid),
                                            _ptr(vis), _stream_handle(stream)))
        return vis

    def finish(self):
        """Synchronise and report deferred device-side errors (MATVIS_EDATA)."""
        self._check(self._L.matvis_finish(self._h))

    def profile(self, enable: bool = True):
        """Time every step's launches with HIP events (launches go direct, not via the graph)."""
        self._check(self._L.matvis_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        """{step: (total device ms, launches)} since the last read."""
        ms = (ctypes.c_double * len(STEPS))()
        n = (ctypes.c_int64 * len(STEPS))()
        self._check(self._L.matvis_profile_read(self._h, ms, n))
        return {name: (ms[i], n[i]) for i, name in enumerate(STEPS)}

    def step_sky(self, lsts, src_radec, stream=None):
        """Alg. 2 step (i): (idx, count, s_hat, za_az) for every time."""
        import torch
        n_time, n_src = lsts.shape[0], src_radec.shape[1]
        _need(lsts, torch.float64, (n_time,), "lsts")
        _need(src_radec, torch.float64, (2, n_src), "src_radec")
        dev = lsts.device
        idx = torch.empty((n_time, n_src), dtype=torch.int32, device=dev)
        count = torch.empty((n_time,), dtype=torch.int32, device=dev)
        s_hat = torch.empty((n_time, 3, n_src), dtype=torch.float64, device=dev)
        za_az = torch.empty((n_time, 2, n_src), dtype=torch.float64, device=dev)
        self._check(self._L.matvis_step_sky(self._h, _ptr(lsts), n_time, _ptr(src_radec), n_src, _ptr(idx),
                                            _ptr(count), _ptr(s_hat), _ptr(za_az), _stream_handle(stream)))
        return idx, count, s_hat, za_az

    def step_interp(self, za_az, grid, stream=None):
        """Alg. 2 step (ii) alone: beam at points za_az [2][n] from one channel's grid."""
        import torch
        c = self.cfg
        n = za_az.shape[1]
        _need(za_az, torch.float64, (2, n), "za_az")
        _need(grid, self.complex_dtype, (c.n_beam, c.n_feed, c.n_ax, c.n_za, c.n_az), "grid")
        A = torch.empty((c.n_beam, c.n_feed, c.n_ax, n), dtype=self.complex_dtype, device=za_az.device)
        self._check(self._L.matvis_step_interp(self._h, _ptr(za_az), n, _ptr(grid), _ptr(A), _stream_handle(stream)))
        return A

    def step_herk(self, Z, stream=None):
        """Step (v) alone: V = Z Z^H for a [n_row][n_col] complex matrix."""
        import torch
        n_row, n_col = Z.shape
        _need(Z, self.complex_dtype, (n_row, n_col), "Z")
        V = torch.empty((n_row, n_row), dtype=self.complex_dtype, device=Z.device)
        self._check(self._L.matvis_step_herk(self._h, _ptr(Z), n_row, n_col, n_col, _ptr(V), _stream_handle(stream)))
        return V

    def set_pairs(self, pairs, n_sub: int = 3) -> int:
        """matvis_set_pairs: plan the sub-matrix product (App. A) for these (a, b) pairs;
        returns the total sub-matrix size in antenna pairs."""
        import numpy as np
        pa = np.ascontiguousarray([p[0] for p in pairs], dtype=np.int32)
        pb = np.ascontiguousarray([p[1] for p in pairs], dtype=np.int32)
        size = ctypes.c_int64()
        self._check(self._L.matvis_set_pairs(self._h, pa.ctypes.data, pb.ctypes.data, len(pa), int(n_sub),
                                             ctypes.byref(size)))
        self._n_pairs = len(pa)
        return int(size.value)

    def simulate_pairs(self, antpos, freqs, lsts, src_radec, src_flux, beam_grid, vis=None, beam_idx=None,
                       stream=None):
        """matvis_simulate_pairs: V of the planned pairs, [t][f][pair][p][q] (allocated if None)."""
        import torch
        c = self.cfg
        n_freq, n_time, n_src = freqs.shape[0], lsts.shape[0], src_radec.shape[1]
        _need(antpos, torch.float64, (c.n_ant, 3), "antpos")
        _need(freqs, torch.float64, (n_freq,), "freqs")
        _need(lsts, torch.float64, (n_time,), "lsts")
        _need(src_radec, torch.float64, (2, n_src), "src_radec")
        _need(src_flux, torch.float64, (4, n_freq, n_src) if c.polarised_sky else (n_freq, n_src), "src_flux")
        _need(beam_grid, self.complex_dtype, (c.n_beam, n_freq, c.n_feed, c.n_ax, c.n_za, c.n_az), "beam_grid")
        if beam_idx is not None:
            _need(beam_idx, torch.int32, (c.n_ant,), "beam_idx")
        shape = (n_time, n_freq, getattr(self, "_n_pairs", 0), c.n_feed, c.n_feed)
        if vis is None:
            vis = torch.empty(shape, dtype=self.complex_dtype, device=antpos.device)
        _need(vis, self.complex_dtype, shape, "vis")
        self._check(self._L.matvis_simulate_pairs(self._h, _ptr(antpos), _ptr(beam_idx), _ptr(freqs), n_freq,
                                                  _ptr(lsts), n_time, _ptr(src_radec), n_src, _ptr(src_flux),
                                                  _ptr(beam_grid), _ptr(vis), _stream_handle(stream)))
        return vis

    def set_surrogate(self, params, nu_min_hz: float, nu_max_hz: float):
        """matvis_set_surrogate: load the learned beams (copied; [MLP_N_PARAMS] for one beam or
        [n_beam][MLP_N_PARAMS], one network per unique beam) and their frequency range."""
        import torch
        nb = self.cfg.n_beam
        _need(params, torch.float32, (MLP_N_PARAMS,) if nb == 1 and params.dim() == 1 else (nb, MLP_N_PARAMS),
              "params")
        self._check(self._L.matvis_set_surrogate(self._h, _ptr(params), float(nu_min_hz), float(nu_max_hz)))

    def close(self):
        if getattr(self, "_h", None):
            self._L.matvis_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def autotune(cfg: Config, antpos, freqs, lsts, src_radec, src_flux, beam_grid, beam_idx=None, vis=None,
             cache_path: Optional[str] = None, stream=None, surrogate=None, nu_range=(100e6, 200e6)):
    """matvis_autotune: (tuned Config, ms per simulate call).  ``vis`` is scratch output;
    ``surrogate`` the learned beam's parameters when cfg.beam_mode is "surrogate"."""
    import torch
    L = load_library()
    n_freq, n_time, n_src = freqs.shape[0], lsts.shape[0], src_radec.shape[1]
    cdt = torch.complex128 if cfg.precision == "fp64" else torch.complex64
    if vis is None:
        vis = torch.empty((n_time, n_freq, cfg.n_ant, cfg.n_ant, cfg.n_feed, cfg.n_feed), dtype=cdt,
                          device=antpos.device)
    best = _Config()
    ms = ctypes.c_double()
    st = L.matvis_autotune(ctypes.byref(cfg._c()), _ptr(antpos), _ptr(beam_idx), _ptr(freqs), n_freq, _ptr(lsts),
                           n_time, _ptr(src_radec), n_src, _ptr(src_flux), _ptr(beam_grid), _ptr(vis),
                           _stream_handle(stream), cache_path.encode() if cache_path else None, ctypes.byref(best),
                           ctypes.byref(ms), _ptr(surrogate), float(nu_range[0]), float(nu_range[1]))
    if st != OK:
        raise MatvisError(st, "matvis_autotune failed")
    tuned = dataclasses.replace(cfg, ksplit=int(best.ksplit), batch_time=int(best.batch_time),
                                src_chunk=int(best.src_chunk), tile=int(best.tile),
                                unfused=bool(best.flags & FLAG_UNFUSED))
    return tuned, float(ms.value)


def redundant_groups(antpos, beam_idx=None, tol_m: float = 1e-3):
    """matvis_redundant_groups (host): (group of every pair (i <= j, lexicographic), representative pairs)."""
    import numpy as np
    x = np.ascontiguousarray(antpos, dtype=np.float64)
    n = x.shape[0]
    npairs = n * (n + 1) // 2
    bi = None if beam_idx is None else np.ascontiguousarray(beam_idx, dtype=np.int32)
    group = np.empty(npairs, dtype=np.int32)
    ra = np.empty(npairs, dtype=np.int32)
    rb = np.empty(npairs, dtype=np.int32)
    nu = ctypes.c_int32()
    _check_lib(load_library().matvis_redundant_groups(x.ctypes.data, None if bi is None else bi.ctypes.data, n,
                                                      float(tol_m), group.ctypes.data, ra.ctypes.data, rb.ctypes.data,
                                                      ctypes.byref(nu)), "matvis_redundant_groups")
    return group, list(zip(ra[:nu.value].tolist(), rb[:nu.value].tolist()))


def submatrix_plan(pairs, n_ant: int, n_sub: int):
    """matvis_submatrix_plan (host): (alpha order, sub-matrix sizes, densities)."""
    import numpy as np
    pa = np.ascontiguousarray([p[0] for p in pairs], dtype=np.int32)
    pb = np.ascontiguousarray([p[1] for p in pairs], dtype=np.int32)
    alpha = np.empty(n_ant, dtype=np.int32)
    sizes = np.empty(max(1, n_sub), dtype=np.int32)
    dens = np.empty(max(1, n_sub), dtype=np.float64)
    na, ns = ctypes.c_int32(), ctypes.c_int32()
    _check_lib(load_library().matvis_submatrix_plan(pa.ctypes.data, pb.ctypes.data, len(pa), int(n_ant), int(n_sub),
                                                    alpha.ctypes.data, sizes.ctypes.data, dens.ctypes.data,
                                                    ctypes.byref(na), ctypes.byref(ns)), "matvis_submatrix_plan")
    return alpha[:na.value].tolist(), sizes[:ns.value].tolist(), dens[:ns.value].tolist()


def _check_lib(st: int, what: str):
    if st != OK:
        raise MatvisError(st, f"{what} failed (details on stderr)")


def mlp_forward(params, x, stream=None):
    """matvis_mlp_forward: learned-beam outputs [n][8] for inputs x [n][3] (synchronous)."""
    import torch
    n = x.shape[0]
    _need(params, torch.float32, (MLP_N_PARAMS,), "params")
    _need(x, torch.float32, (n, 3), "x")
    out = torch.empty((n, 8), dtype=torch.float32, device=x.device)
    _check_lib(load_library().matvis_mlp_forward(_ptr(params), _ptr(x), n, _ptr(out), _stream_handle(stream)),
               "matvis_mlp_forward")
    return out


def mlp_loss_grad(params, x, y, fp32_math: bool = False, stream=None):
    """matvis_mlp_loss_grad: (grad [MLP_N_PARAMS], loss [1]) of the mean squared error (synchronous)."""
    import torch
    n = x.shape[0]
    _need(params, torch.float32, (MLP_N_PARAMS,), "params")
    _need(x, torch.float32, (n, 3), "x")
    _need(y, torch.float32, (n, 8), "y")
    grad = torch.empty_like(params)
    loss = torch.empty((1,), dtype=torch.float32, device=x.device)
    _check_lib(load_library().matvis_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(y), n, 1 if fp32_math else 0,
                                                   _ptr(grad), _ptr(loss), _stream_handle(stream)),
               "matvis_mlp_loss_grad")
    return grad, loss


def mlp_loss_grad_noalloc(params, x, y, grad, loss, fp32_math: bool = False, stream=None):
    """matvis_mlp_loss_grad_noalloc: the same loss and gradient written into the caller's
    grad [MLP_N_PARAMS] and loss [1], with no device allocation (n <= 4096 rows;
    asynchronous on the stream)."""
    import torch
    n = x.shape[0]
    _need(params, torch.float32, (MLP_N_PARAMS,), "params")
    _need(x, torch.float32, (n, 3), "x")
    _need(y, torch.float32, (n, 8), "y")
    _need(grad, torch.float32, (MLP_N_PARAMS,), "grad")
    _need(loss, torch.float32, (1,), "loss")
    _check_lib(load_library().matvis_mlp_loss_grad_noalloc(_ptr(params), _ptr(x), _ptr(y), n, 1 if fp32_math else 0,
                                                           _ptr(grad), _ptr(loss), _stream_handle(stream)),
               "matvis_mlp_loss_grad_noalloc")


def mlp_adam(params, grad, m1, m2, step: int, lr: float, stream=None):
    """matvis_mlp_adam: one Adam step on params (in place)."""
    import torch
    for t, name in ((params, "params"), (grad, "grad"), (m1, "m1"), (m2, "m2")):
        _need(t, torch.float32, (MLP_N_PARAMS,), name)
    _check_lib(load_library().matvis_mlp_adam(_ptr(params), _ptr(grad), _ptr(m1), _ptr(m2), int(step), float(lr),
                                              _stream_handle(stream)), "matvis_mlp_adam")


def beam_samples(grid, dza_rad: float, daz_rad: float, za, az, chan, bicubic: bool = True, chan_freq=None,
                 nu_range=None, stream=None):
    """matvis_beam_samples: targets y [n][8] (and inputs x [n][3] when chan_freq and nu_range are given).

    grid is complex64 [n_chan][n_feed][n_ax][n_za][n_az]; za, az float64 [n]; chan int32 [n].
    """
    import torch
    n_chan, n_feed, n_ax, n_za, n_az = grid.shape
    n = za.shape[0]
    _need(grid, torch.complex64, grid.shape, "grid")
    _need(za, torch.float64, (n,), "za")
    _need(az, torch.float64, (n,), "az")
    _need(chan, torch.int32, (n,), "chan")
    y = torch.empty((n, 8), dtype=torch.float32, device=za.device)
    x = None
    nu0 = nu1 = 0.0
    if chan_freq is not None:
        _need(chan_freq, torch.float64, (n_chan,), "chan_freq")
        nu0, nu1 = (float(v) for v in nu_range)
        x = torch.empty((n, 3), dtype=torch.float32, device=za.device)
    _check_lib(load_library().matvis_beam_samples(_ptr(grid), n_chan, n_feed, n_ax, n_za, n_az, float(dza_rad),
                                                  float(daz_rad), 1 if bicubic else 0, _ptr(za), _ptr(az),
                                                  _ptr(chan), n, _ptr(y), _ptr(chan_freq), nu0, nu1, _ptr(x),
                                                  _stream_handle(stream)), "matvis_beam_samples")
    return y, x


def train_surrogate(params, x, y, batch: int = 4096, epochs: int = 10, lr0: float = 2e-3, lr1: float = 1e-4,
                    seed: int = 0, fp32_math: bool = False, stream=None):
    """matvis_train_surrogate: train params in place; returns the per-epoch mean loss (numpy, float32)."""
    import numpy as np
    import torch
    n = x.shape[0]
    _need(params, torch.float32, (MLP_N_PARAMS,), "params")
    _need(x, torch.float32, (n, 3), "x")
    _need(y, torch.float32, (n, 8), "y")
    hist = np.zeros(epochs, dtype=np.float32)
    _check_lib(load_library().matvis_train_surrogate(_ptr(params), _ptr(x), _ptr(y), n, int(batch), int(epochs),
                                                     float(lr0), float(lr1), int(seed), 1 if fp32_math else 0,
                                                     hist.ctypes.data, _stream_handle(stream)),
               "matvis_train_surrogate")
    return hist


def config_for(wl, precision: str = "fp32", **kw) -> Config:
    """Context configuration sized for a synthetic workload (paper_2312_09763_amd.synth.Workload)."""
    n_za, n_az = wl.beam.shape[-2], wl.beam.shape[-1]
    args = dict(n_ant=wl.n_ant, n_feed=wl.n_feed, n_ax=wl.n_ax, n_beam=wl.beam.shape[0], max_src=max(wl.n_src, 1),
                max_time=wl.n_time, max_freq=wl.n_freq, latitude_rad=wl.latitude, precision=precision,
                beam_mode=wl.interp, n_za=n_za, n_az=n_az, dza_rad=wl.dza, daz_rad=wl.daz)
    args.update(kw)
    return Config(**args)


def device_inputs(wl, precision: str = "fp32", device: str = "cuda", stokes=None):
    """Move a synthetic workload's arrays to the device in the ABI's dtypes
    (src_flux = stokes [4][n_freq][n_src] for a polarised sky when given)."""
    import numpy as np
    import torch
    cd = np.complex128 if precision == "fp64" else np.complex64
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
    return dict(antpos=t(wl.antpos, np.float64), freqs=t(wl.freqs, np.float64), lsts=t(wl.lsts, np.float64),
                src_radec=t(wl.radec, np.float64), src_flux=t(wl.flux if stokes is None else stokes, np.float64),
                beam_grid=t(wl.beam, cd))
