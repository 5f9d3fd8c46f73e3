"""Thin Python binding of the C ABI in include/rw.h (librw.so, gfx950).

Argument marshalling only: every step of the walk, the adjoint, the reductions
and the finalisation runs in the library's HIP kernels.  PyTorch provides
device memory (tensors) and the current HIP stream.  The functions keep the C
names (rw_forward, rw_batch_forward, rw_adjoint, rw_batch_adjoint,
rw_finalize, rw_check, rw_debug_trace, rw_debug_philox).

Importing this module does not load the library; the first call does, and it
raises if librw.so is missing (build it with ``python -m
paper_2606_27604_amd.build``).  There is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librw.so")

RW_OK, RW_E_INVALID, RW_E_HIP, RW_E_NOMEM, RW_E_UNSUPPORTED, RW_E_DEVICE_FLAG = range(6)
RW_FLAG_BAD_PARAMS = 1
RW_FLAG_VERTEX_CAP = 2
RW_FLAG_WEIGHT_CAP = 4


class RwError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_status_name(status)}: {message}")
        self.status = status


class RwGeometryC(ctypes.Structure):
    _fields_ = [
        ("n_media", ctypes.c_int32),
        ("n_bins", ctypes.c_int32),
        ("n_rel", ctypes.c_float),
        ("slab_mm", ctypes.c_float),
        ("r_min_mm", ctypes.c_float),
        ("r_max_mm", ctypes.c_float),
        ("rr_weight", ctypes.c_float),
        ("rr_survive", ctypes.c_float),
        ("max_vertices", ctypes.c_int64),
        ("incidence", ctypes.c_int32),
    ]


class RwMediaC(ctypes.Structure):
    _fields_ = [
        ("sigma_t", ctypes.c_void_p),
        ("albedo", ctypes.c_void_p),
        ("g", ctypes.c_void_p),
        ("weight", ctypes.c_void_p),
        ("weights_are_logits", ctypes.c_int32),
        ("n_sets", ctypes.c_int64),
        ("n_wl", ctypes.c_int64),
        ("wavelength_nm", ctypes.c_void_p),
        ("k_stride", ctypes.c_int64),
        ("unit_base", ctypes.c_int64),
    ]


class RwLayersC(ctypes.Structure):
    _fields_ = [
        ("sigma_t", ctypes.c_void_p),
        ("albedo", ctypes.c_void_p),
        ("g", ctypes.c_void_p),
        ("thickness_mm", ctypes.c_void_p),
        ("n_rel_bottom", ctypes.c_float),
        ("n_units", ctypes.c_int64),
        ("k_stride", ctypes.c_int64),
        ("unit_base", ctypes.c_int64),
    ]


class RwLutC(ctypes.Structure):
    _fields_ = [
        ("R", ctypes.c_void_p),
        ("Pd", ctypes.c_void_p),
        ("n_alpha", ctypes.c_int32),
        ("n_g", ctypes.c_int32),
        ("n_bins", ctypes.c_int32),
        ("alpha_max", ctypes.c_float),
        ("g_max", ctypes.c_float),
        ("r_min_mm", ctypes.c_float),
        ("r_max_mm", ctypes.c_float),
    ]


class RwLutTargetsC(ctypes.Structure):
    _fields_ = [
        ("R", ctypes.c_void_p),
        ("Pd", ctypes.c_void_p),
        ("mass", ctypes.c_void_p),
        ("r_mm", ctypes.c_void_p),
        ("n_r", ctypes.c_int32),
        ("lambda_R", ctypes.c_float),
        ("min_mass", ctypes.c_float),
        ("shape_floor", ctypes.c_float),
        ("shape_form", ctypes.c_int32),
    ]


class RwTallyC(ctypes.Structure):
    _fields_ = [
        ("R", ctypes.c_void_p),
        ("bins", ctypes.c_void_p),
        ("vertices", ctypes.c_void_p),
        ("flags", ctypes.c_void_p),
    ]


class RwBatchOptsC(ctypes.Structure):
    _fields_ = [
        ("use_graph", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("unit_begin", ctypes.c_int64),
        ("unit_end", ctypes.c_int64),
        ("path_mask", ctypes.c_void_p),
    ]


RW_LUT_SHAPE_PAPER, RW_LUT_SHAPE_MIXTURE = 0, 1

EXPORTS = [
    "rw_create", "rw_destroy", "rw_last_error", "rw_status_string", "rw_forward",
    "rw_batch_forward", "rw_adjoint", "rw_batch_adjoint", "rw_finalize", "rw_check",
    "rw_debug_trace", "rw_debug_philox", "rw_version", "rw_layered_forward",
    "rw_layered_adjoint", "rw_debug_trace_layered", "rw_lut_loss_grad", "rw_lut_fit_step",
    "rw_forward_noalloc", "rw_layered_hero_forward", "rw_dwivedi_forward",
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load librw.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library with `python -m paper_2606_27604_amd.build`")
    L = ctypes.CDLL(path)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    P = ctypes.POINTER
    L.rw_create.argtypes = [P(vp), ctypes.c_int]
    L.rw_create.restype = ctypes.c_int
    L.rw_destroy.argtypes = [vp]
    L.rw_destroy.restype = ctypes.c_int
    L.rw_last_error.argtypes = [vp]
    L.rw_last_error.restype = ctypes.c_char_p
    L.rw_status_string.argtypes = [ctypes.c_int]
    L.rw_status_string.restype = ctypes.c_char_p
    L.rw_version.argtypes = []
    L.rw_version.restype = ctypes.c_char_p
    L.rw_forward.argtypes = [vp, P(RwMediaC), P(RwGeometryC), i64, u64, P(RwTallyC), vp]
    L.rw_forward.restype = ctypes.c_int
    L.rw_forward_noalloc.argtypes = [vp, P(RwMediaC), P(RwGeometryC), i64, u64, P(RwTallyC), vp]
    L.rw_forward_noalloc.restype = ctypes.c_int
    L.rw_layered_hero_forward.argtypes = [vp, P(RwLayersC), P(RwGeometryC), i32, i64, u64,
                                          P(RwTallyC), vp]
    L.rw_layered_hero_forward.restype = ctypes.c_int
    L.rw_dwivedi_forward.argtypes = [vp, P(RwMediaC), P(RwGeometryC), i64, u64, ctypes.c_float,
                                     P(RwTallyC), vp]
    L.rw_dwivedi_forward.restype = ctypes.c_int
    L.rw_batch_forward.argtypes = [vp, P(RwMediaC), P(RwGeometryC), vp, i64, u64, P(RwTallyC),
                                   P(RwBatchOptsC), vp]
    L.rw_batch_forward.restype = ctypes.c_int
    L.rw_adjoint.argtypes = [vp, P(RwMediaC), P(RwGeometryC), i64, u64, vp, vp, vp, vp, vp, vp, vp]
    L.rw_adjoint.restype = ctypes.c_int
    L.rw_batch_adjoint.argtypes = [vp, P(RwMediaC), P(RwGeometryC), vp, i64, u64, vp, vp, vp, vp,
                                   vp, vp, P(RwBatchOptsC), vp]
    L.rw_batch_adjoint.restype = ctypes.c_int
    L.rw_finalize.argtypes = [vp, P(RwGeometryC), i64, vp, i64, P(RwTallyC), vp, vp, vp, vp, vp, vp]
    L.rw_finalize.restype = ctypes.c_int
    L.rw_check.argtypes = [vp, vp, P(i32), vp]
    L.rw_check.restype = ctypes.c_int
    L.rw_debug_trace.argtypes = [vp, P(RwMediaC), P(RwGeometryC), vp, i64, i64, u64,
                                 ctypes.c_uint32, vp, vp, vp, vp]
    L.rw_debug_trace.restype = ctypes.c_int
    L.rw_debug_philox.argtypes = [vp, vp, u64, i64, vp, vp]
    L.rw_debug_philox.restype = ctypes.c_int
    L.rw_layered_forward.argtypes = [vp, P(RwLayersC), P(RwGeometryC), vp, i64, u64, P(RwTallyC),
                                     P(RwBatchOptsC), vp]
    L.rw_layered_forward.restype = ctypes.c_int
    L.rw_layered_adjoint.argtypes = [vp, P(RwLayersC), P(RwGeometryC), vp, i64, u64, vp, vp, vp,
                                     vp, vp, vp, P(RwBatchOptsC), vp]
    L.rw_layered_adjoint.restype = ctypes.c_int
    L.rw_debug_trace_layered.argtypes = [vp, P(RwLayersC), P(RwGeometryC), vp, i64, i64, u64,
                                         ctypes.c_uint32, vp, vp, vp]
    L.rw_debug_trace_layered.restype = ctypes.c_int
    L.rw_lut_loss_grad.argtypes = [vp, P(RwLutC), P(RwLutTargetsC), i64, i32, vp, vp, vp, vp]
    L.rw_lut_loss_grad.restype = ctypes.c_int
    L.rw_lut_fit_step.argtypes = [vp, P(RwLutC), P(RwLutTargetsC), i64, i32, vp, vp, vp, i32,
                                  ctypes.c_float, vp, vp]
    L.rw_lut_fit_step.restype = ctypes.c_int
    _lib = L
    return L


def _status_name(st: int) -> str:
    try:
        return load_library().rw_status_string(st).decode()
    except ImportError:
        return f"status {st}"


@dataclass
class Geometry:
    """rw_geometry: radial set-up of 256 log bins over [1e-3, 50] mm, roulette
    1e-4 / 0.1, semi-infinite unless slab_mm > 0."""

    n_media: int = 3
    n_rel: float = 1.4
    slab_mm: float = 0.0
    n_bins: int = 256
    r_min_mm: float = 1e-3
    r_max_mm: float = 50.0
    rr_weight: float = 1e-4
    rr_survive: float = 0.1
    max_vertices: int = 1 << 20
    incidence: int = 0  # 0: normal pencil beam; 1: cosine-weighted lobe

    def c(self) -> RwGeometryC:
        return RwGeometryC(self.n_media, self.n_bins, self.n_rel, self.slab_mm, self.r_min_mm,
                           self.r_max_mm, self.rr_weight, self.rr_survive, self.max_vertices,
                           self.incidence)


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _need(t, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


class Media:
    """Device-resident media parameters, SoA float32 [K, n_units] (unit = set * n_wl + wl)."""

    def __init__(self, sigma_t, albedo, g, weight, n_sets: int, n_wl: int = 1,
                 weights_are_logits: bool = False, wavelength_nm=None, k_stride: int = 0,
                 unit_base: int = 0):
        K = sigma_t.shape[0]
        n = n_sets * n_wl
        cols = k_stride if k_stride else n
        for name, t in (("sigma_t", sigma_t), ("albedo", albedo), ("g", g), ("weight", weight)):
            _need(t, torch.float32, name=name)
            if t.dim() != 2 or t.shape[0] != K or t.shape[1] != cols:
                if not k_stride:
                    raise ValueError(f"{name} must have shape [{K}, {n}]")
        self.sigma_t, self.albedo, self.g, self.weight = sigma_t, albedo, g, weight
        self.K, self.n_sets, self.n_wl = K, n_sets, n_wl
        self.logits = weights_are_logits
        self.wavelength_nm = wavelength_nm
        self.k_stride = k_stride
        self.unit_base = unit_base
        self._c = RwMediaC(_ptr(sigma_t), _ptr(albedo), _ptr(g), _ptr(weight),
                           int(weights_are_logits), n_sets, n_wl, _ptr(wavelength_nm), k_stride,
                           unit_base)

    @property
    def n_units(self) -> int:
        return self.n_sets * self.n_wl

    @classmethod
    def from_numpy(cls, sigma_t, albedo, g, weight, n_sets, n_wl=1, device="cuda",
                   weights_are_logits=False):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).contiguous().to(device)  # noqa: E731
        return cls(f(sigma_t), f(albedo), f(g), f(weight), n_sets, n_wl, weights_are_logits)

    def unit_range(self, begin: int, count: int) -> "Media":
        """A view on units [begin, begin + count) of the same SoA arrays (n_sets = count).
        Its units keep their random-number index (unit_base), so a call on the view
        draws the same random numbers for them as a call on the whole set."""
        stride = self.k_stride or self.n_units
        sub = object.__new__(Media)
        sub.sigma_t, sub.albedo, sub.g, sub.weight = self.sigma_t, self.albedo, self.g, self.weight
        sub.K, sub.n_sets, sub.n_wl = self.K, count, 1
        sub.logits, sub.wavelength_nm, sub.k_stride = self.logits, None, stride
        sub.unit_base = self.unit_base + begin
        es = 4  # float32
        sub._c = RwMediaC(self.sigma_t.data_ptr() + begin * es, self.albedo.data_ptr() + begin * es,
                          self.g.data_ptr() + begin * es, self.weight.data_ptr() + begin * es,
                          int(self.logits), count, 1, None, stride, sub.unit_base)
        return sub


class Layers:
    """Device-resident two-layer tissue (rw_layers): sigma_t, albedo, g float32
    [2, n_units] (row 0 top layer, row 1 bottom layer), thickness float32
    [n_units] (top-layer thickness, mm); n_rel_bottom is the bottom layer's
    index over the outside (the top layer's is Geometry.n_rel)."""

    def __init__(self, sigma_t, albedo, g, thickness_mm, n_rel_bottom: float = 1.4,
                 unit_base: int = 0):
        n = sigma_t.shape[1]
        for name, t in (("sigma_t", sigma_t), ("albedo", albedo), ("g", g)):
            _need(t, torch.float32, (2, n), name)
        _need(thickness_mm, torch.float32, (n,), "thickness_mm")
        self.sigma_t, self.albedo, self.g, self.thickness_mm = sigma_t, albedo, g, thickness_mm
        self.n_rel_bottom = float(n_rel_bottom)
        self.n_units = n
        self.unit_base = unit_base
        self._c = RwLayersC(_ptr(sigma_t), _ptr(albedo), _ptr(g), _ptr(thickness_mm),
                            self.n_rel_bottom, n, n, unit_base)

    @classmethod
    def from_numpy(cls, sigma_t, albedo, g, thickness_mm, n_rel_bottom=1.4, device="cuda"):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).contiguous().to(device)  # noqa: E731
        return cls(f(sigma_t), f(albedo), f(g), f(thickness_mm), n_rel_bottom)


class Tally:
    """Raw FP64 forward sums on the device (layout of rw_tally)."""

    def __init__(self, n_units: int, n_bins: int, device="cuda"):
        self.R = torch.zeros((n_units, 4), dtype=torch.float64, device=device)
        self.bins = torch.zeros((n_units, n_bins + 2, 2), dtype=torch.float64, device=device)
        self.vertices = torch.zeros(n_units, dtype=torch.int64, device=device)
        self.flags = torch.zeros(1, dtype=torch.int32, device=device)
        self._c = RwTallyC(_ptr(self.R), _ptr(self.bins), _ptr(self.vertices), _ptr(self.flags))

    def view(self, begin: int, count: int) -> "Tally":
        """A tally struct addressing units [begin, begin + count) of this one."""
        sub = object.__new__(Tally)
        sub.R, sub.bins = self.R[begin:begin + count], self.bins[begin:begin + count]
        sub.vertices, sub.flags = self.vertices[begin:begin + count], self.flags
        sub._c = RwTallyC(_ptr(sub.R), _ptr(sub.bins), _ptr(sub.vertices), _ptr(sub.flags))
        return sub


class Context:
    """rw_context on one HIP device (device=-1: validation-only, no GPU)."""

    def __init__(self, device: int = 0):
        L = load_library()
        h = ctypes.c_void_p()
        st = L.rw_create(ctypes.byref(h), device)
        if st != RW_OK:
            raise RwError(st, f"rw_create(device={device}) failed")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            load_library().rw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return load_library().rw_last_error(self.h).decode()

    def _check(self, st: int):
        if st != RW_OK:
            raise RwError(st, self.last_error())


def _opts(use_graph=True, autotune=False, unit_begin=0, unit_end=0, path_mask=None):
    return RwBatchOptsC(int(use_graph), int(autotune), unit_begin, unit_end, _ptr(path_mask))


def mask_words(paths_uniform: int) -> int:
    """Words per unit of a live-path mask (rw_batch_opts.path_mask)."""
    return (int(paths_uniform) + 31) // 32


def new_path_mask(n_units: int, paths_uniform: int, device="cuda") -> torch.Tensor:
    """An int32 tensor [n_units, ceil(paths / 32)] to hold a live-path mask."""
    return torch.empty((n_units, mask_words(paths_uniform)), dtype=torch.int32, device=device)


def _check_mask(mask, n_units, paths_uniform):
    if mask is not None:
        _need(mask, torch.int32, (n_units, mask_words(paths_uniform)), "path_mask")


# ---------------------------------------------------------------------------
# entry points, same names as the C ABI
# ---------------------------------------------------------------------------
def rw_forward(ctx: Context, media: Media, geom: Geometry, paths_per_unit: int, seed: int,
               out: Tally, stream=None):
    g = geom.c()
    ctx._check(load_library().rw_forward(ctx.h, ctypes.byref(media._c), ctypes.byref(g),
                                         int(paths_per_unit), int(seed), ctypes.byref(out._c),
                                         _stream(stream)))


def rw_forward_noalloc(ctx: Context, media: Media, geom: Geometry, paths_per_unit: int, seed: int,
                       out: Tally, stream=None):
    g = geom.c()
    ctx._check(load_library().rw_forward_noalloc(ctx.h, ctypes.byref(media._c), ctypes.byref(g),
                                                 int(paths_per_unit), int(seed),
                                                 ctypes.byref(out._c), _stream(stream)))


def rw_batch_forward(ctx: Context, media: Media, geom: Geometry, paths_per_unit, paths_uniform: int,
                     seed: int, out: Tally, use_graph=True, autotune=False, unit_begin=0,
                     unit_end=0, stream=None, path_mask=None):
    if paths_per_unit is not None:
        _need(paths_per_unit, torch.int32, (media.n_units,), "paths_per_unit")
    _check_mask(path_mask, media.n_units, paths_uniform)
    g = geom.c()
    o = _opts(use_graph, autotune, unit_begin, unit_end, path_mask)
    ctx._check(load_library().rw_batch_forward(ctx.h, ctypes.byref(media._c), ctypes.byref(g),
                                               _ptr(paths_per_unit), int(paths_uniform), int(seed),
                                               ctypes.byref(out._c), ctypes.byref(o),
                                               _stream(stream)))


def _adj_args(media, geom, cot_R, cot_bins, grad, grad_sumsq, vertices, flags):
    n, P = media.n_units, 4 * geom.n_media
    if cot_R is not None:
        _need(cot_R, torch.float32, (n,), "cot_R")
    if cot_bins is not None:
        _need(cot_bins, torch.float32, (n, geom.n_bins + 2), "cot_bins")
    _need(grad, torch.float64, (n, P), "grad")
    if grad_sumsq is not None:
        _need(grad_sumsq, torch.float64, (n, P), "grad_sumsq")
    if vertices is not None:
        _need(vertices, torch.int64, (n,), "vertices")
    _need(flags, torch.int32, (1,), "flags")


def rw_adjoint(ctx: Context, media: Media, geom: Geometry, paths_per_unit: int, seed: int, cot_R,
               cot_bins, grad, grad_sumsq, vertices, flags, stream=None):
    _adj_args(media, geom, cot_R, cot_bins, grad, grad_sumsq, vertices, flags)
    g = geom.c()
    ctx._check(load_library().rw_adjoint(ctx.h, ctypes.byref(media._c), ctypes.byref(g),
                                         int(paths_per_unit), int(seed), _ptr(cot_R),
                                         _ptr(cot_bins), _ptr(grad), _ptr(grad_sumsq),
                                         _ptr(vertices), _ptr(flags), _stream(stream)))


def rw_batch_adjoint(ctx: Context, media: Media, geom: Geometry, paths_per_unit, paths_uniform: int,
                     seed: int, cot_R, cot_bins, grad, grad_sumsq, vertices, flags, use_graph=True,
                     autotune=False, unit_begin=0, unit_end=0, stream=None, path_mask=None):
    _adj_args(media, geom, cot_R, cot_bins, grad, grad_sumsq, vertices, flags)
    if paths_per_unit is not None:
        _need(paths_per_unit, torch.int32, (media.n_units,), "paths_per_unit")
    _check_mask(path_mask, media.n_units, paths_uniform)
    g = geom.c()
    o = _opts(use_graph, autotune, unit_begin, unit_end, path_mask)
    ctx._check(load_library().rw_batch_adjoint(
        ctx.h, ctypes.byref(media._c), ctypes.byref(g), _ptr(paths_per_unit), int(paths_uniform),
        int(seed), _ptr(cot_R), _ptr(cot_bins), _ptr(grad), _ptr(grad_sumsq), _ptr(vertices),
        _ptr(flags), ctypes.byref(o), _stream(stream)))


def rw_finalize(ctx: Context, geom: Geometry, n_units: int, paths_per_unit, paths_uniform: int,
                tally: Tally, R_mean=None, R_se=None, Rr=None, Rr_se=None, Pd=None, stream=None):
    g = geom.c()
    ctx._check(load_library().rw_finalize(ctx.h, ctypes.byref(g), int(n_units),
                                          _ptr(paths_per_unit), int(paths_uniform),
                                          ctypes.byref(tally._c), _ptr(R_mean), _ptr(R_se),
                                          _ptr(Rr), _ptr(Rr_se), _ptr(Pd), _stream(stream)))


def rw_check(ctx: Context, flags, stream=None) -> int:
    out = ctypes.c_int32(0)
    st = load_library().rw_check(ctx.h, _ptr(flags), ctypes.byref(out), _stream(stream))
    if st not in (RW_OK, RW_E_DEVICE_FLAG):
        ctx._check(st)
    return out.value


def rw_debug_trace(ctx: Context, media: Media, geom: Geometry, words, n_paths: int, n_blocks: int,
                   seed: int, unit_index: int, events, path_out, path_adj, stream=None):
    g = geom.c()
    ctx._check(load_library().rw_debug_trace(ctx.h, ctypes.byref(media._c), ctypes.byref(g),
                                             _ptr(words), int(n_paths), int(n_blocks), int(seed),
                                             int(unit_index), _ptr(events), _ptr(path_out),
                                             _ptr(path_adj), _stream(stream)))


def rw_layered_forward(ctx: Context, layers: Layers, geom: Geometry, paths_per_unit,
                       paths_uniform: int, seed: int, out: Tally, use_graph=True, autotune=False,
                       unit_begin=0, unit_end=0, stream=None, path_mask=None):
    if paths_per_unit is not None:
        _need(paths_per_unit, torch.int32, (layers.n_units,), "paths_per_unit")
    _check_mask(path_mask, layers.n_units, paths_uniform)
    g = geom.c()
    o = _opts(use_graph, autotune, unit_begin, unit_end, path_mask)
    ctx._check(load_library().rw_layered_forward(ctx.h, ctypes.byref(layers._c), ctypes.byref(g),
                                                 _ptr(paths_per_unit), int(paths_uniform),
                                                 int(seed), ctypes.byref(out._c),
                                                 ctypes.byref(o), _stream(stream)))


def rw_layered_adjoint(ctx: Context, layers: Layers, geom: Geometry, paths_per_unit,
                       paths_uniform: int, seed: int, cot_R, cot_bins, grad, grad_sumsq, vertices,
                       flags, use_graph=True, autotune=False, unit_begin=0, unit_end=0,
                       stream=None, path_mask=None):
    _adj_args(layers, geom, cot_R, cot_bins, grad, grad_sumsq, vertices, flags)
    if paths_per_unit is not None:
        _need(paths_per_unit, torch.int32, (layers.n_units,), "paths_per_unit")
    _check_mask(path_mask, layers.n_units, paths_uniform)
    g = geom.c()
    o = _opts(use_graph, autotune, unit_begin, unit_end, path_mask)
    ctx._check(load_library().rw_layered_adjoint(
        ctx.h, ctypes.byref(layers._c), ctypes.byref(g), _ptr(paths_per_unit), int(paths_uniform),
        int(seed), _ptr(cot_R), _ptr(cot_bins), _ptr(grad), _ptr(grad_sumsq), _ptr(vertices),
        _ptr(flags), ctypes.byref(o), _stream(stream)))


def rw_layered_hero_forward(ctx: Context, layers: Layers, geom: Geometry, n_hero: int,
                            paths_per_group: int, seed: int, out: Tally, stream=None):
    g = geom.c()
    ctx._check(load_library().rw_layered_hero_forward(ctx.h, ctypes.byref(layers._c),
                                                      ctypes.byref(g), int(n_hero),
                                                      int(paths_per_group), int(seed),
                                                      ctypes.byref(out._c), _stream(stream)))


def rw_dwivedi_forward(ctx: Context, media: Media, geom: Geometry, paths_per_unit: int, seed: int,
                       q: float, out: Tally, stream=None):
    g = geom.c()
    ctx._check(load_library().rw_dwivedi_forward(ctx.h, ctypes.byref(media._c), ctypes.byref(g),
                                                 int(paths_per_unit), int(seed), float(q),
                                                 ctypes.byref(out._c), _stream(stream)))


def rw_debug_trace_layered(ctx: Context, layers: Layers, geom: Geometry, words, n_paths: int,
                           n_blocks: int, seed: int, unit_index: int, events, path_out,
                           stream=None):
    g = geom.c()
    ctx._check(load_library().rw_debug_trace_layered(ctx.h, ctypes.byref(layers._c),
                                                     ctypes.byref(g), _ptr(words), int(n_paths),
                                                     int(n_blocks), int(seed), int(unit_index),
                                                     _ptr(events), _ptr(path_out),
                                                     _stream(stream)))


def rw_lut_loss_grad(ctx: Context, lut: RwLutC, targets: RwLutTargetsC, n_units: int,
                     n_media: int, params, grad=None, loss=None, stream=None):
    P = 4 * n_media - 1
    _need(params, torch.float32, (P, n_units), "params")
    if grad is not None:
        _need(grad, torch.float32, (P, n_units), "grad")
    if loss is not None:
        _need(loss, torch.float32, (n_units,), "loss")
    ctx._check(load_library().rw_lut_loss_grad(ctx.h, ctypes.byref(lut), ctypes.byref(targets),
                                               int(n_units), int(n_media), _ptr(params),
                                               _ptr(grad), _ptr(loss), _stream(stream)))


def rw_lut_fit_step(ctx: Context, lut: RwLutC, targets: RwLutTargetsC, n_units: int,
                    n_media: int, params, adam_m, adam_v, step: int, lr: float, loss=None,
                    stream=None):
    P = 4 * n_media - 1
    for name, t in (("params", params), ("adam_m", adam_m), ("adam_v", adam_v)):
        _need(t, torch.float32, (P, n_units), name)
    if loss is not None:
        _need(loss, torch.float32, (n_units,), "loss")
    ctx._check(load_library().rw_lut_fit_step(ctx.h, ctypes.byref(lut), ctypes.byref(targets),
                                              int(n_units), int(n_media), _ptr(params),
                                              _ptr(adam_m), _ptr(adam_v), int(step), float(lr),
                                              _ptr(loss), _stream(stream)))


def rw_debug_philox(ctx: Context, ctr, key: int, out, stream=None):
    n = ctr.shape[0]
    ctx._check(load_library().rw_debug_philox(ctx.h, _ptr(ctr), int(key), int(n), _ptr(out),
                                              _stream(stream)))
