"""ctypes wrapper of the FP64 CPU oracle (``rw_oracle.c``).

TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never imports this module
and this module never imports the product package.

The oracle evaluates the random walk of the paper's mixture-of-media model
(Sec. 4.1, second form of eq. sss: per-path medium choice by weight, then a
homogeneous walk) in FP64, following the estimator conventions listed at the
top of ``rw_oracle.c``; and the same estimator in the two-layer tissue of the
paper's data generator (Sec. 3: a top layer of given thickness over a
semi-infinite bottom layer).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rw_oracle.c")
_LIB = os.path.join(_HERE, "liborc_rw.so")

# tally layout of orc_forward (per unit)
T_SUMX, T_SUMX2, T_SUMT, T_SUMA, T_SPEC, T_CAPPED, T_KILLED, T_NEXIT = range(8)
END_EXIT_TOP, END_EXIT_BOTTOM, END_RR_KILLED, END_CAPPED = 1, 2, 3, 4
END_ABSORBED, END_SPECULAR, END_NO_BLOCKS = 5, 6, 7
EV_START, EV_COLLIDE, EV_REFLECT, EV_EXIT_TOP, EV_EXIT_BOTTOM = 0, 1, 2, 3, 4
EV_RR_KILL, EV_CAP, EV_ABSORB, EV_CROSS = 5, 6, 7, 8


class OrcGeometry(ctypes.Structure):
    _fields_ = [
        ("n_media", ctypes.c_int32),
        ("n_bins", ctypes.c_int32),
        ("n_rel", ctypes.c_double),
        ("slab_mm", ctypes.c_double),
        ("r_min_mm", ctypes.c_double),
        ("r_max_mm", ctypes.c_double),
        ("rr_weight", ctypes.c_double),
        ("rr_survive", ctypes.c_double),
        ("max_vertices", ctypes.c_int64),
        ("analog", ctypes.c_int32),
        ("order_filter", ctypes.c_int32),
        ("incidence", ctypes.c_int32),
    ]


@dataclass
class Geometry:
    """Walk geometry and estimator constants (defaults: the radial set-up with
    256 log bins over [1e-3, 50] mm and the roulette constants 1e-4 / 0.1)."""

    n_media: int = 3
    n_rel: float = 1.0
    slab_mm: float = 0.0  # <= 0: semi-infinite
    n_bins: int = 256
    r_min_mm: float = 1e-3
    r_max_mm: float = 50.0
    rr_weight: float = 1e-4
    rr_survive: float = 0.1
    max_vertices: int = 1 << 20
    analog: bool = False
    order_filter: int = 0
    incidence: int = 0  # 0: normal pencil beam; 1: cosine-weighted lobe

    def c(self) -> OrcGeometry:
        return OrcGeometry(
            self.n_media, self.n_bins, self.n_rel, self.slab_mm, self.r_min_mm,
            self.r_max_mm, self.rr_weight, self.rr_survive, self.max_vertices,
            int(self.analog), self.order_filter, int(self.incidence),
        )


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE semantics, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-Wall", "-Wextra",
             "-o", tmp, _SRC, "-lm", "-lpthread"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _bind(ctypes.CDLL(build()))
    return _lib


class use_library:
    """Temporarily route this module's calls to another build of the oracle
    source (used by the tests that plant mistakes in a copy of the oracle)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _bind(ctypes.CDLL(self.path))
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def compile_source(src_text: str, out_path: str) -> str:
    """Compile oracle source text (e.g. a deliberately broken copy) to out_path."""
    c_path = out_path[:-3] + ".c"
    with open(c_path, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                           "-w", "-o", out_path, c_path, "-lm", "-lpthread"])
    return out_path


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def _bind(L):
    """Declare the argument and return types of the exported functions."""
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    gp = ctypes.POINTER(OrcGeometry)
    L.orc_forward.argtypes = [gp, dp, dp, dp, dp, ctypes.c_int64, i64p, ctypes.c_uint64,
                              ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, dp, dp, i64p]
    L.orc_forward.restype = ctypes.c_int
    L.orc_dwivedi_forward.argtypes = [gp, dp, dp, dp, dp, ctypes.c_int64, i64p, ctypes.c_uint64,
                                      ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double,
                                      ctypes.c_int, dp, dp, i64p]
    L.orc_dwivedi_forward.restype = ctypes.c_int
    L.orc_dwivedi_nu0.argtypes = [ctypes.c_double]
    L.orc_dwivedi_nu0.restype = ctypes.c_double
    L.orc_adjoint.argtypes = [gp, dp, dp, dp, dp, ctypes.c_int64, i64p, ctypes.c_uint64,
                              ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, dp, dp, dp, dp, dp,
                              dp]
    L.orc_adjoint.restype = ctypes.c_int
    L.orc_trace.argtypes = [gp, dp, dp, dp, dp, u32p, ctypes.c_int64, ctypes.c_int64,
                            ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, dp, dp, dp,
                            ctypes.c_double]
    L.orc_trace.restype = ctypes.c_int
    L.orc_layered_forward.argtypes = [gp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int64, i64p,
                                      ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_int, dp, dp, i64p]
    L.orc_layered_forward.restype = ctypes.c_int
    L.orc_layered_hero_forward.argtypes = [gp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int64,
                                           ctypes.c_int, i64p, ctypes.c_uint64, ctypes.c_uint32,
                                           ctypes.c_uint32, ctypes.c_int, dp, dp, i64p]
    L.orc_layered_hero_forward.restype = ctypes.c_int
    L.orc_layered_adjoint.argtypes = [gp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int64, i64p,
                                      ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_int, dp, dp, dp, dp]
    L.orc_layered_adjoint.restype = ctypes.c_int
    L.orc_layered_trace.argtypes = [gp, dp, dp, dp, ctypes.c_double, ctypes.c_double, u32p,
                                    ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                    ctypes.c_uint32, ctypes.c_uint32, dp, dp]
    L.orc_layered_trace.restype = ctypes.c_int
    L.orc_philox.argtypes = [u32p, u32p, u32p, ctypes.c_int64]
    L.orc_philox.restype = None
    L.orc_u01.argtypes = [ctypes.c_uint32]
    L.orc_u01.restype = ctypes.c_double
    L.orc_fresnel.argtypes = [ctypes.c_double, ctypes.c_double]
    L.orc_fresnel.restype = ctypes.c_double
    L.orc_hg_cos.argtypes = [ctypes.c_double, ctypes.c_double]
    L.orc_hg_cos.restype = ctypes.c_double
    L.orc_hg_dlog_dg.argtypes = [ctypes.c_double, ctypes.c_double]
    L.orc_hg_dlog_dg.restype = ctypes.c_double
    L.orc_frame.argtypes = [dp, dp, dp]
    L.orc_frame.restype = None
    L.orc_scatter_dir.argtypes = [dp, ctypes.c_double, ctypes.c_double]
    L.orc_scatter_dir.restype = None
    L.orc_bin_slot.argtypes = [ctypes.c_double, gp]
    L.orc_bin_slot.restype = ctypes.c_int
    return L


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i64ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _u32ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _soa(x, K: int, n_units: int) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(K, n_units))
    return a


def _paths(paths, n_units: int) -> np.ndarray:
    p = np.asarray(paths, dtype=np.int64)
    if p.ndim == 0:
        p = np.full(n_units, int(p), dtype=np.int64)
    return np.ascontiguousarray(p.reshape(n_units))


def default_threads() -> int:
    env = os.environ.get("ORC_THREADS")
    if env:
        return max(1, int(env))
    return max(1, min(os.cpu_count() or 1, 64))


def forward(geo: Geometry, sigma_t, albedo, g, w, paths, seed: int, tag: int = 0,
            n_threads: int | None = None, unit_base: int = 0):
    """Raw FP64 sums per unit.

    Parameters are SoA arrays of shape [K, n_units] (any float dtype; FP32 values
    are taken exactly).  Unit u draws its random numbers as unit unit_base + u.  Returns (tally[n_units, 8], bins[n_units, n_bins+2, 2],
    vertices[n_units])."""
    K = geo.n_media
    sigma_t = np.asarray(sigma_t)
    n_units = sigma_t.size // K
    s, a, gg, ww = (_soa(v, K, n_units) for v in (sigma_t, albedo, g, w))
    p = _paths(paths, n_units)
    tally = np.zeros((n_units, 8))
    bins = np.zeros((n_units, geo.n_bins + 2, 2))
    vert = np.zeros(n_units, dtype=np.int64)
    cg = geo.c()
    rc = lib().orc_forward(ctypes.byref(cg), _dptr(s), _dptr(a), _dptr(gg), _dptr(ww), n_units,
                           _i64ptr(p), seed, tag, unit_base, n_threads or default_threads(),
                           _dptr(tally),
                           _dptr(bins), _i64ptr(vert))
    if rc != 0:
        raise ValueError(f"orc_forward failed with code {rc}")
    return tally, bins, vert


def dwivedi_forward(geo: Geometry, sigma_t, albedo, g, w, paths, seed: int, q: float,
                    tag: int = 0, n_threads: int | None = None, unit_base: int = 0):
    """Raw FP64 sums per unit of the mixture walk with Dwivedi sampling
    (technique probability q in (0, 1); see orc_dwivedi_forward).  Same layout
    as forward()."""
    K = geo.n_media
    sigma_t = np.asarray(sigma_t)
    n_units = sigma_t.size // K
    s, a, gg, ww = (_soa(v, K, n_units) for v in (sigma_t, albedo, g, w))
    p = _paths(paths, n_units)
    tally = np.zeros((n_units, 8))
    bins = np.zeros((n_units, geo.n_bins + 2, 2))
    vert = np.zeros(n_units, dtype=np.int64)
    cg = geo.c()
    rc = lib().orc_dwivedi_forward(ctypes.byref(cg), _dptr(s), _dptr(a), _dptr(gg), _dptr(ww),
                                   n_units, _i64ptr(p), seed, tag, unit_base, float(q),
                                   n_threads or default_threads(), _dptr(tally), _dptr(bins),
                                   _i64ptr(vert))
    if rc != 0:
        raise ValueError(f"orc_dwivedi_forward failed with code {rc}")
    return tally, bins, vert


def dwivedi_nu0(alpha: float) -> float:
    """nu0 of the Dwivedi walk for a single-scattering albedo (clamped to
    [0.3, 1 - 1e-7])."""
    return float(lib().orc_dwivedi_nu0(float(alpha)))


def adjoint(geo: Geometry, sigma_t, albedo, g, w, paths, seed: int, cot_R=None, cot_bins=None,
            tag: int = 0, n_threads: int | None = None, jacobian: bool = False,
            unit_base: int = 0):
    """Score-function gradient sums (see orc_adjoint).  Returns (grad, sumsq) of
    shape [n_units, 4K], plus (jac_R [n_units, 4K], jac_bins [n_units, n_bins+2, 4K])
    when jacobian=True."""
    K = geo.n_media
    sigma_t = np.asarray(sigma_t)
    n_units = sigma_t.size // K
    s, a, gg, ww = (_soa(v, K, n_units) for v in (sigma_t, albedo, g, w))
    p = _paths(paths, n_units)
    P = 4 * K
    cR = None if cot_R is None else np.ascontiguousarray(np.asarray(cot_R, np.float64).reshape(n_units))
    cB = None if cot_bins is None else np.ascontiguousarray(
        np.asarray(cot_bins, np.float64).reshape(n_units, geo.n_bins + 2))
    grad = np.zeros((n_units, P))
    sumsq = np.zeros((n_units, P))
    jR = np.zeros((n_units, P)) if jacobian else None
    jB = np.zeros((n_units, geo.n_bins + 2, P)) if jacobian else None
    cg = geo.c()
    rc = lib().orc_adjoint(ctypes.byref(cg), _dptr(s), _dptr(a), _dptr(gg), _dptr(ww), n_units,
                           _i64ptr(p), seed, tag, unit_base, n_threads or default_threads(),
                           _dptr(cR) if cR is not None else None,
                           _dptr(cB) if cB is not None else None, _dptr(grad), _dptr(sumsq),
                           _dptr(jR) if jacobian else None, _dptr(jB) if jacobian else None)
    if rc != 0:
        raise ValueError(f"orc_adjoint failed with code {rc}")
    if jacobian:
        return grad, sumsq, jR, jB
    return grad, sumsq


def trace(geo: Geometry, sigma_t, albedo, g, w, words=None, n_paths: int | None = None,
          n_blocks: int = 64, seed: int = 0, unit: int = 0, tag: int = 0,
          with_events: bool = True, dwivedi_q: float = 0.0):
    """Per-path replay of one unit.  words: uint32 [n_paths, n_blocks, 4] or None
    (Philox).  dwivedi_q > 0: the Dwivedi walk with that technique probability.
    Returns (events [n_paths, n_blocks, 8], path_out [n_paths, 8],
    path_adj [n_paths, 2])."""
    K = geo.n_media
    s, a, gg, ww = (np.ascontiguousarray(np.asarray(v, np.float64).reshape(K))
                    for v in (sigma_t, albedo, g, w))
    if words is not None:
        words = np.ascontiguousarray(np.asarray(words, dtype=np.uint32))
        n_paths, n_blocks = words.shape[0], words.shape[1]
    assert n_paths is not None
    ev = np.zeros((n_paths, n_blocks, 8)) if with_events else None
    out = np.zeros((n_paths, 8))
    adj = np.zeros((n_paths, 2))
    cg = geo.c()
    rc = lib().orc_trace(ctypes.byref(cg), _dptr(s), _dptr(a), _dptr(gg), _dptr(ww),
                         _u32ptr(words) if words is not None else None, n_paths, n_blocks, seed,
                         unit, tag, _dptr(ev) if ev is not None else None, _dptr(out), _dptr(adj),
                         float(dwivedi_q))
    if rc != 0:
        raise ValueError(f"orc_trace failed with code {rc}")
    return ev, out, adj


def layered_forward(geo: Geometry, sigma_t, albedo, g, thickness, n_bottom: float, paths,
                    seed: int, tag: int = 0, n_threads: int | None = None, unit_base: int = 0):
    """Two-layer tissue: raw FP64 sums per unit, as forward().  sigma_t, albedo,
    g: [2, n_units] (top, bottom layer); thickness: [n_units] top-layer
    thickness in mm; n_bottom: the bottom layer's index relative to the
    outside (the top layer's is geo.n_rel).  geo.n_media must be 2."""
    sigma_t = np.asarray(sigma_t)
    n_units = sigma_t.size // 2
    s, a, gg = (_soa(v, 2, n_units) for v in (sigma_t, albedo, g))
    d = np.ascontiguousarray(np.asarray(thickness, np.float64).reshape(n_units))
    p = _paths(paths, n_units)
    tally = np.zeros((n_units, 8))
    bins = np.zeros((n_units, geo.n_bins + 2, 2))
    vert = np.zeros(n_units, dtype=np.int64)
    cg = geo.c()
    rc = lib().orc_layered_forward(ctypes.byref(cg), _dptr(s), _dptr(a), _dptr(gg), _dptr(d),
                                   float(n_bottom), n_units, _i64ptr(p), seed, tag, unit_base,
                                   n_threads or default_threads(), _dptr(tally), _dptr(bins),
                                   _i64ptr(vert))
    if rc != 0:
        raise ValueError(f"orc_layered_forward failed with code {rc}")
    return tally, bins, vert


def layered_hero_forward(geo: Geometry, sigma_t, albedo, g, thickness, n_bottom: float,
                         n_hero: int, paths, seed: int, tag: int = 0,
                         n_threads: int | None = None, unit_base: int = 0):
    """Hero-wavelength two-layer walk (orc_layered_hero_forward): units in
    groups of n_hero consecutive units sharing one walk, `paths` per group
    (scalar or [n_groups], multiples of n_hero).  Returns (tally, bins,
    vertices) per unit as layered_forward (absorbed weight 0; vertices of the
    paths each unit was hero of)."""
    sigma_t = np.asarray(sigma_t)
    n_units = sigma_t.size // 2
    s, a, gg = (_soa(v, 2, n_units) for v in (sigma_t, albedo, g))
    d = np.ascontiguousarray(np.asarray(thickness, np.float64).reshape(n_units))
    p = _paths(paths, n_units // n_hero)
    tally = np.zeros((n_units, 8))
    bins = np.zeros((n_units, geo.n_bins + 2, 2))
    vert = np.zeros(n_units, dtype=np.int64)
    cg = geo.c()
    rc = lib().orc_layered_hero_forward(ctypes.byref(cg), _dptr(s), _dptr(a), _dptr(gg), _dptr(d),
                                        float(n_bottom), n_units, int(n_hero), _i64ptr(p), seed,
                                        tag, unit_base, n_threads or default_threads(),
                                        _dptr(tally), _dptr(bins), _i64ptr(vert))
    if rc != 0:
        raise ValueError(f"orc_layered_hero_forward failed with code {rc}")
    return tally, bins, vert


def layered_adjoint(geo: Geometry, sigma_t, albedo, g, thickness, n_bottom: float, paths,
                    seed: int, cot_R=None, cot_bins=None, tag: int = 0,
                    n_threads: int | None = None, unit_base: int = 0):
    """Score-function gradient sums of the two-layer walk (see
    orc_layered_adjoint).  Returns (grad, sumsq) of shape [n_units, 8]:
    sigma_t (top, bottom), albedo (top, bottom), g (top, bottom), 0, 0."""
    sigma_t = np.asarray(sigma_t)
    n_units = sigma_t.size // 2
    s, a, gg = (_soa(v, 2, n_units) for v in (sigma_t, albedo, g))
    d = np.ascontiguousarray(np.asarray(thickness, np.float64).reshape(n_units))
    p = _paths(paths, n_units)
    cR = None if cot_R is None else np.ascontiguousarray(np.asarray(cot_R, np.float64).reshape(n_units))
    cB = None if cot_bins is None else np.ascontiguousarray(
        np.asarray(cot_bins, np.float64).reshape(n_units, geo.n_bins + 2))
    grad = np.zeros((n_units, 8))
    sumsq = np.zeros((n_units, 8))
    cg = geo.c()
    rc = lib().orc_layered_adjoint(ctypes.byref(cg), _dptr(s), _dptr(a), _dptr(gg), _dptr(d),
                                   float(n_bottom), n_units, _i64ptr(p), seed, tag, unit_base,
                                   n_threads or default_threads(),
                                   _dptr(cR) if cR is not None else None,
                                   _dptr(cB) if cB is not None else None, _dptr(grad),
                                   _dptr(sumsq))
    if rc != 0:
        raise ValueError(f"orc_layered_adjoint failed with code {rc}")
    return grad, sumsq


def layered_trace(geo: Geometry, sigma_t, albedo, g, thickness: float, n_bottom: float,
                  words=None, n_paths: int | None = None, n_blocks: int = 64, seed: int = 0,
                  unit: int = 0, tag: int = 0):
    """Per-path replay of one two-layer unit (parameters of length 2).  Returns
    (events [n_paths, n_blocks, 8], path_out [n_paths, 8]); path_out[:, 1] is
    the layer the path ended in."""
    s, a, gg = (np.ascontiguousarray(np.asarray(v, np.float64).reshape(2))
                for v in (sigma_t, albedo, g))
    if words is not None:
        words = np.ascontiguousarray(np.asarray(words, dtype=np.uint32))
        n_paths, n_blocks = words.shape[0], words.shape[1]
    assert n_paths is not None
    ev = np.zeros((n_paths, n_blocks, 8))
    out = np.zeros((n_paths, 8))
    cg = geo.c()
    rc = lib().orc_layered_trace(ctypes.byref(cg), _dptr(s), _dptr(a), _dptr(gg),
                                 float(thickness), float(n_bottom),
                                 _u32ptr(words) if words is not None else None, n_paths, n_blocks,
                                 seed, unit, tag, _dptr(ev), _dptr(out))
    if rc != 0:
        raise ValueError(f"orc_layered_trace failed with code {rc}")
    return ev, out


def philox(counters, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(counters, dtype=np.uint32).reshape(-1, 4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.zeros_like(c)
    lib().orc_philox(_u32ptr(c), _u32ptr(k), _u32ptr(out), c.shape[0])
    return out


def u01(word: int) -> float:
    return lib().orc_u01(word)


def fresnel(cos_i: float, n: float) -> float:
    return lib().orc_fresnel(cos_i, n)


def hg_cos(g: float, u: float) -> float:
    return lib().orc_hg_cos(g, u)


def hg_dlog_dg(g: float, mu: float) -> float:
    return lib().orc_hg_dlog_dg(g, mu)


def frame(d):
    d = np.ascontiguousarray(np.asarray(d, np.float64))
    t1 = np.zeros(3)
    t2 = np.zeros(3)
    lib().orc_frame(_dptr(d), _dptr(t1), _dptr(t2))
    return t1, t2


def scatter_dir(d, mu: float, phi: float) -> np.ndarray:
    d = np.ascontiguousarray(np.asarray(d, np.float64)).copy()
    lib().orc_scatter_dir(_dptr(d), mu, phi)
    return d


def bin_slot(r: float, geo: Geometry) -> int:
    cg = geo.c()
    return lib().orc_bin_slot(r, ctypes.byref(cg))


def mean_and_se(sum_x, sum_x2, n):
    """Per-path mean and its standard error from raw sums."""
    sum_x = np.asarray(sum_x, np.float64)
    sum_x2 = np.asarray(sum_x2, np.float64)
    n = np.asarray(n, np.float64)
    mean = sum_x / n
    var = np.maximum(sum_x2 - sum_x * sum_x / n, 0.0) / np.maximum(n - 1.0, 1.0)
    return mean, np.sqrt(var / n)
