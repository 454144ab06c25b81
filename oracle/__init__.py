"""ctypes front-end of the FP64 CPU oracle (``oracle/gf_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the HIP library or its binding.

Every array argument is converted to contiguous float64 (parameters and rays
are float32 inputs promoted exactly).  See ``gf_oracle.c`` for the definitions.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "gf_oracle.c")

GCC_CMD = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", LIB_PATH, SRC_PATH, "-lm"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU code involved)."""
    if force or not os.path.exists(LIB_PATH):
        subprocess.check_call(GCC_CMD)
    return LIB_PATH


_lib = None

_d = C.POINTER(C.c_double)
_f = C.POINTER(C.c_float)
_i32 = C.POINTER(C.c_int32)
_i64 = C.POINTER(C.c_int64)
_u32 = C.POINTER(C.c_uint32)
_u64 = C.POINTER(C.c_uint64)
_I64, _U64 = C.c_int64, C.c_uint64


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.or_w.argtypes = [_d, _d, _I64, _d, _d]
        L.or_set_clamp_eps.argtypes = [C.c_double]
        L.or_segment_integral.argtypes = [_d, _d, C.c_double, _d]
        L.or_cells.argtypes = [_d, _I64, _i32, _d]
        L.or_cell_medians.argtypes = [_d, _I64, _d]
        L.or_mask_cone.argtypes = [_d, _I64, _d, C.c_double, _u32]
        L.or_tau.argtypes = [_d, _I64, C.c_double, C.c_double, _d, _I64, _U64, _u32, C.c_int, C.c_double, _d, _d,
                             _i64]
        L.or_kappa.argtypes = [_d, _I64, C.c_double, C.c_double, _U64, _u32, _d, _I64, _d]
        L.or_lbvh.argtypes = [_d, _I64, C.c_double, C.c_double, _u64, _i32, _i32, _i32, _i32, _f, _u64]
        L.or_lbvh.restype = C.c_int
        L.or_traverse_counts.argtypes = [_d, _I64, C.c_double, C.c_double, _i32, _i32, _i32, _f, _u64, _d, _I64,
                                         _U64, _u32, _i64, _i64]
        L.or_philox.argtypes = [_u32, _u32, _u32, _I64]
        L.or_ratio_T.argtypes = [_d, _I64, C.c_double, C.c_double, _d, _I64, _U64, _u32, C.c_double, C.c_int, _U64,
                                 _d, _d]
        L.or_free_flight.argtypes = [_d, _I64, C.c_double, C.c_double, _d, _I64, _U64, _u32, C.c_int, C.c_int, _U64,
                                     _d, _d]
        L.or_hg_cos.argtypes = [C.c_double, _I64, _U64, _d]
        L.or_segment_cell_weights.argtypes = [_d, _d, _d, _d, _d]
        L.or_sample_cell_weights.argtypes = [_d, _d, _d, _I64, _U64, _d]
        L.or_render.argtypes = [_d, _I64, C.c_double, C.c_double, _d, _I64, _U64, _u32, _d, _U64, _d, _d, _d,
                                _d]
        L.or_tau_grad.argtypes = [_d, _I64, C.c_double, C.c_double, _d, _I64, _U64, _u32, C.c_double, _d, _d]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _bits(b):
    return None if b is None else np.ascontiguousarray(np.asarray(b, dtype=np.uint32))


FULL_MASK = (1 << 12) - 1

# Strategy codes of the per-segment stochastic masks (Appendix B tables)
LEVEL = dict(deterministic=0, uniform=1, power=2, uniform_cv=3, power_cv=4, power_cv_accum=5)
BIN = dict(deterministic=0, threshold=1, uniform=2, importance=3, threshold_uniform=4, mixture=5)


class _clamp:
    """Sets the oracle's adaptive-clamping threshold for one call."""

    def __init__(self, eps):
        self.eps = float(eps)

    def __enter__(self):
        lib().or_set_clamp_eps(self.eps)

    def __exit__(self, *exc):
        lib().or_set_clamp_eps(0.0)


def lod_cells(lod: int) -> int:
    """Cell mask of an LOD level: 0 = all levels, 1 = levels 0-2 (1/2 band),
    2 = levels 0-1 (1/4 band), 3 = level 0 (1/8 band); all orientation bins."""
    nlev = 4 - lod
    return sum(7 << (3 * l) for l in range(nlev))


def faddeeva(z):
    z = np.asarray(z, dtype=np.complex128).ravel()
    zr, zi = _f64(z.real), _f64(z.imag)
    wr, wi = np.empty_like(zr), np.empty_like(zr)
    lib().or_w(_p(zr, _d), _p(zi, _d), len(zr), _p(wr, _d), _p(wi, _d))
    return wr + 1j * wi


def segment_integral(prim, ray, r=3.0):
    """(I, nonempty, h2, ua, ub, Omega, theta, n) of one primitive and one ray."""
    p, ry = _f64(prim), _f64(ray)
    out = np.zeros(8)
    lib().or_segment_integral(_p(p, _d), _p(ry, _d), r, _p(out, _d))
    return out


def cells(params):
    p = _f64(params)
    n = p.shape[0]
    c = np.empty(n, np.int32)
    m = np.zeros(1)
    lib().or_cells(_p(p, _d), n, _p(c, _i32), _p(m, _d))
    return c, float(m[0])


def cell_medians(params):
    p = _f64(params)
    med = np.zeros(12)
    lib().or_cell_medians(_p(p, _d), p.shape[0], _p(med, _d))
    return med


def mask_cone(params, axis=(0.0, 0.0, 1.0), half_angle=np.pi / 4):
    p = _f64(params)
    n = p.shape[0]
    bits = np.zeros((n + 31) // 32, np.uint32)
    ax = _f64(axis)
    lib().or_mask_cone(_p(p, _d), n, _p(ax, _d), half_angle, _p(bits, _u32))
    return bits


def tau(params, rays, rho=1.0, r=3.0, cells=FULL_MASK, bits=None, envelope=False, lod_k=0.0, clamp_eps=0.0):
    """Returns (tau, sum_i |tau_i|, number of hits) per ray."""
    p, ry, b = _f64(params), _f64(rays), _bits(bits)
    nr = ry.shape[0]
    t, a, h = np.empty(nr), np.empty(nr), np.empty(nr, np.int64)
    with _clamp(clamp_eps):
        lib().or_tau(_p(p, _d), p.shape[0], rho, r, _p(ry, _d), nr, cells, _p(b, _u32), int(envelope), lod_k,
                     _p(t, _d), _p(a, _d), _p(h, _i64))
    return t, a, h


def kappa(params, pts, rho=1.0, r=3.0, cells=FULL_MASK, bits=None, clamp_eps=0.0):
    p, x, b = _f64(params), _f64(pts), _bits(bits)
    out = np.empty(x.shape[0])
    with _clamp(clamp_eps):
        lib().or_kappa(_p(p, _d), p.shape[0], rho, r, cells, _p(b, _u32), _p(x, _d), x.shape[0], _p(out, _d))
    return out


def lbvh(params, r=3.0, rho=1.0, clamp_eps=0.0):
    p = _f64(params)
    n = p.shape[0]
    keys = np.empty(n, np.uint64)
    perm = np.empty(n, np.int32)
    left = np.full(max(n - 1, 0), -1, np.int32)
    right = np.full(max(n - 1, 0), -1, np.int32)
    parent = np.empty(2 * n - 1, np.int32)
    aabb = np.empty((2 * n - 1, 6), np.float32)
    cellor = np.empty(2 * n - 1, np.uint64)
    with _clamp(clamp_eps):
        rc = lib().or_lbvh(_p(p, _d), n, rho, r, _p(keys, _u64), _p(perm, _i32), _p(left, _i32), _p(right, _i32),
                           _p(parent, _i32), _p(aabb, _f), _p(cellor, _u64))
    if rc != 0:
        raise ValueError("or_lbvh failed")
    return dict(keys=keys, perm=perm, left=left, right=right, parent=parent, aabb=aabb, cellor=cellor)


def traverse_counts(params, bvh, rays, r=3.0, cells=FULL_MASK, bits=None, rho=1.0, clamp_eps=0.0):
    p, ry, b = _f64(params), _f64(rays), _bits(bits)
    nr = ry.shape[0]
    nn, nh = np.empty(nr, np.int64), np.empty(nr, np.int64)
    with _clamp(clamp_eps):
        lib().or_traverse_counts(_p(p, _d), p.shape[0], rho, r, _p(bvh["perm"], _i32), _p(bvh["left"], _i32),
                                 _p(bvh["right"], _i32), _p(bvh["aabb"], _f), _p(bvh["cellor"], _u64),
                                 _p(ry, _d), nr, cells, _p(b, _u32), _p(nn, _i64), _p(nh, _i64))
    return nn, nh


def philox(ctr, key):
    c = np.ascontiguousarray(np.asarray(ctr, np.uint32).reshape(-1, 4))
    k = np.ascontiguousarray(np.asarray(key, np.uint32).reshape(-1, 2))
    out = np.empty_like(c)
    lib().or_philox(_p(c, _u32), _p(k, _u32), _p(out, _u32), c.shape[0])
    return out


def ratio_T(params, rays, spp, seed, rho=1.0, r=3.0, cells=FULL_MASK, bits=None, lod_k=0.0, clamp_eps=0.0):
    p, ry, b = _f64(params), _f64(rays), _bits(bits)
    nr = ry.shape[0]
    m, v = np.empty(nr), np.empty(nr)
    with _clamp(clamp_eps):
        lib().or_ratio_T(_p(p, _d), p.shape[0], rho, r, _p(ry, _d), nr, cells, _p(b, _u32), lod_k, spp, seed,
                         _p(m, _d), _p(v, _d))
    return m, v


def free_flight(params, rays, spp, seed, rho=1.0, r=3.0, cells=FULL_MASK, bits=None, analytic=False):
    """Free-flight distances (inf on escape) and weights; analytic=True
    inverts the cumulative optical depth by bisection instead of delta
    tracking."""
    p, ry, b = _f64(params), _f64(rays), _bits(bits)
    nr = ry.shape[0]
    t, w = np.empty(nr * spp), np.empty(nr * spp)
    lib().or_free_flight(_p(p, _d), p.shape[0], rho, r, _p(ry, _d), nr, cells, _p(b, _u32), int(analytic), spp,
                         seed, _p(t, _d), _p(w, _d))
    return t.reshape(nr, spp), w.reshape(nr, spp)


def _strat(level, bin, beta, delta):
    lv = LEVEL[level] if isinstance(level, str) else int(level)
    bn = BIN[bin] if isinstance(bin, str) else int(bin)
    return _f64([lv, bn, beta, delta])


def segment_cell_weights(level, bin, med12, v, u, beta=0.0, delta=1.0):
    """Cell weights (12) of one segment with direction v for explicit uniforms u[0..3]."""
    out = np.empty(12)
    st, m, vv, uu = _strat(level, bin, beta, delta), _f64(med12), _f64(v), _f64(u)
    lib().or_segment_cell_weights(_p(st, _d), _p(m, _d), _p(vv, _d), _p(uu, _d), _p(out, _d))
    return out


def sample_cell_weights(level, bin, med12, v, n, seed, beta=0.0, delta=1.0):
    """n draws (n x 12) of a segment's cell weights from the oracle's own streams."""
    out = np.empty((n, 12))
    st, m, vv = _strat(level, bin, beta, delta), _f64(med12), _f64(v)
    lib().or_sample_cell_weights(_p(st, _d), _p(m, _d), _p(vv, _d), n, seed, _p(out, _d))
    return out


def hg_cos(g, n, seed):
    out = np.empty(n)
    lib().or_hg_cos(g, n, seed, _p(out, _d))
    return out


def render(params, rays, spp, seed, rho=1.0, r=3.0, multiple=False, max_scatter=16, albedo=0.9, hg_g=0.0,
           L_env=1.0, stochastic=False, cells=FULL_MASK, bits=None, level="uniform_cv", bin="importance",
           beta=0.0, delta=1.0, analytic=False, shadow_cells=0, lod_k=0.0, clamp_eps=0.0):
    """Returns (L_mean, L_var, primaryT_mean, primaryT_var) per ray.
    stochastic: per-segment masks drawn by the level / bin strategies;
    analytic: free flights by CDF inversion and exact transmittances;
    shadow_cells: cells the single-scattering shadow rays trace (0 = the
    segment's own mask); lod_k: continuous-LOD cutoff of the camera segment."""
    p, ry, b = _f64(params), _f64(rays), _bits(bits)
    nr = ry.shape[0]
    st = _strat(level, bin, beta, delta)
    desc = _f64([spp, int(multiple), max_scatter, albedo, hg_g, L_env, int(stochastic), st[0], st[1], beta, delta,
                 int(analytic), shadow_cells, lod_k])
    Lm, Lv, Tm, Tv = (np.empty(nr) for _ in range(4))
    with _clamp(clamp_eps):
        lib().or_render(_p(p, _d), p.shape[0], rho, r, _p(ry, _d), nr, cells, _p(b, _u32), _p(desc, _d), seed,
                        _p(Lm, _d), _p(Lv, _d), _p(Tm, _d), _p(Tv, _d))
    return Lm, Lv, Tm, Tv


def tau_grad(params, rays, dL_dtau, rho=1.0, r=3.0, cells=FULL_MASK, bits=None, lod_k=0.0, clamp_eps=0.0):
    p, ry, b, g = _f64(params), _f64(rays), _bits(bits), _f64(dL_dtau)
    out = np.empty((p.shape[0], 15))
    with _clamp(clamp_eps):
        lib().or_tau_grad(_p(p, _d), p.shape[0], rho, r, _p(ry, _d), ry.shape[0], cells, _p(b, _u32), lod_k,
                          _p(g, _d), _p(out, _d))
    return out


def clamp_radii(params, rho, eps, r=3.0):
    """Per-primitive truncation radius under adaptive clamping, min(r, E_i)
    with E_i^2 = 2 ln(rho |alpha_i| s_max / (2 pi s0 s1 s2 eps)) (0 when
    E_i^2 <= 0): what the oracle integrates with (see clamp_radius in
    gf_oracle.c)."""
    p = np.asarray(params, np.float64)
    smax = p[:, 7:10].max(axis=1)
    arg = rho * np.abs(p[:, 14]) * smax / (2 * np.pi * p[:, 7] * p[:, 8] * p[:, 9] * eps)
    with np.errstate(divide="ignore", invalid="ignore"):
        E = np.sqrt(2 * np.log(np.where(arg > 1, arg, 1.0)))
    return np.where(arg > 1, np.minimum(E, r), 0.0)
