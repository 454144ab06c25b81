"""Pins of the oracle's stochastic estimators.

* ratio tracking with local majorants: E[T_hat] = exp(-tau) for a signed field;
* weighted delta tracking: distances follow 1 - exp(-tau(0, t)) for a positive
  Gaussian (Kolmogorov-Smirnov), and E[w 1(escape)] = exp(-tau) when signed;
* Henyey-Greenstein sampling: E[cos] = g;
* furnace: albedo 1, no cap, L_env = 1 gives L = 1 (Sec. 3 radiative transfer);
* single scattering against FP64 nested quadrature of the transfer equation.
* Philox4x32-10 against the published known-answer vectors (Salmon et al. 2011).
"""
import math

import numpy as np
import pytest
import scipy.stats as st

import gen
from gen import workloads as W

RHO_TINY = W.rho("tiny256")


def test_philox_known_answers(orc):
    out = orc.philox([[0, 0, 0, 0], [0xffffffff] * 4, [0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344]],
                     [[0, 0], [0xffffffff] * 2, [0xa4093822, 0x299f31d0]])
    assert [hex(x) for x in out[0]] == ["0x6627e8d5", "0xe169c58d", "0xbc57ac4c", "0x9b00dbd8"]
    assert [hex(x) for x in out[1]] == ["0x408f276d", "0x41c83b0e", "0xa20bc7c6", "0x6d5451fd"]
    assert [hex(x) for x in out[2]] == ["0xd16cfe09", "0x94fdcceb", "0x5001e420", "0x24126ea1"]


def _pooled(mean, target, se):
    se = se + 1e-15
    return abs(np.sum(mean - target)) / np.sqrt(np.sum(se ** 2)), np.max(np.abs(mean - target) / se)


def test_ratio_tracking_unbiased_signed(orc):
    params = gen.uniform_scene(256, 0)
    rays = gen.ortho_rays(64, 64)[::61]
    spp = 2000
    tau, _, hits = orc.tau(params, rays, rho=RHO_TINY)
    m, v = orc.ratio_T(params, rays, spp, seed=5, rho=RHO_TINY)
    pooled, worst = _pooled(m, np.exp(-tau), np.sqrt(v / spp))
    assert pooled < 3.0 and worst < 4.5
    assert np.all(m[hits == 0] == 1.0)


def test_ratio_tracking_mask(orc):
    params = gen.uniform_scene(256, 0)
    rays = gen.ortho_rays(64, 64)[::97]
    spp = 1500
    cells = orc.lod_cells(2)
    tau, _, _ = orc.tau(params, rays, rho=RHO_TINY, cells=cells)
    m, v = orc.ratio_T(params, rays, spp, seed=6, rho=RHO_TINY, cells=cells)
    pooled, worst = _pooled(m, np.exp(-tau), np.sqrt(v / spp))
    assert pooled < 3.0 and worst < 4.5
    m0, _ = orc.ratio_T(params, rays, 4, seed=6, rho=RHO_TINY, cells=0)
    assert np.all(m0 == 1.0)


def _gaussian_prim(alpha=1.0, s=(0.1, 0.06, 0.08)):
    p = np.zeros(15)
    p[0:3] = 0.5
    q = np.array([0.9, 0.2, -0.3, 0.25])
    p[3:7] = q / np.linalg.norm(q)
    p[7:10] = s
    p[14] = alpha
    return p[None, :]


def test_free_flight_distribution_positive_gaussian(orc):
    params = _gaussian_prim()
    ray = np.array([[0.52, 0.47, -0.5, 0.0, 0.0, 1.0, 0.0, np.inf]])
    rho = 1.5 / orc.tau(params, ray, rho=1.0)[0][0]
    tau_tot = orc.tau(params, ray, rho=rho)[0][0]
    t, w = orc.free_flight(params, ray, 20000, seed=3, rho=rho)
    assert np.all(w == 1.0)  # positive density: plain delta tracking, no weights
    t = t[0]
    col = t[np.isfinite(t)]
    esc = np.mean(~np.isfinite(t))
    assert abs(esc - math.exp(-tau_tot)) < 4 * math.sqrt(math.exp(-tau_tot) * (1 - math.exp(-tau_tot)) / len(t))
    # conditional CDF of collision distances
    ts = np.sort(col)[:: max(1, len(col) // 2000)]
    rr = np.repeat(ray, len(ts), axis=0)
    rr[:, 7] = ts
    F = 1.0 - np.exp(-orc.tau(params, rr, rho=rho)[0])
    Fcond = F / (1.0 - math.exp(-tau_tot))
    ks = st.kstest(Fcond, "uniform")
    assert ks.pvalue > 1e-3


def test_weighted_delta_tracking_escape_signed(orc):
    params = gen.uniform_scene(256, 0)
    rays = gen.ortho_rays(64, 64)[::89]
    spp = 3000
    tau, _, _ = orc.tau(params, rays, rho=RHO_TINY)
    t, w = orc.free_flight(params, rays, spp, seed=9, rho=RHO_TINY)
    est = np.where(np.isfinite(t), 0.0, w)
    # rays whose expected number of escapes is below 5 cannot estimate their
    # own standard error (all samples collide), so they are left out
    ok = spp * np.exp(-tau) >= 5.0
    assert ok.sum() >= 30
    pooled, worst = _pooled(est.mean(axis=1)[ok], np.exp(-tau[ok]), est.std(axis=1, ddof=1)[ok] / math.sqrt(spp))
    assert pooled < 3.0 and worst < 4.5


def test_hg_sampling_mean_cosine(orc):
    for g in (0.0, 0.3, -0.5, 0.8):
        c = orc.hg_cos(g, 200000, seed=1)
        assert np.all(np.abs(c) <= 1.0)
        assert abs(c.mean() - g) < 4 * c.std() / math.sqrt(len(c))
    c = orc.hg_cos(0.0, 200000, seed=2)
    assert abs(np.mean(c * c) - 1 / 3) < 0.003


def test_furnace_positive_density_is_exact(orc):
    params = gen.uniform_scene(64, 5).astype(np.float64)
    params[:, 10:13] = 0.0
    params[:, 13] = 0.0
    rays = gen.ortho_rays(16, 16)
    L, _, _, _ = orc.render(params, rays, 8, seed=1, rho=0.05, multiple=True, max_scatter=100000, albedo=1.0,
                            hg_g=0.3)
    assert np.all(L == 1.0)


def test_furnace_signed_density_in_mean(orc):
    params = gen.uniform_scene(64, 5)
    rays = gen.ortho_rays(16, 16)[::5]
    spp = 2000
    L, Lv, _, _ = orc.render(params, rays, spp, seed=2, rho=0.004, multiple=True, max_scatter=100000, albedo=1.0,
                             hg_g=0.3)
    pooled, worst = _pooled(L, np.ones_like(L), np.sqrt(Lv / spp))
    assert pooled < 3.0 and worst < 4.5


def _quadrature_scene(n_gabor=0):
    g = np.random.default_rng(4)
    n = 6 + n_gabor
    params = np.zeros((n, 15))
    params[:, 0:3] = 0.5 + 0.08 * g.standard_normal((n, 3))
    q = g.standard_normal((n, 4))
    params[:, 3:7] = q / np.linalg.norm(q, axis=1, keepdims=True)
    params[:, 7:10] = g.uniform(0.05, 0.09, (n, 3))
    params[:, 14] = g.uniform(0.5, 1.5, n)
    if n_gabor:
        # Gabor kernels of the top frequency level on top of the Gaussians
        f = g.standard_normal((n_gabor, 3))
        params[6:, 10:13] = 2.0 * f / np.linalg.norm(f, axis=1, keepdims=True)
        params[6:, 13] = 0.0
    return params


def _single_scattering_reference(orc, params, ray, rho, albedo, shadow_cells=None):
    """L = T(0,inf) L_env + albedo int T(0,t) kappa(t) [int p(w) T_s(x_t, w) dw] dt L_env,
    isotropic p; T_s the shadow transmittance (of the cells shadow_cells when
    given); t by Gauss-Legendre per chord piece, directions by a 3000-point
    Fibonacci sphere."""
    # chord ends of every truncated ellipsoid along the camera ray (numpy geometry)
    brk = [0.0]
    for p in params:
        w, x, y, z = p[3:7] / np.linalg.norm(p[3:7])
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        Si = np.linalg.inv(R @ np.diag(p[7:10] ** 2) @ R.T)
        d = ray[0:3] - p[0:3]
        a, b, c = ray[3:6] @ Si @ ray[3:6], ray[3:6] @ Si @ d, d @ Si @ d - 9.0
        if b * b - a * c > 0:
            brk += [(-b - math.sqrt(b * b - a * c)) / a, (-b + math.sqrt(b * b - a * c)) / a]
    tt = np.array(sorted(t for t in brk if t >= 0.0))
    xg, wg = np.polynomial.legendre.leggauss(24)
    pieces = [(a, b) for a, b in zip(tt[:-1], tt[1:]) if b > a]
    ts = np.concatenate([0.5 * (a + b) + 0.5 * (b - a) * xg for a, b in pieces])
    ws = np.concatenate([0.5 * (b - a) * wg for a, b in pieces])
    pts = ray[0:3][None, :] + ts[:, None] * ray[3:6][None, :]
    kap = orc.kappa(params, pts, rho=rho)
    r0 = np.repeat(ray[None, :], len(ts), axis=0)
    r0[:, 7] = ts
    T0 = np.exp(-orc.tau(params, r0, rho=rho)[0])
    m = 3000
    i = np.arange(m) + 0.5
    zc = 1 - 2 * i / m
    ph = math.pi * (1 + 5 ** 0.5) * i
    dirs = np.stack([np.sqrt(1 - zc * zc) * np.cos(ph), np.sqrt(1 - zc * zc) * np.sin(ph), zc], axis=1)
    keep = kap != 0.0
    inner = np.zeros(len(ts))
    sel = np.where(keep)[0]
    sr = np.zeros((len(sel) * m, 8))
    sr[:, 0:3] = np.repeat(pts[sel], m, axis=0)
    sr[:, 3:6] = np.tile(dirs, (len(sel), 1))
    sr[:, 6], sr[:, 7] = 0.0, np.inf
    cells = orc.FULL_MASK if shadow_cells is None else shadow_cells
    Ts = np.exp(-orc.tau(params, sr, rho=rho, cells=cells)[0]).reshape(len(sel), m)
    inner[sel] = Ts.mean(axis=1)
    Tinf = math.exp(-orc.tau(params, ray[None, :], rho=rho)[0][0])
    return Tinf + albedo * np.sum(ws * T0 * kap * inner)


_QRAY = np.array([0.5, 0.5, -0.5, 0.05, -0.02, 1.0, 0.0, np.inf])
_QRAY[3:6] /= np.linalg.norm(_QRAY[3:6])


@pytest.mark.slow
@pytest.mark.parametrize("analytic", [False, True])
def test_single_scattering_matches_nested_quadrature(orc, analytic):
    """positive kernels: delta tracking and CDF inversion (with exact shadow
    transmittance) both solve the single-scattering transfer equation"""
    params = _quadrature_scene()
    rho, albedo = 0.02, 0.9
    L_ref = _single_scattering_reference(orc, params, _QRAY, rho, albedo)
    spp = 40000 if not analytic else 20000
    L, Lv, _, _ = orc.render(params, _QRAY[None, :], spp, seed=8, rho=rho, multiple=False, albedo=albedo,
                             analytic=analytic)
    se = math.sqrt(Lv[0] / spp)
    assert abs(L[0] - L_ref) < 4 * se + 2e-4


@pytest.mark.slow
def test_zero_nee_matches_nested_quadrature(orc):
    """shadow rays traced against the low-pass level only (Zero-NEE, Sec. 4.5
    implementation details): the estimator converges to the transfer equation
    with the shadow transmittance of level 0, and differs from the full one"""
    params = _quadrature_scene(n_gabor=4)
    c, _ = orc.cells(params)
    assert np.all(c[:6] == 0) and np.all(c[6:] >= 9)
    rho, albedo = 0.03, 0.9
    L_ref = _single_scattering_reference(orc, params, _QRAY, rho, albedo, shadow_cells=0b111)
    L_full = _single_scattering_reference(orc, params, _QRAY, rho, albedo)
    spp = 40000
    L, Lv, _, _ = orc.render(params, _QRAY[None, :], spp, seed=9, rho=rho, multiple=False, albedo=albedo,
                             shadow_cells=0b111)
    se = math.sqrt(Lv[0] / spp)
    assert abs(L[0] - L_ref) < 4 * se + 2e-4
    assert abs(L_ref - L_full) > 8 * se


def test_shadow_cells_full_is_the_default(orc):
    params = gen.uniform_scene(64, 5)
    rays = gen.ortho_rays(8, 8)
    a = orc.render(params, rays, 16, seed=3, rho=0.01, multiple=False)
    b = orc.render(params, rays, 16, seed=3, rho=0.01, multiple=False, shadow_cells=orc.FULL_MASK)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_analytic_free_flight_distribution_positive_gaussian(orc):
    """CDF inversion by bisection: distances follow 1 - exp(-tau(0, t)) and
    the escape probability is exp(-tau) (Kolmogorov-Smirnov), weights 1"""
    params = _gaussian_prim()
    ray = np.array([[0.52, 0.47, -0.5, 0.0, 0.0, 1.0, 0.0, np.inf]])
    rho = 1.5 / orc.tau(params, ray, rho=1.0)[0][0]
    tau_tot = orc.tau(params, ray, rho=rho)[0][0]
    t, w = orc.free_flight(params, ray, 8000, seed=4, rho=rho, analytic=True)
    assert np.all(w == 1.0)
    t = t[0]
    col = t[np.isfinite(t)]
    esc = np.mean(~np.isfinite(t))
    assert abs(esc - math.exp(-tau_tot)) < 4 * math.sqrt(math.exp(-tau_tot) * (1 - math.exp(-tau_tot)) / len(t))
    ts = np.sort(col)[:: max(1, len(col) // 2000)]
    rr = np.repeat(ray, len(ts), axis=0)
    rr[:, 7] = ts
    F = 1.0 - np.exp(-orc.tau(params, rr, rho=rho)[0])
    ks = st.kstest(F / (1.0 - math.exp(-tau_tot)), "uniform")
    assert ks.pvalue > 1e-3
    # each distance solves tau(0, t) = -log(1 - xi) to the bisection tolerance:
    # the optical depth up to the sampled point is an Exp(1) variate
    # truncated at tau_tot, i.e. F above is uniform (checked) and every t lies
    # where the density is non-zero
    assert np.all(np.diff(F) >= 0)


def test_analytic_furnace_positive_density_is_exact(orc):
    params = gen.uniform_scene(64, 5).astype(np.float64)
    params[:, 10:14] = 0.0
    rays = gen.ortho_rays(16, 16)
    L, _, T, _ = orc.render(params, rays, 8, seed=1, rho=0.05, multiple=True, max_scatter=100000, albedo=1.0,
                            hg_g=0.3, analytic=True)
    assert np.all(L == 1.0)
    tau, _, _ = orc.tau(params, rays, rho=0.05)
    assert np.allclose(T, np.exp(-tau), rtol=1e-12, atol=0)


@pytest.mark.slow
def test_analytic_and_delta_tracking_agree_on_positive_field(orc):
    """multiple scattering on a positive field: both free-flight samplers are
    unbiased for the same transfer equation"""
    params = gen.uniform_scene(64, 5).astype(np.float64)
    params[:, 10:14] = 0.0
    rays = gen.ortho_rays(16, 16)[::9]
    spp = 3000
    a = orc.render(params, rays, spp, seed=5, rho=0.05, multiple=True, albedo=0.8, hg_g=0.3, analytic=True)
    d = orc.render(params, rays, spp, seed=6, rho=0.05, multiple=True, albedo=0.8, hg_g=0.3)
    pooled, worst = _pooled(a[0], d[0], np.sqrt((a[1] + d[1]) / spp))
    assert pooled < 3.0 and worst < 4.5
