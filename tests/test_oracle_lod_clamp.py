"""Pins of the continuous LOD cutoff (supplementary "LOD Selection": the
Nyquist limit R / (4 d tan(phi/2)) cycles per unit at distance d) and of
adaptive clamping of the support (Sec. 4.4, in its conservative form).

* LOD: the oracle's optical depth under the cutoff equals the sum, over the
  primitives a brute-force numpy selection keeps, of their single-primitive
  optical depths; no cutoff and an infinite cutoff both give the full depth.
* Clamping: for unit-speed rays the optical depth of every primitive moves by
  at most eps (the error bound the clamped radius is derived from), the bound
  is approached (it is not vacuous), eps = 0 changes nothing, a huge eps
  removes everything, and the density vanishes beyond the clamped radius.
"""
import math

import numpy as np
import pytest

import gen


def _sigma_inv(p):
    w, x, y, z = p[3:7] / np.linalg.norm(p[3:7])
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    return R @ np.diag(1.0 / p[7:10] ** 2) @ R.T


def lod_k_of(width, fov_y_deg):
    """lod_k = R / (4 tan(phi/2)): |f| d <= lod_k keeps a primitive at distance d"""
    return width / (4.0 * math.tan(math.radians(fov_y_deg) / 2))


def test_lod_cutoff_brute_force(orc):
    params = gen.uniform_scene(96, 2).astype(np.float64)
    rays = gen.pinhole_rays(8, 8, eye=(0.5, 0.5, -0.6))[::3].astype(np.float64)
    K = lod_k_of(32, 40.0)
    rho = 0.02
    got, _, _ = orc.tau(params, rays, rho=rho, lod_k=K)
    full, _, _ = orc.tau(params, rays, rho=rho)
    assert np.array_equal(orc.tau(params, rays, rho=rho, lod_k=0.0)[0], full)
    assert np.array_equal(orc.tau(params, rays, rho=rho, lod_k=1e30)[0], full)
    per = np.stack([orc.tau(params[i:i + 1], rays, rho=rho)[0] for i in range(len(params))], axis=1)
    ref = np.zeros(len(rays))
    n_drop = 0
    for k, ray in enumerate(rays):
        o, v = ray[0:3], ray[3:6]
        for i, p in enumerate(params):
            A = _sigma_inv(p)
            tc = -((o - p[0:3]) @ A @ v) / (v @ A @ v)
            keep = tc <= 0 or np.linalg.norm(p[10:13]) * tc * np.linalg.norm(v) <= K
            if keep:
                ref[k] += per[k, i]
            elif per[k, i] != 0.0:
                n_drop += 1
    assert n_drop >= 20
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-15)
    assert np.any(np.abs(got - full) > 1e-6)


def test_lod_cutoff_keeps_low_frequencies(orc):
    params = gen.uniform_scene(64, 3).astype(np.float64)
    params[::2, 10:13] = 0.0  # half the primitives at zero frequency
    rays = gen.ortho_rays(8, 8).astype(np.float64)
    tiny = orc.tau(params, rays, rho=0.02, lod_k=1e-9)[0]
    low = orc.tau(params[::2], rays, rho=0.02)[0]
    assert np.allclose(tiny, low, rtol=1e-12, atol=1e-15)


def _unit_rays(n, seed):
    r = gen.random_rays(n, seed).astype(np.float64)
    r[:, 6], r[:, 7] = -5.0, 5.0  # whole chords
    return r


@pytest.mark.parametrize("eps", [0.2, 1.0])
def test_clamping_error_bound(orc, eps):
    params = gen.uniform_scene(64, 4).astype(np.float64)
    rho = 0.05
    rays = _unit_rays(600, 5)
    radii = orc.clamp_radii(params, rho, eps)
    assert np.any(radii < 3.0) and np.any(radii > 1.0)
    worst = 0.0
    for i in range(len(params)):
        a = orc.tau(params[i:i + 1], rays, rho=rho)[0]
        b = orc.tau(params[i:i + 1], rays, rho=rho, clamp_eps=eps)[0]
        err = np.abs(a - b)
        assert np.all(err <= eps * (1 + 1e-9))
        if radii[i] == 3.0:
            assert np.array_equal(a, b)
        worst = max(worst, err.max())
    assert worst > 0.02 * eps  # the bound is approached, not vacuous


def test_clamping_limits(orc):
    params = gen.uniform_scene(64, 4).astype(np.float64)
    rays = _unit_rays(100, 6)
    full = orc.tau(params, rays, rho=0.05)[0]
    assert np.array_equal(orc.tau(params, rays, rho=0.05, clamp_eps=0.0)[0], full)
    assert np.all(orc.tau(params, rays, rho=0.05, clamp_eps=1e30)[0] == 0.0)
    assert np.all(orc.clamp_radii(params, 0.05, 1e30) == 0.0)


def test_clamped_density_support(orc):
    params = gen.uniform_scene(32, 7).astype(np.float64)
    rho, eps = 0.05, 0.5
    radii = orc.clamp_radii(params, rho, eps)
    g = np.random.default_rng(1)
    for i in np.where((radii > 0.5) & (radii < 2.9))[0][:6]:
        p = params[i:i + 1]
        A = _sigma_inv(p[0])
        d = g.standard_normal((400, 3))
        # points at Mahalanobis radius just inside / outside the clamped radius
        L = np.linalg.cholesky(np.linalg.inv(A))
        u = d / np.linalg.norm(d, axis=1, keepdims=True)
        inside = p[0, 0:3] + (0.98 * radii[i]) * (u @ L.T)
        outside = p[0, 0:3] + (1.02 * radii[i]) * (u @ L.T)
        assert np.all(orc.kappa(p, outside, rho=rho, clamp_eps=eps) == 0.0)
        assert np.all(orc.kappa(p, inside, rho=rho, clamp_eps=eps) == orc.kappa(p, inside, rho=rho))


def test_clamped_lbvh_boxes(orc):
    params = gen.uniform_scene(200, 8).astype(np.float64)
    rho, eps = 0.05, 0.5
    full = orc.lbvh(params)
    cl = orc.lbvh(params, rho=rho, clamp_eps=eps)
    assert np.array_equal(full["perm"], cl["perm"]) and np.array_equal(full["left"], cl["left"])
    n = len(params)
    radii = orc.clamp_radii(params, rho, eps)
    for j in range(n):
        i = cl["perm"][j]
        fb, cb = full["aabb"][n - 1 + j], cl["aabb"][n - 1 + j]
        mu = params[i, 0:3]
        # box half-extents scale with the radius (outward rounding aside)
        ef = (fb[3:] - fb[:3]) / 2
        ec = (cb[3:] - cb[:3]) / 2
        assert np.allclose(ec, ef * radii[i] / 3.0, rtol=1e-5, atol=1e-6)
        assert np.all(cb[:3] <= mu) and np.all(cb[3:] >= mu)
