"""Pins of the oracle's analytic optical-depth gradients: FP64 central
differences (h = 1e-6) of the oracle's own optical depth (itself pinned by
quadrature), and exact invariances (quaternion scale, joint translation of
primitives and rays, linearity in alpha)."""
import numpy as np
import pytest

import gen

H = 1e-6


def _loss_fd(orc, params, rays, wts, i, j, rho, r):
    p = params.astype(np.float64).copy()
    p[i, j] += H
    up = orc.tau(p, rays, rho=rho, r=r)[0] @ wts
    p[i, j] -= 2 * H
    dn = orc.tau(p, rays, rho=rho, r=r)[0] @ wts
    return (up - dn) / (2 * H)


def _scene_and_rays(n=64, seed=0):
    params = gen.uniform_scene(n, seed, smin=0.03, smax=0.12).astype(np.float64)
    g = np.random.default_rng(seed + 100)
    rays = []
    for k in range(160):
        p = params[k % n]
        d = g.standard_normal(3)
        d /= np.linalg.norm(d)
        o = p[0:3] + g.standard_normal(3) * 0.08 - 0.6 * d
        lo = g.uniform(0.0, 0.5)
        rays.append(np.r_[o, d, lo, lo + g.uniform(0.2, 1.2)])
    return params, np.asarray(rays), g.standard_normal(160)


@pytest.mark.parametrize("r", [3.0, 12.0])
def test_gradient_matches_central_differences(orc, r):
    params, rays, wts = _scene_and_rays()
    rho = 0.02
    if r == 3.0:
        # the chord-end derivative diverges like (r^2 - h^2)^-1/2 at tangency:
        # drop rays that pass within 0.02 whitened units of some tangency
        near = np.zeros(len(rays), bool)
        for k, ray in enumerate(rays):
            for p in params:
                out = orc.segment_integral(p, ray, r)
                if out[1] and abs(np.sqrt(out[2]) - r) < 0.02:
                    near[k] = True
        rays, wts = rays[~near], wts[~near]
        assert len(rays) > 120
    an = orc.tau_grad(params, rays, wts, rho=rho, r=r)
    g = np.random.default_rng(3)
    prims = g.choice(len(params), 12, replace=False)
    groups = {"mu": range(0, 3), "q": range(3, 7), "s": range(7, 10), "f": range(10, 13), "phi": [13],
              "alpha": [14]}
    for name, cols in groups.items():
        scale = np.abs(an[:, list(cols)]).max() + 1e-300
        for i in prims:
            for j in cols:
                fd = _loss_fd(orc, params, rays, wts, i, j, rho, r)
                assert abs(fd - an[i, j]) <= 1e-6 * scale + 1e-9 * abs(an[i, j]), (name, i, j, fd, an[i, j])


def test_gradient_invariants(orc):
    params, rays, wts = _scene_and_rays(48, 5)
    rho = 0.02
    an = orc.tau_grad(params, rays, wts, rho=rho)
    # scale invariance of the quaternion: dtau/dq . q = 0
    dots = np.einsum("ij,ij->i", an[:, 3:7], params[:, 3:7])
    assert np.max(np.abs(dots)) <= 1e-10 * np.abs(an[:, 3:7]).max()
    # d/dalpha_i = tau_i / alpha_i: sum_i alpha_i dL/dalpha_i = L (tau linear in alpha)
    L = orc.tau(params, rays, rho=rho)[0] @ wts
    assert abs(np.sum(an[:, 14] * params[:, 14]) - L) <= 1e-10 * (1 + abs(L))
    # translation: moving every mean by e equals moving every ray origin by -e
    e_grad = an[:, 0:3].sum(axis=0)
    for a in range(3):
        r2 = rays.copy()
        r2[:, a] += 1e-6
        up = orc.tau(params, r2, rho=rho)[0] @ wts
        r2[:, a] -= 2e-6
        dn = orc.tau(params, r2, rho=rho)[0] @ wts
        d_origin = (up - dn) / 2e-6
        assert abs(e_grad[a] + d_origin) <= 1e-6 * np.abs(an[:, 0:3]).sum()
