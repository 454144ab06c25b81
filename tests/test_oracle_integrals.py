"""Pins of the oracle's per-primitive line integral and optical depth.

* full-line closed form: the Sec. 4.4 whitened form (K, b, c, d, Omega) and the
  Appendix A boxed form (a, beta, gamma, B, delta) are two derivations; both
  written out here in numpy must equal the oracle's segment integral with the
  truncation pushed out to r = 40;
* zero frequency: the segment integral reduces to a real-erf expression;
* adaptive quadrature of the kernel over the clipped chord (Sec. 3, Eq. 2);
* the mass of one kernel, from its Fourier transform at k = 0 (Appendix C):
  exp(-omega^T Sigma omega / 2);
* invariants of optical depth (phase shift, weight linearity, reversal,
  direction scaling, translation, mask additivity).
"""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

import gen

TWO_PI = 2.0 * math.pi


def frame(p):
    """independent numpy construction of mu, Sigma, omega from one record"""
    p = np.asarray(p, np.float64)
    mu = p[0:3]
    w, x, y, z = p[3:7] / np.linalg.norm(p[3:7])
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    Sig = R @ np.diag(p[7:10] ** 2) @ R.T
    return mu, Sig, R, TWO_PI * p[10:13], p[13], p[14]


def boxed_full_line(p, ray):
    """Appendix A boxed infinite-domain form with a, beta, gamma, B, delta (phase added)."""
    mu, Sig, _, om, phi, _ = frame(p)
    o, v = ray[0:3].astype(np.float64), ray[3:6].astype(np.float64)
    Si = np.linalg.inv(Sig)
    d = o - mu
    a, beta, gam = v @ Si @ v, v @ Si @ d, d @ Si @ d
    B, delta = om @ v, om @ d
    pref = 1.0 / math.sqrt(8 * math.pi ** 3 * np.linalg.det(Sig))
    return (pref * math.sqrt(TWO_PI / a) * math.exp(-0.5 * (gam - beta * beta / a)) * math.exp(-B * B / (2 * a))
            * math.cos(delta - beta * B / a + phi))


def whitened_full_line(p, ray):
    """Sec. 4.4 full-line form with W = S^-1 R^T and k_W = S R^T omega."""
    mu, Sig, R, om, phi, _ = frame(p)
    s = np.asarray(p[7:10], np.float64)
    W = np.diag(1 / s) @ R.T
    kW = np.diag(s) @ R.T @ om
    o, v = ray[0:3].astype(np.float64), ray[3:6].astype(np.float64)
    pW = W @ (o - mu)
    vW = W @ v / np.linalg.norm(W @ v)
    b, c = pW @ vW, pW @ pW
    Om, d = kW @ vW, kW @ pW
    K = 1.0 / (TWO_PI * math.sqrt(np.linalg.det(Sig)) * np.linalg.norm(W @ v))
    return K * math.exp(-0.5 * (c - b * b + Om * Om)) * math.cos(d - Om * b + phi)


@pytest.fixture(scope="module")
def tiny():
    return gen.uniform_scene(256, 0)


def _aimed_rays(params, k, seed, spread=1.5):
    """rays passing near primitive means, with random directions"""
    g = np.random.default_rng(seed)
    out = []
    for i in range(k):
        p = params[i % len(params)]
        d = g.standard_normal(3)
        d /= np.linalg.norm(d)
        off = g.standard_normal(3) * p[7:10].mean() * spread
        o = p[0:3] + off - 0.7 * d
        out.append(np.concatenate([o, d, [-np.inf, np.inf]]))
    return np.asarray(out)


def test_full_line_closed_forms_agree(orc, tiny):
    rays = _aimed_rays(tiny, 200, 1)
    for k, ray in enumerate(rays):
        p = tiny[k % len(tiny)]
        got = orc.segment_integral(p, ray, r=40.0)[0]
        ref1 = boxed_full_line(p, ray)
        ref2 = whitened_full_line(p, ray)
        scale = abs(boxed_full_line(np.r_[p[:10], 0, 0, 0, 0, p[14]], ray))  # envelope scale
        assert abs(ref1 - ref2) <= 1e-10 * scale
        assert abs(got - ref1) <= 1e-10 * scale


def test_zero_frequency_reduces_to_real_erf(orc, tiny):
    rays = _aimed_rays(tiny, 100, 2)
    g = np.random.default_rng(3)
    rays[:, 6] = g.uniform(-1, 0.5, len(rays))
    rays[:, 7] = rays[:, 6] + g.uniform(0.05, 1.5, len(rays))
    for k, ray in enumerate(rays):
        p = tiny[k % len(tiny)].astype(np.float64).copy()
        p[10:13] = 0.0
        out = orc.segment_integral(p, ray)
        mu, Sig, _, _, phi, _ = frame(p)
        Si = np.linalg.inv(Sig)
        o, v = ray[0:3], ray[3:6]
        d = o - mu
        a, beta, gam = v @ Si @ v, v @ Si @ d, d @ Si @ d
        disc = beta * beta - a * (gam - 9.0)
        if disc <= 0:
            assert out[1] == 0
            continue
        tin, tout = (-beta - math.sqrt(disc)) / a, (-beta + math.sqrt(disc)) / a
        ta, tb = max(ray[6], tin), min(ray[7], tout)
        if ta >= tb:
            assert out[1] == 0
            continue
        n = math.sqrt(a)
        tc = -beta / a
        h2 = gam - beta * beta / a
        K = 1.0 / (TWO_PI * math.sqrt(np.linalg.det(Sig)) * n)
        ref = K / 2 * math.exp(-0.5 * h2) * math.cos(phi) * (sp.erf(n * (tb - tc) / math.sqrt(2))
                                                            - sp.erf(n * (ta - tc) / math.sqrt(2)))
        assert abs(out[0] - ref) <= 1e-12 * K


def test_segment_integral_matches_quadrature(orc, tiny):
    rays = np.concatenate([gen.random_rays(48, 3), _aimed_rays(tiny, 150, 4)])
    g = np.random.default_rng(5)
    rays[48:, 6] = g.uniform(-1.0, 0.7, 150)
    rays[48:, 7] = rays[48:, 6] + g.uniform(0.0, 1.0, 150)
    checked = 0
    for k, ray in enumerate(rays):
        idx = range(256) if k < 48 else [(k - 48) % 256]
        for i in idx:
            p = tiny[i]
            out = orc.segment_integral(p, ray)
            mu, Sig, _, om, phi, _ = frame(p)
            Si = np.linalg.inv(Sig)
            o, v = ray[0:3].astype(np.float64), ray[3:6].astype(np.float64)
            d = o - mu
            a, beta, gam = v @ Si @ v, v @ Si @ d, d @ Si @ d
            disc = beta * beta - a * (gam - 9.0)
            if disc <= 0:
                assert out[1] == 0
                continue
            tin, tout = (-beta - math.sqrt(disc)) / a, (-beta + math.sqrt(disc)) / a
            ta, tb = max(ray[6], tin), min(ray[7], tout)
            if ta >= tb:
                assert out[1] == 0
                continue
            cn = 1.0 / math.sqrt((TWO_PI) ** 3 * np.linalg.det(Sig))
            f = lambda t: cn * math.exp(-0.5 * ((d + t * v) @ Si @ (d + t * v))) * math.cos(om @ (d + t * v) + phi)
            e = lambda t: cn * math.exp(-0.5 * ((d + t * v) @ Si @ (d + t * v)))
            val = si.quad(f, ta, tb, limit=400, epsabs=0, epsrel=1e-12)[0]
            env = si.quad(e, ta, tb, epsabs=0, epsrel=1e-12)[0]
            assert abs(val - out[0]) <= 1e-9 * env
            checked += 1
    assert checked > 200


def test_mass_from_fourier_transform_at_zero(orc):
    """Sum of full-line integrals over a fine grid of parallel rays integrates
    the kernel over space: must equal exp(-omega^T Sigma omega / 2)."""
    g = np.random.default_rng(7)
    for trial in range(4):
        p = np.zeros(15)
        p[0:3] = 0.5
        q = g.standard_normal(4)
        p[3:7] = q / np.linalg.norm(q)
        p[7:10] = g.uniform(0.05, 0.1, 3)
        p[10:13] = g.standard_normal(3) * 2.0
        p[13] = g.uniform(0, TWO_PI) if trial else 0.0
        p[14] = 1.0
        _, Sig, _, om, phi, _ = frame(p)
        h = 0.01
        xs = np.arange(-0.5, 1.5, h) + h / 2
        X, Y = np.meshgrid(xs, xs, indexing="ij")
        rays = np.zeros((X.size, 8))
        rays[:, 0], rays[:, 1], rays[:, 2] = X.ravel(), Y.ravel(), -2.0
        rays[:, 5] = 1.0
        rays[:, 6], rays[:, 7] = -np.inf, np.inf
        tau, _, _ = orc.tau(p[None, :], rays, r=40.0)
        mass = tau.sum() * h * h
        ref = math.exp(-0.5 * om @ Sig @ om) * math.cos(phi)
        assert abs(mass - ref) < 1e-9


@pytest.fixture(scope="module")
def tiny_rays():
    return gen.ortho_rays(64, 64)[::37]


def test_tau_ray_matches_quadrature_of_density(orc, tiny):
    """tau = int kappa(x(t)) dt (Sec. 3, Eqs. 1-2) by 60-point Gauss-Legendre on
    every piece between consecutive chord ends (the integrand is smooth there)."""
    rays = gen.ortho_rays(64, 64)[::101]
    rho = 0.0165
    tau, _, _ = orc.tau(tiny, rays, rho=rho)
    xg, wg = np.polynomial.legendre.leggauss(60)
    nonzero = 0
    for k, ray in enumerate(rays):
        brk = []
        o, v = ray[0:3].astype(np.float64), ray[3:6].astype(np.float64)
        for p in tiny:
            mu, Sig, _, _, _, _ = frame(p)
            Si = np.linalg.inv(Sig)
            d = o - mu
            a, beta, gam = v @ Si @ v, v @ Si @ d, d @ Si @ d
            disc = beta * beta - a * (gam - 9.0)
            if disc > 0:
                brk += [(-beta - math.sqrt(disc)) / a, (-beta + math.sqrt(disc)) / a]
        if not brk:
            assert tau[k] == 0.0
            continue
        edges = [0.0] + sorted(b for b in brk if b > 0)
        ts, ws = [], []
        for a_, b_ in zip(edges[:-1], edges[1:]):
            if b_ > a_:
                ts.append(0.5 * (a_ + b_) + 0.5 * (b_ - a_) * xg)
                ws.append(0.5 * (b_ - a_) * wg)
        ts, ws = np.concatenate(ts), np.concatenate(ws)
        total = np.sum(ws * orc.kappa(tiny, o[None, :] + ts[:, None] * v[None, :], rho=rho))
        assert abs(total - tau[k]) < 1e-12 * (1.0 + abs(tau[k]))
        nonzero += 1
    assert nonzero > 20


def test_tau_invariants(orc, tiny, tiny_rays):
    rho = 0.0165
    base, absum, hits = orc.tau(tiny, tiny_rays, rho=rho)
    assert hits.sum() > 0
    # empty mask -> tau = 0 ; full cell mask == unmasked
    t0, _, h0 = orc.tau(tiny, tiny_rays, rho=rho, cells=0)
    assert np.all(t0 == 0) and np.all(h0 == 0)
    # disjoint cell masks add up to the full mask
    parts = sum(orc.tau(tiny, tiny_rays, rho=rho, cells=1 << c)[0] for c in range(12))
    assert np.allclose(parts, base, rtol=0, atol=1e-12 * (1 + absum.max()))
    # phase + pi negates, phase + 2 pi is the identity
    p = tiny.astype(np.float64).copy()
    p[:, 13] += math.pi
    assert np.allclose(orc.tau(p, tiny_rays, rho=rho)[0], -base, atol=1e-12)
    p[:, 13] += math.pi
    assert np.allclose(orc.tau(p, tiny_rays, rho=rho)[0], base, atol=1e-12)
    # linear in alpha
    p = tiny.astype(np.float64).copy()
    p[:, 14] *= 2.5
    assert np.allclose(orc.tau(p, tiny_rays, rho=rho)[0], 2.5 * base, atol=1e-12)
    # direction scaling: v -> c v, t -> t / c scales tau by 1 / c
    r2 = tiny_rays.astype(np.float64).copy()
    r2[:, 3:6] *= 3.0
    assert np.allclose(orc.tau(tiny, r2, rho=rho)[0], base / 3.0, atol=1e-12)
    # reversal on a finite window [a, b]
    r3 = tiny_rays.astype(np.float64).copy()
    r3[:, 6], r3[:, 7] = 0.4, 2.2
    fwd = orc.tau(tiny, r3, rho=rho)[0]
    r4 = r3.copy()
    r4[:, 0:3] = r3[:, 0:3] + (0.4 + 2.2) * r3[:, 3:6]
    r4[:, 3:6] = -r3[:, 3:6]
    assert np.allclose(orc.tau(tiny, r4, rho=rho)[0], fwd, atol=1e-10)
    # rigid translation of scene and rays
    p = tiny.astype(np.float64).copy()
    p[:, 0:3] += np.array([0.25, -0.5, 0.125])
    r5 = tiny_rays.astype(np.float64).copy()
    r5[:, 0:3] += np.array([0.25, -0.5, 0.125])
    assert np.allclose(orc.tau(p, r5, rho=rho)[0], base, atol=1e-9)
