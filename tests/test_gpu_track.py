"""GPU parity of the stochastic path against the FP64 oracle: point density
and majorant validity, ratio-tracking transmittance (mean = exp(-tau)),
single / multiple scattering (GPU and oracle estimates agree in mean within
3 combined standard errors), furnace, exact stochastic-mask expectation, and
bitwise determinism / batch independence."""
import math

import numpy as np
import pytest
import torch

import gen
import oracle
from gen import workloads as W
from gpu_util import dev, host, require_gpu
from strategy_tables import enumerate_outcomes, expected_T

pytestmark = pytest.mark.gpu


def _pooled(a, b, se):
    se = se + 1e-15
    return abs(np.sum(a - b)) / np.sqrt(np.sum(se ** 2)), np.max(np.abs(a - b) / se)


def _check_ratio(Tm, Tv, tau, spp, min_ok):
    """Ratio-tracking means against exp(-tau).  Deep rays (spp exp(-tau) < 5)
    are products of many factors whose mean comes from rare samples that a
    run of this length rarely draws, so their sample variance is no standard
    error: they get a bound relative to exp(-tau) instead (within five
    standard errors plus ten times exp(-tau), and not negative beyond five
    standard errors); the closed-form transmittance of the CDF-inversion
    render pins deep rays exactly (test_gpu_strategies.py)."""
    T = np.exp(-tau)
    ok = spp * T >= 5.0
    assert ok.sum() >= min_ok
    pooled, worst = _pooled(Tm[ok], T[ok], np.sqrt(Tv[ok] / spp))
    assert pooled < 3.0 and worst < 5.0
    se = np.sqrt(Tv[~ok] / spp)
    assert np.all(np.abs(Tm[~ok] - T[~ok]) <= 5.0 * se + 10.0 * T[~ok])


def test_density_and_majorant():
    gf = require_gpu()
    params, rho = W.scene("tiny256"), W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho, majorant_grid=64)
    g = np.random.default_rng(0)
    pts = np.concatenate([params[g.choice(256, 3000), 0:3] + g.normal(0, 0.05, (3000, 3)),
                          g.uniform(-0.1, 1.1, (1000, 3))]).astype(np.float32)
    kap, kb = gf.gf_density(scene, dev(pts))
    kap, kb = host(kap), host(kb)
    ref = oracle.kappa(params, pts, rho=rho)
    env_params = params.astype(np.float64).copy()
    env_params[:, 10:14] = 0.0
    env_params[:, 14] = np.abs(env_params[:, 14])
    env = oracle.kappa(env_params, pts, rho=rho)  # rho sum |alpha| c exp(-M/2) >= |kappa|
    assert np.all(np.abs(kap - ref) <= 2e-5 * env + 1e-6)
    assert np.all(kb >= np.abs(ref) * (1 - 1e-5))
    assert np.all(kb >= env * (1 - 1e-4))


def test_ratio_tracking_mean_is_exp_minus_tau():
    gf = require_gpu()
    params, rays, rho = W.scene("tiny256"), W.rays("tiny256"), W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    sub = rays[::8]
    # signed densities make the per-sample product heavy-tailed (each factor
    # lies in [0, 2]); the sample variance needs many samples to be a
    # reliable standard error
    spp = 16384
    Tm, Tv = gf.gf_transmittance_ratio(scene, dev(sub), spp, seed=11)
    Tm, Tv = host(Tm), host(Tv)
    tau, _, hits = oracle.tau(params, sub, rho=rho)
    _check_ratio(Tm, Tv, tau, spp, min_ok=450)
    assert np.all(Tm[hits == 0] == 1.0)
    # the workload's own output: 16 samples over the whole 64x64 frame
    T16, _ = gf.gf_transmittance_ratio(scene, dev(rays), 16, seed=1, image_width=64)
    assert np.all(np.isfinite(host(T16)))


def test_ratio_tracking_masks():
    gf = require_gpu()
    params, rays, rho = W.scene("tiny256"), W.rays("tiny256")[::16], W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    spp = 4096
    for cells in (gf.gf_mask_lod_cells(2), 0):
        Tm, Tv = gf.gf_transmittance_ratio(scene, dev(rays), spp, seed=3, mask=gf.make_mask(cells))
        tau, _, _ = oracle.tau(params, rays, rho=rho, cells=cells)
        _check_ratio(host(Tm), host(Tv), tau, spp, min_ok=200)


def _render_pair(params, rays, rho, spp_gpu, spp_orc, **kw):
    gf = require_gpu()
    scene = gf.Scene(dev(params), rho=rho)
    d = gf.render_desc(spp=spp_gpu, seed=5, **kw)
    Lm, Lv, Tm, Tv = (host(x) for x in gf.gf_render_rays(scene, dev(rays), d))
    oL, oLv, oT, oTv = oracle.render(params, rays, spp_orc, seed=9, rho=rho, **kw)
    return (Lm, Lv / spp_gpu), (oL, oLv / spp_orc), (Tm, Tv / spp_gpu), (oT, oTv / spp_orc)


def test_single_scattering_matches_oracle_in_mean():
    params, rays, rho = W.scene("tiny256"), W.rays("tiny256")[::32], W.rho("tiny256")
    (g, gv), (o, ov), (gt, gtv), (ot, otv) = _render_pair(params, rays, rho, 4096, 1024, multiple=False,
                                                          albedo=0.9)
    pooled, worst = _pooled(g, o, np.sqrt(gv + ov))
    assert pooled < 3.0 and worst < 5.0
    pooled, worst = _pooled(gt, ot, np.sqrt(gtv + otv))
    assert pooled < 3.0 and worst < 5.0


def test_multiple_scattering_matches_oracle_in_mean():
    params, rays = W.scene("tiny256"), W.rays("tiny256")[::64]
    rho = 0.5 * W.rho("tiny256")
    (g, gv), (o, ov), _, _ = _render_pair(params, rays, rho, 2048, 512, multiple=True, albedo=0.9, hg_g=0.3,
                                          max_scatter=16)
    pooled, worst = _pooled(g, o, np.sqrt(gv + ov))
    assert pooled < 3.0 and worst < 5.0


def test_furnace_positive_density_exact():
    gf = require_gpu()
    params = gen.uniform_scene(64, 5).astype(np.float32)
    params[:, 10:14] = 0.0
    scene = gf.Scene(dev(params), rho=0.05)
    rays = gen.ortho_rays(16, 16)
    d = gf.render_desc(spp=8, multiple=True, max_scatter=1 << 30, albedo=1.0, hg_g=0.3, seed=1)
    L, _, _, _ = gf.gf_render_rays(scene, dev(rays), d)
    assert torch.all(L == 1.0)


def test_stochastic_primary_transmittance_exact_expectation():
    gf = require_gpu()
    params = gen.uniform_scene(128, 3)
    params[:, 10:13] *= 0.2
    rho = 0.004
    rays = gen.random_rays(48, 12)
    scene = gf.Scene(dev(params), rho=rho)
    spp = 20000
    d = gf.render_desc(spp=spp, multiple=True, albedo=0.9, hg_g=0.3, stochastic=True, seed=21, bin="mixture")
    _, _, Tm, Tv = (host(x) for x in gf.gf_render_rays(scene, dev(rays), d))
    med = oracle.cell_medians(params)
    tcs = np.stack([oracle.tau(params, rays, rho=rho, cells=1 << c)[0] for c in range(12)], axis=1)
    exact, keep = [], []
    for ray, tc in zip(rays, tcs):
        out = enumerate_outcomes("uniform_cv", "mixture", med, ray[3:6])
        exact.append(expected_T(out, tc))
        keep.append(max(abs(float(np.dot(w, tc))) for _, w in out) < 0.6)
    exact, keep = np.array(exact), np.array(keep)
    pooled, worst = _pooled(Tm[keep], exact[keep], np.sqrt(Tv[keep] / spp))
    assert pooled < 3.0 and worst < 5.0


def test_render_deterministic_and_batch_independent():
    gf = require_gpu()
    params, rho = W.scene("tiny256"), W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    rays = dev(gen.pinhole_rays(64, 64))
    d = gf.render_desc(spp=2, multiple=True, albedo=0.9, hg_g=0.3, stochastic=True, seed=7)
    a = gf.gf_render_rays(scene, rays, d, image_width=64)[0]
    b = gf.gf_render_rays(scene, rays, d, image_width=0)[0]
    assert torch.equal(a, b)
    # a ray's result depends only on its own index in the launch: rays
    # 1000..1099 kept at their indices, every other ray replaced (reversed
    # order, a different camera), give the same bits
    other = dev(gen.pinhole_rays(64, 64, eye=(1.9, 0.4, -0.8)))[torch.arange(4095, -1, -1, device="cuda")]
    other[1000:1100] = rays[1000:1100]
    c = gf.gf_render_rays(scene, other.contiguous(), d)[0]
    assert torch.equal(a[1000:1100], c[1000:1100])
    assert not torch.equal(a[:1000], c[:1000])
    assert torch.isfinite(a).all() and torch.isfinite(c).all()


def test_render_full_size_sampled_blob100k():
    """the benchmark's render launch (100k primitives, 512^2 pinhole, 8 spp,
    single scattering with closed-form shadow transmittance, 8x8 tiles whose
    shadow rays share a direction per sample and trace as packets),
    repeated with 8 seeds, checked in mean on a seeded sample of pixels (in
    distinct tiles) that the oracle renders one by one with ratio-tracked
    shadow rays"""
    gf = require_gpu()
    params, rays, rho = W.scene("blob100k"), W.rays("blob100k"), W.rho("blob100k")
    scene = gf.Scene(dev(params), rho=rho)
    drays = dev(rays)
    sub = W.pixel_subset(rays.shape[0], k=24, seed=17)
    tiles = (sub // 512 // 8) * 64 + (sub % 512) // 8
    assert len(set(tiles.tolist())) == len(sub)
    runs = 8
    Lsum, Lv_sum = np.zeros(len(sub)), np.zeros(len(sub))
    for seed in range(runs):
        d = gf.render_desc(spp=8, multiple=False, albedo=0.9, seed=1234 + seed, exact_shadow=True)
        L, Lv, _, _ = gf.gf_render_rays(scene, drays, d, image_width=512)
        Lsum += host(L)[sub]
        Lv_sum += host(Lv)[sub]
        print("launch", seed, "done", flush=True)
    g = Lsum / runs
    g_se2 = (Lv_sum / runs) / (8 * runs)
    spp_o = 256
    o, ov, _, _ = oracle.render(params, rays[sub], spp_o, seed=3, rho=rho, multiple=False, albedo=0.9)
    se = np.sqrt(g_se2 + ov / spp_o) + 1e-15
    pooled = abs(np.sum(g - o)) / np.sqrt(np.sum(se ** 2))
    worst = np.max(np.abs(g - o) / se)
    print("pooled %.2f worst %.2f" % (pooled, worst), flush=True)
    assert pooled < 3.0 and worst < 6.0


def _stochastic_expectation(params, rays, rho, level, bin):
    """E[T_hat] of the stochastic primary transmittance, summed exactly over
    the per-segment mask distribution (enumerated from the strategy tables
    with the oracle's cell medians and per-cell optical depths)."""
    med = oracle.cell_medians(params)
    tcs = np.stack([oracle.tau(params, rays, rho=rho, cells=1 << c)[0] for c in range(12)], axis=1)
    return np.array([expected_T(enumerate_outcomes(level, bin, med, ray[3:6]), tc) for ray, tc in zip(rays, tcs)])


def test_render_full_size_multiple_stochastic_blob1m():
    """1M primitives, 1024-wide frame, 4 spp, multiple scattering (HG 0.3,
    albedo 0.9, up to 16 bounces) with per-segment stochastic masks: a
    32-row band of the frame in its launch shape, then the primary
    transmittance of sampled pixels against its exact expectation over the
    mask distribution (oracle optical depths per cell)."""
    gf = require_gpu()
    params, rays, rho = W.scene("blob1m"), W.rays("blob1m"), W.rho("blob1m")
    scene = gf.Scene(dev(params), rho=rho)
    band = rays[496 * 1024:528 * 1024]
    d = gf.render_desc(spp=4, multiple=True, max_scatter=16, albedo=0.9, hg_g=0.3, stochastic=True, seed=41,
                       bin="mixture")
    L, Lv, T, Tv = (host(x) for x in gf.gf_render_rays(scene, dev(band), d, image_width=1024))
    print("band done: mean L %.4f, mean T %.4f" % (L.mean(), T.mean()), flush=True)
    assert np.all(np.isfinite(L)) and np.all(np.isfinite(T))
    assert np.all(np.isfinite(Lv)) and np.all(np.isfinite(Tv))
    # sampled pixels with many samples: a lane runs all samples of its ray,
    # so each pixel's ray is repeated (every copy has its own streams) and
    # the copies' 4-sample means are pooled
    sub = W.pixel_subset(band.shape[0], k=24, seed=23)
    rs = band[sub]
    copies = 512
    d = gf.render_desc(spp=4, multiple=True, max_scatter=16, albedo=0.9, hg_g=0.3, stochastic=True, seed=43,
                       bin="mixture")
    Lc, _, Tc, _ = (host(x) for x in gf.gf_render_rays(scene, dev(np.repeat(rs, copies, axis=0)), d))
    Tc = Tc.reshape(len(rs), copies)
    spp = 4 * copies
    Tm, Tv = Tc.mean(axis=1), Tc.var(axis=1, ddof=1) * 4
    print("sampled pixels done", flush=True)
    exact = _stochastic_expectation(params, rs, rho, "uniform_cv", "mixture")
    ok = spp * exact >= 5.0
    assert ok.sum() >= 8
    pooled, worst = _pooled(Tm[ok], exact[ok], np.sqrt(Tv[ok] / spp))
    print("primary T: pooled %.2f worst %.2f over %d pixels" % (pooled, worst, ok.sum()), flush=True)
    assert pooled < 3.0 and worst < 5.0
    se = np.sqrt(Tv[~ok] / spp)
    assert np.all(np.abs(Tm[~ok] - exact[~ok]) <= 5.0 * se + 10.0 * exact[~ok])
    # the workload's output, radiance, against the oracle's own render of
    # the same pixels with the same strategies (both Monte Carlo: in mean)
    Lc = Lc.reshape(len(rs), copies)
    gL, gLv = Lc.mean(axis=1), Lc.var(axis=1, ddof=1) * 4 / spp
    spp_o = 128
    oL, oLv, _, _ = oracle.render(params, rs, spp_o, seed=8, rho=rho, multiple=True, max_scatter=16, albedo=0.9,
                                  hg_g=0.3, stochastic=True, level="uniform_cv", bin="mixture")
    pooled, worst = _pooled(gL, oL, np.sqrt(gLv + oLv / spp_o))
    print("radiance: pooled %.2f worst %.2f" % (pooled, worst), flush=True)
    assert pooled < 3.0 and worst < 6.0


def test_render_edge_cases():
    """Rays that miss the scene or have an empty window escape with weight 1
    (L = L_env, T = 1, zero variance); an empty mask lets every ray escape;
    a one-ray launch and a ragged 7-ray launch give the same bits for the
    same ray."""
    gf = require_gpu()
    params, rho = W.scene("tiny256"), W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    rays = np.zeros((7, 8), np.float32)
    rays[0:3, 0:3] = [[3.0, 3.0, 3.0], [-2.0, 0.5, 0.5], [0.5, 0.5, 5.0]]  # outside, pointing away
    rays[0:3, 3:6] = [[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0], [0.0, 0.0, 1.0]]
    rays[0:3, 7] = np.inf
    rays[3:5, 0:3] = [[0.5, 0.5, 0.5], [0.3, 0.6, 0.4]]  # inside, empty window
    rays[3:5, 3:6] = [[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]]
    rays[3:5, 6] = rays[3:5, 7] = 0.25
    rays[5:7, 0:3] = [[0.5, 0.5, -1.0], [0.2, 0.7, -1.0]]  # through the volume
    rays[5:7, 5] = 1.0
    rays[5:7, 7] = np.inf
    for multiple in (False, True):
        d = gf.render_desc(spp=4, multiple=multiple, albedo=0.9, hg_g=0.3, seed=13)
        L, Lv, T, Tv = (host(x) for x in gf.gf_render_rays(scene, dev(rays), d))
        assert np.all(L[:5] == 1.0) and np.all(T[:5] == 1.0)
        assert np.all(Lv[:5] == 0.0) and np.all(Tv[:5] == 0.0)
        assert np.all(np.isfinite(L)) and np.all(np.isfinite(T))
        L1, _, T1, _ = (host(x) for x in gf.gf_render_rays(scene, dev(rays[6:7]), d))
        # the ray's streams are keyed by its index: index 6 in the ragged
        # launch is index 0 alone, so compare the launch with itself shifted
        shifted = np.concatenate([rays[6:7], rays[:6]])
        L2, _, T2, _ = (host(x) for x in gf.gf_render_rays(scene, dev(shifted), d))
        assert L1[0] == L2[0] and T1[0] == T2[0]
        d0 = gf.render_desc(spp=4, multiple=multiple, albedo=0.9, hg_g=0.3, seed=13, mask=gf.make_mask(0))
        L0, _, T0, _ = (host(x) for x in gf.gf_render_rays(scene, dev(rays), d0))
        assert np.all(L0 == 1.0) and np.all(T0 == 1.0)
