"""GPU parity of the render options against the FP64 oracle:

* the scene's per-cell median |k_W| against the oracle's medians;
* the stochastic primary transmittance under every strategy pair of the
  two Appendix B tables against its exact expectation, enumerated from the
  tables with the oracle's medians and per-cell optical depths;
* stochastic single / multiple scattering radiance against the oracle's
  render with the same strategies, in mean;
* renders of the 100k-primitive workload under the 1/2 band, 1/4 band and
  45-degree cone masks on sampled pixels, and the cone's primitive bits
  through ratio tracking and the render;
* Zero-NEE shadow rays (low-pass cells only), the continuous LOD cutoff;
* free flights by CDF inversion: exact primary transmittance, radiance in
  mean, the furnace;
* the camera render in a caller workspace and the rejection of invalid rays.

Stochastic checks: GPU and oracle estimates agree in mean, pooled over rays
within 3 combined standard errors, every ray within 5-6.
"""
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


def _small_scene(fscale=0.3, n=128, seed=3):
    params = gen.uniform_scene(n, seed)
    params[:, 10:13] *= fscale
    return params


def _positive(params):
    p = params.copy()
    p[:, 10:14] = 0.0
    return p


def test_cell_medians_match_oracle():
    gf = require_gpu()
    for name in ("tiny256", "blob100k"):
        params = W.scene(name)
        scene = gf.Scene(dev(params), rho=W.rho(name))
        got = np.array(scene.info().cell_median_kw[:], dtype=np.float64)
        ref = oracle.cell_medians(params)
        assert np.allclose(got, ref, rtol=2e-6, atol=1e-6), (name, got, ref)


PAIRS = [("uniform_cv", "importance"), ("uniform_cv", "uniform"), ("uniform_cv", "mixture"),
         ("uniform", "deterministic"), ("power", "importance"), ("power_cv", "threshold_uniform"),
         ("power_cv_accum", "uniform"), ("deterministic", "threshold"), ("deterministic", "importance")]


@pytest.mark.parametrize("level,bin", PAIRS)
def test_stochastic_primary_T_every_strategy(level, bin):
    """E[T_hat] of the camera segment under the pair's per-segment masks
    equals sum over the enumerated outcomes of p exp(-sum_c w_c tau_c)."""
    gf = require_gpu()
    params, rho = _small_scene(), 0.004
    rays = gen.random_rays(48, 12)
    beta, delta = (0.4 if "power" in level else 0.0), 0.6
    scene = gf.Scene(dev(params), rho=rho)
    spp = 16384
    d = gf.render_desc(spp=spp, multiple=True, albedo=0.9, hg_g=0.3, stochastic=True, seed=21, level=level,
                       bin=bin, beta=beta, delta=delta)
    _, _, Tm, Tv = (host(x) for x in gf.gf_render_rays(scene, dev(rays), d))
    med = oracle.cell_medians(params)
    tcs = np.stack([oracle.tau(params, rays, rho=rho, cells=1 << c)[0] for c in range(12)], axis=1)
    exact, keep = [], []
    for ray, tc in zip(rays, tcs):
        out = enumerate_outcomes(level, bin, med, ray[3:6], beta=beta, delta=delta)
        exact.append(expected_T(out, tc))
        keep.append(max(abs(float(np.dot(w, tc))) for _, w in out) < 0.8)
    exact, keep = np.array(exact), np.array(keep)
    assert keep.sum() >= 24
    pooled, worst = _pooled(Tm[keep], exact[keep], np.sqrt(Tv[keep] / spp))
    assert pooled < 3.0 and worst < 5.0, (pooled, worst)


@pytest.mark.parametrize("level,bin,multiple", [("uniform_cv", "importance", True), ("uniform_cv", "mixture", True),
                                                 ("power_cv", "uniform", False)])
def test_stochastic_radiance_matches_oracle(level, bin, multiple):
    gf = require_gpu()
    params, rays = W.scene("tiny256"), W.rays("tiny256")[::64]
    rho = 0.5 * W.rho("tiny256")
    kw = dict(multiple=multiple, albedo=0.9, hg_g=0.3 if multiple else 0.0, max_scatter=16, stochastic=True,
              level=level, bin=bin, beta=0.3 if "power" in level else 0.0)
    scene = gf.Scene(dev(params), rho=rho)
    spp = 4096
    g, gv, _, _ = (host(x) for x in gf.gf_render_rays(scene, dev(rays), gf.render_desc(spp=spp, seed=5, **kw)))
    spp_o = 1024
    o, ov, _, _ = oracle.render(params, rays, spp_o, seed=9, rho=rho, **kw)
    pooled, worst = _pooled(g, o, np.sqrt(gv / spp + ov / spp_o))
    assert pooled < 3.0 and worst < 5.0, (pooled, worst)


def _blob100k_masks(gf, scene, params):
    lod = [gf.gf_mask_lod_cells(k) for k in (1, 2, 3)]
    gbits = gf.gf_mask_cone(scene)
    obits = oracle.mask_cone(params)
    return [("half_band", gf.make_mask(lod[0]), dict(cells=lod[0])),
            ("quarter_band", gf.make_mask(lod[1]), dict(cells=lod[1])),
            ("eighth_band", gf.make_mask(lod[2]), dict(cells=lod[2])),
            ("cone45", gf.make_mask(gf.FULL_CELLS, gbits), dict(bits=obits))]


def test_masked_renders_blob100k_sampled():
    """The benchmark's render (100k Gabors, 512^2 pinhole camera, 8-spp
    single scattering) under the 1/2, 1/4 and 1/8 band (the serving
    workload's levels) and 45-degree cone masks: 24 sampled pixels, each
    ray repeated so that its copies pool many samples, against the oracle's
    render of the same pixels."""
    gf = require_gpu()
    params, rays, rho = W.scene("blob100k"), W.rays("blob100k"), W.rho("blob100k")
    scene = gf.Scene(dev(params), rho=rho)
    sub = W.pixel_subset(rays.shape[0], k=24, seed=31)
    rs = rays[sub]
    copies, spp = 64, 8
    for name, gmask, omask in _blob100k_masks(gf, scene, params):
        d = gf.render_desc(spp=spp, multiple=False, albedo=0.9, seed=77, mask=gmask)
        L, _, _, _ = (host(x) for x in gf.gf_render_rays(scene, dev(np.repeat(rs, copies, axis=0)), d))
        L = L.reshape(len(rs), copies)
        g, gv = L.mean(axis=1), L.var(axis=1, ddof=1) / copies
        spp_o = 256
        o, ov, _, _ = oracle.render(params, rs, spp_o, seed=3, rho=rho, multiple=False, albedo=0.9, **omask)
        pooled, worst = _pooled(g, o, np.sqrt(gv + ov / spp_o))
        print("%s: pooled %.2f worst %.2f" % (name, pooled, worst), flush=True)
        assert pooled < 3.0 and worst < 6.0, name


def test_cone_bits_through_ratio_and_render():
    """The cone's primitive bits (composed with the cells) reach the
    tracking kernels: ratio-tracking means against exp(-tau) of the oracle
    under the same bits, and the render against the oracle's render."""
    gf = require_gpu()
    params, rays, rho = W.scene("tiny256"), W.rays("tiny256")[::16], W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    gbits = gf.gf_mask_cone(scene, axis=(0.3, 0.2, 1.0), half_angle=0.6)
    obits = oracle.mask_cone(params, axis=(0.3, 0.2, 1.0), half_angle=0.6)
    assert np.array_equal(host(gbits).view(np.uint32), obits)
    cells = gf.gf_mask_lod_cells(1)
    m = gf.make_mask(cells, gbits)
    spp = 4096
    Tm, Tv = (host(x) for x in gf.gf_transmittance_ratio(scene, dev(rays), spp, seed=3, mask=m))
    tau, _, _ = oracle.tau(params, rays, rho=rho, cells=cells, bits=obits)
    T = np.exp(-tau)
    ok = spp * T >= 5.0
    assert ok.sum() >= 128
    pooled, worst = _pooled(Tm[ok], T[ok], np.sqrt(Tv[ok] / spp))
    assert pooled < 3.0 and worst < 5.0
    sr = rays[::4]
    L, Lv, _, _ = (host(x) for x in gf.gf_render_rays(scene, dev(sr), gf.render_desc(spp=spp, seed=5, mask=m)))
    o, ov, _, _ = oracle.render(params, sr, 1024, seed=9, rho=rho, cells=cells, bits=obits)
    pooled, worst = _pooled(L, o, np.sqrt(Lv / spp + ov / 1024))
    assert pooled < 3.0 and worst < 5.0


def test_zero_nee_shadow_cells():
    """Single scattering with shadow rays traced against the low-pass cells
    only (Zero-NEE), on a scene with a Gaussian level under weak Gabor
    residuals (weights x 0.1, so that the signed delta-tracking weights stay
    moderate), against the oracle."""
    gf = require_gpu()
    params = gen.blob_scene(3000, 7, base_level=True)
    gabor = np.abs(params[:, 10:13]).sum(axis=1) > 0
    params[gabor, 14] *= np.float32(0.1)
    rho = 0.01
    rays = gen.pinhole_rays(16, 16)
    scene = gf.Scene(dev(params), rho=rho)
    spp = 4096
    d = gf.render_desc(spp=spp, multiple=False, albedo=0.9, seed=5, shadow_cells=0x7)
    L, Lv, _, _ = (host(x) for x in gf.gf_render_rays(scene, dev(rays), d))
    o, ov, _, _ = oracle.render(params, rays, 1024, seed=9, rho=rho, multiple=False, albedo=0.9, shadow_cells=0x7)
    pooled, worst = _pooled(L, o, np.sqrt(Lv / spp + ov / 1024))
    assert pooled < 3.0 and worst < 5.0


def test_continuous_lod_cutoff():
    """lod_k in the mask: optical depth to the D9 bar, ratio tracking and
    the render's camera segment in mean, all against the oracle with the
    same cutoff (which removes a good share of the primitives)."""
    gf = require_gpu()
    params, rays, rho = W.scene("tiny256"), W.rays("tiny256"), W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    K = 20.0
    m = gf.make_mask(lod_k=K)
    tau, _ = gf.gf_optical_depth(scene, dev(rays), m, image_width=64)
    ref, ab, nh = oracle.tau(params, rays, rho=rho, lod_k=K)
    _, _, nh_full = oracle.tau(params, rays, rho=rho)
    assert nh.sum() < 0.8 * nh_full.sum()
    assert np.all(np.abs(host(tau).astype(np.float64) - ref) <= 1e-5 * ab)
    sr = rays[::16]
    spp = 4096
    Tm, Tv = (host(x) for x in gf.gf_transmittance_ratio(scene, dev(sr), spp, seed=3, mask=m))
    T = np.exp(-ref[::16])
    ok = spp * T >= 5.0
    pooled, worst = _pooled(Tm[ok], T[ok], np.sqrt(Tv[ok] / spp))
    assert pooled < 3.0 and worst < 5.0
    sr = rays[::64]
    d = gf.render_desc(spp=spp, multiple=True, hg_g=0.3, seed=5, mask=m)
    L, Lv, _, _ = (host(x) for x in gf.gf_render_rays(scene, dev(sr), d))
    o, ov, _, _ = oracle.render(params, sr, 1024, seed=9, rho=rho, multiple=True, hg_g=0.3, lod_k=K)
    pooled, worst = _pooled(L, o, np.sqrt(Lv / spp + ov / 1024))
    assert pooled < 3.0 and worst < 5.0


def test_cdf_inversion_exact_transmittance():
    """Free flights by CDF inversion: the primary transmittance is exp(-tau)
    of the closed form on every ray (zero variance, deep rays included),
    with fixed, LOD-cut and stochastic masks (for the latter: its mean
    against the exact expectation)."""
    gf = require_gpu()
    params, rays, rho = W.scene("tiny256"), W.rays("tiny256"), W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    for m, okw in ((gf.make_mask(), {}), (gf.make_mask(gf.gf_mask_lod_cells(2), lod_k=25.0),
                                          dict(cells=gf.gf_mask_lod_cells(2), lod_k=25.0))):
        d = gf.render_desc(spp=2, multiple=False, seed=5, analytic=True, mask=m)
        _, _, T, Tv = (host(x) for x in gf.gf_render_rays(scene, dev(rays), d, image_width=64))
        tau, ab, _ = oracle.tau(params, rays, rho=rho, **okw)
        ref = np.exp(-tau)
        assert np.all(Tv == 0.0)
        assert np.all(np.abs(T - ref) <= ref * (3e-5 * ab + 1e-6) + 1e-30), np.max(np.abs(T - ref) / ref)


def test_cdf_inversion_radiance_matches_oracle():
    """Single and multiple scattering with CDF-inversion free flights on a
    non-negative density (Gaussian kernels), against the oracle's CDF
    inversion, in mean; the stochastic masks with it."""
    gf = require_gpu()
    params = _positive(W.scene("tiny256"))
    rays, rho = W.rays("tiny256")[::64], W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    spp = 2048
    for kw in (dict(multiple=False, albedo=0.9), dict(multiple=True, albedo=0.9, hg_g=0.3, max_scatter=16),
               dict(multiple=True, albedo=0.9, hg_g=0.3, max_scatter=16, stochastic=True, level="uniform_cv",
                    bin="importance")):
        g, gv, _, _ = (host(x) for x in gf.gf_render_rays(scene, dev(rays),
                                                           gf.render_desc(spp=spp, seed=5, analytic=True, **kw)))
        o, ov, _, _ = oracle.render(params, rays, 512, seed=9, rho=rho, analytic=True, **kw)
        pooled, worst = _pooled(g, o, np.sqrt(gv / spp + ov / 512))
        assert pooled < 3.0 and worst < 5.0, (kw, pooled, worst)


def test_cdf_inversion_furnace():
    """Albedo 1, no scattering cap: every path scatters with weight 1 until
    it escapes, so every sample returns the environment exactly."""
    gf = require_gpu()
    params = _positive(gen.uniform_scene(64, 5))
    scene = gf.Scene(dev(params), rho=0.05)
    rays = gen.ortho_rays(16, 16)
    d = gf.render_desc(spp=8, multiple=True, max_scatter=1 << 30, albedo=1.0, hg_g=0.3, seed=1, analytic=True)
    L, _, _, _ = gf.gf_render_rays(scene, dev(rays), d)
    assert torch.all(L == 1.0)


def test_camera_render_in_caller_workspace():
    """gf_render over a camera in a caller workspace gives the bits of
    gf_render_rays over the camera's rays; too small or misaligned
    workspaces are rejected before any launch."""
    gf = require_gpu()
    params, rho = W.scene("tiny256"), W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    cam = gf.camera(1, width=48, height=40)
    # each tile's samples run as separate work units (more waves than
    # tiles: the workspaces hold a slice per unit)
    for d in (gf.render_desc(spp=3, multiple=True, hg_g=0.3, seed=11),
              gf.render_desc(spp=8, exact_shadow=True, seed=12)):
        need = gf.gf_render_workspace_size(scene, cam, d)
        ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
        rad, T = gf.gf_render(scene, cam, d, ws[:need])
        rays = gf.gf_camera_rays(cam)
        L, _, Tr, _ = gf.gf_render_rays(scene, rays, d, image_width=48)
        assert torch.equal(rad.view(-1), L) and torch.equal(T.view(-1), Tr)
    with pytest.raises(gf.GfError):
        gf.gf_render(scene, cam, d, ws[:need - 256])
    with pytest.raises(gf.GfError):
        gf.gf_render(scene, cam, d, ws[16:need + 16])


def test_invalid_rays_rejected():
    """NaN/Inf origins or directions, |v| = 0 and tmin > tmax return
    GF_EINVAL from every ray-taking call, which then leaves its outputs
    untouched."""
    gf = require_gpu()
    params, rho = W.scene("tiny256"), W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    good = W.rays("tiny256")[:64].copy()
    bads = []
    for k, (col, val) in enumerate([(0, np.nan), (4, np.inf), (6, -np.inf), (7, np.nan)]):
        b = good.copy()
        b[10 + k, col] = val
        bads.append(b)
    b = good.copy()
    b[3, 3:6] = 0.0
    bads.append(b)
    b = good.copy()
    b[5, 6], b[5, 7] = 2.0, 1.0
    bads.append(b)
    for b in bads:
        r = dev(b)
        out = torch.full((64,), -7.0, device="cuda")
        with pytest.raises(gf.GfError) as e:
            gf._lib._check(gf._lib.lib().gf_optical_depth(scene.handle, gf._lib._ptr(r), 64, 0, gf.make_mask(),
                                                          gf._lib._ptr(out), None, gf._lib._stream()))
        assert e.value.status == gf._lib.GF_EINVAL
        assert torch.all(out == -7.0)
        for call in (lambda: gf.gf_transmittance_ratio(scene, r, 4, 1),
                     lambda: gf.gf_render_rays(scene, r, gf.render_desc(spp=1)),
                     lambda: gf.gf_optical_depth_backward(scene, r, torch.ones(64, device="cuda"))):
            with pytest.raises(gf.GfError) as e:
                call()
            assert e.value.status == gf._lib.GF_EINVAL
    # tmax = +inf and tmin = tmax are valid
    g2 = good.copy()
    g2[:, 7] = np.inf
    g2[0, 6] = g2[0, 7] = 0.5
    tau, _ = gf.gf_optical_depth(scene, dev(g2))
    assert torch.isfinite(tau).all()


def test_closed_form_shadow_transmittance():
    """Delta-tracked free flights with the shadow segment's transmittance in
    closed form: the same mean radiance as the oracle's ratio-tracked
    shadow rays (both estimate exp(-tau) of the shadow segment), on the
    signed tiny scene and, on sampled pixels, the 100k-primitive workload."""
    gf = require_gpu()
    params, rays, rho = W.scene("tiny256"), W.rays("tiny256")[::32], W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    spp = 4096
    d = gf.render_desc(spp=spp, multiple=False, albedo=0.9, seed=5, exact_shadow=True)
    L, Lv, _, _ = (host(x) for x in gf.gf_render_rays(scene, dev(rays), d))
    o, ov, _, _ = oracle.render(params, rays, 1024, seed=9, rho=rho, multiple=False, albedo=0.9)
    pooled, worst = _pooled(L, o, np.sqrt(Lv / spp + ov / 1024))
    assert pooled < 3.0 and worst < 5.0, (pooled, worst)
    params, rays, rho = W.scene("blob100k"), W.rays("blob100k"), W.rho("blob100k")
    scene = gf.Scene(dev(params), rho=rho)
    rs = rays[W.pixel_subset(rays.shape[0], k=24, seed=41)]
    copies = 64
    d = gf.render_desc(spp=8, multiple=False, albedo=0.9, seed=78, exact_shadow=True)
    L, _, _, _ = (host(x) for x in gf.gf_render_rays(scene, dev(np.repeat(rs, copies, axis=0)), d))
    L = L.reshape(len(rs), copies)
    g, gv = L.mean(axis=1), L.var(axis=1, ddof=1) / copies
    o, ov, _, _ = oracle.render(params, rs, 256, seed=4, rho=rho, multiple=False, albedo=0.9)
    pooled, worst = _pooled(g, o, np.sqrt(gv + ov / 256))
    assert pooled < 3.0 and worst < 6.0, (pooled, worst)


def test_tile_shared_shadow_directions_image_launch():
    """Single scattering with closed-form shadow transmittance in an image
    launch (8x8 tiles sharing each sample's shadow direction, packet shadow
    walks): one pixel per tile against the oracle's render in mean, and the
    launch differs from a ray-list launch of the same rays (which draws one
    direction per ray)."""
    gf = require_gpu()
    params, rays, rho = W.scene("tiny256"), W.rays("tiny256"), W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    spp = 2048
    d = gf.render_desc(spp=spp, multiple=False, albedo=0.9, seed=15, exact_shadow=True)
    L, Lv, _, _ = (host(x) for x in gf.gf_render_rays(scene, dev(rays), d, image_width=64))
    px = np.array([(8 * ty + 3) * 64 + 8 * tx + 5 for ty in range(8) for tx in range(8)])
    o, ov, _, _ = oracle.render(params, rays[px], 1024, seed=9, rho=rho, multiple=False, albedo=0.9)
    pooled, worst = _pooled(L[px], o, np.sqrt(Lv[px] / spp + ov / 1024))
    assert pooled < 3.0 and worst < 5.0, (pooled, worst)
    Ll, _, _, _ = (host(x) for x in gf.gf_render_rays(scene, dev(rays), d, image_width=0))
    assert not np.array_equal(L, Ll)
