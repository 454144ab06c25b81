"""The synthetic input recipe: blob scenes are Gabor kernels only by default
(the generator the workloads state) and carry a Gaussian low-pass level only
when asked (every fourth primitive: zero frequency, zero phase, four times a
lognormal weight); uniform scenes are Gabor kernels only; scales stay in their
stated ranges; and the stored extinction scale of the small workloads is what
the calibration script computes from the oracle."""
import numpy as np

import gen
from gen import calibrate_rho
from gen import scenes as S
from gen import workloads as W


def test_blob_scene_default_is_gabor_only():
    p = gen.blob_scene(4000, 7).astype(np.float64)
    assert np.all(np.linalg.norm(p[:, S.F], axis=1) > 0.0)
    s = p[:, S.S]
    assert s.min() >= 0.003 * (1 - 1e-6) and s.max() <= 0.05 * (1 + 1e-6)
    # |f| <= 1 / (smallest scale) for every primitive
    assert np.all(np.linalg.norm(p[:, S.F], axis=1) * s.min(axis=1) <= 1.0 + 1e-5)
    la = np.log(p[:, S.ALPHA])
    assert abs(np.median(la)) < 0.05
    assert np.all((p[:, 0:3] >= 0.0) & (p[:, 0:3] <= 1.0))


def test_blob_scene_low_pass_level():
    p = gen.blob_scene(4000, 7, base_level=True).astype(np.float64)
    q = gen.blob_scene(4000, 7).astype(np.float64)
    base = np.arange(len(p)) % S.GAUSS_EVERY == 0
    assert np.all(p[base][:, S.F] == 0.0) and np.all(p[base][:, S.PHI] == 0.0)
    assert np.all(np.linalg.norm(p[~base][:, S.F], axis=1) > 0.0)
    # only the low-pass primitives differ from the Gabor-only draw
    assert np.array_equal(p[~base], q[~base])
    assert np.array_equal(p[base][:, 0:10], q[base][:, 0:10])
    # the level's weights are the lognormal(0, 0.5) draws times four: the
    # median of log(alpha) is log(4) there and 0 elsewhere
    la = np.log(p[:, S.ALPHA])
    assert abs(np.median(la[base]) - np.log(S.GAUSS_WEIGHT)) < 0.1
    assert abs(np.median(la[~base])) < 0.05


def test_workload_variants():
    assert not W.WORKLOADS["blob100k"].get("base_level", False)
    assert W.WORKLOADS["blob100k_lp"]["base_level"]
    assert "Gabor-only" in W.describe("blob1m")
    assert "low-pass" in W.describe("blob1m_lp")


def test_uniform_scene_is_gabor_only():
    p = W.scene("tiny256").astype(np.float64)
    assert np.all(np.linalg.norm(p[:, S.F], axis=1) > 0.0)
    assert p[:, S.S].min() >= 0.02 * (1 - 1e-6) and p[:, S.S].max() <= 0.1 * (1 + 1e-6)


def test_stored_rho_matches_calibration():
    for name in ("tiny256", "serve10k"):
        assert abs(calibrate_rho.calibrate(name) / W.rho(name) - 1.0) < 1e-12
