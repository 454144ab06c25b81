"""The synthetic input recipe: blob scenes carry a Gaussian low-pass level
(every fourth primitive: zero frequency, zero phase, four times a lognormal
weight), uniform scenes are Gabor kernels only, scales stay in their stated
ranges, and the stored extinction scale of the small workload is what the
calibration script computes from the oracle."""
import numpy as np

import gen
from gen import calibrate_rho
from gen import scenes as S
from gen import workloads as W


def test_blob_scene_low_pass_level():
    p = gen.blob_scene(4000, 7).astype(np.float64)
    base = np.arange(len(p)) % S.GAUSS_EVERY == 0
    assert np.all(p[base][:, S.F] == 0.0) and np.all(p[base][:, S.PHI] == 0.0)
    assert np.all(np.linalg.norm(p[~base][:, S.F], axis=1) > 0.0)
    s = p[:, S.S]
    assert s.min() >= 0.003 * (1 - 1e-6) and s.max() <= 0.05 * (1 + 1e-6)
    # |f| <= 1 / (smallest scale) for every primitive
    assert np.all(np.linalg.norm(p[:, S.F], axis=1) * s.min(axis=1) <= 1.0 + 1e-5)
    # the level's weights are the lognormal(0, 0.5) draws times four: the
    # median of log(alpha) is log(4) there and 0 elsewhere
    la = np.log(p[:, S.ALPHA])
    assert abs(np.median(la[base]) - np.log(S.GAUSS_WEIGHT)) < 0.1
    assert abs(np.median(la[~base])) < 0.05


def test_uniform_scene_is_gabor_only():
    p = W.scene("tiny256").astype(np.float64)
    assert np.all(np.linalg.norm(p[:, S.F], axis=1) > 0.0)
    assert p[:, S.S].min() >= 0.02 * (1 - 1e-6) and p[:, S.S].max() <= 0.1 * (1 + 1e-6)


def test_stored_rho_matches_calibration():
    assert abs(calibrate_rho.calibrate("tiny256") / W.rho("tiny256") - 1.0) < 1e-12
