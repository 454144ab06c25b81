"""Pins of the per-segment stochastic masks (Sec. 4.5.1-4.5.2, Appendix B
tables of frequency-level and orientation-bin strategies):

* every stochastic strategy is unbiased cell by cell (E[w_c] = 1) and its
  probabilities sum to 1, by exact enumeration;
* special cases reduce to known distributions (power law with beta = 0 is
  uniform; the accumulating weights at beta = 0 are P / (P - j); importance
  sampling with equal contributions is uniform; threshold + uniform with a
  threshold above every alignment is deterministic, below every alignment
  uniform);
* the power-law bucket probabilities agree with a direct simulation of
  x = u^(1/(1-beta));
* the oracle's sampler draws outcomes with the enumerated probabilities
  (chi-square) and gives exactly the enumerated weights for each outcome;
* the oracle's ratio-tracked primary transmittance under each strategy
  matches the exact expectation sum_outcomes p exp(-tau_hat).
"""
import math

import numpy as np
import pytest
import scipy.stats as st

import gen
from strategy_tables import enumerate_outcomes, expected_T, expected_weights

LEVELS = ["deterministic", "uniform", "power", "uniform_cv", "power_cv", "power_cv_accum"]
BINS = ["deterministic", "threshold", "uniform", "importance", "threshold_uniform", "mixture"]
STOCHASTIC_BINS = ["deterministic", "uniform", "importance", "mixture"]

MED = np.array([0.0, 0.0, 0.0, 1.5, 2.0, 0.7, 4.0, 3.0, 5.5, 9.0, 12.0, 7.0])
V = np.array([0.3, -0.5, 0.81])


@pytest.mark.parametrize("level", LEVELS)
@pytest.mark.parametrize("bin", STOCHASTIC_BINS)
@pytest.mark.parametrize("beta", [0.0, 0.2, 0.6])
def test_unbiased_by_enumeration(level, bin, beta):
    out = enumerate_outcomes(level, bin, MED, V, beta=beta)
    assert abs(sum(p for p, _ in out) - 1.0) < 1e-12
    assert np.allclose(expected_weights(out), 1.0, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("delta", [0.2, 0.55, 0.9])
def test_threshold_strategies(delta):
    a = np.abs(V) / np.linalg.norm(V)
    keep = (a <= delta).astype(float)
    out = enumerate_outcomes("deterministic", "threshold", MED, V, delta=delta)
    assert len(out) == 1
    w = out[0][1]
    assert np.array_equal(w[:3], np.ones(3))
    for l in (1, 2, 3):
        assert np.array_equal(w[3 * l:3 * l + 3], keep)
    # threshold + uniform: unbiased cell by cell
    out = enumerate_outcomes("uniform_cv", "threshold_uniform", MED, V, delta=delta)
    assert np.allclose(expected_weights(out), 1.0)


def test_special_cases(orc):
    u = lambda *x: np.array(x, np.float64)  # noqa: E731
    # power law at beta = 0 is the uniform level strategy
    for uu in (0.1, 0.3, 0.6, 0.95):
        assert np.allclose(orc.segment_cell_weights("power", "deterministic", MED, V, u(uu, .5, .5, .5), beta=0.0),
                           orc.segment_cell_weights("uniform", "deterministic", MED, V, u(uu, .5, .5, .5)),
                           rtol=1e-14, atol=0)
        assert np.allclose(
            orc.segment_cell_weights("power_cv", "deterministic", MED, V, u(uu, .5, .5, .5), beta=0.0),
            orc.segment_cell_weights("uniform_cv", "deterministic", MED, V, u(uu, .5, .5, .5)), rtol=1e-14, atol=0)
    # uniform: level floor(4u) with weight 4
    w = orc.segment_cell_weights("uniform", "deterministic", MED, V, u(0.6, .5, .5, .5))
    assert np.array_equal(w, np.r_[np.zeros(6), 4 * np.ones(3), np.zeros(3)])
    # accumulating at beta = 0: level j has weight P / (P - j); u = 0.99 traces all levels
    w = orc.segment_cell_weights("power_cv_accum", "deterministic", MED, V, u(0.99, .5, .5, .5), beta=0.0)
    assert np.allclose(w, np.repeat([1.0, 4 / 3, 2.0, 4.0], 3), rtol=1e-15)
    w = orc.segment_cell_weights("power_cv_accum", "deterministic", MED, V, u(0.3, .5, .5, .5), beta=0.0)
    assert np.allclose(w, np.r_[np.ones(3), 4 / 3 * np.ones(3), np.zeros(6)], rtol=1e-15)
    # importance sampling with equal contributions is uniform sampling
    vd = np.ones(3) / math.sqrt(3)
    med_eq = np.repeat([0.0, 2.0, 3.0, 4.0], 3)
    for uu in (0.1, 0.5, 0.9):
        a = orc.segment_cell_weights("deterministic", "importance", med_eq, vd, u(.5, uu, uu, uu))
        b = orc.segment_cell_weights("deterministic", "uniform", med_eq, vd, u(.5, uu, uu, uu))
        assert np.allclose(a, b, rtol=1e-12)
    # threshold + uniform: above every alignment -> deterministic; below every one -> uniform
    for uu in (0.2, 0.7):
        assert np.array_equal(
            orc.segment_cell_weights("deterministic", "threshold_uniform", MED, V, u(.5, uu, uu, uu), delta=1.0),
            np.ones(12))
        assert np.array_equal(
            orc.segment_cell_weights("deterministic", "threshold_uniform", MED, V, u(.5, uu, uu, uu), delta=0.1),
            orc.segment_cell_weights("deterministic", "uniform", MED, V, u(.5, uu, uu, uu)))
    # importance: the picked bin of a level has weight W / w_k
    a = np.abs(V) / np.linalg.norm(V)
    w = orc.segment_cell_weights("deterministic", "importance", MED, V, u(.5, 0.999, 0.001, 0.5))
    for l, uu in ((1, 0.999), (2, 0.001)):
        wk = np.exp(-0.5 * MED[3 * l:3 * l + 3] ** 2 * a ** 2)
        p = wk / wk.sum()
        k = int(np.searchsorted(np.cumsum(p), uu, side="right"))
        assert abs(w[3 * l + k] - 1 / p[k]) <= 1e-12 / p[k]
        assert np.count_nonzero(w[3 * l:3 * l + 3]) == 1


@pytest.mark.parametrize("beta", [0.2, 0.5])
def test_power_law_buckets_by_simulation(orc, beta):
    """bucket frequencies of x = u^(1/(1-beta)) by direct simulation against
    the reciprocal of the oracle's level weights"""
    g = np.random.default_rng(4)
    x = g.random(400000) ** (1 / (1 - beta))
    freq = np.bincount(np.minimum((4 * x).astype(int), 3), minlength=4) / len(x)
    for l in range(4):
        uu = ((l + 0.5) / 4) ** (1 - beta)
        w = orc.segment_cell_weights("power", "deterministic", MED, V, np.array([uu, .5, .5, .5]), beta=beta)
        assert abs(1 / w[3 * l] - freq[l]) < 5 * math.sqrt(freq[l] / len(x))


@pytest.mark.parametrize("level,bin,beta,delta", [("uniform_cv", "importance", 0.0, 1.0),
                                                  ("power_cv_accum", "uniform", 0.2, 1.0),
                                                  ("power", "mixture", 0.4, 1.0),
                                                  ("deterministic", "threshold_uniform", 0.0, 0.5),
                                                  ("power_cv", "importance", 0.2, 1.0)])
def test_oracle_sampler_matches_enumeration(orc, level, bin, beta, delta):
    out = enumerate_outcomes(level, bin, MED, V, beta=beta, delta=delta)
    n = 30000
    draws = orc.sample_cell_weights(level, bin, MED, V, n, seed=8, beta=beta, delta=delta)
    # every draw is one of the enumerated outcomes, with exactly its weights
    idx = np.full(n, -1)
    for j, (_, w) in enumerate(out):
        hit = np.all(np.abs(draws - w) <= 1e-9 * np.maximum(1.0, np.abs(w)), axis=1)
        idx[hit & (idx < 0)] = j
    assert np.all(idx >= 0)
    probs = np.array([p for p, _ in out])
    counts = np.bincount(idx, minlength=len(out))
    big = probs * n >= 5
    exp_counts = probs[big] * n
    obs = counts[big]
    rest_e, rest_o = n - exp_counts.sum(), n - obs.sum()
    if rest_e >= 5:
        exp_counts, obs = np.r_[exp_counts, rest_e], np.r_[obs, rest_o]
    stat = ((obs - exp_counts) ** 2 / exp_counts).sum()
    assert st.chi2.sf(stat, len(obs) - 1) > 1e-4
    # unbiased cell weights from the sampler itself, on the cells whose
    # weighted outcomes are all frequent enough to be sampled (importance
    # sampling gives rarely drawn cells huge weights)
    m, s = draws.mean(axis=0), draws.std(axis=0, ddof=1) / math.sqrt(n) + 1e-12
    ew = expected_weights(out)
    pmin = np.array([min([p for p, w in out if w[c] != 0.0], default=1.0) for c in range(12)])
    ok = pmin * n >= 50
    assert ok.sum() >= 6
    assert np.all(np.abs(m - ew)[ok] < 5 * s[ok] + 1e-12)


def _tau_cells(orc, params, rays, rho):
    return np.stack([orc.tau(params, rays, rho=rho, cells=1 << c)[0] for c in range(12)], axis=1)


@pytest.mark.slow
@pytest.mark.parametrize("level,bin,beta", [("uniform_cv", "importance", 0.0), ("power_cv_accum", "uniform", 0.2),
                                            ("uniform", "mixture", 0.0)])
def test_primary_transmittance_exact_expectation(orc, level, bin, beta):
    """E[T_hat] of the ratio-tracked camera segment = sum over outcomes of
    p exp(-sum_c w_c tau_c) (the Jensen-biased expectation of Sec. 4.5.3)"""
    params = gen.uniform_scene(128, 3)
    params[:, 10:13] *= 0.2
    rho = 0.004
    rays = gen.random_rays(40, 12)
    med = orc.cell_medians(params)
    tc = _tau_cells(orc, params, rays, rho)
    spp = 4000
    _, _, Tm, Tv = orc.render(params, rays, spp, seed=77, rho=rho, multiple=True, hg_g=0.3, stochastic=True,
                              level=level, bin=bin, beta=beta)
    exact, keep = [], []
    for k, ray in enumerate(rays):
        out = enumerate_outcomes(level, bin, med, ray[3:6], beta=beta)
        exact.append(expected_T(out, tc[k]))
        # unbiased optical depth
        assert abs(sum(p * np.dot(w, tc[k]) for p, w in out) - tc[k].sum()) <= 1e-12 * (1 + np.abs(tc[k]).sum())
        keep.append(max(abs(np.dot(w, tc[k])) for _, w in out) < 0.6)
    exact, keep = np.array(exact), np.array(keep)
    assert keep.sum() >= 20
    # Jensen (Sec. 4.5.3): E[exp(-tau_hat)] > exp(-E[tau_hat]) when tau_hat
    # varies, and 1/2 Var(tau_hat) T approximates the gap to second order
    for k, ray in enumerate(rays):
        out = enumerate_outcomes(level, bin, med, ray[3:6], beta=beta)
        th = np.array([np.dot(w, tc[k]) for _, w in out])
        p = np.array([p for p, _ in out])
        var = np.dot(p, th ** 2) - np.dot(p, th) ** 2
        T = math.exp(-tc[k].sum())
        if var > 1e-8 and keep[k]:
            assert exact[k] > T
            assert abs((exact[k] - T) - 0.5 * var * T) < 0.5 * (0.5 * var * T) + 1e-12
    se = np.sqrt(Tv / spp) + 1e-12
    assert abs(np.sum((Tm - exact)[keep])) / np.sqrt(np.sum(se[keep] ** 2)) < 3.0
    assert np.max(np.abs((Tm - exact) / se)[keep]) < 4.5
