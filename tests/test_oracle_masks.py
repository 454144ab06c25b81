"""Pins of the level / bin partition, the cone mask, and the stochastic
per-segment masks (Sec. 4.5.1-4.5.2, Appendix B: uniform + control variate
over levels, importance sampling over orientation bins)."""
import math

import numpy as np
import pytest

import gen


def cells_ref(params):
    f = params[:, 10:13].astype(np.float64)
    f2 = (f[:, 0] * f[:, 0] + f[:, 1] * f[:, 1]) + f[:, 2] * f[:, 2]
    m = f2.max()
    lev = np.where(f2 <= m / 64, 0, np.where(f2 <= m / 16, 1, np.where(f2 <= m / 4, 2, 3)))
    return lev * 3 + np.argmax(f * f, axis=1)


@pytest.mark.parametrize("seed", [0, 1])
def test_cells_match_definition(orc, seed):
    params = gen.blob_scene(5000, seed)
    c, m = orc.cells(params)
    assert np.array_equal(c, cells_ref(params))
    # ties go to the lower axis; zero frequency lands in level 0, bin 0
    p = params[:4].copy()
    p[0, 10:13] = 0.0
    p[1, 10:13] = [1.0, -1.0, 0.5]
    p[2, 10:13] = [0.5, 1.0, -1.0]
    p[3, 10:13] = [0.0, 0.0, 8.0]
    c, _ = orc.cells(p)
    assert c[0] == 0 and c[1] % 3 == 0 and c[2] % 3 == 1 and c[3] == 11


def test_lod_cells_nesting(orc):
    assert orc.lod_cells(0) == orc.FULL_MASK
    assert orc.lod_cells(3) == 0b111
    assert orc.lod_cells(2) == 0b111111
    assert orc.lod_cells(1) == (1 << 9) - 1


def test_cone_mask_matches_definition(orc):
    params = gen.blob_scene(3000, 2)
    bits = orc.mask_cone(params, (0, 0, 1), math.pi / 4)
    f = params[:, 10:13].astype(np.float64)
    keep = f[:, 2] ** 2 <= 0.5 * (f ** 2).sum(axis=1) * (1 + 1e-12)
    got = np.array([(bits[i >> 5] >> (i & 31)) & 1 for i in range(len(params))], bool)
    assert np.array_equal(got, keep)


def test_cell_medians(orc):
    params = gen.blob_scene(3000, 4)
    c, _ = orc.cells(params)
    med = orc.cell_medians(params)
    p = params.astype(np.float64)
    for cell in range(12):
        idx = np.where(c == cell)[0]
        if len(idx) == 0:
            assert med[cell] == 0
            continue
        vals = []
        for i in idx:
            w, x, y, z = p[i, 3:7] / np.linalg.norm(p[i, 3:7])
            R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                          [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                          [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
            vals.append(np.linalg.norm(p[i, 7:10] * (R.T @ (2 * math.pi * p[i, 10:13]))))
        vals = np.sort(vals)
        assert abs(med[cell] - vals[(len(vals) - 1) // 2]) <= 1e-12 * vals.max()


def _stoch_table(orc, params, ray, rho):
    """exact enumeration of the per-segment mask distribution for one ray:
    list of (probability, tau_hat) pairs"""
    med = orc.cell_medians(params)
    tc = [orc.tau(params, ray[None, :], rho=rho, cells=1 << c)[0][0] for c in range(12)]
    tau_L0 = sum(tc[0:3])
    v = ray[3:6] / np.linalg.norm(ray[3:6])
    out = []
    for l in (1, 2, 3):
        w = np.exp(-0.5 * med[3 * l:3 * l + 3] ** 2 * np.abs(v) ** 2)
        p = 0.5 * w / w.sum() + 1.0 / 6.0  # even mixture of importance and uniform bin sampling
        for k in range(3):
            out.append((p[k] / 3.0, tau_L0 + 3.0 / p[k] * tc[3 * l + k]))
    return out, sum(tc)


def test_stochastic_mask_unbiased_tau(orc):
    params = gen.uniform_scene(256, 0)
    rays = gen.random_rays(32, 11)
    for ray in rays:
        tab, full = _stoch_table(orc, params, ray, 0.0166)
        assert abs(sum(p for p, _ in tab) - 1.0) < 1e-14
        assert abs(sum(p * t for p, t in tab) - full) <= 1e-12 * (1 + abs(full))


@pytest.mark.slow
def test_stochastic_primary_transmittance_matches_exact_expectation(orc):
    """E[T_hat] = sum over masks of p(mask) exp(-tau_hat(mask)) (the exact
    Jensen-biased expectation of Sec. 4.5.3); the oracle's ratio-tracked primary
    transmittance under per-segment masks must match it in mean."""
    params = gen.uniform_scene(128, 3)
    params[:, 10:13] *= 0.2  # moderate importance weights
    rho = 0.004  # keeps |tau_hat| small: ratio tracking of a signed field is heavy-tailed otherwise
    rays = gen.random_rays(48, 12)
    spp = 6000
    _, _, Tm, Tv = orc.render(params, rays, spp, seed=77, rho=rho, multiple=True, stochastic=True, hg_g=0.3)
    exact, full_T, var_tau, keep = [], [], [], []
    for ray in rays:
        tab, full = _stoch_table(orc, params, ray, rho)
        exact.append(sum(p * math.exp(-t) for p, t in tab))
        full_T.append(math.exp(-full))
        var_tau.append(sum(p * t * t for p, t in tab) - sum(p * t for p, t in tab) ** 2)
        keep.append(max(abs(t) for _, t in tab) < 0.6)
    exact, keep = np.array(exact), np.array(keep)
    assert keep.sum() >= 30
    se = np.sqrt(Tv / spp) + 1e-12
    z = (Tm - exact) / se
    assert abs(np.sum((Tm - exact)[keep])) / np.sqrt(np.sum(se[keep] ** 2)) < 3.0
    assert np.max(np.abs(z[keep])) < 4.5
    # Jensen: the exact expectation exceeds exp(-E[tau_hat]) whenever tau_hat varies,
    # and 1/2 Var(tau_hat) T approximates the gap to second order
    for e, T, v in zip(exact, full_T, var_tau):
        if v > 1e-8:
            assert e > T
            assert abs((e - T) - 0.5 * v * T) < 0.5 * (0.5 * v * T) + 1e-12
