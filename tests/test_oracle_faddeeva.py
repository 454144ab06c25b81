"""Pins of the oracle's Faddeeva function w(z) (used by the closed-form
segment integral of Sec. 4.4) against library routines and the paper's
Maclaurin series of erf (Sec. 4.4, complex-valued error function)."""
import math

import mpmath
import numpy as np
import pytest
import scipy.special as sp


def test_w_matches_scipy_on_render_domain(orc):
    # arguments met by the segment integral: (+-Omega + i|u|)/sqrt2 with |u| <= r
    g = np.random.default_rng(0)
    z = np.concatenate([
        g.uniform(-80, 80, 20000) + 1j * g.uniform(0, 2.2, 20000),
        g.uniform(-7, 7, 20000) + 1j * g.uniform(0, 9, 20000),
        np.array([0.0, 1e-12, 6.0, 6j, 5.999 + 0.001j, -6.0 + 0j, 0.3j]),
    ])
    w = orc.faddeeva(z)
    ref = sp.wofz(z)
    rel = np.abs(w - ref) / np.abs(ref)
    assert rel.max() < 1e-12


def test_w_matches_mpmath_50_digits(orc):
    mpmath.mp.dps = 50
    pts = [0.1 + 0.2j, 2.5 + 0.01j, -3.7 + 1.9j, 5.9 + 0.0j, 0.0 + 5.9j, 12.0 + 0.5j, -40.0 + 2.0j]
    w = orc.faddeeva(np.array(pts))
    for z, got in zip(pts, w):
        zz = mpmath.mpc(z.real, z.imag)
        ref = complex(mpmath.exp(-zz * zz) * mpmath.erfc(-1j * zz))
        assert abs(got - ref) <= 1e-13 * abs(ref)


def test_w_lower_half_plane_reflection(orc):
    z = np.array([0.5 - 0.5j, -2.0 - 1.0j, 3.0 - 0.2j])
    assert np.allclose(orc.faddeeva(z), sp.wofz(z), rtol=1e-11, atol=0)


def test_erf_from_w_matches_paper_series(orc):
    """erf(z) = 1 - exp(-z^2) w(iz); inside its convergence disc the truncated
    Maclaurin series the paper uses (Sec. 4.4) must agree."""
    g = np.random.default_rng(1)
    z = g.uniform(-1.2, 1.2, 200) + 1j * g.uniform(-1.2, 1.2, 200)
    erf_w = 1.0 - np.exp(-z * z) * orc.faddeeva(1j * z)
    series = np.zeros_like(z)
    for n in range(40):
        series += (-1) ** n * z ** (2 * n + 1) / (math.factorial(n) * (2 * n + 1))
    series *= 2.0 / math.sqrt(math.pi)
    assert np.max(np.abs(erf_w - series)) < 1e-13
    # the paper truncates at 16 terms: accurate only for small |z|
    s16 = sum((-1) ** n * z ** (2 * n + 1) / (math.factorial(n) * (2 * n + 1)) for n in range(16))
    small = np.abs(z) < 1.0
    assert np.max(np.abs(2 / math.sqrt(math.pi) * s16[small] - erf_w[small])) < 1e-12


@pytest.mark.parametrize("z", [0.0, 1.0, 3.0])
def test_w_real_axis_real_part_is_gaussian(orc, z):
    # Re w(x) = exp(-x^2) on the real axis (textbook identity)
    assert abs(orc.faddeeva(np.array([z]))[0].real - math.exp(-z * z)) < 1e-15
