"""Seeded synthetic scenes of Gabor primitives.

This module only draws random inputs.  It holds none of the rendering
arithmetic (no kernel evaluation, no integrals, no acceleration structure):
both the FP64 oracle and the HIP path consume what it produces.

Primitive record, 15 float32 per primitive, in this order:

    mu[3]  q[4] (w, x, y, z; real part first)  s[3]  f[3]  phi  alpha

* ``mu``    kernel mean (Sec. 4.2, Eq. of the 3D anisotropic Gabor kernel)
* ``q``     rotation quaternion, stored normalised; R(q) maps local to world
* ``s``     per-axis standard deviations (the diagonal of S, Sigma = R S S^T R^T)
* ``f``     carrier frequency vector in cycles per unit length (omega = 2 pi f)
* ``phi``   carrier phase in radians
* ``alpha`` kernel weight

The draw order is fixed (one ``numpy.random.Generator(PCG64(seed))``, every
quantity drawn in float64, then cast to float32 at the end):

    [blob field parameters]  mu  q  s  f-direction  f-magnitude  phi  alpha

By default every primitive is a Gabor kernel (a signed field).  With
``base_level=True`` (blob scenes) every fourth primitive (index % 4 == 0) is
then turned into a Gaussian of the low-pass level: f = 0, phi = 0, alpha
scaled by 4 -- a positive base under the Gabor residuals, shaped like the
paper's assets (Sec. 4.3: Gaussians for the low-pass, Gabor kernels for the
remaining bands).
"""
from __future__ import annotations

import numpy as np

N_FIELDS = 15
MU, Q, S, F, PHI, ALPHA = slice(0, 3), slice(3, 7), slice(7, 10), slice(10, 13), 13, 14
GAUSS_EVERY, GAUSS_WEIGHT = 4, 4.0


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _common_tail(g: np.random.Generator, mu: np.ndarray, smin: float, smax: float,
                 base_level: bool = False) -> np.ndarray:
    n = mu.shape[0]
    q = g.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    # log-uniform per-axis scales
    s = np.exp(g.uniform(np.log(smin), np.log(smax), size=(n, 3)))
    fdir = g.standard_normal((n, 3))
    fdir /= np.linalg.norm(fdir, axis=1, keepdims=True)
    # magnitude uniform on [0, 1/s_min] with s_min the primitive's smallest axis
    fmag = g.uniform(0.0, 1.0, size=n) / s.min(axis=1)
    phi = g.uniform(0.0, 2.0 * np.pi, size=n)
    alpha = g.lognormal(0.0, 0.5, size=n)
    if base_level:
        # the pyramid's low-pass level (Sec. 4): every fourth primitive is a
        # zero-frequency kernel (a Gaussian) with 4x the weight, so that the
        # mixture is positive almost everywhere and the Gabor kernels are
        # residuals on top of it
        base = np.arange(n) % GAUSS_EVERY == 0
        fdir[base] = 0.0
        fmag[base] = 0.0
        phi[base] = 0.0
        alpha[base] *= GAUSS_WEIGHT
    out = np.empty((n, N_FIELDS), dtype=np.float64)
    out[:, MU] = mu
    out[:, Q] = q
    out[:, S] = s
    out[:, F] = fdir * fmag[:, None]
    out[:, PHI] = phi
    out[:, ALPHA] = alpha
    return np.ascontiguousarray(out.astype(np.float32))


def uniform_scene(n: int = 256, seed: int = 0, smin: float = 0.02, smax: float = 0.1) -> np.ndarray:
    """Means uniform in the unit cube (the tiny 256-primitive workload)."""
    g = _rng(seed)
    mu = g.uniform(0.0, 1.0, size=(n, 3))
    return _common_tail(g, mu, smin, smax)


def blob_scene(n: int, seed: int, smin: float = 0.003, smax: float = 0.05, n_blobs: int = 64,
               base_level: bool = False) -> np.ndarray:
    """Means drawn from a sum of ``n_blobs`` isotropic Gaussian blobs.

    Blob centres are uniform in [0.15, 0.85]^3, blob radii log-uniform in
    [0.03, 0.15], blob weights uniform in [0.5, 1.5].  A mean is drawn by picking
    a blob with probability proportional to its weight and adding an isotropic
    normal offset of the blob's radius; means outside the unit cube are redrawn.
    With ``base_level`` every fourth primitive belongs to a Gaussian low-pass
    level (off by default: Gabor kernels only).
    """
    g = _rng(seed)
    centres = g.uniform(0.15, 0.85, size=(n_blobs, 3))
    radii = np.exp(g.uniform(np.log(0.03), np.log(0.15), size=n_blobs))
    weights = g.uniform(0.5, 1.5, size=n_blobs)
    p = weights / weights.sum()
    mu = np.empty((n, 3))
    todo = np.arange(n)
    while todo.size:
        b = g.choice(n_blobs, size=todo.size, p=p)
        cand = centres[b] + radii[b, None] * g.standard_normal((todo.size, 3))
        ok = np.all((cand >= 0.0) & (cand <= 1.0), axis=1)
        mu[todo[ok]] = cand[ok]
        todo = todo[~ok]
    return _common_tail(g, mu, smin, smax, base_level=base_level)


def jitter_scene(params: np.ndarray, seed: int, rel: float = 0.05) -> np.ndarray:
    """A perturbed copy of a scene (the target of the differentiation workload).

    mu moves by rel * mean(s) * U[-1,1]^3; q, s, f, alpha are scaled by
    (1 + rel * U[-1,1]) per component (q renormalised); phi moves by
    rel * 2 pi * U[-1,1].
    """
    g = _rng(seed)
    p = params.astype(np.float64).copy()
    n = p.shape[0]
    sbar = p[:, S].mean(axis=1)
    p[:, MU] += rel * sbar[:, None] * g.uniform(-1, 1, size=(n, 3))
    p[:, Q] *= 1.0 + rel * g.uniform(-1, 1, size=(n, 4))
    p[:, Q] /= np.linalg.norm(p[:, Q], axis=1, keepdims=True)
    p[:, S] *= 1.0 + rel * g.uniform(-1, 1, size=(n, 3))
    p[:, F] *= 1.0 + rel * g.uniform(-1, 1, size=(n, 3))
    p[:, PHI] += rel * 2.0 * np.pi * g.uniform(-1, 1, size=n)
    p[:, ALPHA] *= 1.0 + rel * g.uniform(-1, 1, size=n)
    return np.ascontiguousarray(p.astype(np.float32))
