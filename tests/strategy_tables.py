"""Exact enumeration of the per-segment stochastic mask distribution, written
in the tests from the paper's two Appendix B tables (frequency levels;
orientation bins), independently of the oracle's sampler.

enumerate_outcomes(...) -> list of (probability, 12 cell weights).  Cells are
(level, bin), cell = 3 * level + bin; P = 4 levels (level 0 the low-pass
level, which carries no orientation), K = 3 bins with o_k = e_k.
"""
import itertools
import math

import numpy as np

P, K = 4, 3


def level_outcomes(strategy, beta):
    """[(probability, level weights[4])]"""
    e = 1.0 - beta
    out = []
    if strategy == "deterministic":
        return [(1.0, [1.0] * P)]
    if strategy == "uniform":
        for l in range(P):
            w = [0.0] * P
            w[l] = P
            out.append((1.0 / P, w))
        return out
    if strategy in ("power", "power_cv_accum"):
        # bucket [l/P, (l+1)/P) of x = u^(1/(1-beta)) has probability b^(1-beta) - a^(1-beta)
        for l in range(P):
            a, b = l / P, (l + 1) / P
            p = b ** e - a ** e
            w = [0.0] * P
            if strategy == "power":
                w[l] = 1.0 / p
            else:
                # levels 0..l traced; level j is traced whenever the drawn level is >= j
                for j in range(l + 1):
                    w[j] = 1.0 / (1.0 - (j / P) ** e)
            out.append((p, w))
        return out
    if strategy == "uniform_cv":
        for j in range(P - 1):
            w = [1.0] + [0.0] * (P - 1)
            w[1 + j] = P - 1
            out.append((1.0 / (P - 1), w))
        return out
    if strategy == "power_cv":
        for j in range(P - 1):
            a, b = j / (P - 1), (j + 1) / (P - 1)
            p = b ** e - a ** e
            w = [1.0] + [0.0] * (P - 1)
            w[1 + j] = 1.0 / p
            out.append((p, w))
        return out
    raise KeyError(strategy)


def bin_outcomes(strategy, f0, a, delta):
    """[(probability, bin weights[3])] for one level; f0 = the level's three
    cell medians, a = alignments |v_k| / |v|"""
    if strategy == "deterministic":
        return [(1.0, [1.0] * K)]
    if strategy == "threshold":
        return [(1.0, [1.0 if a[k] <= delta else 0.0 for k in range(K)])]
    if strategy == "uniform":
        return [(1.0 / K, [K if j == k else 0.0 for j in range(K)]) for k in range(K)]
    if strategy == "threshold_uniform":
        above = [k for k in range(K) if a[k] > delta]
        base = [1.0 if a[k] <= delta else 0.0 for k in range(K)]
        if not above:
            return [(1.0, base)]
        out = []
        for k in above:
            w = list(base)
            w[k] = len(above)
            out.append((1.0 / len(above), w))
        return out
    # contribution weights w_k = exp(-f0^2 a^2 / 2), scaled by the largest
    lw = [-0.5 * f0[k] ** 2 * a[k] ** 2 for k in range(K)]
    m = max(lw)
    w = [math.exp(x - m) for x in lw]
    W = sum(w)
    if strategy == "importance":
        p = [wk / W for wk in w]
    elif strategy == "mixture":
        p = [0.5 * wk / W + 0.5 / K for wk in w]
    else:
        raise KeyError(strategy)
    return [(p[k], [1.0 / p[k] if j == k else 0.0 for j in range(K)]) for k in range(K) if p[k] > 0.0]


def enumerate_outcomes(level, bin, med12, v, beta=0.0, delta=1.0):
    v = np.asarray(v, np.float64)
    a = list(np.abs(v) / np.linalg.norm(v))
    out = []
    for pl, lw in level_outcomes(level, beta):
        per_level = []
        for l in range(P):
            if l == 0 or lw[l] == 0.0:
                per_level.append([(1.0, [1.0] * K)])
            else:
                per_level.append(bin_outcomes(bin, list(med12[3 * l:3 * l + 3]), a, delta))
        for combo in itertools.product(*per_level):
            p = pl
            wc = []
            for l, (pb, bw) in enumerate(combo):
                p *= pb
                wc.extend(lw[l] * x for x in bw)
            if p > 0.0:
                out.append((p, np.array(wc)))
    return out


def expected_T(outcomes, tau_cells):
    """E[exp(-sum_c w_c tau_c)] over the outcomes (exact Jensen-biased
    expectation of a segment's transmittance estimate)."""
    return sum(p * math.exp(-float(np.dot(w, tau_cells))) for p, w in outcomes)


def expected_weights(outcomes):
    return sum(p * w for p, w in outcomes)
