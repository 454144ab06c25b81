"""Pins of the level / bin partition, the cone mask and the per-cell medians
of |k_W| (Sec. 4.6 implementation details; the stochastic strategies that
use them are pinned in test_oracle_strategies.py)."""
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
