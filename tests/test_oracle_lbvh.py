"""Pins of the oracle's linear BVH (Morton keys, Karras hierarchy, boxes).

Independent re-derivations in numpy: the 63-bit Morton key of each mean, the
binary radix tree built top-down by splitting at the highest differing key bit
(index bits for equal keys), the containment of every truncated ellipsoid in
its leaf box, and the equality of the traversal hit set with brute force.
"""
import math

import numpy as np
import pytest

import gen


def morton_ref(params):
    mu = params[:, 0:3].astype(np.float32)
    lo, hi = mu.min(axis=0).astype(np.float64), mu.max(axis=0).astype(np.float64)
    keys = np.zeros(len(mu), dtype=np.uint64)
    q = np.zeros((len(mu), 3), dtype=np.int64)
    for a in range(3):
        if hi[a] == lo[a]:
            continue
        scale = 2097152.0 / (hi[a] - lo[a])
        q[:, a] = np.minimum(2097151, np.floor((mu[:, a].astype(np.float64) - lo[a]) * scale)).astype(np.int64)
    for b in range(21):
        for a, shift in ((0, 2), (1, 1), (2, 0)):
            keys |= (((q[:, a] >> b) & 1).astype(np.uint64) << np.uint64(3 * b + shift))
    return keys


def radix_tree_ref(keys_sorted):
    """top-down: range [f, l] splits after the last index sharing the longest prefix"""
    n = len(keys_sorted)
    ext = [(int(k) << 32) | j for j, k in enumerate(keys_sorted)]  # 95-bit codes, index tie-break
    out = set()
    stack = [(0, n - 1)]
    while stack:
        f, l = stack.pop()
        if f == l:
            continue
        x = ext[f] ^ ext[l]
        top = x.bit_length() - 1
        # split = last index whose bit `top` equals that of ext[f]
        lo_, hi_ = f, l
        while lo_ + 1 < hi_:
            m = (lo_ + hi_) // 2
            if (ext[m] >> top) & 1 == (ext[f] >> top) & 1:
                lo_ = m
            else:
                hi_ = m
        s = lo_
        out.add((f, l, s))
        stack += [(f, s), (s + 1, l)]
    return out


def tree_ranges(bvh, n):
    """(first, last, split) of every internal node of the oracle tree"""
    L0 = n - 1
    rng = {}

    def visit(i):
        if i >= L0:
            return (i - L0, i - L0)
        a = visit(int(bvh["left"][i]))
        b = visit(int(bvh["right"][i]))
        assert a[1] + 1 == b[0]
        rng[i] = (a[0], b[1], a[1])
        return (a[0], b[1])

    import sys
    sys.setrecursionlimit(100000)
    visit(0)
    return rng


@pytest.mark.parametrize("n,seed,kind", [(256, 0, "uniform"), (3000, 5, "blob"), (2, 1, "uniform"),
                                         (1, 1, "uniform"), (777, 9, "dups")])
def test_lbvh_structure(orc, n, seed, kind):
    if kind == "blob":
        params = gen.blob_scene(n, seed)
    else:
        params = gen.uniform_scene(n, seed)
    if kind == "dups":
        params[:, 0:3] = params[seed % 5, 0:3]  # all means equal: keys all zero
        params[::3, 0:3] = params[1, 0:3] + np.float32(0.25)
    bvh = orc.lbvh(params)
    keys_ref = morton_ref(params)
    order = np.lexsort((np.arange(n), keys_ref))
    assert np.array_equal(bvh["perm"], order.astype(np.int32))
    assert np.array_equal(bvh["keys"], keys_ref[order])
    if n == 1:
        assert bvh["parent"][0] == -1
    else:
        rng = tree_ranges(bvh, n)
        assert len(rng) == n - 1
        assert set(rng.values()) == radix_tree_ref(bvh["keys"])
        # Karras numbering: internal node i is an end point of its own range
        for i, (f, l, _) in rng.items():
            assert i in (f, l)
        # parents consistent, every node but the root has one
        par = bvh["parent"]
        assert par[0] == -1
        for i in range(n - 1):
            assert par[bvh["left"][i]] == i and par[bvh["right"][i]] == i
        assert np.all(par[1:] >= 0)
    # leaf boxes: outward-rounded r * sqrt(diag(Sigma)) around mu
    L0 = n - 1
    for j in range(n):
        p = params[bvh["perm"][j]].astype(np.float64)
        w, x, y, z = p[3:7] / np.sqrt(((p[3] ** 2 + p[4] ** 2) + p[5] ** 2) + p[6] ** 2)
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        e = 3.0 * np.sqrt(((R * p[7:10]) ** 2).sum(axis=1))
        bx = bvh["aabb"][L0 + j].astype(np.float64)
        assert np.all(bx[0:3] <= p[0:3] - e) and np.all(bx[3:6] >= p[0:3] + e)
        # tight: within one float32 ulp
        assert np.all(p[0:3] - e - bx[0:3] <= np.spacing(np.float32(np.abs(bx[0:3]).max() + 1e-30)) * 1.0001)
    # internal boxes are unions, cells are ORs
    for i in range(n - 1):
        a, b = bvh["left"][i], bvh["right"][i]
        assert np.array_equal(bvh["aabb"][i, 0:3], np.minimum(bvh["aabb"][a, 0:3], bvh["aabb"][b, 0:3]))
        assert np.array_equal(bvh["aabb"][i, 3:6], np.maximum(bvh["aabb"][a, 3:6], bvh["aabb"][b, 3:6]))
        assert bvh["cellor"][i] == bvh["cellor"][a] | bvh["cellor"][b]


def test_leaf_box_contains_ellipsoid_surface(orc):
    params = gen.uniform_scene(64, 3)
    bvh = orc.lbvh(params)
    g = np.random.default_rng(0)
    for j in range(64):
        p = params[bvh["perm"][j]].astype(np.float64)
        w, x, y, z = p[3:7] / np.linalg.norm(p[3:7])
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        u = g.standard_normal((2000, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        pts = p[0:3] + 3.0 * (u * p[7:10]) @ R.T
        bx = bvh["aabb"][63 + j]
        assert np.all(pts >= bx[0:3]) and np.all(pts <= bx[3:6])


def test_traversal_hit_set_equals_brute_force(orc):
    params = gen.blob_scene(4000, 7)
    bvh = orc.lbvh(params)
    rays = np.concatenate([gen.pinhole_rays(32, 32), gen.random_rays(512, 8)])
    for cells in (orc.FULL_MASK, orc.lod_cells(2), 0b000000111):
        nn, nh = orc.traverse_counts(params, bvh, rays, cells=cells)
        _, _, hits = orc.tau(params, rays, cells=cells)
        assert np.array_equal(nh, hits)
        assert np.all(nn >= nh)
    bits = orc.mask_cone(params)
    nn, nh = orc.traverse_counts(params, bvh, rays, bits=bits)
    assert np.array_equal(nh, orc.tau(params, rays, bits=bits)[2])
