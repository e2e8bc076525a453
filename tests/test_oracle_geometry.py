"""Pins of the oracle's ray march against brute force.

For every cell (or octree leaf) the length of the ray r + t k, t >= 0, inside
the cell's box is computed independently by slab intersection; the march's
per-cell path lengths must agree to 1e-12, and their sum must equal the chord
through the grid's bounding box.  A uniformly refined octree must reproduce
the Cartesian march of the equivalent lattice segment by segment.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_1705_04702_amd import scenes


def chord(lo, hi, r, k):
    """Length of {r + t k : t >= 0} inside the box [lo, hi] (slab method)."""
    tn, tf = 0.0, np.inf
    for a in range(3):
        if k[a] == 0.0:
            if r[a] < lo[a] or r[a] > hi[a]:
                return 0.0
            continue
        t1 = (lo[a] - r[a]) / k[a]
        t2 = (hi[a] - r[a]) / k[a]
        tn = max(tn, min(t1, t2))
        tf = min(tf, max(t1, t2))
    return max(0.0, tf - tn)


def cartesian_boxes(box, n):
    d = [(box[3 + a] - box[a]) / n[a] for a in range(3)]
    out = {}
    for iz, iy, ix in itertools.product(range(n[2]), range(n[1]), range(n[0])):
        m = ix + n[0] * (iy + n[1] * iz)
        lo = [box[0] + ix * d[0], box[1] + iy * d[1], box[2] + iz * d[2]]
        hi = [lo[0] + d[0], lo[1] + d[1], lo[2] + d[2]]
        out[m] = (lo, hi)
    return out


def octree_boxes(box, leaves, depth):
    lv, lx, ly, lz = leaves
    N = 1 << depth
    d = [(box[3 + a] - box[a]) / N for a in range(3)]
    out = {}
    for m in range(lv.shape[0]):
        size = 1 << (depth - lv[m])
        o = [lx[m] * size, ly[m] * size, lz[m] * size]
        lo = [box[a] + o[a] * d[a] for a in range(3)]
        hi = [box[a] + (o[a] + size) * d[a] for a in range(3)]
        out[m] = (lo, hi)
    return out


def make_cart(box, n):
    nc = n[0] * n[1] * n[2]
    return scenes.Scene(grid_type="cartesian", box=tuple(box), n=tuple(n),
                        density=np.ones(nc, np.float32), lambdas=np.array([1.0]),
                        kappa=np.array([1.0]), albedo=np.array([0.5]), hg_g=np.array([0.0]),
                        lum=np.array([1.0]), source="point_iso", instruments=[])


def make_oct(box, fc, nleaves):
    return scenes.Scene(grid_type="octree", box=tuple(box), first_child=fc,
                        density=np.ones(nleaves, np.float32), lambdas=np.array([1.0]),
                        kappa=np.array([1.0]), albedo=np.array([0.5]), hg_g=np.array([0.0]),
                        lum=np.array([1.0]), source="point_iso", instruments=[])


def random_rays(rng, box, n, outside_frac=0.4):
    lo = np.array(box[:3])
    hi = np.array(box[3:])
    span = hi - lo
    rays = []
    for i in range(n):
        if rng.random() < outside_frac:
            r = lo - 0.5 * span + 2.0 * span * rng.random(3)
        else:
            r = lo + span * rng.random(3)
        k = rng.normal(size=3)
        k /= np.linalg.norm(k)
        rays.append((r, k))
    return rays


def special_rays(box, n):
    """Rays along axes, through cell corners and edges, starting on faces."""
    lo = np.array(box[:3])
    hi = np.array(box[3:])
    d = (hi - lo) / np.array(n)
    corner = lo + d * np.floor(np.array(n) / 2)  # a lattice corner
    rays = []
    for k in ([1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [1, 1, 1], [-1, 1, -1], [0, 1, -1]):
        k = np.array(k, float)
        k /= np.linalg.norm(k)
        rays.append((corner.copy(), k))
        rays.append((lo.copy(), k))
        rays.append((hi.copy(), k))
        rays.append((corner - 3 * (hi - lo) * k, k))  # from outside through a corner
    return rays


def entry_t(lo, hi, r, k):
    tn = 0.0
    for a in range(3):
        if k[a] != 0.0:
            tn = max(tn, min((lo[a] - r[a]) / k[a], (hi[a] - r[a]) / k[a]))
    return tn


def check_against_boxes(sc, boxes, rays, box, generic=True):
    """generic: the ray lies on no cell face, so every cell's chord is unique
    and must match.  Otherwise (rays along faces, edges or through corners)
    each segment must lie in its cell's closed box and the segments must tile
    the chord through the grid."""
    for r, k in rays:
        cells, lens = oracle.march(sc, list(r), list(k))
        assert np.all(lens >= 0.0)
        total = chord(box[:3], box[3:], r, k)
        assert abs(sum(lens) - total) <= 1e-12 * max(1.0, total)
        if generic:
            got = {}
            for c, l in zip(cells, lens):
                got[int(c)] = got.get(int(c), 0.0) + float(l)
            for m, (lo, hi) in boxes.items():
                expect = chord(lo, hi, r, k)
                assert abs(got.get(m, 0.0) - expect) <= 1e-12 * max(1.0, total), (m, r, k)
        else:
            t = entry_t(box[:3], box[3:], r, k) if total > 0 else 0.0
            for c, l in zip(cells, lens):
                mid = np.asarray(r) + (t + 0.5 * l) * np.asarray(k)
                lo, hi = boxes[int(c)]
                tol = 1e-12 * (1.0 + np.abs(mid))
                assert np.all(mid >= np.asarray(lo) - tol) and np.all(mid <= np.asarray(hi) + tol), \
                    (c, r, k, mid)
                t += l


@pytest.mark.parametrize("box,n", [((-1, -1, -1, 1, 1, 1), (2, 2, 2)),
                                   ((0.0, -1.0, 2.0, 3.0, 3.0, 7.0), (3, 4, 5)),
                                   ((-1, -1, -1, 1, 1, 1), (1, 1, 1))])
def test_cartesian_march_brute_force(box, n):
    rng = np.random.default_rng(1)
    sc = make_cart(box, n)
    boxes = cartesian_boxes(box, n)
    check_against_boxes(sc, boxes, random_rays(rng, box, 300), box)
    check_against_boxes(sc, boxes, special_rays(box, n), box, generic=False)


def test_cartesian_march_misses_and_order():
    box = (-1, -1, -1, 1, 1, 1)
    sc = make_cart(box, (4, 4, 4))
    # pointing away from the box
    cells, lens = oracle.march(sc, [3.0, 0.0, 0.0], [1.0, 0.0, 0.0])
    assert len(cells) == 0
    # from the centre along +x: cells 2 and 3 of row (iy=2, iz=2), 0.5 each
    cells, lens = oracle.march(sc, [0.0, 0.0, 0.0], [1.0, 0.0, 0.0])
    assert list(cells) == [2 + 4 * (2 + 4 * 2), 3 + 4 * (2 + 4 * 2)]
    assert np.allclose(lens, [0.5, 0.5], rtol=0, atol=1e-15)
    # along -x from the centre enters the cell below the plane
    cells, lens = oracle.march(sc, [0.0, 0.0, 0.0], [-1.0, 0.0, 0.0])
    assert list(cells) == [1 + 4 * (2 + 4 * 2), 0 + 4 * (2 + 4 * 2)]


@pytest.mark.parametrize("seed,depth", [(0, 3), (1, 4), (2, 2)])
def test_octree_march_brute_force(seed, depth):
    box = (-1.0, -2.0, 0.0, 1.0, 2.0, 3.0)
    fc, leaves, D = scenes.random_octree(depth, 0.45, seed)
    sc = make_oct(box, fc, leaves[0].shape[0])
    boxes = octree_boxes(box, leaves, D)
    rng = np.random.default_rng(seed + 10)
    check_against_boxes(sc, boxes, random_rays(rng, box, 150), box)
    check_against_boxes(sc, boxes, special_rays(box, (8, 8, 8)), box, generic=False)


def test_uniform_octree_equals_cartesian():
    depth = 3
    box = (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)
    fc, leaves, D = scenes.uniform_octree(depth)
    n = 1 << depth
    oc = make_oct(box, fc, leaves[0].shape[0])
    ca = make_cart(box, (n, n, n))
    lv, lx, ly, lz = leaves
    leaf_to_cart = lx + n * (ly + n * lz)
    rng = np.random.default_rng(5)
    for r, k in random_rays(rng, box, 200) + special_rays(box, (n, n, n)):
        c1, l1 = oracle.march(oc, list(r), list(k))
        c2, l2 = oracle.march(ca, list(r), list(k))
        assert list(leaf_to_cart[c1]) == list(c2)
        assert np.array_equal(l1, l2)
