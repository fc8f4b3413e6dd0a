"""Oracle cloud-in-cell on the quadtree (paper Sec. 3.1, Fig. 2: the shape
function of a particle covers its cell and the direct and diagonal
neighbours, through ghost cells at +-1 level where the neighbours differ in
level; charge conservation needs the same shape function for scatter and
gather), pinned by brute force geometry:

  - the charge a particle gives each leaf is its cloud's ghost-cell shares
    spread over the leaves by the area each ghost cell has in each leaf
    (computed here from leaf boxes), up to the integer remainders;
  - on a uniform tree this is the textbook 2D cloud-in-cell (bilinear
    weights on the four nearest cell centres, computed here from the lower
    left centre), and the first moment of the charge is the particle's;
  - charge sums are exact; the gather of any cell field is the deposit's
    weights applied to it (the same shape function both ways); the gather is
    exact for linear fields where the tree is uniform.
"""
import numpy as np
import pytest

import oracle
from paper_1604_07713_amd import inputs as I

H64 = 16      # fraction bits per axis of the FP64 cloud (F = 32)


def tree_desc(base=3, top=5, disk=True, precision=64, r=0.2):
    e = I.species(-I.E_CHARGE, I.M_ELECTRON, 1.0, I.MCC_NONE)
    return I.base_desc(dim=2, precision=precision, length=1.0, dt=1e-12, min_level=base, max_level=top,
                       base_level=base, refine_disk=1 if disk else 0, disk_cx=0.41, disk_cy=0.57, disk_r=r,
                       disk_level=top, species=[e], gas_mass=1.0, field_scheme=I.FIELD_CIC_AMR)


def boxes(o):
    keys, lv = o.leaves()
    cx, cy = I.leaf_corners(keys, lv)
    return cx[:, 0], cy[:, 0], cx[:, 1], cy[:, 2], lv


def cloud_cells(x, y, lv_of, x0, y0, H):
    """The four level-L ghost cells of a particle at (x, y) in leaf of level
    L with low corner (x0, y0): their boxes (folded at the walls) and
    integer shares in units of 2^-2H."""
    h = 2.0 ** -int(lv_of)
    gx = (x - x0) / h - 0.5
    gy = (y - y0) / h - 0.5
    o = 1 << H
    rx = int(np.rint(abs(gx) * o))
    ry = int(np.rint(abs(gy) * o))
    sx = h if gx >= 0 else -h
    sy = h if gy >= 0 else -h
    xn = x0 + sx if 0 <= x0 + sx < 1 else x0        # folded back at a wall
    yn = y0 + sy if 0 <= y0 + sy < 1 else y0
    return [((x0, y0), (o - rx) * (o - ry)), ((xn, y0), rx * (o - ry)),
            ((x0, yn), (o - rx) * ry), ((xn, yn), rx * ry)], h


def brute_shares(o, x, y, w, H):
    """Charge units per leaf of one particle: each ghost cell's share spread
    over the leaves by area overlap."""
    bx0, by0, bx1, by1, lv = boxes(o)
    me = np.nonzero((x >= bx0) & (x < bx1) & (y >= by0) & (y < by1))[0][0]
    cells, h = cloud_cells(x, y, lv[me], bx0[me], by0[me], H)
    out = np.zeros(len(lv))
    for (cx0, cy0), share in cells:
        ox = np.clip(np.minimum(bx1, cx0 + h) - np.maximum(bx0, cx0), 0, None)
        oy = np.clip(np.minimum(by1, cy0 + h) - np.maximum(by0, cy0), 0, None)
        out += w * share * (ox * oy) / (h * h)
    return out


def check_area_overlaps(seed, library=None):
    d = tree_desc()
    o = oracle.Oracle(d, library)
    rng = np.random.Generator(np.random.PCG64(seed))
    for k in range(60):
        x, y = rng.random(2)
        if k < 20:   # near the refined disk: interfaces between levels
            a = rng.random() * 2 * np.pi
            x, y = 0.41 + 0.2 * np.cos(a) + rng.normal(0, 0.02), 0.57 + 0.2 * np.sin(a) + rng.normal(0, 0.02)
            x, y = min(max(x, 0.0), 0.999), min(max(y, 0.0), 0.999)
        w = int(rng.integers(1, 1 << 16))
        o.load(0, np.array([[x, y]]), np.zeros((1, 3)), w=np.array([w], dtype=np.uint32))
        q = o.deposit()[0].astype(np.float64)
        want = brute_shares(o, x, y, w, H64)
        assert int(o.deposit()[0].astype(object).sum()) == w << (2 * H64)     # exact total
        # equal up to the remainder of the integer split among finer leaves
        assert np.max(np.abs(q - want)) <= 64.0, (x, y, np.max(np.abs(q - want)))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_single_particle_shares_are_area_overlaps(seed):
    check_area_overlaps(seed)


def test_uniform_tree_is_textbook_cic_with_exact_moments():
    L = 4
    d = tree_desc(base=L, top=L, disk=False)
    o = oracle.Oracle(d)
    h = 2.0 ** -L
    rng = np.random.Generator(np.random.PCG64(9))
    bx0, by0, bx1, by1, lv = boxes(o)
    for _ in range(40):
        x, y = rng.uniform(0.6 * h, 1 - 0.6 * h, 2)     # away from the walls
        o.load(0, np.array([[x, y]]), np.zeros((1, 3)), w=np.array([1], dtype=np.uint32))
        q = o.deposit()[0].astype(np.float64)
        # textbook: lower-left cell centre and fractions from it
        i0, j0 = int(np.floor(x / h - 0.5)), int(np.floor(y / h - 0.5))
        fx, fy = x / h - 0.5 - i0, y / h - 0.5 - j0
        want = np.zeros(len(lv))
        o_ = 1 << H64
        for di, wx in ((0, 1 - fx), (1, fx)):
            for dj, wy in ((0, 1 - fy), (1, fy)):
                leaf = np.nonzero((np.isclose(bx0, (i0 + di) * h)) & (np.isclose(by0, (j0 + dj) * h)))[0][0]
                want[leaf] += wx * wy * o_ * o_
        assert np.max(np.abs(q - want)) <= 2.0 * o_   # the fixed-point rounding of each axis fraction
        # first moment: the charge-weighted cell centres are the particle's position
        xc, yc = (bx0 + bx1) / 2, (by0 + by1) / 2
        tot = q.sum()
        assert abs((q * xc).sum() / tot - x) <= h * 2.0 ** -(H64) and abs((q * yc).sum() / tot - y) <= h * 2.0 ** -H64


def test_charge_exact_on_refined_tree_with_walls():
    d = tree_desc(base=2, top=6, r=0.3)
    o = oracle.Oracle(d)
    rng = np.random.Generator(np.random.PCG64(4))
    n = 20000
    s = rng.random((n, 2))
    s[:200] = rng.random((200, 2)) * 0.01            # corners and walls
    s[200:400, 0] = 1 - rng.random(200) * 1e-3
    w = rng.integers(1, 1 << 20, n).astype(np.uint32)
    o.load(0, s, np.zeros((n, 3)), w=w)
    q = o.deposit()[0]
    assert int(q.astype(object).sum()) == int(w.astype(object).sum()) << (2 * H64)


def test_gather_is_the_deposit_weights_applied_to_the_field():
    d = tree_desc(base=2, top=5, r=0.25)
    o = oracle.Oracle(d)
    rng = np.random.Generator(np.random.PCG64(5))
    E = rng.normal(0, 1e3, (o.nq(), 2))
    o.field_set(oracle.CELL_E_2D, E)
    pts = rng.random((80, 2))
    got = o.gather(pts)
    for k, (x, y) in enumerate(pts):
        # a heavy particle: the integer split of its shares among finer
        # leaves then rounds at 2^-48 of a share
        o.load(0, np.array([[x, y]]), np.zeros((1, 3)), w=np.array([65536], dtype=np.uint32))
        wts = o.deposit()[0].astype(np.float64) / 2.0 ** (2 * H64 + 16)
        want = wts @ E
        assert np.allclose(got[k], want, rtol=0, atol=1e-11 * np.abs(E).max()), (x, y, got[k], want)


def test_gather_exact_for_linear_field_where_uniform():
    L = 4
    d = tree_desc(base=L, top=L, disk=False)
    o = oracle.Oracle(d)
    bx0, by0, bx1, by1, lv = boxes(o)
    xc, yc = (bx0 + bx1) / 2, (by0 + by1) / 2
    a, b, c = 2.5, -1.75, 0.5
    o.field_set(oracle.CELL_E_2D, np.stack([a + b * xc + c * yc, c - b * xc + a * yc], 1))
    h = 2.0 ** -L
    pts = np.random.Generator(np.random.PCG64(6)).uniform(0.5 * h, 1 - 0.5 * h, (200, 2))
    got = o.gather(pts)
    # the cloud's fractions are rounded to 2^-16 of a cell: exact up to that
    tol = (abs(b) + abs(c) + abs(a)) * h * 2.0 ** -H64 * 2
    assert np.allclose(got[:, 0], a + b * pts[:, 0] + c * pts[:, 1], rtol=0, atol=tol)
    assert np.allclose(got[:, 1], c - b * pts[:, 0] + a * pts[:, 1], rtol=0, atol=tol)
