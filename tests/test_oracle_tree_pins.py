"""Pins of the oracle's quadtree rules that symmetry and invariants alone do
not fix (paper Sec. 3.1: particles reassigned when cells refine or coarsen,
ghost cells at +-1 level for direct and diagonal neighbours; Sec. 3:
potential at cell centres, bilinear gather from nodal E; Sec. 4.3: merging
particles when a cell holds too many).

Each test builds its tree leaf by leaf (explicit-tree input), so the
expected result is written down from the geometry, not taken from the
oracle:
  - the coarsen rule on a hand-built tree, every condition exercised by its
    own sibling group;
  - the coarse-fine face coefficient of the finite-volume operator: exact
    flux of a linear potential across faces between levels, and second-order
    convergence of a manufactured solution on trees with such faces;
  - the cell-to-node potential at hanging nodes, exact for linear
    potentials against the mean of the incident leaf centres;
  - the merge pairing order (velocity octant, |v|^2, id) on one leaf whose
    pairs are listed by hand.
"""
import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.linalg

import oracle
from paper_1604_07713_amd import inputs as I


def morton(x, y):
    k = 0
    for b in range(16):
        k |= ((x >> b) & 1) << (2 * b)
        k |= ((y >> b) & 1) << (2 * b + 1)
    return k


def leaf_key(level, ix, iy):
    sh = 16 - level
    return morton(ix << sh, iy << sh)


def explicit(desc, leaves):
    """leaves: [(level, ix, iy)] in any order -> desc with the explicit tree."""
    leaves = sorted(leaves, key=lambda t: leaf_key(*t))
    d = dict(desc)
    d["leaf_keys"] = np.array([leaf_key(*t) for t in leaves], dtype=np.uint32)
    d["leaf_levels"] = np.array([t[0] for t in leaves], dtype=np.uint8)
    return d, leaves


def box(level, ix, iy):
    h = 2.0 ** -level
    return ix * h, iy * h, (ix + 1) * h, (iy + 1) * h


def points_in(rng, level, ix, iy, n):
    x0, y0, x1, y1 = box(level, ix, iy)
    return np.stack([rng.uniform(x0, x1, n), rng.uniform(y0, y1, n)], axis=1)


# ---------------------------------------------------------------------------
# explicit-tree input
# ---------------------------------------------------------------------------
def _desc(lmin, lmax, **kw):
    d = I.streamer_desc(min_level=lmin, max_level=lmax, precision=64, **kw)
    d["base_level"] = lmin
    return d


def test_explicit_tree_round_trip_and_rejections():
    d = I.quadtree_static_desc(precision=64)
    keys, lv = oracle.Oracle(d).leaves()
    e = dict(d, leaf_keys=keys, leaf_levels=lv, refine_disk=0)
    k2, l2 = oracle.Oracle(e).leaves()
    assert np.array_equal(keys, k2) and np.array_equal(lv, l2)
    uni = [(1, i, j) for i in range(2) for j in range(2)]
    # a gap (one leaf missing), a misaligned key, a level outside the bounds
    for bad in (uni[:3], None, [(0, 0, 0)]):
        if bad is None:
            dd = explicit(_desc(1, 3), uni)[0]
            dd["leaf_keys"] = dd["leaf_keys"].copy()
            dd["leaf_keys"][1] += 1
        else:
            dd = explicit(_desc(1, 3), bad)[0]
        with pytest.raises(oracle.OracleError):
            oracle.Oracle(dd)
    # not 2:1 balanced: a level-3 leaf next to a level-1 leaf
    unbal = [(1, 1, 0), (1, 0, 1), (1, 1, 1), (2, 0, 0), (2, 1, 0), (2, 0, 1)]
    unbal += [(3, 2 + i, 2 + j) for i in range(2) for j in range(2)]
    with pytest.raises(oracle.OracleError):
        oracle.Oracle(explicit(_desc(1, 3), unbal)[0])


# ---------------------------------------------------------------------------
# coarsen rule
# ---------------------------------------------------------------------------
def coarsen_case():
    """Level-2 parents P(i, j), each with four level-3 children, except that
    the SW child of P(2, 2) is refined to level 4.  Sibling groups:
      A = P(0, 0): 10 electrons and 10 ions per child   -> coarsens
      B = P(3, 0): 20 per child (sum 80 > 64)           -> stays
      C = P(0, 3): 16 per child (no child below 16)     -> stays
      D = P(1, 2): 10 per child, a level-4 leaf touches its face   -> stays
      E = P(1, 1): 10 per child, a level-4 leaf touches its corner -> stays
      the four level-4 leaves: 20 each (sum 80)         -> stay
    every other leaf holds 30 (its group sums to 120)."""
    counts_e, counts_i = {}, {}
    leaves = []
    for i in range(4):
        for j in range(4):
            for c in range(4):
                ix, iy = 2 * i + (c & 1), 2 * j + (c >> 1)
                if (i, j) == (2, 2) and c == 0:
                    for q in range(4):
                        t = (4, 2 * ix + (q & 1), 2 * iy + (q >> 1))
                        leaves.append(t)
                        counts_e[t] = 20
                    continue
                t = (3, ix, iy)
                leaves.append(t)
                counts_e[t] = {(0, 0): 10, (3, 0): 20, (0, 3): 16, (1, 2): 10, (1, 1): 10}.get((i, j), 30)
                if (i, j) == (0, 0):
                    counts_i[t] = 10
    return leaves, counts_e, counts_i


def check_coarsen_rule(library=None):
    leaves, ce, ci = coarsen_case()
    d, leaves = explicit(_desc(2, 4), leaves)
    o = oracle.Oracle(d, library)
    rng = np.random.Generator(np.random.PCG64(31))
    pe = np.concatenate([points_in(rng, *t, ce[t]) for t in leaves])
    pi = np.concatenate([points_in(rng, *t, ci[t]) for t in leaves if t in ci])
    o.load(0, pe, np.zeros((len(pe), 3)), ids=np.arange(len(pe), dtype=np.uint32))
    o.load(1, pi, np.zeros((len(pi), 3)), ids=np.arange(len(pe), len(pe) + len(pi), dtype=np.uint32))
    st = o.adapt(16, 64)
    # expected: group A replaced by its level-2 parent, nothing else changes
    a_kids = {(3, x, y) for x in (0, 1) for y in (0, 1)}
    want = [t for t in leaves if t not in a_kids] + [(2, 0, 0)]
    want = sorted(want, key=lambda t: leaf_key(*t))
    keys, lv = o.leaves()
    assert st["coarsened"] == 1 and st["refined"] == 0 and st["balance_refined"] == 0
    assert list(lv) == [t[0] for t in want]
    assert list(keys) == [leaf_key(*t) for t in want]


def test_coarsen_rule_on_hand_built_tree():
    check_coarsen_rule()


# ---------------------------------------------------------------------------
# coarse-fine face coefficient of the FV operator
# ---------------------------------------------------------------------------
def strip_tree(L, axis):
    """Uniform at level L, refined to L + 1 in two strips across the square
    (cells whose centre coordinate along 'axis' is in [0.25, 0.5) or
    [0.625, 0.75)): every coarse-fine face is normal to 'axis', and the faces
    along it join leaves of one level."""
    leaves = []
    n = 2 ** L
    for i in range(n):
        for j in range(n):
            c = i if axis == 0 else j
            u = (c + 0.5) / n
            if 0.25 <= u < 0.5 or 0.625 <= u < 0.75:
                leaves += [(L + 1, 2 * i + (q & 1), 2 * j + (q >> 1)) for q in range(4)]
            else:
                leaves.append((L, i, j))
    return leaves


def fv_strip_case(L, axis, library=None):
    """Dirichlet walls normal to 'axis' (zero), Neumann walls along it.
    Returns (max |A u| over rows away from the Dirichlet walls for the linear
    potential u = coordinate along 'axis', max error of the solution of the
    assembled operator for phi = sin(pi u), f = pi^2 phi, right-hand side
    f h^2)."""
    d = I.streamer_desc(min_level=L, max_level=L + 1, precision=64)
    d.update(field_bc=[1, 1, 0, 0] if axis == 0 else [0, 0, 1, 1], wall_phi=[0.0] * 4, length=1.0, depth_z=1.0)
    d, _ = explicit(d, strip_tree(L, axis))
    o = oracle.Oracle(d, library)
    keys, lv = o.leaves()
    cx, cy = I.leaf_corners(keys, lv)
    lo, hi = (cx[:, 0], cx[:, 1]) if axis == 0 else (cy[:, 0], cy[:, 2])
    u = (lo + hi) / 2
    h = np.ldexp(1.0, -lv.astype(int))
    rows, cols, vals, rhs = o.assemble_2d()
    A = scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(len(keys), len(keys)))
    inner = (lo > 0) & (hi < 1)
    lin = float(np.max(np.abs((A @ u)[inner])))
    exact = np.sin(np.pi * u)
    phi = scipy.sparse.linalg.spsolve(A.tocsc(), np.pi ** 2 * exact * h * h + rhs)
    return lin, float(np.max(np.abs(phi - exact)))


def check_fv_coarse_fine_faces(axis, library=None):
    """Across a face between leaves one level apart the two-point flux of
    a potential varying only normal to the face must equal the face length
    times the gradient: the operator annihilates a linear potential away from
    Dirichlet walls, and a smooth solution converges at second order."""
    errs = []
    for L in (3, 4, 5):
        lin, err = fv_strip_case(L, axis, library)
        assert lin <= 1e-12, (L, lin)
        errs.append(err)
    assert errs[1] < errs[0] / 3.5 and errs[2] < errs[1] / 3.5, errs


@pytest.mark.parametrize("axis", [0, 1])
def test_fv_coarse_fine_faces(axis):
    check_fv_coarse_fine_faces(axis)


# ---------------------------------------------------------------------------
# cell potential -> node potential at hanging nodes
# ---------------------------------------------------------------------------
def node_incidence(keys, lv):
    """node (X, Y in 16-bit units) -> leaves having it as one of their corners"""
    cx, cy = I.leaf_corners(keys, lv)
    inc = {}
    for l in range(len(keys)):
        for c in range(4):
            X, Y = int(round(cx[l, c] * 65536)), int(round(cy[l, c] * 65536))
            inc.setdefault((X, Y), []).append(l)
    return cx, cy, inc


def check_hanging_nodes(dirichlet, library=None):
    d = I.streamer_desc(min_level=2, max_level=5, precision=64)
    d.update(base_level=2, refine_disk=1, disk_cx=0.37, disk_cy=0.61, disk_r=0.2, disk_level=5, length=1.0)
    walls = [0.7, -1.5, 2.0, 3.25]
    d["field_bc"] = [1, 0, 1, 1] if dirichlet else [0, 0, 0, 0]
    d["wall_phi"] = walls
    o = oracle.Oracle(d, library)
    keys, lv = o.leaves()
    cx, cy, inc = node_incidence(keys, lv)
    xc, yc = (cx[:, 0] + cx[:, 1]) / 2, (cy[:, 0] + cy[:, 2]) / 2
    a, bx, by = 0.25, 3.0, -2.0
    o.field_set(oracle.CELL_PHI_2D, a + bx * xc + by * yc)
    cphi = o.corner_phi()
    hanging = 0
    for (X, Y), ls in inc.items():
        if dirichlet and (X == 0 or Y == 0 or Y == 65536):
            # Dirichlet walls in the order x0, x1, y0, y1 (x1 is Neumann here)
            want = walls[0] if X == 0 else (walls[2] if Y == 0 else walls[3])
        else:
            want = a + bx * np.mean(xc[ls]) + by * np.mean(yc[ls])
        for l in ls:
            c = [k for k in range(4) if int(round(cx[l, k] * 65536)) == X and int(round(cy[l, k] * 65536)) == Y][0]
            assert abs(cphi[l, c] - want) <= 1e-13 * (1 + abs(want))
        # a hanging node: on the edge of a coarser leaf that does not have it as a corner
        hanging += int(len(ls) == 2 and 0 < X < 65536 and 0 < Y < 65536)
    assert hanging > 0


@pytest.mark.parametrize("dirichlet", [False, True])
def test_hanging_node_potential_is_mean_of_incident_leaves(dirichlet):
    check_hanging_nodes(dirichlet)


# ---------------------------------------------------------------------------
# merge pairing order
# ---------------------------------------------------------------------------
MERGE_CASE = {   # name: (id, velocity / 1e5); octant bits: vx < 0, vy < 0, vz < 0
    "a": (10, (2, 0, 0)),     # octant 0, |v|^2 4
    "b": (20, (0, 1, 0)),     # octant 0, |v|^2 1
    "c": (30, (-1, 1, 0)),    # octant 1, |v|^2 2
    "d": (5, (-3, 0, 0)),     # octant 1, |v|^2 9
    "e": (3, (0, 0, 2)),      # octant 0, |v|^2 4 (ties a; smaller id)
    "f": (7, (0, -1, 0)),     # octant 2, |v|^2 1
    "g": (1, (-1, 0, 1)),     # octant 1, |v|^2 2 (ties c; smaller id)
    "h": (8, (0, -4, 0)),     # octant 2, |v|^2 16
}
# sorted by (octant, |v|^2, id): b e a | g c d | f h  -> pairs in that order
MERGE_PAIRS = [("b", "e"), ("a", "g"), ("c", "d"), ("f", "h")]


def check_merge_pairs(library=None):
    d = _desc(1, 1)
    o = oracle.Oracle(d, library)
    rng = np.random.Generator(np.random.PCG64(17))
    names = sorted(MERGE_CASE)
    s = rng.uniform(0.0, 0.5, (len(names), 2))                 # all in the SW leaf
    ids = np.array([MERGE_CASE[k][0] for k in names], dtype=np.uint32)
    v = np.array([MERGE_CASE[k][1] for k in names], dtype=np.float64) * 1e5
    o.load(0, s, v, ids=ids)
    o.load(1, s[:0], v[:0], ids=np.zeros(0, dtype=np.uint32))
    st = o.adapt(1, 4)                                          # 8 > 4: one round of pairs
    r = o.read(0)
    assert st["merged_pairs"] == 4 and len(r["id"]) == 4
    at = {k: i for i, k in enumerate(names)}
    for p, q in MERGE_PAIRS:
        keep = min(MERGE_CASE[p][0], MERGE_CASE[q][0])
        j = int(np.nonzero(r["id"] == keep)[0][0])
        assert r["w"][j] == 2 * 65536
        assert np.array_equal(r["v"][j], (v[at[p]] + v[at[q]]) / 2.0)
        assert np.allclose(r["s"][j], (s[at[p]] + s[at[q]]) / 2.0, rtol=0, atol=1e-16)


def test_merge_pairs_in_written_order():
    check_merge_pairs()


# ---------------------------------------------------------------------------
# charge density
# ---------------------------------------------------------------------------
def test_rho_integrates_to_total_charge():
    d = I.streamer_desc(min_level=2, max_level=5, precision=64)
    d.update(base_level=2, refine_disk=1, disk_cx=0.37, disk_cy=0.61, disk_r=0.2, disk_level=5)
    o = oracle.Oracle(d)
    rng = np.random.Generator(np.random.PCG64(6))
    n = 3000
    w = rng.integers(1, 1 << 17, n).astype(np.uint32)
    o.load(0, rng.random((n, 2)), np.zeros((n, 3)), w=w, ids=np.arange(n, dtype=np.uint32))
    o.load(1, rng.random((n // 2, 2)), np.zeros((n // 2, 3)), ids=np.arange(n, n + n // 2, dtype=np.uint32))
    o.deposit()
    keys, lv = o.leaves()
    h = d["length"] * np.ldexp(1.0, -lv.astype(int))
    total = np.sum(o.rho() * h * h * d["depth_z"])
    qe, qi = d["species"][0]["charge"] * d["species"][0]["w0"], d["species"][1]["charge"] * d["species"][1]["w0"]
    want = qe * float(np.sum(w.astype(np.float64))) / 65536.0 + qi * (n // 2)
    assert abs(total - want) <= 1e-12 * abs(qi * n)
    # 1D: the node sums over dx integrate to the charge per unit area
    d1 = I.ccp_desc(ncells=50, ppc=4)
    o1 = oracle.Oracle(d1)
    o1.load(0, rng.random((200, 1)), np.zeros((200, 3)), ids=np.arange(200, dtype=np.uint32))
    o1.deposit()
    dx = d1["length"] / 50
    tot1 = np.sum(o1.rho()) * dx
    want1 = d1["species"][0]["charge"] * d1["species"][0]["w0"] * 200
    assert abs(tot1 - want1) <= 1e-12 * abs(want1)


def test_cell_e_kind_only_on_energy_conserving_slots():
    d = I.ccp_desc(ncells=16, ppc=2)
    o = oracle.Oracle(d)
    with pytest.raises(oracle.OracleError):
        o.field_set(oracle.CELL_E_1D, np.zeros(16))
    d["field_scheme"] = I.FIELD_CIC_EC
    o = oracle.Oracle(d)
    with pytest.raises(oracle.OracleError):
        o.field_set(oracle.NODE_E_1D, np.zeros(17))
    e = np.arange(16, dtype=np.float64) * 10.0 + 1.0
    o.field_set(oracle.CELL_E_1D, e)
    assert np.array_equal(o.field_table()[:16], e) and o.field_table()[16] == 0.0
