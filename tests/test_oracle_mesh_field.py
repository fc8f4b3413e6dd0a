"""Oracle deposit, quadtree locate and field solves pinned to brute force,
exact identities and library solvers (paper Sec. 3: NGP at cell centres, CIC
on the uniform mesh, Poisson for the potential; Sec. 3.1: particles kept in
the leaf cell that contains them, no volume weighting on the adaptive mesh)."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

import oracle
from paper_1604_07713_amd import inputs as I


def leaf_boxes(keys, lv):
    cx, cy = I.leaf_corners(keys, lv)
    return cx[:, 0], cy[:, 0], cx[:, 1], cy[:, 2]


def brute_locate(keys, lv, s):
    x0, y0, x1, y1 = leaf_boxes(keys, lv)
    out = np.empty(len(s), dtype=np.int64)
    for i, (x, y) in enumerate(s):
        hit = np.nonzero((x >= x0) & (x < x1) & (y >= y0) & (y < y1))[0]
        assert len(hit) == 1
        out[i] = hit[0]
    return out


def small_tree_desc(disk_r=0.2, cx=0.37, cy=0.61, base=2, top=5):
    e = I.species(-I.E_CHARGE, I.M_ELECTRON, 1.0, I.MCC_NONE)
    return I.base_desc(dim=2, precision=64, length=1.0, dt=1e-12, min_level=base, max_level=top,
                       base_level=base, refine_disk=1, disk_cx=cx, disk_cy=cy, disk_r=disk_r,
                       disk_level=top, species=[e], gas_mass=1.0)


def check_balanced(keys, lv):
    x0, y0, x1, y1 = leaf_boxes(keys, lv)
    for a in range(len(keys)):
        touch = (x0 <= x1[a]) & (x0[a] <= x1) & (y0 <= y1[a]) & (y0[a] <= y1)
        assert np.all(lv[touch].astype(int) <= int(lv[a]) + 1)


def test_quadtree_disk_mesh_brute_force():
    """The disk-refined mesh equals a direct construction: refine every cell
    whose closed box meets the closed disk, level by level, then balance."""
    d = I.quadtree_static_desc()
    o = oracle.Oracle(d)
    keys, lv = o.leaves()
    assert np.all(np.diff(keys.astype(np.int64)) > 0)          # Morton order
    x0, y0, x1, y1 = leaf_boxes(keys, lv)
    assert abs(np.sum((x1 - x0) * (y1 - y0)) - 1.0) == 0.0
    assert set(np.unique(lv)) <= {6, 7, 8, 9}
    # every level-9 leaf meets the disk or is there for balance; no coarse leaf meets it
    dx = np.maximum(np.maximum(x0 - 0.5, 0), 0.5 - x1)
    dy = np.maximum(np.maximum(y0 - 0.5, 0), 0.5 - y1)
    meets = dx * dx + dy * dy <= 0.15 * 0.15
    assert np.all(lv[meets] == 9)
    assert len(keys) == 23620
    assert list(np.bincount(lv)[6:]) == [3696, 284, 472, 19168]


def test_balance_small_tree():
    o = oracle.Oracle(small_tree_desc())
    keys, lv = o.leaves()
    check_balanced(keys, lv)


def test_locate_brute_force_with_edges():
    o = oracle.Oracle(small_tree_desc())
    keys, lv = o.leaves()
    x0, y0, x1, y1 = leaf_boxes(keys, lv)
    rng = np.random.Generator(np.random.PCG64(11))
    pts = [rng.random((300, 2))]
    # corners, face midpoints and hanging nodes of every leaf (inside the square)
    for xs, ys in ((x0, y0), (x1, y0), (x0, y1), ((x0 + x1) / 2, y0), (x0, (y0 + y1) / 2)):
        pts.append(np.stack([xs, ys], axis=1))
    p1 = np.nextafter(1.0, 0.0)
    pts.append(np.array([[0.0, 0.0], [p1, p1], [0.0, p1], [p1, 0.0], [0.5, 0.5]]))
    P = np.concatenate(pts)
    P = P[np.all(P < 1.0, axis=1)]
    assert np.array_equal(o.locate(P).astype(np.int64), brute_locate(keys, lv, P))


def test_cic_deposit_sums_and_first_moment():
    d = I.ccp_desc(ncells=100, ppc=10)
    for precision, F in ((64, 32), (32, 24)):
        d["precision"] = precision
        o = oracle.Oracle(d)
        rng = np.random.Generator(np.random.PCG64(3))
        n = 1000
        s = rng.random(n)
        w = rng.integers(1, 1 << 16, n, dtype=np.uint32)
        o.load(0, s[:, None], np.zeros((n, 3)), w=w, ids=np.arange(n, dtype=np.uint32))
        q = o.deposit()[0]
        tot = int(np.sum(q.astype(object)))
        assert tot == int(np.sum(w.astype(object))) << F
        # first moment in cells: sum_i i Q_i / 2^F = sum_p w_p g_p within 2^-(F+1) per particle
        s_p = o.read(0)["s"][:, 0]
        g = s_p * 100
        mom = sum(int(i) * int(qi) for i, qi in enumerate(q)) / 2.0 ** F
        exact = float(np.sum(w.astype(np.float64) * g))
        assert abs(mom - exact) <= np.sum(w) * 2.0 ** -(F + 1) + 1e-6 * exact


def test_ngp_deposit_counts_brute_force():
    o = oracle.Oracle(small_tree_desc())
    keys, lv = o.leaves()
    rng = np.random.Generator(np.random.PCG64(5))
    s = rng.random((4000, 2))
    w = rng.integers(1, 1000, 4000, dtype=np.uint32)
    o.load(0, s, np.zeros((4000, 3)), w=w)
    q = o.deposit()[0]
    idx = brute_locate(keys, lv, s)
    assert np.array_equal(q, np.bincount(idx, weights=w, minlength=len(keys)).astype(np.uint64))


def _poisson1d_case(N=64, L=0.05, V=123.0):
    d = I.ccp_desc(ncells=N, ppc=8, length=L)
    o = oracle.Oracle(d)
    return d, o


def test_poisson1d_uniform_charge_gives_parabola():
    N, L, V = 64, 0.05, 123.0
    d, o = _poisson1d_case(N, L, V)
    # uniform ion charge on every node: one ion per node, exactly on the node
    pos = np.arange(N + 1) / N
    pos = pos[pos < 1.0]
    o.load(1, pos[:, None], np.zeros((len(pos), 3)), ids=np.arange(len(pos), dtype=np.uint32))
    q = o.deposit()
    assert np.all(q[1][:N] == (1 << 16) << 32) and q[1][N] == 0
    phi, E = o.field_solve_1d(V)
    dx = L / N
    rho = I.E_CHARGE * d["species"][1]["w0"] / dx      # C/m^3 on nodes 1..N-1
    x = np.arange(N + 1) * dx
    exact = V * (1 - x / L) + rho / (2 * 8.8541878128e-12) * x * (L - x)
    assert np.allclose(phi, exact, rtol=1e-12, atol=1e-12 * V)
    Eex = V / L - rho / 8.8541878128e-12 * (L / 2 - x)
    assert np.allclose(E, Eex, rtol=1e-9, atol=1e-9 * np.max(np.abs(Eex)))


def test_poisson1d_matches_banded_solver():
    N, L, V = 97, 0.067, -37.5
    d, o = _poisson1d_case(N, L, V)
    rng = np.random.Generator(np.random.PCG64(8))
    n = 5000
    o.load(0, rng.random((n, 1)), np.zeros((n, 3)), ids=np.arange(n, dtype=np.uint32))
    o.load(1, rng.random((n, 1)), np.zeros((n, 3)), ids=np.arange(n, 2 * n, dtype=np.uint32))
    q = o.deposit().astype(np.float64)
    phi, E = o.field_solve_1d(V)
    dx = L / N
    F = 32
    kap = [sp["charge"] * sp["w0"] * 2.0 ** -(16 + F) * dx / 8.8541878128e-12 for sp in d["species"]]
    b = q[0] * kap[0] + q[1] * kap[1]
    rhs = b[1:N].copy()
    rhs[0] += V
    ab = np.zeros((3, N - 1))
    ab[0, 1:] = -1
    ab[1, :] = 2
    ab[2, :-1] = -1
    ref = scipy.linalg.solve_banded((1, 1), ab, rhs)
    assert np.allclose(phi[1:N], ref, rtol=1e-10, atol=1e-10 * np.max(np.abs(ref)))
    assert phi[0] == V and phi[N] == 0.0
    assert np.allclose(E[1:N], (phi[:N - 1] - phi[2:]) / (2 * dx), rtol=1e-12, atol=1e-9)


def test_nodal_e_exact_for_linear_potential_on_quadtree():
    d = I.quadtree_static_desc(precision=64)
    o = oracle.Oracle(d)
    keys, lv = o.leaves()
    cx, cy = I.leaf_corners(keys, lv)
    a, b, c = 3.5, -1.25, 0.7
    o.field_set(oracle.CORNER_PHI_2D, a * cx + b * cy + c)
    E = o.field_table()
    assert np.allclose(E[:, :, 0], -a, rtol=1e-12, atol=0)
    assert np.allclose(E[:, :, 1], -b, rtol=1e-12, atol=0)


def test_quadtree_field_first_order_vs_analytic():
    d = I.quadtree_static_desc(precision=64)
    o = oracle.Oracle(d)
    keys, lv = o.leaves()
    cx, cy = I.leaf_corners(keys, lv)
    o.field_set(oracle.CORNER_PHI_2D, I.quadtree_phi(cx, cy))
    E = o.field_table()
    ex, ey = -2 * cx, -0.6 * np.pi * np.cos(2 * np.pi * cy)
    h = np.ldexp(1.0, -lv.astype(int))[:, None]
    # first-order bound from the Taylor remainder of a one-cell difference
    assert np.all(np.abs(E[:, :, 0] - ex) <= 2.0 * h * 1.0001)
    assert np.all(np.abs(E[:, :, 1] - ey) <= 0.3 * (2 * np.pi) ** 2 * h * 1.0001)


def _streamer_small(levels=(3, 5)):
    d = I.streamer_desc(min_level=levels[0], max_level=levels[1], precision=64)
    d["base_level"] = levels[0]
    d["refine_disk"] = 1
    d["disk_cx"], d["disk_cy"], d["disk_r"], d["disk_level"] = 0.4, 0.55, 0.2, levels[1]
    return d


def test_fv_operator_symmetric_and_cg_matches_spsolve():
    d = _streamer_small()
    o = oracle.Oracle(d)
    rng = np.random.Generator(np.random.PCG64(9))
    n = 3000
    o.load(0, rng.random((n, 2)), np.zeros((n, 3)), ids=np.arange(n, dtype=np.uint32))
    o.load(1, rng.normal(0.5, 0.1, (n, 2)).clip(0, 0.999), np.zeros((n, 3)),
           ids=np.arange(n, 2 * n, dtype=np.uint32))
    o.deposit()
    rows, cols, vals, rhs = o.assemble_2d()
    A = scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(o.nq(), o.nq()))
    assert abs(A - A.T).max() < 1e-15
    # constant potential: only Dirichlet faces remain
    ones = A @ np.ones(o.nq())
    assert np.all(ones >= -1e-12)
    ref = scipy.sparse.linalg.spsolve(A.tocsc(), rhs)
    phi, it, rr, rc = o.field_solve_2d(rtol=1e-13)
    assert rc == 0 and rr <= 1e-13
    assert np.allclose(phi, ref, rtol=1e-8, atol=1e-8 * np.max(np.abs(ref)))


def test_fv_uniform_mesh_exact_for_linear_potential():
    d = I.streamer_desc(min_level=4, max_level=4, precision=64)
    d["base_level"] = 4
    o = oracle.Oracle(d)
    phi, it, rr, rc = o.field_solve_2d(rtol=1e-14)
    keys, lv = o.leaves()
    cx, cy = I.leaf_corners(keys, lv)
    yc = (cy[:, 0] + cy[:, 2]) / 2
    exact = d["wall_phi"][3] * yc
    assert np.allclose(phi, exact, rtol=1e-11, atol=1e-9)
    E = o.field_table()
    assert np.allclose(E[:, :, 1], -d["wall_phi"][3] / d["length"], rtol=1e-9)
    assert np.allclose(E[:, :, 0], 0.0, atol=1e-6)


def test_fv_manufactured_solution_converges():
    """phi = sin(pi x) sin(pi y) with zero Dirichlet walls: the FV error
    falls as the uniform mesh is refined (second order on a uniform mesh)."""
    errs = []
    for L in (3, 4, 5):
        d = I.streamer_desc(min_level=L, max_level=L, precision=64)
        d["base_level"] = L
        d["field_bc"] = [1, 1, 1, 1]
        d["wall_phi"] = [0.0] * 4
        d["length"] = 1.0
        d["depth_z"] = 1.0
        o = oracle.Oracle(d)
        keys, lv = o.leaves()
        cx, cy = I.leaf_corners(keys, lv)
        xc, yc = (cx[:, 0] + cx[:, 1]) / 2, (cy[:, 0] + cy[:, 2]) / 2
        # charge per leaf: rho h^2 / eps0 = 2 pi^2 phi h^2 -> weight units of one ion species
        h = 2.0 ** -L
        target = 2 * np.pi ** 2 * np.sin(np.pi * xc) * np.sin(np.pi * yc) * h * h
        kap = I.E_CHARGE * 1.0 * 2.0 ** -16 / 1.0 / 8.8541878128e-12
        wu = np.round(target / kap / 1e6).astype(np.uint32)      # 1e6 particles worth per unit
        d["species"][1]["w0"] = 1e6
        o = oracle.Oracle(d)
        o.load(1, np.stack([xc, yc], 1), np.zeros((len(xc), 3)), w=wu, ids=np.arange(len(xc), dtype=np.uint32))
        o.deposit()
        phi, *_ = o.field_solve_2d(rtol=1e-13)
        errs.append(np.max(np.abs(phi - np.sin(np.pi * xc) * np.sin(np.pi * yc))))
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3


def test_poisson1d_exact_against_rational_elimination():
    """The 1D solve against Gaussian elimination in exact rational arithmetic
    (fractions) of the same tridiagonal system: the oracle's result is the
    exact solution rounded, within a few units in the last place."""
    from fractions import Fraction as Fr
    N, L, V = 13, 0.05, 77.25
    d = I.ccp_desc(ncells=N, ppc=4, length=L)
    o = oracle.Oracle(d)
    rng = np.random.Generator(np.random.PCG64(21))
    for sp in range(2):
        n = 300
        o.load(sp, rng.random((n, 1)), np.zeros((n, 3)), w=rng.integers(1, 1 << 17, n).astype(np.uint32),
               ids=np.arange(sp * n, (sp + 1) * n, dtype=np.uint32))
    q = o.deposit()
    phi, _ = o.field_solve_1d(V)
    dx = L / N
    kap = [Fr(((sp["charge"] * sp["w0"]) * 2.0 ** -48) * dx / 8.8541878128e-12) for sp in d["species"]]
    # exact right-hand side and elimination on tridiag(-1, 2, -1), phi_0 = V, phi_N = 0
    c = [sum(kap[s] * int(q[s][i]) for s in range(2)) for i in range(N + 1)]
    m = N - 1
    diag = [Fr(2)] * m
    rhs = [c[i + 1] for i in range(m)]
    rhs[0] += Fr(V)
    for k in range(1, m):
        f = Fr(-1) / diag[k - 1]
        diag[k] -= f * Fr(-1)
        rhs[k] -= f * rhs[k - 1]
    x = [Fr(0)] * m
    x[m - 1] = rhs[m - 1] / diag[m - 1]
    for k in range(m - 2, -1, -1):
        x[k] = (rhs[k] + x[k + 1]) / diag[k]
    exact = np.array([float(v) for v in x])
    assert phi[0] == V and phi[N] == 0.0
    # a few roundings of terms of either sign: the bound scales with the
    # magnitude of the terms (the species' potentials nearly cancel)
    scale = np.array([abs(float(V * (N - i) / N)) + sum(
        abs(float(kap[s] * sum(min(i, j) * (N - max(i, j)) * int(q[s][j]) for j in range(1, N)) / N))
        for s in range(2)) for i in range(1, N)])
    err = np.abs(phi[1:N] - exact) / scale
    assert err.max() <= 8 * 2.0 ** -52, err.max()
