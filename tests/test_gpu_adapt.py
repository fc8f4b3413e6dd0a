"""GPU quadtree adaptation, split/merge and the 2D avalanche ("streamer")
steps vs the CPU oracle (paper Sec. 3.1 reassignment on refine/coarsen,
Sec. 4.3 splitting and merging, Sec. 3 MCC and Poisson).  Trees, particle
ids, weights, cells and event counts must match exactly; positions and
velocities to 1e-12 (FP64) / 1e-5 (FP32) relative."""
import numpy as np
import pytest

import oracle
from paper_1604_07713_amd import binding as B
from paper_1604_07713_amd import inputs as I
from tests.gpu_common import assert_same_particles, load_both

pytestmark = pytest.mark.gpu
TOL = {64: 1e-12, 32: 1e-5}


def compare_all(o, g, precision, what):
    ko, lo = o.leaves()
    kg, lg = g.leaves(0)
    assert np.array_equal(ko, kg) and np.array_equal(lo, lg), f"{what}: trees differ ({len(ko)} vs {len(kg)} leaves)"
    for sp in range(o.nspecies):
        assert_same_particles(o.read(sp), g.read(0, sp), TOL[precision], f"{what} species {sp}")
    assert o.next_id == g.next_id(0)
    assert np.array_equal(o.deposit(), g.deposit(0)), f"{what}: deposits differ"


def adapt_both(o, g, n_lo=16, n_hi=64):
    so = o.adapt(n_lo, n_hi)
    sg = g.adapt(0, n_lo, n_hi)
    for k in ("refined", "coarsened", "balance_refined", "split_parents", "merged_pairs", "nleaves"):
        assert so[k] == sg[k], (k, so[k], sg[k])
    assert abs(so["merge_energy_change"] - sg["merge_energy_change"]) <= 1e-9 * max(1.0, abs(so["merge_energy_change"]))
    return so


def cluster(n, seed, sigma=0.08, center=0.5):
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.normal(center, sigma, (n, 2)).clip(0.0, np.nextafter(1.0, 0.0))
    ve = rng.standard_normal((n, 3)) * 4e5
    vi = rng.standard_normal((n, 3)) * 3e2
    return pos, ve, vi


@pytest.mark.parametrize("precision", [64, 32])
def test_adapt_cluster_matches(precision):
    d = I.streamer_desc(min_level=2, max_level=7, precision=precision)
    d["base_level"] = 2
    pos, ve, vi = cluster(20000, 7)
    parts = [(pos, ve, None, np.arange(20000, dtype=np.uint32)),
             (pos[:10000], vi[:10000], None, np.arange(20000, 30000, dtype=np.uint32))]
    o, g = load_both(d, parts)
    st = adapt_both(o, g)
    assert st["refined"] > 0 and st["split_parents"] > 0
    compare_all(o, g, precision, "after adapt")
    # a second adapt on the same particles is a fixed point for the tree
    adapt_both(o, g)
    compare_all(o, g, precision, "after second adapt")


def test_adapt_split_and_merge_match():
    # few particles per leaf at the finest allowed level -> split; many -> merge
    d = I.streamer_desc(min_level=3, max_level=3, precision=64)
    d["base_level"] = 3
    rng = np.random.Generator(np.random.PCG64(2))
    pos = np.concatenate([rng.random((30, 2)), rng.random((600, 2)) * 0.125])
    v = rng.standard_normal((630, 3)) * 1e5
    o, g = load_both(d, [(pos, v, None, np.arange(630, dtype=np.uint32)),
                         (pos[:0], v[:0], None, np.zeros(0, dtype=np.uint32))])
    st = adapt_both(o, g)
    assert st["merged_pairs"] > 0 and st["split_parents"] > 0
    compare_all(o, g, 64, "split/merge")


def test_adapt_coarsens_after_removal():
    """The tree of a dense cluster, given explicitly, with most particles
    removed: both sides coarsen it the same way."""
    d = I.streamer_desc(min_level=2, max_level=6, precision=64)
    d["base_level"] = 2
    pos, ve, vi = cluster(20000, 11, sigma=0.05)
    o, g = load_both(d, [(pos, ve, None, np.arange(20000, dtype=np.uint32)),
                         (pos[:0], vi[:0], None, np.zeros(0, dtype=np.uint32))])
    adapt_both(o, g)
    compare_all(o, g, 64, "first")
    # the adapted tree, with a sparse subset of the particles (same on both sides)
    keys, lv = o.leaves()
    d2 = dict(d, leaf_keys=keys, leaf_levels=lv)
    r = o.read(0)
    keep = np.arange(0, len(r["id"]), 40)
    o2, g2 = load_both(d2, [(r["s"][keep], r["v"][keep], r["w"][keep], r["id"][keep]),
                            (r["s"][:0], r["v"][:0], None, np.zeros(0, dtype=np.uint32))])
    assert np.array_equal(g2.leaves(0)[0], keys)
    st = adapt_both(o2, g2)
    assert st["coarsened"] > 0
    compare_all(o2, g2, 64, "after removal")


@pytest.mark.parametrize("precision,ranking,max_level", [(64, 0, 11), (32, 0, 11), (32, 2, 11), (32, 0, 12)])
def test_streamer_steps_with_births_match(precision, ranking, max_level):
    """2D electron avalanche: 1 atm N2-like gas, 30 kV/cm, Gaussian seed of
    electron-ion pairs, levels 5-11, adapt every 10 steps, MCC with
    ionization births; both sides step with the same field table.  ranking 2:
    the GPU ranks the births through id bins instead of pairwise.  Levels up
    to 12 take the point location that ends in a binary search (the lookup
    table stops at level 11)."""
    d = I.streamer_desc(precision=precision, max_level=max_level)
    parts = I.streamer_particles(d, npairs=3000)
    o, g = load_both(d, parts)
    g.set_births_ranking(0, ranking)
    adapt_both(o, g)
    compare_all(o, g, precision, "initial adapt")
    births = 0
    for n in range(30):
        if n % 10 == 0:
            if n:
                adapt_both(o, g)
            o.deposit()
            phi, it, rr, rc = o.field_solve_2d(rtol=1e-10)
            E = o.field_table()
            o.field_set(oracle.CORNER_E_2D, E)
            g.field_set(0, B.CORNER_E_2D, E)
            if n == 0:
                o.leapfrog_start()
                g.leapfrog_start(0)
        so = o.step(n, 1)
        sg = g.step(n, 1)
        for k in ("alive_start", "absorbed", "elastic", "ionization", "births", "numax_violations"):
            assert so[k] == sg[k], (n, k, so[k], sg[k])
        births += so["births"]
    assert births > 0
    compare_all(o, g, precision, "after 30 steps")


def test_cg_solve_matches_oracle_and_direct():
    import scipy.sparse
    import scipy.sparse.linalg
    d = I.streamer_desc(precision=64, min_level=3, max_level=7)
    d["base_level"] = 3
    pos, ve, vi = cluster(20000, 5, sigma=0.1)
    o, g = load_both(d, [(pos, ve, None, np.arange(20000, dtype=np.uint32)),
                         (pos[:15000], vi[:15000], None, np.arange(20000, 35000, dtype=np.uint32))])
    adapt_both(o, g)
    o.deposit()
    g.deposit(0)
    po, ito, rro, rco = o.field_solve_2d(rtol=1e-12)
    pg, itg, rrg, rcg = g.field_solve_2d(0, rtol=1e-12)
    assert rco == 0 and rcg == 0 and rrg <= 1e-12
    rows, cols, vals, rhs = o.assemble_2d()
    A = scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(o.nq(), o.nq()))
    ref = scipy.sparse.linalg.spsolve(A.tocsc(), rhs)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(pg - ref)) <= 1e-8 * scale
    assert np.max(np.abs(pg - po)) <= 1e-8 * scale
    Eo = o.field_table()
    Eg = g.field_table(0)
    assert np.max(np.abs(Eg - Eo)) <= 1e-6 * np.max(np.abs(Eo))


def test_cg_large_grid_deterministic():
    """A 512 x 512 uniform tree (262,144 unknowns, a CG launch with the most
    workgroups it takes and several rows per thread): two solves from the
    same start give the same bits and iteration count (the block partials each launch sums are not overwritten
    by workgroups that finish early), and the true residual of the result
    meets the tolerance."""
    import scipy.sparse
    d = I.streamer_desc(precision=64, min_level=9, max_level=9)
    pos, ve, vi = cluster(200000, 7, sigma=0.1)
    parts = [(pos, ve, None, np.arange(200000, dtype=np.uint32)),
             (pos[:150000], vi[:150000], None, np.arange(200000, 350000, dtype=np.uint32))]
    o, g = load_both(d, parts)
    assert g.nq(0) == 512 * 512
    o.deposit()
    g.deposit(0)
    zero = np.zeros(g.nq(0))
    p1, it1, rr1, rc1 = g.field_solve_2d(0, phi_init=zero, rtol=1e-10)
    p2, it2, rr2, rc2 = g.field_solve_2d(0, phi_init=zero, rtol=1e-10)
    assert rc1 == 0 and rc2 == 0 and it1 > 100
    assert it1 == it2 and np.array_equal(p1, p2)
    rows, cols, vals, rhs = o.assemble_2d()
    A = scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(o.nq(), o.nq()))
    assert np.linalg.norm(rhs - A @ p1) <= 1e-8 * np.linalg.norm(rhs)
