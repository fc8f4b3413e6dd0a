"""Oracle adaptation of the quadtree to the particle count (paper Sec. 3.1:
particles reassigned by position when cells refine or coarsen; Sec. 4.3:
splitting one particle into four in 2D, merging, AMR keeping particles per
cell steady) pinned to tree invariants and exact conservation identities."""
import numpy as np
import pytest

import oracle
from paper_1604_07713_amd import inputs as I
from tests.test_oracle_mesh_field import check_balanced, leaf_boxes, brute_locate


def cluster_desc(lmin=2, lmax=7, precision=64):
    d = I.streamer_desc(min_level=lmin, max_level=lmax, precision=precision)
    d["base_level"] = lmin
    return d


def load_cluster(o, n=20000, seed=7, sigma=0.08):
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.normal(0.5, sigma, (n, 2)).clip(0.0, np.nextafter(1.0, 0.0))
    ve = rng.standard_normal((n, 3)) * 4e5
    vi = rng.standard_normal((n, 3)) * 3e2
    o.load(0, pos, ve, ids=np.arange(n, dtype=np.uint32))
    o.load(1, pos[: n // 2], vi[: n // 2], ids=np.arange(n, n + n // 2, dtype=np.uint32))


def totals(o):
    out = []
    for sp in range(2):
        r = o.read(sp)
        out.append((int(r["w"].astype(np.int64).sum()),
                    (r["w"][:, None].astype(np.float64) * r["v"]).sum(axis=0)))
    return out


@pytest.mark.parametrize("precision", [64, 32])
def test_adapt_invariants(precision):
    d = cluster_desc(precision=precision)
    o = oracle.Oracle(d)
    load_cluster(o)
    before = totals(o)
    st = o.adapt(16, 64)
    keys, lv = o.leaves()
    check_balanced(keys, lv)
    x0, y0, x1, y1 = leaf_boxes(keys, lv)
    assert np.sum((x1 - x0) * (y1 - y0)) == 1.0
    assert lv.min() >= d["min_level"] and lv.max() <= d["max_level"]
    assert st["nleaves"] == len(keys)
    after = totals(o)
    for sp in range(2):
        assert before[sp][0] == after[sp][0]           # weight (charge) exactly conserved
        mom_tol = 1e-9 if precision == 64 else 1e-4
        assert np.allclose(before[sp][1], after[sp][1], rtol=mom_tol, atol=mom_tol * np.abs(before[sp][1]).max())
    # per-leaf counts: above the upper bound only at the finest level; below the lower
    # bound only where no particle can split any more
    for sp in range(2):
        r = o.read(sp)
        assert np.array_equal(r["cell"].astype(np.int64), brute_locate(keys, lv, r["s"]))
        c = np.bincount(r["cell"], minlength=len(keys))
        assert np.all((c <= 64) | (lv == d["max_level"]))
        low = (c > 0) & (c < 16)
        splittable = np.bincount(r["cell"], weights=(r["w"] % 4 == 0), minlength=len(keys)) > 0
        assert not np.any(low & splittable)
    assert st["merge_energy_change"] <= 1e-9 * abs(before[0][0]) * 1e12
    # the deposit after adapt matches the particles
    q = o.deposit()
    for sp in range(2):
        r = o.read(sp)
        assert np.array_equal(q[sp], np.bincount(r["cell"], weights=r["w"], minlength=len(keys)).astype(np.uint64))


def test_split_one_into_four():
    d = cluster_desc(lmin=3, lmax=3)
    o = oracle.Oracle(d)
    rng = np.random.Generator(np.random.PCG64(1))
    n = 20
    pos = rng.random((n, 2))
    v = rng.standard_normal((n, 3))
    o.load(0, pos, v, ids=np.arange(n, dtype=np.uint32))
    o.load(1, pos[:0], v[:0], ids=np.zeros(0, dtype=np.uint32))
    before = o.read(0)
    st = o.adapt(16, 64)
    r = o.read(0)
    # 64 leaves, at most a few particles each: each particle splits until its leaf holds >= 16
    c0 = np.bincount(before["cell"], minlength=64)
    c1 = np.bincount(r["cell"], minlength=64)
    for leaf in range(64):
        n0 = c0[leaf]
        if n0 == 0:
            assert c1[leaf] == 0
            continue
        k = 0
        while n0 * 4 ** k < 16:
            k += 1
        assert c1[leaf] == n0 * 4 ** k
    assert r["w"].astype(np.int64).sum() == n * 65536
    # copies keep position and velocity of their parent; parents keep their id
    for pid in before["id"]:
        j = np.nonzero(r["id"] == pid)[0][0]
        same = np.all(r["s"] == r["s"][j], axis=1) & np.all(r["v"] == r["v"][j], axis=1)
        assert r["w"][same].astype(np.int64).sum() == 65536
    assert o.next_id == n + 3 * st["split_parents"]
    assert len(np.unique(r["id"])) == len(r["id"])


def test_merge_pairs_at_finest_level():
    d = cluster_desc(lmin=2, lmax=2)
    o = oracle.Oracle(d)
    rng = np.random.Generator(np.random.PCG64(2))
    n = 300
    pos = rng.random((n, 2)) * 0.25                       # one level-2 leaf
    v = rng.standard_normal((n, 3)) * 1e5
    o.load(0, pos, v, ids=np.arange(n, dtype=np.uint32))
    o.load(1, pos[:0], v[:0], ids=np.zeros(0, dtype=np.uint32))
    st = o.adapt(16, 64)
    r = o.read(0)
    # 300 -> 150 -> 75 -> 38
    assert len(r["id"]) == 38 and st["merged_pairs"] == 150 + 75 + 37
    assert r["w"].astype(np.int64).sum() == n * 65536
    mom0 = (v * 65536.0).sum(axis=0)
    mom1 = (r["w"][:, None] * r["v"]).sum(axis=0)
    assert np.allclose(mom0, mom1, rtol=1e-12, atol=1e-6 * np.abs(mom0).max())
    assert st["merge_energy_change"] <= 0.0
    assert np.all((r["s"] >= 0) & (r["s"] < 0.25))


def test_adapt_idempotent_without_split_or_coarsen():
    d = cluster_desc()
    o = oracle.Oracle(d)
    load_cluster(o)
    o.adapt(0, 64)
    k1, l1 = o.leaves()
    r1 = o.read(0)
    st = o.adapt(0, 64)
    k2, l2 = o.leaves()
    assert np.array_equal(k1, k2) and np.array_equal(l1, l2)
    assert st["refined"] == 0 and st["coarsened"] == 0 and st["balance_refined"] == 0
    assert np.array_equal(o.read(0)["s"], r1["s"])


def test_coarsen_after_particles_leave():
    """The adapted tree of a dense cluster, given explicitly, with most of the
    particles removed: sibling groups coarsen and the tree stays balanced."""
    d = cluster_desc(lmin=2, lmax=6)
    o = oracle.Oracle(d)
    load_cluster(o, n=20000, sigma=0.05)
    o.adapt(16, 64)
    k1, l1 = o.leaves()
    r = o.read(0)
    keep = np.arange(0, len(r["id"]), 50)
    o2 = oracle.Oracle(dict(d, leaf_keys=k1, leaf_levels=l1))
    o2.load(0, r["s"][keep], r["v"][keep], w=r["w"][keep], ids=r["id"][keep])
    o2.load(1, r["s"][:0], r["v"][:0], ids=np.zeros(0, dtype=np.uint32))
    assert np.array_equal(o2.leaves()[0], k1)
    st = o2.adapt(16, 64)
    keys, lv = o2.leaves()
    check_balanced(keys, lv)
    assert st["coarsened"] > 0 and len(keys) < len(k1)
