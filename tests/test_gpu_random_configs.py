"""Randomised parity: small configurations drawn from fixed seeds, each
stepped on the GPU through the C ABI and by the oracle.  The draws cover
meshes from 2 cells up, particle counts from 1, both precisions, every 1D
coupling (momentum- and energy-conserving CIC, direct implicit), both wall
rules, sort periods, quadtrees and octrees of random depth and refinement
(including octrees deeper than the point-location table), the 2D
collision path with births and adaptation, and batched launches over
several 1D discharges or several avalanches (random work-item sizes, grids,
sort periods and graph replay).  Discrete results bit for bit;
positions and velocities to 1e-12 (FP64) / 1e-5 (FP32) relative."""
import numpy as np
import pytest

import oracle
from paper_1604_07713_amd import binding as B
from paper_1604_07713_amd import inputs as I
from tests.gpu_common import assert_same_particles, ccp_run_both, load_both

pytestmark = pytest.mark.gpu
TOL = {64: 1e-12, 32: 1e-5}
KEYS = ("alive_start", "absorbed", "elastic", "ionization", "cx", "births", "numax_violations", "lost_reflect")


def same_stats(so, sg, what):
    for k in KEYS:
        assert so[k] == sg[k], (what, k, so[k], sg[k])


def draw_1d(seed):
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    scheme = (I.FIELD_CIC_EM, I.FIELD_CIC_EC, I.FIELD_DIPIC)[seed % 3]
    kw = dict(ncells=int(rng.choice([2, 3, 5, 17, 64, 129, 300, 1000])), ppc=int(rng.integers(1, 33)),
              precision=int(rng.choice([32, 64])), voltage=float(rng.uniform(50.0, 600.0)),
              pressure_mtorr=float(rng.uniform(10.0, 100.0)), seed=int(rng.integers(1, 1000)),
              instance_key=int(rng.integers(0, 100)))
    if scheme == I.FIELD_DIPIC:
        d = I.dipic_ccp_desc(**kw)
    else:
        d = I.ccp_desc(**kw)
        d["field_scheme"] = scheme
    d["particle_bc"] = int(rng.choice([I.ABSORB, I.REFLECT]))
    return d, int(rng.choice([0, 7, 20]))


@pytest.mark.parametrize("seed", range(15))
def test_random_1d(seed):
    d, sort_every = draw_1d(seed)
    what = f"seed {seed}: {d['ncells']} cells, ppc {d['extra']['ppc']}, fp{d['precision']}, scheme {d['field_scheme']}"
    o, g, so, sg = ccp_run_both(d, 60, sort_every=sort_every)
    same_stats(so, sg, what)
    for sp in range(2):
        assert_same_particles(o.read(sp), g.read(0, sp), TOL[d["precision"]], f"{what} species {sp}")
    assert o.next_id == g.next_id(0)
    a, b = o.field_table(), g.field_table(0)
    assert np.allclose(a, b, rtol=TOL[d["precision"]], atol=TOL[d["precision"]] * np.abs(a).max()), what
    assert np.array_equal(o.deposit(), g.deposit_read(0)), what


def draw_tree(seed, dim):
    rng = np.random.Generator(np.random.PCG64(2000 + 10 * dim + seed))
    base = int(rng.integers(2, 5 if dim == 3 else 6))
    top = min(base + int(rng.integers(0, 4)), 8 if dim == 3 else 10)
    radius = float(rng.uniform(0.02, 0.4))
    if dim == 3 and seed % 3 == 2:   # deeper than the point-location table (level 7): a small ball at level 8
        top, radius = 8, float(rng.uniform(0.03, 0.08))
    e = I.species(-I.E_CHARGE, I.M_ELECTRON, 1.0, I.MCC_NONE)
    scheme = I.FIELD_CIC_EM if dim == 3 else (I.FIELD_CIC_EM, I.FIELD_CIC_AMR)[seed % 2]
    d = I.base_desc(dim=dim, precision=int(rng.choice([32, 64])), length=1.0, dt=1e-9, min_level=base,
                    max_level=top, base_level=base, refine_disk=1, disk_cx=float(rng.uniform(0.1, 0.9)),
                    disk_cy=float(rng.uniform(0.1, 0.9)), disk_cz=float(rng.uniform(0.1, 0.9)),
                    disk_r=radius, disk_level=top,
                    particle_bc=int(rng.choice([I.ABSORB, I.REFLECT])), seed=int(rng.integers(1, 1000)),
                    species=[e], gas_mass=40.0 * I.AMU, field_scheme=scheme)
    n = int(rng.choice([1, 63, 777, 4000]))
    return d, n, float(rng.uniform(0.2, 5.0)), int(rng.choice([0, 5, 16]))


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("seed", range(9))
def test_random_static_tree(dim, seed):
    d, n, scale, sort_every = draw_tree(seed, dim)
    what = (f"seed {seed}: dim {dim}, levels {d['min_level']}-{d['max_level']}, {n} particles, "
            f"fp{d['precision']}, scheme {d['field_scheme']}")
    if dim == 2:
        s, v, w, ids = I.quadtree_particles(n, seed=seed + 40)
    else:
        s, v, w, ids = I.octree_particles(n, seed=seed + 40)
    o, g = load_both(d, [(s, v, w, ids)])
    keys, lv = o.leaves()
    gk, gl = g.leaves(0)
    assert np.array_equal(keys, gk) and np.array_equal(lv, gl), what
    if dim == 2:
        cx, cy = I.leaf_corners(keys, lv)
        phi, kind_o, kind_g = scale * I.quadtree_phi(cx, cy), oracle.CORNER_PHI_2D, B.CORNER_PHI_2D
    else:
        x, y, z = I.leaf_corners3(keys, lv)
        phi, kind_o, kind_g = scale * I.octree_phi(x, y, z), oracle.CORNER_PHI_3D, B.CORNER_PHI_3D
    o.field_set(kind_o, phi)
    g.field_set(0, kind_g, phi)
    o.leapfrog_start()
    g.leapfrog_start(0)
    so = o.step(0, 40)
    sg = g.step(0, 40, sort_every=sort_every)
    same_stats(so, sg, what)
    assert_same_particles(o.read(0), g.read(0, 0), TOL[d["precision"]], what)
    assert np.array_equal(o.deposit(), g.deposit(0)), what


def adapt_both(o, g):
    so = o.adapt()
    sg = g.adapt(0)
    for k in ("refined", "coarsened", "balance_refined", "split_parents", "merged_pairs", "nleaves"):
        assert so[k] == sg[k], (k, so[k], sg[k])


@pytest.mark.parametrize("seed", range(6))
def test_random_avalanche_with_adaptation(seed):
    """The 2D collision path with births on a dynamic tree: random domain,
    field, levels, seed size and precision, with either coupling (NGP with
    nodal E, or the cloud-in-cell on the tree, Sec. 3.1); 40 steps with an
    adaptation every 10 (refine, coarsen, balance, split, merge), both sides
    on the same field table (the analytic uniform field set at the new
    leaves' corners)."""
    rng = np.random.Generator(np.random.PCG64(3000 + seed))
    lo = int(rng.integers(3, 6))
    side, e0 = float(rng.uniform(0.002, 0.01)), float(rng.uniform(2e6, 4e6))
    d = I.streamer_desc(side=side, precision=int(rng.choice([32, 64])), seed=int(rng.integers(1, 1000)), e0=e0,
                        min_level=lo, max_level=min(lo + int(rng.integers(2, 5)), 10))
    d["field_scheme"] = (I.FIELD_CIC_EM, I.FIELD_CIC_AMR)[seed % 2]   # NGP with nodal E, or the tree cloud-in-cell
    parts = I.streamer_particles(d, npairs=int(rng.integers(200, 3000)), sigma=float(rng.uniform(2e-4, 1e-3)) * side / 0.01,
                                 rng_seed=[3000 + seed])
    what = (f"seed {seed}: levels {d['min_level']}-{d['max_level']}, side {side:.4f}, fp{d['precision']}, "
            f"scheme {d['field_scheme']}")
    o, g = load_both(d, parts)
    births = 0
    for n in range(0, 40, 10):
        adapt_both(o, g)
        keys, lv = o.leaves()
        cx, cy = I.leaf_corners(keys, lv)
        phi = e0 * cy * side
        o.field_set(oracle.CORNER_PHI_2D, phi)
        g.field_set(0, B.CORNER_PHI_2D, phi)
        if n == 0:
            o.leapfrog_start()
            g.leapfrog_start(0)
        so = o.step(n, 10)
        sg = g.step(n, 10, sort_every=4)
        same_stats(so, sg, f"{what} steps {n}..{n + 9}")
        births += so["births"]
    ko, lo_ = o.leaves()
    kg, lg = g.leaves(0)
    assert np.array_equal(ko, kg) and np.array_equal(lo_, lg), what
    for sp in range(2):
        assert_same_particles(o.read(sp), g.read(0, sp), TOL[d["precision"]], f"{what} species {sp}")
    assert o.next_id == g.next_id(0)
    assert np.array_equal(o.deposit(), g.deposit(0)), what


@pytest.mark.parametrize("seed", range(5))
def test_random_batched_1d(seed):
    """Two to six uneven discharges of one precision stepped by one
    persistent launch per step: random meshes, particles per cell,
    couplings, wall rules, work-item size, grid, sort period and graph
    replay, against the oracle slot by slot."""
    rng = np.random.Generator(np.random.PCG64(4000 + seed))
    prec = int(rng.choice([32, 64]))
    descs = []
    for k in range(int(rng.integers(2, 7))):
        d = I.ccp_desc(ncells=int(rng.choice([2, 5, 17, 64, 300, 1000])), ppc=int(rng.integers(1, 25)), precision=prec,
                       voltage=float(rng.uniform(50.0, 600.0)), pressure_mtorr=float(rng.uniform(10.0, 100.0)),
                       seed=int(rng.integers(1, 1000)), instance_key=k)
        d["field_scheme"] = int(rng.choice([I.FIELD_CIC_EM, I.FIELD_CIC_EC]))
        d["particle_bc"] = int(rng.choice([I.ABSORB, I.REFLECT]))
        descs.append(d)
    tile, grid = int(rng.choice([256, 1024, 4096])), int(rng.choice([16, 256, 2048]))
    graph, sort_every = int(rng.choice([0, 0, 5])), int(rng.choice([0, 10, 20]))
    what = f"seed {seed}: {len(descs)} slots fp{prec}, tile {tile}, grid {grid}, graph {graph}, sort {sort_every}"
    nsteps = 40
    vn = np.stack([I.drive_voltage(d, np.arange(1, nsteps + 1)) for d in descs], axis=1)
    g = B.Context(descs)
    orc = [oracle.Oracle(d) for d in descs]
    for j, d in enumerate(descs):
        v0 = float(I.drive_voltage(d, 0))
        for sp, (s, v, w, ids) in enumerate(I.ccp_particles(d)):
            g.load(j, sp, s, v, w, ids)
            orc[j].load(sp, s, v, w, ids)
        g.deposit(j)
        orc[j].deposit()
        g.field_solve_1d(j, v0)
        orc[j].field_solve_1d(v0)
        g.leapfrog_start(j)
        orc[j].leapfrog_start()
    sg = g.step(0, nsteps, vn, solve_field=True, batched=tile, grid=grid, sort_every=sort_every, graph_steps=graph)
    so = [o.step(0, nsteps, vn[:, j], True) for j, o in enumerate(orc)]
    for k in ("elastic", "ionization", "cx", "births", "lost_reflect"):
        assert sg[k] == sum(s[k] for s in so), (what, k)
    for k in ("alive_start", "absorbed", "numax_violations"):
        assert list(sg[k]) == [sum(s[k][i] for s in so) for i in range(2)], (what, k)
    for j, o in enumerate(orc):
        for sp in range(2):
            assert_same_particles(o.read(sp), g.read(j, sp), TOL[prec], f"{what} slot {j} species {sp}")
        assert o.next_id == g.next_id(j), (what, j)
        a, b = o.field_table(), g.field_table(j)
        assert np.allclose(a, b, rtol=TOL[prec], atol=TOL[prec] * np.abs(a).max()), (what, j)
        assert np.array_equal(o.deposit(), g.deposit_read(j)), (what, j)


@pytest.mark.parametrize("seed", range(4))
def test_random_batched_avalanches(seed):
    """Two to four avalanches of one precision on dynamic trees stepped by
    one persistent launch per step (random domains, fields, levels, seed
    sizes, work-item size and grid), with an adaptation every 10 steps,
    against the oracle slot by slot."""
    rng = np.random.Generator(np.random.PCG64(5000 + seed))
    prec = int(rng.choice([32, 64]))
    descs, parts, fields = [], [], []
    for k in range(int(rng.integers(2, 5))):
        lo = int(rng.integers(3, 6))
        side, e0 = float(rng.uniform(0.002, 0.01)), float(rng.uniform(2e6, 4e6))
        d = I.streamer_desc(side=side, precision=prec, seed=int(rng.integers(1, 1000)), e0=e0, min_level=lo,
                            max_level=min(lo + int(rng.integers(2, 5)), 10))
        descs.append(d)
        parts.append(I.streamer_particles(d, npairs=int(rng.integers(200, 2000)),
                                          sigma=float(rng.uniform(2e-4, 1e-3)) * side / 0.01, rng_seed=[5000 + 10 * seed + k]))
        fields.append((e0, side))
    tile, grid = int(rng.choice([256, 1024, 2048])), int(rng.choice([64, 512, 2048]))
    what = f"seed {seed}: {len(descs)} slots fp{prec}, tile {tile}, grid {grid}"
    g = B.Context(descs)
    orc = [oracle.Oracle(d) for d in descs]
    for j in range(len(descs)):
        for sp, (s, v, w, ids) in enumerate(parts[j]):
            g.load(j, sp, s, v, w, ids)
            orc[j].load(sp, s, v, w, ids)
    slots = list(range(len(descs)))
    for n in range(0, 30, 10):
        for j, o in enumerate(orc):
            so, sg = o.adapt(), g.adapt(j)
            for k in ("refined", "coarsened", "balance_refined", "split_parents", "merged_pairs", "nleaves"):
                assert so[k] == sg[k], (what, j, k)
            keys, lv = o.leaves()
            cx, cy = I.leaf_corners(keys, lv)
            e0, side = fields[j]
            o.field_set(oracle.CORNER_PHI_2D, e0 * cy * side)
            g.field_set(j, B.CORNER_PHI_2D, e0 * cy * side)
            if n == 0:
                o.leapfrog_start()
                g.leapfrog_start(j)
        sg = g.step(n, 10, slots=slots, batched=tile, grid=grid, sort_every=4)
        so = [o.step(n, 10) for o in orc]
        for k in ("elastic", "ionization", "cx", "births", "lost_reflect"):
            assert sg[k] == sum(s[k] for s in so), (what, n, k)
        for k in ("alive_start", "absorbed", "numax_violations"):
            assert list(sg[k]) == [sum(s[k][i] for s in so) for i in range(2)], (what, n, k)
    for j, o in enumerate(orc):
        ko, lo_ = o.leaves()
        kg, lg = g.leaves(j)
        assert np.array_equal(ko, kg) and np.array_equal(lo_, lg), (what, j)
        for sp in range(2):
            assert_same_particles(o.read(sp), g.read(j, sp), TOL[prec], f"{what} slot {j} species {sp}")
        assert o.next_id == g.next_id(j), (what, j)
        assert np.array_equal(o.deposit(), g.deposit(j)), (what, j)


@pytest.mark.parametrize("seed", range(4))
def test_random_octree_avalanche(seed):
    """Electron avalanches on static octrees (paper Sec. 4.1 3D runs): random
    cube side, field, refinement depth (past the point-location table for
    some), seed size and spread, precision, births ranking and sort period;
    40 steps with collisions and births against the oracle."""
    rng = np.random.Generator(np.random.PCG64(6000 + seed))
    top = int(rng.integers(5, 9))
    d = I.octree_avalanche_desc(precision=int(rng.choice([32, 64])), seed=int(rng.integers(1, 1000)),
                                side=float(rng.uniform(0.002, 0.008)), e0=float(rng.uniform(2e6, 4e6)), top=top)
    d["disk_r"] = float(rng.uniform(0.05, 0.1)) if top == 8 else float(rng.uniform(0.1, 0.25))   # refined ball
    parts = I.octree_avalanche_particles(d, npairs=int(rng.integers(100, 3000)), sigma=float(rng.uniform(0.05, 0.2)))
    ranking, sort_every = int(rng.choice([0, 1, 2])), int(rng.choice([0, 7, 16]))
    what = f"seed {seed}: levels 4-{top}, fp{d['precision']}, ranking {ranking}, sort {sort_every}"
    o, g = load_both(d, parts)
    g.set_births_ranking(0, ranking)
    keys, lv = o.leaves()
    x, y, z = I.leaf_corners3(keys, lv)
    phi = I.octree_avalanche_phi(d, x * d["length"], y * d["length"], z * d["length"])
    o.field_set(oracle.CORNER_PHI_3D, phi)
    g.field_set(0, B.CORNER_PHI_3D, phi)
    o.leapfrog_start()
    g.leapfrog_start(0)
    births = 0
    for k in range(0, 40, 20):
        so = o.step(k, 20)
        sg = g.step(-1, 20, sort_every=sort_every)
        same_stats(so, sg, f"{what} steps {k}..{k + 19}")
        births += so["births"]
    assert births > 0, what
    for sp in range(2):
        assert_same_particles(o.read(sp), g.read(0, sp), TOL[d["precision"]], f"{what} species {sp}")
    assert o.next_id == g.next_id(0), what
    assert np.array_equal(o.deposit(), g.deposit_read(0)), what
