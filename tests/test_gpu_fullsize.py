"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times.  The oracle cannot step every particle of
these runs, so it steps a sample it can compute one by one: particles of the
collisionless quadtree (each depends only on its own state and the fixed
field) and whole instances of the batched ensemble (each is independent of
the others).  The rest is checked through properties that hold at any size:
the deposit the step loop accumulated equals the integer charge of the
particles it left, every particle sits in the leaf that holds its position,
ids are unique, and charge units are conserved."""
import numpy as np
import pytest

import oracle
from paper_1604_07713_amd import binding as B
from paper_1604_07713_amd import inputs as I
from tests.gpu_common import assert_same_particles

pytestmark = pytest.mark.gpu


def pick(r, ids):
    """Rows of a read() dict (sorted by id) for the given sorted ids."""
    idx = np.searchsorted(r["id"], ids)
    assert np.array_equal(r["id"][idx], ids), "sampled ids missing on the GPU side"
    return {k: r[k][idx] for k in ("id", "w", "cell", "s", "v")}


def spread16(v):
    v = v.astype(np.uint64) & 0xFFFF
    v = (v | (v << 8)) & 0x00FF00FF
    v = (v | (v << 4)) & 0x0F0F0F0F
    v = (v | (v << 2)) & 0x33333333
    v = (v | (v << 1)) & 0x55555555
    return v


def host_locate(keys, s):
    """Leaf of each point of a Morton-ordered quadtree: the last leaf whose
    corner code is <= the point's 16-bit Morton code."""
    X = np.floor(s[:, 0] * 65536.0).astype(np.uint64)
    Y = np.floor(s[:, 1] * 65536.0).astype(np.uint64)
    m = spread16(X) | (spread16(Y) << 1)
    return (np.searchsorted(keys.astype(np.uint64), m, side="right") - 1).astype(np.int64)


@pytest.mark.parametrize("n", [4194304, 16777216])
def test_quadtree_full_size_sampled(n):
    """4,194,304 electrons on the static quadtree (the benchmark's particles),
    and the 16,777,216 of its variant beyond the Infinity Cache, default
    launch grid, 60 steps with the order kept by a sort every 50 steps:
    20,000 particles sampled by id equal the oracle's, and the step loop's
    deposit equals the particles' NGP charge."""
    d = I.quadtree_static_desc()
    s, v, w, ids = I.quadtree_particles(n)
    g = B.Context(d)
    g.load(0, 0, s, v, w, ids)
    o = oracle.Oracle(d)
    okeys, olv = o.leaves()
    gkeys, glv = g.leaves(0)
    assert np.array_equal(okeys, gkeys) and np.array_equal(olv, glv)
    cx, cy = I.leaf_corners(okeys, olv)
    phi = I.quadtree_phi(cx, cy)
    g.field_set(0, B.CORNER_PHI_2D, phi)
    g.sort(0)
    g.leapfrog_start(0)
    nsteps = 60
    sg = g.step(0, nsteps, sort_every=50)
    sample = np.sort(np.random.Generator(np.random.PCG64(11)).choice(n, 20000, replace=False)).astype(np.uint32)
    o.load(0, s[sample], v[sample], w[sample], ids[sample])
    o.field_set(oracle.CORNER_PHI_2D, phi)
    o.leapfrog_start()
    o.step(0, nsteps)
    gr = g.read(0, 0)
    assert len(gr["id"]) == n - sg["absorbed"][0]
    assert_same_particles(o.read(0), pick(gr, sample), 1e-5, "sampled quadtree particles")
    q = g.deposit_read(0)
    ngp = np.bincount(gr["cell"].astype(np.int64), weights=gr["w"].astype(np.float64), minlength=len(gkeys))
    assert np.array_equal(q[0].astype(np.float64), ngp)
    assert np.array_equal(host_locate(gkeys, gr["s"]), gr["cell"].astype(np.int64))


@pytest.mark.parametrize("scheme", [I.FIELD_CIC_EM, I.FIELD_CIC_EC])
def test_ensemble_full_size_sampled(scheme):
    """The 96-instance ensemble at full size, batched FP32 with graph replay
    (work items of 4096 particles, 2048 workgroups), with either 1D coupling:
    three whole instances (smallest, median and largest) equal the oracle's
    run, and every instance keeps its charge units."""
    descs = I.ensemble_descs(count=96, precision=32)
    for d in descs:
        d["field_scheme"] = scheme
    nsteps = 20
    vn = np.stack([I.drive_voltage(d, np.arange(1, nsteps + 1)) for d in descs], axis=1)
    g = B.Context(descs)
    parts = []
    for j, d in enumerate(descs):
        p = I.ensemble_particles(d)
        parts.append(p)
        for sp, (s, v, w, ids) in enumerate(p):
            g.load(j, sp, s, v, w, ids)
        g.deposit(j)
        g.field_solve_1d(j, float(I.drive_voltage(d, 0)))
        g.leapfrog_start(j)
    g.step(0, nsteps, vn, solve_field=True, sort_every=20, batched=4096, grid=2048, graph_steps=10)
    sizes = np.array([len(p[0][0]) + len(p[1][0]) for p in parts])
    order = np.argsort(sizes, kind="stable")
    for j in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        d = descs[j]
        o = oracle.Oracle(d)
        for sp, (s, v, w, ids) in enumerate(parts[j]):
            o.load(sp, s, v, w, ids)
        o.deposit()
        o.field_solve_1d(float(I.drive_voltage(d, 0)))
        o.leapfrog_start()
        o.step(0, nsteps, vn[:, j], True)
        for sp in range(2):
            assert_same_particles(o.read(sp), g.read(j, sp), 1e-5, f"instance {j} species {sp}")
        assert o.next_id == g.next_id(j)
        assert np.array_equal(o.field_table(), g.field_table(j))
    one = 1 << 24   # CIC charge units per weight unit (FP32)
    for j in range(len(descs)):
        q = g.deposit_read(j)
        for sp in range(2):
            r = g.read(j, sp)
            assert int(q[sp].sum()) == int(r["w"].astype(np.uint64).sum()) * one, (j, sp)


def test_streamer_full_config_properties():
    """The avalanche workload (1e4 seed pairs, levels 5-11) for 300 steps with
    adaptation and the CG field solve every 10 steps: after the last step the
    step loop's deposit equals the particles' NGP charge per species, every
    particle sits in the leaf holding its position, ids are unique and below
    the next id, and the leaves stay within the level bounds."""
    d = I.streamer_desc(side=0.01, precision=32)
    g = B.Context(d)
    for sp, (s, v, w, ids) in enumerate(I.streamer_particles(d, npairs=10000)):
        g.load(0, sp, s, v, w, ids)
    g.adapt(0)
    g.field_solve_2d(0, rtol=1e-8, maxit=4000)
    g.leapfrog_start(0)
    births = 0
    for k in range(30):
        st = g.step(-1, 10, sort_every=0)
        births += st["births"]
        if k < 29:
            g.adapt(0)
            g.field_solve_2d(0, rtol=1e-8, maxit=4000)
    assert births > 0
    keys, lv = g.leaves(0)
    assert lv.min() >= d["min_level"] and lv.max() <= d["max_level"]
    q = g.deposit_read(0)
    allids = []
    for sp in range(2):
        r = g.read(0, sp)
        assert np.array_equal(host_locate(keys, r["s"]), r["cell"].astype(np.int64)), f"species {sp}"
        ngp = np.bincount(r["cell"].astype(np.int64), weights=r["w"].astype(np.float64), minlength=len(keys))
        assert np.array_equal(q[sp].astype(np.float64), ngp), f"species {sp}"
        allids.append(r["id"])
    allids = np.concatenate(allids)
    assert len(np.unique(allids)) == len(allids)
    assert allids.max() < g.next_id(0)


def test_streamer_resynced_at_full_size():
    """The avalanche workload (1e4 seed pairs, 1 cm, levels 5-11, adapt and
    CG every 10 steps) run on the GPU to steps 1000 and 1300, where it holds
    about a million particles and more; at each point the GPU's state (tree,
    particles, field table, next id) is loaded into the oracle and both sides
    take 3 more steps, the second time with the binned births ranking.  Ids,
    weights, cells, births, event counts and deposits must match exactly,
    positions and velocities to 1e-5 relative (in practice bitwise)."""
    d = I.streamer_desc(side=0.01, precision=32)
    g = B.Context(d)
    for sp, (s, v, w, ids) in enumerate(I.streamer_particles(d, npairs=10000)):
        g.load(0, sp, s, v, w, ids)
    g.adapt(0)
    g.field_solve_2d(0, rtol=1e-8, maxit=4000)
    g.leapfrog_start(0)
    step = 0
    for stop, ranking in ((1000, 1), (1300, 2)):
        while step < stop:
            g.step(-1, 10, sort_every=0)
            step += 10
            g.adapt(0)
            g.field_solve_2d(0, rtol=1e-8, maxit=4000)
        g.set_births_ranking(0, ranking)
        keys, lv = g.leaves(0)
        E = g.field_table(0)
        parts = [g.read(0, sp) for sp in range(2)]
        n = sum(len(p["id"]) for p in parts)
        o = oracle.Oracle(dict(d, leaf_keys=keys, leaf_levels=lv))
        for sp, p in enumerate(parts):
            o.load(sp, p["s"], p["v"], p["w"], p["id"])
        o.set_next_id(g.next_id(0))
        o.field_set(oracle.CORNER_E_2D, E)
        for sp in range(2):
            assert np.array_equal(o.read(sp)["cell"], parts[sp]["cell"]), f"step {step}: cells on load"
        so = o.step(step, 3)
        sg = g.step(-1, 3, sort_every=0)
        step += 3
        print(f"resync at step {stop}: {n} particles, {so['births']} births in 3 steps", flush=True)
        assert n > 500_000
        for k in ("alive_start", "absorbed", "elastic", "ionization", "births", "numax_violations"):
            assert so[k] == sg[k], (stop, k, so[k], sg[k])
        assert so["births"] > 0
        for sp in range(2):
            assert_same_particles(o.read(sp), g.read(0, sp), 1e-5, f"step {step} species {sp}")
        assert o.next_id == g.next_id(0)
        assert np.array_equal(o.deposit(), g.deposit_read(0)), f"step {step}: deposits differ"
        if step < 1300:
            g.adapt(0)
            g.field_solve_2d(0, rtol=1e-8, maxit=4000)
        g.set_births_ranking(0, 0)
        del o
