"""Batched 2D launch (one persistent launch over many quadtree slots): each
slot's result equals the same slot stepped alone with per-slot launches, bit
for bit, through avalanches with collisions, births (pairwise and binned
ranking), adaptation with split / merge, field solves, sorts, room stops and
HIP graph replay; one slot is also checked against the oracle."""
import numpy as np
import pytest

import oracle
from paper_1604_07713_amd import binding as B
from paper_1604_07713_amd import inputs as I
from tests.gpu_common import assert_same_particles

pytestmark = pytest.mark.gpu


def avalanche_descs(precision, n=5):
    """Uneven avalanche instances: domains 0.25-1 cm, levels up to 10 or 12
    (the deeper trees locate through the binary search), own Philox keys."""
    out = []
    for k in range(n):
        side = [0.01, 0.005, 0.0025, 0.0075, 0.004][k % 5]
        d = I.streamer_desc(side=side, precision=precision, seed=20 + k, instance_key=k,
                            max_level=12 if k % 2 else 10)
        out.append(d)
    return out


def load(ctx, descs, npairs):
    for j, d in enumerate(descs):
        for sp, (s, v, w, ids) in enumerate(I.streamer_particles(d, npairs=npairs[j])):
            ctx.load(j, sp, s, v, w, ids)


def same_state(a, b, nslots, what):
    for j in range(nslots):
        ka, la = a.leaves(j)
        kb, lb = b.leaves(j)
        assert np.array_equal(ka, kb) and np.array_equal(la, lb), f"{what}: slot {j} trees differ"
        for sp in range(2):
            assert_same_particles(a.read(j, sp), b.read(j, sp), 0, f"{what}: slot {j} species {sp}")
        assert a.next_id(j) == b.next_id(j), f"{what}: slot {j} next ids differ"
        assert np.array_equal(a.deposit_read(j), b.deposit_read(j)), f"{what}: slot {j} deposits differ"


def run_avalanche(ctx, nslots, nsteps, every, step_kw):
    stats = []
    for j in range(nslots):
        ctx.adapt(j)
        ctx.field_solve_2d(j, rtol=1e-10, maxit=4000)
        ctx.leapfrog_start(j)
    for k in range(0, nsteps, every):
        stats.append(ctx.step(-1, every, **step_kw))
        for j in range(nslots):
            ctx.adapt(j)
            ctx.field_solve_2d(j, rtol=1e-10, maxit=4000)
    return stats


@pytest.mark.parametrize("precision", [32, 64])
def test_batched_avalanche_equals_plain(precision):
    descs = avalanche_descs(precision)
    npairs = [3000, 1000, 500, 2000, 800]
    a = B.Context(descs)
    b = B.Context(descs)
    load(a, descs, npairs)
    load(b, descs, npairs)
    for j in (1, 3):   # these rank births through id bins, the others pairwise
        a.set_births_ranking(j, 2)
        b.set_births_ranking(j, 2)
    sa = run_avalanche(a, len(descs), 60, 10, dict(batched=1024, grid=96, sort_every=5))
    sb = run_avalanche(b, len(descs), 60, 10, dict(sort_every=5))
    for x, y in zip(sa, sb):
        for k in ("alive_start", "absorbed", "elastic", "ionization", "births", "numax_violations"):
            assert x[k] == y[k], (k, x[k], y[k])
    assert sum(x["births"] for x in sa) > 100
    same_state(a, b, len(descs), "after 60 steps")


def test_batched_static_quadtrees_with_graph_replay():
    """Collisionless slots on static trees (reflecting walls), different disk
    refinements and particle counts: graph replay of the batched launch
    against per-slot launches."""
    descs, parts = [], []
    for k, (r, n) in enumerate([(0.15, 200000), (0.3, 50000), (0.05, 120000)]):
        d = I.quadtree_static_desc(precision=32, seed=2 + k)
        d["disk_r"] = r
        descs.append(d)
        parts.append(I.quadtree_particles(n, seed=2 + k))
    a = B.Context(descs)
    b = B.Context(descs)
    for g in (a, b):
        for j, (s, v, w, ids) in enumerate(parts):
            g.load(j, 0, s, v, w, ids)
            keys, lv = g.leaves(j)
            cx, cy = I.leaf_corners(keys, lv)
            g.field_set(j, B.CORNER_PHI_2D, I.quadtree_phi(cx, cy))
            g.leapfrog_start(j)
    sa = a.step(0, 60, batched=4096, grid=256, sort_every=20, graph_steps=10)
    sb = b.step(0, 60, sort_every=20)
    for k in ("alive_start", "absorbed", "lost_reflect"):
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    for j in range(len(descs)):
        assert_same_particles(a.read(j, 0), b.read(j, 0), 0, f"slot {j}")
        assert np.array_equal(a.deposit_read(j), b.deposit_read(j))


def test_batched_room_stops_equal_unconstrained_plain():
    """Capacities just above one step's worst case of births (strongly
    ionizing gas): batched steps stop slots for room, grow them and continue;
    the result equals per-slot steps with room to spare."""
    npairs = [5000, 2000, 3500]
    descs = []
    for k, n in enumerate(npairs):
        d = I.streamer_desc(precision=32, max_level=8, instance_key=k, seed=30 + k)
        d["species"][0]["sigma_iz"] = 1e-19
        d["species"][0]["eps_iz"] = 5.0
        descs.append(d)
    tight = [dict(d, capacity=((2 * n + 1024 + 255) // 256 * 256 + 512,) * 2) for d, n in zip(descs, npairs)]
    big = [dict(d, capacity=(2_000_000, 2_000_000)) for d in descs]
    a = B.Context(tight)
    b = B.Context(big)
    for g in (a, b):
        load(g, descs, npairs)
        for j in range(3):
            g.field_solve_2d(j, rtol=1e-10)
            g.leapfrog_start(j)
    sa = a.step(0, 96, batched=1024, grid=128)
    sb = b.step(0, 96)
    print("births", sa["births"], "room stops", sa["room_stops"], flush=True)
    assert sa["room_stops"] > 0 and sb["room_stops"] == 0
    assert sa["births"] == sb["births"] > 0
    same_state(a, b, 3, "after 96 steps")


def test_batched_slot_matches_oracle():
    d = I.streamer_desc(precision=64, max_level=10, instance_key=3)
    other = I.streamer_desc(side=0.005, precision=64, max_level=12, instance_key=4)
    parts = I.streamer_particles(d, npairs=2000)
    g = B.Context([d, other])
    o = oracle.Oracle(d)
    for sp, (s, v, w, ids) in enumerate(parts):
        g.load(0, sp, s, v, w, ids)
        o.load(sp, s, v, w, ids)
    for sp, (s, v, w, ids) in enumerate(I.streamer_particles(other, npairs=700)):
        g.load(1, sp, s, v, w, ids)
    o.adapt(16, 64)
    g.adapt(0)
    g.adapt(1)
    o.deposit()
    o.field_solve_2d(rtol=1e-10)
    E = o.field_table()
    o.field_set(oracle.CORNER_E_2D, E)
    g.field_set(0, B.CORNER_E_2D, E)
    g.field_solve_2d(1, rtol=1e-10)
    o.leapfrog_start()
    g.leapfrog_start(0)
    g.leapfrog_start(1)
    so = o.step(0, 40)
    for k in range(0, 40, 10):
        g.step(-1, 10, batched=512, grid=32)
    ro, rg = o.read(0), g.read(0, 0)
    assert so["births"] > 0
    assert_same_particles(ro, rg, 1e-12, "electrons")
    assert_same_particles(o.read(1), g.read(0, 1), 1e-12, "ions")
    assert o.next_id == g.next_id(0)
