"""GPU octree slots (3D, paper Sec. 3.1 quad/octree with cubic cells)
against the oracle, through the C ABI: the tree and point location, the
nodal E table, the trilinear gather, free-running steps with reflecting
walls and sorts, the avalanche with collisions and births (pairwise and
binned ranking), the charge density, the full-size workload sampled by id,
and the calls an octree slot refuses.  Discrete results bit for bit;
positions and velocities to 1e-12 (FP64) / 1e-5 (FP32) relative (bitwise in
practice)."""
import numpy as np
import pytest

import oracle
from paper_1604_07713_amd import binding as B
from paper_1604_07713_amd import inputs as I
from tests.gpu_common import assert_same_particles, load_both

pytestmark = pytest.mark.gpu
TOL = {64: 1e-12, 32: 1e-5}


def small_desc(precision, bc=I.REFLECT, top=5):
    e = I.species(-I.E_CHARGE, I.M_ELECTRON, 1.0, I.MCC_NONE)
    return I.base_desc(dim=3, precision=precision, length=1.0, dt=1e-9, min_level=2, max_level=top, base_level=2,
                       refine_disk=1, disk_cx=0.41, disk_cy=0.57, disk_cz=0.5, disk_r=0.3, disk_level=top,
                       particle_bc=bc, species=[e], gas_mass=1.0)


def set_phi(o, g, slot=0, scale=1.0, fn=I.octree_phi):
    keys, lv = o.leaves()
    x, y, z = I.leaf_corners3(keys, lv)
    phi = fn(x, y, z) * scale
    o.field_set(oracle.CORNER_PHI_3D, phi)
    g.field_set(slot, B.CORNER_PHI_3D, phi)


@pytest.mark.parametrize("precision", [64, 32])
def test_tree_locate_field_and_gather(precision):
    for d in (small_desc(precision), I.octree_static_desc(precision=precision)):
        o = oracle.Oracle(d)
        g = B.Context(d)
        ko, lo = o.leaves()
        kg, lg = g.leaves(0)
        assert np.array_equal(ko, kg) and np.array_equal(lo, lg)
        rng = np.random.Generator(np.random.PCG64(2))
        pts = rng.random((20000, 3))
        x, y, z = I.leaf_corners3(ko, lo)
        corners = np.stack([x[:500, 7], y[:500, 0], z[:500, 3]], 1) % 1.0
        pts = np.concatenate([pts, corners, [[0, 0, 0]]])
        assert np.array_equal(o.locate(pts), g.locate(0, pts))
        set_phi(o, g)
        assert np.array_equal(o.field_table(), g.field_table(0))
        assert np.array_equal(o.gather(pts), g.gather(0, pts))
        E = rng.normal(0, 1e3, (len(ko), 8, 3))
        o.field_set(oracle.CORNER_E_3D, E)
        g.field_set(0, B.CORNER_E_3D, E)
        assert np.array_equal(o.gather(pts), g.gather(0, pts))
        g.close()


@pytest.mark.parametrize("precision", [64, 32])
def test_free_steps_with_walls_and_sorts(precision):
    d = I.octree_static_desc(precision=precision)
    n = 200000
    s, v, w, ids = I.octree_particles(n, seed=3)
    o, g = load_both(d, [(s, v, w, ids)])
    set_phi(o, g)
    o.leapfrog_start()
    g.leapfrog_start(0)
    so = o.step(0, 50)
    sg = g.step(0, 50, sort_every=20)
    for k in ("alive_start", "absorbed", "lost_reflect"):
        assert so[k] == sg[k], (k, so[k], sg[k])
    assert_same_particles(o.read(0), g.read(0, 0), TOL[precision], "octree")
    assert np.array_equal(o.deposit(), g.deposit_read(0))
    qg, rg = g.deposit(0, rho=True)
    assert np.array_equal(o.deposit(), qg)
    assert np.allclose(o.rho(), rg, rtol=1e-15, atol=0)


@pytest.mark.parametrize("precision,ranking", [(64, 0), (32, 0), (32, 2)])
def test_avalanche_with_births(precision, ranking):
    d = I.octree_avalanche_desc(precision=precision)
    parts = I.octree_avalanche_particles(d, npairs=4000)
    o, g = load_both(d, parts)
    g.set_births_ranking(0, ranking)
    L = d["length"]
    set_phi(o, g, fn=lambda x, y, z: I.octree_avalanche_phi(d, x * L, y * L, z * L))
    o.leapfrog_start()
    g.leapfrog_start(0)
    births = 0
    for k in range(0, 80, 20):
        so = o.step(k, 20)
        sg = g.step(-1, 20, sort_every=10)
        for key in ("alive_start", "absorbed", "elastic", "ionization", "births", "numax_violations"):
            assert so[key] == sg[key], (k, key, so[key], sg[key])
        births += so["births"]
    assert births > 50
    for sp in range(2):
        assert_same_particles(o.read(sp), g.read(0, sp), TOL[precision], f"species {sp}")
    assert o.next_id == g.next_id(0)
    assert np.array_equal(o.deposit(), g.deposit_read(0))


def test_full_size_sampled():
    """The 4,194,304-particle octree workload in the benchmark's launch
    configuration against the oracle on 20,000 particles sampled by id (a
    collisionless particle depends only on its own state and the field)."""
    d = I.octree_static_desc(precision=32)
    n = 4194304
    s, v, w, ids = I.octree_particles(n)
    g = B.Context(d)
    g.load(0, 0, s, v, w, ids)
    o = oracle.Oracle(d)
    set_phi(o, g)
    g.leapfrog_start(0)
    g.step(0, 60, sort_every=50)
    pick = np.sort(np.random.Generator(np.random.PCG64(8)).choice(n, 20000, replace=False))
    o.load(0, s[pick], v[pick], w[pick], ids[pick])
    o.leapfrog_start()
    o.step(0, 60)
    ro, rg = o.read(0), g.read(0, 0)
    idx = np.searchsorted(rg["id"], ro["id"])
    sub = {k: rg[k][idx] for k in ("id", "w", "cell", "s", "v")}
    assert_same_particles(ro, sub, TOL[32], "sampled")
    q = g.deposit_read(0)[0]
    keys, lv = g.leaves(0)
    assert int(q.astype(np.int64).sum()) == 65536 * n
    assert np.array_equal(q, np.bincount(rg["cell"], minlength=len(keys)).astype(np.uint64) * 65536)


def test_octree_refuses_batched_adapt_and_solve():
    d = small_desc(32)
    g = B.Context([d, d])
    s, v, w, ids = I.octree_particles(1000)
    for j in range(2):
        g.load(j, 0, s, v, w, ids)
    for call in (lambda: g.step(0, 2, batched=1024), lambda: g.adapt(0), lambda: g.field_solve_2d(0)):
        with pytest.raises(B.PicError) as e:
            call()
        assert e.value.code == B.PIC_E_ARG
    g.close()
