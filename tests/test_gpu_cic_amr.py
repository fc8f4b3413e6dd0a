"""GPU cloud-in-cell on the quadtree (paper Sec. 3.1, Fig. 2) against the
oracle, through the C ABI: the gather of a cell field, the deposit, the
cell-centred field table, free-running steps of the quadtree workload, and
the avalanche with collisions, births and adaptation.  Discrete results and
deposits bit for bit; positions and velocities to 1e-12 (FP64) / 1e-5
(FP32) relative (in practice bitwise)."""
import numpy as np
import pytest

import oracle
from paper_1604_07713_amd import binding as B
from paper_1604_07713_amd import inputs as I
from tests.gpu_common import assert_same_particles, load_both
from tests.test_gpu_adapt import adapt_both, compare_all

pytestmark = pytest.mark.gpu
TOL = {64: 1e-12, 32: 1e-5}


def tree_desc(precision, base=3, top=6, r=0.25, reflect=True):
    e = I.species(-I.E_CHARGE, I.M_ELECTRON, 1.0, I.MCC_NONE)
    return I.base_desc(dim=2, precision=precision, length=1.0, dt=1e-9, min_level=base, max_level=top,
                       base_level=base, refine_disk=1, disk_cx=0.41, disk_cy=0.57, disk_r=r, disk_level=top,
                       particle_bc=I.REFLECT if reflect else I.ABSORB, species=[e], gas_mass=1.0,
                       field_scheme=I.FIELD_CIC_AMR)


@pytest.mark.parametrize("precision", [64, 32])
def test_gather_and_deposit_match(precision):
    d = tree_desc(precision)
    rng = np.random.Generator(np.random.PCG64(3))
    n = 50000
    s = rng.random((n, 2))
    s[:500] = rng.random((500, 2)) * 0.02            # the corner and walls (folded clouds)
    s[500:1000, 1] = 1 - rng.random(500) * 1e-3
    w = rng.integers(1, 1 << 18, n).astype(np.uint32)
    o, g = load_both(d, [(s, np.zeros((n, 3)), w, np.arange(n, dtype=np.uint32))])
    qo = o.deposit()
    qg, rg = g.deposit(0, rho=True)
    assert np.array_equal(qo, qg)
    assert np.array_equal(o.rho(), rg)
    E = rng.normal(0, 1e4, (o.nq(), 2))
    o.field_set(oracle.CELL_E_2D, E)
    g.field_set(0, B.CELL_E_2D, E)
    assert np.array_equal(o.field_table(), g.field_table(0))
    pts = np.concatenate([rng.random((20000, 2)), s[:1000]])
    assert np.array_equal(o.gather(pts), g.gather(0, pts))


@pytest.mark.parametrize("precision", [64, 32])
def test_cell_table_from_potential_and_free_steps(precision):
    d = tree_desc(precision)
    n = 200000
    s, v, w, ids = I.quadtree_particles(n, seed=5)
    o, g = load_both(d, [(s, v, w, ids)])
    keys, lv = o.leaves()
    cx, cy = I.leaf_corners(keys, lv)
    phi = I.quadtree_phi(cx, cy)
    o.field_set(oracle.CORNER_PHI_2D, phi)
    g.field_set(0, B.CORNER_PHI_2D, phi)
    assert np.array_equal(o.field_table(), g.field_table(0))
    o.leapfrog_start()
    g.leapfrog_start(0)
    so = o.step(0, 50)
    sg = g.step(0, 50, sort_every=20)
    for k in ("alive_start", "absorbed", "lost_reflect"):
        assert so[k] == sg[k], (k, so[k], sg[k])
    assert_same_particles(o.read(0), g.read(0, 0), TOL[precision], "quadtree cloud")
    assert np.array_equal(o.deposit(), g.deposit_read(0))


@pytest.mark.parametrize("precision", [64, 32])
def test_avalanche_with_births_and_adapt(precision):
    d = I.streamer_desc(precision=precision, max_level=10)
    d["field_scheme"] = I.FIELD_CIC_AMR
    parts = I.streamer_particles(d, npairs=3000)
    o, g = load_both(d, parts)
    adapt_both(o, g)
    compare_all(o, g, precision, "initial adapt")
    births = 0
    for n in range(60):
        if n % 10 == 0:
            if n:
                adapt_both(o, g)
            o.deposit()
            o.field_solve_2d(rtol=1e-10)
            E = o.field_table()
            o.field_set(oracle.CELL_E_2D, E)
            g.field_set(0, B.CELL_E_2D, E)
            if n == 0:
                o.leapfrog_start()
                g.leapfrog_start(0)
        so = o.step(n, 1)
        sg = g.step(n, 1)
        for k in ("alive_start", "absorbed", "elastic", "ionization", "births", "numax_violations"):
            assert so[k] == sg[k], (n, k, so[k], sg[k])
        births += so["births"]
    assert births > 50
    compare_all(o, g, precision, "after 60 steps")
