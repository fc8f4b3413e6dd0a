"""GPU library vs CPU oracle on identical seeded inputs (through the C ABI).

Discrete results (ids, cells, counts, births, event counts, integer charge
sums, quadtree leaves) must match bit-exactly.  Floating-point particle state
is compared with the stated tolerance (1e-12 relative for FP64 paths, 1e-5
for FP32 paths against the FP32-mirror oracle); in practice it matches
bitwise, because both sides perform the same IEEE operations in the same
order without contraction."""
import math

import numpy as np
import pytest

import oracle
from paper_1604_07713_amd import binding as B
from paper_1604_07713_amd import inputs as I
from tests.gpu_common import assert_same_particles, ccp_run_both, load_both

pytestmark = pytest.mark.gpu

TOL = {64: 1e-12, 32: 1e-5}


def test_philox_matches_oracle():
    rng = np.random.Generator(np.random.PCG64(1))
    ctr = rng.integers(0, 2**32, (4096, 4), dtype=np.uint64).astype(np.uint32)
    key = np.array([0xDEADBEEF, 0x01234567], dtype=np.uint32)
    got = B.philox4x32(ctr, key)
    ref = np.stack([oracle.philox4x32(c, key) for c in ctr])
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("precision", [64, 32])
def test_derived_constants_match(precision):
    for d in (I.ccp_desc(precision=precision), I.streamer_desc(precision=precision)):
        o = oracle.Oracle(d)
        g = B.Context(d)
        for sp in range(len(d["species"])):
            a, b = o.derived(sp), g.derived(0, sp)
            for k in a:
                assert a[k] == b[k], (k, a[k], b[k])
        g.close()


def test_quadtree_mesh_and_locate():
    d = I.quadtree_static_desc()
    o = oracle.Oracle(d)
    g = B.Context(d)
    ko, lo = o.leaves()
    kg, lg = g.leaves(0)
    assert np.array_equal(ko, kg) and np.array_equal(lo, lg)
    assert len(kg) == 23620
    rng = np.random.Generator(np.random.PCG64(3))
    pts = rng.random((20000, 2))
    x0 = (np.arange(0, 1, 1 / 512.0))
    edge = np.stack(np.meshgrid(x0[::7], x0[::5]), -1).reshape(-1, 2)
    p1 = np.nextafter(1.0, 0.0)
    P = np.concatenate([pts, edge, [[0, 0], [p1, p1], [0, p1], [p1, 0]]])
    assert np.array_equal(g.locate(0, P), o.locate(P))


@pytest.mark.parametrize("precision", [64, 32])
def test_quadtree_field_tables_match(precision):
    d = I.quadtree_static_desc(precision=precision)
    o = oracle.Oracle(d)
    g = B.Context(d)
    keys, lv = o.leaves()
    cx, cy = I.leaf_corners(keys, lv)
    phi = I.quadtree_phi(cx, cy)
    o.field_set(oracle.CORNER_PHI_2D, phi)
    g.field_set(0, B.CORNER_PHI_2D, phi)
    assert np.array_equal(o.field_table(), g.field_table(0))
    # cell-centred potential path (node averaging, Dirichlet walls)
    d2 = I.streamer_desc(precision=precision, min_level=3, max_level=6)
    d2["refine_disk"], d2["disk_r"], d2["disk_level"] = 1, 0.2, 6
    o2 = oracle.Oracle(d2)
    g2 = B.Context(d2)
    rng = np.random.Generator(np.random.PCG64(4))
    cphi = rng.standard_normal(o2.nq())
    o2.field_set(oracle.CELL_PHI_2D, cphi)
    g2.field_set(0, B.CELL_PHI_2D, cphi)
    assert np.array_equal(o2.field_table(), g2.field_table(0))


@pytest.mark.parametrize("precision", [64, 32])
def test_deposit_matches_1d_and_2d(precision):
    d = I.ccp_desc(precision=precision, ncells=97, ppc=50)
    o, g = load_both(d, I.ccp_particles(d))
    assert np.array_equal(o.deposit(), g.deposit(0))
    d2 = I.quadtree_static_desc(precision=precision)
    s, v, w, ids = I.quadtree_particles(100000)
    w = (np.arange(100000) % 977 + 1).astype(np.uint32)
    o2, g2 = load_both(d2, [(s, v, w, ids)])
    assert np.array_equal(o2.deposit(), g2.deposit(0))


@pytest.mark.parametrize("ncells,heavy", [(300, False), (4096, False), (8192, True), (2, False)])
def test_poisson1d_matches_bitwise(ncells, heavy):
    """The exact 1D solve (128-bit integer prefix sums rounded once) on the
    GPU equals the oracle's bit for bit, from a few nodes to the largest mesh,
    also with weights near 2^32 (charge sums near 2^64 per node)."""
    d = I.ccp_desc(ncells=ncells, ppc=20)
    parts = I.ccp_particles(d)
    if heavy:
        rng = np.random.Generator(np.random.PCG64(4))
        parts = [(s, v, rng.integers(1 << 31, 1 << 32, len(w), dtype=np.uint64).astype(np.uint32), ids)
                 for (s, v, w, ids) in parts]
    o, g = load_both(d, parts)
    assert np.array_equal(o.deposit(), g.deposit(0))
    po, eo = o.field_solve_1d(321.5)
    pg, eg = g.field_solve_1d(0, 321.5)
    assert np.array_equal(po, pg) and np.array_equal(eo, eg)


@pytest.mark.parametrize("precision", [64, 32])
def test_ccp_400_steps_free_running(precision):
    """The 1D CCP discharge (gap 0.067 m, 128 cells, 64 particles per cell per
    species, 450 V at 13.56 MHz, 30 mTorr argon, null-collision MCC with
    ionization births): one full RF period of 400 steps, field solved on the
    device every step, particles re-sorted every 20 steps."""
    d = I.ccp_desc(precision=precision)
    o, g, so, sg = ccp_run_both(d, 400, sort_every=20)
    for k in ("alive_start", "absorbed", "elastic", "ionization", "cx", "births", "numax_violations"):
        assert so[k] == sg[k], (k, so[k], sg[k])
    assert so["births"] > 0 and so["elastic"] > 0 and so["cx"] > 0
    for sp in range(2):
        assert_same_particles(o.read(sp), g.read(0, sp), TOL[precision], f"species {sp}")
    assert o.next_id == g.next_id(0)
    assert np.array_equal(o.field_table(), g.field_table(0))


@pytest.mark.parametrize("precision", [64, 32])
def test_ccp_energy_conserving_coupling(precision):
    """The CCP discharge with the energy-conserving coupling (the particle
    takes its cell's E): 400 steps free running against the oracle."""
    d = I.ccp_desc(precision=precision)
    d["field_scheme"] = I.FIELD_CIC_EC
    o, g, so, sg = ccp_run_both(d, 400, sort_every=20)
    for k in ("alive_start", "absorbed", "elastic", "ionization", "cx", "births"):
        assert so[k] == sg[k], (k, so[k], sg[k])
    for sp in range(2):
        assert_same_particles(o.read(sp), g.read(0, sp), TOL[precision], f"species {sp}")
    assert o.next_id == g.next_id(0)
    assert np.array_equal(o.field_table(), g.field_table(0))


def test_ccp_binned_births_ranking():
    """The CCP discharge for 200 steps with the births ranked through id bins
    on the GPU: the same newborn ids, hence the same particles, as the
    oracle's ranking by parent id."""
    d = I.ccp_desc(precision=32)
    o, g, so, sg = ccp_run_both(d, 200, sort_every=20, births_ranking=2)
    assert so["births"] > 0 and so["births"] == sg["births"]
    for sp in range(2):
        assert_same_particles(o.read(sp), g.read(0, sp), TOL[32], f"species {sp}")
    assert o.next_id == g.next_id(0)


def test_quadtree_static_steps_bitwise():
    """2D static quadtree (levels 6-9), FP32 particles, reflecting walls, 100 steps."""
    d = I.quadtree_static_desc()
    n = 200000
    s, v, w, ids = I.quadtree_particles(n, seed=5)
    o, g = load_both(d, [(s, v, w, ids)])
    keys, lv = o.leaves()
    cx, cy = I.leaf_corners(keys, lv)
    phi = I.quadtree_phi(cx, cy)
    o.field_set(oracle.CORNER_PHI_2D, phi)
    g.field_set(0, B.CORNER_PHI_2D, phi)
    o.leapfrog_start()
    g.leapfrog_start(0)
    so = o.step(0, 100)
    sg = g.step(0, 100, sort_every=10)
    assert so["alive_start"] == sg["alive_start"] and so["lost_reflect"] == sg["lost_reflect"]
    assert_same_particles(o.read(0), g.read(0, 0), TOL[32])
    assert np.array_equal(o.deposit(), g.deposit(0))
