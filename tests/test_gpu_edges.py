"""Edge cases of the step loop against the oracle: particle counts below one
wave and not a multiple of the batch (lanes past the end must neither load
out of range nor contribute) on the quadtree and the octree, discharges of
one particle per cell (explicit and direct implicit), and instances whose
particles all leave through the walls and which keep stepping empty (1D
explicit and direct implicit, octree)."""
import numpy as np
import pytest

import oracle
from paper_1604_07713_amd import binding as B
from paper_1604_07713_amd import inputs as I
from tests.gpu_common import assert_same_particles, ccp_run_both, load_both

pytestmark = pytest.mark.gpu
TOL = {64: 1e-12, 32: 1e-5}


@pytest.mark.parametrize("n", [1, 5, 63, 257, 513])
def test_quadtree_ragged_counts(n):
    """The static quadtree with n FP32 electrons (fewer than a wave, or a
    ragged last batch), 60 steps with a sort every 10."""
    d = I.quadtree_static_desc()
    s, v, w, ids = I.quadtree_particles(n, seed=9)
    o, g = load_both(d, [(s, v, w, ids)])
    keys, lv = o.leaves()
    cx, cy = I.leaf_corners(keys, lv)
    phi = I.quadtree_phi(cx, cy)
    o.field_set(oracle.CORNER_PHI_2D, phi)
    g.field_set(0, B.CORNER_PHI_2D, phi)
    o.leapfrog_start()
    g.leapfrog_start(0)
    so = o.step(0, 60)
    sg = g.step(0, 60, sort_every=10)
    assert so["alive_start"] == sg["alive_start"]
    assert_same_particles(o.read(0), g.read(0, 0), TOL[32], f"n={n}")
    assert np.array_equal(o.deposit(), g.deposit(0))


@pytest.mark.parametrize("precision", [64, 32])
def test_ccp_one_particle_per_cell(precision):
    """A 16-cell discharge with one electron and one ion per cell (32
    particles, collisions and births on), 200 steps."""
    d = I.ccp_desc(ncells=16, ppc=1, precision=precision)
    o, g, so, sg = ccp_run_both(d, 200, sort_every=20)
    for k in ("alive_start", "absorbed", "elastic", "ionization", "cx", "births"):
        assert so[k] == sg[k], (k, so[k], sg[k])
    for sp in range(2):
        assert_same_particles(o.read(sp), g.read(0, sp), TOL[precision], f"species {sp}")
    assert o.next_id == g.next_id(0)


def test_ccp_all_particles_leave_then_empty_steps():
    """Every particle starts next to the grounded wall moving out: after a
    few steps the instance is empty on both sides, its deposit is zero, and
    30 more steps of an empty instance change nothing."""
    d = I.ccp_desc(ncells=64, ppc=4, precision=64)
    rng = np.random.Generator(np.random.PCG64(13))
    ne = 40
    s = 0.999 + 0.0009 * rng.random((ne, 1))
    ve = np.zeros((ne, 3))
    ve[:, 0] = 1.0e7
    vi = np.zeros((ne, 3))
    vi[:, 0] = 1.0e7
    parts = [(s, ve, None, np.arange(ne, dtype=np.uint32)),
             (s.copy(), vi, None, np.arange(ne, 2 * ne, dtype=np.uint32))]
    o, g = load_both(d, parts)
    o.deposit()
    g.deposit(0)
    v0 = float(I.drive_voltage(d, 0))
    o.field_solve_1d(v0)
    g.field_solve_1d(0, v0)
    o.leapfrog_start()
    g.leapfrog_start(0)
    vn = I.drive_voltage(d, np.arange(1, 41))
    so = o.step(0, 10, vn[:10], True)
    sg = g.step(0, 10, vn[:10], solve_field=True, sort_every=5)
    assert so["absorbed"] == sg["absorbed"] and sg["absorbed"][0] == ne and sg["absorbed"][1] == ne
    for sp in range(2):
        assert len(g.read(0, sp)["id"]) == 0 and len(o.read(sp)["id"]) == 0
    so = o.step(10, 30, vn[10:40], True)
    sg = g.step(10, 30, vn[10:40], solve_field=True, sort_every=5)
    assert sg["alive_start"] == [0, 0] and so["alive_start"] == sg["alive_start"]
    q = g.deposit_read(0)
    assert not np.any(q)
    assert o.next_id == g.next_id(0)
    assert np.array_equal(o.field_table(), g.field_table(0))


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_positions_rounding_to_one_in_fp32_are_refused(dim):
    """A double in [1 - 2^-25, 1) is inside the domain but rounds to 1.0 in
    FP32, outside it: an FP32 slot refuses it at load (as the oracle does), an
    FP64 slot takes it; the point gather refuses it the same way."""
    near = 1.0 - 2.0 ** -26
    for prec, ok in ((32, False), (64, True)):
        if dim == 1:
            d = I.ccp_desc(ncells=16, ppc=4, precision=prec)
        elif dim == 2:
            d = I.quadtree_static_desc(precision=prec)
        else:
            d = I.octree_static_desc(precision=prec)
        g = B.Context(d)
        s = np.full((4, dim), 0.5)
        s[2, dim - 1] = near
        if ok:
            g.load(0, 0, s, np.zeros((4, 3)))
            assert g.count(0, 0) == 4
        else:
            with pytest.raises(B.PicError) as e:
                g.load(0, 0, s, np.zeros((4, 3)))
            assert e.value.code == B.PIC_E_ARG
            with pytest.raises(B.PicError) as e:
                g.gather(0, s)
            assert e.value.code == B.PIC_E_ARG
        g.close()


@pytest.mark.parametrize("n", [1, 5, 63, 257, 513])
def test_octree_ragged_counts(n):
    """The static octree with n FP32 electrons (fewer than a wave, or a
    ragged last range), 40 steps with a sort every 10."""
    d = I.octree_static_desc()
    s, v, w, ids = I.octree_particles(n, seed=9)
    o, g = load_both(d, [(s, v, w, ids)])
    keys, lv = o.leaves()
    x, y, z = I.leaf_corners3(keys, lv)
    phi = I.octree_phi(x, y, z)
    o.field_set(oracle.CORNER_PHI_3D, phi)
    g.field_set(0, B.CORNER_PHI_3D, phi)
    o.leapfrog_start()
    g.leapfrog_start(0)
    so = o.step(0, 40)
    sg = g.step(0, 40, sort_every=10)
    assert so["alive_start"] == sg["alive_start"]
    assert_same_particles(o.read(0), g.read(0, 0), TOL[32], f"n={n}")
    assert np.array_equal(o.deposit(), g.deposit(0))


def test_octree_all_particles_leave_then_empty_steps():
    """Absorbing walls and every electron next to the x = 1 face moving out:
    the instance empties within a few steps, its deposit is zero, and empty
    steps change nothing."""
    d = dict(I.octree_static_desc(precision=64), particle_bc=I.ABSORB)
    rng = np.random.Generator(np.random.PCG64(14))
    n = 300
    s = rng.random((n, 3)) * 0.9 + 0.05
    s[:, 0] = 0.999 + 0.0009 * rng.random(n)
    v = np.zeros((n, 3))
    v[:, 0] = 1.0e7
    o, g = load_both(d, [(s, v, None, np.arange(n, dtype=np.uint32))])
    keys, lv = o.leaves()
    x, y, z = I.leaf_corners3(keys, lv)
    phi = I.octree_phi(x, y, z)
    o.field_set(oracle.CORNER_PHI_3D, phi)
    g.field_set(0, B.CORNER_PHI_3D, phi)
    o.leapfrog_start()
    g.leapfrog_start(0)
    so = o.step(0, 5)
    sg = g.step(0, 5, sort_every=2)
    assert so["absorbed"] == sg["absorbed"] and sg["absorbed"][0] == n
    assert len(g.read(0, 0)["id"]) == 0 and len(o.read(0)["id"]) == 0
    sg = g.step(5, 20, sort_every=3)
    assert sg["alive_start"][0] == 0 and not np.any(g.deposit_read(0))


@pytest.mark.parametrize("precision", [64, 32])
def test_direct_implicit_one_particle_per_cell(precision):
    """The direct implicit discharge on 16 cells with one electron and one
    ion per cell (collisions and births on), 200 steps."""
    d = I.dipic_ccp_desc(ncells=16, ppc=1, precision=precision)
    o, g, so, sg = ccp_run_both(d, 200, sort_every=20)
    for k in ("alive_start", "absorbed", "elastic", "ionization", "cx", "births"):
        assert so[k] == sg[k], (k, so[k], sg[k])
    for sp in range(2):
        assert_same_particles(o.read(sp), g.read(0, sp), TOL[precision], f"species {sp}")
    assert o.next_id == g.next_id(0)
    a, b = o.field_table(), g.field_table(0)
    assert np.allclose(a, b, rtol=TOL[precision], atol=TOL[precision] * np.abs(a).max())


def test_direct_implicit_all_particles_leave_then_empty_steps():
    """A direct implicit slot whose particles all leave through the grounded
    wall: the predictor absorbs them, the field becomes the drive's vacuum
    field (no charge, no susceptibility), and empty steps match the oracle."""
    d = I.dipic_ccp_desc(ncells=64, ppc=4, precision=64)
    rng = np.random.Generator(np.random.PCG64(15))
    ne = 40
    s = 0.999 + 0.0009 * rng.random((ne, 1))
    v = np.zeros((ne, 3))
    v[:, 0] = 1.0e7
    parts = [(s, v, None, np.arange(ne, dtype=np.uint32)),
             (s.copy(), v.copy(), None, np.arange(ne, 2 * ne, dtype=np.uint32))]
    o, g = load_both(d, parts)
    o.deposit()
    g.deposit(0)
    v0 = float(I.drive_voltage(d, 0))
    o.field_solve_1d(v0)
    g.field_solve_1d(0, v0)
    o.leapfrog_start()
    g.leapfrog_start(0)
    vn = I.drive_voltage(d, np.arange(1, 31))
    so = o.step(0, 10, vn[:10], True)
    sg = g.step(0, 10, vn[:10], solve_field=True, sort_every=5)
    assert so["absorbed"] == sg["absorbed"] and sg["absorbed"][0] == ne and sg["absorbed"][1] == ne
    so = o.step(10, 20, vn[10:30], True)
    sg = g.step(10, 20, vn[10:30], solve_field=True, sort_every=5)
    assert sg["alive_start"] == [0, 0] and so["alive_start"] == sg["alive_start"]
    assert not np.any(g.deposit_read(0))
    E = g.field_table(0)
    assert np.array_equal(o.field_table(), E)
    assert np.allclose(E, vn[-1] / d["length"], rtol=1e-12)   # uniform vacuum field of the last drive value
