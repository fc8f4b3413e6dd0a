"""Oracle 3D octree (paper Sec. 3.1: quad/octree, cubic cells; Sec. 3:
gather from nodal E, leapfrog, NGP to the cell) pinned by brute force
geometry and closed forms:

  - the mesh tiles the cube in Morton order, every leaf meeting the refined
    ball sits at its level, the rest are coarser, and the tree is 2:1
    balanced across faces, edges and corners (all pairs of touching leaves);
  - point location equals a brute-force search over leaf boxes (half-open),
    also at nodes, faces, 0 and pred(1);
  - nodal E is exact for a linear potential; the gather is the trilinear
    interpolation of the leaf's corner E, computed here from leaf geometry,
    and is exact for linear E;
  - constant force: leapfrog positions equal x0 + v0 t + a t^2 / 2; a linear
    restoring field gives the closed-form leapfrog oscillation;
  - NGP charge per leaf equals brute-force counts; rho integrates to the
    total charge; reflecting walls keep particles inside on all six faces;
  - collision rates and births in 3D: event counts against n sigma v dt,
    newborn pairs at the parent's position with the next ids.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1604_07713_amd import inputs as I


def small_desc(precision=64, base=2, top=4, r=0.3, c=(0.41, 0.57, 0.5), bc=I.REFLECT):
    e = I.species(-I.E_CHARGE, I.M_ELECTRON, 1.0, I.MCC_NONE)
    return I.base_desc(dim=3, precision=precision, length=1.0, dt=1e-9, min_level=base, max_level=top,
                       base_level=base, refine_disk=1, disk_cx=c[0], disk_cy=c[1], disk_cz=c[2], disk_r=r,
                       disk_level=top, particle_bc=bc, species=[e], gas_mass=1.0)


def boxes(o):
    keys, lv = o.leaves()
    x, y, z = I.leaf_corners3(keys, lv)
    lo = np.stack([x[:, 0], y[:, 0], z[:, 0]], 1)
    hi = np.stack([x[:, 7], y[:, 7], z[:, 7]], 1)
    return keys, lv, lo, hi


def brute_locate(lo, hi, pts):
    out = np.empty(len(pts), dtype=np.int64)
    for i, p in enumerate(pts):
        m = np.nonzero(np.all((p >= lo) & (p < hi), axis=1))[0]
        assert len(m) == 1, (p, m)
        out[i] = m[0]
    return out


def check_mesh(library=None):
    d = small_desc()
    o = oracle.Oracle(d, library)
    keys, lv, lo, hi = boxes(o)
    # Morton tiling of the cube
    span = (8 ** (10 - lv.astype(np.int64)))
    assert keys[0] == 0 and np.array_equal(keys[1:].astype(np.int64), (keys[:-1].astype(np.int64) + span[:-1]))
    assert int(keys[-1]) + int(span[-1]) == 1 << 30
    assert np.sum(np.prod(hi - lo, axis=1)) == 1.0
    # ball rule: leaves meeting the closed ball are at the ball's level; a
    # leaf finer than the base has a parent that met the ball or touched a
    # leaf two levels finer than the parent (2:1 balance), nothing else
    c = np.array([d["disk_cx"], d["disk_cy"], d["disk_cz"]])

    def meets(a, b):
        g = np.maximum(np.maximum(a - c, 0.0), c - b)
        return np.sum(g * g, axis=-1) <= d["disk_r"] ** 2
    assert np.all(lv[meets(lo, hi)] == d["disk_level"])
    assert np.all(lv >= d["base_level"])
    for i in np.nonzero(lv > d["base_level"])[0]:
        hp = 2.0 ** -(int(lv[i]) - 1)
        plo = np.floor(lo[i] / hp) * hp
        phi = plo + hp
        t = np.all((lo <= phi) & (plo <= hi), axis=1)
        assert meets(plo, phi) or np.any(lv[t] >= lv[i] + 1), i
    # 2:1 across faces, edges and corners: every pair of touching closed boxes
    for i in range(len(lv)):
        t = np.all((lo <= hi[i]) & (lo[i] <= hi), axis=1)
        assert np.max(np.abs(lv[t].astype(int) - int(lv[i]))) <= 1, i
    return o, lo, hi


def test_octree_mesh_brute_force():
    check_mesh()


def test_octree_workload_mesh():
    o = oracle.Oracle(I.octree_static_desc(precision=64))
    keys, lv = o.leaves()
    assert np.array_equal(np.bincount(lv, minlength=8)[4:], [3784, 1432, 3832, 37440])


def check_locate(library=None):
    d = small_desc()
    o = oracle.Oracle(d, library)
    keys, lv, lo, hi = boxes(o)
    rng = np.random.Generator(np.random.PCG64(3))
    pts = [rng.random((400, 3))]
    # nodes, face and edge midpoints of some leaves, and the domain's ends
    idx = rng.choice(len(lv), 60, replace=False)
    for k in range(8):
        corner = np.stack([(lo if (k >> a) & 1 == 0 else hi)[idx, a] for a in range(3)], 1)
        pts.append(corner)
    pts.append((lo[idx] + hi[idx]) / 2)
    pts.append(np.stack([lo[idx, 0], (lo[idx, 1] + hi[idx, 1]) / 2, hi[idx, 2]], 1))
    pts = np.concatenate(pts)
    pts = np.clip(pts, 0.0, np.nextafter(1.0, 0.0))
    pts = np.concatenate([pts, [[0, 0, 0], [np.nextafter(1.0, 0.0)] * 3]])
    assert np.array_equal(o.locate(pts).astype(np.int64), brute_locate(lo, hi, pts))


def test_octree_locate_brute_force():
    check_locate()


def check_nodal_e(library=None):
    d = small_desc()
    o = oracle.Oracle(d, library)
    keys, lv = o.leaves()
    x, y, z = I.leaf_corners3(keys, lv)
    a, b, c, e = 0.7, 2.0, -3.0, 1.25
    o.field_set(oracle.CORNER_PHI_3D, a + b * x + c * y + e * z)
    E = o.field_table()
    assert np.allclose(E[..., 0], -b, rtol=0, atol=1e-12)
    assert np.allclose(E[..., 1], -c, rtol=0, atol=1e-12)
    assert np.allclose(E[..., 2], -e, rtol=0, atol=1e-12)


def test_octree_nodal_e_exact_for_linear_potential():
    check_nodal_e()


def check_trilinear(library=None):
    d = small_desc()
    o = oracle.Oracle(d, library)
    keys, lv, lo, hi = boxes(o)
    rng = np.random.Generator(np.random.PCG64(4))
    Ec = rng.normal(0, 1, (len(lv), 8, 3))
    o.field_set(oracle.CORNER_E_3D, Ec)
    pts = rng.random((300, 3))
    got = o.gather(pts)
    leaf = brute_locate(lo, hi, pts)
    f = (pts - lo[leaf]) / (hi[leaf] - lo[leaf])
    want = np.zeros_like(pts)
    for corner in range(8):
        w = np.ones(len(pts))
        for ax in range(3):
            w = w * (f[:, ax] if (corner >> ax) & 1 else 1 - f[:, ax])
        want += w[:, None] * Ec[leaf, corner]
    assert np.allclose(got, want, rtol=0, atol=1e-12)
    # linear E given at the corners is reproduced exactly
    x, y, z = I.leaf_corners3(keys, lv)
    lin = np.stack([2 * x - y, z + 0.5, 3 * y - x + z], -1)
    o.field_set(oracle.CORNER_E_3D, lin)
    got = o.gather(pts)
    assert np.allclose(got, np.stack([2 * pts[:, 0] - pts[:, 1], pts[:, 2] + 0.5,
                                      3 * pts[:, 1] - pts[:, 0] + pts[:, 2]], 1), rtol=0, atol=1e-12)


def test_octree_gather_is_trilinear():
    check_trilinear()


def test_octree_constant_force_leapfrog_exact():
    d = small_desc(bc=I.ABSORB)
    o = oracle.Oracle(d)
    keys, lv = o.leaves()
    x, y, z = I.leaf_corners3(keys, lv)
    g = np.array([30.0, -20.0, 45.0])    # V/m along x, y, z (phi = -g . x)
    o.field_set(oracle.CORNER_PHI_3D, -(g[0] * x + g[1] * y + g[2] * z))
    s0 = np.array([[0.3, 0.6, 0.45], [0.52, 0.41, 0.5]])
    v0 = np.array([[1e3, -2e3, 5e2], [-3e3, 1e3, 2e3]])
    o.load(0, s0, v0)
    o.leapfrog_start()
    n = 40
    o.step(0, n)
    qm = -I.E_CHARGE / I.M_ELECTRON
    t = n * d["dt"]
    want = s0 + (v0 * t + 0.5 * qm * g * t * t) / d["length"]
    assert np.allclose(o.read(0)["s"], want, rtol=0, atol=1e-12)


def test_octree_harmonic_motion_closed_form():
    d = small_desc()
    keys, lv = oracle.Oracle(d).leaves()
    x, y, z = I.leaf_corners3(keys, lv)
    qm = -I.E_CHARGE / I.M_ELECTRON
    w = 2 * math.pi / (40 * d["dt"])        # 40 steps per period
    kk = w * w / qm                         # E = -kk (x - 0.5), so the acceleration is -w^2 (x - 0.5)
    amp = np.array([0.1, 0.05, 0.08])
    th = math.acos(1 - (w * d["dt"]) ** 2 / 2)
    for n in (7, 20, 33):
        o2 = oracle.Oracle(d)
        o2.field_set(oracle.CORNER_E_3D, np.stack([-kk * (x - 0.5), -kk * (y - 0.5), -kk * (z - 0.5)], -1))
        o2.load(0, (0.5 + amp)[None, :], np.zeros((1, 3)))
        o2.leapfrog_start()
        o2.step(0, n)
        # leapfrog with v(-1/2) = -(qm dt/2) E(x0): x_n - 0.5 = amp cos(n theta) exactly
        assert np.allclose(o2.read(0)["s"][0] - 0.5, amp * math.cos(n * th), rtol=0, atol=1e-12)


def test_octree_ngp_deposit_and_rho():
    d = small_desc()
    o = oracle.Oracle(d)
    keys, lv, lo, hi = boxes(o)
    rng = np.random.Generator(np.random.PCG64(5))
    n = 5000
    s = rng.random((n, 3))
    w = rng.integers(1, 1 << 20, n).astype(np.uint32)
    o.load(0, s, np.zeros((n, 3)), w=w)
    q = o.deposit()[0]
    leaf = brute_locate(lo, hi, s)
    assert np.array_equal(q, np.bincount(leaf, weights=w, minlength=len(lv)).astype(np.uint64))
    vol = np.prod(hi - lo, axis=1)
    total = float((o.rho() * vol).sum())
    want = -I.E_CHARGE * float(w.astype(np.float64).sum()) / 65536.0
    assert abs(total - want) <= 1e-12 * abs(want)


def test_octree_reflecting_walls_all_faces():
    d = small_desc()
    o = oracle.Oracle(d)
    rng = np.random.Generator(np.random.PCG64(6))
    n = 3000
    s = rng.random((n, 3))
    v = rng.normal(0, 3e7, (n, 3))          # several cell crossings per step
    o.load(0, s, v)
    o.leapfrog_start()
    st = o.step(0, 20)
    r = o.read(0)
    assert st["absorbed"] == [0, 0] and len(r["id"]) == n
    assert np.all((r["s"] >= 0) & (r["s"] < 1))
    assert np.array_equal(np.abs(r["v"]), np.abs(v))     # no field: reflections only flip signs


def test_octree_collisions_and_births():
    d = I.octree_avalanche_desc(precision=64)
    o = oracle.Oracle(d)
    keys, lv = o.leaves()
    x, y, z = I.leaf_corners3(keys, lv)
    o.field_set(oracle.CORNER_PHI_3D, I.octree_avalanche_phi(d, x * d["length"], y * d["length"],
                                                              z * d["length"]))
    parts = I.octree_avalanche_particles(d, npairs=4000)
    for sp, (s, v, w, ids) in enumerate(parts):
        o.load(sp, s, v, w, ids)
    o.leapfrog_start()
    births = elastic = 0
    for k in range(60):
        before = o.next_id
        st = o.step(k, 1)
        births += st["births"]
        elastic += st["elastic"]
        assert o.next_id == before + 2 * st["births"]
    assert births > 0 and elastic > 0
    e, i = o.read(0), o.read(1)
    born_e = e["id"] >= 8000
    born_i = i["id"] >= 8000
    assert np.all(e["id"][born_e] % 2 == 0) and np.all(i["id"][born_i] % 2 == 1)
    assert np.count_nonzero(born_e) <= births and np.count_nonzero(born_i) == births
    # ions do not move far in 60 steps: a newborn ion sits where its pair was born
    assert np.all((i["s"] >= 0) & (i["s"] < 1))


def test_octree_elastic_rate_matches_cross_section():
    """Elastic events per step at a fixed speed (no field, isotropic):
    N (T / 2^24) a_el |v|, the null-collision candidate rate times the
    elastic share, from the derived constants."""
    d = I.octree_avalanche_desc(precision=64)
    d["species"][0]["sigma_iz"] = 0.0
    o = oracle.Oracle(d)
    n = 40000
    rng = np.random.Generator(np.random.PCG64(9))
    s = 0.3 + 0.4 * rng.random((n, 3))
    speed = 1.5e6
    dirs = rng.normal(size=(n, 3))
    v = speed * dirs / np.linalg.norm(dirs, axis=1)[:, None]
    o.load(0, s, v)
    o.load(1, s[:1], np.zeros((1, 3)), ids=np.array([n], dtype=np.uint32))
    st = o.step(0, 1)
    k = o.derived(0)
    p = k["Tcand"] / 2.0 ** 24 * k["a_el"] * speed
    mean = n * p
    assert abs(st["elastic"] - mean) <= 5 * math.sqrt(mean * (1 - p)), (st["elastic"], mean)
