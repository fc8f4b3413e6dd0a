"""Shared helpers of the GPU parity tests: run the same seeded workload on the
GPU library (through the C ABI) and on the CPU oracle, and compare."""
import numpy as np

import oracle
from paper_1604_07713_amd import binding as B
from paper_1604_07713_amd import inputs as I


def load_both(desc, parts, ctx=None, slot=0):
    o = oracle.Oracle(desc)
    g = ctx if ctx is not None else B.Context(desc)
    for sp, (s, v, w, ids) in enumerate(parts):
        o.load(sp, s, v, w, ids)
        g.load(slot, sp, s, v, w, ids)
    return o, g


def assert_same_particles(a, b, tol, what=""):
    """a, b: dicts from read(); ids must match exactly, weights exactly, and
    positions / velocities to the relative tolerance tol (0 = bitwise)."""
    assert len(a["id"]) == len(b["id"]), f"{what}: counts differ {len(a['id'])} vs {len(b['id'])}"
    assert np.array_equal(a["id"], b["id"]), f"{what}: ids differ"
    assert np.array_equal(a["w"], b["w"]), f"{what}: weights differ"
    assert np.array_equal(a["cell"], b["cell"]), f"{what}: cells differ"
    if len(a["id"]) == 0:
        return
    for k in ("s", "v"):
        x, y = a[k], b[k]
        if tol == 0:
            bad = np.nonzero(np.any(x != y, axis=1))[0]
            assert len(bad) == 0, f"{what}: {k} differs for {len(bad)} particles, first id {a['id'][bad[0]]}: {x[bad[0]]} vs {y[bad[0]]}"
        else:
            scale = np.maximum(np.abs(x), np.abs(y))
            err = np.abs(x - y) / np.where(scale > 0, scale, 1.0)
            assert err.max() <= tol, f"{what}: {k} max rel error {err.max()}"


def ccp_run_both(desc, nsteps, sort_every=20, gpu_kwargs=None, births_ranking=0):
    parts = I.ccp_particles(desc)
    o, g = load_both(desc, parts)
    g.set_births_ranking(0, births_ranking)
    o.deposit()
    g.deposit(0)
    v0 = float(I.drive_voltage(desc, 0))
    o.field_solve_1d(v0)
    g.field_solve_1d(0, v0)
    o.leapfrog_start()
    g.leapfrog_start(0)
    vn = I.drive_voltage(desc, np.arange(1, nsteps + 1))
    so = o.step(0, nsteps, vn, True)
    sg = g.step(0, nsteps, vn, solve_field=True, sort_every=sort_every, **(gpu_kwargs or {}))
    return o, g, so, sg
