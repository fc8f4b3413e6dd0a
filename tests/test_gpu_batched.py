"""Batched ensemble: many uneven 1D CCP instances stepped by one persistent
launch per step (optionally replayed from a captured HIP graph) must give,
instance by instance, exactly the oracle's result -- the same as stepping
each instance alone."""
import numpy as np
import pytest

import oracle
from paper_1604_07713_amd import binding as B
from paper_1604_07713_amd import inputs as I
from tests.gpu_common import assert_same_particles

pytestmark = pytest.mark.gpu
TOL = {64: 1e-12, 32: 1e-5}


def small_ensemble(n=6, precision=32):
    full = I.ensemble_descs(count=n, precision=precision)
    return [I.ccp_desc(ncells=d["ncells"], ppc=8, voltage=d["extra"]["voltage"],
                       pressure_mtorr=d["extra"]["pressure_mtorr"], precision=precision, seed=4, instance_key=k)
            for k, d in enumerate(full)]


def start(ctx_or_oracles, descs, gpu):
    for j, d in enumerate(descs):
        parts = I.ensemble_particles(d)
        v0 = float(I.drive_voltage(d, 0))
        if gpu:
            g = ctx_or_oracles
            for sp, (s, v, w, ids) in enumerate(parts):
                g.load(j, sp, s, v, w, ids)
            g.deposit(j)
            g.field_solve_1d(j, v0)
            g.leapfrog_start(j)
        else:
            o = ctx_or_oracles[j]
            for sp, (s, v, w, ids) in enumerate(parts):
                o.load(sp, s, v, w, ids)
            o.deposit()
            o.field_solve_1d(v0)
            o.leapfrog_start()


@pytest.mark.parametrize("precision,graph", [(32, 0), (32, 10), (64, 0)])
def test_batched_ensemble_matches_oracle(precision, graph):
    check_against_oracle(small_ensemble(precision=precision), precision, graph)


@pytest.mark.parametrize("precision,graph", [(32, 10), (64, 0)])
def test_batched_mixed_field_schemes(precision, graph):
    """Every other instance uses the energy-conserving coupling (cell E,
    no interpolation): the batched launch honours each instance's scheme."""
    descs = small_ensemble(precision=precision)
    for j in range(1, len(descs), 2):
        descs[j]["field_scheme"] = I.FIELD_CIC_EC
    check_against_oracle(descs, precision, graph)


def check_against_oracle(descs, precision, graph):
    nsteps = 60
    vn = np.stack([I.drive_voltage(d, np.arange(1, nsteps + 1)) for d in descs], axis=1)   # [k][slot]
    g = B.Context(descs)
    start(g, descs, True)
    sg = g.step(0, nsteps, vn, solve_field=True, batched=1024, sort_every=20, graph_steps=graph)
    orc = [oracle.Oracle(d) for d in descs]
    start(orc, descs, False)
    tot = dict(alive_start=[0, 0], births=0, elastic=0, cx=0)
    for j, o in enumerate(orc):
        so = o.step(0, nsteps, vn[:, j], True)
        tot["alive_start"][0] += so["alive_start"][0]
        tot["alive_start"][1] += so["alive_start"][1]
        for k in ("births", "elastic", "cx"):
            tot[k] += so[k]
        for sp in range(2):
            assert_same_particles(o.read(sp), g.read(j, sp), TOL[precision], f"slot {j} species {sp}")
        assert o.next_id == g.next_id(j)
        assert np.array_equal(o.field_table(), g.field_table(j))
    assert sg["alive_start"] == tot["alive_start"]
    for k in ("births", "elastic", "cx"):
        assert sg[k] == tot[k], (k, sg[k], tot[k])


def test_batched_equals_plain_per_slot():
    descs = small_ensemble(n=4, precision=32)
    nsteps = 40
    vn = np.stack([I.drive_voltage(d, np.arange(1, nsteps + 1)) for d in descs], axis=1)
    a = B.Context(descs)
    b = B.Context(descs)
    start(a, descs, True)
    start(b, descs, True)
    a.step(0, nsteps, vn, solve_field=True, batched=2048, grid=64)
    b.step(0, nsteps, vn, solve_field=True)
    for j in range(len(descs)):
        for sp in range(2):
            assert_same_particles(a.read(j, sp), b.read(j, sp), 0, f"slot {j} species {sp}")
