"""pic_step_noalloc (the step for callers that cannot allocate device
memory) against pic_step with the same arguments, through the C ABI: two
calls in a row on the same device workspace, the second with a smaller
input; and the refusal of launch tables larger than the workspace."""
import numpy as np
import pytest

from paper_1604_07713_amd import binding as B
from paper_1604_07713_amd import inputs as I
from tests.gpu_common import assert_same_particles

pytestmark = pytest.mark.gpu


def ensemble(n, seed, precision=32):
    descs = I.ensemble_descs(count=n, seed=seed, precision=precision)
    for d in descs:   # keep the test small: at most 1024 cells and 64 particles per cell
        d.update(I.ccp_desc(ncells=min(d["ncells"], 1024), ppc=min(d["extra"]["ppc"], 64), precision=precision,
                            seed=seed, instance_key=d["instance_key"], voltage=d["extra"]["voltage"],
                            pressure_mtorr=d["extra"]["pressure_mtorr"]))
    g = B.Context(descs)
    for j, d in enumerate(descs):
        for sp, (s, v, w, ids) in enumerate(I.ensemble_particles(d)):
            g.load(j, sp, s, v, w, ids)
        g.deposit(j)
        g.field_solve_1d(j, float(I.drive_voltage(d, 0)))
        g.leapfrog_start(j)
    return descs, g


@pytest.mark.parametrize("precision", [32, 64])
def test_noalloc_step_equals_step_twice(precision):
    for call, (n, seed, nsteps) in enumerate([(6, 41, 100), (2, 43, 50)]):   # the second input is smaller
        descs, ref = ensemble(n, seed, precision)
        _, run = ensemble(n, seed, precision)
        vn = np.stack([I.drive_voltage(d, np.arange(1, nsteps + 1)) for d in descs], axis=1)
        kw = dict(solve_field=True, sort_every=20, batched=4096, grid=512)
        sr = ref.step(0, nsteps, vn, **kw)
        st = run.step(0, nsteps, vn, noalloc=True, **kw)
        print(f"call {call}: {n} instances, {nsteps} steps, births {st['births']}", flush=True)
        for k in ("alive_start", "absorbed", "elastic", "ionization", "cx", "births"):
            assert sr[k] == st[k], (call, k, sr[k], st[k])
        for j in range(n):
            for sp in range(2):
                assert_same_particles(ref.read(j, sp), run.read(j, sp), 0, f"call {call} slot {j} species {sp}")
            assert np.array_equal(ref.deposit_read(j), run.deposit_read(j))
            assert np.array_equal(ref.field_table(j), run.field_table(j))
            assert ref.step_index(j) == run.step_index(j) == nsteps
        ref.close()
        run.close()


def test_noalloc_refuses_tables_beyond_the_workspace():
    d = I.ccp_desc(ncells=4096, ppc=4, precision=32)
    g = B.Context(d)
    rng = np.random.Generator(np.random.PCG64(9))
    n = 20_000_000          # work items of 256 particles: 2 x 78125 items, over the workspace
    for sp in range(2):
        g.load(0, sp, I.unit_positions(rng, (n, 1)), np.zeros((n, 3)), None, np.arange(sp * n, (sp + 1) * n, dtype=np.uint32))
    g.deposit(0)
    g.field_solve_1d(0, 0.0)
    with pytest.raises(B.PicError) as e:
        g.step(0, 1, np.zeros((1, 1)), solve_field=True, batched=256, noalloc=True)
    assert e.value.code == B.PIC_E_ARG and "workspace" in str(e.value)
    assert g.step_index(0) == 0
    # the same call through pic_step, which allocates its tables, runs
    g.step(0, 1, np.zeros((1, 1)), solve_field=True, batched=256)
    assert g.step_index(0) == 1
