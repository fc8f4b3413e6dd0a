"""Device memory from the caller's allocator (pic_set_allocator): a context
whose blocks come from torch's caching allocator gives exactly the particles of
a context on the library's own block cache, holds its memory in torch's
accounting while it lives, and returns it when closed."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1604_07713_amd import binding as B
from paper_1604_07713_amd import inputs as I
from tests.gpu_common import assert_same_particles

pytestmark = pytest.mark.gpu


def streamer_run(allocator):
    d = I.streamer_desc(precision=32)
    g = B.Context(d, allocator=allocator)
    for sp, (s, v, w, ids) in enumerate(I.streamer_particles(d, npairs=3000)):
        g.load(0, sp, s, v, w, ids)
    g.adapt(0)
    g.field_solve_2d(0, rtol=1e-8, maxit=4000)
    g.leapfrog_start(0)
    for k in range(6):
        g.step(-1, 10, sort_every=0)
        g.adapt(0)
        g.field_solve_2d(0, rtol=1e-8, maxit=4000)
    return g


def ensemble_run(allocator):
    full = I.ensemble_descs(count=6, precision=32)
    descs = [I.ccp_desc(ncells=d["ncells"], ppc=8, voltage=d["extra"]["voltage"],
                        pressure_mtorr=d["extra"]["pressure_mtorr"], precision=32, seed=4, instance_key=k)
             for k, d in enumerate(full)]
    g = B.Context(descs, allocator=allocator)
    for j, d in enumerate(descs):
        for sp, (s, v, w, ids) in enumerate(I.ensemble_particles(d)):
            g.load(j, sp, s, v, w, ids)
        g.deposit(j)
        g.field_solve_1d(j, float(I.drive_voltage(d, 0)))
        g.leapfrog_start(j)
    nsteps = 40
    vn = np.stack([I.drive_voltage(d, np.arange(1, nsteps + 1)) for d in descs], axis=1)
    g.step(0, nsteps, vn, solve_field=True, sort_every=20, batched=1024, grid=256, graph_steps=10)
    return g, len(descs)


def test_torch_allocator_streamer_identical():
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    a = streamer_run(None)
    b = streamer_run(B.TorchAllocator())
    assert torch.cuda.memory_allocated() > base   # b's blocks are torch's
    keys_a, lv_a = a.leaves(0)
    keys_b, lv_b = b.leaves(0)
    assert np.array_equal(keys_a, keys_b) and np.array_equal(lv_a, lv_b)
    for sp in range(2):
        assert_same_particles(a.read(0, sp), b.read(0, sp), 0, f"species {sp}")
        assert np.array_equal(a.deposit_read(0)[sp], b.deposit_read(0)[sp])
    assert a.next_id(0) == b.next_id(0)
    a.close()
    b.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_torch_allocator_batched_graph_identical():
    a, n = ensemble_run(None)
    b, _ = ensemble_run(B.TorchAllocator())
    for j in range(n):
        for sp in range(2):
            assert_same_particles(a.read(j, sp), b.read(j, sp), 0, f"instance {j} species {sp}")
        assert np.array_equal(a.field_table(j), b.field_table(j))
    a.close()
    b.close()


def test_allocator_rejected_once_instances_are_held():
    d = I.ccp_desc(ncells=32, ppc=4, precision=32)
    g = B.Context(d)
    alloc = B.TorchAllocator()
    rc = B.lib().pic_set_allocator(g.h, C.byref(alloc.struct))
    assert rc == B.PIC_E_STATE
    g.close()
