"""Device allocation failures, injected through the caller's allocator
(pic_set_allocator) at every allocation request of a call, with the launch
checks on (every kernel-side view of a slot is checked on the host against
the slot's live blocks before use, so a stale or short table is an error
rather than a launch):

  - a step that grows an ionizing avalanche (paper Sec. 4.3: births multiply
    the particles): PIC_E_NOMEM leaves the slot at its last committed step,
    and the retry ends bit-identical to a run that never failed; a second
    context on the same stream, stepped between the failure and the retry,
    is unaffected;
  - an adaptation (Sec. 3.1 refinement, Sec. 4.3 split and merge):
    PIC_E_NOMEM marks the slot failed; every later call on it but the counter
    reads and pic_retire returns PIC_E_STATE, and the context's other slot
    goes on equal to a context that never failed;
  - a particle load: PIC_E_NOMEM leaves the slot as it was, and loading again
    gives the state of a load that never failed;
  - batched steps of three ionizing 1D discharges and of two avalanches:
    every slot stays at its last committed step, and each slot's retry ends
    bit-identical;
  - a 2D field solve after an adaptation: PIC_E_NOMEM, and solving again
    gives the same potential bit for bit."""
import numpy as np
import pytest
import torch

from paper_1604_07713_amd import binding as B
from paper_1604_07713_amd import inputs as I
from tests.test_gpu_contract import TIGHT_5000, TIGHT_8192, fast_ionizing, same_state

pytestmark = pytest.mark.gpu


class FailingAllocator:
    """torch's caching allocator behind pic_set_allocator, refusing the
    request numbered fail_at (counted from 1 over the allocator's life)."""

    def __init__(self, fail_at=None):
        self.requests = 0
        self.fail_at = fail_at
        dev = torch.cuda.current_device()

        def _alloc(nbytes, stream, user):
            self.requests += 1
            if self.requests == self.fail_at:
                return None
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0)
            except Exception:
                return None

        def _free(p, user):
            torch.cuda.caching_allocator_delete(p)
        self._alloc = B.ALLOC_FN(_alloc)
        self._free = B.FREE_FN(_free)
        self.struct = B.Allocator(self._alloc, self._free, None)


def avalanche(alloc, stream=None, npairs=5000):
    d = fast_ionizing(I.streamer_desc(precision=32, max_level=8))
    d["capacity"] = TIGHT_5000
    g = B.Context(d, allocator=alloc, stream=stream)
    for sp, (s, v, w, ids) in enumerate(I.streamer_particles(d, npairs=npairs)):
        g.load(0, sp, s, v, w, ids)
    g.field_solve_2d(0, rtol=1e-10)
    g.leapfrog_start(0)
    return g


def test_step_growth_failures_leave_the_last_committed_step():
    ra = FailingAllocator()
    ref = avalanche(ra)
    r0 = ra.requests
    st = ref.step(0, 96)
    sites = ra.requests - r0
    print("requests in the step call", sites, "room stops", st["room_stops"], flush=True)
    assert st["room_stops"] > 0 and sites >= 5
    other_ref = avalanche(FailingAllocator(), npairs=3000)
    other_ref.step(0, 40)
    stream = torch.cuda.Stream()
    for k in range(1, sites + 1):
        a = FailingAllocator(fail_at=r0 + k)
        g = avalanche(a, stream=stream.cuda_stream)
        assert a.requests == r0
        other = avalanche(FailingAllocator(), stream=stream.cuda_stream, npairs=3000)
        with pytest.raises(B.PicError) as e:
            g.step(0, 96)
        assert e.value.code == B.PIC_E_NOMEM, (k, e.value)
        done = g.step_index(0)
        assert 0 <= done < 96, (k, done)
        other.step(0, 40)   # the stream's other context, between the failure and the retry
        g.step(-1, 96 - done)
        same_state(ref, g, what=f"failure at request {k} of {sites}, stopped at step {done}")
        same_state(other_ref, other, what=f"other context, failure at request {k}")
        g.close()
        other.close()
    ref.close()
    other_ref.close()


def two_slots(alloc):
    d = I.streamer_desc(precision=32, max_level=8)
    descs = [dict(d, seed=11), dict(d, seed=12)]
    g = B.Context(descs, allocator=alloc)
    for j, dd in enumerate(descs):
        for sp, (s, v, w, ids) in enumerate(I.streamer_particles(dd, npairs=3000, rng_seed=[40 + j])):
            g.load(j, sp, s, v, w, ids)
        g.field_solve_2d(j, rtol=1e-10)
        g.leapfrog_start(j)
    g.step(0, 30, slots=[0, 1])
    return g


def test_adapt_failures_mark_the_slot_failed():
    ra = FailingAllocator()
    ref = two_slots(ra)
    r0 = ra.requests
    s = ref.adapt(0)
    sites = ra.requests - r0
    print("requests in the adaptation", sites, s, flush=True)
    assert sites >= 10 and s["refined"] + s["split_parents"] > 0
    ref.step(-1, 20, slots=[1])
    ks = sorted(set(np.linspace(1, sites, min(sites, 48)).round().astype(int).tolist()))
    for k in ks:
        a = FailingAllocator(fail_at=r0 + k)
        g = two_slots(a)
        assert a.requests == r0
        with pytest.raises(B.PicError) as e:
            g.adapt(0)
        assert e.value.code == B.PIC_E_NOMEM, (k, e.value)
        calls = (lambda: g.step(-1, 1, slots=[0]), lambda: g.read(0, 0), lambda: g.deposit(0),
                 lambda: g.deposit_read(0), lambda: g.adapt(0), lambda: g.field_solve_2d(0, rtol=1e-8),
                 lambda: g.leaves(0), lambda: g.field_table(0), lambda: g.leapfrog_start(0))
        for call in calls:
            with pytest.raises(B.PicError) as e:
                call()
            assert e.value.code == B.PIC_E_STATE, (k, e.value)
        assert g.count(0, 0) > 0 and g.step_index(0) == 30
        with pytest.raises(B.PicError) as e:   # a batched step over both refuses too
            g.step(-1, 1, slots=[0, 1])
        assert e.value.code == B.PIC_E_STATE
        g.step(-1, 20, slots=[1])
        for sp in range(2):
            np.testing.assert_array_equal(ref.read(1, sp)["id"], g.read(1, sp)["id"])
        same_state(ref, g, 1, 1, what=f"other slot, adaptation failed at request {k} of {sites}")
        g.retire(0)
        g.close()
    ref.close()


def test_load_failures_leave_the_slot_as_it_was():
    d = fast_ionizing(I.streamer_desc(precision=32, max_level=8))
    parts = I.streamer_particles(d, npairs=4000)
    ra = FailingAllocator()
    ref = B.Context(d, allocator=ra)
    r0 = ra.requests
    for sp, (s, v, w, ids) in enumerate(parts):
        ref.load(0, sp, s, v, w, ids)
    sites = ra.requests - r0
    print("requests in the loads", sites, flush=True)
    assert sites >= 3
    for k in range(1, sites + 1):
        a = FailingAllocator(fail_at=r0 + k)
        g = B.Context(d, allocator=a)
        failed = False
        for sp, (s, v, w, ids) in enumerate(parts):
            before = g.count(0, sp)
            try:
                g.load(0, sp, s, v, w, ids)
            except B.PicError as e:
                assert e.code == B.PIC_E_NOMEM, (k, e)
                assert g.count(0, sp) == before   # the slot as it was
                failed = True
                g.load(0, sp, s, v, w, ids)       # again, now granted
        assert failed, k
        same_state(ref, g, what=f"load failed at request {k} of {sites}")
        g.close()
    ref.close()


def ionizing_ensemble(alloc):
    descs = [dict(fast_ionizing(I.ccp_desc(ncells=128, ppc=64, precision=32, instance_key=k, voltage=450.0 + 50 * k)),
                  capacity=TIGHT_8192) for k in range(3)]
    g = B.Context(descs, allocator=alloc)
    for j, d in enumerate(descs):
        for sp, (s, v, w, ids) in enumerate(I.ccp_particles(d)):
            g.load(j, sp, s, v, w, ids)
        g.deposit(j)
        g.field_solve_1d(j, float(I.drive_voltage(d, 0)))
        g.leapfrog_start(j)
    vn = np.stack([I.drive_voltage(d, np.arange(1, 121)) for d in descs], axis=1)
    return g, vn


def test_batched_step_failures_leave_every_slot_at_its_last_committed_step():
    """Three ionizing discharges stepped by one persistent launch per step
    (launch tables, births staging and growth all take device memory): each
    refused request ends the call with every slot at its last committed
    step, and each slot's retry from there ends bit-identical to a run that
    never failed."""
    ra = FailingAllocator()
    ref, vn = ionizing_ensemble(ra)
    r0 = ra.requests
    st = ref.step(0, 120, vn, solve_field=True, sort_every=20, batched=4096)
    sites = ra.requests - r0
    print("requests in the batched step call", sites, "room stops", st["room_stops"], flush=True)
    assert st["room_stops"] > 0 and sites >= 5
    for k in range(1, sites + 1):
        a = FailingAllocator(fail_at=r0 + k)
        g, _ = ionizing_ensemble(a)
        assert a.requests == r0
        with pytest.raises(B.PicError) as e:
            g.step(0, 120, vn, solve_field=True, sort_every=20, batched=4096)
        assert e.value.code == B.PIC_E_NOMEM, (k, e.value)
        for j in range(3):
            done = g.step_index(j)
            assert 0 <= done <= 120, (k, j, done)
            if done < 120:
                g.step(-1, 120 - done, vn[done:, j:j + 1], solve_field=True, sort_every=20, batched=4096, slots=[j])
            same_state(ref, g, j, j, what=f"slot {j}, failure at request {k} of {sites}, stopped at step {done}")
        g.close()
    ref.close()


def adapted_avalanche(alloc):
    d = I.streamer_desc(precision=32, max_level=8)
    g = B.Context(d, allocator=alloc)
    for sp, (s, v, w, ids) in enumerate(I.streamer_particles(d, npairs=3000)):
        g.load(0, sp, s, v, w, ids)
    g.field_solve_2d(0, rtol=1e-10)
    g.leapfrog_start(0)
    g.step(0, 20)
    g.adapt(0)   # a new tree: the next solve builds its stencil anew
    return g


def test_field_solve_failures_leave_the_slot_usable():
    """The 2D solve's stencil and CG workspace (Sec. 3.1 finite volumes on
    the tree) are built after an adaptation: a refused request returns
    PIC_E_NOMEM, and the solve called again gives the same potential and
    field bit for bit, and the same steps after it."""
    ra = FailingAllocator()
    ref = adapted_avalanche(ra)
    r0 = ra.requests
    phi_ref = ref.field_solve_2d(0, rtol=1e-10)[0]
    sites = ra.requests - r0
    print("requests in the field solve", sites, flush=True)
    assert sites >= 5
    ref.step(-1, 10)
    for k in range(1, sites + 1):
        a = FailingAllocator(fail_at=r0 + k)
        g = adapted_avalanche(a)
        assert a.requests == r0
        with pytest.raises(B.PicError) as e:
            g.field_solve_2d(0, rtol=1e-10)
        assert e.value.code == B.PIC_E_NOMEM, (k, e.value)
        phi = g.field_solve_2d(0, rtol=1e-10)[0]
        assert np.array_equal(phi, phi_ref), k
        g.step(-1, 10)
        same_state(ref, g, what=f"field solve failed at request {k} of {sites}")
        g.close()
    ref.close()


def two_avalanches(alloc):
    d = fast_ionizing(I.streamer_desc(precision=32, max_level=8))
    descs = [dict(d, seed=21, capacity=TIGHT_5000), dict(d, seed=22, capacity=TIGHT_5000)]
    g = B.Context(descs, allocator=alloc)
    for j, dd in enumerate(descs):
        for sp, (s, v, w, ids) in enumerate(I.streamer_particles(dd, npairs=5000, rng_seed=[50 + j])):
            g.load(j, sp, s, v, w, ids)
        g.field_solve_2d(j, rtol=1e-10)
        g.leapfrog_start(j)
    return g


def test_batched_2d_step_failures_leave_every_slot_at_its_last_committed_step():
    """Two growing avalanches stepped by one persistent launch per step: each
    refused request ends the call with both slots at their last committed
    steps, and each slot's retry ends bit-identical."""
    ra = FailingAllocator()
    ref = two_avalanches(ra)
    r0 = ra.requests
    st = ref.step(-1, 96, slots=[0, 1], batched=2048, grid=2048)
    sites = ra.requests - r0
    print("requests in the batched 2D step call", sites, "room stops", st["room_stops"], flush=True)
    assert st["room_stops"] > 0 and sites >= 5
    for k in range(1, sites + 1):
        a = FailingAllocator(fail_at=r0 + k)
        g = two_avalanches(a)
        assert a.requests == r0
        with pytest.raises(B.PicError) as e:
            g.step(-1, 96, slots=[0, 1], batched=2048, grid=2048)
        assert e.value.code == B.PIC_E_NOMEM, (k, e.value)
        for j in range(2):
            done = g.step_index(j)
            assert 0 <= done <= 96, (k, j, done)
            if done < 96:
                g.step(-1, 96 - done, slots=[j], batched=2048, grid=2048)
            same_state(ref, g, j, j, what=f"slot {j}, failure at request {k} of {sites}, stopped at step {done}")
        g.close()
    ref.close()
