"""Served request stream: a job's result is the same when it runs alone and
when it shares the GPU with jobs arriving before and after it (continuous
batching: one persistent launch steps every resident 1D job)."""
import numpy as np
import pytest

from paper_1604_07713_amd import serve
from tests.gpu_common import assert_same_particles

pytestmark = pytest.mark.gpu


def ccp(key, arrival, steps, ncells=200, ppc=16):
    return serve.Job(dict(kind="ccp", arrival=arrival, key=key, ncells=ncells, ppc=ppc, voltage=300.0 + key,
                          pressure=40.0 + key, steps=steps))


def streamer(key, arrival, steps):
    return serve.Job(dict(kind="streamer", arrival=arrival, key=key, side=0.004, npairs=800, steps=steps))


def run(jobs, tick_steps=10, lanes=4):
    srv = serve.Server(budget_bytes=8 << 30, tick_steps=tick_steps, keep_results=True, lanes=lanes)
    m = srv.run(jobs, clock="tick")
    res = {j.key: j for j in srv.done}
    srv.close()
    return m, res


@pytest.mark.parametrize("lanes", [1, 4])
def test_job_alone_equals_in_mix(lanes):
    """Avalanches arriving at different ticks (so at different points of
    their adapt / field cycle) share batched 2D launches (all in one lane,
    or spread over four concurrent lanes), beside the 1D jobs' batched
    launches; each job ends as it does alone."""
    _, alone = run([ccp(1, 0, 37)])
    _, alone_s = run([streamer(7, 0, 30)])
    _, alone_t = run([streamer(8, 0, 44)])
    mix = [ccp(3, 0, 55, ncells=300), ccp(1, 1, 37), ccp(4, 2, 23, ppc=8), streamer(7, 1, 30), ccp(5, 3, 61),
           streamer(9, 0, 50), streamer(8, 2, 44)]
    m, res = run(mix, tick_steps=7, lanes=lanes)
    assert m["jobs_done"] == len(mix)
    _, alone1 = run([ccp(1, 0, 37)], tick_steps=7)
    for key, ref in ((1, alone1[1]), (7, alone_s[7]), (8, alone_t[8])):
        for sp in range(2):
            assert_same_particles(ref.result[sp], res[key].result[sp], 0, f"job {key} species {sp}")
    for sp in range(2):
        assert_same_particles(alone[1].result[sp], alone1[1].result[sp], 0, f"job 1 ticks of 10 vs 7, species {sp}")


def test_admission_respects_budget():
    # a budget that fits one job at a time serialises the jobs
    jobs = [ccp(k, 0, 12) for k in range(3)]
    one = jobs[0].projected_bytes()
    srv = serve.Server(budget_bytes=int(one * 1.5), tick_steps=6)
    peak = 0
    orig = srv._admit

    def admit():
        orig()
        nonlocal peak
        peak = max(peak, len(srv.running))
    srv._admit = admit
    m = srv.run(jobs, clock="tick")
    srv.close()
    assert m["jobs_done"] == 3 and peak == 1
