"""Host logic of the serving loop (no GPU): the memory projection that
admission uses, and the growth estimate it is built on."""
import math

from paper_1604_07713_amd import serve


def streamer(npairs=10000, steps=2000):
    return serve.Job(dict(kind="streamer", arrival=0.0, key=1, side=0.01, npairs=npairs, steps=steps))


def ccp(ncells=200, ppc=16, steps=500):
    return serve.Job(dict(kind="ccp", arrival=0.0, key=2, ncells=ncells, ppc=ppc, voltage=300.0, pressure=40.0,
                          steps=steps))


def test_streamer_projection_follows_exponential_growth():
    j = streamer()
    lam = 0.004
    # population now x exp(lam x steps left), two slots per particle of 112 B (FP32)
    peak = j.nparticles * math.exp(lam * j.steps_total)
    expect = 112 * (2 * peak + 8192) + max(1024.0, peak / 16) * 400 + 4 * (1 << 18)
    assert abs(j.projected_bytes(lam) - expect) <= 1e-9 * expect
    # halfway, with the population observed: only the steps left count
    j.steps_done, j.n_now = 1000, 2_000_000
    peak2 = 2_000_000 * math.exp(lam * 1000)
    assert j.projected_bytes(lam) < 112 * (2 * peak2 + 8192) + peak2 / 16 * 400 + 4 * (1 << 18) + 1
    assert j.projected_bytes(lam) > 112 * 2 * peak2
    # no growth assumed: the footprint of the population now
    assert j.projected_bytes(0.0) < j.projected_bytes(lam)


def test_growth_rate_is_the_mean_log_rate():
    j = streamer()
    assert j.growth_rate() is None           # too early to tell
    j.steps_done, j.n_now = 200, j.nparticles * 8
    assert abs(j.growth_rate() - math.log(8) / 200) < 1e-15


def test_ccp_projection_and_precision():
    a = ccp()
    b = serve.Job(dict(a.spec), precision=64)
    assert a.projected_bytes() < b.projected_bytes()   # FP64 particles take more room
    # a discharge grows by at most the assumed factor over its start
    a.n_now = 10 * a.nparticles
    assert a.projected_bytes() > ccp().projected_bytes()
