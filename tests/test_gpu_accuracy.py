"""Error of the FP32 particle path against the FP64 oracle, stated per
result (positions and velocities in FP32, deposits in 64-bit fixed point,
field solves and time bookkeeping in FP64).

  - the quadtree workload (collisionless, fixed field: not chaotic): the
    pointwise relative error of positions and velocities after 100 steps,
    on particles sampled by id, and the share whose leaf differs;
  - the 1D discharge (collisions, births and the self-consistent field:
    chaotic): the divergence horizon (first step whose discrete results
    differ), then counts, mean energies and the density profile after five
    RF periods (2000 steps) against the spread between independent seeds of
    the FP64 oracle (the sampling error of those results).

Each test prints a JSON line with its figures (collected into the accuracy
summary of the measurements)."""
import json

import numpy as np
import pytest

import oracle
from paper_1604_07713_amd import binding as B
from paper_1604_07713_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_quadtree_fp32_pointwise_error():
    d32 = I.quadtree_static_desc(precision=32)
    d64 = I.quadtree_static_desc(precision=64)
    n = 4194304
    s, v, w, ids = I.quadtree_particles(n)
    g = B.Context(d32)
    g.load(0, 0, s, v, w, ids)
    keys, lv = g.leaves(0)
    cx, cy = I.leaf_corners(keys, lv)
    phi = I.quadtree_phi(cx, cy)
    g.field_set(0, B.CORNER_PHI_2D, phi)
    g.sort(0)
    g.leapfrog_start(0)
    g.step(0, 100, sort_every=50)
    sample = np.sort(np.random.Generator(np.random.PCG64(12)).choice(n, 20000, replace=False)).astype(np.uint32)
    o = oracle.Oracle(d64)
    o.load(0, s[sample], v[sample], w[sample], ids[sample])
    o.field_set(oracle.CORNER_PHI_2D, phi)
    o.leapfrog_start()
    o.step(0, 100)
    ro = o.read(0)
    rg = g.read(0, 0)
    keep = np.isin(ro["id"], rg["id"])
    idx = np.searchsorted(rg["id"], ro["id"][keep])
    # position error in units of the domain side; velocity error relative to
    # the particle's speed (a component near zero has no useful relative error)
    ds = np.max(np.abs(ro["s"][keep] - rg["s"][idx]), axis=1)
    dv = np.linalg.norm(ro["v"][keep] - rg["v"][idx], axis=1) / np.linalg.norm(ro["v"][keep], axis=1)
    out = dict(s_abs=dict(max=float(ds.max()), median=float(np.median(ds)), p99=float(np.percentile(ds, 99))),
               v_rel=dict(max=float(dv.max()), median=float(np.median(dv)), p99=float(np.percentile(dv, 99))))
    out["leaf_differs"] = float(np.mean(ro["cell"][keep] != rg["cell"][idx]))
    out["absorbed_or_lost_differ"] = int(np.count_nonzero(~keep))
    print(json.dumps({"accuracy": "quadtree_4M_100_steps_fp32_vs_fp64", **out}), flush=True)
    assert out["s_abs"]["max"] < 1e-5 and out["v_rel"]["p99"] < 1e-5 and out["v_rel"]["max"] < 1e-3
    assert out["leaf_differs"] < 1e-3


def ccp_oracle(precision, seed, nsteps, per_step=False):
    d = I.ccp_desc(precision=precision, seed=seed)
    o = oracle.Oracle(d)
    for sp, (s, v, w, ids) in enumerate(I.ccp_particles(d)):
        o.load(sp, s, v, w, ids)
    o.deposit()
    o.field_solve_1d(float(I.drive_voltage(d, 0)))
    o.leapfrog_start()
    vn = I.drive_voltage(d, np.arange(1, nsteps + 1))
    if not per_step:
        return d, o, o.step(0, nsteps, vn, True)
    return d, o, [o.step(k, 1, vn[k:k + 1], True) for k in range(nsteps)]


def moments(read_e, read_i, d, bins=16):
    me, mi = d["species"][0]["mass"], d["species"][1]["mass"]
    ee = 0.5 * me * np.sum(read_e["v"] ** 2, axis=1) / I.E_CHARGE
    ei = 0.5 * mi * np.sum(read_i["v"] ** 2, axis=1) / I.E_CHARGE
    he = np.histogram(read_e["s"][:, 0], bins=bins, range=(0, 1))[0].astype(float)
    hi = np.histogram(read_i["s"][:, 0], bins=bins, range=(0, 1))[0].astype(float)
    return dict(ne=len(ee), ni=len(ei), mean_e_ev=float(ee.mean()), mean_i_ev=float(ei.mean()), he=he, hi=hi)


def test_ccp_fp32_divergence_horizon_and_statistics():
    nsteps = 2000
    # FP32 on the GPU, one step per call: the per-step discrete results
    d = I.ccp_desc(precision=32, seed=1)
    g = B.Context(d)
    for sp, (s, v, w, ids) in enumerate(I.ccp_particles(d)):
        g.load(0, sp, s, v, w, ids)
    g.deposit(0)
    g.field_solve_1d(0, float(I.drive_voltage(d, 0)))
    g.leapfrog_start(0)
    vn = I.drive_voltage(d, np.arange(1, nsteps + 1))
    sg = [g.step(k, 1, vn[k:k + 1], solve_field=True) for k in range(nsteps)]
    _, o64, so = ccp_oracle(64, 1, nsteps, per_step=True)
    keys = ("alive_start", "absorbed", "elastic", "ionization", "cx", "births")
    horizon = next((k for k in range(nsteps) if any(so[k][x] != sg[k][x] for x in keys)), nsteps)
    m32 = moments(g.read(0, 0), g.read(0, 1), d)
    m64 = moments(o64.read(0), o64.read(1), d)
    # the sampling error of each result: its spread over independent seeds of the FP64 oracle
    seeds = [moments(*(lambda o: (o.read(0), o.read(1)))(ccp_oracle(64, sd, nsteps)[1]), d) for sd in (11, 12, 13, 14)]
    out = dict(divergence_horizon_step=int(horizon))
    worst = 0.0
    for k in ("ne", "ni", "mean_e_ev", "mean_i_ev"):
        spread = float(np.std([m[k] for m in seeds], ddof=1))
        z = abs(m32[k] - m64[k]) / max(spread, 1e-30)
        out[k] = dict(fp32=m32[k], fp64=m64[k], seed_spread=spread, z=z)
        worst = max(worst, z)
    for k in ("he", "hi"):
        spread = np.std([m[k] for m in seeds], axis=0, ddof=1)
        chi2 = float(np.sum((m32[k] - m64[k]) ** 2 / np.maximum(2 * spread ** 2, 1.0)) / len(spread))
        out[k + "_chi2_per_bin"] = chi2
    print(json.dumps({"accuracy": "ccp_2000_steps_fp32_vs_fp64", **out}), flush=True)
    assert horizon > 0
    # within sampling error: every scalar within 4 seed spreads, profiles within chi^2/bin 4
    assert worst < 4.0, out
    assert out["he_chi2_per_bin"] < 4.0 and out["hi_chi2_per_bin"] < 4.0, out
