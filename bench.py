"""Throughput benchmark of the ES-PIC particle loop on one MI355X.

Default workload: the 2D static quadtree (unit square, level 6 base refined
to level 9 inside a centred disk of radius 0.15: 23,620 leaves), 4,194,304
electrons (uniform positions, 1 eV Maxwellian), FP32 particles, static
potential phi = x^2 + 0.3 sin(2 pi y) given at the nodes, reflecting walls.
One step = gather + leapfrog push + walls + locate + deposit for every
particle (no collisions in this workload), plus the periodic re-sort of the
particles by leaf.  Inputs are synthetic and seeded; they are resident in
HBM before the timed region starts.

Beside it (same line, own keys): the same quadtree at 16,777,216 electrons
(state beyond the Infinity Cache), the batched-vs-plain comparisons the
metric names -- 96 uneven 1D discharges and 32 uneven 2D avalanches on
dynamic quadtrees, each stepped by one persistent launch per step over all
instances and by per-instance launches (FP32 and FP64) -- the 2D
avalanche breakdown run, the 3D octree counterpart of the quadtree
workload (4,194,304 electrons, 46,488 leaves), and the 1D discharge at
w_p dt = 2.08 stepped by the direct implicit scheme.

Prints ONE JSON line (metric/value/unit/... plus "roofline" for the
dominant kernel and "cpu_baseline" for the oracle on a bounded sample).

Usage: python bench.py [--gpus 1] [--steps 100] [--warmup 10]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                 # MI355X HBM3E, GB/s
# Algorithmic bytes per particle-update (what the step must move; the field,
# leaf and charge tables are cache resident and not counted):
#  2D FP32 without collisions: read sx, sy, vx, vy, leaf (20 B) and the
#  per-particle weight this layout carries (4 B), write sx, sy, vx, vy, leaf
#  (20 B; the leaf is counted although it is stored only when it changes)
#  -> 44 B.
BYTES_PER_UPDATE_2D = 44
#  1D FP32 with MCC: read s, vx, w, id (16 B), write s, vx (8 B); a particle
#  that collides also moves vy, vz in and out (16 B per collision).
BYTES_PER_UPDATE_1D_MCC = 24
BYTES_PER_COLLISION_1D = 16
#  2D FP32 with MCC (avalanche): read s (8), v (12), leaf, id, w (12); write
#  s, v, leaf (24) -> 56 B.
BYTES_PER_UPDATE_2D_MCC = 56
#  3D FP32 without collisions: read sx, sy, sz, vx, vy, vz, leaf, w (32 B),
#  write sx, sy, sz, vx, vy, vz, leaf (28 B) -> 60 B.
BYTES_PER_UPDATE_3D = 60
#  1D direct implicit step: the predictor reads s, v_x, b, w and writes s,
#  v_x; the corrector reads s, v_x, b, w, id and writes s, v_x, b -> 56 B
#  (FP32), 100 B (FP64).
BYTES_PER_UPDATE_DIPIC = {32: 56, 64: 100}
METRIC = "particle-updates/s (locate+gather+push+MCC+deposit), 2D AMR; batched vs plain"
PROFILE_PMC = os.path.join(ROOT, "profiles", "pmc_traffic.json")


T_START = time.perf_counter()


def note(stage):
    """A progress line on stderr as each stage of the run ends."""
    print(f"[bench] {stage} done at {time.perf_counter() - T_START:.1f} s", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("k_step.hip", "device_util.hpp", "pic_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1604_07713_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel, workload):
    """Calibrated HBM bytes per launch of 'kernel' on 'workload' from the
    committed rocprofv3 PMC summary, if it was taken on the current kernel
    source; else None."""
    try:
        with open(PROFILE_PMC) as f:
            p = json.load(f)
    except (OSError, ValueError):
        return None
    if p.get("kernel_source_hash") != kernel_source_hash():
        return None
    e = p.get("kernels", {}).get(f"{kernel} | {workload}")
    return None if e is None else e.get("hbm_bytes_per_launch")


def roofline(bytes_per_launch, launch_ms, traffic=None):
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic}


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count()
    return model, avail


def streamer_bench(nsteps=2000, npairs=10000, field_every=10, max_wall=120.0):
    """2D streamer breakdown on the dynamic quadtree (1 cm square, levels
    5-11, 30 kV/cm, Gaussian seed of 1e4 pairs, FP32 particles): every 10
    steps the tree is adapted (refine / coarsen with particle split / merge)
    and the FP64 CG field solve is redone.  Reports the particle-loop rate
    (collisions and births included), its kernel's roofline, and the
    whole-run rate with adaptation and field solves."""
    import numpy as np
    import torch
    from paper_1604_07713_amd import binding as B
    from paper_1604_07713_amd import inputs as I
    d = I.streamer_desc(side=0.01, precision=32)
    g = B.Context(d)
    for sp, (s, v, w, ids) in enumerate(I.streamer_particles(d, npairs=npairs)):
        g.load(0, sp, s, v, w, ids)
    g.adapt(0)
    g.field_solve_2d(0, rtol=1e-8, maxit=4000)
    g.leapfrog_start(0)
    t = dict(step=0.0, adapt=0.0, solve=0.0)
    upd = births = cg = 0
    kern_ms = 0.0
    launches = 0
    step = 0
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    while step < nsteps and time.perf_counter() - t_start < max_wall:
        t0 = time.perf_counter()
        st = g.step(-1, field_every, sort_every=0, timing=1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.adapt(0)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        _, it, _, _ = g.field_solve_2d(0, rtol=1e-8, maxit=4000)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        t["step"] += t1 - t0
        t["adapt"] += t2 - t1
        t["solve"] += t3 - t2
        upd += int(st["alive_start"][0] + st["alive_start"][1])
        births += int(st["births"])
        kern_ms += st["loop_ms"]
        launches += st["loop_launches"]
        cg += it
        step += field_every
    wall = time.perf_counter() - t_start
    keys, _ = g.leaves(0)
    out = dict(steps=step, particles_end=int(g.count(0, 0) + g.count(0, 1)), leaves_end=int(len(keys)),
               births=births, particle_loop_updates_per_s=upd / max(t["step"], 1e-12),
               updates_per_s_with_adapt_and_field=upd / wall, particle_loop_s=t["step"], adapt_s=t["adapt"],
               field_solve_s=t["solve"], cg_iterations=cg, wall_s=wall,
               loop_kernel_s=kern_ms * 1e-3,
               workload="1 cm x 1 cm, N2-like gas at 1 atm, 30 kV/cm, 1e4 seed pairs (sigma 0.5 mm), "
                        "levels 5-11, 16-64 particles per leaf, dt 1e-13 s, adapt + FP64 CG every 10 steps")
    # the particle-loop launches (step kernel and births kernels) over the
    # run: 56 B per particle-update, summed over launches
    out["roofline"] = roofline(BYTES_PER_UPDATE_2D_MCC * upd / max(launches, 1), kern_ms / max(launches, 1))
    out["roofline"]["per"] = "mean particle-loop launch (step + births kernels), 56 B per particle-update"
    g.close()
    return out


def _ccp_oracle_run(args):
    """One 1D CCP instance on the FP64 oracle (run in a worker process)."""
    desc, nsteps = args
    import numpy as np
    import oracle
    from paper_1604_07713_amd import inputs as I
    o = oracle.Oracle(desc)
    parts = I.ensemble_particles(desc) if desc.get("from_ensemble") else I.ccp_particles(desc)
    for sp, (s, v, w, ids) in enumerate(parts):
        o.load(sp, s, v, w, ids)
    o.deposit()
    o.field_solve_1d(float(I.drive_voltage(desc, 0)))
    o.leapfrog_start()
    vn = I.drive_voltage(desc, np.arange(1, nsteps + 1))
    t0 = time.perf_counter()
    st = o.step(0, nsteps, vn, True)
    return st["alive_start"][0] + st["alive_start"][1], time.perf_counter() - t0


def cpu_baseline(nparticles, nsteps, seed=2, extra=True):
    """The oracle timed on this host: the quadtree workload on a bounded
    sample (single thread), plus the 1D discharge in full (single thread) and
    8 instances of the ensemble for a bounded number of steps, one process
    per instance."""
    import numpy as np
    import oracle
    from paper_1604_07713_amd import inputs as I
    model, avail = cpu_info()
    d = I.quadtree_static_desc()
    o = oracle.Oracle(d)
    s, v, w, ids = I.quadtree_particles(nparticles, seed=seed)
    o.load(0, s, v, w, ids)
    keys, lv = o.leaves()
    cx, cy = I.leaf_corners(keys, lv)
    o.field_set(oracle.CORNER_PHI_2D, I.quadtree_phi(cx, cy))
    o.leapfrog_start()
    t0 = time.perf_counter()
    st = o.step(0, nsteps)
    dt = time.perf_counter() - t0
    upd = st["alive_start"][0]
    out = dict(value=upd / dt, unit="particle-updates/s", cores=1, kind="oracle",
               sample=f"{nparticles} particles x {nsteps} steps of the same workload, single-threaded "
                      f"FP32-mirror oracle, {dt:.1f} s",
               cpu_model=model, host_threads=avail)
    if not extra:
        return out
    # the octree workload on all its particles for a few steps
    d3 = I.octree_static_desc()
    o3 = oracle.Oracle(d3)
    s3, v3, w3, ids3 = I.octree_particles(nparticles)
    o3.load(0, s3, v3, w3, ids3)
    k3, l3 = o3.leaves()
    x3, y3, z3 = I.leaf_corners3(k3, l3)
    o3.field_set(oracle.CORNER_PHI_3D, I.octree_phi(x3, y3, z3))
    o3.leapfrog_start()
    steps3 = 8
    t0 = time.perf_counter()
    st3 = o3.step(0, steps3)
    t3 = time.perf_counter() - t0
    del o3
    out["octree_sample"] = dict(updates_per_s=st3["alive_start"][0] / t3, cores=1,
                                sample=f"{nparticles} particles x {steps3} steps of the octree workload, "
                                       f"single-threaded FP32-mirror oracle, {t3:.1f} s")
    # the streamer's first 200 of its 2000 steps (adapt and CG every 10)
    ds = I.streamer_desc(side=0.01, precision=32)
    os_ = oracle.Oracle(ds)
    for sp, (s_, v_, w_, i_) in enumerate(I.streamer_particles(ds, npairs=10000)):
        os_.load(sp, s_, v_, w_, i_)
    os_.adapt()
    os_.field_solve_2d(rtol=1e-8, maxit=4000)
    os_.leapfrog_start()
    t_loop = t_all = 0.0
    upd_s = 0
    for k in range(0, 200, 10):
        t0 = time.perf_counter()
        st_s = os_.step(k, 10)
        t1 = time.perf_counter()
        os_.adapt()
        os_.field_solve_2d(rtol=1e-8, maxit=4000)
        t_loop += t1 - t0
        t_all += time.perf_counter() - t0
        upd_s += st_s["alive_start"][0] + st_s["alive_start"][1]
    out["streamer_sample"] = dict(particle_loop_updates_per_s=upd_s / t_loop, updates_per_s_with_adapt_and_field=upd_s / t_all,
                                  cores=1, sample=f"the 2D streamer's first 200 of its 2000 steps (2e4 -> {os_.count(0) + os_.count(1)} "
                                                  f"particles; the full run reaches 3e7), FP32-mirror oracle, {t_all:.1f} s")
    del os_
    # 1D discharge in full: 16,384 particles, 400 steps, FP64
    u, t = _ccp_oracle_run((I.ccp_desc(precision=64), 400))
    out["ccp_full"] = dict(updates_per_s=u / t, cores=1, sample=f"the whole 1D discharge run, 400 steps, FP64, {t:.2f} s")
    # the direct implicit discharge in full: 16,384 particles, 400 steps, FP64
    u, t = _ccp_oracle_run((I.dipic_ccp_desc(precision=64), 400))
    out["dipic_full"] = dict(updates_per_s=u / t, cores=1,
                             sample=f"the whole direct implicit 1D discharge, 400 steps, FP64, {t:.2f} s")
    # ensemble: 8 of the 96 instances, one process each, a bounded number of steps
    from concurrent.futures import ProcessPoolExecutor
    descs = I.ensemble_descs(count=96, precision=64)
    pick = [descs[k] for k in np.linspace(0, 95, 8).astype(int)]
    for d8 in pick:
        d8["from_ensemble"] = True
    steps8 = 100
    workers = max(1, min(8, avail))
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(_ccp_oracle_run, [(d8, steps8) for d8 in pick]))
    wall = time.perf_counter() - t0
    # instances are independent: the aggregate rate is the sum of the
    # processes' own stepping rates (each timed around its step loop)
    rate8 = sum(r[0] / r[1] for r in res)
    out["ensemble_sample"] = dict(updates_per_s=rate8, cores=workers,
                                  sample=f"8 of the 96 instances (evenly spaced), {steps8} of 2000 steps each, "
                                         f"FP64, one process per instance, {wall:.1f} s wall; the full ensemble "
                                         f"(about 2e11 updates with its growth) would take hours at this rate")
    return out


def ensemble_bench(nsteps, ninst=96, tune=True,
                   modes=("batched", "plain_fp32", "plain", "batched_energy_conserving"), shape=None, sort_every=50):
    """Batched ensemble of 1D CCP instances (the 1D discharge's physics, 96
    uneven meshes), with the on-device field solve: the FP32 batched path
    (one persistent launch per step, autotuned work items; the same steps
    replayed from captured HIP graphs are timed beside it), the
    same FP32 arithmetic with per-instance launches (plain_fp32: the
    batching gain alone), the FP64 plain path (per-instance launches; its
    ratio to plain_fp32 is the precision gain alone), and the batched path
    again with the energy-conserving coupling (cell E, no interpolation)."""
    import numpy as np
    import torch
    from paper_1604_07713_amd import autotune
    from paper_1604_07713_amd import binding as B
    from paper_1604_07713_amd import inputs as I
    out = {}
    tuned_batched = None
    precs = {"batched": 32, "plain_fp32": 32, "plain": 64, "batched_energy_conserving": 32}
    for mode in modes:
        prec = precs[mode]
        batched = mode.startswith("batched")
        descs = I.ensemble_descs(count=ninst, precision=prec)
        if mode == "batched_energy_conserving":
            for d in descs:
                d["field_scheme"] = I.FIELD_CIC_EC
        vtab = np.stack([I.drive_voltage(d, np.arange(1, 4000)) for d in descs], axis=1)

        def make():
            g = B.Context(descs)
            for j, d in enumerate(descs):
                for sp, (s, v, w, ids) in enumerate(I.ensemble_particles(d)):
                    g.load(j, sp, s, v, w, ids)
                g.deposit(j)
                g.field_solve_1d(j, float(I.drive_voltage(d, 0)))
                g.leapfrog_start(j)
            return g
        g = make()
        kw = dict(solve_field=True, sort_every=sort_every)
        tuned = None
        if batched:
            if shape:
                tuned = dict(tile=shape[0], grid=shape[1])
            elif tuned_batched:
                tuned = tuned_batched   # same ensemble, same launch shape
            else:
                tuned = autotune.tune(make, descs, vtab) if tune else dict(tile=4096, grid=2048)
            tuned_batched = tuned
            kw.update(batched=tuned["tile"], grid=tuned["grid"])
        g.step(0, 10, vtab[:10], **kw)          # warm-up
        st = g.step(10, nsteps, vtab[10:10 + nsteps], timing=1, **kw)
        kern = st["loop_ms"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st2 = g.step(10 + nsteps, nsteps, vtab[10 + nsteps:10 + 2 * nsteps], **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        graph_rate = None
        if batched:
            # the same steps replayed from a captured HIP graph of 25 steps
            k0 = 10 + 2 * nsteps
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st3 = g.step(k0, nsteps, vtab[k0:k0 + nsteps], graph_steps=25, **kw)
            torch.cuda.synchronize()
            graph_rate = (st3["alive_start"][0] + st3["alive_start"][1]) / (time.perf_counter() - t1)
        upd = st2["alive_start"][0] + st2["alive_start"][1]
        upd_t = st["alive_start"][0] + st["alive_start"][1]
        coll_t = st["elastic"] + st["ionization"] + st["cx"]
        out[mode] = dict(precision=f"fp{prec}", updates_per_s=upd / dt, ms_per_step=dt * 1e3 / nsteps,
                         births_per_step=st2["births"] / nsteps, room_stops=st["room_stops"] + st2["room_stops"],
                         loop_kernel_ms_per_step=kern / nsteps, particles=upd // nsteps,
                         launch=("one persistent launch per step" if batched else "per-instance launches"))
        if graph_rate is not None:
            out[mode]["graph_replay_updates_per_s"] = graph_rate
        if batched and prec == 32:
            # the particle loop of a step (the persistent step launch and the
            # births kernels after it, timed together): 24 B per update + 16 B
            # per collision
            per = (BYTES_PER_UPDATE_1D_MCC * upd_t + BYTES_PER_COLLISION_1D * coll_t) / nsteps
            out[mode]["roofline"] = roofline(per, kern / nsteps)
            out[mode]["roofline"]["per"] = ("batched particle loop of a step (k_step1d_batched<float,true> + births kernels), "
                                            "24 B per update + 16 B per collision")
        if tuned:
            out[mode]["tile"] = tuned["tile"]
            out[mode]["grid"] = tuned["grid"]
        g.close()
        note(f"ensemble {mode}")
    if "batched" in out and "plain" in out:
        out["batched_over_plain"] = out["batched"]["updates_per_s"] / out["plain"]["updates_per_s"]
    if "batched" in out and "plain_fp32" in out:
        out["batched_over_plain_fp32"] = out["batched"]["updates_per_s"] / out["plain_fp32"]["updates_per_s"]
    if "plain_fp32" in out and "plain" in out:
        out["plain_fp32_over_plain_fp64"] = out["plain_fp32"]["updates_per_s"] / out["plain"]["updates_per_s"]
    return out


TILES_2D = (512, 1024, 2048, 4096)
GRIDS_2D = (256, 512, 1024, 2048)


def avalanche_bench(nsteps=200, ninst=32, field_every=10, tune=True, shape=None,
                    modes=("batched", "plain_fp32", "plain")):
    """Batched ensemble of 2D avalanches on dynamic quadtrees, shaped like
    the served stream's 2D jobs (32 instances, sides 0.25-1 cm, 1e3-1e4
    seed pairs, levels 5-11, 30 kV/cm).  Every field_every steps each slot
    adapts its tree (split / merge) and re-solves its field with the FP64 CG
    (per-slot calls, the same in every mode); the particle-loop calls in
    between (locate, gather, push, MCC with births, deposit) are timed: one
    persistent launch per step over all slots (batched, FP32), per-slot
    launches of the same FP32 kernels (plain_fp32: the batching gain alone),
    and per-slot FP64 launches (plain: the paper's method at the oracle's
    precision)."""
    import torch
    from paper_1604_07713_amd import autotune
    from paper_1604_07713_amd import binding as B
    from paper_1604_07713_amd import inputs as I
    out = {}
    tuned = None
    for mode in modes:
        prec = 64 if mode == "plain" else 32
        ens = I.avalanche_ensemble(count=ninst, precision=prec)
        descs = [d for d, _ in ens]

        def make():
            g = B.Context(descs)
            for j, (d, parts) in enumerate(ens):
                for sp, (s, v, w, ids) in enumerate(parts):
                    g.load(j, sp, s, v, w, ids)
                g.adapt(j)
                g.field_solve_2d(j, rtol=1e-8, maxit=4000)
                g.leapfrog_start(j)
            return g
        kw = {}
        if mode == "batched":
            if shape:
                tuned = dict(tile=shape[0], grid=shape[1])
            elif tune:
                npart = sum(len(p[0][0]) * 2 for _, p in ens)
                tuned = autotune.tune(make, descs, None, tiles=TILES_2D, grids=GRIDS_2D, nparticles=npart)
            else:
                tuned = dict(tile=1024, grid=1024)
            kw = dict(batched=tuned["tile"], grid=tuned["grid"])
        g = make()
        t_loop = t_field = 0.0
        upd = births = 0
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(0, nsteps, field_every):
            t0 = time.perf_counter()
            st = g.step(-1, field_every, **kw)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for j in range(ninst):
                g.adapt(j)
                g.field_solve_2d(j, rtol=1e-8, maxit=4000)
            torch.cuda.synchronize()
            t_loop += t1 - t0
            t_field += time.perf_counter() - t1
            upd += int(st["alive_start"][0] + st["alive_start"][1])
            births += int(st["births"])
        wall = time.perf_counter() - t_start
        r = dict(precision=f"fp{prec}", particle_loop_updates_per_s=upd / t_loop,
                 updates_per_s_with_adapt_and_field=upd / wall, particle_loop_ms_per_step=t_loop * 1e3 / nsteps,
                 adapt_and_field_s=t_field, births=births,
                 particles_end=int(sum(g.count(j, 0) + g.count(j, 1) for j in range(ninst))),
                 launch=("one persistent launch per step over all slots" if mode == "batched"
                         else "per-slot launches"))
        if mode == "batched":
            r.update(tile=tuned["tile"], grid=tuned["grid"])
            # one more chunk with events around every step's particle-loop
            # launches (the batched step kernel and the births kernels)
            st = g.step(-1, field_every, timing=1, **kw)
            n_upd = int(st["alive_start"][0] + st["alive_start"][1])
            r["roofline"] = roofline(BYTES_PER_UPDATE_2D_MCC * n_upd / field_every, st["loop_ms"] / field_every)
            r["roofline"]["per"] = "batched particle-loop launch (k_step2d_batched + births), 56 B per particle-update"
        out[mode] = r
        g.close()
        note(f"avalanche ensemble {mode}")
    rate = {m: out[m]["particle_loop_updates_per_s"] for m in out}
    if "batched" in rate and "plain_fp32" in rate:
        out["batched_over_plain_fp32"] = rate["batched"] / rate["plain_fp32"]
    if "batched" in rate and "plain" in rate:
        out["batched_over_plain"] = rate["batched"] / rate["plain"]
    if "plain_fp32" in rate and "plain" in rate:
        out["plain_fp32_over_plain_fp64"] = rate["plain_fp32"] / rate["plain"]
    out["workload"] = (f"{ninst} avalanches (sides 0.25-1 cm, 1e3-1e4 seed pairs, N2-like gas at 1 atm, "
                       f"30 kV/cm, levels 5-11), {nsteps} steps, adapt + FP64 CG every {field_every} steps")
    return out


def quadtree_bench(n, steps, warmup, sort_every, timing_every):
    """The static quadtree workload with n electrons: whole step loop rate
    (timed steps include floor(steps / sort_every) sorts) and the mean
    duration of the step kernel from HIP events on the library's stream."""
    import torch
    from paper_1604_07713_amd import binding as B
    from paper_1604_07713_amd import inputs as I
    d = I.quadtree_static_desc()
    g = B.Context(d)
    s, v, w, ids = I.quadtree_particles(n)
    g.load(0, 0, s, v, w, ids)
    keys, lv = g.leaves(0)
    cx, cy = I.leaf_corners(keys, lv)
    g.field_set(0, B.CORNER_PHI_2D, I.quadtree_phi(cx, cy))
    g.sort(0)
    g.leapfrog_start(0)
    if warmup:
        g.step(0, warmup, sort_every=sort_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = g.step(warmup, steps, sort_every=sort_every, timing=timing_every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g.close()
    updates = st["alive_start"][0]
    kern_ms = st["loop_ms"] / max(st["loop_launches"], 1)
    return dict(updates=updates, seconds=dt, kernel_ms=kern_ms, leaves=int(len(keys)))


def octree_bench(n, steps, warmup, sort_every, timing_every):
    """The static octree workload (unit cube, level 4 refined to level 7
    inside a centred ball of radius 0.15: 46,488 leaves) with n electrons,
    timed like the quadtree workload."""
    import torch
    from paper_1604_07713_amd import binding as B
    from paper_1604_07713_amd import inputs as I
    d = I.octree_static_desc()
    g = B.Context(d)
    s, v, w, ids = I.octree_particles(n)
    g.load(0, 0, s, v, w, ids)
    keys, lv = g.leaves(0)
    x, y, z = I.leaf_corners3(keys, lv)
    g.field_set(0, B.CORNER_PHI_3D, I.octree_phi(x, y, z))
    g.leapfrog_start(0)
    if warmup:
        g.step(0, warmup, sort_every=sort_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = g.step(warmup, steps, sort_every=sort_every, timing=timing_every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g.close()
    updates = st["alive_start"][0]
    kern_ms = st["loop_ms"] / max(st["loop_launches"], 1)
    out = dict(particles=n, leaves=int(len(keys)), steps=steps, updates_per_s=updates / dt,
               ms_per_step=dt * 1e3 / steps, kernel_ms_per_step=kern_ms,
               workload=(f"3D static octree (levels 4-7, {len(keys)} leaves), {n} electrons, trilinear gather + "
                         f"push + reflect + locate + NGP deposit, sort every {sort_every} steps"))
    out["roofline"] = roofline((updates / steps) * BYTES_PER_UPDATE_3D, kern_ms,
                               traffic_from_profile("k_step3d<float,false>", f"octree {n} electrons"))
    out["roofline"]["per"] = "k_step3d<float,false> launch, 60 B per particle-update"
    return out


def dipic_bench(ppc=64, nsteps=400, precision=64, sort_every=20, timing_every=10):
    """The 1D discharge at w_p dt = 2.08 (n0 = 1e16 m^-3, 200 steps per RF
    period, 128 cells, 450 V, 30 mTorr argon with collisions and ionization
    births), stepped by the direct implicit scheme: predictor, implicit field
    solve and corrector every step, re-sorted every sort_every steps."""
    import numpy as np
    import torch
    from paper_1604_07713_amd import binding as B
    from paper_1604_07713_amd import inputs as I
    d = I.dipic_ccp_desc(precision=precision, ppc=ppc)
    g = B.Context(d)
    for sp, (s, v, w, ids) in enumerate(I.ccp_particles(d)):
        g.load(0, sp, s, v, w, ids)
    g.deposit(0)
    g.field_solve_1d(0, float(I.drive_voltage(d, 0)))
    g.leapfrog_start(0)
    vn = I.drive_voltage(d, np.arange(1, nsteps + 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = g.step(0, nsteps, vn, solve_field=True, sort_every=sort_every, timing=timing_every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g.close()
    updates = st["alive_start"][0] + st["alive_start"][1]
    kern_ms = st["loop_ms"] / max(st["loop_launches"], 1)
    per_update = BYTES_PER_UPDATE_DIPIC[precision]
    roof = roofline((updates / nsteps) * per_update, kern_ms)
    roof["per"] = (f"the step's kernels (predictor, implicit field, corrector, births), {per_update} B per "
                   "particle-update (predictor and corrector traffic; collisions' extra bytes left out)")
    return dict(particles_start=2 * d["extra"]["npart"], steps=nsteps, precision=f"fp{precision}",
                updates_per_s=updates / dt, ms_per_step=dt * 1e3 / nsteps, roofline=roof,
                step_kernels_ms=kern_ms, births=st["births"],
                workload=(f"1D discharge, direct implicit (w_p dt 2.08, dx 4.4 Debye lengths), 128 cells x {ppc} "
                          f"per cell per species, {nsteps} steps, sort every {sort_every}"),
                note="step_kernels_ms: predictor + implicit field + corrector + births of one step (HIP events "
                     f"around every {timing_every}th step)")


def dipic_runs():
    """The discharge as the tests run it (FP64, 16,384 particles) and at
    2048 per cell per species in FP32 (524,288 particles)."""
    return dict(discharge_fp64=dipic_bench(), discharge_large_fp32=dipic_bench(ppc=2048, nsteps=200, precision=32))


TIMING_EVERY = 10   # steps between timed launches of the dominant kernel
SORT_EVERY = 50     # re-sort the quadtree and octree particles by leaf every this many steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--particles", type=int, default=4194304)
    ap.add_argument("--large-particles", type=int, default=16777216,
                    help="particles of the labelled large variant whose state exceeds the Infinity Cache (0: skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=24)
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-vs-plain ensemble measurement")
    ap.add_argument("--no-streamer", action="store_true", help="skip the 2D streamer breakdown measurement")
    ap.add_argument("--streamer-steps", type=int, default=2000)
    ap.add_argument("--only-streamer", action="store_true", help="measure only the streamer (profiling)")
    ap.add_argument("--ensemble-steps", type=int, default=100)
    ap.add_argument("--only-ensemble", action="store_true", help="measure only the ensemble (profiling)")
    ap.add_argument("--only-quadtree", action="store_true", help="measure only the quadtree workload (profiling)")
    ap.add_argument("--no-avalanche", action="store_true", help="skip the batched-vs-plain 2D avalanche ensemble")
    ap.add_argument("--no-octree", action="store_true", help="skip the 3D octree workload")
    ap.add_argument("--only-octree", action="store_true", help="measure only the 3D octree workload (profiling)")
    ap.add_argument("--only-avalanche", action="store_true", help="measure only the 2D avalanche ensemble")
    ap.add_argument("--sort-every", type=int, default=SORT_EVERY,
                    help="steps between re-sorts of the quadtree and octree particles by leaf")
    ap.add_argument("--no-dipic", action="store_true", help="skip the direct implicit 1D discharge")
    ap.add_argument("--only-dipic", action="store_true", help="measure only the direct implicit 1D discharge")
    ap.add_argument("--avalanche-steps", type=int, default=200)
    ap.add_argument("--avalanche-modes", default="batched,plain_fp32,plain")
    ap.add_argument("--ensemble-modes", default="batched,plain_fp32,plain,batched_energy_conserving",
                    help="comma-separated ensemble modes to run with --only-ensemble")
    ap.add_argument("--ensemble-sort-every", type=int, default=50)
    ap.add_argument("--tile", type=int, default=0, help="batched work-item size (with --grid: skip the autotuner)")
    ap.add_argument("--grid", type=int, default=0, help="batched persistent grid (with --tile)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="instead of the benchmark, copy this many bytes 10 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (sharding across GPUs is designed, not built); --gpus must be 1"}))
        sys.exit(2)
    profiling = (args.only_ensemble or args.only_streamer or args.only_quadtree or args.only_avalanche
                 or args.only_octree or args.only_dipic or args.copy_probe)
    # the oracle's host timing runs first, before this process touches the GPU
    # (its ensemble sample forks worker processes)
    cpu = None
    if not args.no_cpu and not profiling:
        cpu = cpu_baseline(args.particles, args.cpu_steps)
        note("cpu baseline")

    import numpy as np
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        a = torch.empty(args.copy_probe // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "repeats": 10}), flush=True)
        return
    shape = (args.tile, args.grid) if args.tile and args.grid else None
    if args.only_ensemble:
        print(json.dumps({"ensemble": ensemble_bench(args.ensemble_steps, tune=False,
                                                     modes=tuple(args.ensemble_modes.split(",")),
                                                     shape=shape, sort_every=args.ensemble_sort_every)}),
              flush=True)
        return
    if args.only_streamer:
        print(json.dumps({"streamer": streamer_bench(args.streamer_steps)}), flush=True)
        return
    if args.only_octree:
        print(json.dumps({"octree": octree_bench(args.particles, args.steps, args.warmup, min(args.sort_every, args.steps),
                                                 TIMING_EVERY)}), flush=True)
        return
    if args.only_dipic:
        print(json.dumps({"dipic": dipic_runs()}), flush=True)
        return
    if args.only_avalanche:
        print(json.dumps({"avalanche_ensemble": avalanche_bench(args.avalanche_steps, shape=shape,
                                                                modes=tuple(args.avalanche_modes.split(",")))}),
              flush=True)
        return

    # the timed steps hold floor(steps / sort_every) sorts
    sort_every = min(args.sort_every, args.steps)
    q = quadtree_bench(args.particles, args.steps, args.warmup, sort_every, TIMING_EVERY)
    note(f"quadtree {args.particles}")
    value = q["updates"] / q["seconds"]
    # dominant kernel: the fused 2D step kernel; its mean launch duration from
    # HIP events recorded on the library's stream around the launches of every
    # TIMING_EVERY-th step of the timed loop (events around every launch would
    # add ~8 us per step to the wall time measured above)
    per_launch = (q["updates"] / args.steps) * BYTES_PER_UPDATE_2D
    workload = "quadtree 4194304 electrons" if args.particles == 4194304 else f"quadtree {args.particles} electrons"
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": q["seconds"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2D static quadtree (levels 6-9, 23620 leaves), {args.particles} electrons, "
                               f"gather+push+reflect+locate+NGP deposit, sort every {sort_every} steps "
                               f"({args.steps // sort_every} sorts in the timed steps)",
                   "particles": args.particles, "leaves": q["leaves"], "precision": "fp32 particles, int64 deposit",
                   "kernel_ms_per_step": q["kernel_ms"]},
        "roofline": roofline(per_launch, q["kernel_ms"],
                             traffic_from_profile("k_step<float,false,2,true>", workload)),
    }
    out["roofline"]["per"] = "k_step<float,false,2,true> launch, 44 B per particle-update"
    if args.only_quadtree:
        print(json.dumps(out), flush=True)
        return
    if args.large_particles:
        n = args.large_particles
        ql = quadtree_bench(n, 50, 10, min(args.sort_every, 50), 5)
        note(f"quadtree {n}")
        out["quadtree_large"] = dict(
            particles=n, state_bytes=n * 28,
            note="state beyond the 256 MB Infinity Cache: the bandwidth figure is HBM bandwidth",
            updates_per_s=ql["updates"] / ql["seconds"], ms_per_step=ql["seconds"] * 1e3 / 50,
            kernel_ms_per_step=ql["kernel_ms"],
            roofline=dict(roofline((ql["updates"] / 50) * BYTES_PER_UPDATE_2D, ql["kernel_ms"],
                                   traffic_from_profile("k_step<float,false,2,true>", f"quadtree {n} electrons")),
                          per="k_step<float,false,2,true> launch, 44 B per particle-update"))
    if not args.no_octree:
        out["octree"] = octree_bench(args.particles, args.steps, args.warmup, sort_every, TIMING_EVERY)
        note("octree")
    if not args.no_ensemble:
        out["ensemble"] = ensemble_bench(args.ensemble_steps, shape=shape, sort_every=args.ensemble_sort_every)
        note("ensemble")
    if not args.no_streamer:
        out["streamer"] = streamer_bench(args.streamer_steps)
        note("streamer")
    if not args.no_avalanche:
        out["avalanche_ensemble"] = avalanche_bench(args.avalanche_steps, shape=shape,
                                                    modes=tuple(args.avalanche_modes.split(",")))
        note("avalanche ensemble")
    if not args.no_dipic:
        out["dipic"] = dipic_runs()
        note("dipic")
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
