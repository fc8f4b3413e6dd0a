"""Throughput benchmark of the ES-PIC particle loop on one MI355X.

Default workload: the 2D static quadtree (unit square, level 6 base refined
to level 9 inside a centred disk of radius 0.15: 23,620 leaves), 4,194,304
electrons (uniform positions, 1 eV Maxwellian), FP32 particles, static
potential phi = x^2 + 0.3 sin(2 pi y) given at the nodes, reflecting walls.
One step = gather + leapfrog push + walls + locate + deposit for every
particle (no collisions in this workload), plus the periodic re-sort of the
particles by leaf.  Inputs are synthetic and seeded; they are resident in
HBM before the timed region starts.

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
# algorithmic bytes per particle-update of the 2D FP32 step kernel without
# collisions: read sx, sy, vx, vy, w, leaf (6 x 4 B), write sx, sy, vx, vy
# (4 x 4 B; the leaf index is rewritten only when it changes); the field,
# leaf and charge tables are cache resident.
BYTES_PER_UPDATE_2D = 40
METRIC = "particle-updates/s (locate+gather+push+MCC+deposit), 2D AMR; batched vs plain"
PROFILE_PMC = os.path.join(ROOT, "profiles", "step2d_quadtree_4M_pmc.json")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("k_step.hip", "device_util.hpp", "pic_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1604_07713_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile():
    """Measured HBM bytes per launch of the step kernel from the committed
    rocprofv3 PMC summary, if it was taken on the current kernel source."""
    try:
        with open(PROFILE_PMC) as f:
            p = json.load(f)
    except (OSError, ValueError):
        return None
    if p.get("kernel_source_hash") != kernel_source_hash():
        return None
    return p.get("hbm_bytes_per_launch")


def streamer_bench(nsteps=2000, npairs=10000, field_every=10, max_wall=120.0):
    """2D streamer breakdown on the dynamic quadtree (1 cm square, levels
    5-11, 30 kV/cm, Gaussian seed of 1e4 pairs, FP32 particles): every 10
    steps the tree is adapted (refine / coarsen with particle split / merge)
    and the FP64 CG field solve is redone.  Reports the particle-loop rate
    (collisions and births included) and the whole-run rate with adaptation
    and field solves."""
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
    step = 0
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    while step < nsteps and time.perf_counter() - t_start < max_wall:
        t0 = time.perf_counter()
        st = g.step(-1, field_every, sort_every=0)
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
        cg += it
        step += field_every
    wall = time.perf_counter() - t_start
    keys, _ = g.leaves(0)
    out = dict(steps=step, particles_end=int(g.count(0, 0) + g.count(0, 1)), leaves_end=int(len(keys)),
               births=births, particle_loop_updates_per_s=upd / max(t["step"], 1e-12),
               updates_per_s_with_adapt_and_field=upd / wall, particle_loop_s=t["step"], adapt_s=t["adapt"],
               field_solve_s=t["solve"], cg_iterations=cg, wall_s=wall,
               workload="1 cm x 1 cm, N2-like gas at 1 atm, 30 kV/cm, 1e4 seed pairs (sigma 0.5 mm), "
                        "levels 5-11, 16-64 particles per leaf, dt 1e-13 s, adapt + FP64 CG every 10 steps")
    g.close()
    return out


def cpu_baseline(nparticles, nsteps, seed=2):
    import numpy as np
    import oracle
    from paper_1604_07713_amd import inputs as I
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
    return dict(value=upd / dt, unit="particle-updates/s", cores=1, kind="oracle",
                sample=f"{nparticles} particles x {nsteps} steps of the same workload, single-threaded "
                       f"FP32-mirror oracle, {dt:.1f} s")


def ensemble_bench(nsteps, ninst=96, tune=True, modes=("batched", "plain", "batched_energy_conserving"), shape=None):
    """Batched ensemble of 1D CCP instances (config-0 physics, 96 uneven
    meshes): the FP32 batched path (one persistent launch per step, graph
    replay, autotuned work items) vs the FP64 plain path (per-instance
    launches), both with the on-device field solve; and the batched path
    again with the energy-conserving coupling (cell E, no interpolation)."""
    import numpy as np
    import torch
    from paper_1604_07713_amd import autotune
    from paper_1604_07713_amd import binding as B
    from paper_1604_07713_amd import inputs as I
    out = {}
    tuned_batched = None
    precs = {"batched": 32, "plain": 64, "batched_energy_conserving": 32}
    for mode in modes:
        prec = precs[mode]
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
        kw = dict(solve_field=True, sort_every=20)
        tuned = None
        if mode != "plain":
            if shape:
                tuned = dict(tile=shape[0], grid=shape[1])
            elif tuned_batched:
                tuned = tuned_batched   # same ensemble, same launch shape
            else:
                tuned = autotune.tune(make, descs, vtab) if tune else dict(tile=4096, grid=2048)
            tuned_batched = tuned
        if tuned:
            kw.update(batched=tuned["tile"], grid=tuned["grid"])
        g.step(0, 10, vtab[:10], **kw)          # warm-up
        st = g.step(10, nsteps, vtab[10:10 + nsteps], timing=True, **kw)
        kern = st["loop_ms"]
        if mode != "plain":
            kw["graph_steps"] = 25
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st2 = g.step(10 + nsteps, nsteps, vtab[10 + nsteps:10 + 2 * nsteps], **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        upd = st2["alive_start"][0] + st2["alive_start"][1]
        out[mode] = dict(precision=f"fp{prec}", updates_per_s=upd / dt, ms_per_step=dt * 1e3 / nsteps,
                         births_per_step=st2["births"] / nsteps,
                         loop_kernel_ms_per_step=kern / nsteps, particles=upd // nsteps,
                         launch="one persistent launch per step, HIP graph of 25 steps" if mode != "plain"
                         else "per-instance launches")
        if tuned:
            out[mode]["tile"] = tuned["tile"]
            out[mode]["grid"] = tuned["grid"]
        g.close()
    if "batched" in out and "plain" in out:
        out["batched_over_plain"] = out["batched"]["updates_per_s"] / out["plain"]["updates_per_s"]
    return out


TIMING_EVERY = 10   # steps between timed launches of the dominant kernel


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--particles", type=int, default=4194304)
    ap.add_argument("--sort-every", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=24)
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-vs-plain ensemble measurement")
    ap.add_argument("--no-streamer", action="store_true", help="skip the 2D streamer breakdown measurement")
    ap.add_argument("--streamer-steps", type=int, default=2000)
    ap.add_argument("--only-streamer", action="store_true", help="measure only the streamer (profiling)")
    ap.add_argument("--ensemble-steps", type=int, default=100)
    ap.add_argument("--only-ensemble", action="store_true", help="measure only the ensemble (profiling)")
    ap.add_argument("--ensemble-modes", default="batched,plain,batched_energy_conserving",
                    help="comma-separated ensemble modes to run with --only-ensemble")
    ap.add_argument("--tile", type=int, default=0, help="batched work-item size (with --grid: skip the autotuner)")
    ap.add_argument("--grid", type=int, default=0, help="batched persistent grid (with --tile)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="instead of the benchmark, copy this many bytes 10 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (sharding across GPUs is designed, not built); --gpus must be 1"}))
        sys.exit(2)

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
    from paper_1604_07713_amd import binding as B
    from paper_1604_07713_amd import inputs as I
    if args.only_ensemble:
        shape = (args.tile, args.grid) if args.tile and args.grid else None
        print(json.dumps({"ensemble": ensemble_bench(args.ensemble_steps, tune=False,
                                                     modes=tuple(args.ensemble_modes.split(",")),
                                                     shape=shape)}), flush=True)
        return
    if args.only_streamer:
        print(json.dumps({"streamer": streamer_bench(args.streamer_steps)}), flush=True)
        return

    d = I.quadtree_static_desc()
    n = args.particles
    g = B.Context(d)
    s, v, w, ids = I.quadtree_particles(n)
    g.load(0, 0, s, v, w, ids)
    keys, lv = g.leaves(0)
    cx, cy = I.leaf_corners(keys, lv)
    g.field_set(0, B.CORNER_PHI_2D, I.quadtree_phi(cx, cy))
    g.sort(0)
    g.leapfrog_start(0)
    if args.warmup:
        g.step(0, args.warmup, sort_every=args.sort_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = g.step(args.warmup, args.steps, sort_every=args.sort_every, timing=TIMING_EVERY)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    updates = st["alive_start"][0]
    value = updates / dt
    # dominant kernel: the fused 2D step kernel; its mean launch duration from
    # HIP events recorded on the library's stream around the launches of every
    # TIMING_EVERY-th step of the timed loop (events around every launch would
    # add ~8 us per step to the wall time measured above)
    kern_ms = st["loop_ms"] / max(st["loop_launches"], 1)
    per_launch_bytes = (updates / args.steps) * BYTES_PER_UPDATE_2D
    achieved = per_launch_bytes / (kern_ms * 1e-3) / 1e9
    traffic = traffic_from_profile()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D static quadtree (levels 6-9, 23620 leaves), 4194304 electrons, "
                               "gather+push+reflect+locate+NGP deposit, sort every %d steps" % args.sort_every,
                   "particles": n, "leaves": int(len(keys)), "precision": "fp32 particles, int64 deposit",
                   "kernel_ms_per_step": kern_ms},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic},
    }
    if not args.no_ensemble:
        out["ensemble"] = ensemble_bench(args.ensemble_steps)
    if not args.no_streamer:
        out["streamer"] = streamer_bench(args.streamer_steps)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
