"""Serving loop: continuous batching of ES-PIC jobs on one GPU.

Jobs (1D capacitively coupled discharges and 2D avalanches of different
sizes) arrive over time.  Each admitted job owns a slot of one library
context; its particle and mesh state stay resident on the GPU until it
finishes.  Admission is by projected device memory: ionization makes
particle counts grow, so a job is admitted when the sum of the projected
footprints of the resident jobs and the new one fits the budget.  Every tick
all resident 1D jobs advance together in one persistent batched launch per
step (each at its own step index), and the resident 2D jobs advance with
periodic adaptation and field solves.  Jobs that arrive while others run are
admitted as soon as memory and slots allow, so their work joins the device
stream of the running ones.

CLI: python -m paper_1604_07713_amd.serve --duration 60 --rate 20
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import binding as B
from . import inputs as I

GIB = 1 << 30


class Job:
    def __init__(self, spec, precision=32):
        self.spec = spec
        self.precision = precision
        self.kind = spec["kind"]
        self.arrival = spec["arrival"]
        self.steps_total = int(spec["steps"])
        self.key = spec["key"]
        self.slot = None
        self.steps_done = 0
        self.t_submit = None
        self.t_admit = None
        self.t_done = None
        self.updates = 0
        self.result = None
        if self.kind == "ccp":
            self.desc = I.ccp_desc(ncells=spec["ncells"], ppc=spec["ppc"], voltage=spec["voltage"],
                                   pressure_mtorr=spec["pressure"], precision=precision, seed=5,
                                   instance_key=spec["key"])
            self.nparticles = 2 * spec["ncells"] * spec["ppc"]
        else:
            self.desc = I.streamer_desc(side=spec["side"], precision=precision, seed=5, instance_key=spec["key"])
            self.nparticles = 2 * spec["npairs"]

    def projected_bytes(self, growth_ccp=3.0, growth_streamer=32.0):
        """Device footprint if the population grows by the given factor:
        particle slots (two buffers of s, v, w, id, cell in the particle
        precision) with the library's births/sort headroom, births staging,
        and the mesh."""
        e = self.precision // 8
        if self.kind == "ccp":
            per_slot = 2 * (4 * e + 12) + 11 * e
            slots = 2.0 * growth_ccp * self.nparticles + 8192
            mesh = 8 * 40 * (self.spec["ncells"] + 1)
        else:
            per_slot = 2 * (5 * e + 12) + 12 * e
            slots = 2.0 * growth_streamer * self.nparticles + 8192
            leaves = max(1024.0, growth_streamer * self.nparticles / 16.0)
            mesh = leaves * 400 + 4 * (1 << 18)
        return int(per_slot * slots + mesh)


class Server:
    def __init__(self, budget_bytes=None, tick_steps=25, field_every=10, adapt_every=10, max_slots=512,
                 keep_results=False, stream=None, batched=True):
        self.ctx = B.Context([], stream=stream)
        if budget_bytes is None:
            import torch
            free, total = torch.cuda.mem_get_info()
            budget_bytes = int(total - 16 * GIB)
        self.budget = budget_bytes
        self.tick_steps = tick_steps
        self.field_every = field_every
        self.adapt_every = adapt_every
        self.max_slots = max_slots
        self.keep_results = keep_results
        self.batched = batched   # False: every job steps with its own launches (the plain method)
        self.pending = []
        self.running = {}
        self.done = []
        self.committed = 0
        self.t0 = time.perf_counter()

    # ---- admission ----
    def submit(self, job):
        job.t_submit = time.perf_counter()
        self.pending.append(job)

    def _start(self, job):
        g = self.ctx
        slot = g.admit(job.desc)
        job.slot = slot
        job.t_admit = time.perf_counter()
        if job.kind == "ccp":
            parts = I.ccp_particles(job.desc, rng_seed=[5, job.key])
            for sp, (s, v, w, ids) in enumerate(parts):
                g.load(slot, sp, s, v, w, ids)
            g.deposit(slot)
            g.field_solve_1d(slot, float(I.drive_voltage(job.desc, 0)))
            g.leapfrog_start(slot)
        else:
            parts = I.streamer_particles(job.desc, npairs=job.spec["npairs"], rng_seed=[5, job.key])
            for sp, (s, v, w, ids) in enumerate(parts):
                g.load(slot, sp, s, v, w, ids)
            g.adapt(slot)
            self._solve2d(job)
            g.leapfrog_start(slot)
        # the library's own step counter starts at 0 for a new slot

    def _solve2d(self, job):
        phi, it, rr, rc = self.ctx.field_solve_2d(job.slot, rtol=1e-8, maxit=4000)
        return it

    # ---- stepping ----
    def _step_ccp(self):
        jobs = [j for j in self.running.values() if j.kind == "ccp"]
        if not jobs:
            return 0
        K = self.tick_steps
        full = [j for j in jobs if j.steps_total - j.steps_done >= K]
        rest = [j for j in jobs if j.steps_total - j.steps_done < K]
        upd = 0
        if self.batched:
            groups = ([(full, K)] if full else []) + [([j], j.steps_total - j.steps_done) for j in rest]
        else:
            groups = [([j], min(K, j.steps_total - j.steps_done)) for j in jobs]
        for group, n in groups:
            if n <= 0:
                continue
            vn = np.stack([I.drive_voltage(j.desc, np.arange(j.steps_done + 1, j.steps_done + n + 1))
                           for j in group], axis=1)
            st = self.ctx.step(-1, n, vn, solve_field=True, sort_every=20, batched=1 if self.batched else 0,
                               slots=[j.slot for j in group])
            u = st["alive_start"][0] + st["alive_start"][1]
            upd += u
            for j in group:
                j.steps_done += n
            # attribute updates to jobs by their share of particles (reporting only)
            for j in group:
                j.updates += u / len(group)
        return upd

    def _step_streamers(self):
        upd = 0
        for j in [j for j in self.running.values() if j.kind == "streamer"]:
            n = min(self.tick_steps, j.steps_total - j.steps_done)
            while n > 0:
                chunk = min(n, self.field_every - (j.steps_done % self.field_every))
                st = self.ctx.step(-1, chunk, slots=[j.slot], sort_every=0)
                u = st["alive_start"][0] + st["alive_start"][1]
                upd += u
                j.updates += u
                j.steps_done += chunk
                n -= chunk
                if j.steps_done % self.adapt_every == 0 and j.steps_done < j.steps_total:
                    self.ctx.adapt(j.slot)
                if j.steps_done % self.field_every == 0 and j.steps_done < j.steps_total:
                    self._solve2d(j)
        return upd

    def _retire(self):
        now = time.perf_counter()
        for slot, j in list(self.running.items()):
            if j.steps_done >= j.steps_total:
                if self.keep_results:
                    j.result = [self.ctx.read(slot, sp) for sp in range(2)]
                j.final_counts = [self.ctx.count(slot, sp) for sp in range(2)]
                self.ctx.retire(slot)
                self.committed -= j.projected
                j.t_done = now
                self.done.append(j)
                del self.running[slot]

    def run(self, jobs, max_wall=None, clock="wall"):
        """Serve jobs until all are done (or max_wall seconds).  clock='wall':
        a job is submitted when the wall clock passes its arrival time;
        clock='tick': when the tick counter does (deterministic tests).
        Returns TTR percentiles and the aggregate particle-update rate."""
        jobs = sorted(jobs, key=lambda j: j.arrival)
        t_start = time.perf_counter()
        i = 0
        total_upd = 0
        ticks = 0
        while True:
            now = time.perf_counter() - t_start
            while i < len(jobs) and (jobs[i].arrival <= now if clock == "wall" else jobs[i].arrival <= ticks):
                self.submit(jobs[i])
                i += 1
            self._admit()
            total_upd += self._step_ccp() + self._step_streamers()
            self._retire()
            ticks += 1
            if i >= len(jobs) and not self.pending and not self.running:
                break
            if max_wall is not None and time.perf_counter() - t_start > max_wall:
                break
            if not self.running and not self.pending and i < len(jobs) and clock == "wall":
                time.sleep(max(0.0, min(0.01, jobs[i].arrival - (time.perf_counter() - t_start))))
        wall = time.perf_counter() - t_start
        ttr = np.array([j.t_done - j.t_submit for j in self.done]) if self.done else np.zeros(0)
        return dict(jobs_done=len(self.done), jobs_submitted=i, jobs_pending=len(self.pending),
                    jobs_running=len(self.running), wall_s=wall, ticks=ticks,
                    updates=total_upd, updates_per_s=total_upd / wall if wall > 0 else 0.0,
                    ttr_p50_s=float(np.percentile(ttr, 50)) if len(ttr) else None,
                    ttr_p99_s=float(np.percentile(ttr, 99)) if len(ttr) else None,
                    budget_gib=self.budget / GIB)

    def _admit(self):
        """Admit pending jobs in arrival order while the projected footprint fits."""
        while self.pending and len(self.running) < self.max_slots:
            job = self.pending[0]
            need = job.projected_bytes()
            if self.committed + need > self.budget and self.running:
                break
            self.pending.pop(0)
            self._start(job)
            job.projected = need
            self.committed += need
            self.running[job.slot] = job

    def close(self):
        self.ctx.close()


def make_jobs(rate=20.0, duration=60.0, seed=5, scale=1.0, max_jobs=None, precision=32):
    specs = I.job_stream(rate=rate, duration=duration, seed=seed)
    jobs = []
    for s in specs:
        if s["kind"] == "ccp":
            s = dict(s, steps=max(1, int(s["steps"] * scale)))
        else:
            s = dict(s, steps=max(10, int(s["steps"] * scale)))
        jobs.append(Job(s, precision=precision))
        if max_jobs and len(jobs) >= max_jobs:
            break
    return jobs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--duration", type=float, default=60.0, help="arrival window, s")
    ap.add_argument("--rate", type=float, default=20.0, help="jobs per second")
    ap.add_argument("--max-wall", type=float, default=None, help="stop serving after this many seconds")
    ap.add_argument("--steps-scale", type=float, default=1.0, help="scale every job's step count")
    ap.add_argument("--tick-steps", type=int, default=25)
    ap.add_argument("--plain", action="store_true",
                    help="the plain method: FP64 particles, every job stepped with its own launches")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    jobs = make_jobs(args.rate, args.duration, scale=args.steps_scale, precision=64 if args.plain else 32)
    srv = Server(tick_steps=args.tick_steps, batched=not args.plain)
    m = srv.run(jobs, max_wall=args.max_wall)
    offered = sum(j.nparticles * j.steps_total for j in jobs) / max(args.duration, 1e-9)
    m["offered_updates_per_s_lower_bound"] = offered
    m["ccp_jobs"] = sum(1 for j in jobs if j.kind == "ccp")
    m["streamer_jobs"] = sum(1 for j in jobs if j.kind == "streamer")
    m["method"] = "plain FP64, per-job launches" if args.plain else "batched FP32, one launch for all 1D jobs"
    print(json.dumps(m), flush=True)
    srv.close()


if __name__ == "__main__":
    main()
