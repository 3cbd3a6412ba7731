"""A request loop that serves simulation jobs with continuous batching.

Jobs (a box, its spheres, a step count) arrive over time.  The server admits a
waiting job as soon as its device footprint (lb_footprint_bytes) fits in the
memory budget left by the resident jobs, keeps every admitted lattice resident
on the GPU, and advances all resident jobs together: one graph launch of a
batch (lb_batch_*) moves every member by ``steps_per_launch`` steps.  The host
keeps at most ``ahead`` launches queued on the device (it waits on the event
of the oldest one before queueing another), and before every launch it admits
the jobs that have arrived and fit: a job that arrives while others are on the
GPU joins at the next launch, not at the next completion.  When a job has done
its steps its result is read back, its lattice is freed and its memory goes
back to the budget.

Each job's kernels are the ones it would run alone, so its result is bitwise
the same alone and in the mix.
"""
import time
from dataclasses import dataclass, field

import numpy as np

from . import lbm


@dataclass
class Job:
    params: dict
    particles: dict
    steps: int
    arrival: float = 0.0
    contact_angle: float = 90.0
    name: str = ""


@dataclass
class Result:
    name: str
    arrival: float
    admitted: float
    finished: float
    steps: int
    sites: int
    observables: dict
    populations_digest: str
    extra: dict = field(default_factory=dict)

    @property
    def time_to_result(self):
        return self.finished - self.arrival


def coloured(job):
    """the job's spheres with the particle colour of its contact angle"""
    parts = {k: np.array(v, copy=True) for k, v in job.particles.items()}
    parts["color"][:] = lbm.contact_angle_to_color(job.contact_angle)
    return parts


def digest(lat):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(lat.populations()).tobytes()).hexdigest()


def _finish(lat, job, admitted, t0, clock, keep_digest, keep_density=False):
    """the job's result; a job whose lattice reports an error (e.g. it went
    unstable) finishes with that error instead of observables.  With
    ``keep_density`` the two components' density fields go into ``extra``."""
    sites = job.params["nx"] * job.params["ny"] * job.params["nz"]
    try:
        lat.synchronize()
    except lbm.LBError as e:
        return Result(job.name, job.arrival, admitted, clock() - t0, job.steps, sites, None, "",
                      extra={"error": str(e)})
    obs = lat.observables()
    dg = digest(lat) if keep_digest else ""
    extra = {"rho": lat.fields()["rho"], "precision": lat.precision} if keep_density else {}
    return Result(job.name, job.arrival, admitted, clock() - t0, job.steps, sites, obs, dg, extra=extra)


class Server:
    """Continuous-batching server on one GPU.

    ``budget_bytes``: device memory the resident jobs may use (lb_footprint_bytes
    per job); ``precision``: population storage of every job; ``steps_per_launch``:
    steps per graph launch (every job's step count must be a multiple);
    ``ahead``: launches the host may keep queued on the device;
    ``keep_density``: names of jobs whose density fields the results carry."""

    def __init__(self, budget_bytes, precision="bf16", steps_per_launch=10, keep_digest=False, ahead=2,
                 keep_density=()):
        self.budget = int(budget_bytes)
        self.precision = precision
        self.k = int(steps_per_launch)
        self.keep_digest = keep_digest
        self.ahead = max(1, int(ahead))
        self.keep_density = set(keep_density)
        self.batch_rebuilds = 0
        self.launches = 0

    def footprint(self, job):
        r = float(job.particles["radius"].max()) if len(job.particles["radius"]) else 0.0
        return lbm.footprint_bytes(job.params, len(job.particles["radius"]), r, self.precision)

    def run(self, jobs, clock=time.perf_counter):
        import torch
        for j in jobs:
            if j.steps <= 0 or j.steps % self.k:
                raise ValueError(f"job {j.name}: {j.steps} steps is not a positive multiple of {self.k}")
            if self.footprint(j) > self.budget:
                raise ValueError(f"job {j.name} does not fit the memory budget")
        pending = sorted(jobs, key=lambda j: j.arrival)
        active = []  # [job, lattice, remaining, admitted, bytes]
        used = 0
        batch = None
        inflight = []  # events of the launches queued on the device, oldest first
        results = []
        t0 = clock()
        while pending or active:
            now = clock() - t0
            changed = False
            # admission in arrival order while memory allows (no overtaking)
            while pending and pending[0].arrival <= now and used + self.footprint(pending[0]) <= self.budget:
                j = pending.pop(0)
                lat = lbm.Lattice(j.params, precision=self.precision)
                if len(j.particles["radius"]):
                    lat.add_particles(coloured(j))
                b = self.footprint(j)
                used += b
                active.append([j, lat, j.steps, clock() - t0, b])
                changed = True
            if not active:
                time.sleep(max(0.0, min(pending[0].arrival - now, 0.05)))
                continue
            if changed or batch is None:
                if batch is not None:
                    batch.close()  # waits for its queued launches
                    inflight.clear()
                batch = lbm.Batch([a[1] for a in active], steps_per_launch=self.k)
                self.batch_rebuilds += 1
            # device progress: at most `ahead` launches queued before this one
            while len(inflight) >= self.ahead:
                inflight.pop(0).synchronize()
            batch.step(1)
            ev = torch.cuda.Event()
            ev.record(batch.stream)
            inflight.append(ev)
            self.launches += 1
            done = []
            for a in active:
                a[2] -= self.k
                if a[2] <= 0:
                    done.append(a)
            if done:
                batch.close()
                batch = None
                inflight.clear()
                for a in done:
                    results.append(_finish(a[1], a[0], a[3], t0, clock, self.keep_digest,
                                           a[0].name in self.keep_density))
                    a[1].close()
                    used -= a[4]
                    active.remove(a)
        if batch is not None:
            batch.close()
        return results


def run_alone(jobs, precision="fp32", keep_digest=False, clock=time.perf_counter, keep_density=()):
    """One job at a time in arrival order, each stepped by lb_step alone (the
    comparison point of the server)."""
    results = []
    t0 = clock()
    for j in sorted(jobs, key=lambda j: j.arrival):
        now = clock() - t0
        if j.arrival > now:
            time.sleep(j.arrival - now)
        admitted = clock() - t0
        lat = lbm.Lattice(j.params, precision=precision)
        if len(j.particles["radius"]):
            lat.add_particles(coloured(j))
        lat.step(j.steps)
        results.append(_finish(lat, j, admitted, t0, clock, keep_digest, j.name in set(keep_density)))
        lat.close()
    return results


def summary(results):
    """p50 / p99 time-to-result and jobs per hour over the completed jobs, site
    updates per second over the whole run, and the jobs that failed"""
    ok = [r for r in results if r.observables is not None]
    ttr = np.array([r.time_to_result for r in ok]) if ok else np.zeros(1)
    makespan = max(r.finished for r in results) - min(r.arrival for r in results)
    updates = sum(r.sites * r.steps for r in results)
    return dict(jobs=len(ok), failed=[r.name for r in results if r.observables is None],
                p50_s=float(np.percentile(ttr, 50)), p99_s=float(np.percentile(ttr, 99)),
                makespan_s=float(makespan), jobs_per_hour=float(len(ok) / makespan * 3600.0),
                mlups=float(updates / makespan / 1e6))


def density_error(result, job, short_steps=10):
    """The served result's density fields against the same job stepped alone
    with FP64 storage (the path that matches the oracle to rounding).

    Demixing amplifies any perturbation, so after many steps the interfaces
    of two runs that differ by rounding sit in different places and the
    pointwise difference says little about the storage: the same job with
    FP32 storage is compared with FP64 too, as the control.  Reported: the
    largest |rho - rho_fp64| of the served result and of the FP32 control,
    the same for the first ``short_steps`` steps (where rounding has not yet
    been amplified), the largest relative error of a component's total mass,
    and the relative error of the mean |phi| (phi = order parameter), a
    statistic of the demixed state."""
    def alone(precision, steps):
        j = Job(job.params, job.particles, steps, 0.0, job.contact_angle, job.name)
        return run_alone([j], precision=precision, keep_density=(job.name,))[0].extra["rho"]

    def mean_abs_phi(r):
        tot = r[0] + r[1]
        return float(np.abs((r[0] - r[1])[tot > 0] / tot[tot > 0]).mean())

    ref = alone("fp64", job.steps)
    f32 = alone("fp32", job.steps)
    a = result.extra["rho"]
    mass = np.abs(a.sum(axis=(1, 2, 3)) / ref.sum(axis=(1, 2, 3)) - 1.0)
    short = np.abs(alone(result.extra["precision"], short_steps) - alone("fp64", short_steps)).max()
    return dict(job=job.name, steps=job.steps, max_abs_rho=float(np.abs(a - ref).max()),
                max_abs_rho_fp32_control=float(np.abs(f32 - ref).max()),
                short_steps=short_steps, max_abs_rho_short=float(short),
                max_rel_mass=float(mass.max()),
                rel_mean_abs_phi=abs(mean_abs_phi(a) / mean_abs_phi(ref) - 1.0))
