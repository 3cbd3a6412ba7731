"""Seeded synthetic inputs shared by the GPU path's tests, the oracle's tests and
the benchmark.

This module holds no arithmetic of the method itself: it only draws particle
positions (random sequential addition: the paper places its spheres at random
initial positions, Sec. VI) and assembles the parameter sets of the
benchmark workloads.  The random initial fluid densities are drawn by each
implementation from its own SplitMix64 generator keyed by ``seed``.
"""
import math

import numpy as np

#: parameter keys understood by both the GPU binding and the oracle
PARAM_DEFAULTS = dict(
    nx=16, ny=16, nz=16,
    tau=(1.0, 1.0), g_br=0.08, rho0=1.0, w_face=4.0, w_edge=2.0,
    velocity_mode=1, eq_order=3,
    rho_init=(0.35, 0.35), noise_amp=0.01, seed=1,
    body_accel=(0.0, 0.0, 0.0), wall_axis=-1, wall_vel=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),
    c0_mass_corr=0.0, k_hertz=100.0, lub_hc=2.0 / 3.0, lub_hmin=0.1, lub_mode=1,
    force_average=0,
)


def params(**kw):
    p = dict(PARAM_DEFAULTS)
    for k in kw:
        if k not in PARAM_DEFAULTS:
            raise KeyError(f"unknown parameter {k!r}")
    p.update(kw)
    return p


def empty_particles():
    return dict(pos=np.zeros((0, 3)), vel=np.zeros((0, 3)), omega=np.zeros((0, 3)),
                radius=np.zeros(0), density=np.zeros(0), color=np.zeros(0),
                prescribed=np.zeros(0, dtype=np.int32))


def make_particles(pos, radius, vel=None, omega=None, density=1.0, color=0.0, prescribed=0):
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    n = len(pos)
    full = lambda v: np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)).copy()
    return dict(
        pos=pos.copy(),
        vel=np.zeros((n, 3)) if vel is None else np.asarray(vel, dtype=np.float64).reshape(n, 3).copy(),
        omega=np.zeros((n, 3)) if omega is None else np.asarray(omega, dtype=np.float64).reshape(n, 3).copy(),
        radius=full(radius), density=full(density), color=full(color),
        prescribed=np.broadcast_to(np.asarray(prescribed, dtype=np.int32), (n,)).copy(),
    )


def random_sphere_positions(box, n, radius, seed, min_gap=1.0, max_tries=2_000_000):
    """Random sequential addition of ``n`` spheres of radius ``radius`` (scalar or
    array) in a periodic box ``(nx, ny, nz)``: uniform centres, rejected when any
    centre distance under the minimum image is <= r_a + r_b + min_gap."""
    L = np.asarray(box, dtype=np.float64)
    rad = np.broadcast_to(np.asarray(radius, dtype=np.float64), (n,))
    rng = np.random.Generator(np.random.PCG64(seed))
    cell = float(2 * rad.max() + min_gap)
    ncell = np.maximum((L // cell).astype(int), 1)
    grid = {}
    pos = np.zeros((n, 3))
    k = 0
    tries = 0
    while k < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError(f"could not place {n} spheres (placed {k})")
        c = rng.random(3) * L
        ci = tuple((c // (L / ncell)).astype(int) % ncell)
        ok = True
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    key = ((ci[0] + dx) % ncell[0], (ci[1] + dy) % ncell[1], (ci[2] + dz) % ncell[2])
                    for m in grid.get(key, ()):
                        d = c - pos[m]
                        d -= L * np.round(d / L)
                        if np.dot(d, d) <= (rad[k] + rad[m] + min_gap) ** 2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            pos[k] = c
            grid.setdefault(ci, []).append(k)
            k += 1
    return pos


def sphere_count(box, fraction, radius):
    return int(round(fraction * box[0] * box[1] * box[2] / (4.0 / 3.0 * math.pi * radius ** 3)))


def config(name):
    """Benchmark and parity workloads, returned as (params, particles, steps, precision).

    * ``spinodal32``: 32^3, two components at 0.7 +- 0.01 each, g = 0.1, no
      particles, FP64, 200 steps (spinodal decomposition).
    * ``spheres64``: 64^3, 50:50 at 0.35 +- 0.01 each, g = 0.08, 100 spheres
      of radius 4 (about 10% volume), neutral wettability, particle density 1,
      FP32, 1000 steps.
    * ``bijel256``: 256^3, 50:50 at 0.35 +- 0.01, g = 0.08, 4806 spheres of
      radius 5 (volume fraction 0.15), neutral wettability, FP32, 10000 steps,
      the spheres' fluid force averaged over two steps (force_average 1: with
      each step's force alone the run breaks down near step 5,300).
    """
    if name == "spinodal32":
        p = params(nx=32, ny=32, nz=32, rho_init=(0.7, 0.7), noise_amp=0.01, g_br=0.1, seed=1001)
        return p, empty_particles(), 200, "fp64"
    if name == "spheres64":
        box = (64, 64, 64)
        p = params(nx=64, ny=64, nz=64, rho_init=(0.35, 0.35), noise_amp=0.01, g_br=0.08, seed=1002)
        pos = random_sphere_positions(box, 100, 4.0, seed=1002)
        return p, make_particles(pos, 4.0), 1000, "fp32"
    if name == "bijel256":
        box = (256, 256, 256)
        n = sphere_count(box, 0.15, 5.0)
        p = params(nx=256, ny=256, nz=256, rho_init=(0.35, 0.35), noise_amp=0.01, g_br=0.08, seed=1003,
                   force_average=1)
        pos = random_sphere_positions(box, n, 5.0, seed=1003)
        return p, make_particles(pos, 5.0), 10000, "fp32"
    raise KeyError(name)


def _job(rng, edge, ratio_red, fraction, radius, theta, steps, seed, total=0.7):
    """one box of an ensemble: periodic cube, solvent ratio red:blue, spheres
    at the volume fraction, contact angle theta (degrees; the caller converts
    it to a particle colour).  Its spheres' fluid force is averaged over two
    steps (force_average 1): with the force of each step alone, light spheres
    in some of these dense random boxes run away within a few thousand steps"""
    box = (edge, edge, edge)
    p = params(nx=edge, ny=edge, nz=edge, rho_init=(total * ratio_red, total * (1.0 - ratio_red)),
               noise_amp=0.01, g_br=0.08, seed=seed, force_average=1)
    n = max(1, sphere_count(box, fraction, radius))
    # dense packings (up to 0.3) leave a smaller gap so that random addition
    # does not jam
    pos = random_sphere_positions(box, n, radius, seed=seed, min_gap=1.0 if fraction <= 0.2 else 0.1)
    return dict(params=p, particles=make_particles(pos, radius), steps=int(steps), contact_angle=float(theta))


def ensemble(n_boxes=64, seed=1004, steps=2000):
    """Batched ensemble: ``n_boxes`` independent periodic boxes with edges drawn
    from {32, 48, 64, 96}, solvent ratios 50:50 to 80:20, particle volume
    fractions 0.05-0.25, radii 4-6 and contact angles 60-120 degrees, FP32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    for k in range(n_boxes):
        edge = int(rng.choice([32, 48, 64, 96]))
        jobs.append(_job(rng, edge, float(rng.uniform(0.5, 0.8)), float(rng.uniform(0.05, 0.25)),
                         float(rng.uniform(4.0, 6.0)), float(rng.uniform(60.0, 120.0)), steps, seed * 1000 + k))
    return jobs


def serving_trace(n_jobs=40, seed=1005, rate_per_min=20.0, time_scale=1.0, step_scale=1.0, step_quantum=2):
    """Serving trace: Poisson arrivals at ``rate_per_min`` jobs per minute of
    periodic boxes with edges 48-192, radii 4-8 at volume fractions 0.05-0.3,
    contact angles 45-135 degrees and 2000-20000 steps.  ``time_scale`` divides
    the arrival times and ``step_scale`` multiplies the step counts (a
    compressed trace keeps the mix and shortens the run); step counts are
    rounded to multiples of ``step_quantum``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    jobs = []
    for k in range(n_jobs):
        t += float(rng.exponential(60.0 / rate_per_min)) / time_scale
        edge = int(rng.integers(48, 193))
        steps = float(rng.uniform(2000, 20000)) * step_scale
        steps = max(step_quantum, int(round(steps / step_quantum)) * step_quantum)
        job = _job(rng, edge, float(rng.uniform(0.5, 0.8)), float(rng.uniform(0.05, 0.3)),
                   float(rng.uniform(4.0, 8.0)), float(rng.uniform(45.0, 135.0)), steps, seed * 1000 + k)
        job["arrival"] = t
        jobs.append(job)
    return jobs


def slab_populations(shape, rho_major, rho_minor, z0, z1):
    """Populations (2, 19, nz, ny, nx) of fluid at rest with a red slab
    z0 <= z < z1 (red density rho_major, blue rho_minor) in blue fluid of the
    opposite composition: the flat-interface start of the contact-angle runs
    (Sec. V).  At rest each population is its lattice weight times the density
    (1/3 for the rest direction, 1/18 for the 6 faces, 1/36 for the 12 edges,
    in the library's direction order: rest, faces, edges)."""
    nz, ny, nx = shape
    z = np.arange(nz)[:, None, None]
    red = np.broadcast_to((z >= z0) & (z < z1), shape)
    rho = np.stack([np.where(red, rho_major, rho_minor), np.where(red, rho_minor, rho_major)])
    w = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)
    return rho[:, None] * w[None, :, None, None, None]
