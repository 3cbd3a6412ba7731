"""Batches (one graph launch advancing several lattices), the autotuner and the
continuous-batching server, on the GPU through the C interface.

Graph replays are checked against eager stepping of identical lattices after
every replay, with the program's own eager work and synchronisations between
the replays; every comparison is bitwise (the batch runs the same kernels)."""
import numpy as np
import pytest

from paper_1004_4414_amd import workloads as W

pytestmark = pytest.mark.gpu


def lbm():
    from paper_1004_4414_amd import lbm as _lbm
    return _lbm


def _members():
    """three uneven boxes: spheres with colours, a sphere-free box, a 16-bit box"""
    out = []
    p = W.params(nx=32, ny=32, nz=32, rho_init=(0.4, 0.3), noise_amp=0.02, g_br=0.08, seed=21)
    rng = np.random.default_rng(21)
    pos = W.random_sphere_positions((32, 32, 32), 3, 4.0, seed=21)
    parts = W.make_particles(pos, 4.0, vel=rng.uniform(-0.02, 0.02, (3, 3)), color=[0.05, -0.05, 0.0])
    out.append((p, parts, "fp32"))
    out.append((W.params(nx=40, ny=24, nz=20, rho_init=(0.35, 0.35), noise_amp=0.02, g_br=0.09, seed=22),
                None, "fp32"))
    p3 = W.params(nx=36, ny=36, nz=28, rho_init=(0.35, 0.35), noise_amp=0.02, g_br=0.08, seed=23)
    pos3 = W.random_sphere_positions((36, 36, 28), 2, 5.0, seed=23)
    out.append((p3, W.make_particles(pos3, 5.0), "bf16"))
    return out


def _make(spec):
    p, parts, prec = spec
    lat = lbm().Lattice(p, precision=prec)
    if parts is not None:
        lat.add_particles(parts)
    return lat


def _same(a, b):
    assert np.array_equal(a.populations(), b.populations())
    assert np.array_equal(a.owner(), b.owner())
    if a.num_particles:
        pa, pb = a.particles(), b.particles()
        for k in ("R", "U", "W"):
            assert np.array_equal(pa[k], pb[k]), k


def test_batch_replays_match_eager_stepping():
    specs = _members()
    batched = [_make(s) for s in specs]
    eager = [_make(s) for s in specs]
    batch = lbm().Batch(batched, steps_per_launch=4)
    assert batch.steps_per_launch == 4
    done = 0
    for nl in (1, 2, 1):
        batch.step(nl)
        for e in eager:
            e.step(4 * nl)
        done += 4 * nl
        # eager work of the program itself between replays
        obs = batched[0].observables()
        assert obs["step"] == done
        for b, e in zip(batched, eager):
            _same(b, e)
    batch.close()
    for b, e in zip(batched, eager):
        b.step(2)
        e.step(2)
        _same(b, e)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_shared_launch_batch_matches_eager_stepping(precision):
    """Members of one precision and model are advanced by one launch per stage
    over all of them; uneven boxes (row-aligned 64 x 36 x 20 with spheres,
    ragged 40 x 24 x 20 without, 36^3 with spheres) stay bitwise equal to
    eager stepping; the 36^3 member averages its spheres' fluid force over
    two steps (force_average)."""
    specs = []
    p1 = W.params(nx=64, ny=36, nz=20, rho_init=(0.4, 0.3), noise_amp=0.02, g_br=0.08, seed=51)
    rng = np.random.default_rng(51)
    pos1 = W.random_sphere_positions((64, 36, 20), 4, 4.0, seed=51)
    specs.append((p1, W.make_particles(pos1, 4.0, vel=rng.uniform(-0.02, 0.02, (4, 3)), color=[0.05, 0, -0.05, 0]),
                  precision))
    specs.append((W.params(nx=40, ny=24, nz=20, rho_init=(0.35, 0.35), noise_amp=0.02, g_br=0.09, seed=52),
                  None, precision))
    p3 = W.params(nx=36, ny=36, nz=36, rho_init=(0.35, 0.35), noise_amp=0.02, g_br=0.08, seed=53,
                  force_average=1)
    pos3 = W.random_sphere_positions((36, 36, 36), 3, 5.0, seed=53)
    specs.append((p3, W.make_particles(pos3, 5.0, vel=rng.uniform(-0.02, 0.02, (3, 3))), precision))
    batched = [_make(s) for s in specs]
    eager = [_make(s) for s in specs]
    batch = lbm().Batch(batched, steps_per_launch=6)
    for nl in (1, 3):
        batch.step(nl)
        for e in eager:
            e.step(6 * nl)
        for b, e in zip(batched, eager):
            _same(b, e)
    # a member stepped an odd number of times outside the batch is refused
    batched[1].step(1)
    with pytest.raises(lbm().LBError):
        batch.step(1)
    batched[1].step(1)
    batch.step(1)
    for e in eager:
        e.step(6)
    eager[1].step(2)
    for b, e in zip(batched, eager):
        _same(b, e)
    batch.close()


def test_shared_launch_batch_with_cell_list_member():
    """A member with 1100 spheres takes the cell-list pair search inside the
    shared launches; it and a small member stay bitwise equal to eager stepping."""
    specs = []
    p1 = W.params(nx=64, ny=64, nz=64, rho_init=(0.36, 0.34), noise_amp=0.02, g_br=0.06, seed=61)
    pos1 = W.random_sphere_positions((64, 64, 64), 1100, 1.5, seed=61, min_gap=0.15)
    rng = np.random.default_rng(61)
    specs.append((p1, W.make_particles(pos1, 1.5, vel=rng.uniform(-0.02, 0.02, (1100, 3))), "fp32"))
    p2 = W.params(nx=32, ny=32, nz=32, rho_init=(0.35, 0.35), noise_amp=0.02, g_br=0.08, seed=62)
    specs.append((p2, W.make_particles(W.random_sphere_positions((32, 32, 32), 3, 4.0, seed=62), 4.0), "fp32"))
    batched = [_make(s) for s in specs]
    eager = [_make(s) for s in specs]
    batch = lbm().Batch(batched, steps_per_launch=4)
    batch.step(3)
    for e in eager:
        e.step(12)
    for b, e in zip(batched, eager):
        _same(b, e)
    batch.close()


def test_large_member_keeps_its_own_launches_beside_shared_ones():
    """A member of 2^21 sites (128^3) is captured with its own launches on a
    branch beside the shared launches of two small members; a lone small
    member of the shared kind takes its own launches too.  All stay bitwise
    equal to eager stepping."""
    big = W.params(nx=128, ny=128, nz=128, rho_init=(0.35, 0.35), noise_amp=0.02, g_br=0.08, seed=71)
    rng = np.random.default_rng(71)
    pos = W.random_sphere_positions((128, 128, 128), 40, 5.0, seed=71)
    specs = [(big, W.make_particles(pos, 5.0, vel=rng.uniform(-0.02, 0.02, (40, 3))), "fp32")] + _members()[:2]
    batched = [_make(s) for s in specs]
    eager = [_make(s) for s in specs]
    batch = lbm().Batch(batched, steps_per_launch=4)
    for nl in (1, 2):
        batch.step(nl)
        for e in eager:
            e.step(4 * nl)
        for b, e in zip(batched, eager):
            _same(b, e)
    batch.close()
    lone, lone_eager = _make(_members()[0]), _make(_members()[0])
    batch = lbm().Batch([lone], steps_per_launch=2)
    batch.step(3)
    lone_eager.step(6)
    _same(lone, lone_eager)
    batch.close()


def test_member_with_sweep_side_bounces_in_a_batch():
    """A member whose bounced populations the density sweep forms
    (link_writes = 0), stepped alone before, between and after replays of a
    shared-launch batch (whose steps write every bounce from the link kernel),
    stays bitwise equal to a twin that always writes them."""
    p = W.params(nx=32, ny=32, nz=28, rho_init=(0.36, 0.34), noise_amp=0.02, g_br=0.07, seed=81)
    rng = np.random.default_rng(81)
    pos = W.random_sphere_positions((32, 32, 28), 4, 3.5, seed=81)
    parts = W.make_particles(pos, 3.5, vel=rng.uniform(-0.04, 0.04, (4, 3)), color=[0.05, 0.0, -0.05, 0.0])
    lats = []
    for lw in (0, 1):
        lat = lbm().Lattice(dict(p, link_writes=lw), precision="fp32", kernel="twopass")
        lat.add_particles(parts)
        lats.append(lat)
    a, b = lats
    other = _make(_members()[1])
    a.step(7)
    b.step(7)
    batch = lbm().Batch([a, other], steps_per_launch=4)
    batch.step(2)
    b.step(8)
    a.step(2)
    b.step(2)
    batch.step(1)
    b.step(4)
    a.step(3)
    b.step(3)
    batch.close()
    assert np.array_equal(a.owner(), b.owner())
    assert np.array_equal(a.populations(), b.populations())
    pa, pb = a.particles(), b.particles()
    for k in ("R", "U", "W", "Ffluid", "Tfluid"):
        assert np.array_equal(pa[k], pb[k]), k
    assert a.observables()["covered_total"] == b.observables()["covered_total"]


def test_batch_membership_rules():
    L = lbm()
    a = _make(_members()[1])
    batch = L.Batch([a], steps_per_launch=2)
    with pytest.raises(L.LBError):
        L.Batch([a], steps_per_launch=2)  # already in a batch
    assert a.add_particles(W.make_particles([[5, 5, 5]], 3.0), check=False) == L.LB_ESTATE
    batch.close()
    with pytest.raises(L.LBError):
        L.Batch([a], steps_per_launch=3)  # odd step count


def test_autotune_returns_a_runnable_variant():
    L = lbm()
    p = W.params(nx=48, ny=40, nz=36, seed=31)
    parts = W.make_particles(W.random_sphere_positions((48, 40, 36), 4, 4.0, seed=31), 4.0)
    kernel, tile, ms = L.autotune(p, parts, "fp32", trial_steps=3)
    assert kernel in ("fused", "twopass") and ms > 0.0
    lat = L.Lattice(p, precision="fp32", kernel=kernel, tile=tile)
    lat.add_particles(parts)
    lat.step(2)
    lat.synchronize()


def test_served_results_equal_results_alone():
    from paper_1004_4414_amd import serving as S
    trace = W.serving_trace(5, seed=41, rate_per_min=600.0, step_scale=0.004, step_quantum=4)
    jobs = []
    for k, t in enumerate(trace):
        edge = 24 + 4 * k  # small boxes for the test, the trace's mix otherwise
        p = dict(t["params"], nx=edge, ny=edge, nz=edge)
        pos = W.random_sphere_positions((edge, edge, edge), 1 + k % 3, 4.0, seed=41 + k)
        jobs.append(S.Job(p, W.make_particles(pos, 4.0), t["steps"], arrival=t["arrival"],
                          contact_angle=t["contact_angle"], name=f"job{k}"))
    # a budget that holds about two jobs forces admission by footprint
    fp = S.Server(1, precision="fp32").footprint
    srv = S.Server(budget_bytes=2.2 * max(fp(j) for j in jobs), precision="fp32", steps_per_launch=4,
                   keep_digest=True)
    served = {r.name: r for r in srv.run(jobs)}
    alone = {r.name: r for r in S.run_alone(jobs, precision="fp32", keep_digest=True)}
    assert srv.batch_rebuilds >= 2
    for name, r in alone.items():
        assert served[name].populations_digest == r.populations_digest, name
        assert served[name].observables["step"] == r.observables["step"] == r.steps


class _FakeClock:
    """a clock that advances a fixed amount at every reading"""

    def __init__(self, dt):
        self.t = 0.0
        self.dt = dt

    def __call__(self):
        self.t += self.dt
        return self.t


def test_late_arrival_is_admitted_at_the_next_launch():
    """Continuous batching: a job arriving while another is on the GPU, with
    room in the memory budget, is admitted before the running job completes
    (at a launch boundary), and both results equal the jobs run alone."""
    from paper_1004_4414_amd import serving as S
    p1 = W.params(nx=32, ny=32, nz=32, seed=71)
    p2 = W.params(nx=24, ny=24, nz=24, seed=72)
    a = S.Job(p1, W.make_particles(W.random_sphere_positions((32, 32, 32), 2, 4.0, seed=71), 4.0), 200,
              arrival=0.0, name="early")
    b = S.Job(p2, W.make_particles(W.random_sphere_positions((24, 24, 24), 1, 4.0, seed=72), 4.0), 40,
              arrival=0.3, name="late")
    srv = S.Server(budget_bytes=10 * max(S.Server(1, "fp32").footprint(j) for j in (a, b)), precision="fp32",
                   steps_per_launch=10, keep_digest=True)
    res = {r.name: r for r in srv.run([a, b], clock=_FakeClock(0.05))}
    assert res["late"].admitted >= 0.3
    assert res["late"].admitted < res["early"].finished
    assert res["late"].finished < res["early"].finished  # 4 launches against the early job's 20
    alone = {r.name: r for r in S.run_alone([a, b], precision="fp32", keep_digest=True)}
    for n in ("early", "late"):
        assert res[n].populations_digest == alone[n].populations_digest


def test_jobs_without_steps_are_refused():
    from paper_1004_4414_amd import serving as S
    j = S.Job(W.params(nx=16, ny=16, nz=16), W.empty_particles(), 0, name="empty")
    with pytest.raises(ValueError):
        S.Server(1 << 40, precision="fp32", steps_per_launch=10).run([j])


def _oracle_compare(lat, ref, p, parts):
    g, r = lat.fields(), ref.fields()
    rbar = np.array(p["rho_init"])
    for c in range(2):
        assert np.abs(g["rho"][c] - r["rho"][c]).max() / rbar[c] < 1e-9
    assert np.abs(g["u"] - r["u"]).max() / max(np.abs(r["u"]).max(), 1e-30) < 1e-8
    assert np.array_equal(lat.owner(), ref.owner())
    if parts is not None:
        Pg, Pr = lat.particles(), ref.particles()
        for k in ("R", "U", "W", "Ffluid", "Tfluid"):
            assert np.abs(Pg[k] - Pr[k]).max() < 1e-9, k


def test_batch_members_fp64_match_the_oracle():
    """Two FP64 members (moving coloured spheres; a sphere-free box) advanced
    only by graph launches of a batch, then each compared with the oracle end
    to end: densities 1e-9, velocities 1e-8, the solid map exactly, sphere
    positions, velocities, forces and torques 1e-9."""
    from oracle.oracle import Oracle
    p1 = W.params(nx=20, ny=20, nz=20, rho_init=(0.36, 0.34), noise_amp=0.02, g_br=0.06, seed=31)
    parts = W.make_particles([[5.2, 5.5, 6.1], [14.3, 6.2, 13.7]], [3.0, 2.6],
                             vel=[[0.04, 0.03, -0.02], [-0.03, 0.05, 0.01]], color=[0.05, -0.05],
                             density=[0.8, 1.2])
    p2 = W.params(nx=16, ny=12, nz=10, rho_init=(0.35, 0.35), noise_amp=0.02, g_br=0.09, seed=32)
    lats = [lbm().Lattice(p1, precision="fp64"), lbm().Lattice(p2, precision="fp64")]
    lats[0].add_particles(parts)
    batch = lbm().Batch(lats, steps_per_launch=4)
    batch.step(10)
    batch.close()
    for lat, p, pr in zip(lats, (p1, p2), (parts, None)):
        ref = Oracle(p)
        if pr is not None:
            assert ref.add_particles(pr) == 0
        ref.step(40)
        assert lat.observables()["step"] == 40
        _oracle_compare(lat, ref, p, pr)


def test_served_job_fp64_matches_the_oracle():
    """A job served in FP64 beside another (both resident, advanced by shared
    graph launches) ends with the densities the oracle computes for it alone
    (1e-9 relative)."""
    from oracle.oracle import Oracle
    from paper_1004_4414_amd import serving as S
    p1 = W.params(nx=20, ny=18, nz=16, rho_init=(0.36, 0.34), noise_amp=0.02, g_br=0.06, seed=33)
    a = S.Job(p1, W.make_particles([[6.2, 7.1, 8.3]], 3.0, vel=[[0.03, -0.02, 0.01]]), 30, arrival=0.0,
              contact_angle=70.0, name="a")
    p2 = W.params(nx=24, ny=16, nz=16, seed=34)
    b = S.Job(p2, W.make_particles([[12.0, 8.0, 8.0]], 4.0), 60, arrival=0.0, name="b")
    srv = S.Server(1 << 40, precision="fp64", steps_per_launch=10, keep_density=("a",))
    res = {r.name: r for r in srv.run([a, b], clock=_FakeClock(0.01))}
    ref = Oracle(p1)
    assert ref.add_particles(S.coloured(a)) == 0
    ref.step(30)
    rho = ref.fields()["rho"]
    for c in range(2):
        assert np.abs(res["a"].extra["rho"][c] - rho[c]).max() / p1["rho_init"][c] < 1e-9
