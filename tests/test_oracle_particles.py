"""Pins of the oracle's particle coupling (Secs. III, IV of the paper) against
brute force, conservation laws and the qualitative claims of the paper."""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle_helpers import total_momentum
from paper_1004_4414_amd import workloads as W

C19 = np.array([v for v in itertools.product((-1, 0, 1), repeat=3) if 0 < sum(abs(a) for a in v) <= 2])


def brute_force_geometry(L, centre, r):
    """solid map, link count (fluid x, i with x - c_i solid) and shell count
    (solid sites with a fluid 18-neighbour) of one sphere, by direct counting"""
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    pos = np.stack([x, y, z], -1).astype(float)
    d = pos - np.asarray(centre)
    d -= L * np.round(d / L)
    d2 = (d ** 2).sum(-1)
    solid = d2 < r * r
    links = 0
    shell = np.zeros_like(solid)
    for c in C19:
        nb = np.roll(solid, shift=(c[2], c[1], c[0]), axis=(0, 1, 2))  # nb[x] = solid[x - c]
        links += int((~solid & nb).sum())
        fluid_at_x_plus_c = np.roll(~solid, shift=(-c[2], -c[1], -c[0]), axis=(0, 1, 2))
        shell |= solid & fluid_at_x_plus_c
    return solid, links, int(shell.sum()), d2


# (r, offset) -> (solid sites, links, shell sites), brute-force counts
GEOMETRY = [
    (1.0, (0.0, 0.0, 0.0), 1, 18, 1),
    (1.0, (0.5, 0.5, 0.5), 8, 96, 8),
    (1.5, (0.0, 0.0, 0.0), 19, 186, 18),
    (2.0, (0.0, 0.0, 0.0), 27, 234, 26),
    (4.0, (0.0, 0.0, 0.0), 251, 1050, 170),
    (4.0, (0.5, 0.5, 0.5), 280, 1176, 192),
    (5.0, (0.0, 0.0, 0.0), 485, 1674, 306),
    (5.0, (0.5, 0.5, 0.5), 552, 1896, 344),
    (5.0, (0.25, 0.1, 0.4), 525, 1800, 315),
    (6.0, (0.0, 0.0, 0.0), 895, 2514, 458),
]


@pytest.mark.parametrize("r,off,nsolid,nlinks,nshell", GEOMETRY)
def test_sphere_discretisation_matches_brute_force(r, off, nsolid, nlinks, nshell):
    L = 26
    centre = np.array([9.0, 10.0, 8.0]) + np.array(off)
    solid, links, shell, d2 = brute_force_geometry(L, centre, r)
    # sites near the surface are exact ties (d^2 == r^2, outside under the strict
    # test) or far enough that rounding of the centre cannot move them
    near = np.abs(d2 - r * r) < 1e-4
    assert np.all(d2[near] == r * r)
    assert (int(solid.sum()), links, shell) == (nsolid, nlinks, nshell)
    orc = O.Oracle(W.params(nx=L, ny=L, nz=L, noise_amp=0.0))
    assert orc.add_particles(W.make_particles([centre], r)) == 0
    assert np.array_equal(orc.owner() == 0, solid)
    lk, sh = orc.particle_counts()
    assert (int(lk[0]), int(sh[0])) == (nlinks, nshell)
    # the fluid on the solid sites was removed
    f = orc.populations()
    assert np.all(f[:, :, solid] == 0.0)


def test_overlapping_discretisations_go_to_the_lower_index():
    L = 16
    orc = O.Oracle(W.params(nx=L, ny=L, nz=L, noise_amp=0.0, k_hertz=0.0))
    # two spheres 4.9 apart with radius 2.5: their lattice footprints may share sites only
    # after they move closer; place them touching-but-valid, then move them together
    assert orc.add_particles(W.make_particles([[5.0, 8.0, 8.0], [10.1, 8.0, 8.0]], 2.5)) == 0
    P = orc.particles()
    orc.set_particle_state([[6.2, 8.0, 8.0], [9.0, 8.0, 8.0]], P["U"], P["W"])
    own = orc.owner()
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    in0 = (x - 6.2) ** 2 + (y - 8.0) ** 2 + (z - 8.0) ** 2 < 6.25
    in1 = (x - 9.0) ** 2 + (y - 8.0) ** 2 + (z - 8.0) ** 2 < 6.25
    assert (in0 & in1).sum() > 0
    assert np.all(own[in0] == 0) and np.all(own[in1 & ~in0] == 1)


def test_add_particles_validation():
    orc = O.Oracle(W.params(nx=16, ny=16, nz=16))
    assert orc.add_particles(W.make_particles([[4, 4, 4], [9.9, 4, 4]], 3.0)) == -4  # overlap
    assert orc.add_particles(W.make_particles([[4, 4, 4], [2.1, 4, 15.0]], 3.0)) == -4  # overlap across the boundary
    assert orc.add_particles(W.make_particles([[4, 4, 4]], 5.0)) == -1  # radius > L/4
    assert orc.add_particles(W.make_particles([[4, 4, 4]], 3.0)) == 0
    orc.step(1)
    assert orc.add_particles(W.make_particles([[12, 12, 12]], 2.0)) == -5  # after stepping


def _moving_spheres(c0=0.0, steps=60, g=0.06, seed=4, **kw):
    p = W.params(nx=20, ny=20, nz=20, rho_init=(0.36, 0.34), noise_amp=0.02, g_br=g, seed=seed,
                 c0_mass_corr=c0, **kw)
    orc = O.Oracle(p)
    pos = [[5.2, 5.5, 6.1], [14.3, 6.2, 13.7], [9.6, 14.4, 4.8]]
    vel = [[0.04, 0.03, -0.02], [-0.03, 0.05, 0.01], [0.02, -0.04, 0.05]]
    om = [[0.01, -0.02, 0.015], [0.0, 0.02, -0.01], [-0.02, 0.0, 0.01]]
    assert orc.add_particles(W.make_particles(pos, [3.0, 2.6, 3.3], vel=vel, omega=om,
                                              color=[0.05, -0.05, 0.0], density=[0.6, 1.0, 1.4])) == 0
    return orc


def test_moving_spheres_conserve_total_momentum():
    """Fluid momentum + particle momentum m U + pending impulses is conserved:
    pins the signs of the link exchange, the moving-wall term, the Shan-Chen
    force on the virtual fluid and the covering / uncovering impulses."""
    orc = _moving_spheres()
    p0 = total_momentum(orc)
    scale = orc.sums()["mass"].sum() * 0.05
    orc.step(60)
    c = orc.counts()
    assert c["covered_total"] > 10 and c["uncovered_total"] > 10
    assert np.abs(total_momentum(orc) - p0).max() < 1e-12 * scale


def test_force_average_shifts_the_momentum_balance_by_half_the_end_forces():
    """force_average = 1 (the fluid force entering Eqs. (9), (10) is the mean
    of this step's and the previous step's, this step's alone in the first):
    over steps 1..T the spheres take from the fluid the sum of the fluid
    forces plus half the first step's minus half the last step's, so fluid +
    sphere momentum + pending impulses moves by exactly (F_1 - F_T) / 2 summed
    over the spheres.  A weight other than 1/2, a stale or missing previous
    force, or averaging in the first step breaks the balance or the first
    step's equality with the plain run; the shift itself is far above the
    rounding, so the plain conservation law would fail here."""
    orc = _moving_spheres(force_average=1)
    plain = _moving_spheres()
    p0 = total_momentum(orc)
    scale = orc.sums()["mass"].sum() * 0.05
    orc.step(1)
    plain.step(1)
    a, b = orc.particles(), plain.particles()
    for k in ("R", "U", "W", "Ftotal", "Ttotal"):
        assert np.array_equal(a[k], b[k]), k
    F1 = a["Ffluid"].sum(0)
    prev = a
    for _ in range(59):
        pending = prev["PT"]
        orc.step(1)
        cur = orc.particles()
        # the torque half: the applied torque is the mean of the two reported
        # fluid torques plus the angular impulse pending before the step
        assert np.allclose(cur["Ttotal"], 0.5 * (cur["Tfluid"] + prev["Tfluid"]) + pending, rtol=0, atol=1e-13)
        prev = cur
    shift = 0.5 * (F1 - prev["Ffluid"].sum(0))
    assert np.abs(total_momentum(orc) - p0 - shift).max() < 1e-12 * scale
    assert np.abs(shift).max() > 1e-6 * scale
    assert orc.counts()["covered_total"] > 10


def test_previous_fluid_force_setter_continues_an_averaged_run():
    """A state copied mid-run (positions, velocities, pending impulses,
    populations) into a fresh oracle with force_average 1 continues the
    original bitwise once each sphere's previous fluid force and torque are
    handed over too, and differs without them (the copy then starts the
    average anew)."""
    a = _moving_spheres(force_average=1)
    a.step(10)
    Pa = a.particles()
    copies = []
    for hand_over in (True, False):
        b = _moving_spheres(force_average=1)
        b.set_particle_state(Pa["R"], Pa["U"], Pa["W"], Pa["P"], Pa["PT"])
        if hand_over:
            b.set_previous_fluid_force(Pa["Ffluid"], Pa["Tfluid"])
        b.set_populations(a.populations())
        b.step(5)
        copies.append(b)
    a.step(5)
    Pa, Pb, Pc = a.particles(), copies[0].particles(), copies[1].particles()
    for k in ("R", "U", "W", "Ftotal", "Ttotal"):
        assert np.array_equal(Pa[k], Pb[k]), k
    assert np.array_equal(a.populations(), copies[0].populations())
    assert not np.array_equal(Pa["U"], Pc["U"])


def test_mass_changes_only_by_covering_refilling_and_the_wall_term():
    """The moving-wall term of the bounce-back, covering and refilling are the
    only sources of fluid mass; everything else conserves it exactly."""
    orc = _moving_spheres()
    m0 = orc.sums()["mass"]
    orc.step(40)
    ev = orc.event_mass()
    # exact up to the rounding of ~10^5 additions per step
    assert np.allclose(orc.sums()["mass"], m0 - ev["covered"] + ev["refilled"] + ev["wall"], rtol=1e-11, atol=0)
    assert np.all(np.abs(ev["wall"]) > 1e-6)
    assert np.all(ev["covered"] > 0) and np.all(ev["refilled"] > 0)


def test_mass_correction_counteracts_the_mass_error():
    """Eq. (31): with C_0 > 0 a mass deficit raises the refilled densities."""
    a, b = _moving_spheres(c0=0.0), _moving_spheres(c0=200.0)
    a.step(40)
    b.step(40)
    ma, mb = a.sums()["mass"], b.sums()["mass"]
    m0 = _moving_spheres().sums()["mass"]
    assert np.all(np.abs(mb - m0) < np.abs(ma - m0))


def _c0_pair(c0, rho_init, delta):
    """two lattices with the same history, C_0 = 0 and C_0 = c0: one step, then
    the fluid rescaled per component so that the mass error of Eq. (31),
    Delta rho^c = M^c(now) - M^c(first step), is delta N for both components
    (N = all sites); returns the two lattices, the owner maps before and after
    a second step, and the mass errors"""
    out = []
    for c in (0.0, c0):
        p = W.params(nx=16, ny=16, nz=16, rho_init=rho_init, noise_amp=0.01, g_br=0.05, seed=5, c0_mass_corr=c)
        orc = O.Oracle(p)
        assert orc.add_particles(W.make_particles([[8.1, 8.3, 7.7]], 3.0, vel=[[0.23, 0.11, -0.07]],
                                                  prescribed=1)) == 0
        m0 = orc.sums()["mass"]  # the baseline M(0), taken at the start of the first step
        orc.step(1)
        f = orc.populations()
        m1 = orc.sums()["mass"]
        N = 16 ** 3
        for comp in range(2):
            f[comp] *= (m0[comp] + delta * N) / m1[comp]
        orc.set_populations(f)
        dM = orc.sums()["mass"] - m0
        own_before = orc.owner()
        orc.step(1)
        out.append((orc, own_before, orc.owner(), dM))
    return out


def test_mass_correction_factor_of_eq31():
    """Eq. (31) in closed form on refilled sites.  Everything before the refill
    is the same with and without the correction, so the refilled density
    (the only density of a new fluid site, since sum_i f_i^eq = rho_new) with
    C_0 divided by the one without is 1 - C_0 (sum_c rho_init^c / rho_init^c)
    Delta rho^c / N, with N all lattice sites.  With rho_init = (0.6, 0.2) and
    equal Delta rho^c / N the blue correction is exactly three times the red
    one; dropping the density ratio, or taking N as the fluid sites only,
    fails this."""
    c0, delta = 10.0, 2.5e-3
    rho_init = (0.6, 0.2)
    (a, own_b, own_a, dMa), (b, own_b2, own_a2, dMb) = _c0_pair(c0, rho_init, delta)
    assert np.array_equal(own_b, own_b2) and np.array_equal(own_a, own_a2)
    assert np.allclose(dMa, delta * 16 ** 3, rtol=1e-12) and np.allclose(dMb, dMa, rtol=0, atol=1e-12)
    unc = (own_b >= 0) & (own_a == -1)
    assert unc.sum() == a.counts()["uncovered_last"] == 8
    ra, rb = a.fields()["rho"], b.fields()["rho"]
    ratio = rb[:, unc] / ra[:, unc]  # (2, sites)
    N = 16 ** 3
    for comp in range(2):
        expect = 1.0 - c0 * (sum(rho_init) / rho_init[comp]) * dMb[comp] / N
        assert np.abs(ratio[comp] - expect).max() < 1e-12
    # equal mass errors per site: the blue correction is three times the red one
    assert np.allclose((1.0 - ratio[1]) / (1.0 - ratio[0]), 3.0, rtol=1e-9)
    # sites that were fluid before and after are untouched by the correction
    keep = (own_b == -1) & (own_a == -1)
    assert np.abs(rb[:, keep] - ra[:, keep]).max() == 0.0


def test_colour_sign_sets_the_preferred_fluid():
    """Sec. IV: a positive colour adds red virtual fluid and makes the particle
    prefer red (blue is repelled from its surface); a negative colour the reverse."""
    phis = []
    for col in (0.1, -0.1):
        orc = O.Oracle(W.params(nx=14, ny=14, nz=14, rho_init=(0.35, 0.35), noise_amp=0.0, g_br=0.05))
        assert orc.add_particles(W.make_particles([[7.0, 7.0, 7.0]], 3.0, color=col, prescribed=1)) == 0
        orc.step(40)
        own = orc.owner()
        fluid = own == -1
        near = np.zeros_like(fluid)
        for c in C19:
            near |= np.roll(own == 0, shift=(c[2], c[1], c[0]), axis=(0, 1, 2))
        rho = orc.fields()["rho"]
        phis.append(float((rho[0] - rho[1])[fluid & near].mean()))
    assert phis[0] > 1e-3 and phis[1] < -1e-3


def test_virtual_fluid_removes_the_density_halo():
    """Fig. 1 of the paper: without the virtual fluid the fluid forms a layer of
    raised total density around the particle; with it the layer is absent."""
    dev = {}
    for vf in (1, 0):
        orc = O.Oracle(W.params(nx=16, ny=16, nz=16, rho_init=(0.35, 0.35), noise_amp=0.0, g_br=0.05))
        orc_params = orc.params
        orc = O.Oracle(dict(orc_params, virtual_fluid=vf))
        assert orc.add_particles(W.make_particles([[8.0, 8.0, 8.0]], 4.0, prescribed=1)) == 0
        orc.step(200)
        rho = orc.fields()["rho"].sum(0)
        fluid = orc.owner() == -1
        dev[vf] = np.abs(rho[fluid] - 0.7).max()
    assert dev[1] < 1e-12
    assert dev[0] > 1e-3


def test_fixed_sphere_balances_the_driving_force():
    """A fixed sphere in a body-forced periodic flow: at steady state the fluid
    force on the sphere equals the total force that drives the fluid."""
    a = 2e-5
    orc = O.Oracle(W.params(nx=13, ny=13, nz=13, rho_init=(0.35, 0.35), noise_amp=0.0, g_br=0.0,
                            body_accel=(a, 0.0, 0.0)))
    assert orc.add_particles(W.make_particles([[6.0, 6.0, 6.0]], 2.5, prescribed=1)) == 0
    orc.step(3000)
    F = orc.particles()["Ffluid"][0]
    drive = a * orc.sums()["mass"].sum()
    assert abs(F[0] / drive - 1.0) < 0.01
    assert abs(F[1]) < 1e-3 * drive and abs(F[2]) < 1e-3 * drive


def test_rotating_sphere_feels_an_opposing_torque():
    orc = O.Oracle(W.params(nx=14, ny=14, nz=14, rho_init=(0.35, 0.35), noise_amp=0.0, g_br=0.0))
    om = np.array([0.0, 0.0, 2e-3])
    assert orc.add_particles(W.make_particles([[7.0, 7.0, 7.0]], 3.0, omega=[om], prescribed=1)) == 0
    orc.step(100)
    T = orc.particles()["Tfluid"][0]
    assert T[2] < 0 and abs(T[0]) < 1e-3 * abs(T[2]) and abs(T[1]) < 1e-3 * abs(T[2])
    # Stokes rotational drag 8 pi eta r^3 Omega sets the scale
    eta = 0.7 * O.viscosity(1.0)
    assert 0.3 < -T[2] / (8 * math.pi * eta * 27 * om[2]) < 3.0


def _two_spheres(gap, v, k_hertz=100.0, lub_hc=2.0 / 3.0):
    orc = O.Oracle(W.params(nx=24, ny=16, nz=16, rho_init=(0.0, 0.0), noise_amp=0.0, g_br=0.0,
                            k_hertz=k_hertz, lub_hc=lub_hc))
    x1, x2 = 8.0, 8.0 + 6.0 + gap
    assert orc.add_particles(W.make_particles([[x1, 8.0, 8.0], [x2, 8.0, 8.0]], 3.0,
                                              vel=[[v, 0, 0], [-v, 0, 0]])) == 0
    return orc


def test_hertz_collision_conserves_momentum_and_energy():
    """Eq. (21) in an empty lattice with the lubrication switched off: the
    head-on collision is elastic up to the leap-frog error and conserves
    momentum exactly."""
    orc = _two_spheres(gap=1.0, v=0.01, k_hertz=50.0, lub_hc=0.0)
    m = orc.particles()
    mass = 1.0 * 4.0 / 3.0 * math.pi * 27
    e0 = mass * (0.01 ** 2)
    orc.step(600)
    P = orc.particles()
    assert np.abs(P["U"].sum(0)).max() < 1e-15
    assert P["U"][0, 0] < 0 and P["U"][1, 0] > 0  # they bounced back
    e1 = 0.5 * mass * (P["U"] ** 2).sum()
    assert abs(e1 / e0 - 1.0) < 0.02


def test_lubrication_acts_only_below_the_cutoff_and_is_clamped():
    far = _two_spheres(gap=0.7, v=0.001)
    far.step(1)
    assert np.all(far.particles()["Ftotal"] == 0.0)
    f = []
    for gap in (0.05, 0.1, 0.3):
        o = _two_spheres(gap=gap, v=0.001)
        o.step(1)
        F = o.particles()["Ftotal"]
        assert F[0, 0] < 0 and F[1, 0] > 0 and F[0, 0] == -F[1, 0]  # repels the approach
        f.append(F[0, 0])
    assert f[0] == f[1]  # clamped at h_min = 0.1
    assert abs(f[2]) < abs(f[1])


def _row_of_spheres(n, gap, vel, density, r=3.0):
    """spheres of radius r on a line along x in an empty lattice (no fluid)"""
    nx = int(math.ceil(n * (2 * r + gap))) + 8
    orc = O.Oracle(W.params(nx=nx, ny=16, nz=16, rho_init=(0.0, 0.0), noise_amp=0.0, g_br=0.0))
    xs = [4.0 + r + k * (2 * r + gap) for k in range(n)]
    assert orc.add_particles(W.make_particles([[x, 8.0, 8.0] for x in xs], r, vel=vel, density=density)) == 0
    return orc


def test_lubrication_of_an_isolated_pair_is_backward_euler():
    """Eq. (22) taken implicitly: for one pair the approach speed after a step
    is w / (1 + c (1/m_1 + 1/m_2)) (closed form), even where the explicit
    update c (1/m_1 + 1/m_2) > 2 would reverse and amplify it."""
    r, gap, v, rho_p = 3.0, 0.1, 0.002, 0.05
    orc = _row_of_spheres(2, gap, [[v, 0, 0], [-v, 0, 0]], rho_p, r)
    m = rho_p * 4.0 / 3.0 * math.pi * r ** 3
    nu = (1.0 - 0.5) / 3.0
    c = 6.0 * math.pi * nu * 1.0 * (r * r / (2 * r)) ** 2 * (1.0 / 0.1 - 1.0 / (2.0 / 3.0))
    assert c * 2.0 / m > 2.0  # stiff: the explicit update would be unstable
    orc.step(1)
    U = orc.particles()["U"]
    w_after = U[0, 0] - U[1, 0]
    assert abs(w_after - 2 * v / (1.0 + 2.0 * c / m)) < 1e-15
    assert U[0, 0] == -U[1, 0] and U[0, 0] > 0.0


def _explicit_pair(gap, v, rho_p, r=3.0):
    orc = O.Oracle(W.params(nx=int(2 * (2 * r + gap)) + 8, ny=16, nz=16, rho_init=(0.0, 0.0), noise_amp=0.0,
                            g_br=0.0, lub_mode=0))
    xs = [4.0 + r, 4.0 + 3 * r + gap]
    assert orc.add_particles(W.make_particles([[x, 8.0, 8.0] for x in xs], r, vel=[[v, 0, 0], [-v, 0, 0]],
                                              density=rho_p)) == 0
    return orc


def test_explicit_lubrication_is_eq22_under_the_leapfrog():
    """lub_mode 0: Eq. (22) as printed, evaluated with the latest velocities
    U(t - 1/2) and integrated by the leap-frog of Eqs. (9), (10).  For an
    isolated pair the approach speed after one step is w (1 - c (1/m_1 +
    1/m_2)) and the force on each sphere is -c w along the centre line
    (closed form); in a stiff case (c (1/m_1 + 1/m_2) > 2, at the h_min clamp
    with light spheres) the speed reverses and grows, which is why the
    default mode applies the term implicitly."""
    r, v = 3.0, 0.002
    nu = (1.0 - 0.5) / 3.0
    for gap, rho_p in ((0.3, 1.0), (0.1, 0.05)):
        orc = _explicit_pair(gap, v, rho_p, r)
        m = rho_p * 4.0 / 3.0 * math.pi * r ** 3
        h = max(gap, 0.1)
        c = 6.0 * math.pi * nu * 1.0 * (r * r / (2 * r)) ** 2 * (1.0 / h - 1.0 / (2.0 / 3.0))
        orc.step(1)
        P = orc.particles()
        w = 2 * v
        assert abs(P["Ftotal"][0, 0] + c * w) < 1e-15 and P["Ftotal"][1, 0] == -P["Ftotal"][0, 0]
        w_after = P["U"][0, 0] - P["U"][1, 0]
        assert abs(w_after - w * (1.0 - 2.0 * c / m)) < 1e-15
        if 2.0 * c / m > 2.0:
            assert w_after < -w  # reversed and amplified
        else:
            assert 0.0 < w_after < w


def test_explicit_and_implicit_lubrication_agree_when_soft():
    """Far from the clamp and with heavy spheres the two readings of Eq. (22)
    differ only at second order in c/m over one step."""
    r, v, gap = 3.0, 0.002, 0.5
    a = _explicit_pair(gap, v, 5.0, r)
    b = _row_of_spheres(2, gap, [[v, 0, 0], [-v, 0, 0]], 5.0, r)
    a.step(1)
    b.step(1)
    Ua, Ub = a.particles()["U"], b.particles()["U"]
    m = 5.0 * 4.0 / 3.0 * math.pi * r ** 3
    nu = 0.5 / 3.0
    c = 6.0 * math.pi * nu * (r * r / (2 * r)) ** 2 * (1.0 / gap - 1.5)
    assert 0.0 < c * 2.0 / m < 0.02
    assert abs((Ua[0, 0] - Ua[1, 0]) - (Ub[0, 0] - Ub[1, 0])) < 2 * v * (2 * c / m) ** 2 * 1.01


def test_stiff_lubrication_network_dissipates_and_conserves_momentum():
    """A packed row of light spheres with alternating velocities (stiff: the
    explicit update would grow them geometrically): the shared-mass pair
    impulses only remove kinetic energy, and momentum is exact."""
    vel = [[0.002 * (-1) ** k, 0.0005 * k, 0.0] for k in range(6)]
    orc = _row_of_spheres(6, 0.05, vel, 0.05)
    p0 = orc.particles()
    m = 0.05 * 4.0 / 3.0 * math.pi * 27
    mom0 = (m * p0["U"]).sum(axis=0)
    ke = 0.5 * m * (p0["U"] ** 2).sum()
    for _ in range(10):
        orc.step(1)
        P = orc.particles()
        ke_new = 0.5 * m * (P["U"] ** 2).sum()
        assert ke_new <= ke * (1 + 1e-12)
        ke = ke_new
        assert np.allclose((m * P["U"]).sum(axis=0), mom0, rtol=0, atol=1e-16)
    assert np.abs(orc.particles()["U"][:, 0]).max() < 0.002


def test_runaway_sphere_stops_the_oracle():
    """A sphere that moves a lattice unit or more in one step is outside the
    scheme (the map update takes sub-lattice moves): the oracle stops with an
    error instead of stepping on."""
    p = W.params(nx=16, ny=16, nz=16, noise_amp=0.0, g_br=0.0, seed=3)
    ref = O.Oracle(p)
    assert ref.add_particles(W.make_particles([[8.0, 8.0, 8.0]], 2.0, vel=[[1.5, 0.0, 0.0]], prescribed=1)) == 0
    with pytest.raises(RuntimeError):
        ref.step(3)
    assert ref.counts()["step"] == 1


def test_runaway_criterion_is_per_axis():
    """The limit is one lattice unit per step along each axis (the map update
    walks sub-lattice moves per axis): a sphere moving (0.8, 0.8, 0) per step
    (speed 1.13) continues, one moving exactly 1 along an axis stops."""
    p = W.params(nx=16, ny=16, nz=16, noise_amp=0.0, g_br=0.0, seed=3)
    a = O.Oracle(p)
    assert a.add_particles(W.make_particles([[8.0, 8.0, 8.0]], 2.0, vel=[[0.8, 0.8, 0.0]], prescribed=1)) == 0
    a.step(3)
    assert a.counts()["step"] == 3
    b = O.Oracle(p)
    assert b.add_particles(W.make_particles([[8.0, 8.0, 8.0]], 2.0, vel=[[0.0, -1.0, 0.0]], prescribed=1)) == 0
    with pytest.raises(RuntimeError):
        b.step(3)
    assert b.counts()["step"] == 1


def test_add_particles_refuses_what_the_library_refuses():
    """Spheres need a periodic box (no walls) and a bounding box of
    2 ceil(r) + 7 sites that fits in one period of every axis."""
    orc = O.Oracle(W.params(nx=16, ny=16, nz=16, wall_axis=2))
    assert orc.add_particles(W.make_particles([[8, 8, 8]], 2.0)) == -1
    # r = 4 needs 15 sites; r = 4.01 needs 17
    orc = O.Oracle(W.params(nx=16, ny=16, nz=17))
    assert orc.add_particles(W.make_particles([[8, 8, 8]], 4.01)) == -1
    orc = O.Oracle(W.params(nx=17, ny=17, nz=17))
    assert orc.add_particles(W.make_particles([[8, 8, 8]], 4.01)) == 0
    orc = O.Oracle(W.params(nx=16, ny=16, nz=16))
    assert orc.add_particles(W.make_particles([[8, 8, 8]], 4.0)) == 0
