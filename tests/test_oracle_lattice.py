"""Pins of the oracle's lattice, equilibrium and unit relations against closed
forms (Sec. II of the paper) and against values the paper prints (Sec. VI)."""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_velocity_set_is_d3q19():
    c, zeta, opp = O.lattice()
    # 19 distinct velocities: rest, the 6 faces and the 12 edges of the unit cube
    rows = {tuple(v) for v in c}
    expect = {v for v in itertools.product((-1, 0, 1), repeat=3) if sum(abs(a) for a in v) <= 2}
    assert rows == expect and len(c) == 19
    assert tuple(c[0]) == (0, 0, 0)
    for i in range(19):
        assert np.array_equal(c[opp[i]], -c[i])


def test_weight_moment_identities():
    c, zeta, _ = O.lattice()
    c = c.astype(float)
    assert abs(zeta.sum() - 1.0) < 1e-15
    assert np.allclose((zeta[:, None] * c).sum(0), 0.0, atol=1e-15)
    second = np.einsum("i,ia,ib->ab", zeta, c, c)
    assert np.allclose(second, np.eye(3) / 3.0, atol=1e-15)  # c_s^2 = 1/3
    third = np.einsum("i,ia,ib,ic->abc", zeta, c, c, c)
    assert np.allclose(third, 0.0, atol=1e-15)
    fourth = np.einsum("i,ia,ib,ic,id->abcd", zeta, c, c, c, c)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(fourth, iso, atol=1e-15)  # c_s^4 (three deltas)


@pytest.mark.parametrize("order", [2, 3])
def test_equilibrium_moments_match_maxwellian(order):
    """Sum f^eq = rho, sum f^eq c = rho u, sum f^eq c c = rho (c_s^2 I + u u)
    exactly on D3Q19 for the equilibrium of Eq. (3)."""
    c, _, _ = O.lattice()
    c = c.astype(float)
    rng = np.random.default_rng(5)
    for _ in range(20):
        rho = rng.uniform(0.1, 2.0)
        u = rng.uniform(-0.1, 0.1, 3)
        f = O.equilibrium(rho, u, order)
        assert abs(f.sum() - rho) < 1e-14
        assert np.allclose(f @ c, rho * u, atol=1e-15)
        assert np.allclose(np.einsum("i,ia,ib->ab", f, c, c), rho * (np.eye(3) / 3.0 + np.outer(u, u)), atol=1e-15)


def test_third_order_terms_match_maxwellian_third_moment():
    """The cubic terms of Eq. (3) make the off-diagonal third moment
    sum f^eq c_a c_b^2 equal the Maxwellian's rho (c_s^2 u_a + u_a u_b^2) for a
    velocity in the a-b plane; the second-order equilibrium misses u_a u_b^2."""
    c, _, _ = O.lattice()
    c = c.astype(float)
    rng = np.random.default_rng(6)
    for a, b in [(0, 1), (1, 0), (0, 2), (2, 1)]:
        for _ in range(10):
            u = np.zeros(3)
            u[a], u[b] = rng.uniform(-0.1, 0.1, 2)
            rho = rng.uniform(0.2, 1.5)
            m3 = lambda f: float((f * c[:, a] * c[:, b] ** 2).sum())
            maxwell = rho * (u[a] / 3.0 + u[a] * u[b] ** 2)
            assert abs(m3(O.equilibrium(rho, u, 3)) - maxwell) < 1e-15
            if abs(u[a] * u[b] ** 2) > 1e-6:
                assert abs(m3(O.equilibrium(rho, u, 2)) - maxwell) > 1e-7


def test_effective_mass_limits():
    """Eq. (5): Psi(0) = 0, Psi ~ rho for small rho, Psi -> rho_0 for large rho,
    dPsi/drho = exp(-rho/rho_0)."""
    assert O.psi(0.0, 1.0) == 0.0
    assert abs(O.psi(1e-6, 1.0) - 1e-6) < 1e-12
    assert abs(O.psi(40.0, 1.0) - 1.0) < 1e-15
    for rho0 in (0.5, 1.0, 2.0):
        for r in (0.1, 0.7, 1.3):
            h = 1e-6
            d = (O.psi(r + h, rho0) - O.psi(r - h, rho0)) / (2 * h)
            assert abs(d - math.exp(-r / rho0)) < 1e-8


def test_si_conversion_reproduces_paper():
    """Sec. VI converts lattice units with water's c_s and nu at tau = 1 to
    Delta t = 9.14e-13 s and Delta x = 2.35 nm; that holds only with
    c_s^2 = 1/3 and nu = c_s^2 (tau - 1/2)."""
    g = json.load(open(os.path.join(GOLDEN, "si_conversion.json")))
    cs_lat = math.sqrt(O.cs2())
    nu_lat = O.viscosity(1.0)
    # c_s,SI = cs_lat dx/dt and nu_SI = nu_lat dx^2/dt
    dx = g["nu_water_m2_s"] / nu_lat * cs_lat / g["cs_water_m_s"]
    dt = dx * cs_lat / g["cs_water_m_s"]
    assert round(dx * 1e9, 2) == g["dx_nm"]
    assert float(f"{dt:.3g}") == g["dt_s"]
    assert abs(nu_lat - 1.0 / 6.0) < 1e-16


def test_splitmix64_reference_outputs():
    """Published SplitMix64 sequence for seed 1234567 (first five outputs)."""
    g = json.load(open(os.path.join(GOLDEN, "splitmix64.json")))
    for k, v in enumerate(g["outputs"]):
        assert O.uniform01(g["seed"], k) == (v >> 11) * 2.0 ** -53
