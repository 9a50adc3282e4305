"""Pins for the oracle's external galactic field (Eq. 3 term F_ext; bulge + disk + halo):
finite differences of its potential, circular-speed closed form, Sect. 6.1's orbital period of
about 60 time units at R = 8, and exact L_z conservation for the axisymmetric field (Table 2)."""
import math
import os

import numpy as np
import pytest

from paper_1003_3896_amd import inputs


def test_acceleration_is_minus_gradient(oracle_mod):
    rng = np.random.default_rng(3)
    pts = np.concatenate([rng.uniform(-12, 12, (40, 3)), rng.uniform(-0.5, 0.5, (10, 3)),
                          np.array([[8.0, 0.0, 0.0], [8.0, 0.0, 0.2], [0.3, 0.1, -2.0]])])
    a, _ = oracle_mod.ext_field(pts)
    h = 1e-5
    fd = np.zeros_like(pts)
    for c in range(3):
        dp = np.zeros(3)
        dp[c] = h
        fd[:, c] = -(oracle_mod.ext_field(pts + dp)[1] - oracle_mod.ext_field(pts - dp)[1]) / (2 * h)
    err = np.linalg.norm(a - fd, axis=1) / np.linalg.norm(a, axis=1)
    assert err.max() < 1e-8


def test_component_closed_forms(oracle_mod):
    """Each component alone against its textbook potential at a point."""
    x = np.array([[1.5, -0.5, 0.7]])
    R2 = 1.5 ** 2 + 0.5 ** 2
    r = math.sqrt(R2 + 0.49)
    # bulge only
    _, phi = oracle_mod.ext_field(x, galaxy=(2.0, 0.5, 0.0, 1.0, 1.0, 0.0, 1.0))
    assert abs(phi[0] + 2.0 / (r + 0.5)) < 1e-15
    # disk only
    _, phi = oracle_mod.ext_field(x, galaxy=(0.0, 1.0, 3.0, 2.0, 0.3, 0.0, 1.0))
    assert abs(phi[0] + 3.0 / math.sqrt(R2 + (2.0 + math.sqrt(0.49 + 0.09)) ** 2)) < 1e-15
    # halo only
    _, phi = oracle_mod.ext_field(x, galaxy=(0.0, 1.0, 0.0, 1.0, 1.0, 0.6, 5.0))
    assert abs(phi[0] - 0.18 * math.log(r * r + 25.0)) < 1e-15
    # G scales bulge and disk but not the halo (its amplitude is vh^2)
    a1, _ = oracle_mod.ext_field(x, G=1.0, galaxy=(1.0, 0.5, 1.0, 1.0, 0.3, 0.0, 1.0))
    a2, _ = oracle_mod.ext_field(x, G=2.0, galaxy=(1.0, 0.5, 1.0, 1.0, 0.3, 0.0, 1.0))
    np.testing.assert_allclose(a2, 2 * a1, rtol=1e-15)


def _golden(name):
    """key value pairs of a fixture under tests/golden/ (comment lines start with #)"""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    out = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def test_circular_speed_and_period(oracle_mod):
    """The circular orbit at R = 8 in the oracle's galaxy has the period Sect. 6.1 prints."""
    g = _golden("sect6_orbital_period.txt")
    assert g["radius"] == inputs.ORBIT_R
    a, _ = oracle_mod.ext_field(np.array([[inputs.ORBIT_R, 0.0, 0.0]]))
    vc = math.sqrt(inputs.ORBIT_R * abs(a[0, 0]))
    assert abs(vc - inputs.V_CIRC_8) < 1e-12
    period = 2 * math.pi * inputs.ORBIT_R / vc
    assert abs(period - g["period"]) < g["tolerance"]
    assert a[0, 1] == 0 and a[0, 2] == 0


def test_test_particle_orbit_conserves_energy_and_lz(oracle_mod):
    """A massless tracer on an inclined orbit: sym6 keeps E to ~1e-12 and L_z to rounding."""
    pos = np.array([[8.0, 0.0, 0.3]])
    vel = np.array([[0.05, inputs.V_CIRC_8, 0.04]])
    m = np.array([1.0])
    e0 = oracle_mod.energy(pos, vel, m, 1.0, 0.0, field=True)
    acc = oracle_mod.total_accel(pos, m, 1.0, 0.0, field=True)
    p, v, _ = oracle_mod.step(pos, vel, m, acc, 0.05, 1200, "sym6", 1.0, 0.0, field=True)
    e1 = oracle_mod.energy(p, v, m, 1.0, 0.0, field=True)
    assert abs(e1[3] - e0[3]) / abs(e0[3]) < 1e-11
    assert abs(e1[9] - e0[9]) / abs(e0[9]) < 1e-13
    # it went about once around (t = 60)
    assert np.linalg.norm(p[0, :2]) > 6.0


def test_torque_of_axisymmetric_field_has_no_z_component(oracle_mod):
    pos, vel, m = inputs.plummer(256, 5)
    pos, vel = inputs.on_orbit(pos, vel)
    e = oracle_mod.energy(pos, vel, m, 1.0, 1e-3, field=True)
    assert abs(e[12]) < 1e-14 * abs(e[10:12]).max() + 1e-16


BH_GALAXY = inputs.GALAXY + (50.0, 2e-3)


def test_black_hole_is_minus_gradient_and_closed_form(oracle_mod):
    """The central point mass (Sect. 6.2) alone against its softened Kepler potential, its
    acceleration against the finite difference of the whole field with it, and G scaling."""
    x = np.array([[1.5, -0.5, 0.7], [0.01, 0.002, -0.003]])
    r2 = (x * x).sum(1)
    a, phi = oracle_mod.ext_field(x, galaxy=(0.0, 1.0, 0.0, 1.0, 1.0, 0.0, 1.0, 7.0, 0.05))
    np.testing.assert_allclose(phi, -7.0 / np.sqrt(r2 + 0.0025), rtol=1e-15)
    np.testing.assert_allclose(a, -7.0 * x / ((r2 + 0.0025) ** 1.5)[:, None], rtol=1e-14)
    a2, _ = oracle_mod.ext_field(x, G=3.0, galaxy=(0.0, 1.0, 0.0, 1.0, 1.0, 0.0, 1.0, 7.0, 0.05))
    np.testing.assert_allclose(a2, 3 * a, rtol=1e-15)
    # Mbh = 0 is the 7-parameter galaxy exactly
    pts = np.array([[8.0, 0.1, 0.2], [0.3, -0.2, 0.1]])
    np.testing.assert_array_equal(oracle_mod.ext_field(pts, galaxy=inputs.GALAXY + (0.0, 0.3))[0],
                                  oracle_mod.ext_field(pts)[0])
    rng = np.random.default_rng(8)
    pts = np.concatenate([rng.uniform(-3, 3, (30, 3)), rng.uniform(-0.05, 0.05, (10, 3))])
    a, _ = oracle_mod.ext_field(pts, galaxy=BH_GALAXY)
    h = 1e-6
    fd = np.zeros_like(pts)
    for c in range(3):
        dp = np.zeros(3)
        dp[c] = h
        fd[:, c] = -(oracle_mod.ext_field(pts + dp, galaxy=BH_GALAXY)[1]
                     - oracle_mod.ext_field(pts - dp, galaxy=BH_GALAXY)[1]) / (2 * h)
    err = np.linalg.norm(a - fd, axis=1) / np.linalg.norm(a, axis=1)
    assert err.max() < 1e-7


def test_kepler_orbit_around_the_black_hole(oracle_mod):
    """A tracer around the point mass alone (no galaxy, no softening) on an e = 0.5 orbit follows
    Kepler's equation after one sym6 integration over one and a half periods."""
    M, a_k, e = 5.0, 1.0, 0.5
    gal = (0.0, 1.0, 0.0, 1.0, 1.0, 0.0, 1.0, M, 0.0)
    r_p = a_k * (1 - e)
    v_p = math.sqrt(M * (1 + e) / r_p)
    pos = np.array([[r_p, 0.0, 0.0]])
    vel = np.array([[0.0, v_p, 0.0]])
    m = np.array([1e-9])
    T = 2 * math.pi * math.sqrt(a_k ** 3 / M)
    t = 1.5 * T
    nsteps = 3000
    acc = oracle_mod.total_accel(pos, m, 1.0, 0.0, field=True, galaxy=gal)
    p, v, _ = oracle_mod.step(pos, vel, m, acc, t / nsteps, nsteps, "sym6", 1.0, 0.0, field=True, galaxy=gal)
    # Kepler's equation: mean anomaly at t = 1.5 T is pi -> apocentre on the -x axis
    assert abs(p[0, 0] + a_k * (1 + e)) < 1e-8 and abs(p[0, 1]) < 1e-7
    assert abs(math.hypot(v[0, 0], v[0, 1]) - math.sqrt(M * (1 - e) / (a_k * (1 + e)))) < 1e-8
