"""Pins for the oracle's external galactic field (Eq. 3 term F_ext; bulge + disk + halo):
finite differences of its potential, circular-speed closed form, Sect. 6.1's orbital period of
about 60 time units at R = 8, and exact L_z conservation for the axisymmetric field (Table 2); and
for the Allen & Santillan (1991) Galaxy that Sect. 3 names: the circular speed, escape speed and
total mass its authors give, finite differences inside and beyond the halo cut-off, continuity
there, and the halo's enclosed mass against Gauss's law."""
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


def _as91(G_scale=1.0):
    g = _golden("allen_santillan_1991.txt")
    return g, (g["Mb"], g["ab"], g["Md"], g["ad"], g["bd"], 0.0, 1.0, 0.0, 0.0, 1.0, g["Mh"], g["ah"], g["rcut"])


def test_allen_santillan_published_properties(oracle_mod):
    """At the solar radius the model's circular speed is 220 km/s and its escape speed 536 km/s,
    and its total mass is 9.0e11 solar masses (read off the far field, where every component acts
    as a point mass: M = -r Phi)."""
    g, gal = _as91()
    R0 = g["R0"]
    a, phi = oracle_mod.ext_field(np.array([[R0, 0.0, 0.0]]), galaxy=gal)
    vc = math.sqrt(-a[0, 0] * R0)
    assert abs(vc - g["vc0"]) < 0.05, vc
    vesc = math.sqrt(-2.0 * phi[0])
    assert abs(vesc - g["vesc0"]) < 0.1, vesc
    r = 1e6
    _, phi = oracle_mod.ext_field(np.array([[r, 0.0, 0.0]]), galaxy=gal)
    mtot = -r * phi[0] * g["mass_unit_msun"]
    assert abs(mtot / g["mtot_msun"] - 1.0) < 0.005, mtot


def test_allen_santillan_is_minus_gradient(oracle_mod):
    """-grad Phi by central differences matches the acceleration inside the halo cut-off, beyond
    it, and at points on both sides of it; Phi and the acceleration are continuous across it."""
    g, gal = _as91()
    rng = np.random.default_rng(31)
    u = rng.normal(size=(60, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    radii = np.concatenate([10.0 ** rng.uniform(-1.5, 2.5, 50), [99.0, 101.0, 0.2, 8.5, 30.0, 250.0,
                                                                  99.9, 100.1, 5.0, 1.0]])
    pts = u * radii[:, None]
    a, _ = oracle_mod.ext_field(pts, galaxy=gal)
    fd = np.zeros_like(pts)
    for c in range(3):
        h = 1e-6 * np.maximum(1.0, radii)
        dp = np.zeros_like(pts)
        dp[:, c] = h
        fd[:, c] = -(oracle_mod.ext_field(pts + dp, galaxy=gal)[1] - oracle_mod.ext_field(pts - dp, galaxy=gal)[1]) / (2 * h)
    err = np.linalg.norm(a - fd, axis=1) / np.linalg.norm(a, axis=1)
    assert err.max() < 1e-7, err.max()
    rc = g["rcut"]
    inner = np.array([[rc * (1 - 1e-12), 0.0, 0.0]])
    outer = np.array([[rc * (1 + 1e-12), 0.0, 0.0]])
    ai, pi = oracle_mod.ext_field(inner, galaxy=gal)
    ao, po = oracle_mod.ext_field(outer, galaxy=gal)
    assert abs(pi[0] - po[0]) < 1e-9 * abs(pi[0])
    assert np.abs(ai - ao).max() < 1e-9 * np.abs(ai).max()


def test_allen_santillan_halo_mass_from_gauss(oracle_mod):
    """The halo alone: the radial field times r^2 / G is the mass inside r, which must rise as
    r^2.02 / (1 + (r/ah)^1.02) and stop at the cut-off; the spherical bulge alone has the mass
    Mb r^3 / (r^2 + ab^2)^(3/2) inside r."""
    g, gal = _as91()
    halo = (0.0, 1.0, 0.0, 1.0, 1.0, 0.0, 1.0, 0.0, 0.0, 1.0, g["Mh"], g["ah"], g["rcut"])
    bulge = (g["Mb"], g["ab"], 0.0, 1.0, 1.0, 0.0, 1.0, 0.0, 0.0, 1.0, 0.0, g["ah"], g["rcut"])
    for r in (0.5, 3.0, 12.0, 40.0, 100.0, 150.0, 400.0):
        x = np.array([[0.0, r / math.sqrt(2), r / math.sqrt(2)]])
        m = -(oracle_mod.ext_field(x, G=2.0, galaxy=halo)[0][0] @ x[0]) * r / 2.0
        s = min(r, g["rcut"]) / g["ah"]
        assert abs(m / (g["Mh"] * s ** 2.02 / (1.0 + s ** 1.02)) - 1.0) < 1e-13, r
        mb = -(oracle_mod.ext_field(x, G=2.0, galaxy=bulge)[0][0] @ x[0]) * r / 2.0
        assert abs(mb / (g["Mb"] * r ** 3 / (r * r + g["ab"] ** 2) ** 1.5) - 1.0) < 1e-13, r
    # the enclosed mass grows with r, so the density is positive, and is flat beyond the cut-off
    rs = np.linspace(0.1, 99.0, 200)
    pts = np.stack([rs, np.zeros_like(rs), np.zeros_like(rs)], axis=1)
    m = -oracle_mod.ext_field(pts, galaxy=halo)[0][:, 0] * rs
    assert np.all(np.diff(m) > 0)


def test_allen_santillan_orbits_conserve_energy_and_lz(oracle_mod):
    """Tracers on inclined orbits from the solar circle keep their energy and L_z under the
    oracle's sym6 integration (the field is static and axisymmetric): one that stays inside the
    halo cut-off to 1e-10 (sixth order: 3.3e-9 at dt = 0.01, 6e-12 at 0.005), one that goes out
    past it and back to 2e-8 (the field's derivative jumps at the cut-off, so there the error
    falls only as dt^2: 2.7e-8 at 0.01, 5.3e-9 at 0.005)."""
    g, gal = _as91()
    for vy, tol, crosses in ((30.0, 1e-10, False), (46.0, 2e-8, True)):
        p = np.array([[8.5, 0.0, 0.3]])
        v = np.array([[5.0, vy, 12.0]])
        m = np.array([1.0])
        e0 = oracle_mod.energy(p, v, m, 1.0, 0.0, field=True, galaxy=gal)
        acc = oracle_mod.total_accel(p, m, 1.0, 0.0, field=True, galaxy=gal)
        rmax = 0.0
        for _ in range(20):
            p, v, acc = oracle_mod.step(p, v, m, acc, 0.005, 400, "sym6", 1.0, 0.0, field=True, galaxy=gal)
            rmax = max(rmax, float(np.linalg.norm(p[0])))
        e1 = oracle_mod.energy(p, v, m, 1.0, 0.0, field=True, galaxy=gal)
        assert (rmax > g["rcut"]) == crosses, rmax
        assert abs(e1[3] - e0[3]) / abs(e0[3]) < tol
        assert abs(e1[9] - e0[9]) / abs(e0[9]) < 1e-12
