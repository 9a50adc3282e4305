"""Pins for the oracle's integrators (Sect. 3.1): Kepler two-body orbit against its closed form,
convergence orders 2 (leapfrog) and 6 (symplectic composition), time reversibility, the
composition's order conditions, and energy / angular-momentum behaviour (Sect. 5.1)."""
import math

import numpy as np
import pytest

from paper_1003_3896_amd import inputs


def kepler_state(t, a=1.0, e=0.5, mu=1.0):
    """Relative position and velocity of a Kepler orbit starting at pericentre, from Kepler's
    equation E - e sin E = n t solved by Newton iteration."""
    nmean = math.sqrt(mu / a ** 3)
    M = nmean * t
    E = M if e < 0.8 else math.pi
    for _ in range(100):
        dE = (E - e * math.sin(E) - M) / (1 - e * math.cos(E))
        E -= dE
        if abs(dE) < 1e-16:
            break
    b = a * math.sqrt(1 - e * e)
    x = np.array([a * (math.cos(E) - e), b * math.sin(E), 0.0])
    Edot = nmean / (1 - e * math.cos(E))
    v = np.array([-a * math.sin(E) * Edot, b * math.cos(E) * Edot, 0.0])
    return x, v


def two_body(a=1.0, e=0.5, m1=0.5, m2=0.5, G=1.0):
    mu = G * (m1 + m2)
    r0, v0 = kepler_state(0.0, a, e, mu)
    M = m1 + m2
    pos = np.array([-m2 / M * r0, m1 / M * r0])
    vel = np.array([-m2 / M * v0, m1 / M * v0])
    return pos, vel, np.array([m1, m2])


def kepler_error(oracle_mod, integ, nsteps_per_orbit, orbits=1):
    pos, vel, m = two_body()
    P = 2 * math.pi
    dt = P / nsteps_per_orbit
    acc = oracle_mod.total_accel(pos, m, 1.0, 0.0)
    p, v, a = oracle_mod.step(pos, vel, m, acc, dt, nsteps_per_orbit * orbits, integ, 1.0, 0.0)
    r_num = p[1] - p[0]
    r_ex, _ = kepler_state(P * orbits)
    return np.linalg.norm(r_num - r_ex)


def test_kepler_closed_form_sym6(oracle_mod):
    """One orbit of e = 0.5 with 1024 sym6 steps lands on the closed-form pericentre."""
    assert kepler_error(oracle_mod, "sym6", 1024) < 1e-10


def test_kepler_closed_form_leapfrog(oracle_mod):
    assert kepler_error(oracle_mod, "leapfrog", 4096) < 2e-4


def _slope(oracle_mod, integ, ns):
    errs = [kepler_error(oracle_mod, integ, n) for n in ns]
    h = [1.0 / n for n in ns]
    return np.polyfit(np.log(h), np.log(errs), 1)[0], errs


def test_leapfrog_order_two(oracle_mod):
    s, errs = _slope(oracle_mod, "leapfrog", [256, 512, 1024, 2048])
    assert abs(s - 2.0) < 0.1, (s, errs)


def test_sym6_order_six(oracle_mod):
    s, errs = _slope(oracle_mod, "sym6", [128, 256, 512, 1024])
    assert min(errs) > 1e-13  # above the round-off floor so the slope is the truncation order
    assert abs(s - 6.0) < 0.3, (s, errs)


def test_sym6_coefficients(oracle_mod):
    d, k = oracle_mod.sym6_coefficients()
    w = d
    assert abs(w.sum() - 1.0) < 1e-15
    assert abs(k.sum() - 1.0) < 1e-15
    assert abs((w ** 3).sum()) < 1e-13
    assert abs((w ** 5).sum()) < 1e-13
    # symmetric composition: palindromic drifts and kicks
    assert np.array_equal(d, d[::-1]) and np.array_equal(k, k[::-1])
    # kicks are the merged half-weights of consecutive stages
    assert np.allclose(k[1:-1], 0.5 * (d[:-1] + d[1:]), rtol=0, atol=1e-16)


@pytest.mark.parametrize("integ", ["leapfrog", "sym6"])
def test_time_reversibility(oracle_mod, integ):
    pos, vel, m = inputs.plummer(64, 8)
    eps = 0.05
    acc = oracle_mod.total_accel(pos, m, 1.0, eps)
    p, v, a = oracle_mod.step(pos, vel, m, acc, 1.0 / 256, 100, integ, 1.0, eps)
    p2, v2, a2 = oracle_mod.step(p, -v, m, a, 1.0 / 256, 100, integ, 1.0, eps)
    assert np.abs(p2 - pos).max() < 1e-12
    assert np.abs(v2 + vel).max() < 1e-12


def test_energy_two_body_closed_form(oracle_mod):
    pos, vel, m = two_body()
    for eps in (0.0, 0.1):
        e = oracle_mod.energy(pos, vel, m, 1.0, eps)
        r = np.linalg.norm(pos[1] - pos[0])
        K = 0.5 * (m * (vel ** 2).sum(1)).sum()
        W = -m[0] * m[1] / math.sqrt(r * r + eps * eps)
        assert abs(e[0] - K) < 1e-15 and abs(e[1] - W) < 1e-15 and abs(e[3] - (K + W)) < 1e-15
        # for eps = 0 this is the Kepler energy -G m1 m2 / (2a)
        if eps == 0:
            assert abs(e[3] + 0.125) < 1e-14


def test_energy_conservation_orders(oracle_mod):
    """A short C1-like run: sym6 conserves energy far better than leapfrog, both without drift."""
    pos, vel, m = inputs.plummer(256, 21)
    eps = 1e-2
    e0 = oracle_mod.energy(pos, vel, m, 1.0, eps)[3]
    res = {}
    for integ in ("leapfrog", "sym6"):
        acc = oracle_mod.total_accel(pos, m, 1.0, eps)
        p, v, _ = oracle_mod.step(pos, vel, m, acc, 1.0 / 1024, 50, integ, 1.0, eps)
        res[integ] = abs(oracle_mod.energy(p, v, m, 1.0, eps)[3] - e0) / abs(e0)
    assert res["sym6"] < res["leapfrog"] / 10
    assert res["leapfrog"] < 1e-4


def test_plummer_ic_statistics(oracle_mod):
    """Henon units: E = -1/4, virial ratio 2K/|W| = 1 and half-mass radius 0.769, each to O(N^-1/2)."""
    pos, vel, m = inputs.plummer(4096, 4242)
    e = oracle_mod.energy(pos, vel, m, 1.0, 0.0)
    assert abs(e[3] + 0.25) < 0.0125
    assert abs(2 * e[0] / abs(e[1]) - 1.0) < 0.06
    r = np.sort(np.linalg.norm(pos, axis=1))
    assert abs(r[len(r) // 2] - 0.769) < 0.04
    assert abs(e[13] - 1.0) < 1e-14
    assert np.abs(e[4:7]).max() < 1e-15


def test_free_particles_drift_exactly(oracle_mod):
    """With negligible masses the integrators reduce to x += v t (kicks vanish)."""
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
    vel = np.array([[1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])
    m = np.array([0.0, 0.0])
    for integ in ("leapfrog", "sym6"):
        acc = oracle_mod.total_accel(pos, m, 1.0, 0.0)
        p, v, a = oracle_mod.step(pos, vel, m, acc, 0.125, 8, integ)
        np.testing.assert_allclose(p, pos + vel * 1.0, rtol=0, atol=1e-14)
        assert np.array_equal(v, vel)


@pytest.mark.parametrize("integ", ["leapfrog", "sym6"])
def test_momentum_and_angular_momentum_conserved(oracle_mod, integ):
    """Central, antisymmetric pair forces (after Eq. 2): P and L are invariants of every kick and
    drift, so they survive integration to rounding (3-D, non-planar, moving system)."""
    pos, vel, m = inputs.plummer(32, 33, salpeter=True)
    vel = vel + np.array([0.1, -0.2, 0.05])
    e0 = oracle_mod.energy(pos, vel, m, 1.0, 0.05)
    acc = oracle_mod.total_accel(pos, m, 1.0, 0.05)
    p, v, _ = oracle_mod.step(pos, vel, m, acc, 1.0 / 128, 40, integ, 1.0, 0.05)
    e1 = oracle_mod.energy(p, v, m, 1.0, 0.05)
    assert np.abs(e1[4:7] - e0[4:7]).max() < 1e-15
    assert np.abs(e1[7:10] - e0[7:10]).max() < 1e-13 * np.abs(e0[7:10]).max()


def test_angular_momentum_of_rigid_rotation(oracle_mod):
    """Closed form: particles on a ring of radius r in the plane normal to z, rotating with angular
    speed w, carry L = (0, 0, M r^2 w); rotating the whole set rotates L (covariance)."""
    n, r, w = 12, 0.7, 1.3
    th = 2 * math.pi * np.arange(n) / n
    pos = np.stack([r * np.cos(th), r * np.sin(th), np.zeros(n)], 1)
    vel = np.stack([-r * w * np.sin(th), r * w * np.cos(th), np.zeros(n)], 1)
    m = np.full(n, 1.0 / n)
    e = oracle_mod.energy(pos, vel, m, 1.0, 0.0)
    np.testing.assert_allclose(e[7:10], [0, 0, r * r * w], atol=1e-15)
    c, s = math.cos(0.4), math.sin(0.4)
    R = np.array([[1, 0, 0], [0, c, -s], [0, s, c]]) @ np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    e2 = oracle_mod.energy(pos @ R.T, vel @ R.T, m, 1.0, 0.0)
    np.testing.assert_allclose(e2[7:10], R @ e[7:10], atol=1e-15)
