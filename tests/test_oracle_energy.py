"""Pins for the oracle's diagnostics of Sect. 5.1 that no closed form of the sum itself fixes:
the external torque of Eq. 8, the linear momentum, and the mass-weighted internal force sum.

Each quantity is checked against a different piece of mathematics than its own formula:
  * torque about axis n equals minus the derivative of U_ext = sum m Phi_ext(x) under a rigid
    rotation of the system about n (a finite difference of the potential energy, which the oracle
    computes by another route: Phi, not grad Phi);
  * torque equals the rate of change of L = sum m x cross v along the oracle's own integration
    (internal torques cancel for central pair forces);
  * momentum equals M times the velocity of the centre of mass (the displacement of sum m x / M
    along the integration, divided by the elapsed time);
  * sum m a_int vanishes by the antisymmetry of the pair forces of Eq. 2, and sum m |a_int| of two
    bodies has the closed form 2 G m1 m2 r / (r^2 + eps^2)^{3/2}.
"""
import math

import numpy as np

from paper_1003_3896_amd import inputs

GAL_BH = (1.0, 0.7, 4.5, 3.0, 0.28, 0.7, 12.0, 0.3, 0.05)  # the galaxy plus a central point mass


def rotation(axis, angle):
    """Rotation matrix about coordinate axis 0, 1 or 2 (right-handed)."""
    c, s = math.cos(angle), math.sin(angle)
    i, j = [(1, 2), (2, 0), (0, 1)][axis]
    R = np.eye(3)
    R[i, i] = c
    R[i, j] = -s
    R[j, i] = s
    R[j, j] = c
    return R


def off_axis_tracers(n=9, seed=5):
    """Tracers at distinct off-axis points above and below the disk plane, unequal masses."""
    rng = np.random.default_rng(seed)
    pos = np.column_stack([rng.uniform(-9, 9, n), rng.uniform(-9, 9, n), rng.uniform(-2.5, 2.5, n)])
    vel = rng.normal(0, 0.3, (n, 3))
    mass = rng.uniform(0.2, 1.5, n)
    return pos, vel, mass


def rotation_derivative_torque(oracle_mod, pos, vel, mass, galaxy, h=1e-5):
    """-dU_ext/dtheta about each coordinate axis, by a central difference of rigid rotations."""
    T = np.zeros(3)
    for k in range(3):
        up = oracle_mod.energy(pos @ rotation(k, h).T, vel, mass, 1.0, 0.01, True, galaxy)[2]
        dn = oracle_mod.energy(pos @ rotation(k, -h).T, vel, mass, 1.0, 0.01, True, galaxy)[2]
        T[k] = -(up - dn) / (2 * h)
    return T


def test_torque_is_minus_rotation_derivative_of_external_energy(oracle_mod):
    for galaxy in (None, GAL_BH):
        pos, vel, mass = off_axis_tracers()
        e = oracle_mod.energy(pos, vel, mass, 1.0, 0.01, True, galaxy)
        T_fd = rotation_derivative_torque(oracle_mod, pos, vel, mass, galaxy)
        # the disk flattens the potential: torques about x and y are O(1), about z exactly 0
        assert np.abs(T_fd[:2]).min() > 1e-3
        assert np.abs(e[10:13] - T_fd).max() <= 1e-7 * np.abs(T_fd).max()


def test_torque_per_tracer_and_spherical_limit(oracle_mod):
    """One tracer at a time (the sign and index of every component are exposed), and a spherical
    galaxy (no disk) in which the torque vanishes about every axis."""
    pos, vel, mass = off_axis_tracers(4, 8)
    for i in range(4):
        sl = slice(i, i + 1)
        e = oracle_mod.energy(pos[sl], vel[sl], mass[sl], 1.0, 0.0, True)
        T_fd = rotation_derivative_torque(oracle_mod, pos[sl], vel[sl], mass[sl], None)
        assert np.abs(e[10:13] - T_fd).max() <= 1e-7 * np.abs(T_fd).max()
    sphere = (1.0, 0.7, 0.0, 3.0, 0.28, 0.7, 12.0)
    e = oracle_mod.energy(pos, vel, mass, 1.0, 0.0, True, sphere)
    assert np.abs(e[10:13]).max() <= 1e-15 * np.abs(pos).max() * mass.sum()


def test_torque_is_rate_of_angular_momentum(oracle_mod):
    """dL/dt = torque: central difference of L over one short sym6 step forward and one backward
    from the same state, for an interacting cluster on an inclined orbit in the field."""
    pos, vel, mass = inputs.plummer(48, 77)
    pos = pos * 0.5 + np.array([6.0, 1.0, 1.5])
    vel = vel * 0.5 + np.array([0.1, 0.6, 0.2])
    eps = 0.05
    acc = oracle_mod.total_accel(pos, mass, 1.0, eps, True)
    h = 1e-3
    p1, v1, _ = oracle_mod.step(pos, vel, mass, acc, h, 1, "sym6", 1.0, eps, True)
    p0, v0, _ = oracle_mod.step(pos, vel, mass, acc, -h, 1, "sym6", 1.0, eps, True)
    L1 = oracle_mod.energy(p1, v1, mass, 1.0, eps, True)[7:10]
    L0 = oracle_mod.energy(p0, v0, mass, 1.0, eps, True)[7:10]
    T = oracle_mod.energy(pos, vel, mass, 1.0, eps, True)[10:13]
    dLdt = (L1 - L0) / (2 * h)
    assert np.abs(T[:2]).min() > 1e-2  # T_z = 0: the field is axisymmetric
    assert np.abs(dLdt - T).max() <= 1e-6 * np.abs(T).max()


def test_momentum_moves_centre_of_mass(oracle_mod):
    """P = M dX_cm/dt with distinct bulk velocities per axis (no field: P is conserved, so the
    centre of mass moves uniformly and the relation holds over any interval)."""
    pos, vel, mass = inputs.plummer(64, 31, salpeter=True)
    V = np.array([0.3, -0.7, 1.1])
    vel = vel + V
    eps = 0.02
    e = oracle_mod.energy(pos, vel, mass, 1.0, eps)
    acc = oracle_mod.total_accel(pos, mass, 1.0, eps)
    t = 0.25
    p1, _, _ = oracle_mod.step(pos, vel, mass, acc, t / 64, 64, "leapfrog", 1.0, eps)
    M = mass.sum()
    dX = ((mass[:, None] * p1).sum(0) - (mass[:, None] * pos).sum(0)) / M
    assert np.abs(e[4:7] - M * dX / t).max() <= 1e-12
    assert np.abs(e[4:7] - M * V).max() <= 1e-12  # the Plummer generator leaves zero CoM velocity


def test_internal_force_sum(oracle_mod):
    """sum m a_int = 0 to rounding; two bodies: sum m |a_int| = 2 G m1 m2 r / (r^2 + eps^2)^{3/2}."""
    pos, vel, mass = inputs.plummer(200, 12, salpeter=True)
    for eps in (0.0, 1e-3):
        e = oracle_mod.energy(pos, vel, mass, 1.0, eps, True)
        assert e[18] > 0
        assert e[17] <= 1e-14 * e[18]
        assert abs(e[17] - np.linalg.norm(e[14:17])) <= 1e-30 + 1e-15 * e[17]
    m = np.array([0.25, 1.5])
    p = np.array([[0.1, -0.2, 0.3], [0.7, 0.4, -0.5]])
    r = np.linalg.norm(p[1] - p[0])
    for eps, G in ((0.0, 1.0), (0.3, 2.5)):
        e = oracle_mod.energy(p, np.zeros((2, 3)), m, G, eps)
        ref = 2 * G * m[0] * m[1] * r / (r * r + eps * eps) ** 1.5
        assert abs(e[18] - ref) <= 1e-15 * ref
