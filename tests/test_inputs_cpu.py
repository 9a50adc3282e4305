"""The paper's timing set-up generator (Sect. 3 and 5): a uniform sphere with virial ratio 0.3,
checked against closed forms of a uniform ball and against the oracle's potential energy."""
import math

import numpy as np

import oracle
from paper_1003_3896_amd import inputs


def test_uniform_sphere_geometry_and_kinetic_energy():
    n = 20000
    p, v, m = inputs.uniform_sphere(n, 11)
    r = np.linalg.norm(p, axis=1)
    assert r.max() <= 1.0 + 0.02                       # inside R = 1 (up to the centre-of-mass shift)
    # r^3 of a uniform ball is uniform on [0, 1]: mean 1/2, variance 1/12
    assert abs(np.mean(r ** 3) - 0.5) < 4 * math.sqrt(1 / 12 / n)
    assert np.allclose(m, 1.0 / n) and abs(m.sum() - 1.0) < 1e-12
    assert np.abs(p.mean(axis=0)).max() < 1e-15 and np.abs(v.mean(axis=0)).max() < 1e-15
    k = 0.5 * (m[:, None] * v * v).sum()
    assert abs(k - 0.5 * 0.3 * 0.6) < 1e-12           # K = q |W_continuum| / 2
    # isotropic velocities: each axis carries a third of the kinetic energy
    for d in range(3):
        assert abs((m * v[:, d] ** 2).sum() / (2 * k) - 1 / 3) < 0.02


def test_uniform_sphere_virial_ratio_from_the_oracle():
    """2K / |W| with the oracle's pair-sum potential is 0.3 up to the discreteness of N."""
    n = 3000
    p, v, m = inputs.uniform_sphere(n, 12)
    e = oracle.energy(p, v, m, 1.0, 0.005 / n ** (1 / 3), False)
    q = 2 * e[0] / abs(e[1])
    assert abs(q - 0.3) < 0.02, q


def test_paper_timing_batch():
    b = inputs.paper_timing(480)
    assert b.n == 480 and b.B == 1 and bool(b.field[0])
    assert abs(b.eps[0] - 0.005 / 480 ** (1 / 3)) < 1e-15
    assert b.meta["dt"] == 5e-4 and b.meta["integrator"] == "leapfrog"
    assert inputs.PAPER_SIZES[0] == 480 and inputs.PAPER_SIZES[-1] == 1536000
    cm = (b.mass[:, None] * b.pos).sum(axis=0)
    assert abs(cm[0] - 8.0) < 1e-12 and abs(cm[1]) < 1e-12


def test_black_hole_set_up():
    """Table 8's start: barycentre at (10, 0, 0) with 0.001 of the local circular speed, the point
    mass in cluster-mass units at the galaxy centre; V_CIRC_10 is the galaxy's circular speed."""
    a, _ = oracle.ext_field(np.array([[10.0, 0.0, 0.0]]))
    assert abs(math.sqrt(10 * abs(a[0, 0])) - inputs.V_CIRC_10) < 1e-12
    b = inputs.paper_black_hole(50.0, n=960)
    cm = (b.mass[:, None] * b.pos).sum(axis=0)
    vcm = (b.mass[:, None] * b.vel).sum(axis=0)
    assert abs(cm[0] - 10.0) < 1e-12 and abs(vcm[1] - 0.001 * inputs.V_CIRC_10) < 1e-15
    assert b.galaxy[:7] == inputs.GALAXY and b.galaxy[7] == 50.0 and b.galaxy[8] == b.eps[0]
    assert b.meta["integrator"] == "sym6" and b.meta["dt"] == 1e-4 and b.meta["steps"] == 40000


def test_allen_santillan_parameters_match_the_fixture(oracle_mod):
    """The generator's Allen & Santillan parameter tuple is the one the oracle's pins use, and its
    solar-circle speed is the oracle's circular speed there."""
    from test_oracle_field import _as91
    g, gal = _as91()
    assert tuple(inputs.ALLEN_SANTILLAN) == tuple(gal)
    a, _ = oracle_mod.ext_field(np.array([[inputs.AS91_SUN_R, 0.0, 0.0]]), galaxy=inputs.ALLEN_SANTILLAN)
    assert abs(np.sqrt(-a[0, 0] * inputs.AS91_SUN_R) - inputs.AS91_SUN_VC) < 0.05
