"""The oracle's pins are strong enough: plant a plausible mistake in a COPY of the oracle source
(on the CPU, never in the HIP path), rebuild it, and check that at least one pin rejects it."""
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1003_3896_amd import inputs

SRC = os.path.join(os.path.dirname(oracle.__file__), "nbody_oracle.c")

# (name, original text, planted mistake)
MUTANTS = [
    ("dx-sign", "const double dx = pos[3 * j] - xi;", "const double dx = xi - pos[3 * j];"),
    ("softening-dropped", "dz * dz + e2;", "dz * dz;"),
    ("wrong-power", "const double inv3 = inv * inv * inv;", "const double inv3 = inv * inv;"),
    ("self-term-kept", "if (j == i) continue;", "if (j == i && e2 == 0.0) continue;"),
    ("y-uses-x", "const double dy = pos[3 * j + 1] - yi;", "const double dy = pos[3 * j] - yi;"),
    ("kick-unmerged", "kick8[k] = 0.5 * (w[k - 1] + w[k]);", "kick8[k] = w[k];"),
    ("coef-digit", "W2 = 0.235573213359357;", "W2 = 0.235573213359957;"),
    ("drift-uses-acc", "pos[i] = pos[i] + c * vel[i];", "pos[i] = pos[i] + c * vel[i] * 0.999999;"),
    ("disk-exponent", "const double D3 = D2 * D;", "const double D3 = D2 * D2;"),
    ("disk-z-factor", "G * Md * As / (D3 * s);", "G * Md / (D3 * s);"),
    ("halo-sign", "ph = 0.5 * vh * vh * log(r2 + dh * dh);", "ph = -0.5 * vh * vh * log(r2 + dh * dh);"),
    ("energy-half-missing", "nsum_add(&W, 0.5 * m * pot[i]);", "nsum_add(&W, m * pot[i]);"),
    ("kinetic-half-missing", "nsum_add(&K, 0.5 * m * (v[0]", "nsum_add(&K, 1.0 * m * (v[0]"),
    ("L-index", "nsum_add(&L[2], m * (x[0] * v[1] - x[1] * v[0]));", "nsum_add(&L[2], m * (x[0] * v[1] - x[1] * v[1]));"),
    ("last-kick-missing", "kick(n, vel, acc, Kc[stages] * dt);", ";"),
    ("bh-power", "G * Mbh / (q2 * sqrt(q2))", "G * Mbh / q2"),
    ("bh-softening-dropped", "const double q2 = r2 + ebh * ebh;", "const double q2 = r2;"),
    ("torque-sign", "nsum_add(&T[0], m * (x[1] * ae[2] - x[2] * ae[1]));",
     "nsum_add(&T[0], m * (x[2] * ae[1] - x[1] * ae[2]));"),
    ("torque-index", "nsum_add(&T[1], m * (x[2] * ae[0] - x[0] * ae[2]));",
     "nsum_add(&T[1], m * (x[2] * ae[0] - x[0] * ae[1]));"),
    ("momentum-index", "nsum_add(&P[c], m * v[c]);", "nsum_add(&P[c], m * v[0]);"),
    ("force-sum-mass-dropped", "nsum_add(&F[c], m * a[c]);", "nsum_add(&F[c], a[c]);"),
    ("force-abs-mass-dropped", "nsum_add(&A, m * sqrt(", "nsum_add(&A, sqrt("),
    ("as91-halo-mass-power", "return Mh * (s / ah) * q / (1.0 + q);", "return Mh * q / (1.0 + q);"),
    ("as91-bulge-power", "gb = G * Mb / pow(r2 + ab * ab, 1.5);", "gb = G * Mb / pow(r2 + ab * ab, 1.0);"),
    ("as91-halo-potential-term", "return log(1.0 + q) - 1.02 / (1.0 + q);", "return log(1.0 + q) - 1.0 / (1.0 + q);"),
    ("as91-beyond-cutoff", "ph = -G * as91_halo_mass(rcut, Mh, ah, rcut) / r;",
     "ph = -G * as91_halo_mass(rcut, Mh, ah, rcut) / rcut;"),
]


def _pins():
    """A compact run of the pins from the other oracle test files; returns names of failures."""
    from test_oracle_pairs import _brute_decimal
    from test_oracle_integrators import kepler_error, two_body
    fails = []
    rng = np.random.default_rng(1)
    pos = rng.uniform(-1, 1, (5, 3))
    mass = rng.uniform(0.1, 2, 5)
    for eps in (0.0, 1e-3):
        ra, rp = _brute_decimal(pos, mass, 1.0, eps)
        a, p, absa = oracle.accel(pos, mass, 1.0, eps, want_pot=True, want_abs=True)
        if not (np.linalg.norm(a - ra, axis=1) / np.maximum(absa, 1e-300)).max() <= 2e-15:
            fails.append("brute-accel")
        if not np.abs(p - rp).max() <= 2e-15 * np.abs(rp).max():
            fails.append("brute-pot")
    d, k = oracle.sym6_coefficients()
    if abs((d ** 3).sum()) > 1e-13 or abs((d ** 5).sum()) > 1e-13 or abs(k.sum() - 1) > 1e-15:
        fails.append("sym6-identities")
    errs = [kepler_error(oracle, "sym6", n) for n in (128, 256, 512, 1024)]
    s = np.polyfit(np.log([1 / 128, 1 / 256, 1 / 512, 1 / 1024]), np.log(np.maximum(errs, 1e-300)), 1)[0]
    if abs(s - 6) > 0.3 or errs[-1] > 1e-10:
        fails.append("sym6-order")
    errs = [kepler_error(oracle, "leapfrog", n) for n in (256, 512, 1024, 2048)]
    s = np.polyfit(np.log([1 / 256, 1 / 512, 1 / 1024, 1 / 2048]), np.log(np.maximum(errs, 1e-300)), 1)[0]
    if abs(s - 2) > 0.1:
        fails.append("leapfrog-order")
    # field: finite differences, closed-form circular speed
    pts = rng.uniform(-10, 10, (12, 3))
    a, _ = oracle.ext_field(pts)
    h = 1e-5
    fd = np.zeros_like(pts)
    for c in range(3):
        dp = np.zeros(3)
        dp[c] = h
        fd[:, c] = -(oracle.ext_field(pts + dp)[1] - oracle.ext_field(pts - dp)[1]) / (2 * h)
    if (np.linalg.norm(a - fd, axis=1) / np.linalg.norm(a, axis=1)).max() > 1e-8:
        fails.append("field-fd")
    # the central point mass: closed form and finite differences
    gal = (0.0, 1.0, 0.0, 1.0, 1.0, 0.0, 1.0, 7.0, 0.05)
    xb = rng.uniform(-0.3, 0.3, (6, 3))
    ab, pb = oracle.ext_field(xb, galaxy=gal)
    q2 = (xb * xb).sum(1) + 0.0025
    if np.abs(pb + 7.0 / np.sqrt(q2)).max() > 1e-13 or np.abs(ab + 7.0 * xb / (q2 ** 1.5)[:, None]).max() > 1e-11:
        fails.append("bh-closed-form")
    a8, _ = oracle.ext_field(np.array([[8.0, 0, 0]]))
    if abs(math.sqrt(8 * abs(a8[0, 0])) - inputs.V_CIRC_8) > 1e-12:
        fails.append("field-vc")
    # energy closed form for two bodies, with and without softening
    p2, v2, m2 = two_body()
    for eps in (0.0, 0.1):
        e = oracle.energy(p2, v2, m2, 1.0, eps)
        r = np.linalg.norm(p2[1] - p2[0])
        K = 0.5 * (m2 * (v2 ** 2).sum(1)).sum()
        W = -m2[0] * m2[1] / math.sqrt(r * r + eps * eps)
        L = (m2[:, None] * np.cross(p2, v2)).sum(0)
        if abs(e[0] - K) > 1e-15 or abs(e[1] - W) > 1e-15 or np.abs(e[7:10] - L).max() > 1e-15:
            fails.append("energy-closed-form")
    # angular momentum and momentum are conserved by the integrators for central pair forces
    p3, v3, m3 = inputs.plummer(16, 3)
    v3 = v3 + np.array([0.1, -0.2, 0.05])
    e0 = oracle.energy(p3, v3, m3, 1.0, 0.05)
    acc = oracle.total_accel(p3, m3, 1.0, 0.05)
    p4, v4, _ = oracle.step(p3, v3, m3, acc, 1.0 / 128, 20, "sym6", 1.0, 0.05)
    e1 = oracle.energy(p4, v4, m3, 1.0, 0.05)
    if np.abs(e1[7:10] - e0[7:10]).max() > 1e-13 * np.abs(e0[7:10]).max():
        fails.append("L-conservation")
    # torque against the rotation derivative of U_ext; momentum against the centre-of-mass drift;
    # the internal force sum (zero, and its two-body magnitude)
    from test_oracle_energy import off_axis_tracers, rotation_derivative_torque
    pt, vt, mt = off_axis_tracers()
    et = oracle.energy(pt, vt, mt, 1.0, 0.01, True)
    tfd = rotation_derivative_torque(oracle, pt, vt, mt, None)
    if np.abs(et[10:13] - tfd).max() > 1e-7 * np.abs(tfd).max():
        fails.append("torque-rotation")
    p5, v5, m5 = inputs.plummer(32, 31, salpeter=True)
    v5 = v5 + np.array([0.3, -0.7, 1.1])
    e5 = oracle.energy(p5, v5, m5, 1.0, 0.02)
    p6, _, _ = oracle.step(p5, v5, m5, oracle.total_accel(p5, m5, 1.0, 0.02), 1.0 / 64, 16, "leapfrog", 1.0, 0.02)
    dX = ((m5[:, None] * p6).sum(0) - (m5[:, None] * p5).sum(0)) / 0.25
    if np.abs(e5[4:7] - dX).max() > 1e-12:
        fails.append("momentum-centre-of-mass")
    if not (e5[18] > 0 and e5[17] <= 1e-14 * e5[18]):
        fails.append("force-sum-zero")
    e2b = oracle.energy(p2, v2, m2, 1.0, 0.1)
    r = np.linalg.norm(p2[1] - p2[0])
    if abs(e2b[18] - 2 * m2[0] * m2[1] * r / (r * r + 0.01) ** 1.5) > 1e-15:
        fails.append("force-abs-closed-form")
    # the Allen & Santillan Galaxy: its published circular speed, escape speed and total mass, and
    # -grad Phi by central differences inside and beyond the halo cut-off
    from test_oracle_field import _as91
    g, gal = _as91()
    a0, ph0 = oracle.ext_field(np.array([[g["R0"], 0.0, 0.0]]), galaxy=gal)
    if abs(math.sqrt(max(-a0[0, 0] * g["R0"], 0.0)) - g["vc0"]) > 0.05:
        fails.append("as91-circular-speed")
    if abs(math.sqrt(max(-2.0 * ph0[0], 0.0)) - g["vesc0"]) > 0.1:
        fails.append("as91-escape-speed")
    _, phf = oracle.ext_field(np.array([[1e6, 0.0, 0.0]]), galaxy=gal)
    if abs(-1e6 * phf[0] * g["mass_unit_msun"] / g["mtot_msun"] - 1.0) > 0.005:
        fails.append("as91-total-mass")
    pts = np.array([[0.3, 0.2, 0.1], [8.5, 0.0, 0.3], [40.0, -20.0, 5.0], [150.0, 30.0, -60.0]])
    aa, _ = oracle.ext_field(pts, galaxy=gal)
    fd = np.zeros_like(pts)
    for c in range(3):
        dp = np.zeros(3)
        dp[c] = 1e-5
        fd[:, c] = -(oracle.ext_field(pts + dp, galaxy=gal)[1] - oracle.ext_field(pts - dp, galaxy=gal)[1]) / 2e-5
    if (np.linalg.norm(aa - fd, axis=1) / np.linalg.norm(aa, axis=1)).max() > 1e-7:
        fails.append("as91-gradient")
    return fails


def test_unmutated_oracle_passes_all_pins(oracle_mod):
    assert _pins() == []


@pytest.mark.parametrize("name,orig,bad", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, oracle_mod, name, orig, bad):
    src = open(SRC).read()
    assert src.count(orig) == 1, "mutation anchor not unique: " + orig
    path = tmp_path / ("mutant_%s.c" % name)
    path.write_text(src.replace(orig, bad))
    lib = tmp_path / ("mutant_%s.so" % name)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-o",
                           str(lib), str(path), "-lm"])
    with oracle.use_library(str(lib)):
        fails = _pins()
    assert fails, "planted mistake %s was not caught by any pin" % name
