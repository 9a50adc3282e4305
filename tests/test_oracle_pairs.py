"""Pins for the oracle's pair sum (Sect. 2, Eqs. 2, 4, 5) against facts other than itself:
40-digit Decimal brute force, two-body closed form, momentum and angular-momentum conservation of
the internal forces (the antisymmetry stated after Eq. 2)."""
import decimal
from decimal import Decimal

import numpy as np
import pytest

from paper_1003_3896_amd import inputs


def _brute_decimal(pos, mass, G, eps, prec=40):
    """a_i = G sum_{j != i} m_j d_ij / (|d|^2 + eps^2)^{3/2}, phi_i = -G sum m_j / sqrt(|d|^2+eps^2),
    evaluated in 40-digit decimal arithmetic from the exact binary inputs."""
    ctx = decimal.Context(prec=prec)
    n = len(mass)
    P = [[Decimal(float(v)) for v in row] for row in pos]
    Mm = [Decimal(float(v)) for v in mass]
    e2 = Decimal(float(eps)) * Decimal(float(eps))
    Gd = Decimal(float(G))
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    for i in range(n):
        a = [Decimal(0)] * 3
        p = Decimal(0)
        for j in range(n):
            if j == i:
                continue
            d = [ctx.subtract(P[j][c], P[i][c]) for c in range(3)]
            r2 = ctx.add(ctx.add(ctx.add(ctx.multiply(d[0], d[0]), ctx.multiply(d[1], d[1])),
                                 ctx.multiply(d[2], d[2])), e2)
            inv = ctx.divide(Decimal(1), ctx.sqrt(r2))
            inv3 = ctx.multiply(ctx.multiply(inv, inv), inv)
            for c in range(3):
                a[c] = ctx.add(a[c], ctx.multiply(ctx.multiply(Mm[j], d[c]), inv3))
            p = ctx.add(p, ctx.multiply(Mm[j], inv))
        acc[i] = [float(ctx.multiply(Gd, a[c])) for c in range(3)]
        pot[i] = float(-ctx.multiply(Gd, p))
    return acc, pot


@pytest.mark.parametrize("n", [2, 3, 5, 8])
@pytest.mark.parametrize("eps", [0.0, 1e-3, 0.3])
@pytest.mark.parametrize("seed", [11, 12])
def test_brute_force_decimal(oracle_mod, n, eps, seed):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-1, 1, (n, 3))
    mass = rng.uniform(0.1, 2.0, n)
    G = 1.0 if seed == 11 else 0.75
    ref_a, ref_p = _brute_decimal(pos, mass, G, eps)
    a, p, absa = oracle_mod.accel(pos, mass, G, eps, want_pot=True, want_abs=True)
    # error relative to the sum of magnitudes: conditioning-independent bound for a correct sum
    err = np.linalg.norm(a - ref_a, axis=1) / absa
    assert err.max() <= 2e-15, err
    assert np.abs(p - ref_p).max() <= 2e-15 * np.abs(ref_p).max()


def test_two_body_closed_form(oracle_mod):
    """Two bodies: a_1 = G m_2 d / (d^2 + eps^2)^{3/2}, a_2 = -G m_1 d / (...)."""
    for eps in (0.0, 0.01, 1.0):
        x = np.array([[0.1, -0.2, 0.3], [0.4, 0.5, -0.6]])
        m = np.array([0.25, 0.75])
        G = 2.0
        d = x[1] - x[0]
        r2 = d @ d + eps * eps
        a = oracle_mod.accel(x, m, G, eps)
        np.testing.assert_allclose(a[0], G * m[1] * d / r2 ** 1.5, rtol=1e-15)
        np.testing.assert_allclose(a[1], -G * m[0] * d / r2 ** 1.5, rtol=1e-15)
        a, p = oracle_mod.accel(x, m, G, eps, want_pot=True)
        np.testing.assert_allclose(p, [-G * m[1] / np.sqrt(r2), -G * m[0] / np.sqrt(r2)], rtol=1e-15)


def test_self_term_absent(oracle_mod):
    """A single particle feels nothing and has zero pair potential, for any eps (j != i)."""
    for eps in (0.0, 1e-4, 1.0):
        a, p = oracle_mod.accel(np.array([[1.0, 2.0, 3.0]]), np.array([1.0]), 1.0, eps, want_pot=True)
        assert np.all(a == 0) and np.all(p == 0)


@pytest.mark.parametrize("eps", [0.0, 1e-3])
def test_momentum_and_angular_momentum_conservation(oracle_mod, eps):
    """F_ij = -F_ji: sum_i m_i a_i = 0 and sum_i m_i x_i x a_i = 0 for internal central forces."""
    pos, vel, mass = inputs.plummer(512, 77, salpeter=True)
    a, absa = oracle_mod.accel(pos, mass, 1.0, eps, want_abs=True)
    scale = (mass * absa).sum()
    assert np.abs((mass[:, None] * a).sum(0)).max() / scale < 1e-13
    tq = (mass[:, None] * np.cross(pos, a)).sum(0)
    assert np.abs(tq).max() / (mass * absa * np.linalg.norm(pos, axis=1)).sum() < 1e-13


def test_row_range_matches_full(oracle_mod):
    pos, _, mass = inputs.uniform_box(300, 5)
    full = oracle_mod.accel(pos, mass, 1.0, 1e-2)
    part = oracle_mod.accel(pos, mass, 1.0, 1e-2, rows=(37, 211))
    assert np.array_equal(full[37:211], part)


def test_translation_invariance(oracle_mod):
    """Accelerations depend only on differences: shifting by a power of two changes nothing beyond
    the rounding of the shifted coordinates."""
    pos, _, mass = inputs.uniform_box(200, 6)
    a0, absa = oracle_mod.accel(pos, mass, 1.0, 1e-3, want_abs=True)
    a1 = oracle_mod.accel(pos + 4.0, mass, 1.0, 1e-3)
    err = np.linalg.norm(a1 - a0, axis=1) / absa
    assert err.max() < 1e-12


def test_plummer_mean_field(oracle_mod):
    """Statistical sanity: the radial acceleration of a Plummer sphere follows
    -G M r / (r^2 + a^2)^{3/2} to O(N^-1/2) (a check of inputs + oracle together, loose)."""
    pos, _, mass = inputs.plummer(4096, 99)
    a = oracle_mod.accel(pos, mass, 1.0, 1e-2)
    r = np.linalg.norm(pos, axis=1)
    ar = -(a * pos).sum(1) / np.maximum(r, 1e-12)
    A = inputs.PLUMMER_A
    model = r / (r * r + A * A) ** 1.5
    sel = (r > 0.3) & (r < 3.0)
    rel = np.median(np.abs(ar[sel] - model[sel]) / model[sel])
    assert rel < 0.1
