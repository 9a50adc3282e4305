"""Seeded synthetic inputs shared by the HIP path and the oracle.

Pure NumPy sampling of initial conditions; it holds none of the method's arithmetic (no force,
potential or integration code) and imports neither the HIP binding nor the oracle.

* Plummer spheres in Henon units (G = M = 1, E = -1/4 in expectation, scale a = 3 pi / 16),
  sampled as in Aarseth, Henon & Wielen (1974): radius from the inverse cumulative mass profile
  (mass fractions above 0.999 rejected, i.e. r < 38.7 a), isotropic directions, speeds by
  rejection on q^2 (1 - q^2)^{7/2}.  Centre-of-mass position and velocity are then set to zero.
  No rescaling to an exact energy is done here: that would need the potential energy, which
  belongs to the method.
* Salpeter (1955) masses dN/dm ~ m^-2.35 on [0.1, 100] by inverse-CDF sampling, normalised to a
  total mass of 1, drawn independently of position.
* The workloads the benchmarks and tests use (cluster sizes, softening, time step, galaxy orbit).

Every generator takes an integer seed and uses ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

PLUMMER_A = 3.0 * math.pi / 16.0

# Galaxy parameters {Mb, ab, Md, ad, bd, vh, dh} (G = 1): Hernquist bulge, Miyamoto-Nagai disk,
# logarithmic halo, chosen so that a circular orbit at R = 8 has a period of about 60 time units.
GALAXY = (1.0, 0.7, 4.5, 3.0, 0.28, 0.7, 12.0)
# circular speed of that model at (8, 0, 0): sqrt(R |a_R|); pinned against the oracle's field
V_CIRC_8 = 0.837866164494
V_CIRC_10 = 0.821107211916  # circular speed of the same galaxy at R = 10
ORBIT_R = 8.0

# The Allen & Santillan (1991) Galaxy that Sect. 3 names, as the library's second galaxy model:
# (Mb, ab, Md, ad, bd, vh, dh, Mbh, ebh, model, Mh, ah, rcut) with its published parameters in its
# own units (length kpc, mass 2.32e7 solar masses, G = 1, so velocities in units of 10 km/s):
# spherical bulge, Miyamoto-Nagai disk, spherical halo cut off at 100 kpc (vh, dh unused).
ALLEN_SANTILLAN = (606.0, 0.3873, 3690.0, 5.3178, 0.25, 0.0, 1.0, 0.0, 0.0, 1.0, 4615.0, 12.0, 100.0)
AS91_SUN_R = 8.5      # the solar radius of that model (kpc)
AS91_SUN_VC = 22.0    # its circular speed there (220 km/s), pinned against the oracle's field

DT_DEFAULT = 2.0 ** -11


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _isotropic(rng: np.random.Generator, r: np.ndarray) -> np.ndarray:
    n = r.shape[0]
    z = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * s * np.cos(ph), r * s * np.sin(ph), r * z], axis=1)


def salpeter_masses(n: int, rng: np.random.Generator, alpha: float = 2.35, mlo: float = 0.1,
                    mhi: float = 100.0) -> np.ndarray:
    """Masses from dN/dm ~ m^-alpha on [mlo, mhi] (inverse CDF), normalised to sum 1."""
    k = 1.0 - alpha
    u = rng.uniform(0.0, 1.0, n)
    m = (mlo ** k + u * (mhi ** k - mlo ** k)) ** (1.0 / k)
    return m / m.sum()


def plummer(n: int, seed: int, masses: Optional[np.ndarray] = None, a: float = PLUMMER_A,
            G: float = 1.0, M: float = 1.0, salpeter: bool = False):
    """Plummer sphere of n particles; returns (pos (n,3), vel (n,3), mass (n,)) as float64.

    Draw order from the seeded stream: radii, position directions, speeds (rejection), velocity
    directions, then Salpeter masses if asked.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = _rng(seed)
    # radii: mass fraction X -> r = a (X^(-2/3) - 1)^(-1/2), reject X > 0.999
    X = np.empty(0)
    while X.size < n:
        x = rng.uniform(0.0, 1.0, 2 * n)
        x = x[(x > 0.0) & (x <= 0.999)]
        X = np.concatenate([X, x])
    X = X[:n]
    r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    pos = _isotropic(rng, r)
    # speeds: q with density ~ q^2 (1 - q^2)^3.5 by rejection (max of that density < 0.1)
    q = np.empty(0)
    while q.size < n:
        x4 = rng.uniform(0.0, 1.0, 2 * n)
        x5 = rng.uniform(0.0, 1.0, 2 * n)
        q = np.concatenate([q, x4[0.1 * x5 < x4 * x4 * (1.0 - x4 * x4) ** 3.5]])
    q = q[:n]
    vesc = math.sqrt(2.0 * G * M / a) * (1.0 + (r / a) ** 2) ** -0.25
    vel = _isotropic(rng, q * vesc)
    if masses is None:
        mass = salpeter_masses(n, rng) * M if salpeter else np.full(n, M / n)
    else:
        mass = np.asarray(masses, dtype=np.float64)
    msum = mass.sum()
    pos -= (mass[:, None] * pos).sum(axis=0) / msum
    vel -= (mass[:, None] * vel).sum(axis=0) / msum
    return np.ascontiguousarray(pos), np.ascontiguousarray(vel), np.ascontiguousarray(mass)


def uniform_sphere(n: int, seed: int, q: float = 0.3, R: float = 1.0, G: float = 1.0, M: float = 1.0):
    """Equal-mass particles uniform in a sphere of radius R, velocities isotropic with speeds
    uniform in [0, 1), rescaled so that the virial ratio 2K/|W| equals q (Sect. 3's set-up).

    The potential energy of the rescaling is the continuum value W = -3 G M^2 / (5 R) of a uniform
    sphere (a closed form, not a pair sum).  Draw order: radii, position directions, speeds,
    velocity directions.  Centre of mass at rest at the origin.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = _rng(seed)
    r = R * rng.uniform(0.0, 1.0, n) ** (1.0 / 3.0)
    pos = _isotropic(rng, r)
    vel = _isotropic(rng, rng.uniform(0.0, 1.0, n))
    mass = np.full(n, M / n)
    pos -= pos.mean(axis=0)
    vel -= vel.mean(axis=0)
    k = 0.5 * (mass[:, None] * vel * vel).sum()
    k_target = 0.5 * q * 0.6 * G * M * M / R
    if k > 0.0:
        vel *= math.sqrt(k_target / k)
    return np.ascontiguousarray(pos), np.ascontiguousarray(vel), mass


def paper_timing(n: int, seed: int = 7000):
    """The timing set-up of Sect. 5: the uniform sphere with q = 0.3, eps = 0.005 R / N^(1/3), on a
    circular orbit in the galaxy, leapfrog with dt = 5e-4 crossing times (seed 7000 + n)."""
    p, v, m = uniform_sphere(n, seed + n)
    p, v = on_orbit(p, v)
    return single(p, v, m, 0.005 / n ** (1.0 / 3.0), True, name="uniform-sphere-q0.3-%d" % n,
                  integrator="leapfrog", steps=1000, dt=5e-4)


PAPER_SIZES = [480 * 2 ** k for k in range(12)] + [1536000]  # 480 .. 983040, then 1,536,000
BH_RATIOS = (0.1, 1.0, 50.0, 105.0)  # black-hole to cluster mass ratios of Table 8


def paper_black_hole(ratio: float, n: int = 15360, seed: int = 8000):
    """The collision set-up of Sect. 6.2 (Table 8): the uniform sphere with q = 0.3 and
    eps = 0.005 / N^(1/3), centre of mass at (10, 0, 0) moving at (0, 0.001 v_c, 0), in the galaxy
    with a point mass of `ratio` cluster masses at its centre (softened like a star); sym6 with
    dt = 1e-4 (4e4 steps cover t = [0, 4])."""
    p, v, m = uniform_sphere(n, seed + n)
    p, v = on_orbit(p, v, R=10.0, vc=0.001 * V_CIRC_10)
    eps = 0.005 / n ** (1.0 / 3.0)
    b = single(p, v, m, eps, True, name="black-hole-%g-uniform-sphere-%d" % (ratio, n), integrator="sym6",
               steps=40000, dt=1e-4)
    b.galaxy = GALAXY + (float(ratio), eps)  # the cluster mass is 1
    return b


def uniform_box(n: int, seed: int, scale: float = 1.0, mass_range=(0.5, 1.5)):
    """Uniform random positions in a cube, random masses: generic parity-test input."""
    rng = _rng(seed)
    pos = rng.uniform(-scale, scale, (n, 3))
    vel = rng.uniform(-0.5, 0.5, (n, 3))
    mass = rng.uniform(mass_range[0], mass_range[1], n)
    mass /= mass.sum()
    return pos, vel, mass


# --------------------------------------------------------------------------------------------
# Workloads


@dataclass
class Batch:
    """A ragged batch: clusters concatenated; offsets has B+1 entries."""
    pos: np.ndarray
    vel: np.ndarray
    mass: np.ndarray
    offsets: np.ndarray
    eps: np.ndarray
    field: np.ndarray
    G: float = 1.0
    galaxy: tuple = GALAXY
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.offsets[-1])

    @property
    def B(self) -> int:
        return len(self.offsets) - 1

    def interactions_per_eval(self) -> int:
        sz = np.diff(self.offsets).astype(np.int64)
        return int((sz * sz).sum())


def single(pos, vel, mass, eps, field_on=False, **meta) -> Batch:
    n = pos.shape[0]
    return Batch(pos, vel, mass, np.array([0, n], np.int64), np.array([eps], np.float64),
                 np.array([1 if field_on else 0], np.uint8), meta=dict(meta))


def concat(clusters: List[Batch]) -> Batch:
    pos = np.concatenate([c.pos for c in clusters])
    vel = np.concatenate([c.vel for c in clusters])
    mass = np.concatenate([c.mass for c in clusters])
    sizes = [c.n for c in clusters]
    offsets = np.zeros(len(sizes) + 1, np.int64)
    offsets[1:] = np.cumsum(sizes)
    eps = np.concatenate([c.eps for c in clusters])
    fld = np.concatenate([c.field for c in clusters])
    return Batch(pos, vel, mass, offsets, eps, fld)


def on_orbit(pos, vel, R: float = ORBIT_R, vc: float = V_CIRC_8):
    """Place a cluster's centre of mass at (R,0,0) with velocity (0, vc, 0): a circular planar orbit."""
    pos = pos + np.array([R, 0.0, 0.0])
    vel = vel + np.array([0.0, vc, 0.0])
    return pos, vel


def c1():
    """Plummer N=1024, equal masses, eps=1e-3, no field; 100 leapfrog steps, dt=1/1024, FP64."""
    p, v, m = plummer(1024, 1001)
    return single(p, v, m, 1e-3, False, name="plummer-1024", integrator="leapfrog", steps=100,
                  dt=1.0 / 1024)


def c2(n: int = 65536):
    """Plummer N=65536 with Salpeter masses, eps=1e-4, galaxy field, circular orbit at R=8; sym6."""
    p, v, m = plummer(n, 2002, salpeter=True)
    p, v = on_orbit(p, v)
    return single(p, v, m, 1e-4, True, name="plummer-salpeter-%d-galaxy" % n, integrator="sym6",
                  steps=200, dt=DT_DEFAULT)


def c3(n: int = 262144):
    """Plummer N=262144, equal masses, eps=1e-4, no field; 1000 leapfrog steps, dt=2^-11."""
    p, v, m = plummer(n, 3003)
    return single(p, v, m, 1e-4, False, name="plummer-%d" % n, integrator="leapfrog", steps=1000,
                  dt=DT_DEFAULT)


def c4_sizes(B: int = 512, lo: int = 256, hi: int = 16384, seed: int = 40000) -> np.ndarray:
    rng = _rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), B))).astype(np.int64)


def c4(B: int = 512, lo: int = 256, hi: int = 16384):
    """B independent Plummer clusters, N_c log-uniform in [lo, hi] (seed 4000+c), eps=1e-3; sym6."""
    sizes = c4_sizes(B, lo, hi)
    cl = []
    for c, n in enumerate(sizes):
        p, v, m = plummer(int(n), 4000 + c)
        cl.append(single(p, v, m, 1e-3, False))
    b = concat(cl)
    b.meta = dict(name="ensemble-%d-plummer-%d-%d" % (B, lo, hi), integrator="sym6", steps=100,
                  dt=DT_DEFAULT)
    return b


@dataclass
class Job:
    jid: int
    n: int
    steps: int
    integrator: str
    field: bool
    seed: int
    arrival: float = 0.0
    eps: float = 1e-3
    dt: float = DT_DEFAULT

    def initial_state(self):
        p, v, m = plummer(self.n, self.seed)
        if self.field:
            p, v = on_orbit(p, v)
        return p, v, m

    def evals(self) -> int:
        return self.steps * (1 if self.integrator == "leapfrog" else 7)

    def interactions(self) -> int:
        return self.evals() * self.n * self.n


def c5_jobs(count: int, rate: float, seed: int = 5005, nlo: int = 1024, nhi: int = 65536,
            smin: int = 10, smax: int = 1000) -> List[Job]:
    """Job stream: N log-uniform in [nlo, nhi], steps uniform in [smin, smax], integrator and field
    50/50, Poisson arrivals of the given rate (jobs per second); job j uses seed 5,000,000 + j."""
    rng = _rng(seed)
    jobs = []
    t = 0.0
    for j in range(count):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        n = int(round(math.exp(rng.uniform(math.log(nlo), math.log(nhi)))))
        steps = int(rng.integers(smin, smax + 1))
        integ = "leapfrog" if rng.uniform() < 0.5 else "sym6"
        fld = bool(rng.uniform() < 0.5)
        jobs.append(Job(j, n, steps, integ, fld, 5_000_000 + j, t))
    return jobs
