"""FP64 CPU oracle for the softened direct-summation N-body hot path (NBSymple, Sects. 2-3, 5.1).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import this package.  It shares no code with the HIP library in
``paper_1003_3896_amd`` and neither imports the other; only the seeded input generators
(``paper_1003_3896_amd.inputs``, pure NumPy, none of the method's arithmetic) feed both.

The arithmetic lives in ``nbody_oracle.c`` (plain C, FP64, OpenMP over particles, compiled with
``-O2 -ffp-contract=off``).  This module is argument marshalling plus the per-cluster loop for
ragged batches.

Parity pins (tests/test_oracle_*.py): 40-digit Decimal brute force for N <= 8, two-body closed
forms, momentum conservation, Kepler orbit closed form, h^2 / h^6 convergence slopes, time
reversibility, finite differences of the external potential, circular-velocity closed form.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbody_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

# Galaxy parameters {Mb, ab, Md, ad, bd, vh, dh} (G = 1, Henon units of the cluster):
# Hernquist bulge, Miyamoto-Nagai disk, logarithmic halo.  The paper's Allen & Santillan model is
# named but not printed (Sect. 3); these values give a circular orbit at R = 8 with a period of
# about 60 internal time units, the figure quoted in Sect. 6.1.
GALAXY = (1.0, 0.7, 4.5, 3.0, 0.28, 0.7, 12.0)


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (FP64, no FMA contraction, OpenMP)."""
    with _lock:
        if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            tmp = _LIB + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                                   "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, _LIB)
    return _LIB


def _configure(lib):
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    D = ctypes.c_double
    lib.oracle_accel_range.argtypes = [I64, I64, I64, P, P, D, D, P, P, P]
    lib.oracle_accel.argtypes = [I64, P, P, D, D, P, P, P]
    lib.oracle_ext_field.argtypes = [I64, P, D, P, P, P]
    lib.oracle_energy.argtypes = [I64, P, P, P, D, D, ctypes.c_int, P, P, P]
    lib.oracle_step.argtypes = [I64, P, P, P, P, D, D, ctypes.c_int, P, D, I64, ctypes.c_int]
    lib.oracle_total_accel.argtypes = [I64, P, P, D, D, ctypes.c_int, P, P]
    lib.oracle_sym6_coefficients.argtypes = [P, P]
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


class use_library:
    """Context manager: route this module's calls through another build of the oracle source
    (used by the tests that plant a mistake in a copy of the oracle and check a pin catches it)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _load()
        _lib = _configure(ctypes.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        a = a.reshape(shape)
    return a


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _gal(galaxy):
    """Galaxy parameters as the C side reads them: (Mb, ab, Md, ad, bd, vh, dh, Mbh, ebh, model,
    Mh, ah, rcut); a 7-tuple has no central black hole, and a tuple of 9 or fewer is model 0."""
    g = list(GALAXY if galaxy is None else galaxy)
    return _f64(g + [0.0] * (13 - len(g)))


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_threads(t: int) -> None:
    _load().oracle_set_threads(int(t))


def accel(pos, mass, G=1.0, eps=0.0, rows=None, want_pot=False, want_abs=False):
    """Internal softened acceleration (Eq. 5, j != i) of one cluster.

    Returns acc (m,3) and, if asked, pot (m,) = -G sum m_j/sqrt(r^2+eps^2) (Eq. 4 summed) and
    absa (m,) = G sum m_j |d|/(d^2+eps^2)^{3/2}.  ``rows`` = (i0, i1) restricts the targets.
    """
    lib = _load()
    pos = _f64(pos)
    n = pos.shape[0]
    mass = _f64(mass)
    i0, i1 = (0, n) if rows is None else rows
    m = i1 - i0
    acc = np.empty((m, 3))
    pot = np.empty(m) if want_pot else None
    absa = np.empty(m) if want_abs else None
    lib.oracle_accel_range(n, i0, i1, _p(pos), _p(mass), float(G), float(eps), _p(acc), _p(pot), _p(absa))
    out = [acc]
    if want_pot:
        out.append(pot)
    if want_abs:
        out.append(absa)
    return out[0] if len(out) == 1 else tuple(out)


def ext_field(pos, G=1.0, galaxy=None):
    """External acceleration (n,3) and potential (n,) of the bulge + disk + halo model."""
    lib = _load()
    pos = _f64(pos)
    n = pos.shape[0]
    acc = np.empty((n, 3))
    phi = np.empty(n)
    lib.oracle_ext_field(n, _p(pos), float(G), _p(_gal(galaxy)), _p(acc), _p(phi))
    return acc, phi


def total_accel(pos, mass, G=1.0, eps=0.0, field=False, galaxy=None):
    lib = _load()
    pos = _f64(pos)
    n = pos.shape[0]
    acc = np.empty((n, 3))
    lib.oracle_total_accel(n, _p(pos), _p(_f64(mass)), float(G), float(eps), int(bool(field)),
                           _p(_gal(galaxy)), _p(acc))
    return acc


ENERGY_FIELDS = ("K", "W", "Uext", "E", "Px", "Py", "Pz", "Lx", "Ly", "Lz", "Tx", "Ty", "Tz", "M",
                 "Fx", "Fy", "Fz", "|F|", "sum m|a|", "_")


def energy(pos, vel, mass, G=1.0, eps=0.0, field=False, galaxy=None):
    """Diagnostics of Sect. 5.1 as a 20-vector (layout in ``ENERGY_FIELDS``; F = sum m a_int)."""
    lib = _load()
    pos = _f64(pos)
    n = pos.shape[0]
    out = np.zeros(20)
    scratch = np.empty(4 * n)
    lib.oracle_energy(n, _p(pos), _p(_f64(vel)), _p(_f64(mass)), float(G), float(eps), int(bool(field)),
                      _p(_gal(galaxy)), _p(out), _p(scratch))
    return out


def sym6_coefficients():
    d = np.empty(7)
    k = np.empty(8)
    _load().oracle_sym6_coefficients(_p(d), _p(k))
    return d, k


def step(pos, vel, mass, acc, dt, nsteps, integrator="leapfrog", G=1.0, eps=0.0, field=False, galaxy=None):
    """Advance one cluster; returns new (pos, vel, acc).  ``acc`` must be A(pos) on entry."""
    lib = _load()
    pos = _f64(pos).copy()
    vel = _f64(vel).copy()
    acc = _f64(acc).copy()
    n = pos.shape[0]
    integ = {"leapfrog": 0, "sym6": 1}[integrator]
    lib.oracle_step(n, _p(pos), _p(vel), _p(_f64(mass)), _p(acc), float(G), float(eps), int(bool(field)),
                    _p(_gal(galaxy)), float(dt), int(nsteps), integ)
    return pos, vel, acc


def accel_ragged(pos, mass, offsets, G=1.0, eps=None, field=None, galaxy=None, want_pot=False):
    """Per-cluster total acceleration for a ragged batch (clusters never interact)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    B = len(offsets) - 1
    eps = np.zeros(B) if eps is None else np.broadcast_to(np.asarray(eps, dtype=np.float64), (B,))
    field = np.zeros(B, bool) if field is None else np.broadcast_to(np.asarray(field, bool), (B,))
    pos = _f64(pos)
    mass = _f64(mass)
    acc = np.empty_like(pos)
    pot = np.empty(pos.shape[0]) if want_pot else None
    for b in range(B):
        s, e = offsets[b], offsets[b + 1]
        if want_pot:
            a, p = accel(pos[s:e], mass[s:e], G, eps[b], want_pot=True)
            pot[s:e] = p
        else:
            a = accel(pos[s:e], mass[s:e], G, eps[b])
        if field[b]:
            a = a + ext_field(pos[s:e], G, galaxy)[0]
        acc[s:e] = a
    return (acc, pot) if want_pot else acc
