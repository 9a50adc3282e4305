"""ctypes binding of libnbody.so (C ABI in include/nbody.h), same names as the C functions.

Argument marshalling only: every step of the computation runs in the HIP kernels of
``csrc/``.  Device arrays are passed as ``torch.Tensor`` (float64, contiguous, on the GPU) or
as raw integer device addresses; PyTorch provides device memory and streams, nothing else.
If the library is not built this module raises on first use; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnbody.so")

NB_OK, NB_ERR_ARG, NB_ERR_HIP, NB_ERR_NOMEM, NB_ERR_UNSUPPORTED, NB_ERR_NONFINITE = 0, -1, -2, -3, -4, -5
NB_FP32, NB_FP32C, NB_FP32DS, NB_FP64, NB_FP32DL = 0, 1, 2, 3, 4
NB_GALAXY_HERNQUIST_LOG, NB_GALAXY_ALLEN_SANTILLAN = 0, 1
PREC = {"fp32": NB_FP32, "fp32c": NB_FP32C, "fp32ds": NB_FP32DS, "fp64": NB_FP64, "fp32dl": NB_FP32DL}
# cluster-size classes of the launch-shape table (nbody_set_tile)
N_CLASSES = 4

EXPORTS = (
    "nbody_create", "nbody_destroy", "nbody_workspace_bytes", "nbody_accel", "nbody_substep",
    "nbody_step_leapfrog", "nbody_step_sym6", "nbody_energy", "nbody_last_error", "nbody_set_tile",
    "nbody_get_tile", "nbody_timing_enable", "nbody_timing_read", "nbody_interactions", "nbody_use_graphs",
    "nbody_sym6_coefficients", "nbody_substeps", "nbody_workspace_bytes_max", "nbody_accel_noalloc",
)
# limits of nbody_accel_noalloc (NB_NOALLOC_SCRATCH_BYTES, NB_NOALLOC_TABLE_BYTES in include/nbody.h)
NOALLOC_SCRATCH_BYTES = 256 << 20
NOALLOC_TABLE_BYTES = 4 << 20

ENERGY_FIELDS = ("K", "W", "Uext", "E", "Px", "Py", "Pz", "Lx", "Ly", "Lz", "Tx", "Ty", "Tz", "M",
                 "Fx", "Fy", "Fz", "|F|", "sum m|a|", "nonfinite")
ENERGY_WIDTH = len(ENERGY_FIELDS)


class NBodyError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("nbody error %d: %s" % (code, msg))
        self.code = code


class nbody_galaxy(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_double) for n in ("Mb", "ab", "Md", "ad", "bd", "vh", "dh", "Mbh", "ebh")] +
                [("model", ctypes.c_int32)] + [(n, ctypes.c_double) for n in ("Mh", "ah", "rcut")])


class nbody_system(ctypes.Structure):
    _fields_ = [
        ("nclusters", ctypes.c_int32),
        ("offsets", ctypes.POINTER(ctypes.c_int64)),
        ("G", ctypes.c_double),
        ("eps", ctypes.POINTER(ctypes.c_double)),
        ("field", ctypes.POINTER(ctypes.c_uint8)),
        ("galaxy", nbody_galaxy),
        ("prec", ctypes.c_int32),
    ]


class nbody_tile(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("waves_per_group", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("phased", ctypes.c_int32)]


_lib = None


def lib():
    """Load libnbody.so (raises if it has not been built).

    PyTorch is imported first so that the library binds to the HIP runtime PyTorch already loaded
    (both carry the soname libamdhip64.so.7): one process must not run two HIP runtimes."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads PyTorch's HIP runtime before ours resolves it)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libnbody.so is not built (%s); run __graft_entry__.build() or "
                               "python -m paper_1003_3896_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
        SYS = ctypes.POINTER(nbody_system)
        L.nbody_create.argtypes = [ctypes.c_int, ctypes.POINTER(P)]
        L.nbody_destroy.argtypes = [P]
        L.nbody_destroy.restype = None
        L.nbody_workspace_bytes.argtypes = [P, SYS]
        L.nbody_workspace_bytes.restype = SZ
        L.nbody_workspace_bytes_max.argtypes = [I64, I32]
        L.nbody_workspace_bytes_max.restype = SZ
        L.nbody_accel.argtypes = [P, SYS, P, P, P, P, P, SZ, P]
        L.nbody_accel_noalloc.argtypes = [P, SYS, P, P, P, P, P]
        L.nbody_substep.argtypes = [P, SYS, P, P, P, P, P, P, P, P, SZ, P]
        L.nbody_substeps.argtypes = [P, SYS, P, P, P, P, P, I32, P, SZ, P]
        L.nbody_step_leapfrog.argtypes = [P, SYS, P, P, P, P, D, I32, P, SZ, P]
        L.nbody_step_sym6.argtypes = [P, SYS, P, P, P, P, D, I32, P, SZ, P]
        L.nbody_energy.argtypes = [P, SYS, P, P, P, P, P, SZ, P]
        L.nbody_last_error.restype = ctypes.c_char_p
        L.nbody_set_tile.argtypes = [P, I32, I32, nbody_tile]
        L.nbody_get_tile.argtypes = [P, I32, I32, ctypes.POINTER(nbody_tile)]
        L.nbody_timing_enable.argtypes = [P, ctypes.c_int]
        L.nbody_use_graphs.argtypes = [P, ctypes.c_int]
        L.nbody_sym6_coefficients.argtypes = [P, P]
        L.nbody_timing_read.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(I64)]
        L.nbody_interactions.argtypes = [SYS]
        L.nbody_interactions.restype = I64
        for name in ("nbody_create", "nbody_accel", "nbody_accel_noalloc", "nbody_substep", "nbody_step_leapfrog", "nbody_step_sym6",
                     "nbody_energy", "nbody_set_tile", "nbody_get_tile", "nbody_timing_enable", "nbody_use_graphs",
                     "nbody_sym6_coefficients", "nbody_substeps",
                     "nbody_timing_read"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != NB_OK:
        raise NBodyError(rc, lib().nbody_last_error().decode())


def _addr(x) -> Optional[int]:
    """Device address of a tensor (or an int address, or None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if not x.is_contiguous():
        raise ValueError("device arrays must be contiguous")
    return x.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class System:
    """Host description of a ragged batch (the C ``nbody_system``); keeps its arrays alive."""

    def __init__(self, offsets, eps, field=None, G: float = 1.0,
                 galaxy: Sequence[float] = (1.0, 0.7, 4.5, 3.0, 0.28, 0.7, 12.0), prec=NB_FP32DS):
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        B = len(self.offsets) - 1
        self.eps = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, np.float64), (B,)))
        self.field = None if field is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(field, np.uint8), (B,)))
        self.G = float(G)
        # (Mb, ab, Md, ad, bd, vh, dh, Mbh, ebh, model, Mh, ah, rcut): no black hole if 7 values,
        # model 0 if 9 or fewer
        self.galaxy = tuple(float(v) for v in galaxy) + (0.0,) * (13 - len(galaxy))
        self.prec = PREC[prec] if isinstance(prec, str) else int(prec)
        c = nbody_system()
        c.nclusters = B
        c.offsets = self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        c.G = self.G
        c.eps = self.eps.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        c.field = (self.field.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if self.field is not None
                   else ctypes.POINTER(ctypes.c_uint8)())
        g = self.galaxy
        c.galaxy = nbody_galaxy(*g[:9], int(g[9]), *g[10:])
        c.prec = self.prec
        self._c = c

    @property
    def B(self) -> int:
        return len(self.offsets) - 1

    @property
    def n(self) -> int:
        return int(self.offsets[-1])

    def ref(self):
        return ctypes.byref(self._c)

    def with_prec(self, prec) -> "System":
        return System(self.offsets, self.eps, self.field, self.G, self.galaxy, prec)


def system_from_batch(batch, prec="fp32ds") -> System:
    return System(batch.offsets, batch.eps, batch.field, batch.G, batch.galaxy, prec)


# ---- the C ABI, name for name --------------------------------------------------------------

def nbody_create(device: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(lib().nbody_create(int(device), ctypes.byref(h)))
    return h.value


def nbody_destroy(ctx: int) -> None:
    lib().nbody_destroy(ctx)


def nbody_workspace_bytes(ctx: Optional[int], sys: System) -> int:
    n = lib().nbody_workspace_bytes(ctx, sys.ref())
    if n == 0:
        raise NBodyError(NB_ERR_ARG, lib().nbody_last_error().decode())
    return n


def nbody_workspace_bytes_max(max_particles: int, max_clusters: int) -> int:
    n = lib().nbody_workspace_bytes_max(int(max_particles), int(max_clusters))
    if n == 0:
        raise NBodyError(NB_ERR_ARG, lib().nbody_last_error().decode())
    return n


def nbody_interactions(sys: System) -> int:
    return int(lib().nbody_interactions(sys.ref()))


def nbody_accel(ctx, sys: System, pos, mass, acc, pot, ws, ws_bytes: int, stream=None) -> None:
    _check(lib().nbody_accel(ctx, sys.ref(), _addr(pos), _addr(mass), _addr(acc), _addr(pot), _addr(ws),
                             int(ws_bytes), _stream(stream)))


def nbody_accel_noalloc(ctx, sys: System, pos, mass, acc, pot, stream=None) -> None:
    """nbody_accel with the library's static device scratch instead of a caller workspace."""
    _check(lib().nbody_accel_noalloc(ctx, sys.ref(), _addr(pos), _addr(mass), _addr(acc), _addr(pot),
                                     _stream(stream)))


def nbody_substep(ctx, sys: System, pos, vel, mass, acc, kick_pre, drift, kick_post, ws, ws_bytes: int,
                  stream=None) -> None:
    kp = np.ascontiguousarray(kick_pre, np.float64)
    dr = np.ascontiguousarray(drift, np.float64)
    kq = np.ascontiguousarray(kick_post, np.float64)
    for a in (kp, dr, kq):
        if a.shape != (sys.B,):
            raise ValueError("coefficient arrays must have one entry per cluster")
    P = ctypes.c_void_p
    _check(lib().nbody_substep(ctx, sys.ref(), _addr(pos), _addr(vel), _addr(mass), _addr(acc),
                               kp.ctypes.data_as(P), dr.ctypes.data_as(P), kq.ctypes.data_as(P), _addr(ws),
                               int(ws_bytes), _stream(stream)))


def nbody_substeps(ctx, sys: System, pos, vel, mass, acc, coef, ws, ws_bytes: int, stream=None) -> None:
    """coef: array [nrounds][B][3] of (kick_pre, drift, kick_post)."""
    c = np.ascontiguousarray(coef, np.float64)
    if c.ndim != 3 or c.shape[1:] != (sys.B, 3):
        raise ValueError("coef must have shape (nrounds, B, 3)")
    _check(lib().nbody_substeps(ctx, sys.ref(), _addr(pos), _addr(vel), _addr(mass), _addr(acc),
                                c.ctypes.data_as(ctypes.c_void_p), int(c.shape[0]), _addr(ws), int(ws_bytes),
                                _stream(stream)))


def nbody_step_leapfrog(ctx, sys: System, pos, vel, mass, acc, dt: float, nsteps: int, ws, ws_bytes: int,
                        stream=None) -> None:
    _check(lib().nbody_step_leapfrog(ctx, sys.ref(), _addr(pos), _addr(vel), _addr(mass), _addr(acc), float(dt),
                                     int(nsteps), _addr(ws), int(ws_bytes), _stream(stream)))


def nbody_step_sym6(ctx, sys: System, pos, vel, mass, acc, dt: float, nsteps: int, ws, ws_bytes: int,
                    stream=None) -> None:
    _check(lib().nbody_step_sym6(ctx, sys.ref(), _addr(pos), _addr(vel), _addr(mass), _addr(acc), float(dt),
                                 int(nsteps), _addr(ws), int(ws_bytes), _stream(stream)))


def nbody_energy(ctx, sys: System, pos, vel, mass, out, ws, ws_bytes: int, stream=None) -> None:
    _check(lib().nbody_energy(ctx, sys.ref(), _addr(pos), _addr(vel), _addr(mass), _addr(out), _addr(ws),
                              int(ws_bytes), _stream(stream)))


def nbody_set_tile(ctx, prec, nclass: int, k: int, waves_per_group: int, tile: int, blocks_per_cu: int,
                   phased: int = 0) -> None:
    prec = PREC[prec] if isinstance(prec, str) else prec
    _check(lib().nbody_set_tile(ctx, int(prec), int(nclass),
                                nbody_tile(k, waves_per_group, tile, blocks_per_cu, int(phased))))


def nbody_get_tile(ctx, prec, nclass: int):
    prec = PREC[prec] if isinstance(prec, str) else prec
    t = nbody_tile()
    _check(lib().nbody_get_tile(ctx, int(prec), int(nclass), ctypes.byref(t)))
    return (t.k, t.waves_per_group, t.tile, t.blocks_per_cu, t.phased)


def nbody_sym6_coefficients():
    """(drift weights [7], kick weights [8]) of the 6th-order composition, from the library."""
    d = np.zeros(7)
    k = np.zeros(8)
    _check(lib().nbody_sym6_coefficients(d.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(ctypes.c_void_p)))
    return d, k


def nbody_use_graphs(ctx, enable: bool) -> None:
    _check(lib().nbody_use_graphs(ctx, 1 if enable else 0))


def nbody_timing_enable(ctx, enable: bool) -> None:
    _check(lib().nbody_timing_enable(ctx, 1 if enable else 0))


def nbody_timing_read(ctx):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().nbody_timing_read(ctx, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def nbody_last_error() -> str:
    return lib().nbody_last_error().decode()


# ---- convenience: device state + workspace held together -----------------------------------

class Simulation:
    """Device-resident state of one ragged batch plus its workspace; thin wrapper over the ABI."""

    def __init__(self, batch, prec="fp32ds", device: int = 0, ctx: Optional[int] = None, tuned: bool = True):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda", device)
        self.sys = system_from_batch(batch, prec)
        self.own_ctx = ctx is None
        self.ctx = nbody_create(device) if ctx is None else ctx
        if tuned and self.own_ctx:
            from . import autotune
            autotune.apply(self.ctx)  # launch shapes from the autotuner's cache, if present
        self.ws_bytes = nbody_workspace_bytes(self.ctx, self.sys)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.dev)
        base = self.ws.data_ptr()
        self.ws_addr = (base + 255) & ~255
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.pos = torch.as_tensor(batch.pos, **f64).contiguous()
        self.vel = torch.as_tensor(batch.vel, **f64).contiguous()
        self.mass = torch.as_tensor(batch.mass, **f64).contiguous()
        self.acc = torch.zeros_like(self.pos)
        self.pot = torch.zeros(self.sys.n, **f64)
        self.eout = torch.zeros(self.sys.B, ENERGY_WIDTH, **f64)

    def close(self):
        if self.own_ctx and self.ctx:
            nbody_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def accel(self, pot: bool = False, stream=None):
        nbody_accel(self.ctx, self.sys, self.pos, self.mass, self.acc, self.pot if pot else None, self.ws_addr,
                    self.ws_bytes, stream)
        return self.acc

    def step(self, integrator: str, dt: float, nsteps: int, stream=None):
        fn = nbody_step_leapfrog if integrator == "leapfrog" else nbody_step_sym6
        fn(self.ctx, self.sys, self.pos, self.vel, self.mass, self.acc, dt, nsteps, self.ws_addr, self.ws_bytes,
           stream)

    def substep(self, kick_pre, drift, kick_post, stream=None):
        nbody_substep(self.ctx, self.sys, self.pos, self.vel, self.mass, self.acc, kick_pre, drift, kick_post,
                      self.ws_addr, self.ws_bytes, stream)

    def energy(self, stream=None, prec=None):
        sys = self.sys if prec is None else self.sys.with_prec(prec)
        if prec is not None and nbody_workspace_bytes(self.ctx, sys) > self.ws_bytes:
            raise NBodyError(NB_ERR_ARG, "workspace too small for the energy precision")
        nbody_energy(self.ctx, sys, self.pos, self.vel, self.mass, self.eout, self.ws_addr, self.ws_bytes, stream)
        return self.eout
