"""Helpers for the GPU parity tests: run the HIP path through the C ABI binding and compare with
the oracle on the same seeded inputs."""
import numpy as np

import oracle

# Tolerances on err_i = |a_gpu,i - a_ref,i| / S_i, with S_i = G sum_j m_j |d_ij| / (d^2+eps^2)^{3/2}
# + |a_ext,i| (the sum of the magnitudes of every term of particle i's acceleration).
#   FP64: ~20 FP64 roundings per term                              -> 1e-12 (observed ~1e-16)
#   FP32DS: differences exact to fl32 of the difference; r^2, rsq, the cube and the product add
#   ~8 FP32 roundings (2^-24 each) per term, tile sums folded into FP64 -> 1e-6
#   FP32C: as FP32DS plus the rounding of the centred coordinates themselves, which perturbs a
#   pair term by ~2^-24 |x| / |d| (unbounded for close pairs) -> gated on the median only
#   FP32DL: far j-tiles have coordinate differences within 1.5 x 2^-22 relative (local centring), near
#   ones are double-single -> 1e-6 as FP32DS
TOL = {"fp64": 1e-12, "fp32ds": 1e-6, "fp32dl": 1e-6}
TOL_MEDIAN = {"fp64": 1e-14, "fp32ds": 1e-7, "fp32c": 1e-6, "fp32dl": 1e-7}


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def make_sim(batch, prec):
    from paper_1003_3896_amd import nbody
    return nbody.Simulation(batch, prec)


def oracle_reference(batch, want_pot=False):
    """Per-particle reference acceleration (internal + field), scale S_i, and optional potential."""
    offs = batch.offsets
    n = batch.n
    acc = np.zeros((n, 3))
    scale = np.zeros(n)
    pot = np.zeros(n)
    for b in range(batch.B):
        s, e = offs[b], offs[b + 1]
        a, p, absa = oracle.accel(batch.pos[s:e], batch.mass[s:e], batch.G, batch.eps[b], want_pot=True,
                                  want_abs=True)
        if batch.field[b]:
            ae, _ = oracle.ext_field(batch.pos[s:e], batch.G, batch.galaxy)
            a = a + ae
            absa = absa + np.linalg.norm(ae, axis=1)
        acc[s:e] = a
        scale[s:e] = absa
        pot[s:e] = p
    return (acc, scale, pot) if want_pot else (acc, scale)


def rel_errors(a_gpu, a_ref, scale):
    d = np.linalg.norm(np.asarray(a_gpu) - a_ref, axis=1)
    out = np.zeros_like(d)
    nz = scale > 0
    out[nz] = d[nz] / scale[nz]
    out[~nz] = np.where(d[~nz] == 0, 0.0, np.inf)
    return out


def stats(err):
    return dict(max=float(err.max()), p99=float(np.quantile(err, 0.99)), median=float(np.median(err)))
