"""Helpers for the GPU parity tests: run the HIP path through the C ABI binding and compare with
the oracle on the same seeded inputs."""
import numpy as np

import oracle
from paper_1003_3896_amd import accuracy

# Gates on err_i = |a_gpu,i - a_ref,i| / S_i, S_i = G sum_j m_j |d_ij| / (d^2+eps^2)^{3/2} + |a_ext,i|
# (the sum of the magnitudes of every term of particle i's acceleration), from accuracy.S_MAX and
# accuracy.S_MEDIAN:
#   FP64: ~20 FP64 roundings per term                              -> max 1e-12 (observed ~1e-16)
#   FP32DS: differences exact to fl32 of the difference; r^2, rsq, the cube and the product add
#   ~8 FP32 roundings (2^-24 each) per term, tile sums folded into FP64 -> max 1e-6
#   FP32DL: far j-tiles have coordinate differences within 1.5 x 2^-22 relative (local centring),
#   near ones are double-single -> max 1e-6 as FP32DS
#   FP32C: as FP32DS plus the rounding of the centred coordinates themselves, which perturbs a pair
#   term by ~2^-24 |x| / |d| (unbounded for close pairs) -> median 1e-6, max 1e-3 (a sanity gate
#   that catches a wrong sign, mass or G, not an accuracy claim)
#   FP32: absolute FP32 coordinates and one FP32 sum -> median 1e-6, max 1e-3 (sanity gate)
TOL = accuracy.S_MAX
TOL_MEDIAN = accuracy.S_MEDIAN


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
    return accuracy.s_errors(a_gpu, a_ref, scale)


def stats(err):
    return dict(max=float(err.max()), p99=float(np.quantile(err, 0.99)), median=float(np.median(err)))
