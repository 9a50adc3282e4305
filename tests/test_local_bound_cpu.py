"""The error bound of the local double-single mode's far tiles, checked by emulation on the host.

A work item centres every coordinate on the centre c of its i-particles' bounding box (diagonal
D); a source at |x_j - c| >= 3/4 D is far and its difference to an i-particle is formed in FP32
from the FP32-rounded local coordinates.  The claim: that difference is within 1.5 x 2^-22 |d|
of the exact one.  The emulation rounds exactly as the kernel does (FP64 subtraction of the
centre, rounding to FP32, FP32 subtraction) over random and worst-case placements."""
import numpy as np

BOUND = 1.5 * 2.0 ** -22


def _local_difference_error(xi, xj, c):
    li = (xi - c).astype(np.float32)
    lj = (xj - c).astype(np.float32)
    d32 = (lj - li).astype(np.float64)           # FP32 subtraction, exact in FP64
    d = xj - xi
    return np.linalg.norm(d32 - d, axis=-1) / np.linalg.norm(d, axis=-1)


def test_far_sources_meet_the_bound():
    rng = np.random.default_rng(7)
    worst = 0.0
    for _ in range(200):
        # a box somewhere in a cluster (offset and size over several decades)
        c = rng.uniform(-10, 10, 3)
        half = 10.0 ** rng.uniform(-4, 0) * rng.uniform(0.2, 1.0, 3)
        D = 2 * np.linalg.norm(half)
        xi = c + rng.uniform(-1, 1, (256, 3)) * half
        xi[:8] = c + np.sign(rng.uniform(-1, 1, (8, 3))) * half      # corners: |x_i - c| = D/2
        u = rng.normal(size=(256, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        r = 0.75 * D * (1.0 + 10.0 ** rng.uniform(-9, 1, 256))       # at and beyond the threshold
        xj = c + u * r[:, None]
        err = _local_difference_error(xi[:, None, :], xj[None, :, :], c)
        worst = max(worst, float(err.max()))
    assert worst <= BOUND, worst


def test_the_bound_needs_the_threshold():
    """Sources well inside 3/4 D from the centre can exceed it (the near tiles run
    double-single for that reason)."""
    rng = np.random.default_rng(8)
    c = np.array([8.0, 0.3, -0.2])
    half = np.array([1e-3, 1e-3, 1e-3])
    xi = c + rng.uniform(-1, 1, (512, 3)) * half
    xj = xi + rng.normal(size=(512, 3)) * 1e-9                       # close pairs inside the box
    assert _local_difference_error(xi, xj, c).max() > BOUND
