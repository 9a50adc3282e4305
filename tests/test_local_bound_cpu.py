"""The error bounds of the local double-single mode's far tiles, checked by emulation on the host.

A work item centres every coordinate on the centre c of its i-particles' bounding box (diagonal
D); a source at |x_j - c| >= 3/4 D is far and its difference to an i-particle is formed in FP32
from the FP32-rounded local coordinates.  The claim: that difference is within 1.5 x 2^-22 |d|
of the exact one.  The emulation rounds exactly as the kernel does (FP64 subtraction of the
centre, rounding to FP32, FP32 subtraction) over random and worst-case placements.

In equal-mass clusters, tiles whose sources all lie at least 3/2 D from the centre form r^2 + eps^2
in the expanded form (|x_j|^2 + eps^2) + |x_i|^2 + (-2 x_j).x_i; its eight roundings give at most
32 x 2^-24 relative error there."""
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


XBOUND = 32.0 * 2.0 ** -24


def _fma32(a, b, c):
    """FP32 fused multiply-add: a*b + c formed in extended precision, rounded once to FP32."""
    return (a.astype(np.longdouble) * b.astype(np.longdouble) + c.astype(np.longdouble)).astype(np.float32)


def _expanded_r2_error(xi, xj, c, eps2):
    """Relative error of the expanded r^2 + eps^2 of the pair kernel's equal-mass far tiles, against
    the exact value for the same FP32-rounded local coordinates (the rounding of the coordinates
    themselves is the far tiles' common error, bounded above)."""
    li = (xi - c).astype(np.float32)
    lj = (xj - c).astype(np.float32)
    aj = np.float32(-2.0) * lj                                          # exact scaling
    e2 = np.full(lj.shape[:-1], np.float32(eps2), np.float32)
    cj = _fma32(lj[..., 0], lj[..., 0], _fma32(lj[..., 1], lj[..., 1], _fma32(lj[..., 2], lj[..., 2], e2)))
    qi = (li.astype(np.float64) ** 2).sum(-1).astype(np.float32)
    q = _fma32(aj[..., 0], li[..., 0], cj)
    q = _fma32(aj[..., 1], li[..., 1], q)
    q = _fma32(aj[..., 2], li[..., 2], q)
    r2 = (q.astype(np.float64) + qi.astype(np.float64)).astype(np.float32)  # FP32 add
    d = lj.astype(np.longdouble) - li.astype(np.longdouble)
    exact = (d * d).sum(-1) + np.longdouble(np.float32(eps2))  # the kernel's eps^2 is rounded to FP32
    return np.abs((r2.astype(np.longdouble) - exact) / exact).astype(np.float64)


def _placements(rng, thr, n=256):
    c = rng.uniform(-10, 10, 3)
    half = 10.0 ** rng.uniform(-4, 0) * rng.uniform(0.2, 1.0, 3)
    D = 2 * np.linalg.norm(half)
    xi = c + rng.uniform(-1, 1, (n, 3)) * half
    xi[:8] = c + np.sign(rng.uniform(-1, 1, (8, 3))) * half
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    r = thr * D * (1.0 + 10.0 ** rng.uniform(-9, 1, n))
    # the worst alignment: sources straight out from a corner particle
    u[:8] = (xi[:8] - c) / np.linalg.norm(xi[:8] - c, axis=1, keepdims=True)
    return c, D, xi, c + u * r[:, None]


def test_expanded_far_tiles_meet_their_bound():
    """Sources at least 3/2 D from the centre: the expanded r^2 + eps^2 is within 32 x 2^-24 of the
    exact value, with and without softening."""
    rng = np.random.default_rng(9)
    worst = 0.0
    for t in range(200):
        c, D, xi, xj = _placements(rng, 1.5)
        eps2 = 0.0 if t % 2 else (1e-2 * D) ** 2
        err = _expanded_r2_error(xi[:, None, :], xj[None, :, :], c, eps2)
        worst = max(worst, float(err.max()))
    assert worst <= XBOUND, worst


def test_the_expanded_error_grows_toward_the_centre():
    """The expanded form cancels more the closer the sources come to the frame's centre: its worst
    error at the far-tile threshold of 3/4 D is several times that at 3 D (which is why it gets its
    own, larger threshold)."""
    def worst(thr):
        rng = np.random.default_rng(10)
        w = 0.0
        for _ in range(100):
            c, D, xi, xj = _placements(rng, thr)
            w = max(w, float(_expanded_r2_error(xi[:, None, :], xj[None, :, :], c, 0.0).max()))
        return w
    assert worst(0.75) > 2.0 * worst(3.0)
