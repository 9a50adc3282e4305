"""The no-allocation entry point nbody_accel_noalloc: through the C ABI, bitwise against
nbody_accel on the same inputs, two calls in a row on one context (the second with a smaller
system, so the shared scratch still holds the first call's data), and its host-only limits."""
import numpy as np
import pytest

from paper_1003_3896_amd import autotune, inputs, nbody


def test_noalloc_limits_are_host_checks():
    """Systems beyond the scratch or the table limit are rejected before anything else (no context,
    no GPU needed); a system within both reaches the context check."""
    too_big = nbody.System([0, 9_000_000], [1e-3])
    with pytest.raises(nbody.NBodyError, match="scratch"):
        nbody.nbody_accel_noalloc(None, too_big, None, None, None, None, 0)
    too_many = nbody.System(np.arange(60001), np.full(60000, 1e-3))
    with pytest.raises(nbody.NBodyError, match="staging"):
        nbody.nbody_accel_noalloc(None, too_many, None, None, None, None, 0)
    ok = nbody.System([0, 100], [1e-3])
    with pytest.raises(nbody.NBodyError, match="context is NULL"):
        nbody.nbody_accel_noalloc(None, ok, None, None, None, None, 0)
    assert nbody.nbody_workspace_bytes(None, nbody.System([0, 262144], [1e-4], prec="fp32dl")) <= \
        nbody.NOALLOC_SCRATCH_BYTES


def _batch(sizes, seed):
    cl = []
    for c, n in enumerate(sizes):
        p, v, m = inputs.plummer(n, seed + c, salpeter=(c % 2 == 1))
        if c == 1:
            p, v = inputs.on_orbit(p, v)
        cl.append(inputs.single(p, v, m, 1e-3 if c != 2 else 0.0, c == 1))
    return inputs.concat(cl)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp32dl", "fp32ds", "fp64"])
def test_noalloc_equals_accel_two_calls(prec):
    import torch
    assert torch.cuda.is_available()
    ctx = nbody.nbody_create(0)
    autotune.apply(ctx)
    try:
        # the second system is smaller: the scratch still holds the first call's tables and sums
        for sizes, seed in (((9000, 3000, 700, 65), 900), ((1500, 40), 950)):
            b = _batch(sizes, seed)
            sim = nbody.Simulation(b, prec, ctx=ctx)
            a_ref = sim.accel(pot=True).clone()
            p_ref = sim.pot.clone()
            acc = torch.full_like(sim.acc, float("nan"))
            pot = torch.full_like(sim.pot, float("nan"))
            print("\n[noalloc %s N=%s] call" % (prec, list(sizes)), flush=True)
            nbody.nbody_accel_noalloc(ctx, sim.sys, sim.pos, sim.mass, acc, pot)
            torch.cuda.synchronize()
            assert torch.equal(acc, a_ref)
            assert torch.equal(pot, p_ref)
            acc2 = torch.zeros_like(sim.acc)  # without the potential
            nbody.nbody_accel_noalloc(ctx, sim.sys, sim.pos, sim.mass, acc2, None)
            torch.cuda.synchronize()
            assert torch.equal(acc2, a_ref)
            sim.close()
    finally:
        nbody.nbody_destroy(ctx)
