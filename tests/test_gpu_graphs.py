"""Step graphs: replays of the captured integrator step are bitwise the direct launches, replay after
replay, with the program's own eager work and synchronisations in between; a change of dt or of the
state pointers recaptures."""
import numpy as np
import pytest

from gpu_helpers import torch_dev
from paper_1003_3896_amd import inputs, nbody

pytestmark = pytest.mark.gpu


def _pair(batch, prec):
    a = nbody.Simulation(batch, prec)
    b = nbody.Simulation(batch, prec)
    nbody.nbody_use_graphs(a.ctx, True)
    nbody.nbody_use_graphs(b.ctx, False)
    a.accel()
    b.accel()
    return a, b


def _same(a, b):
    return (np.array_equal(a.pos.cpu().numpy(), b.pos.cpu().numpy())
            and np.array_equal(a.vel.cpu().numpy(), b.vel.cpu().numpy())
            and np.array_equal(a.acc.cpu().numpy(), b.acc.cpu().numpy()))


@pytest.mark.parametrize("integ,prec", [("leapfrog", "fp64"), ("sym6", "fp32ds"), ("leapfrog", "fp32"),
                                        ("sym6", "fp32dl")])
def test_graph_replays_match_eager(integ, prec):
    torch = torch_dev()
    cl = []
    for c, n in enumerate((700, 64, 1300)):
        p, v, m = inputs.plummer(n, 600 + c)
        if c == 2:
            p, v = inputs.on_orbit(p, v)
        cl.append(inputs.single(p, v, m, 1e-3, c == 2))
    batch = inputs.concat(cl)
    g, e = _pair(batch, prec)
    for rep in range(4):
        dt = 1.0 / 512 if rep < 3 else 1.0 / 300  # the last round changes dt: recapture
        g.step(integ, dt, 3)
        e.step(integ, dt, 3)
        torch.cuda.synchronize()
        assert _same(g, e), "replay %d differs" % rep
        # eager work of the program's own between replays
        g.energy()
        e.energy()
        x = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert np.array_equal(g.eout.cpu().numpy(), e.eout.cpu().numpy())
        assert torch.isfinite(x)
    g.close()
    e.close()


def test_graph_follows_new_state_buffers():
    torch = torch_dev()
    b = inputs.c1()
    g, e = _pair(b, "fp64")
    g.step("leapfrog", 1.0 / 1024, 4)
    e.step("leapfrog", 1.0 / 1024, 4)
    # move the state to fresh buffers: the cached graph must not keep writing the old ones
    g.pos = g.pos.clone()
    g.vel = g.vel.clone()
    g.acc = g.acc.clone()
    g.step("leapfrog", 1.0 / 1024, 4)
    e.step("leapfrog", 1.0 / 1024, 4)
    torch.cuda.synchronize()
    assert _same(g, e)


def test_multi_step_graph_with_remainder():
    """19 steps = two replays of an 8-step graph + a 3-step graph: bitwise the eager launches."""
    torch = torch_dev()
    b = inputs.c1()
    for integ in ("leapfrog", "sym6"):
        g, e = _pair(b, "fp32ds")
        g.step(integ, 1.0 / 1024, 19)
        e.step(integ, 1.0 / 1024, 19)
        torch.cuda.synchronize()
        assert _same(g, e), integ
        g.close()
        e.close()
