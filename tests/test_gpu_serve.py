"""The served path on the GPU: jobs that run together in one ragged batch (each at its own stage)
give bitwise the results they give alone, and agree with the oracle."""
import numpy as np
import pytest

import oracle
from gpu_helpers import torch_dev
from paper_1003_3896_amd import inputs
from paper_1003_3896_amd.serve import HipExecutor, Request, Server

pytestmark = pytest.mark.gpu


def _reqs(prec_tag, count=10):
    jobs = inputs.c5_jobs(count, rate=0.0, seed=4242, nlo=128, nhi=3000, smin=2, smax=9)
    out = []
    for j in jobs:
        p, v, m = j.initial_state()
        out.append(Request(j.jid, p, v, m, j.steps, j.integrator, 1.0 / 512, 1e-2, j.field, 0.0))
    return out


@pytest.mark.parametrize("prec,policy,fill", [("fp32ds", "srpt", 2.0 ** 30), ("fp32ds", "srpt", 4e6),
                                              ("fp32ds", "all", 0.0), ("fp64", "srpt", 2.0 ** 30),
                                              ("fp32dl", "srpt", 2.0 ** 30)])
def test_alone_equals_in_mix(prec, policy, fill):
    """20 jobs (sizes 128..3000 across two size classes, both integrators, field on some) served
    together, with queueing, reordering and partial rounds, give bitwise their results alone."""
    torch_dev()
    reqs = _reqs(prec, count=20)
    ex = HipExecutor(capacity=12000, max_clusters=6, prec=prec, energy_prec="fp64")
    mix = Server(ex, policy=policy, fill=fill).run(reqs)  # capacity forces queueing
    for r in reqs:
        assert mix[r.jid].status == "done"
        alone = Server(ex).run([r])[r.jid]
        assert np.array_equal(alone.pos, mix[r.jid].pos) and np.array_equal(alone.vel, mix[r.jid].vel), r.jid
    ex.close()


def test_served_fp64_matches_oracle():
    torch_dev()
    reqs = _reqs("fp64", count=6)
    ex = HipExecutor(capacity=8000, max_clusters=4, prec="fp64")
    res = Server(ex).run(reqs)
    for r in reqs:
        a0 = oracle.total_accel(r.pos, r.mass, 1.0, r.eps, r.field)
        p, v, _ = oracle.step(r.pos, r.vel, r.mass, a0, r.dt, r.steps, r.integrator, 1.0, r.eps, r.field)
        assert np.abs(res[r.jid].pos - p).max() <= 1e-10 * np.abs(p).max()
        e0 = oracle.energy(r.pos, r.vel, r.mass, 1.0, r.eps, r.field)
        assert abs(res[r.jid].energy0[3] - e0[3]) <= 1e-12 * abs(e0[3])
    ex.close()
