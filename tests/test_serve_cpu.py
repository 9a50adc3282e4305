"""Control logic of the continuous-batching server on the CPU (oracle-backed executor): every job
finishes with its solo trajectory, admission respects capacity, oversize and invalid requests are
rejected, cancellation and a non-finite job do not disturb the others."""
import numpy as np
import pytest

import oracle
from fake_executor import FakeExecutor
from paper_1003_3896_amd import inputs, nbody
from paper_1003_3896_amd.serve import Request, Server, latency_stats, stage_schedule

SYM6 = nbody.nbody_sym6_coefficients()


def _req(j, n, steps, integ, fld=False, arrival=0.0, dt=1.0 / 256, eps=1e-2):
    p, v, m = inputs.plummer(n, 700 + j)
    if fld:
        p, v = inputs.on_orbit(p, v)
    return Request(j, p, v, m, steps, integ, dt, eps, fld, arrival)


def _solo_oracle(r):
    a0 = oracle.total_accel(r.pos, r.mass, 1.0, r.eps, r.field)
    return oracle.step(r.pos, r.vel, r.mass, a0, r.dt, r.steps, r.integrator, 1.0, r.eps, r.field)


def test_schedule_matches_integrators():
    s = stage_schedule("leapfrog", 0.1, 3, SYM6)
    assert s[0] == (0.0, 0.0, 0.0) and len(s) == 4 and s[1] == (0.05, 0.1, 0.05)
    s = stage_schedule("sym6", 0.1, 2, SYM6)
    assert len(s) == 1 + 14
    d, k = SYM6
    assert abs(sum(c[1] for c in s) - 0.2) < 1e-15  # drifts add up to the elapsed time
    assert abs(sum(c[0] + c[2] for c in s) - 0.2) < 1e-15  # so do kicks
    with pytest.raises(ValueError):
        stage_schedule("rk4", 0.1, 1, SYM6)


def test_mixed_jobs_match_solo_oracle_runs():
    reqs = [_req(0, 40, 3, "leapfrog"), _req(1, 25, 2, "sym6", True), _req(2, 60, 4, "leapfrog", True),
            _req(3, 33, 1, "sym6")]
    srv = Server(FakeExecutor(capacity=100, max_clusters=3), sym6=SYM6)
    res = srv.run(reqs)
    for r in reqs:
        out = res[r.jid]
        assert out.status == "done"
        p, v, _ = _solo_oracle(r)
        assert np.array_equal(out.pos, p) and np.array_equal(out.vel, v), r.jid
        assert out.rel_energy_error < 1e-3
    # capacity 100 with these sizes forces queueing: no round ran more than 100 particles
    assert max(sum(c) for c in srv.ex.calls) <= 100
    assert max(len(c) for c in srv.ex.calls) <= 3


def test_rejections():
    big = _req(0, 50, 1, "leapfrog")
    bad = _req(1, 10, -1, "leapfrog")
    ok = _req(2, 10, 1, "leapfrog")
    res = Server(FakeExecutor(capacity=20, max_clusters=4), sym6=SYM6).run([big, bad, ok])
    assert res[0].status == "rejected" and res[1].status == "rejected" and res[2].status == "done"


def test_cancel_queued_and_active():
    reqs = [_req(0, 30, 6, "leapfrog"), _req(1, 30, 6, "leapfrog"), _req(2, 30, 3, "leapfrog")]
    srv = Server(FakeExecutor(capacity=60, max_clusters=2), sym6=SYM6)
    srv.cancel(2)   # still queued when cancelled
    srv.run(reqs, max_rounds=2)
    srv.cancel(1)   # active when cancelled
    res = srv.run([])
    assert res[2].status == "cancelled" and res[1].status == "cancelled"
    assert res[0].status == "done"
    p, v, _ = _solo_oracle(reqs[0])
    assert np.array_equal(res[0].pos, p)


def test_nonfinite_job_fails_alone():
    good = _req(0, 30, 3, "leapfrog")
    bad = _req(1, 30, 3, "leapfrog")
    bad.vel = bad.vel.copy()
    bad.vel[3, 0] = np.nan
    res = Server(FakeExecutor(capacity=100, max_clusters=4), sym6=SYM6).run([bad, good])
    assert res[1].status == "failed" and res[0].status == "done"
    p, v, _ = _solo_oracle(good)
    assert np.array_equal(res[0].pos, p)


def test_arrivals_and_latency_stats():
    t = [0.0]

    def clock():
        t[0] += 0.001
        return t[0]

    reqs = [_req(j, 20, 2, "leapfrog", arrival=0.01 * j) for j in range(6)]
    res = Server(FakeExecutor(capacity=50, max_clusters=8), clock=clock, sym6=SYM6).run(reqs)
    st = latency_stats(res)
    assert st["n"] == 6 and 0 < st["p50"] <= st["p99"]
    assert all(res[j].latency > 0 for j in range(6))


def test_short_job_overtakes_long_one():
    """Least-remaining-work order: a short job that arrives while a long one runs goes to the front
    of the arena and, with a fill of one cluster, runs alone until it is done."""
    t = [0.0]

    def clock():
        t[0] += 0.001
        return t[0]

    long_job = _req(0, 40, 30, "leapfrog")
    short = _req(1, 20, 2, "leapfrog", arrival=0.004)
    ex = FakeExecutor(capacity=100, max_clusters=4)
    srv = Server(ex, clock=clock, sym6=SYM6, fill=1.0, max_rounds_per_call=1)
    res = srv.run([long_job, short])
    assert res[1].latency < res[0].latency
    assert ex.reorders >= 1
    # after the short job's admission, every round until it finished advanced it alone
    i = next(k for k, c in enumerate(ex.calls) if c == [20])
    assert ex.calls[i:i + 3] == [[20]] * 3
    for r in (long_job, short):
        p, v, _ = _solo_oracle(r)
        assert np.array_equal(res[r.jid].pos, p) and np.array_equal(res[r.jid].vel, v)


@pytest.mark.parametrize("policy,fill", [("all", 1.0), ("srpt", 1.0), ("srpt", 2000.0)])
def test_policies_give_solo_results(policy, fill):
    reqs = [_req(0, 40, 3, "leapfrog", arrival=0.0), _req(1, 25, 2, "sym6", True, arrival=0.0),
            _req(2, 30, 1, "leapfrog", arrival=0.0)]
    ex = FakeExecutor(capacity=200, max_clusters=4)
    res = Server(ex, sym6=SYM6, policy=policy, fill=fill).run(reqs)
    for r in reqs:
        p, v, _ = _solo_oracle(r)
        assert np.array_equal(res[r.jid].pos, p) and np.array_equal(res[r.jid].vel, v), (policy, r.jid)
    if policy == "all":
        assert ex.calls[0] == [40, 25, 30]
    elif fill == 1.0:
        assert all(len(c) == 1 for c in ex.calls)  # one job per round
    else:
        assert max(len(c) for c in ex.calls) >= 2  # 30^2 + 25^2 < 2000 <= + 40^2: up to three
    with pytest.raises(ValueError):
        Server(ex, policy="fifo")


def test_queue_admits_small_job_past_a_big_one():
    """A queued job too big for the free arena space does not hold back a smaller one behind it
    (least-work admission); in arrival order ("all") it does."""
    for policy, small_first in (("srpt", True), ("all", False)):
        running = _req(0, 60, 6, "leapfrog", arrival=0.0)
        big = _req(1, 60, 1, "leapfrog", arrival=0.0)
        small = _req(2, 30, 1, "leapfrog", arrival=0.0)
        ex = FakeExecutor(capacity=100, max_clusters=4)
        srv = Server(ex, sym6=SYM6, policy=policy, fill=1e9)
        srv.submit(running)
        srv._admit(0.0)
        srv.submit(big)
        srv.submit(small)
        srv._admit(0.0)
        ids = [a.req.jid for a in srv.active]
        assert (2 in ids) == small_first and 1 not in ids, (policy, ids)
        res = srv.run([])
        for r in (running, big, small):
            p, v, _ = _solo_oracle(r)
            assert np.array_equal(res[r.jid].pos, p), (policy, r.jid)
