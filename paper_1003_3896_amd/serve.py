"""Continuous-batching request loop for N-body integration jobs.

Jobs (one isolated cluster each: initial state, integrator, number of steps, softening, field
flag) arrive over time.  The server keeps every admitted job's state on the device in one
particle arena and advances the jobs in rounds: each round is one stage of the ragged batch of
jobs at the front of the arena, every job at its own integrator stage (its own kick/drift
coefficients), and up to 64 rounds go to the device in one ``nbody_substeps`` call.  A job's
first round is an evaluation-only substep (all coefficients 0) that produces its first
acceleration; after that a leapfrog step is one substep (dt/2, dt, dt/2) and a 6th-order step is
seven (the composition's merged kicks and drifts, taken from the library).  Jobs that arrive while
others run are admitted as soon as arena space and cluster slots allow (admission by bytes of
device memory), so their work overlaps on the device with the jobs already running.  By default
the arena is kept in order of remaining work and a round takes the leading jobs until it holds
enough pair interactions to occupy the device, so short jobs finish at their own pace; finished
jobs are retired, their energy evaluated, and the arena compacted.

Because each cluster's arithmetic depends only on its own data and on the pair kernel's fold
pattern (the same tile length and waves per i-group for every cluster size here), a job's result is
bitwise the same whether it ran alone or in a mix.

The device work goes through an executor; ``HipExecutor`` is the GPU one.  Tests drive the same
control logic with a CPU stand-in.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import nbody

STATE_BYTES_PER_PARTICLE = 80  # pos 24 + vel 24 + acc 24 + mass 8 (float64)
SERVE_TILE = (256, 2)          # (j-records per LDS tile, waves per i-group) for every served job


@dataclass
class Request:
    """One integration job.  ``pos``/``vel``/``mass`` are the host initial state."""
    jid: int
    pos: np.ndarray
    vel: np.ndarray
    mass: np.ndarray
    steps: int
    integrator: str = "leapfrog"  # or "sym6"
    dt: float = 2.0 ** -11
    eps: float = 1e-3
    field: bool = False
    arrival: float = 0.0          # seconds after the start of the run

    @property
    def n(self) -> int:
        return int(self.mass.shape[0])

    def evals(self) -> int:
        return self.steps * (1 if self.integrator == "leapfrog" else 7)

    def interactions(self) -> int:
        return self.evals() * self.n * self.n


@dataclass
class Result:
    jid: int
    status: str                   # "done", "failed", "rejected", "cancelled"
    latency: float = float("nan")
    pos: Optional[np.ndarray] = None
    vel: Optional[np.ndarray] = None
    energy0: Optional[np.ndarray] = None
    energy1: Optional[np.ndarray] = None
    reason: str = ""

    @property
    def rel_energy_error(self) -> float:
        if self.energy0 is None or self.energy1 is None:
            return float("nan")
        return abs(self.energy1[3] - self.energy0[3]) / abs(self.energy0[3])


@dataclass
class _Active:
    req: Request
    offset: int
    schedule: np.ndarray          # [rounds, 3] (kick_pre, drift, kick_post) of every round
    cursor: int = 0               # next round to run
    energy0: Optional[np.ndarray] = None
    admitted_at: float = 0.0

    @property
    def left(self) -> int:
        return self.schedule.shape[0] - self.cursor


def stage_schedule(integrator: str, dt: float, steps: int, sym6: Optional[tuple] = None) -> List[tuple]:
    """Coefficient triples of every round of a job: one evaluation-only round, then the steps."""
    rounds = [(0.0, 0.0, 0.0)]
    if integrator == "leapfrog":
        rounds += [(0.5 * dt, 1.0 * dt, 0.5 * dt)] * steps
    elif integrator == "sym6":
        d, k = sym6 if sym6 is not None else nbody.nbody_sym6_coefficients()
        one = [(k[s] * dt, d[s] * dt, (k[7] * dt) if s == 6 else 0.0) for s in range(7)]
        rounds += one * steps
    else:
        raise ValueError("unknown integrator %r" % integrator)
    return rounds


class HipExecutor:
    """Device side of the server: a particle arena, its workspace and the library context."""

    def __init__(self, capacity: int, max_clusters: int, prec: str = "fp32ds", device: int = 0,
                 energy_prec: str = "fp64", tile=None, G: float = 1.0, galaxy=None, max_inflight: int = 2):
        import collections
        import torch
        self.torch = torch
        # calls whose device work may still be queued: bounding them bounds how long a newly admitted
        # job waits behind work enqueued for the jobs already running
        self.max_inflight = int(max_inflight)
        self._inflight = collections.deque()
        self.dev = torch.device("cuda", device)
        self.capacity = int(capacity)
        self.max_clusters = int(max_clusters)
        self.prec = prec
        self.energy_prec = energy_prec
        self.G = G
        self.galaxy = tuple(galaxy) if galaxy is not None else nbody.System([0, 1], [0.0]).galaxy
        self.ctx = nbody.nbody_create(device)
        # no step graphs: the batch layout changes at every job boundary, so most calls would
        # capture a new graph instead of replaying one
        nbody.nbody_use_graphs(self.ctx, False)
        # Results depend on the tile length and the waves per group (the fold pattern), not on the
        # i-particles per lane, blocks per CU or the phased loop: every size class gets the same
        # (tile, waves) and its own tuned rest, so a job's result does not depend on the batch.
        if tile is None:
            from . import autotune
            autotune.apply(self.ctx, fixed_tile={fam: SERVE_TILE for fam in ("f32", "ds", "f64", "dl")})
        else:
            for p in {prec, energy_prec}:
                for ncl in range(nbody.N_CLASSES):
                    nbody.nbody_set_tile(self.ctx, p, ncl, *tile)
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.pos = torch.zeros(self.capacity, 3, **f64)
        self.vel = torch.zeros(self.capacity, 3, **f64)
        self.acc = torch.zeros(self.capacity, 3, **f64)
        self.mass = torch.zeros(self.capacity, **f64)
        self.eout = torch.zeros(self.max_clusters, nbody.ENERGY_WIDTH, **f64)
        self.ws_bytes = self._workspace_bound()
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.dev)
        self.ws_addr = (self.ws.data_ptr() + 255) & ~255

    def _workspace_bound(self) -> int:
        """Workspace for any admissible batch (the library's bound over all systems of at most
        `capacity` particles in at most `max_clusters` clusters)."""
        return nbody.nbody_workspace_bytes_max(self.capacity, self.max_clusters)

    def footprint_bytes(self) -> int:
        return STATE_BYTES_PER_PARTICLE * self.capacity + self.ws_bytes + nbody.ENERGY_WIDTH * 8 * self.max_clusters

    def close(self):
        if self.ctx:
            self.torch.cuda.synchronize()
            nbody.nbody_destroy(self.ctx)
            self.ctx = None

    def load(self, offset: int, req: Request) -> None:
        t = self.torch
        n = req.n
        sl = slice(offset, offset + n)
        self.pos[sl] = t.as_tensor(req.pos, dtype=t.float64).to(self.dev, non_blocking=False)
        self.vel[sl] = t.as_tensor(req.vel, dtype=t.float64).to(self.dev, non_blocking=False)
        self.mass[sl] = t.as_tensor(req.mass, dtype=t.float64).to(self.dev, non_blocking=False)
        self.acc[sl].zero_()

    def _system(self, sizes: Sequence[int], eps: Sequence[float], fld: Sequence[bool], prec: str):
        offs = np.zeros(len(sizes) + 1, np.int64)
        offs[1:] = np.cumsum(sizes)
        return nbody.System(offs, np.asarray(eps, np.float64), np.asarray(fld, np.uint8), self.G, self.galaxy, prec)

    def substeps(self, sizes, eps, fld, coef) -> None:
        """len(coef) rounds over the batch; coef is [rounds][B][3]."""
        sys = self._system(sizes, eps, fld, self.prec)
        nbody.nbody_substeps(self.ctx, sys, self.pos, self.vel, self.mass, self.acc, coef, self.ws_addr,
                             self.ws_bytes)
        ev = self.torch.cuda.Event()
        ev.record()
        self._inflight.append(ev)
        while len(self._inflight) > self.max_inflight:
            self._inflight.popleft().synchronize()

    def energy(self, offset: int, sizes, eps, fld) -> np.ndarray:
        """Diagnostics of the consecutive jobs starting at ``offset`` (one row each)."""
        sys = self._system(sizes, eps, fld, self.energy_prec)
        o = int(offset)
        B = len(sizes)
        nbody.nbody_energy(self.ctx, sys, self.pos.data_ptr() + 24 * o, self.vel.data_ptr() + 24 * o,
                           self.mass.data_ptr() + 8 * o, self.eout.data_ptr(), self.ws_addr, self.ws_bytes)
        return self.eout[:B].cpu().numpy().copy()

    def reorder(self, spans) -> None:
        """Rewrite the arena from offset 0 as the concatenation of the (offset, n) spans, in order."""
        t = self.torch
        idx = np.concatenate([np.arange(o, o + n, dtype=np.int64) for o, n in spans])
        it = t.from_numpy(idx).to(self.dev)
        m = idx.shape[0]
        for buf in (self.pos, self.vel, self.acc, self.mass):
            buf[:m] = buf.index_select(0, it)

    def move(self, src: int, dst: int, n: int) -> None:
        """Move n particles of state from src to dst < src (compaction)."""
        if src == dst or n == 0:
            return
        for buf in (self.pos, self.vel, self.acc, self.mass):
            buf[dst:dst + n] = buf[src:src + n].clone()

    def read(self, offset: int, n: int):
        sl = slice(offset, offset + n)
        return self.pos[sl].cpu().numpy(), self.vel[sl].cpu().numpy()

    def sync(self) -> None:
        self.torch.cuda.synchronize()
        self._inflight.clear()


class Server:
    """Admission, per-round batching, retirement and latency bookkeeping (device work in the
    executor).  ``run(requests)`` replays arrival times against the wall clock."""

    def __init__(self, executor, energy: bool = True, clock=time.perf_counter, sym6=None, round_budget_s: float = 4e-3,
                 rate_estimate: float = 2e12, max_rounds_per_call: int = 64, policy: str = "srpt",
                 fill: float = 2.0 ** 30, on_result=None):
        if policy not in ("srpt", "all"):
            raise ValueError("policy must be 'srpt' or 'all'")
        self.ex = executor
        # "all": every active job advances every round.  "srpt": the arena is kept in order of
        # remaining work (least first) and the rounds advance the leading jobs only, as many as it
        # takes for a round to hold `fill` pair interactions (enough work to occupy the device), so
        # short jobs are not held to the round rate of the largest ones.
        self.policy = policy
        self.fill = float(fill)
        self.on_result = on_result  # called with every Result as it is recorded (progress, logging)
        self.energy = energy
        self.clock = clock
        # rounds are chained in one call while no job starts or ends, up to about round_budget_s of
        # estimated device time (so a job arriving meanwhile waits at most about that long)
        self.round_budget_s = round_budget_s
        self.rate_estimate = rate_estimate
        self.max_rounds_per_call = max_rounds_per_call
        self.sym6 = sym6 if sym6 is not None else nbody.nbody_sym6_coefficients()
        self.active: List[_Active] = []
        self.queue: List[Request] = []
        self.results: Dict[int, Result] = {}
        self.cancelled: set = set()
        self.rounds = 0
        self.interactions = 0

    # -- admission -----------------------------------------------------------------------
    def used(self) -> int:
        return sum(a.req.n for a in self.active)

    def fits(self, req: Request) -> bool:
        return self.used() + req.n <= self.ex.capacity and len(self.active) < self.ex.max_clusters

    def submit(self, req: Request) -> None:
        if req.n < 1 or req.steps < 0 or not (req.dt == req.dt) or req.eps < 0:
            self.results[req.jid] = Result(req.jid, "rejected", reason="invalid request")
            return
        if req.n > self.ex.capacity:
            self.results[req.jid] = Result(req.jid, "rejected", reason="larger than the device arena")
            return
        self.queue.append(req)

    def cancel(self, jid: int) -> None:
        self.cancelled.add(jid)

    def _admit(self, now: float) -> List[_Active]:
        """Admit queued jobs while they fit: in arrival order, stopping at the first that does not
        fit ("all"), or least work first, skipping those that do not fit yet ("srpt")."""
        new = []
        if self.policy == "srpt":
            self.queue.sort(key=lambda r: (r.interactions(), r.arrival, r.jid))
        i = 0
        while i < len(self.queue):
            req = self.queue[i]
            if req.jid in self.cancelled:
                self.queue.pop(i)
                self.results[req.jid] = Result(req.jid, "cancelled")
                continue
            if not self.fits(req):
                if self.policy == "srpt":
                    i += 1
                    continue
                break
            self.queue.pop(i)
            off = self.used()
            self.ex.load(off, req)
            sched = np.array(stage_schedule(req.integrator, req.dt, req.steps, self.sym6), dtype=np.float64)
            act = _Active(req, off, sched, admitted_at=now)
            self.active.append(act)
            new.append(act)
        if new and self.energy:
            e = self.ex.energy(new[0].offset, [a.req.n for a in new], [a.req.eps for a in new],
                               [a.req.field for a in new])
            for a, row in zip(new, e):
                a.energy0 = row
        if new and self.policy == "srpt":
            self._reorder()
        return new

    @staticmethod
    def remaining(a: _Active) -> int:
        """Pair interactions a job still needs."""
        return a.left * a.req.n * a.req.n

    def _reorder(self) -> None:
        """Rearrange the arena in order of remaining work (ties: arrival, then id)."""
        order = sorted(self.active, key=lambda a: (self.remaining(a), a.req.arrival, a.req.jid))
        if all(x is y for x, y in zip(order, self.active)):
            return
        self.ex.reorder([(a.offset, a.req.n) for a in order])
        off = 0
        for a in order:
            a.offset = off
            off += a.req.n
        self.active = order

    def batch(self) -> List[_Active]:
        """The jobs the next rounds advance: a prefix of the arena (see ``policy``)."""
        if self.policy == "all":
            return self.active
        tot = 0
        for i, a in enumerate(self.active):
            tot += a.req.n * a.req.n
            if tot >= self.fill:
                return self.active[:i + 1]
        return self.active

    # -- rounds --------------------------------------------------------------------------
    def chain_length(self, acts: Optional[List[_Active]] = None) -> int:
        """Rounds to run in one call: until the first job of the batch finishes, within the budget."""
        acts = self.active if acts is None else acts
        per_round = sum(a.req.n * a.req.n for a in acts) / self.rate_estimate
        budget = max(1, int(self.round_budget_s / max(per_round, 1e-12)))
        return max(1, min(min(a.left for a in acts), budget, self.max_rounds_per_call))

    def step_rounds(self, rounds: int = 1, acts: Optional[List[_Active]] = None) -> None:
        """``rounds`` rounds over the jobs ``acts`` (default: all active), a prefix of the arena."""
        acts = self.active if acts is None else acts
        coef = np.stack([a.schedule[a.cursor:a.cursor + rounds] for a in acts], axis=1)  # [R][B][3]
        self.ex.substeps([a.req.n for a in acts], [a.req.eps for a in acts], [a.req.field for a in acts], coef)
        self.rounds += rounds
        for a in acts:
            a.cursor += rounds
            self.interactions += rounds * a.req.n * a.req.n

    def step_round(self) -> None:
        self.step_rounds(1)

    def _retire(self, now_fn) -> int:
        done = [a for a in self.active if a.left == 0 or a.req.jid in self.cancelled]
        if not done:
            return 0
        for a in done:
            if a.req.jid in self.cancelled:
                self.results[a.req.jid] = Result(a.req.jid, "cancelled")
                continue
            e1 = None
            if self.energy:
                e1 = self.ex.energy(a.offset, [a.req.n], [a.req.eps], [a.req.field])[0]
            pos, vel = self.ex.read(a.offset, a.req.n)
            bad = (not np.all(np.isfinite(pos))) or (not np.all(np.isfinite(vel))) or (e1 is not None and e1[19] != 0)
            self.results[a.req.jid] = Result(a.req.jid, "failed" if bad else "done", now_fn() - a.req.arrival, pos,
                                             vel, a.energy0, e1, "non-finite state" if bad else "")
            if self.on_result:
                self.on_result(self.results[a.req.jid])
        # compaction: keep survivors in admission order, contiguous from 0
        keep = [a for a in self.active if a not in done]
        off = 0
        for a in keep:
            self.ex.move(a.offset, off, a.req.n)
            a.offset = off
            off += a.req.n
        self.active = keep
        return len(done)

    def run(self, requests: Sequence[Request], max_rounds: Optional[int] = None) -> Dict[int, Result]:
        """Serve the requests; arrival times are seconds after the start of the call."""
        pending = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        now_fn = lambda: self.clock() - t0
        i = 0
        while i < len(pending) or self.queue or self.active:
            now = now_fn()
            while i < len(pending) and pending[i].arrival <= now:
                self.submit(pending[i])
                i += 1
            self._admit(now)
            if not self.active:
                if i < len(pending) and not self.queue:
                    wait = pending[i].arrival - now_fn()
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                    continue
                if self.queue and not self.active:
                    # the head of the queue can never fit: reject it rather than stall
                    r = self.queue.pop(0)
                    self.results[r.jid] = Result(r.jid, "rejected", reason="does not fit")
                continue
            acts = self.batch()
            nr = self.chain_length(acts)
            if max_rounds is not None:
                nr = max(1, min(nr, max_rounds - self.rounds))
            self.step_rounds(nr, acts)
            if any(a.left == 0 for a in acts) or self.cancelled:
                self.ex.sync()
                self._retire(now_fn)
            if max_rounds is not None and self.rounds >= max_rounds:
                break
        self.ex.sync()
        return self.results


def latency_stats(results: Dict[int, Result], skip: int = 0) -> dict:
    lat = sorted(r.latency for j, r in results.items() if r.status == "done" and j >= skip)
    if not lat:
        return {"p50": float("nan"), "p99": float("nan"), "n": 0}
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)), "n": len(lat),
            "mean": float(np.mean(lat))}
