"""CPU stand-in for the server's device executor, backed by the FP64 oracle (tests only)."""
import numpy as np

import oracle


class FakeExecutor:
    def __init__(self, capacity, max_clusters, G=1.0, galaxy=None):
        self.capacity = capacity
        self.max_clusters = max_clusters
        self.G = G
        self.galaxy = galaxy
        self.pos = np.zeros((capacity, 3))
        self.vel = np.zeros((capacity, 3))
        self.acc = np.zeros((capacity, 3))
        self.mass = np.zeros(capacity)
        self.calls = []

    def load(self, offset, req):
        n = req.n
        self.pos[offset:offset + n] = req.pos
        self.vel[offset:offset + n] = req.vel
        self.mass[offset:offset + n] = req.mass
        self.acc[offset:offset + n] = 0.0

    def substeps(self, sizes, eps, fld, coef):
        for r in range(len(coef)):
            self.substep(sizes, eps, fld, coef[r][:, 0], coef[r][:, 1], coef[r][:, 2])

    def substep(self, sizes, eps, fld, kick_pre, drift, kick_post):
        self.calls.append(list(sizes))
        o = 0
        for n, e, f, kp, dr, kq in zip(sizes, eps, fld, kick_pre, drift, kick_post):
            sl = slice(o, o + n)
            self.vel[sl] = self.vel[sl] + kp * self.acc[sl]
            self.pos[sl] = self.pos[sl] + dr * self.vel[sl]
            self.acc[sl] = oracle.total_accel(self.pos[sl], self.mass[sl], self.G, e, bool(f), self.galaxy)
            self.vel[sl] = self.vel[sl] + kq * self.acc[sl]
            o += n

    def energy(self, offset, sizes, eps, fld):
        out = []
        o = offset
        for n, e, f in zip(sizes, eps, fld):
            sl = slice(o, o + n)
            r = oracle.energy(self.pos[sl], self.vel[sl], self.mass[sl], self.G, e, bool(f), self.galaxy)
            r[19] = 0.0 if np.all(np.isfinite(r[:19])) else 1.0
            out.append(r)
            o += n
        return np.array(out)

    def reorder(self, spans):
        self.reorders = getattr(self, "reorders", 0) + 1
        idx = np.concatenate([np.arange(o, o + n) for o, n in spans])
        for b in (self.pos, self.vel, self.acc, self.mass):
            b[:len(idx)] = b[idx]

    def move(self, src, dst, n):
        for b in (self.pos, self.vel, self.acc, self.mass):
            b[dst:dst + n] = b[src:src + n].copy()

    def read(self, offset, n):
        return self.pos[offset:offset + n].copy(), self.vel[offset:offset + n].copy()

    def sync(self):
        pass
