"""Several spatial domains of one particle set on one device (Sec. III.B).

The paper runs one domain per GPU: the particles are cut along the
space-filling curve into flop-balanced pieces (Sec. III.B.1), every domain
keys its particles in the one global box so its tree is a branch of one
global octree, and each domain walks its own tree plus the local essential
trees (LETs) of the others (Sec. III.B.2).  Here every domain is a library
context on the same device; the exchange of particles and LETs between
processes becomes device-to-device copies inside the library.  Every step
runs in the library's kernels; this module only sequences the calls.
"""
from __future__ import annotations

from .binding import Tree


class Domains:
    """p domains of the particles (pos [N,3], mass [N], optional vel):
    a global tree gives the box and the walk costs that the cuts balance,
    then each domain gets its own tree, boundary tree and merged LET."""

    def __init__(self, pos, mass, p, theta, eps, vel=None, cap=1.3, max_boundary=1024,
                 nleaf=16, ncrit=64, curve="morton", far_fp16=False, sampling=None):
        """sampling = (px, py, m1, m2) cuts by the two-level sampling with
        px * py = p processes and m1, m2 samples per process and level;
        None cuts exactly over all keys."""
        n = int(mass.shape[0])
        self.n, self.p = n, int(p)
        self.theta, self.eps = float(theta), float(eps)
        g = Tree(n, nleaf, ncrit, far_fp16, curve=curve)
        if vel is None:
            g.build(pos, mass)
        else:
            g.set_state(pos, vel, mass)
        g.force(theta, eps)  # costs of the cut: this walk's interaction counts
        self.bounds = None
        if sampling is None:
            self.cuts = g.decompose(self.p, cap)
        else:
            px, py, m1, m2 = sampling
            if px * py != self.p:
                raise ValueError("sampling needs px * py == p")
            self.cuts, self.bounds = g.decompose_sampled(px, py, m1, m2, cap)
        box = g.export("box")
        self.lo, self.side = box[:3].copy(), float(box[3])
        self.trees, self.ids, self.slots = [], [], []
        for d in range(self.p):
            lo, hi = int(self.cuts[d]), int(self.cuts[d + 1])
            if hi == lo:
                continue
            dpos, dvel, dmass, dids = g.extract(lo, hi)
            t = Tree(hi - lo, nleaf, ncrit, far_fp16, curve=curve)
            t.set_box(self.lo, self.side)
            t.set_state(dpos, dvel, dmass)
            t.boundary(max_boundary)
            self.trees.append(t)
            self.ids.append(dids)
            self.slots.append((lo, hi))
        g.close()
        self.info = None
        self._streams = []

    def build_lets(self, theta=None):
        """LETs of every other domain for each domain; returns per domain
        the info rows of the sources (boundary tree sufficed, cells,
        particles)."""
        th = self.theta if theta is None else float(theta)
        self.info = []
        for d, t in enumerate(self.trees):
            others = [u for e, u in enumerate(self.trees) if e != d]
            self.info.append(t.let_build(others, th))
        self.theta = th
        return self.info

    def forces(self, eps=None, acc=None, pot=None, streams=4):
        """(acc [N,3], pot [N]) in the caller order of the particles given to
        the constructor: each domain's own walk plus its merged LET walk.
        The domains write disjoint rows, so they run on up to `streams` HIP
        streams at once (default priority), the tail of one domain's walk
        overlapping the next; the caller's stream waits for all of them."""
        import torch
        e = self.eps if eps is None else float(eps)
        if self.info is None:
            self.build_lets()
        if acc is None:
            acc = torch.empty((self.n, 3), dtype=torch.float32, device="cuda")
        if pot is None:
            pot = torch.empty((self.n,), dtype=torch.float32, device="cuda")
        cur = torch.cuda.current_stream()
        k = max(1, min(int(streams), len(self.trees)))
        if k == 1:
            for t, ids in zip(self.trees, self.ids):
                t.force_let(self.theta, e, rows=ids, acc=acc, pot=pot)
            return acc, pot
        if len(self._streams) < k:
            self._streams += [torch.cuda.Stream() for _ in range(k - len(self._streams))]
        for s in self._streams[:k]:
            s.wait_stream(cur)
        for i, (t, ids) in enumerate(zip(self.trees, self.ids)):
            t.force_let(self.theta, e, rows=ids, acc=acc, pot=pot, stream=self._streams[i % k])
        for s in self._streams[:k]:
            cur.wait_stream(s)
        return acc, pot

    def close(self):
        for t in self.trees:
            t.close()
        self.trees = []
