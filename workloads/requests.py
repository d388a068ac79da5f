"""Seeded request streams for the serving loop.

A request is one reservoir model plus a short sequence of source vectors
(repeated solves on the same grid: a moved or rescaled source/sink pair),
arriving at a Poisson-process time.  Large requests come from a small pool
of layered five-spot models; small ones from a pool of ensemble members.
Only inputs are built here; no solver arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .grids import make_config1, make_config3_member, rng_for


@dataclass
class Request:
    rid: int
    arrival: float
    problem: object
    partitions: list
    sources: list
    kind: str
    # filled in by the server
    admitted: float = 0.0
    finished: float = 0.0
    iters: list = field(default_factory=list)
    relres: list = field(default_factory=list)
    status: list = field(default_factory=list)
    dyn_blocks: list = field(default_factory=list)
    solutions: list = field(default_factory=list)
    error: str = ""

    @property
    def cells(self) -> int:
        return int(self.problem.n_active) * len(self.sources)


def source_sequence(prob, rng, k):
    """k sources: the model's own source plus a source/sink pair of strength
    s at two random active cells; each repeat moves one end of the pair to a
    new random cell or rescales the pair by U[0.5, 1.5]."""
    act = np.nonzero(prob.active)[0]
    base = np.asarray(prob.source, dtype=np.float64)
    s = 1.0 if base.sum() == 0 else 0.5 * float(np.abs(base).sum())
    a, b = rng.choice(act, 2, replace=False)
    out = []
    for n in range(k):
        if n > 0:
            if rng.uniform() < 0.5:
                if rng.uniform() < 0.5:
                    a = rng.choice(act)
                else:
                    b = rng.choice(act)
                if a == b:
                    b = act[(np.searchsorted(act, a) + 1) % act.size]
            else:
                s *= rng.uniform(0.5, 1.5)
        q = base.copy()
        q[a] += s
        q[b] -= s
        out.append(q)
    return out


LARGE_PARTS = [{"kind": "cartesian", "coarse_dims": (10, 10, 5)}, {"kind": "cartesian", "coarse_dims": (6, 22, 17)}]
SMALL_PARTS = [{"kind": "cartesian", "coarse_dims": (8, 8, 4)}]


def poisson_stream(n_requests, rate, p_large=0.1, large_pool=4, small_pool=16, seed=0, large_dims=(60, 220, 85)):
    """n_requests requests with exponential gaps of mean 1/rate; each is large
    (a layered five-spot model from a pool) with probability p_large, else an
    ensemble member from a pool; k ~ U{1..5} solves each."""
    rng = rng_for(5, seed)
    larges = [make_config1(dims=large_dims, seed=s) for s in range(large_pool)]
    smalls = [make_config3_member(m) for m in range(small_pool)]
    t = 0.0
    reqs = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate)
        large = rng.uniform() < p_large
        prob = larges[rng.integers(len(larges))] if large else smalls[rng.integers(len(smalls))]
        k = int(rng.integers(1, 6))
        reqs.append(Request(r, t, prob, LARGE_PARTS if large else SMALL_PARTS, source_sequence(prob, rng, k),
                            "large" if large else "small"))
    return reqs


def ensemble_batch(n_members, seed=0):
    """A batch of ensemble members (correlation length, size and permeability
    from the member's seed), all available at time 0, one solve each with the
    member's own source."""
    reqs = []
    for m in range(n_members):
        prob = make_config3_member(m + 1000 * seed)
        reqs.append(Request(m, 0.0, prob, SMALL_PARTS, [np.asarray(prob.source, dtype=np.float64)], "member"))
    return reqs
