"""Seeded serving workload: Poisson arrivals of solve requests.

Arrival gaps are exponential with mean 1/rate from default_rng(seed_arrival).
Each request draws, from default_rng(seed_req) in this order: the dimension
(2 or 3), the number of macros k in [1, kmax], the level in the range of its
dimension, a seed for its affine map and a seed for its right-hand side.  The
mesh is ceil(k/2) unit squares in a strip cut along a diagonal (first k
triangles) or ceil(k/6) unit cubes in a row, 6 Kuhn tetrahedra each (first k),
under a seeded affine map (condition number of J at most 10).  The right-hand
side is U[-1, 1) on interior DoFs and 0 on the Dirichlet boundary.

No part of the method's arithmetic lives here.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import workloads as W


@dataclass
class Req:
    t: float          # arrival time from the start of the run (s)
    dim: int
    k: int
    level: int
    coords: np.ndarray
    cells: np.ndarray
    rhs_seed: int
    tol: float


def requests(n: int = 2000, rate: float = 200.0, levels2=(5, 11), levels3=(5, 11), kmax: int = 64,
             tol: float = 1e-8, seed_arrival: int = 6, seed_req: int = 7) -> list[Req]:
    ra = np.random.default_rng(seed_arrival)
    t = np.cumsum(ra.exponential(1.0 / rate, n))
    rr = np.random.default_rng(seed_req)
    out = []
    for i in range(n):
        dim = int(rr.integers(2, 4))
        k = int(rr.integers(1, kmax + 1))
        lo, hi = levels2 if dim == 2 else levels3
        level = int(rr.integers(lo, hi + 1))
        aff_seed = int(rr.integers(0, 2 ** 31))
        rhs_seed = int(rr.integers(0, 2 ** 31))
        co, ce = W.strip_2d(k) if dim == 2 else W.strip_3d(k)
        J, tr = W.random_affine(dim, aff_seed)
        out.append(Req(float(t[i]), dim, k, level, W.apply_affine(co, J, tr), ce, rhs_seed, tol))
    return out


def replay(server, reqs: list[Req], time_scale: float = 1.0):
    """Submits reqs to server at their arrival times (real time, scaled);
    returns (futures, t_start, t_last_submit)."""
    t0 = time.perf_counter()
    futs = []
    for r in reqs:
        target = t0 + r.t * time_scale
        while True:
            now = time.perf_counter()
            if now >= target:
                break
            time.sleep(min(target - now, 0.002))
        futs.append(server.submit(r.dim, r.coords, r.cells, r.level, r.rhs_seed, r.tol, t_arrival=target))
    return futs, t0, time.perf_counter()
