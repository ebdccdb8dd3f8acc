"""Seeded synthetic meshed transmission grids and load scenarios.

This module only draws random numbers and builds graphs.  It holds none of
the power-flow arithmetic: no admittance matrix, no injections, no Newton
step.  Both the CPU oracle and the GPU library consume the arrays it returns,
so the two sides always see identical inputs.

Recipe (stands in for the paper's pandapower cases, which are not available;
the paper's own scenario scheme is the uniform +-10% load perturbation of its
experimental-setup section, kept here as ``scenario_mode="uniform10"``):

* bus coordinates ~ U[0,1]^2; candidate branches = symmetric 6-nearest-
  neighbour graph, so the meshing is near-planar like a real grid;
* a random spanning tree (Kruskal over U(0,1) weights on the candidates),
  plus the requested number of extra branches drawn uniformly, without
  repetition, from the remaining candidates;
* bus 0 is the slack (|V| = 1, angle 0); a uniform random subset of the
  other buses is PV with |V| setpoint ~ U(0.98, 1.05); the rest are PQ;
* branch r ~ U(0.005, 0.05), x = r * U(3, 10), total line charging
  b ~ U(0, 0.05) (pi model, no taps, no shunts);
* PQ-bus nominal load P0 ~ U(0.1, 1.0), Q0 = P0 * tan(acos(pf)),
  pf ~ U(0.9, 0.98); PV and slack buses carry no load;
* scenario b scales each PQ load by s ~ LogNormal(0, sigma) (same factor
  for P and Q), and every PV bus dispatches 0.95 * sum_b(p_d) / n_PV;
* ``load_factor`` < 1 scales the nominal loads (and hence the dispatch)
  down; it is a feasibility back-off (the recipe's literal load levels do
  not converge from the flat start on the larger grids) and its per-grid
  value was chosen by ``oracle/calibrate_load_factor.py``;
* ``z_scale`` multiplies the drawn r, x and b: per-unit line parameters grow
  with line length, and on the 9241-bus grid (same unit square) the lines
  are sqrt(9241/118) times shorter than on the 118-bus grid.  Without it no
  load level converges from the flat start on that grid.

Random streams: ``numpy.random.default_rng(SeedSequence([seed, grid_id]))``
for the network, ``SeedSequence([seed, grid_id, 1])`` for the scenarios, with
the draw order fixed as written in :func:`make_network` and
:func:`make_scenarios`.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PQ, PV, SLACK = 0, 1, 2


@dataclass(frozen=True)
class GridSpec:
    name: str
    grid_id: int
    n_bus: int
    n_pv: int
    n_branch: int          # spanning tree (n_bus - 1) + extra branches
    batch: int
    sigma: float           # LogNormal sigma of the per-(scenario, bus) load scale
    tol: float             # Newton tolerance on ||F1||_inf in pu
    load_factor: float = 1.0
    z_scale: float = 1.0   # multiplies the drawn r, x and b (per-unit parameters ~ line length)
    knn: int = 6


# Five synthetic workloads.  Branch counts: 14-bus tree + 6 extra; 118-bus
# tree + 60 extra; the others from their average degree (2 * n_branch / n_bus).
SPECS = {
    "c0": GridSpec("c0", 0, 14, 4, 19, 64, 0.10, 1e-8, load_factor=0.9 ** 8),
    "c1": GridSpec("c1", 1, 118, 53, 177, 1024, 0.10, 1e-8, load_factor=0.9 ** 7),
    "c2": GridSpec("c2", 2, 1354, 260, 1896, 4096, 0.15, 1e-8, load_factor=0.9 ** 26),
    "c3": GridSpec("c3", 3, 300, 69, 420, 2048, 0.10, 1e-10, load_factor=0.9 ** 17),
    "c4": GridSpec("c4", 4, 9241, 1400, 12013, 256, 0.10, 1e-8, load_factor=0.9 ** 34,
                   z_scale=(118 / 9241) ** 0.5),
}


@dataclass
class Network:
    """A grid: bus types, branch list (pi model) and nominal setpoints/loads."""
    name: str
    n_bus: int
    bus_type: np.ndarray       # int32 [n_bus], PQ=0 PV=1 SLACK=2
    f: np.ndarray              # int32 [n_branch] from bus
    t: np.ndarray              # int32 [n_branch] to bus
    r: np.ndarray              # float64 [n_branch] series resistance (pu)
    x: np.ndarray              # float64 [n_branch] series reactance (pu)
    bc: np.ndarray             # float64 [n_branch] total line charging (pu)
    vset: np.ndarray           # float64 [n_bus]: |V| setpoint on PV/slack, 1.0 on PQ
    p0: np.ndarray             # float64 [n_bus] nominal active load (PQ buses only)
    q0: np.ndarray             # float64 [n_bus] nominal reactive load
    coords: np.ndarray = field(repr=False, default=None)

    @property
    def n_branch(self) -> int:
        return int(self.f.shape[0])

    @property
    def pq(self) -> np.ndarray:
        return np.flatnonzero(self.bus_type == PQ)

    @property
    def pv(self) -> np.ndarray:
        return np.flatnonzero(self.bus_type == PV)


@dataclass
class Scenarios:
    """A batch of operating points on one network, all arrays [batch, n_bus]."""
    pd: np.ndarray
    qd: np.ndarray
    pg: np.ndarray
    vset: np.ndarray

    @property
    def batch(self) -> int:
        return int(self.pd.shape[0])

    def subset(self, idx) -> "Scenarios":
        idx = np.asarray(idx)
        return Scenarios(self.pd[idx].copy(), self.qd[idx].copy(),
                         self.pg[idx].copy(), self.vset[idx].copy())


class _DSU:
    def __init__(self, n):
        self.p = np.arange(n)

    def find(self, a):
        p = self.p
        while p[a] != a:
            p[a] = p[p[a]]
            a = p[a]
        return a

    def union(self, a, b):
        ra, rb = self.find(a), self.find(b)
        if ra == rb:
            return False
        if ra < rb:
            ra, rb = rb, ra
        self.p[ra] = rb
        return True


def _knn_candidates(coords: np.ndarray, k: int) -> np.ndarray:
    """Symmetric k-nearest-neighbour edge list, sorted, as [m, 2] with a < b."""
    from scipy.spatial import cKDTree
    n = coords.shape[0]
    kk = min(k + 1, n)
    _, nbr = cKDTree(coords).query(coords, k=kk)
    a = np.repeat(np.arange(n), kk - 1)
    b = nbr[:, 1:].reshape(-1)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    keep = lo != hi
    e = np.unique(np.stack([lo[keep], hi[keep]], axis=1), axis=0)
    return e


def _connect_components(coords, edges, n):
    """Add shortest inter-component links until the candidate graph is connected."""
    edges = [tuple(e) for e in edges]
    while True:
        dsu = _DSU(n)
        for a, b in edges:
            dsu.union(a, b)
        roots = np.array([dsu.find(i) for i in range(n)])
        comps = np.unique(roots)
        if comps.size == 1:
            return np.array(sorted(set(edges)), dtype=np.int64)
        sizes = [(np.sum(roots == c), c) for c in comps]
        _, smallest = min(sizes)
        inside = np.flatnonzero(roots == smallest)
        outside = np.flatnonzero(roots != smallest)
        d = ((coords[inside, None, :] - coords[None, outside, :]) ** 2).sum(-1)
        ii, oo = np.unravel_index(np.argmin(d), d.shape)
        a, b = int(inside[ii]), int(outside[oo])
        edges.append((min(a, b), max(a, b)))


def make_network(spec: GridSpec, seed: int = 0) -> Network:
    """Draw one grid.  Draw order: coordinates, tree weights, extra branches,
    PV set, branch r / x-ratio / b, PV setpoints, nominal P0, power factor."""
    n = spec.n_bus
    rng = np.random.default_rng(np.random.SeedSequence([seed, spec.grid_id]))
    coords = rng.random((n, 2))
    cand = _knn_candidates(coords, spec.knn)
    cand = _connect_components(coords, cand, n)
    w = rng.random(cand.shape[0])
    order = np.argsort(w, kind="stable")
    dsu = _DSU(n)
    in_tree = np.zeros(cand.shape[0], dtype=bool)
    for e in order:
        a, b = cand[e]
        if dsu.union(int(a), int(b)):
            in_tree[e] = True
    assert in_tree.sum() == n - 1, "candidate graph is not connected"
    n_extra = spec.n_branch - (n - 1)
    rest = np.flatnonzero(~in_tree)
    if n_extra > rest.size:
        raise ValueError(f"{spec.name}: need {n_extra} extra branches, only {rest.size} candidates")
    extra = np.sort(rng.choice(rest, size=n_extra, replace=False)) if n_extra > 0 else rest[:0]
    chosen = np.concatenate([np.flatnonzero(in_tree), extra])
    chosen.sort()
    edges = cand[chosen]
    m = edges.shape[0]

    bus_type = np.zeros(n, dtype=np.int32)
    bus_type[0] = SLACK
    pv = np.sort(rng.choice(np.arange(1, n), size=spec.n_pv, replace=False))
    bus_type[pv] = PV

    r = rng.uniform(0.005, 0.05, m) * spec.z_scale
    x = r * rng.uniform(3.0, 10.0, m)
    bc = rng.uniform(0.0, 0.05, m) * spec.z_scale

    vset = np.ones(n)
    vset[pv] = rng.uniform(0.98, 1.05, pv.size)

    pq = np.flatnonzero(bus_type == PQ)
    p_nom = rng.uniform(0.1, 1.0, pq.size)
    pf = rng.uniform(0.9, 0.98, pq.size)
    p0 = np.zeros(n)
    q0 = np.zeros(n)
    p0[pq] = p_nom * spec.load_factor
    q0[pq] = p_nom * np.tan(np.arccos(pf)) * spec.load_factor

    return Network(spec.name, n, bus_type, edges[:, 0].astype(np.int32),
                   edges[:, 1].astype(np.int32), r, x, bc, vset, p0, q0, coords)


def make_scenarios(net: Network, spec: GridSpec, batch: int | None = None,
                   seed: int = 0, scenario_mode: str = "lognormal",
                   sigma: float | None = None) -> Scenarios:
    """Draw ``batch`` load scenarios on ``net``.

    ``lognormal``: one LogNormal(0, sigma) factor per (scenario, PQ bus)
    multiplies both P and Q.  ``uniform10``: independent factors
    (1 + eps_P), (1 + eps_Q) with eps ~ U[-0.1, 0.1] per scenario and load.
    """
    batch = spec.batch if batch is None else int(batch)
    sigma = spec.sigma if sigma is None else float(sigma)
    rng = np.random.default_rng(np.random.SeedSequence([seed, spec.grid_id, 1]))
    n = net.n_bus
    pq, pv = net.pq, net.pv
    pd = np.zeros((batch, n))
    qd = np.zeros((batch, n))
    if scenario_mode == "lognormal":
        s = rng.lognormal(0.0, sigma, size=(batch, pq.size))
        pd[:, pq] = net.p0[pq] * s
        qd[:, pq] = net.q0[pq] * s
    elif scenario_mode == "uniform10":
        ep = rng.uniform(-0.1, 0.1, size=(batch, pq.size))
        eq = rng.uniform(-0.1, 0.1, size=(batch, pq.size))
        pd[:, pq] = net.p0[pq] * (1.0 + ep)
        qd[:, pq] = net.q0[pq] * (1.0 + eq)
    else:
        raise ValueError(scenario_mode)
    pg = np.zeros((batch, n))
    if pv.size:
        pg[:, pv] = (0.95 * pd.sum(axis=1) / pv.size)[:, None]
    vset = np.broadcast_to(net.vset, (batch, n)).copy()
    return Scenarios(pd, qd, pg, vset)


def make_case(name: str, batch: int | None = None, seed: int = 0, **kw):
    """(spec, network, scenarios) for one of the named workloads."""
    spec = SPECS[name]
    net = make_network(spec, seed)
    return spec, net, make_scenarios(net, spec, batch, seed, **kw)
