"""Seeded synthetic interior-point KKT sequences shaped like AC optimal power flow.

This module only draws random numbers and assembles matrices; it holds none of the
solver's arithmetic, so both the CPU oracle and the GPU path can consume its output.

The matrix is the z-eliminated Newton system of an interior-point method (the symmetric
block system of Section II, eq. (12)), written with the constraint Jacobian J of size m x n
in the lower-left block:

    K_t = [[H + D_t + delta*I,  J^T       ],
           [J,                  -delta_c*I]]

Grids stand in for the TAMU synthetic grids of Section II / Table I (not available here):

* buses are uniform random points in the unit square; candidate branches join each bus to
  its 7 nearest neighbours; a random spanning tree (minimum spanning tree of the candidate
  graph under i.i.d. uniform weights, i.e. Kruskal on a random order) makes the grid
  connected, and further candidates are added in random order until the branch count is
  round(avg_degree * buses / 2).  Local edges keep the pattern irregular and very sparse
  with no dense blocks, as Section II and III describe for grid KKT systems;
* generators sit on round(gen_frac * buses) distinct random buses;
* primal variables: Vm, Va per bus; Pg, Qg per generator; one slack per flow-limit row;
  constraints: P- and Q-balance per bus and `flows_per_branch` flow-limit rows per branch;
* H is the sum over branches of a symmetrised 4x4 N(0,1) block on (Vm_i, Va_i, Vm_j, Va_j);
  J entries are N(0,1); D is diagonal on all primal variables.

Value schedules (D_y = mu Y^-2 widens as mu -> 0, Section II):

* "fixed":   D = 10^U(-4,4); every stored value of step t is multiplied by (1 + 0.05 z),
             z ~ N(0,1) drawn per symmetric pair;
* "widening": u_i ~ U(-1,1) fixed; D_i(t) = 10^(e_t u_i), e_t = 2 + 8 t/(T-1); H and J
             are multiplied by (1 + 0.05 z) per step; delta and delta_c are constant.

Seeds: numpy.random.default_rng(SeedSequence([0, config_id, stream, k])) with streams
0 graph, 1 generators, 2 base values, 3 D, 4 per-step perturbation (k = t), 5 RHS (k = t).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
from scipy.sparse import csgraph
from scipy.spatial import cKDTree

__all__ = ["GridSpec", "KKTSequence", "CONFIGS", "config", "make_sequence", "closed_form_sizes", "batch_specs",
           "serve_specs", "serve_trace", "SERVE_SIZES", "SERVE_PROBS"]


@dataclasses.dataclass(frozen=True)
class GridSpec:
    name: str
    config_id: int
    buses: int
    avg_degree: float
    gen_frac: float
    steps: int
    schedule: str            # "fixed" or "widening"
    flows_per_branch: int = 2
    delta: float = 1e-8
    delta_c: float = 1e-8
    knn: int = 7


# The three plain-FP64 workloads: 200-bus (10 steps), 25k-bus-shaped (30 steps) and the
# 70k-bus-shaped headline case (50 steps).
CONFIGS = (
    GridSpec("grid200", 0, 200, 2.7, 0.20, 10, "fixed"),
    GridSpec("grid25k", 1, 25_000, 2.5, 0.25, 30, "widening"),
    GridSpec("grid70k", 2, 70_000, 2.5, 0.25, 50, "widening"),
)


def config(i: int) -> GridSpec:
    return CONFIGS[i]


def small(buses: int, *, config_id: int = 100, steps: int = 4, schedule: str = "widening",
          avg_degree: float = 2.5, gen_frac: float = 0.25, flows: int = 2) -> GridSpec:
    """A reduced grid with the same generator rules (for tests)."""
    return GridSpec(f"grid{buses}_s{config_id}", config_id, buses, avg_degree, gen_frac,
                    steps, schedule, flows)


def batch_specs(patterns: int = 8, steps: int = 8, lo: int = 1_000, hi: int = 10_000,
                config_id: int = 3) -> list[GridSpec]:
    """The batched workload: `patterns` grids whose bus counts are drawn log-uniform in
    [lo, hi] (SeedSequence([0, config_id, 6, 0])), same generator rules, `steps` value sets
    each on the widening schedule.  Pattern k uses config id 100 * config_id + k."""
    rng = np.random.default_rng(np.random.SeedSequence([0, config_id, 6, 0]))
    buses = np.round(np.exp(rng.uniform(np.log(lo), np.log(hi), patterns))).astype(int)
    return [GridSpec(f"batch{k}_{int(b)}", 100 * config_id + k, int(b), 2.5, 0.25, steps, "widening")
            for k, b in enumerate(buses)]


SERVE_SIZES = (500, 2_000, 10_000, 25_000)
SERVE_PROBS = (0.4, 0.3, 0.2, 0.1)


def serve_specs(steps: int = 16, config_id: int = 4) -> list[GridSpec]:
    """One pattern per serving grid size, `steps` value sets each (widening schedule);
    pattern k uses config id 100 * config_id + k."""
    return [GridSpec(f"serve{k}_{b}", 100 * config_id + k, b, 2.5, 0.25, steps, "widening")
            for k, b in enumerate(SERVE_SIZES)]


def serve_trace(rate: float, count: int, steps: int = 16, config_id: int = 4, seed_k: int = 0):
    """Poisson arrivals of `count` requests at mean `rate` per second: (arrival time s,
    pattern index drawn with SERVE_PROBS, value-set index, right-hand sides 1..4), from
    SeedSequence([0, config_id, 7, seed_k])."""
    rng = np.random.default_rng(np.random.SeedSequence([0, config_id, 7, seed_k]))
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    pat = rng.choice(len(SERVE_SIZES), size=count, p=SERVE_PROBS)
    val = rng.integers(0, steps, count)
    nrhs = rng.integers(1, 5, count)
    return [(float(a), int(p), int(v), int(r)) for a, p, v, r in zip(t, pat, val, nrhs)]


def closed_form_sizes(buses: int, gens: int, branches: int, flows: int) -> tuple[int, int]:
    """(N, nnz) of the assembled KKT on a simple connected graph."""
    n = 4 * buses + 2 * gens + 2 * flows * branches
    nnz = 14 * buses + (24 + 12 * flows) * branches + 6 * gens
    return n, nnz


def _rng(spec: GridSpec, stream: int, k: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([0, spec.config_id, stream, k]))


def _graph(spec: GridSpec) -> tuple[np.ndarray, np.ndarray]:
    """Branch list (Br x 2, i < j, sorted) and bus coordinates."""
    rng = _rng(spec, 0)
    B = spec.buses
    pts = rng.random((B, 2))
    k = min(spec.knn, B - 1)
    _, nn = cKDTree(pts).query(pts, k + 1)
    a = np.repeat(np.arange(B), k)
    b = nn[:, 1:].reshape(-1)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    cand = np.unique(np.stack([lo, hi], 1), axis=0)
    # bridge components of the candidate graph, if any (rare): join each component that
    # does not hold bus 0 to its nearest bus outside it
    while True:
        g = sp.coo_matrix((np.ones(len(cand)), (cand[:, 0], cand[:, 1])), shape=(B, B))
        ncomp, lab = csgraph.connected_components(g, directed=False)
        if ncomp == 1:
            break
        comp = lab[np.argmax(lab != lab[0])]
        inside = np.flatnonzero(lab == comp)
        outside = np.flatnonzero(lab != comp)
        d, j = cKDTree(pts[outside]).query(pts[inside], 1)
        t = int(np.argmin(d))
        u, v = int(inside[t]), int(outside[j[t]])
        cand = np.unique(np.vstack([cand, [[min(u, v), max(u, v)]]]), axis=0)
    w = rng.random(len(cand)) + 1e-3          # i.i.d. positive weights
    g = sp.coo_matrix((w, (cand[:, 0], cand[:, 1])), shape=(B, B)).tocsr()
    t = csgraph.minimum_spanning_tree(g).tocoo()
    tree = np.unique(np.stack([np.minimum(t.row, t.col), np.maximum(t.row, t.col)], 1), axis=0)
    # remaining candidates in a random order
    key_all = cand[:, 0].astype(np.int64) * B + cand[:, 1]
    key_tree = tree[:, 0].astype(np.int64) * B + tree[:, 1]
    rest = cand[~np.isin(key_all, key_tree)]
    rest = rest[rng.permutation(len(rest))]
    target = int(round(spec.avg_degree * B / 2))
    extra = rest[: max(0, target - len(tree))]
    E = np.unique(np.vstack([tree, extra]), axis=0)
    return E.astype(np.int64), pts


@dataclasses.dataclass
class KKTSequence:
    spec: GridSpec
    n: int                      # KKT order N
    n_primal: int
    rowptr: np.ndarray          # int64[N+1]
    colind: np.ndarray          # int32[nnz], sorted within rows
    pair: np.ndarray            # int64[nnz] symmetric-pair id of each stored entry
    branches: np.ndarray        # int64[Br, 2]
    gen_bus: np.ndarray         # int64[G]
    _hj: np.ndarray             # base H + J values (diag of primal holds H_ii only)
    _dslot: np.ndarray          # CSR slot of each primal diagonal
    _cslot: np.ndarray          # CSR slot of each dual diagonal
    _dbase: np.ndarray          # log10 D ("fixed") or u ("widening")

    @property
    def nnz(self) -> int:
        return int(self.colind.shape[0])

    @property
    def steps(self) -> int:
        return self.spec.steps

    def values(self, t: int) -> np.ndarray:
        """float64[nnz] values of K_t in CSR order."""
        s = self.spec
        z = _rng(s, 4, t).standard_normal(int(self.pair.max()) + 1)
        f = 1.0 + 0.05 * z[self.pair]
        v = np.zeros(self.nnz)
        if s.schedule == "fixed":
            v += self._hj
            v[self._dslot] += 10.0 ** self._dbase + s.delta
            v[self._cslot] += -s.delta_c
            return v * f
        T = max(s.steps, 2)
        e = 2.0 + 8.0 * t / (T - 1)
        v += self._hj * f
        v[self._dslot] += 10.0 ** (e * self._dbase) + s.delta
        v[self._cslot] += -s.delta_c
        return v

    def rhs(self, t: int, nrhs: int = 1) -> np.ndarray:
        b = _rng(self.spec, 5, t).standard_normal((nrhs, self.n))
        return b[0] if nrhs == 1 else b

    def scipy(self, t: int) -> sp.csr_matrix:
        return sp.csr_matrix((self.values(t), self.colind, self.rowptr), shape=(self.n, self.n))


def make_sequence(spec: GridSpec) -> KKTSequence:
    E, _ = _graph(spec)
    B, Br, F = spec.buses, len(E), spec.flows_per_branch
    G = int(round(spec.gen_frac * B))
    gen_bus = _rng(spec, 1).choice(B, G, replace=False).astype(np.int64)
    n_p = 2 * B + 2 * G + F * Br
    m = 2 * B + F * Br
    N = n_p + m
    vm, va = 2 * np.arange(B), 2 * np.arange(B) + 1
    pg, qg = 2 * B + 2 * np.arange(G), 2 * B + 2 * np.arange(G) + 1
    slack0 = 2 * B + 2 * G
    pbal, qbal = n_p + 2 * np.arange(B), n_p + 2 * np.arange(B) + 1
    flow0 = n_p + 2 * B

    rv = _rng(spec, 2)
    # Hessian blocks per branch on (Vm_i, Va_i, Vm_j, Va_j)
    blk = rv.standard_normal((Br, 4, 4))
    blk = 0.5 * (blk + blk.transpose(0, 2, 1))
    idx = np.stack([vm[E[:, 0]], va[E[:, 0]], vm[E[:, 1]], va[E[:, 1]]], 1)
    hr = np.repeat(idx, 4, axis=1).reshape(-1)
    hc = np.tile(idx, (1, 4)).reshape(-1)
    hv = blk.reshape(-1)
    # Jacobian entries (row, col) in a fixed construction order
    jr, jc = [], []
    for rows in (pbal, qbal):
        jr += [rows, rows]
        jc += [vm, va]
        for (a, b) in ((0, 1), (1, 0)):
            jr += [rows[E[:, a]], rows[E[:, a]]]
            jc += [vm[E[:, b]], va[E[:, b]]]
    jr += [pbal[gen_bus], qbal[gen_bus]]
    jc += [pg, qg]
    fr = flow0 + F * np.arange(Br)[:, None] + np.arange(F)[None, :]          # Br x F
    fs = slack0 + F * np.arange(Br)[:, None] + np.arange(F)[None, :]
    for cols in (vm[E[:, 0]], va[E[:, 0]], vm[E[:, 1]], va[E[:, 1]]):
        jr.append(fr.reshape(-1))
        jc.append(np.repeat(cols, F))
    jr.append(fr.reshape(-1))
    jc.append(fs.reshape(-1))
    jr = np.concatenate(jr)
    jc = np.concatenate(jc)
    jv = rv.standard_normal(len(jr))
    dprim = np.arange(n_p)
    ddual = np.arange(n_p, N)
    rows = np.concatenate([hr, jr, jc, dprim, ddual])
    cols = np.concatenate([hc, jc, jr, dprim, ddual])
    vals = np.concatenate([hv, jv, jv, np.zeros(n_p), np.zeros(m)])
    A = sp.coo_matrix((vals, (rows, cols)), shape=(N, N)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    rowptr = A.indptr.astype(np.int64)
    colind = A.indices.astype(np.int32)
    hj = A.data.astype(np.float64).copy()
    # pair ids: index of (min, max) among upper-triangle entries
    r = np.repeat(np.arange(N, dtype=np.int64), np.diff(rowptr))
    c = colind.astype(np.int64)
    key = np.minimum(r, c) * N + np.maximum(r, c)
    _, pair = np.unique(key, return_inverse=True)
    # exact symmetry: every entry takes the value summed at its upper-triangle position
    up = r <= c
    byp = np.zeros(int(pair.max()) + 1)
    byp[pair[up]] = hj[up]
    hj = byp[pair]
    diag_slot = np.flatnonzero(r == c)
    assert len(diag_slot) == N
    dslot = diag_slot[:n_p]
    cslot = diag_slot[n_p:]
    rd = _rng(spec, 3)
    if spec.schedule == "fixed":
        dbase = rd.uniform(-4.0, 4.0, n_p)
    elif spec.schedule == "widening":
        dbase = rd.uniform(-1.0, 1.0, n_p)
    else:
        raise ValueError(spec.schedule)
    return KKTSequence(spec, N, n_p, rowptr, colind, pair.astype(np.int64), E, gen_bus,
                       hj, dslot, cslot, dbase)
