"""ORACLE -- test infrastructure. A plain-Python model of a GPOP run.

Follows the paper's own structure, for tiny graphs only:

* index-range partitions of q vertices (graph partitioning, Sec. 3.1.1);
* aggregated messages, one per (source vertex, neighbouring partition) pair,
  each carrying the source's value and its out-neighbours in that partition
  (message generation, Sec. 3.1.2);
* the partition-node bipartite layout N_i^p(q) for partition-centric scatter
  (Algorithm 3);
* one iteration = scatter of every partition with active vertices in the mode
  the model picks, reInit with initFunc, gather of every partition that
  received messages or kept carried vertices, then filterFunc (Algorithm 2);
* the analytical mode model (performance modelling, Sec. 3.2, Eq. 1).

Readings taken where the paper is silent:
  - inactive vertices of a partition-centric partition send the combine's
    identity, and gather ignores identity messages (no combine, no
    activation), so the mode never changes results;
  - filterFunc runs on carried and on newly activated vertices, also in a
    partition that received no message;
  - PageRank adds the dangling mass D/|V| inside filterFunc; personalised
    PageRank returns it to the seed;
  - r in the partition-centric cost is r^p; the model is evaluated exactly in
    integers after multiplying through by E^p, a tie picks partition-centric.
"""
from __future__ import annotations

import math

import numpy as np
from dataclasses import dataclass, field
from fractions import Fraction
from typing import Dict, List, Tuple

INF32 = 0xFFFFFFFF
SC, PC = "SC", "PC"


# ---------------------------------------------------------------------------
# Partitions and the partition-node bipartite graph
# ---------------------------------------------------------------------------
def num_partitions(n: int, q: int) -> int:
    return max(1, -(-n // q))


def neighbour_groups(g, q: int, v: int) -> List[Tuple[int, List[int], List[int]]]:
    """Messages of vertex v: for each neighbouring partition pq (ascending),
    the local ids of v's out-neighbours in pq, in CSR order, and the CSR edge
    indices they come from."""
    groups: Dict[int, Tuple[List[int], List[int]]] = {}
    for e in range(int(g.offsets[v]), int(g.offsets[v + 1])):
        u = int(g.cols[e])
        ids, edges = groups.setdefault(u // q, ([], []))
        ids.append(u - (u // q) * q)
        edges.append(e)
    return [(pq, groups[pq][0], groups[pq][1]) for pq in sorted(groups)]


@dataclass
class PNG:
    """N_i^p(pq) with each source's destination ids: png[(p, pq)] is the
    list of (v, local ids, edge indices) for ascending v in p."""
    q: int
    k: int
    bins: Dict[Tuple[int, int], List[Tuple[int, List[int], List[int]]]]
    E: List[int]   # E^p: out-edges of partition p
    M: List[int]   # messages of partition p when every vertex is active (= r^p E^p)


def build_png(g, q: int) -> PNG:
    k = num_partitions(g.n, q)
    bins: Dict[Tuple[int, int], list] = {}
    E = [0] * k
    M = [0] * k
    for v in range(g.n):
        p = v // q
        E[p] += int(g.offsets[v + 1]) - int(g.offsets[v])
        for pq, ids, edges in neighbour_groups(g, q, v):
            bins.setdefault((p, pq), []).append((v, ids, edges))
            M[p] += 1
    return PNG(q, k, bins, E, M)


# ---------------------------------------------------------------------------
# Analytical mode model (Eq. 1)
# ---------------------------------------------------------------------------
def pc_cost_bytes(E_p: int, M_p: int, k: int, s_i: int = 4, s_v: int = 4) -> Fraction:
    """E^p((r^p + 1) s_i + 2 r^p s_v) + k s_i with r^p = M^p / E^p."""
    if E_p == 0:
        return Fraction(k * s_i)
    r = Fraction(M_p, E_p)
    return E_p * ((r + 1) * s_i + 2 * r * s_v) + k * s_i


def sc_cost_bytes(E_p: int, M_p: int, Va: int, Ea: int, s_i: int = 4, s_v: int = 4) -> Fraction:
    """2 r^p E_a^p s_v + 3 E_a^p s_i + V_a^p s_i."""
    r = Fraction(M_p, E_p) if E_p else Fraction(0)
    return 2 * r * Ea * s_v + 3 * Ea * s_i + Va * s_i


def choose_mode(E_p: int, M_p: int, Va: int, Ea: int, k: int, bw_ratio=Fraction(2),
                s_i: int = 4, s_v: int = 4) -> str:
    """PC iff cost_PC / BW_PC <= cost_SC / BW_SC, i.e. cost_PC <= ratio * cost_SC
    with ratio = BW_PC / BW_SC (2 by default). Both sides are scaled by E^p
    so the comparison is exact; with E^p = 0 both sides are 0 and PC wins."""
    ratio = Fraction(bw_ratio)
    lhs = pc_cost_bytes(E_p, M_p, k, s_i, s_v) * E_p
    rhs = ratio * sc_cost_bytes(E_p, M_p, Va, Ea, s_i, s_v) * E_p
    return PC if lhs <= rhs else SC


# ---------------------------------------------------------------------------
# Programs: scatterFunc / initFunc / gatherFunc / filterFunc / applyWeight
# ---------------------------------------------------------------------------
@dataclass
class Ctx:
    n: int
    deg: List[int]
    it: int = 0
    dangling: float = 0.0
    params: dict = field(default_factory=dict)


class Program:
    combine = "min"
    identity = INF32
    weighted = False

    def start(self, n, params):  # -> (state, frontier)
        raise NotImplementedError

    def scatter(self, st, v, ctx):
        return st[v]

    def init(self, st, v, ctx):
        return False

    def apply_weight(self, val, w):
        return val

    def gather(self, st, u, val):
        if val < st[u]:
            st[u] = val
            return True
        return False

    def filter(self, st, v, ctx):
        return True

    def before_gather(self, st, active, ctx):
        """Values a program needs from the pre-reInit state (dangling mass)."""
        return None


class BFSLevel(Program):
    def start(self, n, params):
        st = [INF32] * n
        st[params["root"]] = 0
        return st, [params["root"]]

    def scatter(self, st, v, ctx):
        return st[v] + 1


class BFSParent(Program):
    """Algorithm 5 as printed: scatterFunc sends the vertex's own id,
    gatherFunc sets the parent of a vertex that has none, initFunc keeps no
    vertex, filterFunc keeps every vertex gatherFunc set. The first message a
    vertex receives wins; this model gathers bins in source-partition order
    and a bin's messages in source order, so that is the least source id."""

    def start(self, n, params):
        st = [INF32] * n
        st[params["root"]] = params["root"]
        return st, [params["root"]]

    def scatter(self, st, v, ctx):
        return v

    def gather(self, st, u, val):
        if st[u] == INF32:
            st[u] = val
            return True
        return False


class Nibble(Program):
    """Parallel Nibble as the paper writes it, in FP64: scatterFunc sends
    PR/(2 deg), initFunc halves PR and keeps the vertex iff PR >= eps * deg,
    gatherFunc adds, filterFunc keeps iff PR >= eps * deg. A vertex without
    out-edges is never kept (its threshold eps * 0 would keep it forever
    while it has nothing to send)."""
    combine = "sum"
    identity = 0.0

    def start(self, n, params):
        self.eps = float(params["eps"])
        st = [0.0] * n
        st[params["root"]] = 1.0
        return st, [params["root"]]

    def keep(self, x, d):
        return d > 0 and x >= self.eps * d

    def scatter(self, st, v, ctx):
        d = ctx.deg[v]
        return st[v] / (2.0 * d) if d else 0.0

    def init(self, st, v, ctx):
        st[v] = st[v] * 0.5
        return self.keep(st[v], ctx.deg[v])

    def gather(self, st, u, val):
        st[u] += val
        return True

    def filter(self, st, v, ctx):
        return self.keep(st[v], ctx.deg[v])


class CCMinLabel(Program):
    def start(self, n, params):
        return list(range(n)), list(range(n))


class SSSP(Program):
    weighted = True

    def start(self, n, params):
        st = [INF32] * n
        st[params["root"]] = 0
        return st, [params["root"]]

    def apply_weight(self, val, w):
        return min(val + w, INF32)


class CarryBFS(BFSLevel):
    """Selective continuity: a reached vertex stays in the frontier for
    `persist` iterations (initFunc returns true while it is young)."""

    def init(self, st, v, ctx):
        return ctx.it - st[v] + 1 < ctx.params["persist"]


class PageRank(Program):
    combine = "sum"
    identity = None

    def start(self, n, params):
        return [1.0 / n] * n, list(range(n))

    def before_gather(self, st, active, ctx):
        ctx.dangling = sum(st[v] for v in range(ctx.n) if ctx.deg[v] == 0)

    def scatter(self, st, v, ctx):
        return st[v] / ctx.deg[v]

    def init(self, st, v, ctx):
        st[v] = 0.0
        return True

    def gather(self, st, u, val):
        st[u] += val
        return True

    def filter(self, st, v, ctx):
        d = ctx.params.get("damping", 0.85)
        st[v] = (1.0 - d) / ctx.n + d * (st[v] + ctx.dangling / ctx.n)
        return True


class PPR(PageRank):
    def start(self, n, params):
        st = [0.0] * n
        st[params["seed"]] = 1.0
        return st, [params["seed"]]

    def before_gather(self, st, active, ctx):
        ctx.dangling = sum(st[v] for v in active if ctx.deg[v] == 0)

    def filter(self, st, v, ctx):
        a = ctx.params.get("alpha", 0.15)
        s = ctx.params["seed"]
        st[v] = (1.0 - a) * st[v]
        if v == s:
            st[v] += a + (1.0 - a) * ctx.dangling
        return st[v] > 0.0


PROGRAMS = {"bfs": BFSLevel, "cc": CCMinLabel, "sssp": SSSP, "pagerank": PageRank,
            "ppr": PPR, "carry_bfs": CarryBFS, "bfs_parent": BFSParent, "nibble": Nibble}


# ---------------------------------------------------------------------------
# The iteration (Algorithm 2, with Algorithm 3 for partition-centric scatter)
# ---------------------------------------------------------------------------
@dataclass
class IterTrace:
    modes: Dict[int, str]
    Va: Dict[int, int]
    Ea: Dict[int, int]
    bins: Dict[Tuple[int, int], List[Tuple[object, List[int], List[int]]]]
    frontier_out: List[int]


def run(g, q: int, prog_name: str, params: dict, max_iter: int, selector="analytical",
        bw_ratio=Fraction(2), keep_bins: bool = False):
    """Runs up to max_iter iterations or until the frontier empties.
    selector: "analytical", "sc" or "pc" (forced). Returns (state, traces)."""
    prog = PROGRAMS[prog_name]()
    png = build_png(g, q)
    deg = [int(g.offsets[v + 1]) - int(g.offsets[v]) for v in range(g.n)]
    st, frontier = prog.start(g.n, params)
    active = sorted(set(frontier))
    ctx = Ctx(g.n, deg, 0, 0.0, params)
    traces: List[IterTrace] = []
    w = g.weights
    for it in range(max_iter):
        if not active:
            break
        ctx.it = it
        by_part: Dict[int, List[int]] = {}
        for v in active:
            by_part.setdefault(v // q, []).append(v)
        act_set = set(active)
        prog.before_gather(st, active, ctx)
        # ---- Scatter (each p in sPartList writes only its bin row)
        bins: Dict[Tuple[int, int], list] = {}
        modes, Va, Ea = {}, {}, {}
        for p in sorted(by_part):
            verts = by_part[p]
            Va[p] = len(verts)
            Ea[p] = sum(deg[v] for v in verts)
            if selector == "sc":
                mode = SC
            elif selector == "pc":
                mode = PC
            else:
                mode = choose_mode(png.E[p], png.M[p], Va[p], Ea[p], png.k, bw_ratio)
            modes[p] = mode
            if mode == SC:
                for v in verts:
                    groups = neighbour_groups(g, q, v)
                    if not groups:
                        continue  # no out-edge, no message (and no scatterFunc call)
                    val = prog.scatter(st, v, ctx)
                    for pq, ids, edges in groups:
                        bins.setdefault((p, pq), []).append((val, ids, edges))
            else:
                for pq in range(png.k):
                    for v, ids, edges in png.bins.get((p, pq), []):
                        val = prog.scatter(st, v, ctx) if v in act_set else prog.identity
                        bins.setdefault((p, pq), []).append((val, ids, edges))
        # ---- reInit frontier (initFunc on V_a^p, after p's scatter)
        carried = set()
        for v in active:
            if prog.init(st, v, ctx):
                carried.add(v)
        # ---- Gather: every partition with incoming messages or carried vertices
        prelim = set(carried)
        cols = sorted({pq for (_, pq) in bins} | {v // q for v in carried})
        for pq in cols:
            for p in range(png.k):
                for val, ids, edges in bins.get((p, pq), []):
                    if val is prog.identity or (prog.combine == "min" and val == INF32):
                        continue
                    for u_local, e in zip(ids, edges):
                        x = prog.apply_weight(val, int(w[e])) if prog.weighted else val
                        if prog.gather(st, pq * q + u_local, x):
                            prelim.add(pq * q + u_local)
        # ---- filter frontier
        nxt = sorted(v for v in prelim if prog.filter(st, v, ctx))
        traces.append(IterTrace(modes, Va, Ea, bins if keep_bins else {}, nxt))
        active = nxt
    return st, traces
