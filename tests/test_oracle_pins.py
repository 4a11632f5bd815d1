"""Pins the oracle to things other than itself: brute force on tiny graphs,
library routines (scipy.sparse.csgraph), closed forms, hand-derived fixtures
and invariants. Runs on the CPU only."""
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import graphgen as gg
import oracle
from oracle import gpop_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
INF = 0xFFFFFFFF


def graph_from_edges(n, edges, weights=None):
    src = np.array([e[0] for e in edges], np.uint32)
    dst = np.array([e[1] for e in edges], np.uint32)
    off, cols = gg.build_csr(n, src, dst)
    g = gg.Graph(n, off, cols)
    if weights is not None:
        order = np.lexsort((dst, src))
        g.weights = np.array(weights, np.uint8)[order]
    return g


def small_graphs():
    out = []
    for seed in range(6):
        out.append(gg.rmat_graph(5, 3, 100 + seed))
        out.append(gg.er_graph(40, 90, 200 + seed))
    out.append(gg.rmat_graph(5, 4, 300, symmetric=True))
    out.append(graph_from_edges(1, []))
    out.append(graph_from_edges(7, [(0, 0), (0, 0), (1, 2), (2, 1), (5, 6)]))
    return out


def edge_list(g):
    rows = np.repeat(np.arange(g.n), np.diff(g.offsets.astype(np.int64)))
    return rows, g.cols.astype(np.int64)


# ---------------------------------------------------------------- BFS levels
def floyd_warshall_hops(g):
    n = g.n
    d = np.full((n, n), np.inf)
    np.fill_diagonal(d, 0)
    r, c = edge_list(g)
    d[r, c] = np.minimum(d[r, c], 1)
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    return d


@pytest.mark.parametrize("gi", range(15))
def test_bfs_vs_floyd_warshall(gi):
    g = small_graphs()[gi]
    d = floyd_warshall_hops(g)
    for root in range(min(g.n, 6)):
        lv = oracle.bfs_levels(g, root)
        ref = np.where(np.isinf(d[root]), INF, d[root]).astype(np.uint64)
        assert np.array_equal(lv.astype(np.uint64), ref)


def test_bfs_vs_scipy_and_invariants():
    g = gg.rmat_graph(12, 8, 77)
    r, c = edge_list(g)
    A = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(g.n, g.n))
    for root in gg.pick_sources(g.offsets, 3, 4):
        lv = oracle.bfs_levels(g, int(root))
        ref = csgraph.shortest_path(A, unweighted=True, indices=int(root))
        assert np.array_equal(lv.astype(np.float64), np.where(np.isinf(ref), INF, ref))
        # every edge: level[v] <= level[u] + 1 for reached u
        reached = lv[r] != INF
        assert np.all(lv[c[reached]].astype(np.int64) <= lv[r[reached]].astype(np.int64) + 1)


def test_bfs_closed_forms():
    n = 9
    path = graph_from_edges(n, [(i, i + 1) for i in range(n - 1)])
    assert oracle.bfs_levels(path, 0).tolist() == list(range(n))
    star = graph_from_edges(n, [(0, i) for i in range(1, n)])
    assert oracle.bfs_levels(star, 0).tolist() == [0] + [1] * (n - 1)
    assert oracle.bfs_levels(star, 3).tolist() == [INF] * 3 + [0] + [INF] * 5
    comp = graph_from_edges(5, [(i, j) for i in range(5) for j in range(5) if i != j])
    assert oracle.bfs_levels(comp, 2).tolist() == [1, 1, 0, 1, 1]


# -------------------------------------------------------------- CC min label
def dfs_min_label(g):
    r, c = edge_list(g)
    adj = [[] for _ in range(g.n)]
    for a, b in zip(r.tolist(), c.tolist()):
        adj[a].append(b)
        adj[b].append(a)
    lab = [-1] * g.n
    for s in range(g.n):
        if lab[s] >= 0:
            continue
        stack, comp = [s], []
        lab[s] = s
        while stack:
            u = stack.pop()
            comp.append(u)
            for v in adj[u]:
                if lab[v] < 0:
                    lab[v] = s
                    stack.append(v)
    return np.array(lab, np.uint32)


# ---------------------------------------------------------------- BFS parents
def brute_parents(g, root):
    """Levels by repeated relaxation over every edge, then for each reached
    vertex the least in-neighbour one level closer to the root."""
    n = g.n
    lv = [INF] * n
    lv[root] = 0
    r, c = edge_list(g)
    changed = True
    while changed:
        changed = False
        for u, v in zip(r.tolist(), c.tolist()):
            if lv[u] != INF and lv[u] + 1 < lv[v]:
                lv[v] = lv[u] + 1
                changed = True
    par = [INF] * n
    par[root] = root
    for v in range(n):
        if v != root and lv[v] != INF:
            par[v] = min(u for u, w in zip(r.tolist(), c.tolist()) if w == v and lv[u] == lv[v] - 1)
    return np.array(par, np.uint32)


@pytest.mark.parametrize("gi", range(15))
def test_bfs_parents_vs_brute_force(gi):
    g = small_graphs()[gi]
    for root in range(min(g.n, 6)):
        assert np.array_equal(oracle.bfs_parents(g, root), brute_parents(g, root))


def test_bfs_parents_hand_example():
    # 0->1 0->2 1->3 2->3 2->4 3->5 4->5 5->0; vertex 6 has no in-edge.
    g = graph_from_edges(7, [(0, 1), (0, 2), (1, 3), (2, 3), (2, 4), (3, 5), (4, 5), (5, 0)])
    # from 0: 1, 2 at level 1 (parent 0); 3 at level 2 is offered 1 and 2 -> 1;
    # 4 is offered 2; 5 at level 3 is offered 3 and 4 -> 3
    assert oracle.bfs_parents(g, 0).tolist() == [0, 0, 0, 1, 2, 3, INF]
    # from 2: 3, 4 at level 1; 5 at level 2 (3 and 4 -> 3); 0 at level 3 (5);
    # 1 at level 4 (0)
    assert oracle.bfs_parents(g, 2).tolist() == [5, 0, 2, 2, 2, 3, INF]


def test_bfs_parents_tree_validation():
    """Graph500-style checks of the trees at a size brute force cannot reach:
    the root is its own parent, exactly the reachable vertices have parents,
    every tree edge is a graph edge going one level down, and the parent is
    the least such in-neighbour."""
    g = gg.rmat_graph(12, 8, 78)
    r, c = edge_list(g)
    edges = set(zip(r.tolist(), c.tolist()))
    for root in gg.pick_sources(g.offsets, 5, 4):
        root = int(root)
        par = oracle.bfs_parents(g, root)
        lv = oracle.bfs_levels(g, root)
        assert par[root] == root
        reached = lv != INF
        assert np.array_equal(par != INF, reached)
        v = np.nonzero(reached & (np.arange(g.n) != root))[0]
        assert all((int(par[x]), int(x)) in edges for x in v)
        assert np.all(lv[par[v]].astype(np.int64) == lv[v].astype(np.int64) - 1)
        ok = (lv[r] != INF) & (lv[c].astype(np.int64) == lv[r].astype(np.int64) + 1)
        least = np.full(g.n, INF, np.uint64)
        np.minimum.at(least, c[ok], r[ok].astype(np.uint64))
        assert np.array_equal(least[v], par[v].astype(np.uint64))


# ---------------------------------------------------------------- Parallel Nibble
# oracle.nibble is Parallel Nibble (the Nibble application) in FP64. While
# every reached vertex stays active it is exactly the lazy random walk
# x <- (x + A^T D^-1 x) / 2 started at the seed; the thresholds then decide
# which vertices keep walking.

def test_nibble_cycle_is_binomial():
    """On a directed cycle every vertex has one out-edge, so with a tiny eps
    the mass after t < n iterations is the binomial C(t, j) / 2^t at j steps
    ahead of the seed (a lazy walk), and the frontier is the t + 1 vertices
    holding mass."""
    from math import comb
    n, seed = 50, 7
    g = graph_from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    for t in (1, 2, 5, 13):
        r = oracle.nibble(g, seed, 1e-300, t)
        want = np.zeros(n)
        for j in range(t + 1):
            want[(seed + j) % n] = comb(t, j) / 2.0 ** t
        assert r.iters == t
        assert np.array_equal(r.pr, want)
        assert list(r.fsize) == [i + 2 for i in range(t)]


@pytest.mark.parametrize("seed", [0, 3, 11])
def test_nibble_tiny_eps_is_lazy_walk_matrix_power(seed):
    """With every reached vertex kept, t iterations equal the t-th power of
    the lazy walk matrix (I + A^T D^-1) / 2 applied to e_seed (dense numpy;
    duplicate edges count twice), on a symmetric graph whose vertices all
    have out-edges."""
    base = gg.rmat_graph(5, 4, 300, symmetric=True)
    r0, c0 = edge_list(base)
    n = base.n
    ring = [(i, (i + 1) % n) for i in range(n)] + [((i + 1) % n, i) for i in range(n)]
    g = graph_from_edges(n, list(zip(r0.tolist(), c0.tolist())) + ring)
    deg = g.degrees().astype(np.float64)
    assert np.all(deg > 0)
    r, c = edge_list(g)
    P = np.zeros((n, n))
    np.add.at(P, (c, r), 1.0 / deg[r])
    W = 0.5 * (np.eye(n) + P)
    e = np.zeros(n)
    e[seed] = 1.0
    for t in (1, 3, 8):
        want = np.linalg.matrix_power(W, t) @ e
        got = oracle.nibble(g, seed, 1e-300, t)
        assert got.iters == t
        assert np.max(np.abs(got.pr - want)) <= 1e-14


@pytest.mark.parametrize("gi", [0, 1, 4, 7, 12, 14])
def test_nibble_mass_conservation(gi):
    """Mass only moves along edges: the total stays 1, except that an active
    seed without out-edges keeps the half initFunc leaves it and sends
    nothing."""
    g = small_graphs()[gi]
    deg = g.degrees()
    for seed in range(min(4, g.n)):
        for eps in (1.3e-2, 2.7e-3, 1e-300):
            r = oracle.nibble(g, seed, eps, 40)
            total = 1.0 if deg[seed] > 0 else 0.5
            assert abs(r.pr.sum() - total) <= 1e-12
            assert np.all(r.pr >= 0)


def test_nibble_threshold_closed_forms():
    # a star of 8 leaves around 0, both directions: after the first
    # iteration the centre holds 1/2 and every leaf 1/16, a fixed point
    # (every vertex passes its threshold, so all 9 stay active)
    g = graph_from_edges(9, [(0, i) for i in range(1, 9)] + [(i, 0) for i in range(1, 9)])
    for t in (1, 2, 5):
        r = oracle.nibble(g, 0, 1e-3, t)
        assert r.iters == t and list(r.fsize) == [9] * t
        assert np.array_equal(r.pr, np.array([0.5] + [1 / 16] * 8))
    # a leaf's threshold is eps * 1: with eps = 1/10 the leaves (1/16) drop
    # after the first iteration, the centre (1/2 >= 8/10 fails) too
    r = oracle.nibble(g, 0, 0.1, 10)
    assert r.iters == 1 and list(r.fsize) == [0]
    # one edge both ways: the seed keeps 1/2 and sends 1/2, then both stay
    # at 1/2; with eps above 1/2 the seed stops after its first scatter
    g = graph_from_edges(2, [(0, 1), (1, 0)])
    r = oracle.nibble(g, 0, 0.1, 3)
    assert np.array_equal(r.pr, [0.5, 0.5]) and list(r.fsize) == [2, 2, 2]
    r = oracle.nibble(g, 0, 0.75, 10)
    assert np.array_equal(r.pr, [0.5, 0.5]) and r.iters == 1 and list(r.fsize) == [0]
    # a seed without out-edges halves once and stops
    g = graph_from_edges(3, [(1, 2)])
    r = oracle.nibble(g, 0, 1e-3, 10)
    assert r.iters == 1 and list(r.fsize) == [0] and np.array_equal(r.pr, [0.5, 0, 0])


def test_nibble_margin_reports_ties():
    """The reported margin is the least relative distance of a decisive
    threshold test: on a 4-cycle with eps = 1/4 the second iteration holds
    [1/4, 1/2, 1/4] from the seed, two exact ties."""
    g = graph_from_edges(4, [(i, (i + 1) % 4) for i in range(4)])
    r = oracle.nibble(g, 0, 0.25, 2, delta=1e-6)
    assert r.min_margin == 0.0 and r.near >= 2
    # after one iteration the two vertices hold 1/2, twice the threshold
    r = oracle.nibble(g, 0, 0.25, 1, delta=1e-6)
    assert r.min_margin == 1.0 and r.near == 0


@pytest.mark.parametrize("gi", [0, 1, 4, 7, 12])
def test_nibble_gpop_model_equals_oracle(gi):
    """The partitioned GPOP model (bins, both scatter modes, reInit, gather,
    filter) in FP64 follows the direct edge iteration: the same frontiers and
    values to rounding, wherever no decision lies within 1e-9 of its
    threshold."""
    g = small_graphs()[gi]
    checked = 0
    for seed in range(min(3, g.n)):
        for eps in (1.37e-2, 3.1e-3, 1.1e-3):
            ref = oracle.nibble(g, seed, eps, 60, delta=1e-9)
            if ref.near:
                continue
            for sel in ("analytical", "sc", "pc"):
                st, tr = gpop_ref.run(g, 8, "nibble", {"root": seed, "eps": eps}, 60, selector=sel)
                assert [len(t.frontier_out) for t in tr] == list(ref.fsize)
                assert np.max(np.abs(np.array(st, np.float64) - ref.pr)) <= 1e-14
            checked += 1
    assert checked > 0


@pytest.mark.parametrize("gi", range(15))
def test_cc_vs_dfs(gi):
    g = small_graphs()[gi]
    assert np.array_equal(oracle.cc_minlabel(g), dfs_min_label(g))


def test_cc_vs_scipy_and_invariants():
    g = gg.rmat_graph(12, 4, 78, symmetric=True)
    r, c = edge_list(g)
    lab = oracle.cc_minlabel(g)
    A = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(g.n, g.n))
    ncomp, comp = csgraph.connected_components(A, directed=False)
    mins = np.full(ncomp, g.n)
    np.minimum.at(mins, comp, np.arange(g.n))
    assert np.array_equal(lab, mins[comp].astype(np.uint32))
    assert np.all(lab[r] == lab[c])
    assert np.all(lab <= np.arange(g.n))
    assert np.array_equal(lab[lab], lab)


# --------------------------------------------------------------------- SSSP
def bellman_ford(g, root):
    d = [INF] * g.n
    d[root] = 0
    r, c = edge_list(g)
    for _ in range(g.n):
        changed = False
        for e, (u, v) in enumerate(zip(r.tolist(), c.tolist())):
            if d[u] != INF and d[u] + int(g.weights[e]) < d[v]:
                d[v] = d[u] + int(g.weights[e])
                changed = True
        if not changed:
            break
    return np.array(d, np.uint32)


@pytest.mark.parametrize("gi", range(15))
def test_sssp_vs_bellman_ford(gi):
    g = small_graphs()[gi]
    g.weights = gg.edge_weights(g.m, 400 + gi)
    for root in range(min(g.n, 4)):
        assert np.array_equal(oracle.sssp(g, root), bellman_ford(g, root))


def test_sssp_vs_scipy_dijkstra():
    g = gg.rmat_graph(11, 8, 79, weights_seed=80)
    r, c = edge_list(g)
    # duplicates: keep the lightest parallel edge for the library routine
    best = {}
    for e, (u, v) in enumerate(zip(r.tolist(), c.tolist())):
        w = int(g.weights[e])
        if best.get((u, v), 256) > w:
            best[(u, v)] = w
    keys = np.array(list(best.keys()))
    A = sp.csr_matrix((np.array(list(best.values()), np.float64), (keys[:, 0], keys[:, 1])),
                      shape=(g.n, g.n))
    for root in gg.pick_sources(g.offsets, 4, 3):
        ref = csgraph.dijkstra(A, indices=int(root))
        d = oracle.sssp(g, int(root))
        assert np.array_equal(d.astype(np.float64), np.where(np.isinf(ref), INF, ref))
        reached = d[r] != INF
        assert np.all(d[c[reached]].astype(np.int64)
                      <= d[r[reached]].astype(np.int64) + g.weights[reached])


def test_sssp_unit_weights_equal_bfs():
    g = gg.rmat_graph(11, 8, 81)
    ones = np.ones(g.m, np.uint8)
    for root in gg.pick_sources(g.offsets, 5, 3):
        assert np.array_equal(oracle.sssp(g, int(root), ones), oracle.bfs_levels(g, int(root)))


# ----------------------------------------------------------------- PageRank
def dense_pagerank(g, d=0.85, iters=10):
    n = g.n
    r, c = edge_list(g)
    A = np.zeros((n, n))
    np.add.at(A, (r, c), 1.0)
    deg = A.sum(axis=1)
    P = np.zeros((n, n))
    for u in range(n):
        if deg[u] > 0:
            P[:, u] = A[u] / deg[u]
        else:
            P[:, u] = 1.0 / n
    G = d * P + (1 - d) / n
    x = np.full(n, 1.0 / n)
    for _ in range(iters):
        x = G @ x
    return x


@pytest.mark.parametrize("gi", range(15))
def test_pagerank_vs_dense_google_matrix(gi):
    g = small_graphs()[gi]
    for iters in (1, 3, 10):
        x = oracle.pagerank(g, 0.85, iters)
        assert np.allclose(x, dense_pagerank(g, 0.85, iters), rtol=0, atol=1e-14)
        assert abs(x.sum() - 1.0) < 1e-12


def test_pagerank_golden_stars():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "pagerank_star.txt"))
            if l.strip() and not l.startswith("#")]
    sym = graph_from_edges(5, [(0, i) for i in range(1, 5)] + [(i, 0) for i in range(1, 5)])
    dr = graph_from_edges(5, [(0, i) for i in range(1, 5)])
    for kind, it, *vals in rows:
        g = sym if kind == "sym" else dr
        x = oracle.pagerank(g, 0.85, int(it))
        assert np.allclose(x, np.array(vals, float), rtol=0, atol=1e-15)


def test_pagerank_closed_forms():
    n = 7
    cycle = graph_from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    comp = graph_from_edges(n, [(i, j) for i in range(n) for j in range(n) if i != j])
    empty = graph_from_edges(n, [])
    for g in (cycle, comp, empty):
        assert np.allclose(oracle.pagerank(g, 0.85, 10), 1.0 / n, rtol=0, atol=1e-15)


def dense_ppr(g, seed, alpha=0.15, iters=20):
    n = g.n
    r, c = edge_list(g)
    A = np.zeros((n, n))
    np.add.at(A, (r, c), 1.0)
    deg = A.sum(axis=1)
    P = np.zeros((n, n))
    for u in range(n):
        if deg[u] > 0:
            P[:, u] = A[u] / deg[u]
        else:
            P[seed, u] = 1.0
    x = np.zeros(n)
    x[seed] = 1.0
    e = np.zeros(n)
    e[seed] = 1.0
    for _ in range(iters):
        x = alpha * e + (1 - alpha) * (P @ x)
    return x


@pytest.mark.parametrize("gi", range(15))
def test_ppr_vs_dense(gi):
    g = small_graphs()[gi]
    for seed in range(min(3, g.n)):
        x = oracle.ppr(g, seed, 0.15, 20)
        assert np.allclose(x, dense_ppr(g, seed), rtol=0, atol=1e-14)
        assert abs(x.sum() - 1.0) < 1e-12


# ------------------------------------------------- GPOP iteration model
def test_mode_model_golden():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "mode_model.txt"))
            if l.strip() and not l.startswith("#")]
    for Ep, Mp, k, Va, Ea, cpc, csc, mode in rows:
        Ep, Mp, k, Va, Ea = map(int, (Ep, Mp, k, Va, Ea))
        assert gpop_ref.pc_cost_bytes(Ep, Mp, k) == int(cpc)
        assert gpop_ref.sc_cost_bytes(Ep, Mp, Va, Ea) == int(csc)
        assert gpop_ref.choose_mode(Ep, Mp, Va, Ea, k) == mode


def test_all_active_picks_pc():
    # PageRank (every vertex active) always runs partition-centric
    for g in small_graphs():
        png = gpop_ref.build_png(g, 8)
        for p in range(png.k):
            lo, hi = p * 8, min(g.n, p * 8 + 8)
            Ea = int(g.offsets[hi]) - int(g.offsets[lo])
            if png.E[p] == 0:
                continue
            assert gpop_ref.choose_mode(png.E[p], png.M[p], hi - lo, Ea, png.k) == "PC"


def test_png_structure():
    g = gg.rmat_graph(7, 6, 90)
    q = 16
    png = gpop_ref.build_png(g, q)
    seen = []
    for (p, pq), msgs in png.bins.items():
        vs = [v for v, _, _ in msgs]
        assert vs == sorted(vs) and len(set(vs)) == len(vs)
        for v, ids, edges in msgs:
            assert v // q == p
            assert all(int(g.cols[e]) == pq * q + i for i, e in zip(ids, edges))
            seen.extend(edges)
    assert sorted(seen) == list(range(g.m))          # every edge exactly once
    assert sum(png.M) == sum(len(m) for m in png.bins.values())
    assert sum(png.E) == g.m


def test_sc_bins_equal_pc_bins_when_all_active():
    g = gg.rmat_graph(6, 5, 91)
    _, tr_sc = gpop_ref.run(g, 8, "pagerank", {}, 1, selector="sc", keep_bins=True)
    _, tr_pc = gpop_ref.run(g, 8, "pagerank", {}, 1, selector="pc", keep_bins=True)
    assert tr_sc[0].bins == tr_pc[0].bins


@pytest.mark.parametrize("selector", ["analytical", "sc", "pc"])
@pytest.mark.parametrize("gi", [0, 1, 4, 7, 12, 14])
def test_gpop_model_matches_textbook(selector, gi):
    g = small_graphs()[gi]
    g.weights = gg.edge_weights(g.m, 500 + gi)
    q = 8
    for root in range(min(3, g.n)):
        st, _ = gpop_ref.run(g, q, "bfs", {"root": root}, 10 * g.n + 5, selector)
        assert np.array_equal(np.array(st, np.uint32), oracle.bfs_levels(g, root))
        st, _ = gpop_ref.run(g, q, "sssp", {"root": root}, 10 * g.n + 5, selector)
        assert np.array_equal(np.array(st, np.uint32), oracle.sssp(g, root))
        # Algorithm 5 as printed (first message wins, in gather order) against
        # the textbook least-id parent
        st, _ = gpop_ref.run(g, q, "bfs_parent", {"root": root}, 10 * g.n + 5, selector)
        assert np.array_equal(np.array(st, np.uint32), oracle.bfs_parents(g, root))
        st, _ = gpop_ref.run(g, q, "ppr", {"seed": root}, 20, selector)
        assert np.allclose(st, oracle.ppr(g, root), rtol=0, atol=1e-13)
    sym = gg.Graph(g.n, *gg.build_csr(g.n, *gg.symmetrize(*edge_list_u32(g))))
    st, _ = gpop_ref.run(sym, q, "cc", {}, 10 * g.n + 5, selector)
    assert np.array_equal(np.array(st, np.uint32), oracle.cc_minlabel(sym))
    st, _ = gpop_ref.run(g, q, "pagerank", {}, 10, selector)
    assert np.allclose(st, oracle.pagerank(g), rtol=0, atol=1e-14)


def edge_list_u32(g):
    r, c = edge_list(g)
    return r.astype(np.uint32), c.astype(np.uint32)


def test_carry_frontier_closed_form():
    g = gg.rmat_graph(7, 4, 92, symmetric=True)
    root = int(gg.pick_sources(g.offsets, 1, 1)[0])
    lv = oracle.bfs_levels(g, root)
    for persist in (1, 2, 3):
        st, tr = gpop_ref.run(g, 16, "carry_bfs", {"root": root, "persist": persist}, 50)
        assert np.array_equal(np.array(st, np.uint32), lv)
        for it, t in enumerate(tr):
            # after iteration it, active = vertices with level in (it+1-persist, it+1]
            want = [v for v in range(g.n) if lv[v] != INF and it + 1 - persist < lv[v] <= it + 1]
            assert t.frontier_out == want
