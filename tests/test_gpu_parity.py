"""GPU parity: the HIP path through the C-ABI against the oracle, element by
element, on seeded inputs. Integer programs must be bit-exact; PageRank-family
results within 1e-6 max-abs and 1e-5 relative L1 of the FP64 oracle."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import gpop_ref

from gpu_util import make_graph, pr_ok, run_program, torch_cuda

pytestmark = pytest.mark.gpu

INF = 0xFFFFFFFF
SELECTORS = ["analytical", "sc", "pc"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def edges_graph(n, edges, wseed=None):
    src = np.array([e[0] for e in edges], np.uint32)
    dst = np.array([e[1] for e in edges], np.uint32)
    return gg.from_edges(n, src, dst, wseed)


def zoo():
    """(name, graph, log2_part): skewed, uniform, deep, degenerate."""
    out = [
        ("rmat10", gg.rmat_graph(10, 8, 11, weights_seed=12), 8),
        ("rmat11sym", gg.rmat_graph(11, 8, 13, symmetric=True, weights_seed=14), 8),
        ("er3000", gg.er_graph(3000, 24000, 15, weights_seed=16), 8),
        ("path700", edges_graph(700, [(i, i + 1) for i in range(699)] +
                                [(i + 1, i) for i in range(699)], 17), 8),
        ("star", edges_graph(1500, [(0, i) for i in range(1, 1500)] +
                             [(i, 0) for i in range(1, 1500)], 18), 8),
        ("messy", edges_graph(777, [(0, 0), (0, 0), (5, 5), (3, 700), (3, 700), (700, 3),
                                    (776, 0), (0, 776)] +
                              [(i, (i * 37) % 777) for i in range(0, 777, 3)], 19), 8),
        ("single", edges_graph(1, [(0, 0)], 20), 8),
        ("noedges", edges_graph(300, [], 21), 8),
        ("rmat12_q10", gg.rmat_graph(12, 16, 22, weights_seed=23), 10),
    ]
    return out


ZOO = None


def get_zoo():
    global ZOO
    if ZOO is None:
        ZOO = [(name, g, lp, make_graph(g, lp)) for name, g, lp in zoo()]
    return ZOO


def roots_of(g, n=3):
    r = gg.pick_sources(g.offsets, 99, n).tolist()
    return r if r else [0]


@pytest.mark.parametrize("zi", range(9))
@pytest.mark.parametrize("sel", SELECTORS)
def test_bfs_levels(zi, sel):
    name, g, lp, (G, _) = get_zoo()[zi]
    for root in roots_of(g):
        say("bfs", name, sel, "root", root)
        got, iters = run_program(G, "bfs", g.n, root=root, selector=sel)
        ref = oracle.bfs_levels(g, root)
        assert np.array_equal(got, ref), (name, sel, root, np.flatnonzero(got != ref)[:10])


@pytest.mark.parametrize("zi", range(9))
@pytest.mark.parametrize("sel", SELECTORS)
def test_bfs_parents(zi, sel):
    name, g, lp, (G, _) = get_zoo()[zi]
    for root in roots_of(g):
        say("bfs_parent", name, sel, "root", root)
        got, _ = run_program(G, "bfs_parent", g.n, root=root, selector=sel)
        ref = oracle.bfs_parents(g, root)
        assert np.array_equal(got, ref), (name, sel, root, np.flatnonzero(got != ref)[:10])


@pytest.mark.parametrize("gids,combine", [(256, "lds"), (1024, "lds"), (0, "rounds"), (256, "rounds")])
def test_bfs_parents_split_gather_and_combines(gids, combine):
    """Columns split over many gather tasks (partials and merges) and the
    atomic-free combine give the same least-id parents."""
    g = gg.rmat_graph(14, 16, 31, symmetric=True)
    G, _ = make_graph(g, 10, gather_task_ids=gids, combine=combine)
    for root in roots_of(g, 2):
        say("bfs_parent split", gids, combine, "root", root)
        got, _ = run_program(G, "bfs_parent", g.n, root=root)
        assert np.array_equal(got, oracle.bfs_parents(g, root)), (gids, combine, root)


def test_bfs_parents_tree_at_scale():
    """RMAT-20 (16.8M directed edges), default sizes: bit-exact against the
    oracle and a valid BFS tree whose depths are the BFS levels."""
    g = gg.rmat_graph(20, 16, 32)
    G, _ = make_graph(g, 14)
    for root in roots_of(g, 2):
        say("bfs_parent rmat20 root", root)
        got, iters = run_program(G, "bfs_parent", g.n, root=root)
        lv = oracle.bfs_levels(g, root)
        assert np.array_equal(got, oracle.bfs_parents(g, root)), root
        v = np.nonzero((got != INF) & (np.arange(g.n) != root))[0]
        assert np.array_equal(got != INF, lv != INF)
        assert np.all(lv[got[v]].astype(np.int64) == lv[v].astype(np.int64) - 1)
        assert iters == int(lv[lv != INF].max()) + 1


# Parallel Nibble decides its frontier by threshold tests (PR >= eps deg) on
# FP32 values, the oracle on FP64 ones. The kernel's value of a vertex after
# an iteration is a halved own value (exact) plus messages (x * 0.5) / deg
# (one rounding each) summed exactly in 2^-60 fixed point and rounded to
# FP32 once, so its relative error grows by at most 2 * 2^-24 per iteration.
# Policy: a case of at most T iterations is compared only when every
# decisive test of the FP64 run lies more than nibble_delta(T) = 4 T 2^-24
# (relative, twice that bound) from its threshold; then the iteration count
# and the frontier size after every iteration must be identical and the
# values within 1e-6 max-abs and 1e-5 relative L1 of the FP64 oracle. Cases
# closer to a tie are counted as skipped; each test needs checked cases.
def nibble_delta(max_iter):
    return 4.0 * max_iter * 2.0 ** -24


def nibble_check(G, g, seed, eps, max_iter, **kw):
    """True if checked against the FP64 oracle, False if skipped (near tie)."""
    delta = nibble_delta(max_iter)
    ref = oracle.nibble(g, seed, eps, max_iter, delta=delta)
    if ref.near:
        say("nibble skipped (%d decisions within %.2g of their threshold)" % (ref.near, delta), seed, eps)
        return False
    got, iters = run_program(G, "nibble", g.n, root=seed, epsilon=eps, max_iter=max_iter, **kw)
    stats = G.iter_stats()
    fs = [r["active_vertices"] for r in stats[1:iters]] + [G.frontier_size()]
    assert iters == ref.iters, (seed, eps, iters, ref.iters)
    assert fs == list(ref.fsize), (seed, eps)
    assert pr_ok(got, ref.pr), (seed, eps, float(np.max(np.abs(got.astype(np.float64) - ref.pr))))
    return True


@pytest.mark.parametrize("zi", [0, 2, 3, 4, 5, 7, 8])
@pytest.mark.parametrize("sel", SELECTORS)
def test_nibble(zi, sel):
    """Parallel Nibble against the FP64 oracle under the threshold policy."""
    name, g, lp, (G, _) = get_zoo()[zi]
    checked = 0
    for seed in roots_of(g, 2):
        for eps in (1.1e-3, 3.7e-4, 2.3e-5):
            say("nibble", name, sel, seed, eps)
            checked += nibble_check(G, g, seed, eps, 80, selector=sel)
    assert checked >= 2, (name, checked)


@pytest.mark.parametrize("gids,combine", [(256, "lds"), (0, "rounds")])
def test_nibble_split_gather_and_combines(gids, combine):
    g = gg.rmat_graph(12, 8, 33, symmetric=True)
    G, _ = make_graph(g, 9, gather_task_ids=gids, combine=combine)
    checked = 0
    for seed in roots_of(g, 2):
        for eps in (1.3e-4, 3.1e-5):
            say("nibble split", gids, combine, seed, eps)
            checked += nibble_check(G, g, seed, eps, 40)
    assert checked >= 2


def test_nibble_at_scale():
    """RMAT-18 symmetrised (8.4M CSR entries) at the default partition size
    for sum programs (2^13) and the default task sizes: the policy above on
    seeds drawn like the benchmark's."""
    g = gg.rmat_graph(18, 16, gg.BASE_SEED + 44, symmetric=True)
    G, _ = make_graph(g, 13)
    checked = 0
    for seed in [int(s) for s in gg.pick_sources(g.offsets, gg.SOURCE_SEED, 4)]:
        for eps in (1.1e-6, 3.3e-7):
            for max_iter in (12, 30):
                say("nibble rmat18", seed, eps, max_iter)
                checked += nibble_check(G, g, seed, eps, max_iter)
    assert checked >= 6


@pytest.mark.parametrize("zi", range(9))
@pytest.mark.parametrize("sel", SELECTORS)
def test_sssp(zi, sel):
    name, g, lp, (G, _) = get_zoo()[zi]
    for root in roots_of(g, 2):
        say("sssp", name, sel, "root", root)
        got, _ = run_program(G, "sssp", g.n, root=root, selector=sel)
        ref = oracle.sssp(g, root)
        assert np.array_equal(got, ref), (name, sel, root, np.flatnonzero(got != ref)[:10])


@pytest.mark.parametrize("zi", range(9))
@pytest.mark.parametrize("sel", SELECTORS)
def test_cc(zi, sel):
    name, g, lp, _ = get_zoo()[zi]
    sym = gg.from_edges(g.n, *gg.symmetrize(*edge_arrays(g)))
    G, keep = make_graph(sym, lp)
    say("cc", name, sel)
    got, _ = run_program(G, "cc", sym.n, selector=sel)
    ref = oracle.cc_minlabel(sym)
    assert np.array_equal(got, ref), (name, sel, np.flatnonzero(got != ref)[:10])


def edge_arrays(g):
    rows = np.repeat(np.arange(g.n, dtype=np.uint32), np.diff(g.offsets.astype(np.int64)))
    return rows, g.cols.copy()


# Interleaved scatter-gather (Sec. 3.3) in colour classes: BFS levels, SSSP
# distances and CC labels are the unique minimum fixed points, so the results
# must equal the oracle's bit for bit whatever the class count.
@pytest.mark.parametrize("zi", range(9))
@pytest.mark.parametrize("classes", [2, 3, 16])
def test_isg_min_programs(zi, classes):
    name, g, lp, (G, _) = get_zoo()[zi]
    sym = gg.from_edges(g.n, *gg.symmetrize(*edge_arrays(g)))
    GS, keep = make_graph(sym, lp)
    try:
        G.set_isg(classes)
        GS.set_isg(classes)
        for sel in SELECTORS:
            for root in roots_of(g, 2):
                say("isg", classes, name, sel, root)
                got, _ = run_program(G, "bfs", g.n, root=root, selector=sel)
                assert np.array_equal(got, oracle.bfs_levels(g, root)), ("bfs", name, sel, root)
                got, _ = run_program(G, "sssp", g.n, root=root, selector=sel)
                assert np.array_equal(got, oracle.sssp(g, root)), ("sssp", name, sel, root)
            got, _ = run_program(GS, "cc", sym.n, selector=sel)
            assert np.array_equal(got, oracle.cc_minlabel(sym)), ("cc", name, sel)
    finally:
        G.set_isg(0)


@pytest.mark.parametrize("gids,combine", [(256, "lds"), (2048, "lds"), (0, "rounds"), (256, "rounds")])
def test_isg_split_gather_and_combines(gids, combine):
    """Columns split over several gather tasks (held-back columns pass
    through the merge) and the atomic-free combine."""
    g = gg.rmat_graph(14, 16, 35, symmetric=True, weights_seed=36)
    G, _ = make_graph(g, 10, gather_task_ids=gids, combine=combine)
    G.set_isg(4)
    for root in roots_of(g, 2):
        say("isg split", gids, combine, root)
        got, _ = run_program(G, "sssp", g.n, root=root)
        assert np.array_equal(got, oracle.sssp(g, root)), (gids, combine, root)
        got, _ = run_program(G, "bfs", g.n, root=root)
        assert np.array_equal(got, oracle.bfs_levels(g, root)), (gids, combine, root)
    got, _ = run_program(G, "cc", g.n)
    assert np.array_equal(got, oracle.cc_minlabel(g)), (gids, combine)


def test_isg_at_scale_and_fewer_sweeps():
    """RMAT-20 symmetrised, default sizes: CC and SSSP bit-exact with two
    classes; CC needs fewer sweeps (pairs of half-steps) than iterations
    without interleaving."""
    g = gg.rmat_graph(20, 16, 37, symmetric=True, weights_seed=38)
    G, _ = make_graph(g, 14)
    _, it_plain = run_program(G, "cc", g.n)
    G.set_isg(2)
    got, it_isg = run_program(G, "cc", g.n)
    assert np.array_equal(got, oracle.cc_minlabel(g))
    say("cc iterations plain %d, isg half-steps %d" % (it_plain, it_isg))
    assert it_isg <= 2 * it_plain
    root = roots_of(g, 1)[0]
    got, _ = run_program(G, "sssp", g.n, root=root)
    assert np.array_equal(got, oracle.sssp(g, root))


def test_isg_rejects_other_programs():
    import torch
    import paper_1806_08092_amd as gp
    name, g, lp, (G, _) = get_zoo()[0]
    st = torch.empty(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(gp.GpopError) as e:
        G.set_isg(17)
    assert e.value.code == gp.EINVAL
    G.set_isg(2)
    try:
        for prog in ("pagerank", "ppr", "nibble", "bfs_parent", "carry_bfs"):
            with pytest.raises(gp.GpopError) as e:
                G.state_init(prog, st, root=0)
            assert e.value.code == gp.ENOTSUP, prog
        G.set_isg(0)
        G.state_init("pagerank", st)
        with pytest.raises(gp.GpopError) as e:
            G.set_isg(2)
        assert e.value.code == gp.ENOTSUP
    finally:
        G.set_isg(0)


@pytest.mark.parametrize("zi", [0, 1, 2, 4, 5, 7, 8])
@pytest.mark.parametrize("sel", SELECTORS)
def test_pagerank(zi, sel):
    name, g, lp, (G, _) = get_zoo()[zi]
    say("pagerank", name, sel)
    got, iters = run_program(G, "pagerank", g.n, selector=sel, max_iter=10)
    assert iters == 10
    ref = oracle.pagerank(g, 0.85, 10)
    assert pr_ok(got, ref), (name, sel, np.max(np.abs(got - ref)))
    assert abs(float(got.astype(np.float64).sum()) - 1.0) < 1e-5


@pytest.mark.parametrize("zi", [0, 1, 2, 5, 8])
@pytest.mark.parametrize("sel", SELECTORS)
def test_ppr(zi, sel):
    name, g, lp, (G, _) = get_zoo()[zi]
    for seed in roots_of(g, 2):
        say("ppr", name, sel, seed)
        got, _ = run_program(G, "ppr", g.n, root=seed, selector=sel, max_iter=20)
        ref = oracle.ppr(g, seed, 0.15, 20)
        assert pr_ok(got, ref), (name, sel, seed, np.max(np.abs(got - ref)))


@pytest.mark.parametrize("persist", [1, 2, 3])
@pytest.mark.parametrize("sel", SELECTORS)
def test_carry_frontier_sizes(persist, sel):
    # selective continuity: vertices stay active for `persist` iterations
    name, g, lp, (G, _) = get_zoo()[1]
    root = roots_of(g, 1)[0]
    got, iters = run_program(G, "carry_bfs", g.n, root=root, persist=persist, selector=sel)
    lv = oracle.bfs_levels(g, root)
    assert np.array_equal(got, lv)
    stats = G.iter_stats()
    finite = lv[lv != INF].astype(np.int64)
    for it, rec in enumerate(stats):
        want = int(np.sum((finite <= it) & (finite > it - persist)))
        assert rec["active_vertices"] == want, (it, rec, want)


def test_iteration_stats_match_model():
    """Per iteration: active vertices/edges and the SC/PC partition counts
    equal what the oracle's mode model decides for the BFS frontiers."""
    name, g, lp, (G, _) = get_zoo()[8]
    root = roots_of(g, 1)[0]
    got, iters = run_program(G, "bfs", g.n, root=root, selector="analytical")
    lv = oracle.bfs_levels(g, root)
    q = 1 << lp
    png = gpop_ref.build_png(g, q)
    deg = g.degrees()
    stats = G.iter_stats()
    assert len(stats) == iters
    for it, rec in enumerate(stats):
        act = np.flatnonzero(lv == it)
        assert rec["active_vertices"] == len(act)
        assert rec["active_edges"] == int(deg[act].sum())
        nsc = npc = 0
        for p in np.unique(act // q):
            a = act[act // q == p]
            m = gpop_ref.choose_mode(png.E[p], png.M[p], len(a), int(deg[a].sum()), png.k)
            nsc += m == "SC"
            npc += m == "PC"
        assert (rec["sc_parts"], rec["pc_parts"]) == (nsc, npc), (it, rec)


@pytest.mark.parametrize("sel", SELECTORS)
def test_active_list_lists_exactly_the_nonempty_bins(sel):
    """The two-level active list (Sec. 3.1.3): per iteration, gather reads
    exactly the bins that received ids -- every static bin of a
    partition-centric partition, and the bins a source-centric partition's
    active out-edges reach -- counted here from the BFS levels, the mode
    model and the edge list (no gather task is split at these sizes, so each
    bin is counted once)."""
    g, lp = gg.rmat_graph(14, 8, 34, symmetric=True), 8  # k = 64 partitions
    G, _ = make_graph(g, lp, gather_task_ids=1 << 20)  # one task per column
    q = 1 << lp
    png = gpop_ref.build_png(g, q)
    deg = g.degrees()
    src = np.repeat(np.arange(g.n), deg)
    static = {(int(a) // q, int(b) // q) for a, b in zip(src, g.cols)}
    for root in roots_of(g, 2):
        say("active list", sel, root)
        got, iters = run_program(G, "bfs", g.n, root=root, selector=sel)
        lv = oracle.bfs_levels(g, root)
        stats = G.iter_stats()
        assert len(stats) == iters
        for it, rec in enumerate(stats):
            act = np.flatnonzero(lv == it)
            pcs = set()
            for p in np.unique(act // q).tolist():
                a = act[act // q == p]
                m = gpop_ref.choose_mode(png.E[p], png.M[p], len(a), int(deg[a].sum()), png.k)
                if sel == "pc" or (sel == "analytical" and m == "PC"):
                    pcs.add(p)
            e_act = np.isin(src, act)
            sc_bins = {(int(a) // q, int(b) // q) for a, b in zip(src[e_act], g.cols[e_act]) if int(a) // q not in pcs}
            pc_bins = {bn for bn in static if bn[0] in pcs}
            assert rec["gathered_bins"] == len(sc_bins | pc_bins), (sel, root, it, rec)


def test_default_selector_uses_ratio_16():
    """A new graph selects by Eq. 1 with BW_PC / BW_SC = 16 until
    gpop_set_selector changes it."""
    from fractions import Fraction
    torch = torch_cuda()
    name, g, lp, _ = get_zoo()[8]
    G, _ = make_graph(g, lp)
    root = roots_of(g, 1)[0]
    st = torch.empty(g.n, dtype=torch.int32, device="cuda")
    G.state_init("bfs", st, root=root)
    G.set_frontier(torch.tensor([root], dtype=torch.int32, device="cuda"))
    G.run()
    lv = oracle.bfs_levels(g, root)
    assert np.array_equal(st.cpu().numpy().view(np.uint32), lv)
    q = 1 << lp
    png = gpop_ref.build_png(g, q)
    deg = g.degrees()
    for it, rec in enumerate(G.iter_stats()):
        act = np.flatnonzero(lv == it)
        nsc = npc = 0
        for p in np.unique(act // q):
            a = act[act // q == p]
            m = gpop_ref.choose_mode(png.E[p], png.M[p], len(a), int(deg[a].sum()), png.k, Fraction(16))
            nsc += m == "SC"
            npc += m == "PC"
        assert (rec["sc_parts"], rec["pc_parts"]) == (nsc, npc), (it, rec)


def test_pagerank_c1_workload():
    """The PageRank workload itself: directed RMAT scale 16, edge factor 16,
    10 iterations, d = 0.85, against the FP64 oracle."""
    g = gg.workload_pagerank_rmat16()
    G, _ = make_graph(g, 13)
    for sel in SELECTORS:
        got, _ = run_program(G, "pagerank", g.n, selector=sel, max_iter=10)
        ref = oracle.pagerank(g, 0.85, 10)
        err = np.abs(got.astype(np.float64) - ref)
        say("C1 pagerank", sel, "max abs", err.max(), "rel l1", err.sum() / ref.sum())
        assert pr_ok(got, ref)


def test_mode_invariance_bitwise():
    """The mode never changes the arithmetic: forced SC, forced PC and the
    analytical choice give identical bits, also for PageRank."""
    name, g, lp, (G, _) = get_zoo()[8]
    outs = {}
    for prog, kw in [("bfs", dict(root=roots_of(g, 1)[0])), ("pagerank", dict(max_iter=10)),
                     ("ppr", dict(root=roots_of(g, 1)[0], max_iter=20))]:
        res = [run_program(G, prog, g.n, selector=s, **kw)[0] for s in SELECTORS]
        for r in res[1:]:
            assert np.array_equal(r.view(np.uint32), res[0].view(np.uint32)), prog


def test_determinism_repeat():
    name, g, lp, (G, _) = get_zoo()[0]
    a, _ = run_program(G, "pagerank", g.n, max_iter=10)
    b, _ = run_program(G, "pagerank", g.n, max_iter=10)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_partition_sizes_agree():
    g = gg.rmat_graph(13, 8, 31, symmetric=True)
    root = roots_of(g, 1)[0]
    ref = oracle.bfs_levels(g, root)
    for lp in (8, 10, 12, 14):
        G, _ = make_graph(g, lp)
        got, _ = run_program(G, "bfs", g.n, root=root)
        assert np.array_equal(got, ref), lp
        got, _ = run_program(G, "cc", g.n)
        assert np.array_equal(got, oracle.cc_minlabel(g)), lp


def test_bad_frontier_vertex_reported():
    import torch
    import paper_1806_08092_amd as gp
    name, g, lp, (G, _) = get_zoo()[0]
    st = torch.empty(g.n, dtype=torch.int32, device="cuda")
    G.state_init("bfs", st, root=0)
    G.set_frontier(torch.tensor([0, g.n + 5], dtype=torch.int32, device="cuda"))
    with pytest.raises(gp.GpopError) as e:
        G.check()
    assert e.value.code == gp.EINVAL
    G.check()  # cleared


def test_program_parameters_rejected():
    """Bad program parameters fail state_init with EINVAL and change nothing."""
    import torch
    import paper_1806_08092_amd as gp
    name, g, lp, (G, _) = get_zoo()[0]
    st = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for prog, kw in (("nibble", {"epsilon": 0.0}), ("nibble", {"epsilon": float("nan")}),
                     ("nibble", {"epsilon": -1e-3}), ("bfs_parent", {"root": g.n}),
                     ("carry_bfs", {"persist": 0}), ("ppr", {"alpha": 1.5}), (99, {})):
        with pytest.raises(gp.GpopError) as e:
            G.state_init(prog, st, **kw)
        assert e.value.code == gp.EINVAL, (prog, kw)
    got, _ = run_program(G, "nibble", g.n, root=0, epsilon=1e-3)
    assert np.isfinite(got).all()


def test_max_iter_partial_state():
    name, g, lp, (G, _) = get_zoo()[3]  # path: one level per iteration
    got, iters = run_program(G, "bfs", g.n, root=0, max_iter=5)
    assert iters == 5
    assert G.frontier_size() == 1
    ref = oracle.bfs_levels(g, 0)
    assert np.array_equal(got[:6], ref[:6]) and np.all(got[6:] == INF)
    # continuing finishes the traversal
    G.run()
    import torch
    torch.cuda.synchronize()


def test_malformed_csr_rejected():
    import torch
    import paper_1806_08092_amd as gp
    off = torch.tensor([0, 2, 3], dtype=torch.int32, device="cuda")
    for cols in ([1, 0, 1], [0, 5, 1]):  # unsorted row, column out of range
        c = torch.tensor(cols, dtype=torch.int32, device="cuda")
        with pytest.raises(gp.GpopError) as e:
            gp.Graph(off, c, log2_part=8)
        assert e.value.code == gp.EINVAL
    bad_off = torch.tensor([0, 3, 2], dtype=torch.int32, device="cuda")
    with pytest.raises(gp.GpopError):
        gp.Graph(bad_off, torch.tensor([0, 1, 1], dtype=torch.int32, device="cuda"), log2_part=8)


@pytest.mark.parametrize("sc_log2,gids", [(6, 256), (8, 1024), (6, 4096)])
@pytest.mark.parametrize("sel", SELECTORS)
def test_task_splits(sc_log2, gids, sel):
    """Source-centric scatter cut into many small edge tasks (tasks start and
    end inside rows) and gathers split over many tasks plus the merge: results
    must not change."""
    g = gg.rmat_graph(12, 16, 41, weights_seed=42)
    sym = gg.rmat_graph(12, 16, 43, symmetric=True)
    G, _ = make_graph(g, 10, sc_task_log2=sc_log2, gather_task_ids=gids)
    Gs, _ = make_graph(sym, 10, sc_task_log2=sc_log2, gather_task_ids=gids)
    for root in roots_of(g, 2):
        got, _ = run_program(G, "bfs", g.n, root=root, selector=sel)
        assert np.array_equal(got, oracle.bfs_levels(g, root))
        got, _ = run_program(G, "sssp", g.n, root=root, selector=sel)
        assert np.array_equal(got, oracle.sssp(g, root))
        got, _ = run_program(G, "ppr", g.n, root=root, selector=sel, max_iter=20)
        assert pr_ok(got, oracle.ppr(g, root, 0.15, 20))
        got, _ = run_program(Gs, "carry_bfs", sym.n, root=root, persist=2, selector=sel)
        assert np.array_equal(got, oracle.bfs_levels(sym, root))
    got, _ = run_program(Gs, "cc", sym.n, selector=sel)
    assert np.array_equal(got, oracle.cc_minlabel(sym))
    got, _ = run_program(G, "pagerank", g.n, selector=sel, max_iter=10)
    assert pr_ok(got, oracle.pagerank(g, 0.85, 10))


def test_split_results_bitwise_equal_unsplit():
    g = gg.rmat_graph(12, 16, 44)
    G1, _ = make_graph(g, 10)
    G2, _ = make_graph(g, 10, sc_task_log2=6, gather_task_ids=256)
    a, _ = run_program(G1, "pagerank", g.n, max_iter=10)
    b, _ = run_program(G2, "pagerank", g.n, max_iter=10)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("sel", ["analytical", "sc"])
def test_split_scan_units(sel):
    """128 partitions (two blocks of 64 destinations) and 64-edge
    source-centric tasks, so the hub partitions have hundreds of tasks and
    their offset scans are split into one unit per destination block; results
    must match the oracle, and PageRank must be bitwise equal to the run with
    default task sizes."""
    g = gg.rmat_graph(15, 16, 45, weights_seed=46)
    sym = gg.rmat_graph(15, 16, 47, symmetric=True)
    G, _ = make_graph(g, 8, sc_task_log2=6)
    Gs, _ = make_graph(sym, 8, sc_task_log2=6)
    assert G.k == 128
    for root in roots_of(g, 2):
        got, _ = run_program(G, "bfs", g.n, root=root, selector=sel)
        assert np.array_equal(got, oracle.bfs_levels(g, root))
        got, _ = run_program(G, "sssp", g.n, root=root, selector=sel)
        assert np.array_equal(got, oracle.sssp(g, root))
        got, _ = run_program(G, "ppr", g.n, root=root, selector=sel, max_iter=20)
        assert pr_ok(got, oracle.ppr(g, root, 0.15, 20))
    got, _ = run_program(Gs, "cc", sym.n, selector=sel)
    assert np.array_equal(got, oracle.cc_minlabel(sym))
    a, _ = run_program(G, "pagerank", g.n, selector=sel, max_iter=10)
    assert pr_ok(a, oracle.pagerank(g, 0.85, 10))
    G1, _ = make_graph(g, 8)
    b, _ = run_program(G1, "pagerank", g.n, selector=sel, max_iter=10)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    # every active out-edge of a source-centric partition is one id: the
    # per-unit totals of a split scan must add up to it
    run_program(G, "bfs", g.n, root=roots_of(g, 1)[0], selector=sel)
    st = G.iter_stats()
    assert sum(r["sc_ids"] for r in st) > 0
    assert all(r["sc_ids"] == r["sc_active_edges"] for r in st)


def _hub_graph():
    """Many small messages into a few hubs: every vertex links to hubs 0, 1
    and 2 (hub 0 twice), plus a ring; 6000 vertices in 2^8-vertex
    partitions, so each bin holds a few dozen ids and a single combine round
    sees the same hub many times."""
    n = 6000
    edges = []
    for v in range(3, n):
        edges += [(v, 0), (v, 0), (v, 1), (v, 2), (v, (v + 1) % n)]
    edges += [(0, 5), (1, 6), (2, 7)]
    return edges_graph(n, edges)


@pytest.mark.parametrize("sel", SELECTORS)
@pytest.mark.parametrize("gids", [0, 256])
def test_sum_programs_with_hub_destinations(sel, gids):
    g = _hub_graph()
    G, _ = make_graph(g, 8, gather_task_ids=gids)
    ref = oracle.pagerank(g, 0.85, 10)
    got, _ = run_program(G, "pagerank", g.n, selector=sel, max_iter=10)
    assert pr_ok(got, ref), np.max(np.abs(got.astype(np.float64) - ref))
    ref = oracle.ppr(g, 7, 0.15, 20)
    got, _ = run_program(G, "ppr", g.n, root=7, selector=sel, max_iter=20)
    assert pr_ok(got, ref), np.max(np.abs(got.astype(np.float64) - ref))


def test_sum_with_hub_destinations_is_mode_and_split_invariant():
    g = _hub_graph()
    outs = []
    for gids in (0, 256):
        G, _ = make_graph(g, 8, gather_task_ids=gids)
        for sel in SELECTORS:
            got, _ = run_program(G, "pagerank", g.n, selector=sel, max_iter=10)
            outs.append(got.view(np.uint32))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("zi", [0, 1, 2, 4, 5, 8])
def test_atomic_free_combine_gives_the_same_bits(zi):
    """The atomic-free combine (write-verify / tag rounds) and the LDS
    combine give identical results for every program."""
    name, g, lp, (G, _) = get_zoo()[zi]
    R, _ = make_graph(g, lp, combine="rounds")
    root = roots_of(g, 1)[0]
    for prog, kw in [("bfs", {}), ("cc", {}), ("sssp", {}), ("pagerank", {"max_iter": 10}),
                     ("ppr", {"max_iter": 20})]:
        a, ia = run_program(G, prog, g.n, root=root, **kw)
        b, ib = run_program(R, prog, g.n, root=root, **kw)
        assert ia == ib and np.array_equal(a.view(np.uint32), b.view(np.uint32)), (name, prog)
    ref = oracle.bfs_levels(g, root)
    got, _ = run_program(R, "bfs", g.n, root=root)
    assert np.array_equal(got, ref)


def test_atomic_free_combine_on_hub_graph_and_splits():
    g = _hub_graph()
    for gids in (0, 256):
        A, _ = make_graph(g, 8, gather_task_ids=gids)
        R, _ = make_graph(g, 8, gather_task_ids=gids, combine="rounds")
        for prog, kw in [("pagerank", {"max_iter": 10}), ("ppr", {"root": 7, "max_iter": 20}), ("cc", {})]:
            a, _ = run_program(A, prog, g.n, **kw)
            b, _ = run_program(R, prog, g.n, **kw)
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (gids, prog)


@pytest.mark.gpu
@pytest.mark.parametrize("sel", ["analytical", "sc", "pc"])
def test_relabelled_rmat(sel):
    # the locality workload's input form: RMAT with vertex ids randomly
    # permuted, so hubs land in every partition and every bin fills
    g0 = gg.rmat_graph(14, 16, gg.BASE_SEED + 41, symmetric=True)
    g, perm = gg.permute_vertices(g0, gg.BASE_SEED + 42)
    root0 = roots_of(g0, 1)[0]
    G, _ = make_graph(g, 11)
    got, _ = run_program(G, "bfs", g.n, root=int(perm[root0]), selector=sel)
    ref = oracle.bfs_levels(g, int(perm[root0]))
    assert np.array_equal(got, ref)
    # levels are invariant under the relabelling
    assert np.array_equal(got[perm], oracle.bfs_levels(g0, root0))
    got, _ = run_program(G, "cc", g.n, selector=sel)
    assert np.array_equal(got, oracle.cc_minlabel(g))


@pytest.mark.gpu
def test_largest_partition_size():
    # q = 2^15, the largest partition the library takes: min programs fit the
    # LDS and agree with the oracle; sum programs need 8 bytes per vertex and
    # are refused; sizes outside [8, 15] are rejected
    import paper_1806_08092_amd as gp
    g = gg.rmat_graph(16, 8, gg.BASE_SEED + 43, symmetric=True)
    G, (off, cols, w) = make_graph(g, 15)
    assert G.info().q == 1 << 15 and G.info().k == 2
    root = roots_of(g, 1)[0]
    for sel in ("analytical", "sc", "pc"):
        got, _ = run_program(G, "bfs", g.n, root=root, selector=sel)
        assert np.array_equal(got, oracle.bfs_levels(g, root)), sel
        got, _ = run_program(G, "cc", g.n, selector=sel)
        assert np.array_equal(got, oracle.cc_minlabel(g)), sel
    for prog in ("pagerank", "nibble"):
        with pytest.raises(gp.GpopError) as e:
            run_program(G, prog, g.n, root=root, max_iter=2)
        assert e.value.code == gp.ENOTSUP, prog
    for lp in (7, 16):
        with pytest.raises(gp.GpopError) as e:
            gp.Graph(off, cols, w, log2_part=lp)
        assert e.value.code == gp.EINVAL, lp
