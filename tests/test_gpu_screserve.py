"""GPU parity of the two ways a source-centric task reserves bin slots.

Per message piece (one device-wide atomic each) and per bin (the wave counts
its pieces per bin in LDS, reserves each bin's share with one atomic, then
walks its task again) must both give the oracle's results, bit for bit equal
to each other (only the order of messages inside a bin differs, and the
combines do not depend on it: minima, and sums in exact fixed point), with
the same per-iteration statistics. Every partition is scattered
source-centric in the "sc" cases; the cases include hubs whose runs into one
partition are longer than a piece (256 edges), tasks that start inside such
runs, and weighted programs."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

from gpu_util import make_graph, pr_ok, run_program, torch_cuda

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def edges_graph(n, src, dst, wseed=None):
    return gg.from_edges(n, np.asarray(src, np.uint32), np.asarray(dst, np.uint32), wseed)


def hub_graph():
    """2^14 vertices in 64 partitions of 256: vertex 0 points at every vertex
    (runs of 256 edges into each partition, one piece each), vertex 300 at
    every vertex of partitions 0-2 twice over through a second hub 301 (runs
    that fill whole partitions), plus a sparse random layer."""
    n = 1 << 14
    rng = np.random.default_rng(41)
    src = [0] * n + [300] * 768 + [301] * 700
    dst = list(range(n)) + list(range(768)) + list(rng.choice(768, 700, replace=False))
    m = 3 * n
    src += rng.integers(0, n, m).tolist()
    dst += rng.integers(0, n, m).tolist()
    s, d = np.array(src, np.uint32), np.array(dst, np.uint32)
    return edges_graph(n, np.concatenate([s, d]), np.concatenate([d, s]), 43)


def cases():
    return [
        ("rmat11sym", gg.rmat_graph(11, 8, 13, symmetric=True, weights_seed=14), 8, 0),
        ("er3000", gg.er_graph(3000, 24000, 15, weights_seed=16), 8, 0),
        ("star", edges_graph(1500, list(range(1, 1500)) + [0] * 1499,
                             [0] * 1499 + list(range(1, 1500)), 18), 8, 0),
        ("single", edges_graph(1, [0], [0], 20), 8, 0),
        ("noedges", edges_graph(300, [], [], 21), 8, 0),
        ("hub", hub_graph(), 8, 0),
        ("hub_small_tasks", hub_graph(), 8, 6),
        ("rmat14sym", gg.rmat_graph(14, 16, 31, symmetric=True, weights_seed=32), 10, 0),
    ]


CASES = None


def get_cases():
    global CASES
    if CASES is None:
        CASES = []
        for name, g, lp, sct in cases():
            Gs = {m: make_graph(g, lp, sc_task_log2=sct, sc_reserve=m)[0] for m in ("piece", "bin")}
            CASES.append((name, g, Gs))
    return CASES


def run_both(Gs, g, prog, sel, **kw):
    out = {}
    for m, G in Gs.items():
        got, iters = run_program(G, prog, g.n, selector=sel, **kw)
        st = G.iter_stats()
        out[m] = (got, iters, [(r["sc_msgs"], r["sc_ids"], r["gathered_ids"]) for r in st])
    a, b = out["piece"], out["bin"]
    assert a[1] == b[1], (prog, sel, "iterations", a[1], b[1])
    assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32)), (prog, sel, "results differ")
    assert a[2] == b[2], (prog, sel, "per-iteration source-centric messages, ids, gathered ids")
    return a[0], a[1]


def roots_of(g, n=2):
    r = gg.pick_sources(g.offsets, 99, n).tolist()
    return r if r else [0]


@pytest.mark.parametrize("ci", range(8))
@pytest.mark.parametrize("sel", ["sc", "analytical"])
def test_min_programs(ci, sel):
    torch_cuda()
    name, g, Gs = get_cases()[ci]
    for root in roots_of(g) + ([0] if name.startswith("hub") else []):
        say("screserve", name, sel, "root", root)
        got, _ = run_both(Gs, g, "bfs", sel, root=root, bw_ratio=2.0)
        assert np.array_equal(got, oracle.bfs_levels(g, root)), (name, sel, root)
        got, _ = run_both(Gs, g, "bfs_parent", sel, root=root)
        assert np.array_equal(got, oracle.bfs_parents(g, root)), (name, sel, root)
        got, _ = run_both(Gs, g, "sssp", sel, root=root)
        assert np.array_equal(got, oracle.sssp(g, root)), (name, sel, root)
    got, _ = run_both(Gs, g, "cc", sel)
    if name != "er3000":  # symmetric graphs: min labels are the components
        assert np.array_equal(got, oracle.cc_minlabel(g)), (name, sel)


@pytest.mark.parametrize("ci", range(8))
def test_sum_programs_source_centric(ci):
    torch_cuda()
    name, g, Gs = get_cases()[ci]
    say("screserve pagerank", name)
    got, iters = run_both(Gs, g, "pagerank", "sc", max_iter=10)
    assert iters == 10
    assert pr_ok(got, oracle.pagerank(g, 0.85, 10)), name
    for seed in roots_of(g):
        got, _ = run_both(Gs, g, "ppr", "sc", root=seed, max_iter=20)
        assert pr_ok(got, oracle.ppr(g, seed, 0.15, 20)), (name, seed)
