"""GPU parity of the column-stream gather of partition-centric bins.

Gather can read the static ids of partition-centric bins either bin by bin
(pc_stream "off") or from each destination partition's column stream (pc_stream
"on": 256-id chunks that span several bins, a bin-start bitmap and a per-chunk
table of message offsets). Both must give the oracle's results, bit for bit
equal to each other for every program (the sums are exact fixed-point sums),
with the same per-iteration statistics. The cases cover dense iterations (every
partition partition-centric), mixed ones (bins of source-centric or inactive
sources inside a chunk read the identity words), columns split over several
gather tasks, and columns whose bins are so small that chunks need padding
runs (at most 62 bins start inside one chunk)."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

from gpu_util import INF, make_graph, pr_ok, run_program, torch_cuda

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def edges_graph(n, src, dst, wseed=None):
    return gg.from_edges(n, np.asarray(src, np.uint32), np.asarray(dst, np.uint32), wseed)


def fragmented_graph(symmetric):
    """2^16 vertices in 256 partitions of 256: partition 0 receives one edge
    from every partition (its column holds 256 one-id bins, so its first
    chunks fill up with bin starts and padding moves bins to the next
    chunk); partition 7 receives a few ids from every partition; plus a
    sparse random layer so that most vertices are reachable."""
    n, q = 1 << 16, 256
    rng = np.random.default_rng(5)
    src, dst = [], []
    for p in range(n // q):
        src.append(p * q + 1)
        dst.append(p % q)
        for j in range(3):
            src.append(p * q + 2 + j)
            dst.append(7 * q + (p * 3 + j) % q)
    m = 4 * n
    src.extend(rng.integers(0, n, m).tolist())
    dst.extend(rng.integers(0, n, m).tolist())
    src, dst = np.array(src, np.uint32), np.array(dst, np.uint32)
    if symmetric:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    return edges_graph(n, src, dst, 77)


def cases():
    return [
        ("rmat10", gg.rmat_graph(10, 8, 11, weights_seed=12), 8, 0),
        ("rmat11sym", gg.rmat_graph(11, 8, 13, symmetric=True, weights_seed=14), 8, 0),
        ("er3000", gg.er_graph(3000, 24000, 15, weights_seed=16), 8, 0),
        ("star", edges_graph(1500, list(range(1, 1500)) + [0] * 1499,
                             [0] * 1499 + list(range(1, 1500)), 18), 8, 0),
        ("single", edges_graph(1, [0], [0], 20), 8, 0),
        ("noedges", edges_graph(300, [], [], 21), 8, 0),
        ("rmat12_q10", gg.rmat_graph(12, 16, 22, weights_seed=23), 10, 0),
        ("rmat14sym_split", gg.rmat_graph(14, 16, 31, symmetric=True, weights_seed=32), 10, 256),
        ("fragmented", fragmented_graph(False), 8, 0),
        ("fragmented_sym_split", fragmented_graph(True), 8, 512),
    ]


CASES = None


def get_cases():
    global CASES
    if CASES is None:
        CASES = []
        for name, g, lp, gids in cases():
            Gs = {m: make_graph(g, lp, gather_task_ids=gids, pc_stream=m)[0] for m in ("on", "off")}
            CASES.append((name, g, Gs))
    return CASES


def roots_of(g, n=2):
    r = gg.pick_sources(g.offsets, 99, n).tolist()
    return r if r else [0]


def run_both(Gs, g, prog, sel, **kw):
    out = {}
    for m, G in Gs.items():
        got, iters = run_program(G, prog, g.n, selector=sel, **kw)
        out[m] = (got, iters, [r["gathered_ids"] for r in G.iter_stats()],
                  [r["gathered_bins"] for r in G.iter_stats()])
    a, b = out["on"], out["off"]
    assert a[1] == b[1], (prog, sel, "iterations", a[1], b[1])
    assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32)), (prog, sel, "results differ")
    assert a[2] == b[2], (prog, sel, "gathered ids per iteration", a[2], b[2])
    assert a[3] == b[3], (prog, sel, "gathered bins per iteration", a[3], b[3])
    return a[0], a[1]


@pytest.mark.parametrize("ci", range(10))
@pytest.mark.parametrize("sel", ["analytical", "pc"])
def test_min_programs(ci, sel):
    torch_cuda()
    name, g, Gs = get_cases()[ci]
    for root in roots_of(g):
        say("stream", name, sel, "root", root)
        got, _ = run_both(Gs, g, "bfs", sel, root=root, bw_ratio=16.0)
        assert np.array_equal(got, oracle.bfs_levels(g, root)), (name, sel, root)
        got, _ = run_both(Gs, g, "bfs_parent", sel, root=root)
        assert np.array_equal(got, oracle.bfs_parents(g, root)), (name, sel, root)
        got, _ = run_both(Gs, g, "sssp", sel, root=root)
        assert np.array_equal(got, oracle.sssp(g, root)), (name, sel, root)
        got, _ = run_both(Gs, g, "carry_bfs", sel, root=root, persist=2)
        assert np.array_equal(got, oracle.bfs_levels(g, root)), (name, sel, root)
    got, _ = run_both(Gs, g, "cc", sel)
    if "sym" in name or name in ("star", "single", "noedges"):
        assert np.array_equal(got, oracle.cc_minlabel(g)), (name, sel)


@pytest.mark.parametrize("ci", range(10))
@pytest.mark.parametrize("sel", ["analytical", "pc"])
def test_sum_programs(ci, sel):
    torch_cuda()
    name, g, Gs = get_cases()[ci]
    say("stream pagerank", name, sel)
    got, iters = run_both(Gs, g, "pagerank", sel, max_iter=10)
    assert iters == 10
    assert pr_ok(got, oracle.pagerank(g, 0.85, 10)), name
    for seed in roots_of(g):
        say("stream ppr / nibble", name, sel, seed)
        got, _ = run_both(Gs, g, "ppr", sel, root=seed, max_iter=20)
        assert pr_ok(got, oracle.ppr(g, seed, 0.15, 20)), (name, seed)
        run_both(Gs, g, "nibble", sel, root=seed, max_iter=30, epsilon=3.7e-5)


def test_auto_mode_at_scale():
    """RMAT-18 symmetrised at the default sizes: the default (auto) layout
    choice gives the oracle's BFS levels and CC labels, and the same bits
    as both fixed layouts."""
    torch_cuda()
    g = gg.rmat_graph(18, 16, gg.BASE_SEED + 61, symmetric=True)
    Gs = {m: make_graph(g, 14, pc_stream=m)[0] for m in ("auto", "on", "off")}
    for root in gg.pick_sources(g.offsets, gg.SOURCE_SEED, 2).tolist():
        say("stream rmat18 bfs", root)
        ref = oracle.bfs_levels(g, root)
        for m, G in Gs.items():
            got, iters = run_program(G, "bfs", g.n, root=root, bw_ratio=16.0)
            assert np.array_equal(got, ref), (m, root)
            assert iters == int(ref[ref != INF].max()) + 1
    ref = oracle.cc_minlabel(g)
    for m, G in Gs.items():
        got, _ = run_program(G, "cc", g.n, bw_ratio=16.0)
        assert np.array_equal(got, ref), m
