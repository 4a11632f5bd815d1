"""Columns whose bins come from more source partitions than a gather
workgroup lists at once (512): symmetrised RMAT-18 with q = 256 gives
k = 1024 partitions, and its busiest columns receive bins from more than
512 of them, so their gather takes the bins in several windows. BFS levels,
CC and SSSP stay bit-exact against the oracle under the analytical, the
all source-centric and the all partition-centric selection, and with both
source-centric reservation modes."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import make_graph, run_program

pytestmark = pytest.mark.gpu

_G = {}


def graph(sc_reserve="auto", task_ids=0):
    key = (sc_reserve, task_ids)
    if key not in _G:
        g = gg.rmat_graph(18, 8, 31, symmetric=True, weights_seed=32)
        G, _ = make_graph(g, 8, sc_reserve=sc_reserve, gather_task_ids=task_ids)
        _G[key] = (g, G)
    return _G[key]


def test_columns_span_several_windows():
    g, G = graph()
    assert G.info().k == 1024
    # source partitions with an edge into each column (host-side, from the CSR)
    deg = np.diff(g.offsets.astype(np.int64))
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg) >> 8
    dst = g.cols.astype(np.int64) >> 8
    pairs = np.unique(dst * 1024 + src)
    per_col = np.bincount(pairs // 1024, minlength=1024)
    assert per_col.max() > 512, per_col.max()


@pytest.mark.parametrize("sel,reserve", [("analytical", "auto"), ("sc", "auto"), ("pc", "auto"),
                                         ("sc", "bin"), ("analytical", "piece")])
def test_bfs_cc_sssp(sel, reserve):
    # reserve: how source-centric tasks reserve bin slots (per bin: a k-word
    # LDS row per wave, 1024 words here)
    g, G = graph(reserve)
    for root in gg.pick_sources(g.offsets, 33, 2).tolist():
        got, _ = run_program(G, "bfs", g.n, root=root, selector=sel)
        ref = oracle.bfs_levels(g, root)
        assert np.array_equal(got, ref), ("bfs", sel, root, np.flatnonzero(got != ref)[:10])
        got, _ = run_program(G, "sssp", g.n, root=root, selector=sel)
        ref = oracle.sssp(g, root)
        assert np.array_equal(got, ref), ("sssp", sel, root, np.flatnonzero(got != ref)[:10])
    got, _ = run_program(G, "cc", g.n, selector=sel)
    ref = oracle.cc_minlabel(g)
    assert np.array_equal(got, ref), ("cc", sel, np.flatnonzero(got != ref)[:10])


def test_split_tasks_take_their_source_ranges():
    # gather tasks of about 2^14 ids: the heavy columns split into tasks that
    # each list only the bins of their own source-partition range
    g, G = graph("auto", 1 << 14)
    got, _ = run_program(G, "cc", g.n, selector="sc")
    assert np.array_equal(got, oracle.cc_minlabel(g))
    assert max(r["split_tasks"] for r in G.iter_stats()) > 0
    for root in gg.pick_sources(g.offsets, 34, 2).tolist():
        got, _ = run_program(G, "bfs", g.n, root=root, selector="analytical")
        ref = oracle.bfs_levels(g, root)
        assert np.array_equal(got, ref), ("bfs", root, np.flatnonzero(got != ref)[:10])
