"""GPU parity at the benchmarked sizes, in the launch configuration the bench
times (default partition sizes, task sizes and Eq. 1 at the library's default
bandwidth ratio of 16):

- BFS levels and min-label CC on RMAT scale 22 ef16, symmetrised
  (4,194,304 vertices, 134,217,728 CSR entries, 2^14-vertex partitions);
- SSSP with u8 weights on RMAT scale 24 ef16 and on Erdos-Renyi 2^24 vertices
  of degree 16 (268,435,456 directed edges each, k = 1024 partitions).

Every output element is compared bit-exactly with the oracle. The ER case
also checks the shortest-path certificate (feasible on every edge, tight on
every reached vertex, reached set = reachable set), which fixes the distances
of a positively weighted graph by itself."""
import sys
import time

import numpy as np
import pytest

import graphgen as gg
import oracle

from gpu_util import make_graph, run_program, sssp_certificate, torch_cuda

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

INF = 0xFFFFFFFF


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_bfs_cc_rmat22_full_size():
    torch_cuda()
    t = time.perf_counter()
    g = gg.workload_bfs_cc_rmat22()
    say("rmat22 sym generated in %.1f s: V=%d E=%d" % (time.perf_counter() - t, g.n, g.m))
    G, _ = make_graph(g, 14)
    for root in gg.pick_sources(g.offsets, gg.SOURCE_SEED, 2).tolist():
        say("bfs rmat22 root", root)
        got, iters = run_program(G, "bfs", g.n, root=root, bw_ratio=16.0)
        ref = oracle.bfs_levels(g, root)
        bad = np.flatnonzero(got != ref)
        assert bad.size == 0, (root, bad[:8], got[bad[:8]], ref[bad[:8]])
        assert iters == int(ref[ref != INF].max()) + 1
    say("cc rmat22")
    got, _ = run_program(G, "cc", g.n, bw_ratio=16.0)
    ref = oracle.cc_minlabel(g)
    bad = np.flatnonzero(got != ref)
    assert bad.size == 0, (bad[:8], got[bad[:8]], ref[bad[:8]])


def test_sssp_rmat24_full_size():
    torch_cuda()
    t = time.perf_counter()
    g = gg.workload_sssp_rmat24()
    say("rmat24 generated in %.1f s: V=%d E=%d" % (time.perf_counter() - t, g.n, g.m))
    G, _ = make_graph(g, 14)
    root = int(gg.pick_sources(g.offsets, gg.SOURCE_SEED, 1)[0])
    say("sssp rmat24 root", root)
    got, _ = run_program(G, "sssp", g.n, root=root, bw_ratio=16.0)
    t = time.perf_counter()
    ref = oracle.sssp(g, root)
    say("oracle %.1f s" % (time.perf_counter() - t))
    bad = np.flatnonzero(got != ref)
    assert bad.size == 0, (root, bad[:8], got[bad[:8]], ref[bad[:8]])


def test_sssp_er24_full_size():
    torch_cuda()
    t = time.perf_counter()
    g = gg.workload_sssp_er24()
    say("er24 generated in %.1f s: V=%d E=%d" % (time.perf_counter() - t, g.n, g.m))
    G, _ = make_graph(g, 14)
    root = int(gg.pick_sources(g.offsets, gg.SOURCE_SEED, 1)[0])
    say("sssp er24 root", root)
    got, _ = run_program(G, "sssp", g.n, root=root, bw_ratio=16.0)
    say("certificate")
    sssp_certificate(g, root, got)
    t = time.perf_counter()
    ref = oracle.sssp(g, root)
    say("oracle %.1f s" % (time.perf_counter() - t))
    bad = np.flatnonzero(got != ref)
    assert bad.size == 0, (root, bad[:8], got[bad[:8]], ref[bad[:8]])
