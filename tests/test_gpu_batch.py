"""GPU tests of batched runs: many seeds on one graph and many uneven graphs
in one launch sequence (recorded HIP graph or direct launches), against the
oracle and bitwise against single runs."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import make_graph, pr_ok, run_program, torch_cuda

pytestmark = pytest.mark.gpu


def _states(torch, n, count):
    return [torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(count)]


@pytest.mark.parametrize("eager", [False, True])
def test_batch_bfs_seeds_match_oracle_and_single_runs(eager):
    torch = torch_cuda()
    import paper_1806_08092_amd as gp
    g = gg.rmat_graph(12, 8, seed=gg.BASE_SEED + 80, symmetric=True)
    G, _ = make_graph(g, 8)
    seeds = [int(s) for s in gg.pick_sources(g.offsets, gg.SOURCE_SEED + 3, 16)]
    B = gp.Batch([G] * len(seeds))
    st = _states(torch, g.n, len(seeds))
    for rep in range(2):  # a second run replays the recorded graph
        B.state_init("bfs", st, roots=seeds)
        for i, s in enumerate(seeds):
            B.set_frontier(i, torch.tensor([s], dtype=torch.int32, device="cuda"))
        iters = B.run(eager=eager)
        B.check()
        torch.cuda.synchronize()
        for i, s in enumerate(seeds):
            lv = oracle.bfs_levels(g, s)
            got = st[i].cpu().numpy().view(np.uint32)
            assert np.array_equal(got, lv), (rep, i)
            _, single_iters = run_program(G, "bfs", g.n, root=s)
            assert iters[i] == single_iters


def test_batch_graph_replay_equals_eager_with_work_in_between():
    torch = torch_cuda()
    import paper_1806_08092_amd as gp
    g = gg.rmat_graph(11, 16, seed=gg.BASE_SEED + 81, symmetric=True, weights_seed=gg.BASE_SEED + 82)
    G, _ = make_graph(g, 8)
    seeds = [int(s) for s in gg.pick_sources(g.offsets, gg.SOURCE_SEED + 4, 6)]
    B = gp.Batch([G] * len(seeds))
    st = _states(torch, g.n, len(seeds))
    outs = []
    for eager in (True, False, False, False):
        B.state_init("sssp", st, roots=seeds)
        for i, s in enumerate(seeds):
            B.set_frontier(i, torch.tensor([s], dtype=torch.int32, device="cuda"))
        B.run(eager=eager)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy().copy() for x in st])
        run_program(G, "cc", g.n)  # other work on the graph between replays
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)
    for i, s in enumerate(seeds):
        assert np.array_equal(outs[0][i].view(np.uint32), oracle.sssp(g, s))


def test_batch_ppr_seeds_bitwise_equal_single_runs():
    torch = torch_cuda()
    import paper_1806_08092_amd as gp
    g = gg.rmat_graph(12, 8, seed=gg.BASE_SEED + 83, symmetric=True)
    G, _ = make_graph(g, 9)
    seeds = [int(s) for s in gg.pick_sources(g.offsets, gg.SOURCE_SEED + 5, 8)]
    B = gp.Batch([G] * len(seeds))
    st = _states(torch, g.n, len(seeds))
    B.state_init("ppr", st, roots=seeds, alpha=0.15)
    for i, s in enumerate(seeds):
        B.set_frontier(i, torch.tensor([s], dtype=torch.int32, device="cuda"))
    iters = B.run(max_iter=20)
    B.check()
    assert all(it == 20 for it in iters)
    for i, s in enumerate(seeds):
        got = st[i].cpu().numpy().view(np.float32)
        ref = oracle.ppr(g, s, 0.15, 20)
        assert pr_ok(got, ref)
        single, _ = run_program(G, "ppr", g.n, root=s, max_iter=20)
        assert np.array_equal(got.view(np.uint32), single.view(np.uint32))


@pytest.mark.parametrize("eager", [False, True])
def test_batch_bfs_parents_and_nibble_equal_single_runs(eager):
    """The two newest programs batched over seeds: BFS parents against the
    oracle, and both bitwise against single runs (iteration counts too)."""
    torch = torch_cuda()
    import paper_1806_08092_amd as gp
    g = gg.rmat_graph(12, 8, seed=gg.BASE_SEED + 84, symmetric=True)
    G, _ = make_graph(g, 9)
    seeds = [int(s) for s in gg.pick_sources(g.offsets, gg.SOURCE_SEED + 6, 8)]
    B = gp.Batch([G] * len(seeds))
    st = _states(torch, g.n, len(seeds))
    for prog, kw in (("bfs_parent", {}), ("nibble", {"epsilon": 1e-5})):
        B.state_init(prog, st, roots=seeds, **kw)
        for i, s in enumerate(seeds):
            B.set_frontier(i, torch.tensor([s], dtype=torch.int32, device="cuda"))
        iters = B.run(max_iter=40, eager=eager)
        B.check()
        torch.cuda.synchronize()
        for i, s in enumerate(seeds):
            got = st[i].cpu().numpy().view(np.uint32)
            if prog == "bfs_parent":
                assert np.array_equal(got, oracle.bfs_parents(g, s)), (prog, i)
            single, single_iters = run_program(G, prog, g.n, root=s, max_iter=40, **kw)
            assert np.array_equal(got, single.view(np.uint32)), (prog, i)
            assert iters[i] == single_iters, (prog, i)


def _uneven_graphs(symmetric):
    """Directed graphs for PageRank; min-label CC needs symmetric ones."""
    out = []
    for i in range(7):
        scale = 8 + (i % 5)
        ef = 4 * (1 + (i % 4))
        lp = 8 + (i % 3)
        out.append((gg.rmat_graph(scale, ef, seed=gg.BASE_SEED + 90 + i, symmetric=symmetric), lp))
    if symmetric:
        src, dst = gg.symmetrize(*gg.er_edges(5000, 15000, gg.BASE_SEED + 99))
        out.append((gg.from_edges(5000, src, dst), 9))
    else:
        out.append((gg.er_graph(5000, 30000, seed=gg.BASE_SEED + 99), 9))
    return out


@pytest.mark.parametrize("prog", ["pagerank", "cc"])
def test_batch_uneven_graphs(prog):
    torch = torch_cuda()
    import paper_1806_08092_amd as gp
    items = _uneven_graphs(prog == "cc")
    Gs = [make_graph(g, lp)[0] for g, lp in items]
    B = gp.Batch(Gs)
    st = [torch.empty(g.n, dtype=torch.int32, device="cuda") for g, _ in items]
    B.state_init(prog, st)
    for i in range(len(items)):
        B.set_frontier_all(i)
    max_iter = 10 if prog == "pagerank" else 1 << 20
    B.run(max_iter=max_iter)
    B.check()
    for i, (g, _) in enumerate(items):
        single, _ = run_program(Gs[i], prog, g.n, max_iter=max_iter)
        got = st[i].cpu().numpy()
        assert np.array_equal(got.view(np.uint32), single.view(np.uint32)), i
        if prog == "pagerank":
            assert pr_ok(got.view(np.float32), oracle.pagerank(g, 0.85, 10)), i
        else:
            assert np.array_equal(got.view(np.uint32), oracle.cc_minlabel(g)), i


def test_batch_iteration_limit_and_errors():
    torch = torch_cuda()
    import paper_1806_08092_amd as gp
    g = gg.rmat_graph(10, 8, seed=gg.BASE_SEED + 84, symmetric=True)
    G, _ = make_graph(g, 8)
    B = gp.Batch([G, G])
    st = _states(torch, g.n, 2)
    with pytest.raises(gp.GpopError):
        B.run()  # before state_init
    B.state_init("bfs", st, roots=[0, 1])
    B.set_frontier(0, torch.tensor([0], dtype=torch.int32, device="cuda"))
    B.set_frontier(1, torch.tensor([1], dtype=torch.int32, device="cuda"))
    iters = B.run(max_iter=2)
    assert iters == [2, 2]
    for i in range(2):
        want, _ = run_program(G, "bfs", g.n, root=i, max_iter=2)
        assert np.array_equal(st[i].cpu().numpy().view(np.uint32), want)
    with pytest.raises(gp.GpopError) as e:
        B.set_frontier(0, torch.tensor([0], dtype=torch.int32, device="cuda"))  # after running
    assert e.value.code == gp.ESTATE
    with pytest.raises(gp.GpopError) as e:
        B.state_init("bfs", st, roots=[0, g.n])  # root out of range
    assert e.value.code == gp.EINVAL


@pytest.mark.parametrize("prog", ["pagerank", "bfs"])
def test_autotune_choice_is_fastest_tried_and_correct(prog):
    torch = torch_cuda()
    import paper_1806_08092_amd as gp
    g = gg.rmat_graph(13, 8, seed=gg.BASE_SEED + 85, symmetric=(prog == "bfs"))
    off, cols, w = gp.upload_csr(g)
    root = int(gg.pick_sources(g.offsets, gg.SOURCE_SEED, 1)[0])
    front = None if prog == "pagerank" else torch.tensor([root], dtype=torch.int32, device="cuda")
    best, table = gp.autotune(off, cols, w, prog, root=root, frontier=front, max_iter=3, reps=1)
    ran = [(c, ms) for c, ms, _ in table if ms >= 0]
    assert ran and best in [c for c, _ in ran]
    assert min(ms for _, ms in ran) == [ms for c, ms in ran if c == best][0]
    G = gp.Graph(off, cols, w, **best)
    if prog == "pagerank":
        got, _ = run_program(G, "pagerank", g.n, max_iter=10)
        assert pr_ok(got, oracle.pagerank(g, 0.85, 10))
    else:
        got, _ = run_program(G, "bfs", g.n, root=root)
        assert np.array_equal(got, oracle.bfs_levels(g, root))


@pytest.mark.parametrize("sel", ["analytical", "sc"])
def test_batch_at_scale_rmat18(sel):
    """A batch of 16 BFS and then 8 SSSP runs on RMAT-18 symmetrised at the
    default partition size (k = 16), under Eq. 1 at the default ratio and
    with every partition source-centric: every run equals the oracle, and
    per-run iteration counts equal single runs'."""
    torch = torch_cuda()
    import paper_1806_08092_amd as gp
    g = gg.rmat_graph(18, 16, seed=gg.BASE_SEED + 86, symmetric=True, weights_seed=gg.BASE_SEED + 87)
    G, _ = make_graph(g, 14)
    G.set_selector(sel, 16.0)
    for prog, count in (("bfs", 16), ("sssp", 8)):
        seeds = [int(s) for s in gg.pick_sources(g.offsets, gg.SOURCE_SEED + 7, count)]
        B = gp.Batch([G] * count)
        st = _states(torch, g.n, count)
        B.state_init(prog, st, roots=seeds)
        for i, s in enumerate(seeds):
            B.set_frontier(i, torch.tensor([s], dtype=torch.int32, device="cuda"))
        iters = B.run()
        B.check()
        torch.cuda.synchronize()
        for i, s in enumerate(seeds):
            want = oracle.bfs_levels(g, s) if prog == "bfs" else oracle.sssp(g, s)
            assert np.array_equal(st[i].cpu().numpy().view(np.uint32), want), (prog, sel, i)
        for i in (0, count - 1):
            _, single_iters = run_program(G, prog, g.n, root=seeds[i], selector=sel, bw_ratio=16.0)
            assert iters[i] == single_iters, (prog, sel, i)
        B.close()
