"""Helpers for GPU tests: run a program through the C-ABI on seeded inputs."""
import numpy as np

import graphgen as gg

INF = 0xFFFFFFFF


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def make_graph(g, log2_part, sc_task_log2=0, gather_task_ids=0, combine="lds", pc_stream="auto",
               sc_reserve="auto"):
    import paper_1806_08092_amd as gp
    off, cols, w = gp.upload_csr(g)
    G = gp.Graph(off, cols, w, log2_part=log2_part, sc_task_log2=sc_task_log2,
                 gather_task_ids=gather_task_ids, combine=combine, pc_stream=pc_stream,
                 sc_reserve=sc_reserve)
    return G, (off, cols, w)


def run_program(G, prog, n, root=0, persist=1, selector="analytical", max_iter=1 << 20,
                damping=0.85, alpha=0.15, bw_ratio=2.0, frontier=None, epsilon=1e-6):
    """Runs one program to completion (or max_iter) and returns the state as
    a numpy array (uint32 or float32) plus the iterations run."""
    torch = torch_cuda()
    import paper_1806_08092_amd as gp
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    G.set_selector(selector, bw_ratio)
    G.state_init(prog, st, root=root, persist=persist, damping=damping, alpha=alpha, epsilon=epsilon)
    if frontier is not None:
        G.set_frontier(torch.as_tensor(np.asarray(frontier, np.int32), device="cuda"))
    elif prog in ("cc", "pagerank"):
        G.set_frontier_all()
    else:
        G.set_frontier(torch.tensor([root], dtype=torch.int32, device="cuda"))
    iters = G.run(max_iter)
    G.check()
    torch.cuda.synchronize()
    out = st.cpu().numpy()
    if prog in ("pagerank", "ppr", "nibble"):
        return out.view(np.float32), iters
    return out.view(np.uint32), iters


def pr_ok(x32, ref64, max_abs=1e-6, rel_l1=1e-5):
    x = x32.astype(np.float64)
    return (np.max(np.abs(x - ref64)) <= max_abs and
            np.sum(np.abs(x - ref64)) <= rel_l1 * np.sum(np.abs(ref64)))


def sssp_certificate(g, root, dist):
    """Shortest-path certificate for positive weights: dist[root] = 0; every
    edge u -> v with dist[u] finite has dist[v] <= dist[u] + w; every reached
    v != root has an in-edge with equality; the reached set is the set
    reachable from root (BFS levels). Together these force dist to equal the
    shortest-path distances."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.offsets.astype(np.int64)))
    dst = g.cols.astype(np.int64)
    w = g.weights.astype(np.int64)
    d = dist.astype(np.int64)
    fin = d[src] != INF
    assert d[root] == 0
    import oracle
    reach = oracle.bfs_levels(g, root) != INF
    assert np.array_equal(dist != INF, reach)
    cand = d[src[fin]] + w[fin]
    assert np.all(d[dst[fin]] <= cand)
    tight = np.zeros(g.n, bool)
    tight[dst[fin][d[dst[fin]] == cand]] = True
    tight[root] = True
    assert np.all(tight[reach])
