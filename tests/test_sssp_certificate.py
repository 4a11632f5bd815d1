"""The shortest-path certificate used by the full-size GPU tests accepts the
oracle's distances and rejects planted mistakes (CPU only)."""
import numpy as np
import pytest

import graphgen as gg
import oracle

from gpu_util import INF, sssp_certificate


@pytest.mark.parametrize("kind", ["rmat", "er"])
def test_certificate_accepts_oracle_and_rejects_mistakes(kind):
    if kind == "rmat":
        g = gg.rmat_graph(12, 16, 41, weights_seed=42)
    else:
        g = gg.er_graph(4096, 65536, 43, weights_seed=44)
    root = int(gg.pick_sources(g.offsets, 45, 1)[0])
    d = oracle.sssp(g, root)
    sssp_certificate(g, root, d)
    reached = np.flatnonzero((d != INF) & (np.arange(g.n) != root))
    rng = np.random.default_rng(46)
    for v in rng.choice(reached, 4, replace=False):
        for delta in (-1, 1):
            bad = d.copy()
            bad[v] = np.uint32(int(bad[v]) + delta)
            with pytest.raises(AssertionError):
                sssp_certificate(g, root, bad)
    bad = d.copy()
    bad[root] = 1
    with pytest.raises(AssertionError):
        sssp_certificate(g, root, bad)
    unreached = np.flatnonzero(d == INF)
    if unreached.size:
        bad = d.copy()
        bad[unreached[0]] = 7
        with pytest.raises(AssertionError):
            sssp_certificate(g, root, bad)
