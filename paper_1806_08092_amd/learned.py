"""Training-set collection and training of the learned scatter-mode selector.

Orchestration only: features, per-partition scatter timings, the network's
gradient and Adam all run in libgpop's kernels (gpop_features,
gpop_probe_scatter, gpop_mlp_*); this module loops over iterations and
batches. The selector is described in include/gpop_mlp.h.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import MLP_IN, Mlp


@dataclass
class Samples:
    """Per-(iteration, active partition) training rows: raw features and the
    cost of the partition's iteration in each mode (microseconds): its
    measured scatter time plus, when collected with gather costs, the ids the
    mode sends to gather times that iteration's measured gather time per id
    (source-centric mode sends one id per active out-edge, partition-centric
    mode every static id of the partition)."""
    x: np.ndarray        # n x 12 float32
    t_sc: np.ndarray     # n float32
    t_pc: np.ndarray     # n float32
    it: np.ndarray       # n int32, iteration of the row
    tot_sc: List[float]  # whole SC / PC scatter time of each iteration
    tot_pc: List[float]

    @staticmethod
    def concat(parts: List["Samples"]) -> "Samples":
        return Samples(np.concatenate([p.x for p in parts]), np.concatenate([p.t_sc for p in parts]),
                       np.concatenate([p.t_pc for p in parts]), np.concatenate([p.it for p in parts]),
                       sum((p.tot_sc for p in parts), []), sum((p.tot_pc for p in parts), []))

    def __len__(self):
        return self.x.shape[0]


def collect(G, max_iter: int = 1 << 20, stream=None, gather_cost: bool = True) -> Samples:
    """Runs the program bound to G (state and frontier already set) to the
    end, probing both scatter modes before every iteration. With gather_cost
    the iterations run with profiling on, and each row's mode costs include
    the modelled gather time of the ids the mode sends."""
    xs, tsc, tpc, its, tot_sc, tot_pc = [], [], [], [], [], []
    if gather_cost:
        G.profile_enable(True)
    try:
        for it in range(max_iter):
            if G.frontier_size(stream) == 0:
                break
            f = G.features(stream).cpu().numpy()
            a, ta = G.probe_scatter("sc", stream)
            b, tb = G.probe_scatter("pc", stream)
            act = f[:, 0] > 0          # log1p(V_a) > 0: the partition scatters
            a = a[act].astype(np.float64)
            b = b[act].astype(np.float64)
            before = G.profile_read(stream) if gather_cost else None
            G.iterate(stream)
            if gather_cost:
                after = G.profile_read(stream)
                g_ms = sum(after[k][0] - before[k][0] for k in ("gather", "merge"))
                rec = G.iter_stats(stream)[-1]
                ids = rec["sc_ids"] + rec["pc_ids"]
                per_id = g_ms * 1e3 / ids if ids else 0.0
                a = a + per_id * np.expm1(f[act, 1].astype(np.float64))   # E_a ids
                b = b + per_id * np.expm1(f[act, 2].astype(np.float64))   # E^p ids
            xs.append(f[act])
            tsc.append(a.astype(np.float32))
            tpc.append(b.astype(np.float32))
            its.append(np.full(int(act.sum()), it, np.int32))
            tot_sc.append(ta)
            tot_pc.append(tb)
    finally:
        if gather_cost:
            G.profile_enable(False)
    if not xs:
        return Samples(np.zeros((0, MLP_IN), np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32),
                       np.zeros(0, np.int32), [], [])
    return Samples(np.concatenate(xs).astype(np.float32), np.concatenate(tsc), np.concatenate(tpc),
                   np.concatenate(its), tot_sc, tot_pc)


def train(data: Samples, init_params: np.ndarray, steps: int = 2000, batch: int = 4096, lr: float = 1e-3,
          seed: int = 0, stream=None) -> Mlp:
    """Trains a model on `data` with minibatches drawn uniformly with a
    seeded generator; returns the Mlp (its .model is what the selector
    reads)."""
    import torch
    dev = "cuda"
    x = torch.from_numpy(np.ascontiguousarray(data.x, np.float32)).to(dev)
    a = torch.from_numpy(np.ascontiguousarray(data.t_sc, np.float32)).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(data.t_pc, np.float32)).to(dev)
    mlp = Mlp()
    mlp.init(torch.from_numpy(np.asarray(init_params, np.float32)).to(dev), x, stream)
    n = x.shape[0]
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    for _ in range(steps):
        if n <= batch:
            xb, ab, bb = x, a, b
        else:
            idx = torch.randint(0, n, (batch,), device=dev, generator=gen)
            xb, ab, bb = x[idx].contiguous(), a[idx].contiguous(), b[idx].contiguous()
        mlp.train_step(xb, ab, bb, lr=lr, stream=stream)
    return mlp


def choice_cost(pick_pc: np.ndarray, data: Samples) -> float:
    """Total measured scatter time of the given per-row choices."""
    return float(np.where(pick_pc, data.t_pc, data.t_sc).sum())


def analytical_choice(data: Samples, bw_ratio: float = 16.0) -> np.ndarray:
    """Eq. 1's choice for each row from the last feature, which is
    log(cost_PC / cost_SC) (PC iff cost_PC <= ratio cost_SC)."""
    return data.x[:, 11].astype(np.float64) <= math.log(bw_ratio)


def calibrate_offset(mlp, time_runs, offsets=(-1.0, 0.0, 0.5, 1.0, 2.0, 4.0, 8.0, 16.0), stream=None):
    """Moves the network's decision threshold to where whole runs are
    fastest. The per-row labels price each mode with every partition
    scattering in it, so they miss how modes interact in one iteration; the
    threshold corrects the resulting bias. Each candidate offset is added to
    the output bias in turn (Mlp.shift_logit), time_runs() times whole runs
    on training graphs (ms), and the fastest offset stays in the model (the
    one nearer 0 on a tie). Returns (offset, {offset: ms})."""
    cur = 0.0
    res = {}
    for d in offsets:
        mlp.shift_logit(float(d) - cur, stream)
        cur = float(d)
        res[float(d)] = float(time_runs())
    best = min(res, key=lambda d: (res[d], abs(d)))
    mlp.shift_logit(best - cur, stream)
    return best, res


def calibrate_ratio(data: Samples, grid: Optional[np.ndarray] = None) -> float:
    """The bandwidth ratio whose Eq. 1 choices cost least on `data`."""
    if grid is None:
        grid = 2.0 ** np.arange(-4.0, 8.01, 0.25)
    costs = [choice_cost(analytical_choice(data, r), data) for r in grid]
    return float(grid[int(np.argmin(costs))])
