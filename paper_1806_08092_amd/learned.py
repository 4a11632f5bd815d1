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
    # with gather costs: the scatter-only times of the rows, and per iteration
    # the measured gather + merge time (us) with the ids each mode sent
    s_sc: Optional[np.ndarray] = None
    s_pc: Optional[np.ndarray] = None
    g_us: Optional[np.ndarray] = None
    g_sc_ids: Optional[np.ndarray] = None
    g_pc_ids: Optional[np.ndarray] = None

    @staticmethod
    def concat(parts: List["Samples"]) -> "Samples":
        out = Samples(np.concatenate([p.x for p in parts]), np.concatenate([p.t_sc for p in parts]),
                      np.concatenate([p.t_pc for p in parts]), np.concatenate([p.it for p in parts]),
                      sum((p.tot_sc for p in parts), []), sum((p.tot_pc for p in parts), []))
        if all(p.g_us is not None for p in parts):
            # rows point at their iteration in the concatenated per-iteration arrays
            base = np.cumsum([0] + [len(p.g_us) for p in parts[:-1]])
            out.it = np.concatenate([p.it + b for p, b in zip(parts, base)]).astype(np.int32)
            for f in ("s_sc", "s_pc", "g_us", "g_sc_ids", "g_pc_ids"):
                setattr(out, f, np.concatenate([getattr(p, f) for p in parts]))
        return out

    def __len__(self):
        return self.x.shape[0]


def collect(G, max_iter: int = 1 << 20, stream=None, gather_cost: bool = True) -> Samples:
    """Runs the program bound to G (state and frontier already set) to the
    end, probing both scatter modes before every iteration. With gather_cost
    the iterations run with profiling on, and each row's mode costs include
    the modelled gather time of the ids the mode sends."""
    xs, tsc, tpc, its, tot_sc, tot_pc = [], [], [], [], [], []
    ssc, spc, gus, gsi, gpi = [], [], [], [], []
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
                ssc.append(a.astype(np.float32))
                spc.append(b.astype(np.float32))
                gus.append(g_ms * 1e3)
                gsi.append(rec["sc_ids"])
                gpi.append(rec["pc_ids"])
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
    out = Samples(np.concatenate(xs).astype(np.float32), np.concatenate(tsc), np.concatenate(tpc),
                  np.concatenate(its), tot_sc, tot_pc)
    if gather_cost:
        out.s_sc, out.s_pc = np.concatenate(ssc), np.concatenate(spc)
        out.g_us = np.array(gus, np.float64)
        out.g_sc_ids = np.array(gsi, np.float64)
        out.g_pc_ids = np.array(gpi, np.float64)
    return out


def relabel_by_id_kind(data: Samples):
    """Gather cost per id fitted separately for the ids of source-centric
    bins and of partition-centric bins: the measured gather + merge time of
    every training iteration against the two id counts, non-negative least
    squares without intercept. Relabels every row as its scatter time plus
    the ids its mode sends times that mode's fitted cost. Returns (samples,
    us per SC id, us per PC id)."""
    from scipy.optimize import nnls
    A = np.stack([data.g_sc_ids, data.g_pc_ids], axis=1)
    (c_sc, c_pc), _ = nnls(A, data.g_us)
    ea = np.expm1(data.x[:, 1].astype(np.float64))   # E_a ids (source-centric)
    ep = np.expm1(data.x[:, 2].astype(np.float64))   # E^p ids (partition-centric)
    out = Samples(data.x, (data.s_sc + c_sc * ea).astype(np.float32), (data.s_pc + c_pc * ep).astype(np.float32),
                  data.it, data.tot_sc, data.tot_pc, data.s_sc, data.s_pc, data.g_us, data.g_sc_ids,
                  data.g_pc_ids)
    return out, float(c_sc), float(c_pc)


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


def calibrate_offset(mlp, time_runs, offsets=(-1.0, 0.0, 0.5, 1.0, 2.0, 4.0, 8.0, 16.0), stream=None,
                     min_gain: float = 0.01):
    """Moves the network's decision threshold to where whole runs are
    fastest. The per-row labels price each mode with every partition
    scattering in it, so they miss how modes interact in one iteration; the
    threshold corrects the resulting bias. Each candidate offset is added to
    the output bias in turn (Mlp.shift_logit), time_runs() times whole runs
    on training graphs (ms), and the fastest offset stays in the model (the
    one nearer 0 on a tie). An offset must beat no offset by min_gain (a
    fraction of its time), or the network stays as trained: smaller
    differences are timing noise. Returns (offset, {offset: ms})."""
    cur = 0.0
    res = {}
    for d in offsets:
        mlp.shift_logit(float(d) - cur, stream)
        cur = float(d)
        res[float(d)] = float(time_runs())
    if 0.0 not in res:
        mlp.shift_logit(0.0 - cur, stream)
        cur = 0.0
        res[0.0] = float(time_runs())
    best = min(res, key=lambda d: (res[d], abs(d)))
    if res[best] > res[0.0] * (1.0 - min_gain):
        best = 0.0
    mlp.shift_logit(best - cur, stream)
    return best, res


def calibrate_margin(mlp, time_runs, margins=(math.inf, 8.0, 4.0, 2.0, 1.0, 0.5, 0.0), stream=None,
                     min_gain: float = 0.01):
    """Chooses how far the network is trusted: with margin m the selector
    takes the network's mode only where |logit| >= m and Eq. 1's elsewhere
    (m = inf: Eq. 1 alone; m = 0: the network alone). time_runs() times whole
    runs on training graphs (ms) under each candidate; a finite margin must
    beat Eq. 1 alone by min_gain (a fraction of its time), else the margin
    stays inf. Returns (margin, {margin: ms}); the model keeps the margin."""
    res = {}
    for m in margins:
        mlp.set_margin(float(m), stream)
        res[float(m)] = float(time_runs())
    if math.inf not in res:
        mlp.set_margin(math.inf, stream)
        res[math.inf] = float(time_runs())
    best = min(res, key=lambda m: (res[m], -m))
    if res[best] > res[math.inf] * (1.0 - min_gain):
        best = math.inf
    mlp.set_margin(best, stream)
    return best, res


def calibrate_ratio(data: Samples, grid: Optional[np.ndarray] = None) -> float:
    """The bandwidth ratio whose Eq. 1 choices cost least on `data`."""
    if grid is None:
        grid = 2.0 ** np.arange(-4.0, 8.01, 0.25)
    costs = [choice_cost(analytical_choice(data, r), data) for r in grid]
    return float(grid[int(np.argmin(costs))])
