"""Seeded synthetic graph inputs shared by the oracle and the GPU path.

Input preparation only: RMAT / Erdos-Renyi edge lists, CSR with sorted rows,
symmetrisation, uint8 edge weights and source selection. Nothing here performs
any step of the partition-centric scatter/gather method.

The evaluation section's synthetic graphs are RMAT graphs "with default
settings" and degree 16 (evaluation section, datasets paragraph and Table 2);
the workloads below use a=0.57, b=0.19, c=0.19, d=0.05 with edge factor 16,
and integer SSSP weights uniform on [1, 255].
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")

#: Base seed of every named workload; each input adds a fixed offset.
BASE_SEED = 1806080920

RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = False) -> str:
    """Compile libgraphgen.so with gcc (OpenMP). Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        u64, u32, i32, dbl, vp = (ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_void_p)
        _lib.gg_draw.restype = u64
        _lib.gg_draw.argtypes = [u64, u64]
        _lib.gg_rmat_edges.argtypes = [i32, u64, dbl, dbl, dbl, u64, vp, vp]
        _lib.gg_er_edges.argtypes = [u64, u64, u64, vp, vp]
        _lib.gg_symmetrize.argtypes = [u64, vp, vp, vp, vp]
        _lib.gg_build_csr.restype = i32
        _lib.gg_build_csr.argtypes = [u64, u64, vp, vp, vp, vp]
        _lib.gg_weights.argtypes = [u64, u64, u32, vp]
        _lib.gg_sources.restype = u32
        _lib.gg_sources.argtypes = [u64, vp, u64, u32, vp]
    return _lib


def _p(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def draw(seed: int, counter: int) -> int:
    """SplitMix64 output for (seed, counter)."""
    return int(_L().gg_draw(seed & (2**64 - 1), counter))


def rmat_edges(scale: int, m: int, seed: int, abc=RMAT_ABC):
    src = np.empty(m, dtype=np.uint32)
    dst = np.empty(m, dtype=np.uint32)
    a, b, c = abc
    _L().gg_rmat_edges(scale, m, a, b, c, seed, _p(src), _p(dst))
    return src, dst


def er_edges(n: int, m: int, seed: int):
    src = np.empty(m, dtype=np.uint32)
    dst = np.empty(m, dtype=np.uint32)
    _L().gg_er_edges(n, m, seed, _p(src), _p(dst))
    return src, dst


def symmetrize(src: np.ndarray, dst: np.ndarray):
    m = src.shape[0]
    osrc = np.empty(2 * m, dtype=np.uint32)
    odst = np.empty(2 * m, dtype=np.uint32)
    _L().gg_symmetrize(m, _p(np.ascontiguousarray(src, np.uint32)),
                       _p(np.ascontiguousarray(dst, np.uint32)), _p(osrc), _p(odst))
    return osrc, odst


def build_csr(n: int, src: np.ndarray, dst: np.ndarray):
    src = np.ascontiguousarray(src, np.uint32)
    dst = np.ascontiguousarray(dst, np.uint32)
    m = src.shape[0]
    offsets = np.empty(n + 1, dtype=np.uint32)
    cols = np.empty(max(m, 1), dtype=np.uint32)[:m]
    if _L().gg_build_csr(n, m, _p(src), _p(dst), _p(offsets), _p(cols) if m else 0) != 0:
        raise ValueError("edge endpoint out of range or too many edges")
    return offsets, cols


def edge_weights(m: int, seed: int, span: int = 255) -> np.ndarray:
    w = np.empty(max(m, 1), dtype=np.uint8)[:m]
    if m:
        _L().gg_weights(m, seed, span, _p(w))
    return w


def pick_sources(offsets: np.ndarray, seed: int, count: int) -> np.ndarray:
    out = np.empty(max(count, 1), dtype=np.uint32)
    n = offsets.shape[0] - 1
    got = _L().gg_sources(n, _p(np.ascontiguousarray(offsets, np.uint32)), seed, count, _p(out))
    return out[:got].copy()


@dataclass
class Graph:
    """A CSR graph: offsets u32[n+1], cols u32[m] (rows ascending), optional u8 weights."""
    n: int
    offsets: np.ndarray
    cols: np.ndarray
    weights: Optional[np.ndarray] = None
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.cols.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets.astype(np.int64))


def from_edges(n: int, src, dst, weights_seed: Optional[int] = None, name: str = "") -> Graph:
    off, cols = build_csr(n, np.asarray(src, np.uint32), np.asarray(dst, np.uint32))
    w = edge_weights(cols.shape[0], weights_seed) if weights_seed is not None else None
    return Graph(n, off, cols, w, name)


def rmat_graph(scale: int, edge_factor: int = 16, seed: int = BASE_SEED, abc=RMAT_ABC,
               symmetric: bool = False, weights_seed: Optional[int] = None) -> Graph:
    n = 1 << scale
    src, dst = rmat_edges(scale, edge_factor * n, seed, abc)
    if symmetric:
        src, dst = symmetrize(src, dst)
    name = "rmat%d_ef%d%s" % (scale, edge_factor, "_sym" if symmetric else "")
    return from_edges(n, src, dst, weights_seed, name)


def er_graph(n: int, m: int, seed: int, weights_seed: Optional[int] = None) -> Graph:
    src, dst = er_edges(n, m, seed)
    return from_edges(n, src, dst, weights_seed, "er_n%d_m%d" % (n, m))


def permute_vertices(g: Graph, seed: int):
    """The same graph with vertex ids relabelled by a seeded uniform random
    permutation (vertex v becomes perm[v]); returns (graph, perm). It
    destroys the locality of RMAT's id order: nearly every edge then joins
    two different index-range partitions. Unweighted graphs only."""
    if g.weights is not None:
        raise ValueError("permute_vertices takes unweighted graphs")
    perm = np.random.Generator(np.random.PCG64(seed)).permutation(g.n).astype(np.uint32)
    src = np.repeat(np.arange(g.n, dtype=np.uint32), g.degrees())
    off, cols = build_csr(g.n, perm[src], perm[g.cols])
    return Graph(g.n, off, cols, None, g.name + "_perm"), perm


def inter_partition_fraction(g: Graph, log2_part: int) -> float:
    """Fraction of CSR entries whose endpoints lie in different partitions of
    2^log2_part consecutive ids."""
    src = np.repeat(np.arange(g.n, dtype=np.uint32), g.degrees())
    return float(np.count_nonzero((src >> log2_part) != (g.cols >> log2_part))) / max(g.m, 1)


# Named workloads (seed offsets fixed so every run sees the same bytes).
def workload_pagerank_rmat16() -> Graph:
    """PageRank input: directed RMAT scale 16, edge factor 16 (1,048,576 edges)."""
    return rmat_graph(16, 16, BASE_SEED + 1)


def workload_bfs_cc_rmat22() -> Graph:
    """BFS / CC input: RMAT scale 22, edge factor 16, symmetrised (134,217,728 entries)."""
    return rmat_graph(22, 16, BASE_SEED + 2, symmetric=True)


def workload_sssp_rmat24() -> Graph:
    """SSSP input: directed RMAT scale 24, edge factor 16, weights U{1..255}."""
    return rmat_graph(24, 16, BASE_SEED + 3, weights_seed=BASE_SEED + 4)


def workload_sssp_er24() -> Graph:
    """SSSP input, non-skewed: G(2^24, 16 * 2^24), weights U{1..255}."""
    n = 1 << 24
    return er_graph(n, 16 * n, BASE_SEED + 5, weights_seed=BASE_SEED + 4)


SOURCE_SEED = BASE_SEED + 6


def mlp_init_params(seed: int) -> np.ndarray:
    """Seeded He-normal initial weights of the selector network (12 -> 64 ->
    64 -> 1), biases zero, in the parameter order W1[64][12], b1[64],
    W2[64][64], b2[64], w3[64], b3. float32 [5057]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w1 = rng.standard_normal(64 * 12) * np.sqrt(2.0 / 12)
    w2 = rng.standard_normal(64 * 64) * np.sqrt(2.0 / 64)
    w3 = rng.standard_normal(64) * np.sqrt(2.0 / 64)
    z = np.zeros(64)
    return np.concatenate([w1, z, w2, z, w3, [0.0]]).astype(np.float32)
