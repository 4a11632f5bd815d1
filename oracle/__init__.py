"""ORACLE -- test infrastructure, not part of the product path.

Plain, slow, obviously-correct CPU implementations of what the
partition-centric scatter/gather path computes. Only ``tests/``, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may
import this package. It shares no code with the GPU library (no kernels,
headers, tables or helpers); the only common dependency is the seeded input
generator in ``graphgen``, which holds none of the method's arithmetic.

Contents
  * textbook results (``oracle.c`` via ctypes): BFS levels, min-label
    connected components, integer-weight SSSP, FP64 PageRank and
    personalised PageRank;
  * ``nibble``: FP64 Parallel Nibble with the distance of every frontier
    decision from its threshold (``oracle.c``);
  * ``gpop_ref``: the GPOP iteration itself (scatter in source- or
    partition-centric mode, reInit, gather, filter) and the analytical mode
    model, written out in pure Python for tiny graphs;
  * ``mlp_ref``: FP64 forward/backward of the learned mode selector's MLP.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

INF32 = 0xFFFFFFFF


def build(force: bool = False) -> str:
    """Compile liboracle.so (plain single-threaded C, gcc -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        u32, i32, dbl, vp = ctypes.c_uint32, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        for name, args in [
            ("oracle_bfs_levels", [u32, vp, vp, u32, vp]),
            ("oracle_bfs_parents", [u32, vp, vp, u32, vp]),
            ("oracle_cc_minlabel", [u32, vp, vp, vp]),
            ("oracle_sssp", [u32, vp, vp, vp, u32, vp]),
            ("oracle_pagerank", [u32, vp, vp, dbl, u32, vp]),
            ("oracle_ppr", [u32, vp, vp, dbl, u32, u32, vp]),
            ("oracle_nibble", [u32, vp, vp, u32, dbl, u32, dbl, vp, vp, vp, vp, vp]),
        ]:
            fn = getattr(_lib, name)
            fn.restype = i32
            fn.argtypes = args
    return _lib


def _p(a):
    return 0 if a is None else np.ascontiguousarray(a).ctypes.data


def _csr(g):
    off = np.ascontiguousarray(g.offsets, np.uint32)
    cols = np.ascontiguousarray(g.cols, np.uint32)
    if cols.size == 0:
        cols = np.zeros(1, np.uint32)
    return off, cols


def bfs_levels(g, root: int) -> np.ndarray:
    off, cols = _csr(g)
    out = np.empty(g.n, np.uint32)
    if _L().oracle_bfs_levels(g.n, _p(off), _p(cols), root, _p(out)) != 0:
        raise ValueError("bad root or allocation failure")
    return out


def bfs_parents(g, root: int) -> np.ndarray:
    """Parent of each vertex in the BFS tree of root (least-id in-neighbour one
    level closer; root: itself; unreached: 0xFFFFFFFF)."""
    off, cols = _csr(g)
    out = np.empty(g.n, np.uint32)
    if _L().oracle_bfs_parents(g.n, _p(off), _p(cols), root, _p(out)) != 0:
        raise ValueError("bad root or allocation failure")
    return out


def cc_minlabel(g) -> np.ndarray:
    off, cols = _csr(g)
    out = np.empty(g.n, np.uint32)
    if _L().oracle_cc_minlabel(g.n, _p(off), _p(cols), _p(out)) != 0:
        raise MemoryError
    return out


def sssp(g, root: int, weights=None) -> np.ndarray:
    off, cols = _csr(g)
    w = g.weights if weights is None else weights
    w = None if w is None else np.ascontiguousarray(w, np.uint8)
    if w is not None and w.size == 0:
        w = np.zeros(1, np.uint8)
    out = np.empty(g.n, np.uint32)
    rc = _L().oracle_sssp(g.n, _p(off), _p(cols), _p(w), root, _p(out))
    if rc == -2:
        raise OverflowError("distance does not fit uint32")
    if rc != 0:
        raise ValueError("bad root or allocation failure")
    return out


def pagerank(g, damping: float = 0.85, iters: int = 10) -> np.ndarray:
    off, cols = _csr(g)
    out = np.empty(g.n, np.float64)
    if _L().oracle_pagerank(g.n, _p(off), _p(cols), damping, iters, _p(out)) != 0:
        raise MemoryError
    return out


def ppr(g, seed: int, alpha: float = 0.15, iters: int = 20) -> np.ndarray:
    off, cols = _csr(g)
    out = np.empty(g.n, np.float64)
    if _L().oracle_ppr(g.n, _p(off), _p(cols), alpha, iters, seed, _p(out)) != 0:
        raise ValueError("bad seed or allocation failure")
    return out


class NibbleResult:
    """FP64 Parallel Nibble: ``pr`` (float64 [n]), ``fsize`` (frontier size
    after each iteration), ``iters``, ``min_margin`` (least relative distance
    of a decisive threshold test from its threshold) and ``near`` (decisive
    tests closer than the requested delta)."""

    def __init__(self, pr, fsize, iters, min_margin, near):
        self.pr, self.fsize, self.iters, self.min_margin, self.near = pr, fsize, iters, min_margin, near


def nibble(g, seed: int, eps: float, max_iter: int = 20, delta: float = 1e-4) -> NibbleResult:
    off, cols = _csr(g)
    pr = np.empty(g.n, np.float64)
    fs = np.zeros(max(1, max_iter), np.uint64)
    it = ctypes.c_uint32()
    mm = ctypes.c_double()
    near = ctypes.c_uint64()
    if _L().oracle_nibble(g.n, _p(off), _p(cols), seed, eps, max_iter, delta, _p(pr), _p(fs),
                          ctypes.addressof(it), ctypes.addressof(mm), ctypes.addressof(near)) != 0:
        raise ValueError("bad seed or allocation failure")
    return NibbleResult(pr, fs[:it.value].astype(np.int64), it.value, mm.value, near.value)
