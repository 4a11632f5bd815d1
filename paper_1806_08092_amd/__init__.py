"""Python binding of libgpop.so: argument marshalling only.

Every step of the scatter/gather iteration runs in the library's HIP kernels;
PyTorch provides device memory (the workspace and the caller's arrays) and the
stream. Names follow include/gpop.h. Importing this module does not touch the
GPU; loading the library fails loudly if it has not been built.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpop.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HEADERS = [os.path.join(INCLUDE, "gpop.h"), os.path.join(INCLUDE, "gpop_mlp.h")]

# status codes
OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENOTSUP = range(6)
# programs
BFS_LEVEL, CC_MINLABEL, SSSP_U32, PAGERANK_F32, PPR_F32, CARRY_BFS, BFS_PARENT, NIBBLE_F32 = range(8)
PROGRAMS = {"bfs": BFS_LEVEL, "cc": CC_MINLABEL, "sssp": SSSP_U32, "pagerank": PAGERANK_F32,
            "ppr": PPR_F32, "carry_bfs": CARRY_BFS, "bfs_parent": BFS_PARENT, "nibble": NIBBLE_F32}
COMBINE_LDS, COMBINE_ROUNDS = 0, 1
COMBINES = {"lds": COMBINE_LDS, "rounds": COMBINE_ROUNDS}
PCSTREAM_AUTO, PCSTREAM_OFF, PCSTREAM_ON = 0, 1, 2
PCSTREAMS = {"auto": PCSTREAM_AUTO, "off": PCSTREAM_OFF, "on": PCSTREAM_ON}
SCRES_AUTO, SCRES_PIECE, SCRES_BIN = 0, 1, 2
SCRESERVES = {"auto": SCRES_AUTO, "piece": SCRES_PIECE, "bin": SCRES_BIN}
# selectors
SEL_ANALYTICAL, SEL_FORCE_SC, SEL_FORCE_PC, SEL_LEARNED = range(4)
SELECTORS = {"analytical": SEL_ANALYTICAL, "sc": SEL_FORCE_SC, "pc": SEL_FORCE_PC,
             "learned": SEL_LEARNED}
MODE_NONE, MODE_SC, MODE_PC = 0, 1, 2
KERNELS = ["plan", "scatter_sc", "scatter_pc", "gather", "merge"]
# learned selector (include/gpop_mlp.h)
MLP_IN, MLP_HIDDEN, MLP_PARAMS, MLP_MODEL_BYTES = 12, 64, 5057, 10240
MLP_MAGIC = 0x504C4D47
MLP_NOALLOC_MAX_SAMPLES = 16384


class GpopError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("gpop error %d: %s" % (code, msg))
        self.code = code


class GraphDesc(ctypes.Structure):
    _fields_ = [("num_vertices", ctypes.c_uint32), ("reserved0", ctypes.c_uint32),
                ("num_edges", ctypes.c_uint64), ("offsets", ctypes.c_void_p),
                ("cols", ctypes.c_void_p), ("weights", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("log2_part", ctypes.c_uint32), ("sc_task_log2", ctypes.c_uint32),
                ("gather_task_ids", ctypes.c_uint32), ("combine", ctypes.c_uint32),
                ("pc_stream", ctypes.c_uint32), ("sc_reserve", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 2)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("q", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("workspace_bytes", ctypes.c_uint64), ("reserved", ctypes.c_uint64 * 6)]


class Params(ctypes.Structure):
    _fields_ = [("root", ctypes.c_uint32), ("persist", ctypes.c_uint32),
                ("damping", ctypes.c_float), ("alpha", ctypes.c_float),
                ("epsilon", ctypes.c_float), ("reserved", ctypes.c_uint32 * 3)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("q", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("num_vertices", ctypes.c_uint64), ("num_edges", ctypes.c_uint64),
                ("num_messages", ctypes.c_uint64), ("nonempty_bins", ctypes.c_uint64),
                ("reserved", ctypes.c_uint64 * 6)]


class IterStats(ctypes.Structure):
    _fields_ = [("active_vertices", ctypes.c_uint64), ("active_edges", ctypes.c_uint64),
                ("sc_parts", ctypes.c_uint32), ("pc_parts", ctypes.c_uint32),
                ("sc_msgs", ctypes.c_uint64), ("sc_ids", ctypes.c_uint64),
                ("pc_msgs", ctypes.c_uint64), ("pc_ids", ctypes.c_uint64),
                ("gathered_ids", ctypes.c_uint64), ("gather_parts", ctypes.c_uint32),
                ("split_tasks", ctypes.c_uint32), ("sc_active_vertices", ctypes.c_uint64),
                ("sc_active_edges", ctypes.c_uint64), ("pc_vertices", ctypes.c_uint64),
                ("merged_parts", ctypes.c_uint64), ("learned_fallbacks", ctypes.c_uint32),
                ("gathered_bins", ctypes.c_uint32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_ if f != "reserved"}


TUNE_MAX = 64


class TuneResult(ctypes.Structure):
    _fields_ = [("best", Options), ("best_ms", ctypes.c_float), ("n_tried", ctypes.c_uint32),
                ("run_ms", ctypes.c_float * TUNE_MAX), ("prep_ms", ctypes.c_float * TUNE_MAX)]


_lib = None

_SIGS = {
    "gpop_abi_version": (ctypes.c_int, []),
    "gpop_last_error": (ctypes.c_char_p, []),
    "gpop_plan": (ctypes.c_int, [ctypes.POINTER(GraphDesc), ctypes.POINTER(Options),
                                 ctypes.POINTER(PlanInfo)]),
    "gpop_graph_create": (ctypes.c_int, [ctypes.POINTER(GraphDesc), ctypes.POINTER(Options),
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "gpop_graph_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "gpop_graph_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(GraphInfo)]),
    "gpop_state_init": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Params),
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "gpop_set_frontier": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                         ctypes.c_void_p]),
    "gpop_set_frontier_all": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "gpop_set_selector": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_float,
                                         ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]),
    "gpop_set_isg": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    "gpop_scatter": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "gpop_gather": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "gpop_iterate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "gpop_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                ctypes.c_void_p]),
    "gpop_frontier_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64),
                                          ctypes.c_void_p]),
    "gpop_iterations": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)]),
    "gpop_iter_stats_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(IterStats),
                                            ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                            ctypes.c_void_p]),
    "gpop_modes_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "gpop_check": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "gpop_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "gpop_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p]),
    "gpop_stream_ceiling": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                           ctypes.c_void_p]),
    "gpop_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "gpop_probe_scatter": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_float), ctypes.c_void_p]),
    "gpop_mlp_init": (ctypes.c_int, [ctypes.c_void_p] * 6 + [ctypes.c_uint32, ctypes.c_void_p]),
    "gpop_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "gpop_mlp_grad_workspace": (ctypes.c_size_t, [ctypes.c_uint32]),
    "gpop_mlp_grad": (ctypes.c_int, [ctypes.c_void_p] * 4 + [ctypes.c_uint32] + [ctypes.c_void_p] * 3
                      + [ctypes.c_size_t, ctypes.c_void_p]),
    "gpop_mlp_grad_noalloc": (ctypes.c_int, [ctypes.c_void_p] * 4 + [ctypes.c_uint32] + [ctypes.c_void_p] * 3),
    "gpop_mlp_adam": (ctypes.c_int, [ctypes.c_void_p] * 5 + [ctypes.c_uint32, ctypes.c_float,
                                                             ctypes.c_void_p]),
    "gpop_mlp_train_step": (ctypes.c_int, [ctypes.c_void_p] * 7 + [ctypes.c_uint32, ctypes.c_uint32,
                                                                   ctypes.c_float]
                            + [ctypes.c_void_p] * 3 + [ctypes.c_size_t, ctypes.c_void_p]),
    "gpop_mlp_shift_logit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p]),
    "gpop_mlp_set_margin": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p]),
    "gpop_batch_plan": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64)]),
    "gpop_batch_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "gpop_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "gpop_batch_state_init": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "gpop_batch_set_frontier": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                               ctypes.c_uint32, ctypes.c_void_p]),
    "gpop_batch_set_frontier_all": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p]),
    "gpop_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "gpop_batch_check": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "gpop_autotune_candidates": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p,
                                                ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]),
    "gpop_autotune": (ctypes.c_int, [ctypes.POINTER(GraphDesc), ctypes.c_int, ctypes.POINTER(Params),
                                     ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(TuneResult)]),
}


def lib():
    """Loads libgpop.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgpop.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_symbols() -> Sequence[str]:
    """Function names declared in include/*.h."""
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(gpop_\w+)\s*\(", text, re.M)))


def _check(rc: int):
    if rc != OK:
        raise GpopError(rc, lib().gpop_last_error().decode())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def plan(num_vertices: int, num_edges: int, log2_part: int = 14, sc_task_log2: int = 0,
         gather_task_ids: int = 0, pc_stream="auto") -> PlanInfo:
    d = GraphDesc(num_vertices, 0, num_edges, None, None, None)
    pc_stream = PCSTREAMS[pc_stream] if isinstance(pc_stream, str) else int(pc_stream)
    o = Options(log2_part, sc_task_log2, gather_task_ids, 0, pc_stream)
    out = PlanInfo()
    _check(lib().gpop_plan(ctypes.byref(d), ctypes.byref(o), ctypes.byref(out)))
    return out


class Graph:
    """A preprocessed graph on the GPU. `offsets`, `cols` (int32/uint32) and
    optional `weights` (uint8) are CUDA tensors the caller keeps alive; the
    workspace is allocated here as a torch tensor and owned by this object."""

    def __init__(self, offsets, cols, weights=None, log2_part: int = 14, stream=None,
                 sc_task_log2: int = 0, gather_task_ids: int = 0, combine="lds", pc_stream="auto",
                 sc_reserve="auto"):
        import torch
        self._keep = (offsets, cols, weights)
        n = offsets.numel() - 1
        m = cols.numel()
        self.desc = GraphDesc(n, 0, m, offsets.data_ptr(), cols.data_ptr() if m else 0,
                              None if weights is None else weights.data_ptr())
        combine = COMBINES[combine] if isinstance(combine, str) else int(combine)
        pc_stream = PCSTREAMS[pc_stream] if isinstance(pc_stream, str) else int(pc_stream)
        sc_reserve = SCRESERVES[sc_reserve] if isinstance(sc_reserve, str) else int(sc_reserve)
        self.opts = Options(log2_part, sc_task_log2, gather_task_ids, combine, pc_stream, sc_reserve)
        info = PlanInfo()
        _check(lib().gpop_plan(ctypes.byref(self.desc), ctypes.byref(self.opts), ctypes.byref(info)))
        self.q, self.k = info.q, info.k
        self.workspace = torch.empty(info.workspace_bytes + 256, dtype=torch.uint8, device=offsets.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        h = ctypes.c_void_p()
        _check(lib().gpop_graph_create(ctypes.byref(self.desc), ctypes.byref(self.opts),
                                       ctypes.c_void_p(aligned), info.workspace_bytes,
                                       _stream(stream), ctypes.byref(h)))
        self.h = h
        self.n, self.m = n, m
        self.prog = None
        self.state = None

    def close(self):
        if getattr(self, "h", None):
            lib().gpop_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> GraphInfo:
        out = GraphInfo()
        _check(lib().gpop_graph_get_info(self.h, ctypes.byref(out)))
        return out

    def state_init(self, prog, state, root: int = 0, persist: int = 1, damping: float = 0.85,
                   alpha: float = 0.15, epsilon: float = 1e-6, stream=None):
        prog = PROGRAMS[prog] if isinstance(prog, str) else int(prog)
        p = Params(root, persist, damping, alpha, epsilon)
        _check(lib().gpop_state_init(self.h, prog, ctypes.byref(p), _ptr(state), _stream(stream)))
        self.prog, self.state = prog, state

    def set_frontier(self, vertices, stream=None):
        _check(lib().gpop_set_frontier(self.h, _ptr(vertices), vertices.numel(), _stream(stream)))

    def set_frontier_all(self, stream=None):
        _check(lib().gpop_set_frontier_all(self.h, _stream(stream)))

    def set_selector(self, kind="analytical", bw_ratio: float = 16.0, s_i: int = 4, s_v: int = 4,
                     mlp=None):
        kind = SELECTORS[kind] if isinstance(kind, str) else int(kind)
        _check(lib().gpop_set_selector(self.h, kind, bw_ratio, s_i, s_v, _ptr(mlp)))

    def set_isg(self, classes: int):
        """Interleaved scatter-gather in `classes` colour classes (0: off)."""
        _check(lib().gpop_set_isg(self.h, classes))

    def features(self, stream=None):
        """k x 12 float32 CUDA tensor of the learned selector's features."""
        import torch
        out = torch.empty((self.k, MLP_IN), dtype=torch.float32, device="cuda")
        _check(lib().gpop_features(self.h, _ptr(out), _stream(stream)))
        return out

    def probe_scatter(self, kind, stream=None):
        """Per-partition scatter time (us, numpy float32 [k]) of the current
        frontier in mode `kind` ("sc" or "pc"), and the whole scatter time."""
        import numpy as np
        kind = SELECTORS[kind] if isinstance(kind, str) else int(kind)
        out = np.zeros(self.k, dtype=np.float32)
        tot = ctypes.c_float()
        _check(lib().gpop_probe_scatter(self.h, kind, ctypes.c_void_p(out.ctypes.data),
                                        ctypes.byref(tot), _stream(stream)))
        return out, tot.value

    def scatter(self, stream=None):
        _check(lib().gpop_scatter(self.h, _stream(stream)))

    def gather(self, stream=None):
        _check(lib().gpop_gather(self.h, _stream(stream)))

    def iterate(self, stream=None):
        _check(lib().gpop_iterate(self.h, _stream(stream)))

    def run(self, max_iter: int = 1 << 30, stream=None) -> int:
        it = ctypes.c_uint32()
        _check(lib().gpop_run(self.h, max_iter, ctypes.byref(it), _stream(stream)))
        return it.value

    def frontier_size(self, stream=None) -> int:
        out = ctypes.c_uint64()
        _check(lib().gpop_frontier_size(self.h, ctypes.byref(out), _stream(stream)))
        return out.value

    def iterations(self) -> int:
        out = ctypes.c_uint32()
        _check(lib().gpop_iterations(self.h, ctypes.byref(out)))
        return out.value

    def iter_stats(self, stream=None):
        cap = 4096
        buf = (IterStats * cap)()
        n = ctypes.c_uint32()
        _check(lib().gpop_iter_stats_read(self.h, buf, cap, ctypes.byref(n), _stream(stream)))
        return [buf[i].as_dict() for i in range(n.value)]

    def modes(self, stream=None):
        import numpy as np
        out = np.zeros(self.k, dtype=np.uint8)
        _check(lib().gpop_modes_read(self.h, ctypes.c_void_p(out.ctypes.data), _stream(stream)))
        return out

    def check(self, stream=None):
        _check(lib().gpop_check(self.h, _stream(stream)))

    def profile_enable(self, on: bool = True):
        _check(lib().gpop_profile_enable(self.h, 1 if on else 0))

    def profile_read(self, stream=None):
        nk = len(KERNELS)
        ms = (ctypes.c_double * nk)()
        n = (ctypes.c_uint64 * nk)()
        _check(lib().gpop_profile_read(self.h, ms, n, _stream(stream)))
        return {KERNELS[i]: (ms[i], int(n[i])) for i in range(nk)}


def autotune_candidates(prog, num_vertices: int, num_edges: int):
    """Default tuning candidates (list of dicts) for a program and graph size."""
    prog = PROGRAMS[prog] if isinstance(prog, str) else int(prog)
    buf = (Options * TUNE_MAX)()
    n = ctypes.c_uint32()
    _check(lib().gpop_autotune_candidates(prog, num_vertices, num_edges, buf, TUNE_MAX, ctypes.byref(n)))
    return [{"log2_part": buf[i].log2_part, "sc_task_log2": buf[i].sc_task_log2,
             "gather_task_ids": buf[i].gather_task_ids} for i in range(n.value)]


def autotune(offsets, cols, weights, prog, root: int = 0, persist: int = 1, damping: float = 0.85,
             alpha: float = 0.15, frontier=None, max_iter: int = 3, reps: int = 2, candidates=None,
             stream=None, epsilon: float = 1e-6):
    """Times the candidates (default: autotune_candidates) through
    gpop_autotune and returns (best options dict, per-candidate list of
    (options, run_ms, prep_ms))."""
    import torch
    prog_id = PROGRAMS[prog] if isinstance(prog, str) else int(prog)
    n, m = offsets.numel() - 1, cols.numel()
    cands = candidates or autotune_candidates(prog_id, n, m)
    carr = (Options * len(cands))(*[Options(c["log2_part"], c["sc_task_log2"], c["gather_task_ids"])
                                    for c in cands])
    desc = GraphDesc(n, 0, m, offsets.data_ptr(), cols.data_ptr() if m else 0,
                     None if weights is None else weights.data_ptr())
    need = 0
    for i in range(len(cands)):
        info = PlanInfo()
        if lib().gpop_plan(ctypes.byref(desc), ctypes.byref(carr[i]), ctypes.byref(info)) == OK:
            need = max(need, info.workspace_bytes)
    ws = torch.empty(need + 256, dtype=torch.uint8, device=offsets.device)
    aligned = (ws.data_ptr() + 255) & ~255
    state = torch.empty(n, dtype=torch.int32, device=offsets.device)
    p = Params(root, persist, damping, alpha, epsilon)
    res = TuneResult()
    _check(lib().gpop_autotune(ctypes.byref(desc), prog_id, ctypes.byref(p), _ptr(frontier),
                               0 if frontier is None else frontier.numel(), max_iter, reps, carr, len(cands),
                               ctypes.c_void_p(aligned), need, _ptr(state), _stream(stream), ctypes.byref(res)))
    best = {"log2_part": res.best.log2_part, "sc_task_log2": res.best.sc_task_log2,
            "gather_task_ids": res.best.gather_task_ids}
    return best, [(cands[i], res.run_ms[i], res.prep_ms[i]) for i in range(len(cands))]


BATCH_EAGER = 1


class Batch:
    """Many runs of one program launched together (include/gpop.h, batches):
    `graphs` is a list of Graph objects (repeat one for several seeds). The
    workspace is a torch tensor owned by this object."""

    def __init__(self, graphs, stream=None):
        import torch
        self.graphs = list(graphs)
        self.n = len(self.graphs)
        self._harr = (ctypes.c_void_p * self.n)(*[g.h.value for g in self.graphs])
        need = ctypes.c_uint64()
        _check(lib().gpop_batch_plan(self._harr, self.n, ctypes.byref(need)))
        self.workspace = torch.empty(need.value + 256, dtype=torch.uint8, device="cuda")
        aligned = (self.workspace.data_ptr() + 255) & ~255
        h = ctypes.c_void_p()
        _check(lib().gpop_batch_create(self._harr, self.n, ctypes.c_void_p(aligned), need.value,
                                       _stream(stream), ctypes.byref(h)))
        self.h = h
        self.states = None

    def close(self):
        if getattr(self, "h", None):
            lib().gpop_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state_init(self, prog, states, roots=None, persist: int = 1, damping: float = 0.85,
                   alpha: float = 0.15, epsilon: float = 1e-6, stream=None):
        prog = PROGRAMS[prog] if isinstance(prog, str) else int(prog)
        roots = [0] * self.n if roots is None else list(roots)
        prm = (Params * self.n)(*[Params(int(r), persist, damping, alpha, epsilon) for r in roots])
        ptrs = (ctypes.c_void_p * self.n)(*[s.data_ptr() for s in states])
        _check(lib().gpop_batch_state_init(self.h, prog, prm, ptrs, _stream(stream)))
        self.states = list(states)

    def set_frontier(self, run: int, vertices, stream=None):
        _check(lib().gpop_batch_set_frontier(self.h, run, _ptr(vertices), vertices.numel(), _stream(stream)))

    def set_frontier_all(self, run: int, stream=None):
        _check(lib().gpop_batch_set_frontier_all(self.h, run, _stream(stream)))

    def run(self, max_iter: int = 1 << 30, eager: bool = False, stream=None):
        iters = (ctypes.c_uint32 * self.n)()
        _check(lib().gpop_batch_run(self.h, max_iter, BATCH_EAGER if eager else 0, iters, _stream(stream)))
        return list(iters)

    def check(self, stream=None):
        _check(lib().gpop_batch_check(self.h, _stream(stream)))


class Mlp:
    """Device buffers of one learned-selector model (include/gpop_mlp.h):
    the model the selector reads, f32 masters, Adam moments, the last
    gradient and loss. Every computation runs in the library's kernels."""

    def __init__(self):
        import torch
        self.model = torch.zeros(MLP_MODEL_BYTES // 4, dtype=torch.int32, device="cuda")
        self.master = torch.zeros(MLP_PARAMS, dtype=torch.float32, device="cuda")
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.grad = torch.zeros_like(self.master)
        self.loss = torch.zeros(2, dtype=torch.float32, device="cuda")
        self.ws = None
        self.step = 0

    def init(self, init_params, x, stream=None):
        """init_params: f32 [5057] CUDA tensor; x: n x 12 training features."""
        _check(lib().gpop_mlp_init(_ptr(self.model), _ptr(self.master), _ptr(self.m), _ptr(self.v),
                                   _ptr(init_params), _ptr(x), x.shape[0], _stream(stream)))
        self.step = 0

    def forward(self, x, stream=None):
        import torch
        out = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
        _check(lib().gpop_mlp_forward(_ptr(self.model), _ptr(x), x.shape[0], _ptr(out), _stream(stream)))
        return out

    def _workspace(self, n):
        import torch
        need = lib().gpop_mlp_grad_workspace(n)
        if self.ws is None or self.ws.numel() * 4 < need:
            self.ws = torch.empty((need + 3) // 4, dtype=torch.float32, device="cuda")
        return self.ws

    def compute_grad(self, x, t_sc, t_pc, stream=None):
        ws = self._workspace(x.shape[0])
        _check(lib().gpop_mlp_grad(_ptr(self.model), _ptr(x), _ptr(t_sc), _ptr(t_pc), x.shape[0],
                                   _ptr(self.grad), _ptr(self.loss), _ptr(ws), ws.numel() * 4,
                                   _stream(stream)))
        return self.grad

    def compute_grad_noalloc(self, x, t_sc, t_pc, grad=None, loss=None, stream=None):
        """gpop_mlp_grad_noalloc: the gradient without a workspace (the
        library's fixed per-GPU scratch array); writes `grad` / `loss`
        (default: this object's buffers)."""
        grad = self.grad if grad is None else grad
        loss = self.loss if loss is None else loss
        _check(lib().gpop_mlp_grad_noalloc(_ptr(self.model), _ptr(x), _ptr(t_sc), _ptr(t_pc), x.shape[0],
                                           _ptr(grad), _ptr(loss), _stream(stream)))
        return grad

    def adam(self, lr=1e-3, stream=None):
        self.step += 1
        _check(lib().gpop_mlp_adam(_ptr(self.model), _ptr(self.master), _ptr(self.m), _ptr(self.v),
                                   _ptr(self.grad), self.step, lr, _stream(stream)))

    def set_margin(self, margin, stream=None):
        """Confidence margin of the learned selector (gpop_mlp_set_margin):
        partitions with |logit| below it keep Eq. 1's mode."""
        _check(lib().gpop_mlp_set_margin(_ptr(self.model), ctypes.c_float(margin), _stream(stream)))

    def shift_logit(self, delta, stream=None):
        """Adds delta to the output bias (gpop_mlp_shift_logit)."""
        _check(lib().gpop_mlp_shift_logit(_ptr(self.model), _ptr(self.master), ctypes.c_float(delta),
                                          _stream(stream)))

    def train_step(self, x, t_sc, t_pc, lr=1e-3, stream=None):
        ws = self._workspace(x.shape[0])
        self.step += 1
        _check(lib().gpop_mlp_train_step(_ptr(self.model), _ptr(self.master), _ptr(self.m), _ptr(self.v),
                                         _ptr(x), _ptr(t_sc), _ptr(t_pc), x.shape[0], self.step, lr,
                                         _ptr(self.grad), _ptr(self.loss), _ptr(ws), ws.numel() * 4,
                                         _stream(stream)))


STREAM_READ, STREAM_COPY, STREAM_WIDEN, STREAM_SEGMENTS = 0, 1, 2, 3


def stream_ceiling(mix: int, src, dst, nbytes: int, stream=None):
    """One launch of the library's reference stream for access mix `mix`
    over `nbytes` bytes of the device tensor `src` (gpop_stream_ceiling)."""
    _check(lib().gpop_stream_ceiling(int(mix), _ptr(src), _ptr(dst), int(nbytes), _stream(stream)))


def upload_csr(g, device="cuda"):
    """Copies a host CSR (numpy offsets/cols[/weights]) to device tensors."""
    import numpy as np
    import torch
    off = torch.from_numpy(np.ascontiguousarray(g.offsets).view(np.int32)).to(device)
    cols = torch.from_numpy(np.ascontiguousarray(g.cols).view(np.int32)).to(device)
    w = None
    if getattr(g, "weights", None) is not None:
        w = torch.from_numpy(np.ascontiguousarray(g.weights)).to(device)
    return off, cols, w
