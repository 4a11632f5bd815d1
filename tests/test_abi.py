"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and rejects malformed arguments in host-only calls."""
import ctypes

import pytest

import paper_1806_08092_amd as gp


def test_library_exports_header_symbols():
    L = gp.lib()
    names = gp.header_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert L.gpop_abi_version() == 1


def test_plan_sizes():
    info = gp.plan(1 << 22, 1 << 27, 14)
    assert info.q == 16384 and info.k == 256
    # workspace grows linearly with E (ids, weights and message slots per
    # edge: the partition-centric messages and, separately, the
    # source-centric ones, which are sized for M <= E)
    a = gp.plan(1 << 20, 1 << 24, 14).workspace_bytes
    b = gp.plan(1 << 20, 1 << 25, 14).workspace_bytes
    assert 9 * (1 << 24) < b - a < 24 * (1 << 24)


@pytest.mark.parametrize("n,m,lp", [(0, 10, 14), (100, 2**32 - 1, 14), (100, 10, 7), (100, 10, 16),
                                    (1 << 25, 10, 12)])
def test_plan_rejects(n, m, lp):
    with pytest.raises(gp.GpopError) as e:
        gp.plan(n, m, lp)
    assert e.value.code == gp.EINVAL


def test_null_arguments_rejected():
    L = gp.lib()
    assert L.gpop_plan(None, None, None) == gp.EINVAL
    assert L.gpop_graph_destroy(None) == gp.OK
    assert L.gpop_scatter(None, None) == gp.EINVAL
    assert L.gpop_gather(None, None) == gp.EINVAL
    assert L.gpop_run(None, 1, None, None) == gp.EINVAL
    assert b"NULL" in L.gpop_last_error()


def test_create_rejects_unaligned_workspace_without_touching_device():
    d = gp.GraphDesc(100, 0, 10, 0x1000, 0x2000, None)
    o = gp.Options(10)
    h = ctypes.c_void_p()
    rc = gp.lib().gpop_graph_create(ctypes.byref(d), ctypes.byref(o), ctypes.c_void_p(0x1001),
                                    1 << 30, None, ctypes.byref(h))
    assert rc == gp.EINVAL and not h.value
    rc = gp.lib().gpop_graph_create(ctypes.byref(d), ctypes.byref(o), ctypes.c_void_p(0x1000),
                                    16, None, ctypes.byref(h))
    assert rc == gp.ENOMEM


def test_selector_entry_points_reject_bad_arguments_on_host():
    L = gp.lib()
    fake = ctypes.c_void_p(256)  # never dereferenced: each call fails before any device work
    assert L.gpop_features(None, fake, None) == gp.EINVAL
    assert L.gpop_probe_scatter(None, gp.SEL_FORCE_SC, None, None, None) == gp.EINVAL
    assert L.gpop_mlp_init(None, fake, fake, fake, fake, fake, 10, None) == gp.EINVAL
    assert L.gpop_mlp_init(fake, fake, fake, fake, fake, fake, 0, None) == gp.EINVAL
    assert L.gpop_mlp_forward(None, fake, 1, fake, None) == gp.EINVAL
    assert L.gpop_mlp_grad(fake, fake, fake, fake, 0, fake, None, fake, 1 << 20, None) == gp.EINVAL
    assert L.gpop_mlp_grad(fake, fake, fake, fake, 100, fake, None, fake, 16, None) == gp.ENOMEM
    assert L.gpop_mlp_adam(fake, fake, fake, fake, fake, 0, 1e-3, None) == gp.EINVAL
    assert L.gpop_mlp_adam(fake, fake, fake, fake, fake, 1, -1.0, None) == gp.EINVAL
    assert b"Adam" in L.gpop_last_error() or b"lr" in L.gpop_last_error()
    assert L.gpop_mlp_shift_logit(None, fake, 1.0, None) == gp.EINVAL
    assert L.gpop_mlp_shift_logit(fake, None, 1.0, None) == gp.EINVAL
    assert L.gpop_mlp_shift_logit(fake, fake, float("nan"), None) == gp.EINVAL
    assert L.gpop_mlp_shift_logit(fake, fake, float("inf"), None) == gp.EINVAL


def test_mlp_workspace_size():
    L = gp.lib()
    # one partial row (5057 gradients + loss + weight sum) per 64 samples
    assert L.gpop_mlp_grad_workspace(1) == 5059 * 4
    assert L.gpop_mlp_grad_workspace(64) == 5059 * 4
    assert L.gpop_mlp_grad_workspace(65) == 2 * 5059 * 4


def test_batch_entry_points_reject_bad_arguments_on_host():
    L = gp.lib()
    n = ctypes.c_uint64()
    assert L.gpop_batch_plan(None, 0, ctypes.byref(n)) == gp.EINVAL
    arr = (ctypes.c_void_p * 2)(None, None)
    assert L.gpop_batch_plan(arr, 2, ctypes.byref(n)) == gp.EINVAL
    assert L.gpop_batch_destroy(None) == gp.OK
    assert L.gpop_batch_run(None, 10, 0, None, None) == gp.EINVAL
    assert L.gpop_batch_state_init(None, 0, None, None, None) == gp.EINVAL
    assert L.gpop_batch_set_frontier(None, 0, None, 0, None) == gp.EINVAL
    assert L.gpop_batch_check(None, None) == gp.EINVAL


def test_autotune_candidates():
    # PageRank's 64-bit accumulators rule out 2^15-vertex partitions
    pr = gp.autotune_candidates("pagerank", 1 << 22, 1 << 27)
    bfs = gp.autotune_candidates("bfs", 1 << 22, 1 << 27)
    assert {c["log2_part"] for c in pr} == {12, 13, 14}
    assert {c["log2_part"] for c in bfs} == {12, 13, 14, 15}
    assert len(bfs) == 16 and len(pr) == 12
    # a small graph needs no partition larger than itself
    small = gp.autotune_candidates("bfs", 3000, 20000)
    assert {c["log2_part"] for c in small} == {12}
    L = gp.lib()
    n = ctypes.c_uint32()
    assert L.gpop_autotune_candidates(0, 100, 100, None, 0, ctypes.byref(n)) == gp.EINVAL
    assert L.gpop_autotune(None, 0, None, None, 0, 1, 1, None, 0, None, 0, None, None, None) == gp.EINVAL


def test_plan_rejects_unknown_combine():
    d = gp.GraphDesc(1000, 0, 5000, None, None, None)
    info = gp.PlanInfo()
    L = gp.lib()
    assert L.gpop_plan(ctypes.byref(d), ctypes.byref(gp.Options(10, 0, 0, 2)), ctypes.byref(info)) == gp.EINVAL
    assert L.gpop_plan(ctypes.byref(d), ctypes.byref(gp.Options(10, 0, 0, 1)), ctypes.byref(info)) == gp.OK


def test_plan_pc_stream_modes():
    """pc_stream selects where gather reads partition-centric ids: unknown
    modes are rejected, and without column streams the workspace is smaller
    (the streams hold a copy of every static id, its weight, and per 256-id
    chunk a bin-start bitmap and table)."""
    d = gp.GraphDesc(1 << 20, 0, 1 << 24, None, None, None)
    L = gp.lib()
    info = gp.PlanInfo()
    assert L.gpop_plan(ctypes.byref(d), ctypes.byref(gp.Options(14, 0, 0, 0, 3)), ctypes.byref(info)) == gp.EINVAL
    ws = {m: gp.plan(1 << 20, 1 << 24, 14, pc_stream=m).workspace_bytes for m in ("auto", "off", "on")}
    assert ws["auto"] == ws["on"]
    assert ws["auto"] - ws["off"] >= (1 << 24) * 3  # 2-byte ids + 1-byte weights of every edge


def test_plan_sc_reserve_modes():
    """sc_reserve picks how source-centric tasks reserve bin slots; unknown
    modes and nonzero reserved words are rejected, known ones plan."""
    d = gp.GraphDesc(1 << 20, 0, 1 << 24, None, None, None)
    L = gp.lib()
    info = gp.PlanInfo()
    for m in (gp.SCRES_AUTO, gp.SCRES_PIECE, gp.SCRES_BIN):
        assert L.gpop_plan(ctypes.byref(d), ctypes.byref(gp.Options(14, 0, 0, 0, 0, m)), ctypes.byref(info)) == gp.OK
    assert L.gpop_plan(ctypes.byref(d), ctypes.byref(gp.Options(14, 0, 0, 0, 0, 3)), ctypes.byref(info)) == gp.EINVAL
    o = gp.Options(14, 0, 0, 0, 0, 0)
    o.reserved[1] = 1
    assert L.gpop_plan(ctypes.byref(d), ctypes.byref(o), ctypes.byref(info)) == gp.EINVAL


def test_stream_ceiling_rejects_bad_arguments_on_host():
    # every one of these is refused before anything is launched
    L = gp.lib()
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20)  # never dereferenced
    assert L.gpop_stream_ceiling(5, a, b, 1 << 20, None) == gp.EINVAL  # unknown mix
    assert L.gpop_stream_ceiling(-1, a, b, 1 << 20, None) == gp.EINVAL
    assert L.gpop_stream_ceiling(gp.STREAM_READ, None, b, 1 << 20, None) == gp.EINVAL
    assert L.gpop_stream_ceiling(gp.STREAM_COPY, a, None, 1 << 20, None) == gp.EINVAL
    assert L.gpop_stream_ceiling(gp.STREAM_COPY, ctypes.c_void_p((1 << 20) + 8), b, 1 << 20, None) == gp.EINVAL
    assert L.gpop_stream_ceiling(gp.STREAM_COPY, a, ctypes.c_void_p((2 << 20) + 4), 1 << 20, None) == gp.EINVAL
    assert L.gpop_stream_ceiling(gp.STREAM_COPY, a, b, 0, None) == gp.EINVAL
    assert L.gpop_stream_ceiling(gp.STREAM_COPY, a, b, 24, None) == gp.EINVAL  # not a multiple of 16
    assert L.gpop_stream_ceiling(gp.STREAM_WIDEN, a, b, 20, None) == gp.EINVAL  # not a multiple of 8
    assert L.gpop_stream_ceiling(gp.STREAM_READ, a, b, 1 << 40, None) == gp.EINVAL
    assert L.gpop_stream_ceiling(gp.STREAM_SEGMENTS, a, b, 3 * 512, None) == gp.EINVAL  # 3 segments
    assert L.gpop_stream_ceiling(gp.STREAM_SEGMENTS, a, b, 256, None) == gp.EINVAL  # half a segment
    assert L.gpop_stream_ceiling(4, a, b, 1 << 20, None) == gp.EINVAL
