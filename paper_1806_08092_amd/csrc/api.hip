// C ABI of the engine: argument checks, workspace carving, preprocessing and
// the iteration driver. No device memory is allocated here; every buffer is
// a slice of the caller's workspace.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <queue>
#include <cmath>
#include <string>
#include <vector>

#include "launch.h"

using namespace gpop;

namespace {

constexpr uint32_t kPcTaskMin = 32768;  // least message slots per partition-centric task

thread_local std::string g_err;

}  // namespace

namespace gpop {

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(GPOP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace gpop

namespace {


struct Pending {
    int kid;
    hipEvent_t a, b;
};

// Records a fixed number of iterations of one or more runs as a HIP graph
// and replays it until every run has finished or paused. Profiling records
// an event pair around each kernel group of each iteration.
struct Runner {
    hipStream_t cap = nullptr;  // used only to record
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int prog = -1;
    bool prof = false;
    bool learned = false;
    uint32_t chunk = 4;
    std::vector<hipEvent_t> ev;  // 2 * GPOP_KERNEL_COUNT per recorded iteration

    void drop() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        prog = -1;
    }
    ~Runner() {
        drop();
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

}  // namespace

struct gpop_graph {
    Dev G{};
    Params P{};
    int prog = -1;
    uint32_t* state = nullptr;
    uint64_t M = 0;
    uint64_t M_sc = 0;  // source-centric message slots (after the identity words)
    uint64_t nonempty_bins = 0;
    bool prof = false;
    bool limited = false;  // a finite iteration limit may be set on the device
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double prof_ms[GPOP_KERNEL_COUNT] = {};
    uint64_t prof_n[GPOP_KERNEL_COUNT] = {};
    // the graph's own run, launched through the batched kernels as a batch
    // of one: [0] the run, [1] / [2] source- / partition-centric probes
    Inst h_tab[3]{};
    Inst* d_tab = nullptr;
    BatchGrid grid{}, probe_grid[2]{};
    Runner run;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Task sizes of a graph: the largest source-centric task in work units (at
// least 1024 and at least 4k, so the per-task count row stays small next to
// the task; lighter iterations use smaller tasks) and ids per gather task
// (about 256-512 tasks over all bins, so that the workgroups that finish early
// in a dense iteration pick up further tasks; heavier partitions are split
// over several).
struct Sizes {
    uint32_t s, sc_shift;
    uint64_t q, k, T;
    uint32_t pc_stream;  // GPOP_PCSTREAM_*
};

Sizes sizes_for(uint32_t V, uint64_t E, uint32_t s, const gpop_options* o) {
    Sizes z{};
    z.s = s;
    z.q = 1ull << s;
    z.k = (V + z.q - 1) / z.q;
    z.sc_shift = 10;
    while ((1ull << z.sc_shift) < 4 * z.k) ++z.sc_shift;
    if (o && o->sc_task_log2) z.sc_shift = o->sc_task_log2;
    // about 512 tasks, or 256 when there are 4096 destination partitions
    // (enough columns to fill the chip without splitting as many)
    const uint64_t ntask = std::min<uint64_t>(512, std::max<uint64_t>(256, (1ull << 20) / z.k));
    z.T = std::max<uint64_t>(1ull << 16, E / ntask);
    if (o && o->gather_task_ids) z.T = o->gather_task_ids;
    z.pc_stream = o ? o->pc_stream : GPOP_PCSTREAM_AUTO;
    return z;
}

// Source-centric tasks of one iteration: a task holds at most 2^sc_shift work
// units (an active vertex is one unit, each of its out-edges one more); the
// plan takes smaller tasks when the iteration's units are few, never more
// than 2 x kScTaskTarget of them (plus one partial task per partition).
uint64_t max_sctask_for(uint32_t V, uint64_t E, const Sizes& z) {
    return std::max<uint64_t>((E + V) >> z.sc_shift, 2ull * kScTaskTarget) + z.k + 1;
}

// Bounds of the column streams (chunks, entries): every non-empty bin is
// padded by at most 3 null ids to a multiple of 4 positions, and every
// column by less than one chunk. Streams are built for partitions of at most
// 2^14 vertices (the null id is q, which needs the local-id field's 15th bit).
bool cs_enabled(const Sizes& z) { return z.pc_stream != GPOP_PCSTREAM_OFF && z.s <= 14; }
uint64_t cs_bins_max(uint64_t E, const Sizes& z) { return std::min<uint64_t>(E, z.k * z.k); }
uint64_t cs_chunks_max(uint64_t E, const Sizes& z) {
    if (!cs_enabled(z)) return 0;
    return (E + 3 * cs_bins_max(E, z) + kChunk - 1) / kChunk + z.k + 1;
}
uint64_t cs_entries_max(uint64_t E, const Sizes& z) {
    if (!cs_enabled(z)) return 0;
    return cs_chunks_max(E, z) + cs_bins_max(E, z) + z.k + 1;
}

uint64_t max_gtask_for(uint64_t E, const Sizes& z) {
    return (E + 512ull * z.k * z.k) / z.T + z.k + 1;
}

size_t carve(Dev* G, char* base, uint32_t V, uint64_t E, const Sizes& z, Inst** tab = nullptr,
             uint32_t** boff = nullptr) {
    size_t o = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + o : nullptr;
        o += align256(bytes ? bytes : 1);
        return p;
    };
    const uint64_t q = z.q;
    const uint64_t k = z.k;
    const uint64_t kk = k * k;
    const uint64_t E_pad = align256(E ? E : 1);
    const uint64_t nch = E_pad / kChunk;
    const uint64_t ntask = E / kPcTaskMin + k + 1;
    const uint64_t nsct = max_sctask_for(V, E, z);
    const uint64_t ngt = max_gtask_for(E, z);
    G->part_E = (uint32_t*)take(k * 4);
    G->part_M = (uint32_t*)take(k * 4);
    G->bin_moff = (uint32_t*)take((kk + 1) * 4);
    G->bin_ioff = (uint32_t*)take((kk + 1) * 4);
    G->cm = (uint4*)take(kk * 16);
    G->sc_mo = (uint32_t*)take(kk * 4);
    G->sc_mor = (uint32_t*)take((kk + 1) * 4);
    const uint64_t kw = (k + 63) / 64;
    G->colsrc = (uint64_t*)take(k * kw * 8);
    G->spre = (uint32_t*)take(kk * 4);
    G->png_src = (uint16_t*)take(E_pad * 2);
    G->png_ids = (uint16_t*)take(E_pad * 2);
    G->png_w = (uint8_t*)take(E_pad);
    G->png_chunk = (uint32_t*)take(nch * 4);
    G->pctask = (uint4*)take(ntask * 16);
    {
        const uint64_t nc = cs_chunks_max(E, z), ne = cs_entries_max(E, z);
        G->cs_c0 = (uint32_t*)take((k + 1) * 4);
        G->cs_ids = (uint16_t*)take(nc * kChunk * 2);
        G->cs_w = (uint8_t*)take(nc * kChunk);
        G->cs_lm = (uint64_t*)take(nc * 8);
        G->cs_tabo = (uint32_t*)take((nc + 1) * 4);
        G->cs_ent = (uint2*)take((ne + 64) * 8);
    }
    G->bld_t0 = (uint32_t*)take((k + 1) * 4);
    G->gtask = (uint4*)take(ngt * 32);
    G->gsplit = (uint4*)take(k * 16);
    G->gpart = (uint32_t*)take(ngt * q * 8);
    G->gflag = (uint32_t*)take(ngt * 4);
    G->mtot = (uint4*)take(k * kMaxMergeChunks * 16);
    // partition-centric messages (M <= E), the identity words, then the
    // source-centric message slots (at most M + E / kPiece)
    G->data = (uint32_t*)take((2 * E_pad + E_pad / kPiece + kIdWords) * 4);
    G->sc_ids = (uint16_t*)take(E_pad * 2);
    G->sc_w = (uint8_t*)take(E_pad);
    G->sc_chunk = (uint32_t*)take(nch * 4);
    G->sc_cnt = (uint2*)take(kk * 8);
    G->nz = (uint8_t*)take(k * kw * 64);
    G->cact = (uint32_t*)take(k * 4);
    G->pcmask = (uint64_t*)take(kw * 8);
    G->scmask = (uint64_t*)take(kw * 8);
    G->sc_tt = (uint2*)take(nsct * 8);
    G->sc_sh = (uint8_t*)take(k);
    G->sc_t0 = (uint32_t*)take((k + 1) * 4);
    G->sc_tc = (uint2*)take(((E >> z.sc_shift) + k + 1) * k * 8);  // build tasks x k
    G->gat_ids = (uint32_t*)take(ngt * 4);
    G->gat_ran = (uint32_t*)take((ngt + k) * 4);
    G->mode = (uint8_t*)take(k);
    for (int b = 0; b < 2; ++b) {
        G->flist[b] = (uint16_t*)take(k * q * 2);
        G->fbits[b] = (uint32_t*)take(k * q / 8);
        G->fVa[b] = (uint32_t*)take(k * 4);
        G->fEa[b] = (uint32_t*)take(k * 4);
        G->fpre[b] = (uint32_t*)take(k * q * 4);
        G->dpart[b] = (double*)take(k * 8);
    }
    G->marks = (uint8_t*)take(k * q);
    G->cnt_m = (uint32_t*)take(kk * 4);
    G->cnt_i = (uint32_t*)take(kk * 4);
    G->scan_tmp = (uint32_t*)take(scan_tmp_words(kk) * 4);
    G->ctrl = (Ctrl*)take(sizeof(Ctrl));
    G->log = (gpop_iter_stats*)take(kLogCap * sizeof(gpop_iter_stats));
    G->pfill = (float*)take(k * 4);
    G->pskew = (float*)take(k * 4);
    G->mode_l = (uint8_t*)take(k);
    G->mlp = (gpop_mlp_model*)take(sizeof(gpop_mlp_model));
    G->probe = (unsigned long long*)take(3 * k * 8);
    Inst* t = (Inst*)take(3 * sizeof(Inst));
    uint32_t* b = (uint32_t*)take(6 * 2 * 4);
    if (tab) *tab = t;
    if (boff) *boff = b;
    return o;
}

// Column streams of the partition-centric ids (the layout is described with
// the cs_* fields of Dev). Each destination partition's non-empty bins are
// laid out in source order, each from a multiple of 4 positions, so that a
// decoding lane's four positions never span two bins. The walk over bins is
// done here on the host from the per-bin id counts (row-major, bin[p][q] at
// p*k+q), in row order with per-column state; the per-id work (copying ids
// and weights, counting message starts) is done by launch_cs_fill.
struct ColWalk {
    uint64_t pos = 0;      // stream position inside the column (a multiple of 4 between bins)
    uint64_t chunks = 0, entries = 0;
};

int build_streams(Dev& G, const Sizes& z, const std::vector<uint32_t>& cnti, hipStream_t st) {
    const uint32_t k = G.k;
    if (!cs_enabled(z)) {
        G.n_chunks = 0;
        return GPOP_OK;
    }
    std::vector<ColWalk> w(k);
    std::vector<uint64_t> cbase(k + 1, 0), ebase(k + 1, 0);
    std::vector<uint64_t> lm;
    std::vector<uint32_t> tabo;
    std::vector<uint2> ent;
    // pass 0 counts chunks and entries per column; pass 1 writes them
    for (int pass = 0; pass < 2; ++pass) {
        for (uint32_t q = 0; q < k; ++q) w[q] = ColWalk{};
        auto chunk_begin = [&](uint32_t q, uint32_t p, uint64_t x0) {  // entry 0 of a new chunk
            ColWalk& c = w[q];
            if (pass) {
                const uint64_t ch = cbase[q] + c.chunks;
                tabo[ch] = (uint32_t)(ebase[q] + c.entries);
                ent[ebase[q] + c.entries] = make_uint2((uint32_t)x0, p | (q << 16));
            }
            ++c.chunks;
            ++c.entries;
        };
        auto lane_start = [&](uint32_t q, uint32_t p) {  // a bin (or padding, p = 0xFFFF) at lane pos/4 > 0
            ColWalk& c = w[q];
            const uint32_t t = (uint32_t)(c.pos % kChunk);
            if (pass) {
                lm[cbase[q] + c.chunks - 1] |= 1ull << (t / 4);
                ent[ebase[q] + c.entries] = make_uint2(t, p | (q << 16));
            }
            ++c.entries;
        };
        for (uint32_t p = 0; p < k; ++p) {
            const uint32_t* row = cnti.data() + (size_t)p * k;
            for (uint32_t q = 0; q < k; ++q) {
                const uint32_t ic = row[q];
                if (!ic) continue;
                ColWalk& c = w[q];
                if (c.pos % kChunk) lane_start(q, p);
                // chunks that begin inside [pos, pos + ic), entry 0 = this bin
                const uint64_t first = (c.pos + kChunk - 1) / kChunk, last = (c.pos + ic - 1) / kChunk;
                for (uint64_t ch = first; ch <= last; ++ch) chunk_begin(q, p, ch * kChunk - c.pos);
                c.pos += (ic + 3u) & ~3u;  // null ids fill the bin's last lane
            }
        }
        for (uint32_t q = 0; q < k; ++q) {
            ColWalk& c = w[q];
            if (c.pos % kChunk) lane_start(q, 0xFFFFu);  // padding to the end of the last chunk
        }
        if (pass == 0) {
            for (uint32_t q = 0; q < k; ++q) {
                cbase[q + 1] = cbase[q] + w[q].chunks;
                ebase[q + 1] = ebase[q] + w[q].entries;
            }
            if (cbase[k] > cs_chunks_max(G.E, z) || ebase[k] > cs_entries_max(G.E, z))
                return fail(GPOP_EDEVICE, "internal: column stream bound exceeded");
            if (cbase[k] * kChunk >= 0xFFFFFFFFull)
                return fail(GPOP_ENOTSUP, "column streams of %llu positions exceed 2^32",
                            (unsigned long long)(cbase[k] * kChunk));
            lm.assign(cbase[k], 0ull);
            tabo.assign(cbase[k] + 1, 0u);
            ent.assign(ebase[k] + 64, make_uint2(0u, 0xFFFFu));
            tabo[cbase[k]] = (uint32_t)ebase[k];
        }
    }
    G.n_chunks = (uint32_t)cbase[k];
    std::vector<uint32_t> c0(k + 1);
    for (uint32_t q = 0; q <= k; ++q) c0[q] = (uint32_t)cbase[q];
    HIP_OR_RETURN(hipMemcpyAsync(G.cs_c0, c0.data(), c0.size() * 4, hipMemcpyHostToDevice, st), "write stream bases");
    if (G.n_chunks) {
        HIP_OR_RETURN(hipMemcpyAsync(G.cs_lm, lm.data(), lm.size() * 8, hipMemcpyHostToDevice, st),
                      "write stream lane starts");
        HIP_OR_RETURN(hipMemcpyAsync(G.cs_tabo, tabo.data(), tabo.size() * 4, hipMemcpyHostToDevice, st),
                      "write stream tables");
        HIP_OR_RETURN(hipMemcpyAsync(G.cs_ent, ent.data(), ent.size() * 8, hipMemcpyHostToDevice, st),
                      "write stream entries");
        HIP_OR_RETURN(launch_cs_fill(G, st), "fill column streams");
    }
    // the host vectors must outlive the copies
    HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
    return GPOP_OK;
}

int check_desc(const gpop_graph_desc* d, const gpop_options* o, uint32_t* s_out) {
    if (!d) return fail(GPOP_EINVAL, "desc is NULL");
    if (d->num_vertices == 0) return fail(GPOP_EINVAL, "graph has no vertex");
    if (d->num_edges >= 0xFFFFFFFFull) return fail(GPOP_EINVAL, "E must be < 2^32 - 1");
    if (d->reserved0) return fail(GPOP_EINVAL, "reserved0 must be zero");
    uint32_t s = 14;
    if (o) {
        for (int i = 0; i < 2; ++i)
            if (o->reserved[i]) return fail(GPOP_EINVAL, "options.reserved must be zero");
        if (o->sc_reserve > GPOP_SCRES_BIN) return fail(GPOP_EINVAL, "unknown sc_reserve mode %u", o->sc_reserve);
        if (o->combine > GPOP_COMBINE_ROUNDS) return fail(GPOP_EINVAL, "unknown combine %u", o->combine);
        if (o->pc_stream > GPOP_PCSTREAM_ON) return fail(GPOP_EINVAL, "unknown pc_stream mode %u", o->pc_stream);
        if (o->log2_part) s = o->log2_part;
        if (o->sc_task_log2 && (o->sc_task_log2 < 6 || o->sc_task_log2 > 24))
            return fail(GPOP_EINVAL, "sc_task_log2 must be 0 or in [6, 24]");
        if (o->gather_task_ids && o->gather_task_ids < 256)
            return fail(GPOP_EINVAL, "gather_task_ids must be 0 or >= 256");
    }
    if (s < 8 || s > 15) return fail(GPOP_EINVAL, "log2_part must be in [8, 15]");
    const uint64_t q = 1ull << s;
    const uint64_t k = (d->num_vertices + q - 1) / q;
    if (k > 4096) return fail(GPOP_EINVAL, "too many partitions (k = %llu > 4096); raise log2_part",
                              (unsigned long long)k);
    *s_out = s;
    return GPOP_OK;
}

hipEvent_t get_event(gpop_graph* g) {
    if (!g->pool.empty()) {
        hipEvent_t e = g->pool.back();
        g->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

template <class F>
int timed(gpop_graph* g, int kid, hipStream_t s, F&& f, const char* what) {
    hipEvent_t a = nullptr, b = nullptr;
    if (g->prof) {
        a = get_event(g);
        b = get_event(g);
        if (a && b) (void)hipEventRecord(a, s);
    }
    hipError_t e = f();
    if (e != hipSuccess) return hip_fail(e, what);
    if (g->prof && a && b) {
        (void)hipEventRecord(b, s);
        g->pending.push_back({kid, a, b});
    }
    return GPOP_OK;
}

int collect_profile(gpop_graph* g) {
    for (const Pending& p : g->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g->prof_ms[p.kid] += ms;
            g->prof_n[p.kid] += 1;
        }
        g->pool.push_back(p.a);
        g->pool.push_back(p.b);
    }
    g->pending.clear();
    return GPOP_OK;
}

// One iteration of every run of B; ev (2 * GPOP_KERNEL_COUNT events, or
// nullptr) brackets plan, SC scatter, PC scatter, gather and merge.
hipError_t launch_iteration(const BatchGrid& B, int prog, hipStream_t st, const hipEvent_t* ev) {
    hipError_t e = hipSuccess;
    auto mark = [&](int i) {
        if (ev && e == hipSuccess) e = hipEventRecord(ev[i], st);
    };
    mark(0);
    if (e == hipSuccess) e = launch_batch_select(B, st);
    if (e == hipSuccess) e = launch_batch_plan(B, st);
    mark(1);
    mark(2);
    if (e == hipSuccess) e = launch_batch_sc(B, prog, st);
    mark(3);
    mark(4);
    if (e == hipSuccess) e = launch_batch_pc(B, prog, st);
    mark(5);
    mark(6);
    if (e == hipSuccess) e = launch_batch_gather(B, prog, st);
    mark(7);
    mark(8);
    if (e == hipSuccess) e = launch_batch_merge(B, prog, st);
    mark(9);
    return e;
}

int runner_record(Runner& R, const BatchGrid& B, int prog, bool prof, uint32_t* d_status) {
    R.drop();
    if (!R.cap && hipStreamCreateWithFlags(&R.cap, hipStreamNonBlocking) != hipSuccess)
        return fail(GPOP_EDEVICE, "cannot create the recording stream");
    const size_t nev = prof ? (size_t)2 * GPOP_KERNEL_COUNT * R.chunk : 0;
    while (R.ev.size() < nev) {
        hipEvent_t e = nullptr;
        HIP_OR_RETURN(hipEventCreate(&e), "event");
        R.ev.push_back(e);
    }
    HIP_OR_RETURN(prepare_batch_scatter(B, prog), "kernel attributes");
    HIP_OR_RETURN(prepare_batch_gather(B, prog), "kernel attributes");
    HIP_OR_RETURN(hipStreamBeginCapture(R.cap, hipStreamCaptureModeRelaxed), "begin capture");
    hipError_t e = hipSuccess;
    for (uint32_t c = 0; c < R.chunk && e == hipSuccess; ++c)
        e = launch_iteration(B, prog, R.cap, prof ? &R.ev[(size_t)2 * GPOP_KERNEL_COUNT * c] : nullptr);
    if (e == hipSuccess && d_status) e = launch_batch_status(B, d_status, R.cap);
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(R.cap, &gr);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return hip_fail(e != hipSuccess ? e : e2, "record iterations");
    }
    R.graph = gr;
    HIP_OR_RETURN(hipGraphInstantiate(&R.exec, gr, nullptr, nullptr, 0), "instantiate iterations");
    R.prog = prog;
    R.prof = prof;
    R.learned = B.learned;
    return GPOP_OK;
}

// Replays the recorded iterations (or launches them directly when `eager`)
// until `finished()` reports that every run has finished or paused. The
// limit set on the device bounds the replays: max_iter / chunk + 2 suffice.
template <class F>
int runner_run(Runner& R, const BatchGrid& B, int prog, bool prof, bool eager, uint32_t max_iter,
               uint32_t* d_status, hipStream_t st, double* prof_ms, uint64_t* prof_n, F&& finished) {
    if (!eager && (R.prog != prog || R.prof != prof || R.learned != B.learned || !R.exec)) {
        int rc = runner_record(R, B, prog, prof, d_status);
        if (rc) return rc;
    }
    if (eager) {
        HIP_OR_RETURN(prepare_batch_scatter(B, prog), "kernel attributes");
        HIP_OR_RETURN(prepare_batch_gather(B, prog), "kernel attributes");
    }
    const uint64_t passes = (uint64_t)max_iter / R.chunk + 2;
    for (uint64_t r = 0; r < passes; ++r) {
        if (eager) {
            for (uint32_t c = 0; c < R.chunk; ++c)
                HIP_OR_RETURN(launch_iteration(B, prog, st, nullptr), "iteration");
            if (d_status) HIP_OR_RETURN(launch_batch_status(B, d_status, st), "run status");
        } else {
            HIP_OR_RETURN(hipGraphLaunch(R.exec, st), "replay iterations");
        }
        bool done = false;
        int rc = finished(done);  // synchronises the stream
        if (rc) return rc;
        if (prof && !eager) {
            for (uint32_t c = 0; c < R.chunk; ++c)
                for (int k = 0; k < GPOP_KERNEL_COUNT; ++k) {
                    float ms = 0.f;
                    const size_t i = (size_t)2 * GPOP_KERNEL_COUNT * c + 2 * k;
                    if (hipEventElapsedTime(&ms, R.ev[i], R.ev[i + 1]) == hipSuccess) {
                        prof_ms[k] += ms;
                        prof_n[k] += 1;
                    }
                }
        }
        if (done) break;
    }
    return GPOP_OK;
}

constexpr size_t kLdsPerWorkgroup = 160 * 1024;  // gfx950: on-chip memory a workgroup may use

int cu_count() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) return 256;
    return v;
}

// Slice length of the partition-centric scatter tasks, from a few sizes, by a
// model of an iteration where every partition scatters: workgroups (two per
// CU while the partition's q state words fit twice in LDS) take the slices
// longest first; a slice costs its slots plus a reload of its partition's
// state, about q * 4 / 6 slot-equivalents (a slot moves 6 bytes). The least
// modelled finish time wins, the longer slice on a tie. Long slices reload
// less state; short ones leave a smaller last round.
uint64_t pc_task_slots(const std::vector<uint32_t>& partM, uint64_t q) {
    const uint64_t per_cu = std::max<uint64_t>(1, std::min<uint64_t>(2, kLdsPerWorkgroup / (q * 4)));
    const size_t nslot = (size_t)cu_count() * per_cu;
    const double fix = (double)q * 4.0 / 6.0;
    const uint64_t cand[] = {kPcTaskMin, 49152, 65536, 98304, 131072, 196608, 262144};
    uint64_t best_len = 65536;
    double best = 0.0;
    bool have = false;
    std::vector<double> len;
    for (const uint64_t L : cand) {
        len.clear();
        for (const uint32_t m : partM)
            for (uint64_t a = 0; a < m; a += L) len.push_back((double)std::min<uint64_t>(m - a, L));
        std::sort(len.begin(), len.end(), [](double x, double y) { return x > y; });
        std::priority_queue<double, std::vector<double>, std::greater<double>> busy;
        for (size_t i = 0; i < nslot; ++i) busy.push(0.0);
        double finish = 0.0;
        for (const double l : len) {
            const double t = busy.top() + fix + l;
            busy.pop();
            busy.push(t);
            finish = std::max(finish, t);
        }
        if (!have || finish <= best) {
            best = finish;
            best_len = L;
            have = true;
        }
    }
    return best_len;
}

int max_lds_per_block() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 65536;
    return v;
}

}  // namespace

extern "C" {

int gpop_abi_version(void) { return GPOP_ABI_VERSION; }

const char* gpop_last_error(void) { return g_err.c_str(); }

int gpop_plan(const gpop_graph_desc* desc, const gpop_options* opts, gpop_plan_info* out) {
    uint32_t s;
    int rc = check_desc(desc, opts, &s);
    if (rc) return rc;
    if (!out) return fail(GPOP_EINVAL, "out is NULL");
    Dev G{};
    memset(out, 0, sizeof *out);
    out->q = 1u << s;
    out->k = (desc->num_vertices + out->q - 1) / out->q;
    out->workspace_bytes = carve(&G, nullptr, desc->num_vertices, desc->num_edges,
                                 sizes_for(desc->num_vertices, desc->num_edges, s, opts));
    return GPOP_OK;
}

int gpop_graph_create(const gpop_graph_desc* desc, const gpop_options* opts, void* d_ws,
                      size_t ws_bytes, void* stream, gpop_graph** out) {
    uint32_t s;
    int rc = check_desc(desc, opts, &s);
    if (rc) return rc;
    if (!out) return fail(GPOP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!desc->offsets || (!desc->cols && desc->num_edges))
        return fail(GPOP_EINVAL, "offsets/cols must be device pointers");
    if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(GPOP_EINVAL, "workspace must be 256-byte aligned");
    Dev G{};
    const Sizes z = sizes_for(desc->num_vertices, desc->num_edges, s, opts);
    const size_t need = carve(&G, nullptr, desc->num_vertices, desc->num_edges, z);
    if (ws_bytes < need)
        return fail(GPOP_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    Inst* d_tab = nullptr;
    uint32_t* d_boff = nullptr;
    carve(&G, (char*)d_ws, desc->num_vertices, desc->num_edges, z, &d_tab, &d_boff);
    G.V = desc->num_vertices;
    G.E = desc->num_edges;
    G.s = s;
    G.q = 1u << s;
    G.k = (G.V + G.q - 1) / G.q;
    G.kw = (G.k + 63) / 64;
    G.nbits = 0;
    while ((1u << G.nbits) < G.k) ++G.nbits;
    G.off = desc->offsets;
    G.cols = desc->cols;
    G.w = desc->weights;
    hipStream_t st = (hipStream_t)stream;

    G.sc_shift = z.sc_shift;
    G.max_sctask = (uint32_t)max_sctask_for(G.V, G.E, z);
    if (sc_lds_bytes(G.k) > (size_t)max_lds_per_block() ||
        gather_lds_bytes(P_BFS, G.q, false) + 2048 > (size_t)max_lds_per_block())
        return fail(GPOP_ENOTSUP, "partition of %u vertices does not fit the LDS", G.q);

    HIP_OR_RETURN(hipMemsetAsync(G.ctrl, 0, sizeof(Ctrl), st), "clear control block");
    HIP_OR_RETURN(launch_validate(G, st), "validate CSR");
    Ctrl hc;
    HIP_OR_RETURN(hipMemcpyAsync(&hc, G.ctrl, sizeof hc, hipMemcpyDeviceToHost, st), "read control");
    HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
    if (!hc.csr_err) {
        HIP_OR_RETURN(launch_validate_edges(G, st), "validate CSR");
        HIP_OR_RETURN(hipMemcpyAsync(&hc, G.ctrl, sizeof hc, hipMemcpyDeviceToHost, st), "read control");
        HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
    }
    if (hc.csr_err) {
        static const char* why[] = {"", "offsets[0] != 0", "decreasing offsets or offset > E",
                                    "offsets[V] != E", "column index >= V", "row not sorted ascending"};
        return fail(GPOP_EINVAL, "malformed CSR: %s", why[hc.csr_err < 6 ? hc.csr_err : 0]);
    }
    const uint64_t kk = (uint64_t)G.k * G.k;
    HIP_OR_RETURN(launch_part_E(G, st), "partition edges");
    std::vector<uint32_t> partE(G.k), bld(G.k + 1);
    HIP_OR_RETURN(hipMemcpyAsync(partE.data(), G.part_E, G.k * 4, hipMemcpyDeviceToHost, st), "read E^p");
    HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
    {
        uint64_t t = 0;
        for (uint32_t p = 0; p < G.k; ++p) {
            bld[p] = (uint32_t)t;
            t += ((uint64_t)partE[p] + (1ull << G.sc_shift) - 1) >> G.sc_shift;
        }
        bld[G.k] = (uint32_t)t;
        G.n_bldtask = (uint32_t)t;
    }
    HIP_OR_RETURN(hipMemcpyAsync(G.bld_t0, bld.data(), (G.k + 1) * 4, hipMemcpyHostToDevice, st),
                  "write build tasks");
    HIP_OR_RETURN(launch_sc_build(G, 0, st), "count bins");
    HIP_OR_RETURN(launch_scan_excl(G.cnt_m, G.bin_moff, kk, G.scan_tmp, st), "scan messages");
    HIP_OR_RETURN(launch_scan_excl(G.cnt_i, G.bin_ioff, kk, G.scan_tmp, st), "scan ids");
    HIP_OR_RETURN(launch_part_M(G, st), "partition messages");
    HIP_OR_RETURN(launch_colmajor(G, st), "column table");
    HIP_OR_RETURN(launch_colsrc(G, st), "column source masks");
    // source-centric message slots: per bin its capacity (cnt_m becomes it),
    // scanned into the counter array, which is cleared below
    uint64_t m_sc = 0;
    {
        uint32_t* sx = reinterpret_cast<uint32_t*>(G.sc_cnt);  // kk * 8 bytes >= (kk + 1) words
        HIP_OR_RETURN(launch_sc_cap(G, st), "source-centric capacities");
        HIP_OR_RETURN(launch_scan_excl(G.cnt_m, sx, kk, G.scan_tmp, st), "scan source-centric capacities");
        uint32_t tot[2];
        HIP_OR_RETURN(hipMemcpyAsync(&tot[0], G.bin_moff + kk, 4, hipMemcpyDeviceToHost, st), "read M");
        HIP_OR_RETURN(hipMemcpyAsync(&tot[1], sx + kk, 4, hipMemcpyDeviceToHost, st), "read SC slots");
        HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
        m_sc = tot[1];
        if ((uint64_t)tot[0] + kIdWords + m_sc >= 0x80000000ull)
            return fail(GPOP_ENOTSUP, "graph has %llu + %llu message slots; at most 2^31 - 1 supported",
                        (unsigned long long)tot[0], (unsigned long long)m_sc);
        HIP_OR_RETURN(launch_sc_mo(G, sx, tot[0] + kIdWords, st), "source-centric message offsets");
    }
    // source-centric counters and marks start clear (each scatter clears what
    // the one before it stamped)
    HIP_OR_RETURN(hipMemsetAsync(G.cact, 0, (size_t)G.k * 4, st), "clear column stamps");
    HIP_OR_RETURN(hipMemsetAsync(G.sc_cnt, 0, kk * 8, st), "clear bin counters");
    HIP_OR_RETURN(hipMemsetAsync(G.nz, 0, (size_t)G.k * G.kw * 64, st), "clear bin marks");
    HIP_OR_RETURN(launch_sc_build(G, 1, st), "fill PNG");

    std::vector<uint32_t> partM(G.k), cnti(kk), ioff(kk + 1);
    HIP_OR_RETURN(hipMemcpyAsync(partM.data(), G.part_M, G.k * 4, hipMemcpyDeviceToHost, st), "read M");
    HIP_OR_RETURN(hipMemcpyAsync(cnti.data(), G.cnt_i, kk * 4, hipMemcpyDeviceToHost, st), "read counts");
    HIP_OR_RETURN(hipMemcpyAsync(ioff.data(), G.bin_ioff, (kk + 1) * 4, hipMemcpyDeviceToHost, st),
                  "read offsets");
    HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
    // partition-centric scatter tasks: slices of each partition's message range
    const uint64_t pc_len = pc_task_slots(partM, G.q);
    std::vector<uint4> tasks;
    uint64_t slot = 0;
    for (uint32_t p = 0; p < G.k; ++p) {
        for (uint64_t a = 0; a < partM[p]; a += pc_len) {
            const uint64_t b = std::min<uint64_t>(partM[p], a + pc_len);
            tasks.push_back(make_uint4(p, (uint32_t)(slot + a), (uint32_t)(slot + b), 0));
        }
        slot += partM[p];
    }
    // workgroups start in task order: longest slices first
    std::stable_sort(tasks.begin(), tasks.end(),
                     [](const uint4& x, const uint4& y) { return x.z - x.y > y.z - y.y; });
    if (slot >= 0x80000000ull)
        return fail(GPOP_ENOTSUP, "graph has %llu messages; at most 2^31 - 1 supported",
                    (unsigned long long)slot);
    uint64_t nz = 0;
    for (uint64_t i = 0; i < kk; ++i) nz += cnti[i] != 0;
    G.n_pctask = (uint32_t)tasks.size();
    if (!tasks.empty())
        HIP_OR_RETURN(hipMemcpyAsync(G.pctask, tasks.data(), tasks.size() * sizeof(uint4),
                                     hipMemcpyHostToDevice, st), "write task table");
    // gather tasks: each destination partition's static 256-id pieces, in
    // source-partition order, cut into ranges of about gather_task_ids ids
    const uint64_t T = z.T;
    const uint64_t max_gt = max_gtask_for(G.E, z);
    std::vector<uint4> gt, gs;
    std::vector<uint64_t> sp(G.k);
    uint32_t nslot = 0;
    for (uint32_t q = 0; q < G.k; ++q) {
        uint64_t tot = 0;
        for (uint32_t p = 0; p < G.k; ++p) {
            const uint64_t r = (uint64_t)p * G.k + q;
            const uint64_t c = cnti[r], o = ioff[r];
            sp[p] = c ? (o + c - 1) / kChunk - o / kChunk + 1 : 0;
            tot += sp[p];
        }
        uint64_t nt = (tot * kChunk + T - 1) / T;
        nt = std::max<uint64_t>(1, std::min<uint64_t>(nt, 64));
        uint32_t p = 0;
        uint64_t before = 0;  // static pieces of bins p' < p
        for (uint64_t j = 0; j < nt; ++j) {
            const uint64_t a = tot * j / nt, b = tot * (j + 1) / nt;
            while (p + 1 < G.k && before + sp[p] <= a) before += sp[p++];
            uint32_t plo = nt == 1 ? 0 : p;
            uint64_t blo = nt == 1 ? 0 : before;
            uint32_t phi = plo;
            uint64_t acc = blo;
            if (nt == 1) phi = G.k - 1;
            else {
                while (phi + 1 < G.k && acc + sp[phi] < b) acc += sp[phi++];
            }
            const uint32_t s0 = (uint32_t)(a - blo), s1 = (uint32_t)(b - blo);
            const uint32_t sl = nt > 1 ? nslot++ : 0u;
            gt.push_back(make_uint4(q, plo, phi, (uint32_t)(nt << 16) | (uint32_t)j));
            gt.push_back(make_uint4(s0, s1, sl, 0));
        }
        if (nt > 1) gs.push_back(make_uint4(q, 0u, (uint32_t)nt, nslot - (uint32_t)nt));
    }
    if (gt.size() / 2 > max_gt) return fail(GPOP_EDEVICE, "internal: gather task bound exceeded");
    {
        // Workgroups start in task order: the largest tasks (static pieces)
        // go first, so that a dense iteration ends on small ones instead of
        // leaving a partly filled last round of large ones. Each entry is
        // self-contained (split partials are addressed by slot), so the order
        // is free.
        const size_t nt = gt.size() / 2;
        std::vector<uint32_t> ord(nt);
        std::vector<uint64_t> wt(nt);
        for (size_t t = 0; t < nt; ++t) {
            ord[t] = (uint32_t)t;
            const uint4 a = gt[2 * t], b = gt[2 * t + 1];
            if ((a.w >> 16) > 1) wt[t] = b.y - b.x;
            else {
                uint64_t tot = 0;
                for (uint32_t p = 0; p < G.k; ++p) {
                    const uint64_t r = (uint64_t)p * G.k + a.x, c = cnti[r], o = ioff[r];
                    tot += c ? (o + c - 1) / kChunk - o / kChunk + 1 : 0;
                }
                wt[t] = tot;
            }
        }
        std::stable_sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) { return wt[x] > wt[y]; });
        std::vector<uint4> sorted(gt.size());
        for (size_t t = 0; t < nt; ++t) {
            sorted[2 * t] = gt[2 * ord[t]];
            sorted[2 * t + 1] = gt[2 * ord[t] + 1];
        }
        gt.swap(sorted);
    }
    G.n_gtask = (uint32_t)(gt.size() / 2);
    G.n_gsplit = (uint32_t)gs.size();
    G.combine = opts ? opts->combine : GPOP_COMBINE_LDS;
    G.whole_ids = (uint32_t)std::min<uint64_t>(z.T / 2, 0x7FFFFFFFull);
    HIP_OR_RETURN(hipMemcpyAsync(G.gtask, gt.data(), gt.size() * sizeof(uint4), hipMemcpyHostToDevice, st),
                  "write gather tasks");
    if (!gs.empty())
        HIP_OR_RETURN(hipMemcpyAsync(G.gsplit, gs.data(), gs.size() * sizeof(uint4), hipMemcpyHostToDevice,
                                     st), "write split list");
    G.idb = (uint32_t)slot;
    G.pcs_mode = z.pc_stream;
    G.scres_mode = opts ? opts->sc_reserve : GPOP_SCRES_AUTO;
    HIP_OR_RETURN(hipMemsetD32Async((hipDeviceptr_t)(G.data + G.idb), 0xFFFFFFFF, kIdWords, st),
                  "write identity words");
    if ((rc = build_streams(G, z, cnti, st))) return rc;
    HIP_OR_RETURN(launch_part_static(G, st), "partition features");
    Ctrl hc2;
    HIP_OR_RETURN(hipMemcpyAsync(&hc2, G.ctrl, sizeof hc2, hipMemcpyDeviceToHost, st), "read control");
    HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
    if (hc2.bug) return fail(GPOP_EDEVICE, "internal error while building the partition layout");

    // the graph's own run as a batch of one: per kernel, blocks [0, n)
    const uint32_t nb[6] = {(G.k + 31) / 32, std::min<uint32_t>((G.max_sctask + kScWaves - 1) / kScWaves, 2048u),
                            (G.k + 3) / 4, G.n_pctask, G.n_gtask, G.n_gsplit * merge_chunks(G.q)};
    uint32_t hb[12];
    for (int j = 0; j < 6; ++j) {
        hb[2 * j] = 0;
        hb[2 * j + 1] = nb[j];
    }
    HIP_OR_RETURN(hipMemcpyAsync(d_boff, hb, sizeof hb, hipMemcpyHostToDevice, st), "write run grid");
    HIP_OR_RETURN(hipStreamSynchronize(st), "sync");

    gpop_graph* g = new (std::nothrow) gpop_graph();
    if (!g) return fail(GPOP_ENOMEM, "host allocation failed");
    g->G = G;
    g->M = slot;
    g->M_sc = m_sc;
    g->nonempty_bins = nz;
    g->P.selector = GPOP_SEL_ANALYTICAL;
    g->P.s_i = 4;
    g->P.s_v = 4;
    g->P.ratio_num = 16 * 1024;  // BW_PC / BW_SC = 16 (measured on this GPU; the paper's CPU figure is 2)
    g->P.ratio_den = 1024;
    g->d_tab = d_tab;
    BatchGrid& B = g->grid;
    B.tab = d_tab;
    B.n = 1;
    B.b_select = d_boff;
    B.b_sc = d_boff + 2;
    B.b_clr = d_boff + 4;
    B.b_pc = d_boff + 6;
    B.b_gather = d_boff + 8;
    B.b_merge = d_boff + 10;
    B.nb_select = nb[0];
    B.nb_sc = nb[1];
    B.nb_clr = nb[2];
    B.nb_pc = nb[3];
    B.nb_gather = nb[4];
    B.nb_merge = nb[5];
    B.k_max = G.k;
    B.q_max = G.q;
    B.rounds = G.combine == GPOP_COMBINE_ROUNDS;
    B.learned = false;
    B.streams = G.n_chunks != 0;
    B.view = &g->G;
    for (int i = 0; i < 2; ++i) {
        g->probe_grid[i] = B;
        g->probe_grid[i].tab = d_tab + 1 + i;
    }
    *out = g;
    return GPOP_OK;
}

int gpop_graph_destroy(gpop_graph* g) {
    if (!g) return GPOP_OK;
    for (const Pending& p : g->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : g->pool) (void)hipEventDestroy(e);
    delete g;
    return GPOP_OK;
}

int gpop_graph_get_info(const gpop_graph* g, gpop_graph_info* out) {
    if (!g || !out) return fail(GPOP_EINVAL, "NULL argument");
    memset(out, 0, sizeof *out);
    out->q = g->G.q;
    out->k = g->G.k;
    out->num_vertices = g->G.V;
    out->num_edges = g->G.E;
    out->num_messages = g->M;
    out->nonempty_bins = g->nonempty_bins;
    return GPOP_OK;
}

namespace {

// Programs whose result does not depend on the order of updates (a minimum
// fixed point), so that interleaved scatter-gather leaves it unchanged.
bool isg_program(int prog) {
    return prog == GPOP_PROG_BFS_LEVEL || prog == GPOP_PROG_CC_MINLABEL || prog == GPOP_PROG_SSSP_U32;
}

// Argument checks shared by gpop_state_init and gpop_batch_state_init.
int check_program(const gpop_graph* g, gpop_program prog, const gpop_params* prm) {
    if ((int)prog < 0 || (int)prog > GPOP_PROG_NIBBLE_F32) return fail(GPOP_EINVAL, "unknown program %d", (int)prog);
    const bool rooted = prog != GPOP_PROG_CC_MINLABEL && prog != GPOP_PROG_PAGERANK_F32;
    if (rooted && prm->root >= g->G.V) return fail(GPOP_EINVAL, "root %u >= V", prm->root);
    if (prog == GPOP_PROG_CARRY_BFS && prm->persist == 0) return fail(GPOP_EINVAL, "persist must be >= 1");
    if (prog == GPOP_PROG_SSSP_U32 && !g->G.w && g->G.E > 0) return fail(GPOP_EINVAL, "SSSP needs edge weights");
    if (prog == GPOP_PROG_PAGERANK_F32 && !(prm->damping >= 0.f && prm->damping <= 1.f))
        return fail(GPOP_EINVAL, "damping must be in [0, 1]");
    if (prog == GPOP_PROG_PPR_F32 && !(prm->alpha >= 0.f && prm->alpha <= 1.f))
        return fail(GPOP_EINVAL, "alpha must be in [0, 1]");
    if (prog == GPOP_PROG_NIBBLE_F32 && !(prm->epsilon > 0.f && std::isfinite(prm->epsilon)))
        return fail(GPOP_EINVAL, "epsilon must be finite and > 0");
    if (g->P.isg > 1 && !isg_program(prog))
        return fail(GPOP_ENOTSUP, "interleaved scatter-gather is on; program %d does not take it", (int)prog);
    const bool rounds = g->G.combine == GPOP_COMBINE_ROUNDS;
    if (gather_lds_bytes(prog, g->G.q, rounds) + 2048 > (size_t)max_lds_per_block())
        return fail(GPOP_ENOTSUP, "program %d needs %zu bytes of LDS at q = %u; use a smaller partition",
                    (int)prog, gather_lds_bytes(prog, g->G.q, rounds), g->G.q);
    return GPOP_OK;
}

void program_params(const gpop_graph* g, const gpop_params* prm, Params* P) {
    P->root = prm->root;
    P->persist = prm->persist;
    P->damping = prm->damping;
    P->alpha = prm->alpha;
    P->eps = prm->epsilon;
    P->inv_n = 1.0 / (double)g->G.V;
}

}  // namespace

namespace {

// Writes the graph's run table (the run and its two probe variants).
int upload_tab(gpop_graph* g, hipStream_t st) {
    for (int i = 0; i < 3; ++i) {
        g->h_tab[i].G = g->G;
        g->h_tab[i].P = g->P;
        g->h_tab[i].state = g->state;
    }
    g->h_tab[0].P.probe = 0;
    g->h_tab[1].P.probe = 1;
    g->h_tab[1].P.selector = GPOP_SEL_FORCE_SC;
    g->h_tab[2].P.probe = 1;
    g->h_tab[2].P.selector = GPOP_SEL_FORCE_PC;
    HIP_OR_RETURN(hipMemcpyAsync(g->d_tab, g->h_tab, sizeof g->h_tab, hipMemcpyHostToDevice, st), "write run table");
    HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
    return GPOP_OK;
}

Ctrl read_ctrl(const gpop_graph* g, hipStream_t st, int* rc) {
    Ctrl hc{};
    *rc = GPOP_OK;
    if (hipMemcpyAsync(&hc, g->G.ctrl, sizeof hc, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        *rc = fail(GPOP_EDEVICE, "read control");
    return hc;
}

}  // namespace

int gpop_state_init(gpop_graph* g, gpop_program prog, const gpop_params* prm, void* d_state,
                    void* stream) {
    if (!g || !prm || !d_state) return fail(GPOP_EINVAL, "NULL argument");
    int rc = check_program(g, prog, prm);
    if (rc) return rc;
    g->prog = (int)prog;
    g->state = (uint32_t*)d_state;
    program_params(g, prm, &g->P);
    hipStream_t st = (hipStream_t)stream;
    HIP_OR_RETURN(launch_state_init(g->G, g->P, g->prog, g->state, st), "state init");
    g->limited = false;
    if ((rc = upload_tab(g, st))) return rc;
    HIP_OR_RETURN(prepare_batch_scatter(g->grid, g->prog), "kernel attributes");
    HIP_OR_RETURN(prepare_batch_gather(g->grid, g->prog), "kernel attributes");
    return GPOP_OK;
}

int gpop_set_frontier(gpop_graph* g, const uint32_t* d_vertices, uint32_t n, void* stream) {
    if (!g) return fail(GPOP_EINVAL, "NULL graph");
    if (n && !d_vertices) return fail(GPOP_EINVAL, "NULL vertex array");
    HIP_OR_RETURN(launch_set_frontier(g->G, d_vertices, n, 0, (hipStream_t)stream), "set frontier");
    return GPOP_OK;
}

int gpop_set_frontier_all(gpop_graph* g, void* stream) {
    if (!g) return fail(GPOP_EINVAL, "NULL graph");
    HIP_OR_RETURN(launch_set_frontier(g->G, nullptr, 0, 1, (hipStream_t)stream), "set frontier");
    return GPOP_OK;
}

int gpop_set_selector(gpop_graph* g, gpop_selector kind, float bw_ratio, uint32_t s_i,
                      uint32_t s_v, const void* d_mlp) {
    if (!g) return fail(GPOP_EINVAL, "NULL graph");
    if ((int)kind < 0 || (int)kind > GPOP_SEL_LEARNED) return fail(GPOP_EINVAL, "unknown selector");
    if (!(bw_ratio > 0.f) || !std::isfinite(bw_ratio) || bw_ratio > 1e6f)
        return fail(GPOP_EINVAL, "bw_ratio must be finite and > 0");
    if (s_i < 1 || s_i > 16 || s_v < 1 || s_v > 16) return fail(GPOP_EINVAL, "s_i, s_v in [1, 16]");
    if (kind == GPOP_SEL_LEARNED && d_mlp) {
        // validate on the host, then keep a private copy in the workspace
        gpop_mlp_model h;
        HIP_OR_RETURN(hipMemcpy(&h, d_mlp, sizeof h, hipMemcpyDeviceToHost), "read model");
        if (h.magic != GPOP_MLP_MAGIC || h.n_params != GPOP_MLP_PARAMS)
            return fail(GPOP_EINVAL, "not a gpop_mlp_model (bad magic or parameter count)");
        for (int i = 0; i < GPOP_MLP_IN; ++i)
            if (!std::isfinite(h.mean[i]) || !std::isfinite(h.inv_std[i]) || !(h.inv_std[i] > 0.f))
                return fail(GPOP_EINVAL, "model standardisation %d is not finite and positive", i);
        for (int j = 0; j < GPOP_MLP_PARAMS; ++j)
            if ((h.w[j] & 0x7F80u) == 0x7F80u) return fail(GPOP_EINVAL, "model weight %d is not finite", j);
        if (!(h.margin >= 0.f)) return fail(GPOP_EINVAL, "model margin must be >= 0");
        HIP_OR_RETURN(hipMemcpy(g->G.mlp, &h, sizeof h, hipMemcpyHostToDevice), "write model");
        // an infinite margin: the plan applies Eq. 1 and no selection kernel runs
        g->P.learned_eq1 = std::isinf(h.margin) ? 1u : 0u;
    }
    g->P.selector = (uint32_t)kind;
    g->P.ratio_num = (uint32_t)std::lround((double)bw_ratio * 1024.0);
    if (g->P.ratio_num == 0) g->P.ratio_num = 1;
    g->P.ratio_den = 1024;
    g->P.s_i = s_i;
    g->P.s_v = s_v;
    if (kind == GPOP_SEL_LEARNED && !d_mlp) g->P.selector = GPOP_SEL_ANALYTICAL;
    g->grid.learned = g->P.selector == GPOP_SEL_LEARNED && !g->P.learned_eq1;
    if (g->prog >= 0) return upload_tab(g, nullptr);  // the run reads its parameters on the device
    return GPOP_OK;
}

int gpop_set_isg(gpop_graph* g, uint32_t classes) {
    if (!g) return fail(GPOP_EINVAL, "NULL graph");
    if (classes > 16) return fail(GPOP_EINVAL, "at most 16 colour classes (got %u)", classes);
    if (classes > 1 && g->prog >= 0 && !isg_program(g->prog))
        return fail(GPOP_ENOTSUP, "program %d does not take interleaved scatter-gather", g->prog);
    g->P.isg = classes > 1 ? classes : 0;
    if (g->prog >= 0) return upload_tab(g, nullptr);  // the run reads its parameters on the device
    return GPOP_OK;
}

int gpop_features(gpop_graph* g, float* d_out, void* stream) {
    if (!g || !d_out) return fail(GPOP_EINVAL, "NULL argument");
    HIP_OR_RETURN(launch_features(g->G, g->P, d_out, (hipStream_t)stream), "features");
    return GPOP_OK;
}

int gpop_probe_scatter(gpop_graph* g, gpop_selector kind, float* h_us, float* h_total_us, void* stream) {
    if (!g) return fail(GPOP_EINVAL, "NULL graph");
    if (g->prog < 0) return fail(GPOP_ESTATE, "gpop_state_init not called");
    if (kind != GPOP_SEL_FORCE_SC && kind != GPOP_SEL_FORCE_PC)
        return fail(GPOP_EINVAL, "probe kind must be GPOP_SEL_FORCE_SC or GPOP_SEL_FORCE_PC");
    hipStream_t st = (hipStream_t)stream;
    const Dev& G = g->G;
    const uint32_t k = G.k;
    const BatchGrid& B = g->probe_grid[kind == GPOP_SEL_FORCE_SC ? 0 : 1];
    hipEvent_t ev[2];
    HIP_OR_RETURN(hipEventCreate(&ev[0]), "event");
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return fail(GPOP_EDEVICE, "event");
    }
    struct Guard {
        hipEvent_t* e;
        ~Guard() {
            (void)hipEventDestroy(e[0]);
            (void)hipEventDestroy(e[1]);
        }
    } guard{ev};
    HIP_OR_RETURN(launch_fill_u8((uint8_t*)G.probe, 3ull * k * 8, 0, st), "clear probe");
    HIP_OR_RETURN(launch_batch_plan(B, st), "probe plan");
    HIP_OR_RETURN(hipEventRecord(ev[0], st), "event");
    if (kind == GPOP_SEL_FORCE_SC) HIP_OR_RETURN(launch_batch_sc(B, g->prog, st), "probe scatter SC");
    else HIP_OR_RETURN(launch_batch_pc(B, g->prog, st), "probe scatter PC");
    HIP_OR_RETURN(hipEventRecord(ev[1], st), "event");
    int rc;
    const Ctrl hc = read_ctrl(g, st, &rc);
    if (rc) return rc;
    std::vector<unsigned long long> acc(3ull * k);
    std::vector<uint32_t> va(k);
    HIP_OR_RETURN(hipMemcpyAsync(acc.data(), G.probe, acc.size() * 8, hipMemcpyDeviceToHost, st), "read probe");
    HIP_OR_RETURN(hipMemcpyAsync(va.data(), G.fVa[hc.pos & 1u], k * 4, hipMemcpyDeviceToHost, st),
                  "read frontier sizes");
    HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
    float ms = 0.f;
    HIP_OR_RETURN(hipEventElapsedTime(&ms, ev[0], ev[1]), "elapsed");
    const double total_us = (double)ms * 1e3;
    double sum = 0.0;
    std::vector<double> wt(k, 0.0);
    for (uint32_t p = 0; p < k; ++p) {
        if (!va[p]) continue;
        wt[p] = kind == GPOP_SEL_FORCE_SC ? (double)acc[p] + (double)acc[k + p] : (double)acc[2 * k + p];
        sum += wt[p];
    }
    if (h_us)
        for (uint32_t p = 0; p < k; ++p) h_us[p] = sum > 0.0 ? (float)(total_us * wt[p] / sum) : 0.f;
    if (h_total_us) *h_total_us = (float)total_us;
    return GPOP_OK;
}

int gpop_scatter(gpop_graph* g, void* stream) {
    if (!g) return fail(GPOP_EINVAL, "NULL graph");
    if (g->prog < 0) return fail(GPOP_ESTATE, "gpop_state_init not called");
    hipStream_t st = (hipStream_t)stream;
    const BatchGrid& B = g->grid;
    if (g->limited) {  // lift a limit an earlier gpop_run left behind
        HIP_OR_RETURN(launch_batch_limits(B, 0xFFFFFFFFu, st), "iteration limit");
        g->limited = false;
    }
    int rc;
    if ((rc = timed(g, GPOP_KERNEL_PLAN, st,
                    [&] {
                        hipError_t e = launch_batch_select(B, st);
                        return e != hipSuccess ? e : launch_batch_plan(B, st);
                    },
                    "plan")))
        return rc;
    if ((rc = timed(g, GPOP_KERNEL_SCATTER_SC, st, [&] { return launch_batch_sc(B, g->prog, st); }, "scatter SC")))
        return rc;
    return timed(g, GPOP_KERNEL_SCATTER_PC, st, [&] { return launch_batch_pc(B, g->prog, st); }, "scatter PC");
}

int gpop_gather(gpop_graph* g, void* stream) {
    if (!g) return fail(GPOP_EINVAL, "NULL graph");
    if (g->prog < 0) return fail(GPOP_ESTATE, "gpop_state_init not called");
    hipStream_t st = (hipStream_t)stream;
    int rc = timed(g, GPOP_KERNEL_GATHER, st, [&] { return launch_batch_gather(g->grid, g->prog, st); }, "gather");
    if (rc) return rc;
    return timed(g, GPOP_KERNEL_MERGE, st, [&] { return launch_batch_merge(g->grid, g->prog, st); }, "merge");
}

int gpop_iterate(gpop_graph* g, void* stream) {
    int rc = gpop_scatter(g, stream);
    if (rc) return rc;
    return gpop_gather(g, stream);
}

int gpop_run(gpop_graph* g, uint32_t max_iter, uint32_t* h_iters, void* stream) {
    if (!g) return fail(GPOP_EINVAL, "NULL graph");
    if (g->prog < 0) return fail(GPOP_ESTATE, "gpop_state_init not called");
    hipStream_t st = (hipStream_t)stream;
    HIP_OR_RETURN(launch_batch_limits(g->grid, max_iter, st), "iteration limit");
    g->limited = true;
    Ctrl hc{};
    auto finished = [&](bool& done) {
        int r;
        hc = read_ctrl(g, st, &r);
        done = hc.done != 0;
        return r;
    };
    int rc = GPOP_OK;
    if (g->prof) {
        // profiling brackets every kernel group with events on the stream,
        // so the iterations are launched directly rather than replayed
        const uint64_t passes = (uint64_t)max_iter / g->run.chunk + 2;
        for (uint64_t r = 0; r < passes && !rc; ++r) {
            for (uint32_t c = 0; c < g->run.chunk && !rc; ++c) {
                rc = timed(g, GPOP_KERNEL_PLAN, st,
                           [&] {
                               hipError_t e = launch_batch_select(g->grid, st);
                               return e != hipSuccess ? e : launch_batch_plan(g->grid, st);
                           },
                           "plan");
                if (!rc) rc = timed(g, GPOP_KERNEL_SCATTER_SC, st, [&] { return launch_batch_sc(g->grid, g->prog, st); }, "scatter SC");
                if (!rc) rc = timed(g, GPOP_KERNEL_SCATTER_PC, st, [&] { return launch_batch_pc(g->grid, g->prog, st); }, "scatter PC");
                if (!rc) rc = timed(g, GPOP_KERNEL_GATHER, st, [&] { return launch_batch_gather(g->grid, g->prog, st); }, "gather");
                if (!rc) rc = timed(g, GPOP_KERNEL_MERGE, st, [&] { return launch_batch_merge(g->grid, g->prog, st); }, "merge");
            }
            bool done = false;
            if (!rc) rc = finished(done);
            if (done) break;
        }
    } else {
        rc = runner_run(g->run, g->grid, g->prog, false, false, max_iter, nullptr, st, nullptr, nullptr, finished);
    }
    if (rc) return rc;
    if (h_iters) *h_iters = hc.pos - hc.run_start;
    return GPOP_OK;
}

int gpop_frontier_size(gpop_graph* g, uint64_t* h_out, void* stream) {
    if (!g || !h_out) return fail(GPOP_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    int rc;
    const Ctrl hc = read_ctrl(g, st, &rc);
    if (rc) return rc;
    std::vector<uint32_t> va(g->G.k);
    HIP_OR_RETURN(hipMemcpyAsync(va.data(), g->G.fVa[hc.pos & 1u], g->G.k * 4, hipMemcpyDeviceToHost, st),
                  "read frontier sizes");
    HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
    uint64_t t = 0;
    for (uint32_t x : va) t += x;
    *h_out = t;
    return GPOP_OK;
}

int gpop_iterations(const gpop_graph* g, uint32_t* h_out) {
    if (!g || !h_out) return fail(GPOP_EINVAL, "NULL argument");
    int rc;
    const Ctrl hc = read_ctrl(g, nullptr, &rc);
    if (rc) return rc;
    *h_out = hc.pos;
    return GPOP_OK;
}

int gpop_iter_stats_read(gpop_graph* g, gpop_iter_stats* h_out, uint32_t max_records,
                         uint32_t* h_count, void* stream) {
    if (!g || !h_count || (max_records && !h_out)) return fail(GPOP_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    HIP_OR_RETURN(launch_finalize(g->G, st), "finalize stats");
    int rc;
    const Ctrl hc = read_ctrl(g, st, &rc);
    if (rc) return rc;
    const uint32_t avail = std::min<uint32_t>(hc.pos, kLogCap);
    const uint32_t n = std::min(avail, max_records);
    const uint32_t first = hc.pos - avail;
    for (uint32_t i = 0; i < n; ++i) {
        HIP_OR_RETURN(hipMemcpyAsync(h_out + i, g->G.log + ((first + i) % kLogCap), sizeof(gpop_iter_stats),
                                     hipMemcpyDeviceToHost, st), "read stats");
    }
    HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
    *h_count = n;
    return GPOP_OK;
}

int gpop_modes_read(gpop_graph* g, uint8_t* h_modes, void* stream) {
    if (!g || !h_modes) return fail(GPOP_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    HIP_OR_RETURN(hipMemcpyAsync(h_modes, g->G.mode, g->G.k, hipMemcpyDeviceToHost, st), "read modes");
    HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
    return GPOP_OK;
}

int gpop_check(gpop_graph* g, void* stream) {
    if (!g) return fail(GPOP_EINVAL, "NULL graph");
    hipStream_t st = (hipStream_t)stream;
    uint32_t err = 0, bug = 0;
    HIP_OR_RETURN(hipMemcpyAsync(&err, &g->G.ctrl->err, 4, hipMemcpyDeviceToHost, st), "read error word");
    HIP_OR_RETURN(hipMemcpyAsync(&bug, &g->G.ctrl->bug, 4, hipMemcpyDeviceToHost, st), "read error word");
    HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
    if (bug) return fail(GPOP_EDEVICE, "internal error: inconsistent bin detected by gather");
    if (err) {
        HIP_OR_RETURN(hipMemsetAsync(&g->G.ctrl->err, 0, 4, st), "clear error word");
        HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
        return fail(GPOP_EINVAL, "a vertex id >= V was passed to gpop_set_frontier");
    }
    return GPOP_OK;
}

int gpop_profile_enable(gpop_graph* g, int enable) {
    if (!g) return fail(GPOP_EINVAL, "NULL graph");
    g->prof = enable != 0;
    for (int i = 0; i < GPOP_KERNEL_COUNT; ++i) {
        g->prof_ms[i] = 0;
        g->prof_n[i] = 0;
    }
    return GPOP_OK;
}

int gpop_profile_read(gpop_graph* g, double* h_ms, uint64_t* h_launches, void* stream) {
    if (!g) return fail(GPOP_EINVAL, "NULL graph");
    HIP_OR_RETURN(hipStreamSynchronize((hipStream_t)stream), "sync");
    collect_profile(g);
    for (int i = 0; i < GPOP_KERNEL_COUNT; ++i) {
        if (h_ms) h_ms[i] = g->prof_ms[i];
        if (h_launches) h_launches[i] = g->prof_n[i];
    }
    return GPOP_OK;
}

int gpop_stream_ceiling(int mix, const void* d_src, void* d_dst, uint64_t bytes, void* stream) {
    if (mix != GPOP_STREAM_READ && mix != GPOP_STREAM_COPY && mix != GPOP_STREAM_WIDEN &&
        mix != GPOP_STREAM_SEGMENTS)
        return fail(GPOP_EINVAL, "unknown stream mix %d", mix);
    if (!d_src || !d_dst) return fail(GPOP_EINVAL, "NULL pointer");
    if ((reinterpret_cast<uintptr_t>(d_src) | reinterpret_cast<uintptr_t>(d_dst)) & 15u)
        return fail(GPOP_EINVAL, "pointers must be 16-byte aligned");
    const uint64_t unit = mix == GPOP_STREAM_WIDEN ? 8u : 16u;
    if (bytes == 0 || bytes % unit || bytes >= (1ull << 40))
        return fail(GPOP_EINVAL, "bytes must be a nonzero multiple of %llu below 2^40", (unsigned long long)unit);
    if (mix == GPOP_STREAM_SEGMENTS && (bytes % 512u || ((bytes / 512u) & (bytes / 512u - 1u))))
        return fail(GPOP_EINVAL, "bytes / 512 must be a power of two");
    HIP_OR_RETURN(launch_stream_ceiling(mix, d_src, d_dst, bytes / unit, (hipStream_t)stream), "stream ceiling");
    return GPOP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: many runs of one program, every kernel launched once per iteration
// for all runs, the iteration sequence captured as a HIP graph.
// ---------------------------------------------------------------------------
struct gpop_batch {
    std::vector<gpop_graph*> graphs;
    std::vector<Inst> inst;          // host copy of the run table
    Inst* d_tab = nullptr;
    uint32_t* d_status = nullptr;    // {done, iterations} per run
    std::vector<uint32_t> h_status;
    BatchGrid grid{};
    int prog = -1;
    bool frontier_ok = false;
    Runner run;
};

namespace {

// Per-run buffers (everything an iteration writes); nullptr base: sizing.
size_t carve_run(Dev* D, char* base, const gpop_graph* g) {
    size_t o = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + o : nullptr;
        o += align256(bytes ? bytes : 1);
        return p;
    };
    const Dev& S = g->G;
    const uint64_t k = S.k, q = S.q, kk = k * k;
    const uint64_t E_pad = align256(S.E ? S.E : 1);
    const uint64_t ngt = S.n_gtask ? S.n_gtask : 1;
    // partition-centric messages, the identity words, source-centric message slots
    D->data = (uint32_t*)take((g->M + kIdWords + g->M_sc) * 4);
    D->sc_ids = (uint16_t*)take(E_pad * 2);
    D->sc_w = S.w ? (uint8_t*)take(E_pad) : nullptr;
    D->sc_chunk = (uint32_t*)take(E_pad / kChunk * 4);
    D->sc_cnt = (uint2*)take(kk * 8);
    D->nz = (uint8_t*)take(k * ((k + 63) / 64) * 64);
    D->cact = (uint32_t*)take(k * 4);
    D->pcmask = (uint64_t*)take((k + 63) / 64 * 8);
    D->scmask = (uint64_t*)take((k + 63) / 64 * 8);
    D->sc_tt = (uint2*)take((uint64_t)S.max_sctask * 8);
    D->sc_sh = (uint8_t*)take(k);
    D->sc_t0 = (uint32_t*)take((k + 1) * 4);
    D->gat_ids = (uint32_t*)take(ngt * 4);
    D->gat_ran = (uint32_t*)take((ngt + k) * 4);
    D->mode = (uint8_t*)take(k);
    D->mode_l = (uint8_t*)take(k);
    for (int b = 0; b < 2; ++b) {
        D->flist[b] = (uint16_t*)take(k * q * 2);
        D->fbits[b] = (uint32_t*)take(k * q / 8);
        D->fVa[b] = (uint32_t*)take(k * 4);
        D->fEa[b] = (uint32_t*)take(k * 4);
        D->fpre[b] = (uint32_t*)take(k * q * 4);
        D->dpart[b] = (double*)take(k * 8);
    }
    D->marks = (uint8_t*)take(k * q);
    D->ctrl = (Ctrl*)take(sizeof(Ctrl));
    D->log = (gpop_iter_stats*)take(kLogCap * sizeof(gpop_iter_stats));
    D->probe = (unsigned long long*)take(3 * k * 8);
    D->gpart = (uint32_t*)take(ngt * q * 8);
    D->gflag = (uint32_t*)take(ngt * 4);
    D->mtot = (uint4*)take(k * kMaxMergeChunks * 16);
    return o;
}

size_t batch_header_bytes(uint32_t n) {
    return align256((size_t)n * sizeof(Inst)) + align256(6 * ((size_t)n + 1) * 4) + align256((size_t)n * 8);
}

int batch_check_graphs(gpop_graph* const* graphs, uint32_t n) {
    if (!graphs || n == 0) return fail(GPOP_EINVAL, "a batch needs at least one graph");
    for (uint32_t i = 0; i < n; ++i)
        if (!graphs[i]) return fail(GPOP_EINVAL, "graph %u is NULL", i);
    return GPOP_OK;
}

}  // namespace

int gpop_batch_plan(gpop_graph* const* graphs, uint32_t n, uint64_t* ws_bytes) {
    int rc = batch_check_graphs(graphs, n);
    if (rc) return rc;
    if (!ws_bytes) return fail(GPOP_EINVAL, "ws_bytes is NULL");
    uint64_t t = batch_header_bytes(n);
    for (uint32_t i = 0; i < n; ++i) {
        Dev D{};
        t += carve_run(&D, nullptr, graphs[i]);
    }
    *ws_bytes = t;
    return GPOP_OK;
}

int gpop_batch_create(gpop_graph* const* graphs, uint32_t n, void* d_ws, size_t ws_bytes, void* stream,
                      gpop_batch** out) {
    int rc = batch_check_graphs(graphs, n);
    if (rc) return rc;
    if (!out) return fail(GPOP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(GPOP_EINVAL, "workspace must be 256-byte aligned");
    uint64_t need = 0;
    if ((rc = gpop_batch_plan(graphs, n, &need))) return rc;
    if (ws_bytes < need) return fail(GPOP_ENOMEM, "batch workspace %zu bytes < %llu needed", ws_bytes,
                                     (unsigned long long)need);
    hipStream_t st = (hipStream_t)stream;
    gpop_batch* b = new (std::nothrow) gpop_batch();
    if (!b) return fail(GPOP_ENOMEM, "host allocation failed");
    b->graphs.assign(graphs, graphs + n);
    b->inst.resize(n);
    b->h_status.assign(2 * (size_t)n, 0);
    char* base = (char*)d_ws;
    b->d_tab = (Inst*)base;
    uint32_t* boff = (uint32_t*)(base + align256((size_t)n * sizeof(Inst)));
    b->d_status = (uint32_t*)(base + align256((size_t)n * sizeof(Inst)) + align256(6 * ((size_t)n + 1) * 4));
    size_t o = batch_header_bytes(n);
    std::vector<uint32_t> hb(6 * ((size_t)n + 1), 0);
    const uint32_t sc_cap = std::max<uint32_t>(16u, 2048u / n);
    uint32_t k_max = 0, q_max = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const gpop_graph* g = graphs[i];
        Inst& I = b->inst[i];
        I.G = g->G;  // static arrays shared with the graph
        o += carve_run(&I.G, base + o, g);
        I.P = g->P;
        I.state = nullptr;
        const Dev& S = g->G;
        const uint32_t nb[6] = {(S.k + 31) / 32, std::min<uint32_t>((S.max_sctask + kScWaves - 1) / kScWaves, sc_cap),
                                (S.k + 3) / 4, S.n_pctask, S.n_gtask, S.n_gsplit * merge_chunks(S.q)};
        for (int j = 0; j < 6; ++j) hb[(size_t)j * (n + 1) + i + 1] = hb[(size_t)j * (n + 1) + i] + nb[j];
        k_max = std::max(k_max, S.k);
        q_max = std::max(q_max, S.q);
        HIP_OR_RETURN(hipMemsetAsync(I.G.ctrl, 0, sizeof(Ctrl), st), "clear run control");
        // source-centric counters and marks start clear (each scatter clears
        // what the one before it stamped)
        HIP_OR_RETURN(hipMemsetAsync(I.G.cact, 0, (size_t)S.k * 4, st), "clear column stamps");
        HIP_OR_RETURN(hipMemsetAsync(I.G.sc_cnt, 0, (size_t)S.k * S.k * 8, st), "clear bin counters");
        HIP_OR_RETURN(hipMemsetAsync(I.G.nz, 0, (size_t)S.k * S.kw * 64, st), "clear bin marks");
        HIP_OR_RETURN(hipMemsetD32Async((hipDeviceptr_t)(I.G.data + S.idb), 0xFFFFFFFF, kIdWords, st),
                      "write identity words");
    }
    BatchGrid& B = b->grid;
    B.tab = b->d_tab;
    B.n = n;
    const uint32_t* bo[6];
    uint32_t tot[6];
    for (int j = 0; j < 6; ++j) {
        bo[j] = boff + (size_t)j * (n + 1);
        tot[j] = hb[(size_t)j * (n + 1) + n];
    }
    B.b_select = bo[0];
    B.b_sc = bo[1];
    B.b_clr = bo[2];
    B.b_pc = bo[3];
    B.b_gather = bo[4];
    B.b_merge = bo[5];
    B.nb_select = tot[0];
    B.nb_sc = tot[1];
    B.nb_clr = tot[2];
    B.nb_pc = tot[3];
    B.nb_gather = tot[4];
    B.nb_merge = tot[5];
    B.k_max = k_max;
    B.q_max = q_max;
    B.rounds = graphs[0]->G.combine == GPOP_COMBINE_ROUNDS;
    B.learned = false;
    B.streams = false;
    for (uint32_t i = 0; i < n; ++i) {
        B.learned = B.learned || (graphs[i]->P.selector == GPOP_SEL_LEARNED && !graphs[i]->P.learned_eq1);
        B.streams = B.streams || graphs[i]->G.n_chunks != 0;
    }
    for (uint32_t i = 1; i < n; ++i)
        if (graphs[i]->G.combine != graphs[0]->G.combine) {
            delete b;
            return fail(GPOP_EINVAL, "every graph of a batch must use the same combine option");
        }
    if (sc_lds_bytes(k_max) > (size_t)max_lds_per_block()) {
        delete b;
        return fail(GPOP_ENOTSUP, "k = %u partitions need more LDS than a workgroup has", k_max);
    }
    HIP_OR_RETURN(hipMemcpyAsync(boff, hb.data(), hb.size() * 4, hipMemcpyHostToDevice, st), "write batch grid");
    HIP_OR_RETURN(hipMemcpyAsync(b->d_tab, b->inst.data(), n * sizeof(Inst), hipMemcpyHostToDevice, st),
                  "write run table");
    HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
    *out = b;
    return GPOP_OK;
}

int gpop_batch_destroy(gpop_batch* b) {
    delete b;
    return GPOP_OK;
}

int gpop_batch_state_init(gpop_batch* b, gpop_program prog, const gpop_params* prm, void* const* d_states,
                          void* stream) {
    if (!b || !prm || !d_states) return fail(GPOP_EINVAL, "NULL argument");
    const uint32_t n = (uint32_t)b->inst.size();
    for (uint32_t i = 0; i < n; ++i) {
        if (!d_states[i]) return fail(GPOP_EINVAL, "state %u is NULL", i);
        int rc = check_program(b->graphs[i], prog, &prm[i]);
        if (rc) return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    for (uint32_t i = 0; i < n; ++i) {
        Inst& I = b->inst[i];
        I.P = b->graphs[i]->P;  // the graph's selector settings
        program_params(b->graphs[i], &prm[i], &I.P);
        I.P.probe = 0;
        I.state = (uint32_t*)d_states[i];
        HIP_OR_RETURN(launch_state_init(I.G, I.P, (int)prog, I.state, st), "state init");
    }
    HIP_OR_RETURN(hipMemcpyAsync(b->d_tab, b->inst.data(), n * sizeof(Inst), hipMemcpyHostToDevice, st),
                  "write run table");
    HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
    b->prog = (int)prog;
    b->frontier_ok = true;
    return GPOP_OK;
}

int gpop_batch_set_frontier(gpop_batch* b, uint32_t run, const uint32_t* d_vertices, uint32_t n, void* stream) {
    if (!b) return fail(GPOP_EINVAL, "NULL batch");
    if (run >= b->inst.size()) return fail(GPOP_EINVAL, "run %u out of range", run);
    if (n && !d_vertices) return fail(GPOP_EINVAL, "NULL vertex array");
    if (!b->frontier_ok) return fail(GPOP_ESTATE, "set the frontier after gpop_batch_state_init, before running");
    HIP_OR_RETURN(launch_set_frontier(b->inst[run].G, d_vertices, n, 0, (hipStream_t)stream), "set frontier");
    return GPOP_OK;
}

int gpop_batch_set_frontier_all(gpop_batch* b, uint32_t run, void* stream) {
    if (!b) return fail(GPOP_EINVAL, "NULL batch");
    if (run >= b->inst.size()) return fail(GPOP_EINVAL, "run %u out of range", run);
    if (!b->frontier_ok) return fail(GPOP_ESTATE, "set the frontier after gpop_batch_state_init, before running");
    HIP_OR_RETURN(launch_set_frontier(b->inst[run].G, nullptr, 0, 1, (hipStream_t)stream), "set frontier");
    return GPOP_OK;
}

int gpop_batch_run(gpop_batch* b, uint32_t max_iter, uint32_t flags, uint32_t* h_iters, void* stream) {
    if (!b) return fail(GPOP_EINVAL, "NULL batch");
    if (b->prog < 0) return fail(GPOP_ESTATE, "gpop_batch_state_init not called");
    if (flags & ~(uint32_t)GPOP_BATCH_EAGER) return fail(GPOP_EINVAL, "unknown flags 0x%x", flags);
    hipStream_t st = (hipStream_t)stream;
    const uint32_t n = (uint32_t)b->inst.size();
    b->frontier_ok = false;
    HIP_OR_RETURN(launch_batch_limits(b->grid, max_iter, st), "iteration limit");
    int rc = runner_run(b->run, b->grid, b->prog, false, (flags & GPOP_BATCH_EAGER) != 0, max_iter, b->d_status, st,
                        nullptr, nullptr, [&](bool& done) {
                            if (hipMemcpyAsync(b->h_status.data(), b->d_status, 8 * (size_t)n,
                                               hipMemcpyDeviceToHost, st) != hipSuccess ||
                                hipStreamSynchronize(st) != hipSuccess)
                                return fail(GPOP_EDEVICE, "read run status");
                            done = true;
                            for (uint32_t i = 0; i < n; ++i) done = done && b->h_status[2 * i] != 0;
                            return (int)GPOP_OK;
                        });
    if (rc) return rc;
    if (h_iters)
        for (uint32_t i = 0; i < n; ++i) h_iters[i] = b->h_status[2 * i + 1];
    return GPOP_OK;
}

int gpop_batch_check(gpop_batch* b, void* stream) {
    if (!b) return fail(GPOP_EINVAL, "NULL batch");
    hipStream_t st = (hipStream_t)stream;
    for (size_t i = 0; i < b->inst.size(); ++i) {
        Ctrl hc;
        HIP_OR_RETURN(hipMemcpyAsync(&hc, b->inst[i].G.ctrl, sizeof hc, hipMemcpyDeviceToHost, st), "read control");
        HIP_OR_RETURN(hipStreamSynchronize(st), "sync");
        if (hc.bug) return fail(GPOP_EDEVICE, "internal error in run %zu: inconsistent bin", i);
        if (hc.err) return fail(GPOP_EINVAL, "run %zu: a frontier vertex id was >= V", i);
    }
    return GPOP_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: partition size and bin tile shape per graph and program.
// ---------------------------------------------------------------------------
int gpop_autotune_candidates(gpop_program prog, uint32_t num_vertices, uint64_t num_edges, gpop_options* out,
                             uint32_t cap, uint32_t* n) {
    if (!out || !n) return fail(GPOP_EINVAL, "NULL argument");
    if ((int)prog < 0 || (int)prog > GPOP_PROG_NIBBLE_F32) return fail(GPOP_EINVAL, "unknown program %d", (int)prog);
    (void)num_edges;
    uint32_t c = 0;
    for (uint32_t lp = 12; lp <= 15; ++lp) {
        if (gather_lds_bytes((int)prog, 1u << lp, false) + 2048 > kLdsPerWorkgroup) continue;
        const uint32_t gids[2] = {0, 1u << 16};
        const uint32_t scs[2] = {0, 12};
        for (uint32_t a = 0; a < 2; ++a)
            for (uint32_t b = 0; b < 2; ++b) {
                if (c >= cap) return fail(GPOP_EINVAL, "capacity %u too small", cap);
                gpop_options o{};
                o.log2_part = lp;
                o.gather_task_ids = gids[a];
                o.sc_task_log2 = scs[b];
                out[c++] = o;
            }
        if ((1ull << lp) >= num_vertices) break;  // larger partitions add nothing
    }
    *n = c;
    return GPOP_OK;
}

int gpop_autotune(const gpop_graph_desc* desc, gpop_program prog, const gpop_params* prm,
                  const uint32_t* d_frontier, uint32_t n_frontier, uint32_t max_iter, uint32_t reps,
                  const gpop_options* cands, uint32_t n_cand, void* d_ws, size_t ws_bytes, void* d_state,
                  void* stream, gpop_tune_result* out) {
    if (!desc || !prm || !cands || !d_ws || !d_state || !out) return fail(GPOP_EINVAL, "NULL argument");
    if (n_cand == 0 || n_cand > GPOP_TUNE_MAX) return fail(GPOP_EINVAL, "n_cand must be in [1, %d]", GPOP_TUNE_MAX);
    if (n_frontier && !d_frontier) return fail(GPOP_EINVAL, "NULL frontier");
    if (reps == 0) reps = 1;
    memset(out, 0, sizeof *out);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_OR_RETURN(hipEventCreate(&e0), "event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(GPOP_EDEVICE, "event");
    }
    int best = -1;
    int rc = GPOP_OK;
    for (uint32_t c = 0; c < n_cand && rc == GPOP_OK; ++c) {
        out->run_ms[c] = -1.f;
        out->prep_ms[c] = -1.f;
        gpop_plan_info pi;
        if (gpop_plan(desc, &cands[c], &pi) != GPOP_OK || pi.workspace_bytes > ws_bytes) continue;
        (void)hipEventRecord(e0, st);
        gpop_graph* g = nullptr;
        if (gpop_graph_create(desc, &cands[c], d_ws, ws_bytes, stream, &g) != GPOP_OK) continue;
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float pms = 0.f;
        (void)hipEventElapsedTime(&pms, e0, e1);
        out->prep_ms[c] = pms;
        if (check_program(g, prog, prm) != GPOP_OK) {
            gpop_graph_destroy(g);
            continue;
        }
        float bestc = -1.f;
        for (uint32_t r = 0; r < reps && rc == GPOP_OK; ++r) {
            (void)hipEventRecord(e0, st);
            rc = gpop_state_init(g, prog, prm, d_state, stream);
            if (!rc) rc = d_frontier ? gpop_set_frontier(g, d_frontier, n_frontier, stream)
                                     : gpop_set_frontier_all(g, stream);
            if (!rc) rc = gpop_run(g, max_iter, nullptr, stream);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (!rc && (bestc < 0.f || ms < bestc)) bestc = ms;
        }
        gpop_graph_destroy(g);
        if (rc) break;
        out->run_ms[c] = bestc;
        out->n_tried++;
        if (best < 0 || bestc < out->best_ms) {
            best = (int)c;
            out->best_ms = bestc;
            out->best = cands[c];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (best < 0) return fail(GPOP_ENOTSUP, "no candidate could run");
    return GPOP_OK;
}
