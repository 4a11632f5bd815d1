// Device-side layout and wavefront primitives of the gfx950 engine.
//
// Bins (message generation, Sec. 3.1.2): every partition pair (p, q) owns a
// message range [bin_moff, +M(p,q)) of the value array `data` and an id range
// [bin_ioff, +E(p,q)) of an id array, both in row-major (p, q) order so one
// partition's partition-centric scatter writes one contiguous stretch
// (Algorithm 3 writes bin[p][q] before bin[p][q+1]). Ids are 16-bit local
// destination ids with bit 15 marking the first id of a message; the
// partition-centric ids are static (png_ids, written once), the
// source-centric ids are rewritten each iteration (sc_ids) at the same
// positions. A chunk table holds, for every 256-id-aligned position, the
// index of the message containing it, so any 256-id chunk of a bin can be
// decoded on its own.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gpop.h"

namespace gpop {

constexpr uint32_t kChunk = 256;          // ids per decode chunk
constexpr uint32_t kFlag = 0x8000u;       // message-start bit of an id
constexpr uint32_t kLocalMask = 0x7FFFu;  // local destination id bits
constexpr uint32_t kIdentMin = 0xFFFFFFFFu;  // min-combine identity ("no message")
constexpr uint32_t kIdentSum = 0x80000000u;  // sum-combine identity: -0.0f bits
constexpr uint32_t kLogCap = 4096;        // per-iteration stats records
constexpr uint8_t kFallbackMark = 0x80u;  // a learned mode the network left to Eq. 1
constexpr uint32_t kIdWords = 320;        // identity words after the messages (a 256-position chunk plus a lane's 4)
constexpr uint32_t kScWaves = 4;          // independent source-centric task waves per workgroup
constexpr uint32_t kMergeSpan = 1024;     // vertices per workgroup of a split-partition merge
constexpr uint32_t kMaxMergeChunks = 32;  // q / kMergeSpan at the largest partition (2^15)
constexpr double kFix = 1152921504606846976.0;      // 2^60: fixed-point scale of sums
constexpr double kInvFix = 8.673617379884035e-19;   // 2^-60

enum Prog : int {
    P_BFS = GPOP_PROG_BFS_LEVEL,
    P_CC = GPOP_PROG_CC_MINLABEL,
    P_SSSP = GPOP_PROG_SSSP_U32,
    P_PR = GPOP_PROG_PAGERANK_F32,
    P_PPR = GPOP_PROG_PPR_F32,
    P_CARRY = GPOP_PROG_CARRY_BFS,
    P_PARENT = GPOP_PROG_BFS_PARENT,
    P_NIBBLE = GPOP_PROG_NIBBLE_F32,
};

__host__ __device__ constexpr bool is_sum(int prog) { return prog == P_PR || prog == P_PPR || prog == P_NIBBLE; }
__host__ __device__ constexpr bool is_weighted(int prog) { return prog == P_SSSP; }
// gatherFunc sets an unvisited vertex only (BFS parents); the other min
// programs keep any smaller value
__host__ __device__ constexpr bool first_write(int prog) { return prog == P_PARENT; }
// Source-centric tasks per iteration the plan aims for: one per wave of the
// largest scatter grid (2048 workgroups of kScWaves waves).
constexpr uint32_t kScTaskTarget = 8192;
// Smallest source-centric task, log2 of its work units.
constexpr uint32_t kScShiftFloor = 6;
// Source-centric scatter cuts a message into pieces of at most this many
// edges (each with its own flag and value), so no task holds a long one.
constexpr uint32_t kPiece = 256;
// Workgroups that merge one split partition of q vertices.
__host__ __device__ constexpr uint32_t merge_chunks(uint32_t q) { return q > kMergeSpan ? q / kMergeSpan : 1u; }

struct Ctrl {
    uint32_t done;        // bit 0: frontier became empty; bit 1: paused at max_it
    uint32_t iters;       // iterations whose plan found active vertices
    uint32_t err;         // bad vertex id passed to set_frontier
    uint32_t csr_err;     // CSR validation failure code
    uint32_t bug;         // a kernel found an inconsistent bin (internal error)
    uint32_t n_sctask;    // source-centric tasks of the current iteration
    uint64_t frontier;    // sum of V_a at the last plan
    double dangling;      // PageRank-family dangling mass of the current frontier
    uint32_t fin_it;      // records below this iteration are final
    uint32_t pc_stream;   // gather reads partition-centric ids from the column streams
    uint32_t pos;         // iterations run so far (index of the next plan)
    uint32_t max_it;      // a plan at this index pauses the run (done bit 2)
    uint32_t run_start;   // pos when the current run began
    uint32_t n_pcpart;    // partitions scattered partition-centric in the current iteration
    uint32_t sc_agg;      // source-centric tasks reserve per bin (1) or per piece (0)
    uint32_t dense_gather;  // the wide gather kernel takes this iteration (column streams, few SC ids)
    uint32_t pad[46];
};

// Everything the kernels read or write, by value in each launch.
struct Dev {
    uint32_t V, k, s, q;      // vertices, partitions, log2 q, q
    uint32_t kw;              // 64-bit words of a k-bit partition mask
    uint32_t nbits;           // bits needed for a partition id
    uint32_t n_pctask;        // partition-centric scatter tasks (static)
    uint32_t sc_shift;        // log2 of the active edges per source-centric task
    uint32_t max_sctask;      // bound on source-centric tasks per iteration
    uint32_t n_bldtask;       // tasks of the preprocessing build
    uint32_t n_gtask;         // gather tasks (static)
    uint32_t n_gsplit;        // partitions whose gather is split over tasks
    uint32_t combine;         // GPOP_COMBINE_*
    uint32_t whole_ids;       // a split partition with at most this many ids is gathered by one task
    uint32_t pcs_mode;        // GPOP_PCSTREAM_*
    uint32_t scres_mode;      // GPOP_SCRES_*
    uint32_t idb;             // data[idb, idb + kIdWords): combine identities (min and sum), never written
    uint32_t n_chunks;        // chunks of all column streams
    uint64_t E;
    const uint32_t* off;
    const uint32_t* cols;
    const uint8_t* w;
    // static (preprocessing)
    uint32_t* part_E;         // [k] out-edges of partition p
    uint32_t* part_M;         // [k] messages of p when all of it is active
    uint32_t* bin_moff;       // [k*k+1] row-major message offsets
    uint32_t* bin_ioff;       // [k*k+1] row-major id offsets
    uint4* cm;                // [k*k] column-major {moff, ioff, mcnt, icnt}, index q*k+p
    uint64_t* colsrc;         // [k*kw] static: bit p of column q's words set iff bin[p][q] has ids
    uint32_t* spre;           // [k*k] static: 256-id pieces of bins[0..p)[q], index q*k+p
    uint16_t* png_src;        // [M] local source id of each message
    uint16_t* png_ids;        // [E_pad] static ids
    uint8_t* png_w;           // [E_pad] static weights
    uint32_t* png_chunk;      // [E_pad/256]
    uint4* pctask;            // [n_pctask] {p, slot_begin, slot_end, 0}
    // column streams of the partition-centric ids (static; built for
    // partitions of at most 2^14 vertices): column q's chunks are
    // [cs_c0[q], cs_c0[q+1]); chunk c holds stream positions [256c, 256c+256),
    // four per lane of the wave that decodes it. Every bin starts at a
    // multiple of 4 (its last lane is filled with null ids: local id q, no
    // message start), so a lane's four positions always belong to one bin.
    // Bit l of cs_lm[c] marks a bin (or the padding run at a column's end)
    // starting at lane l > 0. Chunk c's entries [cs_tabo[c], cs_tabo[c+1])
    // are, for the bin at position 0 and then each lane start in order,
    // {adj, src | mt << 16}: the data index of a position i is
    // adj[b] + (message starts at positions 1..i), b = lane starts at lanes
    // 1..i/4; src is the source partition (0xFFFF: padding, whose adj points
    // into the identity words) and mt the message starts at positions
    // 1..start.
    uint32_t* cs_c0;          // [k+1]
    uint16_t* cs_ids;         // [n_chunks*256] ids (local id | message-start flag)
    uint8_t* cs_w;            // [n_chunks*256] weights
    uint64_t* cs_lm;          // [n_chunks] lanes that start a bin
    uint32_t* cs_tabo;        // [n_chunks+1]
    uint2* cs_ent;            // [entries + 64]
    uint32_t* bld_t0;         // [k+1] task prefix of the build (all vertices active)
    uint4* gtask;             // [2*n_gtask] {q, p_lo, p_hi, nt<<16|j}, {s0, s1, slot, 0}
    uint4* gsplit;            // [n_gsplit] {q, 0, nt, first slot}
    uint32_t* gpart;          // partial results of split gathers, q (u32) or 2q (u64) words per slot
    uint32_t* gflag;          // [slots] a split task wrote its partial
    uint4* mtot;              // [k*kMaxMergeChunks] per merge chunk {kept, kept out-edges, dangling sum (f64 bits)}
    // per iteration
    uint32_t* data;           // [M] message values
    uint16_t* sc_ids;         // [E_pad]
    uint8_t* sc_w;            // [E_pad]
    uint32_t* sc_chunk;       // [E_pad/256]
    uint2* sc_cnt;            // [k*k] column-major {mcnt, icnt} of SC bins: reservation counters,
                              // zero outside the stamped columns
    uint8_t* nz;              // [k*kw*64] column-major, column stride kw*64: SC bin[p][q] received ids
                              // (1 / 0; valid for partitions scattered source-centric)
    uint32_t* cact;           // [k] column q received SC ids in the iteration with this plan index
                              // (0: its counters and marks are clear)
    uint64_t* pcmask;         // [kw] partitions scattered partition-centric this iteration
    uint64_t* scmask;         // [kw] partitions scattered source-centric this iteration
    uint2* sc_tt;             // [max_sctask] {messages, ids} written by each SC task
    uint32_t* sc_mo;          // [k*k] column-major: data index of SC bin[p][q]'s first message slot
    uint32_t* sc_mor;         // [k*k+1] the same, row-major (scatter), then the end of the last bin
    uint8_t* sc_sh;           // [k] log2 work units per source-centric task of each partition
    uint32_t* sc_t0;          // [k+1] exclusive prefix of SC tasks per partition
    uint2* sc_tc;             // [n_bldtask*k] build: per-(task, q) counts, then bases
    uint32_t* gat_ids;        // [n_gtask] ids combined per gather task
    uint32_t* gat_ran;        // [n_gtask + n_gsplit] 1 whole partition, 2 partial, 3 merge, 0 idle
    uint8_t* mode;            // [k]
    uint16_t* flist[2];       // [k*q] frontier lists (local ids, ascending)
    uint32_t* fbits[2];       // [k*q/32] frontier bitmaps
    uint32_t* fVa[2];         // [k]
    uint32_t* fEa[2];         // [k]
    uint32_t* fpre[2];        // [k*q] active-edge prefix of each frontier entry
    double* dpart[2];         // [k] dangling partial sums
    uint8_t* marks;           // [k*q] set_frontier scratch
    uint32_t* cnt_m;          // [k*k] preprocessing counts, row-major
    uint32_t* cnt_i;          // [k*k]
    uint32_t* scan_tmp;       // scan scratch
    Ctrl* ctrl;
    gpop_iter_stats* log;     // [kLogCap]
    // learned selector
    float* pfill;             // [k] non-empty PNG bins of row p / k
    float* pskew;             // [k] log(max / mean out-degree) of partition p
    uint8_t* mode_l;          // [k] modes the learned selector picked for the next plan
    gpop_mlp_model* mlp;      // the selector's copy of the model
    unsigned long long* probe;  // [3k] wave time of probe tasks: SC count, SC write, PC
};

// Program parameters and the mode model.
struct Params {
    uint32_t root, persist;
    float damping, alpha;
    float eps;                // Nibble threshold
    double inv_n;             // 1 / V
    uint32_t selector;        // gpop_selector
    uint32_t s_i, s_v;        // model element sizes (bytes)
    uint32_t ratio_num, ratio_den;  // BW_PC / BW_SC as a fraction
    uint32_t probe;           // scatter kernels time their tasks into Dev::probe
    uint32_t isg;             // interleaved scatter-gather: colour classes (0 or 1: off)
    uint32_t learned_eq1;     // learned selector whose margin is infinite: Eq. 1 decides every partition
};

// Interleaved scatter-gather (Sec. 3.3) in colour classes: partitions are
// cut into isg contiguous index ranges; iteration it scatters only the
// active partitions of class it mod isg, and every other active partition
// keeps its frontier, so it scatters later with the values the gathers in
// between have already improved.
__host__ __device__ __forceinline__ uint32_t isg_class(uint32_t p, uint32_t k, uint32_t classes) {
    return (uint32_t)(((uint64_t)p * classes) / k);
}
__host__ __device__ __forceinline__ bool isg_holds(const Params& P, uint32_t p, uint32_t k, uint32_t it) {
    return P.isg > 1u && isg_class(p, k, P.isg) != it % P.isg;
}

// One run of a batch: its graph view (static arrays shared with the graph,
// per-run arrays of its own), its parameters and its state array.
struct Inst {
    Dev G;
    Params P;
    uint32_t* state;
};

// A global-memory pointer every lane holds the same value of, made opaque to
// the compiler (it stays a scalar value and keeps its address space).
// A pointer into device memory, the same in every lane, marked as global
// memory. Pointers read from the view in memory are otherwise generic, and
// accesses through them become flat instructions, which also count against
// the LDS wait counter (an LDS read then waits for the flat access as well).
// The value goes through readfirstlane so that the compiler cannot fold the
// address-space casts away.
template <class T>
__device__ __forceinline__ T* gptr(T* p) {
    const uint64_t u = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    typedef __attribute__((address_space(1))) T GlobalT;
    return (T*)(GlobalT*)(((uint64_t)hi << 32) | lo);
}

// Batched launches: instance i owns blocks [boff[i], boff[i+1]) of the grid.
__device__ __forceinline__ uint32_t batch_find(const uint32_t* __restrict__ boff, uint32_t n, uint32_t b) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (boff[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Number of set bits of m among lanes below the calling lane.
__device__ __forceinline__ uint32_t popc_lt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__popcll(m); }

// The value of lane l (l the same in every lane).
__device__ __forceinline__ uint32_t readlane_u32(uint32_t x, uint32_t l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, (int)l);
}

// Inclusive prefix sum over the 64 lanes of a wave.
// Inclusive prefix sum across the wave with DPP: shifts by 1, 2, 4, 8 lanes
// inside each row of 16, then the last lane of row 0 is added to row 1 and
// of row 2 to row 3 (row_bcast:15), then the last lane of row 1 to rows 2
// and 3 (row_bcast:31). Lanes without a source read 0.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return x;
}
// The value of lane 63 (a scalar read, no LDS traffic).
__device__ __forceinline__ uint32_t last_lane(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Wave sums: the DPP inclusive scan of wave_incl_scan, then lane 63's value
// read into a scalar register (the same in every lane). 64-bit values move
// through DPP as two 32-bit halves with the same control. The tree is the
// same on every call, so floating-point sums are reproducible bit for bit.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, ROWS, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, ROWS, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t lane63_u64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) { return last_lane(wave_incl_scan(x)); }
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
    x += dpp_u64<0x111, 0xF>(x);  // row_shr:1
    x += dpp_u64<0x112, 0xF>(x);  // row_shr:2
    x += dpp_u64<0x114, 0xF>(x);  // row_shr:4
    x += dpp_u64<0x118, 0xF>(x);  // row_shr:8
    x += dpp_u64<0x142, 0xA>(x);  // row_bcast:15
    x += dpp_u64<0x143, 0xC>(x);  // row_bcast:31
    return lane63_u64(x);
}
__device__ __forceinline__ double f64_dpp_add(double y, uint64_t b, int step) {
    uint64_t t = 0;
    switch (step) {
        case 0: t = dpp_u64<0x111, 0xF>(b); break;
        case 1: t = dpp_u64<0x112, 0xF>(b); break;
        case 2: t = dpp_u64<0x114, 0xF>(b); break;
        case 3: t = dpp_u64<0x118, 0xF>(b); break;
        case 4: t = dpp_u64<0x142, 0xA>(b); break;
        default: t = dpp_u64<0x143, 0xC>(b); break;
    }
    return y + __longlong_as_double((long long)t);
}
__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
    for (int step = 0; step < 6; ++step) x = f64_dpp_add(x, (uint64_t)__double_as_longlong(x), step);
    return __longlong_as_double((long long)lane63_u64((uint64_t)__double_as_longlong(x)));
}

// 256-id decode pieces touched by the id range [ioff, ioff + icnt).
__host__ __device__ __forceinline__ uint32_t pieces_of(uint32_t ioff, uint32_t icnt) {
    return icnt ? (ioff + icnt - 1u) / kChunk - ioff / kChunk + 1u : 0u;
}

__device__ __forceinline__ bool test_bit(const uint32_t* bits, uint32_t i) {
    return (bits[i >> 5] >> (i & 31)) & 1u;
}

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
    uint32_t c = a + b;
    return c < a ? 0xFFFFFFFFu : c;
}

// scatterFunc of each program for an active vertex v (global id).
template <int PROG>
__device__ __forceinline__ uint32_t scatter_value(const Dev& G, const uint32_t* st, uint32_t v) {
    if constexpr (PROG == P_BFS || PROG == P_CARRY) {
        return st[v] + 1u;
    } else if constexpr (PROG == P_CC || PROG == P_SSSP) {
        return st[v];
    } else if constexpr (PROG == P_PARENT) {
        return v;
    } else if constexpr (PROG == P_NIBBLE) {
        const uint32_t* __restrict__ off = gptr(G.off);
        const uint32_t deg = off[v + 1] - off[v];
        const float x = __uint_as_float(st[v]);
        return __float_as_uint(deg ? (x * 0.5f) / (float)deg : 0.0f);
    } else {
        const uint32_t* __restrict__ off = gptr(G.off);
        uint32_t deg = off[v + 1] - off[v];
        float x = __uint_as_float(st[v]);
        return __float_as_uint(deg ? x / (float)deg : 0.0f);
    }
}

template <int PROG>
__device__ __forceinline__ uint32_t ident_of() {
    return is_sum(PROG) ? kIdentSum : kIdentMin;
}

}  // namespace gpop
