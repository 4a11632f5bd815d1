// Scatter phase: mode selection, source-centric scatter and partition-centric
// scatter (Algorithm 2 scatter phase; Algorithm 3; Sec. 3.2).
#include <algorithm>

#include "launch.h"
#include "select_dev.h"

namespace gpop {

// ---------------------------------------------------------------------------
// Source-centric scatter (Algorithm 2, scatter loop): for active v in
// ascending order, for each neighbouring partition q in ascending order,
// insert {val[v], ids of v's out-neighbours in q} into bin[p][q] (Sec. 3.1.2,
// source-centric mode). A message is a maximal run of one vertex's edges into
// one q (rows are sorted, so it is v's whole neighbourhood in q); its first id
// carries the message-start flag and its value is written once.
//
// GPU form, per iteration: the active vertices of partition p and their
// out-edges, taken in (vertex, edge) order with one work unit per vertex and
// one per edge, are cut into tasks of about C consecutive units (C chosen per
// iteration so that the tasks fill the chip; a hub's row spreads over many
// tasks). One wave owns one task. The task moves both ends of its range
// forward to the next message boundary, so it owns exactly the messages that
// start inside its range and no message is split between tasks. For each
// message the wave reserves its slots with one 64-bit atomic add of
// {1, length} on the bin's {message, id} counter: the old value gives the
// message index and the first id slot at once, so every message is a
// contiguous run of its bin and message indices follow id order, which is
// what the gather's decoding needs. The order of messages inside a bin is the
// order of the reservations; no combine depends on it (minima, and sums in
// exact fixed point). The first reservation in a bin marks it nonempty and
// stamps its column (the two levels of the active list); before the next
// source-centric scatter one pass clears exactly the stamped columns' counters
// and marks. There is no per-task count table and no offset scan, so the
// metadata a task moves is proportional to the messages it writes.
//
// The static partition-node layout (N_i^p(q) in png_src and the static ids
// that partition-centric scatter reuses every iteration, Algorithm 3) is
// built once at preprocessing with every vertex active and a deterministic
// order, in three passes over edge tasks:
//   count pass  - each task counts ids and message starts per destination q;
//   scan pass   - per (p, q), an exclusive scan over the tasks of p gives each
//                 task its base in bin[p][q] (and the bin's totals);
//   write pass  - each task replays its edges and writes at base + rank.
// Inside a task, lanes that hold edges to the same q are grouped with a
// ballot match on the bits of q; only the lowest lane of a group updates the
// wave's LDS counter row, so no two lanes touch the same word.
// ---------------------------------------------------------------------------

// Largest i in [0, n) with key(i) <= x, for a non-decreasing key with
// key(0) <= x. One wave searches 64 ways at once: a round is one load per
// lane, and ceil(log64 n) rounds suffice (instead of log2 n dependent loads).
template <class F>
__device__ __forceinline__ uint32_t wave_search(uint32_t n, uint32_t x, F key) {
    const uint32_t lane = lane_id();
    uint32_t lo = 0;
    while (n > 1) {
        const uint32_t stride = (n + 63u) >> 6;
        const uint32_t o = lane * stride;
        const bool le = o < n && key(lo + o) <= x;
        const uint32_t j = popc64(ballot(le)) - 1u;  // lane 0 always holds
        lo += j * stride;
        n = min(stride, n - j * stride);
    }
    return lo;
}

// The partition that owns task t: largest p with t0[p] <= t (t0 is a
// non-decreasing task prefix over k partitions, t < t0[k]).
__device__ __forceinline__ uint32_t task_owner(const uint32_t* t0, uint32_t k, uint32_t t) {
    return wave_search(k, t, [&](uint32_t i) { return t0[i]; });
}

// Lane of the edge with flat index f among 64 vertices whose edge counts have
// the inclusive prefix incl (the largest o with incl[o - 1] <= f).
__device__ __forceinline__ uint32_t owner_lane(uint32_t incl, uint32_t f) {
    uint32_t o = 0;
#pragma unroll
    for (uint32_t step = 32; step >= 1; step >>= 1) {
        const uint32_t c = __shfl(incl, (int)(o + step - 1), 64);
        if (c <= f) o += step;
    }
    return o;
}


// ---------------------------------------------------------------- build

// Build pass over the edge range [f0, f1) of partition p (every vertex of p,
// edges in CSR order) with one wave.
// WRITE = false: adds per-destination id and message counts to (ci, cm).
// WRITE = true : (ci, cm) hold the task's bases; writes the static layout.
template <bool WRITE>
__device__ __forceinline__ void bld_wave_task(const Dev& G, uint32_t p, uint32_t f0, uint32_t f1,
                                              uint32_t* ci, uint32_t* cm) {
    const uint32_t lane = lane_id();
    const uint32_t k = G.k, s = G.s, qmask = G.q - 1u;
    const uint32_t vbase = p << s;
    const uint32_t nv = min(G.q, G.V - vbase);
    const uint32_t* __restrict__ off = gptr(G.off);
    const uint32_t* __restrict__ cols = gptr(G.cols);
    const uint32_t* __restrict__ rmoff = gptr(G.bin_moff) + (size_t)p * k;
    const uint32_t* __restrict__ rioff = gptr(G.bin_ioff) + (size_t)p * k;
    const uint32_t base_off = off[vbase];
    auto pre = [&](uint32_t i) -> uint32_t { return off[vbase + i] - base_off; };
    // first vertex whose edges reach f0
    const uint32_t lo = wave_search(nv, f0, pre);
    for (uint32_t i0 = lo; i0 < nv; i0 += 64) {
        const uint32_t vl = i0 + lane;
        const bool vv = vl < nv;
        const uint32_t v = vbase + vl;
        const uint32_t rs = vv ? off[v] : 0u;
        const uint32_t deg = vv ? off[v + 1] - rs : 0u;
        const uint32_t pr = vv ? rs - base_off : 0u;
        const uint32_t clo = max(pr, f0);
        const uint32_t chi = min(pr + deg, f1);
        const uint32_t cdeg = (vv && chi > clo) ? chi - clo : 0u;
        const uint32_t cst = rs + (clo - pr);
        const uint32_t incl = wave_incl_scan(cdeg);
        const uint32_t total = last_lane(incl);
        for (uint32_t g0 = 0; g0 < total; g0 += 64) {
            const uint32_t f = g0 + lane;
            const bool valid = f < total;
            const uint32_t o = owner_lane(incl, f);
            const uint32_t o_rs = __shfl(rs, (int)o, 64);
            const uint32_t o_cst = __shfl(cst, (int)o, 64);
            const uint32_t o_incl = __shfl(incl, (int)o, 64);
            const uint32_t o_cdeg = __shfl(cdeg, (int)o, 64);
            const uint32_t o_vl = __shfl(vl, (int)o, 64);
            const uint32_t e = o_cst + (f - (o_incl - o_cdeg));
            const uint32_t col = valid ? cols[e] : 0u;
            const uint32_t key = col >> s;
            const bool flag = valid && (e == o_rs || (cols[e - 1] >> s) != key);
            uint64_t peers = ballot(valid);
            for (uint32_t b = 0; b < G.nbits; ++b) {
                const bool bit = (key >> b) & 1u;
                const uint64_t m = ballot(valid && bit);
                peers &= bit ? m : ~m;
            }
            const uint64_t fpeers = ballot(flag) & peers;
            const uint32_t rank_i = popc_lt(peers);
            const uint32_t m_le = popc_lt(fpeers) + (flag ? 1u : 0u);
            uint32_t bi = 0, bm = 0;
            if (valid) {
                bi = ci[key];
                bm = cm[key];
            }
            if (valid && rank_i == 0) {
                ci[key] = bi + popc64(peers);
                cm[key] = bm + popc64(fpeers);
            }
            if (WRITE && valid) {
                const uint32_t pos = rioff[key] + bi + rank_i;
                const uint32_t midx = bm + m_le - 1u;
                // positions must stay inside the capacity the count pass gave bin[p][key]
                if (pos >= rioff[key + 1] || midx >= rmoff[key + 1] - rmoff[key]) {
                    gptr(G.ctrl)->bug = 1;
                } else {
                    if (flag) gptr(G.png_src)[rmoff[key] + midx] = (uint16_t)o_vl;
                    gptr(G.png_ids)[pos] = (uint16_t)((col & qmask) | (flag ? kFlag : 0u));
                    if (gptr(G.w)) gptr(G.png_w)[pos] = gptr(G.w)[e];
                    if ((pos & (kChunk - 1)) == 0) gptr(G.png_chunk)[pos / kChunk] = midx;
                }
            }
        }
        if (i0 + 64 >= nv || pre(i0 + 64) >= f1) break;
    }
}

// Count pass (WRITE = false) and write pass (WRITE = true) of the build tasks.
template <bool WRITE>
__global__ __launch_bounds__(kScWaves * 64) void k_bld_pass(Dev G) {
    const uint32_t k = G.k;
    const uint32_t* __restrict__ t0 = gptr(G.bld_t0);
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    extern __shared__ uint32_t lds[];
    uint32_t* ci = lds + wave * 2 * k;
    uint32_t* cm = ci + k;
    for (uint32_t t = blockIdx.x * kScWaves + wave; t < G.n_bldtask; t += gridDim.x * kScWaves) {
        uint2* __restrict__ tc = gptr(G.sc_tc) + (size_t)t * k;
        for (uint32_t j = lane; j < k; j += 64) {
            if constexpr (WRITE) {
                const uint2 b = tc[j];
                cm[j] = b.x;
                ci[j] = b.y;
            } else {
                cm[j] = 0;
                ci[j] = 0;
            }
        }
        const uint32_t p = task_owner(t0, k, t);
        const uint32_t f0 = (t - t0[p]) << G.sc_shift;
        const uint32_t f1 = min(f0 + (1u << G.sc_shift), gptr(G.part_E)[p]);
        bld_wave_task<WRITE>(G, p, f0, f1, ci, cm);
        if constexpr (!WRITE) {
            for (uint32_t j = lane; j < k; j += 64) tc[j] = make_uint2(cm[j], ci[j]);
        }
    }
}

// Scan pass of the build: per source partition p (one workgroup) and each
// destination q, exclusive scan of the task counts over the tasks of p (in
// place), giving each task its base in bin[p][q]; the totals are the bin's
// message and id counts. 16 strips of tasks x 64 destinations per round:
// strip sums are scanned in LDS, then each strip rewrites its counts as
// bases. Loads go in batches of 8 so that a strip keeps several in flight.
__global__ __launch_bounds__(1024) void k_bld_scan(Dev G) {
    const uint32_t p = blockIdx.x, k = G.k;
    const uint32_t* __restrict__ t0 = gptr(G.bld_t0);
    const uint32_t tb = t0[p], n = t0[p + 1] - tb;
    const uint32_t tid = threadIdx.x, ql = tid & 63u, strip = tid >> 6;
    __shared__ uint32_t s_m[16][64], s_i[16][64];
    const uint32_t per = (n + 15u) / 16u;
    const uint32_t a = min(strip * per, n), b = min(a + per, n);
    for (uint32_t q0 = 0; q0 < k; q0 += 64) {
        const uint32_t q = q0 + ql;
        const bool qin = q < k;
        uint2* __restrict__ col = gptr(G.sc_tc) + (size_t)tb * k + q;
        uint32_t sm = 0, si = 0;
        if (qin) {
            uint32_t t = a;
            for (; t + 8u <= b; t += 8u) {
                uint2 c[8];
#pragma unroll
                for (uint32_t j = 0; j < 8; ++j) c[j] = col[(size_t)(t + j) * k];
#pragma unroll
                for (uint32_t j = 0; j < 8; ++j) {
                    sm += c[j].x;
                    si += c[j].y;
                }
            }
            for (; t < b; ++t) {
                const uint2 c = col[(size_t)t * k];
                sm += c.x;
                si += c.y;
            }
        }
        s_m[strip][ql] = sm;
        s_i[strip][ql] = si;
        __syncthreads();
        uint32_t rm = 0, ri = 0, tm = 0, ti = 0;
        for (uint32_t w = 0; w < 16; ++w) {
            if (w < strip) {
                rm += s_m[w][ql];
                ri += s_i[w][ql];
            }
            tm += s_m[w][ql];
            ti += s_i[w][ql];
        }
        __syncthreads();
        if (qin) {
            uint32_t t = a;
            for (; t + 8u <= b; t += 8u) {
                uint2 x[8];
#pragma unroll
                for (uint32_t j = 0; j < 8; ++j) x[j] = col[(size_t)(t + j) * k];
#pragma unroll
                for (uint32_t j = 0; j < 8; ++j) {
                    col[(size_t)(t + j) * k] = make_uint2(rm, ri);
                    rm += x[j].x;
                    ri += x[j].y;
                }
            }
            for (; t < b; ++t) {
                const uint2 x = col[(size_t)t * k];
                col[(size_t)t * k] = make_uint2(rm, ri);
                rm += x.x;
                ri += x.y;
            }
            if (strip == 0) {
                gptr(G.cnt_m)[(size_t)p * k + q] = tm;
                gptr(G.cnt_i)[(size_t)p * k + q] = ti;
            }
        }
    }
}

size_t sc_lds_bytes(uint32_t k) { return (size_t)kScWaves * 2 * k * 4; }

hipError_t launch_sc_build(const Dev& G, int fill, hipStream_t st) {
    const size_t lds = sc_lds_bytes(G.k);
    const uint32_t blocks = std::min<uint32_t>((G.n_bldtask + kScWaves - 1) / kScWaves, 2048u);
    hipError_t e = hipSuccess;
    if (fill) {
        if (blocks == 0) return hipSuccess;
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bld_pass<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_bld_pass<true>, dim3(blocks), dim3(kScWaves * 64), lds, st, G);
        return hipGetLastError();
    }
    if (blocks) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bld_pass<false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_bld_pass<false>, dim3(blocks), dim3(kScWaves * 64), lds, st, G);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // the scan also writes the zero counts of bins without edges
    hipLaunchKernelGGL(k_bld_scan, dim3(G.k), dim3(1024), 0, st, G);
    return hipGetLastError();
}

// ------------------------------------------------------------ iterations

// First edge of the run (the stretch of a sorted row into one partition) that
// edge e of the row starting at rs belongs to; key = cols[e] >> s.
// Wave-uniform.
__device__ __forceinline__ uint32_t run_start(const uint32_t* __restrict__ cols, uint32_t rs, uint32_t e,
                                              uint32_t key, uint32_t s) {
    if ((cols[rs] >> s) == key) return rs;
    // the last edge before the run: largest j with cols[rs + j] >> s <= key - 1
    const uint32_t j = wave_search(e - rs + 1u, key - 1u, [&](uint32_t i) { return cols[rs + i] >> s; });
    return rs + j + 1u;
}

// First piece boundary at or after unit x of a partition's source-centric
// units (end: their number). A piece is at most kPiece edges of one run,
// starting at the run's start or kPiece, 2 kPiece, ... edges after it. The
// boundary is x itself if x is a vertex's unit or a piece's first edge, else
// the end of the piece x falls in. r_out: the run start of the boundary's edge
// (when the boundary is an edge). Wave-uniform.
__device__ __forceinline__ uint32_t sc_cut(uint32_t x, uint32_t end, uint32_t nact, uint32_t vbase,
                                           uint32_t s, const uint32_t* __restrict__ off,
                                           const uint32_t* __restrict__ cols,
                                           const uint16_t* __restrict__ alist,
                                           const uint32_t* __restrict__ fpre, uint32_t& r_out) {
    r_out = 0;
    if (x >= end) return end;
    const uint32_t i = wave_search(nact, x, [&](uint32_t j) { return fpre[j] + j; });
    const uint32_t u = fpre[i] + i;  // the vertex's own unit; its edges follow
    if (x == u) return x;
    const uint32_t v = vbase + alist[i];
    const uint32_t rs = off[v], re = off[v + 1];
    const uint32_t e = rs + (x - u - 1u);
    const uint32_t key = cols[e] >> s;
    const uint32_t r0 = e == rs ? rs : run_start(cols, rs, e, key, s);
    r_out = r0;
    if (((e - r0) & (kPiece - 1u)) == 0) return x;
    // the piece ends at the next multiple of kPiece after its run start, or
    // earlier where the run ends
    const uint32_t lim = min(r0 + ((e - r0) | (kPiece - 1u)) + 1u, re);
    uint32_t y = e + 1u;
    for (; y < lim; y += 64u) {
        const uint32_t yy = y + lane_id();
        const uint64_t stop = ballot(yy >= lim || (cols[yy] >> s) != key);
        if (stop) {
            y += (uint32_t)__builtin_ctzll(stop);
            break;
        }
    }
    y = min(y, lim);
    if (y < re) r_out = (cols[y] >> s) == key ? r0 : y;
    return x + (y - e);
}

// How a task reserves its pieces' slots.
enum ScKind : int {
    SC_DIRECT = 0,  // one global atomic per piece
    SC_COUNT = 1,   // pass 1 of a large task: per-bin totals in the wave's LDS row
    SC_WRITE = 2,   // pass 2: slots from the row, which holds the task's bases
};

// One source-centric task: the units [f0, f1) of partition p moved to piece
// boundaries (see above). n_msg / n_ids count the messages (runs) started and
// the ids written. row: the wave's LDS row of k {message, id} words
// (SC_COUNT, SC_WRITE).
template <int PROG, int KIND>
__device__ __forceinline__ void sc_task(const Dev& G, const uint32_t* __restrict__ state, uint32_t p,
                                        uint32_t f0, uint32_t f1, uint32_t end, uint32_t nact,
                                        uint32_t stamp, const uint16_t* __restrict__ alist,
                                        const uint32_t* __restrict__ fpre, uint32_t& n_msg,
                                        uint32_t& n_ids, unsigned long long* row) {
    const uint32_t lane = lane_id();
    const uint32_t k = G.k, s = G.s, qmask = G.q - 1u;
    const uint32_t vbase = p << s;
    const uint32_t* __restrict__ off = gptr(G.off);
    const uint32_t* __restrict__ cols = gptr(G.cols);
    const uint32_t* __restrict__ rioff = gptr(G.bin_ioff) + (size_t)p * k;
    const uint32_t* __restrict__ smor = gptr(G.sc_mor) + (size_t)p * k;  // row p: cached
    unsigned long long* __restrict__ cnt = reinterpret_cast<unsigned long long*>(gptr(G.sc_cnt));
    uint32_t r_first, r_unused;
    const uint32_t b0 = sc_cut(f0, end, nact, vbase, s, off, cols, alist, fpre, r_first);
    const uint32_t b1 = sc_cut(f1, end, nact, vbase, s, off, cols, alist, fpre, r_unused);
    if (b0 >= b1) return;
    auto pre = [&](uint32_t i) -> uint32_t { return fpre[i] + i; };
    const uint64_t below_eq = lane == 63u ? ~0ull : (2ull << lane) - 1ull;  // lanes <= this one
    // first active vertex whose units reach b0
    const uint32_t lo = wave_search(nact, b0, pre);
    for (uint32_t i0 = lo; i0 < nact; i0 += 64) {
        const uint32_t ii = i0 + lane;
        const bool vv = ii < nact;
        const uint32_t v = vbase + (vv ? (uint32_t)alist[ii] : 0u);
        const uint32_t rs = vv ? off[v] : 0u;
        const uint32_t deg = vv ? off[v + 1] - rs : 0u;
        const uint32_t pr = vv ? pre(ii) : 0u;
        const uint32_t clo = max(pr + 1u, b0);
        const uint32_t chi = min(pr + 1u + deg, b1);
        const uint32_t cdeg = (vv && chi > clo) ? chi - clo : 0u;
        const uint32_t cst = rs + (clo - pr - 1u);
        const uint32_t val = (KIND != SC_COUNT && cdeg) ? scatter_value<PROG>(G, state, v) : 0u;
        const uint32_t incl = wave_incl_scan(cdeg);
        const uint32_t total = last_lane(incl);
        // carried from the previous 64 edges: the open piece (first id slot,
        // flat index of its first edge, message index) and the open run's
        // first edge (the task's first edge may lie inside a run)
        uint32_t c_slot = 0, c_f = 0, c_m = 0, c_rs = i0 == lo ? r_first : 0u;
        for (uint32_t g0 = 0; g0 < total; g0 += 64) {
            const uint32_t f = g0 + lane;
            const bool valid = f < total;
            const uint32_t o = owner_lane(incl, f);
            const uint32_t o_rs = __shfl(rs, (int)o, 64);
            const uint32_t o_cst = __shfl(cst, (int)o, 64);
            const uint32_t o_incl = __shfl(incl, (int)o, 64);
            const uint32_t o_cdeg = __shfl(cdeg, (int)o, 64);
            const uint32_t o_val = __shfl(val, (int)o, 64);
            const uint32_t e = o_cst + (f - (o_incl - o_cdeg));
            const uint32_t col = valid ? cols[e] : 0u;
            // the edge before (same row) for the run-start test, loaded together with it
            const uint32_t prevc = (valid && e != o_rs) ? cols[e - 1] : 0u;
            const uint32_t key = col >> s;
            // bounds of bin[p][key] (ids and message slots), loaded before the
            // reservation below so that they are in flight together with it
            uint32_t ib = 0, iend = 0, mb = 0, mend = 0;
            if (KIND != SC_COUNT && valid) {
                ib = rioff[key];
                iend = rioff[key + 1];
                mb = smor[key];
                mend = smor[key + 1];
            }
            // run starts, then piece starts: kPiece-aligned offsets from the run start
            const bool rflag = valid && (e == o_rs || (prevc >> s) != key);
            const uint64_t rfm = ballot(rflag);
            const uint64_t rmine = rfm & below_eq;
            const uint32_t r_e = __shfl(e, (int)(rmine ? 63u - (uint32_t)__builtin_clzll(rmine) : 0u), 64);
            const uint32_t r0 = rmine ? r_e : c_rs;
            const bool flag = valid && ((e - r0) & (kPiece - 1u)) == 0;
            const uint64_t fm = ballot(flag);
            n_msg += popc64(rfm);
            n_ids += popc64(ballot(valid));
            if (rfm) c_rs = readlane_u32(e, 63u - (uint32_t)__builtin_clzll(rfm));
            // A piece that starts here ends at the next start in these 64
            // edges; the last one may run on, to the end of its vertex's edges
            // in the task, the end of its run or kPiece edges.
            const uint32_t lf = fm ? 63u - (uint32_t)__builtin_clzll(fm) : 0u;
            uint32_t len_last = 0;
            if (fm) {
                const uint32_t fl = g0 + lf;
                const uint32_t el = readlane_u32(e, lf), kl = readlane_u32(key, lf);
                const uint32_t lim = min(el + kPiece, el + (readlane_u32(o_incl, lf) - fl));
                uint32_t y = el + (g0 + 64u - fl);  // its first edge after these 64
                for (; y < lim; y += 64u) {
                    const uint32_t yy = y + lane;
                    const uint64_t stop = ballot(yy >= lim || (cols[yy] >> s) != kl);
                    if (stop) {
                        y += (uint32_t)__builtin_ctzll(stop);
                        break;
                    }
                }
                len_last = min(y, lim) - el;
            }
            const uint64_t after = fm & ~below_eq;
            unsigned long long old = 0;
            if (flag) {
                const uint32_t len = after ? (uint32_t)__builtin_ctzll(after) - lane : len_last;
                const unsigned long long add = 1ull | ((unsigned long long)len << 32);
                if constexpr (KIND == SC_DIRECT) {
                    old = atomicAdd(cnt + (size_t)key * k + p, add);
                    if (old == 0ull) {  // first piece of the bin this iteration
                        gptr(G.nz)[(size_t)key * G.kw * 64u + p] = 1;
                        gptr(G.cact)[key] = stamp;
                    }
                } else {
                    old = atomicAdd(row + key, add);  // LDS
                }
            }
            if constexpr (KIND == SC_COUNT) continue;
            const uint32_t o_slot = (uint32_t)(old >> 32), o_m = (uint32_t)old;
            // each edge belongs to the latest piece start at or below its lane
            const uint64_t mine = fm & below_eq;
            const uint32_t own = mine ? 63u - (uint32_t)__builtin_clzll(mine) : 0u;
            const uint32_t s_slot = __shfl(o_slot, (int)own, 64), s_m = __shfl(o_m, (int)own, 64);
            const uint32_t slot = mine ? s_slot + (lane - own) : c_slot + (f - c_f);
            const uint32_t midx = mine ? s_m : c_m;
            if (fm) {
                c_slot = readlane_u32(o_slot, lf);
                c_m = readlane_u32(o_m, lf);
                c_f = g0 + lf;
            }
            if (valid) {
                const uint32_t icap = iend - ib, mcap = mend - mb;
                // the reservation must stay inside the capacity of bin[p][key]
                if (slot >= icap || midx >= mcap) {
                    gptr(G.ctrl)->bug = 1;
                } else {
                    const uint32_t pos = ib + slot;
                    if (flag) gptr(G.data)[mb + midx] = o_val;
                    gptr(G.sc_ids)[pos] = (uint16_t)((col & qmask) | (flag ? kFlag : 0u));
                    if constexpr (is_weighted(PROG)) gptr(G.sc_w)[pos] = gptr(G.w)[e];
                    if ((pos & (kChunk - 1)) == 0) gptr(G.sc_chunk)[pos / kChunk] = midx;
                }
            }
        }
        if (i0 + 64 >= nact || pre(i0 + 64) >= b1) break;
    }
}

// The iteration index: the plan has already advanced pos, except in a probe.
__device__ __forceinline__ uint32_t scatter_it(const Inst& I) { return gptr(I.G.ctrl)->pos - (I.P.probe ? 0u : 1u); }

// The source-centric tasks of an iteration. AGG = false: one global atomic per
// piece. AGG = true (iterations whose tasks are large next to k, where a task
// holds many pieces per bin): the wave counts its pieces per bin in its LDS
// row, reserves each bin's share with one global atomic, then walks the task
// again and takes slots from the row. The plan picks one of the two per
// iteration; the other kernel returns at once.
template <int PROG, bool AGG>
__global__ __launch_bounds__(kScWaves * 64) void kb_sc_scatter(const Inst* __restrict__ tab,
                                                               const uint32_t* __restrict__ boff,
                                                               uint32_t n) {
    const uint32_t bi = batch_find(boff, n, blockIdx.x);
    const Inst& I = tab[bi];
    const Dev& G = I.G;
    const Ctrl* C = gptr(G.ctrl);
    if (C->done || (C->sc_agg != 0u) != AGG) return;
    const uint32_t it = scatter_it(I), cur = it & 1u;
    // the gather of this iteration looks for the stamp; a probe's (never
    // gathered) must still be nonzero, so that the next clear finds it
    const uint32_t stamp = I.P.probe ? C->pos | 0x80000000u : C->pos;
    const uint32_t ntask = C->n_sctask, nblk = boff[bi + 1] - boff[bi];
    const uint32_t* __restrict__ t0 = gptr(G.sc_t0);
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t k = G.k;
    extern __shared__ unsigned long long sc_rows[];
    unsigned long long* row = AGG ? sc_rows + (size_t)wave * k : nullptr;
    if constexpr (AGG)
        for (uint32_t j = lane; j < k; j += 64u) row[j] = 0ull;
    for (uint32_t t = (blockIdx.x - boff[bi]) * kScWaves + wave; t < ntask; t += nblk * kScWaves) {
        const uint64_t t_beg = I.P.probe ? wall_clock64() : 0;
        const uint32_t p = task_owner(t0, k, t);
        const uint32_t sh = gptr(G.sc_sh)[p];
        const uint32_t nact = gptr(G.fVa[cur])[p];
        const uint32_t end = gptr(G.fEa[cur])[p] + nact;
        const uint32_t f0 = (t - t0[p]) << sh;
        const uint32_t f1 = min(f0 + (1u << sh), end);
        const uint32_t vbase = p << G.s;
        const uint16_t* __restrict__ alist = gptr(G.flist[cur]) + vbase;
        const uint32_t* __restrict__ fpre = gptr(G.fpre[cur]) + vbase;
        uint32_t n_msg = 0, n_ids = 0;
        if constexpr (!AGG) {
            sc_task<PROG, SC_DIRECT>(G, gptr(I.state), p, f0, f1, end, nact, stamp, alist, fpre, n_msg, n_ids,
                                     nullptr);
        } else {
            uint32_t u0 = 0, u1 = 0;
            sc_task<PROG, SC_COUNT>(G, gptr(I.state), p, f0, f1, end, nact, stamp, alist, fpre, u0, u1, row);
            // the task's share of each bin it writes: one reservation per bin;
            // the row then holds the task's bases
            unsigned long long* __restrict__ cnt = reinterpret_cast<unsigned long long*>(gptr(G.sc_cnt));
            for (uint32_t j = lane; j < k; j += 64u) {
                const unsigned long long c = row[j];
                if (c == 0ull) continue;
                const unsigned long long old = atomicAdd(cnt + (size_t)j * k + p, c);
                if (old == 0ull) {  // first pieces of the bin this iteration
                    gptr(G.nz)[(size_t)j * G.kw * 64u + p] = 1;
                    gptr(G.cact)[j] = stamp;
                }
                row[j] = old;
            }
            sc_task<PROG, SC_WRITE>(G, gptr(I.state), p, f0, f1, end, nact, stamp, alist, fpre, n_msg, n_ids,
                                    row);
            for (uint32_t j = lane; j < k; j += 64u) row[j] = 0ull;
        }
        if (lane == 0) {
            gptr(G.sc_tt)[t] = make_uint2(n_msg, n_ids);
            if (I.P.probe)  // one wave's time, charged to its partition
                atomicAdd(gptr(G.probe) + k + p, (unsigned long long)(wall_clock64() - t_beg));
        }
    }
}

// Before a source-centric scatter: the counters and nonempty marks of every
// column an earlier one stamped go back to zero, then the stamps. One wave
// per column; an unstamped column costs one load.
__global__ __launch_bounds__(256) void kb_sc_clear(const Inst* __restrict__ tab,
                                                   const uint32_t* __restrict__ boff, uint32_t n) {
    const uint32_t bi = batch_find(boff, n, blockIdx.x);
    const Dev& G = tab[bi].G;
    if (gptr(G.ctrl)->done) return;
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t nblk = boff[bi + 1] - boff[bi];
    const uint32_t nw = G.kw * 8u;  // 8-partition words of a column's marks
    for (uint32_t q = (blockIdx.x - boff[bi]) * 4u + wave; q < G.k; q += nblk * 4u) {
        if (gptr(G.cact)[q] == 0u) continue;
        uint64_t* __restrict__ mw = reinterpret_cast<uint64_t*>(gptr(G.nz) + (size_t)q * G.kw * 64u);
        uint2* __restrict__ c = gptr(G.sc_cnt) + (size_t)q * G.k;
        for (uint32_t j = lane; j < nw; j += 64u) {
            const uint64_t m = mw[j];
            if (!m) continue;
            mw[j] = 0;
            for (uint32_t b = 0; b < 8u; ++b)
                if ((m >> (8u * b)) & 1u) c[8u * j + b] = make_uint2(0u, 0u);
        }
        if (lane == 0) gptr(G.cact)[q] = 0u;
    }
}


// ---------------------------------------------------------------------------
// Partition-centric scatter (Algorithm 3): for every q and every v in
// N_i^p(q), write val[v] into bin[p][q]. The static source list png_src makes
// this a pure stream: slot i of the partition's message range gets the value
// of source png_src[i]. The partition's outgoing values are staged once in
// LDS (the partition's vertex data is the cached working set), inactive
// vertices contribute the combine identity. Work is cut into static slices of
// a partition's slots (their length chosen per graph when it is built), so
// hub partitions spread over many workgroups.
// ---------------------------------------------------------------------------
// Partition-centric workgroup: the partition's values sit in LDS (q words), so
// two workgroups fit a CU; 16 waves each keep enough loads in flight.
constexpr uint32_t kPcT = 1024;

template <int PROG>
__device__ __forceinline__ void pc_body(const Dev& G, const Params& P, const uint32_t* __restrict__ state,
                                        uint32_t it, uint32_t task) {
    if (gptr(G.ctrl)->done) return;
    const uint4 t = gptr(G.pctask)[task];
    const uint32_t p = t.x;
    if (gptr(G.mode)[p] != GPOP_MODE_PC) return;
    uint64_t t_beg = 0;
    if (P.probe) {
        __syncthreads();
        t_beg = wall_clock64();
    }
    const uint32_t cur = it & 1u;
    const uint32_t vbase = p << G.s;
    const uint32_t nv = min(G.q, G.V - vbase);
    extern __shared__ uint32_t mv[];
    const uint32_t* __restrict__ bits = gptr(G.fbits[cur]) + (vbase >> 5);
    for (uint32_t v = threadIdx.x; v < nv; v += kPcT)
        mv[v] = test_bit(bits, v) ? scatter_value<PROG>(G, state, vbase + v) : ident_of<PROG>();
    __syncthreads();
    const uint16_t* __restrict__ src = gptr(G.png_src);
    uint32_t* __restrict__ data = gptr(G.data);
    // aligned middle in groups of 4 slots (8-byte source loads, 16-byte
    // stores), two groups per thread per step
    const uint32_t a = t.y, b = t.z;
    const uint32_t a4 = min((a + 3u) & ~3u, b);
    for (uint32_t i = a + threadIdx.x; i < a4; i += kPcT) data[i] = mv[src[i]];
    const uint32_t b4 = a4 + ((b - a4) & ~3u);
    auto group = [&](uint32_t i) {
        const uint2 sv = *reinterpret_cast<const uint2*>(src + i);
        uint4 o;
        o.x = mv[sv.x & 0xFFFFu];
        o.y = mv[sv.x >> 16];
        o.z = mv[sv.y & 0xFFFFu];
        o.w = mv[sv.y >> 16];
        *reinterpret_cast<uint4*>(data + i) = o;
    };
    uint32_t i = a4 + 4u * threadIdx.x;
    for (; i + 4u * kPcT < b4; i += 8u * kPcT) {
        const uint2 s0 = *reinterpret_cast<const uint2*>(src + i);
        const uint2 s1 = *reinterpret_cast<const uint2*>(src + i + 4u * kPcT);
        uint4 o0, o1;
        o0.x = mv[s0.x & 0xFFFFu];
        o0.y = mv[s0.x >> 16];
        o0.z = mv[s0.y & 0xFFFFu];
        o0.w = mv[s0.y >> 16];
        o1.x = mv[s1.x & 0xFFFFu];
        o1.y = mv[s1.x >> 16];
        o1.z = mv[s1.y & 0xFFFFu];
        o1.w = mv[s1.y >> 16];
        *reinterpret_cast<uint4*>(data + i) = o0;
        *reinterpret_cast<uint4*>(data + i + 4u * kPcT) = o1;
    }
    if (i < b4) group(i);
    for (uint32_t j = b4 + threadIdx.x; j < b; j += kPcT) data[j] = mv[src[j]];
    if (P.probe) {  // every wave's time, charged to the partition
        __syncthreads();
        if (threadIdx.x == 0)
            atomicAdd(gptr(G.probe) + 2 * G.k + p, (unsigned long long)(kPcT / 64) * (wall_clock64() - t_beg));
    }
}

template <int PROG>
__global__ __launch_bounds__(kPcT) void kb_pc(const Inst* __restrict__ tab, const uint32_t* __restrict__ boff,
                                             uint32_t n) {
    const uint32_t i = batch_find(boff, n, blockIdx.x);
    const Inst& I = tab[i];
    pc_body<PROG>(I.G, I.P, gptr(I.state), scatter_it(I), blockIdx.x - boff[i]);
}


// Fills the stats record of iteration it - 1 (source-centric totals and ids
// gathered) from per-partition values the previous iteration wrote. Reads
// mode[], so it must run before the next plan overwrites it.
__device__ __forceinline__ void finalize_prev(const Dev& G, uint32_t it) {
    __shared__ uint64_t red[7][16];
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u, B = blockDim.x;
    uint64_t v[7] = {0, 0, 0, 0, 0, 0, 0};  // sc msgs, sc ids, ids, whole, partial, merged, bins
    const uint32_t nt = G.n_gtask + G.n_gsplit;
    // Loads go out in batches before the sums that use them: the first four
    // task marks per thread, then the source-centric task records.
    constexpr uint32_t kTB = 4;
    auto task_batch = [&](uint32_t t0, uint32_t* ids, uint32_t* ran) {
#pragma unroll
        for (uint32_t u = 0; u < kTB; ++u) {
            const uint32_t t = t0 + u * B;
            ids[u] = t < G.n_gtask ? gptr(G.gat_ids)[t] : 0u;
            ran[u] = t < nt ? gptr(G.gat_ran)[t] : 0u;
        }
    };
    auto task_sum = [&](const uint32_t* ids, const uint32_t* ran) {
#pragma unroll
        for (uint32_t u = 0; u < kTB; ++u) {
            v[2] += ids[u];
            v[3] += (ran[u] & 3u) == 1;
            v[4] += (ran[u] & 3u) == 2;
            v[5] += (ran[u] & 3u) == 3;
            v[6] += ran[u] >> 2;
        }
    };
    uint32_t ids0[kTB], ran0[kTB];
    task_batch(tid, ids0, ran0);
    // source-centric messages and ids: one record per task of that iteration
    const uint32_t nsct = gptr(G.ctrl)->n_sctask;
    constexpr uint32_t kSB = 8;  // task records loaded at once
    for (uint32_t t0 = tid; t0 < nsct; t0 += kSB * B) {
        uint2 c[kSB];
#pragma unroll
        for (uint32_t u = 0; u < kSB; ++u) {
            const uint32_t t = t0 + u * B;
            c[u] = t < nsct ? gptr(G.sc_tt)[t] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (uint32_t u = 0; u < kSB; ++u) {
            v[0] += c[u].x;
            v[1] += c[u].y;
        }
    }
    task_sum(ids0, ran0);
    for (uint32_t t0 = tid + kTB * B; t0 < nt; t0 += kTB * B) {
        uint32_t ids[kTB], ran[kTB];
        task_batch(t0, ids, ran);
        task_sum(ids, ran);
    }
    for (int j = 0; j < 7; ++j) v[j] = wave_sum_u64(v[j]);
    if (lane == 0)
        for (int j = 0; j < 7; ++j) red[j][wave] = v[j];
    __syncthreads();
    if (tid == 0) {
        uint64_t t[7] = {0, 0, 0, 0, 0, 0, 0};
        for (uint32_t w = 0; w < blockDim.x / 64; ++w)
            for (int j = 0; j < 7; ++j) t[j] += red[j][w];
        gpop_iter_stats* r = gptr(G.log) + ((it - 1) % kLogCap);
        r->sc_msgs = t[0];
        r->sc_ids = t[1];
        r->gathered_ids = t[2];
        r->gather_parts = (uint32_t)t[3];
        r->split_tasks = (uint32_t)t[4];
        r->merged_parts = t[5];
        r->gathered_bins = (uint32_t)t[6];
    }
    __syncthreads();
}

// Runs finalize_prev once per iteration: a probe scatter or a stats read may
// come before the plan of the same iteration, and both rewrite what it reads.
__device__ __forceinline__ void finalize_once(const Dev& G, uint32_t it) {
    // Every thread reads the mark; thread 0 rewrites it only after the
    // barriers inside finalize_prev, which each thread reaches after its read.
    if (it > 0 && gptr(G.ctrl)->fin_it < it) {
        finalize_prev(G, it);
        if (threadIdx.x == 0) gptr(G.ctrl)->fin_it = it;
    }
}

__global__ __launch_bounds__(1024) void k_finalize(Dev G) { finalize_once(G, gptr(G.ctrl)->pos); }

// The plan runs as one workgroup of kPlanT threads per run.
constexpr uint32_t kPlanT = 512;
constexpr uint32_t kPlanW = kPlanT / 64;

__device__ __forceinline__ void plan_body(const Dev& G, const Params& P, uint32_t it) {
    Ctrl* C = gptr(G.ctrl);
    if (C->done) return;
    if (!P.probe && it >= C->max_it) {  // the run's iteration limit: pause
        if (threadIdx.x == 0) C->done = 2u;
        return;
    }
    const uint32_t cur = it & 1u;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    // This iteration's inputs of every partition (thread tid holds partitions
    // tid, tid + kPlanT, ...) are loaded before the previous iteration's
    // statistics are finalised, so that all their loads overlap.
    constexpr uint32_t kPJ = 4096 / kPlanT;  // k <= 4096
    uint32_t f_va[kPJ], f_ea[kPJ], f_E[kPJ], f_M[kPJ];
    double f_d[kPJ];
#pragma unroll
    for (uint32_t j = 0; j < kPJ; ++j) {
        const uint32_t p = j * kPlanT + tid;
        const bool in = p < G.k;
        f_va[j] = in ? gptr(G.fVa[cur])[p] : 0u;
        f_ea[j] = in ? gptr(G.fEa[cur])[p] : 0u;
        f_E[j] = in ? gptr(G.part_E)[p] : 0u;
        f_M[j] = in ? gptr(G.part_M)[p] : 0u;
        f_d[j] = in ? gptr(G.dpart[cur])[p] : 0.0;
    }
    finalize_once(G, it);
    __shared__ uint64_t red[10][kPlanW];
    __shared__ double dred[kPlanW];
    __shared__ uint32_t s_w[kPlanW];
    uint64_t va = 0, ea = 0, nsc = 0, npc = 0, pcm = 0, pci = 0, sva = 0, sea = 0, pcv = 0, nfb = 0;
    double dang = 0.0;
    uint32_t msc = 0;  // most active edges of one source-centric partition (the thread's)
    // pass 1: modes and totals; the source-centric work units (active
    // vertices + active out-edges) of each partition go to LDS
    __shared__ uint32_t s_units[4096];  // k <= 4096; 0xFFFFFFFF: not source-centric
#pragma unroll
    for (uint32_t j = 0; j < kPJ; ++j) {
        const uint32_t p0 = j * kPlanT;
        if (p0 >= G.k) break;  // uniform
        const uint32_t p = p0 + tid;
        uint8_t md = GPOP_MODE_NONE;
        if (p < G.k) {
            const uint32_t Va = f_va[j], Ea = f_ea[j], Ep = f_E[j], Mp = f_M[j];
            if (Va) {
                if (P.selector == GPOP_SEL_FORCE_SC) md = GPOP_MODE_SC;
                else if (P.selector == GPOP_SEL_FORCE_PC) md = GPOP_MODE_PC;
                else if (P.selector == GPOP_SEL_LEARNED && P.learned_eq1) {
                    md = analytical_mode_of(G, P, Ep, Mp, Va, Ea);  // the network decides nothing
                    nfb += 1;
                } else if (P.selector == GPOP_SEL_LEARNED) {
                    const uint8_t ml = gptr(G.mode_l)[p];
                    md = ml & (uint8_t)~kFallbackMark;
                    nfb += ml >> 7;
                }
                else md = analytical_mode_of(G, P, Ep, Mp, Va, Ea);
                // interleaved scatter-gather: a partition of another colour
                // class stays active without scattering this iteration
                if (isg_holds(P, p, G.k, it)) md = GPOP_MODE_NONE;
            }
            gptr(G.mode)[p] = md;
            va += Va;
            ea += Ea;
            uint32_t units = 0xFFFFFFFFu;
            if (md == GPOP_MODE_PC) {
                ++npc;
                pcm += Mp;
                pci += Ep;
                pcv += min(G.q, G.V - (p << G.s));
            } else if (md == GPOP_MODE_SC) {
                ++nsc;
                sva += Va;
                sea += Ea;
                msc = max(msc, Ea);
                units = (uint32_t)min<uint64_t>((uint64_t)Va + Ea, 0xFFFFFFFEull);
            }
            s_units[p] = units;
            dang += f_d[j];
        }
        // level-2 masks of the active list: the partitions scattered in each
        // mode, one 64-bit word per wave
        const uint64_t pcw = ballot(md == GPOP_MODE_PC), scw = ballot(md == GPOP_MODE_SC);
        if (lane == 0 && p0 + 64u * wave < G.k) {
            gptr(G.pcmask)[(p0 >> 6) + wave] = pcw;
            gptr(G.scmask)[(p0 >> 6) + wave] = scw;
        }
    }
    // task size of this iteration: about kScTaskTarget tasks, between
    // 2^kScShiftFloor and 2^sc_shift work units
    __shared__ uint64_t s_sc_units[kPlanW];
    __shared__ uint32_t s_msc[kPlanW];  // the wave's largest source-centric partition (active edges)
    {
        const uint64_t w = wave_sum_u64(sva + sea);
        if (lane == 0) s_sc_units[wave] = w;
        for (int o = 32; o > 0; o >>= 1) msc = max(msc, (uint32_t)__shfl_xor((int)msc, o, 64));
        if (lane == 0) s_msc[wave] = msc;
    }
    __syncthreads();
    uint32_t sh;
    {
        uint64_t tot = 0;
        for (uint32_t w = 0; w < kPlanW; ++w) tot += s_sc_units[w];
        const uint32_t hi = G.sc_shift, lo = min(kScShiftFloor, hi);
        const uint64_t per = tot / kScTaskTarget;
        uint32_t l = 0;
        while (l < 40u && (2ull << l) <= per) ++l;  // floor(log2 per) for per >= 1
        sh = per == 0 ? lo : max(lo, min(hi, l));
    }
    // pass 2: tasks of the source-centric partitions, an exclusive scan in
    // partition order
    uint32_t tcarry = 0;  // source-centric tasks of the partitions before this block
    for (uint32_t p0 = 0; p0 < G.k; p0 += kPlanT) {
        const uint32_t p = p0 + tid;
        const uint32_t units = p < G.k ? s_units[p] : 0xFFFFFFFFu;
        uint32_t ntask = 0;
        if (units != 0xFFFFFFFFu) {
            ntask = (uint32_t)(((uint64_t)units + (1ull << sh) - 1ull) >> sh);
            gptr(G.sc_sh)[p] = (uint8_t)sh;
        }
        const uint32_t incl = wave_incl_scan(ntask);
        if (lane == 63) s_w[wave] = incl;
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (uint32_t w = 0; w < kPlanW; ++w) {
            if (w < wave) before += s_w[w];
            tot += s_w[w];
        }
        if (p < G.k) gptr(G.sc_t0)[p] = tcarry + before + incl - ntask;
        tcarry += tot;
        __syncthreads();
    }
    va = wave_sum_u64(va);
    ea = wave_sum_u64(ea);
    nsc = wave_sum_u64(nsc);
    npc = wave_sum_u64(npc);
    pcm = wave_sum_u64(pcm);
    pci = wave_sum_u64(pci);
    sva = wave_sum_u64(sva);
    sea = wave_sum_u64(sea);
    pcv = wave_sum_u64(pcv);
    nfb = wave_sum_u64(nfb);
    dang = wave_sum_f64(dang);
    if (lane == 0) {
        red[0][wave] = va;
        red[1][wave] = ea;
        red[2][wave] = nsc;
        red[3][wave] = npc;
        red[4][wave] = pcm;
        red[5][wave] = pci;
        red[6][wave] = sva;
        red[7][wave] = sea;
        red[8][wave] = pcv;
        red[9][wave] = nfb;
        dred[wave] = dang;
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t t[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        double d = 0.0;
        for (uint32_t w = 0; w < kPlanW; ++w) {
            for (int j = 0; j < 10; ++j) t[j] += red[j][w];
            d += dred[w];
        }
        gptr(G.sc_t0)[G.k] = tcarry;
        C->n_sctask = tcarry;
        // tasks of at least 2k units hold many pieces per bin: reserve per bin
        C->sc_agg = G.scres_mode == GPOP_SCRES_BIN ||
                    (G.scres_mode == GPOP_SCRES_AUTO && (1u << sh) >= 2u * G.k) ? 1u : 0u;
        C->n_pcpart = (uint32_t)t[3];
        // gather reads the partition-centric ids from the column streams
        // when their partitions hold at least half of the edges (a stream
        // chunk is read whole, whatever the mode of its bins' sources)
        C->pc_stream = (G.n_chunks != 0u && t[3] != 0u &&
                        (G.pcs_mode == GPOP_PCSTREAM_ON || 2ull * t[5] >= G.E)) ? 1u : 0u;
        // the wide gather kernel reads the streams and the source-centric bins
        // (small ones one per lane, larger ones one wave each): taken when
        // those hold at most an eighth of the partition-centric ids and no
        // source-centric partition has more than 64 active edges per
        // destination partition on average (a hub partition's bins would each
        // keep one wave busy while its workgroup waits); not with interleaved
        // scatter-gather, whose held-back columns kb_gather keeps
        uint32_t msc_all = 0;
        for (uint32_t w = 0; w < kPlanW; ++w) msc_all = max(msc_all, s_msc[w]);
        C->dense_gather = (C->pc_stream != 0u && P.isg <= 1u &&
                           (t[3] == G.k || (8ull * t[7] <= t[5] && (uint64_t)msc_all <= 64ull * G.k))) ? 1u : 0u;
        if (tcarry > G.max_sctask) {  // cannot happen (the bound covers every task size): stop
            C->bug = 1;
            C->done = 1;
        }
        C->frontier = t[0];
        C->dangling = d;
        if (t[0] == 0) {
            C->done = 1;
        } else if (!P.probe) {
            C->iters = it + 1;
            C->pos = it + 1;
            gpop_iter_stats* r = gptr(G.log) + (it % kLogCap);
            r->active_vertices = t[0];
            r->active_edges = t[1];
            r->sc_parts = (uint32_t)t[2];
            r->pc_parts = (uint32_t)t[3];
            r->pc_msgs = t[4];
            r->pc_ids = t[5];
            r->sc_active_vertices = t[6];
            r->sc_active_edges = t[7];
            r->pc_vertices = t[8];
            r->learned_fallbacks = (uint32_t)t[9];
            r->sc_msgs = 0;
            r->sc_ids = 0;
            r->gathered_ids = 0;
            r->gather_parts = 0;
            r->split_tasks = 0;
            r->merged_parts = 0;
            r->gathered_bins = 0;
        }
    }
}

// One workgroup per run; the iteration index comes from the run's control
// block.
__global__ __launch_bounds__(kPlanT) void kb_plan(const Inst* __restrict__ tab) {
    const Inst& I = tab[blockIdx.x];
    plan_body(I.G, I.P, gptr(I.G.ctrl)->pos);
}

// A single run's plan with its view as a kernel argument: the compiler may
// then re-read view fields instead of keeping them all in registers (read
// from memory they spill); the parameters still come from the run table.
__global__ __launch_bounds__(kPlanT) void k_plan1(Dev G, const Params* __restrict__ pp) {
    const Params P = *pp;
    plan_body(G, P, gptr(G.ctrl)->pos);
}

template <int PROG>
static hipError_t prep_batch_scatter_p(const BatchGrid& B) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kb_sc_scatter<PROG, true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sc_lds_bytes(B.k_max));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kb_pc<PROG>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)(B.q_max * 4));
}

template <int PROG>
static hipError_t launch_batch_sc_p(const BatchGrid& B, hipStream_t st) {
    if (B.nb_sc) {
        hipLaunchKernelGGL(kb_sc_clear, dim3(B.nb_clr), dim3(256), 0, st, B.tab, B.b_clr, B.n);
        hipLaunchKernelGGL((kb_sc_scatter<PROG, false>), dim3(B.nb_sc), dim3(kScWaves * 64), 0, st, B.tab,
                           B.b_sc, B.n);
        hipLaunchKernelGGL((kb_sc_scatter<PROG, true>), dim3(B.nb_sc), dim3(kScWaves * 64),
                           sc_lds_bytes(B.k_max), st, B.tab, B.b_sc, B.n);
    }
    return hipGetLastError();
}

template <int PROG>
static hipError_t launch_batch_pc_p(const BatchGrid& B, hipStream_t st) {
    if (B.nb_pc)
        hipLaunchKernelGGL(kb_pc<PROG>, dim3(B.nb_pc), dim3(kPcT), (size_t)B.q_max * 4, st, B.tab, B.b_pc, B.n);
    return hipGetLastError();
}

#define GPOP_PROG_SWITCH(fn, ...)                             \
    switch (prog) {                                           \
        case P_BFS: return fn<P_BFS>(__VA_ARGS__);            \
        case P_CC: return fn<P_CC>(__VA_ARGS__);              \
        case P_SSSP: return fn<P_SSSP>(__VA_ARGS__);          \
        case P_PR: return fn<P_PR>(__VA_ARGS__);              \
        case P_PPR: return fn<P_PPR>(__VA_ARGS__);            \
        case P_CARRY: return fn<P_CARRY>(__VA_ARGS__);        \
        case P_PARENT: return fn<P_PARENT>(__VA_ARGS__);      \
        case P_NIBBLE: return fn<P_NIBBLE>(__VA_ARGS__);      \
    }                                                         \
    return hipErrorInvalidValue;

hipError_t prepare_batch_scatter(const BatchGrid& B, int prog) { GPOP_PROG_SWITCH(prep_batch_scatter_p, B) }

hipError_t launch_batch_plan(const BatchGrid& B, hipStream_t st) {
    if (B.view) hipLaunchKernelGGL(k_plan1, dim3(1), dim3(kPlanT), 0, st, *B.view, &B.tab->P);
    else hipLaunchKernelGGL(kb_plan, dim3(B.n), dim3(kPlanT), 0, st, B.tab);
    return hipGetLastError();
}

hipError_t launch_batch_sc(const BatchGrid& B, int prog, hipStream_t st) { GPOP_PROG_SWITCH(launch_batch_sc_p, B, st) }

hipError_t launch_batch_pc(const BatchGrid& B, int prog, hipStream_t st) { GPOP_PROG_SWITCH(launch_batch_pc_p, B, st) }

#undef GPOP_PROG_SWITCH


hipError_t launch_finalize(const Dev& G, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, st, G);
    return hipGetLastError();
}

}  // namespace gpop
