// Gather phase (Algorithm 2: reInit, gather, filter) plus state and frontier
// initialisation.
#include "launch.h"

namespace gpop {

// Gather workgroups are 8 waves; with a 16K-vertex partition of 4-byte state
// two of them fit the 160 KB LDS of a CU, so one can wait on a barrier while
// the other streams bins.
constexpr uint32_t kGT = 512;
constexpr uint32_t kGW = kGT / 64;
// Bins of at most this many ids are gathered one per lane (a task covering
// whole bins only): a sparse frontier spreads few ids over many bins, and a
// 256-id piece per such bin would leave most of its lanes idle.
constexpr uint32_t kSmallBin = 8;

// Words of a partition bitmask (k <= 4096 partitions).
constexpr uint32_t kMaxMaskWords = 64;

// Bits [lo, hi] of 64-bit word w of a partition mask.
__device__ __forceinline__ uint64_t range_bits(uint32_t w, uint32_t lo, uint32_t hi) {
    const uint32_t a = w * 64u, b = a + 63u;
    if (hi < a || lo > b) return 0ull;
    uint64_t m = ~0ull;
    if (lo > a) m &= ~0ull << (lo - a);
    if (hi < b) m &= ~0ull >> (b - hi);
    return m;
}

// Programs whose initFunc keeps vertices active need a per-vertex carry flag
// (the PageRank family keeps it in the top bit of its accumulator).
__host__ __device__ constexpr bool has_carry(int prog) { return prog == P_CARRY; }
constexpr unsigned long long kCarried = 1ull << 63;  // sum programs: vertex was active before scatter

// LDS layout of the gather workgroup (bytes, all offsets 16-aligned). The
// bin-list arrays double as scratch for the frontier masks in the filter.
struct GatherLds {
    size_t state, tag, carry, amask, pcm, bl_ioff, bl_icnt, bl_moff, bl_mcnt, bl_jlo, bl_scan, total;
};

// `rounds`: the atomic-free combine, whose sum programs need a 16-bit tag per
// vertex.
__host__ __device__ inline GatherLds gather_layout(int prog, uint32_t q, bool rounds = false) {
    GatherLds L{};
    size_t o = 0;
    // the state, plus one spare word (index q) that null stream ids combine into
    L.state = o;  o += ((size_t)(q + 1) * (is_sum(prog) ? 8 : 4) + 15) / 16 * 16;
    L.tag = o;    o += (rounds && is_sum(prog)) ? ((size_t)q * 2 + 15) / 16 * 16 : 0;
    L.carry = o;  o += has_carry(prog) ? ((size_t)q + 15) / 16 * 16 : 0;
    L.amask = o;  o += kMaxMaskWords * 8;
    L.pcm = o;    o += kMaxMaskWords * 8;
    L.bl_ioff = o; o += kGT * 4;
    L.bl_icnt = o; o += kGT * 4;
    L.bl_moff = o; o += kGT * 4;
    L.bl_mcnt = o; o += kGT * 4;
    L.bl_jlo = o;  o += kGT * 4;
    L.bl_scan = o; o += (kGT + 4) * 4;
    L.total = o;
    return L;
}

size_t gather_lds_bytes(int prog, uint32_t q, bool rounds) { return gather_layout(prog, q, rounds).total; }

// Exclusive prefix of a 0..7 per-lane count across the wave, from bit-plane
// ballots.
__device__ __forceinline__ uint32_t wave_excl_small(uint32_t c) {
    return popc_lt(ballot(c & 1u)) + 2u * popc_lt(ballot(c & 2u)) + 4u * popc_lt(ballot(c & 4u));
}

template <uint32_t NW>
struct GatherSharedT {
    uint32_t wc[NW], wp[NW], ws[NW], wsm[NW];
    uint64_t r64[NW];
    double rd[NW];
};
using GatherShared = GatherSharedT<kGW>;

// Programs whose frontier can only come from vertices that received a
// message: a partition with no incoming message leaves an empty frontier,
// whatever was active before.
__host__ __device__ constexpr bool msg_only(int prog) { return !is_sum(prog) && !has_carry(prog); }

// reInit frontier: initFunc on the vertices that were active before scatter.
// (Min programs start the on-chip copy at the identity, so initFunc reads the
// stored value.)
template <int PROG, uint32_t NT = kGT>
__device__ __forceinline__ void reinit(const Dev& G, const Params& P, const uint32_t* __restrict__ state,
                                       uint32_t it, uint32_t cq, uint32_t* st32, uint8_t* carry) {
    if constexpr (has_carry(PROG) || is_sum(PROG)) {
        const uint32_t cur = it & 1u;
        const uint32_t vbase = cq << G.s;
        const uint32_t prevVa = gptr(G.fVa[cur])[cq];
        const uint16_t* __restrict__ prev = gptr(G.flist[cur]) + vbase;
        for (uint32_t i = threadIdx.x; i < prevVa; i += NT) {
            const uint32_t u = prev[i];
            if constexpr (PROG == P_CARRY) carry[u] = (it + 1u - state[vbase + u]) < P.persist;
            else reinterpret_cast<unsigned long long*>(st32)[u] |= kCarried;  // value restarts at 0, stays active
        }
    }
}

// filterFunc on carried and newly activated vertices, state write-back and
// compaction of the next frontier (ascending list, bitmap, active-edge
// prefix, V_a, E_a, dangling partial sum). A min-program vertex is newly
// activated when its combined value is below the value still in memory; a
// sum-program vertex when it received a non-zero amount. Wave w owns a
// contiguous vertex range: pass 1 applies the filter, writes the state and
// counts kept vertices and their out-edges (keep masks go to LDS scratch),
// one scan across waves gives every wave its offsets, pass 2 writes the
// frontier.
template <int PROG, uint32_t NW = kGW>
__device__ __forceinline__ void finish_partition(const Dev& G, const Params& P, uint32_t* __restrict__ state,
                                 uint32_t it, uint32_t cq, uint32_t* st32,
                                 unsigned long long* acc, const uint8_t* carry,
                                 uint64_t* kscratch, GatherSharedT<NW>& sh, uint32_t ids_done,
                                 uint32_t task, bool carry_col) {
    constexpr bool SUM = is_sum(PROG);
    // 64-vertex groups per step of pass 1: their global loads are issued together
    constexpr uint32_t U = 8;
    const uint32_t nxt = (it & 1u) ^ 1u;
    const uint32_t vbase = cq << G.s, Q = G.q;
    const uint32_t nv = min(Q, G.V - vbase);
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    const double dang = SUM ? gptr(G.ctrl)->dangling : 0.0;
    const uint32_t* __restrict__ off = gptr(G.off);
    const uint32_t per = ((Q / NW) + 63u) & ~63u;  // vertices per wave, multiple of 64
    const uint32_t wb = wave * per;
    const uint32_t wend = min(wb + per, Q);
    // pass 1 leaves the out-degree of each kept vertex in the LDS slot its
    // value used (sum programs: the upper word of the accumulator)
    uint32_t* degl = SUM ? reinterpret_cast<uint32_t*>(acc) : st32;
    const uint32_t dsh = SUM ? 1u : 0u, dadd = SUM ? 1u : 0u;
    uint32_t cnt = 0, edges = 0;
    double my_d = 0.0;
    for (uint32_t g0 = wb; g0 < wend; g0 += 64u * U) {
        uint32_t mv[U], sv[U], o0[U], o1[U];
        unsigned long long av[U];
        float xv[U];
        bool keep[U], need[U];
#pragma unroll
        for (uint32_t i = 0; i < U; ++i) {
            const uint32_t u = g0 + 64u * i + lane;
            const bool in = g0 + 64u * i < wend && u < nv;
            if constexpr (!SUM) mv[i] = in ? st32[u] : kIdentMin;  // least message (identity: none)
            else av[i] = in ? acc[u] : 0ull;  // an amount arrived, or active before scatter
        }
        if constexpr (!SUM) {
            // a column held back by interleaved scatter-gather keeps its
            // active vertices (the current frontier bitmap), one word per 32
            uint32_t hw[U];
#pragma unroll
            for (uint32_t i = 0; i < U; ++i) {
                const uint32_t u = g0 + 64u * i + lane;
                hw[i] = (carry_col && g0 + 64u * i < wend && u < nv)
                            ? gptr(G.fbits[it & 1u])[(vbase + u) >> 5] : 0u;
            }
#pragma unroll
            for (uint32_t i = 0; i < U; ++i)
                sv[i] = mv[i] != kIdentMin ? state[vbase + g0 + 64u * i + lane] : 0u;
#pragma unroll
            for (uint32_t i = 0; i < U; ++i) {
                const uint32_t u = g0 + 64u * i + lane;
                const bool hit = mv[i] != kIdentMin && (first_write(PROG) ? sv[i] == kIdentMin : mv[i] < sv[i]);
                keep[i] = hit || ((hw[i] >> (u & 31u)) & 1u);
                if constexpr (has_carry(PROG)) {
                    const bool in = g0 + 64u * i < wend && u < nv;
                    keep[i] = keep[i] || (in && carry[u]);
                }
                if (hit) state[vbase + u] = mv[i];
                need[i] = keep[i];
            }
        } else {
#pragma unroll
            for (uint32_t i = 0; i < U; ++i) {
                const uint32_t v = vbase + g0 + 64u * i + lane;
                keep[i] = false;
                need[i] = av[i] != 0ull;
                xv[i] = 0.f;
                if (need[i]) {
                    const double y = (double)(av[i] & ~kCarried) * kInvFix;
                    if constexpr (PROG == P_NIBBLE) {
                        // initFunc halved the value of a vertex active before
                        // scatter; any other vertex keeps its value. Both add
                        // the arrived amount in the same fixed point.
                        const float old = __uint_as_float(state[v]);
                        const float base = (av[i] & kCarried) ? old * 0.5f : old;
                        const unsigned long long b = __double2ull_rn((double)base * kFix);
                        xv[i] = (float)((double)((av[i] & ~kCarried) + b) * kInvFix);
                    } else if constexpr (PROG == P_PR) {
                        const double d = (double)P.damping;
                        xv[i] = (float)((1.0 - d) * P.inv_n + d * (y + dang * P.inv_n));
                        keep[i] = true;
                    } else {
                        const double al = (double)P.alpha;
                        double xd = (1.0 - al) * y;
                        if (v == P.root) xd += al + (1.0 - al) * dang;
                        xv[i] = (float)xd;
                        keep[i] = xv[i] > 0.0f;
                    }
                    state[v] = __float_as_uint(xv[i]);
                }
            }
        }
        // out-degrees: of kept vertices (frontier edges), and for sum programs
        // of every vertex that got a value (dangling mass)
#pragma unroll
        for (uint32_t i = 0; i < U; ++i) {
            const uint32_t v = vbase + g0 + 64u * i + lane;
            o0[i] = need[i] ? off[v] : 0u;
            o1[i] = need[i] ? off[v + 1] : 0u;
        }
        if constexpr (PROG == P_NIBBLE) {  // filterFunc: PR >= eps * deg (never without out-edges)
#pragma unroll
            for (uint32_t i = 0; i < U; ++i) {
                const uint32_t d = o1[i] - o0[i];
                keep[i] = need[i] && d > 0u && xv[i] >= P.eps * (float)d;
            }
        }
#pragma unroll
        for (uint32_t i = 0; i < U; ++i) {
            if (g0 + 64u * i >= wend) break;  // uniform
            const uint32_t u = g0 + 64u * i + lane;
            const uint32_t deg = keep[i] ? o1[i] - o0[i] : 0u;
            if constexpr (SUM) {
                if (need[i] && o1[i] == o0[i]) my_d += (double)xv[i];
            }
            if (u < nv) degl[(u << dsh) + dadd] = deg;
            const uint64_t km = ballot(keep[i]);
            if (lane == 0) kscratch[(g0 >> 6) + i] = km;
            cnt += popc64(km);
            edges += deg;
        }
    }
    edges = wave_sum_u32(edges);
    if (lane == 0) {
        sh.wc[wave] = cnt;
        sh.ws[wave] = edges;
    }
    __syncthreads();
    uint32_t pos = 0, epos = 0, tot = 0, etot = 0;
    for (uint32_t w = 0; w < NW; ++w) {
        if (w < wave) {
            pos += sh.wc[w];
            epos += sh.ws[w];
        }
        tot += sh.wc[w];
        etot += sh.ws[w];
    }
    uint16_t* __restrict__ nlist = gptr(G.flist[nxt]) + vbase;
    uint32_t* __restrict__ npre = gptr(G.fpre[nxt]) + vbase;
    uint32_t* __restrict__ nbits = gptr(G.fbits[nxt]) + (vbase >> 5);
    // the wave's bitmap words, one per lane
    for (uint32_t w = (wb >> 5) + lane; w < (wend >> 5); w += 64) {
        const uint64_t km = kscratch[w >> 1];
        nbits[w] = (w & 1u) ? (uint32_t)(km >> 32) : (uint32_t)km;
    }
    for (uint32_t u0 = wb; u0 < wend; u0 += 64) {
        const uint32_t u = u0 + lane;
        const uint64_t km = kscratch[u0 >> 6];
        if (km == 0) continue;  // nothing kept in these 64 vertices
        const bool keep = (km >> lane) & 1u;
        const uint32_t deg = keep ? degl[(u << dsh) + dadd] : 0u;
        const uint32_t dincl = wave_incl_scan(deg);
        if (keep) {
            const uint32_t at = pos + popc_lt(km);
            nlist[at] = (uint16_t)u;
            npre[at] = epos + dincl - deg;
        }
        pos += popc64(km);
        epos += last_lane(dincl);
    }
    my_d = wave_sum_f64(my_d);
    const uint64_t ids64 = wave_sum_u64((uint64_t)ids_done);
    if (lane == 0) {
        sh.r64[wave] = ids64;
        sh.rd[wave] = my_d;
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t ni = 0;
        double d = 0.0;
        for (uint32_t w = 0; w < NW; ++w) {
            ni += sh.r64[w];
            d += sh.rd[w];
        }
        gptr(G.fVa[nxt])[cq] = tot;
        gptr(G.fEa[nxt])[cq] = etot;
        gptr(G.dpart[nxt])[cq] = d;
        if (task != 0xFFFFFFFFu) gptr(G.gat_ids)[task] = (uint32_t)ni;
    }
}

// Partition-centric ids of one column read from its stream, chunks
// [c_lo, c_hi): wave w takes chunks c_lo + w, c_lo + w + NW, ..., SPW per
// round. Lane l decodes chunk positions 4l..4l+3, which belong to one bin
// (bins start at multiples of 4). Its entry is the number of lane starts at
// lanes 1..l (a popcount of the chunk's lane-start mask); the entry's adj
// value comes from the lane that holds the entry (ds_bpermute; a chunk has at
// most 64 entries) and the message index from one wave scan of the
// message-start flags. One 16-byte load at data[adj + message starts before
// 4l] then holds the values of all four positions (a bin's messages are
// contiguous). A bin whose source did not scatter partition-centric this
// iteration (or a padding run) reads the identity words instead, so no id
// needs a mask of its own; values equal to the identity (inactive sources
// included) skip the LDS combine, and null ids (local id q) combine into a
// spare LDS word past the partition's state and are not counted.
// The next round's ids, weights and entries are loaded before the current
// round is decoded; the chunks' table offsets and lane-start masks one round
// earlier still, with scalar loads.
template <int PROG, bool WIDE, uint32_t NW = kGW, uint32_t SPW = 4>
__device__ __forceinline__ uint32_t stream_gather(const Dev& G, uint32_t c_lo, uint32_t c_hi, bool dense,
                                                  const uint64_t* pcm, uint32_t* st32,
                                                  unsigned long long* acc) {
    constexpr bool SUM = is_sum(PROG);
    typedef __attribute__((address_space(4))) const uint32_t CU32;  // read with scalar loads
    typedef __attribute__((address_space(4))) const uint64_t CU64;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // the range is the same in every lane: keep its arithmetic scalar
    c_lo = __builtin_amdgcn_readfirstlane(c_lo);
    c_hi = __builtin_amdgcn_readfirstlane(c_hi);
    const uint32_t n = c_hi - c_lo;
    const uint32_t nrounds = (n + NW * SPW - 1) / (NW * SPW);
    const uint2* __restrict__ ids = reinterpret_cast<const uint2*>(gptr(G.cs_ids));
    const uint32_t* __restrict__ wts = reinterpret_cast<const uint32_t*>(gptr(G.cs_w));
    CU64* lmp = (CU64*)reinterpret_cast<uint64_t>(gptr(G.cs_lm));
    CU32* tabo = (CU32*)reinterpret_cast<uint64_t>(gptr(G.cs_tabo));
    const uint2* __restrict__ ent = gptr(G.cs_ent);
    const uint32_t* __restrict__ data = gptr(G.data);
    const uint32_t k = G.k, idb = G.idb, nulld = G.q;
    // message-start flags of the lane's positions after the byte gather
    // below (bit 8j + 7 = position 4l + j); position 0 of the chunk is not
    // counted
    const uint32_t mm = lane == 0 ? 0x80808000u : 0x80808080u;
    // four message values: below 4 GiB of data, one 16-byte buffer load with
    // a 32-bit byte offset
    const __amdgpu_buffer_rsrc_t drsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t*>(data), (short)0, (int)0xFFFFFFFF, (int)0x00020000);
    auto msg4 = [&](uint32_t d) -> uint4 {
        if constexpr (WIDE) return make_uint4(data[d], data[d + 1], data[d + 2], data[d + 3]);
        else {
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(drsrc, (int)(d << 2), 0, 0);
            return make_uint4((uint32_t)v[0], (uint32_t)v[1], (uint32_t)v[2], (uint32_t)v[3]);
        }
    };
    auto piece = [&](uint32_t r, uint32_t pi) -> uint32_t { return (r * SPW + pi) * NW + wave; };
    auto chunk = [&](uint32_t r, uint32_t pi) -> uint32_t {
        const uint32_t i = piece(r, pi);
        return i < n ? c_lo + i : c_lo;  // past the range: re-read the first chunk, not combined
    };
    // per chunk of the next round: table offsets and lane-start mask (scalar)
    uint32_t tb_n[SPW], te_n[SPW];
    uint64_t lm_n[SPW];
    uint2 raw_n[SPW], ent_n[SPW];
    uint32_t w_n[SPW];
    auto fetch_meta = [&](uint32_t r, uint32_t* tb, uint32_t* te, uint64_t* lm) {
#pragma unroll
        for (uint32_t pi = 0; pi < SPW; ++pi) {
            const uint32_t c = chunk(r, pi);
            tb[pi] = tabo[c];
            te[pi] = tabo[c + 1];
            lm[pi] = lmp[c];
        }
    };
    auto fetch = [&](uint32_t r, const uint32_t* tb, const uint32_t* te) {
#pragma unroll
        for (uint32_t pi = 0; pi < SPW; ++pi) {
            const uint32_t c = chunk(r, pi);
            raw_n[pi] = gptr(ids + (size_t)c * 64)[lane];
            // lanes past the chunk's table read its last entry (one fetch)
            ent_n[pi] = gptr(ent + tb[pi])[min(lane, te[pi] - tb[pi] - 1u)];
            w_n[pi] = 0u;
            if constexpr (is_weighted(PROG)) w_n[pi] = gptr(wts + (size_t)c * 64)[lane];
        }
    };
    uint32_t my_ids = 0;  // non-identity ids the lane combined
    if (nrounds == 0) return 0;
    uint32_t tb_a[SPW], te_a[SPW];
    uint64_t lm_a[SPW];
    fetch_meta(0, tb_a, te_a, lm_a);
    fetch(0, tb_a, te_a);
    fetch_meta(1, tb_n, te_n, lm_n);
    for (uint32_t r = 0; r < nrounds; ++r) {
        uint2 raw[SPW], ev[SPW];
        uint32_t wv[SPW], tb_b[SPW], te_b[SPW];
        uint64_t lmc[SPW], lm_b[SPW];
#pragma unroll
        for (uint32_t pi = 0; pi < SPW; ++pi) {
            raw[pi] = raw_n[pi];
            ev[pi] = ent_n[pi];
            wv[pi] = w_n[pi];
            lmc[pi] = lm_a[pi];
            tb_b[pi] = tb_n[pi];
            te_b[pi] = te_n[pi];
            lm_b[pi] = lm_n[pi];
        }
        // loads of the next round (chunks past the range re-read the first)
        fetch_meta(r + 2, tb_n, te_n, lm_n);
        fetch(r + 1, tb_b, te_b);
#pragma unroll
        for (uint32_t pi = 0; pi < SPW; ++pi) lm_a[pi] = lm_b[pi];
        // the round's chunks go through each step together, so that their
        // scans, ds_bpermutes and loads overlap one another's latency
        uint32_t adjv[SPW], hb[SPW], mex[SPW];
        uint4 v4[SPW];
#pragma unroll
        for (uint32_t pi = 0; pi < SPW; ++pi) {
            adjv[pi] = ev[pi].x;
            if (!dense) {
                const uint32_t src = ev[pi].y & 0xFFFFu;
                if (src < k && !((pcm[src >> 6] >> (src & 63u)) & 1ull)) adjv[pi] = idb - (ev[pi].y >> 16);
            }
            // a chunk past the task's range (a re-read of its first chunk)
            // reads the identity words: its combines change nothing
            if (piece(r, pi) >= n) adjv[pi] = idb;
            hb[pi] = __builtin_amdgcn_perm(raw[pi].y, raw[pi].x, 0x07050301u) & mm;
            mex[pi] = (uint32_t)__popc(hb[pi]);
        }
#pragma unroll
        for (uint32_t pi = 0; pi < SPW; ++pi) mex[pi] = wave_incl_scan(mex[pi]) - mex[pi];
#pragma unroll
        for (uint32_t pi = 0; pi < SPW; ++pi) {
            // entry of the lane: lane starts at lanes 1..lane
            const uint32_t b = popc_lt(lmc[pi]) + (uint32_t)((lmc[pi] >> lane) & 1ull);
            const uint32_t d0 = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(b << 2), (int)adjv[pi]) + mex[pi] +
                                ((hb[pi] >> 7) & 1u);
            v4[pi] = msg4(d0);
        }
#pragma unroll
        for (uint32_t pi = 0; pi < SPW; ++pi) {
            // message of position 4l + j relative to that of 4l: the starts at 4l+1..4l+j
            // word r of the four loaded, r = the message starts at
            // positions 4l+1..4l+j, by bit selects (m* = 0 or all ones)
            const uint32_t m1 = (uint32_t)__builtin_amdgcn_sbfe((int)hb[pi], 15, 1);
            const uint32_t m2 = (uint32_t)__builtin_amdgcn_sbfe((int)hb[pi], 23, 1);
            const uint32_t m3 = (uint32_t)__builtin_amdgcn_sbfe((int)hb[pi], 31, 1);
            const uint32_t a = v4[pi].x, bb = v4[pi].y, cc = v4[pi].z, dd = v4[pi].w;
            auto bfi = [](uint32_t m, uint32_t y, uint32_t x) { return (m & y) | (~m & x); };
            const uint32_t t1 = bfi(m1, cc, bb), t2 = bfi(m1, dd, cc);
            uint32_t xv[4];
            xv[0] = a;
            xv[1] = bfi(m1, bb, a);
            xv[2] = bfi(m2, t1, xv[1]);
            xv[3] = bfi(m3, bfi(m2, t2, t1), xv[2]);
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                uint32_t x = xv[j];
                if constexpr (is_weighted(PROG)) x = sat_add(x, (wv[pi] >> (8u * j)) & 0xFFu);
                const uint32_t d = ((j < 2 ? raw[pi].x : raw[pi].y) >> (16u * (j & 1u))) & kLocalMask;
                const bool real = d != nulld;
                // an identity (a source that did not scatter, padding) changes
                // nothing and is not combined: its LDS operation would only add
                // bank conflicts at a random word
                if constexpr (SUM) {
                    const bool use = (int32_t)x >= 0 && real;  // identities and padding read negative words
                    my_ids += use ? 1u : 0u;
                    if (use) atomicAdd(acc + d, __double2ull_rn((double)__uint_as_float(x) * kFix));
                } else {
                    my_ids += (x != kIdentMin && real) ? 1u : 0u;
                    if (x != kIdentMin) atomicMin(st32 + d, x);
                }
            }
        }
    }
    return my_ids;
}

// An iteration in which gather reads the column streams and source-centric
// bins hold few ids (the plan decides): kb_gather_dense runs it with wider
// workgroups and kb_gather returns.
__device__ __forceinline__ bool dense_stream_iteration(const Dev& G) {
    return gptr(G.ctrl)->dense_gather != 0u;
}

// Workgroup of the dense gather: 16 waves. Without the bin-list arrays its LDS
// is the partition's state plus the filter's keep masks, so two workgroups
// share a CU (32 waves, at most 64 registers per lane), twice the waves the
// general gather can keep in flight on the column streams.
constexpr uint32_t kDT = 1024;
constexpr uint32_t kDW = kDT / 64;

struct DenseLds {
    size_t state, carry, keep, pcm, scm, total;
};
__host__ __device__ inline DenseLds dense_layout(int prog, uint32_t q) {
    DenseLds L{};
    size_t o = 0;
    L.state = o;  o += ((size_t)(q + 1) * (is_sum(prog) ? 8 : 4) + 15) / 16 * 16;  // plus the spare word
    L.carry = o;  o += has_carry(prog) ? ((size_t)q + 15) / 16 * 16 : 0;
    L.keep = o;   o += ((size_t)q / 64 + 1) * 8;
    L.pcm = o;    o += 64 * 8;  // k-bit source masks (k <= 4096)
    L.scm = o;    o += 64 * 8;
    L.total = o;
    return L;
}

// The source-centric bins of source partitions [p_lo, p_hi] marked in scm.
// A task of a split column takes the bins whose first static piece lies in
// its piece range [s0, s1) (counted from the first piece of bin p_lo), so
// every bin has one owner. The waves take the task's bins in turn, 64 at a
// time, one per lane: a lane walks a bin of at most 8 ids by itself (message
// index: the starts seen so far), a larger bin is taken by the whole wave, 64
// ids a step (message index: the bin's first plus the starts before the id).
// Returns the ids with a value the lane combined.
template <int PROG>
__device__ __forceinline__ uint32_t dense_sc_bins(const Dev& G, uint32_t cq, uint32_t p_lo, uint32_t p_hi,
                                                  bool split, uint32_t s0, uint32_t s1, const uint64_t* scm,
                                                  uint32_t* st32, unsigned long long* acc) {
    constexpr bool SUM = is_sum(PROG);
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t k = G.k;
    const uint64_t below_eq = lane == 63u ? ~0ull : (2ull << lane) - 1ull;
    const uint16_t* __restrict__ ids = gptr(G.sc_ids);
    const uint8_t* __restrict__ wts = gptr(G.sc_w);
    const uint32_t* __restrict__ data = gptr(G.data);
    const uint2* __restrict__ cnt = gptr(G.sc_cnt) + (size_t)cq * k;
    const uint4* __restrict__ cmc = gptr(G.cm) + (size_t)cq * k;
    const uint32_t* __restrict__ smo = gptr(G.sc_mo) + (size_t)cq * k;
    const uint32_t* __restrict__ spre = gptr(G.spre) + (size_t)cq * k;
    const uint32_t sbase = spre[p_lo];
    uint32_t my_ids = 0;
    auto combine = [&](uint32_t d, uint32_t v, bool use) {
        if constexpr (SUM) {
            use = use && (int32_t)v >= 0;
            my_ids += use ? 1u : 0u;
            atomicAdd(acc + d, use ? __double2ull_rn((double)__uint_as_float(v) * kFix) : 0ull);
        } else {
            if (!use) v = kIdentMin;
            my_ids += v != kIdentMin ? 1u : 0u;
            atomicMin(st32 + d, v);
        }
    };
    // one group: lane j < n holds bin gp
    auto group = [&](uint32_t n, uint32_t gp) {
        const bool valid = lane < n;
        uint32_t icnt = 0, ioff = 0, moff = 0;
        if (valid) {
            icnt = cnt[gp].y;
            ioff = cmc[gp].y;
            moff = smo[gp];
        }
        const bool small = valid && icnt <= 8u;
        if (small) {
            uint32_t m = 0xFFFFFFFFu;  // message index of the id
            for (uint32_t i = 0; i < icnt; ++i) {
                const uint32_t id = ids[ioff + i];
                m += (id & kFlag) ? 1u : 0u;
                uint32_t v = data[moff + m];
                if constexpr (is_weighted(PROG)) v = sat_add(v, wts[ioff + i]);
                combine(id & kLocalMask, v, true);
            }
        }
        uint64_t big = ballot(valid && !small);
        while (big) {
            const uint32_t j = (uint32_t)__builtin_ctzll(big);
            big &= big - 1ull;
            const uint32_t bn = readlane_u32(icnt, j), bo = readlane_u32(ioff, j), bm = readlane_u32(moff, j);
            uint32_t before = 0;  // message starts before this step
            for (uint32_t x = 0; x < bn; x += 64u) {
                const uint32_t i = x + lane;
                const bool ok = i < bn;
                const uint32_t id = ok ? (uint32_t)ids[bo + i] : 0u;
                const uint64_t fm = ballot(ok && (id & kFlag));
                uint32_t v = SUM ? kIdentSum : kIdentMin;
                if (ok) {
                    v = data[bm + before + popc64(fm & below_eq) - 1u];
                    if constexpr (is_weighted(PROG)) v = sat_add(v, wts[bo + i]);
                }
                combine(id & kLocalMask, v, ok);
                before += popc64(fm);
            }
        }
    };
    uint32_t rank = 0, n = 0, gp = 0;
    for (uint32_t w = p_lo >> 6; w <= (p_hi >> 6); ++w) {
        uint64_t m = scm[w] & range_bits(w, p_lo, p_hi);
        while (m) {
            const uint32_t b = (uint32_t)__builtin_ctzll(m);
            m &= m - 1ull;
            const uint32_t p = 64u * w + b;
            if (split) {
                const uint32_t sp = spre[p] - sbase;
                if (sp < s0 || sp >= s1) continue;  // another task of the column owns the bin
            }
            if ((rank++ % kDW) != wave) continue;
            if (lane == n) gp = p;
            if (++n == 64u) {
                group(64u, gp);
                n = 0;
            }
        }
    }
    if (n) group(n, gp);
    return my_ids;
}

// The gather task of a dense iteration: the task table, the split of heavy
// columns and the partial results are those of gather_body; the task's share
// of the column stream is all it reads.
template <int PROG>
__device__ __forceinline__ void dense_body(const Dev& G, const Params& P, uint32_t* __restrict__ state,
                                           uint32_t it, uint32_t task) {
    if (gptr(G.ctrl)->done || !dense_stream_iteration(G)) return;
    constexpr bool SUM = is_sum(PROG);
    const uint4 TA = gptr(G.gtask)[2 * task], TB = gptr(G.gtask)[2 * task + 1];
    const uint32_t cq = TA.x, nt = TA.w >> 16, jt = TA.w & 0xFFFFu;
    uint32_t p_lo = TA.y, p_hi = TA.z;
    const uint32_t slot = TB.z;
    bool split = nt > 1;
    const uint32_t cur = it & 1u, nxt = cur ^ 1u;
    const uint32_t k = G.k, Q = G.q;
    const uint32_t vbase = cq << G.s;
    const uint32_t nv = min(Q, G.V - vbase);
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    extern __shared__ __align__(16) unsigned char smem[];
    const DenseLds L = dense_layout(PROG, Q);
    uint32_t* st32 = reinterpret_cast<uint32_t*>(smem + L.state);
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem + L.state);
    uint8_t* carry = smem + L.carry;
    __shared__ GatherSharedT<kDW> sh;

    // Source masks of the column when some partition did not scatter
    // partition-centric: pcm, bins whose source did (read from the stream);
    // scm, source-centric bins with ids (the column's stamp says whether any).
    const bool mixed = gptr(G.ctrl)->n_pcpart != k;
    uint64_t* pcm = reinterpret_cast<uint64_t*>(smem + L.pcm);
    uint64_t* scm = reinterpret_cast<uint64_t*>(smem + L.scm);
    if (mixed) {
        const bool sc_col = gptr(G.cact)[cq] == it + 1u;
        const uint32_t g = tid;  // byte g covers partitions [8g, 8g + 8); k <= 4096 = 8 * 512
        if (g < G.kw * 8u) {
            uint32_t scb = 0;
            if (sc_col) {
                const uint64_t f = *reinterpret_cast<const uint64_t*>(gptr(G.nz) + (size_t)cq * G.kw * 64u + 8u * g);
                uint32_t bits = 0;
#pragma unroll
                for (int j = 0; j < 8; ++j) bits |= (uint32_t)((f >> (8 * j)) & 1u) << j;
                scb = bits & reinterpret_cast<const uint8_t*>(gptr(G.scmask))[g];
            }
            reinterpret_cast<uint8_t*>(pcm)[g] = (uint8_t)(reinterpret_cast<const uint8_t*>(
                gptr(G.colsrc) + (size_t)cq * G.kw)[g] & reinterpret_cast<const uint8_t*>(gptr(G.pcmask))[g]);
            reinterpret_cast<uint8_t*>(scm)[g] = (uint8_t)scb;
        }
        __syncthreads();
    }
    auto bit = [&](const uint64_t* m, uint32_t p) -> bool { return (m[p >> 6] >> (p & 63u)) & 1ull; };

    // a split column whose ids fit one task is gathered whole by its first
    // task (the ids of its listed bins: every static id of a partition-centric
    // source, the reserved ids of a source-centric one)
    if (split) {
        const uint4* __restrict__ cmcol = gptr(G.cm) + (size_t)cq * k;
        const uint2* __restrict__ sccol = gptr(G.sc_cnt) + (size_t)cq * k;
        uint32_t c = 0;
        for (uint32_t p = tid; p < k; p += kDT) {
            if (!mixed) c += cmcol[p].w;
            else if (bit(pcm, p)) c += cmcol[p].w;
            else if (bit(scm, p)) c += sccol[p].y;
        }
        c = wave_sum_u32(c);
        if (lane == 0) sh.wc[wave] = c;
        __syncthreads();
        uint32_t tot = 0;
        for (uint32_t w = 0; w < kDW; ++w) tot += sh.wc[w];
        __syncthreads();
        if (tot <= G.whole_ids) {
            if (jt != 0) {
                if (tid == 0) {
                    gptr(G.gflag)[slot] = 0;
                    gptr(G.gat_ids)[task] = 0;
                    gptr(G.gat_ran)[task] = 0;
                }
                return;
            }
            if (tid == 0) gptr(G.gflag)[slot] = 2;  // the merge skips this partition
            split = false;
            p_lo = 0;
            p_hi = k - 1;
        }
    }
    // statistics: the listed bins of the task's source range, as kb_gather
    // counts them (in a dense iteration every non-empty static bin)
    uint32_t mine = 0, sc_mine = 0;
    if (tid < G.kw) {
        const uint64_t r = range_bits(tid, p_lo, p_hi);
        if (mixed) {
            mine = (uint32_t)__popcll((pcm[tid] | scm[tid]) & r);
            sc_mine = (uint32_t)__popcll(scm[tid] & r);
        } else {
            mine = (uint32_t)__popcll(gptr(G.colsrc)[(size_t)cq * G.kw + tid] & r);
        }
    }
    mine = wave_sum_u32(mine);  // kw <= 64: wave 0 holds the sum
    sc_mine = __syncthreads_or(sc_mine != 0u) ? 1u : 0u;  // some source-centric bin in the range
    const uint32_t c0 = gptr(G.cs_c0)[cq], c1 = gptr(G.cs_c0)[cq + 1];
    uint32_t cs_lo = c0, cs_hi = c1;
    if (split) {
        const uint64_t C = c1 - c0;
        cs_lo = c0 + (uint32_t)(C * jt / nt);
        cs_hi = c0 + (uint32_t)(C * (jt + 1u) / nt);
    }
    const bool any = cs_hi > cs_lo || sc_mine != 0u || (!split && !msg_only(PROG) && gptr(G.fVa[cur])[cq] > 0);
    if (!any) {
        if (tid == 0) {
            if (split) {
                gptr(G.gflag)[slot] = 0;
            } else {
                gptr(G.fVa[nxt])[cq] = 0;
                gptr(G.fEa[nxt])[cq] = 0;
                gptr(G.dpart[nxt])[cq] = 0.0;
            }
            gptr(G.gat_ids)[task] = 0;
            gptr(G.gat_ran)[task] = mine << 2;
        }
        return;
    }
    if (tid == 0) gptr(G.gat_ran)[task] = (split ? 2u : 1u) | (mine << 2);
    for (uint32_t u = tid; u < Q; u += kDT) {
        if constexpr (SUM) acc[u] = 0ull;
        else st32[u] = kIdentMin;
        if constexpr (has_carry(PROG)) carry[u] = 0;
    }
    __syncthreads();
    if (!split) {
        reinit<PROG, kDT>(G, P, state, it, cq, st32, carry);
        __syncthreads();
    }
    uint32_t my_ids;
    if (G.idb < (1u << 30) - kIdWords) my_ids = stream_gather<PROG, false, kDW, 2>(G, cs_lo, cs_hi, !mixed, pcm, st32, acc);
    else my_ids = stream_gather<PROG, true, kDW, 2>(G, cs_lo, cs_hi, !mixed, pcm, st32, acc);
    if (sc_mine) my_ids += dense_sc_bins<PROG>(G, cq, p_lo, p_hi, split, TB.x, TB.y, scm, st32, acc);
    __syncthreads();
    if (split) {
        if constexpr (SUM) {
            unsigned long long* out = reinterpret_cast<unsigned long long*>(gptr(G.gpart)) + (size_t)slot * Q;
            for (uint32_t u = tid; u < nv; u += kDT) out[u] = acc[u];
        } else {
            uint32_t* out = gptr(G.gpart) + (size_t)slot * 2 * Q;
            for (uint32_t u = tid; u < nv; u += kDT) out[u] = st32[u];
        }
        const uint64_t ids64 = wave_sum_u64((uint64_t)my_ids);
        if (lane == 0) sh.r64[wave] = ids64;
        __syncthreads();
        if (tid == 0) {
            uint64_t ni = 0;
            for (uint32_t w = 0; w < kDW; ++w) ni += sh.r64[w];
            gptr(G.gflag)[slot] = 1;
            gptr(G.gat_ids)[task] = (uint32_t)ni;
        }
        return;
    }
    finish_partition<PROG, kDW>(G, P, state, it, cq, st32, acc, carry,
                                reinterpret_cast<uint64_t*>(smem + L.keep), sh, my_ids, task, false);
}

// Gather task: a contiguous range [s0, s1) of the static 256-id pieces of the
// bins bin[p][cq], p in [p_lo, p_hi], taken in p order. The destination
// partition's state lives in LDS (the cached vertex data of Sec. 3): every
// message updates on-chip state, every bin piece is read once, sequentially.
// Partitions whose bins hold few ids get one task that also runs reInit and
// the filter; heavy partitions (RMAT hubs) get several tasks that each leave
// a partial result for k_merge.
//
// Bins are enumerated through the two-level active list (Sec. 3.1.3): the
// source-centric scatter stamps every column that receives source-centric ids
// (level 1, cact) and flags each non-empty source-centric bin (nz); the plan
// writes the masks of the partitions scattered in each mode. A task first
// builds its column's k-bit mask of bins with ids this iteration --
// partition-centric sources from the static column mask, source-centric ones
// from the flags, read only when the column is stamped -- and then reads the
// counts of those bins alone: a column without messages costs two loads, a
// sparse one a few words per 64 source partitions.
// Each wave decodes a contiguous run of pieces: message index of an id =
// chunk-table base + number of message-start flags after the piece start.
//
// Combining touches only the workgroup's own LDS copy of the partition (no
// global atomics, no locks), in one of two ways chosen per graph:
//  - LDS combine (default): every message is one LDS min (min programs) or
//    one LDS 64-bit integer add of its value in units of 2^-60 (sum
//    programs); no rounds and no barriers inside the message loop.
//  - atomic-free rounds (ROUNDS): min programs: every pending lane reads the
//    state word and writes its value if smaller; after a barrier each lane
//    re-reads, and only lanes whose value is still smaller stay pending. Each
//    round lowers every contested word strictly, so the loop ends with the
//    exact minimum whatever the write order. Sum programs: every pending lane
//    writes its slot number into the destination's tag, the lane whose tag
//    survived adds; after four rounds the leftovers (high in-degree vertices)
//    are first summed per destination inside each wave, leaving at most one
//    entry per destination per wave for the last rounds.
// Both give the same bits: min is order-independent and the sums are exact
// integer sums.
template <int PROG, bool ROUNDS>
__device__ __forceinline__ void gather_body(const Dev& G, const Params& P, uint32_t* __restrict__ state,
                                            uint32_t it, uint32_t task) {
    if (gptr(G.ctrl)->done) return;
    if constexpr (!ROUNDS) {
        if (dense_stream_iteration(G)) return;  // kb_gather_dense gathers every column
    }
    constexpr bool SUM = is_sum(PROG);
    constexpr uint32_t IDENT = is_sum(PROG) ? kIdentSum : kIdentMin;
    // pieces per wave per combine round (the atomic-free sum keeps two, for registers)
    constexpr uint32_t PPW = (ROUNDS && SUM) ? 2 : 4;
    const uint4 TA = gptr(G.gtask)[2 * task], TB = gptr(G.gtask)[2 * task + 1];
    const uint32_t cq = TA.x, nt = TA.w >> 16, jt = TA.w & 0xFFFFu;
    uint32_t p_lo = TA.y, p_hi = TA.z;
    // the two id / weight / chunk arrays a piece may come from, as uniform
    // values (a per-lane choice between two fields of the view would
    // otherwise become a per-lane load of the pointer itself)
    const uint16_t* __restrict__ ids_sc = gptr(G.sc_ids);
    const uint16_t* __restrict__ ids_pc = gptr(G.png_ids);
    const uint8_t* __restrict__ w_sc = gptr(G.sc_w);
    const uint8_t* __restrict__ w_pc = gptr(G.png_w);
    const uint32_t* __restrict__ ch_sc = gptr(G.sc_chunk);
    const uint32_t* __restrict__ ch_pc = gptr(G.png_chunk);
    const uint32_t* __restrict__ data = gptr(G.data);
    uint32_t s0 = TB.x, s1 = TB.y;
    const uint32_t slot = TB.z;
    bool split = nt > 1;
    const uint32_t cur = it & 1u, nxt = cur ^ 1u;
    const uint32_t k = G.k, Q = G.q;
    const uint32_t vbase = cq << G.s;
    const uint32_t nv = min(Q, G.V - vbase);
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    const uint4* __restrict__ cmcol = gptr(G.cm) + (size_t)cq * k;
    const uint2* __restrict__ sccol = gptr(G.sc_cnt) + (size_t)cq * k;

    extern __shared__ __align__(16) unsigned char smem[];
    const GatherLds L = gather_layout(PROG, Q, ROUNDS);
    uint32_t* st32 = reinterpret_cast<uint32_t*>(smem + L.state);
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem + L.state);
    uint16_t* tag = reinterpret_cast<uint16_t*>(smem + L.tag);
    uint8_t* carry = smem + L.carry;   // kept active by initFunc
    uint32_t* bl_ioff = reinterpret_cast<uint32_t*>(smem + L.bl_ioff);
    uint32_t* bl_icnt = reinterpret_cast<uint32_t*>(smem + L.bl_icnt);
    uint32_t* bl_moff = reinterpret_cast<uint32_t*>(smem + L.bl_moff);  // bit 31: SC bin
    uint32_t* bl_mcnt = reinterpret_cast<uint32_t*>(smem + L.bl_mcnt);
    uint32_t* bl_jlo = reinterpret_cast<uint32_t*>(smem + L.bl_jlo);
    uint32_t* bl_scan = reinterpret_cast<uint32_t*>(smem + L.bl_scan);
    __shared__ GatherShared sh;

    // ---- the two-level active list. Level 1: does column cq receive
    //      anything? (stamped by the source-centric scatter; partition-centric
    //      sources exist only if some partition scattered in that mode).
    //      Level 2: the k-bit mask of source partitions whose bin to cq holds
    //      ids, built one byte (8 partitions) per thread with independent
    //      loads: partition-centric sources from the static column mask,
    //      source-centric ones from the scatter's marks.
    uint64_t* amask = reinterpret_cast<uint64_t*>(smem + L.amask);
    uint64_t* pcm = reinterpret_cast<uint64_t*>(smem + L.pcm);
    bool col_pc = false;  // some partition-centric source has a bin in this column
    {
        const bool sc_col = gptr(G.cact)[cq] == it + 1u;
        const bool pc_any = gptr(G.ctrl)->n_pcpart != 0u;
        uint8_t* ab = reinterpret_cast<uint8_t*>(amask);
        uint8_t* pb = reinterpret_cast<uint8_t*>(pcm);
        const uint32_t g = tid;  // byte g covers partitions [8g, 8g + 8); k <= 4096 = 8 * kGT
        if (g < G.kw * 8u) {
            uint32_t scb = 0, pcb = 0;
            if (sc_col) {
                const uint64_t f = *reinterpret_cast<const uint64_t*>(gptr(G.nz) + (size_t)cq * G.kw * 64u + 8u * g);
                uint32_t bits = 0;
#pragma unroll
                for (int j = 0; j < 8; ++j) bits |= (uint32_t)((f >> (8 * j)) & 1u) << j;
                scb = bits & reinterpret_cast<const uint8_t*>(gptr(G.scmask))[g];
            }
            if (pc_any)
                pcb = reinterpret_cast<const uint8_t*>(gptr(G.colsrc) + (size_t)cq * G.kw)[g] &
                      reinterpret_cast<const uint8_t*>(gptr(G.pcmask))[g];
            ab[g] = (uint8_t)(scb | pcb);
            pb[g] = (uint8_t)pcb;
            col_pc = pcb != 0u;
        }
    }
    col_pc = __syncthreads_or(col_pc);
    auto abit = [&](uint32_t p) -> bool { return (amask[p >> 6] >> (p & 63u)) & 1ull; };
    auto pcbit = [&](uint32_t p) -> bool { return (pcm[p >> 6] >> (p & 63u)) & 1ull; };
    // partition-centric bins from the column stream this iteration (the bin
    // list below then takes only the source-centric ones)
    const bool use_stream = !ROUNDS && col_pc && gptr(G.ctrl)->pc_stream != 0u;

    // ---- a split partition with few ids this iteration (a sparse frontier)
    //      is gathered whole by its first task: no partial results, no merge
    if (split) {
        uint32_t c = 0;
        for (uint32_t p = tid; p < k; p += kGT) {
            if (!abit(p)) continue;
            c += pcbit(p) ? cmcol[p].w : sccol[p].y;
        }
        c = wave_sum_u32(c);
        if (lane == 0) sh.wc[wave] = c;
        __syncthreads();
        uint32_t tot = 0;
        for (uint32_t w = 0; w < kGW; ++w) tot += sh.wc[w];
        __syncthreads();
        if (tot <= G.whole_ids) {
            if (jt != 0) {
                if (tid == 0) {
                    gptr(G.gflag)[slot] = 0;
                    gptr(G.gat_ids)[task] = 0;
                    gptr(G.gat_ran)[task] = 0;
                }
                return;
            }
            if (tid == 0) gptr(G.gflag)[slot] = 2;  // the merge skips this partition
            split = false;
            p_lo = 0;
            p_hi = k - 1;
            s0 = 0;
            s1 = 0xFFFFFFFFu;
        }
    }

    // ---- anything to do for this task? (bins with ids in its source range,
    //      or, for programs that carry vertices, an active set to filter)
    uint32_t mine = 0, mine_l = 0;  // listed bins of the thread's byte inside [p_lo, p_hi] (all; bin-list path)
    uint32_t lbits = 0;               // those of the bin-list path, as bits of the byte
    if (tid < G.kw * 8u) {
        const uint32_t byte = reinterpret_cast<const uint8_t*>(amask)[tid];
        const uint32_t lbyte = use_stream ? byte & ~(uint32_t)reinterpret_cast<const uint8_t*>(pcm)[tid] : byte;
        const uint64_t r = range_bits(tid >> 3, p_lo, p_hi) >> (8u * (tid & 7u));
        mine = (uint32_t)__popc(byte & (uint32_t)(r & 0xFFu));
        lbits = lbyte & (uint32_t)(r & 0xFFu);
        mine_l = (uint32_t)__popc(lbits);
    }
    const uint32_t wbins = wave_sum_u32(mine);
    if (lane == 0) sh.wsm[wave] = wbins;
    // rank of the thread's first bin-list bin among those of the task (bytes
    // are in source-partition order)
    const uint32_t lincl = wave_incl_scan(mine_l);
    if (lane == 63) sh.wp[wave] = lincl;
    // this task's share of the column stream
    uint32_t cs_lo = 0, cs_hi = 0;
    if (use_stream) {
        const uint32_t c0 = gptr(G.cs_c0)[cq], c1 = gptr(G.cs_c0)[cq + 1];
        if (split) {
            const uint64_t C = c1 - c0;
            cs_lo = c0 + (uint32_t)(C * jt / nt);
            cs_hi = c0 + (uint32_t)(C * (jt + 1u) / nt);
        } else {
            cs_lo = c0;
            cs_hi = c1;
        }
    }
    // a column held back by interleaved scatter-gather keeps its frontier
    const bool carry_col = !SUM && isg_holds(P, cq, k, it) && gptr(G.fVa[cur])[cq] > 0;
    const bool any = __syncthreads_or(mine_l > 0u || (tid == 0 && (cs_hi > cs_lo || (!split && (carry_col ||
                                      (!msg_only(PROG) && gptr(G.fVa[cur])[cq] > 0))))));
    uint32_t nbins = 0, lrank = lincl - mine_l, nlisted = 0;
    for (uint32_t w = 0; w < kGW; ++w) {
        nbins += sh.wsm[w];
        if (w < wave) lrank += sh.wp[w];
        nlisted += sh.wp[w];
    }
    if (!any) {
        if (tid == 0) {
            if (split) {
                gptr(G.gflag)[slot] = 0;
            } else {
                gptr(G.fVa[nxt])[cq] = 0;
                gptr(G.fEa[nxt])[cq] = 0;
                gptr(G.dpart[nxt])[cq] = 0.0;
            }
            gptr(G.gat_ids)[task] = 0;
            // listed bins in this task's source range whose ids another task
            // of the column reads from the stream still count as gathered
            gptr(G.gat_ran)[task] = nbins << 2;
        }
        return;
    }
    if (tid == 0) gptr(G.gat_ran)[task] = (split ? 2u : 1u) | (nbins << 2);

    // ---- LDS copy of the partition at the combine identity (the filter
    //      compares it with the stored values)
    for (uint32_t u = tid; u < Q; u += kGT) {
        if constexpr (SUM) acc[u] = 0ull;
        else st32[u] = kIdentMin;
        if constexpr (has_carry(PROG)) carry[u] = 0;
    }
    __syncthreads();
    if (!split) {
        reinit<PROG>(G, P, state, it, cq, st32, carry);
        __syncthreads();
    }

    // ---- gather the task's pieces, bins in windows of kGT bin-list bins
    //      (ascending source partition), so that a column with few listed
    //      bins takes one window whatever their partitions
    uint32_t my_ids = 0;
    if constexpr (!ROUNDS) {
        if (use_stream) {
            const bool dense = gptr(G.ctrl)->n_pcpart == k;
            if (G.idb < (1u << 30) - kIdWords) my_ids += stream_gather<PROG, false>(G, cs_lo, cs_hi, dense, pcm, st32, acc);
            else my_ids += stream_gather<PROG, true>(G, cs_lo, cs_hi, dense, pcm, st32, acc);
        }
    }
    // static pieces of the bins before p_lo: the task's piece range [s0, s1)
    // counts from there
    const uint32_t sbase = gptr(G.spre)[(size_t)cq * k + p_lo];
    for (uint32_t j0 = 0; j0 < nlisted; j0 += kGT) {
        // the window's partitions, listed in bl_jlo (rewritten with the
        // window's bins only after the barrier that follows the reads)
        for (uint32_t m = lbits, r = lrank; m; m &= m - 1u, ++r)
            if (r >= j0 && r < j0 + kGT) bl_jlo[r - j0] = 8u * tid + (uint32_t)__builtin_ctz(m);
        __syncthreads();
        const bool inr = j0 + tid < nlisted;
        const uint32_t p = inr ? bl_jlo[tid] : 0u;
        const bool is_pc = inr && pcbit(p);
        const uint32_t md = !inr ? GPOP_MODE_NONE : (is_pc ? GPOP_MODE_PC : GPOP_MODE_SC);
        uint32_t ioff = 0, icnt = 0, moff = 0, mcnt = 0, SP = 0;
        if (inr) {
            const uint4 c = cmcol[p];
            ioff = c.y;
            moff = c.x;
            SP = gptr(G.spre)[(size_t)cq * k + p] - sbase;
            if (is_pc) {
                icnt = c.w;
                mcnt = c.z;
            } else {
                const uint2 d = sccol[p];
                icnt = d.y;
                mcnt = d.x;
                moff = gptr(G.sc_mo)[(size_t)cq * k + p];  // source-centric message slots
            }
        }
        const uint32_t dp = pieces_of(ioff, icnt);
        // a task that covers whole bins takes a bin of at most kSmallBin ids
        // with one lane (below) instead of as pieces of 256-id chunks
        const bool small = !ROUNDS && !split && icnt > 0 && icnt <= kSmallBin;
        // pieces of this bin that fall in [s0, s1)
        const uint32_t jlo = s0 > SP ? s0 - SP : 0u;
        const uint32_t jhi = min(dp, s1 > SP ? s1 - SP : 0u);
        const uint32_t npieces = (jhi > jlo && !small) ? jhi - jlo : 0u;
        const bool nz = npieces > 0;
        const uint64_t bm = ballot(nz);
        const uint64_t sm = ballot(small);
        const uint32_t pincl = wave_incl_scan(npieces);
        if (lane == 63) {
            sh.wc[wave] = popc64(bm);
            sh.wp[wave] = pincl;
            sh.wsm[wave] = popc64(sm);
        }
        __syncthreads();
        uint32_t boff = 0, poff = 0, nb = 0, npt = 0, soff = 0, ns = 0;
        for (uint32_t w = 0; w < kGW; ++w) {
            const uint32_t c = sh.wc[w], pc = sh.wp[w], sc = sh.wsm[w];
            if (w < wave) {
                boff += c;
                poff += pc;
                soff += sc;
            }
            nb += c;
            npt += pc;
            ns += sc;
        }
        if (small) {  // small bins from the top of the bin arrays (nb + ns <= kGT)
            const uint32_t b = kGT - 1u - (soff + popc_lt(sm));
            bl_ioff[b] = ioff;
            bl_icnt[b] = icnt;
            bl_moff[b] = moff | (md == GPOP_MODE_SC ? 0x80000000u : 0u);
            bl_mcnt[b] = mcnt;
        }
        if (nz) {
            const uint32_t b = boff + popc_lt(bm);
            bl_ioff[b] = ioff;
            bl_icnt[b] = icnt;
            bl_moff[b] = moff | (md == GPOP_MODE_SC ? 0x80000000u : 0u);
            bl_mcnt[b] = mcnt;
            bl_jlo[b] = jlo;
            bl_scan[b] = poff + pincl - npieces;
        }
        if (tid == 0) bl_scan[nb] = npt;  // sentinel
        __syncthreads();

        // every wave takes a contiguous run of pieces; rounds of PPW pieces
        // per wave, then all waves combine
        const uint32_t per_w = (npt + kGW - 1) / kGW;
        const uint32_t pw0 = min(wave * per_w, npt), pw1 = min(pw0 + per_w, npt);
        uint32_t bcur = 0;
        {
            uint32_t lo = 0, hi = nb ? nb : 1u;
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (bl_scan[mid] <= pw0) lo = mid; else hi = mid;
            }
            bcur = lo;
        }
        const uint32_t nrounds = (per_w + PPW - 1) / PPW;
        // Phase 1 of a round (piece metadata, id / weight / chunk-base loads)
        // is issued one round ahead, so that those loads are in flight while
        // the wave decodes and combines the current round.
        uint64_t n_raw[PPW];
        uint32_t n_wts[PPW], n_lo[PPW], n_hi[PPW], n_x0[PPW], n_mb[PPW], n_moff[PPW], n_mcnt[PPW];
        auto fetch = [&](uint32_t r) {
#pragma unroll
            for (uint32_t pi = 0; pi < PPW; ++pi) {
                const uint32_t pid = pw0 + r * PPW + pi;
                const bool live = pid < pw1;
                // a piece past the run stays in the bin of the run's last
                // piece (pw1 >= 1 whenever a round runs)
                const uint32_t pq = min(pid, pw1 - 1u);
                while (pq >= bl_scan[bcur + 1]) ++bcur;
                const uint32_t b = bcur;
                const uint32_t bioff = bl_ioff[b], bicnt = bl_icnt[b], bmo = bl_moff[b];
                n_mcnt[pi] = bl_mcnt[b];
                const bool sc = bmo & 0x80000000u;
                n_moff[pi] = bmo & 0x7FFFFFFFu;
                const uint32_t c = bioff / kChunk + bl_jlo[b] + (pid - bl_scan[b]);
                const uint32_t lo = max(bioff, c * kChunk);
                const uint32_t hi = live ? min(bioff + bicnt, c * kChunk + kChunk) : 0u;
                const uint32_t x0 = c * kChunk + lane * 4u;
                n_lo[pi] = lo;
                n_hi[pi] = hi;
                n_x0[pi] = x0;
                const bool vm = x0 + 3u >= lo && x0 < hi;
                // The loads are unconditional: a lane with no id of the piece
                // (or a piece past the wave's run) reads the 4-id group that
                // holds the bin's first id, inside the chunk-padded arrays, and
                // its words are masked off in phase 2. Loads behind a branch
                // would leave the compiler unable to count the loads in flight,
                // and the wait for this round's data would then also wait for
                // the next round's.
                const uint32_t xa = vm ? x0 : (bioff & ~3u);
                n_raw[pi] = *reinterpret_cast<const uint64_t*>((sc ? ids_sc : ids_pc) + xa);
                n_wts[pi] = 0;
                if constexpr (is_weighted(PROG))
                    n_wts[pi] = *reinterpret_cast<const uint32_t*>((sc ? w_sc : w_pc) + xa);
                // the chunk's first message index; the first piece of a bin
                // counts from the bin's first message (bit 31 of the message
                // offset says which, applied where the value is used, so that
                // nothing here waits on the load)
                const uint32_t need_mb = (uint32_t)live & (uint32_t)(lo != bioff);
                n_mb[pi] = (sc ? ch_sc : ch_pc)[need_mb ? c : bioff / kChunk];
                n_moff[pi] |= need_mb << 31;
            }
        };
        if (nrounds) fetch(0);
        for (uint32_t r = 0; r < nrounds; ++r) {
            uint32_t dst[4 * PPW], val[4 * PPW];
            uint32_t pend = 0;
            uint64_t raw[PPW];
            uint32_t wts[PPW], lo_x[PPW], hi_x[PPW], x0[PPW], mb[PPW], bmoff[PPW], bmcnt[PPW];
#pragma unroll
            for (uint32_t pi = 0; pi < PPW; ++pi) {
                raw[pi] = n_raw[pi];
                wts[pi] = n_wts[pi];
                lo_x[pi] = n_lo[pi];
                hi_x[pi] = n_hi[pi];
                x0[pi] = n_x0[pi];
                mb[pi] = n_mb[pi];
                bmoff[pi] = n_moff[pi];
                bmcnt[pi] = n_mcnt[pi];
            }
            // the fetch past the last round reads only in-bin words of pieces
            // that are not live; it is not skipped, so that no branch holds loads
            fetch(r + 1);
            // phase 2: message indices and value loads
            uint32_t vmaskall = 0;
            bool bad = false;
#pragma unroll
            for (uint32_t pi = 0; pi < PPW; ++pi) {
                uint32_t vmask = 0, fmask = 0, fc = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t x = x0[pi] + j;
                    const uint32_t id = (uint32_t)(raw[pi] >> (16 * j)) & 0xFFFFu;
                    const bool v = x >= lo_x[pi] && x < hi_x[pi];
                    const bool f = v && x > lo_x[pi] && (id & kFlag);
                    vmask |= (uint32_t)v << j;
                    fmask |= (uint32_t)f << j;
                    fc += f;
                    dst[4 * pi + j] = id & kLocalMask;
                }
                const bool from_chunk = bmoff[pi] >> 31;
                bmoff[pi] &= 0x7FFFFFFFu;
                uint32_t midx = (from_chunk ? mb[pi] : 0u) + wave_excl_small(fc);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    midx += (fmask >> j) & 1u;
                    // an id outside its bin's messages or partition marks an
                    // inconsistent bin: it is dropped (never read or written
                    // out of range) and reported once per round
                    const bool ok = (vmask >> j) & 1u;
                    const bool oob = midx >= bmcnt[pi] || dst[4 * pi + j] >= nv;
                    bad = bad || (ok && oob);
                    const bool use = ok && !oob;
                    vmask &= ~((uint32_t)(ok && oob) << j);
                    // unused lanes read the bin's first message (in range:
                    // a bin with ids has messages), so the load is unconditional
                    val[4 * pi + j] = data[bmoff[pi] + (use ? midx : 0u)];
                }
                vmaskall |= vmask << (4 * pi);
            }
            // phase 3: drop identity messages, apply weights, combine. The LDS
            // combine is unconditional: a lane with nothing to add applies the
            // identity (min with the identity, add of 0, both no-ops) to LDS
            // word `lane`, which spreads such lanes over the banks.
            unsigned long long fx[(SUM && ROUNDS) ? 4 * PPW : 1];
#pragma unroll
            for (uint32_t j = 0; j < 4 * PPW; ++j) {
                uint32_t x = ((vmaskall >> j) & 1u) ? val[j] : IDENT;
                const bool use = x != IDENT;
                if constexpr (is_weighted(PROG)) x = use ? sat_add(x, (wts[j / 4] >> (8 * (j % 4))) & 0xFFu) : IDENT;
                val[j] = x;
                my_ids += use ? 1u : 0u;
                if constexpr (!ROUNDS) {
                    const uint32_t d = use ? dst[j] : lane;
                    if constexpr (SUM)
                        atomicAdd(acc + d, use ? __double2ull_rn((double)__uint_as_float(x) * kFix) : 0ull);
                    else
                        atomicMin(st32 + d, x);
                } else if (use) {
                    if constexpr (SUM) fx[j] = __double2ull_rn((double)__uint_as_float(x) * kFix);
                    pend |= 1u << j;
                }
            }
            if (ballot(bad)) {
                if (lane == 0) gptr(G.ctrl)->bug = 1;
                bad = false;
            }
            if constexpr (ROUNDS && !SUM) {
                // write-verify rounds for the min combine
                // A lane whose value is not below the word it reads is done
                // for good (words only decrease); only lanes that wrote must
                // check, after the barrier, that their write survived.
                for (;;) {
#pragma unroll
                    for (uint32_t j = 0; j < 4 * PPW; ++j) {
                        if ((pend >> j) & 1u) {
                            if (val[j] < st32[dst[j]]) st32[dst[j]] = val[j];
                            else pend &= ~(1u << j);
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (uint32_t j = 0; j < 4 * PPW; ++j)
                        if (((pend >> j) & 1u) && !(val[j] < st32[dst[j]])) pend &= ~(1u << j);
                    if (!__syncthreads_or(pend != 0)) break;
                }
            }
            if constexpr (ROUNDS && SUM) {
                // Exact fixed-point sum. Tag rounds: every pending entry
                // writes its slot number into its destination's tag, the
                // entry whose tag survived adds. Each round retires one entry
                // per destination, so a destination hit many times in one
                // round (a high in-degree vertex) would take as many rounds;
                // after four rounds the leftovers are first summed per
                // destination inside each wave, which leaves at most one
                // entry per destination per wave for the final rounds.
                bool left = true;
                for (int tr = 0; tr < 4 && left; ++tr) {
#pragma unroll
                    for (uint32_t j = 0; j < 4 * PPW; ++j)
                        if ((pend >> j) & 1u) tag[dst[j]] = (uint16_t)(tid * 4u * PPW + j);
                    __syncthreads();
#pragma unroll
                    for (uint32_t j = 0; j < 4 * PPW; ++j) {
                        if (((pend >> j) & 1u) && tag[dst[j]] == (uint16_t)(tid * 4u * PPW + j)) {
                            acc[dst[j]] += fx[j];
                            pend &= ~(1u << j);
                        }
                    }
                    left = __syncthreads_or(pend != 0);
                }
                if (left) {
                    uint32_t adst[4 * PPW];
                    unsigned long long afx[4 * PPW];
                    uint32_t apend = 0, na = 0;
                    for (;;) {  // one destination of this wave per pass
                        const uint64_t bl = ballot(pend != 0);
                        if (!bl) break;
                        uint32_t mykey = 0;
                        bool found = false;
#pragma unroll
                        for (uint32_t j = 0; j < 4 * PPW; ++j) {
                            if (!found && ((pend >> j) & 1u)) {
                                mykey = dst[j];
                                found = true;
                            }
                        }
                        const uint32_t key = (uint32_t)__shfl((int)mykey, (int)(__ffsll((long long)bl) - 1), 64);
                        unsigned long long sum = 0;
#pragma unroll
                        for (uint32_t j = 0; j < 4 * PPW; ++j) {
                            if (((pend >> j) & 1u) && dst[j] == key) {
                                sum += fx[j];
                                pend &= ~(1u << j);
                            }
                        }
                        sum = wave_sum_u64(sum);
                        const uint32_t tl = na & 63u, ts = na >> 6;
#pragma unroll
                        for (uint32_t j = 0; j < 4 * PPW; ++j) {
                            if (lane == tl && j == ts) {
                                adst[j] = key;
                                afx[j] = sum;
                                apend |= 1u << j;
                            }
                        }
                        ++na;
                    }
                    for (;;) {  // at most kGW contenders per destination
#pragma unroll
                        for (uint32_t j = 0; j < 4 * PPW; ++j)
                            if ((apend >> j) & 1u) tag[adst[j]] = (uint16_t)(tid * 4u * PPW + j);
                        __syncthreads();
#pragma unroll
                        for (uint32_t j = 0; j < 4 * PPW; ++j) {
                            if (((apend >> j) & 1u) && tag[adst[j]] == (uint16_t)(tid * 4u * PPW + j)) {
                                acc[adst[j]] += afx[j];
                                apend &= ~(1u << j);
                            }
                        }
                        if (!__syncthreads_or(apend != 0)) break;
                    }
                }
            }
        }
        // small bins, one per thread: the bin's ids, message indices counted
        // from its first message (no chunk table), values, combine
        if constexpr (!ROUNDS) {
            for (uint32_t sb = tid; sb < ns; sb += kGT) {
                const uint32_t b = kGT - 1u - sb;
                const uint32_t bio = bl_ioff[b], bic = bl_icnt[b], bmo = bl_moff[b], bmc = bl_mcnt[b];
                const bool sc = bmo & 0x80000000u;
                const uint16_t* __restrict__ sid = (sc ? ids_sc : ids_pc) + bio;
                const uint8_t* __restrict__ swt = (sc ? w_sc : w_pc) + bio;
                const uint32_t* __restrict__ sval = data + (bmo & 0x7FFFFFFFu);
                uint32_t idv[kSmallBin], mi[kSmallBin], vv[kSmallBin], wv[kSmallBin];
#pragma unroll
                for (uint32_t i = 0; i < kSmallBin; ++i) idv[i] = i < bic ? sid[i] : 0u;
#pragma unroll
                for (uint32_t i = 0; i < kSmallBin; ++i) {
                    wv[i] = 0u;
                    if constexpr (is_weighted(PROG)) wv[i] = i < bic ? swt[i] : 0u;
                }
                uint32_t m = 0;
                bool sbad = false;
#pragma unroll
                for (uint32_t i = 0; i < kSmallBin; ++i) {
                    if (i > 0 && (idv[i] & kFlag)) ++m;
                    const bool ok = i < bic;
                    const bool oob = m >= bmc || (idv[i] & kLocalMask) >= nv;
                    sbad = sbad || (ok && oob);
                    mi[i] = (ok && !oob) ? m : 0xFFFFFFFFu;
                }
#pragma unroll
                for (uint32_t i = 0; i < kSmallBin; ++i) vv[i] = sval[mi[i] != 0xFFFFFFFFu ? mi[i] : 0u];
#pragma unroll
                for (uint32_t i = 0; i < kSmallBin; ++i) {
                    uint32_t x = mi[i] != 0xFFFFFFFFu ? vv[i] : IDENT;
                    const bool use = x != IDENT;
                    if constexpr (is_weighted(PROG)) x = use ? sat_add(x, wv[i]) : IDENT;
                    my_ids += use ? 1u : 0u;
                    const uint32_t d = use ? (idv[i] & kLocalMask) : lane;
                    if constexpr (SUM)
                        atomicAdd(acc + d, use ? __double2ull_rn((double)__uint_as_float(x) * kFix) : 0ull);
                    else
                        atomicMin(st32 + d, x);
                }
                if (sbad) gptr(G.ctrl)->bug = 1;  // inconsistent bin (never read or written out of range)
            }
        }
        __syncthreads();
    }
    __syncthreads();  // the stream's combines are complete before the state is read

    if (split) {
        // partial result of this task for the merge
        if constexpr (SUM) {
            unsigned long long* out = reinterpret_cast<unsigned long long*>(gptr(G.gpart)) + (size_t)slot * Q;
            for (uint32_t u = tid; u < nv; u += kGT) out[u] = acc[u];
        } else {
            uint32_t* out = gptr(G.gpart) + (size_t)slot * 2 * Q;
            for (uint32_t u = tid; u < nv; u += kGT) out[u] = st32[u];
        }
        const uint64_t ids64 = wave_sum_u64((uint64_t)my_ids);
        if (lane == 0) sh.r64[wave] = ids64;
        __syncthreads();
        if (tid == 0) {
            uint64_t ni = 0;
            for (uint32_t w = 0; w < kGW; ++w) ni += sh.r64[w];
            gptr(G.gflag)[slot] = 1;
            gptr(G.gat_ids)[task] = (uint32_t)ni;
        }
        return;
    }
    finish_partition<PROG>(G, P, state, it, cq, st32, acc, carry,
                           reinterpret_cast<uint64_t*>(bl_ioff), sh, my_ids, task, carry_col);
}

template <int PROG, bool ROUNDS>
__global__ __launch_bounds__(kGT) __attribute__((amdgpu_waves_per_eu(4))) void kb_gather(const Inst* __restrict__ tab,
                                                    const uint32_t* __restrict__ boff, uint32_t n) {
    const uint32_t i = batch_find(boff, n, blockIdx.x);
    const Inst& I = tab[i];
    gather_body<PROG, ROUNDS>(I.G, I.P, gptr(I.state), gptr(I.G.ctrl)->pos - 1u, blockIdx.x - boff[i]);
}

template <int PROG>
__global__ __launch_bounds__(kDT) __attribute__((amdgpu_waves_per_eu(8))) void kb_gather_dense(
    const Inst* __restrict__ tab, const uint32_t* __restrict__ boff, uint32_t n) {
    const uint32_t i = batch_find(boff, n, blockIdx.x);
    const Inst& I = tab[i];
    dense_body<PROG>(I.G, I.P, gptr(I.state), gptr(I.G.ctrl)->pos - 1u, blockIdx.x - boff[i]);
}

// Merge of a partition whose gather was split over several tasks, in two
// kernels over chunks of kMergeSpan vertices (several workgroups per
// partition, so that a few heavy partitions still spread over the chip):
//  - merge_part: per chunk, the state (min programs) or zero (sum programs),
//    reInit from the frontier bitmap, the combine of the written partials
//    (min, or exact fixed-point sum), the filter and the state write-back;
//    the keep bits go to the next frontier bitmap, the chunk's kept count,
//    kept out-edges and dangling sum to mtot;
//  - merge_list: per chunk, the next frontier list and active-edge prefix
//    from the bitmap, at the offsets the earlier chunks' counts give; chunk 0
//    writes the partition's V_a, E_a and dangling sum (chunk order, so the
//    sum is the same on every run).
constexpr uint32_t kMT = 256;        // merge workgroup
constexpr uint32_t kMW = kMT / 64;
constexpr uint32_t kMU = kMergeSpan / kMT;  // vertices per thread
// partials loaded at once: 8 of 32-bit (min programs), 4 of 64-bit (sums)
__host__ __device__ constexpr uint32_t merge_pj(int prog) { return is_sum(prog) ? 4u : 8u; }
constexpr uint32_t kWholeCol = 0xFFFFFFFFu;

template <int PROG>
__device__ __forceinline__ void merge_part_body(const Dev& G, const Params& P, uint32_t* __restrict__ state,
                                                uint32_t it, uint32_t local) {
    if (gptr(G.ctrl)->done) return;
    constexpr bool SUM = is_sum(PROG);
    const uint32_t Q = G.q, C = merge_chunks(Q), R = Q / C;
    const uint32_t sidx = local / C, c = local - sidx * C;
    const uint4 S = gptr(G.gsplit)[sidx];
    const uint32_t cq = S.x, nt = S.z, slot0 = S.w;
    const uint32_t vbase = cq << G.s;
    const uint32_t nv = min(Q, G.V - vbase);
    const uint32_t cur = it & 1u, nxt = cur ^ 1u;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    __shared__ uint32_t s_wl[64];  // written partials, compacted (at most 64 tasks per partition)
    __shared__ uint32_t s_nw;
    __shared__ uint32_t s_wc[kMW], s_we[kMW];
    __shared__ double s_wd[kMW];
    if (wave == 0) {
        const uint32_t f = lane < nt ? gptr(G.gflag)[slot0 + lane] : 0u;
        const uint32_t f0 = (uint32_t)__shfl((int)f, 0, 64);
        const uint64_t wm = ballot(f != 0u);
        if (f) s_wl[popc_lt(wm)] = slot0 + lane;
        if (lane == 0) s_nw = f0 == 2u ? kWholeCol : popc64(wm);
    }
    __syncthreads();
    const uint32_t nw = s_nw;
    const bool lead = c == 0 && tid == 0;
    if (nw == kWholeCol) {  // gathered whole by its first task
        if (lead) gptr(G.gat_ran)[G.n_gtask + sidx] = 0;
        return;
    }
    // interleaved scatter-gather: a held-back column keeps its frontier
    const bool carry_col = !SUM && isg_holds(P, cq, G.k, it);
    const bool prev = (!msg_only(PROG) || carry_col) && gptr(G.fVa[cur])[cq] > 0;  // frontier bitmap of cq is current
    if (nw == 0 && !prev) {
        if (lead) {
            gptr(G.fVa[nxt])[cq] = 0;
            gptr(G.fEa[nxt])[cq] = 0;
            gptr(G.dpart[nxt])[cq] = 0.0;
            gptr(G.gat_ran)[G.n_gtask + sidx] = 0;
        }
        return;
    }
    if (lead) gptr(G.gat_ran)[G.n_gtask + sidx] = 3;

    const uint32_t ulo = c * R, nu = R / kMT;
    const uint32_t* __restrict__ pbits = gptr(G.fbits[cur]) + (vbase >> 5);
    uint32_t* __restrict__ nbits = gptr(G.fbits[nxt]) + (vbase >> 5);
    const uint32_t* __restrict__ off = gptr(G.off);
    const double dang = SUM ? gptr(G.ctrl)->dangling : 0.0;
    // the thread's vertices u = ulo + kMT * i + tid: combined value (min
    // programs: least message, identity if none), initFunc's keep-active flag
    uint32_t m[kMU];
    unsigned long long a[kMU];
    bool was[kMU];
#pragma unroll
    for (uint32_t i = 0; i < kMU; ++i) {
        const uint32_t u = ulo + kMT * i + tid;
        const bool in = i < nu && u < nv;
        was[i] = in && prev && test_bit(pbits, u);
        if constexpr (SUM) a[i] = 0ull;
        else m[i] = kIdentMin;
    }
    constexpr uint32_t kPJ = merge_pj(PROG);
    for (uint32_t w = 0; w < nw; w += kPJ) {
        if constexpr (SUM) {
            const unsigned long long* part = reinterpret_cast<const unsigned long long*>(gptr(G.gpart));
            unsigned long long x[kPJ][kMU];
#pragma unroll
            for (uint32_t r = 0; r < kPJ; ++r) {
                const bool ok = w + r < nw;
                const unsigned long long* pj = part + (size_t)s_wl[ok ? w + r : w] * Q;
#pragma unroll
                for (uint32_t i = 0; i < kMU; ++i) {
                    const uint32_t u = ulo + kMT * i + tid;
                    x[r][i] = (ok && i < nu && u < nv) ? pj[u] : 0ull;
                }
            }
#pragma unroll
            for (uint32_t r = 0; r < kPJ; ++r)
#pragma unroll
                for (uint32_t i = 0; i < kMU; ++i) a[i] += x[r][i];
        } else {
            uint32_t x[kPJ][kMU];
#pragma unroll
            for (uint32_t r = 0; r < kPJ; ++r) {
                // past the end, re-read the first partial of the group: min
                // is idempotent
                const uint32_t* pj = gptr(G.gpart) + (size_t)s_wl[w + r < nw ? w + r : w] * 2 * Q;
#pragma unroll
                for (uint32_t i = 0; i < kMU; ++i) {
                    const uint32_t u = ulo + kMT * i + tid;
                    x[r][i] = (i < nu && u < nv) ? pj[u] : 0xFFFFFFFFu;
                }
            }
#pragma unroll
            for (uint32_t r = 0; r < kPJ; ++r)
#pragma unroll
                for (uint32_t i = 0; i < kMU; ++i) m[i] = min(m[i], x[r][i]);
        }
    }
    // filterFunc and state write-back, as for a single-task partition; the
    // stored values of the thread's vertices, then their offsets, are
    // loaded together
    uint32_t cnt = 0, edges = 0;
    double my_d = 0.0;
    bool keep[kMU], need[kMU];
    float xv[kMU];
    uint32_t o0[kMU], o1[kMU];
    if constexpr (!SUM) {
        uint32_t m0[kMU];
#pragma unroll
        for (uint32_t i = 0; i < kMU; ++i) {
            const uint32_t u = ulo + kMT * i + tid;
            const bool in = i < nu && u < nv;
            // the stored value is read only where it is compared
            m0[i] = (in && (m[i] != kIdentMin || (has_carry(PROG) && was[i]))) ? state[vbase + u] : 0u;
        }
#pragma unroll
        for (uint32_t i = 0; i < kMU; ++i) {
            const uint32_t u = ulo + kMT * i + tid;
            const bool in = i < nu && u < nv;
            const bool hit = in && m[i] != kIdentMin && (first_write(PROG) ? m0[i] == kIdentMin : m[i] < m0[i]);
            keep[i] = hit || (carry_col && was[i]);
            if constexpr (has_carry(PROG)) keep[i] = keep[i] || (in && was[i] && (it + 1u - m0[i]) < P.persist);
            if (hit) state[vbase + u] = m[i];
            need[i] = keep[i];
            xv[i] = 0.f;
        }
    } else {
#pragma unroll
        for (uint32_t i = 0; i < kMU; ++i) {
            const uint32_t u = ulo + kMT * i + tid;
            const uint32_t v = vbase + u;
            const bool in = i < nu && u < nv;
            keep[i] = false;
            xv[i] = 0.f;
            need[i] = in && (a[i] != 0ull || was[i]);  // received an amount, or was active before scatter
            if (need[i]) {
                const double y = (double)a[i] * kInvFix;
                if constexpr (PROG == P_NIBBLE) {
                    const float old = __uint_as_float(state[v]);
                    const float base = was[i] ? old * 0.5f : old;
                    const unsigned long long b = __double2ull_rn((double)base * kFix);
                    xv[i] = (float)((double)(a[i] + b) * kInvFix);
                } else if constexpr (PROG == P_PR) {
                    const double d = (double)P.damping;
                    xv[i] = (float)((1.0 - d) * P.inv_n + d * (y + dang * P.inv_n));
                    keep[i] = true;
                } else {
                    const double al = (double)P.alpha;
                    double xd = (1.0 - al) * y;
                    if (v == P.root) xd += al + (1.0 - al) * dang;
                    xv[i] = (float)xd;
                    keep[i] = xv[i] > 0.0f;
                }
                state[v] = __float_as_uint(xv[i]);
            }
        }
    }
#pragma unroll
    for (uint32_t i = 0; i < kMU; ++i) {
        const uint32_t v = vbase + ulo + kMT * i + tid;
        o0[i] = need[i] ? off[v] : 0u;
        o1[i] = need[i] ? off[v + 1] : 0u;
    }
    if constexpr (PROG == P_NIBBLE) {  // filterFunc: PR >= eps * deg (never without out-edges)
#pragma unroll
        for (uint32_t i = 0; i < kMU; ++i) {
            const uint32_t d = o1[i] - o0[i];
            keep[i] = need[i] && d > 0u && xv[i] >= P.eps * (float)d;
        }
    }
#pragma unroll
    for (uint32_t i = 0; i < kMU; ++i) {
        if (i < nu) {
            if constexpr (SUM) {
                if (need[i] && o1[i] == o0[i]) my_d += (double)xv[i];
            }
            if (keep[i]) edges += o1[i] - o0[i];
            const uint64_t km = ballot(keep[i]);
            if (lane == 0) {
                const uint32_t wi = (ulo + kMT * i + wave * 64u) >> 5;
                nbits[wi] = (uint32_t)km;
                nbits[wi + 1] = (uint32_t)(km >> 32);
            }
            cnt += popc64(km);
        }
    }
    edges = wave_sum_u32(edges);
    my_d = wave_sum_f64(my_d);
    if (lane == 0) {
        s_wc[wave] = cnt;
        s_we[wave] = edges;
        s_wd[wave] = my_d;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t tc = 0, te = 0;
        double td = 0.0;
        for (uint32_t w = 0; w < kMW; ++w) {
            tc += s_wc[w];
            te += s_we[w];
            td += s_wd[w];
        }
        const unsigned long long db = (unsigned long long)__double_as_longlong(td);
        gptr(G.mtot)[(size_t)sidx * C + c] = make_uint4(tc, te, (uint32_t)db, (uint32_t)(db >> 32));
    }
}

__device__ __forceinline__ void merge_list_body(const Dev& G, uint32_t it, uint32_t local) {
    if (gptr(G.ctrl)->done) return;
    const uint32_t Q = G.q, C = merge_chunks(Q), R = Q / C;
    const uint32_t sidx = local / C, c = local - sidx * C;
    if (gptr(G.gat_ran)[G.n_gtask + sidx] != 3u) return;
    const uint32_t cq = gptr(G.gsplit)[sidx].x;
    const uint32_t vbase = cq << G.s;
    const uint32_t nxt = (it & 1u) ^ 1u;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    __shared__ uint32_t s_wc[kMW], s_we[kMW], s_base[2];
    if (wave == 0) {
        const uint4 t = lane < C ? gptr(G.mtot)[(size_t)sidx * C + lane] : make_uint4(0u, 0u, 0u, 0u);
        const uint32_t before = wave_sum_u32(lane < c ? t.x : 0u);
        const uint32_t ebefore = wave_sum_u32(lane < c ? t.y : 0u);
        const double d = __longlong_as_double((long long)(((unsigned long long)t.w << 32) | t.z));
        if (c == 0) {
            const uint32_t tot = wave_sum_u32(t.x), etot = wave_sum_u32(t.y);
            double sd = 0.0;
            for (uint32_t j = 0; j < C; ++j) sd += __shfl(d, (int)j, 64);
            if (lane == 0) {
                gptr(G.fVa[nxt])[cq] = tot;
                gptr(G.fEa[nxt])[cq] = etot;
                gptr(G.dpart[nxt])[cq] = sd;
            }
        }
        if (lane == 0) {
            s_base[0] = before;
            s_base[1] = ebefore;
        }
    }
    // wave w lists the vertices [ulo + w * per, ulo + (w + 1) * per)
    const uint32_t per = R / kMW, ng = per / 64;
    const uint32_t ub = c * R + wave * per;
    const uint32_t* __restrict__ bits = gptr(G.fbits[nxt]) + (vbase >> 5);
    const uint32_t* __restrict__ off = gptr(G.off) + vbase;
    uint32_t deg[kMU];
    uint64_t km[kMU];
    uint32_t cnt = 0, edges = 0;
    // bitmap words of every group first, then the offsets of the kept
    // vertices, each batch issued together
#pragma unroll
    for (uint32_t g = 0; g < kMU; ++g) {
        const uint32_t u0 = ub + 64u * g;
        km[g] = g < ng ? ((uint64_t)bits[u0 >> 5] | ((uint64_t)bits[(u0 >> 5) + 1] << 32)) : 0ull;
    }
    uint32_t o0[kMU], o1[kMU];
#pragma unroll
    for (uint32_t g = 0; g < kMU; ++g) {
        const uint32_t u = ub + 64u * g + lane;
        const bool kp = (km[g] >> lane) & 1u;
        o0[g] = kp ? off[u] : 0u;
        o1[g] = kp ? off[u + 1] : 0u;
    }
#pragma unroll
    for (uint32_t g = 0; g < kMU; ++g) {
        deg[g] = o1[g] - o0[g];
        cnt += popc64(km[g]);
        edges += deg[g];
    }
    edges = wave_sum_u32(edges);
    if (lane == 0) {
        s_wc[wave] = cnt;
        s_we[wave] = edges;
    }
    __syncthreads();
    uint32_t pos = s_base[0], epos = s_base[1];
    for (uint32_t w = 0; w < wave; ++w) {
        pos += s_wc[w];
        epos += s_we[w];
    }
    uint16_t* __restrict__ nlist = gptr(G.flist[nxt]) + vbase;
    uint32_t* __restrict__ npre = gptr(G.fpre[nxt]) + vbase;
#pragma unroll
    for (uint32_t g = 0; g < kMU; ++g) {
        if (g < ng) {
            const uint32_t u = ub + 64u * g + lane;
            const uint32_t dincl = wave_incl_scan(deg[g]);
            if ((km[g] >> lane) & 1u) {
                const uint32_t at = pos + popc_lt(km[g]);
                nlist[at] = (uint16_t)u;
                npre[at] = epos + dincl - deg[g];
            }
            pos += popc64(km[g]);
            epos += last_lane(dincl);
        }
    }
}

template <int PROG>
__global__ __launch_bounds__(kMT) void kb_merge_part(const Inst* __restrict__ tab,
                                                     const uint32_t* __restrict__ boff, uint32_t n) {
    const uint32_t i = batch_find(boff, n, blockIdx.x);
    const Inst& I = tab[i];
    merge_part_body<PROG>(I.G, I.P, gptr(I.state), gptr(I.G.ctrl)->pos - 1u, blockIdx.x - boff[i]);
}

__global__ __launch_bounds__(kMT) void kb_merge_list(const Inst* __restrict__ tab,
                                                     const uint32_t* __restrict__ boff, uint32_t n) {
    const uint32_t i = batch_find(boff, n, blockIdx.x);
    const Inst& I = tab[i];
    merge_list_body(I.G, gptr(I.G.ctrl)->pos - 1u, blockIdx.x - boff[i]);
}

// Batched: run status {done, iterations} per run, and the iteration limit of
// the next batched run (relative to where each run stands).
__global__ void kb_status(const Inst* __restrict__ tab, uint32_t n, uint32_t* __restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Ctrl* C = tab[i].G.ctrl;  // one run per lane: not a uniform pointer
    out[2 * i] = C->done;
    out[2 * i + 1] = C->pos - C->run_start;  // iterations of the current run
}

__global__ void kb_limits(const Inst* __restrict__ tab, uint32_t n, uint32_t max_iter) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Ctrl* C = tab[i].G.ctrl;  // one run per lane: not a uniform pointer
    const uint64_t lim = (uint64_t)C->pos + max_iter;
    C->max_it = lim > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)lim;
    C->run_start = C->pos;
    C->done &= ~2u;  // resume a paused run
}

template <int PROG>
static hipError_t prep_batch_gather_p(const BatchGrid& B) {
    const bool r = B.rounds;
    hipError_t e = hipFuncSetAttribute(
        r ? reinterpret_cast<const void*>(kb_gather<PROG, true>) : reinterpret_cast<const void*>(kb_gather<PROG, false>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)gather_lds_bytes(PROG, B.q_max, r));
    if (e == hipSuccess && !r && B.streams)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(kb_gather_dense<PROG>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)dense_layout(PROG, B.q_max).total);
    return e;
}

template <int PROG>
static hipError_t launch_batch_gather_p(const BatchGrid& B, hipStream_t st) {
    const size_t lds = gather_lds_bytes(PROG, B.q_max, B.rounds);
    if (B.nb_gather) {
        if (B.rounds)
            hipLaunchKernelGGL((kb_gather<PROG, true>), dim3(B.nb_gather), dim3(kGT), lds, st, B.tab, B.b_gather, B.n);
        else
            hipLaunchKernelGGL((kb_gather<PROG, false>), dim3(B.nb_gather), dim3(kGT), lds, st, B.tab, B.b_gather, B.n);
        // dense iterations of graphs with column streams (the kernel returns
        // at once in any other iteration)
        if (!B.rounds && B.streams)
            hipLaunchKernelGGL(kb_gather_dense<PROG>, dim3(B.nb_gather), dim3(kDT), dense_layout(PROG, B.q_max).total, st,
                               B.tab, B.b_gather, B.n);
    }
    return hipGetLastError();
}

template <int PROG>
static hipError_t launch_batch_merge_p(const BatchGrid& B, hipStream_t st) {
    if (B.nb_merge) {
        hipLaunchKernelGGL(kb_merge_part<PROG>, dim3(B.nb_merge), dim3(kMT), 0, st, B.tab, B.b_merge, B.n);
        hipLaunchKernelGGL(kb_merge_list, dim3(B.nb_merge), dim3(kMT), 0, st, B.tab, B.b_merge, B.n);
    }
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

hipError_t prepare_batch_gather(const BatchGrid& B, int prog) { GPOP_PROG_SWITCH(prep_batch_gather_p, B) }

hipError_t launch_batch_gather(const BatchGrid& B, int prog, hipStream_t st) {
    GPOP_PROG_SWITCH(launch_batch_gather_p, B, st)
}

hipError_t launch_batch_merge(const BatchGrid& B, int prog, hipStream_t st) {
    GPOP_PROG_SWITCH(launch_batch_merge_p, B, st)
}

#undef GPOP_PROG_SWITCH

hipError_t launch_batch_limits(const BatchGrid& B, uint32_t max_iter, hipStream_t st) {
    hipLaunchKernelGGL(kb_limits, dim3((B.n + 63) / 64), dim3(64), 0, st, B.tab, B.n, max_iter);
    return hipGetLastError();
}

hipError_t launch_batch_status(const BatchGrid& B, uint32_t* out, hipStream_t st) {
    hipLaunchKernelGGL(kb_status, dim3((B.n + 63) / 64), dim3(64), 0, st, B.tab, B.n, out);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Initial vertex values (val[] initialisation of each application) and the
// dangling partial sums of the initial state, one workgroup per partition.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_state_init(Dev G, Params P, int prog,
                                                    uint32_t* __restrict__ state) {
    const uint32_t p = blockIdx.x;
    const uint32_t vbase = p << G.s;
    const uint32_t nv = min(G.q, G.V - vbase);
    __shared__ double s_rd[4];
    double my_d = 0.0;
    for (uint32_t u = threadIdx.x; u < nv; u += 256) {
        const uint32_t v = vbase + u;
        uint32_t x;
        switch (prog) {
            case P_CC: x = v; break;
            case P_PR: x = __float_as_uint((float)P.inv_n); break;
            case P_PPR: x = __float_as_uint(v == P.root ? 1.0f : 0.0f); break;
            case P_PARENT: x = v == P.root ? v : 0xFFFFFFFFu; break;
            case P_NIBBLE: x = __float_as_uint(v == P.root ? 1.0f : 0.0f); break;
            default: x = v == P.root ? 0u : 0xFFFFFFFFu; break;
        }
        state[v] = x;
        if ((prog == P_PR || prog == P_PPR) && gptr(G.off)[v + 1] == gptr(G.off)[v])
            my_d += (double)__uint_as_float(x);
    }
    my_d = wave_sum_f64(my_d);
    if ((threadIdx.x & 63u) == 0) s_rd[threadIdx.x >> 6] = my_d;
    __syncthreads();
    if (threadIdx.x == 0) {
        gptr(G.dpart[0])[p] = s_rd[0] + s_rd[1] + s_rd[2] + s_rd[3];
        gptr(G.dpart[1])[p] = 0.0;
        gptr(G.fVa[0])[p] = 0;
        gptr(G.fEa[0])[p] = 0;
        gptr(G.fVa[1])[p] = 0;
        gptr(G.fEa[1])[p] = 0;
        gptr(G.mode)[p] = GPOP_MODE_NONE;
    }
    if (p == 0 && threadIdx.x == 0) {
        gptr(G.ctrl)->done = 0;
        gptr(G.ctrl)->iters = 0;
        gptr(G.ctrl)->frontier = 0;
        gptr(G.ctrl)->dangling = 0.0;
        gptr(G.ctrl)->fin_it = 0;
        gptr(G.ctrl)->pos = 0;
        gptr(G.ctrl)->max_it = 0xFFFFFFFFu;
        gptr(G.ctrl)->run_start = 0;
    }
}

hipError_t launch_state_init(const Dev& G, const Params& P, int prog, uint32_t* state,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_state_init, dim3(G.k), dim3(256), 0, st, G, P, prog, state);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// loadFrontier: byte marks (plain idempotent stores, so duplicates are
// harmless), then per-partition ballot compaction into the list, bitmap and
// V_a / E_a of frontier buffer `buf`.
// ---------------------------------------------------------------------------
__global__ void k_fill_u8(uint8_t* __restrict__ p, uint64_t n, uint8_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_u8, dim3((uint32_t)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

__global__ void k_mark(Dev G, const uint32_t* __restrict__ verts, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t v = verts[i];
        if (v < G.V) gptr(G.marks)[v] = 1;
        else gptr(G.ctrl)->err = 1;
    }
}

__global__ __launch_bounds__(1024) void k_marks_to_frontier(Dev G, int all) {
    const uint32_t p = blockIdx.x;
    const uint32_t buf = gptr(G.ctrl)->pos & 1u;  // the buffer the next plan reads
    const uint32_t vbase = p << G.s;
    const uint32_t nv = min(G.q, G.V - vbase);
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    __shared__ uint32_t s_wc[16], s_ws[16];
    uint16_t* list = gptr(G.flist[buf]) + vbase;
    uint32_t* pre = gptr(G.fpre[buf]) + vbase;
    uint32_t* bits = gptr(G.fbits[buf]) + (vbase >> 5);
    uint32_t running = 0, erun = 0;
    for (uint32_t u0 = 0; u0 < nv; u0 += 1024) {
        const uint32_t u = u0 + tid;
        const bool keep = u < nv && (all || gptr(G.marks)[vbase + u]);
        const uint32_t deg = keep ? gptr(G.off)[vbase + u + 1] - gptr(G.off)[vbase + u] : 0u;
        const uint64_t bm = ballot(keep);
        const uint32_t dincl = wave_incl_scan(deg);
        if (lane == 0 && u0 + wave * 64u < G.q) {
            const uint32_t wi = (u0 + wave * 64u) >> 5;
            bits[wi] = (uint32_t)bm;
            bits[wi + 1] = (uint32_t)(bm >> 32);
        }
        if (lane == 63) {
            s_wc[wave] = popc64(bm);
            s_ws[wave] = dincl;
        }
        __syncthreads();
        uint32_t before = 0, tot = 0, eb = 0, et = 0;
        for (uint32_t w = 0; w < 16; ++w) {
            if (w < wave) {
                before += s_wc[w];
                eb += s_ws[w];
            }
            tot += s_wc[w];
            et += s_ws[w];
        }
        if (keep) {
            const uint32_t pos = running + before + popc_lt(bm);
            list[pos] = (uint16_t)u;
            pre[pos] = erun + eb + dincl - deg;
        }
        running += tot;
        erun += et;
        __syncthreads();
    }
    if (tid == 0) {
        gptr(G.fVa[buf])[p] = running;
        gptr(G.fEa[buf])[p] = erun;
    }
    if (p == 0 && tid == 0) {
        gptr(G.ctrl)->done = 0;
    }
}

hipError_t launch_set_frontier(const Dev& G, const uint32_t* verts, uint32_t n, int all, hipStream_t st) {
    if (!all) {
        const uint64_t nm = (uint64_t)G.k * G.q;
        hipLaunchKernelGGL(k_fill_u8, dim3(1024), dim3(256), 0, st, G.marks, nm, (uint8_t)0);
        if (n) {
            const uint32_t blocks = min(1024u, (n + 255u) / 256u);
            hipLaunchKernelGGL(k_mark, dim3(blocks), dim3(256), 0, st, G, verts, n);
        }
    }
    hipLaunchKernelGGL(k_marks_to_frontier, dim3(G.k), dim3(1024), 0, st, G, all);
    return hipGetLastError();
}

}  // namespace gpop
