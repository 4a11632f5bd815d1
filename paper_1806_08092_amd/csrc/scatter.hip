// Scatter phase: mode selection, source-centric scatter and partition-centric
// scatter (Algorithm 2 scatter phase; Algorithm 3; Sec. 3.2).
#include "launch.h"

namespace gpop {

// ---------------------------------------------------------------------------
// Ordered multi-split of one partition's edges by destination partition.
//
// Source-centric scatter (Algorithm 2, scatter loop): for active v in
// ascending order, for each neighbouring partition q in ascending order,
// insert {val[v], ids of v's out-neighbours in q} into bin[p][q]. Successive
// messages to q land at consecutive insertion points of bin[p][q]
// (Sec. 3.1.2, source-centric mode). On the GPU the insertion points are
// exclusive prefix sums: a workgroup of W waves takes the active list in
// rounds of W*R vertices (wave w owns a contiguous block of R), flattens the
// edges of 64 vertices at a time across the lanes, groups lanes by
// destination partition with a ballot match on the partition id bits, counts
// per (wave, q) in LDS (pass 0), scans the counts across waves (so wave w
// starts where wave w-1 ends), and writes (pass 1). Only the lowest lane of
// each match group touches a counter, so no two lanes of a wave update the
// same word and no atomics are needed; waves own disjoint counter rows.
//
// The same routine builds the static partition-node layout once with every
// vertex active: MODE 1 counts messages and ids per (p, q), MODE 2 writes
// N_i^p(q) (png_src) and the static ids (Algorithm 3 reuses them).
// MODE 0 is the per-iteration source-centric scatter.
// ---------------------------------------------------------------------------
constexpr uint32_t kR = 256;  // vertices per wave per round

template <int PROG, int MODE, int W>
__global__ __launch_bounds__(W * 64) void k_sc(Dev G, Params P, const uint32_t* __restrict__ state,
                                               uint32_t it) {
    const uint32_t p = blockIdx.x;
    const uint32_t cur = it & 1u;
    if constexpr (MODE == 0) {
        if (G.ctrl->done) return;
        if (G.mode[p] != GPOP_MODE_SC) return;
    }
    const uint32_t k = G.k, s = G.s, qmask = G.q - 1u;
    const uint32_t vbase = p << s;
    const uint32_t nv = min(G.q, G.V - vbase);
    const uint32_t nact = (MODE == 0) ? G.fVa[cur][p] : nv;
    const uint16_t* __restrict__ alist = G.flist[cur] + vbase;
    const uint32_t* __restrict__ rmoff = G.bin_moff + (size_t)p * k;
    const uint32_t* __restrict__ rioff = G.bin_ioff + (size_t)p * k;
    const uint32_t* __restrict__ off = G.off;
    const uint32_t* __restrict__ cols = G.cols;

    extern __shared__ uint32_t lds[];
    uint32_t* cnt_i = lds;              // [W][k] ids per (wave, q)
    uint32_t* cnt_m = lds + W * k;      // [W][k] messages per (wave, q)
    uint32_t* gi = lds + 2 * W * k;     // [k] running ids of bin[p][q]
    uint32_t* gm = gi + k;              // [k] running messages of bin[p][q]

    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    for (uint32_t j = tid; j < k; j += W * 64) {
        gi[j] = 0;
        gm[j] = 0;
    }

    for (uint32_t rbase = 0; rbase < nact; rbase += W * kR) {
        for (uint32_t j = tid; j < W * k; j += W * 64) {
            cnt_i[j] = 0;
            cnt_m[j] = 0;
        }
        __syncthreads();
        const uint32_t wbeg = rbase + wave * kR;
        const uint32_t wend = min(wbeg + kR, nact);
        uint32_t* my_i = cnt_i + wave * k;
        uint32_t* my_m = cnt_m + wave * k;

        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1) {
                __syncthreads();
                // exclusive scan of the counts over waves, per destination q
                for (uint32_t j = tid; j < k; j += W * 64) {
                    uint32_t ri = gi[j], rm = gm[j];
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        uint32_t ti = cnt_i[w * k + j], tm = cnt_m[w * k + j];
                        cnt_i[w * k + j] = ri;
                        cnt_m[w * k + j] = rm;
                        ri += ti;
                        rm += tm;
                    }
                    gi[j] = ri;
                    gm[j] = rm;
                }
                __syncthreads();
                if constexpr (MODE == 1) break;
            }
            for (uint32_t x0 = wbeg; x0 < wend; x0 += 64) {
                const uint32_t i = x0 + lane;
                const bool vv = i < wend;
                const uint32_t vl = vv ? ((MODE == 0) ? (uint32_t)alist[i] : i) : 0u;
                const uint32_t v = vbase + vl;
                const uint32_t rs = vv ? off[v] : 0u;
                const uint32_t deg = vv ? off[v + 1] - rs : 0u;
                uint32_t val = vl;
                if constexpr (MODE == 0) {
                    if (vv && pass == 1) val = scatter_value<PROG>(G, state, v);
                }
                const uint32_t incl = wave_incl_scan(deg);
                const uint32_t total = __shfl(incl, 63, 64);
                for (uint32_t f0 = 0; f0 < total; f0 += 64) {
                    const uint32_t f = f0 + lane;
                    const bool valid = f < total;
                    // owner lane: number of window vertices whose edges end at or before f
                    uint32_t o = 0;
#pragma unroll
                    for (uint32_t step = 32; step >= 1; step >>= 1) {
                        uint32_t c = __shfl(incl, (int)(o + step - 1), 64);
                        if (c <= f) o += step;
                    }
                    const uint32_t o_rs = __shfl(rs, (int)o, 64);
                    const uint32_t o_incl = __shfl(incl, (int)o, 64);
                    const uint32_t o_deg = __shfl(deg, (int)o, 64);
                    const uint32_t o_val = __shfl(val, (int)o, 64);
                    const uint32_t e = o_rs + (f - (o_incl - o_deg));
                    const uint32_t col = valid ? cols[e] : 0u;
                    const uint32_t key = col >> s;
                    const bool flag = valid && (e == o_rs || (cols[e - 1] >> s) != key);
                    // lanes with the same destination partition
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
                        bi = my_i[key];
                        bm = my_m[key];
                    }
                    if (valid && rank_i == 0) {
                        my_i[key] = bi + popc64(peers);
                        my_m[key] = bm + popc64(fpeers);
                    }
                    if (pass == 1 && valid) {
                        const uint32_t pos = rioff[key] + bi + rank_i;
                        const uint32_t midx = bm + m_le - 1u;
                        // positions must stay inside the static capacity of bin[p][key]
                        if (pos >= rioff[key + 1] || midx >= rmoff[key + 1] - rmoff[key]) {
                            G.ctrl->bug = 1;
                            continue;
                        }
                        const uint16_t idw = (uint16_t)((col & qmask) | (flag ? kFlag : 0u));
                        if constexpr (MODE == 0) {
                            if (flag) G.data[rmoff[key] + midx] = o_val;
                            G.sc_ids[pos] = idw;
                            if constexpr (is_weighted(PROG)) G.sc_w[pos] = G.w[e];
                            if ((pos & (kChunk - 1)) == 0) G.sc_chunk[pos / kChunk] = midx;
                        } else {
                            if (flag) G.png_src[rmoff[key] + midx] = (uint16_t)o_val;
                            G.png_ids[pos] = idw;
                            if (G.w) G.png_w[pos] = G.w[e];
                            if ((pos & (kChunk - 1)) == 0) G.png_chunk[pos / kChunk] = midx;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }

    // epilogue: per-bin totals of this source partition
    if constexpr (MODE == 0) {
        uint32_t tm = 0, ti = 0;
        for (uint32_t j = tid; j < k; j += W * 64) {
            G.sc_cnt[(size_t)j * k + p] = make_uint2(gm[j], gi[j]);
            tm += gm[j];
            ti += gi[j];
        }
        tm = wave_sum_u32(tm);
        ti = wave_sum_u32(ti);
        __syncthreads();
        if (lane == 0) {
            cnt_i[wave] = ti;
            cnt_m[wave] = tm;
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t a = 0, b = 0;
            for (int w = 0; w < W; ++w) {
                a += cnt_m[w];
                b += cnt_i[w];
            }
            G.sc_tot[p] = make_uint2(a, b);
        }
    } else if constexpr (MODE == 1) {
        for (uint32_t j = tid; j < k; j += W * 64) {
            G.cnt_m[(size_t)p * k + j] = gm[j];
            G.cnt_i[(size_t)p * k + j] = gi[j];
        }
    }
}

int sc_waves_for(uint32_t k) {
    // (2W + 2) * k words of LDS must fit in 80 KB
    if ((2 * 4 + 2) * (size_t)k * 4 <= 81920) return 4;
    if ((2 * 2 + 2) * (size_t)k * 4 <= 81920) return 2;
    return 1;
}

size_t sc_lds_bytes(uint32_t k, int waves) { return (size_t)(2 * waves + 2) * k * 4; }

template <int PROG, int MODE, int W>
static hipError_t launch_sc_w(const Dev& G, const Params& P, const uint32_t* state, uint32_t it,
                              hipStream_t st) {
    const size_t lds = sc_lds_bytes(G.k, W);
    auto fn = k_sc<PROG, MODE, W>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(G.k), dim3(W * 64), lds, st, G, P, state, it);
    return hipGetLastError();
}

template <int PROG, int MODE>
static hipError_t launch_sc_any(const Dev& G, const Params& P, const uint32_t* state, uint32_t it,
                                hipStream_t st) {
    switch (sc_waves_for(G.k)) {
        case 4: return launch_sc_w<PROG, MODE, 4>(G, P, state, it, st);
        case 2: return launch_sc_w<PROG, MODE, 2>(G, P, state, it, st);
        default: return launch_sc_w<PROG, MODE, 1>(G, P, state, it, st);
    }
}

hipError_t launch_sc_build(const Dev& G, int fill, hipStream_t st) {
    Params P{};
    return fill ? launch_sc_any<P_BFS, 2>(G, P, nullptr, 0, st)
                : launch_sc_any<P_BFS, 1>(G, P, nullptr, 0, st);
}

hipError_t launch_scatter_sc(const Dev& G, const Params& P, int prog, const uint32_t* state,
                             uint32_t it, hipStream_t st) {
    switch (prog) {
        case P_BFS: return launch_sc_any<P_BFS, 0>(G, P, state, it, st);
        case P_CC: return launch_sc_any<P_CC, 0>(G, P, state, it, st);
        case P_SSSP: return launch_sc_any<P_SSSP, 0>(G, P, state, it, st);
        case P_PR: return launch_sc_any<P_PR, 0>(G, P, state, it, st);
        case P_PPR: return launch_sc_any<P_PPR, 0>(G, P, state, it, st);
        case P_CARRY: return launch_sc_any<P_CARRY, 0>(G, P, state, it, st);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Partition-centric scatter (Algorithm 3): for every q and every v in
// N_i^p(q), write val[v] into bin[p][q]. The static source list png_src makes
// this a pure stream: slot i of the partition's message range gets the value
// of source png_src[i]. The partition's outgoing values are staged once in
// LDS (the partition's vertex data is the cached working set), inactive
// vertices contribute the combine identity. Work is cut into static tasks of
// at most kPcTask slots so hub partitions spread over many workgroups.
// ---------------------------------------------------------------------------
template <int PROG>
__global__ __launch_bounds__(256) void k_pc(Dev G, Params P, const uint32_t* __restrict__ state,
                                            uint32_t it) {
    if (G.ctrl->done) return;
    const uint4 t = G.pctask[blockIdx.x];
    const uint32_t p = t.x;
    if (G.mode[p] != GPOP_MODE_PC) return;
    const uint32_t cur = it & 1u;
    const uint32_t vbase = p << G.s;
    const uint32_t nv = min(G.q, G.V - vbase);
    extern __shared__ uint32_t mv[];
    const uint32_t* __restrict__ bits = G.fbits[cur] + (vbase >> 5);
    for (uint32_t v = threadIdx.x; v < nv; v += 256)
        mv[v] = test_bit(bits, v) ? scatter_value<PROG>(G, state, vbase + v) : ident_of<PROG>();
    __syncthreads();
    const uint16_t* __restrict__ src = G.png_src;
    uint32_t* __restrict__ data = G.data;
    // aligned middle in groups of 4 slots (8-byte source loads, 16-byte stores)
    uint32_t a = t.y, b = t.z;
    uint32_t a4 = min((a + 3u) & ~3u, b);
    for (uint32_t i = a + threadIdx.x; i < a4; i += 256) data[i] = mv[src[i]];
    uint32_t b4 = a4 + ((b - a4) & ~3u);
    for (uint32_t i = a4 + 4u * threadIdx.x; i < b4; i += 1024) {
        const uint2 sv = *reinterpret_cast<const uint2*>(src + i);
        uint4 o;
        o.x = mv[sv.x & 0xFFFFu];
        o.y = mv[sv.x >> 16];
        o.z = mv[sv.y & 0xFFFFu];
        o.w = mv[sv.y >> 16];
        *reinterpret_cast<uint4*>(data + i) = o;
    }
    for (uint32_t i = b4 + threadIdx.x; i < b; i += 256) data[i] = mv[src[i]];
}

template <int PROG>
static hipError_t launch_pc_p(const Dev& G, const Params& P, const uint32_t* state, uint32_t it,
                              hipStream_t st) {
    if (G.n_pctask == 0) return hipSuccess;
    const size_t lds = (size_t)G.q * 4;
    auto fn = k_pc<PROG>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(G.n_pctask), dim3(256), lds, st, G, P, state, it);
    return hipGetLastError();
}

hipError_t launch_scatter_pc(const Dev& G, const Params& P, int prog, const uint32_t* state,
                             uint32_t it, hipStream_t st) {
    switch (prog) {
        case P_BFS: return launch_pc_p<P_BFS>(G, P, state, it, st);
        case P_CC: return launch_pc_p<P_CC>(G, P, state, it, st);
        case P_SSSP: return launch_pc_p<P_SSSP>(G, P, state, it, st);
        case P_PR: return launch_pc_p<P_PR>(G, P, state, it, st);
        case P_PPR: return launch_pc_p<P_PPR>(G, P, state, it, st);
        case P_CARRY: return launch_pc_p<P_CARRY>(G, P, state, it, st);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Mode selection (Sec. 3.2, Eq. 1). With r^p = M^p / E^p the
// partition-centric volume E^p((r^p+1)s_i + 2 r^p s_v) + k s_i is the integer
// (M^p + E^p) s_i + 2 M^p s_v + k s_i, and E^p times the source-centric volume
// 2 r^p E_a s_v + 3 E_a s_i + V_a s_i is 2 M^p E_a s_v + (3 E_a + V_a) s_i E^p.
// PC is chosen iff cost_PC / BW_PC <= cost_SC / BW_SC, evaluated exactly in
// 128-bit integers with BW_PC / BW_SC = ratio_num / ratio_den; ties pick PC.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint8_t analytical_mode(const Dev& G, const Params& P, uint32_t p,
                                                   uint32_t Va, uint32_t Ea) {
    typedef unsigned __int128 u128;
    const uint64_t Ep = G.part_E[p], Mp = G.part_M[p];
    const uint64_t si = P.s_i, sv = P.s_v;
    const uint64_t cost_pc = (Mp + Ep) * si + 2ull * Mp * sv + (uint64_t)G.k * si;
    const u128 lhs = (u128)cost_pc * Ep * P.ratio_den;
    const u128 sc_scaled = (u128)(2ull * sv) * Mp * Ea + (u128)((3ull * Ea + Va) * si) * Ep;
    const u128 rhs = sc_scaled * P.ratio_num;
    return lhs <= rhs ? (uint8_t)GPOP_MODE_PC : (uint8_t)GPOP_MODE_SC;
}

// Fills the stats record of iteration it - 1 (source-centric totals and ids
// gathered) from per-partition values the previous iteration wrote. Reads
// mode[], so it must run before the next plan overwrites it.
__device__ void finalize_prev(const Dev& G, uint32_t it) {
    __shared__ uint64_t red[4][16];
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    uint64_t scm = 0, sci = 0, gid = 0, gpt = 0;
    for (uint32_t p = tid; p < G.k; p += blockDim.x) {
        if (G.mode[p] == GPOP_MODE_SC) {
            const uint2 t = G.sc_tot[p];
            scm += t.x;
            sci += t.y;
        }
        const uint32_t g = G.gat_ids[p];
        gid += g;
        gpt += g ? 1u : 0u;
    }
    scm = wave_sum_u64(scm);
    sci = wave_sum_u64(sci);
    gid = wave_sum_u64(gid);
    gpt = wave_sum_u64(gpt);
    if (lane == 0) {
        red[0][wave] = scm;
        red[1][wave] = sci;
        red[2][wave] = gid;
        red[3][wave] = gpt;
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t a = 0, b = 0, c = 0, d = 0;
        for (uint32_t w = 0; w < blockDim.x / 64; ++w) {
            a += red[0][w];
            b += red[1][w];
            c += red[2][w];
            d += red[3][w];
        }
        gpop_iter_stats* r = G.log + ((it - 1) % kLogCap);
        r->sc_msgs = a;
        r->sc_ids = b;
        r->gathered_ids = c;
        r->gather_parts = (uint32_t)d;
    }
    __syncthreads();
}

__global__ __launch_bounds__(1024) void k_finalize(Dev G, uint32_t it) {
    if (it > 0) finalize_prev(G, it);
}

__global__ __launch_bounds__(1024) void k_plan(Dev G, Params P, uint32_t it) {
    Ctrl* C = G.ctrl;
    if (C->done) return;
    const uint32_t cur = it & 1u;
    if (it > 0) finalize_prev(G, it);
    __shared__ uint64_t red[6][16];
    __shared__ double dred[16];
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    uint64_t va = 0, ea = 0, nsc = 0, npc = 0, pcm = 0, pci = 0;
    double dang = 0.0;
    for (uint32_t p = tid; p < G.k; p += 1024) {
        const uint32_t Va = G.fVa[cur][p], Ea = G.fEa[cur][p];
        uint8_t md = GPOP_MODE_NONE;
        if (Va) {
            if (P.selector == GPOP_SEL_FORCE_SC) md = GPOP_MODE_SC;
            else if (P.selector == GPOP_SEL_FORCE_PC) md = GPOP_MODE_PC;
            else md = analytical_mode(G, P, p, Va, Ea);
        }
        G.mode[p] = md;
        va += Va;
        ea += Ea;
        nsc += md == GPOP_MODE_SC;
        npc += md == GPOP_MODE_PC;
        if (md == GPOP_MODE_PC) {
            pcm += G.part_M[p];
            pci += G.part_E[p];
        }
        dang += G.dpart[cur][p];
    }
    va = wave_sum_u64(va);
    ea = wave_sum_u64(ea);
    nsc = wave_sum_u64(nsc);
    npc = wave_sum_u64(npc);
    pcm = wave_sum_u64(pcm);
    pci = wave_sum_u64(pci);
    dang = wave_sum_f64(dang);
    if (lane == 0) {
        red[0][wave] = va;
        red[1][wave] = ea;
        red[2][wave] = nsc;
        red[3][wave] = npc;
        red[4][wave] = pcm;
        red[5][wave] = pci;
        dred[wave] = dang;
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t t[6] = {0, 0, 0, 0, 0, 0};
        double d = 0.0;
        for (int w = 0; w < 16; ++w) {
            for (int j = 0; j < 6; ++j) t[j] += red[j][w];
            d += dred[w];
        }
        C->frontier = t[0];
        C->dangling = d;
        if (t[0] == 0) {
            C->done = 1;
        } else {
            C->iters = it + 1;
            gpop_iter_stats* r = G.log + (it % kLogCap);
            r->active_vertices = t[0];
            r->active_edges = t[1];
            r->sc_parts = (uint32_t)t[2];
            r->pc_parts = (uint32_t)t[3];
            r->pc_msgs = t[4];
            r->pc_ids = t[5];
            r->sc_msgs = 0;
            r->sc_ids = 0;
            r->gathered_ids = 0;
            r->gather_parts = 0;
        }
    }
}

hipError_t launch_plan(const Dev& G, const Params& P, uint32_t it, hipStream_t st) {
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, st, G, P, it);
    return hipGetLastError();
}

hipError_t launch_finalize(const Dev& G, uint32_t it, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, st, G, it);
    return hipGetLastError();
}

}  // namespace gpop
