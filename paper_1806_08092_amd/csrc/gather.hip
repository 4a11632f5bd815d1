// Gather phase (Algorithm 2: reInit, gather, filter) plus state and frontier
// initialisation.
#include "launch.h"

namespace gpop {

constexpr uint32_t kGT = 1024;    // gather threads per workgroup
constexpr uint32_t kGW = kGT / 64;

// LDS layout of the gather workgroup (bytes, all offsets 16-aligned).
struct GatherLds {
    size_t state, flag_a, flag_b, tag, bl_ioff, bl_icnt, bl_moff, bl_mcnt, bl_scan, total;
};

__host__ __device__ inline GatherLds gather_layout(bool sum, uint32_t q) {
    GatherLds L{};
    size_t o = 0;
    L.state = o;  o += (size_t)q * (sum ? 8 : 4);
    L.tag = o;    o += sum ? ((size_t)q * 2 + 15) / 16 * 16 : 0;
    L.flag_a = o; o += ((size_t)q + 15) / 16 * 16;
    L.flag_b = o; o += ((size_t)q + 15) / 16 * 16;
    L.bl_ioff = o; o += kGT * 4;
    L.bl_icnt = o; o += kGT * 4;
    L.bl_moff = o; o += kGT * 4;
    L.bl_mcnt = o; o += kGT * 4;
    L.bl_scan = o; o += (kGT + 4) * 4;
    L.total = o;
    return L;
}

size_t gather_lds_bytes(int prog, uint32_t q) { return gather_layout(is_sum(prog), q).total; }

// Exclusive prefix of a 0..7 per-lane count across the wave, from bit-plane
// ballots.
__device__ __forceinline__ uint32_t wave_excl_small(uint32_t c) {
    return popc_lt(ballot(c & 1u)) + 2u * popc_lt(ballot(c & 2u)) + 4u * popc_lt(ballot(c & 4u));
}

// One workgroup per destination partition cq. The partition's vertex state
// lives in LDS for the whole phase (the cached vertex data of Sec. 3: each
// message updates on-chip state, each bin is read once, sequentially).
//
// Bins bin[p][cq] are enumerated from the per-partition modes and counts (the
// two-level active list: a partition is gathered only if some bin of its
// column is non-empty or it has active vertices; inside it only non-empty
// bins are read). Each bin is cut into 256-id-aligned pieces that one wave
// decodes on its own: message index of an id = chunk-table base + number of
// message-start flags after the piece start.
//
// Combining is atomic-free. For min programs each round every pending lane
// reads the state word and writes its value if smaller; after a barrier each
// lane re-reads, and only lanes whose value is still smaller stay pending.
// Every round lowers each contested word strictly, so the loop ends with the
// exact minimum whatever the write order. For sum programs a round lets every
// pending lane write its slot number into a per-vertex tag; after a barrier
// the lane that finds its own number adds its value (one writer per word),
// the rest retry. Sums are accumulated as 64-bit integers in units of 2^-60,
// so the result is exact and independent of the order of additions.
template <int PROG>
__global__ __launch_bounds__(kGT) void k_gather(Dev G, Params P, uint32_t* __restrict__ state,
                                                uint32_t it) {
    if (G.ctrl->done) return;
    constexpr bool SUM = is_sum(PROG);
    constexpr uint32_t IDENT = is_sum(PROG) ? kIdentSum : kIdentMin;
    const uint32_t cq = blockIdx.x, cur = it & 1u, nxt = cur ^ 1u;
    const uint32_t k = G.k, s = G.s, Q = G.q;
    const uint32_t vbase = cq << s;
    const uint32_t nv = min(Q, G.V - vbase);
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    const uint32_t prevVa = G.fVa[cur][cq];
    const uint4* __restrict__ cmcol = G.cm + (size_t)cq * k;
    const uint2* __restrict__ sccol = G.sc_cnt + (size_t)cq * k;

    extern __shared__ __align__(16) unsigned char smem[];
    const GatherLds L = gather_layout(SUM, Q);
    uint32_t* st32 = reinterpret_cast<uint32_t*>(smem + L.state);
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem + L.state);
    uint16_t* tag = reinterpret_cast<uint16_t*>(smem + L.tag);
    uint8_t* hit = smem + L.flag_a;     // improved (min) / received (sum)
    uint8_t* carry = smem + L.flag_b;   // kept active by initFunc
    uint32_t* bl_ioff = reinterpret_cast<uint32_t*>(smem + L.bl_ioff);
    uint32_t* bl_icnt = reinterpret_cast<uint32_t*>(smem + L.bl_icnt);
    uint32_t* bl_moff = reinterpret_cast<uint32_t*>(smem + L.bl_moff);  // bit 31: SC bin
    uint32_t* bl_mcnt = reinterpret_cast<uint32_t*>(smem + L.bl_mcnt);
    uint32_t* bl_scan = reinterpret_cast<uint32_t*>(smem + L.bl_scan);
    __shared__ uint32_t s_wc[kGW];
    __shared__ uint32_t s_wp[kGW];
    __shared__ uint64_t s_r64[3][kGW];
    __shared__ double s_rd[kGW];

    // ---- is there anything to do for this partition?
    int any = prevVa > 0;
    for (uint32_t p = tid; p < k && !any; p += kGT) {
        const uint32_t md = G.mode[p];
        const uint32_t ic = md == GPOP_MODE_PC ? cmcol[p].w : (md == GPOP_MODE_SC ? sccol[p].y : 0u);
        any |= ic > 0;
    }
    any = __syncthreads_or(any);
    if (!any) {
        if (tid == 0) {
            G.fVa[nxt][cq] = 0;
            G.fEa[nxt][cq] = 0;
            G.dpart[nxt][cq] = 0.0;
            G.gat_ids[cq] = 0;
        }
        return;
    }

    // ---- load the partition's state into LDS
    for (uint32_t u = tid; u < Q; u += kGT) {
        if constexpr (SUM) acc[u] = 0ull;
        else st32[u] = u < nv ? state[vbase + u] : 0xFFFFFFFFu;
        hit[u] = 0;
        carry[u] = 0;
    }
    __syncthreads();

    // ---- reInit frontier: initFunc on the vertices active before scatter
    const uint16_t* __restrict__ prev = G.flist[cur] + vbase;
    for (uint32_t i = tid; i < prevVa; i += kGT) {
        const uint32_t u = prev[i];
        if constexpr (PROG == P_CARRY) {
            carry[u] = (it + 1u - st32[u]) < P.persist;
        } else if constexpr (SUM) {
            carry[u] = 1;  // PageRank family: value restarts at 0, vertex stays active
        }
    }
    __syncthreads();

    // ---- gather all non-empty bins bin[p][cq]
    uint32_t my_ids = 0;
    for (uint32_t p0 = 0; p0 < k; p0 += kGT) {
        const uint32_t p = p0 + tid;
        uint32_t md = p < k ? G.mode[p] : GPOP_MODE_NONE;
        uint32_t ioff = 0, icnt = 0, moff = 0, mcnt = 0;
        if (md != GPOP_MODE_NONE) {
            const uint4 c = cmcol[p];
            ioff = c.y;
            moff = c.x;
            if (md == GPOP_MODE_PC) {
                icnt = c.w;
                mcnt = c.z;
            } else {
                const uint2 d = sccol[p];
                icnt = d.y;
                mcnt = d.x;
            }
        }
        const bool nz = icnt > 0;
        const uint32_t npieces = nz ? (ioff + icnt - 1u) / kChunk - ioff / kChunk + 1u : 0u;
        // compact non-empty bins in p order and scan their piece counts
        const uint64_t bm = ballot(nz);
        const uint32_t pincl = wave_incl_scan(npieces);
        if (lane == 63) {
            s_wc[wave] = popc64(bm);
            s_wp[wave] = pincl;
        }
        __syncthreads();
        uint32_t boff = 0, poff = 0, nb = 0, npt = 0;
        for (uint32_t w = 0; w < kGW; ++w) {
            const uint32_t c = s_wc[w], pc = s_wp[w];
            if (w < wave) {
                boff += c;
                poff += pc;
            }
            nb += c;
            npt += pc;
        }
        if (nz) {
            const uint32_t b = boff + popc_lt(bm);
            bl_ioff[b] = ioff;
            bl_icnt[b] = icnt;
            bl_moff[b] = moff | (md == GPOP_MODE_SC ? 0x80000000u : 0u);
            bl_mcnt[b] = mcnt;
            bl_scan[b] = poff + pincl - npieces;
        }
        __syncthreads();

        for (uint32_t r0 = 0; r0 < npt; r0 += kGW) {
            const uint32_t pid = r0 + wave;
            uint32_t dst[4], val[4];
            unsigned long long fx[4];
            uint32_t pend = 0;
            if (pid < npt) {
                // bin holding piece pid: last b with bl_scan[b] <= pid
                uint32_t lo = 0, hi = nb;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (bl_scan[mid] <= pid) lo = mid; else hi = mid;
                }
                const uint32_t b = lo;
                const uint32_t bioff = bl_ioff[b], bicnt = bl_icnt[b], bmo = bl_moff[b];
                const uint32_t bmcnt = bl_mcnt[b];
                const bool sc = bmo & 0x80000000u;
                const uint32_t bmoff = bmo & 0x7FFFFFFFu;
                const uint32_t c = bioff / kChunk + (pid - bl_scan[b]);
                const uint32_t lo_x = max(bioff, c * kChunk);
                const uint32_t hi_x = min(bioff + bicnt, c * kChunk + kChunk);
                const uint16_t* __restrict__ ids = sc ? G.sc_ids : G.png_ids;
                const uint32_t mbase = (lo_x == bioff) ? 0u : (sc ? G.sc_chunk[c] : G.png_chunk[c]);
                const uint32_t x0 = c * kChunk + lane * 4u;
                uint64_t raw = 0;
                if (x0 + 3u >= lo_x && x0 < hi_x)
                    raw = *reinterpret_cast<const uint64_t*>(ids + x0);
                uint32_t wts = 0;
                if constexpr (is_weighted(PROG)) {
                    if (x0 + 3u >= lo_x && x0 < hi_x)
                        wts = *reinterpret_cast<const uint32_t*>((sc ? G.sc_w : G.png_w) + x0);
                }
                uint32_t vmask = 0, fmask = 0, fc = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t x = x0 + j;
                    const uint32_t id = (uint32_t)(raw >> (16 * j)) & 0xFFFFu;
                    const bool v = x >= lo_x && x < hi_x;
                    const bool f = v && x > lo_x && (id & kFlag);
                    vmask |= (uint32_t)v << j;
                    fmask |= (uint32_t)f << j;
                    fc += f;
                    dst[j] = id & kLocalMask;
                }
                uint32_t midx = mbase + wave_excl_small(fc);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    midx += (fmask >> j) & 1u;
                    if (((vmask >> j) & 1u) && (midx >= bmcnt || dst[j] >= nv)) {
                        G.ctrl->bug = 1;  // inconsistent bin: never read or write out of range
                        vmask &= ~(1u << j);
                    }
                    if ((vmask >> j) & 1u) {
                        uint32_t x = G.data[bmoff + midx];
                        if (x != IDENT) {
                            if constexpr (is_weighted(PROG)) x = sat_add(x, (wts >> (8 * j)) & 0xFFu);
                            val[j] = x;
                            if constexpr (SUM)
                                fx[j] = __double2ull_rn((double)__uint_as_float(x) * kFix);
                            pend |= 1u << j;
                            ++my_ids;
                        }
                    }
                }
            }
            if constexpr (!SUM) {
                // write-verify rounds for the min combine
                for (;;) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if ((pend >> j) & 1u) {
                            if (val[j] < st32[dst[j]]) {
                                st32[dst[j]] = val[j];
                                hit[dst[j]] = 1;
                            }
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (((pend >> j) & 1u) && !(val[j] < st32[dst[j]])) pend &= ~(1u << j);
                    if (!__syncthreads_or(pend != 0)) break;
                }
            } else {
                // tagged rounds for the exact fixed-point sum
                for (;;) {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if ((pend >> j) & 1u) tag[dst[j]] = (uint16_t)(tid * 4u + j);
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if (((pend >> j) & 1u) && tag[dst[j]] == (uint16_t)(tid * 4u + j)) {
                            acc[dst[j]] += fx[j];
                            hit[dst[j]] = 1;
                            pend &= ~(1u << j);
                        }
                    }
                    if (!__syncthreads_or(pend != 0)) break;
                }
            }
        }
        __syncthreads();
    }

    // ---- filter frontier, write state back, compact the next frontier
    const double dang = SUM ? G.ctrl->dangling : 0.0;
    uint32_t running = 0;
    uint64_t my_ea = 0;
    double my_d = 0.0;
    uint16_t* __restrict__ nlist = G.flist[nxt] + vbase;
    uint32_t* __restrict__ nbits = G.fbits[nxt] + (vbase >> 5);
    for (uint32_t u0 = 0; u0 < nv; u0 += kGT) {
        const uint32_t u = u0 + tid;
        const bool in = u < nv;
        bool keep = false;
        uint32_t deg = 0;
        if (in) {
            const uint32_t v = vbase + u;
            deg = G.off[v + 1] - G.off[v];
            const bool prelim = hit[u] || carry[u];
            if constexpr (!SUM) {
                keep = prelim;  // filterFunc returns true for the min programs
                if (hit[u]) state[v] = st32[u];
            } else if constexpr (PROG == P_PR) {
                if (prelim) {
                    const double y = (double)acc[u] * kInvFix;
                    const double d = (double)P.damping;
                    const float x = (float)((1.0 - d) * P.inv_n + d * (y + dang * P.inv_n));
                    state[v] = __float_as_uint(x);
                    keep = true;
                    if (deg == 0) my_d += (double)x;
                }
            } else {  // P_PPR
                if (prelim) {
                    const double y = (double)acc[u] * kInvFix;
                    const double a = (double)P.alpha;
                    double xd = (1.0 - a) * y;
                    if (v == P.root) xd += a + (1.0 - a) * dang;
                    const float x = (float)xd;
                    state[v] = __float_as_uint(x);
                    keep = x > 0.0f;
                    if (deg == 0) my_d += (double)x;
                }
            }
        }
        const uint64_t bm = ballot(keep);
        if (lane == 0 && u0 + wave * 64u < Q) {
            const uint32_t wi = (u0 + wave * 64u) >> 5;
            nbits[wi] = (uint32_t)bm;
            nbits[wi + 1] = (uint32_t)(bm >> 32);
        }
        if (lane == 0) s_wc[wave] = popc64(bm);
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (uint32_t w = 0; w < kGW; ++w) {
            if (w < wave) before += s_wc[w];
            tot += s_wc[w];
        }
        if (keep) {
            nlist[running + before + popc_lt(bm)] = (uint16_t)u;
            my_ea += deg;
        }
        running += tot;
        __syncthreads();
    }
    // deterministic reductions: per-thread partials, butterfly per wave, waves in order
    my_ea = wave_sum_u64(my_ea);
    uint64_t ids64 = wave_sum_u64((uint64_t)my_ids);
    my_d = wave_sum_f64(my_d);
    if (lane == 0) {
        s_r64[0][wave] = my_ea;
        s_r64[1][wave] = ids64;
        s_rd[wave] = my_d;
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t ea = 0, ni = 0;
        double d = 0.0;
        for (uint32_t w = 0; w < kGW; ++w) {
            ea += s_r64[0][w];
            ni += s_r64[1][w];
            d += s_rd[w];
        }
        G.fVa[nxt][cq] = running;
        G.fEa[nxt][cq] = (uint32_t)ea;
        G.dpart[nxt][cq] = d;
        G.gat_ids[cq] = (uint32_t)ni;
    }
}

template <int PROG>
static hipError_t launch_gather_p(const Dev& G, const Params& P, uint32_t* state, uint32_t it,
                                  hipStream_t st) {
    const size_t lds = gather_lds_bytes(PROG, G.q);
    auto fn = k_gather<PROG>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(G.k), dim3(kGT), lds, st, G, P, state, it);
    return hipGetLastError();
}

hipError_t launch_gather(const Dev& G, const Params& P, int prog, uint32_t* state, uint32_t it,
                         hipStream_t st) {
    switch (prog) {
        case P_BFS: return launch_gather_p<P_BFS>(G, P, state, it, st);
        case P_CC: return launch_gather_p<P_CC>(G, P, state, it, st);
        case P_SSSP: return launch_gather_p<P_SSSP>(G, P, state, it, st);
        case P_PR: return launch_gather_p<P_PR>(G, P, state, it, st);
        case P_PPR: return launch_gather_p<P_PPR>(G, P, state, it, st);
        case P_CARRY: return launch_gather_p<P_CARRY>(G, P, state, it, st);
    }
    return hipErrorInvalidValue;
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
            default: x = v == P.root ? 0u : 0xFFFFFFFFu; break;
        }
        state[v] = x;
        if ((prog == P_PR || prog == P_PPR) && G.off[v + 1] == G.off[v])
            my_d += (double)__uint_as_float(x);
    }
    my_d = wave_sum_f64(my_d);
    if ((threadIdx.x & 63u) == 0) s_rd[threadIdx.x >> 6] = my_d;
    __syncthreads();
    if (threadIdx.x == 0) {
        G.dpart[0][p] = s_rd[0] + s_rd[1] + s_rd[2] + s_rd[3];
        G.dpart[1][p] = 0.0;
        G.fVa[0][p] = 0;
        G.fEa[0][p] = 0;
        G.fVa[1][p] = 0;
        G.fEa[1][p] = 0;
        G.gat_ids[p] = 0;
        G.mode[p] = GPOP_MODE_NONE;
    }
    if (p == 0 && threadIdx.x == 0) {
        G.ctrl->done = 0;
        G.ctrl->iters = 0;
        G.ctrl->frontier = 0;
        G.ctrl->dangling = 0.0;
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

__global__ void k_mark(Dev G, const uint32_t* __restrict__ verts, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t v = verts[i];
        if (v < G.V) G.marks[v] = 1;
        else G.ctrl->err = 1;
    }
}

__global__ __launch_bounds__(1024) void k_marks_to_frontier(Dev G, int all, uint32_t buf) {
    const uint32_t p = blockIdx.x;
    const uint32_t vbase = p << G.s;
    const uint32_t nv = min(G.q, G.V - vbase);
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    __shared__ uint32_t s_wc[16];
    __shared__ uint64_t s_e[16];
    uint16_t* list = G.flist[buf] + vbase;
    uint32_t* bits = G.fbits[buf] + (vbase >> 5);
    uint32_t running = 0;
    uint64_t my_ea = 0;
    for (uint32_t u0 = 0; u0 < nv; u0 += 1024) {
        const uint32_t u = u0 + tid;
        const bool keep = u < nv && (all || G.marks[vbase + u]);
        const uint64_t bm = ballot(keep);
        if (lane == 0 && u0 + wave * 64u < G.q) {
            const uint32_t wi = (u0 + wave * 64u) >> 5;
            bits[wi] = (uint32_t)bm;
            bits[wi + 1] = (uint32_t)(bm >> 32);
        }
        if (lane == 0) s_wc[wave] = popc64(bm);
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (uint32_t w = 0; w < 16; ++w) {
            if (w < wave) before += s_wc[w];
            tot += s_wc[w];
        }
        if (keep) {
            list[running + before + popc_lt(bm)] = (uint16_t)u;
            my_ea += G.off[vbase + u + 1] - G.off[vbase + u];
        }
        running += tot;
        __syncthreads();
    }
    my_ea = wave_sum_u64(my_ea);
    if (lane == 0) s_e[wave] = my_ea;
    __syncthreads();
    if (tid == 0) {
        uint64_t e = 0;
        for (int w = 0; w < 16; ++w) e += s_e[w];
        G.fVa[buf][p] = running;
        G.fEa[buf][p] = (uint32_t)e;
    }
    if (p == 0 && tid == 0) {
        G.ctrl->done = 0;
    }
}

hipError_t launch_set_frontier(const Dev& G, const uint32_t* verts, uint32_t n, int all,
                               uint32_t buf, hipStream_t st) {
    if (!all) {
        const uint64_t nm = (uint64_t)G.k * G.q;
        hipLaunchKernelGGL(k_fill_u8, dim3(1024), dim3(256), 0, st, G.marks, nm, (uint8_t)0);
        if (n) {
            const uint32_t blocks = min(1024u, (n + 255u) / 256u);
            hipLaunchKernelGGL(k_mark, dim3(blocks), dim3(256), 0, st, G, verts, n);
        }
    }
    hipLaunchKernelGGL(k_marks_to_frontier, dim3(G.k), dim3(1024), 0, st, G, all, buf);
    return hipGetLastError();
}

}  // namespace gpop
