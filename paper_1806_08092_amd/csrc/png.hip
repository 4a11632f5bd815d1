// Preprocessing: CSR validation, per-partition statistics, bin offsets and
// the column-major bin table the gather reads (graph partitioning Sec. 3.1.1,
// message generation Sec. 3.1.2, PNG layout of Algorithm 3).
#include "launch.h"

namespace gpop {

// Error codes written to Ctrl::csr_err (plain stores: any writer sets it).
// 1 offsets[0] != 0, 2 decreasing offsets or offsets beyond E,
// 3 offsets[V] != E, 4 column >= V, 5 row not sorted ascending.
// Vertex pass: offsets, and a row-start mark for every non-empty row in a
// byte array over the edges (marks start at zero).
__global__ void k_validate_rows(Dev G, uint8_t* __restrict__ rowstart) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= G.V) return;
    const uint32_t a = G.off[v], b = G.off[v + 1];
    if (v == 0 && a != 0) G.ctrl->csr_err = 1;
    if (a > b || (uint64_t)b > G.E) {
        G.ctrl->csr_err = 2;
        return;
    }
    if (v == G.V - 1 && (uint64_t)b != G.E) G.ctrl->csr_err = 3;
    if (b > a) rowstart[a] = 1;
}

// Edge pass: every column < V, and non-decreasing inside each row.
__global__ void k_validate_edges(Dev G, const uint8_t* __restrict__ rowstart) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < G.E;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t c = G.cols[e];
        if (c >= G.V) G.ctrl->csr_err = 4;
        else if (e > 0 && !rowstart[e] && G.cols[e - 1] > c) G.ctrl->csr_err = 5;
    }
}

__global__ void k_zero_u8(uint8_t* __restrict__ p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// The edge pass runs only when the offsets are valid (checked by the caller
// between the two launches), so every row index it reads is in range.
hipError_t launch_validate(const Dev& G, hipStream_t st) {
    uint8_t* marks = G.sc_w;  // E_pad bytes, unused until the first iteration
    hipLaunchKernelGGL(k_zero_u8, dim3(2048), dim3(256), 0, st, marks, G.E);
    hipLaunchKernelGGL(k_validate_rows, dim3((G.V + 255) / 256), dim3(256), 0, st, G, marks);
    return hipGetLastError();
}

hipError_t launch_validate_edges(const Dev& G, hipStream_t st) {
    if (G.E == 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate_edges, dim3(4096), dim3(256), 0, st, G, G.sc_w);
    return hipGetLastError();
}

// E^p: out-edges of the index range of partition p.
__global__ void k_part_E(Dev G) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= G.k) return;
    const uint32_t lo = p << G.s;
    const uint32_t hi = min(lo + G.q, G.V);
    G.part_E[p] = G.off[hi] - G.off[lo];
}

hipError_t launch_part_E(const Dev& G, hipStream_t st) {
    hipLaunchKernelGGL(k_part_E, dim3((G.k + 255) / 256), dim3(256), 0, st, G);
    return hipGetLastError();
}

// -------------------------------------------------- exclusive scan (u32)
constexpr uint32_t kScanT = 256, kScanPer = 16, kScanTile = kScanT * kScanPer;

size_t scan_tmp_words(uint64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

__device__ uint32_t block_excl_scan(uint32_t x, uint32_t* total) {
    __shared__ uint32_t s_w[kScanT / 64];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan(x);
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (uint32_t w = 0; w < kScanT / 64; ++w) {
        if (w < wave) before += s_w[w];
        tot += s_w[w];
    }
    __syncthreads();
    *total = tot;
    return before + incl - x;
}

__global__ __launch_bounds__(kScanT) void k_scan_tiles(const uint32_t* __restrict__ in, uint64_t n,
                                                       uint32_t* __restrict__ tile_sums) {
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanPer;
    uint32_t s = 0;
    for (uint32_t j = 0; j < kScanPer; ++j)
        if (base + j < n) s += in[base + j];
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanT) void k_scan_sums(uint32_t* __restrict__ sums, uint32_t nt,
                                                      uint32_t* __restrict__ out_total) {
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nt; b0 += kScanT) {
        const uint32_t i = b0 + threadIdx.x;
        const uint32_t x = i < nt ? sums[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(x, &tot);
        if (i < nt) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *out_total = carry;
}

__global__ __launch_bounds__(kScanT) void k_scan_apply(const uint32_t* __restrict__ in, uint64_t n,
                                                       const uint32_t* __restrict__ tile_off,
                                                       uint32_t* __restrict__ out) {
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t s = 0;
    for (uint32_t j = 0; j < kScanPer; ++j) {
        v[j] = base + j < n ? in[base + j] : 0u;
        s += v[j];
    }
    uint32_t tot;
    uint32_t run = tile_off[blockIdx.x] + block_excl_scan(s, &tot);
    for (uint32_t j = 0; j < kScanPer; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
}

// out[i] = sum of in[0..i) for i <= n (n + 1 entries). tmp holds
// scan_tmp_words(n) words.
hipError_t launch_scan_excl(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* tmp,
                            hipStream_t st) {
    const uint32_t nt = (uint32_t)((n + kScanTile - 1) / kScanTile);
    if (nt) hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(kScanT), 0, st, in, n, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanT), 0, st, tmp, nt, out + n);
    if (nt) hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(kScanT), 0, st, in, n, tmp, out);
    return hipGetLastError();
}

// M^p from the row-major message offsets.
__global__ void k_part_M(Dev G) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= G.k) return;
    const size_t k = G.k;
    G.part_M[p] = G.bin_moff[(p + 1) * k] - G.bin_moff[p * k];
}

hipError_t launch_part_M(const Dev& G, hipStream_t st) {
    hipLaunchKernelGGL(k_part_M, dim3((G.k + 255) / 256), dim3(256), 0, st, G);
    return hipGetLastError();
}

// Column-major copy: cm[q*k + p] = {moff, ioff, mcnt, icnt} of bin[p][q].
__global__ void k_colmajor(Dev G) {
    const uint64_t kk = (uint64_t)G.k * G.k;
    for (uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; o < kk;
         o += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t q = o / G.k, p = o % G.k;
        const uint64_t r = p * G.k + q;
        G.cm[o] = make_uint4(G.bin_moff[r], G.bin_ioff[r], G.cnt_m[r], G.cnt_i[r]);
    }
}

hipError_t launch_colmajor(const Dev& G, hipStream_t st) {
    const uint64_t kk = (uint64_t)G.k * G.k;
    const uint64_t want = (kk + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(k_colmajor, dim3(blocks), dim3(256), 0, st, G);
    return hipGetLastError();
}

// Source-centric message capacity of each bin. Source-centric scatter cuts
// every message (a maximal run of one vertex's edges into q) into pieces of at
// most kPiece edges, each with its own start flag and value, so a bin holds at
// most runs + ids / kPiece of them. Overwrites cnt_m, whose last reader is the
// column-major table.
__global__ void k_sc_cap(Dev G) {
    const uint64_t kk = (uint64_t)G.k * G.k;
    for (uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; o < kk;
         o += (uint64_t)gridDim.x * blockDim.x)
        G.cnt_m[o] += G.cnt_i[o] / kPiece;
}

// Data index of each source-centric bin's first message slot, base plus the
// row-major exclusive prefix sx of the capacities: row-major (with the end of
// the last bin) for the scatter, column-major for the gather.
__global__ void k_sc_mo(Dev G, const uint32_t* __restrict__ sx, uint32_t base) {
    const uint64_t kk = (uint64_t)G.k * G.k;
    for (uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; o <= kk;
         o += (uint64_t)gridDim.x * blockDim.x) {
        G.sc_mor[o] = base + sx[o];
        if (o == kk) continue;
        const uint64_t q = o / G.k, p = o % G.k;
        G.sc_mo[o] = base + sx[p * G.k + q];
    }
}

static uint32_t kk_blocks(const Dev& G) {
    const uint64_t want = ((uint64_t)G.k * G.k + 255) / 256;
    return (uint32_t)(want < 4096 ? want : 4096);
}

hipError_t launch_sc_cap(const Dev& G, hipStream_t st) {
    hipLaunchKernelGGL(k_sc_cap, dim3(kk_blocks(G)), dim3(256), 0, st, G);
    return hipGetLastError();
}

hipError_t launch_sc_mo(const Dev& G, const uint32_t* sx, uint32_t base, hipStream_t st) {
    hipLaunchKernelGGL(k_sc_mo, dim3(kk_blocks(G)), dim3(256), 0, st, G, sx, base);
    return hipGetLastError();
}

// Static level-2 tables of the active list, one wave per column q: the
// source-partition bitmask of q's non-empty bins (colsrc) and the exclusive
// prefix of the bins' 256-id pieces in source order (spre), which places any
// bin inside the column's static piece enumeration without a scan.
__global__ __launch_bounds__(256) void k_colsrc(Dev G) {
    const uint32_t q = blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    if (q >= G.k) return;
    const uint4* __restrict__ col = G.cm + (size_t)q * G.k;
    uint32_t run = 0;
    for (uint32_t p0 = 0; p0 < G.k; p0 += 64) {
        const uint32_t p = p0 + lane;
        const uint4 c = p < G.k ? col[p] : make_uint4(0u, 0u, 0u, 0u);
        const uint32_t sp = pieces_of(c.y, c.w);
        const uint32_t incl = wave_incl_scan(sp);
        if (p < G.k) G.spre[(size_t)q * G.k + p] = run + incl - sp;
        const uint64_t m = ballot(c.w > 0u);
        if (lane == 0) G.colsrc[(size_t)q * G.kw + (p0 >> 6)] = m;
        run += last_lane(incl);
    }
}

hipError_t launch_colsrc(const Dev& G, hipStream_t st) {
    hipLaunchKernelGGL(k_colsrc, dim3((G.k + 3) / 4), dim3(256), 0, st, G);
    return hipGetLastError();
}

// Column streams, per-id part (one wave per chunk, after the host walk has
// written each chunk's lane-start mask, table offset and raw entries:
// entry 0 {offset of the chunk start inside its bin, src | q << 16}, lane
// starts {start position, src | q << 16}, src = 0xFFFF for padding).
// Lane l covers chunk positions 4l..4l+3, all in one bin: it copies their ids
// and weights from the bin's per-bin layout, fills the bin's last lane past
// its ids with null ids (local id q, not a message start, weight 0) and the
// padding run with one-id messages to vertices 0..63 (identity values then
// spread over the LDS banks), and counts message starts. The entries are
// then rewritten in their final form {adj, src | mt << 16} (see Dev::cs_ent).
__device__ __forceinline__ uint32_t bperm(uint32_t lane_src, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(lane_src << 2), (int)v);
}

__global__ __launch_bounds__(256) void k_cs_fill(Dev G) {
    const uint32_t c = blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    if (c >= G.n_chunks) return;
    const uint32_t k = G.k;
    const uint32_t tb = G.cs_tabo[c], ne = G.cs_tabo[c + 1] - tb;
    const uint64_t lm = G.cs_lm[c];
    if (ne == 0 || ne > 64 || ne != 1u + (uint32_t)__popcll(lm) || (lm & 1ull)) {
        if (lane == 0) G.ctrl->bug = 1;
        return;
    }
    const uint2 e = G.cs_ent[tb + min(lane, ne - 1u)];
    const uint32_t q = G.cs_ent[tb].y >> 16;
    const uint32_t src = e.y & 0xFFFFu;
    const bool pad = src == 0xFFFFu;
    // start position of the entry's run in the chunk (lanes past the table
    // hold a copy of its last entry, which they never use)
    const uint32_t t = (lane == 0 || lane >= ne) ? 0u : e.x;
    const uint32_t x0 = lane == 0 ? e.x : 0u;  // entry 0: offset of the chunk start inside its bin
    const bool sane = q < k && (pad || src < k) && t < kChunk && (t & 3u) == 0u;
    if (__builtin_amdgcn_read_exec() != ballot(sane)) {  // an inconsistent table (internal error)
        if (lane == 0) G.ctrl->bug = 1;
        return;
    }
    const uint4 cb = pad ? make_uint4(0u, 0u, 0u, 0u) : G.cm[(size_t)q * k + src];  // {moff, ioff, mcnt, icnt}
    if (ballot(lane == 0 && (pad || x0 >= cb.w))) {  // the chunk start lies inside bin 0
        if (lane == 0) G.ctrl->bug = 1;
        return;
    }
    // per-bin position of chunk position i for this entry: ioff + x0 + i - t
    const uint32_t rbase = cb.y + x0 - t;
    const uint32_t rend = cb.y + cb.w;          // end of the bin in the per-bin layout
    // the lane's entry: lane starts at lanes 1..lane
    const uint32_t bl = popc_lt(lm) + (uint32_t)((lm >> lane) & 1ull);
    const uint32_t rb = bperm(bl, rbase), re = bperm(bl, rend), pj = bperm(bl, pad ? 1u : 0u);
    uint32_t ids[4], wv[4], mflag = 0;
    bool bad = false;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t i = 4u * lane + j;
        if (pj) {
            ids[j] = kFlag | (i & 63u);
            wv[j] = 0u;
        } else {
            const uint32_t r = rb + i;
            if (r < re) {
                ids[j] = G.png_ids[r];
                wv[j] = G.w ? G.png_w[r] : 0u;
            } else {
                ids[j] = G.q;  // null id after the bin's last id
                wv[j] = 0u;
                bad = bad || j == 0;  // a lane starts with an id of its bin
            }
        }
        if (i > 0 && (ids[j] & kFlag)) mflag |= 1u << j;
    }
    if (bad) G.ctrl->bug = 1;
    uint2 iw;
    iw.x = ids[0] | (ids[1] << 16);
    iw.y = ids[2] | (ids[3] << 16);
    reinterpret_cast<uint2*>(G.cs_ids)[(size_t)c * 64 + lane] = iw;
    reinterpret_cast<uint32_t*>(G.cs_w)[(size_t)c * 64 + lane] = wv[0] | (wv[1] << 8) | (wv[2] << 16) | (wv[3] << 24);
    // message starts at positions 1..4l, inclusive
    const uint32_t mc = __popc(mflag);
    const uint32_t m0 = wave_incl_scan(mc) - mc + (mflag & 1u);
    // message starts at positions 1..t of each entry's start t (entry 0: 0)
    const uint32_t mt = lane == 0 ? 0u : bperm(t >> 2, m0);
    // entry 0: message index (inside bin 0) of the message holding the chunk
    // start, counted from the per-bin chunk table and up to 255 flags
    uint32_t midx0 = 0;
    {
        const uint32_t ioff0 = __builtin_amdgcn_readfirstlane(cb.y);
        const uint32_t xx0 = __builtin_amdgcn_readfirstlane(x0);
        if (xx0) {
            const uint32_t y = ioff0 + xx0, y0 = y & ~(kChunk - 1u);
            const uint32_t lo = y0 > ioff0 ? y0 : ioff0;
            const uint32_t base = y0 > ioff0 ? G.png_chunk[y0 / kChunk] : 0u;
            uint32_t f = 0;
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                const uint32_t r = lo + 1u + 4u * lane + j;
                if (r <= y) f += (G.png_ids[r] & kFlag) ? 1u : 0u;
            }
            midx0 = base + wave_sum_u32(f);
        }
    }
    if (lane < ne) {
        uint32_t adj;
        if (pad) adj = G.idb - mt;
        else if (lane == 0) adj = cb.x + midx0;
        else adj = cb.x - mt;
        G.cs_ent[tb + lane] = make_uint2(adj, src | (mt << 16));
    }
}

hipError_t launch_cs_fill(const Dev& G, hipStream_t st) {
    if (!G.n_chunks) return hipSuccess;
    hipLaunchKernelGGL(k_cs_fill, dim3((G.n_chunks + 3) / 4), dim3(256), 0, st, G);
    return hipGetLastError();
}

}  // namespace gpop
