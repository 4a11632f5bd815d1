// Learned scatter-mode selection on the device: the static per-partition
// features (once per graph), the per-iteration selection that the plan of a
// learned-selector iteration reads, and the feature export used to build
// training sets. Feature definitions and the network are in gpop_mlp.h.
#include "launch.h"
#include "select_dev.h"

namespace gpop {

// Static features of partition p (one workgroup each): the fraction of row
// p's bins that hold partition-centric messages and the log of max over
// mean out-degree.
__global__ __launch_bounds__(256) void k_part_static(Dev G) {
    const uint32_t p = blockIdx.x, tid = threadIdx.x;
    const uint32_t vbase = p << G.s;
    const uint32_t nv = min(G.q, G.V - vbase);
    uint32_t maxd = 0, nz = 0;
    for (uint32_t v = tid; v < nv; v += 256) maxd = max(maxd, gptr(G.off)[vbase + v + 1] - gptr(G.off)[vbase + v]);
    const uint32_t* row = gptr(G.bin_moff) + (size_t)p * G.k;
    for (uint32_t q = tid; q < G.k; q += 256) nz += row[q + 1] > row[q];
    __shared__ uint32_t s_max[4], s_nz[4];
    for (int o = 32; o > 0; o >>= 1) {
        maxd = max(maxd, (uint32_t)__shfl_xor((int)maxd, o));
        nz += (uint32_t)__shfl_xor((int)nz, o);
    }
    if ((tid & 63u) == 0) {
        s_max[tid >> 6] = maxd;
        s_nz[tid >> 6] = nz;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t m = 0, z = 0;
        for (int w = 0; w < 4; ++w) {
            m = max(m, s_max[w]);
            z += s_nz[w];
        }
        const uint32_t Ep = gptr(G.part_E)[p];
        gptr(G.pfill)[p] = (float)((double)z / (double)G.k);
        gptr(G.pskew)[p] = Ep ? (float)log((double)m * (double)nv / (double)Ep) : 0.f;
    }
}

// Sum of E_a over all partitions / |E| (every wave computes it).
__device__ inline float active_edge_fraction(const Dev& G, uint32_t cur) {
    uint64_t s = 0;
    for (uint32_t j = lane_id(); j < G.k; j += 64) s += gptr(G.fEa[cur])[j];
    s = wave_sum_u64(s);
    return G.E ? (float)((double)s / (double)G.E) : 0.f;
}

// Learned selection for the plan of iteration `it`: one lane per partition.
__device__ __forceinline__ void select_body(const Dev& G, const Params& P, uint32_t it, uint32_t bid) {
    if (gptr(G.ctrl)->done) return;
    const uint32_t cur = it & 1u;
    const float ea_frac = active_edge_fraction(G, cur);
    const uint32_t p = bid * 64 + lane_id();
    if (p >= G.k) return;
    const uint32_t Va = gptr(G.fVa[cur])[p];
    if (!Va) {
        gptr(G.mode_l)[p] = GPOP_MODE_NONE;
        return;
    }
    const uint32_t Ea = gptr(G.fEa[cur])[p];
    float f[GPOP_MLP_IN];
    partition_features(G, P, p, Va, Ea, it, ea_frac, f);
    float z;
    uint8_t md;
    // an infinite margin leaves every partition to Eq. 1 (no network pass)
    const float margin = gptr(G.mlp)->margin;
    if (margin != INFINITY && mlp_logit(gptr(G.mlp), f, &z) && fabsf(z) >= margin) {
        md = z >= 0.f ? (uint8_t)GPOP_MODE_PC : (uint8_t)GPOP_MODE_SC;
    } else {
        // an input the network was not trained on, or a logit inside the
        // confidence margin: Eq. 1 decides
        // left to Eq. 1: bit 7 marks the fallback, which the plan counts
        md = (uint8_t)(analytical_mode(G, P, p, Va, Ea) | kFallbackMark);
    }
    gptr(G.mode_l)[p] = md;
}

// Batched: runs whose selector is not the learned one skip.
__global__ __launch_bounds__(64) void kb_select(const Inst* __restrict__ tab,
                                                const uint32_t* __restrict__ boff, uint32_t n) {
    const uint32_t i = batch_find(boff, n, blockIdx.x);
    const Inst& I = tab[i];
    if (I.P.selector != GPOP_SEL_LEARNED || I.P.learned_eq1) return;
    select_body(I.G, I.P, gptr(I.G.ctrl)->pos, blockIdx.x - boff[i]);
}

__global__ __launch_bounds__(64) void k_features(Dev G, Params P, float* __restrict__ out) {
    const uint32_t it = gptr(G.ctrl)->pos;
    const uint32_t cur = it & 1u;
    const float ea_frac = active_edge_fraction(G, cur);
    const uint32_t p = blockIdx.x * 64 + lane_id();
    if (p >= G.k) return;
    float f[GPOP_MLP_IN];
    partition_features(G, P, p, gptr(G.fVa[cur])[p], gptr(G.fEa[cur])[p], it, ea_frac, f);
    for (int i = 0; i < GPOP_MLP_IN; ++i) out[(size_t)p * GPOP_MLP_IN + i] = f[i];
}

hipError_t launch_batch_select(const BatchGrid& B, hipStream_t st) {
    if (B.nb_select == 0 || !B.learned) return hipSuccess;
    hipLaunchKernelGGL(kb_select, dim3(B.nb_select), dim3(64), 0, st, B.tab, B.b_select, B.n);
    return hipGetLastError();
}

hipError_t launch_part_static(const Dev& G, hipStream_t st) {
    hipLaunchKernelGGL(k_part_static, dim3(G.k), dim3(256), 0, st, G);
    return hipGetLastError();
}


hipError_t launch_features(const Dev& G, const Params& P, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_features, dim3((G.k + 63) / 64), dim3(64), 0, st, G, P, out);
    return hipGetLastError();
}

}  // namespace gpop
