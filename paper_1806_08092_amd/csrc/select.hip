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

// ---------------------------------------------------------------------------
// The network on the matrix cores, 32 partitions per wave. The two hidden
// layers are 32 x 32 x 8 bf16 MFMA tiles with f32 accumulation, in transposed
// form (rows: hidden units, columns: partitions): H1^T = W1 [X | 1]^T and
// H2^T = W2 H1^T. With that orientation the accumulator of one layer is, lane
// by lane and register by register, the B operand of the next (lane l holds
// column l % 32 and rows 8 (r / 4) + 4 (l / 32) + r % 4 of register r; a B
// operand of K-step j takes rows 8 j + 4 (l / 32) + i), so no data moves
// between the layers. The inputs of each layer are rounded to bf16 (round to
// nearest even): the standardised features, with the bias folded in as a
// 13th input of value 1, and the first hidden layer after its ReLU.
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ bf16x4 bf16x4_of(float a, float b, float c, float d) {
    bf16x4 r;
    r[0] = (short)f32_to_bf16_bits(a);
    r[1] = (short)f32_to_bf16_bits(b);
    r[2] = (short)f32_to_bf16_bits(c);
    r[3] = (short)f32_to_bf16_bits(d);
    return r;
}

// Four consecutive bf16 weights starting at element j (j a multiple of 4
// from an 8-byte aligned model).
__device__ __forceinline__ bf16x4 w4(const uint16_t* __restrict__ w, uint32_t j) {
    const uint2 u = *reinterpret_cast<const uint2*>(w + j);
    bf16x4 r;
    r[0] = (short)(u.x & 0xFFFFu);
    r[1] = (short)(u.x >> 16);
    r[2] = (short)(u.y & 0xFFFFu);
    r[3] = (short)(u.y >> 16);
    return r;
}

// Logit of the partition of column l % 32 from its standardised features x
// (every lane holds its column's 12 values; both halves of the wave compute
// the same logit).
__device__ __forceinline__ float mlp_logit_mfma(const gpop_mlp_model* __restrict__ M, const float* x) {
    const uint32_t lane = lane_id(), h = lane >> 5, c = lane & 31u;
    const uint16_t* __restrict__ w = M->w;
    // B operand of layer 1: inputs 8 j + 4 h + i of column c; input 12 is the
    // constant 1 that multiplies b1, inputs 13..15 are zero
    const bf16x4 xb0 = h ? bf16x4_of(x[4], x[5], x[6], x[7]) : bf16x4_of(x[0], x[1], x[2], x[3]);
    const bf16x4 xb1 = h ? bf16x4_of(1.f, 0.f, 0.f, 0.f) : bf16x4_of(x[8], x[9], x[10], x[11]);
    f32x16 d1[2];
#pragma unroll
    for (uint32_t mt = 0; mt < 2; ++mt) {
        const uint32_t o = 32u * mt + c;  // hidden unit of this lane's A row
        const bf16x4 a0 = w4(w, GPOP_MLP_W1 + o * GPOP_MLP_IN + 4u * h);
        bf16x4 a1;
        if (h) {
            a1 = bf16x4{(short)w[GPOP_MLP_B1 + o], 0, 0, 0};
        } else {
            a1 = w4(w, GPOP_MLP_W1 + o * GPOP_MLP_IN + 8u);
        }
        f32x16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a0, xb0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1, xb1, acc, 0, 0, 0);
        d1[mt] = acc;
    }
    // layer 2: K-step j takes registers 4 (j % 4) .. + 3 of tile j / 4
    f32x16 d2[2];
#pragma unroll
    for (uint32_t mt = 0; mt < 2; ++mt)
        d2[mt] = f32x16{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (uint32_t j = 0; j < 8; ++j) {
        const f32x16& src = d1[j >> 2];
        const uint32_t r0 = 4u * (j & 3u);
        const bf16x4 hb = bf16x4_of(fmaxf(src[r0], 0.f), fmaxf(src[r0 + 1], 0.f), fmaxf(src[r0 + 2], 0.f),
                                    fmaxf(src[r0 + 3], 0.f));
#pragma unroll
        for (uint32_t mt = 0; mt < 2; ++mt) {
            const uint32_t o = 32u * mt + c;
            const bf16x4 a = w4(w, GPOP_MLP_W2 + o * GPOP_MLP_HIDDEN + 8u * j + 4u * h);
            d2[mt] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, hb, d2[mt], 0, 0, 0);
        }
    }
    // output layer over this lane's 32 units of layer 2, then the other half's
    float z = 0.f;
#pragma unroll
    for (uint32_t mt = 0; mt < 2; ++mt) {
#pragma unroll
        for (uint32_t g = 0; g < 4; ++g) {
            const uint32_t o = 32u * mt + 8u * g + 4u * h;  // units o .. o + 3: registers 4 g .. 4 g + 3
            const bf16x4 b2 = w4(w, GPOP_MLP_B2 + o), w3 = w4(w, GPOP_MLP_W3 + o);
#pragma unroll
            for (uint32_t i = 0; i < 4; ++i) {
                const float a = d2[mt][4u * g + i] + bf16_bits_to_f32((uint16_t)b2[i]);
                z = fmaf(bf16_bits_to_f32((uint16_t)w3[i]), fmaxf(a, 0.f), z);
            }
        }
    }
    z += __shfl_xor(z, 32, 64);
    return z + bf16_bits_to_f32(w[GPOP_MLP_B3]);
}

// Learned selection for the plan of iteration `it`: one wave per 32
// partitions (lanes l and l + 32 hold partition l % 32).
__device__ __forceinline__ void select_body(const Dev& G, const Params& P, uint32_t it, uint32_t bid) {
    if (gptr(G.ctrl)->done) return;
    const uint32_t cur = it & 1u;
    const float ea_frac = active_edge_fraction(G, cur);
    const uint32_t lane = lane_id();
    const uint32_t p = bid * 32u + (lane & 31u);
    const bool in = p < G.k;
    const uint32_t Va = in ? gptr(G.fVa[cur])[p] : 0u;
    const uint32_t Ea = in ? gptr(G.fEa[cur])[p] : 0u;
    const gpop_mlp_model* __restrict__ M = gptr(G.mlp);
    float x[GPOP_MLP_IN];
    bool ok = Va != 0u;
    if (ok) {
        float f[GPOP_MLP_IN];
        partition_features(G, P, p, Va, Ea, it, ea_frac, f);
#pragma unroll
        for (int i = 0; i < GPOP_MLP_IN; ++i) {
            x[i] = (f[i] - M->mean[i]) * M->inv_std[i];
            ok = ok && fabsf(x[i]) <= 6.f;
        }
    } else {
#pragma unroll
        for (int i = 0; i < GPOP_MLP_IN; ++i) x[i] = 0.f;
    }
    if (!ok) {  // keep the matrix inputs finite; Eq. 1 decides this partition
#pragma unroll
        for (int i = 0; i < GPOP_MLP_IN; ++i) x[i] = 0.f;
    }
    const float z = mlp_logit_mfma(M, x);  // every lane takes part
    if (!in || lane >= 32u) return;
    if (!Va) {
        gptr(G.mode_l)[p] = GPOP_MODE_NONE;
        return;
    }
    // an infinite margin leaves every partition to Eq. 1 (no network pass)
    const float margin = M->margin;
    uint8_t md;
    if (margin != INFINITY && ok && isfinite(z) && fabsf(z) >= margin) {
        md = z >= 0.f ? (uint8_t)GPOP_MODE_PC : (uint8_t)GPOP_MODE_SC;
    } else {
        // an input the network was not trained on, or a logit inside the
        // confidence margin: Eq. 1 decides; bit 7 marks the fallback, which
        // the plan counts
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
