// Per-partition scatter-mode selection: the analytical model (Sec. 3.2,
// Eq. 1) and the learned selector's features and network (gpop_mlp.h).
#pragma once

#include "gpop_dev.h"

namespace gpop {

// ---------------------------------------------------------------------------
// Mode selection (Sec. 3.2, Eq. 1). With r^p = M^p / E^p the
// partition-centric volume E^p((r^p+1)s_i + 2 r^p s_v) + k s_i is the integer
// (M^p + E^p) s_i + 2 M^p s_v + k s_i, and E^p times the source-centric volume
// 2 r^p E_a s_v + 3 E_a s_i + V_a s_i is 2 M^p E_a s_v + (3 E_a + V_a) s_i E^p.
// PC is chosen iff cost_PC / BW_PC <= cost_SC / BW_SC, evaluated exactly in
// 128-bit integers with BW_PC / BW_SC = ratio_num / ratio_den; ties pick PC.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint8_t analytical_mode_of(const Dev& G, const Params& P, uint64_t Ep, uint64_t Mp,
                                                      uint32_t Va, uint32_t Ea) {
    typedef unsigned __int128 u128;
    const uint64_t si = P.s_i, sv = P.s_v;
    const uint64_t cost_pc = (Mp + Ep) * si + 2ull * Mp * sv + (uint64_t)G.k * si;
    const u128 lhs = (u128)cost_pc * Ep * P.ratio_den;
    const u128 sc_scaled = (u128)(2ull * sv) * Mp * Ea + (u128)((3ull * Ea + Va) * si) * Ep;
    const u128 rhs = sc_scaled * P.ratio_num;
    return lhs <= rhs ? (uint8_t)GPOP_MODE_PC : (uint8_t)GPOP_MODE_SC;
}

__device__ __forceinline__ uint8_t analytical_mode(const Dev& G, const Params& P, uint32_t p,
                                                   uint32_t Va, uint32_t Ea) {
    return analytical_mode_of(G, P, gptr(G.part_E)[p], gptr(G.part_M)[p], Va, Ea);
}

__device__ __forceinline__ float bf16_bits_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// f32 -> bf16 bits, round to nearest even; NaN maps to a quiet NaN.
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x0040u);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// The GPOP_MLP_IN features of partition p (definitions in gpop_mlp.h).
// ea_frac is the sum of E_a over all partitions divided by |E|.
__device__ inline void partition_features(const Dev& G, const Params& P, uint32_t p, uint32_t Va,
                                          uint32_t Ea, uint32_t it, float ea_frac, float* f) {
    const uint32_t Ep = gptr(G.part_E)[p], Mp = gptr(G.part_M)[p];
    const uint32_t nv = min(G.q, G.V - (p << G.s));
    f[0] = log1pf((float)Va);
    f[1] = log1pf((float)Ea);
    f[2] = log1pf((float)Ep);
    f[3] = log1pf((float)Mp);
    f[4] = Ep ? (float)((double)Mp / (double)Ep) : 0.f;
    f[5] = (float)((double)Va / (double)nv);
    f[6] = Ep ? (float)((double)Ea / (double)Ep) : 0.f;
    f[7] = gptr(G.pfill)[p];
    f[8] = gptr(G.pskew)[p];
    f[9] = log1pf((float)it);
    f[10] = ea_frac;
    const double si = P.s_i, sv = P.s_v;
    const double cost_pc = ((double)Mp + (double)Ep) * si + 2.0 * (double)Mp * sv + (double)G.k * si;
    const double cost_sc = (Ep ? 2.0 * sv * (double)Mp * (double)Ea / (double)Ep : 0.0) +
                           (3.0 * (double)Ea + (double)Va) * si;
    f[11] = cost_sc > 0.0 ? (float)log(cost_pc / cost_sc) : 0.f;
}

// The network's logit for raw features f. Returns false when a standardised
// feature leaves [-6, 6] or the logit is not finite (the caller then falls
// back to Eq. 1). Every lane reads the same weights, so they come through
// scalar loads.
__device__ inline bool mlp_logit(const gpop_mlp_model* __restrict__ M, const float* f, float* out) {
    float x[GPOP_MLP_IN];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < GPOP_MLP_IN; ++i) {
        x[i] = (f[i] - M->mean[i]) * M->inv_std[i];
        ok = ok && fabsf(x[i]) <= 6.f;
    }
    const uint16_t* __restrict__ w = M->w;
    float h1[GPOP_MLP_HIDDEN];
#pragma unroll
    for (int o = 0; o < GPOP_MLP_HIDDEN; ++o) {
        float a = bf16_bits_to_f32(w[GPOP_MLP_B1 + o]);
#pragma unroll
        for (int i = 0; i < GPOP_MLP_IN; ++i)
            a = fmaf(bf16_bits_to_f32(w[GPOP_MLP_W1 + o * GPOP_MLP_IN + i]), x[i], a);
        h1[o] = fmaxf(a, 0.f);
    }
    float z = bf16_bits_to_f32(w[GPOP_MLP_B3]);
#pragma unroll 4
    for (int o = 0; o < GPOP_MLP_HIDDEN; ++o) {
        float a = bf16_bits_to_f32(w[GPOP_MLP_B2 + o]);
#pragma unroll
        for (int i = 0; i < GPOP_MLP_HIDDEN; ++i)
            a = fmaf(bf16_bits_to_f32(w[GPOP_MLP_W2 + o * GPOP_MLP_HIDDEN + i]), h1[i], a);
        z = fmaf(bf16_bits_to_f32(w[GPOP_MLP_W3 + o]), fmaxf(a, 0.f), z);
    }
    *out = z;
    return ok && isfinite(z);
}

}  // namespace gpop
