// Host-side launchers of the engine's kernels (one translation unit each).
#pragma once

#include "gpop_dev.h"

namespace gpop {

// error reporting of the C ABI (api.hip): sets gpop_last_error, returns code
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

#define HIP_OR_RETURN(expr, what)                              \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return ::gpop::hip_fail(e_, what); \
    } while (0)

// preprocessing (png.hip)
hipError_t launch_validate(const Dev& G, hipStream_t st);
hipError_t launch_validate_edges(const Dev& G, hipStream_t st);
hipError_t launch_part_E(const Dev& G, hipStream_t st);
hipError_t launch_scan_excl(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* tmp,
                            hipStream_t st);
size_t scan_tmp_words(uint64_t n);
hipError_t launch_part_M(const Dev& G, hipStream_t st);
hipError_t launch_colmajor(const Dev& G, hipStream_t st);
hipError_t launch_sc_cap(const Dev& G, hipStream_t st);
hipError_t launch_sc_mo(const Dev& G, const uint32_t* sx, uint32_t base, hipStream_t st);
hipError_t launch_colsrc(const Dev& G, hipStream_t st);
hipError_t launch_cs_fill(const Dev& G, hipStream_t st);

// scatter side (scatter.hip)
size_t sc_lds_bytes(uint32_t k);
hipError_t launch_sc_build(const Dev& G, int fill, hipStream_t st);
hipError_t launch_finalize(const Dev& G, hipStream_t st);

// gather side (gather.hip)
size_t gather_lds_bytes(int prog, uint32_t q, bool rounds);
hipError_t launch_state_init(const Dev& G, const Params& P, int prog, uint32_t* state,
                             hipStream_t st);
// learned selector (select.hip)
hipError_t launch_part_static(const Dev& G, hipStream_t st);
hipError_t launch_features(const Dev& G, const Params& P, float* out, hipStream_t st);

// batched runs: one launch per kernel covers every run of a batch
struct BatchGrid {
    const Inst* tab;              // [n] device
    uint32_t n;
    // per kernel: device block prefix over the runs (n + 1 entries) and its total
    const uint32_t* b_select;
    const uint32_t* b_sc;
    const uint32_t* b_clr;
    const uint32_t* b_pc;
    const uint32_t* b_gather;
    const uint32_t* b_merge;
    uint32_t nb_select, nb_sc, nb_clr, nb_pc, nb_gather, nb_merge;
    uint32_t k_max, q_max;
    bool rounds;                  // atomic-free combine (every run of a batch uses the same)
    bool learned = true;          // some run uses the learned selector (else its kernel is not launched)
    bool streams = false;         // some run's graph has column streams (the dense gather kernel is launched)
    const Dev* view = nullptr;    // a single run's view on the host, passed by value where it helps
};
hipError_t prepare_batch_scatter(const BatchGrid& B, int prog);
hipError_t prepare_batch_gather(const BatchGrid& B, int prog);
hipError_t launch_batch_select(const BatchGrid& B, hipStream_t st);
hipError_t launch_batch_plan(const BatchGrid& B, hipStream_t st);
hipError_t launch_batch_sc(const BatchGrid& B, int prog, hipStream_t st);
hipError_t launch_batch_pc(const BatchGrid& B, int prog, hipStream_t st);
hipError_t launch_batch_gather(const BatchGrid& B, int prog, hipStream_t st);
hipError_t launch_batch_merge(const BatchGrid& B, int prog, hipStream_t st);
hipError_t launch_batch_limits(const BatchGrid& B, uint32_t max_iter, hipStream_t st);
hipError_t launch_batch_status(const BatchGrid& B, uint32_t* out, hipStream_t st);

hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t v, hipStream_t st);
// mix 0: read vecs 16-byte vectors of src (dst: one word, written at most
// once); 1: copy them to dst; 2: widen vecs groups of four 16-bit words of
// src to four 32-bit words of dst; 3: read vecs 16-byte vectors of src as
// 512-byte segments in a scattered order (vecs / 32 a power of two).
hipError_t launch_stream_ceiling(int mix, const void* src, void* dst, uint64_t vecs, hipStream_t st);
hipError_t launch_set_frontier(const Dev& G, const uint32_t* verts, uint32_t n, int all, hipStream_t st);

}  // namespace gpop
