// Training and inference of the learned scatter-mode selector (gpop_mlp.h):
// model start-up with feature standardisation, batched logits, the gradient
// of the regret-weighted cross-entropy, and Adam on f32 masters with bf16
// copies. The network is 12 -> 64 -> 64 -> 1; a chunk of 64 samples maps to
// one wave (one sample per lane for the forward and backward pass, one
// parameter column per lane for the sums over samples), so every reduction
// runs in a fixed order and the gradient is reproducible bit for bit.
#include <cmath>
#include <cstddef>
#include <mutex>

#include "launch.h"
#include "select_dev.h"

namespace gpop {
namespace {

constexpr int kIn = GPOP_MLP_IN, kH = GPOP_MLP_HIDDEN, kP = GPOP_MLP_PARAMS;
constexpr int kRow = kH + 1;       // padded LDS row: lane-strided rows stay conflict-free
constexpr int kPart = kP + 2;      // per-chunk partial: gradient, loss, weight sum

__global__ __launch_bounds__(256) void k_mlp_init(gpop_mlp_model* __restrict__ M, float* __restrict__ master,
                                                  float* __restrict__ mom1, float* __restrict__ mom2,
                                                  const float* __restrict__ init,
                                                  const float* __restrict__ x, uint32_t n) {
    __shared__ double red[256];
    __shared__ double mean[kIn];
    const uint32_t tid = threadIdx.x;
    for (int f = 0; f < kIn; ++f) {  // two passes per feature, fixed order
        double s = 0.0;
        for (uint32_t i = tid; i < n; i += 256) s += (double)x[(size_t)i * kIn + f];
        red[tid] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < (uint32_t)o) red[tid] += red[tid + o];
            __syncthreads();
        }
        if (tid == 0) mean[f] = red[0] / (double)n;
        __syncthreads();
        const double mu = mean[f];
        s = 0.0;
        for (uint32_t i = tid; i < n; i += 256) {
            const double d = (double)x[(size_t)i * kIn + f] - mu;
            s += d * d;
        }
        red[tid] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < (uint32_t)o) red[tid] += red[tid + o];
            __syncthreads();
        }
        if (tid == 0) {
            const double sd = sqrt(red[0] / (double)n);
            M->mean[f] = (float)mu;
            M->inv_std[f] = (float)(1.0 / fmax(sd, 1e-6));
        }
        __syncthreads();
    }
    for (uint32_t j = tid; j < (uint32_t)kP; j += 256) {
        master[j] = init[j];
        mom1[j] = 0.f;
        mom2[j] = 0.f;
        M->w[j] = f32_to_bf16_bits(init[j]);
    }
    for (uint32_t j = tid; j < 8; j += 256) M->pad[j] = 0;
    if (tid == 0) {
        M->magic = GPOP_MLP_MAGIC;
        M->n_params = kP;
        M->pad0 = 0;
        M->margin = 0.f;
    }
}

__global__ __launch_bounds__(256) void k_mlp_forward(const gpop_mlp_model* __restrict__ M,
                                                     const float* __restrict__ x, uint32_t n,
                                                     float* __restrict__ out) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float f[kIn];
    for (int j = 0; j < kIn; ++j) f[j] = x[(size_t)i * kIn + j];
    float z;
    (void)mlp_logit(M, f, &z);
    out[i] = z;
}

__device__ __forceinline__ float wbf(const uint16_t* __restrict__ w, int j) {
    return bf16_bits_to_f32(w[j]);
}

// One chunk of 64 samples per wave: forward and backward per lane, then the
// per-parameter sums over the chunk, written as one partial row.
__global__ __launch_bounds__(64) void k_mlp_grad_chunk(const gpop_mlp_model* __restrict__ M,
                                                       const float* __restrict__ x,
                                                       const float* __restrict__ t_sc,
                                                       const float* __restrict__ t_pc, uint32_t n,
                                                       float* __restrict__ part) {
    __shared__ float xs[64][kIn + 1];
    __shared__ float h1[64][kRow], h2[64][kRow], d1[64][kRow], d2[64][kRow];
    __shared__ float gs[64];
    const uint32_t lane = threadIdx.x;
    const uint32_t i = blockIdx.x * 64 + lane;
    const bool valid = i < n;
    const uint16_t* __restrict__ w = M->w;

    // forward
    float xh[kIn];
    for (int j = 0; j < kIn; ++j) {
        xh[j] = valid ? (x[(size_t)i * kIn + j] - M->mean[j]) * M->inv_std[j] : 0.f;
        xs[lane][j] = xh[j];
    }
    for (int o = 0; o < kH; ++o) {
        float a = wbf(w, GPOP_MLP_B1 + o);
#pragma unroll
        for (int j = 0; j < kIn; ++j) a = fmaf(wbf(w, GPOP_MLP_W1 + o * kIn + j), xh[j], a);
        h1[lane][o] = valid ? fmaxf(a, 0.f) : 0.f;
    }
    float z = wbf(w, GPOP_MLP_B3);
    for (int o = 0; o < kH; ++o) {
        float a = wbf(w, GPOP_MLP_B2 + o);
#pragma unroll 16
        for (int j = 0; j < kH; ++j) a = fmaf(wbf(w, GPOP_MLP_W2 + o * kH + j), h1[lane][j], a);
        const float r = valid ? fmaxf(a, 0.f) : 0.f;
        h2[lane][o] = r;
        z = fmaf(wbf(w, GPOP_MLP_W3 + o), r, z);
    }

    // loss and dL/dz (unnormalised: the reduce divides by the weight sum)
    float g = 0.f, loss = 0.f, c = 0.f;
    if (valid) {
        const float a = t_sc[i], b = t_pc[i];
        c = fabsf(a - b);
        const float y = b < a ? 1.f : 0.f;
        const float sig = 1.f / (1.f + expf(-z));
        g = c * (sig - y);
        loss = c * (fmaxf(z, 0.f) - y * z + log1pf(expf(-fabsf(z))));
    }
    gs[lane] = g;

    // backward through the two hidden layers
    for (int o = 0; o < kH; ++o) d2[lane][o] = h2[lane][o] > 0.f ? g * wbf(w, GPOP_MLP_W3 + o) : 0.f;
    for (int j = 0; j < kH; ++j) {
        float a = 0.f;
#pragma unroll 16
        for (int o = 0; o < kH; ++o) a = fmaf(wbf(w, GPOP_MLP_W2 + o * kH + j), d2[lane][o], a);
        d1[lane][j] = h1[lane][j] > 0.f ? a : 0.f;
    }
    __syncthreads();

    // sums over the chunk's samples, in sample order
    float* __restrict__ out = part + (size_t)blockIdx.x * kPart;
    for (int idx = lane; idx < kH * kIn; idx += 64) {
        const int o = idx / kIn, j = idx - o * kIn;
        float a = 0.f;
        for (int s = 0; s < 64; ++s) a = fmaf(d1[s][o], xs[s][j], a);
        out[GPOP_MLP_W1 + idx] = a;
    }
    {
        float a = 0.f, b = 0.f, e = 0.f;
        for (int s = 0; s < 64; ++s) {
            a += d1[s][lane];
            b += d2[s][lane];
            e = fmaf(gs[s], h2[s][lane], e);
        }
        out[GPOP_MLP_B1 + lane] = a;
        out[GPOP_MLP_B2 + lane] = b;
        out[GPOP_MLP_W3 + lane] = e;
    }
    for (int o = 0; o < kH; ++o) {
        float a = 0.f;
        for (int s = 0; s < 64; ++s) a = fmaf(d2[s][o], h1[s][lane], a);
        out[GPOP_MLP_W2 + o * kH + lane] = a;
    }
    // b3, loss and weight sum: wave sums in lane order via LDS
    __syncthreads();
    xs[lane][0] = loss;
    xs[lane][1] = c;
    __syncthreads();
    if (lane == 0) {
        float gb = 0.f, l = 0.f, cs = 0.f;
        for (int s = 0; s < 64; ++s) {
            gb += gs[s];
            l += xs[s][0];
            cs += xs[s][1];
        }
        out[GPOP_MLP_B3] = gb;
        out[kP] = l;
        out[kP + 1] = cs;
    }
}

// Sums the chunk partials of every parameter in chunk order (f64) and
// divides by the batch's weight sum.
__global__ __launch_bounds__(256) void k_mlp_grad_reduce(const float* __restrict__ part, uint32_t nchunk,
                                                         float* __restrict__ grad,
                                                         float* __restrict__ loss) {
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= (uint32_t)(kP + 1)) return;
    double cs = 0.0, s = 0.0;
    for (uint32_t b = 0; b < nchunk; ++b) {
        cs += (double)part[(size_t)b * kPart + kP + 1];
        s += (double)part[(size_t)b * kPart + j];
    }
    const double v = cs > 0.0 ? s / cs : 0.0;
    if (j < (uint32_t)kP) {
        grad[j] = (float)v;
    } else if (loss) {
        loss[0] = (float)v;
        loss[1] = (float)cs;
    }
}

__global__ __launch_bounds__(256) void k_mlp_adam(gpop_mlp_model* __restrict__ M, float* __restrict__ master,
                                                  float* __restrict__ mom1, float* __restrict__ mom2,
                                                  const float* __restrict__ grad, float lr, float c1,
                                                  float c2) {
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= (uint32_t)kP) return;
    const float g = grad[j];
    const float m = 0.9f * mom1[j] + 0.1f * g;
    const float v = 0.999f * mom2[j] + 0.001f * g * g;
    mom1[j] = m;
    mom2[j] = v;
    const float th = master[j] - lr * (m * c1) / (sqrtf(v * c2) + 1e-8f);
    master[j] = th;
    M->w[j] = f32_to_bf16_bits(th);
}

// Adds delta to the output bias (master and its bf16 copy).
__global__ __launch_bounds__(64) void k_mlp_shift(gpop_mlp_model* __restrict__ M, float* __restrict__ master,
                                                 float delta) {
    if (threadIdx.x != 0) return;
    const float b = master[GPOP_MLP_B3] + delta;
    master[GPOP_MLP_B3] = b;
    M->w[GPOP_MLP_B3] = f32_to_bf16_bits(b);
}

uint32_t nchunks(uint32_t n) { return (n + 63u) / 64u; }

// Chunk partials of gpop_mlp_grad_noalloc: a fixed array in device memory,
// one copy per GPU, held until the process ends. Host code must not pass
// `scratch` itself to a kernel (on the host it names a stand-in, not the
// device copy); it uses the address hipGetSymbolAddress reports for the
// current device.
constexpr uint32_t kNoAllocChunks = GPOP_MLP_NOALLOC_MAX_SAMPLES / 64u;
static __device__ __align__(256) float scratch[(size_t)kNoAllocChunks * kPart];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up once per device with
// that device current.
int scratch_of_current_device(float** out) {
    int dev = 0;
    HIP_OR_RETURN(hipGetDevice(&dev), "current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(GPOP_ENOTSUP, "device index %d >= %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIP_OR_RETURN(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "address of the gradient scratch");
        if (!p) return fail(GPOP_EDEVICE, "no device address for the gradient scratch");
        g_scratch_dev[dev] = (float*)p;
    }
    *out = g_scratch_dev[dev];
    return GPOP_OK;
}

// The two gradient kernels over a partial buffer of at least nchunks(n) rows.
int launch_grad(const gpop_mlp_model* d_model, const float* d_x, const float* d_t_sc, const float* d_t_pc,
                uint32_t n, float* d_grad, float* d_loss, float* part, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_grad_chunk, dim3(nchunks(n)), dim3(64), 0, st, d_model, d_x, d_t_sc, d_t_pc, n,
                       part);
    HIP_OR_RETURN(hipGetLastError(), "mlp gradient");
    hipLaunchKernelGGL(k_mlp_grad_reduce, dim3((kP + 1 + 255) / 256), dim3(256), 0, st, part, nchunks(n),
                       d_grad, d_loss);
    HIP_OR_RETURN(hipGetLastError(), "mlp gradient reduce");
    return GPOP_OK;
}

}  // namespace
}  // namespace gpop

using namespace gpop;

extern "C" {

int gpop_mlp_init(gpop_mlp_model* d_model, float* d_master, float* d_m, float* d_v,
                  const float* d_init, const float* d_x, uint32_t n, void* stream) {
    if (!d_model || !d_master || !d_m || !d_v || !d_init || !d_x) return fail(GPOP_EINVAL, "NULL argument");
    if (n == 0) return fail(GPOP_EINVAL, "no training samples");
    hipLaunchKernelGGL(k_mlp_init, dim3(1), dim3(256), 0, (hipStream_t)stream, d_model, d_master, d_m, d_v,
                       d_init, d_x, n);
    HIP_OR_RETURN(hipGetLastError(), "mlp init");
    return GPOP_OK;
}

int gpop_mlp_forward(const gpop_mlp_model* d_model, const float* d_x, uint32_t n, float* d_logits,
                     void* stream) {
    if (!d_model || (n && (!d_x || !d_logits))) return fail(GPOP_EINVAL, "NULL argument");
    if (n == 0) return GPOP_OK;
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_model, d_x,
                       n, d_logits);
    HIP_OR_RETURN(hipGetLastError(), "mlp forward");
    return GPOP_OK;
}

size_t gpop_mlp_grad_workspace(uint32_t n) { return (size_t)nchunks(n) * kPart * sizeof(float); }

int gpop_mlp_grad(const gpop_mlp_model* d_model, const float* d_x, const float* d_t_sc, const float* d_t_pc,
                  uint32_t n, float* d_grad, float* d_loss, void* d_ws, size_t ws_bytes, void* stream) {
    if (!d_model || !d_x || !d_t_sc || !d_t_pc || !d_grad || !d_ws) return fail(GPOP_EINVAL, "NULL argument");
    if (n == 0) return fail(GPOP_EINVAL, "no samples");
    if (ws_bytes < gpop_mlp_grad_workspace(n))
        return fail(GPOP_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, gpop_mlp_grad_workspace(n));
    return launch_grad(d_model, d_x, d_t_sc, d_t_pc, n, d_grad, d_loss, (float*)d_ws, (hipStream_t)stream);
}

int gpop_mlp_grad_noalloc(const gpop_mlp_model* d_model, const float* d_x, const float* d_t_sc,
                          const float* d_t_pc, uint32_t n, float* d_grad, float* d_loss, void* stream) {
    if (!d_model || !d_x || !d_t_sc || !d_t_pc || !d_grad) return fail(GPOP_EINVAL, "NULL argument");
    if (n == 0) return fail(GPOP_EINVAL, "no samples");
    if (n > GPOP_MLP_NOALLOC_MAX_SAMPLES)
        return fail(GPOP_EINVAL, "%u samples > GPOP_MLP_NOALLOC_MAX_SAMPLES (%u): use gpop_mlp_grad with a workspace",
                    n, (unsigned)GPOP_MLP_NOALLOC_MAX_SAMPLES);
    float* part = nullptr;
    const int rc = scratch_of_current_device(&part);
    if (rc) return rc;
    return launch_grad(d_model, d_x, d_t_sc, d_t_pc, n, d_grad, d_loss, part, (hipStream_t)stream);
}

int gpop_mlp_adam(gpop_mlp_model* d_model, float* d_master, float* d_m, float* d_v, const float* d_grad,
                  uint32_t step, float lr, void* stream) {
    if (!d_model || !d_master || !d_m || !d_v || !d_grad) return fail(GPOP_EINVAL, "NULL argument");
    if (step == 0) return fail(GPOP_EINVAL, "Adam steps count from 1");
    if (!(lr > 0.f) || !std::isfinite(lr)) return fail(GPOP_EINVAL, "lr must be finite and > 0");
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)step)));
    hipLaunchKernelGGL(k_mlp_adam, dim3((kP + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_model,
                       d_master, d_m, d_v, d_grad, lr, c1, c2);
    HIP_OR_RETURN(hipGetLastError(), "mlp adam");
    return GPOP_OK;
}

int gpop_mlp_train_step(gpop_mlp_model* d_model, float* d_master, float* d_m, float* d_v, const float* d_x,
                        const float* d_t_sc, const float* d_t_pc, uint32_t n, uint32_t step, float lr,
                        float* d_grad, float* d_loss, void* d_ws, size_t ws_bytes, void* stream) {
    int rc = gpop_mlp_grad(d_model, d_x, d_t_sc, d_t_pc, n, d_grad, d_loss, d_ws, ws_bytes, stream);
    if (rc) return rc;
    return gpop_mlp_adam(d_model, d_master, d_m, d_v, d_grad, step, lr, stream);
}

int gpop_mlp_shift_logit(gpop_mlp_model* d_model, float* d_master, float delta, void* stream) {
    if (!d_model || !d_master) return fail(GPOP_EINVAL, "NULL argument");
    if (!std::isfinite(delta)) return fail(GPOP_EINVAL, "delta must be finite");
    hipLaunchKernelGGL(k_mlp_shift, dim3(1), dim3(64), 0, (hipStream_t)stream, d_model, d_master, delta);
    HIP_OR_RETURN(hipGetLastError(), "mlp shift");
    return GPOP_OK;
}

int gpop_mlp_set_margin(gpop_mlp_model* d_model, float margin, void* stream) {
    if (!d_model) return fail(GPOP_EINVAL, "NULL argument");
    if (!(margin >= 0.f)) return fail(GPOP_EINVAL, "margin must be >= 0 (or +inf)");
    static_assert(offsetof(gpop_mlp_model, margin) % 4 == 0, "margin is 4-byte aligned");
    static_assert(sizeof(gpop_mlp_model) == 10240, "model layout");
    // the value is on this function's stack: wait for the copy before returning
    HIP_OR_RETURN(hipMemcpyAsync(reinterpret_cast<char*>(d_model) + offsetof(gpop_mlp_model, margin), &margin,
                                 sizeof margin, hipMemcpyHostToDevice, (hipStream_t)stream),
                  "write margin");
    HIP_OR_RETURN(hipStreamSynchronize((hipStream_t)stream), "sync");
    return GPOP_OK;
}

}  // extern "C"
