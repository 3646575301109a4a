// A small MLP that scores candidate mini-bucket partitions (2 hidden layers
// of `hidden` ReLU units, one linear output): FP32 training kernels (forward,
// backward, Adam) and a BF16 inference kernel (bf16 weights and activations,
// fp32 accumulation).
//
// Parameters (fp32, contiguous): W1[H][F], b1[H], W2[H][H], b2[H], W3[H], b3.
// Row j of W1 / W2 holds the input weights of hidden unit j.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>

#include "bx_internal.h"

namespace bx {

// Per-sample deltas of bx_mlp_backward_noalloc (BX_MLP_NOALLOC_MAX_BATCH
// samples x 2 hidden layers of 128 units, fp32: 4 MiB on each GPU).
static __device__ __align__(256) float scratch[(size_t)BX_MLP_NOALLOC_MAX_BATCH * 2 * 128];

namespace {

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return set_error(BX_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kSB = 8;          // samples per workgroup
constexpr int kMaxIn = 64;      // input features at most
constexpr int kHidden = 128;    // hidden units (one thread each)

struct Layout {
    int64_t w1, b1, w2, b2, w3, b3, total;
};

__host__ __device__ inline Layout layout(int F, int H) {
    Layout l;
    l.w1 = 0;
    l.b1 = l.w1 + (int64_t)H * F;
    l.w2 = l.b1 + H;
    l.b2 = l.w2 + (int64_t)H * H;
    l.w3 = l.b2 + H;
    l.b3 = l.w3 + H;
    l.total = l.b3 + 1;
    return l;
}

// fp32 -> bf16, round to nearest, ties to even (finite inputs)
__device__ inline uint16_t to_bf16(float f) {
    const uint32_t b = __float_as_uint(f);
    return (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// forward pass of kSB samples per workgroup; hidden unit j = thread j.
// act[b] = [h1 (H) | h2 (H)] after ReLU.
__global__ __launch_bounds__(kHidden) void mlp_forward_kernel(const float *p, const float *x, float *act,
                                                              float *y, int batch, int F) {
    const int H = kHidden;
    const Layout L = layout(F, H);
    __shared__ float xs[kSB][kMaxIn];
    __shared__ float h1s[kSB][kHidden];
    __shared__ float part[kSB][kHidden];
    const int j = threadIdx.x;
    const int b0 = blockIdx.x * kSB;
    for (int t = j; t < kSB * F; t += H) {
        const int s = t / F, i = t - s * F;
        xs[s][i] = b0 + s < batch ? x[(int64_t)(b0 + s) * F + i] : 0.f;
    }
    __syncthreads();
    for (int s = 0; s < kSB; ++s) {
        float a = p[L.b1 + j];
        for (int i = 0; i < F; ++i) a += p[L.w1 + (int64_t)j * F + i] * xs[s][i];
        a = a > 0.f ? a : 0.f;
        h1s[s][j] = a;
        if (b0 + s < batch) act[(int64_t)(b0 + s) * 2 * H + j] = a;
    }
    __syncthreads();
    for (int s = 0; s < kSB; ++s) {
        float a = p[L.b2 + j];
        for (int k = 0; k < H; ++k) a += p[L.w2 + (int64_t)j * H + k] * h1s[s][k];
        a = a > 0.f ? a : 0.f;
        if (b0 + s < batch) act[(int64_t)(b0 + s) * 2 * H + H + j] = a;
        part[s][j] = p[L.w3 + j] * a;
    }
    __syncthreads();
    if (j < kSB && b0 + j < batch) {
        float a = p[L.b3];
        for (int k = 0; k < H; ++k) a += part[j][k];
        y[b0 + j] = a;
    }
}

// per-sample deltas: d2 = dy * W3 * [h2 > 0], d1 = (W2^T d2) * [h1 > 0];
// work[b] = [d1 (H) | d2 (H)]
__global__ __launch_bounds__(kHidden) void mlp_delta_kernel(const float *p, const float *act, const float *dy,
                                                            float *work, int batch, int F) {
    const int H = kHidden;
    const Layout L = layout(F, H);
    __shared__ float d2s[kSB][kHidden];
    const int j = threadIdx.x;
    const int b0 = blockIdx.x * kSB;
    for (int s = 0; s < kSB; ++s) {
        float d = 0.f;
        if (b0 + s < batch) {
            const float h2 = act[(int64_t)(b0 + s) * 2 * H + H + j];
            d = h2 > 0.f ? dy[b0 + s] * p[L.w3 + j] : 0.f;
            work[(int64_t)(b0 + s) * 2 * H + H + j] = d;
        }
        d2s[s][j] = d;
    }
    __syncthreads();
    for (int s = 0; s < kSB; ++s) {
        if (b0 + s >= batch) break;
        float a = 0.f;
        for (int q = 0; q < H; ++q) a += d2s[s][q] * p[L.w2 + (int64_t)q * H + j];
        const float h1 = act[(int64_t)(b0 + s) * 2 * H + j];
        work[(int64_t)(b0 + s) * 2 * H + j] = h1 > 0.f ? a : 0.f;
    }
}

// gradient of every parameter, summed over the batch (one thread each)
__global__ void mlp_grad_kernel(const float *x, const float *act, const float *dy, const float *work, float *g,
                                int batch, int F) {
    const int H = kHidden;
    const Layout L = layout(F, H);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= L.total) return;
    float a = 0.f;
    if (t < L.b1) {                                 // W1[j][i]: d1[j] * x[i]
        const int j = (int)(t / F), i = (int)(t - (int64_t)j * F);
        for (int b = 0; b < batch; ++b) a += work[(int64_t)b * 2 * H + j] * x[(int64_t)b * F + i];
    } else if (t < L.w2) {                          // b1[j]
        const int j = (int)(t - L.b1);
        for (int b = 0; b < batch; ++b) a += work[(int64_t)b * 2 * H + j];
    } else if (t < L.b2) {                          // W2[j][k]: d2[j] * h1[k]
        const int64_t o = t - L.w2;
        const int j = (int)(o / H), k = (int)(o - (int64_t)j * H);
        for (int b = 0; b < batch; ++b) a += work[(int64_t)b * 2 * H + H + j] * act[(int64_t)b * 2 * H + k];
    } else if (t < L.w3) {                          // b2[j]
        const int j = (int)(t - L.b2);
        for (int b = 0; b < batch; ++b) a += work[(int64_t)b * 2 * H + H + j];
    } else if (t < L.b3) {                          // W3[j]: dy * h2[j]
        const int j = (int)(t - L.w3);
        for (int b = 0; b < batch; ++b) a += dy[b] * act[(int64_t)b * 2 * H + H + j];
    } else {                                        // b3
        for (int b = 0; b < batch; ++b) a += dy[b];
    }
    g[t] = a;
}

__global__ void mlp_adam_kernel(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                                float b2, float eps, float c1, float c2) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

// loss = mean (y - t)^2 and dy = 2 (y - t) / batch; one workgroup of 256
__global__ __launch_bounds__(256) void mlp_mse_kernel(const float *y, const float *t, float *dy, float *loss,
                                                      int batch) {
    __shared__ float red[256];
    const float inv = 1.f / (float)batch;
    float acc = 0.f;
    for (int b = threadIdx.x; b < batch; b += 256) {
        const float d = y[b] - t[b];
        dy[b] = 2.f * inv * d;
        acc += d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] * inv;
}

__global__ void mlp_pack_kernel(const float *p, uint16_t *q, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) q[t] = to_bf16(p[t]);
}

// inference with bf16 weights and activations, fp32 accumulation
__global__ __launch_bounds__(kHidden) void mlp_infer_bf16_kernel(const uint16_t *q, const float *x, float *y,
                                                                 int batch, int F) {
    const int H = kHidden;
    const Layout L = layout(F, H);
    __shared__ float xs[kSB][kMaxIn];
    __shared__ float h1s[kSB][kHidden];
    __shared__ float part[kSB][kHidden];
    const int j = threadIdx.x;
    const int b0 = blockIdx.x * kSB;
    for (int t = j; t < kSB * F; t += H) {
        const int s = t / F, i = t - s * F;
        xs[s][i] = b0 + s < batch ? from_bf16(to_bf16(x[(int64_t)(b0 + s) * F + i])) : 0.f;
    }
    __syncthreads();
    for (int s = 0; s < kSB; ++s) {
        float a = from_bf16(q[L.b1 + j]);
        for (int i = 0; i < F; ++i) a += from_bf16(q[L.w1 + (int64_t)j * F + i]) * xs[s][i];
        a = a > 0.f ? a : 0.f;
        h1s[s][j] = from_bf16(to_bf16(a));
    }
    __syncthreads();
    for (int s = 0; s < kSB; ++s) {
        float a = from_bf16(q[L.b2 + j]);
        for (int k = 0; k < H; ++k) a += from_bf16(q[L.w2 + (int64_t)j * H + k]) * h1s[s][k];
        a = a > 0.f ? a : 0.f;
        part[s][j] = from_bf16(q[L.w3 + j]) * from_bf16(to_bf16(a));
    }
    __syncthreads();
    if (j < kSB && b0 + j < batch) {
        float a = from_bf16(q[L.b3]);
        for (int k = 0; k < H; ++k) a += part[j][k];
        y[b0 + j] = a;
    }
}

bx_status check(const bx_mlp *m, int32_t batch) {
    if (!m) return set_error(BX_E_INVALID, "mlp is NULL");
    if (m->hidden != kHidden) return set_error(BX_E_UNSUPPORTED, "hidden width must be 128");
    if (m->n_in < 1 || m->n_in > kMaxIn) return set_error(BX_E_UNSUPPORTED, "1..64 input features");
    if (batch < 0) return set_error(BX_E_INVALID, "batch < 0");
    return BX_OK;
}

// ------------------------------------------- backward pass without allocation
// The backward pass's per-sample deltas live in a file-scope device array
// instead of a caller buffer.  Each GPU holds its own copy (4 MiB, for
// kNoAllocMaxBatch samples) until the process ends; its device address is
// looked up once per device with that device current and kept per device.
// The delta kernel writes every entry the gradient kernel then reads (rows
// [0, batch)), so nothing is cleared between calls.  Calls on one GPU share
// the array: overlapping calls race.
constexpr int32_t kNoAllocMaxBatch = BX_MLP_NOALLOC_MAX_BATCH;
static_assert(sizeof(scratch) == sizeof(float) * (size_t)kNoAllocMaxBatch * 2 * kHidden, "scratch size");
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kNoAllocMaxDevices] = {};

bx_status scratch_for_current_device(float **out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices) return set_error(BX_E_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_error(BX_E_DEVICE, "hipGetSymbolAddress returned NULL");
        g_scratch_ptr[dev] = static_cast<float *>(p);
    }
    *out = g_scratch_ptr[dev];
    return BX_OK;
}

}  // namespace

int64_t mlp_num_params(int32_t n_in, int32_t hidden) { return layout(n_in, hidden).total; }

bx_status mlp_forward(const bx_mlp *m, const float *x, float *act, float *y, int32_t batch, void *stream) {
    bx_status s = check(m, batch);
    if (s != BX_OK) return s;
    if (!m->d_params || !x || !act || !y) return set_error(BX_E_INVALID, "NULL device pointer");
    if (batch == 0) return BX_OK;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((batch + kSB - 1) / kSB), dim3(kHidden), 0,
                       static_cast<hipStream_t>(stream), m->d_params, x, act, y, batch, m->n_in);
    HIP_TRY(hipGetLastError());
    return BX_OK;
}

bx_status mlp_backward(const bx_mlp *m, const float *x, const float *act, const float *dy, float *grads,
                       float *work, int32_t batch, void *stream) {
    bx_status s = check(m, batch);
    if (s != BX_OK) return s;
    if (!m->d_params || !x || !act || !dy || !grads || !work) return set_error(BX_E_INVALID, "NULL device pointer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (batch > 0)
        hipLaunchKernelGGL(mlp_delta_kernel, dim3((batch + kSB - 1) / kSB), dim3(kHidden), 0, st, m->d_params,
                           act, dy, work, batch, m->n_in);
    const int64_t n = mlp_num_params(m->n_in, m->hidden);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, act, dy, work,
                       grads, batch, m->n_in);
    HIP_TRY(hipGetLastError());
    return BX_OK;
}

bx_status mlp_backward_noalloc(const bx_mlp *m, const float *x, const float *act, const float *dy, float *grads,
                               int32_t batch, void *stream) {
    bx_status s = check(m, batch);
    if (s != BX_OK) return s;
    if (batch > kNoAllocMaxBatch)
        return set_error(BX_E_TOO_LARGE, "batch " + std::to_string(batch) + " exceeds the " +
                                             std::to_string(kNoAllocMaxBatch) +
                                             " samples the static backward scratch holds");
    float *work = nullptr;
    s = scratch_for_current_device(&work);
    if (s != BX_OK) return s;
    return mlp_backward(m, x, act, dy, grads, work, batch, stream);
}

bx_status mlp_adam(const bx_mlp *m, const float *grads, float *mom, float *vel, float lr, float beta1,
                   float beta2, float eps, int32_t step, void *stream) {
    bx_status s = check(m, 0);
    if (s != BX_OK) return s;
    if (!m->d_params || !grads || !mom || !vel) return set_error(BX_E_INVALID, "NULL device pointer");
    if (step < 1) return set_error(BX_E_INVALID, "step counts from 1");
    const int64_t n = mlp_num_params(m->n_in, m->hidden);
    const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), m->d_params, grads, mom, vel, n, lr, beta1, beta2, eps,
                       c1, c2);
    HIP_TRY(hipGetLastError());
    return BX_OK;
}

bx_status mlp_pack_bf16(const bx_mlp *m, void *stream) {
    bx_status s = check(m, 0);
    if (s != BX_OK) return s;
    if (!m->d_params || !m->d_params_bf16) return set_error(BX_E_INVALID, "NULL device pointer");
    const int64_t n = mlp_num_params(m->n_in, m->hidden);
    hipLaunchKernelGGL(mlp_pack_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), m->d_params, m->d_params_bf16, n);
    HIP_TRY(hipGetLastError());
    return BX_OK;
}

bx_status mlp_mse(const float *y, const float *t, float *dy, float *loss, int32_t batch, void *stream) {
    if (batch < 1) return set_error(BX_E_INVALID, "batch < 1");
    if (!y || !t || !dy || !loss) return set_error(BX_E_INVALID, "NULL device pointer");
    hipLaunchKernelGGL(mlp_mse_kernel, dim3(1), dim3(256), 0, static_cast<hipStream_t>(stream), y, t, dy, loss,
                       batch);
    HIP_TRY(hipGetLastError());
    return BX_OK;
}

bx_status mlp_infer_bf16(const bx_mlp *m, const float *x, float *y, int32_t batch, void *stream) {
    bx_status s = check(m, batch);
    if (s != BX_OK) return s;
    if (!m->d_params_bf16 || !x || !y) return set_error(BX_E_INVALID, "NULL device pointer");
    if (batch == 0) return BX_OK;
    hipLaunchKernelGGL(mlp_infer_bf16_kernel, dim3((batch + kSB - 1) / kSB), dim3(kHidden), 0,
                       static_cast<hipStream_t>(stream), m->d_params_bf16, x, y, batch, m->n_in);
    HIP_TRY(hipGetLastError());
    return BX_OK;
}

// Chooser used by bx_plan_create_learned: the candidates' features go to the
// device, the bf16 network scores them, and each decision takes the best
// candidate whose score exceeds the greedy candidate's by more than `margin`
// (otherwise the greedy partition).
bx_status mlp_choose(void *vctx, int32_t n_dec, const int32_t *dec_inst, const int32_t *off, const float *feats,
                     int32_t *choices) {
    (void)dec_inst;
    LearnedCtx *ctx = static_cast<LearnedCtx *>(vctx);
    const int32_t n = off[n_dec];
    const size_t need = (size_t)n * (kPartFeatures + 1) * sizeof(float);
    if (need > ctx->buf_bytes) return set_error(BX_E_NOMEM, "device buffer too small for the partition features");
    hipStream_t st = static_cast<hipStream_t>(ctx->stream);
    float *dx = static_cast<float *>(ctx->d_buf);
    float *dy = dx + (size_t)n * kPartFeatures;
    HIP_TRY(hipMemcpyAsync(dx, feats, (size_t)n * kPartFeatures * sizeof(float), hipMemcpyHostToDevice, st));
    bx_status s = mlp_infer_bf16(ctx->model, dx, dy, n, ctx->stream);
    if (s != BX_OK) return s;
    std::vector<float> score(n);
    HIP_TRY(hipMemcpyAsync(score.data(), dy, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int32_t d = 0; d < n_dec; ++d) {
        int32_t best = 0;
        float best_gain = ctx->margin;
        for (int32_t c = off[d] + 1; c < off[d + 1]; ++c) {
            const float gain = score[c] - score[off[d]];
            if (gain > best_gain) { best_gain = gain; best = c - off[d]; }
        }
        choices[d] = best;
    }
    return BX_OK;
}

}  // namespace bx
