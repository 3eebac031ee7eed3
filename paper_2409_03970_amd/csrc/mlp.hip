// The learned key-CDF model: an fp32 perceptron 1 -> 32 -> 32 -> 1 with ReLU
// that maps a key to (an estimate of) its rank fraction.  It predicts the
// partition points of the parallel merge (Sec. 2.1); an exact bounded search
// corrects every prediction, so sort results never depend on it.
//
// Kernels (plain VALU fp32; the model is far too small for matrix cores):
//   forward      one thread per sample, parameters staged in LDS;
//   backward     phase 1: one thread per sample computes its forward values
//                and the per-sample factors of every gradient entry;
//                phase 2: each workgroup sums a fixed chunk of samples for all
//                1153 entries (+ the loss) in sample order;
//                phase 3: one thread per entry sums the chunk partials in
//                chunk order -- every sum has a fixed order, so reruns are
//                bitwise identical;
//   adam         one thread per parameter (Kingma and Ba 2015, Algorithm 1);
//   minibatch    sample positions from SplitMix64 (Steele, Lea, Flood 2014)
//                on a counter, key -> x, position/m -> target.
#include "hvms.h"
#include "hvms_internal.h"
#include "mlp_common.h"

namespace hvms {

namespace {

constexpr int H = 32;
constexpr int NP = HVMS_CDF_PARAMS;  // 1153
constexpr int NREC = 4 + 4 * H;      // per-sample record: x, dy, sq, pad, h1, dz1, h2, dz2
constexpr int CHUNK = 128;           // samples per phase-2 workgroup

__global__ __launch_bounds__(256) void cdf_forward_kernel(const float *__restrict__ p,
                                                          const float *__restrict__ x,
                                                          float *__restrict__ y, int64_t b)
{
    __shared__ float P[NP];
    for (int i = threadIdx.x; i < NP; i += blockDim.x)
        P[i] = p[i];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = cdf_eval(P, x[i]);
}

// The model sampled on the unit interval: table[i] = F(i / 2^16), i <= 2^16.
// The co-rank predictor reads it instead of evaluating the model per merge
// pair and pass (see cdf_lookup).
__global__ __launch_bounds__(256) void cdf_table_kernel(const float *__restrict__ p,
                                                        float *__restrict__ table)
{
    __shared__ float P[NP];
    for (int i = threadIdx.x; i < NP; i += blockDim.x)
        P[i] = p[i];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= kCdfTableSteps)
        table[i] = cdf_eval(P, (float)i * (1.0f / kCdfTableSteps));
}

// Phase 1: rec[f * b + i] holds field f of sample i.
__global__ __launch_bounds__(256) void cdf_bwd_samples_kernel(const float *__restrict__ p,
                                                              const float *__restrict__ x,
                                                              const float *__restrict__ tgt,
                                                              float *__restrict__ rec, int64_t b)
{
    __shared__ float P[NP];
    for (int i = threadIdx.x; i < NP; i += blockDim.x)
        P[i] = p[i];
    __syncthreads();
    const float *W1 = P, *b1 = P + H, *W2 = P + 2 * H, *b2 = P + 2 * H + H * H;
    const float *W3 = P + 3 * H + H * H;
    const float b3 = P[4 * H + H * H];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float xi = x[i];
        float h1[H], z2[H];
#pragma unroll
        for (int u = 0; u < H; ++u)
            h1[u] = fmaf(W1[u], xi, b1[u]);  // z1 for now
        float y = b3;
#pragma unroll
        for (int o = 0; o < H; ++o) {
            float z = b2[o];
#pragma unroll
            for (int u = 0; u < H; ++u)
                z = fmaf(W2[o * H + u], fmaxf(h1[u], 0.0f), z);
            z2[o] = z;
            y = fmaf(W3[o], fmaxf(z, 0.0f), y);
        }
        const float diff = y - tgt[i];
        const float dy = 2.0f * diff / (float)b;
        rec[0 * b + i] = xi;
        rec[1 * b + i] = dy;
        rec[2 * b + i] = diff * diff;
        rec[3 * b + i] = 0.0f;
        float dz2[H];
#pragma unroll
        for (int o = 0; o < H; ++o) {
            dz2[o] = z2[o] > 0.0f ? dy * W3[o] : 0.0f;
            rec[(4 + 2 * H + o) * b + i] = fmaxf(z2[o], 0.0f);  // h2
            rec[(4 + 3 * H + o) * b + i] = dz2[o];
        }
#pragma unroll
        for (int u = 0; u < H; ++u) {
            float dh = 0.0f;
#pragma unroll
            for (int o = 0; o < H; ++o)
                dh = fmaf(dz2[o], W2[o * H + u], dh);
            rec[(4 + u) * b + i] = fmaxf(h1[u], 0.0f);                  // h1
            rec[(4 + H + u) * b + i] = h1[u] > 0.0f ? dh : 0.0f;       // dz1
        }
    }
}

// Factor pair of gradient entry j: g_j = sum_i rec[fa(j)][i] * rec[fb(j)][i]
// (fb = -1 means a plain sum); entry NP is the loss (sum of squares / b).
__device__ __forceinline__ void entry_fields(int j, int &fa, int &fb)
{
    if (j < H) {                 // W1[u]: dz1[u] * x
        fa = 4 + H + j;
        fb = 0;
    } else if (j < 2 * H) {      // b1[u]: dz1[u]
        fa = 4 + H + (j - H);
        fb = -1;
    } else if (j < 2 * H + H * H) {  // W2[o][u]: dz2[o] * h1[u]
        const int q = j - 2 * H;
        fa = 4 + 3 * H + q / H;
        fb = 4 + q % H;
    } else if (j < 3 * H + H * H) {  // b2[o]: dz2[o]
        fa = 4 + 3 * H + (j - 2 * H - H * H);
        fb = -1;
    } else if (j < 4 * H + H * H) {  // W3[o]: dy * h2[o]
        fa = 1;
        fb = 4 + 2 * H + (j - 3 * H - H * H);
    } else if (j < NP) {         // b3: dy
        fa = 1;
        fb = -1;
    } else {                     // loss: sq
        fa = 2;
        fb = -1;
    }
}

// Phase 2: partial[c * (NP + 1) + j] = sum over the samples of chunk c.
__global__ __launch_bounds__(256) void cdf_bwd_partial_kernel(const float *__restrict__ rec,
                                                              float *__restrict__ partial, int64_t b)
{
    __shared__ float R[NREC][CHUNK];
    const int64_t c = blockIdx.x;
    const int64_t i0 = c * CHUNK;
    const int cnt = (int)(b - i0 < CHUNK ? b - i0 : CHUNK);
    for (int q = threadIdx.x; q < NREC * CHUNK; q += blockDim.x) {
        const int f = q / CHUNK, k = q % CHUNK;
        R[f][k] = k < cnt ? rec[f * b + i0 + k] : 0.0f;
    }
    __syncthreads();
    for (int j = threadIdx.x; j <= NP; j += blockDim.x) {
        int fa, fb;
        entry_fields(j, fa, fb);
        float s = 0.0f;
        if (fb < 0) {
            for (int k = 0; k < cnt; ++k)
                s += R[fa][k];
        } else {
            for (int k = 0; k < cnt; ++k)
                s = fmaf(R[fa][k], R[fb][k], s);
        }
        partial[c * (NP + 1) + j] = s;
    }
}

// Phase 3: chunk partials in chunk order.
__global__ __launch_bounds__(256) void cdf_bwd_final_kernel(const float *__restrict__ partial,
                                                            int64_t nchunks, int64_t b,
                                                            float *__restrict__ grad,
                                                            float *__restrict__ loss)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > NP)
        return;
    float s = 0.0f;
    for (int64_t c = 0; c < nchunks; ++c)
        s += partial[c * (NP + 1) + j];
    if (j < NP)
        grad[j] = s;
    else
        loss[0] = s / (float)b;
}

__global__ __launch_bounds__(256) void cdf_adam_kernel(float *__restrict__ p, float *__restrict__ m,
                                                       float *__restrict__ v,
                                                       const float *__restrict__ g, float lr,
                                                       float beta1, float beta2, float eps,
                                                       float bc1, float bc2)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= NP)
        return;
    const float gj = g[j];
    const float mj = beta1 * m[j] + (1.0f - beta1) * gj;
    const float vj = beta2 * v[j] + (1.0f - beta2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    p[j] -= lr * (mj / bc1) / (sqrtf(vj / bc2) + eps);
}

__global__ void cdf_zero_kernel(float *__restrict__ a, float *__restrict__ b)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < NP) {
        a[j] = 0.0f;
        b[j] = 0.0f;
    }
}

// Minibatch of training step `step`: position i_k = SplitMix64(seed, step *
// 2^32 + k) mod m of the sorted sample; x_k its key on the unit interval,
// target i_k / m.
__global__ __launch_bounds__(256) void cdf_batch_kernel(const int32_t *__restrict__ sorted,
                                                        int64_t m, int64_t batch, uint64_t seed,
                                                        uint64_t step, float *__restrict__ x,
                                                        float *__restrict__ t)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= batch)
        return;
    const uint64_t r = splitmix64(seed, (step << 32) + (uint64_t)k);
    const int64_t i = (int64_t)(r % (uint64_t)m);
    x[k] = key_to_unit(sorted[i]);
    t[k] = (float)((double)i / (double)m);
}

// out[k] = keys[SplitMix64(seed, k) mod n]: a uniform sample with replacement.
__global__ __launch_bounds__(256) void cdf_sample_kernel(const int32_t *__restrict__ keys, int64_t n,
                                                         int64_t m, uint64_t seed,
                                                         int32_t *__restrict__ out)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * blockDim.x)
        out[k] = keys[splitmix64(seed, (uint64_t)k) % (uint64_t)n];
}

struct BwdWs {
    int64_t rec, partial, total;
};

BwdWs bwd_layout(int64_t b)
{
    BwdWs w;
    const int64_t nchunks = (b + CHUNK - 1) / CHUNK;
    w.rec = 0;
    w.partial = ((NREC * b * 4) + 255) & ~(int64_t)255;
    w.total = w.partial + (((nchunks * (NP + 1) * 4) + 255) & ~(int64_t)255);
    return w;
}

hipError_t backward(const float *p, const float *x, const float *t, float *grad, float *loss,
                    int64_t b, char *ws, hipStream_t s)
{
    const BwdWs w = bwd_layout(b);
    float *rec = (float *)(ws + w.rec);
    float *partial = (float *)(ws + w.partial);
    const int64_t nchunks = (b + CHUNK - 1) / CHUNK;
    int64_t blocks = (b + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(cdf_bwd_samples_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, x, t,
                       rec, b);
    hipLaunchKernelGGL(cdf_bwd_partial_kernel, dim3((unsigned)nchunks), dim3(256), 0, s, rec,
                       partial, b);
    hipLaunchKernelGGL(cdf_bwd_final_kernel, dim3((NP + 1 + 255) / 256), dim3(256), 0, s, partial,
                       nchunks, b, grad, loss);
    return hipGetLastError();
}

hipError_t adam(float *p, float *m, float *v, const float *g, int step, float lr, float beta1,
                float beta2, float eps, hipStream_t s)
{
    const float bc1 = (float)(1.0 - pow((double)beta1, (double)step));
    const float bc2 = (float)(1.0 - pow((double)beta2, (double)step));
    hipLaunchKernelGGL(cdf_adam_kernel, dim3((NP + 255) / 256), dim3(256), 0, s, p, m, v, g, lr,
                       beta1, beta2, eps, bc1, bc2);
    return hipGetLastError();
}

struct TrainWs {
    int64_t x, t, grad, loss, bwd, total;
};

TrainWs train_layout(int64_t batch)
{
    TrainWs w;
    auto a = [](int64_t v) { return (v + 255) & ~(int64_t)255; };
    w.x = 0;
    w.t = a(batch * 4);
    w.grad = w.t + a(batch * 4);
    w.loss = w.grad + a(NP * 4);
    w.bwd = w.loss + 256;
    w.total = w.bwd + bwd_layout(batch).total;
    return w;
}

int status(hipError_t e)
{
    if (e == hipSuccess)
        return HVMS_OK;
    set_last_hip_error((int)e);
    return HVMS_ERR_HIP;
}

int check(void *ws, size_t bytes, int64_t need)
{
    if (!ws || (int64_t)bytes < need || ((uintptr_t)ws & 255))
        return HVMS_ERR_WORKSPACE;
    return HVMS_OK;
}

}  // namespace

hipError_t launch_cdf_table(const float *params, float *table, hipStream_t s)
{
    hipLaunchKernelGGL(cdf_table_kernel, dim3((kCdfTableSteps + 256) / 256), dim3(256), 0, s,
                       params, table);
    return hipGetLastError();
}

}  // namespace hvms

using namespace hvms;

extern "C" {

int64_t hvms_cdf_param_count(void) { return HVMS_CDF_PARAMS; }

int hvms_cdf_forward(const float *d_params, const float *d_x, float *d_y, int64_t b, void *stream)
{
    if (b < 0 || (b > 0 && (!d_params || !d_x || !d_y)))
        return HVMS_ERR_INVALID_ARG;
    if (b == 0)
        return HVMS_OK;
    int64_t blocks = (b + 255) / 256;
    if (blocks > 8192)
        blocks = 8192;
    hipLaunchKernelGGL(cdf_forward_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, d_params, d_x, d_y, b);
    return status(hipGetLastError());
}

int64_t hvms_cdf_workspace_bytes(int64_t b)
{
    if (b < 0)
        return HVMS_ERR_INVALID_ARG;
    return bwd_layout(b).total;
}

int hvms_cdf_backward(const float *d_params, const float *d_x, const float *d_t, float *d_grad,
                      float *d_loss, int64_t b, void *d_ws, size_t ws_bytes, void *stream)
{
    if (b <= 0 || !d_params || !d_x || !d_t || !d_grad || !d_loss)
        return HVMS_ERR_INVALID_ARG;
    const int st = check(d_ws, ws_bytes, bwd_layout(b).total);
    if (st)
        return st;
    return status(backward(d_params, d_x, d_t, d_grad, d_loss, b, (char *)d_ws,
                           (hipStream_t)stream));
}

int hvms_cdf_adam_step(float *d_params, float *d_m, float *d_v, const float *d_grad, int32_t step,
                       float lr, float beta1, float beta2, float eps, void *stream)
{
    if (!d_params || !d_m || !d_v || !d_grad || step < 1 || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f))
        return HVMS_ERR_INVALID_ARG;
    return status(adam(d_params, d_m, d_v, d_grad, step, lr, beta1, beta2, eps,
                       (hipStream_t)stream));
}

int64_t hvms_cdf_train_workspace_bytes(int64_t batch)
{
    if (batch <= 0)
        return HVMS_ERR_INVALID_ARG;
    return train_layout(batch).total;
}

int hvms_cdf_train(float *d_params, float *d_m, float *d_v, const int32_t *d_sorted, int64_t m,
                   int64_t batch, int32_t steps, float lr, uint64_t seed, void *d_ws,
                   size_t ws_bytes, void *stream)
{
    if (!d_params || !d_m || !d_v || !d_sorted || m <= 0 || batch <= 0 || steps < 0)
        return HVMS_ERR_INVALID_ARG;
    const TrainWs w = train_layout(batch);
    int st = check(d_ws, ws_bytes, w.total);
    if (st)
        return st;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)d_ws;
    float *x = (float *)(ws + w.x), *t = (float *)(ws + w.t), *g = (float *)(ws + w.grad);
    float *loss = (float *)(ws + w.loss);
    hipLaunchKernelGGL(cdf_zero_kernel, dim3((NP + 255) / 256), dim3(256), 0, s, d_m, d_v);
    for (int step = 1; step <= steps; ++step) {
        hipLaunchKernelGGL(cdf_batch_kernel, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0,
                           s, d_sorted, m, batch, seed, (uint64_t)(step - 1), x, t);
        hipError_t e = backward(d_params, x, t, g, loss, batch, ws + w.bwd, s);
        if (e == hipSuccess)
            e = adam(d_params, d_m, d_v, g, step, lr, 0.9f, 0.999f, 1e-8f, s);
        st = status(e);
        if (st)
            return st;
    }
    return HVMS_OK;
}

int hvms_cdf_sample_i32(const int32_t *d_keys, int64_t n, int64_t m, uint64_t seed,
                        int32_t *d_out, void *stream)
{
    if (n < 0 || m < 0 || (m > 0 && (n == 0 || !d_keys || !d_out)))
        return HVMS_ERR_INVALID_ARG;
    if (m == 0)
        return HVMS_OK;
    int64_t blocks = (m + 255) / 256;
    if (blocks > 16384)
        blocks = 16384;
    hipLaunchKernelGGL(cdf_sample_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       d_keys, n, m, seed, d_out);
    return status(hipGetLastError());
}

}  // extern "C"
