// Device training and evaluation of the 1-64-64-1 ReLU CDF network used by
// the learned bucket path (not part of the paper).
//
// Parameters (4353 floats, one device vector):
//   W1[64] b1[64] W2[64*64] (row-major: W2[i*64+j] feeds hidden-1 unit j into
//   hidden-2 unit i) b2[64] w3[64] b3
//   y(u) = w3 . relu(W2 relu(W1 u + b1) + b2) + b3,   loss = mean (y - t)^2
//
// Training is data parallel over work-groups, two launches per step: every
// work-group takes 32 samples, computes its partial gradient in LDS with every
// sum in a fixed order and writes it out; then every work-group of the second
// launch sums a slice of the parameters over all partials in work-group order
// and applies Adam (Kingma & Ba) to it.  No floating-point atomics anywhere,
// so a run is bit reproducible.
#include <hip/hip_runtime.h>

#include "gs_device.h"
#include "gs_internal.h"
#include "gs_mlp.h"

namespace gs {

namespace {

constexpr int HID = 64;
constexpr int OW1 = 0, OB1 = 64, OW2 = 128, OB2 = 128 + 64 * 64, OW3 = OB2 + 64, OB3 = OW3 + 64;
static_assert(OB3 + 1 == kMlpParams, "parameter layout");
constexpr int TR_NT = 256;
constexpr int SPW = 32;                 // samples per work-group per step
constexpr int RS = HID + 1;             // padded LDS row stride (no bank conflicts)

struct TrainLds {
    float p[kMlpParams + 3];
    float g[kMlpParams + 3];
    float w2[HID * RS];                 // W2 with padded rows
    float u[SPW], t[SPW], dy[SPW], y[SPW];
    float z1[SPW * RS], h1[SPW * RS];
    float z2[SPW * RS], h2[SPW * RS];
    float g2[SPW * RS], g1[SPW * RS];
    float red[TR_NT / 64][64];
    float loss;
};

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Partial loss (sum of squared errors) and gradient (sums over this group's
// SPW samples) into L.g / L.loss; L.p holds the parameters, L.u / L.t the
// samples.  inv_batch = 1 / total batch over all work-groups.  Each thread
// computes a small block of outputs with its operands in registers; every
// sum runs over its index in increasing order.
__device__ void wg_loss_grad(TrainLds &L, float inv_batch)
{
    static_assert(TR_NT == 256 && SPW == 32 && HID == 64, "thread blocking below");
    const int tid = threadIdx.x;
    for (int k = tid; k < HID * HID; k += TR_NT) L.w2[(k >> 6) * RS + (k & 63)] = L.p[OW2 + k];
    for (int idx = tid; idx < SPW * HID; idx += TR_NT) {
        const int s = idx / HID, j = idx % HID;
        const float z = fmaf(L.p[OW1 + j], L.u[s], L.p[OB1 + j]);
        L.z1[s * RS + j] = z;
        L.h1[s * RS + j] = z > 0.f ? z : 0.f;
    }
    __syncthreads();
    // hidden layer 2: thread block of 2 samples x 4 units
    {
        const int s0 = 2 * (tid & 15), i0 = 4 * (tid >> 4);
        float acc[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[a][c] = L.p[OB2 + i0 + c];
#pragma unroll 8
        for (int j = 0; j < HID; ++j) {
            const float h0 = L.h1[s0 * RS + j], h1v = L.h1[(s0 + 1) * RS + j];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float w = L.w2[(i0 + c) * RS + j];
                acc[0][c] = fmaf(w, h0, acc[0][c]);
                acc[1][c] = fmaf(w, h1v, acc[1][c]);
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                L.z2[(s0 + a) * RS + i0 + c] = acc[a][c];
                L.h2[(s0 + a) * RS + i0 + c] = acc[a][c] > 0.f ? acc[a][c] : 0.f;
            }
    }
    __syncthreads();
    if (tid < SPW) {
        const int s = tid;
        float y = L.p[OB3];
#pragma unroll 16
        for (int i = 0; i < HID; ++i) y = fmaf(L.p[OW3 + i], L.h2[s * RS + i], y);
        const float r = y - L.t[s];
        L.y[s] = r * r;
        L.dy[s] = 2.f * r * inv_batch;
    }
    __syncthreads();
    if (tid == 0) {
        float acc = 0.f;
        for (int s = 0; s < SPW; ++s) acc += L.y[s];
        L.loss = acc;
    }
    for (int idx = tid; idx < SPW * HID; idx += TR_NT) {
        const int s = idx / HID, i = idx % HID;
        L.g2[s * RS + i] = L.z2[s * RS + i] > 0.f ? L.dy[s] * L.p[OW3 + i] : 0.f;
    }
    __syncthreads();
    // dW2[i][j] = sum_s g2[s][i] h1[s][j]: thread block of 4 x 4
    {
        const int i0 = 4 * (tid >> 4), j0 = 4 * (tid & 15);
        float acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[a][c] = 0.f;
#pragma unroll 8
        for (int s = 0; s < SPW; ++s) {
            float gv[4], hv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) gv[a] = L.g2[s * RS + i0 + a];
#pragma unroll
            for (int c = 0; c < 4; ++c) hv[c] = L.h1[s * RS + j0 + c];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[a][c] = fmaf(gv[a], hv[c], acc[a][c]);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) L.g[OW2 + (i0 + a) * HID + j0 + c] = acc[a][c];
    }
    // g1[s][j] = [z1 > 0] sum_i W2[i][j] g2[s][i]: thread block of 2 x 4
    {
        const int s0 = 2 * (tid & 15), j0 = 4 * (tid >> 4);
        float acc[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[a][c] = 0.f;
#pragma unroll 8
        for (int i = 0; i < HID; ++i) {
            const float g0 = L.g2[s0 * RS + i], g1v = L.g2[(s0 + 1) * RS + i];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float w = L.w2[i * RS + j0 + c];
                acc[0][c] = fmaf(w, g0, acc[0][c]);
                acc[1][c] = fmaf(w, g1v, acc[1][c]);
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int o = (s0 + a) * RS + j0 + c;
                L.g1[o] = L.z1[o] > 0.f ? acc[a][c] : 0.f;
            }
    }
    if (tid < HID) {
        const int i = tid;
        float db2 = 0.f, dw3 = 0.f;
#pragma unroll 8
        for (int s = 0; s < SPW; ++s) {
            db2 += L.g2[s * RS + i];
            dw3 = fmaf(L.dy[s], L.h2[s * RS + i], dw3);
        }
        L.g[OB2 + i] = db2;
        L.g[OW3 + i] = dw3;
    }
    if (tid == HID) {
        float db3 = 0.f;
        for (int s = 0; s < SPW; ++s) db3 += L.dy[s];
        L.g[OB3] = db3;
    }
    __syncthreads();
    if (tid < HID) {
        const int j = tid;
        float dw1 = 0.f, db1 = 0.f;
#pragma unroll 8
        for (int s = 0; s < SPW; ++s) {
            dw1 = fmaf(L.g1[s * RS + j], L.u[s], dw1);
            db1 += L.g1[s * RS + j];
        }
        L.g[OW1 + j] = dw1;
        L.g[OB1 + j] = db1;
    }
    __syncthreads();
}

}  // namespace

// ---------------------------------------------------------------------------
// initialisation: He-normal hidden weights (N(0, 2/fan_in)) from the seed;
// the first layer's biases put unit j's ReLU kink at u = (j + 0.5) / 64,
// spreading the kinks over the input range [0, 1] instead of stacking them all
// at 0 (a 1-D input otherwise gives a network that starts out linear on
// (0, 1]); the output layer starts at zero, so an untrained network predicts
// exactly 0 (the learned path fits a correction to the linear CDF)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float he_normal(uint64_t seed, int p, float sd)
{
    const uint64_t a = mix64(seed ^ (0x9E3779B97F4A7C15ull * (uint64_t)(2 * p + 1)));
    const uint64_t b = mix64(a ^ 0xD1B54A32D192ED03ull);
    const double u1 = ((double)(a >> 11) + 1.0) * (1.0 / 9007199254740992.0);   // (0, 1]
    const double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
    return (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2)) * sd;
}

__global__ void mlp_init_kernel(float *params, uint64_t seed)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    float v = 0.f;
    if (p < OB1) v = he_normal(seed, p, sqrtf(2.f));                        // W1, fan_in 1
    else if (p < OW2) {
        const int j = p - OB1;
        v = -he_normal(seed, OW1 + j, sqrtf(2.f)) * ((float)j + 0.5f) / (float)HID;
    } else if (p < OB2) v = he_normal(seed, p, sqrtf(2.f / HID));
    params[p] = v;
}

// ---------------------------------------------------------------------------
// training: two ordinary launches per step
// ---------------------------------------------------------------------------
// Step part 1, nwg work-groups of TR_NT threads (batch = nwg * 32): every
// work-group's partial gradient and loss of its 32 samples.  If full_batch,
// the samples are the first `batch` in order, else 32 per group are drawn
// (with replacement) by a counter-based hash of (seed, step, slot).
__global__ __launch_bounds__(TR_NT) void mlp_step_grad_kernel(const float *params, const float *su,
                                                              const float *st, int64_t S, int step,
                                                              uint64_t seed, int full_batch, float *partial,
                                                              const unsigned *gate)
{
    __shared__ TrainLds L;
    if (gate && *gate) return;
    const int wg = blockIdx.x, tid = threadIdx.x;
    const int batch = (int)gridDim.x * SPW;
    for (int k = tid; k < kMlpParams; k += TR_NT) L.p[k] = params[k];
    if (tid < SPW) {
        const int slot = wg * SPW + tid;
        int64_t idx;
        if (full_batch) idx = slot < S ? slot : S - 1;
        else idx = (int64_t)(mix64(seed ^ ((uint64_t)(step + 1) << 32) ^ (uint64_t)slot) % (uint64_t)S);
        L.u[tid] = su[idx];
        L.t[tid] = st[idx];
    }
    __syncthreads();
    wg_loss_grad(L, 1.f / (float)batch);
    float *pw = partial + (size_t)wg * (kMlpParams + 1);
    for (int k = tid; k < kMlpParams; k += TR_NT) pw[k] = L.g[k];
    if (tid == 0) pw[kMlpParams] = L.loss;
}

// Step part 2: every work-group sums a 64-parameter slice of the gradient
// over the nwg partials -- lane k of quarter q sums the partials of groups
// [q*nq, (q+1)*nq) in group order, then the four quarter sums are added in
// quarter order (a fixed order, so a run is bit reproducible) -- and applies
// Adam (Kingma & Ba) to it.  Work-group 0 also records the mean loss of the
// first and the last step.
__global__ __launch_bounds__(TR_NT) void mlp_step_adam_kernel(float *params, float *adam_m, float *adam_v,
                                                              const float *partial, int nwg, int step, int steps,
                                                              float lr, float *losses, const unsigned *gate)
{
    __shared__ float red[TR_NT / 64][64];
    if (gate && *gate) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)(step + 1));
    const float c2 = 1.f - powf(b2, (float)(step + 1));
    const int tid = threadIdx.x, q = tid >> 6, kl = tid & 63;
    const int nq = (nwg + 3) / 4;
    const int w0 = q * nq, w1 = min(w0 + nq, nwg);
    const int k = blockIdx.x * 64 + kl;
    float g = 0.f;
    if (k < kMlpParams) {
        int w = w0;
        for (; w + 8 <= w1; w += 8) {
            float v8[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) v8[r] = partial[(size_t)(w + r) * (kMlpParams + 1) + k];
#pragma unroll
            for (int r = 0; r < 8; ++r) g += v8[r];
        }
        for (; w < w1; ++w) g += partial[(size_t)w * (kMlpParams + 1) + k];
    }
    red[q][kl] = g;
    __syncthreads();
    if (q == 0 && k < kMlpParams) {
        const float gs = ((red[0][kl] + red[1][kl]) + red[2][kl]) + red[3][kl];
        const float m = b1 * adam_m[k] + (1.f - b1) * gs;
        const float v = b2 * adam_v[k] + (1.f - b2) * gs * gs;
        adam_m[k] = m;
        adam_v[k] = v;
        params[k] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
    }
    if (blockIdx.x == 0 && tid == 0 && losses && (step == 0 || step == steps - 1)) {
        float l = 0.f;
        for (int w = 0; w < nwg; ++w) l += partial[(size_t)w * (kMlpParams + 1) + kMlpParams];
        l /= (float)(nwg * SPW);
        losses[step == 0 ? 0 : 1] = l;
        if (steps == 1) losses[1] = l;
    }
}

// Loss and gradient of one batch (test hook and building block): same code as
// training; nwg = batch / 32 groups, then an ordered reduction.
__global__ __launch_bounds__(TR_NT) void mlp_grad_partial_kernel(const float *params, const float *u,
                                                                 const float *t, int batch,
                                                                 float *partial)
{
    __shared__ TrainLds L;
    const int wg = blockIdx.x, tid = threadIdx.x;
    for (int k = tid; k < kMlpParams; k += TR_NT) L.p[k] = params[k];
    if (tid < SPW) {
        L.u[tid] = u[wg * SPW + tid];
        L.t[tid] = t[wg * SPW + tid];
    }
    __syncthreads();
    wg_loss_grad(L, 1.f / (float)batch);
    float *pw = partial + (size_t)wg * (kMlpParams + 1);
    for (int k = tid; k < kMlpParams; k += TR_NT) pw[k] = L.g[k];
    if (tid == 0) pw[kMlpParams] = L.loss;
}

__global__ void mlp_grad_reduce_kernel(const float *partial, int nwg, int batch, float *grad, float *loss)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > kMlpParams) return;
    float g = 0.f;
    for (int w = 0; w < nwg; ++w) g += partial[(size_t)w * (kMlpParams + 1) + k];
    if (k < kMlpParams) grad[k] = g;
    else *loss = g / (float)batch;
}

// ---------------------------------------------------------------------------
// network evaluation (knot table and test hook)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float mlp_eval(const float *p, float u)
{
    float h1[HID];
#pragma unroll
    for (int j = 0; j < HID; ++j) {
        const float z = fmaf(p[OW1 + j], u, p[OB1 + j]);
        h1[j] = z > 0.f ? z : 0.f;
    }
    float y = p[OB3];
    for (int i = 0; i < HID; ++i) {
        float a = p[OB2 + i];
#pragma unroll
        for (int j = 0; j < HID; ++j) a = fmaf(p[OW2 + i * HID + j], h1[j], a);
        y = fmaf(p[OW3 + i], a > 0.f ? a : 0.f, y);
    }
    return y;
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *params, const float *u, int64_t count,
                                                          float *y, int64_t knots, const unsigned *gate)
{
    __shared__ float p[kMlpParams];
    if (gate && *gate) return;
    for (int k = threadIdx.x; k < kMlpParams; k += blockDim.x) p[k] = params[k];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    // knots > 0: evaluate at u = i / knots; else at the given inputs
    const float x = knots > 0 ? (float)((double)i / (double)knots) : u[i];
    y[i] = mlp_eval(p, x);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t mlp_init(float *params, uint64_t seed, hipStream_t st)
{
    hipLaunchKernelGGL(mlp_init_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, params, seed);
    return hipGetLastError();
}

hipError_t mlp_train(float *params, float *m, float *v, const float *su, const float *stgt, int64_t S,
                     int steps, int batch, float lr, uint64_t seed, int full_batch, float *partial,
                     float *losses, const unsigned *gate, hipStream_t st)
{
    const int nwg = batch / SPW;
    for (int step = 0; step < steps; ++step) {
        hipLaunchKernelGGL(mlp_step_grad_kernel, dim3(nwg), dim3(TR_NT), 0, st, (const float *)params, su, stgt, S,
                           step, seed, full_batch, partial, gate);
        hipLaunchKernelGGL(mlp_step_adam_kernel, dim3((kMlpParams + 63) / 64), dim3(TR_NT), 0, st, params, m, v,
                           (const float *)partial, nwg, step, steps, lr, losses, gate);
    }
    return hipGetLastError();
}

hipError_t mlp_loss_grad(const float *params, const float *u, const float *t, int batch, float *partial,
                         float *grad, float *loss, hipStream_t st)
{
    const int nwg = batch / SPW;
    hipLaunchKernelGGL(mlp_grad_partial_kernel, dim3(nwg), dim3(TR_NT), 0, st, params, u, t, batch, partial);
    hipLaunchKernelGGL(mlp_grad_reduce_kernel, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, st,
                       (const float *)partial, nwg, batch, grad, loss);
    return hipGetLastError();
}

hipError_t mlp_forward(const float *params, const float *u, int64_t count, float *y, int64_t knots,
                       const unsigned *gate, hipStream_t st)
{
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, params, u,
                       count, y, knots, gate);
    return hipGetLastError();
}

int mlp_samples_per_group() { return SPW; }

}  // namespace gs
