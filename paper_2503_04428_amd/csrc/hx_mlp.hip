// Learned slope limiter: standalone BF16-MFMA inference, training-sample extraction from fine
// FP64 solutions, and the FP32 training kernels (forward + backward + Adam).
#include <hip/hip_runtime.h>

#include <mutex>

#include "hx_launch.h"
#include "hx_mlp.h"

namespace hx {

// ---------------------------------------------------------------------------- inference

// phi for n normalised stencils x[n][4]; one wave per 16-stencil tile (grid-stride)
__global__ void __launch_bounds__(256) mlp_eval_kernel(const float* __restrict__ w, const float* __restrict__ x,
                                                       long long n, float* __restrict__ phi)
{
    const int lane = threadIdx.x & 63;
    MlpLane m;
    mlp_load(w, lane, m);
    const long long ntile = (n + 15) / 16;
    const long long wave = (long long)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const long long nwave = (long long)gridDim.x * (blockDim.x / 64);
    for (long long t = wave; t < ntile; t += nwave) {
        const long long e = t * 16 + (lane & 15);
        bf16x4_t xb = {0, 0, 0, 0};
        if (lane < 16 && e < n)
            xb = pack_x(x[4 * e], x[4 * e + 1], x[4 * e + 2], x[4 * e + 3]);
        const float p = mlp_tile(m, xb);
        if (lane < 16 && e < n)
            phi[e] = p;
    }
}

// ---------------------------------------------------------------------------- training samples

// One sample per (row, coarse cell, primitive) of a batch of 1D FP64 solutions on fine grids of
// nf cells (layout [5][nrows][nf]).  Coarse conserved states are averages of `ratio` fine cells;
// the input stencil is the four undivided differences of the coarse primitive around the cell,
// normalised by their largest magnitude; the label is the least-squares slope of the fine
// primitive values inside the coarse cell, times the coarse width.  Samples where the TVD
// region forces a zero slope (or too close to the row ends) get weight 0.
__device__ __forceinline__ void coarse_prim(const double* __restrict__ U, long long plane, long long row_off,
                                            int ratio, int i, double gm1, double* w)
{
    double q[5] = {0, 0, 0, 0, 0};
    for (int f = 0; f < ratio; f++)
#pragma unroll
        for (int v = 0; v < 5; v++)
            q[v] += U[v * plane + row_off + (long long)i * ratio + f];
#pragma unroll
    for (int v = 0; v < 5; v++)
        q[v] = q[v] / ratio;
    const double inv = 1.0 / q[0];
    w[0] = q[0];
    w[1] = q[1] * inv;
    w[2] = q[2] * inv;
    w[3] = q[3] * inv;
    w[4] = gm1 * (q[4] - 0.5 * (q[1] * w[1] + q[2] * w[2] + q[3] * w[3]));
}

__global__ void __launch_bounds__(256) mlp_features_kernel(const double* __restrict__ U, int nrows, int nf,
                                                           int ratio, double gamma, float* __restrict__ xo,
                                                           float* __restrict__ ao, float* __restrict__ to,
                                                           float* __restrict__ wo)
{
    const int nc = nf / ratio;
    const long long total = (long long)nrows * nc;
    const long long plane = (long long)nrows * nf;
    const double gm1 = gamma - 1.0;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < total;
         c += (long long)gridDim.x * blockDim.x) {
        const int row = (int)(c / nc), i = (int)(c % nc);
        const long long row_off = (long long)row * nf;
        double W[5][5];  // coarse primitives of cells i-2..i+2
        const bool inside = i >= 2 && i <= nc - 3;
        if (inside)
            for (int s = 0; s < 5; s++)
                coarse_prim(U, plane, row_off, ratio, i - 2 + s, gm1, W[s]);
        for (int v = 0; v < 5; v++) {
            const long long e = c * 5 + v;
            float xv[4] = {0, 0, 0, 0}, a = 0, t = 0, wt = 0;
            if (inside) {
                const double d[4] = {W[1][v] - W[0][v], W[2][v] - W[1][v], W[3][v] - W[2][v], W[4][v] - W[3][v]};
                double s = 0.0;
                for (int k = 0; k < 4; k++)
                    s = fmax(s, fabs(d[k]));
                if (d[1] * d[2] > 0.0 && s > 0.0) {
                    // least-squares slope of the fine primitive values across the coarse cell
                    double num = 0.0, den = 0.0;
                    const double mid = 0.5 * (ratio - 1);
                    for (int f = 0; f < ratio; f++) {
                        double q[5];
#pragma unroll
                        for (int u = 0; u < 5; u++)
                            q[u] = U[u * plane + row_off + (long long)i * ratio + f];
                        const double inv = 1.0 / q[0];
                        double wf;
                        if (v == 0)
                            wf = q[0];
                        else if (v < 4)
                            wf = q[v] * inv;
                        else
                            wf = gm1 * (q[4] - 0.5 * (q[1] * (q[1] * inv) + q[2] * (q[2] * inv) + q[3] * (q[3] * inv)));
                        num += (f - mid) * wf;
                        den += (f - mid) * (f - mid);
                    }
                    const double slope = ratio * num / den;
                    for (int k = 0; k < 4; k++)
                        xv[k] = (float)(d[k] / s);
                    a = (float)(d[1] / s);
                    t = (float)(slope / s);
                    wt = 1.0f;
                }
            }
            xo[4 * e] = xv[0];
            xo[4 * e + 1] = xv[1];
            xo[4 * e + 2] = xv[2];
            xo[4 * e + 3] = xv[3];
            ao[e] = a;
            to[e] = t;
            wo[e] = wt;
        }
    }
}

// ---------------------------------------------------------------------------- training

// tanh-form GELU and its derivative, the value in the deployed form z s with s = 1 / (1 + 2^(z (G1 +
// G3 z^2))) (gelu_f of the fused evaluation, the same operations); the derivative of z s(y(z)),
// y = 2 k (z + 0.044715 z^3), is s + z s (1 - s) y'(z)
__device__ __forceinline__ float gelu_train(float z, float& dg)
{
    constexpr float G1 = (float)(-2.0 * 0.7978845608028654 * 1.4426950408889634);
    constexpr float G3 = (float)(-2.0 * 0.7978845608028654 * 0.044715 * 1.4426950408889634);
    const float sg = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z * (G1 + G3 * z * z)));
    const float k = 0.7978845608028654f;
    dg = sg + z * sg * (1.0f - sg) * (2.0f * k) * (1.0f + 3.0f * 0.044715f * z * z);
    return z * sg;
}

__device__ __forceinline__ float wave_sum_f(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int GB = 256;  // threads per gradient block
constexpr int GW = GB / 64;  // waves per gradient block

// Per-sample FP32 forward/backward of L = sum wt (phi a - t)^2 (unnormalised), with FP32 parameters
// and activations and the GELU and output sigmoid in the forms the fused BF16 evaluation uses
// (exp2 and reciprocal); the BF16 roundings of the deployed network are left out of training (the
// deployed loss on the training samples is measured beside the FP32 one); per-block sums of
// the 1249 gradients, of the loss and of the weights go to part[block][1251].  Every wave adds its
// wave sums into its own LDS row (one lane writes, so each row is summed in sample order), and the
// rows are added in wave order at the end: the result does not depend on wave timing.
__global__ void __launch_bounds__(GB) mlp_grad_kernel(const float* __restrict__ w, const float* __restrict__ x,
                                                      const float* __restrict__ a, const float* __restrict__ t,
                                                      const float* __restrict__ wt, long long n,
                                                      float* __restrict__ part)
{
    __shared__ float sw[MLP_NPARAM];
    __shared__ float sg[GW][MLP_NPARAM + 2];
    for (int i = threadIdx.x; i < MLP_NPARAM; i += GB)
        sw[i] = w[i];
    for (int i = threadIdx.x; i < GW * (MLP_NPARAM + 2); i += GB)
        sg[i / (MLP_NPARAM + 2)][i % (MLP_NPARAM + 2)] = 0.0f;
    __syncthreads();
    const float* W1 = sw + MLP_W1;
    const float* b1 = sw + MLP_B1;
    const float* W2 = sw + MLP_W2;
    const float* b2 = sw + MLP_B2;
    const float* w3 = sw + MLP_W3;
    const float b3 = sw[MLP_B3];
    const bool lane0 = (threadIdx.x & 63) == 0;
    float* row = sg[threadIdx.x >> 6];

    for (long long base = (long long)blockIdx.x * GB; base < n; base += (long long)gridDim.x * GB) {
        const long long e = base + threadIdx.x;
        const bool live = e < n;
        float xi[4] = {0, 0, 0, 0}, ae = 0, te = 0, we = 0;
        if (live) {
            xi[0] = x[4 * e];
            xi[1] = x[4 * e + 1];
            xi[2] = x[4 * e + 2];
            xi[3] = x[4 * e + 3];
            ae = a[e];
            te = t[e];
            we = wt[e];
        }
        float h1[32], g1[32], h2[32], g2[32];
        for (int o = 0; o < 32; o++) {
            float s = b1[o];
            for (int i = 0; i < 4; i++)
                s += W1[o * 4 + i] * xi[i];
            h1[o] = gelu_train(s, g1[o]);
        }
        for (int o = 0; o < 32; o++) {
            float s = b2[o];
            for (int i = 0; i < 32; i++)
                s += W2[o * 32 + i] * h1[i];
            h2[o] = gelu_train(s, g2[o]);
        }
        float z = b3;
        for (int i = 0; i < 32; i++)
            z += w3[i] * h2[i];
        const float phi = 2.0f * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
        const float err = phi * ae - te;
        const float loss = we * err * err;
        const float dz = 2.0f * we * err * ae * phi * (1.0f - 0.5f * phi);
        // wave sums, added by lane 0 into the wave's own row
        float r = wave_sum_f(loss);
        if (lane0)
            row[MLP_NPARAM] += r;
        r = wave_sum_f(we);
        if (lane0)
            row[MLP_NPARAM + 1] += r;
        r = wave_sum_f(dz);
        if (lane0)
            row[MLP_B3] += r;
        float d2[32];
        for (int o = 0; o < 32; o++) {
            r = wave_sum_f(dz * h2[o]);
            if (lane0)
                row[MLP_W3 + o] += r;
            d2[o] = dz * w3[o] * g2[o];
        }
        for (int o = 0; o < 32; o++) {
            r = wave_sum_f(d2[o]);
            if (lane0)
                row[MLP_B2 + o] += r;
            for (int i = 0; i < 32; i++) {
                r = wave_sum_f(d2[o] * h1[i]);
                if (lane0)
                    row[MLP_W2 + o * 32 + i] += r;
            }
        }
        for (int i = 0; i < 32; i++) {
            float dh = 0.0f;
            for (int o = 0; o < 32; o++)
                dh += W2[o * 32 + i] * d2[o];
            const float d1 = dh * g1[i];
            r = wave_sum_f(d1);
            if (lane0)
                row[MLP_B1 + i] += r;
            for (int k = 0; k < 4; k++) {
                r = wave_sum_f(d1 * xi[k]);
                if (lane0)
                    row[MLP_W1 + i * 4 + k] += r;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < MLP_NPARAM + 2; i += GB) {
        float s = sg[0][i];
        for (int v = 1; v < GW; v++)
            s += sg[v][i];
        part[(long long)blockIdx.x * (MLP_NPARAM + 2) + i] = s;
    }
}

// fixed-order sum of the block partials; grad = sum / sum(wt), loss = sum / sum(wt)
__global__ void __launch_bounds__(256) mlp_grad_final_kernel(const float* __restrict__ part, int nb,
                                                             float* __restrict__ grad, float* __restrict__ loss)
{
    __shared__ float wsum;
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int b = 0; b < nb; b++)
            s += part[(long long)b * (MLP_NPARAM + 2) + MLP_NPARAM + 1];
        wsum = s;
    }
    __syncthreads();
    const float inv = wsum > 0.0f ? 1.0f / wsum : 0.0f;
    for (int i = threadIdx.x; i < MLP_NPARAM + 1; i += blockDim.x) {
        float s = 0.0f;
        for (int b = 0; b < nb; b++)
            s += part[(long long)b * (MLP_NPARAM + 2) + i];
        if (i < MLP_NPARAM)
            grad[i] = s * inv;
        else
            loss[0] = s * inv;
    }
}

__global__ void mlp_adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, int step, float lr, float b1, float b2, float eps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MLP_NPARAM)
        return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - powf(b1, (float)step));
    const float vh = vi / (1.0f - powf(b2, (float)step));
    w[i] -= lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------- launchers

hipError_t launch_mlp_eval(const float* w, const float* x, long long n, float* phi, hipStream_t s)
{
    const long long ntile = (n + 15) / 16;
    long long nb = (ntile + 3) / 4;
    if (nb > 4096)
        nb = 4096;
    if (nb < 1)
        nb = 1;
    mlp_eval_kernel<<<(int)nb, 256, 0, s>>>(w, x, n, phi);
    return hipGetLastError();
}

hipError_t launch_mlp_features(const double* U, int nrows, int nf, int ratio, double gamma, float* x, float* a,
                               float* t, float* wt, hipStream_t s)
{
    const long long total = (long long)nrows * (nf / ratio);
    long long nb = (total + 255) / 256;
    if (nb > 8192)
        nb = 8192;
    if (nb < 1)
        nb = 1;
    mlp_features_kernel<<<(int)nb, 256, 0, s>>>(U, nrows, nf, ratio, gamma, x, a, t, wt);
    return hipGetLastError();
}

constexpr int MLP_GRAD_MAX_BLOCKS = 1024;  // largest grid of mlp_grad_kernel

int mlp_grad_blocks(long long n)
{
    long long nb = (n + GB - 1) / GB;
    return (int)(nb > MLP_GRAD_MAX_BLOCKS ? MLP_GRAD_MAX_BLOCKS : (nb < 1 ? 1 : nb));
}

hipError_t launch_mlp_grad(const float* w, const float* x, const float* a, const float* t, const float* wt,
                           long long n, float* grad, float* loss, float* part, hipStream_t s)
{
    const int nb = mlp_grad_blocks(n);
    mlp_grad_kernel<<<nb, GB, 0, s>>>(w, x, a, t, wt, n, part);
    mlp_grad_final_kernel<<<1, 256, 0, s>>>(part, nb, grad, loss);
    return hipGetLastError();
}

// Scratch of the allocation-free gradient entry point: the block partials of the largest grid
// mlp_grad_kernel is launched with (1024 x 1251 floats, 5.1 MB).  Every device the library runs
// on holds its own copy until the process ends; calls on one device share it.
static __device__ __align__(256) float scratch[MLP_GRAD_MAX_BLOCKS * (MLP_NPARAM + 2)];

constexpr int MLP_SCRATCH_MAX_DEVICES = 64;

// Device address of this device's copy of the scratch array, looked up once per device (the
// array's name in host code is only a stand-in for the symbol, not a device address).
static hipError_t scratch_address(float** ptr)
{
    static std::mutex mu;
    static float* addr[MLP_SCRATCH_MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= MLP_SCRATCH_MAX_DEVICES)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        addr[dev] = static_cast<float*>(p);
    }
    *ptr = addr[dev];
    return hipSuccess;
}

size_t mlp_grad_scratch_bytes() { return sizeof(scratch); }

hipError_t launch_mlp_grad_noalloc(const float* w, const float* x, const float* a, const float* t, const float* wt,
                                   long long n, float* grad, float* loss, hipStream_t s)
{
    if (sizeof(float) * (size_t)mlp_grad_blocks(n) * (MLP_NPARAM + 2) > sizeof(scratch))
        return hipErrorInvalidValue;  // cannot happen while the grid is capped at the array's rows
    float* part = nullptr;
    const hipError_t e = scratch_address(&part);
    if (e != hipSuccess)
        return e;
    return launch_mlp_grad(w, x, a, t, wt, n, grad, loss, part, s);
}

hipError_t launch_mlp_adam(float* w, const float* g, float* m, float* v, int step, float lr, float b1, float b2,
                           float eps, hipStream_t s)
{
    mlp_adam_kernel<<<(MLP_NPARAM + 255) / 256, 256, 0, s>>>(w, g, m, v, step, lr, b1, b2, eps);
    return hipGetLastError();
}

}  // namespace hx
