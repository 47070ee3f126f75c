// Kernels compiled ahead of time into the library (no expression inside):
// the streaming copy used as the bandwidth ceiling, and the cost-model MLP
// (forward, backward, Adam).  FP32, plain vector ALU: the MLP is 32-64-64 and
// far too small for matrix cores to matter.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "coot.h"

namespace {

typedef unsigned int u32;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// dst[i] = src[i] in 16-byte units: one pass, 4 vectors per thread, streaming
// (nontemporal) loads and stores like the fused kernels; the byte tail is done
// by the last block.  It is the plain-copy ceiling the fused kernels are
// measured against, and the known-size kernel the HBM byte counters are
// calibrated on.
__global__ void __launch_bounds__(256) coot_copy16(u32x4* __restrict__ dst, const u32x4* __restrict__ src, int64_t nv,
                                                   unsigned char* __restrict__ dtail,
                                                   const unsigned char* __restrict__ stail, int64_t ntail)
{
    const int64_t step = (int64_t)gridDim.x * blockDim.x * 4;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x * 4 + threadIdx.x; b < nv; b += step) {
        u32x4 r[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int64_t v = b + (int64_t)e * blockDim.x;
            if (v < nv) r[e] = __builtin_nontemporal_load(src + v);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int64_t v = b + (int64_t)e * blockDim.x;
            if (v < nv) __builtin_nontemporal_store(r[e], dst + v);
        }
    }
    if (blockIdx.x == gridDim.x - 1)
        for (int64_t i = threadIdx.x; i < ntail; i += blockDim.x) dtail[i] = stail[i];
}

// Streaming probes with a given read/write mix, nontemporal, one pass, EPT
// vectors of 16 bytes per thread (the launch shapes of the fused
// element-wise kernels).  KIND 0 copies.  KIND 1 reads only: the loads are
// folded into a per-thread XOR that is stored only if all its bits are set
// (the loads cannot be dropped; random data never stores).  KIND 2 writes
// only.  KIND 3 reads two streams and writes one (dst = a XOR b), the mix of
// a two-operand element-wise tree.
template <int KIND, int EPT>
__global__ void __launch_bounds__(256) coot_probe16(u32x4* __restrict__ dst, const u32x4* __restrict__ src, int64_t nv)
{
    const int64_t step = (int64_t)gridDim.x * blockDim.x * EPT;
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x * EPT + threadIdx.x; b < nv; b += step) {
        u32x4 r[EPT], q[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t v = b + (int64_t)e * blockDim.x;
            if (v < nv) {
                if (KIND != 2) r[e] = __builtin_nontemporal_load(src + v);
                if (KIND == 3) q[e] = __builtin_nontemporal_load(src + nv + v);
            }
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t v = b + (int64_t)e * blockDim.x;
            if (v < nv) {
                if (KIND == 0) __builtin_nontemporal_store(r[e], dst + v);
                if (KIND == 1) acc ^= r[e];
                if (KIND == 2) __builtin_nontemporal_store(u32x4{(u32)v, 0u, 0u, 0u}, dst + v);
                if (KIND == 3) __builtin_nontemporal_store(r[e] ^ q[e], dst + v);
            }
        }
    }
    if (KIND == 1 && (acc.x & acc.y & acc.z & acc.w) == 0xffffffffu) dst[0] = acc;
}

template <int KIND>
void probe_shape(int shape, int64_t nv, u32x4* d, const u32x4* sv, hipStream_t st)
{
    // (vectors per thread, threads per block) of shapes 0..3
    static const int ept[4] = {4, 1, 1, 2}, blk[4] = {256, 64, 256, 128};
    const int64_t per = (int64_t)ept[shape] * blk[shape];
    int64_t grid = (nv + per - 1) / per;
    if (grid > INT64_C(0x7fffffff)) grid = INT64_C(0x7fffffff);
    if (grid < 1) grid = 1;
    const dim3 g((unsigned)grid), b((unsigned)blk[shape]);
    switch (shape) {
    case 0: hipLaunchKernelGGL((coot_probe16<KIND, 4>), g, b, 0, st, d, sv, nv); break;
    case 1: hipLaunchKernelGGL((coot_probe16<KIND, 1>), g, b, 0, st, d, sv, nv); break;
    case 2: hipLaunchKernelGGL((coot_probe16<KIND, 1>), g, b, 0, st, d, sv, nv); break;
    default: hipLaunchKernelGGL((coot_probe16<KIND, 2>), g, b, 0, st, d, sv, nv); break;
    }
}

// Tiled probes: each stream a column-major matrix of 16384 rows of 4-byte
// elements and `cols` columns (a multiple of 64), moved in tiles of 2^LR rows
// x 2^(12-LR) columns, a block per tile (grid-stride); wave w's step kk
// covers tile elements 64*(w + 4*kk) + [0, 64) in column order, so a wave
// access is 64 consecutive rows.  KIND 0 copies, KIND 3 writes a XOR b.
template <int KIND, int LR>
__global__ void __launch_bounds__(256) coot_probe_tiled(u32* __restrict__ dst, const u32* __restrict__ src, int64_t cols)
{
    constexpr int LC = 12 - LR, MASK = (1 << LR) - 1;
    constexpr int64_t N = 16384;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t tr = N >> LR, nt = tr * (cols >> LC), second = N * cols;
    for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        const int64_t i0 = (t % tr) << LR, j0 = (t / tr) << LC;
        u32 v[16];
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const int e = 64 * (w + 4 * kk);
            const int64_t off = i0 + (e & MASK) + lane + (j0 + (e >> LR)) * N;
            v[kk] = __builtin_nontemporal_load(src + off);
            if (KIND == 3) v[kk] ^= __builtin_nontemporal_load(src + second + off);
        }
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const int e = 64 * (w + 4 * kk);
            __builtin_nontemporal_store(v[kk], dst + (i0 + (e & MASK) + lane + (j0 + (e >> LR)) * N));
        }
    }
}

template <int KIND>
void probe_tiled(int shape, int64_t bytes, void* d, const void* s, int grid_cap, hipStream_t st)
{
    const int64_t cols = bytes / (16384 * 4), tiles = cols * 4;   // 4096-element tiles
    const dim3 g((unsigned)(tiles < grid_cap ? tiles : grid_cap)), b(256);
    u32* dd = (u32*)d;
    const u32* ss = (const u32*)s;
    switch (shape) {
    case 0: hipLaunchKernelGGL((coot_probe_tiled<KIND, 6>), g, b, 0, st, dd, ss, cols); break;
    case 1: hipLaunchKernelGGL((coot_probe_tiled<KIND, 8>), g, b, 0, st, dd, ss, cols); break;
    case 2: hipLaunchKernelGGL((coot_probe_tiled<KIND, 10>), g, b, 0, st, dd, ss, cols); break;
    default: hipLaunchKernelGGL((coot_probe_tiled<KIND, 12>), g, b, 0, st, dd, ss, cols); break;
    }
}

}  // namespace

namespace {

// ---- MLP 32 -> 64 (ReLU) -> 64 -----------------------------------------------
// params: W1[32][64] b1[64] W2[64][64] b2[64]; row-major, W[i][j] input i -> output j.
constexpr int NI = COOT_MLP_IN, NH = COOT_MLP_HID, NO = COOT_MLP_OUT;
constexpr int OFF_B1 = NI * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NO;

// one block of 64 threads per sample: thread j computes hidden unit j, then output j
__global__ void __launch_bounds__(64) mlp_fwd(const float* __restrict__ P, const float* __restrict__ X, int B,
                                              float* __restrict__ Y, float* __restrict__ Z1, float* __restrict__ H)
{
    __shared__ float xs[NI];
    __shared__ float hs[NH];
    const int j = threadIdx.x;
    for (int s = blockIdx.x; s < B; s += gridDim.x) {
        if (j < NI) xs[j] = X[(int64_t)s * NI + j];
        __syncthreads();
        float z = P[OFF_B1 + j];
        for (int i = 0; i < NI; ++i) z += xs[i] * P[i * NH + j];
        float h = z > 0.0f ? z : 0.0f;
        if (Z1) Z1[(int64_t)s * NH + j] = z;
        if (H) H[(int64_t)s * NH + j] = h;
        hs[j] = h;
        __syncthreads();
        float y = P[OFF_B2 + j];
        for (int i = 0; i < NH; ++i) y += hs[i] * P[OFF_W2 + i * NO + j];
        Y[(int64_t)s * NO + j] = y;
        __syncthreads();
    }
}

// dY = 2 M (Y - T) / sum(M); dZ1 = (dY W2^T) * (Z1 > 0).  One block per sample.
__global__ void __launch_bounds__(64) mlp_bwd_rows(const float* __restrict__ P, const float* __restrict__ Y,
                                                   const float* __restrict__ T, const float* __restrict__ M, int B,
                                                   const float* __restrict__ Z1, const float* __restrict__ msum,
                                                   float* __restrict__ dY, float* __restrict__ dZ1)
{
    __shared__ float dys[NO];
    const int j = threadIdx.x;
    const float inv = 1.0f / msum[0];
    for (int s = blockIdx.x; s < B; s += gridDim.x) {
        int64_t o = (int64_t)s * NO + j;
        float d = 2.0f * M[o] * (Y[o] - T[o]) * inv;
        dY[o] = d;
        dys[j] = d;
        __syncthreads();
        float g = 0.0f;
        for (int k = 0; k < NO; ++k) g += dys[k] * P[OFF_W2 + j * NO + k];
        dZ1[(int64_t)s * NH + j] = Z1[(int64_t)s * NH + j] > 0.0f ? g : 0.0f;
        __syncthreads();
    }
}

// sum of the mask and the masked squared error, fixed order (one block)
__global__ void __launch_bounds__(256) mlp_loss(const float* __restrict__ Y, const float* __restrict__ T,
                                                const float* __restrict__ M, int64_t n, float* __restrict__ out)
{
    __shared__ double sm[256], se[256];
    double a = 0.0, e = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double d = (double)Y[i] - (double)T[i];
        a += M[i];
        e += (double)M[i] * d * d;
    }
    sm[threadIdx.x] = a;
    se[threadIdx.x] = e;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sm[threadIdx.x] += sm[threadIdx.x + s];
            se[threadIdx.x] += se[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = (float)sm[0];
        out[1] = (float)(sm[0] > 0 ? se[0] / sm[0] : 0.0);
    }
}

// Weight gradients: G[i][j] = sum_s A[s][i] * D[s][j] (one thread per (i, j),
// samples in a fixed order) and bias gradients gb[j] = sum_s D[s][j].
__global__ void __launch_bounds__(64) mlp_wgrad(const float* __restrict__ A, int na, const float* __restrict__ D, int nd,
                                                int B, float* __restrict__ G, float* __restrict__ gb)
{
    const int i = blockIdx.x, j = threadIdx.x;
    if (j >= nd) return;
    if (i < na) {
        float acc = 0.0f;
        for (int s = 0; s < B; ++s) acc += A[(int64_t)s * na + i] * D[(int64_t)s * nd + j];
        G[i * nd + j] = acc;
    } else {
        float acc = 0.0f;
        for (int s = 0; s < B; ++s) acc += D[(int64_t)s * nd + j];
        gb[j] = acc;
    }
}

__global__ void __launch_bounds__(256) mlp_adam(float* __restrict__ w, const float* __restrict__ g,
                                                float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                                float b1, float b2, float eps, float c1, float c2)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float mh = mi / c1, vh = vi / c2;
    w[i] -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace

extern "C" {

int coot_copy_launch(void* dst, const void* src, int64_t bytes, int cus, void* stream)
{
    int64_t nv = bytes / 16;
    int64_t tail = bytes - nv * 16;
    // one pass: a block per 1024 vectors (the grid-stride loop only runs
    // again beyond 2^31 - 1 blocks)
    (void)cus;
    int64_t need = (nv + 1023) / 1024;
    int64_t grid = need < INT64_C(0x7fffffff) ? need : INT64_C(0x7fffffff);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(coot_copy16, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, (u32x4*)dst,
                       (const u32x4*)src, nv, (unsigned char*)dst + nv * 16, (const unsigned char*)src + nv * 16, tail);
    return hipGetLastError() == hipSuccess ? 0 : -8;
}

int coot_probe_launch(int kind, int shape, void* dst, const void* src, int64_t bytes, void* stream)
{
    const int64_t nv = bytes / 16;
    u32x4* d = (u32x4*)dst;
    const u32x4* sv = (const u32x4*)src;
    hipStream_t st = (hipStream_t)stream;
    if (shape < 0 || shape > 3) return -10;
    switch (kind) {
    case COOT_PROBE_COPY: probe_shape<0>(shape, nv, d, sv, st); break;
    case COOT_PROBE_READ: probe_shape<1>(shape, nv, d, sv, st); break;
    case COOT_PROBE_WRITE: probe_shape<2>(shape, nv, d, sv, st); break;
    case COOT_PROBE_READ2_WRITE1: probe_shape<3>(shape, nv, d, sv, st); break;
    case COOT_PROBE_TILED_COPY: probe_tiled<0>(shape, bytes, dst, src, 16384, st); break;
    case COOT_PROBE_TILED_READ2_WRITE1: probe_tiled<3>(shape, bytes, dst, src, 16384, st); break;
    default: return -10;
    }
    return hipGetLastError() == hipSuccess ? 0 : -8;
}

int coot_mlp_forward_launch(const float* P, const float* X, int B, float* Y, float* Z1, float* H, void* stream)
{
    int grid = B < 4096 ? B : 4096;
    if (grid < 1) return 0;
    hipLaunchKernelGGL(mlp_fwd, dim3(grid), dim3(64), 0, (hipStream_t)stream, P, X, B, Y, Z1, H);
    return hipGetLastError() == hipSuccess ? 0 : -8;
}

int coot_mlp_backward_launch(const float* P, const float* X, const float* T, const float* M, int B, float* grad,
                             float* loss, float* ws, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    float* Y = ws;
    float* Z1 = Y + (int64_t)B * NO;
    float* H = Z1 + (int64_t)B * NH;
    float* red = H + (int64_t)B * NH;  // [0] = sum(M), [1] = loss
    float* dY = Y;                     // Y is consumed by mlp_bwd_rows before dY overwrites it per element
    float* dZ1 = Z1;                   // likewise for Z1
    int grid = B < 4096 ? B : 4096;
    if (grid < 1) return 0;
    hipLaunchKernelGGL(mlp_fwd, dim3(grid), dim3(64), 0, st, P, X, B, Y, Z1, H);
    hipLaunchKernelGGL(mlp_loss, dim3(1), dim3(256), 0, st, Y, T, M, (int64_t)B * NO, red);
    hipLaunchKernelGGL(mlp_bwd_rows, dim3(grid), dim3(64), 0, st, P, Y, T, M, B, Z1, red, dY, dZ1);
    // dW2 = H^T dY, db2 = sum dY ; dW1 = X^T dZ1, db1 = sum dZ1
    hipLaunchKernelGGL(mlp_wgrad, dim3(NH + 1), dim3(64), 0, st, H, NH, dY, NO, B, grad + OFF_W2, grad + OFF_B2);
    hipLaunchKernelGGL(mlp_wgrad, dim3(NI + 1), dim3(64), 0, st, X, NI, dZ1, NH, B, grad, grad + OFF_B1);
    if (loss && hipMemcpyAsync(loss, red + 1, sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess) return -8;
    return hipGetLastError() == hipSuccess ? 0 : -8;
}

int coot_mlp_adam_launch(float* w, const float* g, float* m, float* v, int n, int t, float lr, float b1, float b2,
                         float eps, void* stream)
{
    float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(mlp_adam, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, w, g, m, v, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError() == hipSuccess ? 0 : -8;
}

}  // extern "C"
