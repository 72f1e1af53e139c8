// qrmc_mlp.hip -- the surrogate network of the learned form: a product of
// bfloat16 operands on the matrix cores with FP32 accumulation for every
// layer of the forward and backward pass, the activations, the loss
// gradient and the Adam update.  Network: features (16) -> silu(W1 f + b1)
// (256) -> silu(W2 h1 + b2) (256) -> w3 . h2 + b3.
#include <cmath>

#include "qrmc_mlp.h"

namespace qrmc {

typedef short mlp_s16x4 __attribute__((ext_vector_type(4)));
typedef float mlp_f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float x) {
    const __bf16 b = (__bf16)x;
    return __builtin_bit_cast(short, b);
}

__device__ __forceinline__ float sigmoidf_(float z) { return 1.0f / (1.0f + expf(-z)); }

// v_mfma_f32_16x16x16_bf16: lane l holds A[l%16][4(l/16) + e] and
// B[4(l/16) + e][l%16] (e = 0..3) and receives D[4(l/16) + r][l%16].
// A block of 4 waves computes a 64 x 64 tile of C, each wave 32 x 32.
// With a K split (gridDim.z > 1), slice z sums k in [z kz, (z+1) kz) into
// C + z M ldc (a partial product, no accumulation).
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, int kz, const float *__restrict__ A,
                                                   int64_t sai, int64_t sak, const float *__restrict__ B,
                                                   int64_t sbk, int64_t sbj, float *__restrict__ C,
                                                   int64_t ldc, int accumulate) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kb = blockIdx.z * kz, ke = min(K, kb + kz);
    C += (int64_t)blockIdx.z * M * ldc;
    const int i0 = blockIdx.y * 64 + (wave >> 1) * 32, j0 = blockIdx.x * 64 + (wave & 1) * 32;
    const int r16 = lane & 15, kq = (lane >> 4) * 4;
    mlp_f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mlp_f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += 16) {
        mlp_s16x4 av[2], bv[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int i = i0 + 16 * t + r16, j = j0 + 16 * t + r16;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = k0 + kq + e;
                av[t][e] = bf16_bits((i < M && k < ke) ? A[(int64_t)i * sai + (int64_t)k * sak] : 0.f);
                bv[t][e] = bf16_bits((j < N && k < ke) ? B[(int64_t)k * sbk + (int64_t)j * sbj] : 0.f);
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + 16 * a + kq + r, j = j0 + 16 * b + r16;
                if (i < M && j < N) {
                    float *c = C + (int64_t)i * ldc + j;
                    *c = (accumulate ? *c : 0.f) + acc[a][b][r];
                }
            }
}

// C[i][j] = (accumulate ? C : 0) + sum_z W[z][i][j], z ascending
__global__ void sum_slices_kernel(int M, int N, int nz, const float *__restrict__ W, float *__restrict__ C,
                                  int64_t ldc, int accumulate) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)M * N) return;
    const int64_t i = idx / N, j = idx % N;
    float sum = accumulate ? C[i * ldc + j] : 0.f;
    for (int z = 0; z < nz; ++z) sum += W[((int64_t)z * M + i) * N + j];
    C[i * ldc + j] = sum;
}

__global__ void bias_silu_kernel(int64_t n, int H, float *__restrict__ Z, const float *__restrict__ b,
                                 float *__restrict__ Hout) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * H) return;
    const float z = Z[idx] + b[idx % H];
    Z[idx] = z;
    Hout[idx] = z * sigmoidf_(z);
}

// one wave per point: lanes stride the hidden units, then a fixed-order
// butterfly over the wave
__global__ void out_layer_kernel(int64_t n, int H, const float *__restrict__ X, const float *__restrict__ w,
                                 const float *__restrict__ b0, float *__restrict__ y) {
    const int64_t p = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= n) return;
    float s = 0.f;
    for (int h = lane; h < H; h += 64) s = fmaf(w[h], X[p * H + h], s);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) y[p] = s + b0[0];
}

__global__ void loss_kernel(int64_t n, const float *__restrict__ y, const float *__restrict__ t,
                            float *__restrict__ dy, double *__restrict__ partial) {
    __shared__ double red[256];
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double r2 = 0.0;
    if (p < n) {
        const float r = y[p] - t[p];
        dy[p] = 2.0f * r / (float)n;
        r2 = (double)r * r;
    }
    red[threadIdx.x] = r2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Column sums in two fixed-order stages: block (column group, row slice)
// sums its rows (4 row phases per column, combined in order), then the
// slices are added in order.
constexpr int kColSlices = 32;
__global__ void colsum_kernel(int64_t n, int H, const float *__restrict__ X, const float *__restrict__ w,
                              float *__restrict__ part) {
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int h = blockIdx.x * 64 + c;
    const int64_t rows = (n + kColSlices - 1) / kColSlices;
    const int64_t p0 = blockIdx.y * rows, p1 = min(n, p0 + rows);
    float sacc = 0.f;
    if (h < H)
        for (int64_t p = p0 + ph; p < p1; p += 4) sacc = fmaf(w ? w[p] : 1.0f, X[p * H + h], sacc);
    red[ph][c] = sacc;
    __syncthreads();
    if (ph == 0 && h < H) part[(int64_t)blockIdx.y * H + h] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

__global__ void colsum_finish_kernel(int H, const float *__restrict__ part, float *__restrict__ out) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= H) return;
    float sacc = 0.f;
    for (int z = 0; z < kColSlices; ++z) sacc += part[(int64_t)z * H + h];
    out[h] = sacc;
}

__global__ void dz_out_kernel(int64_t n, int H, const float *__restrict__ dy, const float *__restrict__ w3,
                              const float *__restrict__ Z, float *__restrict__ dZ) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * H) return;
    const float z = Z[idx], sg = sigmoidf_(z);
    dZ[idx] = dy[idx / H] * w3[idx % H] * (sg * (1.0f + z * (1.0f - sg)));
}

__global__ void dsilu_kernel(int64_t n, int H, const float *__restrict__ Z, float *__restrict__ dH) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * H) return;
    const float z = Z[idx], sg = sigmoidf_(z);
    dH[idx] *= sg * (1.0f + z * (1.0f - sg));
}

__global__ void adam_kernel(int64_t n, float *__restrict__ th, const float *__restrict__ g,
                            float *__restrict__ m, float *__restrict__ v, float c1, float c2, float lr) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    // 1 - beta as its own constant: 1.0f - 0.999f is 5e-5 off 0.001 in FP32
    const float b1 = 0.9f, omb1 = 0.1f, b2 = 0.999f, omb2 = 0.001f, eps = 1e-8f;
    const float mk = b1 * m[k] + omb1 * g[k];
    const float vk = b2 * v[k] + omb2 * g[k] * g[k];
    m[k] = mk;
    v[k] = vk;
    th[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// uniform fan-in initialisation (W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)),
// biases 0) from Philox stream 2, counter (parameter index, 0, 0)
__global__ void mlp_init_kernel(float *__restrict__ th, uint64_t seed) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kMlpParams) return;
    float scale = 0.f;
    if (k < kOffB1) scale = 1.0f / sqrtf((float)kMlpIn);
    else if (k >= kOffW2 && k < kOffB2) scale = 1.0f / sqrtf((float)kMlpHid);
    else if (k >= kOffW3 && k < kOffB3) scale = 1.0f / sqrtf((float)kMlpHid);
    th[k] = scale == 0.f ? 0.f : scale * (float)(2.0 * uniform_at(seed, 2u, (uint64_t)k, 0u, 0u) - 1.0);
}

__global__ void features_kernel(int32_t nu, int32_t d, int64_t n, const double *__restrict__ x, int64_t ldx,
                                float *__restrict__ f) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * kMlpIn) return;
    const int64_t p = idx / kMlpIn;
    const int l = (int)(idx % kMlpIn);
    f[idx] = l < d ? (float)(2.0 * law_cdf(nu, x[l * ldx + p]) - 1.0) : 0.f;
}

__global__ void heldout_kernel(int64_t n, const float *__restrict__ y, const double *__restrict__ t, double mu,
                               double sigma, double *__restrict__ partial) {
    __shared__ double ra[256], rb[256];
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (p < n) {
        const double e = mu + sigma * (double)y[p] - t[p];
        a = e * e;
        b = t[p] * t[p];
    }
    ra[threadIdx.x] = a;
    rb[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            ra[threadIdx.x] += ra[threadIdx.x + o];
            rb[threadIdx.x] += rb[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = ra[0];
        partial[2 * blockIdx.x + 1] = rb[0];
    }
}

__global__ void to_float_kernel(int64_t n, const double *__restrict__ x, double mu, double inv_sigma,
                                float *__restrict__ y) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) y[p] = (float)((x[p] - mu) * inv_sigma);
}

static inline unsigned nblocks(int64_t n, int64_t b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_gemm(int M, int N, int K, const float *A, int64_t sai, int64_t sak, const float *B,
                       int64_t sbk, int64_t sbj, float *C, int64_t ldc, bool accumulate, float *work,
                       int64_t work_floats, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int64_t tiles = (int64_t)nblocks(N, 64) * nblocks(M, 64);
    // split long reductions over few output tiles
    int nz = 1;
    if (tiles < 256 && K >= 512 && work) {
        nz = (int)std::min<int64_t>(std::min<int64_t>(K / 256, 64), work_floats / ((int64_t)M * N));
        if (nz < 2) nz = 1;
    }
    const int kz = nz == 1 ? K : (((K + nz - 1) / nz + 15) / 16) * 16;
    if (nz > 1) nz = (K + kz - 1) / kz;
    if (nz == 1) {
        hipLaunchKernelGGL(gemm_kernel, dim3(nblocks(N, 64), nblocks(M, 64), 1), dim3(256), 0, s, M, N, K, K, A,
                           sai, sak, B, sbk, sbj, C, ldc, accumulate ? 1 : 0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(gemm_kernel, dim3(nblocks(N, 64), nblocks(M, 64), nz), dim3(256), 0, s, M, N, K, kz, A, sai,
                       sak, B, sbk, sbj, work, (int64_t)N, 0);
    hipLaunchKernelGGL(sum_slices_kernel, dim3(nblocks((int64_t)M * N, 256)), dim3(256), 0, s, M, N, nz, work, C,
                       ldc, accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_bias_silu(int64_t n, int H, float *Z, const float *b, float *Hout, hipStream_t s) {
    hipLaunchKernelGGL(bias_silu_kernel, dim3(nblocks(n * H, 256)), dim3(256), 0, s, n, H, Z, b, Hout);
    return hipGetLastError();
}

hipError_t launch_out_layer(int64_t n, int H, const float *X, const float *w, const float *b0, float *y,
                            hipStream_t s) {
    hipLaunchKernelGGL(out_layer_kernel, dim3(nblocks(n, 4)), dim3(256), 0, s, n, H, X, w, b0, y);
    return hipGetLastError();
}

hipError_t launch_loss(int64_t n, const float *y, const float *t, float *dy, double *partial, hipStream_t s) {
    hipLaunchKernelGGL(loss_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, n, y, t, dy, partial);
    return hipGetLastError();
}

hipError_t launch_colsum(int64_t n, int H, const float *X, const float *w, float *out, float *work,
                         hipStream_t s) {
    hipLaunchKernelGGL(colsum_kernel, dim3(nblocks(H, 64), kColSlices), dim3(256), 0, s, n, H, X, w, work);
    hipLaunchKernelGGL(colsum_finish_kernel, dim3(nblocks(H, 64)), dim3(64), 0, s, H, work, out);
    return hipGetLastError();
}

hipError_t launch_dz_out(int64_t n, int H, const float *dy, const float *w3, const float *Z, float *dZ,
                         hipStream_t s) {
    hipLaunchKernelGGL(dz_out_kernel, dim3(nblocks(n * H, 256)), dim3(256), 0, s, n, H, dy, w3, Z, dZ);
    return hipGetLastError();
}

hipError_t launch_dsilu(int64_t n, int H, const float *Z, float *dH, hipStream_t s) {
    hipLaunchKernelGGL(dsilu_kernel, dim3(nblocks(n * H, 256)), dim3(256), 0, s, n, H, Z, dH);
    return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float *theta, const float *g, float *m, float *v, int64_t step, float lr,
                       hipStream_t s) {
    const float c1 = (float)(1.0 - std::pow(0.9, (double)step));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)step));
    hipLaunchKernelGGL(adam_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, n, theta, g, m, v, c1, c2, lr);
    return hipGetLastError();
}

hipError_t launch_mlp_init(float *theta, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(mlp_init_kernel, dim3(nblocks(kMlpParams, 256)), dim3(256), 0, s, theta, seed);
    return hipGetLastError();
}

hipError_t launch_features(int32_t nu, int32_t d, int64_t n, const double *x, int64_t ldx, float *f,
                           hipStream_t s) {
    hipLaunchKernelGGL(features_kernel, dim3(nblocks(n * kMlpIn, 256)), dim3(256), 0, s, nu, d, n, x, ldx, f);
    return hipGetLastError();
}

hipError_t launch_heldout(int64_t n, const float *y, const double *t, double mu, double sigma, double *partial,
                          hipStream_t s) {
    hipLaunchKernelGGL(heldout_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, n, y, t, mu, sigma, partial);
    return hipGetLastError();
}

hipError_t launch_to_float(int64_t n, const double *x, double mu, double inv_sigma, float *y, hipStream_t s) {
    hipLaunchKernelGGL(to_float_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, n, x, mu, inv_sigma, y);
    return hipGetLastError();
}

}  // namespace qrmc
