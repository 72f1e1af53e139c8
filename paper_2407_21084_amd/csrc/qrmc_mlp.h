// qrmc_mlp.h -- launchers of the surrogate-network kernels (learned form).
#pragma once

#include "qrmc_common.h"

namespace qrmc {

constexpr int kMlpIn = QR_MLP_IN;
constexpr int kMlpHid = QR_MLP_HIDDEN;
// offsets of the parameter blocks in the flat FP32 vector
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + (int64_t)kMlpHid * kMlpIn;
constexpr int64_t kOffW2 = kOffB1 + kMlpHid;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kMlpHid * kMlpHid;
constexpr int64_t kOffW3 = kOffB2 + kMlpHid;
constexpr int64_t kOffB3 = kOffW3 + kMlpHid;
constexpr int64_t kMlpParams = kOffB3 + 1;
static_assert(kMlpParams == QR_MLP_NPARAMS, "parameter layout");

// C[M][N] (ldc) = (accumulate ? C : 0) + A B with A(i,k) = A[i sai + k sak],
// B(k,j) = B[k sbk + j sbj] (FP32 in memory, bfloat16 operands, FP32 sums).
// Long sums over few output tiles are split over K into `work` (FP32) and
// added in slice order.
hipError_t launch_gemm(int M, int N, int K, const float *A, int64_t sai, int64_t sak, const float *B,
                       int64_t sbk, int64_t sbj, float *C, int64_t ldc, bool accumulate, float *work,
                       int64_t work_floats, hipStream_t s);
constexpr int64_t kColsumWork = 32 * 256;  // floats of workspace launch_colsum needs for H <= 256
// Z[n][H] += b (row broadcast); Hout = silu(Z)
hipError_t launch_bias_silu(int64_t n, int H, float *Z, const float *b, float *Hout, hipStream_t s);
// y[p] = w . X[p][:] + b0  (X [n][H])
hipError_t launch_out_layer(int64_t n, int H, const float *X, const float *w, const float *b0, float *y,
                            hipStream_t s);
// r = y - t; dy = 2 r / n; partial[block] = sum r^2 (blocks of 256)
hipError_t launch_loss(int64_t n, const float *y, const float *t, float *dy, double *partial, hipStream_t s);
// out[h] = sum_p w[p] X[p][h]  (w = NULL: weights 1); work: kColsumWork floats
hipError_t launch_colsum(int64_t n, int H, const float *X, const float *w, float *out, float *work,
                         hipStream_t s);
// dZ[p][h] = dy[p] w3[h] silu'(Z[p][h])
hipError_t launch_dz_out(int64_t n, int H, const float *dy, const float *w3, const float *Z, float *dZ,
                         hipStream_t s);
// dH[p][h] *= silu'(Z[p][h])
hipError_t launch_dsilu(int64_t n, int H, const float *Z, float *dH, hipStream_t s);
hipError_t launch_adam(int64_t n, float *theta, const float *g, float *m, float *v, int64_t step, float lr,
                       hipStream_t s);
hipError_t launch_mlp_init(float *theta, uint64_t seed, hipStream_t s);
// f[p][l] = 2 F(x[l][p]) - 1 (l < d), 0 otherwise; x SoA [d][n] (stride ldx)
// features 2 F_nu(x_l) - 1 of the sampling law nu (qr_law)
hipError_t launch_features(int32_t nu, int32_t d, int64_t n, const double *x, int64_t ldx, float *f,
                           hipStream_t s);
// sums of (mu + sigma y - t)^2 and t^2 per block of 256: partial[2 block], partial[2 block + 1]
hipError_t launch_heldout(int64_t n, const float *y, const double *t, double mu, double sigma, double *partial,
                          hipStream_t s);
hipError_t launch_to_float(int64_t n, const double *x, double mu, double inv_sigma, float *y, hipStream_t s);

}  // namespace qrmc
