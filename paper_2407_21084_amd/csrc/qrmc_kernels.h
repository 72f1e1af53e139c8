// qrmc_kernels.h -- launchers of the HIP kernels (host side declarations).
#pragma once

#include "qrmc_common.h"

namespace qrmc {

constexpr int kPathBlock = 128;   // threads per block of the path / eval kernels
#ifndef QRMC_PATH_P
#define QRMC_PATH_P 2
#endif
constexpr int kPathP = QRMC_PATH_P;  // paths per thread of the value-only path kernel
// Shape of the projection kernel for a basis of dimension d: paths per lane,
// waves per block and the largest task (consecutive traversal nodes) a block
// accumulates.  The widest shape whose LDS (the lanes' phase factors and the
// waves' task accumulators) fits is taken; the basis cuts its tasks to the
// same size.
struct ProjShape {
    int P, waves, task_max;
};
ProjShape proj_shape(int32_t d);
// coefficient rows (double2, traversal order) are zero-padded to whole
// 64-node chunks plus two chunks of read-ahead
__host__ __device__ constexpr int64_t coef_ld(int64_t nrep) { return ((nrep + 63) / 64 + 2) * 64; }

constexpr int kBatchRT = 8;       // instances per pass of the batched path kernel
constexpr int kPassTM = 64;       // nodes per task of the pass projection
constexpr int kPassWaves = 4;     // waves per block of the pass projection

// Per-pass parameters of a batch (device memory, one per context): members
// per pass, the driver parameter and the cloud size of slot k of pass p at
// f_a[p kBatchRT + k] and m[p kBatchRT + k] (m = 0 for an empty slot).
struct DevBatch {
    int32_t count[QR_MAX_BATCH];
    double f_a[QR_MAX_BATCH * kBatchRT];
    int64_t m[QR_MAX_BATCH * kBatchRT];
};

struct BatchArgs {
    const DevProblem *P;
    int32_t d;  // problem dimension (paths are simulated in all d coordinates)
    const DevBatch *B;
    int32_t pass;
    Walk W;
    int32_t i;
    int64_t M;
    uint64_t seed;
    const double2 *alpha_b;  // [N][ld][kBatchRT] of this pass
    int64_t ld;
    double *S;   // [kBatchRT][M] of this pass
    double2 *e;  // start-point phase factors e^{2 pi i F(x_l)}, [d][M]
};

// Reduced-precision path kernel.  The coefficient tiles of row j are at
// tiles + j tile_ld (uint2 units); a row holds ceil(nrep / 32) groups of
// T x 64 uint2 (T = mfma_tile_groups).
struct MfmaArgs {
    const DevProblem *P;
    Walk W;
    int32_t i;
    int64_t M;
    uint64_t seed;
    const uint2 *tiles;
    int64_t tile_ld;
    double *S;
    double2 *e;  // start-point phase factors, [d][M]
};

struct PathArgs {
    const DevProblem *P;
    Walk W;
    int32_t i;
    int64_t M;
    uint64_t seed;
    const double2 *alpha_int;  // [N][ld]
    int64_t ld;
    double *S;
    double2 *e;  // start-point phase factors e^{2 pi i F(x_l)}, [d][M]
    double *x0;
    double *xs;   // path state [d][ldx], ldx >= path_state_ld(M, grad)
    int64_t ldx;
    double *f0 = nullptr;  // [2][M]: the driver sum's first term f(t_i, ...) Delta_i and the
                           // value the driver read on that step, or NULL
};

hipError_t launch_gather(const double *alpha, int32_t row0, int32_t nrows, int64_t nrep, int64_t ld,
                         int64_t nfuncs, const int32_t *canon_of_trav, double2 *alpha_int,
                         hipStream_t s);
hipError_t launch_pad(int32_t nrows, int64_t nrep, int64_t ld, double2 *alpha_int, hipStream_t s);
// y <- y D, grad <- D (grad + y q x / (1+|x|^2)) with D = (1+|x|^2)^{q/2}
hipError_t launch_undamp(int32_t d, double q, const double *x, int64_t n, double *y, double *grad, hipStream_t s);
// cosine rows [row0, row0 + nrows) of acos ([.][ncos]) into carrier rows of
// acar ([.][2 nrep - 1]); one carrier row into one cosine row
hipError_t launch_cos_expand(const double *acos, int32_t row0, int32_t nrows, int64_t ncos, int64_t nrep,
                             const int32_t *cos_of_rep, const double *rep_scale, double *acar, hipStream_t s);
hipError_t launch_cos_fold(const double *acar_row, int64_t ncos, const int32_t *fold_off, const int32_t *fold_idx,
                           const double *rep_scale, double *acos_row, hipStream_t s);
// damp: the problem's damping exponent q is non-zero
// feat: 0 plain problem, 1 damping q > 0, 2 damping and state-dependent b, sigma
hipError_t launch_path(int db, int cap, bool grad, int feat, const PathArgs &a, hipStream_t s);
// tasks must have been cut to proj_shape(W.d).task_max nodes (task_max is checked)
hipError_t launch_project(int cap, const Walk &W, const double2 *e, int64_t lde, const double *S, int64_t M,
                          int64_t paths_per_split, int32_t ntasks, int32_t nsplit, const Task *tasks,
                          const TaskItem *items, int32_t task_max, double2 *partial, int64_t nrep,
                          hipStream_t s);
// bad (device, or NULL): atomically raised to `step` if a coefficient is not finite
hipError_t launch_reduce(const double2 *partial, int32_t nsplit, int64_t nrep, double M,
                         double2 *alpha_int_row, double *alpha_row,
                         const int32_t *canon_of_trav, int32_t *bad, int32_t step, hipStream_t s);
hipError_t launch_set_flag(int32_t *flag, int32_t v, hipStream_t s);
hipError_t launch_eval(int cap, bool grad, const Walk &W, const double2 *alpha_int_row,
                       const double *x, int64_t n, double *y, double *grad_out, hipStream_t s);
hipError_t launch_x_to_e(int32_t nu, int32_t d, const double *x, int64_t n, double2 *e, hipStream_t s);
// ybar at n points with the basis split across blocks (the projection's
// tasks and shape): e = phase factors [d][n]; partial: ceil(ntasks / waves) x n
// doubles of workspace; y[n] = sum of the groups in order
size_t eval_tasks_lds(int32_t d);
hipError_t launch_eval_tasks(int cap, const Walk &W, const double2 *e, int64_t n, int64_t pps, int32_t ntasks,
                             int32_t nsplit, const Task *tasks, const TaskItem *items, int32_t task_max,
                             const double2 *row, double *partial, double *y, hipStream_t s);
hipError_t launch_sample(int32_t nu, int32_t d, uint64_t seed, uint32_t stream_id, int32_t i, int64_t m0,
                         int64_t n, double *x, hipStream_t s);

hipError_t launch_batched_path(int db, int cap, const BatchArgs &a, hipStream_t s);
// partial [split][n_part][R]: R = 1, n_part = nrep_sub (the instance's own
// projection) or the pass projection's R slots over n_part pass-walk nodes
hipError_t launch_reduce_batched(const double2 *partial, int32_t nsplit, int64_t nrep_sub, int64_t n_part,
                                 int32_t R, double M, const int32_t *ft, const int32_t *canon_of_trav,
                                 const int32_t *pass_pos, double2 *alpha_b_row, int32_t slot,
                                 double *alpha_row, int32_t *bad, int32_t step, hipStream_t s);
// the projection of a pass: kBatchRT responses (S [kBatchRT][M], member r
// using its first m_r[r] paths, m_r device) on the pass walk's tasks of
// kPassTM nodes; partial [nsplit][nrep][kBatchRT] double2
int pass_paths_per_lane(int32_t d);
size_t project_pass_lds_bytes(int32_t d);
hipError_t launch_project_pass(int cap, const Walk &W, const double2 *e, int64_t lde, const double *S, int64_t M,
                               const int64_t *m_r, int64_t pps, int32_t ntasks, int32_t nsplit, const Task *tasks,
                               const TaskItem *items, double2 *partial, int64_t nrep, hipStream_t s);
hipError_t launch_zero(double *p, int64_t n, hipStream_t s);
hipError_t launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s);

// Z of the multistep scheme: responses out[r][m] = (S[m] - f0[m]) dW_{i,k0+r}(m) / Delta_i
// for r < nk (0 for nk <= r < kBatchRT), dW the first increment of path m's stream
// Z responses out[r][M] for the Brownian components k0 + r, r < nk: the
// multistep response (y0 NULL) or the one-step one (y0 = ybar_{i+1} at X_i);
// f0 [2][M] from the path kernel (first term, value read on the first step)
hipError_t launch_z_responses(const DevProblem *P, uint64_t seed, int32_t i, int64_t M, int32_t k0, int32_t nk,
                              const double *S, const double *f0, const double *y0, double *out, hipStream_t s);
// g at n points x [d][n]
hipError_t launch_g_points(int db, const DevProblem *P, const double *x, int64_t n, double *y, hipStream_t s);
// canonical row of response slot `slot` of a pass-projection partial [nsplit][nrep][R]
hipError_t launch_reduce_slot(const double2 *partial, int32_t nsplit, int64_t nrep, int32_t R, int32_t slot,
                              double M, const int32_t *canon_of_trav, double *alpha_row, int32_t *bad, int32_t step,
                              hipStream_t s);


// step-major path simulation (learned form); x, u SoA [d][M]
hipError_t launch_sm_start(const DevProblem *P, int32_t nu, int32_t i, int64_t M, uint64_t seed, double *x, double2 *e,
                           double *S, hipStream_t s);
hipError_t launch_sm_euler(int db, const DevProblem *P, int32_t i, int32_t j, int64_t M, uint64_t seed, double *x,
                           double *H, hipStream_t s);
hipError_t launch_sm_accum(const DevProblem *P, int32_t j, int64_t m0, int64_t n, const double *y64,
                           const float *y32, double mu, double sigma, const double *H, double *S, hipStream_t s);
hipError_t launch_sm_final(int db, const DevProblem *P, int64_t M, const double *x, const double *H, double *S,
                           hipStream_t s);
hipError_t launch_moments(int64_t n, const double *t, double *partial, hipStream_t s);
size_t mfma_path_lds_bytes(int32_t d);
hipError_t launch_mfma_path(int db, int cap, bool grad, int prec, const MfmaArgs &a, hipStream_t s);
int mfma_tile_groups(int db, int d, bool grad);
// half: the cosine basis's half-frequency walk (gradient weights pi k, not 2 pi k)
hipError_t launch_pack_tiles(int prec, const double2 *alpha_int_row, int64_t nrep, const int32_t *trav,
                             int32_t d, int32_t T, bool half, uint2 *out, hipStream_t s);
size_t path_lds_bytes(int32_t d, bool grad, int P);
// paths the path kernel's grid covers (M rounded up to whole blocks)
int64_t path_state_ld(int64_t M, bool grad);

}  // namespace qrmc
