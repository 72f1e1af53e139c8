// qrmc_kernels.h -- launchers of the HIP kernels (host side declarations).
#pragma once

#include "qrmc_common.h"

namespace qrmc {

constexpr int kPathBlock = 128;   // threads per block of the path / eval kernels
constexpr int kProjWaves = 4;     // waves per block of the projection kernel
constexpr int kProjChunk = 8;     // nodes per cross-lane reduction of the projection
constexpr int kTaskMax = 256;     // nodes per projection task

struct PathArgs {
    const DevProblem *P;
    SetRule R;
    int32_t i;
    int64_t M;
    uint64_t seed;
    const double2 *alpha_int;  // [N][ld]
    const uint32_t *ops;       // [nrep + kOpPad]
    int64_t nrep, ld;
    double *S, *u, *x0;
};

hipError_t launch_gather(const double *alpha, int32_t row0, int32_t nrows, int64_t nrep, int64_t ld,
                         int64_t nfuncs, const int32_t *canon_of_trav, double2 *alpha_int,
                         hipStream_t s);
hipError_t launch_pad(int32_t nrows, int64_t nrep, int64_t ld, double2 *alpha_int, hipStream_t s);
hipError_t launch_path(int db, int cap, bool grad, const PathArgs &a, hipStream_t s);
hipError_t launch_project(int cap, const SetRule &R, const double *u, const double *S, int64_t M,
                          int64_t paths_per_split, int32_t ntasks, int32_t nsplit, const Task *tasks,
                          const TaskItem *items, double2 *partial, int64_t nrep, hipStream_t s);
hipError_t launch_reduce(const double2 *partial, int32_t nsplit, int64_t nrep, double M,
                         double2 *alpha_int_row, double *alpha_row,
                         const int32_t *canon_of_trav, hipStream_t s);
hipError_t launch_eval(int cap, bool grad, const SetRule &R, const double2 *alpha_int_row,
                       const uint32_t *ops, int64_t nrep, const double *x, int64_t n, double *y,
                       double *grad_out, hipStream_t s);
hipError_t launch_x_to_u(int32_t d, const double *x, int64_t n, double *u, hipStream_t s);
hipError_t launch_sample(int32_t d, uint64_t seed, uint32_t stream_id, int32_t i, int64_t m0,
                         int64_t n, double *x, hipStream_t s);

size_t project_lds_bytes(int32_t d);

}  // namespace qrmc
