// qrmc_factored.h -- the expansion evaluation as a matrix product over paths.
//
// Split the coordinates into a leading block A (the first dA) and a trailing
// block B.  Every representative k = (kA, kB) of the index set has
//   sqrt2 (a_c cos + a_s sin)(2 pi k.u) = Re[ beta_k e^{2 pi i kA.uA} e^{2 pi i kB.uB} ],
//   beta_k = sqrt2 (a_c - i a_s)   (beta_0 = alpha_0 for the constant),
// so the expansion of eq (yqi:bar:M) at a point is
//   ybar = Re sum_r EA(r) C(r),   C(r) = sum_c beta[r][c] EB(c),
// with rows r = the A-parts {0} u {kA : first non-zero > 0} and columns c = all
// B-parts.  For the index sets here the columns of a row are a prefix of the
// columns sorted by their weight (hyperbolic crosses: the B-part's weight is at
// most level / the A-part's weight; tensor sets: every column), so the
// coefficients form a staircase matrix.  For a tile of paths, C is a product
// of that matrix with the paths' EB values: dense, and run on the matrix
// cores (v_mfma_f32_16x16x32 with 16-bit operands and FP32 accumulation),
// while EA and EB come from per-path tables e^{2 pi i m u_l} (phases reduced in
// FP64).  The row 0 holds the constant (column kB = 0) and the
// representatives (0, kB) with kB's first non-zero positive; its other
// columns are zero.
#pragma once

#include <stdint.h>

#include <vector>

#include "qrmc_common.h"

namespace qrmc {

constexpr int kFacRows = 8;     // complex rows per row tile (16 real rows of the product)
constexpr int kFacCols = 16;    // complex columns per K-block (32 real K)
constexpr int kFacNnz = 8;      // factors per row or column code
constexpr int kFacPaths = 16;   // paths per wave (the product's N dimension)

// Factors of one row (A-part) or column (B-part): entry t is +(l TS + m) for
// e^{2 pi i m u_l}, -(l TS + m) for its conjugate, 0 for the factor 1.
struct FacCode {
    int16_t e[kFacNnz];
};

struct FacTile {
    int32_t nkb;   // K-blocks (16 columns each) of the tile's longest row
    int32_t nnz;   // largest number of factors among the tile's rows
    int64_t off;   // first coefficient block of the tile (blocks of 64 lanes x 16 bytes)
};

struct FactorLayout {
    int32_t d = 0, dA = 0;
    int32_t TS = 0;              // table stride: largest magnitude + 1
    int32_t nrow = 0, nrt = 0;   // rows, row tiles of kFacRows
    int32_t ncol = 0, nkb = 0;   // columns, K-blocks over all columns
    int64_t nblocks = 0;         // coefficient blocks of one time step
    std::vector<FacTile> tiles;  // [nrt]
    std::vector<FacCode> rows;   // [nrt * kFacRows], unused rows all-zero
    std::vector<FacCode> cols;   // [nkb * kFacCols], unused columns all-zero
    std::vector<int32_t> colnnz; // [nkb] largest number of factors among a K-block's columns
    // canonical representative of entry (rr, cc) of coefficient block b at
    // ent[(b kFacRows + rr) kFacCols + cc], -1 where the entry is zero
    std::vector<int32_t> ent;
    double cost = 0.0;           // the cost model's figure for the chosen split
};

// Build the factored layout of an index set (canonical representatives, row-
// major [nrep][d], lexicographic) for the best split the cost model finds
// with at most max_nkb K-blocks.  Returns false if no split qualifies.
bool build_factor_layout(int32_t d, int32_t kind, int32_t level, const int32_t *canon, int64_t nrep,
                         int32_t max_nkb, FactorLayout *out);

// Device view of a layout (one per basis and device).
struct FacDev {
    const FacTile *tiles;
    const FacCode *rows;
    const FacCode *cols;
    const int32_t *colnnz;
    const int32_t *ent;
    int32_t nrt, nkb, TS, dA, d;
    int64_t nblocks;
};

struct FacPathArgs {
    const DevProblem *P;
    FacDev F;
    int32_t i;
    int64_t M;
    uint64_t seed;
    const uint4 *coef;   // [N][nblocks][64] 16-bit coefficient blocks
    double *S;           // [M]
    double2 *e;          // start-point phase factors e^{2 pi i F(x_l)}, [d][M]
};

// largest K-block count the path kernel's instances cache
constexpr int kFacMaxNkb = 24;

// A projection task: R consecutive row tiles from rt0, K-blocks from kb0
// (template tmpl).
struct FacTask {
    int32_t rt0, R, tmpl, kb0;
};
constexpr int kFacTemplates = 4;
void build_fac_tasks(const FactorLayout &L, std::vector<FacTask> tasks[kFacTemplates]);
hipError_t launch_fac_project(int prec, int tmpl, const FacDev &F, const FacTask *tasks, int32_t ntasks,
                              const double2 *e, const double *S, int64_t M, int64_t per_unit, int32_t units,
                              float *partial, hipStream_t s);
hipError_t launch_fac_reduce(const float *partial, int32_t units, int64_t nblocks, const int32_t *ent, double M,
                             double *alpha_row, int32_t *bad, int32_t step, hipStream_t s);
// entries of a path's tables e^{2 pi i m u_l} (l < d, m < TS) in LDS, padded
// to an odd count so that the 16 paths of a lane group fall in distinct banks
__host__ __device__ inline int32_t fac_stride(int32_t d, int32_t TS) { return (d * TS) | 1; }
// waves per block of the path kernel for a table of d x TS entries per path
int fac_waves(int32_t d, int32_t TS);
hipError_t launch_fac_pack(int prec, const double *alpha_row, const int32_t *ent, int64_t nblocks,
                           uint4 *out, hipStream_t s);
hipError_t launch_fac_path(int db, int prec, const FacPathArgs &a, hipStream_t s);

}  // namespace qrmc
