/*
 * qrmc.h -- C ABI of libqrmc, an MI355X (gfx950) implementation of the
 * quasi-regression Monte-Carlo (QRMC) backward step of Gobet, Lopez-Salas and
 * Vazquez, "Quasi-Regression Monte-Carlo scheme for semi-linear PDEs and BSDEs
 * with large scale parallelization on GPUs" (arXiv 2407.21084).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns a qr_status; nothing throws across the ABI.  On a
 *    non-zero status, qr_last_error() returns a thread-local message.
 *  - "device" pointers are HIP device allocations (e.g. the data pointer of a
 *    torch tensor on a ROCm device) owned by the caller; "host" pointers are
 *    ordinary memory owned by the caller and only read during the call.
 *  - Device work is enqueued on the HIP stream passed as `stream` (NULL = the
 *    null stream) and is asynchronous: results are valid once the stream has
 *    been synchronised.  Arguments are validated on the host before anything
 *    is launched; asynchronous device faults surface at the next
 *    synchronising call as QR_EDEVICE.
 *  - A context (qr_ctx) owns device workspace and must not be used from two
 *    host threads or on two streams at the same time.
 *  - Floating-point arguments and results are IEEE binary64, except the
 *    network entry points of the learned form (qr_mlp_*), which take binary32
 *    parameters, features and outputs.
 *
 * Mathematical objects (paper notation)
 * -------------------------------------
 *  - Decoupled FBSDE / semi-linear PDE of Sec. 1, eqs (fbsde), (eds), (pde):
 *    drift b, diffusion sigma, driver f, terminal condition g, horizon T.
 *  - Time grid t_0 < ... < t_N (Sec. 2.1.1), Euler scheme eq (markov:euler).
 *  - Sampling law nu of assumption (A_nu): a product of identical
 *    one-dimensional laws with CDF F, chosen per basis (qr_law): the
 *    standard logistic law F(x) = 1/(1+e^{-x}) (default), or the paper's own
 *    Student's t law with mu = 2 and Cauchy law (Sec. 5).
 *  - Basis (Sec. 2.2, Lemma 2.1 with the Fourier basis of the torus):
 *    phi_0 = 1 and, for each representative k of {k,-k} (first non-zero
 *    coordinate positive), sqrt2 cos(2 pi k.F(x)) and sqrt2 sin(2 pi k.F(x)),
 *    orthonormal in L2(nu).
 *  - Index sets Gamma over Z^d (Sec. 2.3.3).
 *  - Algorithm 1 (GQRMDP) with damping q = 0 and a constant truncation
 *    level L for T_L.
 *
 * Coefficient layout ("canonical order"): for a basis with R representatives
 * k_0 = 0 < k_1 < ... < k_{R-1} in lexicographic order of integer vectors,
 * a coefficient row has n_funcs = 2R-1 entries: entry 0 multiplies phi_0 = 1,
 * entry 2r-1 multiplies sqrt2 cos(2 pi k_r.F(x)), entry 2r multiplies
 * sqrt2 sin(2 pi k_r.F(x)).  A coefficient table is row-major [N][n_funcs],
 * row i holding ybar_i (ybar_N = g is not stored).
 *
 * Random streams: every random number is drawn from Philox4x32-10 (Salmon et
 * al., SC'11).  Draw r of sample m at time index i of stream s uses
 * key (seed_lo, seed_hi ^ s), counter (m_lo, m_hi, i, r >> 1) and words
 * (w0,w1) for even r, (w2,w3) for odd r; U = ((w_a<<20 | w_b>>12) + 1/2) 2^-52.
 * Stream 0: solver paths (start point draws r = 0..d-1, then nbm normals per
 * Euler step: r = d + (j-i) nbm + k).  Stream 1: test points.  Streams 2
 * and 3: training and held-out points of the learned form (time index i =
 * the time index of the fitted expansion); stream 2 also initialises the
 * network (counter (parameter index, 0, 0)).
 */
#ifndef QRMC_H
#define QRMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QR_MAX_D 16    /* maximum state / Brownian dimension            */
#define QR_MAX_DAMPING 64 /* largest damping exponent q                 */
#define QR_MAX_N 128   /* maximum number of time steps                  */

typedef enum {
    QR_OK = 0,
    QR_EINVAL = -1,   /* invalid argument (message says which)            */
    QR_ENOMEM = -2,   /* device or host allocation failed                 */
    QR_EDEVICE = -3,  /* HIP runtime or launch error                      */
    QR_ERANGE = -4,   /* size overflow (index set, M, workspace)          */
    QR_ENUMERIC = -5, /* non-finite coefficient produced (qr_ctx_numeric_status) */
    QR_ENOTSUP = -6   /* valid request outside what this library supports */
} qr_status;

/* Message for the last failing call on this thread ("" if none). */
const char *qr_last_error(void);

/* Library version string. */
const char *qr_version(void);

/* ---------------------------------------------------------------------- */
/* Index sets and basis (Sec. 2.3.3 "Multi-indices sets", Lemma 2.1)       */
/* ---------------------------------------------------------------------- */
typedef enum {
    QR_SET_TENSOR = 0, /* {k in Z^d : max_l |k_l| <= level}  (Gamma_F)        */
    QR_SET_HC_MAX = 1, /* {k in Z^d : prod_l max(1,|k_l|) <= level} (Gamma_H) */
    QR_SET_HC_1P = 2,  /* {k in Z^d : prod_l (1+|k_l|) <= level}              */
    QR_SET_TOTAL = 3   /* {k in Z^d : sum_l |k_l| <= level}   (Gamma_T)       */
} qr_set_kind;

typedef struct qr_basis qr_basis; /* opaque, library-owned */

/* One-dimensional marginal nu_l of the sampling law (assumption (A_nu)).
 * The paper's experiments use Student's t laws (Example "Student's
 * t-distribution", Sec. 5, eq (Fnui:Fnulinv)):
 *   QR_LAW_LOGISTIC: F(x) = 1/(1+e^{-x}), F^{-1}(u) = ln u - ln(1-u);
 *   QR_LAW_STUDENT2: mu = 2, density (1+x^2)^{-3/2}/2,
 *                    F(x) = (1 + x/sqrt(1+x^2))/2, F^{-1}(u) = (u-1/2)/sqrt(u(1-u));
 *   QR_LAW_CAUCHY:   mu = 1, density 1/(pi (1+x^2)),
 *                    F(x) = 1/2 + atan(x)/pi, F^{-1}(u) = tan(pi (u - 1/2)). */
typedef enum {
    QR_LAW_LOGISTIC = 0,
    QR_LAW_STUDENT2 = 1,
    QR_LAW_CAUCHY = 2
} qr_law;

/* Build the index set of kind `kind` and level `level` in dimension d
 * (1 <= d <= QR_MAX_D; level >= 0 for the tensor and total-degree sets,
 * level >= 1 for the hyperbolic crosses, whose sets are empty below 1) and
 * its basis metadata.
 * Host only; no device is touched.  *out receives a handle to free with
 * qr_basis_free.  QR_ERANGE if the set has more than 2^31 representatives. */
qr_status qr_build_basis(int32_t d, int32_t kind, int32_t level, qr_basis **out);

/* As qr_build_basis, for the sampling law `law` (qr_law; QR_EINVAL if
 * unknown).  The basis functions in x are phi_k o F_law (Lemma 2.1), and every
 * call that takes this basis draws its start points X_i ~ nu (Algorithm 1)
 * and maps points to the cube with this law.  qr_build_basis is this call
 * with QR_LAW_LOGISTIC. */
qr_status qr_build_basis_law(int32_t d, int32_t kind, int32_t level, int32_t law, qr_basis **out);

/* The sampling law of a basis (qr_law) into *law. */
qr_status qr_basis_law(const qr_basis *b, int32_t *law);

/* Family of basis functions of a qr_basis. */
typedef enum {
    QR_BASIS_FOURIER = 0, /* the Fourier functions above, over Z^d          */
    QR_BASIS_COSINE = 1   /* the paper's cosine functions over N^d (below)  */
} qr_basis_family;

/* The paper's own basis (Sec. 2.2, Lemma 2.1, eq (nu_basis_functions) with
 * the cosine system of L2([0,1]), and eq (phi:dim:d)): for k in N^d,
 *   phi_k(x) = prod_l c_{k_l}(F(x_l)),  c_0 = 1,  c_m(u) = sqrt2 cos(m pi u),
 * orthonormal in L2(nu), over the index set {k in N^d : k in Gamma} with Gamma
 * of kind `kind` (Gamma_F, Gamma_H, the (1+|k|) cross or Gamma_T; Sec. 2.3.3)
 * and level `level`, limits as in qr_build_basis_law.  A coefficient row of
 * this basis has n_funcs = #(Gamma over N^d) entries, entry c multiplying
 * phi_k for the c-th vector k in lexicographic order (qr_basis_indices).
 * Every entry point that takes a basis accepts this one except the batched
 * and learned forms (QR_ENOTSUP).  The kernels evaluate and project it
 * through the identity, for a vector k with n non-zero coordinates,
 *   phi_k(x) = 2^{1 - n/2} sum cos(pi k'.F(x))   (n >= 1),
 * the sum over the 2^{n-1} vectors k' of Z^d with |k'_l| = k_l and first
 * non-zero coordinate positive: the Fourier walk over the Z^d set of the same
 * kind and level at half the frequency. */
qr_status qr_build_basis_cos(int32_t d, int32_t kind, int32_t level, int32_t law, qr_basis **out);

/* The family of a basis (qr_basis_family) into *family. */
qr_status qr_basis_family_of(const qr_basis *b, int32_t *family);

/* n_funcs = |Gamma| (real basis functions), n_reps = representatives
 * (n_funcs = 2 n_reps - 1; for a cosine basis n_reps = n_funcs, the vectors
 * of N^d), max_nnz = largest number of non-zero coordinates of a k in the
 * set.  Any output pointer may be NULL. */
qr_status qr_basis_info(const qr_basis *b, int64_t *n_funcs, int64_t *n_reps, int32_t *max_nnz);

/* Copy the representatives in canonical (lexicographic) order into
 * reps_out, host memory of n_reps * d int32 (row-major [n_reps][d]); for a
 * cosine basis the vectors of N^d in the order of its coefficient rows. */
qr_status qr_basis_indices(const qr_basis *b, int32_t *reps_out);

/* Release a basis (and any device copies it holds). NULL is accepted. */
void qr_basis_free(qr_basis *b);

/* ---------------------------------------------------------------------- */
/* Problem description                                                     */
/* ---------------------------------------------------------------------- */
typedef enum {
    QR_F_LINEAR = 0,     /* f = h(t,x)                                     */
    QR_F_SIN = 1,        /* f = a sin(y) + h(t,x)                          */
    QR_F_ALLEN_CAHN = 2, /* f = y - y^3 + h(t,x)                           */
    QR_F_ZRAT = 3,       /* f = a |z|^2/(1+|z|^2) + y/(1+y^2) + h(t,x)     */
    QR_F_PAPER = 4       /* f = min(1, (y - u(t,x))^2) + h(t,x)            */
} qr_driver_kind;

/*
 * Semi-linear problem with a manufactured closed-form solution
 *   u(t,x) = B + A exp(-c (T - t)) cos(w.x + p),   g = u(T, .),
 * where h is the source that makes u solve eq (pde) for the chosen driver:
 *   h = -(d_t u + b.grad u + 1/2 tr(sigma sigma^T hess u)) - f_nl(u, sigma^T grad u).
 * Drift b(t,x)_l = b0_l + b1_l x_l + b2_l sin(x_l) and diffusion
 *   sigma(t,x)_{lk} = (1 + v_l cos(x_l + omega t)) sigma_{lk}
 * (sigma: d x nbm, row-major; v = sigma_v, omega = sigma_omega), which is
 * bounded, Lipschitz in x and, for |v_l| < 1 and sigma sigma^T positive
 * definite, uniformly elliptic (assumption (A_{b,sigma}), Thm "Norm-stability").
 * With b2 = v = 0 (zero-initialised fields) sigma is constant.
 * z = sigma(t_{j+1}, X_{j+1})^T grad_x ybar_{j+1} along the paths.  T = t[N].
 * clamp: level L of the truncation T_L applied to y (use INFINITY for none).
 * damping_q: damping exponent q >= 0 of eq (yqi) (at most QR_MAX_DAMPING).
 * With q > 0 the coefficients describe ybar^{(q)}_i = y_i / (1+|x|^2)^{q/2}
 * (Algorithm 1): along the paths the expansion is multiplied back by
 * (1+|x_{j+1}|^2)^{q/2} before T_L and the driver (its x-gradient by the
 * product rule), and each response is divided by (1+|X_i|^2)^{q/2};
 * qr_eval returns the expansion itself.
 * QR_F_PAPER is the driver of the paper's Sec. 5 benchmark, eq (pde2OnlyY):
 * with B = 1 + kappa, A = 1, c = lambda^2 d / 2, w = (lambda, ..., lambda)
 * and p = -pi/2, u = 1 + kappa + sin(lambda sum_l x_l) e^{lambda^2 d (t - T)/2}
 * solves the PDE with b = 0, sigma = I, h = 0 (the quadratic term vanishes on
 * u itself, and h computed from the formula above is zero up to rounding).
 * The paths read u(t_j, X_j) at the start of each step.  Only the plain FP64 entry points
 * (qr_backward_step, qr_solve, qr_solve_from in FP64, qr_path_responses)
 * take q > 0, and those and the Z regression take a non-zero b2 or v; the
 * reduced-precision, batched and learned forms return QR_ENOTSUP for either.
 * All arrays are inline; entries beyond d / nbm / N are ignored.
 */
typedef struct {
    int32_t d;                 /* 1..QR_MAX_D                               */
    int32_t nbm;               /* 1..QR_MAX_D                               */
    int32_t N;                 /* 1..QR_MAX_N                               */
    int32_t driver;            /* qr_driver_kind                            */
    double f_a;                /* driver parameter a                        */
    double clamp;              /* T_L level (> 0)                           */
    double t[QR_MAX_N + 1];    /* t_0 < t_1 < ... < t_N                     */
    double b0[QR_MAX_D];
    double b1[QR_MAX_D];
    double sigma[QR_MAX_D * QR_MAX_D]; /* [d][nbm] row-major               */
    double sol_A, sol_c, sol_p;
    double sol_w[QR_MAX_D];
    double damping_q;          /* damping exponent q >= 0 (0: none)          */
    double sol_B;              /* constant offset B of u (0 for the family)  */
    double b2[QR_MAX_D];       /* bounded drift part b2_l sin(x_l)           */
    double sigma_v[QR_MAX_D];  /* |v_l| < 1: state dependence of row l       */
    double sigma_omega;        /* time frequency omega of that dependence    */
} qr_problem;

/* ---------------------------------------------------------------------- */
/* Context                                                                 */
/* ---------------------------------------------------------------------- */
typedef struct qr_ctx qr_ctx; /* opaque, library-owned */

/* Create a context on HIP device `device`; device workspace is allocated
 * lazily and grown on demand.  QR_EDEVICE if the device is unusable. */
qr_status qr_ctx_create(int32_t device, qr_ctx **out);

/* Synchronise with the context's last stream and release all workspace. */
void qr_ctx_destroy(qr_ctx *ctx);

/* Cap the device workspace the context may hold (bytes; 0 = no cap, the
 * default).  A call whose workspace would grow past the cap returns
 * QR_ENOMEM before it allocates or launches anything; workspace already held
 * is kept.  The basis tables (per basis, not per context) are not counted. */
qr_status qr_ctx_set_mem_limit(qr_ctx *ctx, int64_t bytes);

/* Device workspace currently held by the context, in bytes. */
qr_status qr_ctx_mem_held(const qr_ctx *ctx, int64_t *bytes);

/* Enable (1) or disable (0) per-kernel timing with HIP events recorded on
 * the launch stream around every kernel the library enqueues. */
qr_status qr_ctx_set_timing(qr_ctx *ctx, int32_t enable);

/* Non-finite coefficients.  Every entry point that writes rows of alpha
 * records on the device the largest time index i whose row came out with a
 * NaN or infinite coefficient (for instance a driver that overflows along the
 * paths).  The full solves (qr_solve, qr_solve_prec, qr_solve_learned,
 * qr_solve_batched) clear the record when they start and, when their work
 * has completed (they synchronise the stream at the end), return
 * QR_ENUMERIC naming that time index.  qr_backward_step and
 * qr_backward_step_prec stay asynchronous: this call synchronises the
 * context's last stream, stores the recorded index in *step (-1 for none; step
 * may be NULL), clears it and returns QR_ENUMERIC if one was recorded. */
qr_status qr_ctx_numeric_status(qr_ctx *ctx, int32_t *step);

/* Accumulated timings (ms) and launch counts since the last reset, for
 * kernel class `which`: 0 = path simulation + expansion evaluation
 * (path kernel), 1 = projection, 2 = projection reduction, 3 = coefficient
 * gather.  Synchronises the events it reads. */
qr_status qr_ctx_kernel_time(qr_ctx *ctx, int32_t which, double *ms, int64_t *launches);
qr_status qr_ctx_reset_timing(qr_ctx *ctx);

/* ---------------------------------------------------------------------- */
/* The backward step (Algorithm 1, eqs (yqi:bar:M), (Aqi:bar:M),           */
/* (Sqi:bar:M)) and the full backward induction                            */
/* ---------------------------------------------------------------------- */

/* One backward iteration i (0 <= i < N): draws a fresh cloud of M start
 * points X_i ~ nu (stream 0), Euler-simulates each path to t_N, evaluates
 * ybar_{j+1} (rows j+1 of alpha, or g for j+1 = N) along it, accumulates
 *   S = g(X_N) + sum_{j=i}^{N-1} f(t_j, X_j, T_L(ybar_{j+1}(X_{j+1})), z_{j+1}) (t_{j+1}-t_j)
 * and writes row i of alpha with (1/M) sum_m S_m phi_k(X_i^m).
 * alpha: device, [N][n_funcs] canonical order; rows i+1..N-1 are read,
 * row i is written.  1 <= M <= 2^31 - 1. */
qr_status qr_backward_step(qr_ctx *ctx, const qr_problem *prob, const qr_basis *basis, int32_t i,
                           int64_t M, uint64_t seed, double *alpha, void *stream);

/* Full backward induction i = N-1, ..., 0 (all rows of alpha written).
 * Bit for bit the same rows as qr_backward_step called for i = N-1, ..., 0
 * on one alpha table. */
qr_status qr_solve(qr_ctx *ctx, const qr_problem *prob, const qr_basis *basis, int64_t M,
                   uint64_t seed, double *alpha, void *stream);

/* Resume a backward induction (Algorithm 1) at time index i_start
 * (0 <= i_start < N): rows i_start+1..N-1 of alpha are read as saved from an
 * earlier run, rows i_start..0 are written.  `precision` as in qr_solve_prec.
 * With the same problem, basis, M, seed, precision and reduced-precision
 * kernel, the rows written equal those of the uninterrupted solve bit for
 * bit (qr_solve and qr_solve_prec are this call with i_start = N-1). */
qr_status qr_solve_from(qr_ctx *ctx, const qr_problem *prob, const qr_basis *basis, int32_t i_start,
                        int64_t M, uint64_t seed, int32_t precision, double *alpha, void *stream);

/* Schemes of the Z regression (Sec. 1). */
typedef enum {
    QR_Z_MULTISTEP = 0, /* eq (MDP:intro:0a): R_m = S_m without its term j = i */
    QR_Z_ONESTEP = 1    /* eq (ODP:intro:a): R_m = T_L(ybar_{i+1}(X_{i+1})) - T_L(ybar_{i+1}(X_i)) */
} qr_z_scheme;

/* The backward step with the gradient component: the regression of Z_i
 * beside that of Y_i, eq (MDP:intro:0b).  Row i of alpha is written exactly
 * as qr_backward_step writes it, and for each Brownian component k < nbm
 *   alpha_z[i][k][.] = (1/M) sum_m R_m (W^k_{i+1} - W^k_i)_m / Delta_i phi_.(X_i^m),
 * where the increment is the one the path took on its first step (the
 * normal r = d + k of stream 0 at time index i, times sqrt(Delta_i)) and the
 * response R_m is, by `scheme`:
 *   QR_Z_MULTISTEP: S_m of the step without its term j = i, eq (MDP:intro:0a);
 *     the Monte-Carlo variance carries the whole remaining path and grows as
 *     1/Delta_i;
 *   QR_Z_ONESTEP: the value the driver read on the path's first step,
 *     T_L(ybar_{i+1}(X_{i+1})) (ybar_N = g), less T_L(ybar_{i+1}(X_i)), eq
 *     (ODP:intro:a); the subtracted term is a function of X_i and leaves the
 *     conditional expectation unchanged, and for a smooth ybar_{i+1} the
 *     variance is of order one.  One more evaluation of ybar_{i+1} per path.
 * Z_i(x) is then sum alpha_z[i][k][.] phi_.(x) (qr_eval on that row), an
 * estimate of sigma^T grad u(t_i, x).
 * alpha_z: device [N][nbm][n_funcs] canonical order; slice i is written.
 * FP64, Fourier basis and q = 0 only (QR_ENOTSUP otherwise); an unknown
 * scheme is QR_EINVAL; other arguments and errors as in qr_backward_step. */
qr_status qr_backward_step_z(qr_ctx *ctx, const qr_problem *prob, const qr_basis *basis, int32_t i,
                             int64_t M, uint64_t seed, int32_t scheme, double *alpha, double *alpha_z,
                             void *stream);

/* qr_backward_step_z for i = N-1, ..., 0: alpha equals qr_solve's bit for
 * bit and every slice of alpha_z is written. */
qr_status qr_solve_z(qr_ctx *ctx, const qr_problem *prob, const qr_basis *basis, int64_t M,
                     uint64_t seed, int32_t scheme, double *alpha, double *alpha_z, void *stream);

/* Evaluate ybar = sum_k alpha_k phi_k at n points, phi_k = (Fourier
 * function) o F of the basis's sampling law (with a damping exponent q > 0
 * the caller multiplies by (1+|x|^2)^{q/2} to obtain y).
 * alpha_row: device [n_funcs] canonical order; x: device SoA [d][n];
 * y: device [n]; grad: device SoA [d][n] receiving grad_x ybar, or NULL. */
qr_status qr_eval(qr_ctx *ctx, const qr_basis *basis, const double *alpha_row, int64_t n,
                  const double *x, double *y, double *grad, void *stream);

/* qr_eval (values only) for point sets too small to fill the device one
 * walk per thread, as the learned form's training pairs are: the basis is
 * split across blocks (the projection's tasks), each block sums its tasks'
 * terms for a slice of the points, and the blocks' sums are added in a fixed
 * order.  Same values as qr_eval up to the order of the additions.
 * 0 <= n <= 2^17 (QR_EINVAL otherwise); Fourier basis only (QR_ENOTSUP).
 * Workspace: 16 d n bytes of phase factors and 8 n ceil(tasks / 8) bytes of
 * group sums, held by the context. */
qr_status qr_eval_split(qr_ctx *ctx, const qr_basis *basis, const double *alpha_row, int64_t n,
                        const double *x, double *y, void *stream);

/* The prediction y_i of the problem at n points from its row of
 * coefficients: qr_eval, times (1+|x|^2)^{q/2} for the problem's damping
 * exponent q (eq (yqi)), with the gradient by the product rule,
 * D (grad ybar + ybar q x / (1+|x|^2)).  Arguments as in qr_eval; with
 * q = 0 it is qr_eval. */
qr_status qr_eval_y(qr_ctx *ctx, const qr_problem *prob, const qr_basis *basis, const double *alpha_row,
                    int64_t n, const double *x, double *y, double *grad, void *stream);

/* ---------------------------------------------------------------------- */
/* Evaluation without allocation                                           */
/* ---------------------------------------------------------------------- */

/* Largest coefficient-row staging of qr_eval_noalloc, in 16-byte entries
 * (8 MiB per GPU, held from the first qr_ctx_create on that GPU until the
 * process ends).  A basis of R representatives needs 64 (ceil(R/64) + 2)
 * entries, so R <= 524,160. */
#define QR_NOALLOC_ROW_MAX (1 << 19)

/* Upload the basis tables to the context's device now (the set-up call of
 * qr_eval_noalloc; any other entry point does it on first use).  May
 * allocate device memory, once per basis and device. */
qr_status qr_basis_upload(qr_ctx *ctx, const qr_basis *basis);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): qr_eval with the same arguments,
 * outputs and kernels, that calls no allocating routine.  Its only scratch,
 * the coefficient row in the kernels' layout, is a fixed device array of
 * QR_NOALLOC_ROW_MAX entries per GPU (QR_ERANGE for a larger basis); the
 * basis must already be resident on the context's device (qr_basis_upload;
 * QR_EINVAL otherwise).  Every call on a GPU uses that GPU's one array, and
 * each call rewrites all of it that it reads: calls that overlap on one GPU
 * (two host threads, or two streams not ordered with each other) race. */
qr_status qr_eval_noalloc(qr_ctx *ctx, const qr_basis *basis, const double *alpha_row, int64_t n,
                          const double *x, double *y, double *grad, void *stream);

/* ---------------------------------------------------------------------- */
/* Pieces of the step, exposed for testing and for callers that supply    */
/* their own samples                                                       */
/* ---------------------------------------------------------------------- */

/* Projection alone (eq (Aqi:bar:M) on given samples):
 * alpha_row[k] = (1/n) sum_p s_p phi_k(x_p), phi_k of the basis's law.
 * x: device SoA [d][n]; s: device [n]; alpha_row: device [n_funcs]. */
qr_status qr_project(qr_ctx *ctx, const qr_basis *basis, int64_t n, const double *x,
                     const double *s, double *alpha_row, void *stream);

/* Path simulation and responses alone: writes S_m (eq (Sqi:bar:M)) for
 * m = 0..M-1 of step i into s (device [M]) and, if x0 is not NULL, the start
 * points X_i^m into x0 (device SoA [d][M]).  alpha as in qr_backward_step. */
qr_status qr_path_responses(qr_ctx *ctx, const qr_problem *prob, const qr_basis *basis, int32_t i,
                            int64_t M, uint64_t seed, const double *alpha, double *s, double *x0,
                            void *stream);

/* nu-distributed points of stream `stream_id` at time index i:
 * x[l][m] = F^{-1}(U(seed, stream_id, m0 + m, i, l)), device SoA [d][n]. */
qr_status qr_sample_points(qr_ctx *ctx, int32_t d, uint64_t seed, uint32_t stream_id, int32_t i,
                           int64_t m0, int64_t n, double *x, void *stream);

/* As qr_sample_points, with F^{-1} of the law `law` (qr_law) instead of the
 * logistic law's. */
qr_status qr_sample_points_law(qr_ctx *ctx, int32_t law, int32_t d, uint64_t seed, uint32_t stream_id,
                               int32_t i, int64_t m0, int64_t n, double *x, void *stream);

/* ---------------------------------------------------------------------- */
/* Reduced-precision form                                                  */
/* ---------------------------------------------------------------------- */

/* Arithmetic of the expansion evaluation along the paths (eq (yqi:bar:M)).
 * QR_PREC_F64: everything in FP64 (qr_solve).  QR_PREC_BF16 / QR_PREC_F16:
 * phase reduction F(x) -> e^{2 pi i u} in FP64, the basis walk in FP32, basis
 * values and coefficients rounded to 16 bits (bfloat16 or IEEE half) and
 * contracted on the matrix cores with FP32 accumulation; for drivers that
 * depend on z the d gradient components are further right-hand sides of the
 * same contraction.  The path simulation, driver sum, projection and alpha
 * reduction stay FP64. */
typedef enum { QR_PREC_F64 = 0, QR_PREC_BF16 = 1, QR_PREC_F16 = 2 } qr_precision;

/* Kernel of the reduced-precision form (qr_ctx_set_prec_kernel).
 *  QR_PREC_KERNEL_WALK: the basis traversal of the FP64 path in FP32, each
 *    basis value rounded to 16 bits and contracted with the coefficients on
 *    the matrix cores (value and gradient right-hand sides).
 *  QR_PREC_KERNEL_FACTORED: the coordinates are split in two blocks A | B;
 *    every representative is (kA, kB), so the expansion at a point is
 *    Re sum_kA e^{2 pi i kA.uA} sum_kB beta(kA,kB) e^{2 pi i kB.uB} with
 *    beta = sqrt2 (a_c - i a_s) (beta = alpha_0 for the constant).  Over a tile
 *    of paths the inner sums are a product of the staircase matrix beta with
 *    the paths' e^{2 pi i kB.uB} values, run on the matrix cores with 16-bit
 *    operands and FP32 accumulation; the factors e^{2 pi i m u_l} come from
 *    per-path tables (phase in FP64, stored FP32).  Drivers that depend on z
 *    are not supported (QR_ENOTSUP when forced).
 *  QR_PREC_KERNEL_AUTO (default): the factored kernel where it applies, the
 *    walk otherwise. */
typedef enum {
    QR_PREC_KERNEL_AUTO = 0,
    QR_PREC_KERNEL_WALK = 1,
    QR_PREC_KERNEL_FACTORED = 2
} qr_prec_kernel;

/* Choose the kernel of the reduced-precision entry points of this context
 * (qr_prec_kernel; QR_EINVAL if unknown). */
qr_status qr_ctx_set_prec_kernel(qr_ctx *ctx, int32_t kind);

/* The factored layout of a basis (host only; built on first use): the split
 * dA (the first dA coordinates form block A), the row tiles of 8 A-parts, the
 * K-blocks of 16 B-parts over all B-parts, and the 16-bit coefficient blocks
 * per time step (64 lanes x 16 bytes each).  Any output may be NULL;
 * QR_ENOTSUP if no split qualifies. */
qr_status qr_basis_factored(const qr_basis *basis, int32_t *split, int32_t *n_row_tiles,
                            int32_t *n_kblocks, int64_t *n_blocks);

/* qr_backward_step / qr_solve with the expansion evaluation in `precision`.
 * Arguments and outputs as there; QR_PREC_F64 is the plain path. */
qr_status qr_backward_step_prec(qr_ctx *ctx, const qr_problem *prob, const qr_basis *basis,
                                int32_t i, int64_t M, uint64_t seed, int32_t precision,
                                double *alpha, void *stream);
qr_status qr_solve_prec(qr_ctx *ctx, const qr_problem *prob, const qr_basis *basis, int64_t M,
                        uint64_t seed, int32_t precision, double *alpha, void *stream);

/* ---------------------------------------------------------------------- */
/* Learned form: a network surrogate of ybar_j per time index              */
/* ---------------------------------------------------------------------- */

/* The surrogate (not part of the paper's method): features f in R^16 ->
 * h1 = silu(W1 f + b1) (256) -> h2 = silu(W2 h1 + b2) (256) -> w3 . h2 + b3,
 * silu(z) = z / (1 + e^-z).  Parameters: one FP32 vector, blocks in the order
 * W1 [256][16] (row = output unit), b1 [256], W2 [256][256], b2 [256],
 * w3 [256], b3 [1].  Products run on the matrix cores with bfloat16 operands
 * and FP32 accumulation.  Features of a state x: 2 F(x_l) - 1 for l < d and
 * 0 up to 16 (d <= 16), F of the basis's sampling law in qr_solve_learned and
 * of the logistic law in qr_mlp_features. */
#define QR_MLP_IN 16
#define QR_MLP_HIDDEN 256
#define QR_MLP_NPARAMS (QR_MLP_HIDDEN * QR_MLP_IN + QR_MLP_HIDDEN + QR_MLP_HIDDEN * QR_MLP_HIDDEN + \
                        QR_MLP_HIDDEN + QR_MLP_HIDDEN + 1)
#define QR_MLP_MAX_BATCH 65536

/* Fan-in uniform initialisation (biases 0) from Philox stream 2 of seed.
 * params: device [QR_MLP_NPARAMS]. */
qr_status qr_mlp_init(qr_ctx *ctx, float *params, uint64_t seed, void *stream);
/* feat[p][l] (device [n][16]) from x (device SoA [d][n]), 1 <= d <= 16. */
qr_status qr_mlp_features(qr_ctx *ctx, int32_t d, int64_t n, const double *x, float *feat, void *stream);
/* y[p] (device [n]) = network(feat[p]); any n >= 0 (processed in chunks). */
qr_status qr_mlp_forward(qr_ctx *ctx, const float *params, int64_t n, const float *feat, float *y,
                         void *stream);
/* Mean squared error over n <= QR_MLP_MAX_BATCH pairs and its gradient:
 * grad (device [QR_MLP_NPARAMS]) is overwritten, *loss (host) receives the
 * loss after the stream has completed the work. */
qr_status qr_mlp_loss_grad(qr_ctx *ctx, const float *params, int64_t n, const float *feat,
                           const float *target, float *grad, double *loss, void *stream);
/* One bias-corrected Adam step (beta1 0.9, beta2 0.999, eps 1e-8) number
 * `step` >= 1 on device vectors params, m, v given grad. */
qr_status qr_mlp_adam(qr_ctx *ctx, float *params, const float *grad, float *m, float *v, int64_t step,
                      float lr, void *stream);

typedef struct {
    int64_t train_points;   /* pairs (X, ybar_j(X)) per time index, X from stream 2 */
    int64_t heldout_points; /* held-out pairs, X from stream 3 */
    int32_t epochs;         /* passes over the training pairs */
    int32_t batch;          /* pairs per Adam step, <= QR_MLP_MAX_BATCH */
    float lr;               /* Adam step size */
    double gate;            /* use the surrogate iff its held-out relative L2 error <= gate */
    double reject;          /* > 0: screen each time index first: the fit on the first
                               1/32 of the training and held-out pairs, all epochs, ended as
                               soon as its held-out error is <= reject; a screen still above
                               reject after its last epoch ends the time index (no full fit,
                               no surrogate); 0: always run the full fit */
} qr_learn_opts;

typedef struct {
    double heldout_rel_l2;  /* ||surrogate - ybar_j|| / ||ybar_j|| on the held-out points */
    double train_loss;      /* mean squared error of the last epoch (normalised targets) */
    int32_t trained;        /* a surrogate was fitted for this time index */
    int32_t used;           /* it replaced the expansion along the paths */
    double target_mean;     /* the surrogate predicts (ybar_j - target_mean) / target_sd */
    double target_sd;
    int32_t epochs_run;     /* epochs of the last fit run (the screen's after a rejection) */
} qr_learn_report;

/* qr_solve (the driver must not depend on z) where, after row j of alpha is
 * known (1 <= j <= N-1), a surrogate of ybar_j is fitted on the method's own
 * pairs and, if it passes the gate, evaluated along the paths instead of
 * the |Gamma|-term expansion (ybar_j = target_mean + target_sd * network);
 * otherwise the expansion is used (and is the result).  report: host [N],
 * entry j for time index j.  params: device [N][QR_MLP_NPARAMS] receiving
 * the fitted parameters of every time index (zero where none was fitted),
 * or NULL.  The surrogate only changes how ybar_j is evaluated at X_j; the
 * path simulation, projection and alpha reduction are those of qr_solve, and
 * an iteration i whose later time indices all use the expansion runs
 * qr_solve's own kernels. */
qr_status qr_solve_learned(qr_ctx *ctx, const qr_problem *prob, const qr_basis *basis, int64_t M,
                           uint64_t seed, const qr_learn_opts *opts, double *alpha,
                           qr_learn_report *report, float *params, void *stream);

/* ---------------------------------------------------------------------- */
/* Batched form: several PDE instances solved on one shared cloud          */
/* ---------------------------------------------------------------------- */

#define QR_MAX_BATCH 64

/* One instance of a batch.  The paths of a decoupled FBSDE do not depend on
 * the driver or the terminal condition (eqs (fbsde), (eds)), so instances
 * that share d, nbm, the time grid, b, sigma, the sampling law and the seed
 * can share one cloud of start points and Euler paths.  Instance r uses
 *   - its own driver parameter f_a (the problem's driver kind),
 *   - the first d coordinates only (1 <= d <= problem d; its solution must
 *     not depend on the others),
 *   - the index set of the basis' kind at its own level (<= basis level,
 *     >= 1 for the hyperbolic crosses) restricted to vectors supported on
 *     those d coordinates,
 *   - the first M paths of the shared cloud (1 <= M <= the cloud size).
 * Its coefficients equal those of qr_solve for the problem with that f_a, on
 * that index set (embedded in the problem's d coordinates) and that M, up to
 * summation order. */
typedef struct {
    double f_a;
    int32_t d;
    int32_t level;
    int64_t M;
} qr_instance;

/* Solve R (1 <= R <= QR_MAX_BATCH) instances on one cloud of max_r M_r
 * paths.  alpha: device [R][N][n_funcs] (canonical order); coefficients of
 * functions outside an instance's index set are written as 0.  The driver
 * must not depend on z (QR_ENOTSUP otherwise).  inst: host array of R. */
qr_status qr_solve_batched(qr_ctx *ctx, const qr_problem *prob, const qr_basis *basis, int32_t R,
                           const qr_instance *inst, uint64_t seed, double *alpha, void *stream);

/* The batched solve as one HIP graph, for callers that repeat it (the same
 * instances and seed on new data in the same buffers, or serving loops):
 * qr_batch_graph_create plans the solve like qr_solve_batched, allocates the
 * device buffers it needs as the graph's own (so later calls on the context
 * cannot move them), runs the solve once on `stream` (alpha then holds its
 * result) and captures every launch of it into a graph; each
 * qr_batch_graph_launch replays the whole backward induction of every pass
 * with one launch, writing alpha again.  `stream` must not be the null
 * stream.  The graph reads the basis's device tables and the context's
 * non-finite record (qr_ctx_numeric_status reports a replay's rows): the
 * basis and the context must outlive it, and the basis must stay on the
 * context's device.  qr_batch_graph_destroy synchronises the device and
 * frees the graph and its buffers (NULL is accepted). */
typedef struct qr_batch_graph qr_batch_graph; /* opaque, library-owned */
qr_status qr_batch_graph_create(qr_ctx *ctx, const qr_problem *prob, const qr_basis *basis, int32_t R,
                                const qr_instance *inst, uint64_t seed, double *alpha, void *stream,
                                qr_batch_graph **out);
qr_status qr_batch_graph_launch(qr_batch_graph *graph, void *stream);
void qr_batch_graph_destroy(qr_batch_graph *graph);

/* Host-side copies of the scalar device routines, for unit tests on
 * machines without a GPU.  qr_host_uniform follows the stream layout above;
 * qr_host_norm_icdf is the device inverse normal CDF (Wichura's AS241,
 * PPND16); qr_host_philox writes the 4 output words for a counter / key. */
double qr_host_uniform(uint64_t seed, uint32_t stream_id, uint64_t m, uint32_t i, uint32_t r);
double qr_host_norm_icdf(double u);
void qr_host_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

#ifdef __cplusplus
}
#endif
#endif /* QRMC_H */
