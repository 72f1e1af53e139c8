/*
 * qrmc_oracle.c -- plain FP64 CPU oracle for the quasi-regression Monte-Carlo
 * (QRMC) scheme of Gobet, Lopez-Salas and Vazquez (arXiv 2407.21084).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file: it exists so that tests, the smoke check and the CPU-baseline
 * leg of the benchmark can check the GPU library against an independent,
 * obviously-correct implementation.  It shares no code, header, table or
 * constant generator with the HIP library; both sides only consume the same
 * counter-based random streams, each implementing the published Philox4x32-10
 * generator on its own.
 *
 * Everything is written for clarity, not speed: every basis function is
 * evaluated directly with libm cos/sin of its own phase, sums over Monte-Carlo
 * samples run in sample order with Neumaier compensation, and the only
 * parallelism (OpenMP) is over independent paths or independent coefficients,
 * so results do not depend on the thread count.
 *
 * Paper passages followed (section / equation / algorithm names of the paper):
 *   - decoupled FBSDE and semi-linear PDE: Sec. 1, eqs (fbsde), (eds), (pde)
 *   - multistep dynamic programming equation: Sec. 2.1.1, eq (MDP:fcs)
 *   - Euler scheme of X from a randomised start X_i ~ nu: eq (markov:euler),
 *     assumption (A_nu)
 *   - orthonormal basis phi_k = C_k o F_nu: Sec. 2.2, Lemma 2.1, eqs (relation:1/2)
 *   - GQRMDP Algorithm 1: eqs (yqi:bar:M), (Aqi:bar:M), (Sqi:bar:M), damping q = 0
 *   - soft truncation T_L: notation (vi) of Sec. 1
 *   - index sets Gamma_F / Gamma_H: Sec. 2.3.3 "Multi-indices sets"
 *   - error indicators MSE_max / MSE_av: Sec. 5, eq (mse)
 *   - Z by Brownian-weight regression: Sec. 1, eqs (MDP:intro:0a) (multistep)
 *     and (ODP:intro:a) (one step)
 *   - state-dependent drift and diffusion: assumption (A_{b,sigma})
 *
 * Where the problem statement used here departs from the paper's own
 * experiments (sampling law, basis, index sets, driver, random generator),
 * it is read as follows:
 *   - nu is a product of identical one-dimensional laws, chosen per problem:
 *     the standard logistic law F(x) = 1/(1+e^-x), or one of the paper's
 *     own two (Sec. 5): Student's t with mu = 2 in the scaling of Example
 *     "Student's t-distribution" (density 0.5 (1+x^2)^{-3/2}) and its mu = 1
 *     case, the Cauchy law (density 1/(pi (1+x^2)));
 *   - the basis is the real Fourier basis on the torus composed with F:
 *     phi_0 = 1, and for each representative k (first non-zero coordinate
 *     positive) sqrt2 cos(2 pi k.F(x)) and sqrt2 sin(2 pi k.F(x));
 *   - index sets are taken over Z^d, symmetric in each coordinate;
 *   - the driver may depend on z = sigma^T grad y (explicit: evaluated at
 *     X_{j+1} together with y);
 *   - a damping exponent q >= 0 (eq (yqi)): the expansions approximate
 *     y_i / (1+|x|^2)^{q/2}; q = 0 gives y_i itself.  The factor on the y
 *     handed to the driver, the division of the response and the projection
 *     target are each pinned (Lemma 3.1 with Gaussian moments, an exact
 *     identity, Lemma 3.1 by quadrature);
 *   - a constant truncation level L;
 *   - the paper's own variant is also available: its cosine basis on N^d
 *     (Lemma 2.1, eq (phi:dim:d)) over the sets Gamma_F, Gamma_H and Gamma_T
 *     of Sec. 2.3.3, and the driver of its Sec. 5 benchmark, eq (pde2OnlyY),
 *     f = min(1, (y - u(t,x))^2) with u = 1 + kappa + sin(lambda sum x)
 *     e^{lambda^2 d (t-T)/2} (the family B + A e^{-c(T-t)} cos(w.x + p)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXD 16
#define OR_MAXN 256

/* ------------------------------------------------------------------------ */
/* Problem description (the oracle's own struct; mirrored by oracle/__init__.py) */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t d;        /* state dimension                                   */
    int32_t nbm;      /* Brownian dimension                                */
    int32_t N;        /* number of time steps                              */
    int32_t driver;   /* 0: f=h, 1: a sin y + h, 2: y - y^3 + h,
                         3: a|z|^2/(1+|z|^2) + y/(1+y^2) + h,
                         4: min(1, (y - u(t,x))^2) + h (Sec. 5)            */
    int32_t nu;       /* sampling law: 0 logistic, 1 Student mu=2, 2 Cauchy  */
    double f_a;       /* driver parameter a                                */
    double clamp;     /* truncation level L of T_L (INFINITY: none)        */
    double t[OR_MAXN + 1];          /* time grid t_0 < ... < t_N           */
    double b0[OR_MAXD], b1[OR_MAXD];/* drift b(t,x)_l = b0_l + b1_l x_l + b2_l sin x_l */
    double sigma[OR_MAXD * OR_MAXD];/* diffusion sigma(t,x)_lk = (1 + v_l cos(x_l + omega t)) sigma_lk, d x nbm, row-major */
    double sol_A, sol_c, sol_p;     /* u(t,x) = B + A e^{-c(T-t)} cos(w.x+p) */
    double sol_w[OR_MAXD];
    double damping_q;               /* damping exponent q >= 0 (eq (yqi))  */
    double sol_B;                   /* constant offset B of u              */
    int32_t basis;                  /* 0: Fourier on Z^d, 1: cosine on N^d */
    double b2[OR_MAXD];             /* bounded drift part                  */
    double sigma_v[OR_MAXD];        /* state dependence v_l of sigma's row l */
    double sigma_omega;             /* its time frequency omega            */
} or_problem;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from the      */
/* published definition: 10 rounds of two 32x32->64 multiplications with    */
/* the constants 0xD2511F53 / 0xCD9E8D57 and a Weyl key schedule with       */
/* increments 0x9E3779B9 / 0xBB67AE85.                                      */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/*
 * Stream layout (a reading: the paper uses an inline MRG32k3a, Sec. 4).
 * Draw number r of sample m at time index i in stream s:
 *   key     = (seed_lo, seed_hi XOR s)
 *   counter = (m_lo, m_hi, i, r >> 1)
 *   words   = (w0, w1) if r even, (w2, w3) if r odd
 *   n       = (w_first << 20) | (w_second >> 12)      (52 bits)
 *   U       = (n + 1/2) * 2^-52                       (exact, in (0,1))
 */
double or_uniform(uint64_t seed, uint32_t stream, uint64_t m, uint32_t i, uint32_t r)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ stream};
    uint32_t ctr[4] = {(uint32_t)m, (uint32_t)(m >> 32), i, r >> 1};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    uint32_t a = (r & 1u) ? w[2] : w[0];
    uint32_t b = (r & 1u) ? w[3] : w[1];
    uint64_t n = ((uint64_t)a << 20) | (uint64_t)(b >> 12);
    return ((double)n + 0.5) * 0x1p-52;
}

/* ------------------------------------------------------------------------ */
/* Laws                                                                      */
/* ------------------------------------------------------------------------ */

/* Standard normal CDF through the complementary error function. */
static double or_norm_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/* Lower-tail normal quantile for q in (0, 1/2]: a rough rational start
 * (Abramowitz & Stegun 26.2.23, |error| < 4.5e-4) refined by Halley steps on
 * Phi(x) - q = 0, using Phi' = pdf and Phi'' = -x pdf. */
static double or_norm_lower_quantile(double q)
{
    double t = sqrt(-2.0 * log(q));
    double x = -(t - (2.515517 + 0.802853 * t + 0.010328 * t * t) /
                     (1.0 + 1.432788 * t + 0.189269 * t * t + 0.001308 * t * t * t));
    for (int it = 0; it < 4; ++it) {
        double f = or_norm_cdf(x) - q;
        double pdf = exp(-0.5 * x * x) / sqrt(2.0 * M_PI);
        double e = f / pdf;
        x = x - e / (1.0 + 0.5 * x * e);
    }
    return x;
}

/* Inverse standard normal CDF.  For u > 1/2 the symmetric lower tail of 1-u
 * is used (1-u is exact for the uniforms produced above). */
double or_norm_icdf(double u)
{
    if (u == 0.5) return 0.0;
    if (u < 0.5) return or_norm_lower_quantile(u);
    return -or_norm_lower_quantile(1.0 - u);
}

/* Standard logistic law: F(x) = 1/(1+e^{-x}), F^{-1}(u) = ln u - ln(1-u). */
double or_logistic_cdf(double x) { return 1.0 / (1.0 + exp(-x)); }
double or_logistic_icdf(double u) { return log(u) - log(1.0 - u); }

/* The one-dimensional marginal nu_l of the sampling law (assumption (A_nu)),
 * its CDF F and inverse, as functions of the law's code:
 *   0: standard logistic, density F (1 - F);
 *   1: Student's t with mu = 2 scaled as in Example "Student's
 *      t-distribution" (density c_mu (1+x^2)^{-(mu+1)/2}, c_2 = 1/2), whose F
 *      and F^{-1} are given in closed form in Sec. 5, eq (Fnui:Fnulinv):
 *      F(x) = (x / sqrt(x^2+1) + 1) / 2, F^{-1}(u) = (u - 1/2) / sqrt(u (1-u));
 *   2: the mu = 1 case, the Cauchy law of Sec. 5: density 1/(pi (1+x^2)),
 *      F(x) = 1/2 + atan(x)/pi, F^{-1}(u) = tan(pi (u - 1/2)) = -cot(pi u). */
double or_law_cdf(int nu, double x)
{
    switch (nu) {
    case 0: return or_logistic_cdf(x);
    case 1: return 0.5 * (x / sqrt(x * x + 1.0) + 1.0);
    case 2: return 0.5 + atan(x) / M_PI;
    }
    return NAN;
}

double or_law_icdf(int nu, double u)
{
    switch (nu) {
    case 0: return or_logistic_icdf(u);
    case 1: return (u - 0.5) / sqrt(u * (1.0 - u));
    /* tan(pi (u - 1/2)) = -cot(pi u), evaluated away from the pole: near
     * u = 0 or 1 the product pi (u - 1/2) would lose the small distance to
     * -+pi/2 to rounding */
    case 2: return u < 0.5 ? -1.0 / tan(M_PI * u) : 1.0 / tan(M_PI * (1.0 - u));
    }
    return NAN;
}

double or_law_pdf(int nu, double x)
{
    switch (nu) {
    case 0: { double F = or_logistic_cdf(x); return F * (1.0 - F); }
    case 1: return 0.5 * pow(1.0 + x * x, -1.5);
    case 2: return 1.0 / (M_PI * (1.0 + x * x));
    }
    return NAN;
}

/* ------------------------------------------------------------------------ */
/* Index sets (Sec. 2.3.3), taken over Z^d (or N^d when nonneg != 0).       */
/*   kind 0: tensor      max_l |k_l| <= level                               */
/*   kind 1: hyperbolic  prod_l max(1,|k_l|) <= level                       */
/*   kind 2: hyperbolic  prod_l (1+|k_l|) <= level                          */
/*   kind 3: total degree sum_l |k_l| <= level                              */
/* The enumeration walks coordinates in order with values ascending, so the */
/* output is in lexicographic order of the integer vectors.                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    int d, kind, level, nonneg, reps_only;
    int32_t *out;
    int64_t cap, count;
    int32_t cur[OR_MAXD];
} or_enum_state;

/* Can the partial vector cur[0..upto) still be completed inside the set?
 * (Zero coordinates never increase any of the four measures.) */
static int or_partial_ok(const or_enum_state *s, int upto)
{
    long long acc = (s->kind == 1 || s->kind == 2) ? 1 : 0;
    for (int l = 0; l < upto; ++l) {
        long long a = s->cur[l] < 0 ? -(long long)s->cur[l] : s->cur[l];
        switch (s->kind) {
        case 0: if (a > s->level) return 0; break;
        case 1: acc *= (a > 1 ? a : 1); if (acc > s->level) return 0; break;
        case 2: acc *= (1 + a); if (acc > s->level) return 0; break;
        case 3: acc += a; if (acc > s->level) return 0; break;
        }
    }
    return 1;
}

static int or_is_representative(const int32_t *k, int d)
{
    for (int l = 0; l < d; ++l) {
        if (k[l] > 0) return 1;
        if (k[l] < 0) return 0;
    }
    return 1; /* the zero vector */
}

static void or_enum_rec(or_enum_state *s, int l)
{
    if (l == s->d) {
        if (s->reps_only && !or_is_representative(s->cur, s->d)) return;
        if (s->out && s->count < s->cap)
            memcpy(s->out + s->count * s->d, s->cur, sizeof(int32_t) * s->d);
        s->count++;
        return;
    }
    int lo = s->nonneg ? 0 : -s->level;
    for (int v = lo; v <= s->level; ++v) {
        s->cur[l] = v;
        if (!or_partial_ok(s, l + 1)) continue;
        or_enum_rec(s, l + 1);
    }
    s->cur[l] = 0;
}

/* Enumerate the set.  reps_only=1 keeps only the representatives of
 * {k,-k} (first non-zero coordinate positive, plus the zero vector).
 * Writes up to cap vectors (row-major [count][d]) and returns the count,
 * or -1 on invalid arguments. */
int64_t or_enumerate(int d, int kind, int level, int nonneg, int reps_only,
                     int32_t *out, int64_t cap)
{
    if (d < 1 || d > OR_MAXD || kind < 0 || kind > 3 || level < 0) return -1;
    or_enum_state s;
    memset(&s, 0, sizeof s);
    s.d = d; s.kind = kind; s.level = level; s.nonneg = nonneg;
    s.reps_only = reps_only; s.out = out; s.cap = cap;
    or_enum_rec(&s, 0);
    return s.count;
}

/* ------------------------------------------------------------------------ */
/* Basis functions (Lemma 2.1 / eq (relation:1) with the Fourier basis).    */
/* Real index 0 = 1; representative r >= 1 gives index 2r-1 = sqrt2 cos and */
/* index 2r = sqrt2 sin of 2 pi k_r . F(x).                                  */
/* ------------------------------------------------------------------------ */

/* Phase k.u reduced to [-1/2, 1/2]. */
static double or_phase(const int32_t *k, const double *u, int d)
{
    double th = 0.0;
    for (int l = 0; l < d; ++l) th += (double)k[l] * u[l];
    return th - rint(th);
}

/* The paper's cosine basis on N^d (Lemma 2.1 and the tensor products of
 * eq (phi:dim:d)): phi_k(x) = prod_l c_{k_l}(F(x_l)), c_0 = 1,
 * c_m(u) = sqrt2 cos(m pi u).  One function per vector k (reps holds all of
 * the set, lexicographic). */
static double or_cos_factor(int m, double u) { return m == 0 ? 1.0 : sqrt(2.0) * cos((double)m * M_PI * u); }

static double or_cos_value(const int32_t *k, const double *u, int d)
{
    double v = 1.0;
    for (int l = 0; l < d; ++l) v *= or_cos_factor(k[l], u[l]);
    return v;
}

/* number of basis functions of a set of nrep vectors */
static int64_t or_nfuncs_of(int basis, int64_t nrep) { return basis == 1 ? nrep : 2 * nrep - 1; }

void or_basis_values(int d, int nu, int basis, int64_t nrep, const int32_t *reps, const double *x, double *phi)
{
    double u[OR_MAXD];
    for (int l = 0; l < d; ++l) u[l] = or_law_cdf(nu, x[l]);
    if (basis == 1) {
        for (int64_t r = 0; r < nrep; ++r) phi[r] = or_cos_value(reps + r * d, u, d);
        return;
    }
    phi[0] = 1.0;
    for (int64_t r = 1; r < nrep; ++r) {
        double th = 2.0 * M_PI * or_phase(reps + r * d, u, d);
        phi[2 * r - 1] = sqrt(2.0) * cos(th);
        phi[2 * r] = sqrt(2.0) * sin(th);
    }
}

/* Expansion ybar(x) = sum_k alpha_k phi_k(x) (eq (yqi:bar:M)) and, when
 * grad != NULL, its x-gradient by the chain rule through F (dF/dx = nu_l).
 * The sum runs in basis order with Neumaier compensation. */
static double or_expansion_cos(int d, int nu, int64_t nrep, const int32_t *reps, const double *alpha,
                               const double *x, double *grad);

static double or_expansion(int d, int nu, int basis, int64_t nrep, const int32_t *reps, const double *alpha,
                           const double *x, double *grad)
{
    if (basis == 1) return or_expansion_cos(d, nu, nrep, reps, alpha, x, grad);
    double u[OR_MAXD], dudx[OR_MAXD];
    for (int l = 0; l < d; ++l) {
        u[l] = or_law_cdf(nu, x[l]);
        dudx[l] = or_law_pdf(nu, x[l]);
    }
    double s = alpha[0], c = 0.0;
    double gs[OR_MAXD], gc[OR_MAXD];
    for (int l = 0; l < d; ++l) { gs[l] = 0.0; gc[l] = 0.0; }
    for (int64_t r = 1; r < nrep; ++r) {
        const int32_t *k = reps + r * d;
        double th = 2.0 * M_PI * or_phase(k, u, d);
        double ct = cos(th), st = sin(th);
        double term = sqrt(2.0) * (alpha[2 * r - 1] * ct + alpha[2 * r] * st);
        double t = s + term;
        c += (fabs(s) >= fabs(term)) ? (s - t) + term : (term - t) + s;
        s = t;
        if (grad) {
            /* d/du_l of sqrt2 (a cos th + b sin th) = sqrt2 2 pi k_l (b cos th - a sin th) */
            double g = sqrt(2.0) * 2.0 * M_PI * (alpha[2 * r] * ct - alpha[2 * r - 1] * st);
            for (int l = 0; l < d; ++l) {
                if (k[l] == 0) continue;
                double gt = (double)k[l] * g;
                double tt = gs[l] + gt;
                gc[l] += (fabs(gs[l]) >= fabs(gt)) ? (gs[l] - tt) + gt : (gt - tt) + gs[l];
                gs[l] = tt;
            }
        }
    }
    if (grad)
        for (int l = 0; l < d; ++l) grad[l] = (gs[l] + gc[l]) * dudx[l];
    return s + c;
}

/* The cosine expansion sum_k alpha_k phi_k(x) and its x-gradient:
 * d phi_k / d x_l = (prod_{j != l} c_{k_j}(u_j)) c'_{k_l}(u_l) nu_l(x_l) with
 * c'_m(u) = -sqrt2 m pi sin(m pi u). */
static double or_expansion_cos(int d, int nu, int64_t nrep, const int32_t *reps, const double *alpha,
                               const double *x, double *grad)
{
    double u[OR_MAXD], dudx[OR_MAXD];
    for (int l = 0; l < d; ++l) {
        u[l] = or_law_cdf(nu, x[l]);
        dudx[l] = or_law_pdf(nu, x[l]);
    }
    double s = 0.0, c = 0.0;
    double gs[OR_MAXD], gc[OR_MAXD];
    for (int l = 0; l < d; ++l) { gs[l] = 0.0; gc[l] = 0.0; }
    for (int64_t r = 0; r < nrep; ++r) {
        const int32_t *k = reps + r * d;
        double term = alpha[r] * or_cos_value(k, u, d);
        double t = s + term;
        c += (fabs(s) >= fabs(term)) ? (s - t) + term : (term - t) + s;
        s = t;
        if (grad) {
            for (int l = 0; l < d; ++l) {
                if (k[l] == 0) continue;
                double g = alpha[r] * -sqrt(2.0) * (double)k[l] * M_PI * sin((double)k[l] * M_PI * u[l]);
                for (int j = 0; j < d; ++j)
                    if (j != l) g *= or_cos_factor(k[j], u[j]);
                double tt = gs[l] + g;
                gc[l] += (fabs(gs[l]) >= fabs(g)) ? (gs[l] - tt) + g : (g - tt) + gs[l];
                gs[l] = tt;
            }
        }
    }
    if (grad)
        for (int l = 0; l < d; ++l) grad[l] = (gs[l] + gc[l]) * dudx[l];
    return s + c;
}

/* Evaluate ybar (and optionally grad, row-major [n][d]) at n points. */
void or_eval(int d, int nu, int basis, int64_t nrep, const int32_t *reps, const double *alpha_row, int64_t n,
             const double *x, double *y, double *grad)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < n; ++p)
        y[p] = or_expansion(d, nu, basis, nrep, reps, alpha_row, x + p * d, grad ? grad + p * d : NULL);
}

/* ------------------------------------------------------------------------ */
/* Manufactured solution family u(t,x) = A e^{-c(T-t)} cos(w.x + p) and the  */
/* source h that makes it solve (pde) for the chosen driver:                */
/*   h = -(d_t u + b.grad u + 1/2 tr(sigma sigma^T hess u)) - f_nl(u, sigma^T grad u) */
/* ------------------------------------------------------------------------ */
static double or_T(const or_problem *P) { return P->t[P->N]; }

double or_msol_u(const or_problem *P, double t, const double *x)
{
    double th = P->sol_p;
    for (int l = 0; l < P->d; ++l) th += P->sol_w[l] * x[l];
    return P->sol_B + P->sol_A * exp(-P->sol_c * (or_T(P) - t)) * cos(th);
}

/* gradient of u in x */
static void or_msol_grad(const or_problem *P, double t, const double *x, double *g)
{
    double th = P->sol_p;
    for (int l = 0; l < P->d; ++l) th += P->sol_w[l] * x[l];
    double a = -P->sol_A * exp(-P->sol_c * (or_T(P) - t)) * sin(th);
    for (int l = 0; l < P->d; ++l) g[l] = a * P->sol_w[l];
}

/* Coefficients of the forward SDE (assumption (A_{b,sigma})): drift
 * b(t,x)_l and diffusion sigma(t,x)_{lk}.  Bounded in x apart from the
 * affine part b1_l x_l, Lipschitz in x, and uniformly elliptic when
 * |v_l| < 1 and the constant sigma is (Thm "Norm-stability"). */
static double or_drift(const or_problem *P, double t, const double *x, int l)
{
    (void)t;
    return P->b0[l] + P->b1[l] * x[l] + P->b2[l] * sin(x[l]);
}

static double or_sigma(const or_problem *P, double t, const double *x, int l, int k)
{
    return (1.0 + P->sigma_v[l] * cos(x[l] + P->sigma_omega * t)) * P->sigma[l * P->nbm + k];
}

/* z = sigma(t,x)^T v  (v a d-vector, z an nbm-vector) */
static void or_sigmaT(const or_problem *P, double t, const double *x, const double *v, double *z)
{
    for (int k = 0; k < P->nbm; ++k) {
        double s = 0.0;
        for (int l = 0; l < P->d; ++l) s += or_sigma(P, t, x, l, k) * v[l];
        z[k] = s;
    }
}

/* nonlinear part of the driver, f = f_nl(t, x, y, z) + h(t, x); the Sec. 5
 * benchmark's f_nl = min(1, (y - u(t,x))^2) is the only one that reads (t, x) */
static double or_fnl(const or_problem *P, double t, const double *x, double y, const double *z)
{
    switch (P->driver) {
    case 4: {
        double e = y - or_msol_u(P, t, x);
        double e2 = e * e;
        return e2 < 1.0 ? e2 : 1.0;
    }
    case 0: return 0.0;
    case 1: return P->f_a * sin(y);
    case 2: return y - y * y * y;
    case 3: {
        double z2 = 0.0;
        for (int k = 0; k < P->nbm; ++k) z2 += z[k] * z[k];
        return P->f_a * z2 / (1.0 + z2) + y / (1.0 + y * y);
    }
    }
    return NAN;
}

double or_msol_h(const or_problem *P, double t, const double *x)
{
    int d = P->d;
    double u = or_msol_u(P, t, x);
    double gu[OR_MAXD], z[OR_MAXD];
    or_msol_grad(P, t, x, gu);
    /* the offset B drops out of every derivative */
    double dt_u = P->sol_c * (u - P->sol_B);
    double b_grad = 0.0;
    for (int l = 0; l < d; ++l) b_grad += or_drift(P, t, x, l) * gu[l];
    /* hess u = -(u - B) w w^T, so 1/2 tr(sigma sigma^T hess u) = -1/2 (u - B) |sigma(t,x)^T w|^2 */
    double sw[OR_MAXD];
    or_sigmaT(P, t, x, P->sol_w, sw);
    double sw2 = 0.0;
    for (int k = 0; k < P->nbm; ++k) sw2 += sw[k] * sw[k];
    double diff = -0.5 * (u - P->sol_B) * sw2;
    or_sigmaT(P, t, x, gu, z);
    return -(dt_u + b_grad + diff) - or_fnl(P, t, x, u, z);
}

/* terminal condition g = u(T, .) and its gradient */
static double or_g(const or_problem *P, const double *x) { return or_msol_u(P, or_T(P), x); }

/* T_L: clamp to [-L, L] */
static double or_trunc(const or_problem *P, double y)
{
    double L = P->clamp;
    if (y > L) return L;
    if (y < -L) return -L;
    return y;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (GQRMDP) with damping exponent q.                            */
/* ------------------------------------------------------------------------ */

/* Damping factor (1+|x|^2)^{q/2} of eq (yqi). */
double or_damping(const or_problem *P, const double *x)
{
    double r2 = 0.0;
    for (int l = 0; l < P->d; ++l) r2 += x[l] * x[l];
    return pow(1.0 + r2, 0.5 * P->damping_q);
}

/* y_{j+1}(x) recovered from the expansion of ybar^{(q)}_{j+1}: the
 * expansion times (1+|x|^2)^{q/2} (eqs (yqi), (Sqi:bar:M)), and, when
 * grad != NULL, its x-gradient by the product rule:
 * grad y = D grad ybar + ybar q D x / (1+|x|^2). */
double or_eval_y(const or_problem *P, int64_t nrep, const int32_t *reps, const double *alpha_row,
                 const double *x, double *grad)
{
    int d = P->d;
    double yb = or_expansion(d, P->nu, P->basis, nrep, reps, alpha_row, x, grad);
    if (P->damping_q == 0.0) return yb;
    double r2 = 0.0;
    for (int l = 0; l < d; ++l) r2 += x[l] * x[l];
    double D = pow(1.0 + r2, 0.5 * P->damping_q);
    if (grad)
        for (int l = 0; l < d; ++l) grad[l] = D * grad[l] + yb * P->damping_q * D * x[l] / (1.0 + r2);
    return yb * D;
}


/* Start point X_i^i of path m: d uniforms of stream 0 through F^{-1}. */
static void or_start_point(const or_problem *P, uint64_t seed, int32_t i, uint64_t m, double *x)
{
    for (int l = 0; l < P->d; ++l)
        x[l] = or_law_icdf(P->nu, or_uniform(seed, 0u, m, (uint32_t)i, (uint32_t)l));
}

/* ------------------------------------------------------------------------ */
/* Surrogate network of the learned form (not part of the paper's method):   */
/* features f_l = 2 F(x_l) - 1 (l < d, 0 up to 16), h1 = silu(W1 f + b1),    */
/* h2 = silu(W2 h1 + b2), out = w3 . h2 + b3, parameters in the order W1     */
/* [256][16] (row = output unit), b1, W2 [256][256], b2, w3, b3.  The two    */
/* matrix products take bfloat16 operands (nearest, ties to even, from the   */
/* binary32 value): the network's arithmetic as the learned form defines it; */
/* the sums themselves are exact here (FP64).                                */
/* ------------------------------------------------------------------------ */
#define OR_MLP_IN 16
#define OR_MLP_HID 256

static double or_bf16(double a)
{
    float f = (float)a;
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    u = ((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16) << 16;
    memcpy(&f, &u, sizeof f);
    return (double)f;
}

static double or_silu(double z) { return z / (1.0 + exp(-z)); }

double or_mlp_forward(const double *theta, int nu, int d, const double *x)
{
    const double *W1 = theta, *b1 = W1 + OR_MLP_HID * OR_MLP_IN, *W2 = b1 + OR_MLP_HID;
    const double *b2 = W2 + OR_MLP_HID * OR_MLP_HID, *w3 = b2 + OR_MLP_HID, *b3 = w3 + OR_MLP_HID;
    double f[OR_MLP_IN], h1[OR_MLP_HID], out = b3[0];
    for (int l = 0; l < OR_MLP_IN; ++l) f[l] = l < d ? or_bf16(2.0 * or_law_cdf(nu, x[l]) - 1.0) : 0.0;
    for (int o = 0; o < OR_MLP_HID; ++o) {
        double z = b1[o];
        for (int l = 0; l < OR_MLP_IN; ++l) z += or_bf16(W1[o * OR_MLP_IN + l]) * f[l];
        h1[o] = or_bf16(or_silu(z));
    }
    for (int o = 0; o < OR_MLP_HID; ++o) {
        double z = b2[o];
        for (int k = 0; k < OR_MLP_HID; ++k) z += or_bf16(W2[o * OR_MLP_HID + k]) * h1[k];
        out += w3[o] * or_silu(z);
    }
    return out;
}

/* Response S_i of eq (Sqi:bar:M) along path m, using the expansions
 * alpha rows i+1..N-1 (row j holds ybar_j; ybar_N = g) or, for the time
 * indices j with nets[j] != NULL (learned form), y_j(x) = mu[j] + sd[j] *
 * network_j(x) in place of the expansion. */
static double or_path_response_ex(const or_problem *P, int64_t nrep, const int32_t *reps, int32_t i,
                                  uint64_t seed, uint64_t m, const double *alpha,
                                  const double *const *nets, const double *mu, const double *sd,
                                  double *first, double *y_first);

double or_path_response(const or_problem *P, int64_t nrep, const int32_t *reps, int32_t i,
                        uint64_t seed, uint64_t m, const double *alpha)
{
    return or_path_response_ex(P, nrep, reps, i, seed, m, alpha, NULL, NULL, NULL, NULL, NULL);
}

/* first (if not NULL) receives the term j = i of the driver sum, f(t_i, ...) Delta_i;
 * y_first the value the driver reads on that step, T_L(ybar_{i+1}(X_{i+1})) (g at i = N-1) */
static double or_path_response_ex(const or_problem *P, int64_t nrep, const int32_t *reps, int32_t i,
                                  uint64_t seed, uint64_t m, const double *alpha,
                                  const double *const *nets, const double *mu, const double *sd,
                                  double *first, double *y_first)
{
    int d = P->d, nbm = P->nbm, N = P->N;
    int64_t nf = or_nfuncs_of(P->basis, nrep);
    double x[OR_MAXD], xn[OR_MAXD], dw[OR_MAXD], grad[OR_MAXD], z[OR_MAXD];
    or_start_point(P, seed, i, m, x);
    double S = 0.0;
    for (int j = i; j < N; ++j) {
        double dt = P->t[j + 1] - P->t[j];
        for (int k = 0; k < nbm; ++k) {
            uint32_t r = (uint32_t)(d + (j - i) * nbm + k);
            dw[k] = sqrt(dt) * or_norm_icdf(or_uniform(seed, 0u, m, (uint32_t)i, r));
        }
        /* Euler step, eq (markov:euler), coefficients at (t_j, X_j) */
        for (int l = 0; l < d; ++l) {
            double s = 0.0;
            for (int k = 0; k < nbm; ++k) s += or_sigma(P, P->t[j], x, l, k) * dw[k];
            xn[l] = x[l] + or_drift(P, P->t[j], x, l) * dt + s;
        }
        double y;
        int need_z = (P->driver == 3);
        if (j + 1 < N && nets && nets[j + 1]) {
            y = mu[j + 1] + sd[j + 1] * or_mlp_forward(nets[j + 1], P->nu, d, xn);
        } else if (j + 1 < N) {
            y = or_eval_y(P, nrep, reps, alpha + (int64_t)(j + 1) * nf, xn, need_z ? grad : NULL);
        } else {
            y = or_g(P, xn);
            if (need_z) or_msol_grad(P, or_T(P), xn, grad);
        }
        y = or_trunc(P, y);
        if (j == i && y_first) *y_first = y;
        /* z_{j+1} = sigma(t_{j+1}, X_{j+1})^T grad ybar_{j+1}(X_{j+1}) */
        if (need_z) or_sigmaT(P, P->t[j + 1], xn, grad, z);
        double term = (or_fnl(P, P->t[j], x, y, z) + or_msol_h(P, P->t[j], x)) * dt;
        if (j == i && first) *first = term;
        S += term;
        for (int l = 0; l < d; ++l) x[l] = xn[l];
    }
    S += or_g(P, x);
    /* the response of the damped quantity: divided by (1+|X_i|^2)^{q/2} */
    if (P->damping_q != 0.0) {
        double xi[OR_MAXD];
        or_start_point(P, seed, i, m, xi);
        S /= or_damping(P, xi);
    }
    return S;
}

/* Projection (eq (Aqi:bar:M)): alpha_k = (1/n) sum_p s_p phi_k(x_p), and the
 * scale A_k = (1/n) sum_p |s_p phi_k(x_p)|.  x is row-major [n][d]. */
void or_project(int d, int nu, int basis, int64_t nrep, const int32_t *reps, int64_t n, const double *x,
                const double *s, double *alpha, double *absum)
{
    int64_t nf = or_nfuncs_of(basis, nrep);
    double *u = (double *)malloc(sizeof(double) * (size_t)(n * d));
    for (int64_t p = 0; p < n * d; ++p) u[p] = or_law_cdf(nu, x[p]);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t f = 0; f < nf; ++f) {
        int64_t r = basis == 1 ? f : (f + 1) / 2;
        const int32_t *k = reps + r * d;
        double sum = 0.0, comp = 0.0, asum = 0.0;
        for (int64_t p = 0; p < n; ++p) {
            double phi;
            if (basis == 1) {
                phi = or_cos_value(k, u + p * d, d);
            } else if (f == 0) {
                phi = 1.0;
            } else {
                double th = 2.0 * M_PI * or_phase(k, u + p * d, d);
                phi = (f & 1) ? sqrt(2.0) * cos(th) : sqrt(2.0) * sin(th);
            }
            double term = s[p] * phi;
            double t = sum + term;
            comp += (fabs(sum) >= fabs(term)) ? (sum - t) + term : (term - t) + sum;
            sum = t;
            asum += fabs(term);
        }
        alpha[f] = (sum + comp) / (double)n;
        if (absum) absum[f] = asum / (double)n;
    }
    free(u);
}

/* One backward iteration i of Algorithm 1: fills alpha row i from rows
 * i+1..N-1 with a fresh cloud of M paths.  Optionally returns the start
 * points (row-major [M][d]), the responses S [M] and the scale row A [nf]. */
int or_backward_step_learned(const or_problem *P, int64_t nrep, const int32_t *reps, int32_t i,
                             int64_t M, uint64_t seed, double *alpha, double *absum,
                             const double *const *nets, const double *mu, const double *sd);

int or_backward_step(const or_problem *P, int64_t nrep, const int32_t *reps, int32_t i,
                     int64_t M, uint64_t seed, double *alpha, double *absum, double *x_out,
                     double *s_out)
{
    if (i < 0 || i >= P->N || M <= 0) return -1;
    int d = P->d;
    int64_t nf = or_nfuncs_of(P->basis, nrep);
    double *x = (double *)malloc(sizeof(double) * (size_t)(M * d));
    double *S = (double *)malloc(sizeof(double) * (size_t)M);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t m = 0; m < M; ++m) {
        or_start_point(P, seed, i, (uint64_t)m, x + m * d);
        S[m] = or_path_response(P, nrep, reps, i, seed, (uint64_t)m, alpha);
    }
    or_project(d, P->nu, P->basis, nrep, reps, M, x, S, alpha + (int64_t)i * nf, absum);
    if (x_out) memcpy(x_out, x, sizeof(double) * (size_t)(M * d));
    if (s_out) memcpy(s_out, S, sizeof(double) * (size_t)M);
    free(x);
    free(S);
    return 0;
}

/* Z of the multistep scheme, eq (MDP:intro:0a), at time index i (q = 0):
 * with the paths, streams and later rows of or_backward_step, the response
 * of path m is S^Z_m = g(X_N) + sum_{j=i+1}^{N-1} f_j Delta_j (the driver sum
 * without its term j = i) times the first Brownian increment
 * dW_{i,k}(m) / Delta_i (the normals r = d + k of the path's stream), and
 * alpha_z[k][f] = (1/M) sum_m S^Z_m dW_{i,k}(m) / Delta_i phi_f(X_i^m) for
 * k < nbm (row-major [nbm][n_funcs]); absum_z likewise, or NULL. */
int or_backward_step_z(const or_problem *P, int64_t nrep, const int32_t *reps, int32_t i,
                       int64_t M, uint64_t seed, const double *alpha, double *alpha_z, double *absum_z)
{
    if (i < 0 || i >= P->N || M <= 0 || P->damping_q != 0.0) return -1;
    int d = P->d, nbm = P->nbm;
    int64_t nf = or_nfuncs_of(P->basis, nrep);
    double dt = P->t[i + 1] - P->t[i];
    double *x = (double *)malloc(sizeof(double) * (size_t)(M * d));
    double *SZ = (double *)malloc(sizeof(double) * (size_t)M);
    double *r = (double *)malloc(sizeof(double) * (size_t)M);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t m = 0; m < M; ++m) {
        double first = 0.0;
        or_start_point(P, seed, i, (uint64_t)m, x + m * d);
        double S = or_path_response_ex(P, nrep, reps, i, seed, (uint64_t)m, alpha, NULL, NULL, NULL, &first, NULL);
        SZ[m] = S - first;
    }
    for (int k = 0; k < nbm; ++k) {
        for (int64_t m = 0; m < M; ++m) {
            double dw = sqrt(dt) * or_norm_icdf(or_uniform(seed, 0u, (uint64_t)m, (uint32_t)i, (uint32_t)(d + k)));
            r[m] = SZ[m] * dw / dt;
        }
        or_project(d, P->nu, P->basis, nrep, reps, M, x, r, alpha_z + (int64_t)k * nf,
                   absum_z ? absum_z + (int64_t)k * nf : NULL);
    }
    free(x);
    free(SZ);
    free(r);
    return 0;
}

/* Z of the one-step scheme, eq (ODP:intro:a), at time index i (q = 0): the
 * response of path m is T_L(ybar_{i+1}(X_{i+1})) - T_L(ybar_{i+1}(X_i))
 * (ybar_N = g), the value the driver reads on the path's first step less the
 * same function at the start point; the second term is a function of X_i,
 * so it leaves the conditional expectation against dW unchanged and removes
 * most of the variance.  alpha_z as in or_backward_step_z. */
int or_backward_step_z1(const or_problem *P, int64_t nrep, const int32_t *reps, int32_t i,
                        int64_t M, uint64_t seed, const double *alpha, double *alpha_z, double *absum_z)
{
    if (i < 0 || i >= P->N || M <= 0 || P->damping_q != 0.0) return -1;
    int d = P->d, nbm = P->nbm;
    int64_t nf = or_nfuncs_of(P->basis, nrep);
    double dt = P->t[i + 1] - P->t[i];
    double *x = (double *)malloc(sizeof(double) * (size_t)(M * d));
    double *D = (double *)malloc(sizeof(double) * (size_t)M);
    double *r = (double *)malloc(sizeof(double) * (size_t)M);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t m = 0; m < M; ++m) {
        double first = 0.0, y1 = 0.0;
        or_start_point(P, seed, i, (uint64_t)m, x + m * d);
        (void)or_path_response_ex(P, nrep, reps, i, seed, (uint64_t)m, alpha, NULL, NULL, NULL, &first, &y1);
        double y0 = (i + 1 < P->N) ? or_eval_y(P, nrep, reps, alpha + (int64_t)(i + 1) * nf, x + m * d, NULL)
                                   : or_g(P, x + m * d);
        D[m] = y1 - or_trunc(P, y0);
    }
    for (int k = 0; k < nbm; ++k) {
        for (int64_t m = 0; m < M; ++m) {
            double dw = sqrt(dt) * or_norm_icdf(or_uniform(seed, 0u, (uint64_t)m, (uint32_t)i, (uint32_t)(d + k)));
            r[m] = D[m] * dw / dt;
        }
        or_project(d, P->nu, P->basis, nrep, reps, M, x, r, alpha_z + (int64_t)k * nf,
                   absum_z ? absum_z + (int64_t)k * nf : NULL);
    }
    free(x);
    free(D);
    free(r);
    return 0;
}

/* One backward iteration of the learned form: as or_backward_step, with
 * the surrogate nets[j] (a parameter vector, or NULL for the expansion) and
 * its target scaling mu[j], sd[j] in place of the expansion of ybar_j along
 * the paths (arrays of N entries; entries j <= i are not read). */
int or_backward_step_learned(const or_problem *P, int64_t nrep, const int32_t *reps, int32_t i,
                             int64_t M, uint64_t seed, double *alpha, double *absum,
                             const double *const *nets, const double *mu, const double *sd)
{
    if (i < 0 || i >= P->N || M <= 0) return -1;
    int d = P->d;
    int64_t nf = or_nfuncs_of(P->basis, nrep);
    double *x = (double *)malloc(sizeof(double) * (size_t)(M * d));
    double *S = (double *)malloc(sizeof(double) * (size_t)M);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t m = 0; m < M; ++m) {
        or_start_point(P, seed, i, (uint64_t)m, x + m * d);
        S[m] = or_path_response_ex(P, nrep, reps, i, seed, (uint64_t)m, alpha, nets, mu, sd, NULL, NULL);
    }
    or_project(d, P->nu, P->basis, nrep, reps, M, x, S, alpha + (int64_t)i * nf, absum);
    free(x);
    free(S);
    return 0;
}

/* Full backward induction i = N-1..0 (Algorithm 1). alpha is [N][nf]. */
int or_solve(const or_problem *P, int64_t nrep, const int32_t *reps, int64_t M, uint64_t seed,
             double *alpha)
{
    for (int32_t i = P->N - 1; i >= 0; --i) {
        int rc = or_backward_step(P, nrep, reps, i, M, seed, alpha, NULL, NULL, NULL);
        if (rc) return rc;
    }
    return 0;
}

/* nu-distributed points (stream `stream`, time index i), row-major [n][d]. */
void or_sample_points(int d, int nu, uint64_t seed, uint32_t stream, int32_t i, int64_t m0,
                      int64_t n, double *x)
{
    for (int64_t p = 0; p < n; ++p)
        for (int l = 0; l < d; ++l)
            x[p * d + l] = or_law_icdf(
                nu, or_uniform(seed, stream, (uint64_t)(m0 + p), (uint32_t)i, (uint32_t)l));
}

/* Error indicators of Sec. 5, eq (mse) (natural logarithms), computed on
 * n points per time index drawn from stream 1, against u(t_i, .), the
 * prediction being the expansion times (1+|x|^2)^{q/2}:
 *   out[0] = MSE_max, out[1] = MSE_av, out[2] = relative L2 error at t_0. */
void or_errors(const or_problem *P, int64_t nrep, const int32_t *reps, const double *alpha,
               uint64_t seed, int64_t n, double *out)
{
    int d = P->d, N = P->N;
    int64_t nf = or_nfuncs_of(P->basis, nrep);
    double worst = 0.0, total = 0.0, e0 = 0.0, u0 = 0.0;
    double *x = (double *)malloc(sizeof(double) * (size_t)(n * d));
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    for (int i = 0; i < N; ++i) {
        or_sample_points(d, P->nu, seed, 1u, i, 0, n, x);
        or_eval(d, P->nu, P->basis, nrep, reps, alpha + (int64_t)i * nf, n, x, y, NULL);
        for (int64_t p = 0; p < n; ++p) y[p] *= or_damping(P, x + p * d);
        double se = 0.0, su = 0.0;
        for (int64_t p = 0; p < n; ++p) {
            double uex = or_msol_u(P, P->t[i], x + p * d);
            se += (uex - y[p]) * (uex - y[p]);
            su += uex * uex;
        }
        if (se / (double)n > worst) worst = se / (double)n;
        total += se;
        if (i == 0) { e0 = se; u0 = su; }
    }
    out[0] = log(worst);
    out[1] = log(total / ((double)n * (double)N));
    out[2] = sqrt(e0 / u0);
    free(x);
    free(y);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
