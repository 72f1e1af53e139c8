// qrmc_common.h -- scalar routines shared by the HIP kernels and their host
// mirrors (random streams, laws), plus the structures the host hands to the
// kernels.  Everything here is __host__ __device__ so the host build of the
// library can expose the same arithmetic for unit tests without a GPU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qrmc.h"

namespace qrmc {

constexpr int kMaxD = QR_MAX_D;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds, multipliers
// 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 / 0xBB67AE85.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__host__ __device__ inline uint32_t mulhi32(uint32_t a, uint32_t b) {
#ifdef __HIP_DEVICE_COMPILE__
    return __umulhi(a, b);
#else
    return (uint32_t)(((uint64_t)a * (uint64_t)b) >> 32);
#endif
}

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = mulhi32(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = mulhi32(0xCD9E8D57u, c.z);
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// 52-bit uniform in (0,1) from two words: ((a << 20 | b >> 12) + 1/2) 2^-52.
__host__ __device__ inline double words_to_uniform(uint32_t a, uint32_t b) {
    const uint64_t n = ((uint64_t)a << 20) | (uint64_t)(b >> 12);
    return ((double)n + 0.5) * 0x1p-52;
}

// Sequential reader of draws r = r0, r0+1, ... of sample m, time index i, in
// one stream: each Philox block yields two uniforms; the second is kept.
struct PhiloxStream {
    uint32_t k0, k1, m_lo, m_hi, i;
    uint32_t r;
    double spare;

    __host__ __device__ PhiloxStream(uint64_t seed, uint32_t stream, uint64_t m, uint32_t ti,
                                     uint32_t r0)
        : k0((uint32_t)seed), k1((uint32_t)(seed >> 32) ^ stream), m_lo((uint32_t)m),
          m_hi((uint32_t)(m >> 32)), i(ti), r(r0), spare(0.0) {
        if (r & 1u) {
            const U4 w = philox4x32_10(U4{m_lo, m_hi, i, r >> 1}, k0, k1);
            spare = words_to_uniform(w.z, w.w);
        }
    }

    __host__ __device__ inline double next() {
        double u;
        if (r & 1u) {
            u = spare;
        } else {
            const U4 w = philox4x32_10(U4{m_lo, m_hi, i, r >> 1}, k0, k1);
            u = words_to_uniform(w.x, w.y);
            spare = words_to_uniform(w.z, w.w);
        }
        ++r;
        return u;
    }
};

__host__ __device__ inline double uniform_at(uint64_t seed, uint32_t stream, uint64_t m, uint32_t i,
                                             uint32_t r) {
    const U4 w = philox4x32_10(U4{(uint32_t)m, (uint32_t)(m >> 32), i, r >> 1}, (uint32_t)seed,
                               (uint32_t)(seed >> 32) ^ stream);
    return (r & 1u) ? words_to_uniform(w.z, w.w) : words_to_uniform(w.x, w.y);
}

// ---------------------------------------------------------------------------
// Inverse standard normal CDF: Wichura, "Algorithm AS 241: The percentage
// points of the normal distribution", Applied Statistics 37 (1988), PPND16
// (rational approximations in three regions, ~1e-16 relative accuracy).
// ---------------------------------------------------------------------------
__host__ __device__ inline double norm_icdf(double p) {
    const double q = p - 0.5;
    if (fabs(q) <= 0.425) {
        const double r = 0.180625 - q * q;
        const double num =
            (((((((2.5090809287301226727e+3 * r + 3.3430575583588128105e+4) * r +
                  6.7265770927008700853e+4) * r + 4.5921953931549871457e+4) * r +
                1.3731693765509461125e+4) * r + 1.9715909503065514427e+3) * r +
              1.3314166789178437745e+2) * r + 3.3871328727963666080e0);
        const double den =
            (((((((5.2264952788528545610e+3 * r + 2.8729085735721942674e+4) * r +
                  3.9307895800092710610e+4) * r + 2.1213794301586595867e+4) * r +
                5.3941960214247511077e+3) * r + 6.8718700749205790830e+2) * r +
              4.2313330701600911252e+1) * r + 1.0);
        return q * num / den;
    }
    double r = (q < 0.0) ? p : 1.0 - p;
    r = sqrt(-log(r));
    double v;
    if (r <= 5.0) {
        r -= 1.6;
        const double num =
            (((((((7.74545014278341407640e-4 * r + 2.27238449892691845833e-2) * r +
                  2.41780725177450611770e-1) * r + 1.27045825245236838258e0) * r +
                3.64784832476320460504e0) * r + 5.76949722146069140550e0) * r +
              4.63033784615654529590e0) * r + 1.42343711074968357734e0);
        const double den =
            (((((((1.05075007164441684324e-9 * r + 5.47593808499534494600e-4) * r +
                  1.51986665636164571966e-2) * r + 1.48103976427480074590e-1) * r +
                6.89767334985100004550e-1) * r + 1.67638483018380384940e0) * r +
              2.05319162663775882187e0) * r + 1.0);
        v = num / den;
    } else {
        r -= 5.0;
        const double num =
            (((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r +
                  1.24266094738807843860e-3) * r + 2.65321895265761230930e-2) * r +
                2.96560571828504891230e-1) * r + 1.78482653991729133580e0) * r +
              5.46378491116411436990e0) * r + 6.65790464350110377720e0);
        const double den =
            (((((((2.04426310338993978564e-15 * r + 1.42151175831644588870e-7) * r +
                  1.84631831751005468180e-5) * r + 7.86869131145613259100e-4) * r +
                1.48753612908506148525e-2) * r + 1.36929880922735805310e-1) * r +
              5.99832206555887937690e-1) * r + 1.0);
        v = num / den;
    }
    return (q < 0.0) ? -v : v;
}

// Standard logistic law: F(x) = 1/(1+e^{-x}), F^{-1}(u) = ln u - ln(1-u).
__host__ __device__ inline double logistic_icdf(double u) { return log(u) - log(1.0 - u); }
__host__ __device__ inline double logistic_cdf(double x) { return 1.0 / (1.0 + exp(-x)); }

// One-dimensional marginal nu_l of the sampling law (qr_law):
//  - QR_LAW_STUDENT2: Student's t with mu = 2 in the scaling of the paper's
//    Example "Student's t-distribution", density (1+x^2)^{-3/2} / 2, whose
//    F and F^{-1} are closed forms (Sec. 5, eq (Fnui:Fnulinv)):
//    F(x) = (1 + x / sqrt(1+x^2)) / 2 and F^{-1}(u) = (u - 1/2) / sqrt(u (1-u));
//  - QR_LAW_CAUCHY (mu = 1): density 1 / (pi (1+x^2)), F(x) = 1/2 + atan(x)/pi,
//    F^{-1}(u) = tan(pi (u - 1/2)), here as -cos(pi u) / sin(pi u) with the
//    argument folded to (0, 1/2] so that the tails keep their relative
//    accuracy (sincospi takes u itself, no product with pi);
//  - otherwise the standard logistic law.
// Bit kLawHalf of a law code is not part of the law: it marks the cosine
// basis, whose kernels take the phase factors e^{i pi F(x)} at half the
// Fourier frequency (see nl_unit_phase); the laws below ignore it.
constexpr int32_t kLawHalf = 8;
constexpr int32_t kLawMask = 7;

__device__ inline double law_icdf(int32_t nu, double u) {
    nu &= kLawMask;
    if (nu == QR_LAW_STUDENT2) return (u - 0.5) / sqrt(u * (1.0 - u));
    if (nu == QR_LAW_CAUCHY) {
        const double v = u < 0.5 ? u : 1.0 - u;  // exact for u >= 1/2
        double sn, cs;
        sincospi(v, &sn, &cs);
        return u < 0.5 ? -cs / sn : cs / sn;
    }
    return logistic_icdf(u);
}
__device__ inline double law_cdf(int32_t nu, double x) {
    nu &= kLawMask;
    if (nu == QR_LAW_STUDENT2) return 0.5 + 0.5 * (x / sqrt(fma(x, x, 1.0)));
    if (nu == QR_LAW_CAUCHY) return 0.5 + atan(x) * M_1_PI;
    return logistic_cdf(x);
}
// density nu_l(x) = dF/dx, given x and u = F(x)
__device__ inline double law_pdf(int32_t nu, double x, double u) {
    nu &= kLawMask;
    if (nu == QR_LAW_STUDENT2) {
        const double r = 1.0 / fma(x, x, 1.0);
        return 0.5 * r * sqrt(r);
    }
    if (nu == QR_LAW_CAUCHY) return M_1_PI / fma(x, x, 1.0);
    return u * (1.0 - u);
}

// ---------------------------------------------------------------------------
// Structures handed to the kernels
// ---------------------------------------------------------------------------

// Problem as the kernels read it (device memory, one per context), with the
// closed-form pieces of the manufactured solution pre-combined on the host.
struct DevProblem {
    int32_t d, nbm, N, driver;
    int32_t nu;                       // law code of the basis in use (qr_law | kLawHalf)
    double f_a, clamp, T;
    double sw2;                       // |sigma^T w|^2
    double t[QR_MAX_N + 1];
    double b0[kMaxD], b1[kMaxD];
    double sigma[kMaxD * kMaxD];      // [d][nbm]
    double sol_A, sol_c, sol_p, sol_B;
    double sol_w[kMaxD];
    double sw[kMaxD];                 // sigma^T w
    double dq;                        // damping exponent q (0: none)
    // state-dependent coefficients: drift part b2_l sin(x_l), row scale
    // 1 + sv_l cos(x_l + somega t) of sigma; sdep = 1 iff any is non-zero
    double b2[kMaxD], sv[kMaxD];
    double somega;
    int32_t sdep;
};

// Index-set rule of the traversal: a node with budget P (the root has P = 1)
// may take a next coordinate of magnitude m iff m <= mmax and its child's
// budget, P (a m + b) for the product rules or P + m for the sum rule
// (add = 1), is at most L.
//   tensor  (max |k_l| <= K):            a = 0, b = 1, mmax = K, L = 1
//   hc_max  (prod max(1,|k_l|) <= L):    a = 1, b = 0, mmax = L
//   hc_1p   (prod (1+|k_l|) <= L):       a = 1, b = 1, mmax = L
//   total   (sum |k_l| <= K):            add = 1, mmax = K, L = K + 1
//           (budget 1 + the sum so far)
struct SetRule {
    int32_t a, b, L, mmax, d, add;
};

__host__ __device__ inline SetRule make_rule(int32_t kind, int32_t level, int32_t d) {
    if (kind == QR_SET_TENSOR) return SetRule{0, 1, 1, level, d, 0};
    if (kind == QR_SET_HC_MAX) return SetRule{1, 0, level, level, d, 0};
    if (kind == QR_SET_TOTAL) return SetRule{0, 0, level + 1, level, d, 1};
    return SetRule{1, 1, level, level, d, 0};
}

__host__ __device__ inline int32_t rule_child(const SetRule &R, int32_t P, int32_t m) {
    return R.add ? P + m : P * (R.a * m + R.b);
}

__host__ __device__ inline bool rule_ok(const SetRule &R, int32_t P, int32_t m) {
    return (m <= R.mmax) & (rule_child(R, P, m) <= R.L);
}

constexpr int kMaxDepthCap = 8;

// Branch-light form of the same rule used by the kernels' walk: a node with
// budget Pb extends by magnitudes m = 1, 2, ... while its child's budget,
// w = Pb (m + b) (a = 0) or w = Pb + m (a = 1, total degree), is at most L:
// w runs from Pb (1 + b) + a in steps of (a ? 1 : Pb); the child's
// budget is w when c = 1 (hyperbolic crosses, total degree) or stays Pb = 1
// (c = 0, tensor set); a child has children iff its budget <= Lc.
// The walk also carries the law code nu of the basis (qr_law, plus kLawHalf
// for the cosine basis): the basis functions in x are the Fourier functions
// of the torus composed with F_nu.
struct Walk {
    int32_t b, L, Lc, c, d, nu, a;
};

__host__ __device__ inline Walk make_walk(int32_t kind, int32_t level, int32_t d, int32_t nu) {
    if (kind == QR_SET_TENSOR) return Walk{0, level, level, 0, d, nu, 0};
    if (kind == QR_SET_HC_MAX) return Walk{0, level, level, 1, d, nu, 0};
    if (kind == QR_SET_TOTAL) return Walk{0, level + 1, level, 1, d, nu, 1};
    return Walk{1, level, level / 2, 1, d, nu, 0};
}

// Root of a run of the depth-first traversal used by the projection: the
// node k (by its non-zero coordinates) and whether its whole subtree follows.
struct TaskItem {
    int32_t depth;   // number of non-zero coordinates (0: the zero vector)
    int32_t last;    // last non-zero coordinate (-1 for the zero vector)
    int32_t prod;    // budget product of the node
    int32_t full;    // 1: node and all its descendants; 0: the node alone
    int32_t coord[kMaxDepthCap];
    int32_t val[kMaxDepthCap];
};

// A projection task: items [item_begin, item_end) covering the consecutive
// traversal indices [rep_begin, rep_begin + rep_count).
struct Task {
    int32_t item_begin, item_end;
    int32_t rep_begin, rep_count;
};

}  // namespace qrmc
