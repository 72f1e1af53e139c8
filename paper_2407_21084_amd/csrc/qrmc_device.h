// qrmc_device.h -- device routines shared by the kernel translation units:
// wave-level ordering, the per-coordinate transcendental calls and the
// closed-form pieces of the manufactured problems.
#pragma once

#include "qrmc_common.h"

namespace qrmc {

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Per-coordinate transcendental work.  Called O(d) times per Euler step
// against O(|Gamma|) basis work, so they stay out of line: their FP64
// coefficients (which this ISA cannot take as literals in three-operand
// instructions) are then materialised per call instead of being hoisted into
// registers that would stay live across the basis traversal.
// ---------------------------------------------------------------------------
__device__ __noinline__ double nl_norm_icdf(double u) { return norm_icdf(u); }
// The logistic law keeps one-argument calls of its own; the other laws go
// through a second set, chosen by a wave-uniform branch at the call site, so
// the default path carries no law argument across the basis traversal.
__device__ __noinline__ double nl_icdf_logistic(double u) { return logistic_icdf(u); }
__device__ __noinline__ double nl_icdf_other(int32_t nu, double u) { return law_icdf(nu, u); }
__device__ __noinline__ double nl_pdf_logistic(double x) {
    const double u = logistic_cdf(x);
    return u * (1.0 - u);
}
__device__ __noinline__ double nl_pdf_other(int32_t nu, double x) { return law_pdf(nu, x, law_cdf(nu, x)); }
__device__ __noinline__ double2 nl_unit_phase_logistic(double x) {
    // e^{2 pi i F(x)}
    double sn, cs;
    sincospi(2.0 * logistic_cdf(x), &sn, &cs);
    return make_double2(cs, sn);
}
// e^{2 pi i F(x)}, or e^{i pi F(x)} for a law code with kLawHalf (the cosine
// basis walks the Fourier tree at half the frequency)
__device__ __noinline__ double2 nl_unit_phase_other(int32_t nu, double x) {
    double sn, cs;
    sincospi(((nu & kLawHalf) ? 1.0 : 2.0) * law_cdf(nu, x), &sn, &cs);
    return make_double2(cs, sn);
}
// d/du of the node e^{i theta k.u} is i theta k e^{...}: theta = 2 pi, or pi
// at half frequency
__device__ __forceinline__ double phase_freq(int32_t nu) { return (nu & kLawHalf) ? M_PI : 2.0 * M_PI; }
// F^{-1}(u), dF/dx at x and e^{2 pi i F(x)} of the law nu (qr_law)
__device__ __forceinline__ double nl_icdf(int32_t nu, double u) {
    return nu == QR_LAW_LOGISTIC ? nl_icdf_logistic(u) : nl_icdf_other(nu, u);
}
__device__ __forceinline__ double nl_pdf(int32_t nu, double x) {
    return nu == QR_LAW_LOGISTIC ? nl_pdf_logistic(x) : nl_pdf_other(nu, x);
}
__device__ __forceinline__ double2 nl_unit_phase(int32_t nu, double x) {
    return nu == QR_LAW_LOGISTIC ? nl_unit_phase_logistic(x) : nl_unit_phase_other(nu, x);
}
// The same with the law stated wave-uniform (readfirstlane: it is the same
// for the whole launch), so that the choice is a scalar branch, not a
// lane-masked one.  Measured: 2.5 % faster for the reduced-precision walk,
// 1.2 % slower for the FP64 path kernel, which keeps the forms above.
__device__ __forceinline__ int32_t uniform_law(int32_t nu) { return __builtin_amdgcn_readfirstlane(nu); }
__device__ __forceinline__ double nl_icdf_u(int32_t nu, double u) {
    return uniform_law(nu) == QR_LAW_LOGISTIC ? nl_icdf_logistic(u) : nl_icdf_other(nu, u);
}
__device__ __forceinline__ double nl_pdf_u(int32_t nu, double x) {
    return uniform_law(nu) == QR_LAW_LOGISTIC ? nl_pdf_logistic(x) : nl_pdf_other(nu, x);
}
__device__ __forceinline__ double2 nl_unit_phase_u(int32_t nu, double x) {
    return uniform_law(nu) == QR_LAW_LOGISTIC ? nl_unit_phase_logistic(x) : nl_unit_phase_other(nu, x);
}
__device__ __noinline__ double2 nl_sincos(double th) {
    // (sin th, cos th); sincospi avoids the large-argument reduction
    double sn, cs;
    sincospi(th * M_1_PI, &sn, &cs);
    return make_double2(sn, cs);
}
__device__ __noinline__ double nl_exp(double a) { return exp(a); }
// damping factor D = (1+|x|^2)^{q/2} of eq (yqi) at the point x (d
// coordinates at stride ldx), and q / (1+|x|^2) = (dD/dx_l) / (D x_l)
__device__ __noinline__ double2 nl_damping_at(const DevProblem *P, const double *x, int64_t ldx) {
    double r2 = 0.0;
    for (int l = 0; l < P->d; ++l) r2 = fma(x[l * ldx], x[l * ldx], r2);
    return make_double2(pow(1.0 + r2, 0.5 * P->dq), P->dq / (1.0 + r2));
}
// the damping factor at the start point X_i of path m, redrawn from stream 0
__device__ __noinline__ double nl_start_damping(const DevProblem *P, uint64_t seed, int64_t m, int32_t i) {
    PhiloxStream rs(seed, 0u, (uint64_t)m, (uint32_t)i, 0u);
    double r2 = 0.0;
    for (int l = 0; l < P->d; ++l) {
        const double x = law_icdf(P->nu, rs.next());
        r2 = fma(x, x, r2);
    }
    return pow(1.0 + r2, 0.5 * P->dq);
}
__device__ __noinline__ double nl_sin(double a) { return sin(a); }
// state-dependent coefficients at (t, x_l): .x = 1 + v_l cos(x_l + omega t),
// the scale of row l of sigma(t,x); .y = b2_l sin(x_l), the bounded drift part
__device__ __noinline__ double2 nl_state_coef(const DevProblem *P, double t, double xl, int l) {
    return make_double2(fma(P->sv[l], cos(fma(P->somega, t, xl)), 1.0), P->b2[l] * sin(xl));
}

// ---------------------------------------------------------------------------
// Manufactured problem pieces (closed forms of u, g, h; see qrmc.h)
// ---------------------------------------------------------------------------
// f_nl(t, x, y, z) with z2 = |z|^2 and uc = u(t, x) (read by QR_F_PAPER only)
__device__ __forceinline__ double fnl(const DevProblem *P, double y, double z2, double uc) {
    switch (P->driver) {
    case QR_F_SIN: return P->f_a * nl_sin(y);
    case QR_F_ALLEN_CAHN: return y - y * y * y;
    case QR_F_ZRAT: return P->f_a * z2 / (1.0 + z2) + y / (1.0 + y * y);
    case QR_F_PAPER: {
        const double e = y - uc;
        return fmin(1.0, e * e);
    }
    default: return 0.0;
    }
}

// h(t, x) into .x and u(t, x) into .y; SDEP: b and sigma at (t, x)
template <int DB, bool SDEP = false>
__device__ __forceinline__ double2 h_source(const DevProblem *P, double t, const double *x, int d) {
    const double E = P->sol_A * nl_exp(-P->sol_c * (P->T - t));
    double th = P->sol_p, bw = 0.0;
#pragma unroll
    for (int l = 0; l < DB; ++l) {
        if (l < d) {
            th = fma(P->sol_w[l], x[l], th);
            bw = fma(fma(P->b1[l], x[l], P->b0[l]), P->sol_w[l], bw);
        }
    }
    double sw2 = P->sw2;             // |sigma^T w|^2
    if constexpr (SDEP) {
        double rs[DB];
#pragma unroll
        for (int l = 0; l < DB; ++l) {
            rs[l] = 0.0;
            if (l < d) {
                const double2 c = nl_state_coef(P, t, x[l], l);
                rs[l] = c.x;
                bw = fma(c.y, P->sol_w[l], bw);
            }
        }
        sw2 = 0.0;
        for (int k = 0; k < P->nbm; ++k) {
            double v = 0.0;
#pragma unroll
            for (int l = 0; l < DB; ++l)
                if (l < d) v = fma(P->sigma[l * P->nbm + k] * rs[l], P->sol_w[l], v);
            sw2 = fma(v, v, sw2);
        }
    }
    const double2 sc = nl_sincos(th);
    const double sn = sc.x, cs = sc.y;
    const double v = E * cs;         // u - B: the offset drops out of every derivative
    const double u = v + P->sol_B;
    const double gscale = -E * sn;  // grad u = gscale * w
    const double z2 = gscale * gscale * sw2;
    return make_double2(-(P->sol_c * v + gscale * bw - 0.5 * v * sw2) - fnl(P, u, z2, u), u);
}

template <int DB>
__device__ __forceinline__ double g_term(const DevProblem *P, const double *x, int d, double *grad) {
    double th = P->sol_p;
#pragma unroll
    for (int l = 0; l < DB; ++l)
        if (l < d) th = fma(P->sol_w[l], x[l], th);
    const double2 sc = nl_sincos(th);
    const double sn = sc.x, cs = sc.y;
    if (grad) {
#pragma unroll
        for (int l = 0; l < DB; ++l)
            if (l < d) grad[l] = -P->sol_A * sn * P->sol_w[l];
    }
    return fma(P->sol_A, cs, P->sol_B);
}

__device__ __forceinline__ double clamp_abs(double y, double L) {
    return y > L ? L : (y < -L ? -L : y);
}


// ---------------------------------------------------------------------------
// 16-bit operands of the matrix cores: two FP32 values rounded to nearest
// (bfloat16 or IEEE half) in one 32-bit word, the first in the low half.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));

template <int PREC>
__device__ __forceinline__ uint32_t pack16x2(float a, float b) {
    if constexpr (PREC == QR_PREC_BF16) {
        const bf16x2_t v = {(__bf16)a, (__bf16)b};
        return __builtin_bit_cast(uint32_t, v);
    } else {
        const f16x2_t v = {(_Float16)a, (_Float16)b};
        return __builtin_bit_cast(uint32_t, v);
    }
}

// ---------------------------------------------------------------------------
// Launch helpers (host)
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int64_t b) { return (unsigned)((n + b - 1) / b); }

constexpr size_t kLdsDefault = 64 * 1024;   // dynamic LDS a launch gets without opting in
constexpr size_t kLdsMax = 160 * 1024;      // LDS of one CU (gfx950)

// Opt a kernel in to `bytes` of dynamic LDS (once per kernel and size).
static inline hipError_t allow_lds(const void *kernel, size_t bytes, size_t &granted) {
    if (bytes <= granted) return hipSuccess;
    if (bytes > kLdsMax) return hipErrorInvalidValue;
    const hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) granted = bytes;
    return e;
}

}  // namespace qrmc
