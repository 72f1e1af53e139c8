// qrmc_kernels.hip -- gfx950 kernels of the QRMC backward step.
//
// One backward iteration i of Algorithm 1 (GQRMDP, eqs (yqi:bar:M),
// (Aqi:bar:M), (Sqi:bar:M)) runs as
//   path_kernel     P paths per thread: start draw X_i ~ nu, Euler steps
//                   (eq (markov:euler)), expansion ybar_{j+1}(X_{j+1}) by the
//                   basis traversal below, driver sum S_i;
//   project_kernel  (task of the traversal) x (slice of paths): the same
//                   traversal at X_i, S-weighted, summed over lanes through
//                   LDS, partial sums per slice;
//   reduce_kernel   fixed-order sum over slices, scaling by 1/M.
//
// Basis traversal.  Every representative k != 0 is its parent (k with the
// last non-zero coordinate l removed) or its previous sibling (|k_l| - 1)
// times one factor e^{+-2 pi i u_l}, so e^{2 pi i k.u} costs one complex
// multiplication: nodes are visited depth-first, coordinates l ascending,
// sign + before -, magnitudes ascending.  All lanes of a wave walk the same
// nodes, so loop bounds are wave-uniform (scalar registers) and the
// coefficient stream is shared by the wave (vector-loaded chunks parked in
// LDS); the per-lane factors e^{2 pi i u_l} sit in LDS and the chain of
// values lives in registers.  A thread carries P points through the walk,
// so the scalar control of each node is paid once for P points' worth of
// FP64 work.
#include "qrmc_kernels.h"
#include "qrmc_device.h"

namespace qrmc {

// values at the P points of a thread, in FP64 (R = double) or, for the
// reduced-precision form, FP32 (R = float)
template <int P, class R = double>
struct Pts {
    R re[P], im[P];
};

template <int P, class R>
__device__ __forceinline__ Pts<P, R> cmul(const Pts<P, R> &a, const Pts<P, R> &b) {
    Pts<P, R> r;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        r.re[q] = fma(a.re[q], b.re[q], -(a.im[q] * b.im[q]));
        r.im[q] = fma(a.re[q], b.im[q], a.im[q] * b.re[q]);
    }
    return r;
}

template <int P, class R = double>
__device__ __forceinline__ Pts<P, R> unit() {
    Pts<P, R> r;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        r.re[q] = 1.0;
        r.im[q] = 0.0;
    }
    return r;
}


// Per-lane LDS slots of a thread's P points: e^{2 pi i u_l} of point q at
// E[(l P + q) stride], gradient accumulators (d ybar / d u_l up to 2 pi) at
// G[(l P + q) stride].
template <class R>
struct Cplx;
template <>
struct Cplx<double> {
    using T = double2;
};
template <>
struct Cplx<float> {
    using T = float2;
};

template <int P, class R = double>
struct LanePts {
    using C2 = typename Cplx<R>::T;
    C2 *E;
    R *G;
    int stride;
    __device__ __forceinline__ Pts<P, R> e(int l) const {
        Pts<P, R> r;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const C2 v = E[(l * P + q) * stride];
            r.re[q] = v.x;
            r.im[q] = v.y;
        }
        return r;
    }
    __device__ __forceinline__ void set_e(int l, int q, C2 v) const { E[(l * P + q) * stride] = v; }
    __device__ __forceinline__ R &g(int l, int q) const { return G[(l * P + q) * stride]; }
};


// ---------------------------------------------------------------------------
// The walk.  A node with budget Pb (product of the weights of its non-zero
// coordinates, or 1 + their sum for the total-degree set) extends along
// coordinate l with magnitudes m = 1, 2, ... as long as its child's budget
// w = Pb (m + b) (or Pb + m) is at most L; the child's budget is w
// (hyperbolic crosses, total degree) or stays 1 (tensor set, c = 0); the
// child has children iff its budget is at most Lc.  See make_walk in
// qrmc_common.h.
// ---------------------------------------------------------------------------
template <int T, int CAP, int P, class R, class Sink>
__device__ __forceinline__ typename Sink::Acc visit(const Pts<P, R> &parent, const int p, const int Pb,
                                                    const Walk &W, const LanePts<P, R> &L, Sink &sink) {
    typename Sink::Acc acc{};
    // (the budget step between magnitudes, W.a ? 1 : Pb, is formed at each
    // increment: a value held across the recursion would cost registers)
#pragma unroll 1
    for (int l = p + 1; l < W.d; ++l) {
        const bool more = l + 1 < W.d;
        [[maybe_unused]] R gl[P];
        if constexpr (Sink::kGrad) {
#pragma unroll
            for (int q = 0; q < P; ++q) gl[q] = 0.0;
        }
#pragma unroll 1
        for (int s = 0; s < (T == 0 ? 1 : 2); ++s) {
            // chain factor e^{+-2 pi i u_l}, re-read per sign to keep one
            // complex value per point live instead of two
            Pts<P, R> es = L.e(l);
            if (s) {
#pragma unroll
                for (int q = 0; q < P; ++q) es.im[q] = -es.im[q];
            }
            Pts<P, R> v = parent;
            [[maybe_unused]] R km = s ? -1.0 : 1.0;
            if constexpr (Sink::kSplit) {
                // Value-only sinks that ask for it: the magnitudes whose node
                // has children (budget w for hyperbolic crosses, Pb for the
                // tensor set, at most Lc, and a later coordinate) come first,
                // since w grows with the magnitude; the rest of the chain, all
                // leaves, runs without the recursion test.
                static_assert(!Sink::kGrad, "split chains are value-only");
                int w = Pb * (1 + W.b) + W.a;
                if constexpr (T + 1 < CAP) {
                    const int wc = more ? (W.c ? W.Lc : (Pb <= W.Lc ? W.L : 0)) : 0;
#pragma unroll 1
                    for (; w <= W.L && w <= wc; w += W.a ? 1 : Pb) {
                        v = cmul(v, es);
                        sink.node(v, acc);
                        Sink::add(acc, visit<T + 1, CAP, P>(v, l, W.c ? w : Pb, W, L, sink));
                    }
                }
                // two leaves per trip, so that the running value alternates
                // between two registers instead of being copied back each node
                const int stp = W.a ? 1 : Pb;
#pragma unroll 1
                for (; w + stp <= W.L; w += 2 * stp) {
                    const Pts<P, R> v2 = cmul(v, es);
                    sink.node(v2, acc);
                    v = cmul(v2, es);
                    sink.node(v, acc);
                }
                if (w <= W.L) {
                    v = cmul(v, es);
                    sink.node(v, acc);
                }
            } else {
                // largest magnitude whose node has children (see above)
                [[maybe_unused]] const int wc = more ? (W.c ? W.Lc : (Pb <= W.Lc ? W.L : 0)) : 0;
#pragma unroll 1
                for (int w = Pb * (1 + W.b) + W.a; w <= W.L; w += W.a ? 1 : Pb) {
                    v = cmul(v, es);
                    if constexpr (Sink::kGrad) {
                        R gs[P];
                        sink.node_g(v, acc, gs);
                        if constexpr (T + 1 < CAP) {
                            if (w <= wc) {
                                const int child = W.c ? w : Pb;
                                const typename Sink::Acc c = visit<T + 1, CAP, P>(v, l, child, W, L, sink);
                                Sink::add(acc, c);
#pragma unroll
                                for (int q = 0; q < P; ++q) gs[q] += c.g[q];
                            }
                        }
#pragma unroll
                        for (int q = 0; q < P; ++q) gl[q] = fma(km, gs[q], gl[q]);
                        km += s ? -1.0 : 1.0;
                    } else {
                        sink.node(v, acc);
                        if constexpr (T + 1 < CAP) {
                            const int child = W.c ? w : Pb;
                            if (more && child <= W.Lc) Sink::add(acc, visit<T + 1, CAP, P>(v, l, child, W, L, sink));
                        }
                    }
                }
            }
        }
        if constexpr (Sink::kGrad) {
#pragma unroll
            for (int q = 0; q < P; ++q) L.g(l, q) += gl[q];
        }
    }
    return acc;
}

// Start the walk below a node of runtime depth `depth` (< CAP).
template <int T, int CAP, int P, class R, class Sink>
__device__ __forceinline__ void visit_from(int depth, const Pts<P, R> &v, int p, int Pb, const Walk &W,
                                           const LanePts<P, R> &L, Sink &sink) {
    if constexpr (T < CAP) {
        if (depth == T) {
            (void)visit<T, CAP, P>(v, p, Pb, W, L, sink);
            return;
        }
        visit_from<T + 1, CAP, P>(depth, v, p, Pb, W, L, sink);
    }
}

// ---------------------------------------------------------------------------
// Expansion evaluation: y = sum_r a_r.x Re(e_r) + a_r.y Im(e_r) with the
// internal coefficients a_r = (sqrt2 alpha_cos, sqrt2 alpha_sin), a_0 =
// (alpha_0, 0); with gradients, g_r = a_r.y Re(e_r) - a_r.x Im(e_r) (d/du of
// the node up to 2 pi k).  The coefficient pair of the next node is requested
// as soon as the current one is consumed, so the scalar load overlaps the
// next node's complex multiply.
// ---------------------------------------------------------------------------
// Value-only walks keep one running sum in the sink (no per-level partial
// sums live across the recursion); with gradients each level returns its
// subtree's value and gradient sums, which the gradient chain needs.
template <int P, bool GRAD>
struct EvalAcc {};
template <int P>
struct EvalAcc<P, true> {
    double y[P], g[P];
};

// Coefficients arrive by vector loads, one 64-node chunk per load (lane q
// holds the pair of node 64c + q), issued a chunk ahead of use.  When the
// walk enters a chunk, the wave stores it to its LDS slot; each node's pair
// is then read from there (one broadcast LDS read, requested a node ahead).
// Vector loads and LDS reads complete in order, so the read-ahead is never
// drained by the wait for the current pair, which is what a scalar-load
// stream has to do on every node.
template <int P, bool GRAD>
struct EvalSink {
    static constexpr bool kGrad = GRAD;
    static constexpr bool kSplit = !GRAD;  // split chains carry no gradient sums
    using Acc = EvalAcc<P, GRAD>;
    double2 *slot;        // this wave's LDS copy of the current chunk [64]
    const double2 *next;  // this lane's entry of the chunk after `buf`
    double2 buf;          // this lane's entry of the next chunk
    double2 pc;           // pair of the node about to be visited
    int n;                // its index (wave-uniform)

    __device__ __forceinline__ void init(const double2 *row, double2 *wave_slot) {
        const int lane = __lane_id();
        const double2 *r = row + lane;
        slot = wave_slot;
        slot[lane] = r[0];
        buf = r[64];
        next = r + 128;
        wave_sync();
        pc = slot[0];
        n = 0;
    }
    __device__ __forceinline__ void coeff(double &cx, double &cy) const {
        cx = pc.x;
        cy = pc.y;
    }
    __device__ __forceinline__ void advance() {
        const int nn = __builtin_amdgcn_readfirstlane(n) + 1;
        n = nn;
        if ((nn & 63) == 0) {
            wave_sync();
            slot[__lane_id()] = buf;
            buf = *next;
            next += 64;
            wave_sync();
        }
        pc = slot[nn & 63];
    }
    double ysum[P];  // value-only walks: the running sum

    __device__ __forceinline__ void node(const Pts<P> &v, Acc &acc) {
        double cx, cy;
        coeff(cx, cy);
#pragma unroll
        for (int q = 0; q < P; ++q) {
            if constexpr (GRAD)
                acc.y[q] = fma(cx, v.re[q], fma(cy, v.im[q], acc.y[q]));
            else
                ysum[q] = fma(cx, v.re[q], fma(cy, v.im[q], ysum[q]));
        }
        advance();
    }
    __device__ __forceinline__ void node_g(const Pts<P> &v, Acc &acc, double *gs) {
        double cx, cy;
        coeff(cx, cy);
#pragma unroll
        for (int q = 0; q < P; ++q) {
            acc.y[q] = fma(cx, v.re[q], fma(cy, v.im[q], acc.y[q]));
            gs[q] = fma(cy, v.re[q], -(cx * v.im[q]));
            if constexpr (GRAD) acc.g[q] += gs[q];
        }
        advance();
    }
    __device__ __forceinline__ static void add(Acc &x, const Acc &y) {
        if constexpr (GRAD) {
#pragma unroll
            for (int q = 0; q < P; ++q) {
                x.y[q] += y.y[q];
                x.g[q] += y.g[q];
            }
        }
    }
};

// ybar at the thread's P points.  The row is zero-padded to a whole number
// of 64-node chunks plus two (read ahead); wave_slot is the wave's LDS chunk
// slot (64 double2).  With vector-loaded coefficients every lane of the wave
// must be active.
template <int CAP, int P, bool GRAD>
__device__ __forceinline__ void tree_eval(const double2 *alpha_row, double2 *wave_slot, const Walk &W,
                                          const LanePts<P> &L, double *y) {
    EvalSink<P, GRAD> s;
    s.init(alpha_row, wave_slot);
#pragma unroll
    for (int q = 0; q < P; ++q) s.ysum[q] = 0.0;
    typename EvalSink<P, GRAD>::Acc root{};
    const Pts<P> one = unit<P>();
    s.node(one, root);
    const auto acc = visit<0, CAP, P>(one, -1, 1, W, L, s);
#pragma unroll
    for (int q = 0; q < P; ++q) {
        if constexpr (GRAD)
            y[q] = root.y[q] + acc.y[q];
        else
            y[q] = s.ysum[q];
    }
}

// ---------------------------------------------------------------------------
// path_kernel: P paths per thread of backward iteration i.  Thread t of
// block b carries paths m_q = b kPathBlock P + q kPathBlock + t.
// alpha_int rows have stride ld = coef_ld(nrep) double2.
// LDS per thread: E slots [d][P] double2, gradient slots [d][P] double
// (GRAD); per wave a 64-pair coefficient chunk.  The path state lives in
// HBM (xg, [d][ldx]).
// ---------------------------------------------------------------------------
size_t path_lds_bytes(int32_t d, bool grad, int P) {
    return (size_t)d * kPathBlock * P * (sizeof(double2) + (grad ? sizeof(double) : 0)) +
           (size_t)(kPathBlock / 64) * 64 * sizeof(double2);
}

// Three waves per SIMD (168 VGPRs): a few spills of values that live across
// the whole traversal cost less than the latency the third wave hides
// (measured; also for the gradient walk, where 256 VGPRs and two waves were
// slower).
#ifndef QRMC_PATH_WAVES_PER_EU
#define QRMC_PATH_WAVES_PER_EU 3
#endif
// FEAT: 0 the plain problem, 1 a damping exponent q > 0, 2 also the
// state-dependent drift and diffusion (each its own instances, so that the
// plain kernels carry no code for either; with q = 0 the damping code is
// exact: D = 1 and its gradient term vanishes).
template <int DB, int CAP, bool GRAD, int P, int FEAT>
__global__ __launch_bounds__(kPathBlock)
__attribute__((amdgpu_waves_per_eu(QRMC_PATH_WAVES_PER_EU)))
void path_kernel(
    const DevProblem *__restrict__ P0, const Walk W, const int32_t i, const int64_t M,
    const uint64_t seed, const double2 *__restrict__ alpha_int, const int64_t ld,
    double *__restrict__ S_out, double2 *__restrict__ e_out, double *__restrict__ x_out,
    double *__restrict__ xg, const int64_t ldx, double *__restrict__ f0_out) {
    constexpr bool DAMP = FEAT >= 1, SDEP = FEAT == 2;
    extern __shared__ double2 lds[];
    const int tid = threadIdx.x;
    const int d = P0->d, nbm = P0->nbm, N = P0->N;
    const LanePts<P> L{lds + tid,
                       GRAD ? reinterpret_cast<double *>(lds + d * P * kPathBlock) + tid : nullptr,
                       kPathBlock};
    // coefficient chunk slot of this wave, after the per-lane slots
    double2 *wave_slot = reinterpret_cast<double2 *>(reinterpret_cast<double *>(lds + d * P * kPathBlock) +
                                                     (GRAD ? d * P * kPathBlock : 0)) +
                         (tid >> 6) * 64;

    const int64_t base = (int64_t)blockIdx.x * kPathBlock * P + tid;
    // path state parked in HBM ([d][ldx], this thread's points at base +
    // q kPathBlock) while the traversal runs
    xg += base;
    double S[P];
    // start points X_i^i = F^{-1}(U), U from stream 0 draws r = 0..d-1
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int64_t m = base + (int64_t)q * kPathBlock;
        PhiloxStream rs(seed, 0u, (uint64_t)m, (uint32_t)i, 0u);
        for (int l = 0; l < d; ++l) {
            const double x = nl_icdf(P0->nu, rs.next());
            xg[l * ldx + q * kPathBlock] = x;
            if (m < M) {
                if (e_out) e_out[l * M + m] = nl_unit_phase(P0->nu, x);
                if (x_out) x_out[l * M + m] = x;
            }
        }
        S[q] = 0.0;
    }

    for (int j = i; j < N; ++j) {
        // Re-read the problem each step instead of pinning every parameter in
        // scalar registers across the basis traversal.
        const DevProblem *__restrict__ Pj = P0;
        asm volatile("" : "+s"(Pj));
        const double tj = Pj->t[j];
        const double dt = Pj->t[j + 1] - tj;
        const double sq = sqrt(dt);
        double hj[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int64_t m = base + (int64_t)q * kPathBlock;
            double x[DB];
#pragma unroll
            for (int l = 0; l < DB; ++l) x[l] = (l < d) ? xg[l * ldx + q * kPathBlock] : 0.0;
            // the source term only needs X_j; the Sec. 5 driver also reads
            // u(t_j, X_j), parked in the path state's row d
            const double2 hu = h_source<DB, SDEP>(Pj, tj, x, d);
            hj[q] = hu.x;
            if (Pj->driver == QR_F_PAPER) xg[d * ldx + q * kPathBlock] = hu.y;
            // Euler step, eq (markov:euler): normals r = d + (j-i) nbm + k
            PhiloxStream rs(seed, 0u, (uint64_t)m, (uint32_t)i, (uint32_t)(d + (j - i) * nbm));
            if constexpr (SDEP) {
                // b and sigma at (t_j, X_j): the noise of row l is scaled as a whole
                double sc[DB], nz[DB];
#pragma unroll
                for (int l = 0; l < DB; ++l) {
                    sc[l] = 0.0;
                    nz[l] = 0.0;
                    if (l < d) {
                        const double2 c = nl_state_coef(Pj, tj, x[l], l);
                        sc[l] = c.x;
                        x[l] = fma(fma(Pj->b1[l], x[l], Pj->b0[l]) + c.y, dt, x[l]);
                    }
                }
#pragma unroll 1
                for (int k = 0; k < nbm; ++k) {
                    const double dwk = sq * nl_norm_icdf(rs.next());
#pragma unroll
                    for (int l = 0; l < DB; ++l)
                        if (l < d) nz[l] = fma(Pj->sigma[l * nbm + k], dwk, nz[l]);
                }
#pragma unroll
                for (int l = 0; l < DB; ++l)
                    if (l < d) x[l] = fma(sc[l], nz[l], x[l]);
            } else {
#pragma unroll
                for (int l = 0; l < DB; ++l)
                    if (l < d) x[l] = fma(fma(Pj->b1[l], x[l], Pj->b0[l]), dt, x[l]);
#pragma unroll 1
                for (int k = 0; k < nbm; ++k) {
                    const double dwk = sq * nl_norm_icdf(rs.next());
#pragma unroll
                    for (int l = 0; l < DB; ++l)
                        if (l < d) x[l] = fma(Pj->sigma[l * nbm + k], dwk, x[l]);
                }
            }
#pragma unroll
            for (int l = 0; l < DB; ++l)
                if (l < d) xg[l * ldx + q * kPathBlock] = x[l];
        }
        // xs now holds X_{j+1}
        double y[P];
        double z2[P];
        if (j + 1 < N) {
            for (int l = 0; l < d; ++l) {
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    L.set_e(l, q, nl_unit_phase(Pj->nu, xg[l * ldx + q * kPathBlock]));
                    if constexpr (GRAD) L.g(l, q) = 0.0;
                }
            }
            tree_eval<CAP, P, GRAD>(alpha_int + (int64_t)(j + 1) * ld, wave_slot, W, L, y);
#pragma unroll
            for (int q = 0; q < P; ++q) {
                z2[q] = 0.0;
                // with damping the expansion is ybar^{(q)} = y / D, D = (1+|x|^2)^{q/2}
                // (eq (yqi)): y = ybar D, grad y = D (grad ybar + ybar q x / (1+|x|^2))
                [[maybe_unused]] double2 D = make_double2(1.0, 0.0);
                if constexpr (DAMP) D = nl_damping_at(Pj, xg + q * kPathBlock, ldx);
                if constexpr (GRAD) {
                    double gx[DB];
#pragma unroll
                    for (int l = 0; l < DB; ++l) {
                        gx[l] = 0.0;
                        if (l < d) {
                            const double xv = xg[l * ldx + q * kPathBlock];
                            gx[l] = phase_freq(Pj->nu) * L.g(l, q) * nl_pdf(Pj->nu, xv);
                            if constexpr (DAMP) gx[l] = D.x * fma(y[q] * D.y, xv, gx[l]);
                            // z = sigma(t_{j+1}, X_{j+1})^T grad y
                            if constexpr (SDEP) gx[l] *= nl_state_coef(Pj, Pj->t[j + 1], xv, l).x;
                        }
                    }
                    for (int k = 0; k < nbm; ++k) {
                        double zk = 0.0;
#pragma unroll
                        for (int l = 0; l < DB; ++l)
                            if (l < d) zk = fma(Pj->sigma[l * nbm + k], gx[l], zk);
                        z2[q] = fma(zk, zk, z2[q]);
                    }
                }
                if constexpr (DAMP) y[q] *= D.x;
            }
        } else {
#pragma unroll
            for (int q = 0; q < P; ++q) {
                double x[DB], gx[DB];
#pragma unroll
                for (int l = 0; l < DB; ++l) x[l] = (l < d) ? xg[l * ldx + q * kPathBlock] : 0.0;
                y[q] = g_term<DB>(Pj, x, d, GRAD ? gx : nullptr);
                z2[q] = 0.0;
                if constexpr (GRAD) {
                    if constexpr (SDEP) {
#pragma unroll
                        for (int l = 0; l < DB; ++l)
                            if (l < d) gx[l] *= nl_state_coef(Pj, Pj->T, x[l], l).x;
                    }
                    for (int k = 0; k < nbm; ++k) {
                        double zk = 0.0;
#pragma unroll
                        for (int l = 0; l < DB; ++l)
                            if (l < d) zk = fma(Pj->sigma[l * nbm + k], gx[l], zk);
                        z2[q] = fma(zk, zk, z2[q]);
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const double yq = clamp_abs(y[q], Pj->clamp);
            const double uc = Pj->driver == QR_F_PAPER ? xg[d * ldx + q * kPathBlock] : 0.0;
            const double f = fnl(Pj, yq, z2[q], uc) + hj[q];
            S[q] = fma(f, dt, S[q]);
            if (f0_out && j == i) {
                // for the Z regression: the first term (the multistep responses
                // leave it out) and the value the driver read on that step
                const int64_t m = base + (int64_t)q * kPathBlock;
                if (m < M) {
                    f0_out[m] = S[q];
                    f0_out[M + m] = yq;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int64_t m = base + (int64_t)q * kPathBlock;
        double x[DB];
#pragma unroll
        for (int l = 0; l < DB; ++l) x[l] = (l < d) ? xg[l * ldx + q * kPathBlock] : 0.0;
        double Sq = S[q] + g_term<DB>(P0, x, d, nullptr);
        // the response of the damped quantity (Algorithm 1): over (1+|X_i|^2)^{q/2}
        if constexpr (DAMP) Sq /= nl_start_damping(P0, seed, m, i);
        if (m < M) S_out[m] = Sq;
    }
}

// ---------------------------------------------------------------------------
// project_kernel: block (task of the traversal, slice of paths).  Each wave
// runs 64 P paths at a time through the task's nodes (P per lane); per node,
// a lane forms the S-weighted sum of its points' values, the sums are folded
// across the lanes four nodes at a time (below) into per-wave accumulators,
// and the block finally adds its waves in a fixed order and writes the
// slice's partial sums.
// ---------------------------------------------------------------------------
// Cross-lane sums of the projection, four nodes at a time, in registers.
// The real and imaginary parts of a node are folded across lanes L and L^32
// (v_permlane32_swap: one half of the wave keeps the real parts, the other the
// imaginary ones), two such nodes across L^16 (v_permlane16_swap), two pairs
// across the mirror lane of a row of 16 (DPP row_mirror, bit 3 differs), and
// the three low lane bits by DPP mirrors and quad permutes.  Each lane then
// holds the full 64-lane sum of one (node, part) of the group, the same value
// in eight lanes.  Which one is found once per kernel by running the same folds
// on indicator values (fold_slot), so nothing depends on which half of a swap
// keeps which operand.  The order of every addition is fixed.
__device__ __forceinline__ uint32_t lo32(double x) { return (uint32_t)__double_as_longlong(x); }
__device__ __forceinline__ uint32_t hi32(double x) {
    return (uint32_t)((uint64_t)__double_as_longlong(x) >> 32);
}
__device__ __forceinline__ double from32(uint32_t lo, uint32_t hi) {
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
// a kept by one half of the wave, b by the other; each lane gets its half's
// value summed with the partner lane's
__device__ __forceinline__ double fold32(double a, double b) {
    const auto l = __builtin_amdgcn_permlane32_swap(lo32(a), lo32(b), false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi32(a), hi32(b), false, false);
    return from32(l[0], h[0]) + from32(l[1], h[1]);
}
__device__ __forceinline__ double fold16(double a, double b) {
    const auto l = __builtin_amdgcn_permlane16_swap(lo32(a), lo32(b), false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi32(a), hi32(b), false, false);
    return from32(l[0], h[0]) + from32(l[1], h[1]);
}
constexpr int kDppRowMirror = 0x140;      // lane i <- 15 - i within a row of 16
constexpr int kDppRowHalfMirror = 0x141;  // lane i <- 7 - i within 8
constexpr int kDppQuadXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppQuadXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
template <int CTRL>
__device__ __forceinline__ double dpp_read(double x) {
    // every source lane of these patterns exists, so bound_ctrl never applies
    return from32((uint32_t)__builtin_amdgcn_mov_dpp((int)lo32(x), CTRL, 0xf, 0xf, true),
                  (uint32_t)__builtin_amdgcn_mov_dpp((int)hi32(x), CTRL, 0xf, 0xf, true));
}
// lanes with bit 3 clear keep a, the others b; each adds its mirror lane's
__device__ __forceinline__ double fold8(double a, double b, bool bit3) {
    const double send = bit3 ? a : b;
    const double keep = bit3 ? b : a;
    return keep + dpp_read<kDppRowMirror>(send);
}
// plain sum over the eight lanes that differ in bits 0..2
__device__ __forceinline__ double fold_low(double f) {
    f += dpp_read<kDppRowHalfMirror>(f);
    f += dpp_read<kDppQuadXor2>(f);
    f += dpp_read<kDppQuadXor1>(f);
    return f;
}
// 2 j + part of the sum a lane holds after the folds of nodes j = 0..3
// (indicators 2^(2j+part) entered on lane 0; every lane of the wave active)
__device__ __forceinline__ int fold_slot(int lane) {
    double h[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        h[j] = fold32(lane == 0 ? (double)(1 << (2 * j)) : 0.0, lane == 0 ? (double)(2 << (2 * j)) : 0.0);
    const double f = fold_low(fold8(fold16(h[0], h[1]), fold16(h[2], h[3]), (lane >> 3) & 1));
    return __builtin_ctz((uint32_t)f | 256u) & 7;
}

template <int P>
struct ProjSink {
    static constexpr bool kGrad = false;
    static constexpr bool kSplit = false;  // measured: slower at d = 10
    struct Acc {};
    __device__ __forceinline__ static void add(Acc &, const Acc &) {}
    double *acc;     // wave accumulators, doubles [task_max][2]
    double s[P];     // the lane's responses (0 for paths past the slice)
    double b1, b2;   // folds of the group's first node and of its first pair
    int c;           // nodes of the current group taken, 0..3 (wave-uniform)
    int base;        // task-local index of the group's first node (wave-uniform)
    int slot;        // fold_slot of this lane
    bool lead;       // one lane of the eight holding a sum adds it to acc
    bool bit3;

    __device__ __forceinline__ void take(double re, double im) {
        const double h = fold32(re, im);
        if (!(c & 1)) {
            b1 = h;
        } else {
            const double g = fold16(b1, h);
            if (!(c & 2)) {
                b2 = g;
            } else {
                const double f = fold_low(fold8(b2, g, bit3));
                if (lead) acc[base * 2 + slot] += f;
                base += 4;
            }
        }
        c = (c + 1) & 3;
    }

    __device__ __forceinline__ void node(const Pts<P> &v, Acc &) {
        double re = s[0] * v.re[0], im = s[0] * v.im[0];
#pragma unroll
        for (int q = 1; q < P; ++q) {
            re = fma(s[q], v.re[q], re);
            im = fma(s[q], v.im[q], im);
        }
        take(re, im);
    }

    // complete a partial group with zero nodes
    __device__ __forceinline__ void flush() {
        while (c) take(0.0, 0.0);
    }
};

// The same folds for R responses per point (the members of a batched pass on
// their shared cloud): node n of the task and response r form the virtual node
// n R + r, so the wave accumulators are [task_max][R][2] and a group of four
// takes holds four responses of one node (R is a multiple of 4).
template <int P, int R>
struct ProjSinkR {
    static_assert(R % 4 == 0, "groups of four takes must stay within a node");
    static constexpr bool kGrad = false;
    static constexpr bool kSplit = false;
    struct Acc {};
    __device__ __forceinline__ static void add(Acc &, const Acc &) {}
    ProjSink<P> f;     // the fold state (f.s unused)
    double s[R][P];    // the lane's responses per member (0 past the member's cloud)

    __device__ __forceinline__ void node(const Pts<P> &v, Acc &) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double re = s[r][0] * v.re[0], im = s[r][0] * v.im[0];
#pragma unroll
            for (int q = 1; q < P; ++q) {
                re = fma(s[r][q], v.re[q], re);
                im = fma(s[r][q], v.im[q], im);
            }
            f.take(re, im);
        }
    }
    __device__ __forceinline__ void flush() { f.flush(); }
};

static size_t project_lds_bytes(int32_t d, int P, int waves, int task_max) {
    return (size_t)waves * task_max * 2 * sizeof(double) + (size_t)d * P * 64 * sizeof(double2) +
           (size_t)P * 64 * sizeof(double);
}

// Block (group of WAVES tasks, slice of paths): wave w walks task
// blockIdx.x WAVES + w, and all waves walk the same 64 P paths at a time,
// whose phase factors and responses the block stages once per batch in LDS
// (so a slice is read once per group of tasks, not once per task).  Each
// wave folds its own task's sums (ProjSink) into its accumulators and writes
// them as the slice's partial sums of that task.  Tasks are ordered by size,
// so the waves of a block finish a batch at about the same time.
template <int CAP, int P, int WAVES, int TM>
__global__ __launch_bounds__(WAVES * 64) void project_kernel(
    const Walk W, const double2 *__restrict__ e_in, const int64_t lde, const double *__restrict__ s_in,
    const int64_t M, const int64_t paths_per_split, const int32_t ntasks, const Task *__restrict__ tasks,
    const TaskItem *__restrict__ items, double2 *__restrict__ partial, const int64_t nrep) {
    static_assert(TM % 4 == 0, "groups of four nodes must tile a task");
    constexpr int NT = WAVES * 64, B = 64 * P;
    extern __shared__ double2 lds[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int d = W.d;
    double *accs = reinterpret_cast<double *>(lds);                          // [WAVES][TM][2]
    double2 *Es = reinterpret_cast<double2 *>(accs + WAVES * TM * 2);         // [d][P][64]
    double *Ss = reinterpret_cast<double *>(Es + d * B);                     // [P][64]

    double *acc = accs + wave * TM * 2;
    const LanePts<P> L{Es + lane, nullptr, 64};

    const int32_t t = (int32_t)blockIdx.x * WAVES + wave;
    const bool active = t < ntasks;  // wave-uniform
    const Task task = active ? tasks[t] : Task{0, 0, 0, 0};
    const int64_t m0 = (int64_t)blockIdx.y * paths_per_split;
    const int64_t m1 = min(M, m0 + paths_per_split);

    for (int r = lane; r < TM * 2; r += 64) acc[r] = 0.0;

    ProjSink<P> sink;
    sink.acc = acc;
    sink.slot = fold_slot(lane);
    sink.lead = (lane & 7) == 0;
    sink.bit3 = (lane >> 3) & 1;
    const int ne = d * B;
    for (int64_t gb = m0; gb < m1; gb += B) {
        __syncthreads();  // every wave is done with the previous batch
        // entry j = (l P + q) 64 + lane' holds coordinate l of path gb + q 64 + lane'
        for (int j = tid; j < ne; j += NT) {
            const int l = j / B, r = j - l * B;
            const int64_t m = gb + r;
            Es[j] = m < m1 ? e_in[l * lde + m] : make_double2(1.0, 0.0);
        }
        for (int j = tid; j < B; j += NT) {
            const int64_t m = gb + j;
            Ss[j] = m < m1 ? s_in[m] : 0.0;
        }
        __syncthreads();
        if (!active) continue;
#pragma unroll
        for (int q = 0; q < P; ++q) sink.s[q] = Ss[q * 64 + lane];
        sink.c = 0;
        sink.base = 0;
        for (int it = task.item_begin; it < task.item_end; ++it) {
            const TaskItem &I = items[it];
            Pts<P> v = unit<P>();
            for (int k = 0; k < I.depth; ++k) {
                Pts<P> e = L.e(I.coord[k]);
                int n = I.val[k];
                if (n < 0) {
#pragma unroll
                    for (int q = 0; q < P; ++q) e.im[q] = -e.im[q];
                    n = -n;
                }
                for (int r = 0; r < n; ++r) v = cmul(v, e);
            }
            typename ProjSink<P>::Acc none;
            sink.node(v, none);
            if (I.full) visit_from<0, CAP, P>(I.depth, v, I.last, I.prod, W, L, sink);
        }
        if (sink.c) sink.flush();
    }
    if (!active) return;
    wave_sync();
    double *out = reinterpret_cast<double *>(partial + (int64_t)blockIdx.y * nrep + task.rep_begin);
    for (int r = lane; r < task.rep_count * 2; r += 64) out[r] = acc[r];
}

// Evaluation with the basis split across blocks, for point sets too small
// to fill the chip one walk per thread: block (group of WAVES tasks, slice of
// points) as in project_kernel; wave w holds the coefficients of task
// WAVES blockIdx.x + w in LDS and sums, per lane, a_r.x Re + a_r.y Im over the
// task's nodes for its P points; per batch the waves' sums are added in wave
// order and written to partial[group][m] (sum_groups_kernel adds the groups).
template <int P>
struct TaskEvalSink {
    static constexpr bool kGrad = false;
    static constexpr bool kSplit = true;
    struct Acc {};
    __device__ __forceinline__ static void add(Acc &, const Acc &) {}
    const double2 *coef;  // the task's coefficient pairs in LDS, task-local traversal order
    int n;                // task-local index of the next node (wave-uniform)
    double y[P];
    __device__ __forceinline__ void node(const Pts<P> &v, Acc &) {
        const double2 a = coef[n++];
#pragma unroll
        for (int q = 0; q < P; ++q) y[q] = fma(a.x, v.re[q], fma(a.y, v.im[q], y[q]));
    }
};

static size_t eval_tasks_lds_bytes(int32_t d, int P, int waves, int task_max) {
    return (size_t)waves * task_max * sizeof(double2) + (size_t)d * P * 64 * sizeof(double2) +
           (size_t)waves * P * 64 * sizeof(double);
}

template <int CAP, int P, int WAVES, int TM>
__global__ __launch_bounds__(WAVES * 64) void eval_tasks_kernel(
    const Walk W, const double2 *__restrict__ e_in, const int64_t n, const int64_t points_per_split,
    const int32_t ntasks, const Task *__restrict__ tasks, const TaskItem *__restrict__ items,
    const double2 *__restrict__ row, double *__restrict__ partial) {
    constexpr int NT = WAVES * 64, B = 64 * P;
    extern __shared__ double2 lds[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int d = W.d;
    double2 *cw = lds + wave * TM;                                     // [WAVES][TM]
    double2 *Es = lds + WAVES * TM;                                    // [d][P][64]
    double *Ys = reinterpret_cast<double *>(Es + d * B);               // [WAVES][P][64]
    const LanePts<P> L{Es + lane, nullptr, 64};

    const int32_t t = (int32_t)blockIdx.x * WAVES + wave;
    const bool active = t < ntasks;  // wave-uniform
    const Task task = active ? tasks[t] : Task{0, 0, 0, 0};
    for (int r = lane; r < task.rep_count; r += 64) cw[r] = row[task.rep_begin + r];
    const int64_t m0 = (int64_t)blockIdx.y * points_per_split;
    const int64_t m1 = min(n, m0 + points_per_split);

    TaskEvalSink<P> sink;
    sink.coef = cw;
    const int ne = d * B;
    for (int64_t gb = m0; gb < m1; gb += B) {
        __syncthreads();  // the previous batch's readers of Es and Ys are done
        for (int j = tid; j < ne; j += NT) {
            const int l = j / B, r = j - l * B;
            const int64_t m = gb + r;
            Es[j] = m < m1 ? e_in[l * n + m] : make_double2(1.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < P; ++q) sink.y[q] = 0.0;
        if (active) {
            sink.n = 0;
            for (int it = task.item_begin; it < task.item_end; ++it) {
                const TaskItem &I = items[it];
                Pts<P> v = unit<P>();
                for (int k = 0; k < I.depth; ++k) {
                    Pts<P> e = L.e(I.coord[k]);
                    int nn = I.val[k];
                    if (nn < 0) {
#pragma unroll
                        for (int q = 0; q < P; ++q) e.im[q] = -e.im[q];
                        nn = -nn;
                    }
                    for (int r = 0; r < nn; ++r) v = cmul(v, e);
                }
                typename TaskEvalSink<P>::Acc none;
                sink.node(v, none);
                if (I.full) visit_from<0, CAP, P>(I.depth, v, I.last, I.prod, W, L, sink);
            }
        }
#pragma unroll
        for (int q = 0; q < P; ++q) Ys[(wave * P + q) * 64 + lane] = sink.y[q];
        __syncthreads();
        for (int j = tid; j < B; j += NT) {
            const int64_t m = gb + j;
            if (m < m1) {
                double acc = 0.0;
#pragma unroll
                for (int w = 0; w < WAVES; ++w) acc += Ys[w * B + j];
                partial[(int64_t)blockIdx.x * n + m] = acc;
            }
        }
    }
}

__global__ void sum_groups_kernel(const double *__restrict__ partial, int32_t ngroups, int64_t n,
                                  double *__restrict__ y) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double acc = 0.0;
    for (int32_t g = 0; g < ngroups; ++g) acc += partial[(int64_t)g * n + m];
    y[m] = acc;
}

// project_pass_kernel: the projection of a batched pass, R members on the pass's
// cloud at once (one walk of the pass's set and one read of the phase factors
// per point for all members): member r's response at path m is S[r M + m]
// for m < m_r and 0 beyond (its own cloud is the first m_r paths).  Partial
// sums [split][node][R] (double2); the members' own nodes are picked and
// scaled by reduce_batched_kernel.
template <int CAP, int P, int R, int WAVES, int TM>
__global__ __launch_bounds__(WAVES * 64) void project_pass_kernel(
    const Walk W, const double2 *__restrict__ e_in, const int64_t lde, const double *__restrict__ s_in,
    const int64_t M, const int64_t *__restrict__ m_r, const int64_t paths_per_split, const Task *__restrict__ tasks,
    const TaskItem *__restrict__ items, double2 *__restrict__ partial, const int64_t nrep) {
    static_assert(TM % 4 == 0, "groups of four nodes must tile a task");
    extern __shared__ double2 lds[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int d = W.d;
    double *accs = reinterpret_cast<double *>(lds);   // [WAVES][TM][R][2]
    double2 *Es = lds + WAVES * TM * R;              // [WAVES][d][P][64]

    double *acc = accs + wave * TM * R * 2;
    const LanePts<P> L{Es + wave * d * P * 64 + lane, nullptr, 64};

    const Task task = tasks[blockIdx.x];
    const int64_t m0 = (int64_t)blockIdx.y * paths_per_split;
    const int64_t m1 = min(M, m0 + paths_per_split);
    int64_t mr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) mr[r] = m_r[r];

    for (int r = lane; r < TM * R * 2; r += 64) acc[r] = 0.0;
    wave_sync();

    ProjSinkR<P, R> sink;
    sink.f.acc = acc;
    sink.f.slot = fold_slot(lane);
    sink.f.lead = (lane & 7) == 0;
    sink.f.bit3 = (lane >> 3) & 1;
    for (int64_t gb = m0 + wave * 64 * P; gb < m1; gb += WAVES * 64 * P) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int64_t m = gb + q * 64 + lane;
            const bool live = m < m1;
#pragma unroll
            for (int r = 0; r < R; ++r) sink.s[r][q] = (live && m < mr[r]) ? s_in[r * M + m] : 0.0;
            for (int l = 0; l < d; ++l) L.set_e(l, q, live ? e_in[l * lde + m] : make_double2(1.0, 0.0));
        }
        sink.f.c = 0;
        sink.f.base = 0;
        for (int it = task.item_begin; it < task.item_end; ++it) {
            const TaskItem &I = items[it];
            Pts<P> v = unit<P>();
            for (int t = 0; t < I.depth; ++t) {
                Pts<P> e = L.e(I.coord[t]);
                int n = I.val[t];
                if (n < 0) {
#pragma unroll
                    for (int q = 0; q < P; ++q) e.im[q] = -e.im[q];
                    n = -n;
                }
                for (int k = 0; k < n; ++k) v = cmul(v, e);
            }
            typename ProjSinkR<P, R>::Acc none;
            sink.node(v, none);
            if (I.full) visit_from<0, CAP, P>(I.depth, v, I.last, I.prod, W, L, sink);
        }
        if (sink.f.c) sink.flush();
    }
    __syncthreads();
    double *out = reinterpret_cast<double *>(partial + ((int64_t)blockIdx.y * nrep + task.rep_begin) * R);
    for (int r = tid; r < task.rep_count * R * 2; r += WAVES * 64) {
        double sacc = 0.0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) sacc += accs[w * TM * R * 2 + r];
        out[r] = sacc;
    }
}

// ---------------------------------------------------------------------------
// reduce_kernel: alpha_i from the slice partial sums, fixed order
// ---------------------------------------------------------------------------
__global__ void reduce_kernel(const double2 *__restrict__ partial, int32_t nsplit, int64_t nrep,
                              double M, double2 *__restrict__ alpha_int_row,
                              double *__restrict__ alpha_row,
                              const int32_t *__restrict__ canon_of_trav, int32_t *__restrict__ bad,
                              int32_t step) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep) return;
    double sx = 0.0, sy = 0.0;
    for (int s = 0; s < nsplit; ++s) {
        const double2 p = partial[(int64_t)s * nrep + r];
        sx += p.x;
        sy += p.y;
    }
    if (bad && !(isfinite(sx) && isfinite(sy))) atomicMax(bad, step);
    if (r == 0) {
        const double a0 = sx / M;
        alpha_int_row[0] = make_double2(a0, 0.0);
        if (alpha_row) alpha_row[0] = a0;
    } else {
        const double mc = sx / M, ms = sy / M;
        // the kernels' row is formed from the rounded public coefficients,
        // exactly as gather_kernel forms it from a stored row: a solve then
        // equals its steps run one by one, and resumes from saved rows, bit
        // for bit
        const double ac = M_SQRT2 * mc, as = M_SQRT2 * ms;
        alpha_int_row[r] = make_double2(M_SQRT2 * ac, M_SQRT2 * as);
        if (alpha_row) {
            const int64_t c = canon_of_trav[r];
            alpha_row[2 * c - 1] = ac;
            alpha_row[2 * c] = as;
        }
    }
}

// canonical rows [row0, row0+nrows) -> internal traversal-order rows (stride ld)
__global__ void gather_kernel(const double *__restrict__ alpha, int32_t row0, int32_t nrows,
                              int64_t nrep, int64_t ld, int64_t nfuncs,
                              const int32_t *__restrict__ canon_of_trav,
                              double2 *__restrict__ alpha_int) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nrows * nrep) return;
    const int64_t row = row0 + idx / nrep, r = idx % nrep;
    const double *src = alpha + row * nfuncs;
    const int64_t c = canon_of_trav[r];
    alpha_int[row * ld + r] = (r == 0) ? make_double2(src[0], 0.0)
                                       : make_double2(M_SQRT2 * src[2 * c - 1],
                                                      M_SQRT2 * src[2 * c]);
}

// zero the padding entries [nrep, ld) of rows [0, nrows)
__global__ void pad_kernel(int32_t nrows, int64_t nrep, int64_t ld, double2 *__restrict__ alpha_int) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t padn = ld - nrep;
    if (idx >= (int64_t)nrows * padn) return;
    alpha_int[(idx / padn) * ld + nrep + idx % padn] = make_double2(0.0, 0.0);
}

// ---------------------------------------------------------------------------
// eval_kernel: ybar (and its x-gradient) at given points, one thread each
// ---------------------------------------------------------------------------
template <int CAP, bool GRAD>
__global__ __launch_bounds__(kPathBlock) void eval_kernel(const Walk W,
                                                          const double2 *__restrict__ alpha_int_row,
                                                          const double *__restrict__ x,
                                                          const int64_t n, double *__restrict__ y,
                                                          double *__restrict__ grad) {
    extern __shared__ double2 lds[];
    const int tid = threadIdx.x;
    const int64_t pl = (int64_t)blockIdx.x * kPathBlock + tid;
    const bool live = pl < n;
    const int64_t p = live ? pl : n - 1;  // every lane walks: the coefficient stream is shared by the wave
    const int d = W.d;
    const LanePts<1> L{lds + tid, GRAD ? reinterpret_cast<double *>(lds + d * kPathBlock) + tid : nullptr,
                       kPathBlock};
    for (int l = 0; l < d; ++l) {
        L.set_e(l, 0, nl_unit_phase(W.nu, x[l * n + p]));
        if constexpr (GRAD) L.g(l, 0) = 0.0;
    }
    double2 *wave_slot = reinterpret_cast<double2 *>(reinterpret_cast<double *>(lds + d * kPathBlock) +
                                                     (GRAD ? d * kPathBlock : 0)) +
                         (tid >> 6) * 64;
    double yv;
    tree_eval<CAP, 1, GRAD>(alpha_int_row, wave_slot, W, L, &yv);
    if (!live) return;
    y[p] = yv;
    if constexpr (GRAD) {
        for (int l = 0; l < d; ++l) {
            grad[l * n + p] = phase_freq(W.nu) * L.g(l, 0) * nl_pdf(W.nu, x[l * n + p]);
        }
    }
}

__global__ void x_to_e_kernel(int32_t nu, int32_t d, const double *__restrict__ x, int64_t n,
                              double2 *__restrict__ e) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < (int64_t)d * n) e[idx] = nl_unit_phase(nu, x[idx]);
}

__global__ void sample_kernel(int32_t nu, int32_t d, uint64_t seed, uint32_t stream_id, int32_t i,
                              int64_t m0, int64_t n, double *__restrict__ x) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    PhiloxStream rs(seed, stream_id, (uint64_t)(m0 + p), (uint32_t)i, 0u);
    for (int l = 0; l < d; ++l) x[l * n + p] = law_icdf(nu, rs.next());
}

// ---------------------------------------------------------------------------
// Reduced-precision form.  The walk runs in FP32 from phase factors reduced
// in FP64; each node's value is rounded to 16 bits (bf16 or f16) and parked
// in this lane's LDS slots; every kMfmaGroup nodes the group is contracted
// on the matrix cores with the row's coefficient tiles, accumulating in FP32.
//
// v_mfma_f32_4x4x4_16b: 16 blocks of D(4x4) += A(4x4) B(4x4).  Lane
// l = 4b + j holds B[b][k][j] (k = 0..3) and receives D[b][i][j] (i = 0..3).
// Here B = basis values: block b = pair of nodes (k = Re, Im of node 2b,
// Re, Im of node 2b+1) at the lane's own path (column j, so lane l is path
// l), and A = coefficients of that pair for 4 right-hand sides (rows i),
// broadcast from block b's lanes (CBSZ 4, ABID b) to all blocks.  D rows are
// right-hand sides: 0 = ybar, 1 + l = d ybar / d u_l.  T groups of 4
// right-hand sides take T instructions per pair.
// ---------------------------------------------------------------------------
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 h16x4 __attribute__((ext_vector_type(4)));

template <int PREC, int ABID>
__device__ __forceinline__ f32x4 mfma_pair(uint2 a, uint2 b, f32x4 c) {
    if constexpr (PREC == QR_PREC_BF16)
        return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(__builtin_bit_cast(s16x4, a),
                                                      __builtin_bit_cast(s16x4, b), c, 4, ABID, 0);
    else
        return __builtin_amdgcn_mfma_f32_4x4x4f16(__builtin_bit_cast(h16x4, a),
                                                  __builtin_bit_cast(h16x4, b), c, 4, ABID, 0);
}

constexpr int kMfmaGroup = 32;  // nodes per contraction group (16 pairs)

template <int PREC, int T>
struct MfmaSink {
    static constexpr bool kGrad = false;
    static constexpr bool kSplit = true;
    struct Acc {};
    uint32_t *stage;       // this lane's 16-bit pairs: stage[(node pair) 128 + half], lane offset applied
    const uint2 *tiles;    // coefficient tiles of the next group: [T][64] uint2, lane offset applied
    uint2 a[T];            // this lane's A operands of the current group
    f32x4 acc[T];
    int c;                 // nodes of the current group so far (wave-uniform)

    __device__ __forceinline__ void load_tiles() {
#pragma unroll
        for (int t = 0; t < T; ++t) a[t] = tiles[t * 64];
        tiles += T * 64;
    }
    template <int B>
    __device__ __forceinline__ void pair() {
        const uint2 b = *reinterpret_cast<const uint2 *>(stage + B * 128);
#pragma unroll
        for (int t = 0; t < T; ++t) acc[t] = mfma_pair<PREC, B>(a[t], b, acc[t]);
    }
    template <int B>
    __device__ __forceinline__ void pairs() {
        if constexpr (B < kMfmaGroup / 2) {
            pair<B>();
            pairs<B + 1>();
        }
    }
    __device__ __forceinline__ void flush() {
        pairs<0>();
        load_tiles();
        c = 0;
    }
    __device__ __forceinline__ void node(const Pts<1, float> &v, Acc &) {
        // the counter is the same in every lane: keep it (and the offset) scalar
        const int cu = __builtin_amdgcn_readfirstlane(c);
        stage[(cu >> 1) * 128 + (cu & 1)] = pack16x2<PREC>(v.re[0], v.im[0]);
        c = cu + 1;
        if (c == kMfmaGroup) flush();
    }
    __device__ __forceinline__ static void add(Acc &, const Acc &) {}
};

template <int DB, int CAP, bool GRAD, int T, int PREC>
__global__ __launch_bounds__(kPathBlock) void mfma_path_kernel(
    const DevProblem *__restrict__ P0, const Walk W, const int32_t i, const int64_t M,
    const uint64_t seed, const uint2 *__restrict__ tiles, const int64_t tile_ld,
    double *__restrict__ S_out, double2 *__restrict__ e_out) {
    // T groups of 4 right-hand sides: 1 (ybar) or 1 + d <= 4 T (with gradients)
    extern __shared__ double2 lds[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int d = P0->d, nbm = P0->nbm, N = P0->N;
    // LDS: staged pairs [waves][16][64] uint2 | phase factors [d][128] float2 | path state [d][128] double
    uint32_t *stage = reinterpret_cast<uint32_t *>(lds) + wave * (kMfmaGroup / 2) * 128;
    float2 *E = reinterpret_cast<float2 *>(reinterpret_cast<uint2 *>(lds) + (kPathBlock / 64) * (kMfmaGroup / 2) * 64);
    double *xs = reinterpret_cast<double *>(E + d * kPathBlock) + tid;
    const LanePts<1, float> L{E + tid, nullptr, kPathBlock};
    // stale slots of a partial group meet zero coefficients: keep them finite
    for (int k = 0; k < kMfmaGroup; ++k) stage[(k >> 1) * 128 + 2 * lane + (k & 1)] = 0u;

    const int64_t m = (int64_t)blockIdx.x * kPathBlock + tid;  // paths past M run on and are not stored
    {
        PhiloxStream rs(seed, 0u, (uint64_t)m, (uint32_t)i, 0u);
        for (int l = 0; l < d; ++l) {
            const double x = nl_icdf_u(P0->nu, rs.next());
            xs[l * kPathBlock] = x;
            if (e_out && m < M) e_out[l * M + m] = nl_unit_phase_u(P0->nu, x);
        }
    }
    double S = 0.0;
    for (int j = i; j < N; ++j) {
        const DevProblem *__restrict__ Pj = P0;
        asm volatile("" : "+s"(Pj));
        const double tj = Pj->t[j];
        const double dt = Pj->t[j + 1] - tj;
        double hj, uj;
        {
            double x[DB];
#pragma unroll
            for (int l = 0; l < DB; ++l) x[l] = (l < d) ? xs[l * kPathBlock] : 0.0;
            const double2 hu = h_source<DB>(Pj, tj, x, d);
            hj = hu.x;
            uj = hu.y;
            const double sq = sqrt(dt);
            PhiloxStream rs(seed, 0u, (uint64_t)m, (uint32_t)i, (uint32_t)(d + (j - i) * nbm));
#pragma unroll
            for (int l = 0; l < DB; ++l)
                if (l < d) x[l] = fma(fma(Pj->b1[l], x[l], Pj->b0[l]), dt, x[l]);
#pragma unroll 1
            for (int k = 0; k < nbm; ++k) {
                const double dwk = sq * nl_norm_icdf(rs.next());
#pragma unroll
                for (int l = 0; l < DB; ++l)
                    if (l < d) x[l] = fma(Pj->sigma[l * nbm + k], dwk, x[l]);
            }
#pragma unroll
            for (int l = 0; l < DB; ++l)
                if (l < d) xs[l * kPathBlock] = x[l];
        }
        double y, z2 = 0.0;
        if (j + 1 < N) {
            for (int l = 0; l < d; ++l) {
                const double2 e = nl_unit_phase_u(Pj->nu, xs[l * kPathBlock]);
                L.set_e(l, 0, make_float2((float)e.x, (float)e.y));
            }
            MfmaSink<PREC, T> sink;
            sink.stage = stage + 2 * lane;
            sink.tiles = tiles + (int64_t)(j + 1) * tile_ld + lane;
            sink.c = 0;
#pragma unroll
            for (int t = 0; t < T; ++t) sink.acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
            sink.load_tiles();
            typename MfmaSink<PREC, T>::Acc none{};
            const Pts<1, float> one = unit<1, float>();
            sink.node(one, none);
            (void)visit<0, CAP, 1>(one, -1, 1, W, L, sink);
            if (sink.c) sink.template pairs<0>();
            y = (double)sink.acc[0][0];
            if constexpr (GRAD) {
                double gx[DB];
#pragma unroll
                for (int l = 0; l < DB; ++l) {
                    gx[l] = 0.0;
                    if (l < d) {
                        gx[l] = (double)sink.acc[(l + 1) / 4][(l + 1) % 4] * nl_pdf_u(Pj->nu, xs[l * kPathBlock]);
                    }
                }
                for (int k = 0; k < nbm; ++k) {
                    double zk = 0.0;
#pragma unroll
                    for (int l = 0; l < DB; ++l)
                        if (l < d) zk = fma(Pj->sigma[l * nbm + k], gx[l], zk);
                    z2 = fma(zk, zk, z2);
                }
            }
        } else {
            double x[DB], gx[DB];
#pragma unroll
            for (int l = 0; l < DB; ++l) x[l] = (l < d) ? xs[l * kPathBlock] : 0.0;
            y = g_term<DB>(Pj, x, d, GRAD ? gx : nullptr);
            if constexpr (GRAD) {
                for (int k = 0; k < nbm; ++k) {
                    double zk = 0.0;
#pragma unroll
                    for (int l = 0; l < DB; ++l)
                        if (l < d) zk = fma(Pj->sigma[l * nbm + k], gx[l], zk);
                    z2 = fma(zk, zk, z2);
                }
            }
        }
        S = fma(fnl(Pj, clamp_abs(y, Pj->clamp), z2, uj) + hj, dt, S);
    }
    double x[DB];
#pragma unroll
    for (int l = 0; l < DB; ++l) x[l] = (l < d) ? xs[l * kPathBlock] : 0.0;
    const double Sm = S + g_term<DB>(P0, x, d, nullptr);
    if (m < M) S_out[m] = Sm;
}

size_t mfma_path_lds_bytes(int32_t d) {
    return (size_t)(kPathBlock / 64) * (kMfmaGroup / 2) * 64 * sizeof(uint2) +
           (size_t)d * kPathBlock * (sizeof(float2) + sizeof(double));
}

// Coefficient tiles of one row: tile[g][t][lane] holds, for lane 4b + r, the
// 16-bit coefficients of right-hand side 4t + r on nodes 32g + 2b and
// 32g + 2b + 1: (Re, Im) weights, ybar = sum a.x Re + a.y Im and
// d ybar / d u_l = sum theta k_l (a.y Re - a.x Im), theta = 2 pi (pi for
// the cosine basis's half-frequency walk).  Nodes past nrep and right-hand
// sides past d are zero.
template <int PREC>
__global__ void pack_tiles_kernel(const double2 *__restrict__ alpha_int_row, int64_t nrep,
                                  const int32_t *__restrict__ trav, int32_t d, int32_t T,
                                  int64_t ngroups, double theta, uint2 *__restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ngroups * T * 64) return;
    const int lane = (int)(idx % 64), t = (int)((idx / 64) % T);
    const int64_t g = idx / (64 * T);
    const int b = lane >> 2, rhs = 4 * t + (lane & 3);
    uint32_t w[2];
    for (int h = 0; h < 2; ++h) {
        const int64_t n = g * kMfmaGroup + 2 * b + h;
        double cr = 0.0, ci = 0.0;
        if (n < nrep) {
            const double2 a = alpha_int_row[n];
            if (rhs == 0) {
                cr = a.x;
                ci = a.y;
            } else if (rhs <= d) {
                const double k2p = theta * (double)trav[n * d + rhs - 1];
                cr = k2p * a.y;
                ci = -k2p * a.x;
            }
        }
        w[h] = pack16x2<PREC>((float)cr, (float)ci);
    }
    out[idx] = make_uint2(w[0], w[1]);
}

// ---------------------------------------------------------------------------
// Step-major path simulation (learned form).  The cloud's states live in
// HBM and the paths advance one time step per launch, so that ybar_{j+1}
// can be evaluated for the whole cloud at once, by the expansion
// (eval_kernel) or by the surrogate network.  Random numbers and arithmetic
// are those of path_kernel, step by step.
// ---------------------------------------------------------------------------
__global__ void sm_start_kernel(const DevProblem *__restrict__ P0, int32_t nu, int32_t i, int64_t M,
                                uint64_t seed, double *__restrict__ x, double2 *__restrict__ e,
                                double *__restrict__ S) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    PhiloxStream rs(seed, 0u, (uint64_t)m, (uint32_t)i, 0u);
    for (int l = 0; l < P0->d; ++l) {
        const double xv = nl_icdf(nu, rs.next());
        x[l * M + m] = xv;
        e[l * M + m] = nl_unit_phase(nu, xv);
    }
    S[m] = 0.0;
}

// X_j -> X_{j+1} in place; H = h(t_j, X_j)
template <int DB>
__global__ void sm_euler_kernel(const DevProblem *__restrict__ P0, int32_t i, int32_t j, int64_t M,
                                uint64_t seed, double *__restrict__ xg, double *__restrict__ H) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const int d = P0->d, nbm = P0->nbm;
    const double tj = P0->t[j], dt = P0->t[j + 1] - tj, sq = sqrt(dt);
    double x[DB];
#pragma unroll
    for (int l = 0; l < DB; ++l) x[l] = (l < d) ? xg[l * M + m] : 0.0;
    H[m] = h_source<DB>(P0, tj, x, d).x;
    PhiloxStream rs(seed, 0u, (uint64_t)m, (uint32_t)i, (uint32_t)(d + (j - i) * nbm));
#pragma unroll
    for (int l = 0; l < DB; ++l)
        if (l < d) x[l] = fma(fma(P0->b1[l], x[l], P0->b0[l]), dt, x[l]);
    for (int k = 0; k < nbm; ++k) {
        const double dwk = sq * nl_norm_icdf(rs.next());
#pragma unroll
        for (int l = 0; l < DB; ++l)
            if (l < d) x[l] = fma(P0->sigma[l * nbm + k], dwk, x[l]);
    }
#pragma unroll
    for (int l = 0; l < DB; ++l)
        if (l < d) xg[l * M + m] = x[l];
}

// S += (f(T_L(y)) + H) dt with y = y64 (expansion) or mu + sigma y32
// (surrogate), over paths [m0, m0 + n)
__global__ void sm_accum_kernel(const DevProblem *__restrict__ P0, int32_t j, int64_t m0, int64_t n,
                                const double *__restrict__ y64, const float *__restrict__ y32, double mu,
                                double sigma, const double *__restrict__ H, double *__restrict__ S) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t m = m0 + k;
    const double dt = P0->t[j + 1] - P0->t[j];
    const double y = y64 ? y64[k] : mu + sigma * (double)y32[k];
    S[m] = fma(fnl(P0, clamp_abs(y, P0->clamp), 0.0, 0.0) + H[m], dt, S[m]);
}

// the last step: y = g(X_N), then S += g(X_N)
template <int DB>
__global__ void sm_final_kernel(const DevProblem *__restrict__ P0, int64_t M, const double *__restrict__ xg,
                                const double *__restrict__ H, double *__restrict__ S) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const int d = P0->d, j = P0->N - 1;
    const double dt = P0->t[j + 1] - P0->t[j];
    double x[DB];
#pragma unroll
    for (int l = 0; l < DB; ++l) x[l] = (l < d) ? xg[l * M + m] : 0.0;
    const double g = g_term<DB>(P0, x, d, nullptr);
    const double Sj = fma(fnl(P0, clamp_abs(g, P0->clamp), 0.0, 0.0) + H[m], dt, S[m]);
    S[m] = Sj + g;
}

// first two moments of t (partials per block of 256: sum, sum of squares)
__global__ void moments_kernel(int64_t n, const double *__restrict__ t, double *__restrict__ partial) {
    __shared__ double ra[256], rb[256];
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double v = p < n ? t[p] : 0.0;
    ra[threadIdx.x] = v;
    rb[threadIdx.x] = v * v;
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

// ---------------------------------------------------------------------------
// Batched form: instances sharing the cloud.  One walk per path serves RT
// instances: each node's value is contracted with RT coefficient pairs (one
// scalar load of 16 RT bytes), so the complex multiply and the walk's scalar
// control are shared by the RT instances.  Instance coefficients of a pass
// are interleaved per node: row[node][RT] double2.
// ---------------------------------------------------------------------------
// The pass's coefficient stream (RT pairs per node, 16 RT bytes) arrives in
// chunks of kLoads x 1 KB (kLoads 16-byte vector loads per lane) requested a
// chunk ahead (vector loads complete in order); when the walk enters a chunk
// the wave parks it in its LDS slot, and each node's RT pairs are broadcast
// LDS reads.
template <int RT>
struct BatchSink {
    static constexpr bool kGrad = false;
    static constexpr bool kSplit = true;
    struct Acc {};
    static constexpr int kLoads = 4;
    static constexpr int kNodes = kLoads * 64 / RT;  // nodes per chunk
    double2 *slot;        // this wave's copy of the current chunk [kNodes][RT]
    const double2 *next;  // this lane's part of the chunk after `buf`
    double2 buf[kLoads];  // this lane's part of the next chunk
    int n;                // node about to be visited (wave-uniform)
    double y[RT];

    __device__ __forceinline__ void init(const double2 *row, double2 *wave_slot) {
        const double2 *r = row + __lane_id();
        slot = wave_slot;
#pragma unroll
        for (int k = 0; k < kLoads; ++k) slot[k * 64 + __lane_id()] = r[k * 64];
#pragma unroll
        for (int k = 0; k < kLoads; ++k) buf[k] = r[(kLoads + k) * 64];
        next = r + 2 * kLoads * 64;
        n = 0;
        wave_sync();
#pragma unroll
        for (int k = 0; k < RT; ++k) y[k] = 0.0;
    }
    __device__ __forceinline__ void node(const Pts<1> &v, Acc &) {
        const int nu = __builtin_amdgcn_readfirstlane(n);
        const double2 *p = slot + (nu % kNodes) * RT;
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const double2 c = p[r];
            y[r] = fma(c.x, v.re[0], fma(c.y, v.im[0], y[r]));
        }
        n = nu + 1;
        if ((nu + 1) % kNodes == 0) {
            wave_sync();
#pragma unroll
            for (int k = 0; k < kLoads; ++k) slot[k * 64 + __lane_id()] = buf[k];
#pragma unroll
            for (int k = 0; k < kLoads; ++k) buf[k] = next[k * 64];
            next += kLoads * 64;
            wave_sync();
        }
    }
    __device__ __forceinline__ static void add(Acc &, const Acc &) {}
};

__device__ __forceinline__ double fnl_a(int kind, double a, double y) {
    switch (kind) {
    case QR_F_SIN: return a * nl_sin(y);
    case QR_F_ALLEN_CAHN: return y - y * y * y;
    default: return 0.0;
    }
}

// One path per thread; RT instances per launch (pass).  The part of the
// source term h that does not involve the driver is shared; the driver
// parameter f_a is the instance's.
template <int DB, int CAP, int RT>
__global__ __launch_bounds__(kPathBlock) void batched_path_kernel(
    const DevProblem *__restrict__ P0, const DevBatch *__restrict__ B, const int32_t pass,
    const Walk W, const int32_t i, const int64_t M, const uint64_t seed,
    const double2 *__restrict__ alpha_b, const int64_t ld, double *__restrict__ S_out,
    double2 *__restrict__ e_out) {
    extern __shared__ double2 lds[];
    const int tid = threadIdx.x;
    // paths past M run on and are not stored: every lane takes part in the
    // wave's coefficient stream
    const int64_t m = (int64_t)blockIdx.x * kPathBlock + tid;
    const int d = P0->d, nbm = P0->nbm, N = P0->N;
    const LanePts<1> L{lds + tid, nullptr, kPathBlock};
    double *xs = reinterpret_cast<double *>(lds + d * kPathBlock) + tid;
    double2 *wave_slot = reinterpret_cast<double2 *>(reinterpret_cast<double *>(lds + d * kPathBlock) + d * kPathBlock) +
                         (tid >> 6) * (BatchSink<RT>::kLoads * 64);

    {
        PhiloxStream rs(seed, 0u, (uint64_t)m, (uint32_t)i, 0u);
        for (int l = 0; l < d; ++l) {
            const double x = nl_icdf(P0->nu, rs.next());
            xs[l * kPathBlock] = x;
            if (e_out && m < M) e_out[l * M + m] = nl_unit_phase(P0->nu, x);
        }
    }
    double S[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) S[r] = 0.0;

    for (int j = i; j < N; ++j) {
        const DevProblem *__restrict__ Pj = P0;
        asm volatile("" : "+s"(Pj));
        const double tj = Pj->t[j];
        const double dt = Pj->t[j + 1] - tj;
        double x[DB];
#pragma unroll
        for (int l = 0; l < DB; ++l) x[l] = (l < d) ? xs[l * kPathBlock] : 0.0;
        // source term at X_j without its driver part: -(d_t u + L u)
        double hbase, uval;
        {
            const double E = Pj->sol_A * nl_exp(-Pj->sol_c * (Pj->T - tj));
            double th = Pj->sol_p, bw = 0.0;
#pragma unroll
            for (int l = 0; l < DB; ++l) {
                if (l < d) {
                    th = fma(Pj->sol_w[l], x[l], th);
                    bw = fma(fma(Pj->b1[l], x[l], Pj->b0[l]), Pj->sol_w[l], bw);
                }
            }
            const double2 sc = nl_sincos(th);
            const double v = E * sc.y;  // u - B
            const double gscale = -E * sc.x;
            hbase = -(Pj->sol_c * v + gscale * bw - 0.5 * v * Pj->sw2);
            uval = v + Pj->sol_B;
        }
        {
            const double sq = sqrt(dt);
            PhiloxStream rs(seed, 0u, (uint64_t)m, (uint32_t)i, (uint32_t)(d + (j - i) * nbm));
#pragma unroll
            for (int l = 0; l < DB; ++l)
                if (l < d) x[l] = fma(fma(Pj->b1[l], x[l], Pj->b0[l]), dt, x[l]);
#pragma unroll 1
            for (int k = 0; k < nbm; ++k) {
                const double dwk = sq * nl_norm_icdf(rs.next());
#pragma unroll
                for (int l = 0; l < DB; ++l)
                    if (l < d) x[l] = fma(Pj->sigma[l * nbm + k], dwk, x[l]);
            }
#pragma unroll
            for (int l = 0; l < DB; ++l)
                if (l < d) xs[l * kPathBlock] = x[l];
        }
        double y[RT];
        if (j + 1 < N) {
            for (int l = 0; l < W.d; ++l) L.set_e(l, 0, nl_unit_phase(Pj->nu, xs[l * kPathBlock]));
            BatchSink<RT> sink;
            sink.init(alpha_b + (int64_t)(j + 1) * ld * RT, wave_slot);
            typename BatchSink<RT>::Acc none{};
            const Pts<1> one = unit<1>();
            sink.node(one, none);
            (void)visit<0, CAP, 1>(one, -1, 1, W, L, sink);
#pragma unroll
            for (int r = 0; r < RT; ++r) y[r] = sink.y[r];
        } else {
#pragma unroll
            for (int l = 0; l < DB; ++l) x[l] = (l < d) ? xs[l * kPathBlock] : 0.0;
            const double g = g_term<DB>(Pj, x, d, nullptr);
#pragma unroll
            for (int r = 0; r < RT; ++r) y[r] = g;
        }
        const int kind = Pj->driver;
        const double cl = Pj->clamp;
        const DevBatch *__restrict__ Bj = B;
        asm volatile("" : "+s"(Bj));
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const double ar = Bj->f_a[pass * RT + r];
            const double f = fnl_a(kind, ar, clamp_abs(y[r], cl)) + (hbase - fnl_a(kind, ar, uval));
            S[r] = fma(f, dt, S[r]);
        }
    }
    double x[DB];
#pragma unroll
    for (int l = 0; l < DB; ++l) x[l] = (l < d) ? xs[l * kPathBlock] : 0.0;
    const double g = g_term<DB>(P0, x, d, nullptr);
    const int cnt = B->count[pass];
#pragma unroll
    for (int r = 0; r < RT; ++r)
        if (r < cnt && m < M) S_out[(int64_t)r * M + m] = S[r] + g;
}

// Row i of one instance from its slice partial sums.  The instance's own
// index set is a sub-walk of the basis: node t of it is node ft[t] of the
// basis traversal, which sits at pass_pos[ft[t]] in the coefficient layout of
// the instance's pass (a walk containing the instance's).  Coefficients the
// instance does not have stay as zero-filled.
// partial: [split][n_part][R] with the instance's node t at index t (R = 1,
// n_part = nrep_sub: its own projection) or at its node of the pass walk
// pass_pos[ft[t]] and column slot (R > 1: the pass projection)
__global__ void reduce_batched_kernel(const double2 *__restrict__ partial, int32_t nsplit,
                                      int64_t nrep_sub, int64_t n_part, int32_t R, double M,
                                      const int32_t *__restrict__ ft,
                                      const int32_t *__restrict__ canon_of_trav,
                                      const int32_t *__restrict__ pass_pos,
                                      double2 *__restrict__ alpha_b_row, int32_t slot,
                                      double *__restrict__ alpha_row, int32_t *__restrict__ bad, int32_t step) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrep_sub) return;
    const int64_t pi = R == 1 ? t : (int64_t)pass_pos[ft[t]] * R + slot;
    double sx = 0.0, sy = 0.0;
    for (int s = 0; s < nsplit; ++s) {
        const double2 p = partial[(int64_t)s * n_part * R + pi];
        sx += p.x;
        sy += p.y;
    }
    if (bad && !(isfinite(sx) && isfinite(sy))) atomicMax(bad, step);
    const int64_t r = ft[t];
    double2 *dst = alpha_b_row + (int64_t)pass_pos[r] * kBatchRT + slot;
    if (r == 0) {
        const double a0 = sx / M;
        *dst = make_double2(a0, 0.0);
        alpha_row[0] = a0;
    } else {
        const double mc = sx / M, ms = sy / M;
        *dst = make_double2(2.0 * mc, 2.0 * ms);
        const int64_t c = canon_of_trav[r];
        alpha_row[2 * c - 1] = M_SQRT2 * mc;
        alpha_row[2 * c] = M_SQRT2 * ms;
    }
}

// Z of eq (MDP:intro:0a): the multistep sum without its first term, times the
// first Brownian increment over Delta_i (the normals r = d + k of the stream)
__global__ void z_responses_kernel(const DevProblem *__restrict__ P, uint64_t seed, int32_t i, int64_t M, int32_t k0,
                                   int32_t nk, const double *__restrict__ S, const double *__restrict__ f0,
                                   const double *__restrict__ y0, double *__restrict__ out) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const double dt = P->t[i + 1] - P->t[i];
    // multistep (y0 NULL): the sum without its first term; one step: the value
    // the driver read on the first step less T_L(ybar_{i+1}(X_i))
    const double sz = (y0 ? f0[M + m] - clamp_abs(y0[m], P->clamp) : S[m] - f0[m]) / dt;
    const double sq = sqrt(dt);
    for (int r = 0; r < kBatchRT; ++r) {
        double v = 0.0;
        if (r < nk) v = sz * (sq * norm_icdf(uniform_at(seed, 0u, (uint64_t)m, (uint32_t)i, (uint32_t)(P->d + k0 + r))));
        out[(int64_t)r * M + m] = v;
    }
}

__global__ void reduce_slot_kernel(const double2 *__restrict__ partial, int32_t nsplit, int64_t nrep, int32_t R,
                                   int32_t slot, double M, const int32_t *__restrict__ canon_of_trav,
                                   double *__restrict__ alpha_row, int32_t *__restrict__ bad, int32_t step) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrep) return;
    double sx = 0.0, sy = 0.0;
    for (int s = 0; s < nsplit; ++s) {
        const double2 p = partial[((int64_t)s * nrep + t) * R + slot];
        sx += p.x;
        sy += p.y;
    }
    if (bad && !(isfinite(sx) && isfinite(sy))) atomicMax(bad, step);
    if (t == 0) {
        alpha_row[0] = sx / M;
    } else {
        const int64_t c = canon_of_trav[t];
        alpha_row[2 * c - 1] = M_SQRT2 * (sx / M);
        alpha_row[2 * c] = M_SQRT2 * (sy / M);
    }
}

__global__ void zero_kernel(double *__restrict__ p, int64_t n) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) p[idx] = 0.0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_gather(const double *alpha, int32_t row0, int32_t nrows, int64_t nrep, int64_t ld,
                         int64_t nfuncs, const int32_t *canon_of_trav, double2 *alpha_int,
                         hipStream_t s) {
    const int64_t total = (int64_t)nrows * nrep;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, alpha, row0,
                       nrows, nrep, ld, nfuncs, canon_of_trav, alpha_int);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cosine basis over N^d and its carrier.  For k in N^d with n non-zero
// coordinates, phi_k = prod_l sqrt2^{[k_l > 0]} cos(pi k_l u_l) is, by the
// product-to-sum identity, 2^{(1-n)/2} times the sum of sqrt2 cos(pi k'.u)
// over the 2^{n-1} representatives k' of Z^d with |k'_l| = k_l.  A cosine
// row therefore expands to the carrier row (Fourier canonical layout at half
// frequency) carrier[2c-1] = s_c alpha[k(c)], carrier[2c] = 0,
// carrier[0] = alpha[0] (s_c = 2^{(1-n)/2}), and the projection of S on phi_k
// folds from the carrier's projections on sqrt2 cos(pi k'.u):
// alpha[k] = s_k sum_{c of k} carrier[2c-1] (fixed order).
// ---------------------------------------------------------------------------
__global__ void cos_expand_kernel(const double *__restrict__ acos, int32_t row0, int32_t nrows, int64_t ncos,
                                  int64_t nrep, const int32_t *__restrict__ cos_of_rep,
                                  const double *__restrict__ rep_scale, double *__restrict__ acar) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nrows * nrep) return;
    const int64_t row = row0 + idx / nrep, c = idx % nrep;
    const double a = acos[row * ncos + cos_of_rep[c]];
    double *dst = acar + row * (2 * nrep - 1);
    if (c == 0) {
        dst[0] = a;
    } else {
        dst[2 * c - 1] = rep_scale[c] * a;
        dst[2 * c] = 0.0;
    }
}

__global__ void cos_fold_kernel(const double *__restrict__ acar_row, int64_t ncos,
                                const int32_t *__restrict__ fold_off, const int32_t *__restrict__ fold_idx,
                                const double *__restrict__ rep_scale, double *__restrict__ acos_row) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ncos) return;
    const int32_t b = fold_off[k], e = fold_off[k + 1];
    const int32_t c0 = fold_idx[b];
    if (c0 == 0) {
        acos_row[k] = acar_row[0];
        return;
    }
    double sum = 0.0;
    for (int32_t q = b; q < e; ++q) sum += acar_row[2 * (int64_t)fold_idx[q] - 1];
    acos_row[k] = rep_scale[c0] * sum;
}

hipError_t launch_cos_expand(const double *acos, int32_t row0, int32_t nrows, int64_t ncos, int64_t nrep,
                             const int32_t *cos_of_rep, const double *rep_scale, double *acar, hipStream_t s) {
    const int64_t total = (int64_t)nrows * nrep;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(cos_expand_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, acos, row0, nrows, ncos,
                       nrep, cos_of_rep, rep_scale, acar);
    return hipGetLastError();
}

hipError_t launch_cos_fold(const double *acar_row, int64_t ncos, const int32_t *fold_off, const int32_t *fold_idx,
                           const double *rep_scale, double *acos_row, hipStream_t s) {
    if (ncos == 0) return hipSuccess;
    hipLaunchKernelGGL(cos_fold_kernel, dim3(blocks_for(ncos, 256)), dim3(256), 0, s, acar_row, ncos, fold_off,
                       fold_idx, rep_scale, acos_row);
    return hipGetLastError();
}

// y = ybar D and grad y = D (grad ybar + ybar q x / (1+|x|^2)), D = (1+|x|^2)^{q/2}
// (eq (yqi)), in place at n points (x SoA [d][n]; grad SoA [d][n] or NULL)
__global__ void undamp_kernel(int32_t d, double q, const double *__restrict__ x, int64_t n, double *__restrict__ y,
                              double *__restrict__ grad) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double r2 = 0.0;
    for (int l = 0; l < d; ++l) r2 = fma(x[l * n + p], x[l * n + p], r2);
    const double D = pow(1.0 + r2, 0.5 * q), w = q / (1.0 + r2);
    const double yb = y[p];
    if (grad)
        for (int l = 0; l < d; ++l) grad[l * n + p] = D * fma(yb * w, x[l * n + p], grad[l * n + p]);
    y[p] = yb * D;
}

hipError_t launch_undamp(int32_t d, double q, const double *x, int64_t n, double *y, double *grad, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(undamp_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, q, x, n, y, grad);
    return hipGetLastError();
}

hipError_t launch_pad(int32_t nrows, int64_t nrep, int64_t ld, double2 *alpha_int, hipStream_t s) {
    const int64_t total = (int64_t)nrows * (ld - nrep);
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(pad_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, nrows, nrep, ld,
                       alpha_int);
    return hipGetLastError();
}


int64_t path_state_ld(int64_t M, bool grad) {
    const int64_t per = (int64_t)kPathBlock * (grad ? 1 : kPathP);
    return (M + per - 1) / per * per;
}

template <int DB, int CAP, bool GRAD, int FEAT>
static hipError_t path_t(const PathArgs &a, hipStream_t s) {
    constexpr int P = GRAD ? 1 : kPathP;
    const size_t lds = path_lds_bytes(a.W.d, GRAD, P);
    static size_t granted = kLdsDefault;
    const hipError_t e = allow_lds((const void *)path_kernel<DB, CAP, GRAD, P, FEAT>, lds, granted);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((path_kernel<DB, CAP, GRAD, P, FEAT>), dim3(blocks_for(a.M, (int64_t)kPathBlock * P)),
                       dim3(kPathBlock), lds, s, a.P, a.W, a.i, a.M, a.seed, a.alpha_int, a.ld, a.S,
                       a.e, a.x0, a.xs, a.ldx, a.f0);
    return hipGetLastError();
}

template <int DB, bool GRAD, int FEAT>
static hipError_t path_cap(int cap, const PathArgs &a, hipStream_t s) {
    switch (cap) {
    case 2: return path_t<DB, 2, GRAD, FEAT>(a, s);
    case 4: return path_t<DB, 4, GRAD, FEAT>(a, s);
    case 6: if constexpr (DB >= 6) return path_t<DB, 6, GRAD, FEAT>(a, s); break;
    case 8: if constexpr (DB >= 8) return path_t<DB, 8, GRAD, FEAT>(a, s); break;
    }
    return hipErrorInvalidValue;
}

template <int FEAT>
static hipError_t path_db(int db, int cap, bool grad, const PathArgs &a, hipStream_t s) {
    switch (db) {
    case 4: return grad ? path_cap<4, true, FEAT>(cap, a, s) : path_cap<4, false, FEAT>(cap, a, s);
    case 8: return grad ? path_cap<8, true, FEAT>(cap, a, s) : path_cap<8, false, FEAT>(cap, a, s);
    case 16: return grad ? path_cap<16, true, FEAT>(cap, a, s) : path_cap<16, false, FEAT>(cap, a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_path(int db, int cap, bool grad, int feat, const PathArgs &a, hipStream_t s) {
    switch (feat) {
    case 0: return path_db<0>(db, cap, grad, a, s);
    case 1: return path_db<1>(db, cap, grad, a, s);
    case 2: return path_db<2>(db, cap, grad, a, s);
    }
    return hipErrorInvalidValue;
}

template <int CAP, int P, int WAVES, int TM>
static hipError_t project_t(const Walk &W, const double2 *e, int64_t lde, const double *S, int64_t M, int64_t pps,
                            int32_t ntasks, int32_t nsplit, const Task *tasks,
                            const TaskItem *items, double2 *partial, int64_t nrep, hipStream_t s) {
    const size_t lds = project_lds_bytes(W.d, P, WAVES, TM);
    static size_t granted = kLdsDefault;
    const hipError_t err = allow_lds((const void *)project_kernel<CAP, P, WAVES, TM>, lds, granted);
    if (err != hipSuccess) return err;
    const unsigned groups = (unsigned)((ntasks + WAVES - 1) / WAVES);
    hipLaunchKernelGGL((project_kernel<CAP, P, WAVES, TM>), dim3(groups, (unsigned)nsplit), dim3(WAVES * 64), lds,
                       s, W, e, lde, S, M, pps, ntasks, tasks, items, partial, nrep);
    return hipGetLastError();
}

// The shapes (paths per lane, waves, task size), in order of preference; the
// first whose LDS fits is used.
#ifndef QRMC_PROJ_SHAPES
#define QRMC_PROJ_SHAPES {4, 8, 512}, {2, 8, 512}, {1, 8, 512}
#endif
constexpr ProjShape kProjShapes[3] = {QRMC_PROJ_SHAPES};

ProjShape proj_shape(int32_t d) {
    for (const ProjShape &p : kProjShapes)
        if (project_lds_bytes(d, p.P, p.waves, p.task_max) <= kLdsMax) return p;
    return kProjShapes[2];
}

template <int CAP, int I>
static hipError_t project_i(const Walk &W, const double2 *e, int64_t lde, const double *S, int64_t M, int64_t pps,
                            int32_t ntasks, int32_t nsplit, const Task *tasks, const TaskItem *items,
                            double2 *partial, int64_t nrep, hipStream_t s) {
    constexpr ProjShape p = kProjShapes[I];
    return project_t<CAP, p.P, p.waves, p.task_max>(W, e, lde, S, M, pps, ntasks, nsplit, tasks, items, partial,
                                                       nrep, s);
}

template <int CAP>
static hipError_t project_p(const Walk &W, const double2 *e, int64_t lde, const double *S, int64_t M, int64_t pps,
                            int32_t ntasks, int32_t nsplit, const Task *tasks, const TaskItem *items,
                            int32_t task_max, double2 *partial, int64_t nrep, hipStream_t s) {
    const ProjShape p = proj_shape(W.d);
    if (task_max != p.task_max || project_lds_bytes(W.d, p.P, p.waves, p.task_max) > kLdsMax)
        return hipErrorInvalidValue;
    const auto same = [&](const ProjShape &q) { return q.P == p.P && q.waves == p.waves && q.task_max == p.task_max; };
    if (same(kProjShapes[0])) return project_i<CAP, 0>(W, e, lde, S, M, pps, ntasks, nsplit, tasks, items, partial, nrep, s);
    if (same(kProjShapes[1])) return project_i<CAP, 1>(W, e, lde, S, M, pps, ntasks, nsplit, tasks, items, partial, nrep, s);
    return project_i<CAP, 2>(W, e, lde, S, M, pps, ntasks, nsplit, tasks, items, partial, nrep, s);
}

hipError_t launch_project(int cap, const Walk &W, const double2 *e, int64_t lde, const double *S, int64_t M,
                          int64_t paths_per_split, int32_t ntasks, int32_t nsplit, const Task *tasks,
                          const TaskItem *items, int32_t task_max, double2 *partial, int64_t nrep,
                          hipStream_t s) {
    switch (cap) {
    case 2: return project_p<2>(W, e, lde, S, M, paths_per_split, ntasks, nsplit, tasks, items, task_max, partial, nrep, s);
    case 4: return project_p<4>(W, e, lde, S, M, paths_per_split, ntasks, nsplit, tasks, items, task_max, partial, nrep, s);
    case 6: return project_p<6>(W, e, lde, S, M, paths_per_split, ntasks, nsplit, tasks, items, task_max, partial, nrep, s);
    case 8: return project_p<8>(W, e, lde, S, M, paths_per_split, ntasks, nsplit, tasks, items, task_max, partial, nrep, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(const double2 *partial, int32_t nsplit, int64_t nrep, double M,
                         double2 *alpha_int_row, double *alpha_row,
                         const int32_t *canon_of_trav, int32_t *bad, int32_t step, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3(blocks_for(nrep, 256)), dim3(256), 0, s, partial, nsplit,
                       nrep, M, alpha_int_row, alpha_row, canon_of_trav, bad, step);
    return hipGetLastError();
}

__global__ void set_flag_kernel(int32_t *__restrict__ flag, int32_t v) { *flag = v; }

hipError_t launch_set_flag(int32_t *flag, int32_t v, hipStream_t s) {
    hipLaunchKernelGGL(set_flag_kernel, dim3(1), dim3(1), 0, s, flag, v);
    return hipGetLastError();
}

template <int CAP, bool GRAD>
static hipError_t eval_t(const Walk &W, const double2 *a, const double *x, int64_t n, double *y,
                         double *g, hipStream_t s) {
    const size_t lds = (size_t)W.d * kPathBlock * (sizeof(double2) + (GRAD ? sizeof(double) : 0)) +
                       (size_t)(kPathBlock / 64) * 64 * sizeof(double2);
    hipLaunchKernelGGL((eval_kernel<CAP, GRAD>), dim3(blocks_for(n, kPathBlock)), dim3(kPathBlock),
                       lds, s, W, a, x, n, y, g);
    return hipGetLastError();
}

hipError_t launch_eval(int cap, bool grad, const Walk &W, const double2 *alpha_int_row,
                       const double *x, int64_t n, double *y, double *grad_out, hipStream_t s) {
    if (n == 0) return hipSuccess;
#define QR_EVAL_CAP(C)                                                              \
    case C:                                                                         \
        return grad ? eval_t<C, true>(W, alpha_int_row, x, n, y, grad_out, s)       \
                    : eval_t<C, false>(W, alpha_int_row, x, n, y, grad_out, s);
    switch (cap) {
        QR_EVAL_CAP(2)
        QR_EVAL_CAP(4)
        QR_EVAL_CAP(6)
        QR_EVAL_CAP(8)
    }
#undef QR_EVAL_CAP
    return hipErrorInvalidValue;
}

template <int CAP, int I>
static hipError_t eval_tasks_i(const Walk &W, const double2 *e, int64_t n, int64_t pps, int32_t ntasks,
                               int32_t nsplit, const Task *tasks, const TaskItem *items, const double2 *row,
                               double *partial, hipStream_t s) {
    constexpr ProjShape p = kProjShapes[I];
    const size_t lds = eval_tasks_lds_bytes(W.d, p.P, p.waves, p.task_max);
    static size_t granted = kLdsDefault;
    const hipError_t err = allow_lds((const void *)eval_tasks_kernel<CAP, p.P, p.waves, p.task_max>, lds, granted);
    if (err != hipSuccess) return err;
    const unsigned groups = (unsigned)((ntasks + p.waves - 1) / p.waves);
    hipLaunchKernelGGL((eval_tasks_kernel<CAP, p.P, p.waves, p.task_max>), dim3(groups, (unsigned)nsplit),
                       dim3(p.waves * 64), lds, s, W, e, n, pps, ntasks, tasks, items, row, partial);
    return hipGetLastError();
}

template <int CAP>
static hipError_t eval_tasks_p(const Walk &W, const double2 *e, int64_t n, int64_t pps, int32_t ntasks,
                               int32_t nsplit, const Task *tasks, const TaskItem *items, int32_t task_max,
                               const double2 *row, double *partial, hipStream_t s) {
    const ProjShape p = proj_shape(W.d);
    if (task_max != p.task_max || eval_tasks_lds_bytes(W.d, p.P, p.waves, p.task_max) > kLdsMax)
        return hipErrorInvalidValue;
    const auto same = [&](const ProjShape &q) { return q.P == p.P && q.waves == p.waves && q.task_max == p.task_max; };
    if (same(kProjShapes[0])) return eval_tasks_i<CAP, 0>(W, e, n, pps, ntasks, nsplit, tasks, items, row, partial, s);
    if (same(kProjShapes[1])) return eval_tasks_i<CAP, 1>(W, e, n, pps, ntasks, nsplit, tasks, items, row, partial, s);
    return eval_tasks_i<CAP, 2>(W, e, n, pps, ntasks, nsplit, tasks, items, row, partial, s);
}

size_t eval_tasks_lds(int32_t d) {
    const ProjShape p = proj_shape(d);
    return eval_tasks_lds_bytes(d, p.P, p.waves, p.task_max);
}

hipError_t launch_eval_tasks(int cap, const Walk &W, const double2 *e, int64_t n, int64_t pps, int32_t ntasks,
                             int32_t nsplit, const Task *tasks, const TaskItem *items, int32_t task_max,
                             const double2 *row, double *partial, double *y, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipError_t err = hipErrorInvalidValue;
    switch (cap) {
    case 2: err = eval_tasks_p<2>(W, e, n, pps, ntasks, nsplit, tasks, items, task_max, row, partial, s); break;
    case 4: err = eval_tasks_p<4>(W, e, n, pps, ntasks, nsplit, tasks, items, task_max, row, partial, s); break;
    case 6: err = eval_tasks_p<6>(W, e, n, pps, ntasks, nsplit, tasks, items, task_max, row, partial, s); break;
    case 8: err = eval_tasks_p<8>(W, e, n, pps, ntasks, nsplit, tasks, items, task_max, row, partial, s); break;
    }
    if (err != hipSuccess) return err;
    const int32_t groups = (ntasks + proj_shape(W.d).waves - 1) / proj_shape(W.d).waves;
    hipLaunchKernelGGL(sum_groups_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, partial, groups, n, y);
    return hipGetLastError();
}

hipError_t launch_x_to_e(int32_t nu, int32_t d, const double *x, int64_t n, double2 *e, hipStream_t s) {
    const int64_t total = (int64_t)d * n;
    hipLaunchKernelGGL(x_to_e_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, nu, d, x, n, e);
    return hipGetLastError();
}

hipError_t launch_sample(int32_t nu, int32_t d, uint64_t seed, uint32_t stream_id, int32_t i, int64_t m0,
                         int64_t n, double *x, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(sample_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, nu, d, seed, stream_id,
                       i, m0, n, x);
    return hipGetLastError();
}


template <int DB, int CAP>
static hipError_t batched_t(const BatchArgs &a, hipStream_t s) {
    const size_t lds = (size_t)a.d * kPathBlock * (sizeof(double2) + sizeof(double)) +
                       (size_t)(kPathBlock / 64) * BatchSink<kBatchRT>::kLoads * 64 * sizeof(double2);
    static size_t granted = kLdsDefault;
    const hipError_t e = allow_lds((const void *)batched_path_kernel<DB, CAP, kBatchRT>, lds, granted);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((batched_path_kernel<DB, CAP, kBatchRT>), dim3(blocks_for(a.M, kPathBlock)),
                       dim3(kPathBlock), lds, s, a.P, a.B, a.pass, a.W, a.i, a.M, a.seed, a.alpha_b,
                       a.ld, a.S, a.e);
    return hipGetLastError();
}

template <int DB>
static hipError_t batched_cap(int cap, const BatchArgs &a, hipStream_t s) {
    switch (cap) {
    case 2: return batched_t<DB, 2>(a, s);
    case 4: return batched_t<DB, 4>(a, s);
    case 6: if constexpr (DB >= 6) return batched_t<DB, 6>(a, s); break;
    case 8: if constexpr (DB >= 8) return batched_t<DB, 8>(a, s); break;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_batched_path(int db, int cap, const BatchArgs &a, hipStream_t s) {
    switch (db) {
    case 4: return batched_cap<4>(cap, a, s);
    case 8: return batched_cap<8>(cap, a, s);
    case 16: return batched_cap<16>(cap, a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_reduce_batched(const double2 *partial, int32_t nsplit, int64_t nrep_sub, int64_t n_part,
                                 int32_t R, double M, const int32_t *ft, const int32_t *canon_of_trav,
                                 const int32_t *pass_pos, double2 *alpha_b_row, int32_t slot,
                                 double *alpha_row, int32_t *bad, int32_t step, hipStream_t s) {
    hipLaunchKernelGGL(reduce_batched_kernel, dim3(blocks_for(nrep_sub, 256)), dim3(256), 0, s, partial,
                       nsplit, nrep_sub, n_part, R, M, ft, canon_of_trav, pass_pos, alpha_b_row, slot, alpha_row,
                       bad, step);
    return hipGetLastError();
}

// pass projection: tasks of kPassTM nodes, kPassWaves waves, two paths per
// lane up to d = 6 and one above (the accumulators of R responses per node
// and the phase factors share the LDS: 20 KB per wave)
int pass_paths_per_lane(int32_t d) { return d <= 6 ? 2 : 1; }

size_t project_pass_lds_bytes(int32_t d) {
    return (size_t)kPassWaves * ((size_t)kPassTM * kBatchRT * sizeof(double2) +
                                 (size_t)d * 64 * pass_paths_per_lane(d) * sizeof(double2));
}

template <int CAP, int P>
static hipError_t project_pass_t(const Walk &W, const double2 *e, int64_t lde, const double *S, int64_t M,
                                 const int64_t *m_r, int64_t pps, int32_t ntasks, int32_t nsplit, const Task *tasks,
                                 const TaskItem *items, double2 *partial, int64_t nrep, hipStream_t s) {
    const size_t lds = project_pass_lds_bytes(W.d);
    static size_t granted = kLdsDefault;
    const auto kern = project_pass_kernel<CAP, P, kBatchRT, kPassWaves, kPassTM>;
    const hipError_t err = allow_lds((const void *)kern, lds, granted);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(kern, dim3((unsigned)ntasks, (unsigned)nsplit), dim3(kPassWaves * 64), lds, s, W, e, lde, S,
                       M, m_r, pps, tasks, items, partial, nrep);
    return hipGetLastError();
}

hipError_t launch_project_pass(int cap, const Walk &W, const double2 *e, int64_t lde, const double *S, int64_t M,
                               const int64_t *m_r, int64_t pps, int32_t ntasks, int32_t nsplit, const Task *tasks,
                               const TaskItem *items, double2 *partial, int64_t nrep, hipStream_t s) {
    if (project_pass_lds_bytes(W.d) > kLdsMax) return hipErrorInvalidValue;
    const bool two = pass_paths_per_lane(W.d) == 2;
#define QR_PASS_CAP(C)                                                                                           \
    case C:                                                                                                      \
        return two ? project_pass_t<C, 2>(W, e, lde, S, M, m_r, pps, ntasks, nsplit, tasks, items, partial, nrep, s) \
                   : project_pass_t<C, 1>(W, e, lde, S, M, m_r, pps, ntasks, nsplit, tasks, items, partial, nrep, s);
    switch (cap) {
        QR_PASS_CAP(2)
        QR_PASS_CAP(4)
        QR_PASS_CAP(6)
        QR_PASS_CAP(8)
    }
#undef QR_PASS_CAP
    return hipErrorInvalidValue;
}

hipError_t launch_z_responses(const DevProblem *P, uint64_t seed, int32_t i, int64_t M, int32_t k0, int32_t nk,
                              const double *S, const double *f0, const double *y0, double *out, hipStream_t s) {
    hipLaunchKernelGGL(z_responses_kernel, dim3(blocks_for(M, 256)), dim3(256), 0, s, P, seed, i, M, k0, nk, S, f0,
                       y0, out);
    return hipGetLastError();
}

template <int DB>
__global__ void g_points_kernel(const DevProblem *__restrict__ P, const double *__restrict__ x, int64_t n,
                                double *__restrict__ y) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const int d = P->d;
    double xv[DB];
#pragma unroll
    for (int l = 0; l < DB; ++l) xv[l] = l < d ? x[l * n + m] : 0.0;
    y[m] = g_term<DB>(P, xv, d, nullptr);
}

hipError_t launch_g_points(int db, const DevProblem *P, const double *x, int64_t n, double *y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    switch (db) {
    case 4: hipLaunchKernelGGL(g_points_kernel<4>, dim3(blocks_for(n, 256)), dim3(256), 0, s, P, x, n, y); break;
    case 8: hipLaunchKernelGGL(g_points_kernel<8>, dim3(blocks_for(n, 256)), dim3(256), 0, s, P, x, n, y); break;
    case 16: hipLaunchKernelGGL(g_points_kernel<16>, dim3(blocks_for(n, 256)), dim3(256), 0, s, P, x, n, y); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce_slot(const double2 *partial, int32_t nsplit, int64_t nrep, int32_t R, int32_t slot,
                              double M, const int32_t *canon_of_trav, double *alpha_row, int32_t *bad, int32_t step,
                              hipStream_t s) {
    hipLaunchKernelGGL(reduce_slot_kernel, dim3(blocks_for(nrep, 256)), dim3(256), 0, s, partial, nsplit, nrep, R,
                       slot, M, canon_of_trav, alpha_row, bad, step);
    return hipGetLastError();
}

__global__ void fill_i64_kernel(int64_t *__restrict__ p, int64_t n, int64_t v) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) p[idx] = v;
}

hipError_t launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i64_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

template <int DB, int CAP, bool GRAD, int T, int PREC>
static hipError_t mfma_path_t(const MfmaArgs &a, hipStream_t s) {
    const size_t lds = mfma_path_lds_bytes(a.W.d);
    static size_t granted = kLdsDefault;
    const hipError_t e = allow_lds((const void *)mfma_path_kernel<DB, CAP, GRAD, T, PREC>, lds, granted);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((mfma_path_kernel<DB, CAP, GRAD, T, PREC>), dim3(blocks_for(a.M, kPathBlock)),
                       dim3(kPathBlock), lds, s, a.P, a.W, a.i, a.M, a.seed, a.tiles, a.tile_ld, a.S, a.e);
    return hipGetLastError();
}

template <int DB, bool GRAD, int T, int PREC>
static hipError_t mfma_path_cap(int cap, const MfmaArgs &a, hipStream_t s) {
    switch (cap) {
    case 2: return mfma_path_t<DB, 2, GRAD, T, PREC>(a, s);
    case 4: return mfma_path_t<DB, 4, GRAD, T, PREC>(a, s);
    case 6: if constexpr (DB >= 6) return mfma_path_t<DB, 6, GRAD, T, PREC>(a, s); break;
    case 8: if constexpr (DB >= 8) return mfma_path_t<DB, 8, GRAD, T, PREC>(a, s); break;
    }
    return hipErrorInvalidValue;
}

// right-hand-side groups: the smallest T with 1 + d <= 4 T among those the
// dimension bucket instantiates (value only: T = 1)
int mfma_tile_groups(int db, int d, bool grad) {
    if (!grad) return 1;
    const int T = (d + 4) / 4;
    const int lo = db <= 8 ? 2 : 3;
    return T < lo ? lo : T;
}

template <int DB, int PREC>
static hipError_t mfma_path_g(int cap, bool grad, int T, const MfmaArgs &a, hipStream_t s) {
    if (!grad) return mfma_path_cap<DB, false, 1, PREC>(cap, a, s);
    if constexpr (DB == 4) {
        if (T == 2) return mfma_path_cap<4, true, 2, PREC>(cap, a, s);
    } else if constexpr (DB == 8) {
        if (T == 2) return mfma_path_cap<8, true, 2, PREC>(cap, a, s);
        if (T == 3) return mfma_path_cap<8, true, 3, PREC>(cap, a, s);
    } else {
        if (T == 3) return mfma_path_cap<16, true, 3, PREC>(cap, a, s);
        if (T == 4) return mfma_path_cap<16, true, 4, PREC>(cap, a, s);
        if (T == 5) return mfma_path_cap<16, true, 5, PREC>(cap, a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_mfma_path(int db, int cap, bool grad, int prec, const MfmaArgs &a, hipStream_t s) {
    if (prec != QR_PREC_BF16 && prec != QR_PREC_F16) return hipErrorInvalidValue;
    const bool bf = prec == QR_PREC_BF16;
    const int T = mfma_tile_groups(db, a.W.d, grad);
    switch (db) {
    case 4: return bf ? mfma_path_g<4, QR_PREC_BF16>(cap, grad, T, a, s) : mfma_path_g<4, QR_PREC_F16>(cap, grad, T, a, s);
    case 8: return bf ? mfma_path_g<8, QR_PREC_BF16>(cap, grad, T, a, s) : mfma_path_g<8, QR_PREC_F16>(cap, grad, T, a, s);
    case 16: return bf ? mfma_path_g<16, QR_PREC_BF16>(cap, grad, T, a, s) : mfma_path_g<16, QR_PREC_F16>(cap, grad, T, a, s);
    }
    return hipErrorInvalidValue;
}


hipError_t launch_pack_tiles(int prec, const double2 *alpha_int_row, int64_t nrep, const int32_t *trav,
                             int32_t d, int32_t T, bool half, uint2 *out, hipStream_t s) {
    const int64_t ngroups = (nrep + kMfmaGroup - 1) / kMfmaGroup;
    const int64_t total = ngroups * T * 64;
    const double theta = half ? M_PI : 2.0 * M_PI;
    if (prec == QR_PREC_BF16)
        hipLaunchKernelGGL(pack_tiles_kernel<QR_PREC_BF16>, dim3(blocks_for(total, 256)), dim3(256), 0, s,
                           alpha_int_row, nrep, trav, d, T, ngroups, theta, out);
    else if (prec == QR_PREC_F16)
        hipLaunchKernelGGL(pack_tiles_kernel<QR_PREC_F16>, dim3(blocks_for(total, 256)), dim3(256), 0, s,
                           alpha_int_row, nrep, trav, d, T, ngroups, theta, out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

static inline unsigned sm_blocks(int64_t n) { return blocks_for(n, 256); }

hipError_t launch_sm_start(const DevProblem *P, int32_t nu, int32_t i, int64_t M, uint64_t seed, double *x, double2 *e,
                           double *S, hipStream_t s) {
    hipLaunchKernelGGL(sm_start_kernel, dim3(sm_blocks(M)), dim3(256), 0, s, P, nu, i, M, seed, x, e, S);
    return hipGetLastError();
}

hipError_t launch_sm_euler(int db, const DevProblem *P, int32_t i, int32_t j, int64_t M, uint64_t seed, double *x,
                           double *H, hipStream_t s) {
    switch (db) {
    case 4: hipLaunchKernelGGL(sm_euler_kernel<4>, dim3(sm_blocks(M)), dim3(256), 0, s, P, i, j, M, seed, x, H); break;
    case 8: hipLaunchKernelGGL(sm_euler_kernel<8>, dim3(sm_blocks(M)), dim3(256), 0, s, P, i, j, M, seed, x, H); break;
    case 16: hipLaunchKernelGGL(sm_euler_kernel<16>, dim3(sm_blocks(M)), dim3(256), 0, s, P, i, j, M, seed, x, H); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sm_accum(const DevProblem *P, int32_t j, int64_t m0, int64_t n, const double *y64,
                           const float *y32, double mu, double sigma, const double *H, double *S, hipStream_t s) {
    hipLaunchKernelGGL(sm_accum_kernel, dim3(sm_blocks(n)), dim3(256), 0, s, P, j, m0, n, y64, y32, mu, sigma, H, S);
    return hipGetLastError();
}

hipError_t launch_sm_final(int db, const DevProblem *P, int64_t M, const double *x, const double *H, double *S,
                           hipStream_t s) {
    switch (db) {
    case 4: hipLaunchKernelGGL(sm_final_kernel<4>, dim3(sm_blocks(M)), dim3(256), 0, s, P, M, x, H, S); break;
    case 8: hipLaunchKernelGGL(sm_final_kernel<8>, dim3(sm_blocks(M)), dim3(256), 0, s, P, M, x, H, S); break;
    case 16: hipLaunchKernelGGL(sm_final_kernel<16>, dim3(sm_blocks(M)), dim3(256), 0, s, P, M, x, H, S); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_moments(int64_t n, const double *t, double *partial, hipStream_t s) {
    hipLaunchKernelGGL(moments_kernel, dim3(sm_blocks(n)), dim3(256), 0, s, n, t, partial);
    return hipGetLastError();
}

}  // namespace qrmc
