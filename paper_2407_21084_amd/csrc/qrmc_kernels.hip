// qrmc_kernels.hip -- gfx950 kernels of the QRMC backward step.
//
// One backward iteration i of Algorithm 1 (GQRMDP, eqs (yqi:bar:M),
// (Aqi:bar:M), (Sqi:bar:M)) runs as
//   path_kernel     one thread per path: start draw X_i ~ nu, Euler steps
//                   (eq (markov:euler)), expansion ybar_{j+1}(X_{j+1}) by the
//                   basis traversal below, driver sum S_i;
//   project_kernel  (task of basis functions) x (slice of paths): the same
//                   traversal at X_i, S-weighted, reduced over lanes through
//                   LDS, partial sums per slice;
//   reduce_kernel   fixed-order sum over slices, scaling by 1/M.
//
// Basis traversal.  Every representative k != 0 is reached from a node with
// one coordinate fewer or one unit smaller in its last non-zero coordinate,
// so e^{2 pi i k.u} costs one complex multiplication by e^{+-2 pi i u_l}:
// nodes are visited depth-first, coordinates l ascending, sign + before -,
// magnitudes m ascending.  All lanes of a wave walk the same sequence of
// nodes, so the loop bounds and the coefficient stream are wave-uniform: the
// coefficients come through scalar loads, the per-lane values e^{2 pi i u_l}
// sit in LDS (one 16-byte slot per lane and coordinate), and the chain of
// values lives in registers.
#include "qrmc_kernels.h"

namespace qrmc {

#define QR_CONST __attribute__((address_space(4)))

struct cplx {
    double re, im;
};

__device__ __forceinline__ cplx cmul(const cplx a, const cplx b) {
    return cplx{fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-lane LDS slots: e^{2 pi i u_l} at E[l * stride], gradient accumulators
// (d ybar / d u_l up to 2 pi) at G[l * stride].
struct LaneLds {
    double2 *E;
    double *G;
    int stride;
    __device__ __forceinline__ cplx e(int l) const {
        const double2 v = E[l * stride];
        return cplx{v.x, v.y};
    }
    __device__ __forceinline__ void grad_add(int l, double g) const { G[l * stride] += g; }
};

// Per-coordinate transcendental work of the path kernel.  Called O(d) times
// per Euler step against O(|Gamma|) basis work, so they stay out of line:
// their FP64 coefficients (which gfx9-class VOP3 cannot take as literals) are
// then materialised per call instead of being hoisted into registers that
// would stay live across the basis traversal.
__device__ __noinline__ double nl_norm_icdf(double u) { return norm_icdf(u); }
__device__ __noinline__ double nl_logistic_icdf(double u) { return logistic_icdf(u); }
__device__ __noinline__ double nl_logistic_cdf(double x) { return logistic_cdf(x); }
__device__ __noinline__ double2 nl_unit_phase(double x) {
    // e^{2 pi i F(x)}
    double sn, cs;
    sincospi(2.0 * logistic_cdf(x), &sn, &cs);
    return make_double2(cs, sn);
}
__device__ __noinline__ double2 nl_sincos_exp(double th, double a) {
    // (sin th, exp(a)), th reduced through sincospi
    double sn, cs;
    sincospi(th * M_1_PI, &sn, &cs);
    (void)cs;
    return make_double2(sn, exp(a));
}
__device__ __noinline__ double2 nl_sincos(double th) {
    double sn, cs;
    sincospi(th * M_1_PI, &sn, &cs);
    return make_double2(sn, cs);
}
__device__ __noinline__ double nl_exp(double a) { return exp(a); }
__device__ __noinline__ double nl_sin(double a) { return sin(a); }

// Children of a node at depth T (T non-zero coordinates, last one p, budget
// product P) with value `parent`, in traversal order.  Each level keeps its
// own accumulators (returned to the caller), which keeps the values that
// cross loop levels few.  With gradients, `g` of the returned accumulator is
// the sum over all visited subtrees of the sink's per-node values, from which
// the caller applies the chain rule for its own coordinate.
template <int T, int CAP, class Sink>
__device__ __forceinline__ typename Sink::Acc visit(const cplx parent, const int p, const int P,
                                                    const SetRule &R, const LaneLds &L,
                                                    Sink &sink) {
    typename Sink::Acc acc{};
#pragma unroll 1
    for (int l = p + 1; l < R.d; ++l) {
        const cplx e = L.e(l);
        double gl = 0.0;
#pragma unroll 1
        for (int s = 0; s < (T == 0 ? 1 : 2); ++s) {
            const cplx es{e.re, s ? -e.im : e.im};
            cplx v = parent;
#pragma unroll 1
            for (int m = 1; rule_ok(R, P, m); ++m) {
                v = cmul(v, es);
                double gsub = sink.node(v, acc);
                if constexpr (T + 1 < CAP) {
                    const int P2 = rule_child(R, P, m);
                    if (l + 1 < R.d && rule_ok(R, P2, 1)) {
                        const typename Sink::Acc c = visit<T + 1, CAP>(v, l, P2, R, L, sink);
                        Sink::add(acc, c);
                        if constexpr (Sink::kGrad) gsub += c.g;
                    }
                }
                if constexpr (Sink::kGrad) gl = fma(s ? -(double)m : (double)m, gsub, gl);
            }
        }
        if constexpr (Sink::kGrad) L.grad_add(l, gl);
    }
    return acc;
}

// Start the traversal below a node of runtime depth `depth` (< CAP).
template <int T, int CAP, class Sink>
__device__ __forceinline__ void visit_from(int depth, const cplx v, int p, int P, const SetRule &R,
                                           const LaneLds &L, Sink &sink) {
    if constexpr (T < CAP) {
        if (depth == T) {
            (void)visit<T, CAP>(v, p, P, R, L, sink);
            return;
        }
        visit_from<T + 1, CAP>(depth, v, p, P, R, L, sink);
    }
}

// ---------------------------------------------------------------------------
// Expansion evaluation sink: y = sum_r a_r.x Re(e_r) + a_r.y Im(e_r) with the
// internal coefficients a_r = (sqrt2 alpha_cos, sqrt2 alpha_sin), a_0 = (alpha_0, 0);
// with gradients, g_r = a_r.y Re(e_r) - a_r.x Im(e_r) (d/du of the node up to 2 pi k).
// ---------------------------------------------------------------------------
template <bool GRAD>
struct EvalAccT {
    double y;
};
template <>
struct EvalAccT<true> {
    double y, g;
};

typedef __attribute__((address_space(3))) double lds_double;

// Coefficient row staged through LDS: a ring of 4 chunks of kPathBlock nodes
// shared by the block.  While chunk k is traversed, chunks k and k+1 are in
// the ring and chunk k+3 is on its way into registers; at the boundary into
// chunk k (one barrier) the block stores chunk k+2 into the slot of chunk
// k-2 and requests chunk k+3.  All threads of the block walk the same node
// sequence, so the barriers are uniform.  Coefficients of the next node are
// read one node ahead.
template <bool GRAD>
struct EvalSink {
    static constexpr bool kGrad = GRAD;
    using Acc = EvalAccT<GRAD>;
    const double2 *g;   // row in global memory
    int64_t n;          // readable entries of the row
    lds_double *ring;   // LDS [4 * kPathBlock][2]
    double2 pend;       // this thread's node of the chunk in flight
    int tid;
    int idx;            // node about to be visited
    double2 nxt;        // its coefficients

    __device__ __forceinline__ double2 fetch(int64_t r) const {
        return r < n ? g[r] : make_double2(0.0, 0.0);
    }
    __device__ __forceinline__ void start() {
#pragma unroll
        for (int c = 0; c < 3; ++c) put(c * kPathBlock + tid, fetch((int64_t)c * kPathBlock + tid));
        pend = fetch(3 * (int64_t)kPathBlock + tid);
        __syncthreads();
        idx = 0;
        nxt = get(0);
    }
    __device__ __forceinline__ void put(int slot, const double2 v) {
        ring[2 * slot] = v.x;
        ring[2 * slot + 1] = v.y;
    }
    __device__ __forceinline__ double2 get(int slot) const {
        return make_double2(ring[2 * slot], ring[2 * slot + 1]);
    }
    __device__ __forceinline__ void boundary(int k) {  // entering chunk k >= 1
        __syncthreads();
        put(((k + 2) & 3) * kPathBlock + tid, pend);
        pend = fetch((int64_t)(k + 3) * kPathBlock + tid);
    }
    __device__ __forceinline__ double node(const cplx v, Acc &acc) {
        const double cx = nxt.x, cy = nxt.y;
        acc.y = fma(cx, v.re, fma(cy, v.im, acc.y));
        ++idx;
        if ((idx & (kPathBlock - 1)) == 0) boundary(idx / kPathBlock);
        nxt = get(idx & (4 * kPathBlock - 1));
        if constexpr (GRAD) {
            const double gr = fma(cy, v.re, -(cx * v.im));
            acc.g += gr;
            return gr;
        }
        return 0.0;
    }
    __device__ __forceinline__ static void add(Acc &a, const Acc &b) {
        a.y += b.y;
        if constexpr (GRAD) a.g += b.g;
    }
};

// Expansion at the lane's point by the depth-first traversal.  Every thread of
// the block must call it (the coefficient staging uses block barriers).
template <int CAP, bool GRAD>
__device__ __forceinline__ double tree_eval(const double2 *alpha_row, int64_t nrow, double2 *ring,
                                            const SetRule &R, const LaneLds &L) {
    EvalSink<GRAD> s{alpha_row, nrow, (lds_double *)ring, make_double2(0.0, 0.0),
                     (int)threadIdx.x, 0, make_double2(0.0, 0.0)};
    s.start();
    typename EvalSink<GRAD>::Acc root{};
    const cplx one{1.0, 0.0};
    s.node(one, root);
    const auto acc = visit<0, CAP>(one, -1, 1, R, L, s);
    // the ring is reused by the next call: let every wave finish reading it
    __syncthreads();
    return root.y + acc.y;
}

// ---------------------------------------------------------------------------
// Flat node program (value-only paths): the registers v[t] hold the current
// node value at each depth t and mult[t] the factor of the chain at depth t;
// a uniform switch on the op's depth keeps every register index static.
// ---------------------------------------------------------------------------
template <int CAP>
struct Flat {
    cplx v[CAP + 1];
    cplx mult[CAP + 1];
};

template <int T, int CAP>
__device__ __forceinline__ void flat_step(Flat<CAP> &st, const uint32_t op, const LaneLds &L) {
    if constexpr (T == 0) {
        (void)op;
    } else if (op & kOpNew) {
        cplx e = L.e((int)((op >> 5) & 15u));
        if (op & kOpNeg) e.im = -e.im;
        st.mult[T] = e;
        st.v[T] = cmul(st.v[T - 1], e);
    } else {
        st.v[T] = cmul(st.v[T], st.mult[T]);
    }
}

// Apply `op` and hand the node value to `use`.
template <int CAP, class F>
__device__ __forceinline__ void flat_node(Flat<CAP> &st, const uint32_t op, const LaneLds &L, F &&use) {
#define QR_FLAT_CASE(T)                       \
    case T:                                   \
        if constexpr (T <= CAP) {             \
            flat_step<T, CAP>(st, op, L);     \
            use(st.v[T]);                     \
        }                                     \
        break;
    switch (op & 15u) {
        QR_FLAT_CASE(0)
        QR_FLAT_CASE(1)
        QR_FLAT_CASE(2)
        QR_FLAT_CASE(3)
        QR_FLAT_CASE(4)
        QR_FLAT_CASE(5)
        QR_FLAT_CASE(6)
        QR_FLAT_CASE(7)
        QR_FLAT_CASE(8)
    default: break;
    }
#undef QR_FLAT_CASE
}

// ybar at the lane's point: nodes 0..nrep-1 in groups of 8 whose ops and
// coefficients arrive through batched scalar loads (rows padded by kOpPad).
template <int CAP>
__device__ __forceinline__ double flat_eval(const double2 *alpha_row, const uint32_t *ops,
                                            const int64_t nrep, const LaneLds &L) {
    const QR_CONST double *a = (const QR_CONST double *)alpha_row;
    const QR_CONST uint32_t *o = (const QR_CONST uint32_t *)ops;
    Flat<CAP> st;
    st.v[0] = cplx{1.0, 0.0};
#pragma unroll
    for (int t = 1; t <= CAP; ++t) {
        st.v[t] = cplx{0.0, 0.0};
        st.mult[t] = cplx{1.0, 0.0};
    }
    double yre = 0.0, yim = 0.0;
#pragma unroll 1
    for (int64_t r = 0; r < nrep; r += 8) {
        uint32_t op[8];
        double ax[8], ay[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            op[q] = o[r + q];
            ax[q] = a[2 * (r + q)];
            ay[q] = a[2 * (r + q) + 1];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            flat_node<CAP>(st, op[q], L, [&](const cplx v) {
                yre = fma(ax[q], v.re, yre);
                yim = fma(ay[q], v.im, yim);
            });
        }
    }
    return yre + yim;
}

// ---------------------------------------------------------------------------
// Manufactured problem pieces (closed forms of u, g, h; see qrmc.h)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double fnl(const DevProblem *P, double y, double z2) {
    switch (P->driver) {
    case QR_F_SIN: return P->f_a * nl_sin(y);
    case QR_F_ALLEN_CAHN: return y - y * y * y;
    case QR_F_ZRAT: return P->f_a * z2 / (1.0 + z2) + y / (1.0 + y * y);
    default: return 0.0;
    }
}

template <int DB>
__device__ __forceinline__ double h_source(const DevProblem *P, double t, const double *x, int d) {
    const double E = P->sol_A * nl_exp(-P->sol_c * (P->T - t));
    double th = P->sol_p, bw = 0.0;
#pragma unroll
    for (int l = 0; l < DB; ++l) {
        if (l < d) {
            th = fma(P->sol_w[l], x[l], th);
            bw = fma(fma(P->b1[l], x[l], P->b0[l]), P->sol_w[l], bw);
        }
    }
    const double2 sc = nl_sincos(th);  // sincospi avoids the large-argument reduction
    const double sn = sc.x, cs = sc.y;
    const double u = E * cs;
    const double gscale = -E * sn;  // grad u = gscale * w
    const double z2 = gscale * gscale * P->sw2;
    return -(P->sol_c * u + gscale * bw - 0.5 * u * P->sw2) - fnl(P, u, z2);
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
    return P->sol_A * cs;
}

__device__ __forceinline__ double clamp_abs(double y, double L) {
    return y > L ? L : (y < -L ? -L : y);
}

// ---------------------------------------------------------------------------
// path_kernel: one thread per path of backward iteration i.
// alpha_int rows have stride ld = nrep + kOpPad double2.
// ---------------------------------------------------------------------------
template <int DB, int CAP, bool GRAD>
__global__ __launch_bounds__(kPathBlock) void path_kernel(
    const DevProblem *__restrict__ P0, const SetRule R, const int32_t i, const int64_t M,
    const uint64_t seed, const double2 *__restrict__ alpha_int, const uint32_t *__restrict__ ops,
    const int64_t nrep, const int64_t ld, double *__restrict__ S_out, double *__restrict__ u_out,
    double *__restrict__ x_out) {
    extern __shared__ double2 lds[];
    const int tid = threadIdx.x;
    // lanes past M simulate a path too (block barriers), but store nothing
    const int64_t m = (int64_t)blockIdx.x * kPathBlock + tid;
    const bool live = m < M;
    const int d = P0->d, nbm = P0->nbm, N = P0->N;
    double2 *ring = lds;
    double2 *lane_base = lds + 4 * kPathBlock;
    const LaneLds L{lane_base + tid,
                    GRAD ? reinterpret_cast<double *>(lane_base + d * kPathBlock) + tid : nullptr,
                    kPathBlock};
    // the path state waits in LDS while the traversal runs
    double *xs = reinterpret_cast<double *>(lane_base + d * kPathBlock) + (GRAD ? d * kPathBlock : 0) + tid;

    PhiloxStream rs(seed, 0u, (uint64_t)m, (uint32_t)i, 0u);
    double x[DB];
#pragma unroll
    for (int l = 0; l < DB; ++l) {
        x[l] = 0.0;
        if (l < d) {
            x[l] = nl_logistic_icdf(rs.next());
            if (live && u_out) u_out[l * M + m] = nl_logistic_cdf(x[l]);
            if (live && x_out) x_out[l * M + m] = x[l];
        }
    }

    double S = 0.0;
    for (int j = i; j < N; ++j) {
        // Re-read the problem each step instead of pinning every parameter in
        // scalar registers across the basis traversal.
        const DevProblem *__restrict__ P = P0;
        asm volatile("" : "+s"(P));
        const double tj = P->t[j];
        const double dt = P->t[j + 1] - tj;
        // the source term only needs X_j: take it before X_j is overwritten
        const double hj = h_source<DB>(P, tj, x, d);
        {
            // Euler step, eq (markov:euler); one normal at a time keeps the
            // quantile evaluations sequential (few live registers)
            const double sq = sqrt(dt);
#pragma unroll
            for (int l = 0; l < DB; ++l)
                if (l < d) x[l] = fma(fma(P->b1[l], x[l], P->b0[l]), dt, x[l]);
#pragma unroll 1
            for (int k = 0; k < nbm; ++k) {
                const double dwk = sq * nl_norm_icdf(rs.next());
#pragma unroll
                for (int l = 0; l < DB; ++l)
                    if (l < d) x[l] = fma(P->sigma[l * nbm + k], dwk, x[l]);
            }
        }
        // x now holds X_{j+1}
        double y, gx[DB];
        if (j + 1 < N) {
#pragma unroll
            for (int l = 0; l < DB; ++l) {
                if (l < d) {
                    L.E[l * kPathBlock] = nl_unit_phase(x[l]);
                    if constexpr (GRAD) L.G[l * kPathBlock] = 0.0;
                }
            }
            const double2 *row = alpha_int + (int64_t)(j + 1) * ld;
#pragma unroll
            for (int l = 0; l < DB; ++l)
                if (l < d) xs[l * kPathBlock] = x[l];
            asm volatile("" ::: "memory");
            if constexpr (GRAD) {
                y = tree_eval<CAP, true>(row, ld, ring, R, L);
#pragma unroll
                for (int l = 0; l < DB; ++l) {
                    if (l < d) {
                        const double u = nl_logistic_cdf(x[l]);
                        gx[l] = 2.0 * M_PI * L.G[l * kPathBlock] * (u * (1.0 - u));
                    }
                }
            } else {
#ifdef QRMC_FLAT_EVAL
                y = flat_eval<CAP>(row, ops, nrep, L);
#else
                (void)ops;
                y = tree_eval<CAP, false>(row, ld, ring, R, L);
#endif
            }
            asm volatile("" ::: "memory");
#pragma unroll
            for (int l = 0; l < DB; ++l)
                if (l < d) x[l] = xs[l * kPathBlock];
        } else {
            y = g_term<DB>(P, x, d, GRAD ? gx : nullptr);
        }
        y = clamp_abs(y, P->clamp);
        double z2 = 0.0;
        if constexpr (GRAD) {
#pragma unroll
            for (int k = 0; k < DB; ++k) {
                if (k < nbm) {
                    double zk = 0.0;
#pragma unroll
                    for (int l = 0; l < DB; ++l)
                        if (l < d) zk = fma(P->sigma[l * nbm + k], gx[l], zk);
                    z2 = fma(zk, zk, z2);
                }
            }
        }
        const double f = fnl(P, y, z2) + hj;
        S = fma(f, dt, S);
    }
    S += g_term<DB>(P0, x, d, nullptr);
    if (live) S_out[m] = S;
}

// ---------------------------------------------------------------------------
// project_kernel: block (task of the traversal, slice of paths).
// Each wave runs 64 paths at a time through the task's nodes; node values
// times S go to a per-wave LDS buffer and are summed over the lanes every
// kProjChunk nodes into per-wave accumulators; the block finally adds its
// waves in a fixed order and writes the slice's partial sums.
// ---------------------------------------------------------------------------
struct ProjSink {
    static constexpr bool kGrad = false;
    struct Acc {};
    __device__ __forceinline__ static void add(Acc &, const Acc &) {}
    double2 *row;    // this lane's row of the wave buffer: row[c]
    double2 *wbuf;   // wave buffer [64][kProjChunk + 1]
    double *acc;     // wave accumulators, doubles [kTaskMax][2]
    double s;        // this lane's response (0 for lanes past the slice)
    int c;           // nodes in the current chunk (wave-uniform)
    int base;        // task-local index of the chunk's first node (wave-uniform)
    int lane;

    __device__ __forceinline__ double node(const cplx v, Acc &) {
        row[c] = make_double2(s * v.re, s * v.im);
        if (++c == kProjChunk) flush();
        return 0.0;
    }

    // Sum the chunk over the 64 lanes: lane q adds the 16 lanes of quarter
    // q>>4 for value q&15 (node (q&15)>>1, component q&1); the quarters are
    // then combined by two xor-shuffles in a fixed order.
    __device__ __forceinline__ void flush() {
        wave_sync();
        const int val = lane & 15, rep = val >> 1, quarter = lane >> 4;
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const double2 w = wbuf[(quarter * 16 + k) * (kProjChunk + 1) + rep];
            sum += (val & 1) ? w.y : w.x;
        }
        sum += __shfl_xor(sum, 16);
        sum += __shfl_xor(sum, 32);
        if (lane < 16 && rep < c) acc[(base + rep) * 2 + (val & 1)] += sum;
        wave_sync();
        base += c;
        c = 0;
    }
};

size_t project_lds_bytes(int32_t d) {
    return (size_t)kProjWaves *
           ((size_t)64 * (kProjChunk + 1) * sizeof(double2) + (size_t)kTaskMax * sizeof(double2) +
            (size_t)d * 64 * sizeof(double2));
}

template <int CAP>
__global__ __launch_bounds__(kProjWaves * 64) void project_kernel(
    const SetRule R, const double *__restrict__ u_in, const double *__restrict__ s_in,
    const int64_t M, const int64_t paths_per_split, const Task *__restrict__ tasks,
    const TaskItem *__restrict__ items, double2 *__restrict__ partial, const int64_t nrep) {
    extern __shared__ double2 lds[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int d = R.d;
    double2 *bufs = lds;
    double *accs = reinterpret_cast<double *>(lds + kProjWaves * 64 * (kProjChunk + 1));
    double2 *Es = lds + kProjWaves * 64 * (kProjChunk + 1) + kProjWaves * kTaskMax;

    double2 *wbuf = bufs + wave * 64 * (kProjChunk + 1);
    double *acc = accs + wave * kTaskMax * 2;
    const LaneLds L{Es + wave * d * 64 + lane, nullptr, 64};

    const Task task = tasks[blockIdx.x];
    const int64_t m0 = (int64_t)blockIdx.y * paths_per_split;
    const int64_t m1 = min(M, m0 + paths_per_split);

    for (int r = lane; r < kTaskMax * 2; r += 64) acc[r] = 0.0;
    wave_sync();

    ProjSink sink{wbuf + lane * (kProjChunk + 1), wbuf, acc, 0.0, 0, 0, lane};
    for (int64_t gb = m0 + wave * 64; gb < m1; gb += kProjWaves * 64) {
        const int64_t m = gb + lane;
        const bool live = m < m1;
        sink.s = live ? s_in[m] : 0.0;
        for (int l = 0; l < d; ++l) {
            const double u = live ? u_in[l * M + m] : 0.25;
            double sn, cs;
            sincospi(2.0 * u, &sn, &cs);
            L.E[l * 64] = make_double2(cs, sn);
        }
        sink.c = 0;
        sink.base = 0;
        for (int it = task.item_begin; it < task.item_end; ++it) {
            const TaskItem &I = items[it];
            cplx v{1.0, 0.0};
            for (int t = 0; t < I.depth; ++t) {
                cplx e = L.e(I.coord[t]);
                int n = I.val[t];
                if (n < 0) {
                    e.im = -e.im;
                    n = -n;
                }
                for (int q = 0; q < n; ++q) v = cmul(v, e);
            }
            ProjSink::Acc none;
            sink.node(v, none);
            if (I.full) visit_from<0, CAP>(I.depth, v, I.last, I.prod, R, L, sink);
        }
        if (sink.c) sink.flush();
    }
    __syncthreads();
    double *out = reinterpret_cast<double *>(partial + (int64_t)blockIdx.y * nrep + task.rep_begin);
    for (int r = tid; r < task.rep_count * 2; r += kProjWaves * 64) {
        double sacc = 0.0;
#pragma unroll
        for (int w = 0; w < kProjWaves; ++w) sacc += accs[w * kTaskMax * 2 + r];
        out[r] = sacc;
    }
}

// ---------------------------------------------------------------------------
// reduce_kernel: alpha_i from the slice partial sums, fixed order
// ---------------------------------------------------------------------------
__global__ void reduce_kernel(const double2 *__restrict__ partial, int32_t nsplit, int64_t nrep,
                              double M, double2 *__restrict__ alpha_int_row,
                              double *__restrict__ alpha_row,
                              const int32_t *__restrict__ canon_of_trav) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep) return;
    double sx = 0.0, sy = 0.0;
    for (int s = 0; s < nsplit; ++s) {
        const double2 p = partial[(int64_t)s * nrep + r];
        sx += p.x;
        sy += p.y;
    }
    if (r == 0) {
        const double a0 = sx / M;
        alpha_int_row[0] = make_double2(a0, 0.0);
        if (alpha_row) alpha_row[0] = a0;
    } else {
        const double mc = sx / M, ms = sy / M;
        alpha_int_row[r] = make_double2(2.0 * mc, 2.0 * ms);
        if (alpha_row) {
            const int64_t c = canon_of_trav[r];
            alpha_row[2 * c - 1] = M_SQRT2 * mc;
            alpha_row[2 * c] = M_SQRT2 * ms;
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
__global__ __launch_bounds__(kPathBlock) void eval_kernel(const SetRule R,
                                                          const double2 *__restrict__ alpha_int_row,
                                                          const uint32_t *__restrict__ ops,
                                                          const int64_t nrep,
                                                          const double *__restrict__ x,
                                                          const int64_t n, double *__restrict__ y,
                                                          double *__restrict__ grad) {
    extern __shared__ double2 lds[];
    const int tid = threadIdx.x;
    // lanes past n evaluate a dummy point (block barriers) and store nothing
    const int64_t p0 = (int64_t)blockIdx.x * kPathBlock + tid;
    const bool live = p0 < n;
    const int64_t p = live ? p0 : n - 1;
    const int d = R.d;
    double2 *ring = lds;
    double2 *lane_base = lds + 4 * kPathBlock;
    const LaneLds L{lane_base + tid,
                    GRAD ? reinterpret_cast<double *>(lane_base + d * kPathBlock) + tid : nullptr,
                    kPathBlock};
    for (int l = 0; l < d; ++l) {
        const double u = logistic_cdf(x[l * n + p]);
        double sn, cs;
        sincospi(2.0 * u, &sn, &cs);
        L.E[l * kPathBlock] = make_double2(cs, sn);
        if constexpr (GRAD) L.G[l * kPathBlock] = 0.0;
    }
    const int64_t ld = nrep + kOpPad;
    if constexpr (GRAD) {
        const double yv = tree_eval<CAP, true>(alpha_int_row, ld, ring, R, L);
        if (live) {
            y[p] = yv;
            for (int l = 0; l < d; ++l) {
                const double u = logistic_cdf(x[l * n + p]);
                grad[l * n + p] = 2.0 * M_PI * L.G[l * kPathBlock] * (u * (1.0 - u));
            }
        }
    } else {
#ifdef QRMC_FLAT_EVAL
        const double yv = flat_eval<CAP>(alpha_int_row, ops, nrep, L);
#else
        (void)ops;
        const double yv = tree_eval<CAP, false>(alpha_int_row, ld, ring, R, L);
#endif
        if (live) y[p] = yv;
    }
}

__global__ void x_to_u_kernel(int32_t d, const double *__restrict__ x, int64_t n,
                              double *__restrict__ u) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < (int64_t)d * n) u[idx] = logistic_cdf(x[idx]);
}

__global__ void sample_kernel(int32_t d, uint64_t seed, uint32_t stream_id, int32_t i, int64_t m0,
                              int64_t n, double *__restrict__ x) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    PhiloxStream rs(seed, stream_id, (uint64_t)(m0 + p), (uint32_t)i, 0u);
    for (int l = 0; l < d; ++l) x[l * n + p] = logistic_icdf(rs.next());
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_gather(const double *alpha, int32_t row0, int32_t nrows, int64_t nrep, int64_t ld,
                         int64_t nfuncs, const int32_t *canon_of_trav, double2 *alpha_int,
                         hipStream_t s) {
    const int64_t total = (int64_t)nrows * nrep;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, alpha, row0,
                       nrows, nrep, ld, nfuncs, canon_of_trav, alpha_int);
    return hipGetLastError();
}

hipError_t launch_pad(int32_t nrows, int64_t nrep, int64_t ld, double2 *alpha_int, hipStream_t s) {
    const int64_t total = (int64_t)nrows * (ld - nrep);
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(pad_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, nrows, nrep, ld,
                       alpha_int);
    return hipGetLastError();
}

template <int DB, int CAP, bool GRAD>
static hipError_t path_t(const PathArgs &a, hipStream_t s) {
    const size_t lds = 4 * kPathBlock * sizeof(double2) +
                       (size_t)a.R.d * kPathBlock * (sizeof(double2) + sizeof(double) + (GRAD ? sizeof(double) : 0));
    hipLaunchKernelGGL((path_kernel<DB, CAP, GRAD>), dim3(blocks_for(a.M, kPathBlock)),
                       dim3(kPathBlock), lds, s, a.P, a.R, a.i, a.M, a.seed, a.alpha_int, a.ops,
                       a.nrep, a.ld, a.S, a.u, a.x0);
    return hipGetLastError();
}

template <int DB, bool GRAD>
static hipError_t path_cap(int cap, const PathArgs &a, hipStream_t s) {
    switch (cap) {
    case 2: return path_t<DB, 2, GRAD>(a, s);
    case 4: return path_t<DB, 4, GRAD>(a, s);
    case 6: if constexpr (DB >= 6) return path_t<DB, 6, GRAD>(a, s); break;
    case 8: if constexpr (DB >= 8) return path_t<DB, 8, GRAD>(a, s); break;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_path(int db, int cap, bool grad, const PathArgs &a, hipStream_t s) {
    switch (db) {
    case 4: return grad ? path_cap<4, true>(cap, a, s) : path_cap<4, false>(cap, a, s);
    case 8: return grad ? path_cap<8, true>(cap, a, s) : path_cap<8, false>(cap, a, s);
    case 16: return grad ? path_cap<16, true>(cap, a, s) : path_cap<16, false>(cap, a, s);
    }
    return hipErrorInvalidValue;
}

template <int CAP>
static hipError_t project_t(const SetRule &R, const double *u, const double *S, int64_t M, int64_t pps,
                            int32_t ntasks, int32_t nsplit, const Task *tasks,
                            const TaskItem *items, double2 *partial, int64_t nrep, hipStream_t s) {
    const size_t lds = project_lds_bytes(R.d);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)project_kernel<CAP>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)project_lds_bytes(kMaxD));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(project_kernel<CAP>, dim3((unsigned)ntasks, (unsigned)nsplit),
                       dim3(kProjWaves * 64), lds, s, R, u, S, M, pps, tasks, items, partial, nrep);
    return hipGetLastError();
}

hipError_t launch_project(int cap, const SetRule &R, const double *u, const double *S, int64_t M,
                          int64_t paths_per_split, int32_t ntasks, int32_t nsplit, const Task *tasks,
                          const TaskItem *items, double2 *partial, int64_t nrep, hipStream_t s) {
    switch (cap) {
    case 2: return project_t<2>(R, u, S, M, paths_per_split, ntasks, nsplit, tasks, items, partial, nrep, s);
    case 4: return project_t<4>(R, u, S, M, paths_per_split, ntasks, nsplit, tasks, items, partial, nrep, s);
    case 6: return project_t<6>(R, u, S, M, paths_per_split, ntasks, nsplit, tasks, items, partial, nrep, s);
    case 8: return project_t<8>(R, u, S, M, paths_per_split, ntasks, nsplit, tasks, items, partial, nrep, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(const double2 *partial, int32_t nsplit, int64_t nrep, double M,
                         double2 *alpha_int_row, double *alpha_row,
                         const int32_t *canon_of_trav, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3(blocks_for(nrep, 256)), dim3(256), 0, s, partial, nsplit,
                       nrep, M, alpha_int_row, alpha_row, canon_of_trav);
    return hipGetLastError();
}

template <int CAP, bool GRAD>
static hipError_t eval_t(const SetRule &R, const double2 *a, const uint32_t *ops, int64_t nrep,
                         const double *x, int64_t n, double *y, double *g, hipStream_t s) {
    const size_t lds = 4 * kPathBlock * sizeof(double2) +
                       (size_t)R.d * kPathBlock * (sizeof(double2) + (GRAD ? sizeof(double) : 0));
    hipLaunchKernelGGL((eval_kernel<CAP, GRAD>), dim3(blocks_for(n, kPathBlock)), dim3(kPathBlock),
                       lds, s, R, a, ops, nrep, x, n, y, g);
    return hipGetLastError();
}

hipError_t launch_eval(int cap, bool grad, const SetRule &R, const double2 *alpha_int_row,
                       const uint32_t *ops, int64_t nrep, const double *x, int64_t n, double *y,
                       double *grad_out, hipStream_t s) {
    if (n == 0) return hipSuccess;
#define QR_EVAL_CAP(C)                                                                   \
    case C:                                                                              \
        return grad ? eval_t<C, true>(R, alpha_int_row, ops, nrep, x, n, y, grad_out, s) \
                    : eval_t<C, false>(R, alpha_int_row, ops, nrep, x, n, y, grad_out, s);
    switch (cap) {
        QR_EVAL_CAP(2)
        QR_EVAL_CAP(4)
        QR_EVAL_CAP(6)
        QR_EVAL_CAP(8)
    }
#undef QR_EVAL_CAP
    return hipErrorInvalidValue;
}

hipError_t launch_x_to_u(int32_t d, const double *x, int64_t n, double *u, hipStream_t s) {
    const int64_t total = (int64_t)d * n;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(x_to_u_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, d, x, n, u);
    return hipGetLastError();
}

hipError_t launch_sample(int32_t d, uint64_t seed, uint32_t stream_id, int32_t i, int64_t m0,
                         int64_t n, double *x, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(sample_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, seed, stream_id,
                       i, m0, n, x);
    return hipGetLastError();
}

}  // namespace qrmc
