// qrmc_api.hip -- host side of libqrmc: index sets and basis metadata,
// context and workspace, argument validation and the C entry points of qrmc.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "qrmc_factored.h"
#include "qrmc_kernels.h"
#include "qrmc_mlp.h"

using namespace qrmc;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static qr_status fail(qr_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

static qr_status hipfail(hipError_t e, const char *what) {
    return fail(QR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define QR_HIP(call, what)                                  \
    do {                                                    \
        hipError_t _e = (call);                             \
        if (_e != hipSuccess) return hipfail(_e, what);     \
    } while (0)

extern "C" const char *qr_last_error(void) { return g_last_error.c_str(); }
extern "C" const char *qr_version(void) { return "qrmc 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// basis
// ---------------------------------------------------------------------------
struct qr_basis {
    int32_t d = 0, kind = 0, level = 0;
    int32_t law = QR_LAW_LOGISTIC;       // sampling law nu (qr_law)
    int64_t nrep = 0;
    int32_t max_nnz = 0;
    std::vector<int32_t> trav;           // [nrep][d] traversal order
    std::vector<int32_t> canon;          // [nrep][d] lexicographic order
    std::vector<int32_t> canon_of_trav;  // traversal index -> canonical index
    std::vector<TaskItem> items;         // projection task items
    std::vector<Task> tasks;             // projection tasks of at most task_max nodes
    int32_t task_max = 0;                // proj_shape(d).task_max
    // device copies (one device at a time)
    std::mutex mu;
    int dev = -1;
    int32_t *d_canon_of_trav = nullptr;
    int32_t *d_trav = nullptr;
    TaskItem *d_items = nullptr;
    Task *d_tasks = nullptr;
    int64_t ld() const { return coef_ld(nrep); }
    // Sub-walks (same kind, d' <= d, level' <= level) built on demand for the
    // batched form and owned by this basis.  In a sub-walk, ft maps its
    // traversal index to the parent's, inv the parent's to its own (or -1).
    std::vector<qr_basis *> subs;
    std::vector<int32_t> ft, inv;
    int32_t *d_ft = nullptr, *d_inv = nullptr;
    // Factored layout of the reduced-precision form (built on first use; fac
    // stays null if no split qualifies) and its device copy.
    bool fac_tried = false;
    FactorLayout *fac = nullptr;
    FacDev d_fac{};
    // projection tasks per template (host counts, device lists)
    int32_t fac_ntasks[kFacTemplates] = {};
    FacTask *d_fac_tasks[kFacTemplates] = {};
    // Cosine basis over N^d (qr_build_basis_cos).  Everything above describes
    // its carrier, the Z^d basis of the same kind and level walked at half
    // frequency, whose coefficient rows ("carrier rows", Fourier canonical
    // layout) the kernels use; the caller's rows hold one coefficient per
    // vector of N^d.
    bool cos = false;
    int64_t ncos = 0;
    std::vector<int32_t> cvec;        // [ncos][d] vectors of N^d, lexicographic
    std::vector<int32_t> cos_of_rep;  // carrier representative (canonical) -> vector of N^d
    std::vector<double> rep_scale;    // 2^{(1-n)/2}, n = non-zero coordinates (1 for k = 0)
    std::vector<int32_t> fold_off;    // [ncos + 1]: the representatives of vector c are
    std::vector<int32_t> fold_idx;    //   fold_idx[fold_off[c] .. fold_off[c+1])
    int32_t *d_cos_of_rep = nullptr, *d_fold_off = nullptr, *d_fold_idx = nullptr;
    double *d_rep_scale = nullptr;
    // Tasks of kPassTM nodes for the pass projection of the batched form
    // (built on first use, for the sub-walks that passes walk).
    bool ptasks_built = false;
    std::vector<TaskItem> pitems;
    std::vector<Task> ptasks;
    TaskItem *d_pitems = nullptr;
    Task *d_ptasks = nullptr;
    // coefficients per row: the caller's layout, and the carrier's
    int64_t nf() const { return cos ? ncos : 2 * nrep - 1; }
    int64_t nfc() const { return 2 * nrep - 1; }
    // law code of the kernels: the law, plus the half-frequency flag
    int32_t code() const { return law | (cos ? kLawHalf : 0); }
};

namespace {

constexpr int64_t kMaxReps = (int64_t)1 << 28;

struct Builder {
    SetRule R;
    std::vector<int32_t> cur;
    std::vector<int32_t> &trav;
    std::vector<int64_t> &subtree;
    std::vector<TaskItem> &nodes;
    bool overflow = false;
    int32_t max_depth = 0;

    void push(int depth, int l, int prod) {
        if ((int64_t)subtree.size() >= kMaxReps) {
            overflow = true;
            return;
        }
        trav.insert(trav.end(), cur.begin(), cur.end());
        subtree.push_back(1);
        TaskItem n{};
        n.depth = depth;
        n.last = depth == 0 ? -1 : l;
        n.prod = prod;
        n.full = 1;
        int t = 0;
        for (int c = 0; c < R.d; ++c) {
            if (cur[c] != 0) {
                if (t < kMaxDepthCap) {
                    n.coord[t] = c;
                    n.val[t] = cur[c];
                }
                ++t;
            }
        }
        nodes.push_back(n);
        max_depth = std::max(max_depth, depth);
    }

    // Mirror of the device traversal order (visit<T> in qrmc_kernels.hip).
    void visit(int T, int p, int P) {
        for (int l = p + 1; l < R.d && !overflow; ++l) {
            for (int s = 0; s < (T == 0 ? 1 : 2); ++s) {
                for (int m = 1; rule_ok(R, P, m) && !overflow; ++m) {
                    cur[l] = s ? -m : m;
                    const int P2 = rule_child(R, P, m);
                    const int64_t me = (int64_t)subtree.size();
                    push(T + 1, l, P2);
                    if (l + 1 < R.d && rule_ok(R, P2, 1)) visit(T + 1, l, P2);
                    if (!overflow) subtree[me] = (int64_t)subtree.size() - me;
                }
            }
            cur[l] = 0;
        }
    }
};

// Cut the traversal order into tasks of at most task_max consecutive nodes,
// each a run of items (a node with its whole subtree, or a node alone when
// its subtree exceeds task_max).
void build_tasks(const std::vector<TaskItem> &nodes, const std::vector<int64_t> &subtree, int64_t task_max,
                 std::vector<TaskItem> &items, std::vector<Task> &tasks) {
    const int64_t n = (int64_t)nodes.size();
    Task cur{0, 0, 0, 0};
    auto close = [&]() {
        if (cur.rep_count > 0) {
            cur.item_end = (int32_t)items.size();
            tasks.push_back(cur);
        }
        cur = Task{(int32_t)items.size(), 0, 0, 0};
    };
    int64_t r = 0;
    while (r < n) {
        const int64_t sz = subtree[r];
        if (sz <= task_max - cur.rep_count) {
            if (cur.rep_count == 0) cur.rep_begin = (int32_t)r;
            TaskItem it = nodes[r];
            it.full = 1;
            items.push_back(it);
            cur.rep_count += (int32_t)sz;
            r += sz;
        } else if (sz <= task_max) {
            close();
        } else {
            if (cur.rep_count + 1 > task_max) close();
            if (cur.rep_count == 0) cur.rep_begin = (int32_t)r;
            TaskItem it = nodes[r];
            it.full = 0;
            items.push_back(it);
            cur.rep_count += 1;
            r += 1;
        }
    }
    close();
}

}  // namespace

extern "C" qr_status qr_build_basis(int32_t d, int32_t kind, int32_t level, qr_basis **out) {
    return qr_build_basis_law(d, kind, level, QR_LAW_LOGISTIC, out);
}

extern "C" qr_status qr_build_basis_law(int32_t d, int32_t kind, int32_t level, int32_t law, qr_basis **out) {
    if (!out) return fail(QR_EINVAL, "qr_build_basis: out is NULL");
    *out = nullptr;
    if (d < 1 || d > QR_MAX_D) return fail(QR_EINVAL, "qr_build_basis: d=%d outside [1,%d]", d, QR_MAX_D);
    if (kind < QR_SET_TENSOR || kind > QR_SET_TOTAL)
        return fail(QR_EINVAL, "qr_build_basis: unknown set kind %d", kind);
    if (level < 0 || level > (1 << 20)) return fail(QR_EINVAL, "qr_build_basis: level=%d out of range", level);
    if (level < 1 && (kind == QR_SET_HC_MAX || kind == QR_SET_HC_1P))
        return fail(QR_EINVAL, "qr_build_basis: a hyperbolic cross of level %d is empty", level);
    if (law < QR_LAW_LOGISTIC || law > QR_LAW_CAUCHY)
        return fail(QR_EINVAL, "qr_build_basis: unknown sampling law %d", law);

    qr_basis *b = new (std::nothrow) qr_basis();
    if (!b) return fail(QR_ENOMEM, "qr_build_basis: out of host memory");
    b->d = d;
    b->kind = kind;
    b->level = level;
    b->law = law;
    std::vector<int64_t> subtree;
    std::vector<TaskItem> nodes;
    try {
        Builder B{make_rule(kind, level, d), std::vector<int32_t>(d, 0), b->trav, subtree, nodes};
        B.push(0, 0, 1);  // the zero vector
        B.visit(0, -1, 1);
        if (B.overflow) {
            delete b;
            return fail(QR_ERANGE, "qr_build_basis: more than %lld representatives", (long long)kMaxReps);
        }
        b->nrep = (int64_t)subtree.size();
        subtree[0] = b->nrep;
        b->max_nnz = B.max_depth;

        // canonical (lexicographic) order and the permutation
        std::vector<int64_t> order(b->nrep);
        for (int64_t r = 0; r < b->nrep; ++r) order[r] = r;
        const int32_t *T = b->trav.data();
        std::sort(order.begin(), order.end(), [&](int64_t a, int64_t c) {
            return std::lexicographical_compare(T + a * d, T + a * d + d, T + c * d, T + c * d + d);
        });
        b->canon.resize((size_t)b->nrep * d);
        b->canon_of_trav.resize(b->nrep);
        for (int64_t c = 0; c < b->nrep; ++c) {
            std::memcpy(&b->canon[c * d], T + order[c] * d, sizeof(int32_t) * d);
            b->canon_of_trav[order[c]] = (int32_t)c;
        }
        b->task_max = proj_shape(d).task_max;
        build_tasks(nodes, subtree, b->task_max, b->items, b->tasks);
        // costliest first (nodes plus the complex products that start each
        // item from the root): the waves of a projection block walk
        // consecutive tasks and wait for each other after every batch of paths
        std::vector<int64_t> cost(b->tasks.size());
        for (size_t t = 0; t < b->tasks.size(); ++t) {
            const Task &T = b->tasks[t];
            int64_t c = T.rep_count;
            for (int32_t it = T.item_begin; it < T.item_end; ++it)
                for (int32_t k = 0; k < b->items[it].depth; ++k) c += std::abs(b->items[it].val[k]);
            cost[t] = c;
        }
        std::vector<size_t> by_cost(b->tasks.size());
        for (size_t t = 0; t < by_cost.size(); ++t) by_cost[t] = t;
        std::stable_sort(by_cost.begin(), by_cost.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
        std::vector<Task> sorted(by_cost.size());
        for (size_t t = 0; t < by_cost.size(); ++t) sorted[t] = b->tasks[by_cost[t]];
        b->tasks.swap(sorted);
    } catch (const std::bad_alloc &) {
        delete b;
        return fail(QR_ENOMEM, "qr_build_basis: out of host memory");
    }
    *out = b;
    return QR_OK;
}

// The cosine basis over N^d: its carrier (the Z^d set of the same kind and
// level, whose set rules depend on |k_l| only, so that {|k'| : k' in it} is
// exactly the N^d set) and the maps between the two coefficient layouts.
extern "C" qr_status qr_build_basis_cos(int32_t d, int32_t kind, int32_t level, int32_t law, qr_basis **out) {
    qr_status st = qr_build_basis_law(d, kind, level, law, out);
    if (st) return st;
    qr_basis *b = *out;
    try {
        const int64_t R = b->nrep;
        const int32_t *K = b->canon.data();
        std::vector<int32_t> absv((size_t)R * d);
        for (int64_t i = 0; i < R * d; ++i) absv[i] = std::abs(K[i]);
        std::vector<int64_t> order(R);
        for (int64_t r = 0; r < R; ++r) order[r] = r;
        const int32_t *A = absv.data();
        auto less = [&](int64_t a, int64_t c) {
            return std::lexicographical_compare(A + a * d, A + a * d + d, A + c * d, A + c * d + d);
        };
        std::stable_sort(order.begin(), order.end(), less);
        b->cos_of_rep.assign(R, -1);
        b->rep_scale.assign(R, 1.0);
        b->fold_off.clear();
        b->fold_idx.clear();
        b->cvec.clear();
        for (int64_t q = 0; q < R; ++q) {
            const int64_t r = order[q];
            if (q == 0 || less(order[q - 1], r)) {
                b->fold_off.push_back((int32_t)b->fold_idx.size());
                b->cvec.insert(b->cvec.end(), A + r * d, A + r * d + d);
            }
            int n = 0;
            for (int l = 0; l < d; ++l) n += A[r * d + l] != 0;
            b->cos_of_rep[r] = (int32_t)(b->fold_off.size() - 1);
            // 2^{(1-n)/2}: exact power of two for odd n, sqrt2 times one for even n
            b->rep_scale[r] = n == 0 ? 1.0 : ((n & 1) ? std::ldexp(1.0, (1 - n) / 2) : std::ldexp(M_SQRT2, -n / 2));
            b->fold_idx.push_back((int32_t)r);
        }
        b->ncos = (int64_t)b->fold_off.size();
        b->fold_off.push_back((int32_t)b->fold_idx.size());
        // every vector of N^d in the set has 2^{n-1} representatives (1 for k = 0)
        for (int64_t c = 0; c < b->ncos; ++c) {
            int n = 0;
            for (int l = 0; l < d; ++l) n += b->cvec[c * d + l] != 0;
            const int64_t want = n == 0 ? 1 : ((int64_t)1 << (n - 1));
            if (b->fold_off[c + 1] - b->fold_off[c] != want) {
                qr_basis_free(b);
                *out = nullptr;
                return fail(QR_ENUMERIC, "qr_build_basis_cos: vector %lld has %d representatives, expected %lld",
                            (long long)c, b->fold_off[c + 1] - b->fold_off[c], (long long)want);
            }
        }
    } catch (const std::bad_alloc &) {
        qr_basis_free(b);
        *out = nullptr;
        return fail(QR_ENOMEM, "qr_build_basis_cos: out of host memory");
    }
    b->cos = true;
    return QR_OK;
}

extern "C" qr_status qr_basis_law(const qr_basis *b, int32_t *law) {
    if (!b || !law) return fail(QR_EINVAL, "qr_basis_law: NULL argument");
    *law = b->law;
    return QR_OK;
}

extern "C" qr_status qr_basis_family_of(const qr_basis *b, int32_t *family) {
    if (!b || !family) return fail(QR_EINVAL, "qr_basis_family_of: NULL argument");
    *family = b->cos ? QR_BASIS_COSINE : QR_BASIS_FOURIER;
    return QR_OK;
}

extern "C" qr_status qr_basis_info(const qr_basis *b, int64_t *n_funcs, int64_t *n_reps,
                                   int32_t *max_nnz) {
    if (!b) return fail(QR_EINVAL, "qr_basis_info: basis is NULL");
    if (n_funcs) *n_funcs = b->nf();
    if (n_reps) *n_reps = b->cos ? b->ncos : b->nrep;
    if (max_nnz) *max_nnz = b->max_nnz;
    return QR_OK;
}

extern "C" qr_status qr_basis_indices(const qr_basis *b, int32_t *reps_out) {
    if (!b || !reps_out) return fail(QR_EINVAL, "qr_basis_indices: NULL argument");
    const std::vector<int32_t> &v = b->cos ? b->cvec : b->canon;
    std::memcpy(reps_out, v.data(), sizeof(int32_t) * v.size());
    return QR_OK;
}

static void basis_free_device(qr_basis *b) {
    if (b->dev >= 0) {
        int cur = 0;
        hipGetDevice(&cur);
        hipSetDevice(b->dev);
        hipDeviceSynchronize();
        hipFree(b->d_canon_of_trav);
        hipFree(b->d_trav);
        hipFree(b->d_items);
        hipFree(b->d_tasks);
        hipFree(b->d_ft);
        hipFree(b->d_inv);
        hipFree((void *)b->d_fac.tiles);
        hipFree((void *)b->d_fac.rows);
        hipFree((void *)b->d_fac.cols);
        hipFree((void *)b->d_fac.colnnz);
        hipFree((void *)b->d_fac.ent);
        for (int t = 0; t < kFacTemplates; ++t) hipFree(b->d_fac_tasks[t]);
        hipFree(b->d_pitems);
        hipFree(b->d_ptasks);
        hipFree(b->d_cos_of_rep);
        hipFree(b->d_fold_off);
        hipFree(b->d_fold_idx);
        hipFree(b->d_rep_scale);
        hipSetDevice(cur);
    }
    b->d_pitems = nullptr;
    b->d_ptasks = nullptr;
    b->d_cos_of_rep = nullptr;
    b->d_fold_off = nullptr;
    b->d_fold_idx = nullptr;
    b->d_rep_scale = nullptr;
    b->d_fac = FacDev{};
    for (int t = 0; t < kFacTemplates; ++t) {
        b->d_fac_tasks[t] = nullptr;
        b->fac_ntasks[t] = 0;
    }
    b->d_canon_of_trav = nullptr;
    b->d_trav = nullptr;
    b->d_items = nullptr;
    b->d_tasks = nullptr;
    b->d_ft = nullptr;
    b->d_inv = nullptr;
    b->dev = -1;
}

extern "C" void qr_basis_free(qr_basis *b) {
    if (!b) return;
    for (qr_basis *sb : b->subs) qr_basis_free(sb);
    basis_free_device(b);
    delete b->fac;
    delete b;
}

// The sub-walk of `b` for (d2, level2), built once and kept by `b`.  Its
// traversal is the parent's traversal restricted to the vectors of the
// smaller set (a depth-first pre-order restricted to a set closed under
// taking the parent or previous sibling), which is checked here.
static qr_status sub_basis(qr_basis *b, int32_t d2, int32_t level2, qr_basis **out) {
    std::lock_guard<std::mutex> lock(b->mu);
    for (qr_basis *sb : b->subs)
        if (sb->d == d2 && sb->level == level2) {
            *out = sb;
            return QR_OK;
        }
    qr_basis *sb = nullptr;
    qr_status st = qr_build_basis_law(d2, b->kind, level2, b->law, &sb);
    if (st) return st;
    try {
        sb->ft.resize(sb->nrep);
        sb->inv.assign(b->nrep, -1);
        const int d = b->d;
        int64_t j = 0;
        for (int64_t t = 0; t < sb->nrep; ++t) {
            const int32_t *v = &sb->trav[t * d2];
            for (;; ++j) {
                if (j >= b->nrep) {
                    qr_basis_free(sb);
                    return fail(QR_ENUMERIC, "sub-walk (d=%d, level=%d) is not a subsequence of the basis",
                                d2, level2);
                }
                const int32_t *w = &b->trav[j * d];
                bool eq = std::equal(v, v + d2, w);
                for (int l = d2; l < d && eq; ++l) eq = w[l] == 0;
                if (eq) break;
            }
            sb->ft[t] = (int32_t)j;
            sb->inv[j] = (int32_t)t;
            ++j;
        }
        b->subs.push_back(sb);
    } catch (const std::bad_alloc &) {
        qr_basis_free(sb);
        return fail(QR_ENOMEM, "sub-walk: out of host memory");
    }
    *out = sb;
    return QR_OK;
}

template <class T>
static qr_status upload_vec(T **dst, const std::vector<T> &v) {
    QR_HIP(hipMalloc((void **)dst, sizeof(T) * std::max<size_t>(v.size(), 1)), "hipMalloc(basis tables)");
    if (!v.empty())
        QR_HIP(hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice), "hipMemcpy(basis tables)");
    return QR_OK;
}

// Upload the basis tables to `dev` (current device) once.
static qr_status basis_on_device(qr_basis *b, int dev) {
    std::lock_guard<std::mutex> lock(b->mu);
    if (b->dev == dev) return QR_OK;
    if (b->dev >= 0) basis_free_device(b);
    QR_HIP(hipMalloc(&b->d_canon_of_trav, sizeof(int32_t) * b->nrep), "hipMalloc(basis)");
    QR_HIP(hipMalloc(&b->d_trav, sizeof(int32_t) * b->trav.size()), "hipMalloc(basis)");
    QR_HIP(hipMemcpy(b->d_trav, b->trav.data(), sizeof(int32_t) * b->trav.size(), hipMemcpyHostToDevice),
           "hipMemcpy(basis)");
    QR_HIP(hipMalloc(&b->d_items, sizeof(TaskItem) * b->items.size()), "hipMalloc(basis)");
    QR_HIP(hipMalloc(&b->d_tasks, sizeof(Task) * b->tasks.size()), "hipMalloc(basis)");
    QR_HIP(hipMemcpy(b->d_canon_of_trav, b->canon_of_trav.data(), sizeof(int32_t) * b->nrep,
                     hipMemcpyHostToDevice), "hipMemcpy(basis)");
    QR_HIP(hipMemcpy(b->d_items, b->items.data(), sizeof(TaskItem) * b->items.size(),
                     hipMemcpyHostToDevice), "hipMemcpy(basis)");
    QR_HIP(hipMemcpy(b->d_tasks, b->tasks.data(), sizeof(Task) * b->tasks.size(),
                     hipMemcpyHostToDevice), "hipMemcpy(basis)");
    if (!b->ft.empty()) {
        QR_HIP(hipMalloc(&b->d_ft, sizeof(int32_t) * b->ft.size()), "hipMalloc(basis)");
        QR_HIP(hipMalloc(&b->d_inv, sizeof(int32_t) * b->inv.size()), "hipMalloc(basis)");
        QR_HIP(hipMemcpy(b->d_ft, b->ft.data(), sizeof(int32_t) * b->ft.size(), hipMemcpyHostToDevice),
               "hipMemcpy(basis)");
        QR_HIP(hipMemcpy(b->d_inv, b->inv.data(), sizeof(int32_t) * b->inv.size(), hipMemcpyHostToDevice),
               "hipMemcpy(basis)");
    }
    if (b->cos) {
        qr_status st;
        if ((st = upload_vec(&b->d_cos_of_rep, b->cos_of_rep))) return st;
        if ((st = upload_vec(&b->d_fold_off, b->fold_off))) return st;
        if ((st = upload_vec(&b->d_fold_idx, b->fold_idx))) return st;
        if ((st = upload_vec(&b->d_rep_scale, b->rep_scale))) return st;
    }
    b->dev = dev;
    return QR_OK;
}

// The pass-projection tasks of a basis on its device (host lists built once
// by walking the set again; the basis must be resident on the device).
static qr_status basis_pass_tasks_on_device(qr_basis *b) {
    std::lock_guard<std::mutex> lock(b->mu);
    if (!b->ptasks_built) {
        try {
            std::vector<int32_t> trav;
            std::vector<int64_t> subtree;
            std::vector<TaskItem> nodes;
            Builder B{make_rule(b->kind, b->level, b->d), std::vector<int32_t>(b->d, 0), trav, subtree, nodes};
            B.push(0, 0, 1);
            B.visit(0, -1, 1);
            if (B.overflow || (int64_t)subtree.size() != b->nrep)
                return fail(QR_ENUMERIC, "pass tasks: the walk of the set changed size");
            subtree[0] = b->nrep;
            build_tasks(nodes, subtree, kPassTM, b->pitems, b->ptasks);
        } catch (const std::bad_alloc &) {
            return fail(QR_ENOMEM, "pass tasks: out of host memory");
        }
        b->ptasks_built = true;
    }
    if (!b->d_ptasks) {
        qr_status st;
        if ((st = upload_vec(&b->d_pitems, b->pitems))) return st;
        if ((st = upload_vec(&b->d_ptasks, b->ptasks))) return st;
    }
    return QR_OK;
}

// The factored layout of a basis (host), built once; false if none qualifies.
static bool basis_factored(qr_basis *b) {
    std::lock_guard<std::mutex> lock(b->mu);
    if (!b->fac_tried) {
        b->fac_tried = true;
        FactorLayout *L = new (std::nothrow) FactorLayout();
        if (L && build_factor_layout(b->d, b->kind, b->level, b->canon.data(), b->nrep, kFacMaxNkb, L))
            b->fac = L;
        else
            delete L;
    }
    return b->fac != nullptr;
}

// Device copy of the factored layout (the basis must be on `dev` already).
static qr_status basis_factored_on_device(qr_basis *b) {
    std::lock_guard<std::mutex> lock(b->mu);
    if (!b->fac) return fail(QR_ENOTSUP, "basis has no factored layout");
    if (b->d_fac.tiles) return QR_OK;
    const FactorLayout &L = *b->fac;
    FacDev F{};
    qr_status st;
    if ((st = upload_vec((FacTile **)&F.tiles, L.tiles))) return st;
    if ((st = upload_vec((FacCode **)&F.rows, L.rows))) return st;
    if ((st = upload_vec((FacCode **)&F.cols, L.cols))) return st;
    if ((st = upload_vec((int32_t **)&F.colnnz, L.colnnz))) return st;
    if ((st = upload_vec((int32_t **)&F.ent, L.ent))) return st;
    F.nrt = L.nrt;
    F.nkb = L.nkb;
    F.TS = L.TS;
    F.dA = L.dA;
    F.d = L.d;
    F.nblocks = L.nblocks;
    std::vector<FacTask> tasks[kFacTemplates];
    build_fac_tasks(L, tasks);
    for (int t = 0; t < kFacTemplates; ++t) {
        if ((st = upload_vec(&b->d_fac_tasks[t], tasks[t]))) return st;
        b->fac_ntasks[t] = (int32_t)tasks[t].size();
    }
    b->d_fac = F;
    return QR_OK;
}

extern "C" qr_status qr_basis_factored(const qr_basis *bc, int32_t *split, int32_t *n_row_tiles,
                                       int32_t *n_kblocks, int64_t *n_blocks) {
    qr_basis *b = const_cast<qr_basis *>(bc);
    if (!b) return fail(QR_EINVAL, "qr_basis_factored: basis is NULL");
    if (!basis_factored(b)) return fail(QR_ENOTSUP, "qr_basis_factored: no split of this index set qualifies");
    if (split) *split = b->fac->dA;
    if (n_row_tiles) *n_row_tiles = b->fac->nrt;
    if (n_kblocks) *n_kblocks = b->fac->nkb;
    if (n_blocks) *n_blocks = b->fac->nblocks;
    return QR_OK;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
namespace {
struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Timed {
    int which;
    hipEvent_t a, b;
};
}  // namespace

// streams of a batched solve (the caller's and three of the context's)
constexpr int kBatchStreams = 4;

struct qr_ctx {
    int dev = 0;
    hipStream_t last = nullptr;
    DevProblem *d_prob = nullptr;
    DevProblem h_prob{};
    bool prob_valid = false;
    Buf S, u, alpha_int, partial, row, alpha_b, tiles, xstate, fcoef, fpartial;
    // cosine basis: the carrier table [N][2R-1] and one carrier row
    Buf calpha, crow;
    // Z regression: the sums' first terms [M], responses [8][M], cloud sizes [8]
    Buf zf0, zresp, zm, zx0, zy0;
    // evaluation split across blocks: phase factors [d][n], group sums [groups][n]
    Buf ete, etp;
    // batched solve: side streams (default priority) with their own responses,
    // phase factors and partial sums, so that independent passes overlap
    hipStream_t bstream[kBatchStreams - 1] = {};
    Buf bS[kBatchStreams - 1], bu[kBatchStreams - 1], bpart[kBatchStreams - 1];
    hipEvent_t bfork = nullptr, bjoin[kBatchStreams - 1] = {};
    int32_t prec_kernel = QR_PREC_KERNEL_AUTO;
    // surrogate network workspace: activations of up to kMlpChunk rows
    Buf mf, mz1, mh1, mz2, mh2, mdz, mdh, my, mdy, mpart, mwork, mcwork;
    // learned solve: cloud state, per-step source term, expansion values,
    // surrogate parameters per time index, Adam state, training pairs
    Buf lx, lh, ly, lparams, lgrad, lm, lv, ltx, ltt, ltf, lff, lhx, lht, lhf, lhy;
    DevBatch *d_batch = nullptr;
    // largest time index whose coefficients came out non-finite since the
    // last read (-1: none), raised by the reduction kernels
    int32_t *d_bad = nullptr;
    bool timing = false;
    // workspace held by the buffers above, and the cap set by
    // qr_ctx_set_mem_limit (0: none)
    int64_t held = 0, mem_limit = 0;
    std::vector<Timed> pending;
    std::vector<hipEvent_t> pool;
    double ms[4] = {0, 0, 0, 0};
    int64_t launches[4] = {0, 0, 0, 0};
};

static qr_status ensure(qr_ctx *c, Buf &b, size_t bytes, const char *what) {
    if (b.bytes >= bytes) return QR_OK;
    if (c->mem_limit > 0 && c->held - (int64_t)b.bytes + (int64_t)bytes > c->mem_limit)
        return fail(QR_ENOMEM, "workspace %s: %zu bytes would take the context's workspace to %lld bytes, "
                               "over its limit of %lld", what, bytes,
                    (long long)(c->held - (int64_t)b.bytes + (int64_t)bytes), (long long)c->mem_limit);
    QR_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (b.p) hipFree(b.p);
    c->held -= (int64_t)b.bytes;
    b.p = nullptr;
    b.bytes = 0;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        hipGetLastError();
        return fail(QR_ENOMEM, "workspace %s: cannot allocate %zu bytes", what, bytes);
    }
    b.bytes = bytes;
    c->held += (int64_t)bytes;
    return QR_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free evaluation (qr_eval_noalloc): the caller's
// coefficient row converted to the kernels' layout (double2, traversal order,
// zero read-ahead chunks).  Each GPU holds its own copy of the array for the
// life of the process.  Host code never passes `scratch` itself to a kernel
// (on the host the name is a stand-in, not a device address): the device
// address is looked up once per device, with that device current, and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double2 scratch[QR_NOALLOC_ROW_MAX];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double2 *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Look up the device address of `scratch` on `dev` (the current device).
static qr_status scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(QR_ENOTSUP, "device %d: scratch table holds %d devices", dev,
                                                   kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return QR_OK;
    void *ptr = nullptr;
    QR_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(QR_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = (double2 *)ptr;
    return QR_OK;
}

static double2 *scratch_of(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
}

extern "C" qr_status qr_ctx_create(int32_t device, qr_ctx **out) {
    if (!out) return fail(QR_EINVAL, "qr_ctx_create: out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(QR_EDEVICE, "qr_ctx_create: no HIP device available");
    if (device < 0 || device >= n) return fail(QR_EINVAL, "qr_ctx_create: device %d of %d", device, n);
    QR_HIP(hipSetDevice(device), "hipSetDevice");
    qr_status sst = scratch_init(device);
    if (sst) return sst;
    qr_ctx *c = new (std::nothrow) qr_ctx();
    if (!c) return fail(QR_ENOMEM, "qr_ctx_create: out of host memory");
    c->dev = device;
    e = hipMalloc(&c->d_prob, sizeof(DevProblem));
    if (e != hipSuccess) {
        delete c;
        return hipfail(e, "hipMalloc(problem)");
    }
    e = hipMalloc(&c->d_bad, sizeof(int32_t));
    if (e == hipSuccess) e = launch_set_flag(c->d_bad, -1, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        hipFree(c->d_prob);
        if (c->d_bad) hipFree(c->d_bad);
        delete c;
        return hipfail(e, "hipMalloc(numeric flag)");
    }
    *out = c;
    return QR_OK;
}

extern "C" void qr_ctx_destroy(qr_ctx *c) {
    if (!c) return;
    hipSetDevice(c->dev);
    hipDeviceSynchronize();
    for (Buf *b : {&c->S, &c->u, &c->alpha_int, &c->partial, &c->row, &c->alpha_b, &c->tiles, &c->xstate, &c->fcoef,
                   &c->fpartial, &c->calpha, &c->crow, &c->zf0, &c->zresp, &c->zm, &c->zx0, &c->zy0, &c->ete, &c->etp, &c->mf, &c->mz1, &c->mh1, &c->mz2, &c->mh2, &c->mdz, &c->mdh, &c->my, &c->mdy, &c->mpart, &c->mwork,
                   &c->mcwork, &c->lx, &c->lh, &c->ly, &c->lparams, &c->lgrad, &c->lm, &c->lv, &c->ltx, &c->ltt,
                   &c->ltf, &c->lff, &c->lhx, &c->lht, &c->lhf, &c->lhy})
        if (b->p) hipFree(b->p);
    for (int k = 0; k < kBatchStreams - 1; ++k) {
        for (Buf *b : {&c->bS[k], &c->bu[k], &c->bpart[k]})
            if (b->p) hipFree(b->p);
        if (c->bstream[k]) hipStreamDestroy(c->bstream[k]);
        if (c->bjoin[k]) hipEventDestroy(c->bjoin[k]);
    }
    if (c->bfork) hipEventDestroy(c->bfork);
    hipFree(c->d_prob);
    hipFree(c->d_bad);
    if (c->d_batch) hipFree(c->d_batch);
    for (auto &t : c->pending) {
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    for (auto e : c->pool) hipEventDestroy(e);
    delete c;
}

extern "C" qr_status qr_ctx_set_prec_kernel(qr_ctx *c, int32_t kind) {
    if (!c) return fail(QR_EINVAL, "qr_ctx_set_prec_kernel: ctx is NULL");
    if (kind < QR_PREC_KERNEL_AUTO || kind > QR_PREC_KERNEL_FACTORED)
        return fail(QR_EINVAL, "qr_ctx_set_prec_kernel: unknown kernel choice %d", kind);
    c->prec_kernel = kind;
    return QR_OK;
}

extern "C" qr_status qr_ctx_set_mem_limit(qr_ctx *c, int64_t bytes) {
    if (!c) return fail(QR_EINVAL, "qr_ctx_set_mem_limit: ctx is NULL");
    if (bytes < 0) return fail(QR_EINVAL, "qr_ctx_set_mem_limit: negative limit %lld", (long long)bytes);
    c->mem_limit = bytes;
    return QR_OK;
}

extern "C" qr_status qr_ctx_mem_held(const qr_ctx *c, int64_t *bytes) {
    if (!c || !bytes) return fail(QR_EINVAL, "qr_ctx_mem_held: NULL argument");
    *bytes = c->held;
    return QR_OK;
}

extern "C" qr_status qr_ctx_set_timing(qr_ctx *c, int32_t enable) {
    if (!c) return fail(QR_EINVAL, "qr_ctx_set_timing: ctx is NULL");
    c->timing = enable != 0;
    return QR_OK;
}

static void harvest(qr_ctx *c) {
    for (auto &t : c->pending) {
        hipEventSynchronize(t.b);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            c->ms[t.which] += ms;
            c->launches[t.which] += 1;
        }
        c->pool.push_back(t.a);
        c->pool.push_back(t.b);
    }
    c->pending.clear();
}

extern "C" qr_status qr_ctx_kernel_time(qr_ctx *c, int32_t which, double *ms, int64_t *launches) {
    if (!c || which < 0 || which > 3) return fail(QR_EINVAL, "qr_ctx_kernel_time: bad argument");
    hipSetDevice(c->dev);
    harvest(c);
    if (ms) *ms = c->ms[which];
    if (launches) *launches = c->launches[which];
    return QR_OK;
}

extern "C" qr_status qr_ctx_reset_timing(qr_ctx *c) {
    if (!c) return fail(QR_EINVAL, "qr_ctx_reset_timing: ctx is NULL");
    hipSetDevice(c->dev);
    harvest(c);
    for (int k = 0; k < 4; ++k) {
        c->ms[k] = 0;
        c->launches[k] = 0;
    }
    return QR_OK;
}

static hipEvent_t take_event(qr_ctx *c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
}

// Launch wrapper: records events around the launch when timing is on.
template <class F>
static qr_status timed(qr_ctx *c, int which, hipStream_t s, const char *what, F &&launch) {
    hipEvent_t a = nullptr, b = nullptr;
    if (c->timing) {
        a = take_event(c);
        b = take_event(c);
        hipEventRecord(a, s);
    }
    hipError_t e = launch();
    if (e != hipSuccess) return hipfail(e, what);
    if (c->timing) {
        hipEventRecord(b, s);
        c->pending.push_back(Timed{which, a, b});
    }
    return QR_OK;
}

// ---------------------------------------------------------------------------
// validation and problem upload
// ---------------------------------------------------------------------------
// a problem whose drift or diffusion depends on the state (b2 or v non-zero)
static bool state_dependent(const qr_problem *p) {
    for (int l = 0; l < p->d; ++l)
        if (p->b2[l] != 0.0 || p->sigma_v[l] != 0.0) return true;
    return false;
}

static qr_status check_problem(const qr_problem *p, const qr_basis *b) {
    if (!p) return fail(QR_EINVAL, "problem is NULL");
    if (p->d < 1 || p->d > QR_MAX_D) return fail(QR_EINVAL, "problem: d=%d outside [1,%d]", p->d, QR_MAX_D);
    if (p->nbm < 1 || p->nbm > QR_MAX_D)
        return fail(QR_EINVAL, "problem: nbm=%d outside [1,%d]", p->nbm, QR_MAX_D);
    if (p->N < 1 || p->N > QR_MAX_N) return fail(QR_EINVAL, "problem: N=%d outside [1,%d]", p->N, QR_MAX_N);
    if (p->driver < QR_F_LINEAR || p->driver > QR_F_PAPER)
        return fail(QR_EINVAL, "problem: unknown driver %d", p->driver);
    if (!std::isfinite(p->sol_B)) return fail(QR_EINVAL, "problem: offset B not finite");
    if (!(p->clamp > 0.0)) return fail(QR_EINVAL, "problem: clamp must be > 0 (INFINITY for none)");
    if (!(p->damping_q >= 0.0 && p->damping_q <= QR_MAX_DAMPING))
        return fail(QR_EINVAL, "problem: damping exponent q=%g outside [0,%g]", p->damping_q, (double)QR_MAX_DAMPING);
    for (int j = 0; j < p->N; ++j)
        if (!(p->t[j + 1] > p->t[j]) || !std::isfinite(p->t[j + 1]) || !std::isfinite(p->t[j]))
            return fail(QR_EINVAL, "problem: time grid not strictly increasing at j=%d", j);
    for (int v = 0; v < p->d * p->nbm; ++v)
        if (!std::isfinite(p->sigma[v])) return fail(QR_EINVAL, "problem: sigma not finite");
    for (int l = 0; l < p->d; ++l) {
        if (!std::isfinite(p->b2[l])) return fail(QR_EINVAL, "problem: b2 not finite");
        if (!(std::fabs(p->sigma_v[l]) < 1.0))
            return fail(QR_EINVAL, "problem: |sigma_v[%d]| = %g must be < 1 (uniform ellipticity)", l, p->sigma_v[l]);
    }
    if (!std::isfinite(p->sigma_omega)) return fail(QR_EINVAL, "problem: sigma_omega not finite");
    if (b && b->d != p->d) return fail(QR_EINVAL, "basis dimension %d != problem dimension %d", b->d, p->d);
    return QR_OK;
}

static qr_status check_basis_device(const qr_basis *b) {
    if (!b) return fail(QR_EINVAL, "basis is NULL");
    if (b->max_nnz > kMaxDepthCap)
        return fail(QR_ENOTSUP, "basis has vectors with %d non-zero coordinates (device limit %d)",
                    b->max_nnz, kMaxDepthCap);
    if (2 * b->nrep - 1 > ((int64_t)1 << 31) - 1) return fail(QR_ERANGE, "basis too large");
    return QR_OK;
}

static int depth_cap(int32_t max_nnz) {
    return max_nnz <= 2 ? 2 : (max_nnz <= 4 ? 4 : (max_nnz <= 6 ? 6 : 8));
}

static int dim_bucket(int32_t d, int32_t nbm) {
    const int m = std::max(d, nbm);
    return m <= 4 ? 4 : (m <= 8 ? 8 : 16);
}

// The device copy of the problem also carries the sampling law of the basis
// used with it, so the path kernels read it from memory per step instead of
// keeping it in a register across the basis traversal.
static DevProblem make_dev_problem(const qr_problem *p, int32_t law) {
    DevProblem h{};
    h.d = p->d;
    h.nbm = p->nbm;
    h.N = p->N;
    h.driver = p->driver;
    h.nu = law;
    h.f_a = p->f_a;
    h.clamp = p->clamp;
    h.T = p->t[p->N];
    for (int j = 0; j <= p->N; ++j) h.t[j] = p->t[j];
    for (int l = 0; l < p->d; ++l) {
        h.b0[l] = p->b0[l];
        h.b1[l] = p->b1[l];
        h.sol_w[l] = p->sol_w[l];
        for (int k = 0; k < p->nbm; ++k) h.sigma[l * p->nbm + k] = p->sigma[l * p->nbm + k];
    }
    h.sol_A = p->sol_A;
    h.sol_c = p->sol_c;
    h.sol_p = p->sol_p;
    h.sol_B = p->sol_B;
    h.dq = p->damping_q;
    h.sdep = state_dependent(p) ? 1 : 0;
    for (int l = 0; l < p->d; ++l) {
        h.b2[l] = p->b2[l];
        h.sv[l] = p->sigma_v[l];
    }
    h.somega = p->sigma_omega;
    double sw2 = 0.0;
    for (int k = 0; k < p->nbm; ++k) {
        double v = 0.0;
        for (int l = 0; l < p->d; ++l) v += p->sigma[l * p->nbm + k] * p->sol_w[l];
        h.sw[k] = v;
        sw2 += v * v;
    }
    h.sw2 = sw2;
    return h;
}

static qr_status upload_problem(qr_ctx *c, const qr_problem *p, int32_t law, hipStream_t s) {
    const DevProblem h = make_dev_problem(p, law);
    if (c->prob_valid && std::memcmp(&h, &c->h_prob, sizeof h) == 0) return QR_OK;
    // the previous problem may still be read by queued kernels
    QR_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (c->last && c->last != s) QR_HIP(hipStreamSynchronize(c->last), "hipStreamSynchronize");
    QR_HIP(hipMemcpy(c->d_prob, &h, sizeof h, hipMemcpyHostToDevice), "hipMemcpy(problem)");
    c->h_prob = h;
    c->prob_valid = true;
    return QR_OK;
}

static qr_status begin(qr_ctx *c, void *stream) {
    if (!c) return fail(QR_EINVAL, "ctx is NULL");
    QR_HIP(hipSetDevice(c->dev), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    if (c->last && c->last != s) QR_HIP(hipStreamSynchronize(c->last), "hipStreamSynchronize");
    c->last = s;
    return QR_OK;
}

// The numeric flag: cleared on the stream, read after the stream completes.
static qr_status numeric_clear(qr_ctx *c, hipStream_t s) {
    QR_HIP(launch_set_flag(c->d_bad, -1, s), "set_flag_kernel");
    return QR_OK;
}

static qr_status numeric_read(qr_ctx *c, hipStream_t s, int32_t *step) {
    int32_t h = -1;
    QR_HIP(hipMemcpyAsync(&h, c->d_bad, sizeof h, hipMemcpyDeviceToHost, s), "hipMemcpyAsync(numeric flag)");
    QR_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (step) *step = h;
    if (h < 0) return QR_OK;
    qr_status st = numeric_clear(c, s);
    if (st) return st;
    return fail(QR_ENUMERIC, "non-finite coefficient at time index %d (latest in the backward order)", h);
}

extern "C" qr_status qr_ctx_numeric_status(qr_ctx *c, int32_t *step) {
    if (!c) return fail(QR_EINVAL, "qr_ctx_numeric_status: ctx is NULL");
    QR_HIP(hipSetDevice(c->dev), "hipSetDevice");
    return numeric_read(c, c->last, step);
}

// ---------------------------------------------------------------------------
// step pieces
// ---------------------------------------------------------------------------
#ifndef QRMC_PROJ_BLOCKS
#define QRMC_PROJ_BLOCKS 4096
#endif
// blocks a projection aims at (many per CU, so that the last round is short)
constexpr int64_t kProjBlocks = QRMC_PROJ_BLOCKS;

static void split_plan(const qr_basis *b, int64_t M, int32_t *nsplit, int64_t *pps) {
    const ProjShape sh = proj_shape(b->d);
    // blocks are (group of sh.waves tasks) x slice; a slice is walked 64 P paths at a time
    const int64_t ngroups = std::max<int64_t>(1, ((int64_t)b->tasks.size() + sh.waves - 1) / sh.waves);
    const int64_t group = (int64_t)64 * sh.P;
    int64_t want = (kProjBlocks + ngroups - 1) / ngroups;
    const int64_t maxs = std::max<int64_t>(1, (M + 4 * group - 1) / (4 * group));
    want = std::max<int64_t>(1, std::min(want, maxs));
    int64_t per = (M + want - 1) / want;
    per = (per + group - 1) / group * group;
    *pps = per;
    *nsplit = (int32_t)((M + per - 1) / per);
}

// step: the time index of the row (its non-finite coefficients are
// recorded), or -1 for a projection that is not a step of the method
static qr_status project_and_reduce(qr_ctx *c, const qr_basis *b, const double2 *u, const double *S,
                                    int64_t M, double2 *alpha_int_row, double *alpha_row, int32_t step,
                                    hipStream_t s) {
    int32_t nsplit;
    int64_t pps;
    split_plan(b, M, &nsplit, &pps);
    qr_status st = ensure(c, c->partial, sizeof(double2) * (size_t)nsplit * b->nrep, "partial");
    if (st) return st;
    const int cap = depth_cap(b->max_nnz);
    double2 *partial = (double2 *)c->partial.p;
    st = timed(c, 1, s, "project_kernel", [&] {
        return launch_project(cap, make_walk(b->kind, b->level, b->d, b->code()), u, M, S, M, pps,
                              (int32_t)b->tasks.size(), nsplit, b->d_tasks, b->d_items, b->task_max,
                              partial, b->nrep, s);
    });
    if (st) return st;
    return timed(c, 2, s, "reduce_kernel", [&] {
        return launch_reduce(partial, nsplit, b->nrep, (double)M, alpha_int_row, alpha_row,
                             b->d_canon_of_trav, step >= 0 ? c->d_bad : nullptr, step, s);
    });
}

static qr_status run_path(qr_ctx *c, const qr_problem *p, const qr_basis *b, int32_t i, int64_t M,
                          uint64_t seed, const double2 *alpha_int, double *S, double2 *u, double *x0,
                          hipStream_t s, double *f0 = nullptr) {
    const bool grad = p->driver == QR_F_ZRAT;
    const int64_t ldx = path_state_ld(M, grad);
    // rows 0..d-1: X_j; row d: u(t_j, X_j) for the Sec. 5 driver
    qr_status st = ensure(c, c->xstate, sizeof(double) * (size_t)(p->d + 1) * ldx, "path state");
    if (st) return st;
    PathArgs a{c->d_prob, make_walk(b->kind, b->level, b->d, b->code()), i, M, seed, alpha_int, b->ld(), S, u, x0,
               (double *)c->xstate.p, ldx, f0};
    return timed(c, 0, s, "path_kernel", [&] {
        return launch_path(dim_bucket(p->d, p->nbm), depth_cap(b->max_nnz), p->driver == QR_F_ZRAT,
                           state_dependent(p) ? 2 : (p->damping_q != 0.0 ? 1 : 0), a, s);
    });
}

static qr_status check_M(int64_t M) {
    if (M < 1 || M > (int64_t)INT32_MAX) return fail(QR_EINVAL, "M=%lld outside [1, 2^31-1]", (long long)M);
    return QR_OK;
}

static qr_status prepare(qr_ctx *c, const qr_problem *p, qr_basis *b, int64_t M, void *stream) {
    qr_status st = begin(c, stream);
    if (st) return st;
    if ((st = check_problem(p, b))) return st;
    if ((st = check_basis_device(b))) return st;
    if ((st = check_M(M))) return st;
    if ((st = basis_on_device(b, c->dev))) return st;
    if ((st = upload_problem(c, p, b->code(), (hipStream_t)stream))) return st;
    if ((st = ensure(c, c->S, sizeof(double) * (size_t)M, "S"))) return st;
    if ((st = ensure(c, c->u, sizeof(double2) * (size_t)M * p->d, "phase factors"))) return st;
    if ((st = ensure(c, c->alpha_int, sizeof(double2) * (size_t)p->N * b->ld(), "alpha"))) return st;
    // zero the padding columns read by the batched coefficient loads
    QR_HIP(launch_pad(p->N, b->nrep, b->ld(), (double2 *)c->alpha_int.p, (hipStream_t)stream), "pad_kernel");
    return QR_OK;
}

// The coefficient table the kernels take: the caller's for a Fourier basis;
// for a cosine basis the context's carrier table, rows [r0, N) expanded from
// the caller's cosine rows.
static qr_status carrier_in(qr_ctx *c, const qr_basis *b, const double *alpha, int32_t r0, int32_t N, double **A,
                            hipStream_t s) {
    if (!b->cos) {
        *A = const_cast<double *>(alpha);
        return QR_OK;
    }
    qr_status st = ensure(c, c->calpha, sizeof(double) * (size_t)N * b->nfc(), "carrier coefficients");
    if (st) return st;
    *A = (double *)c->calpha.p;
    if (r0 >= N) return QR_OK;
    return timed(c, 3, s, "cos_expand_kernel", [&] {
        return launch_cos_expand(alpha, r0, N - r0, b->ncos, b->nrep, b->d_cos_of_rep, b->d_rep_scale, *A, s);
    });
}

// After a step has written carrier row i of A: the caller's cosine row i by
// folding it, then carrier row i (and, if alpha_int is given, the kernels'
// row i) replaced by the expansion of that cosine row, which is what the
// later steps evaluate.
static qr_status carrier_out(qr_ctx *c, const qr_basis *b, double *A, double *alpha, int32_t i, double2 *alpha_int,
                             hipStream_t s) {
    if (!b->cos) return QR_OK;
    double *arow = A + (int64_t)i * b->nfc();
    double *crow = alpha + (int64_t)i * b->ncos;
    qr_status st = timed(c, 3, s, "cos_fold_kernel", [&] {
        return launch_cos_fold(arow, b->ncos, b->d_fold_off, b->d_fold_idx, b->d_rep_scale, crow, s);
    });
    if (st) return st;
    st = timed(c, 3, s, "cos_expand_kernel", [&] {
        return launch_cos_expand(alpha, i, 1, b->ncos, b->nrep, b->d_cos_of_rep, b->d_rep_scale, A, s);
    });
    if (st || !alpha_int) return st;
    return timed(c, 3, s, "gather_kernel", [&] {
        return launch_gather(A, i, 1, b->nrep, b->ld(), b->nfc(), b->d_canon_of_trav, alpha_int, s);
    });
}

extern "C" qr_status qr_backward_step(qr_ctx *c, const qr_problem *p, const qr_basis *bc, int32_t i,
                                      int64_t M, uint64_t seed, double *alpha, void *stream) {
    qr_basis *b = const_cast<qr_basis *>(bc);
    qr_status st = prepare(c, p, b, M, stream);
    if (st) return st;
    if (!alpha) return fail(QR_EINVAL, "qr_backward_step: alpha is NULL");
    if (i < 0 || i >= p->N) return fail(QR_EINVAL, "qr_backward_step: i=%d outside [0,%d)", i, p->N);
    hipStream_t s = (hipStream_t)stream;
    double2 *ai = (double2 *)c->alpha_int.p;
    const int64_t nf = b->nfc();
    double *A;
    if ((st = carrier_in(c, b, alpha, i + 1, p->N, &A, s))) return st;
    st = timed(c, 3, s, "gather_kernel", [&] {
        return launch_gather(A, i + 1, p->N - 1 - i, b->nrep, b->ld(), nf, b->d_canon_of_trav, ai, s);
    });
    if (st) return st;
    double *S = (double *)c->S.p;
    double2 *u = (double2 *)c->u.p;
    if ((st = run_path(c, p, b, i, M, seed, ai, S, u, nullptr, s))) return st;
    if ((st = project_and_reduce(c, b, u, S, M, ai + (int64_t)i * b->ld(), A + (int64_t)i * nf, i, s))) return st;
    return carrier_out(c, b, A, alpha, i, nullptr, s);
}

// The backward induction i = i0, ..., 0 in FP64, rows i0+1..N-1 of alpha given.
static qr_status solve_f64_from(qr_ctx *c, const qr_problem *p, qr_basis *b, int32_t i0, int64_t M, uint64_t seed,
                                double *alpha, void *stream) {
    qr_status st = prepare(c, p, b, M, stream);
    if (st) return st;
    if (!alpha) return fail(QR_EINVAL, "qr_solve: alpha is NULL");
    if (i0 < 0 || i0 >= p->N) return fail(QR_EINVAL, "qr_solve_from: i_start=%d outside [0,%d)", i0, p->N);
    hipStream_t s = (hipStream_t)stream;
    double2 *ai = (double2 *)c->alpha_int.p;
    const int64_t nf = b->nfc();
    double *S = (double *)c->S.p;
    double2 *u = (double2 *)c->u.p;
    double *A;
    if ((st = carrier_in(c, b, alpha, i0 + 1, p->N, &A, s))) return st;
    st = timed(c, 3, s, "gather_kernel", [&] {
        return launch_gather(A, i0 + 1, p->N - 1 - i0, b->nrep, b->ld(), nf, b->d_canon_of_trav, ai, s);
    });
    if (st) return st;
    if ((st = numeric_clear(c, s))) return st;
    for (int32_t i = i0; i >= 0; --i) {
        if ((st = run_path(c, p, b, i, M, seed, ai, S, u, nullptr, s))) return st;
        if ((st = project_and_reduce(c, b, u, S, M, ai + (int64_t)i * b->ld(), A + (int64_t)i * nf, i, s)))
            return st;
        if ((st = carrier_out(c, b, A, alpha, i, ai, s))) return st;
    }
    return numeric_read(c, s, nullptr);
}

extern "C" qr_status qr_solve(qr_ctx *c, const qr_problem *p, const qr_basis *bc, int64_t M,
                              uint64_t seed, double *alpha, void *stream) {
    if (!p) return fail(QR_EINVAL, "problem is NULL");
    return solve_f64_from(c, p, const_cast<qr_basis *>(bc), p->N - 1, M, seed, alpha, stream);
}

namespace {
void pass_split_plan(const qr_basis *w, int64_t M, int32_t *nsplit, int64_t *pps);
}  // namespace

// Z rows of time index i from the step just run: its responses S, first
// terms and first-step values f0 in the context, the start points' phase
// factors u (and, for the one-step scheme, the start points X_i in zx0);
// nbm projections, kBatchRT at a time on the basis's pass tasks.
static qr_status project_z(qr_ctx *c, const qr_problem *p, qr_basis *b, int32_t i, int64_t M, uint64_t seed,
                           int32_t scheme, double *alpha_z, hipStream_t s) {
    qr_status st;
    if ((st = basis_pass_tasks_on_device(b))) return st;
    int32_t nsplit;
    int64_t pps;
    pass_split_plan(b, M, &nsplit, &pps);
    if ((st = ensure(c, c->zresp, sizeof(double) * (size_t)M * kBatchRT, "Z responses"))) return st;
    if ((st = ensure(c, c->zm, sizeof(int64_t) * kBatchRT, "Z cloud sizes"))) return st;
    if ((st = ensure(c, c->partial, sizeof(double2) * (size_t)nsplit * b->nrep * kBatchRT, "partial"))) return st;
    QR_HIP(launch_fill_i64((int64_t *)c->zm.p, kBatchRT, M, s), "fill_kernel");
    const int64_t nf = b->nfc();
    double *zr = (double *)c->zresp.p;
    double2 *partial = (double2 *)c->partial.p;
    const double *y0 = nullptr;
    if (scheme == QR_Z_ONESTEP) {
        // ybar_{i+1} (g for i = N-1) at the start points
        double *zy0 = (double *)c->zy0.p;
        const double *x0 = (const double *)c->zx0.p;
        if (i + 1 < p->N) {
            const double2 *row = (const double2 *)c->alpha_int.p + (int64_t)(i + 1) * b->ld();
            st = timed(c, 0, s, "eval_kernel", [&] {
                return launch_eval(depth_cap(b->max_nnz), false, make_walk(b->kind, b->level, b->d, b->code()), row,
                                   x0, M, zy0, nullptr, s);
            });
            if (st) return st;
        } else {
            QR_HIP(launch_g_points(dim_bucket(p->d, p->nbm), c->d_prob, x0, M, zy0, s), "g_points_kernel");
        }
        y0 = zy0;
    }
    for (int32_t k0 = 0; k0 < p->nbm; k0 += kBatchRT) {
        const int32_t nk = std::min<int32_t>(kBatchRT, p->nbm - k0);
        QR_HIP(launch_z_responses(c->d_prob, seed, i, M, k0, nk, (const double *)c->S.p, (const double *)c->zf0.p, y0,
                                  zr, s),
               "z_responses_kernel");
        st = timed(c, 1, s, "project_pass_kernel", [&] {
            return launch_project_pass(depth_cap(b->max_nnz), make_walk(b->kind, b->level, b->d, b->code()),
                                       (const double2 *)c->u.p, M, zr, M, (const int64_t *)c->zm.p, pps,
                                       (int32_t)b->ptasks.size(), nsplit, b->d_ptasks, b->d_pitems, partial, b->nrep,
                                       s);
        });
        if (st) return st;
        for (int32_t r = 0; r < nk; ++r) {
            st = timed(c, 2, s, "reduce_slot_kernel", [&] {
                return launch_reduce_slot(partial, nsplit, b->nrep, kBatchRT, r, (double)M, b->d_canon_of_trav,
                                          alpha_z + ((int64_t)i * p->nbm + k0 + r) * nf, c->d_bad, i, s);
            });
            if (st) return st;
        }
    }
    return QR_OK;
}

static qr_status check_z(qr_ctx *c, const qr_problem *p, const qr_basis *b, int64_t M, int32_t scheme,
                         const double *alpha_z) {
    if (!alpha_z) return fail(QR_EINVAL, "Z regression: alpha_z is NULL");
    if (scheme != QR_Z_MULTISTEP && scheme != QR_Z_ONESTEP) return fail(QR_EINVAL, "Z regression: scheme %d", scheme);
    if (p->damping_q != 0.0) return fail(QR_ENOTSUP, "Z regression: damping exponent q must be 0");
    if (b->cos) return fail(QR_ENOTSUP, "Z regression: the cosine basis is not supported");
    if (project_pass_lds_bytes(p->d) > (size_t)160 * 1024) return fail(QR_ENOTSUP, "Z regression: d=%d", p->d);
    qr_status st;
    if ((st = ensure(c, c->zf0, sizeof(double) * 2 * (size_t)M, "first terms"))) return st;
    if (scheme == QR_Z_ONESTEP) {
        if ((st = ensure(c, c->zx0, sizeof(double) * (size_t)p->d * M, "start points"))) return st;
        if ((st = ensure(c, c->zy0, sizeof(double) * (size_t)M, "start-point values"))) return st;
    }
    return QR_OK;
}

extern "C" qr_status qr_backward_step_z(qr_ctx *c, const qr_problem *p, const qr_basis *bc, int32_t i, int64_t M,
                                        uint64_t seed, int32_t scheme, double *alpha, double *alpha_z,
                                        void *stream) {
    qr_basis *b = const_cast<qr_basis *>(bc);
    qr_status st = prepare(c, p, b, M, stream);
    if (st) return st;
    if (!alpha) return fail(QR_EINVAL, "qr_backward_step_z: alpha is NULL");
    if (i < 0 || i >= p->N) return fail(QR_EINVAL, "qr_backward_step_z: i=%d outside [0,%d)", i, p->N);
    if ((st = check_z(c, p, b, M, scheme, alpha_z))) return st;
    hipStream_t s = (hipStream_t)stream;
    double2 *ai = (double2 *)c->alpha_int.p;
    const int64_t nf = b->nfc();
    st = timed(c, 3, s, "gather_kernel", [&] {
        return launch_gather(alpha, i + 1, p->N - 1 - i, b->nrep, b->ld(), nf, b->d_canon_of_trav, ai, s);
    });
    if (st) return st;
    double *S = (double *)c->S.p;
    double2 *u = (double2 *)c->u.p;
    double *x0 = scheme == QR_Z_ONESTEP ? (double *)c->zx0.p : nullptr;
    if ((st = run_path(c, p, b, i, M, seed, ai, S, u, x0, s, (double *)c->zf0.p))) return st;
    if ((st = project_and_reduce(c, b, u, S, M, ai + (int64_t)i * b->ld(), alpha + (int64_t)i * nf, i, s))) return st;
    return project_z(c, p, b, i, M, seed, scheme, alpha_z, s);
}

extern "C" qr_status qr_solve_z(qr_ctx *c, const qr_problem *p, const qr_basis *bc, int64_t M, uint64_t seed,
                                int32_t scheme, double *alpha, double *alpha_z, void *stream) {
    qr_basis *b = const_cast<qr_basis *>(bc);
    qr_status st = prepare(c, p, b, M, stream);
    if (st) return st;
    if (!alpha) return fail(QR_EINVAL, "qr_solve_z: alpha is NULL");
    if ((st = check_z(c, p, b, M, scheme, alpha_z))) return st;
    hipStream_t s = (hipStream_t)stream;
    double2 *ai = (double2 *)c->alpha_int.p;
    const int64_t nf = b->nfc();
    double *S = (double *)c->S.p;
    double2 *u = (double2 *)c->u.p;
    double *x0 = scheme == QR_Z_ONESTEP ? (double *)c->zx0.p : nullptr;
    if ((st = numeric_clear(c, s))) return st;
    for (int32_t i = p->N - 1; i >= 0; --i) {
        if ((st = run_path(c, p, b, i, M, seed, ai, S, u, x0, s, (double *)c->zf0.p))) return st;
        if ((st = project_and_reduce(c, b, u, S, M, ai + (int64_t)i * b->ld(), alpha + (int64_t)i * nf, i, s)))
            return st;
        if ((st = project_z(c, p, b, i, M, seed, scheme, alpha_z, s))) return st;
    }
    return numeric_read(c, s, nullptr);
}

extern "C" qr_status qr_path_responses(qr_ctx *c, const qr_problem *p, const qr_basis *bc, int32_t i,
                                       int64_t M, uint64_t seed, const double *alpha, double *s_out,
                                       double *x0, void *stream) {
    qr_basis *b = const_cast<qr_basis *>(bc);
    qr_status st = prepare(c, p, b, M, stream);
    if (st) return st;
    if (!alpha || !s_out) return fail(QR_EINVAL, "qr_path_responses: NULL alpha or s");
    if (i < 0 || i >= p->N) return fail(QR_EINVAL, "qr_path_responses: i=%d outside [0,%d)", i, p->N);
    hipStream_t s = (hipStream_t)stream;
    double2 *ai = (double2 *)c->alpha_int.p;
    const int64_t nf = b->nfc();
    double *A;
    if ((st = carrier_in(c, b, alpha, i + 1, p->N, &A, s))) return st;
    st = timed(c, 3, s, "gather_kernel", [&] {
        return launch_gather(A, i + 1, p->N - 1 - i, b->nrep, b->ld(), nf, b->d_canon_of_trav, ai, s);
    });
    if (st) return st;
    return run_path(c, p, b, i, M, seed, ai, s_out, nullptr, x0, s);
}

extern "C" qr_status qr_project(qr_ctx *c, const qr_basis *bc, int64_t n, const double *x,
                                const double *s_in, double *alpha_row, void *stream) {
    qr_basis *b = const_cast<qr_basis *>(bc);
    qr_status st = begin(c, stream);
    if (st) return st;
    if ((st = check_basis_device(b))) return st;
    if ((st = check_M(n))) return st;
    if (!x || !s_in || !alpha_row) return fail(QR_EINVAL, "qr_project: NULL argument");
    if ((st = basis_on_device(b, c->dev))) return st;
    if ((st = ensure(c, c->u, sizeof(double2) * (size_t)n * b->d, "phase factors"))) return st;
    if ((st = ensure(c, c->row, sizeof(double2) * (size_t)b->ld(), "row"))) return st;
    hipStream_t s = (hipStream_t)stream;
    double2 *u = (double2 *)c->u.p;
    QR_HIP(launch_x_to_e(b->code(), b->d, x, n, u, s), "x_to_e_kernel");
    if (!b->cos) return project_and_reduce(c, b, u, s_in, n, (double2 *)c->row.p, alpha_row, -1, s);
    if ((st = ensure(c, c->crow, sizeof(double) * (size_t)b->nfc(), "carrier row"))) return st;
    double *crow = (double *)c->crow.p;
    if ((st = project_and_reduce(c, b, u, s_in, n, (double2 *)c->row.p, crow, -1, s))) return st;
    QR_HIP(launch_cos_fold(crow, b->ncos, b->d_fold_off, b->d_fold_idx, b->d_rep_scale, alpha_row, s),
           "cos_fold_kernel");
    return QR_OK;
}

extern "C" qr_status qr_eval(qr_ctx *c, const qr_basis *bc, const double *alpha_row, int64_t n,
                             const double *x, double *y, double *grad, void *stream) {
    qr_basis *b = const_cast<qr_basis *>(bc);
    qr_status st = begin(c, stream);
    if (st) return st;
    if ((st = check_basis_device(b))) return st;
    if (n < 0 || n > (int64_t)INT32_MAX * 64) return fail(QR_EINVAL, "qr_eval: n out of range");
    if (n == 0) return QR_OK;
    if (!alpha_row || !x || !y) return fail(QR_EINVAL, "qr_eval: NULL argument");
    if ((st = basis_on_device(b, c->dev))) return st;
    if ((st = ensure(c, c->row, sizeof(double2) * (size_t)b->ld(), "row"))) return st;
    hipStream_t s = (hipStream_t)stream;
    double2 *row = (double2 *)c->row.p;
    const int64_t nf = b->nfc();
    if (b->cos) {
        if ((st = ensure(c, c->crow, sizeof(double) * (size_t)nf, "carrier row"))) return st;
        double *crow = (double *)c->crow.p;
        QR_HIP(launch_cos_expand(alpha_row, 0, 1, b->ncos, b->nrep, b->d_cos_of_rep, b->d_rep_scale, crow, s),
               "cos_expand_kernel");
        alpha_row = crow;
    }
    QR_HIP(launch_pad(1, b->nrep, b->ld(), row, s), "pad_kernel");
    QR_HIP(launch_gather(alpha_row, 0, 1, b->nrep, b->ld(), nf, b->d_canon_of_trav, row, s), "gather_kernel");
    QR_HIP(launch_eval(depth_cap(b->max_nnz), grad != nullptr, make_walk(b->kind, b->level, b->d, b->code()), row, x,
                       n, y, grad, s),
           "eval_kernel");
    return QR_OK;
}

// Point sets up to this size are evaluated with the basis split across
// blocks (eval_tasks_kernel); larger ones one walk per thread (eval_kernel),
// which fills the chip from 2^17 points on.
constexpr int64_t kEvalTasksMax = (int64_t)1 << 17;

// ybar = row at n points x (SoA [d][n]) into y; value only.
static qr_status eval_points(qr_ctx *c, const qr_basis *b, const double2 *row, const double *x, int64_t n,
                             double *y, hipStream_t s) {
    const int cap = depth_cap(b->max_nnz);
    const Walk W = make_walk(b->kind, b->level, b->d, b->code());
    if (n > kEvalTasksMax || eval_tasks_lds(b->d) > (size_t)160 * 1024 || b->tasks.empty())
        return timed(c, 0, s, "eval_kernel", [&] { return launch_eval(cap, false, W, row, x, n, y, nullptr, s); });
    const ProjShape sh = proj_shape(b->d);
    const int64_t ntasks = (int64_t)b->tasks.size();
    const int64_t groups = (ntasks + sh.waves - 1) / sh.waves;
    const int64_t B = (int64_t)64 * sh.P;
    const int64_t want = std::max<int64_t>(1, std::min<int64_t>((kProjBlocks + groups - 1) / groups, (n + B - 1) / B));
    int64_t pps = (n + want - 1) / want;
    pps = (pps + B - 1) / B * B;
    const int32_t nsplit = (int32_t)((n + pps - 1) / pps);
    qr_status st;
    if ((st = ensure(c, c->ete, sizeof(double2) * (size_t)b->d * n, "phase factors"))) return st;
    if ((st = ensure(c, c->etp, sizeof(double) * (size_t)groups * n, "group sums"))) return st;
    double2 *e = (double2 *)c->ete.p;
    QR_HIP(launch_x_to_e(b->code(), b->d, x, n, e, s), "x_to_e_kernel");
    return timed(c, 0, s, "eval_tasks_kernel", [&] {
        return launch_eval_tasks(cap, W, e, n, pps, (int32_t)ntasks, nsplit, b->d_tasks, b->d_items, b->task_max,
                                 row, (double *)c->etp.p, y, s);
    });
}

extern "C" qr_status qr_eval_split(qr_ctx *c, const qr_basis *bc, const double *alpha_row, int64_t n,
                                   const double *x, double *y, void *stream) {
    qr_basis *b = const_cast<qr_basis *>(bc);
    qr_status st = begin(c, stream);
    if (st) return st;
    if ((st = check_basis_device(b))) return st;
    if (n < 0 || n > kEvalTasksMax) return fail(QR_EINVAL, "qr_eval_split: n=%lld outside [0, %lld]", (long long)n,
                                                (long long)kEvalTasksMax);
    if (n == 0) return QR_OK;
    if (!alpha_row || !x || !y) return fail(QR_EINVAL, "qr_eval_split: NULL argument");
    if (b->cos) return fail(QR_ENOTSUP, "qr_eval_split: the cosine basis is not supported");
    if (eval_tasks_lds(b->d) > (size_t)160 * 1024) return fail(QR_ENOTSUP, "qr_eval_split: d=%d", b->d);
    if ((st = basis_on_device(b, c->dev))) return st;
    if ((st = ensure(c, c->row, sizeof(double2) * (size_t)b->ld(), "row"))) return st;
    hipStream_t s = (hipStream_t)stream;
    double2 *row = (double2 *)c->row.p;
    QR_HIP(launch_pad(1, b->nrep, b->ld(), row, s), "pad_kernel");
    QR_HIP(launch_gather(alpha_row, 0, 1, b->nrep, b->ld(), b->nfc(), b->d_canon_of_trav, row, s), "gather_kernel");
    return eval_points(c, b, row, x, n, y, s);
}

extern "C" qr_status qr_eval_y(qr_ctx *c, const qr_problem *p, const qr_basis *bc, const double *alpha_row,
                               int64_t n, const double *x, double *y, double *grad, void *stream) {
    qr_status st = check_problem(p, bc);
    if (st) return st;
    if ((st = qr_eval(c, bc, alpha_row, n, x, y, grad, stream))) return st;
    if (p->damping_q == 0.0 || n == 0) return QR_OK;
    QR_HIP(launch_undamp(p->d, p->damping_q, x, n, y, grad, (hipStream_t)stream), "undamp_kernel");
    return QR_OK;
}

extern "C" qr_status qr_basis_upload(qr_ctx *c, const qr_basis *bc) {
    qr_basis *b = const_cast<qr_basis *>(bc);
    if (!c) return fail(QR_EINVAL, "qr_basis_upload: ctx is NULL");
    qr_status st = check_basis_device(b);
    if (st) return st;
    QR_HIP(hipSetDevice(c->dev), "hipSetDevice");
    return basis_on_device(b, c->dev);
}

// qr_eval with the coefficient row staged in this device's `scratch` instead
// of context workspace: no allocation of any kind.  The basis must already be
// resident on the context's device (qr_basis_upload, or any earlier call with
// it on this device).  Calls that overlap on one GPU share the scratch.
extern "C" qr_status qr_eval_noalloc(qr_ctx *c, const qr_basis *bc, const double *alpha_row, int64_t n,
                                     const double *x, double *y, double *grad, void *stream) {
    const qr_basis *b = bc;
    qr_status st = begin(c, stream);
    if (st) return st;
    if ((st = check_basis_device(b))) return st;
    if (n < 0 || n > (int64_t)INT32_MAX * 64) return fail(QR_EINVAL, "qr_eval_noalloc: n out of range");
    if (b->cos) return fail(QR_ENOTSUP, "qr_eval_noalloc: the cosine basis needs a carrier row (use qr_eval)");
    if (b->ld() > (int64_t)QR_NOALLOC_ROW_MAX)
        return fail(QR_ERANGE, "qr_eval_noalloc: basis of %lld representatives needs %lld scratch entries (limit %d)",
                    (long long)b->nrep, (long long)b->ld(), QR_NOALLOC_ROW_MAX);
    int resident;
    {
        std::lock_guard<std::mutex> lock(const_cast<qr_basis *>(b)->mu);
        resident = b->dev;
    }
    if (resident != c->dev)
        return fail(QR_EINVAL, "qr_eval_noalloc: basis is not resident on device %d (call qr_basis_upload first)",
                    c->dev);
    if (n == 0) return QR_OK;
    if (!alpha_row || !x || !y) return fail(QR_EINVAL, "qr_eval_noalloc: NULL argument");
    double2 *row = scratch_of(c->dev);
    if (!row) return fail(QR_EDEVICE, "qr_eval_noalloc: scratch of device %d not initialised", c->dev);
    hipStream_t s = (hipStream_t)stream;
    const int64_t nf = 2 * b->nrep - 1;
    // the read-ahead chunks must read as zero: cleared by a kernel on every call,
    // since the previous call may have left another basis's row there
    QR_HIP(launch_pad(1, b->nrep, b->ld(), row, s), "pad_kernel");
    QR_HIP(launch_gather(alpha_row, 0, 1, b->nrep, b->ld(), nf, b->d_canon_of_trav, row, s), "gather_kernel");
    QR_HIP(launch_eval(depth_cap(b->max_nnz), grad != nullptr, make_walk(b->kind, b->level, b->d, b->code()), row, x,
                       n, y, grad, s),
           "eval_kernel");
    return QR_OK;
}

extern "C" qr_status qr_sample_points(qr_ctx *c, int32_t d, uint64_t seed, uint32_t stream_id,
                                      int32_t i, int64_t m0, int64_t n, double *x, void *stream) {
    return qr_sample_points_law(c, QR_LAW_LOGISTIC, d, seed, stream_id, i, m0, n, x, stream);
}

extern "C" qr_status qr_sample_points_law(qr_ctx *c, int32_t law, int32_t d, uint64_t seed,
                                          uint32_t stream_id, int32_t i, int64_t m0, int64_t n, double *x,
                                          void *stream) {
    qr_status st = begin(c, stream);
    if (st) return st;
    if (law < QR_LAW_LOGISTIC || law > QR_LAW_CAUCHY)
        return fail(QR_EINVAL, "qr_sample_points: unknown sampling law %d", law);
    if (d < 1 || d > QR_MAX_D) return fail(QR_EINVAL, "qr_sample_points: d=%d", d);
    if (n < 0 || m0 < 0 || !x) return fail(QR_EINVAL, "qr_sample_points: bad n/m0/x");
    QR_HIP(launch_sample(law, d, seed, stream_id, i, m0, n, x, (hipStream_t)stream), "sample_kernel");
    return QR_OK;
}

// ---------------------------------------------------------------------------
// reduced-precision form
// ---------------------------------------------------------------------------
namespace {
struct TilePlan {
    int T;
    int64_t ld;  // uint2 per row: one spare group for the walk's prefetch past the last group
};
TilePlan tile_plan(const qr_problem *p, const qr_basis *b) {
    const bool grad = p->driver == QR_F_ZRAT;
    const int T = mfma_tile_groups(dim_bucket(p->d, p->nbm), p->d, grad);
    const int64_t ngroups = (b->nrep + 31) / 32;
    return TilePlan{T, (ngroups + 1) * T * 64};
}
}  // namespace

static qr_status prepare_prec(qr_ctx *c, const qr_problem *p, qr_basis *b, int64_t M, int32_t prec,
                              void *stream, TilePlan *tp) {
    if (prec != QR_PREC_BF16 && prec != QR_PREC_F16)
        return fail(QR_EINVAL, "precision %d is not one of QR_PREC_F64/BF16/F16", prec);
    qr_status st = prepare(c, p, b, M, stream);
    if (st) return st;
    if (p->damping_q != 0.0) return fail(QR_ENOTSUP, "reduced-precision form: damping exponent q must be 0");
    if (state_dependent(p)) return fail(QR_ENOTSUP, "reduced-precision form: state-dependent b2 or sigma_v");
    *tp = tile_plan(p, b);
    if ((st = ensure(c, c->tiles, sizeof(uint2) * (size_t)p->N * tp->ld, "coefficient tiles"))) return st;
    // the spare groups are read ahead and never used; keep them defined
    QR_HIP(launch_zero((double *)c->tiles.p, (int64_t)(sizeof(uint2) / sizeof(double)) * p->N * tp->ld,
                       (hipStream_t)stream), "zero_kernel");
    return QR_OK;
}

static qr_status pack_row(qr_ctx *c, const qr_problem *p, const qr_basis *b, int32_t prec, const TilePlan &tp,
                          int32_t row, hipStream_t s) {
    const double2 *ai = (const double2 *)c->alpha_int.p + (int64_t)row * b->ld();
    uint2 *out = (uint2 *)c->tiles.p + (int64_t)row * tp.ld;
    return timed(c, 3, s, "pack_tiles_kernel",
                 [&] { return launch_pack_tiles(prec, ai, b->nrep, b->d_trav, p->d, tp.T, b->cos, out, s); });
}

static qr_status run_mfma_path(qr_ctx *c, const qr_problem *p, const qr_basis *b, int32_t prec,
                               const TilePlan &tp, int32_t i, int64_t M, uint64_t seed, hipStream_t s) {
    MfmaArgs a{c->d_prob, make_walk(b->kind, b->level, b->d, b->code()), i, M, seed, (const uint2 *)c->tiles.p, tp.ld,
               (double *)c->S.p, (double2 *)c->u.p};
    return timed(c, 0, s, "mfma_path_kernel", [&] {
        return launch_mfma_path(dim_bucket(p->d, p->nbm), depth_cap(b->max_nnz), p->driver == QR_F_ZRAT, prec,
                                a, s);
    });
}

// Whether the reduced-precision form runs the factored kernel for this
// problem and basis (the context's choice, the driver, the basis's layout and
// the kernel's LDS); *st is set when the choice cannot be honoured.
static bool use_factored(qr_ctx *c, const qr_problem *p, qr_basis *b, qr_status *st) {
    *st = QR_OK;
    if (c->prec_kernel == QR_PREC_KERNEL_WALK) return false;
    const bool forced = c->prec_kernel == QR_PREC_KERNEL_FACTORED;
    const char *why = nullptr;
    if (p->driver == QR_F_ZRAT)
        why = "the factored kernel evaluates no gradients (z-dependent driver)";
    else if (!basis_factored(b))
        why = "no split of the index set qualifies for the factored kernel";
    else {
        const size_t lds = (size_t)fac_waves(b->d, b->fac->TS) * kFacPaths * fac_stride(b->d, b->fac->TS) *
                           sizeof(float2);
        if (lds > 160 * 1024) why = "the factored kernel's tables exceed the LDS of a CU";
    }
    if (!why) return true;
    if (forced) *st = fail(QR_ENOTSUP, "reduced-precision form: %s", why);
    return false;
}

static qr_status prepare_fac(qr_ctx *c, const qr_problem *p, qr_basis *b) {
    qr_status st = basis_factored_on_device(b);
    if (st) return st;
    return ensure(c, c->fcoef, sizeof(uint4) * (size_t)p->N * b->fac->nblocks * 64, "factored coefficients");
}

static qr_status fac_pack_row(qr_ctx *c, const qr_basis *b, int32_t prec, const double *alpha_row, int32_t row,
                              hipStream_t s) {
    uint4 *out = (uint4 *)c->fcoef.p + (size_t)row * b->fac->nblocks * 64;
    return timed(c, 3, s, "fac_pack_kernel",
                 [&] { return launch_fac_pack(prec, alpha_row, b->d_fac.ent, b->fac->nblocks, out, s); });
}

static qr_status run_fac_path(qr_ctx *c, const qr_problem *p, const qr_basis *b, int32_t prec, int32_t i,
                              int64_t M, uint64_t seed, hipStream_t s) {
    FacPathArgs a{c->d_prob, b->d_fac, i, M, seed, (const uint4 *)c->fcoef.p, (double *)c->S.p,
                  (double2 *)c->u.p};
    return timed(c, 0, s, "fac_path_kernel",
                 [&] { return launch_fac_path(dim_bucket(p->d, p->nbm), prec, a, s); });
}

// Units (waves) of the factored projection: each takes a share of the paths
// for one task; about 8192 waves in all, at least 256 paths per unit.
static int32_t fac_units(const qr_basis *b, int64_t M) {
    int32_t ntasks = 0;
    for (int t = 0; t < kFacTemplates; ++t) ntasks += b->fac_ntasks[t];
    const int waves = fac_waves(b->d, b->fac->TS);
    int64_t u = 8192 / std::max(1, ntasks);
    u = std::min<int64_t>(u, (M + 255) / 256);
    u = std::max<int64_t>(1, std::min<int64_t>(u, 512));
    return (int32_t)((u + waves - 1) / waves * waves);
}

static qr_status fac_project(qr_ctx *c, const qr_basis *b, int32_t prec, int64_t M, double *alpha_row,
                             int32_t step, hipStream_t s) {
    const int32_t units = fac_units(b, M);
    int64_t per = (M + units - 1) / units;
    per = (per + kFacPaths - 1) / kFacPaths * kFacPaths;
    qr_status st = ensure(c, c->fpartial, sizeof(float) * 256 * (size_t)units * b->fac->nblocks, "factored partials");
    if (st) return st;
    float *partial = (float *)c->fpartial.p;
    for (int t = 0; t < kFacTemplates; ++t) {
        if (!b->fac_ntasks[t]) continue;
        st = timed(c, 1, s, "fac_project_kernel", [&] {
            return launch_fac_project(prec, t, b->d_fac, b->d_fac_tasks[t], b->fac_ntasks[t], (const double2 *)c->u.p,
                                      (const double *)c->S.p, M, per, units, partial, s);
        });
        if (st) return st;
    }
    return timed(c, 2, s, "fac_reduce_kernel", [&] {
        return launch_fac_reduce(partial, units, b->fac->nblocks, b->d_fac.ent, (double)M, alpha_row, c->d_bad, step,
                                 s);
    });
}

extern "C" qr_status qr_backward_step_prec(qr_ctx *c, const qr_problem *p, const qr_basis *bc, int32_t i,
                                           int64_t M, uint64_t seed, int32_t prec, double *alpha,
                                           void *stream) {
    if (prec == QR_PREC_F64) return qr_backward_step(c, p, bc, i, M, seed, alpha, stream);
    qr_basis *b = const_cast<qr_basis *>(bc);
    TilePlan tp;
    qr_status st = prepare_prec(c, p, b, M, prec, stream, &tp);
    if (st) return st;
    if (!alpha) return fail(QR_EINVAL, "qr_backward_step_prec: alpha is NULL");
    if (i < 0 || i >= p->N) return fail(QR_EINVAL, "qr_backward_step_prec: i=%d outside [0,%d)", i, p->N);
    hipStream_t s = (hipStream_t)stream;
    double2 *ai = (double2 *)c->alpha_int.p;
    const int64_t nf = b->nfc();
    const bool fac = use_factored(c, p, b, &st);
    if (st) return st;
    double *A;
    if ((st = carrier_in(c, b, alpha, i + 1, p->N, &A, s))) return st;
    if (fac) {
        if ((st = prepare_fac(c, p, b))) return st;
        for (int32_t r = i + 1; r < p->N; ++r)
            if ((st = fac_pack_row(c, b, prec, A + (int64_t)r * nf, r, s))) return st;
        if ((st = run_fac_path(c, p, b, prec, i, M, seed, s))) return st;
        if ((st = fac_project(c, b, prec, M, A + (int64_t)i * nf, i, s))) return st;
    } else {
        st = timed(c, 3, s, "gather_kernel", [&] {
            return launch_gather(A, i + 1, p->N - 1 - i, b->nrep, b->ld(), nf, b->d_canon_of_trav, ai, s);
        });
        if (st) return st;
        for (int32_t r = i + 1; r < p->N; ++r)
            if ((st = pack_row(c, p, b, prec, tp, r, s))) return st;
        if ((st = run_mfma_path(c, p, b, prec, tp, i, M, seed, s))) return st;
        if ((st = project_and_reduce(c, b, (double2 *)c->u.p, (double *)c->S.p, M, ai + (int64_t)i * b->ld(),
                                     A + (int64_t)i * nf, i, s)))
            return st;
    }
    return carrier_out(c, b, A, alpha, i, nullptr, s);
}

extern "C" qr_status qr_solve_from(qr_ctx *c, const qr_problem *p, const qr_basis *bc, int32_t i0, int64_t M,
                                   uint64_t seed, int32_t prec, double *alpha, void *stream) {
    if (prec == QR_PREC_F64) return solve_f64_from(c, p, const_cast<qr_basis *>(bc), i0, M, seed, alpha, stream);
    qr_basis *b = const_cast<qr_basis *>(bc);
    TilePlan tp;
    qr_status st = prepare_prec(c, p, b, M, prec, stream, &tp);
    if (st) return st;
    if (!alpha) return fail(QR_EINVAL, "qr_solve_prec: alpha is NULL");
    if (i0 < 0 || i0 >= p->N) return fail(QR_EINVAL, "qr_solve_from: i_start=%d outside [0,%d)", i0, p->N);
    hipStream_t s = (hipStream_t)stream;
    double2 *ai = (double2 *)c->alpha_int.p;
    const int64_t nf = b->nfc();
    const bool fac = use_factored(c, p, b, &st);
    if (st) return st;
    if (fac && (st = prepare_fac(c, p, b))) return st;
    double *A;
    if ((st = carrier_in(c, b, alpha, i0 + 1, p->N, &A, s))) return st;
    // the given rows in the kernels' layouts
    if (fac) {
        for (int32_t r = i0 + 1; r < p->N; ++r)
            if ((st = fac_pack_row(c, b, prec, A + (int64_t)r * nf, r, s))) return st;
    } else {
        st = timed(c, 3, s, "gather_kernel", [&] {
            return launch_gather(A, i0 + 1, p->N - 1 - i0, b->nrep, b->ld(), nf, b->d_canon_of_trav, ai, s);
        });
        if (st) return st;
        for (int32_t r = i0 + 1; r < p->N; ++r)
            if ((st = pack_row(c, p, b, prec, tp, r, s))) return st;
    }
    if ((st = numeric_clear(c, s))) return st;
    for (int32_t i = i0; i >= 0; --i) {
        st = fac ? run_fac_path(c, p, b, prec, i, M, seed, s) : run_mfma_path(c, p, b, prec, tp, i, M, seed, s);
        if (st) return st;
        st = fac ? fac_project(c, b, prec, M, A + (int64_t)i * nf, i, s)
                 : project_and_reduce(c, b, (double2 *)c->u.p, (double *)c->S.p, M, ai + (int64_t)i * b->ld(),
                                      A + (int64_t)i * nf, i, s);
        if (st) return st;
        if ((st = carrier_out(c, b, A, alpha, i, fac ? nullptr : ai, s))) return st;
        if (i > 0) {
            st = fac ? fac_pack_row(c, b, prec, A + (int64_t)i * nf, i, s) : pack_row(c, p, b, prec, tp, i, s);
            if (st) return st;
        }
    }
    return numeric_read(c, s, nullptr);
}

extern "C" qr_status qr_solve_prec(qr_ctx *c, const qr_problem *p, const qr_basis *bc, int64_t M,
                                   uint64_t seed, int32_t prec, double *alpha, void *stream) {
    if (!p) return fail(QR_EINVAL, "problem is NULL");
    return qr_solve_from(c, p, bc, p->N - 1, M, seed, prec, alpha, stream);
}

// ---------------------------------------------------------------------------
// surrogate network (learned form)
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kMlpChunk = QR_MLP_MAX_BATCH;       // rows of the activation workspace
constexpr int64_t kGemmWork = (int64_t)64 * kMlpHid * kMlpHid;  // split-K partials (floats)
}  // namespace

// room for two partial sums per block of 256 over n items
static qr_status ensure_partials(qr_ctx *c, int64_t n) {
    return ensure(c, c->mpart, sizeof(double) * (size_t)(2 * ((n + 255) / 256) + 2), "partials");
}

static qr_status mlp_workspace(qr_ctx *c, int64_t rows) {
    qr_status st;
    const size_t act = sizeof(float) * (size_t)rows * kMlpHid;
    if ((st = ensure(c, c->mf, sizeof(float) * (size_t)rows * kMlpIn, "network features"))) return st;
    for (Buf *b : {&c->mz1, &c->mh1, &c->mz2, &c->mh2, &c->mdz, &c->mdh})
        if ((st = ensure(c, *b, act, "network activations"))) return st;
    if ((st = ensure(c, c->my, sizeof(float) * (size_t)rows, "network outputs"))) return st;
    if ((st = ensure(c, c->mdy, sizeof(float) * (size_t)rows, "network outputs"))) return st;
    if ((st = ensure_partials(c, rows))) return st;
    if ((st = ensure(c, c->mwork, sizeof(float) * (size_t)kGemmWork, "gemm workspace"))) return st;
    if ((st = ensure(c, c->mcwork, sizeof(float) * (size_t)kColsumWork, "column sums"))) return st;
    return QR_OK;
}

// forward pass of n <= kMlpChunk rows; leaves Z1, H1, Z2, H2 in the workspace
static hipError_t mlp_fwd(qr_ctx *c, const float *th, int64_t n, const float *f, float *y, hipStream_t s) {
    float *Z1 = (float *)c->mz1.p, *H1 = (float *)c->mh1.p, *Z2 = (float *)c->mz2.p, *H2 = (float *)c->mh2.p;
    float *w = (float *)c->mwork.p;
    hipError_t e;
    const int N = (int)n;
    // Z1 = F W1^T: B(k, j) = W1[j][k]
    if ((e = launch_gemm(N, kMlpHid, kMlpIn, f, kMlpIn, 1, th + kOffW1, 1, kMlpIn, Z1, kMlpHid, false, w, kGemmWork, s)))
        return e;
    if ((e = launch_bias_silu(n, kMlpHid, Z1, th + kOffB1, H1, s))) return e;
    if ((e = launch_gemm(N, kMlpHid, kMlpHid, H1, kMlpHid, 1, th + kOffW2, 1, kMlpHid, Z2, kMlpHid, false, w,
                         kGemmWork, s)))
        return e;
    if ((e = launch_bias_silu(n, kMlpHid, Z2, th + kOffB2, H2, s))) return e;
    return launch_out_layer(n, kMlpHid, H2, th + kOffW3, th + kOffB3, y, s);
}

// loss partials into mpart, gradient into g (all blocks overwritten)
static hipError_t mlp_bwd(qr_ctx *c, const float *th, int64_t n, const float *f, const float *t, float *g,
                          hipStream_t s) {
    hipError_t e;
    if ((e = mlp_fwd(c, th, n, f, (float *)c->my.p, s))) return e;
    float *Z1 = (float *)c->mz1.p, *H1 = (float *)c->mh1.p, *Z2 = (float *)c->mz2.p, *H2 = (float *)c->mh2.p;
    float *dZ = (float *)c->mdz.p, *dH = (float *)c->mdh.p, *dy = (float *)c->mdy.p;
    float *w = (float *)c->mwork.p, *cw = (float *)c->mcwork.p;
    const int N = (int)n;
    if ((e = launch_loss(n, (float *)c->my.p, t, dy, (double *)c->mpart.p, s))) return e;
    if ((e = launch_colsum(n, kMlpHid, H2, dy, g + kOffW3, cw, s))) return e;
    if ((e = launch_colsum(n, 1, dy, nullptr, g + kOffB3, cw, s))) return e;
    if ((e = launch_dz_out(n, kMlpHid, dy, th + kOffW3, Z2, dZ, s))) return e;
    // dW2 = dZ^T H1
    if ((e = launch_gemm(kMlpHid, kMlpHid, N, dZ, 1, kMlpHid, H1, kMlpHid, 1, g + kOffW2, kMlpHid, false, w,
                         kGemmWork, s)))
        return e;
    if ((e = launch_colsum(n, kMlpHid, dZ, nullptr, g + kOffB2, cw, s))) return e;
    // dH1 = dZ W2, then through silu'
    if ((e = launch_gemm(N, kMlpHid, kMlpHid, dZ, kMlpHid, 1, th + kOffW2, kMlpHid, 1, dH, kMlpHid, false, w,
                         kGemmWork, s)))
        return e;
    if ((e = launch_dsilu(n, kMlpHid, Z1, dH, s))) return e;
    // dW1 = dZ1^T F
    if ((e = launch_gemm(kMlpHid, kMlpIn, N, dH, 1, kMlpHid, f, kMlpIn, 1, g + kOffW1, kMlpIn, false, w, kGemmWork,
                         s)))
        return e;
    return launch_colsum(n, kMlpHid, dH, nullptr, g + kOffB1, cw, s);
}

static qr_status read_partials(qr_ctx *c, int64_t nblocks, int stride, double *out, hipStream_t s) {
    std::vector<double> h((size_t)nblocks * stride);
    QR_HIP(hipMemcpyAsync(h.data(), c->mpart.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s),
           "hipMemcpyAsync(partials)");
    QR_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (int k = 0; k < stride; ++k) out[k] = 0.0;
    for (int64_t b = 0; b < nblocks; ++b)
        for (int k = 0; k < stride; ++k) out[k] += h[(size_t)b * stride + k];
    return QR_OK;
}

extern "C" qr_status qr_mlp_init(qr_ctx *c, float *params, uint64_t seed, void *stream) {
    qr_status st = begin(c, stream);
    if (st) return st;
    if (!params) return fail(QR_EINVAL, "qr_mlp_init: params is NULL");
    QR_HIP(launch_mlp_init(params, seed, (hipStream_t)stream), "mlp_init_kernel");
    return QR_OK;
}

extern "C" qr_status qr_mlp_features(qr_ctx *c, int32_t d, int64_t n, const double *x, float *feat, void *stream) {
    qr_status st = begin(c, stream);
    if (st) return st;
    if (d < 1 || d > kMlpIn) return fail(QR_EINVAL, "qr_mlp_features: d=%d outside [1,%d]", d, kMlpIn);
    if (n < 0) return fail(QR_EINVAL, "qr_mlp_features: n < 0");
    if (n == 0) return QR_OK;
    if (!x || !feat) return fail(QR_EINVAL, "qr_mlp_features: NULL argument");
    QR_HIP(launch_features(QR_LAW_LOGISTIC, d, n, x, n, feat, (hipStream_t)stream), "features_kernel");
    return QR_OK;
}

extern "C" qr_status qr_mlp_forward(qr_ctx *c, const float *params, int64_t n, const float *feat, float *y,
                                    void *stream) {
    qr_status st = begin(c, stream);
    if (st) return st;
    if (n < 0) return fail(QR_EINVAL, "qr_mlp_forward: n < 0");
    if (n == 0) return QR_OK;
    if (!params || !feat || !y) return fail(QR_EINVAL, "qr_mlp_forward: NULL argument");
    if ((st = mlp_workspace(c, std::min(n, kMlpChunk)))) return st;
    hipStream_t s = (hipStream_t)stream;
    for (int64_t p0 = 0; p0 < n; p0 += kMlpChunk) {
        const int64_t k = std::min(kMlpChunk, n - p0);
        QR_HIP(mlp_fwd(c, params, k, feat + p0 * kMlpIn, y + p0, s), "mlp forward");
    }
    return QR_OK;
}

extern "C" qr_status qr_mlp_loss_grad(qr_ctx *c, const float *params, int64_t n, const float *feat,
                                      const float *target, float *grad, double *loss, void *stream) {
    qr_status st = begin(c, stream);
    if (st) return st;
    if (n < 1 || n > kMlpChunk) return fail(QR_EINVAL, "qr_mlp_loss_grad: n=%lld outside [1,%lld]", (long long)n,
                                            (long long)kMlpChunk);
    if (!params || !feat || !target || !grad) return fail(QR_EINVAL, "qr_mlp_loss_grad: NULL argument");
    if ((st = mlp_workspace(c, n))) return st;
    hipStream_t s = (hipStream_t)stream;
    QR_HIP(mlp_bwd(c, params, n, feat, target, grad, s), "mlp backward");
    if (loss) {
        double sum;
        if ((st = read_partials(c, (n + 255) / 256, 1, &sum, s))) return st;
        *loss = sum / (double)n;
    }
    return QR_OK;
}

extern "C" qr_status qr_mlp_adam(qr_ctx *c, float *params, const float *grad, float *m, float *v, int64_t step,
                                 float lr, void *stream) {
    qr_status st = begin(c, stream);
    if (st) return st;
    if (!params || !grad || !m || !v) return fail(QR_EINVAL, "qr_mlp_adam: NULL argument");
    if (step < 1) return fail(QR_EINVAL, "qr_mlp_adam: step must be >= 1");
    if (!(lr > 0.f)) return fail(QR_EINVAL, "qr_mlp_adam: lr must be > 0");
    QR_HIP(launch_adam(kMlpParams, params, grad, m, v, step, lr, (hipStream_t)stream), "adam_kernel");
    return QR_OK;
}

// Fit a network to ybar_j (row j of alpha_int) on the first nt training and
// nh held-out pairs, `epochs` epochs of mini-batches of B.
static qr_status fit_pairs(qr_ctx *c, const qr_problem *p, const qr_basis *b, int32_t j, uint64_t seed,
                           const qr_learn_opts *o, int64_t nt, int64_t nh, int64_t B, int epochs, float *th,
                           double *mu, double *sigma, qr_learn_report *rep, hipStream_t s, bool screen = false) {
    qr_status st;
    const int d = p->d;
    double *tx = (double *)c->ltx.p, *tt = (double *)c->ltt.p, *hx = (double *)c->lhx.p, *ht = (double *)c->lht.p;
    float *tf = (float *)c->ltf.p, *ff = (float *)c->lff.p, *hf = (float *)c->lhf.p, *hy = (float *)c->lhy.p;
    const double2 *row = (const double2 *)c->alpha_int.p + (int64_t)j * b->ld();
    // pairs (X, ybar_j(X)): training from stream 2, held-out from stream 3, at time index j
    QR_HIP(launch_sample(b->law, d, seed, 2u, j, 0, nt, tx, s), "sample_kernel");
    QR_HIP(launch_sample(b->law, d, seed, 3u, j, 0, nh, hx, s), "sample_kernel");
    if ((st = eval_points(c, b, row, tx, nt, tt, s))) return st;
    if ((st = eval_points(c, b, row, hx, nh, ht, s))) return st;
    // targets normalised by their mean and standard deviation
    QR_HIP(launch_moments(nt, tt, (double *)c->mpart.p, s), "moments_kernel");
    double mom[2];
    if ((st = read_partials(c, (nt + 255) / 256, 2, mom, s))) return st;
    const double mean = mom[0] / (double)nt;
    double var = mom[1] / (double)nt - mean * mean;
    const double sd = var > 1e-300 ? std::sqrt(var) : 1.0;
    *mu = mean;
    *sigma = sd;
    QR_HIP(launch_to_float(nt, tt, mean, 1.0 / sd, tf, s), "to_float_kernel");
    QR_HIP(launch_features(b->law, d, nt, tx, nt, ff, s), "features_kernel");
    QR_HIP(launch_features(b->law, d, nh, hx, nh, hf, s), "features_kernel");
    // Adam over mini-batches in a fixed order
    QR_HIP(launch_mlp_init(th, seed ^ (0x9E3779B97F4A7C15ull * (uint64_t)(j + 1)), s), "mlp_init_kernel");
    QR_HIP(launch_zero((double *)c->lm.p, kMlpParams / 2 + 1, s), "zero_kernel");
    QR_HIP(launch_zero((double *)c->lv.p, kMlpParams / 2 + 1, s), "zero_kernel");
    float *g = (float *)c->lgrad.p, *m = (float *)c->lm.p, *v = (float *)c->lv.p;
    // held-out relative error of the current parameters against the expansion
    auto heldout = [&](double *err) -> qr_status {
        for (int64_t p0 = 0; p0 < nh; p0 += kMlpChunk) {
            const int64_t k = std::min(kMlpChunk, nh - p0);
            QR_HIP(mlp_fwd(c, th, k, hf + p0 * kMlpIn, hy + p0, s), "mlp forward");
        }
        QR_HIP(launch_heldout(nh, hy, ht, mean, sd, (double *)c->mpart.p, s), "heldout_kernel");
        double ab[2];
        const qr_status rs = read_partials(c, (nh + 255) / 256, 2, ab, s);
        if (rs) return rs;
        *err = ab[1] > 0.0 ? std::sqrt(ab[0] / ab[1]) : INFINITY;
        return QR_OK;
    };
    const int64_t nb = nt / B;
    int64_t step = 0;
    double last = NAN;
    rep->trained = 1;
    rep->used = 0;
    for (int e = 0; e < epochs; ++e) {
        double ep = 0.0;
        for (int64_t bi = 0; bi < nb; ++bi) {
            QR_HIP(mlp_bwd(c, th, B, ff + bi * B * kMlpIn, tf + bi * B, g, s), "mlp backward");
            QR_HIP(launch_adam(kMlpParams, th, g, m, v, ++step, o->lr, s), "adam_kernel");
            if (e + 1 == epochs) {
                double l;
                if ((st = read_partials(c, (B + 255) / 256, 1, &l, s))) return st;
                ep += l / (double)B;
            }
        }
        rep->epochs_run = e + 1;
        if (e + 1 == epochs) last = ep / (double)nb;
        if (screen && e + 1 < epochs) {
            // the screen stops as soon as it is within `reject`
            double err;
            if ((st = heldout(&err))) return st;
            if (err <= o->reject) {
                rep->heldout_rel_l2 = err;
                rep->train_loss = last;
                return QR_OK;
            }
        }
    }
    if ((st = heldout(&rep->heldout_rel_l2))) return st;
    rep->train_loss = last;
    rep->used = rep->heldout_rel_l2 <= o->gate ? 1 : 0;
    return QR_OK;
}

// Fit the surrogate of ybar_j for time index j.  With reject > 0 a screen
// comes first: the fit on the first 1/kScreenShare of the training and
// held-out pairs (the expansion evaluated at that share of the points, which
// is most of a fit's cost), with every epoch, stopping once its held-out
// error is within `reject`; a network still above `reject` after the last
// epoch is not fitted further.  A passed screen is followed by the full fit.
constexpr int64_t kScreenShare = 32;

static qr_status fit_surrogate(qr_ctx *c, const qr_problem *p, const qr_basis *b, int32_t j, uint64_t seed,
                              const qr_learn_opts *o, float *th, double *mu, double *sigma,
                              qr_learn_report *rep, hipStream_t s) {
    if (o->reject > 0.0) {
        const int64_t nt = o->train_points / kScreenShare, nh = std::max<int64_t>(1, o->heldout_points / kScreenShare);
        const int64_t B = std::min<int64_t>(o->batch, nt);
        if (B >= 64 && o->epochs >= 1) {
            qr_status st = fit_pairs(c, p, b, j, seed, o, nt, nh, B, o->epochs, th, mu, sigma, rep, s, true);
            if (st) return st;
            if (rep->heldout_rel_l2 > o->reject) {
                rep->used = 0;
                return QR_OK;
            }
        }
    }
    return fit_pairs(c, p, b, j, seed, o, o->train_points, o->heldout_points, o->batch, o->epochs, th, mu, sigma, rep,
                     s);
}

extern "C" qr_status qr_solve_learned(qr_ctx *c, const qr_problem *p, const qr_basis *bc, int64_t M,
                                      uint64_t seed, const qr_learn_opts *o, double *alpha,
                                      qr_learn_report *report, float *params_out, void *stream) {
    qr_basis *b = const_cast<qr_basis *>(bc);
    if (!o || !report) return fail(QR_EINVAL, "qr_solve_learned: NULL opts or report");
    if (o->epochs < 0 || o->batch < 64 || o->batch > QR_MLP_MAX_BATCH || o->train_points < o->batch ||
        o->heldout_points < 1 || !(o->lr > 0.f) || !(o->gate >= 0.0) || !(o->reject >= 0.0))
        return fail(QR_EINVAL, "qr_solve_learned: invalid options (epochs >= 0, 64 <= batch <= %d, "
                               "train_points >= batch, heldout_points >= 1, lr > 0, gate >= 0, reject >= 0)",
                    QR_MLP_MAX_BATCH);
    qr_status st = prepare(c, p, b, M, stream);
    if (st) return st;
    if (!alpha) return fail(QR_EINVAL, "qr_solve_learned: alpha is NULL");
    if (p->driver == QR_F_ZRAT)
        return fail(QR_ENOTSUP, "qr_solve_learned: the driver depends on z (the surrogate has no gradient)");
    if (p->damping_q != 0.0) return fail(QR_ENOTSUP, "qr_solve_learned: damping exponent q must be 0");
    if (state_dependent(p)) return fail(QR_ENOTSUP, "qr_solve_learned: state-dependent b2 or sigma_v");
    if (b->cos) return fail(QR_ENOTSUP, "qr_solve_learned: the cosine basis is not supported");
    if (p->driver == QR_F_PAPER) return fail(QR_ENOTSUP, "qr_solve_learned: the Sec. 5 driver is not supported");
    hipStream_t s = (hipStream_t)stream;
    const int d = p->d, N = p->N;
    const int64_t nt = o->train_points, nh = o->heldout_points;
    const int64_t chunk = std::min(M, kMlpChunk);
    if ((st = mlp_workspace(c, std::max(chunk, std::min<int64_t>(std::max<int64_t>(o->batch, nh), kMlpChunk)))))
        return st;
    // partial sums over the training pairs (moments) and the held-out pairs
    if ((st = ensure_partials(c, std::max(nt, nh)))) return st;
    if ((st = ensure(c, c->lx, sizeof(double) * (size_t)d * M, "cloud state"))) return st;
    if ((st = ensure(c, c->lh, sizeof(double) * (size_t)M, "source term"))) return st;
    if ((st = ensure(c, c->ly, sizeof(double) * (size_t)M, "expansion values"))) return st;
    // two spare floats: the buffer is cleared in whole doubles
    if ((st = ensure(c, c->lparams, sizeof(float) * ((size_t)N * kMlpParams + 2), "surrogate parameters"))) return st;
    for (Buf *bb : {&c->lgrad, &c->lm, &c->lv})
        if ((st = ensure(c, *bb, sizeof(float) * (size_t)(kMlpParams + 1), "Adam state"))) return st;
    if ((st = ensure(c, c->ltx, sizeof(double) * (size_t)d * nt, "training pairs"))) return st;
    if ((st = ensure(c, c->ltt, sizeof(double) * (size_t)nt, "training pairs"))) return st;
    if ((st = ensure(c, c->ltf, sizeof(float) * (size_t)nt, "training pairs"))) return st;
    if ((st = ensure(c, c->lff, sizeof(float) * (size_t)nt * kMlpIn, "training pairs"))) return st;
    if ((st = ensure(c, c->lhx, sizeof(double) * (size_t)d * nh, "held-out pairs"))) return st;
    if ((st = ensure(c, c->lht, sizeof(double) * (size_t)nh, "held-out pairs"))) return st;
    if ((st = ensure(c, c->lhf, sizeof(float) * (size_t)nh * kMlpIn, "held-out pairs"))) return st;
    if ((st = ensure(c, c->lhy, sizeof(float) * (size_t)nh, "held-out pairs"))) return st;

    std::vector<double> mu(N, 0.0), sg(N, 1.0);
    for (int j = 0; j < N; ++j) report[j] = qr_learn_report{0.0, 0.0, 0, 0, 0.0, 1.0, 0};
    const int db = dim_bucket(p->d, p->nbm);
    const int cap = depth_cap(b->max_nnz);
    const Walk W = make_walk(b->kind, b->level, b->d, b->code());
    double *x = (double *)c->lx.p, *H = (double *)c->lh.p, *y = (double *)c->ly.p;
    double *S = (double *)c->S.p;
    double2 *u = (double2 *)c->u.p;
    double2 *ai = (double2 *)c->alpha_int.p;
    float *params = (float *)c->lparams.p;
    const int64_t nf = 2 * b->nrep - 1;
    // parameters of time indices without a surrogate read as zero
    QR_HIP(launch_zero((double *)params, (int64_t)N * kMlpParams / 2 + 1, s), "zero_kernel");
    if ((st = numeric_clear(c, s))) return st;
    for (int32_t i = N - 1; i >= 0; --i) {
        bool any_used = false;
        for (int32_t j = i + 1; j < N; ++j) any_used = any_used || report[j].used;
        if (!any_used) {
            // every later time index uses its expansion: the fused path kernel of qr_solve
            if ((st = run_path(c, p, b, i, M, seed, ai, S, u, nullptr, s))) return st;
            if ((st = project_and_reduce(c, b, u, S, M, ai + (int64_t)i * b->ld(), alpha + (int64_t)i * nf, i, s)))
                return st;
            if (i >= 1 && o->epochs > 0) {
                if ((st = fit_surrogate(c, p, b, i, seed, o, params + (int64_t)i * kMlpParams, &mu[i], &sg[i],
                                        &report[i], s)))
                    return st;
                report[i].target_mean = mu[i];
                report[i].target_sd = sg[i];
            }
            continue;
        }
        QR_HIP(launch_sm_start(c->d_prob, b->law, i, M, seed, x, u, S, s), "sm_start_kernel");
        for (int32_t j = i; j < N; ++j) {
            QR_HIP(launch_sm_euler(db, c->d_prob, i, j, M, seed, x, H, s), "sm_euler_kernel");
            if (j + 1 == N) {
                QR_HIP(launch_sm_final(db, c->d_prob, M, x, H, S, s), "sm_final_kernel");
            } else if (report[j + 1].used) {
                const float *th = params + (int64_t)(j + 1) * kMlpParams;
                for (int64_t m0 = 0; m0 < M; m0 += kMlpChunk) {
                    const int64_t k = std::min(kMlpChunk, M - m0);
                    QR_HIP(launch_features(b->law, d, k, x + m0, M, (float *)c->mf.p, s), "features_kernel");
                    st = timed(c, 0, s, "mlp forward",
                               [&] { return mlp_fwd(c, th, k, (const float *)c->mf.p, (float *)c->my.p, s); });
                    if (st) return st;
                    QR_HIP(launch_sm_accum(c->d_prob, j, m0, k, nullptr, (const float *)c->my.p, mu[j + 1],
                                           sg[j + 1], H, S, s),
                           "sm_accum_kernel");
                }
            } else {
                const double2 *row = ai + (int64_t)(j + 1) * b->ld();
                st = timed(c, 0, s, "eval_kernel", [&] { return launch_eval(cap, false, W, row, x, M, y, nullptr, s); });
                if (st) return st;
                QR_HIP(launch_sm_accum(c->d_prob, j, 0, M, y, nullptr, 0.0, 1.0, H, S, s), "sm_accum_kernel");
            }
        }
        if ((st = project_and_reduce(c, b, u, S, M, ai + (int64_t)i * b->ld(), alpha + (int64_t)i * nf, i, s)))
            return st;
        if (i >= 1 && o->epochs > 0) {
            if ((st = fit_surrogate(c, p, b, i, seed, o, params + (int64_t)i * kMlpParams, &mu[i], &sg[i], &report[i],
                                    s)))
                return st;
            report[i].target_mean = mu[i];
            report[i].target_sd = sg[i];
        }
    }
    if (params_out)
        QR_HIP(hipMemcpyAsync(params_out, params, sizeof(float) * (size_t)N * kMlpParams, hipMemcpyDeviceToDevice, s),
               "hipMemcpyAsync(params)");
    return numeric_read(c, s, nullptr);
}

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------
namespace {
struct PassPlan {
    int32_t d = 0, level = 0;
    int64_t M = 0;
    qr_basis *walk = nullptr;  // sub-walk of the pass (contains every member's)
    int64_t off = 0;           // offset of its coefficient rows in the batch buffer (double2)
    std::vector<int32_t> members;
    bool shared = false;       // one projection of the pass for all members
    int32_t nsplit = 0;        // slices of the pass projection
    int64_t pps = 0;           // paths per slice
};

// Vector instructions per node and 128 paths of the two projections
// (measured at d = 6): the single-response kernel, and the pass kernel for
// all kBatchRT responses at once (its per-response cross-lane folds dominate).
constexpr double kProjCostOwn = 35.0, kProjCostPass = 126.0;

// Slices of a pass projection: as split_plan, for the pass tasks.
void pass_split_plan(const qr_basis *w, int64_t M, int32_t *nsplit, int64_t *pps) {
    const int64_t ntasks = std::max<int64_t>(1, (int64_t)w->ptasks.size());
    const int64_t group = (int64_t)kPassWaves * 64 * pass_paths_per_lane(w->d);
    int64_t want = (2048 + ntasks - 1) / ntasks;
    const int64_t maxs = std::max<int64_t>(1, (M + 4 * group - 1) / (4 * group));
    want = std::max<int64_t>(1, std::min(want, maxs));
    int64_t per = (M + want - 1) / want;
    per = (per + group - 1) / group * group;
    *pps = per;
    *nsplit = (int32_t)((M + per - 1) / per);
}
}  // namespace

namespace {
// A planned batched solve: each instance's own sub-walk, the passes, and the
// sizes of the buffers they need.
struct BatchPlan {
    std::vector<qr_basis *> own;
    std::vector<PassPlan> passes;
    int64_t Mmax = 0, total = 0, partial_max = 0;
    DevBatch hb{};
};
// Device buffers a batched solve reads and writes.
struct BatchBufs {
    const DevProblem *prob;
    const DevBatch *batch;
    double *S;
    double2 *u, *ab, *partial;
};
}  // namespace

// Validation, passes and device tables of a batched solve (host work and
// basis uploads only; no workspace is touched).
static qr_status plan_batched(qr_ctx *c, const qr_problem *p, qr_basis *b, int32_t R, const qr_instance *inst,
                              const double *alpha, BatchPlan &pl) {
    qr_status st;
    if ((st = check_problem(p, b))) return st;
    if ((st = check_basis_device(b))) return st;
    if (R < 1 || R > QR_MAX_BATCH) return fail(QR_EINVAL, "qr_solve_batched: R=%d outside [1,%d]", R, QR_MAX_BATCH);
    if (!inst || !alpha) return fail(QR_EINVAL, "qr_solve_batched: NULL instances or alpha");
    if (p->driver == QR_F_ZRAT)
        return fail(QR_ENOTSUP, "qr_solve_batched: the driver depends on z (gradients are not batched)");
    if (p->damping_q != 0.0) return fail(QR_ENOTSUP, "qr_solve_batched: damping exponent q must be 0");
    if (state_dependent(p)) return fail(QR_ENOTSUP, "qr_solve_batched: state-dependent b2 or sigma_v");
    if (b->cos) return fail(QR_ENOTSUP, "qr_solve_batched: the cosine basis is not supported");
    if (p->driver == QR_F_PAPER) return fail(QR_ENOTSUP, "qr_solve_batched: the Sec. 5 driver is not supported");
    for (int r = 0; r < R; ++r) {
        const qr_instance &I = inst[r];
        if (I.d < 1 || I.d > p->d) return fail(QR_EINVAL, "instance %d: d=%d outside [1,%d]", r, I.d, p->d);
        const int lmin = b->kind == QR_SET_TENSOR ? 0 : 1;
        if (I.level < lmin || I.level > b->level)
            return fail(QR_EINVAL, "instance %d: level=%d outside [%d,%d]", r, I.level, lmin, b->level);
        if ((st = check_M(I.M))) return st;
        if (!std::isfinite(I.f_a)) return fail(QR_EINVAL, "instance %d: f_a not finite", r);
        pl.Mmax = std::max(pl.Mmax, I.M);
    }

    // Passes of up to kBatchRT instances.  A pass walks the set of its first
    // member and simulates its cloud, so the cost of a pass is set by its
    // first member; greedily, the costliest remaining instance opens a pass
    // and takes along the costliest others that fit inside its envelope
    // (d, level and M no larger), which ride at no extra walk cost.
    std::vector<qr_basis *> &own = pl.own;
    own.assign(R, nullptr);
    std::vector<double> cost(R);
    for (int r = 0; r < R; ++r) {
        if ((st = sub_basis(b, inst[r].d, inst[r].level, &own[r]))) return st;
        cost[r] = (double)inst[r].M * (double)own[r]->nrep;
    }
    std::vector<int32_t> rem(R);
    for (int r = 0; r < R; ++r) rem[r] = r;
    std::stable_sort(rem.begin(), rem.end(), [&](int32_t a, int32_t q) { return cost[a] > cost[q]; });
    std::vector<PassPlan> &passes = pl.passes;
    while (!rem.empty()) {
        PassPlan P;
        const qr_instance &H = inst[rem[0]];
        P.d = H.d;
        P.level = H.level;
        P.M = H.M;
        std::vector<int32_t> left;
        for (int32_t r : rem) {
            const qr_instance &I = inst[r];
            if ((int)P.members.size() < kBatchRT && I.d <= P.d && I.level <= P.level && I.M <= P.M)
                P.members.push_back(r);
            else
                left.push_back(r);
        }
        rem.swap(left);
        passes.push_back(std::move(P));
    }
    for (PassPlan &P : passes) {
        if ((st = sub_basis(b, P.d, P.level, &P.walk))) return st;
        P.off = pl.total;
        pl.total += (int64_t)p->N * P.walk->ld() * kBatchRT;
    }
    if ((st = basis_on_device(b, c->dev))) return st;
    for (qr_basis *sb : b->subs)
        if ((st = basis_on_device(sb, c->dev))) return st;
    if (project_pass_lds_bytes(p->d) > (size_t)160 * 1024)
        return fail(QR_ENOTSUP, "qr_solve_batched: the pass projection's LDS exceeds a CU at d=%d", p->d);
    // The pass projection walks the pass's whole set over its whole cloud for
    // every member slot; it is taken where that costs less than the members'
    // own projections (members close to the pass's envelope), by the cost
    // model above.
    for (PassPlan &P : passes) {
        double own_cost = 0.0;
        for (int32_t r : P.members) own_cost += kProjCostOwn * (double)inst[r].M * (double)own[r]->nrep;
        P.shared = kProjCostPass * (double)P.M * (double)P.walk->nrep < own_cost;
        if (P.shared) {
            if ((st = basis_pass_tasks_on_device(P.walk))) return st;
            pass_split_plan(P.walk, P.M, &P.nsplit, &P.pps);
            pl.partial_max = std::max(pl.partial_max, (int64_t)P.nsplit * P.walk->nrep * kBatchRT);
        } else {
            for (int32_t r : P.members) {
                int32_t nsplit;
                int64_t pps;
                split_plan(own[r], inst[r].M, &nsplit, &pps);
                pl.partial_max = std::max(pl.partial_max, (int64_t)nsplit * own[r]->nrep);
            }
        }
    }
    // instance parameters in pass-slot order
    const int npass = (int)passes.size();
    for (int ps = 0; ps < npass; ++ps) {
        pl.hb.count[ps] = (int32_t)passes[ps].members.size();
        for (size_t k = 0; k < passes[ps].members.size(); ++k) {
            pl.hb.f_a[ps * kBatchRT + k] = inst[passes[ps].members[k]].f_a;
            pl.hb.m[ps * kBatchRT + k] = inst[passes[ps].members[k]].M;
        }
    }
    return QR_OK;
}

// Every launch of a planned batched solve, in order, on stream s (kernels
// only: it can be captured into a graph).
// Passes are independent of each other (own members, coefficients and output
// rows): pass ps runs on streams[ps % K] with that stream's buffers Bk[ps % K]
// (responses, phase factors, partial sums); all of a pass's steps are on one
// stream, in order.  streams[0] is the caller's stream; the others wait for
// it after the clearing and it waits for them at the end (the caller records
// the events).
static qr_status enqueue_batched(qr_ctx *c, const qr_problem *p, const qr_basis *b, int32_t R,
                                 const qr_instance *inst, const BatchPlan &pl, const BatchBufs *Bk,
                                 const hipStream_t *streams, int K, uint64_t seed, double *alpha) {
    qr_status st;
    const int64_t nf = 2 * b->nrep - 1;
    hipStream_t s0 = streams[0];
    QR_HIP(launch_zero(alpha, (int64_t)R * p->N * nf, s0), "zero_kernel");
    QR_HIP(launch_zero((double *)Bk[0].ab, 2 * pl.total, s0), "zero_kernel");
    const int db = dim_bucket(p->d, p->nbm);
    if ((st = numeric_clear(c, s0))) return st;
    if (K > 1) {
        QR_HIP(hipEventRecord(c->bfork, s0), "hipEventRecord");
        for (int k = 1; k < K; ++k) QR_HIP(hipStreamWaitEvent(streams[k], c->bfork, 0), "hipStreamWaitEvent");
    }
    const int npass = (int)pl.passes.size();
    for (int32_t i = p->N - 1; i >= 0; --i) {
        for (int ps = 0; ps < npass; ++ps) {
            const PassPlan &P = pl.passes[ps];
            const BatchBufs &B = Bk[ps % K];
            hipStream_t s = streams[ps % K];
            const int64_t ld = P.walk->ld();
            BatchArgs a{B.prob, p->d, B.batch, ps, make_walk(b->kind, P.level, P.d, b->law), i, P.M, seed,
                        B.ab + P.off, ld, B.S, B.u};
            st = timed(c, 0, s, "batched_path_kernel",
                       [&] { return launch_batched_path(db, depth_cap(P.walk->max_nnz), a, s); });
            if (st) return st;
            if (P.shared) {
                // one projection of the pass for all its members (the shared walk
                // and phase factors), then each member's own coefficients from it
                st = timed(c, 1, s, "project_pass_kernel", [&] {
                    return launch_project_pass(depth_cap(P.walk->max_nnz), make_walk(b->kind, P.level, P.d, b->code()),
                                               B.u, P.M, B.S, P.M, B.batch->m + (int64_t)ps * kBatchRT, P.pps,
                                               (int32_t)P.walk->ptasks.size(), P.nsplit, P.walk->d_ptasks,
                                               P.walk->d_pitems, B.partial, P.walk->nrep, s);
                });
                if (st) return st;
            }
            for (size_t k = 0; k < P.members.size(); ++k) {
                const int32_t r = P.members[k];
                const qr_basis *ob = pl.own[r];
                const int64_t Mr = inst[r].M;
                int32_t nsplit = P.nsplit;
                if (!P.shared) {
                    // the member's own projection: its set on its own cloud
                    int64_t pps;
                    split_plan(ob, Mr, &nsplit, &pps);
                    st = timed(c, 1, s, "project_kernel", [&] {
                        return launch_project(depth_cap(ob->max_nnz), make_walk(b->kind, ob->level, ob->d, b->code()),
                                              B.u, P.M, B.S + (int64_t)k * P.M, Mr, pps, (int32_t)ob->tasks.size(),
                                              nsplit, ob->d_tasks, ob->d_items, ob->task_max, B.partial, ob->nrep, s);
                    });
                    if (st) return st;
                }
                st = timed(c, 2, s, "reduce_batched_kernel", [&] {
                    return launch_reduce_batched(B.partial, nsplit, ob->nrep, P.shared ? P.walk->nrep : ob->nrep,
                                                 P.shared ? kBatchRT : 1, (double)Mr, ob->d_ft, b->d_canon_of_trav,
                                                 P.walk->d_inv, B.ab + P.off + (int64_t)i * ld * kBatchRT, (int32_t)k,
                                                 alpha + ((int64_t)r * p->N + i) * nf, c->d_bad, i, s);
                });
                if (st) return st;
            }
        }
    }
    if (K > 1) {
        for (int k = 1; k < K; ++k) {
            QR_HIP(hipEventRecord(c->bjoin[k - 1], streams[k]), "hipEventRecord");
            QR_HIP(hipStreamWaitEvent(s0, c->bjoin[k - 1], 0), "hipStreamWaitEvent");
        }
    }
    return QR_OK;
}

extern "C" qr_status qr_solve_batched(qr_ctx *c, const qr_problem *p, const qr_basis *bc, int32_t R,
                                      const qr_instance *inst, uint64_t seed, double *alpha,
                                      void *stream) {
    qr_basis *b = const_cast<qr_basis *>(bc);
    qr_status st = begin(c, stream);
    if (st) return st;
    BatchPlan pl;
    if ((st = plan_batched(c, p, b, R, inst, alpha, pl))) return st;
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_problem(c, p, b->law, s))) return st;
    if ((st = ensure(c, c->S, sizeof(double) * (size_t)pl.Mmax * kBatchRT, "S"))) return st;
    if ((st = ensure(c, c->u, sizeof(double2) * (size_t)pl.Mmax * p->d, "phase factors"))) return st;
    if ((st = ensure(c, c->alpha_b, sizeof(double2) * (size_t)pl.total, "batch coefficients"))) return st;
    if ((st = ensure(c, c->partial, sizeof(double2) * (size_t)pl.partial_max, "partial"))) return st;
    if (!c->d_batch) QR_HIP(hipMalloc(&c->d_batch, sizeof(DevBatch)), "hipMalloc(batch)");
    // queued kernels may read the old instance parameters (on this stream or,
    // from an earlier batched solve, on the context's side streams)
    QR_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (int k = 0; k < kBatchStreams - 1; ++k)
        if (c->bstream[k]) QR_HIP(hipStreamSynchronize(c->bstream[k]), "hipStreamSynchronize");
    QR_HIP(hipMemcpy(c->d_batch, &pl.hb, sizeof pl.hb, hipMemcpyHostToDevice), "hipMemcpy(batch)");
    // one stream per pass up to kBatchStreams, each with its own buffers
    const int K = std::max(1, std::min<int>(kBatchStreams, (int)pl.passes.size()));
    BatchBufs Bk[kBatchStreams];
    hipStream_t ss[kBatchStreams] = {s};
    Bk[0] = BatchBufs{c->d_prob, c->d_batch, (double *)c->S.p, (double2 *)c->u.p, (double2 *)c->alpha_b.p,
                      (double2 *)c->partial.p};
    for (int k = 1; k < K; ++k) {
        if (!c->bstream[k - 1]) {
            QR_HIP(hipStreamCreateWithFlags(&c->bstream[k - 1], hipStreamNonBlocking), "hipStreamCreate");
            QR_HIP(hipEventCreateWithFlags(&c->bjoin[k - 1], hipEventDisableTiming), "hipEventCreate");
        }
        if ((st = ensure(c, c->bS[k - 1], sizeof(double) * (size_t)pl.Mmax * kBatchRT, "S"))) return st;
        if ((st = ensure(c, c->bu[k - 1], sizeof(double2) * (size_t)pl.Mmax * p->d, "phase factors"))) return st;
        if ((st = ensure(c, c->bpart[k - 1], sizeof(double2) * (size_t)pl.partial_max, "partial"))) return st;
        ss[k] = c->bstream[k - 1];
        Bk[k] = BatchBufs{c->d_prob, c->d_batch, (double *)c->bS[k - 1].p, (double2 *)c->bu[k - 1].p,
                          (double2 *)c->alpha_b.p, (double2 *)c->bpart[k - 1].p};
    }
    if (K > 1 && !c->bfork) QR_HIP(hipEventCreateWithFlags(&c->bfork, hipEventDisableTiming), "hipEventCreate");
    if ((st = enqueue_batched(c, p, b, R, inst, pl, Bk, ss, K, seed, alpha))) return st;
    return numeric_read(c, s, nullptr);
}

// A batched solve captured into a HIP graph, with device buffers of its own
// (problem, instance parameters, responses, phase factors, coefficient and
// partial-sum workspace), so that later calls on the context cannot move
// what the graph reads.
struct qr_batch_graph {
    qr_ctx *ctx = nullptr;
    int dev = -1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *mem[6] = {};
};

extern "C" void qr_batch_graph_destroy(qr_batch_graph *gr) {
    if (!gr) return;
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(gr->dev);
    hipDeviceSynchronize();
    if (gr->exec) hipGraphExecDestroy(gr->exec);
    if (gr->graph) hipGraphDestroy(gr->graph);
    for (void *m : gr->mem) hipFree(m);
    hipSetDevice(cur);
    delete gr;
}

extern "C" qr_status qr_batch_graph_create(qr_ctx *c, const qr_problem *p, const qr_basis *bc, int32_t R,
                                           const qr_instance *inst, uint64_t seed, double *alpha, void *stream,
                                           qr_batch_graph **out) {
    if (!out) return fail(QR_EINVAL, "qr_batch_graph_create: out is NULL");
    *out = nullptr;
    if (!stream) return fail(QR_EINVAL, "qr_batch_graph_create: capture needs a stream other than the null stream");
    qr_basis *b = const_cast<qr_basis *>(bc);
    qr_status st = begin(c, stream);
    if (st) return st;
    BatchPlan pl;
    if ((st = plan_batched(c, p, b, R, inst, alpha, pl))) return st;
    hipStream_t s = (hipStream_t)stream;
    qr_batch_graph *gr = new (std::nothrow) qr_batch_graph();
    if (!gr) return fail(QR_ENOMEM, "qr_batch_graph_create: out of host memory");
    gr->ctx = c;
    gr->dev = c->dev;
    const size_t bytes[6] = {sizeof(DevProblem), sizeof(DevBatch), sizeof(double) * (size_t)pl.Mmax * kBatchRT,
                             sizeof(double2) * (size_t)pl.Mmax * p->d, sizeof(double2) * (size_t)pl.total,
                             sizeof(double2) * (size_t)std::max<int64_t>(pl.partial_max, 1)};
    for (int k = 0; k < 6; ++k) {
        if (hipMalloc(&gr->mem[k], bytes[k]) != hipSuccess) {
            hipGetLastError();
            qr_batch_graph_destroy(gr);
            return fail(QR_ENOMEM, "qr_batch_graph_create: cannot allocate %zu bytes", bytes[k]);
        }
    }
    const DevProblem hp = make_dev_problem(p, b->law);
    if (hipMemcpy(gr->mem[0], &hp, sizeof hp, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(gr->mem[1], &pl.hb, sizeof pl.hb, hipMemcpyHostToDevice) != hipSuccess) {
        qr_batch_graph_destroy(gr);
        return fail(QR_EDEVICE, "qr_batch_graph_create: upload failed");
    }
    const BatchBufs B{(const DevProblem *)gr->mem[0], (const DevBatch *)gr->mem[1], (double *)gr->mem[2],
                      (double2 *)gr->mem[3], (double2 *)gr->mem[4], (double2 *)gr->mem[5]};
    // one eager solve first (kernel attributes set, errors reported eagerly);
    // then the same launches captured
    if ((st = enqueue_batched(c, p, b, R, inst, pl, &B, &s, 1, seed, alpha))) {
        qr_batch_graph_destroy(gr);
        return st;
    }
    const bool timing = c->timing;
    c->timing = false;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = enqueue_batched(c, p, b, R, inst, pl, &B, &s, 1, seed, alpha);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(s, &g);
        gr->graph = g;
        if (!st && e2 != hipSuccess) e = e2;
    }
    c->timing = timing;
    if (!st && e == hipSuccess) e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
    if (st || e != hipSuccess) {
        hipGetLastError();
        qr_batch_graph_destroy(gr);
        return st ? st : fail(QR_EDEVICE, "qr_batch_graph_create: capture failed (%s)", hipGetErrorString(e));
    }
    *out = gr;
    return QR_OK;
}

extern "C" qr_status qr_batch_graph_launch(qr_batch_graph *gr, void *stream) {
    if (!gr) return fail(QR_EINVAL, "qr_batch_graph_launch: graph is NULL");
    qr_status st = begin(gr->ctx, stream);
    if (st) return st;
    QR_HIP(hipGraphLaunch(gr->exec, (hipStream_t)stream), "hipGraphLaunch");
    return QR_OK;
}

// ---------------------------------------------------------------------------
// host mirrors of the scalar device routines
// ---------------------------------------------------------------------------
extern "C" double qr_host_uniform(uint64_t seed, uint32_t stream_id, uint64_t m, uint32_t i, uint32_t r) {
    return uniform_at(seed, stream_id, m, i, r);
}

extern "C" double qr_host_norm_icdf(double u) { return norm_icdf(u); }

extern "C" void qr_host_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const U4 w = philox4x32_10(U4{ctr[0], ctr[1], ctr[2], ctr[3]}, key[0], key[1]);
    out[0] = w.x;
    out[1] = w.y;
    out[2] = w.z;
    out[3] = w.w;
}
