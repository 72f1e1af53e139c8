// qrmc_factored.hip -- factored form of the expansion evaluation (layout,
// coefficient packing and the reduced-precision path kernel built on it).
#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

#include "qrmc_device.h"
#include "qrmc_factored.h"
#include "qrmc_kernels.h"

namespace qrmc {

// ---------------------------------------------------------------------------
// Host: the staircase layout of an index set for a split dA | d - dA
// ---------------------------------------------------------------------------
static int32_t part_weight(int32_t kind, const int32_t *v, int n) {
    int32_t w = 1;
    for (int l = 0; l < n; ++l) {
        const int32_t m = std::abs(v[l]);
        if (kind == QR_SET_HC_MAX)
            w *= std::max(1, m);
        else if (kind == QR_SET_HC_1P)
            w *= 1 + m;
        else if (kind == QR_SET_TOTAL)
            w += m;
    }
    return w;
}

static bool make_code(const int32_t *v, int n, int l0, int32_t TS, FacCode *c, int *nnz) {
    *c = FacCode{};
    int t = 0;
    for (int l = 0; l < n; ++l) {
        if (v[l] == 0) continue;
        if (t == kFacNnz) return false;
        const int32_t idx = (l0 + l) * TS + std::abs(v[l]);
        c->e[t++] = (int16_t)(v[l] > 0 ? idx : -idx);
    }
    *nnz = t;
    return true;
}

static bool layout_for_split(int32_t d, int32_t kind, const int32_t *canon, int64_t nrep, int32_t dA,
                             int32_t TS, int32_t max_nkb, FactorLayout *out) {
    const int dB = d - dA;
    using Key = std::vector<int32_t>;
    // columns: every B-part of the set (both signs), sorted by weight, then lexicographically
    std::map<Key, int32_t> colpos;
    for (int64_t r = 0; r < nrep; ++r) {
        Key kb(canon + r * d + dA, canon + r * d + d);
        colpos.emplace(kb, 0);
        for (auto &x : kb) x = -x;
        colpos.emplace(kb, 0);
    }
    std::vector<Key> cols;
    cols.reserve(colpos.size());
    for (auto &kv : colpos) cols.push_back(kv.first);
    std::stable_sort(cols.begin(), cols.end(), [&](const Key &a, const Key &b) {
        return part_weight(kind, a.data(), dB) < part_weight(kind, b.data(), dB);
    });
    if ((int64_t)cols.size() > (int64_t)max_nkb * kFacCols) return false;
    for (size_t c = 0; c < cols.size(); ++c) colpos[cols[c]] = (int32_t)c;
    // rows: the zero A-part, then the A-parts of the representatives (first non-zero > 0)
    std::map<Key, int32_t> rowid;
    std::vector<Key> rowkeys;
    rowid.emplace(Key(dA, 0), 0);
    rowkeys.push_back(Key(dA, 0));
    struct Entry {
        int32_t col;
        int32_t rep;
    };
    std::vector<std::vector<Entry>> entries(1);
    for (int64_t r = 0; r < nrep; ++r) {
        Key ka(canon + r * d, canon + r * d + dA);
        auto it = rowid.find(ka);
        int32_t row;
        if (it == rowid.end()) {
            row = (int32_t)rowkeys.size();
            rowid.emplace(ka, row);
            rowkeys.push_back(ka);
            entries.emplace_back();
        } else {
            row = it->second;
        }
        Key kb(canon + r * d + dA, canon + r * d + d);
        entries[row].push_back(Entry{colpos[kb], (int32_t)r});
    }
    const int32_t nrow = (int32_t)rowkeys.size();
    std::vector<int32_t> len(nrow, 0), nnz(nrow, 0);
    std::vector<FacCode> rcode(nrow);
    for (int32_t r = 0; r < nrow; ++r) {
        for (const Entry &e : entries[r]) len[r] = std::max(len[r], e.col + 1);
        // the columns of a row other than row 0 are a prefix of the weight order
        if (r > 0 && (int32_t)entries[r].size() != len[r]) return false;
        if (!make_code(rowkeys[r].data(), dA, 0, TS, &rcode[r], &nnz[r])) return false;
    }
    // row order: row 0 first, then longer rows first, then more factors first
    std::vector<int32_t> order(nrow);
    for (int32_t r = 0; r < nrow; ++r) order[r] = r;
    std::stable_sort(order.begin() + 1, order.end(), [&](int32_t a, int32_t b) {
        if (len[a] != len[b]) return len[a] > len[b];
        return nnz[a] > nnz[b];
    });
    FactorLayout L;
    L.d = d;
    L.dA = dA;
    L.TS = TS;
    L.nrow = nrow;
    L.nrt = (nrow + kFacRows - 1) / kFacRows;
    L.ncol = (int32_t)cols.size();
    L.nkb = (L.ncol + kFacCols - 1) / kFacCols;
    L.cols.assign((size_t)L.nkb * kFacCols, FacCode{});
    L.colnnz.assign(L.nkb, 0);
    for (int32_t c = 0; c < L.ncol; ++c) {
        int n = 0;
        if (!make_code(cols[c].data(), dB, dA, TS, &L.cols[c], &n)) return false;
        L.colnnz[c / kFacCols] = std::max(L.colnnz[c / kFacCols], n);
    }
    L.rows.assign((size_t)L.nrt * kFacRows, FacCode{});
    L.tiles.resize(L.nrt);
    int64_t off = 0;
    double cost = 0.0;
    for (int32_t t = 0; t < L.nrt; ++t) {
        FacTile ft{0, 0, off};
        for (int rr = 0; rr < kFacRows; ++rr) {
            const int32_t q = t * kFacRows + rr;
            if (q >= nrow) break;
            const int32_t r = order[q];
            L.rows[q] = rcode[r];
            ft.nkb = std::max(ft.nkb, (len[r] + kFacCols - 1) / kFacCols);
            ft.nnz = std::max(ft.nnz, nnz[r]);
        }
        ft.nkb = std::max(ft.nkb, 1);
        L.tiles[t] = ft;
        off += ft.nkb;
        // cycles of one tile for 16 paths: the two rows' factor products and the
        // epilogue on the vector ALU (4 cycles per instruction), 16 per product block
        cost += 4.0 * (20 + 14 * ft.nnz) + 16.0 * ft.nkb;
    }
    for (int32_t k = 0; k < L.nkb; ++k) cost += 4.0 * 4 * (6 + 7 * L.colnnz[k]);
    L.nblocks = off;
    L.ent.assign((size_t)L.nblocks * kFacRows * kFacCols, -1);
    std::vector<char> seen(nrep, 0);
    for (int32_t t = 0; t < L.nrt; ++t) {
        for (int rr = 0; rr < kFacRows; ++rr) {
            const int32_t q = t * kFacRows + rr;
            if (q >= nrow) break;
            for (const Entry &e : entries[order[q]]) {
                const int32_t kb = e.col / kFacCols, cc = e.col % kFacCols;
                if (kb >= L.tiles[t].nkb) return false;
                const int64_t b = L.tiles[t].off + kb;
                L.ent[(b * kFacRows + rr) * kFacCols + cc] = e.rep;
                if (seen[e.rep]++) return false;
            }
        }
    }
    for (int64_t r = 0; r < nrep; ++r)
        if (!seen[r]) return false;
    L.cost = cost;
    *out = std::move(L);
    return true;
}

bool build_factor_layout(int32_t d, int32_t kind, int32_t level, const int32_t *canon, int64_t nrep,
                         int32_t max_nkb, FactorLayout *out) {
    (void)level;
    int32_t mmax = 0;
    for (int64_t v = 0; v < nrep * d; ++v) mmax = std::max(mmax, std::abs(canon[v]));
    const int32_t TS = mmax + 1;
    bool found = false;
    for (int32_t dA = 0; dA < std::max(d, 1); ++dA) {
        FactorLayout L;
        if (!layout_for_split(d, kind, canon, nrep, dA, TS, max_nkb, &L)) continue;
        if (!found || L.cost < out->cost) {
            *out = std::move(L);
            found = true;
        }
    }
    return found;
}

// Projection tasks: consecutive row tiles whose K-blocks fit one of the
// templates (R row tiles x NKBT K-blocks, R NKBT = 8 accumulator blocks per
// wave); a row tile of more than 8 K-blocks is cut into tasks of 8 K-blocks
// (kb0 = 0, 8, ...) of the last template.  Row tiles are in order of
// non-increasing K-block count, so a task's first tile has the most.
static const int kTmplR[kFacTemplates] = {8, 4, 2, 1};
static const int kTmplK[kFacTemplates] = {1, 2, 4, 8};

void build_fac_tasks(const FactorLayout &L, std::vector<FacTask> tasks[kFacTemplates]) {
    for (int t = 0; t < kFacTemplates; ++t) tasks[t].clear();
    const int last = kFacTemplates - 1;
    int32_t rt = 0;
    while (rt < L.nrt) {
        const int32_t k = L.tiles[rt].nkb;
        if (k > kTmplK[last]) {
            for (int32_t kb0 = 0; kb0 < k; kb0 += kTmplK[last]) tasks[last].push_back(FacTask{rt, 1, last, kb0});
            ++rt;
            continue;
        }
        int t = 0;
        while (kTmplK[t] < k) ++t;
        int32_t n = 0;
        while (n < kTmplR[t] && rt + n < L.nrt) ++n;
        tasks[t].push_back(FacTask{rt, n, t, 0});
        rt += n;
    }
}

// ---------------------------------------------------------------------------
// Device
// ---------------------------------------------------------------------------
// Tables that no kernel writes while it runs, read through the constant
// address space so that wave-uniform reads become scalar loads.
#define CONSTANT_AS __attribute__((address_space(4)))
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <int PREC>
__device__ __forceinline__ f32x4 fac_mfma(uint4 a, uint4 b, f32x4 c) {
    if constexpr (PREC == QR_PREC_BF16)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                        __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                       __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

// Coefficient blocks for v_mfma_f32_16x16x32: lane l holds A[l % 16][8 (l / 16) .. + 7].
// Real row 2 rr + 0 gives Re C (entries beta_r, -beta_i against EB_r, EB_i),
// real row 2 rr + 1 gives Im C (beta_i, beta_r); K element 8 g + 2 q + {0, 1} is
// (EB_r, EB_i) of complex column 4 g + q of the block.
template <int PREC>
__global__ void fac_pack_kernel(const double *__restrict__ alpha, const int32_t *__restrict__ ent,
                                int64_t nblocks, uint4 *__restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nblocks * 64) return;
    const int64_t b = idx / 64;
    const int lane = (int)(idx % 64);
    const int rr = (lane & 15) >> 1, part = lane & 1, g = lane >> 4;
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int32_t rep = ent[(b * kFacRows + rr) * kFacCols + 4 * g + q];
        double br = 0.0, bi = 0.0;
        if (rep == 0) {
            br = alpha[0];
        } else if (rep > 0) {
            br = M_SQRT2 * alpha[2 * (int64_t)rep - 1];
            bi = -M_SQRT2 * alpha[2 * (int64_t)rep];
        }
        w[q] = part == 0 ? pack16x2<PREC>((float)br, (float)-bi) : pack16x2<PREC>((float)bi, (float)br);
    }
    out[idx] = make_uint4(w[0], w[1], w[2], w[3]);
}

// a row tile's record (the tile table is read-only while kernels run: read
// through the constant address space, wave-uniform, as scalar loads)
__device__ __forceinline__ FacTile fac_tile(const FacTile *t, int i) {
    const FacTile CONSTANT_AS *c = (const FacTile CONSTANT_AS *)t;
    FacTile r;
    r.nkb = c[i].nkb;
    r.nnz = c[i].nnz;
    r.off = c[i].off;
    return r;
}

// the value of the partner lane (lane ^ 1), by a DPP quad permutation
__device__ __forceinline__ float2 swap_pair(float2 v) {
    constexpr int kQuadSwap = 0xB1;  // quad_perm [1, 0, 3, 2]
    const int x = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v.x), kQuadSwap, 0xf, 0xf, true);
    const int y = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v.y), kQuadSwap, 0xf, 0xf, true);
    return make_float2(__builtin_bit_cast(float, x), __builtin_bit_cast(float, y));
}

__device__ __forceinline__ float2 fcmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}

// table entry of a code element: e^{2 pi i m u_l} at T[l TS + m], conjugated for e < 0
__device__ __forceinline__ float2 fac_tab(const float2 *T, int e) {
    const float2 v = T[e < 0 ? -e : e];
    return make_float2(v.x, e < 0 ? -v.y : v.y);
}

// product of the first nnz factors of a code (nnz wave-uniform; an unused
// element 0 reads T[0] = 1)
__device__ __forceinline__ float2 fac_value(const float2 *T, const uint4 c, int nnz) {
    const uint32_t wd[4] = {c.x, c.y, c.z, c.w};
    float2 v = fac_tab(T, (int)(int16_t)(wd[0] & 0xffffu));
#pragma unroll
    for (int t = 1; t < kFacNnz; ++t)
        if (t < nnz) v = fcmul(v, fac_tab(T, (int)(int16_t)(wd[t >> 1] >> (16 * (t & 1)))));
    return v;
}

// acc += blocks KB.. of a row tile (the first nk of NKB; nk wave-uniform): a
// chain of branches that leaves at the tile's last block, each block's B
// operand a register of the cache (constant index)
template <int NKB, int PREC, int KB>
__device__ __forceinline__ void fac_blocks(f32x4 &acc, const uint4 *cb, const uint4 (&eb)[NKB], int nk) {
    if constexpr (KB < NKB) {
        if (KB < nk) {
            acc = fac_mfma<PREC>(cb[KB * 64], eb[KB], acc);
            fac_blocks<NKB, PREC, KB + 1>(acc, cb, eb, nk);
        }
    }
}

int fac_waves(int32_t d, int32_t TS) {
    const size_t per_wave = (size_t)kFacPaths * fac_stride(d, TS) * sizeof(float2);
    for (int w = 4; w > 1; w /= 2)
        if (per_wave * w <= 64 * 1024) return w;
    return 1;
}

// ---------------------------------------------------------------------------
// fac_path_kernel: backward iteration i of Algorithm 1 in the reduced-precision
// form, the expansion evaluated as a product over paths.  A wave carries 16
// paths: lane l holds path l % 16 (the product's column) and works on the
// product rows of its group l / 16; the path simulation itself is repeated in
// the four lanes of a path (its cost is a few percent of the evaluation).
// Per evaluation point: the lanes of a path write its tables
// e^{2 pi i m u_l} (FP64 phase, recurrence in m in FP64, stored FP32) for the
// coordinates l = lane group mod 4; EB of every column is formed once and
// kept as the product's B operands; each row tile is then one product block
// per K-block, followed by EA of the lane's two rows and Re(EA C).
// ---------------------------------------------------------------------------
#ifndef QRMC_FAC_WAVES_PER_EU
#define QRMC_FAC_WAVES_PER_EU 3
#endif
template <int DB, int NKB, int PREC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QRMC_FAC_WAVES_PER_EU)))
void fac_path_kernel(const DevProblem *__restrict__ P0, const FacDev F,
                                                       const int32_t i, const int64_t M, const uint64_t seed,
                                                       const uint4 *__restrict__ coef, double *__restrict__ S_out,
                                                       double2 *__restrict__ e_out) {
    extern __shared__ float2 ftab[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, p = lane & 15;
    const int d = P0->d, nbm = P0->nbm, N = P0->N;
    const int TS = F.TS;
    float2 *T = ftab + (size_t)(wv * kFacPaths + p) * fac_stride(d, TS);
    const int64_t m = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wv) * kFacPaths + p;
    const int nu = __builtin_amdgcn_readfirstlane(P0->nu);

    double x[DB];
    {
        PhiloxStream rs(seed, 0u, (uint64_t)m, (uint32_t)i, 0u);
#pragma unroll
        for (int l = 0; l < DB; ++l) {
            x[l] = 0.0;
            if (l < d) {
                x[l] = nl_icdf_u(nu, rs.next());
                if (g == 0 && m < M && e_out) e_out[l * M + m] = nl_unit_phase_u(nu, x[l]);
            }
        }
    }
    double S = 0.0;
    for (int j = i; j < N; ++j) {
        const DevProblem *__restrict__ Pj = P0;
        const double tj = Pj->t[j];
        const double dt = Pj->t[j + 1] - tj;
        const double sq = sqrt(dt);
        const double2 hu = h_source<DB>(Pj, tj, x, d);
        const double hj = hu.x, uj = hu.y;
        {
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
        }
        double y;
        if (j + 1 < N) {
            // tables of coordinates l = 4 s + g
#pragma unroll
            for (int s4 = 0; s4 < (DB + 3) / 4; ++s4) {
                // lane group g takes coordinate 4 s4 + g: the candidates pass
                // through an empty asm so that the choice stays a register
                // select (folded into a load with a lane-dependent index, it
                // would move the whole state x to scratch memory)
                double c0 = x[4 * s4];
                double c1 = 4 * s4 + 1 < DB ? x[4 * s4 + 1] : 0.0;
                double c2 = 4 * s4 + 2 < DB ? x[4 * s4 + 2] : 0.0;
                double c3 = 4 * s4 + 3 < DB ? x[4 * s4 + 3] : 0.0;
                asm("" : "+v"(c0), "+v"(c1), "+v"(c2), "+v"(c3));
                const double xs = g == 0 ? c0 : (g == 1 ? c1 : (g == 2 ? c2 : c3));
                const int l = 4 * s4 + g;
                if (l < d) {
                    const double2 e1 = nl_unit_phase_u(nu, xs);
                    double2 v = make_double2(1.0, 0.0);
                    float2 *Tl = T + l * TS;
                    Tl[0] = make_float2(1.0f, 0.0f);
                    for (int mm = 1; mm < TS; ++mm) {
                        v = make_double2(fma(v.x, e1.x, -(v.y * e1.y)), fma(v.x, e1.y, v.y * e1.x));
                        Tl[mm] = make_float2((float)v.x, (float)v.y);
                    }
                }
            }
            wave_sync();
            // B operands: EB of complex columns 16 kb + 4 g + q at this lane's path
            uint4 eb[NKB];
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb) {
                eb[kb] = make_uint4(0, 0, 0, 0);
                if (kb < F.nkb) {
                    const int nz = ((const int32_t CONSTANT_AS *)F.colnnz)[kb];
                    uint32_t w[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float2 v = fac_value(T, *reinterpret_cast<const uint4 *>(F.cols + kb * kFacCols + 4 * g + q), nz);
                        w[q] = pack16x2<PREC>(v.x, v.y);
                    }
                    eb[kb] = make_uint4(w[0], w[1], w[2], w[3]);
                }
            }
            const uint4 *cj = coef + (size_t)(j + 1) * F.nblocks * 64 + lane;
            const uint4 *rcode = reinterpret_cast<const uint4 *>(F.rows) + 2 * g;
            float yp = 0.0f;
            // the first coefficient block and the lane's two row codes of a tile
            // are loaded one tile ahead, so their latency overlaps the current tile
            FacTile tl = fac_tile(F.tiles, 0);
            FacTile tn = fac_tile(F.tiles, F.nrt > 1 ? 1 : 0);
            uint4 a0 = cj[tl.off * 64];
            uint4 c0 = rcode[0], c1 = rcode[1];
#pragma unroll 1
            for (int rt = 0; rt < F.nrt; ++rt) {
                const int rn = rt + 1 < F.nrt ? rt + 1 : rt;
                const FacTile tnn = fac_tile(F.tiles, rt + 2 < F.nrt ? rt + 2 : rn);
                const uint4 a0n = cj[tn.off * 64];
                const uint4 c0n = rcode[rn * kFacRows], c1n = rcode[rn * kFacRows + 1];
                f32x4 acc = fac_mfma<PREC>(a0, eb[0], f32x4{0.0f, 0.0f, 0.0f, 0.0f});
                if (tl.nkb > 1) fac_blocks<NKB, PREC, 1>(acc, cj + tl.off * 64, eb, tl.nkb);
                const float2 ea0 = fac_value(T, c0, tl.nnz);
                const float2 ea1 = fac_value(T, c1, tl.nnz);
                yp = fmaf(ea0.x, acc[0], yp);
                yp = fmaf(-ea0.y, acc[1], yp);
                yp = fmaf(ea1.x, acc[2], yp);
                yp = fmaf(-ea1.y, acc[3], yp);
                tl = tn;
                tn = tnn;
                a0 = a0n;
                c0 = c0n;
                c1 = c1n;
            }
            yp += __shfl_xor(yp, 16);
            yp += __shfl_xor(yp, 32);
            y = (double)yp;
            wave_sync();
        } else {
            y = g_term<DB>(Pj, x, d, nullptr);
        }
        const double yc = clamp_abs(y, Pj->clamp);
        S = fma(fnl(Pj, yc, 0.0, uj) + hj, dt, S);
    }
    S += g_term<DB>(P0, x, d, nullptr);
    if (g == 0 && m < M) S_out[m] = S;
}

// ---------------------------------------------------------------------------
// fac_project_kernel: alpha of eq (Aqi:bar:M) in the factored layout.  The
// entry (r, c) of a coefficient block is Z[r][c] = sum_p S_p EA_p(r) EB_p(c);
// for a block of 16 paths this is one product per coefficient block with
//   A (16 real rows x 32 K): row 2 rr + 0 = (W_r, -W_i), row 2 rr + 1 = (W_i, W_r)
//     over the paths (K element 8 g + 2 t + {0,1} = path 4 g + t), W = S EA(rr);
//   B (32 K x 16 columns): (EB_r, EB_i) of column cc at path 4 g + t;
//   D: Re Z and Im Z of rows 2 g, 2 g + 1 (lane l holds column l % 16).
// A wave (one "unit") accumulates, in FP32, the blocks of a task (R row tiles
// of at most NKBT K-blocks each) over its share of the paths and writes them
// as a partial sum; fac_reduce_kernel adds the units in a fixed order in FP64.
// The per-path tables come from the start points' phase factors e^{2 pi i u_l}
// by the FP64 recurrence in m, as along the paths.
// ---------------------------------------------------------------------------
template <int R, int NKBT, int PREC>
__global__ __launch_bounds__(256) void fac_project_kernel(const FacDev F, const FacTask *__restrict__ tasks,
                                                          const double2 *__restrict__ e, const double *__restrict__ S,
                                                          const int64_t M, const int64_t per_unit,
                                                          const int32_t units, float *__restrict__ partial) {
    extern __shared__ float2 ftab[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, q = lane & 15;
    const int d = F.d, TS = F.TS;
    const int stride = fac_stride(d, TS);
    float2 *Tw = ftab + (size_t)wv * kFacPaths * stride;
    const FacTask task = tasks[blockIdx.x];
    const int32_t unit = blockIdx.y * (blockDim.x >> 6) + wv;
    // K-blocks kb0 .. kb0 + nkb[r] - 1 of row tile rt0 + r
    const int kb0 = task.kb0;
    int nkb[R];
    int nnz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        nkb[r] = 0;
        nnz[r] = 0;
        if (r < task.R) {
            const FacTile tl = fac_tile(F.tiles, task.rt0 + r);
            nkb[r] = tl.nkb - kb0 < NKBT ? tl.nkb - kb0 : NKBT;
            nnz[r] = tl.nnz;
        }
    }
    f32x4 acc[R][NKBT];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int kb = 0; kb < NKBT; ++kb) acc[r][kb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int64_t p0 = (int64_t)unit * per_unit;
    const int64_t p1 = p0 + per_unit < M ? p0 + per_unit : M;
    for (int64_t k0 = p0; k0 < p1; k0 += kFacPaths) {
        // tables of path k0 + q, coordinates l = 4 s + g (the factor 1 past M)
        const int64_t mq = k0 + q;
        for (int l = g; l < d; l += 4) {
            const double2 e1 = mq < p1 ? e[l * M + mq] : make_double2(1.0, 0.0);
            double2 v = make_double2(1.0, 0.0);
            float2 *Tl = Tw + q * stride + l * TS;
            Tl[0] = make_float2(1.0f, 0.0f);
            for (int mm = 1; mm < TS; ++mm) {
                v = make_double2(fma(v.x, e1.x, -(v.y * e1.y)), fma(v.x, e1.y, v.y * e1.x));
                Tl[mm] = make_float2((float)v.x, (float)v.y);
            }
        }
        float s4[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t mp = k0 + 4 * g + t;
            s4[t] = mp < p1 ? (float)S[mp] : 0.0f;
        }
        wave_sync();
        uint4 bop[NKBT];
#pragma unroll
        for (int kb = 0; kb < NKBT; ++kb) {
            bop[kb] = make_uint4(0, 0, 0, 0);
            if (kb < nkb[0]) {
                const int nz = ((const int32_t CONSTANT_AS *)F.colnnz)[kb0 + kb];
                const uint4 cc = *reinterpret_cast<const uint4 *>(F.cols + (kb0 + kb) * kFacCols + q);
                uint32_t w[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float2 v = fac_value(Tw + (4 * g + t) * stride, cc, nz);
                    w[t] = pack16x2<PREC>(v.x, v.y);
                }
                bop[kb] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r < task.R) {
                const uint4 rc = *reinterpret_cast<const uint4 *>(F.rows + (task.rt0 + r) * kFacRows + (q >> 1));
                // lanes q and q ^ 1 need EA of the same row at the same four
                // paths: each forms two of them and takes the other two from
                // its partner (quad permutation [1, 0, 3, 2])
                const int h = 2 * (q & 1);
                const float2 m0 = fac_value(Tw + (4 * g + h) * stride, rc, nnz[r]);
                const float2 m1 = fac_value(Tw + (4 * g + h + 1) * stride, rc, nnz[r]);
                const float2 o0 = swap_pair(m0), o1 = swap_pair(m1);
                const float2 eas[4] = {h ? o0 : m0, h ? o1 : m1, h ? m0 : o0, h ? m1 : o1};
                uint32_t w[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float2 ea = eas[t];
                    const float wr = s4[t] * ea.x, wi = s4[t] * ea.y;
                    w[t] = (q & 1) ? pack16x2<PREC>(wi, wr) : pack16x2<PREC>(wr, -wi);
                }
                const uint4 aop = make_uint4(w[0], w[1], w[2], w[3]);
#pragma unroll
                for (int kb = 0; kb < NKBT; ++kb)
                    if (kb < nkb[r]) acc[r][kb] = fac_mfma<PREC>(aop, bop[kb], acc[r][kb]);
            }
        }
        wave_sync();
    }
    // partial sums of this unit: [unit][block][64 lanes][4]
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (r < task.R) {
            const int64_t off = fac_tile(F.tiles, task.rt0 + r).off + kb0;
#pragma unroll
            for (int kb = 0; kb < NKBT; ++kb)
                if (kb < nkb[r]) {
                    float4 *dst = reinterpret_cast<float4 *>(partial + (((int64_t)unit * F.nblocks + off + kb) * 64 + lane) * 4);
                    *dst = make_float4(acc[r][kb][0], acc[r][kb][1], acc[r][kb][2], acc[r][kb][3]);
                }
        }
    }
}

// Sum of the units' partial sums in unit order (FP64), scaled by 1/M, into
// the canonical row: entry (rr, cc) of block b is held by lane 16 (rr / 2) + cc
// at components 2 (rr % 2) + {0, 1} = (Re Z, Im Z).
__global__ void fac_reduce_kernel(const float *__restrict__ partial, int32_t units, int64_t nblocks,
                                  const int32_t *__restrict__ ent, double inv_m, double *__restrict__ alpha,
                                  int32_t *__restrict__ bad, int32_t step) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nblocks * kFacRows * kFacCols) return;
    const int32_t rep = ent[idx];
    if (rep < 0) return;
    const int64_t b = idx / (kFacRows * kFacCols);
    const int rr = (int)((idx / kFacCols) % kFacRows), cc = (int)(idx % kFacCols);
    const int lane = 16 * (rr >> 1) + cc, comp = 2 * (rr & 1);
    double zr = 0.0, zi = 0.0;
    for (int32_t u = 0; u < units; ++u) {
        const float *src = partial + (((int64_t)u * nblocks + b) * 64 + lane) * 4 + comp;
        zr += (double)src[0];
        zi += (double)src[1];
    }
    if (bad && !(isfinite(zr) && isfinite(zi))) atomicMax(bad, step);
    if (rep == 0) {
        alpha[0] = zr * inv_m;
    } else {
        alpha[2 * (int64_t)rep - 1] = M_SQRT2 * zr * inv_m;
        alpha[2 * (int64_t)rep] = M_SQRT2 * zi * inv_m;
    }
}

hipError_t launch_fac_pack(int prec, const double *alpha_row, const int32_t *ent, int64_t nblocks, uint4 *out,
                           hipStream_t s) {
    const int64_t total = nblocks * 64;
    if (total == 0) return hipSuccess;
    const unsigned nb = (unsigned)((total + 255) / 256);
    if (prec == QR_PREC_BF16)
        hipLaunchKernelGGL(fac_pack_kernel<QR_PREC_BF16>, dim3(nb), dim3(256), 0, s, alpha_row, ent, nblocks, out);
    else if (prec == QR_PREC_F16)
        hipLaunchKernelGGL(fac_pack_kernel<QR_PREC_F16>, dim3(nb), dim3(256), 0, s, alpha_row, ent, nblocks, out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int DB, int NKB, int PREC>
static hipError_t fac_path_t(const FacPathArgs &a, hipStream_t s) {
    const int waves = fac_waves(a.F.d, a.F.TS);
    const size_t lds = (size_t)waves * kFacPaths * fac_stride(a.F.d, a.F.TS) * sizeof(float2);
    static size_t granted = kLdsDefault;
    const hipError_t e = allow_lds((const void *)fac_path_kernel<DB, NKB, PREC>, lds, granted);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((fac_path_kernel<DB, NKB, PREC>), dim3(blocks_for(a.M, (int64_t)waves * kFacPaths)),
                       dim3(64 * waves), lds, s, a.P, a.F, a.i, a.M, a.seed, a.coef, a.S, a.e);
    return hipGetLastError();
}

template <int DB, int PREC>
static hipError_t fac_path_nkb(const FacPathArgs &a, hipStream_t s) {
    if (a.F.nkb <= 4) return fac_path_t<DB, 4, PREC>(a, s);
    if (a.F.nkb <= 8) return fac_path_t<DB, 8, PREC>(a, s);
    if (a.F.nkb <= 12) return fac_path_t<DB, 12, PREC>(a, s);
    if (a.F.nkb <= 16) return fac_path_t<DB, 16, PREC>(a, s);
    if (a.F.nkb <= 18) return fac_path_t<DB, 18, PREC>(a, s);
    if (a.F.nkb <= 20) return fac_path_t<DB, 20, PREC>(a, s);
    if (a.F.nkb <= kFacMaxNkb) return fac_path_t<DB, kFacMaxNkb, PREC>(a, s);
    return hipErrorInvalidValue;
}

template <int PREC>
static hipError_t fac_path_db(int db, const FacPathArgs &a, hipStream_t s) {
    switch (db) {
    case 4: return fac_path_nkb<4, PREC>(a, s);
    case 8: return fac_path_nkb<8, PREC>(a, s);
    case 16: return fac_path_nkb<16, PREC>(a, s);
    }
    return hipErrorInvalidValue;
}

template <int R, int NKBT, int PREC>
static hipError_t fac_project_t(const FacDev &F, const FacTask *tasks, int32_t ntasks, const double2 *e,
                                const double *S, int64_t M, int64_t per_unit, int32_t units, float *partial,
                                hipStream_t s) {
    const int waves = fac_waves(F.d, F.TS);
    const size_t lds = (size_t)waves * kFacPaths * fac_stride(F.d, F.TS) * sizeof(float2);
    static size_t granted = kLdsDefault;
    const hipError_t e0 = allow_lds((const void *)fac_project_kernel<R, NKBT, PREC>, lds, granted);
    if (e0 != hipSuccess) return e0;
    hipLaunchKernelGGL((fac_project_kernel<R, NKBT, PREC>), dim3(ntasks, units / waves), dim3(64 * waves), lds, s,
                       F, tasks, e, S, M, per_unit, units, partial);
    return hipGetLastError();
}

template <int PREC>
static hipError_t fac_project_p(int tmpl, const FacDev &F, const FacTask *tasks, int32_t ntasks, const double2 *e,
                                const double *S, int64_t M, int64_t per_unit, int32_t units, float *partial,
                                hipStream_t s) {
    switch (tmpl) {
    case 0: return fac_project_t<8, 1, PREC>(F, tasks, ntasks, e, S, M, per_unit, units, partial, s);
    case 1: return fac_project_t<4, 2, PREC>(F, tasks, ntasks, e, S, M, per_unit, units, partial, s);
    case 2: return fac_project_t<2, 4, PREC>(F, tasks, ntasks, e, S, M, per_unit, units, partial, s);
    case 3: return fac_project_t<1, 8, PREC>(F, tasks, ntasks, e, S, M, per_unit, units, partial, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_fac_project(int prec, int tmpl, const FacDev &F, const FacTask *tasks, int32_t ntasks,
                              const double2 *e, const double *S, int64_t M, int64_t per_unit, int32_t units,
                              float *partial, hipStream_t s) {
    if (ntasks == 0 || M == 0) return hipSuccess;
    if (units % fac_waves(F.d, F.TS) != 0) return hipErrorInvalidValue;
    if (prec == QR_PREC_BF16)
        return fac_project_p<QR_PREC_BF16>(tmpl, F, tasks, ntasks, e, S, M, per_unit, units, partial, s);
    if (prec == QR_PREC_F16)
        return fac_project_p<QR_PREC_F16>(tmpl, F, tasks, ntasks, e, S, M, per_unit, units, partial, s);
    return hipErrorInvalidValue;
}

hipError_t launch_fac_reduce(const float *partial, int32_t units, int64_t nblocks, const int32_t *ent, double M,
                             double *alpha_row, int32_t *bad, int32_t step, hipStream_t s) {
    const int64_t total = nblocks * kFacRows * kFacCols;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(fac_reduce_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, partial, units, nblocks, ent,
                       1.0 / M, alpha_row, bad, step);
    return hipGetLastError();
}

hipError_t launch_fac_path(int db, int prec, const FacPathArgs &a, hipStream_t s) {
    if (a.M <= 0) return hipSuccess;
    if (prec == QR_PREC_BF16) return fac_path_db<QR_PREC_BF16>(db, a, s);
    if (prec == QR_PREC_F16) return fac_path_db<QR_PREC_F16>(db, a, s);
    return hipErrorInvalidValue;
}

}  // namespace qrmc
