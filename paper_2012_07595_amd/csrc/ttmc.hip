// Tensor-times-block products over a stored (1,2)-symmetric tensor
// (section "Multilinear tensor-matrix multiplication" mode products; Algorithm 3 step (i); section "Block-Krylov methods for (1,2)-symmetric tensors").
//
//   FREE3  T3(k, a + px*b) = sum_{stored (i<=j,k,v)} v*(X(i,a)Y(j,b) + [i!=j] X(j,a)Y(i,b))
//          sym-half (Y = X): columns b*(b+1)/2 + a, a <= b (triunfold_3)
//   FREE1  T1(r, b + py*c) = sum_{full entries (r,col,k,v)} v*Y(col,b)*Z(k,c)
//   MODE3  t(q, c)         = sum_{k in fibre of stored pair q} v*Z(k,c)
//
// Narrow widths (the block-Krylov and gradient products) run in
// `ttmc_wave`: one 64-lane wave per work item, each lane owning an exact
// PA x PB block of the output row in registers (PA, PB <= 5), G lanes per
// entry so widths 5, 10, 20 tile without padding.  A heavy item is a chunk
// of one long segment: lanes stride its entries and the wave reduces through
// LDS; a light item is a run of short segments, one lane group per segment,
// written straight from registers.  Split segments leave partial rows that
// `ttmc_fixup` sums in slot order, so results are deterministic and no
// atomics are used.
//
// The wide symmetric product of the core formation, A.(X, X)_{1,2} with
// k1 columns, runs in `ttmc_sym_wide`: one workgroup per (slice, 64x64
// output tile pair) stages the gathered factor rows of 32 entries at a time
// in LDS and accumulates a 4x4 register tile per thread.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "bks_internal.h"

namespace bks {

namespace {

constexpr int kMaxP = 5;
constexpr int kStageBytes = 10240;  // LDS staging budget of one wave
constexpr int kIdxRegs = 2;         // batch entries held in registers per lane

enum { MODE_TWO = 0, MODE_ONE = 1, MODE_M3 = 2 };
enum { OUT_RECT = 0, OUT_SYM = 1 };

// 16-byte vector of the compute type (the unit of every row gather); native
// vector types keep register arrays of them in registers.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef int i32x2 __attribute__((ext_vector_type(2)));
template <typename CT> struct Vec;
template <> struct Vec<float> {
    using T = f32x4;
    static constexpr int V = 4;
};
template <> struct Vec<double> {
    using T = f64x2;
    static constexpr int V = 2;
};

__host__ __device__ constexpr int pad_to(int x, int v) { return (x + v - 1) / v * v; }

// Launch geometry shared by host and kernel.  Factors arrive block-packed:
// row r of a packed factor holds its lane blocks one after another, block t
// in [t*PAD, t*PAD + P) of the row and zero padding up to PAD (a multiple of
// one 16-byte vector), so every gather is an aligned vector load.
struct Geo {
    int px, py;        // logical widths
    int W1, W2;        // packed row widths (elements)
    int PAD1, PAD2;    // padded lane-block widths
    int G;             // lanes per entry
    int ga;            // lane blocks across the first output index
    int NB;            // entries staged per batch
    int PS;            // LDS plane stride in 16-byte units
    int same;          // FREE3: Y rows are X rows
    int outmode;
    int q;             // output columns
    int offv, offw, offa, offb;  // LDS element offsets (compute type)
};

// Read P consecutive row values of one staged entry.  Rows sit in LDS
// unit-major: 16-byte unit u of entry e of a plane set is at
// p + u * pse + e * V (pse = plane stride in elements), so lanes that read
// consecutive entries read consecutive 16-byte words (no bank conflicts).
template <typename CT, int P>
__device__ __forceinline__ void lds_block(const CT *p, int pse, CT (&r)[P]) {
    using VT4 = typename Vec<CT>::T;
    constexpr int V = Vec<CT>::V;
#pragma unroll
    for (int u = 0; u < P / V; ++u) {
        const VT4 x = *reinterpret_cast<const VT4 *>(p + u * pse);
#pragma unroll
        for (int t = 0; t < V; ++t) r[V * u + t] = x[t];
    }
#pragma unroll
    for (int t = P / V * V; t < P; ++t) r[t] = p[(t / V) * pse + (t % V)];
}

__device__ __forceinline__ int out_col(int alpha, int beta, int px, int outmode) {
    if (outmode == OUT_SYM) return beta * (beta + 1) / 2 + alpha;
    return alpha + px * beta;
}

// Lane group g of an entry owns output block (a, b): column-major over a
// ga x gb grid for rectangular outputs, the upper triangle a <= b in
// column order for the symmetric half, (0, g) for the mode-3 product.
template <int MODE>
__device__ __forceinline__ void lane_block(int g, const Geo &geo, int &a, int &b) {
    if constexpr (MODE == MODE_M3) {
        a = 0;
        b = g;
    } else {
        if (geo.outmode == OUT_SYM) {
            b = 0;
            while ((b + 1) * (b + 2) / 2 <= g) ++b;
            a = g - b * (b + 1) / 2;
        } else {
            b = g / geo.ga;
            a = g - b * geo.ga;
        }
    }
}

// Stage the packed factor rows of `cnt` entries into LDS, NR rows per
// entry (row_of(e, w), w < NR), each row U = W / V 16-byte units.  Lanes
// work as spl = 64 / U entries of U units (lane = e * U + u), so the units
// of one row are loaded by neighbouring lanes (fewer cache lines per lane
// quad); row w, unit u of entry e goes to dst + ((w * U + u) * PS + e) * V,
// and the plane stride PS = NB + 4 puts neighbouring lanes' stores in
// different banks.  Each lane issues its
// gathers for kGather / NR entries before the first LDS store so their
// latencies overlap.  `after_issue()` runs once, right after the first
// round of gathers is issued: that round is straight-line code, so loads
// started there (the next batch's indices) stay in flight while the
// gathered rows are stored.
constexpr int kGather = 8;

template <typename CT, int NR, typename RowOf>
__device__ __forceinline__ void gather_round(const CT *__restrict__ F, int W, int cnt, int base,
                                             int spl, int lu, RowOf row_of,
                                             typename Vec<CT>::T (&r)[kGather / NR][NR]) {
    using VT4 = typename Vec<CT>::T;
    constexpr int V = Vec<CT>::V;
#pragma unroll
    for (int x = 0; x < kGather / NR; ++x) {
        // every lane loads (entries past the end re-read entry 0's rows,
        // which are in bounds), so the loads carry no control flow
        const int e = base + x * spl;
        const int ee = e < cnt ? e : 0;
#pragma unroll
        for (int w = 0; w < NR; ++w)
            r[x][w] = *reinterpret_cast<const VT4 *>(F + row_of(ee, w) * W + lu * V);
    }
}

template <typename CT, int NR>
__device__ __forceinline__ void store_round(CT *dst, int U, int PS, int cnt, int base, int spl,
                                            int lu, const typename Vec<CT>::T (&r)[kGather / NR][NR]) {
    using VT4 = typename Vec<CT>::T;
    constexpr int V = Vec<CT>::V;
#pragma unroll
    for (int x = 0; x < kGather / NR; ++x) {
        const int e = base + x * spl;
        if (e < cnt)
#pragma unroll
            for (int w = 0; w < NR; ++w)
                *reinterpret_cast<VT4 *>(dst + ((int64_t)(w * U + lu) * PS + e) * V) = r[x][w];
    }
}

template <typename CT, int NR, typename RowOf, typename Hook>
__device__ __forceinline__ void stage_rows(const CT *__restrict__ F, int W, int PS, int cnt,
                                           CT *dst, RowOf row_of, Hook after_issue) {
    using VT4 = typename Vec<CT>::T;
    constexpr int V = Vec<CT>::V;
    const int U = W / V;
    if (U > 64) {
        after_issue();
        for (int e = 0; e < cnt; ++e)
            for (int w = 0; w < NR; ++w) {
                const int64_t row = row_of(e, w);
                for (int u = threadIdx.x; u < U; u += 64)
                    *reinterpret_cast<VT4 *>(dst + ((int64_t)(w * U + u) * PS + e) * V) =
                        *reinterpret_cast<const VT4 *>(F + row * W + u * V);
            }
        return;
    }
    const int spl = 64 / U;
    int ls = threadIdx.x / U;
    const int lu = threadIdx.x - ls * U;
    const bool act = ls < spl;
    if (!act) ls = cnt;  // idle lanes: every entry they touch is past the end
    const int luc = act ? lu : 0;
    constexpr int K = kGather / NR;
    VT4 r[K][NR];
    gather_round<CT, NR>(F, W, cnt, ls, spl, luc, row_of, r);
    after_issue();
    store_round<CT, NR>(dst, U, PS, cnt, ls, spl, luc, r);
    for (int base = ls + K * spl; base < cnt; base += K * spl) {
        gather_round<CT, NR>(F, W, cnt, base, spl, luc, row_of, r);
        store_round<CT, NR>(dst, U, PS, cnt, base, spl, luc, r);
    }
}

// One work item per 64-lane wave.  Entries are taken in batches of NB:
// the wave loads their index pairs and values coalesced, gathers every
// factor row they touch into LDS with one aligned vector per lane (rows of
// one entry are read by neighbouring lanes, so each row costs one cache
// line), then each lane multiplies out its PA x PB output block from LDS.
// Heavy items split a long segment into chunks (lanes stride the entries,
// LDS tree at the end); light items hold whole short segments, one lane
// group per segment.
template <typename VT, typename CT, int PA, int PB, int MODE>
__global__ __launch_bounds__(64) void ttmc_wave(
    const Item *__restrict__ items, const int64_t *__restrict__ segptr,
    const int2 *__restrict__ c12, const int32_t *__restrict__ ck, const VT *__restrict__ val,
    const CT *__restrict__ F1, const CT *__restrict__ F2, Geo geo,
    CT *__restrict__ out, int64_t ldo, CT *__restrict__ partial) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    CT *lds = reinterpret_cast<CT *>(lds_raw);
    i32x2 *s_idx = reinterpret_cast<i32x2 *>(lds_raw);
    const i32x2 *__restrict__ cp = reinterpret_cast<const i32x2 *>(c12);
    CT *s_v = lds + geo.offv;
    CT *s_w = lds + geo.offw;
    CT *s_a = lds + geo.offa;
    CT *s_b = lds + geo.offb;

    const Item it = items[blockIdx.x];
    const int lane = threadIdx.x;
    const int G = geo.G;
    const int E = 64 / G;
    const int el = lane / G;
    const int g = lane - el * G;
    const bool active = el < E;
    int ba = 0, bb = 0;
    if (active) lane_block<MODE>(g, geo, ba, bb);
    const int offa = ba * geo.PAD1, offb = bb * geo.PAD2;
    const bool heavy = it.seg_end < 0;
    const int NB = geo.NB;

    CT acc[PA][PB];
#pragma unroll
    for (int a = 0; a < PA; ++a)
#pragma unroll
        for (int b = 0; b < PB; ++b) acc[a][b] = CT(0);

    int64_t beg, end, s0 = 0, s1 = 0;
    int64_t myseg = -1;
    if (heavy) {
        beg = it.beg;
        end = it.end;
    } else {
        beg = segptr[it.seg];
        end = segptr[it.seg_end];
        myseg = (int64_t)it.seg + el;
        if (active && myseg < it.seg_end) {
            s0 = segptr[myseg];
            s1 = segptr[myseg + 1];
        }
    }

    const int nA = MODE == MODE_TWO ? 2 : (MODE == MODE_ONE ? 1 : 0);
    const int nB = MODE == MODE_TWO ? (geo.same ? 0 : 2) : 1;
    // element offsets of this lane's first unit in each staged plane set
    constexpr int V = Vec<CT>::V;
    const int pse = geo.PS * V;
    const int U1 = geo.W1 / V;
    const int UB = (MODE == MODE_TWO && geo.same) ? U1 : geo.W2 / V;
    const CT *rowsB = (MODE == MODE_TWO && geo.same) ? s_a : s_b;
    const int pa0 = (offa / V) * pse, pa1 = (U1 + offa / V) * pse;
    const int pb0 = (offb / V) * pse, pb1 = (UB + offb / V) * pse;

    // index pairs and values of the next batch are loaded into registers
    // while the current one is gathered and multiplied (NB <= 64 kIdxRegs)
    i32x2 pc[kIdxRegs];
    VT pv[kIdxRegs];
    auto fetch = [&](int64_t b0) {
        const int cnt = (int)min<int64_t>(NB, end - b0);
#pragma unroll
        for (int u = 0; u < kIdxRegs; ++u) {
            // unconditional, clamped into the batch (see stage_rows)
            const int x = min(lane + 64 * u, cnt - 1);
            if constexpr (MODE == MODE_M3)
                pc[u] = i32x2{0, ck[b0 + x]};
            else
                pc[u] = cp[b0 + x];
            pv[u] = val ? val[b0 + x] : VT(1);
        }
    };
    if (beg < end) fetch(beg);
    for (int64_t b0 = beg; b0 < end; b0 += NB) {
        const int cnt = (int)min<int64_t>(NB, end - b0);
#pragma unroll
        for (int u = 0; u < kIdxRegs; ++u) {
            const int x = lane + 64 * u;
            if (x < cnt) {
                const i32x2 c = pc[u];
                s_idx[x] = c;
                const CT v = static_cast<CT>(pv[u]);
                s_v[x] = v;
                if constexpr (MODE == MODE_TWO) s_w[x] = (c.x != c.y) ? v : CT(0);
            }
        }
        __syncthreads();
        // unconditional (the last batch re-reads itself) so no branch
        // separates these loads from the gathers' waits
        auto next = [&]() { fetch(b0 + NB < end ? b0 + NB : b0); };
        auto none = []() {};
        const int PS = geo.PS;
        if constexpr (MODE == MODE_TWO) {
            // row 0: i, row 1: j
            auto ij = [&](int e, int w) {
                const i32x2 c = s_idx[e];
                return (int64_t)(w ? c.y : c.x);
            };
            if (geo.same) {
                stage_rows<CT, 2>(F1, geo.W1, PS, cnt, s_a, ij, next);
            } else {
                stage_rows<CT, 2>(F1, geo.W1, PS, cnt, s_a, ij, none);
                stage_rows<CT, 2>(F2, geo.W2, PS, cnt, s_b, ij, next);
            }
        } else {
            auto rk = [&](int e, int) { return (int64_t)s_idx[e].y; };
            if constexpr (MODE == MODE_ONE) {
                stage_rows<CT, 1>(F1, geo.W1, PS, cnt, s_a,
                                  [&](int e, int) { return (int64_t)s_idx[e].x; }, next);
                stage_rows<CT, 1>(F2, geo.W2, PS, cnt, s_b, rk, none);
            } else {
                stage_rows<CT, 1>(F2, geo.W2, PS, cnt, s_b, rk, next);
            }
        }
        (void)nA;
        (void)nB;
        __syncthreads();

        int lo, hi, step;
        if (heavy) {
            lo = active ? el : cnt;
            hi = cnt;
            step = E;
        } else {
            lo = (int)max<int64_t>(s0 - b0, 0);
            hi = (int)min<int64_t>(s1 - b0, cnt);
            step = 1;
        }
        for (int e = lo; e < hi; e += step) {
            const CT v = s_v[e];
            if constexpr (MODE == MODE_M3) {
                CT zb[PB];
                lds_block<CT, PB>(s_b + pb0 + e * V, pse, zb);
#pragma unroll
                for (int b = 0; b < PB; ++b) acc[0][b] = fma(v, zb[b], acc[0][b]);
            } else if constexpr (MODE == MODE_ONE) {
                CT ya[PA], zb[PB];
                lds_block<CT, PA>(s_a + pa0 + e * V, pse, ya);
                lds_block<CT, PB>(s_b + pb0 + e * V, pse, zb);
#pragma unroll
                for (int a = 0; a < PA; ++a) {
                    const CT x = v * ya[a];
#pragma unroll
                    for (int b = 0; b < PB; ++b) acc[a][b] = fma(x, zb[b], acc[a][b]);
                }
            } else {
                // A.(X, Y)_{1,2} gets v X(i,:)^T Y(j,:) and, off the
                // diagonal, the mirrored entry's v X(j,:)^T Y(i,:)
                const CT w = s_w[e];
                CT xi[PA], xj[PA], yi[PB], yj[PB];
                lds_block<CT, PA>(s_a + pa0 + e * V, pse, xi);
                lds_block<CT, PA>(s_a + pa1 + e * V, pse, xj);
                lds_block<CT, PB>(rowsB + pb0 + e * V, pse, yi);
                lds_block<CT, PB>(rowsB + pb1 + e * V, pse, yj);
#pragma unroll
                for (int a = 0; a < PA; ++a) {
                    const CT x1 = v * xi[a], x2 = w * xj[a];
#pragma unroll
                    for (int b = 0; b < PB; ++b)
                        acc[a][b] = fma(x2, yi[b], fma(x1, yj[b], acc[a][b]));
                }
            }
        }
        __syncthreads();
    }

    const int a0 = ba * PA, bl0 = bb * PB;
    if (heavy) {
        CT *red = lds;
#pragma unroll
        for (int a = 0; a < PA; ++a)
#pragma unroll
            for (int b = 0; b < PB; ++b) red[lane * PA * PB + a * PB + b] = acc[a][b];
        __syncthreads();
        const int nout = G * PA * PB;
        for (int o = lane; o < nout; o += 64) {
            const int gg = o / (PA * PB);
            const int ab = o - gg * PA * PB;
            const int a = ab / PB, b = ab - (ab / PB) * PB;
            int ga_, gb_;
            lane_block<MODE>(gg, geo, ga_, gb_);
            const int alpha = ga_ * PA + a, beta = gb_ * PB + b;
            if (alpha >= geo.px || beta >= geo.py) continue;
            if (geo.outmode == OUT_SYM && alpha > beta) continue;
            CT s = CT(0);
            for (int x = 0; x < E; ++x) s += red[(x * G + gg) * PA * PB + ab];
            const int col = out_col(alpha, beta, geo.px, geo.outmode);
            if (it.slot < 0)
                out[(int64_t)it.seg * ldo + col] = s;
            else
                partial[(int64_t)it.slot * geo.q + col] = s;
        }
    } else if (active && myseg < it.seg_end) {
#pragma unroll
        for (int a = 0; a < PA; ++a)
#pragma unroll
            for (int b = 0; b < PB; ++b) {
                const int alpha = a0 + a, beta = bl0 + b;
                if (alpha < geo.px && beta < geo.py &&
                    (geo.outmode == OUT_RECT || alpha <= beta))
                    out[myseg * ldo + out_col(alpha, beta, geo.px, geo.outmode)] = acc[a][b];
            }
    }
}

// Block-pack a factor: out(r, t*PAD + u) = F(r, t*P + u) for u < P and
// t*P + u < p, else 0.
template <typename CT>
__global__ __launch_bounds__(256) void pack_blocks(const CT *__restrict__ F, int64_t ld,
                                                   int64_t rows, int p, int P, int PAD, int W,
                                                   CT *__restrict__ out) {
    const int64_t total = rows * W;
    for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < total;
         x += (int64_t)gridDim.x * 256) {
        const int64_t r = x / W;
        const int c = (int)(x - r * W);
        const int t = c / PAD, u = c - t * PAD;
        const int col = t * P + u;
        out[x] = (u < P && col < p) ? F[r * ld + col] : CT(0);
    }
}

// ---------------------------------------------------------------- register-direct
// Narrow products with the whole output block of a segment in each lane's
// registers (P1 x P2 accumulators, the upper triangle only for a symmetric
// half).  A group of L lanes (a power of two, from the item) takes one
// segment and strides its entries, so the group's loads of indices and
// values are coalesced; each lane gathers its entries' factor rows straight
// into registers with aligned 16-byte loads from the block-packed copies,
// U entries at a time so that their loads are in flight together.  The group
// then sums its lanes with cross-lane shuffles in a fixed butterfly order
// (deterministic) and its first lane writes the row, or, for a chunk of a
// split segment, the chunk's partial slot.  Four independent waves per
// workgroup, one item per wave.
template <typename CT, int P>
__device__ __forceinline__ void row_load(const CT *__restrict__ F, int64_t row, int W,
                                         CT (&r)[P]) {
    using VT4 = typename Vec<CT>::T;
    constexpr int V = Vec<CT>::V;
    constexpr int NV = (P + V - 1) / V;
    const VT4 *p = reinterpret_cast<const VT4 *>(F + row * W);
#pragma unroll
    for (int u = 0; u < NV; ++u) {
        const VT4 x = p[u];
#pragma unroll
        for (int t = 0; t < V; ++t)
            if (u * V + t < P) r[u * V + t] = x[t];
    }
}

template <typename VT, typename CT, int MODE, int P1, int P2, bool SYM, int U>
__global__ __launch_bounds__(256) void ttmc_reg(
    const Item *__restrict__ items, int64_t nitems, const int64_t *__restrict__ segptr,
    const int2 *__restrict__ c12, const int32_t *__restrict__ ck, const VT *__restrict__ val,
    const CT *__restrict__ F1, int W1, const CT *__restrict__ F2, int W2, CT *__restrict__ out,
    int64_t ldo, CT *__restrict__ partial, int q) {
    const int lane = threadIdx.x & 63;
    const int64_t wi = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wi >= nitems) return;
    const Item it = items[wi];
    const bool heavy = it.seg_end < 0;
    const int L = heavy ? 64 : it.pad;
    const int gl = lane & (L - 1);
    const int64_t seg = heavy ? (int64_t)it.seg : (int64_t)it.seg + lane / L;
    const bool own = heavy || seg < it.seg_end;
    int64_t beg = 0, end = 0;
    if (heavy) {
        beg = it.beg;
        end = it.end;
    } else if (own) {
        beg = segptr[seg];
        end = segptr[seg + 1];
    }

    CT acc[P1][P2];
#pragma unroll
    for (int a = 0; a < P1; ++a)
#pragma unroll
        for (int b = 0; b < P2; ++b) acc[a][b] = CT(0);

    for (int64_t e0 = beg + gl; e0 < end; e0 += (int64_t)L * U) {
        // U entries per lane: indices and values first (clamped into the
        // segment, weight 0 past its end), then every row gather, then the
        // products
        i32x2 c[U];
        CT v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + (int64_t)L * u;
            const int64_t ec = e < end ? e : e0;
            if constexpr (MODE == MODE_M3)
                c[u] = i32x2{0, ck[ec]};
            else
                c[u] = reinterpret_cast<const i32x2 *>(c12)[ec];
            const CT x = val ? static_cast<CT>(val[ec]) : CT(1);
            v[u] = e < end ? x : CT(0);
        }
        if constexpr (MODE == MODE_M3) {
            CT z[U][P2];
#pragma unroll
            for (int u = 0; u < U; ++u) row_load<CT, P2>(F2, c[u].y, W2, z[u]);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int b = 0; b < P2; ++b) acc[0][b] = fma(v[u], z[u][b], acc[0][b]);
        } else if constexpr (MODE == MODE_ONE) {
            CT y[U][P1], z[U][P2];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                row_load<CT, P1>(F1, c[u].x, W1, y[u]);
                row_load<CT, P2>(F2, c[u].y, W2, z[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int a = 0; a < P1; ++a) {
                    const CT x = v[u] * y[u][a];
#pragma unroll
                    for (int b = 0; b < P2; ++b) acc[a][b] = fma(x, z[u][b], acc[a][b]);
                }
        } else {
            // v X(i,:)^T Y(j,:) and, off the diagonal, the mirrored entry's
            // v X(j,:)^T Y(i,:)
            CT xi[U][P1], xj[U][P1];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                row_load<CT, P1>(F1, c[u].x, W1, xi[u]);
                row_load<CT, P1>(F1, c[u].y, W1, xj[u]);
            }
            if constexpr (SYM) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const CT w = c[u].x != c[u].y ? v[u] : CT(0);
#pragma unroll
                    for (int a = 0; a < P1; ++a) {
                        const CT x1 = v[u] * xi[u][a], x2 = w * xj[u][a];
#pragma unroll
                        for (int b = a; b < P2; ++b)
                            acc[a][b] = fma(x2, xi[u][b], fma(x1, xj[u][b], acc[a][b]));
                    }
                }
            } else {
                CT yi[U][P2], yj[U][P2];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    row_load<CT, P2>(F2, c[u].x, W2, yi[u]);
                    row_load<CT, P2>(F2, c[u].y, W2, yj[u]);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const CT w = c[u].x != c[u].y ? v[u] : CT(0);
#pragma unroll
                    for (int a = 0; a < P1; ++a) {
                        const CT x1 = v[u] * xi[u][a], x2 = w * xj[u][a];
#pragma unroll
                        for (int b = 0; b < P2; ++b)
                            acc[a][b] = fma(x2, yi[u][b], fma(x1, yj[u][b], acc[a][b]));
                    }
                }
            }
        }
    }

    // butterfly sum over the group's lanes (all lanes of the wave take part,
    // each group within itself)
    for (int off = L >> 1; off > 0; off >>= 1)
#pragma unroll
        for (int a = 0; a < P1; ++a)
#pragma unroll
            for (int b = 0; b < P2; ++b)
                if (!SYM || a <= b) acc[a][b] += __shfl_xor(acc[a][b], off, 64);
    if (!own || gl != 0) return;
    CT *dst = (heavy && it.slot >= 0) ? partial + (int64_t)it.slot * q : out + seg * ldo;
#pragma unroll
    for (int a = 0; a < P1; ++a)
#pragma unroll
        for (int b = 0; b < P2; ++b) {
            if (SYM && a > b) continue;
            const int col = MODE == MODE_M3 ? b : (SYM ? b * (b + 1) / 2 + a : a + P1 * b);
            dst[col] = acc[a][b];
        }
}

// Sum the partial rows of one split segment: 256 threads as (slot lane,
// column); each lane sums a strided subset of the slots, then a fixed-order
// tree over the lanes in LDS (deterministic).
// (Tree levels call it with out = partial, ldo = q: the slots read and the
// slot written are disjoint.)
template <typename CT>
__global__ __launch_bounds__(256) void ttmc_fixup(const Fixup *__restrict__ fix,
                                                  const CT *partial, int q, CT *out,
                                                  int64_t ldo) {
    __shared__ CT red[256];
    const Fixup f = fix[blockIdx.x];
    const int cols = q < 256 ? q : 256;
    int lanes = 256 / cols;
    int pw = 1;
    while (pw * 2 <= lanes) pw *= 2;
    lanes = pw;
    const int tid = threadIdx.x;
    const int col_l = tid % cols, sl = tid / cols;
    for (int c0 = 0; c0 < q; c0 += cols) {
        const int col = c0 + col_l;
        CT s = CT(0);
        if (sl < lanes && col < q)
            for (int x = sl; x < f.nslots; x += lanes)
                s += partial[(int64_t)(f.first_slot + x) * q + col];
        red[tid] = s;
        __syncthreads();
        for (int w = lanes / 2; w > 0; w >>= 1) {
            if (sl < w) red[tid] += red[tid + w * cols];
            __syncthreads();
        }
        if (sl == 0 && col < q) out[(int64_t)f.seg * ldo + col] = red[tid];
        __syncthreads();
    }
}

// ---------------------------------------------------------------- wide sym
constexpr int kTile = 64;
constexpr int kChunk = 32;

template <typename VT, typename CT>
__global__ __launch_bounds__(256) void ttmc_sym_wide(
    const int64_t *__restrict__ segptr, const int2 *__restrict__ c12,
    const VT *__restrict__ val, const CT *__restrict__ X,
    int64_t ldx, int p, int ntile, CT *__restrict__ out, int64_t ldo) {
    __shared__ CT xai[kChunk][kTile];
    __shared__ CT xbj[kChunk][kTile];
    __shared__ CT xaj[kChunk][kTile];
    __shared__ CT xbi[kChunk][kTile];
    const int npair = ntile * (ntile + 1) / 2;
    const int64_t k = blockIdx.x / npair;
    int pr = blockIdx.x - (int)(k * npair);
    int ta = 0;
    while (pr >= ntile - ta) {
        pr -= ntile - ta;
        ++ta;
    }
    const int tb = ta + pr;
    const int tid = threadIdx.x;
    const int ty = tid / 16, tx = tid % 16;
    CT acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = CT(0);
    const int64_t e0 = segptr[k], e1 = segptr[k + 1];
    for (int64_t base = e0; base < e1; base += kChunk) {
        const int cnt = (int)min<int64_t>(kChunk, e1 - base);
        // stage gathered rows: 256 threads fill 4 arrays of kChunk x kTile
        for (int x = tid; x < kChunk * kTile; x += 256) {
            const int e = x / kTile, c = x - (x / kTile) * kTile;
            CT vi = CT(0), vj = CT(0), wi = CT(0), wj = CT(0);
            if (e < cnt) {
                const int64_t ee = base + e;
                const int2 ij = c12[ee];
                const int i = ij.x, j = ij.y;
                const CT v = static_cast<CT>(val[ee]);
                const CT w = (i != j) ? v : CT(0);
                const int ca = ta * kTile + c, cb = tb * kTile + c;
                if (ca < p) {
                    vi = v * X[(int64_t)i * ldx + ca];
                    wj = w * X[(int64_t)j * ldx + ca];
                }
                if (cb < p) {
                    vj = X[(int64_t)j * ldx + cb];
                    wi = X[(int64_t)i * ldx + cb];
                }
            }
            xai[e][c] = vi;
            xbj[e][c] = vj;
            xaj[e][c] = wj;
            xbi[e][c] = wi;
        }
        __syncthreads();
        for (int e = 0; e < cnt; ++e) {
            CT a1[4], b1[4], a2[4], b2[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                a1[a] = xai[e][ty * 4 + a];
                a2[a] = xaj[e][ty * 4 + a];
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                b1[b] = xbj[e][tx * 4 + b];
                b2[b] = xbi[e][tx * 4 + b];
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    acc[a][b] = fma(a1[a], b1[b], acc[a][b]);
                    acc[a][b] = fma(a2[a], b2[b], acc[a][b]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int alpha = ta * kTile + ty * 4 + a, beta = tb * kTile + tx * 4 + b;
            if (alpha < p && beta < p && alpha <= beta)
                out[k * ldo + beta * (beta + 1) / 2 + alpha] = acc[a][b];
        }
}

// ---------------------------------------------------------------- wide sym, Gram form
// A.(X, X)_{1,2} for wide X as a sum of per-entry outer products: with
// v' = v off the diagonal and v / 2 on it (i = j), the symmetric result of
// slice k is M + M^T, M = sum over stored (i, j, k) of v' X(i,:)^T X(j,:).
// One workgroup of T x T threads (an R x R register tile each, T*R >= p)
// accumulates M for one item (a slice or a chunk of a long slice) from
// rows of the block-packed X staged in LDS, kGramChunk entries at a time,
// and writes it to its partial slot; `sym_gram_reduce` sums a slice's
// chunks in order and writes the upper triangle of M + M^T.
constexpr int kGramChunk = 16;
constexpr int64_t kGramItems = 4096;  // target number of slice chunks per product

template <typename VT, typename CT, int R>
__global__ __launch_bounds__(256) void ttmc_sym_gram(const Item *__restrict__ items,
                                                     const int2 *__restrict__ c12,
                                                     const VT *__restrict__ val,
                                                     const CT *__restrict__ Xp, int T, int RP,
                                                     int p, CT *__restrict__ part) {
    using VT4 = typename Vec<CT>::T;
    constexpr int V = Vec<CT>::V;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int W = T * RP;  // packed row width (elements)
    const int U = W / V;
    CT *s_xi = reinterpret_cast<CT *>(lds_raw);  // [kGramChunk][W], scaled by v'
    CT *s_xj = s_xi + kGramChunk * W;           // [kGramChunk][W]
    CT *s_v = s_xj + kGramChunk * W;            // [kGramChunk]
    i32x2 *s_ij = reinterpret_cast<i32x2 *>(s_v + pad_to(kGramChunk, V));
    const i32x2 *__restrict__ cp = reinterpret_cast<const i32x2 *>(c12);

    const Item it = items[blockIdx.x];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int ty = tid / T, tx = tid - (tid / T) * T;
    const bool active = ty < T;
    CT acc[R][R];
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) acc[a][b] = CT(0);
    // staging walk: thread -> (entry, unit of the entry's two rows)
    const int two_u = 2 * U;
    const int e0 = tid / two_u, r0 = tid - e0 * two_u;
    const int de = nth / two_u, dr = nth - de * two_u;

    for (int64_t b0 = it.beg; b0 < it.end; b0 += kGramChunk) {
        const int cnt = (int)min<int64_t>(kGramChunk, it.end - b0);
        for (int x = tid; x < cnt; x += nth) {
            const i32x2 c = cp[b0 + x];
            const CT v = static_cast<CT>(val[b0 + x]);
            s_ij[x] = c;
            s_v[x] = c.x == c.y ? v * CT(0.5) : v;
        }
        __syncthreads();
        for (int e = e0, rem = r0; e < cnt;) {
            const int w = rem >= U ? 1 : 0;
            const int u = rem - w * U;
            const i32x2 c = s_ij[e];
            VT4 d = reinterpret_cast<const VT4 *>(Xp + (int64_t)(w ? c.y : c.x) * W)[u];
            if (!w) d = d * s_v[e];
            reinterpret_cast<VT4 *>((w ? s_xj : s_xi) + e * W)[u] = d;
            e += de;
            rem += dr;
            if (rem >= two_u) {
                rem -= two_u;
                ++e;
            }
        }
        __syncthreads();
        if (active) {
            for (int e = 0; e < cnt; ++e) {
                CT xa[R], xb[R];
                lds_block<CT, R>(s_xi + e * W + ty * RP, V, xa);
                lds_block<CT, R>(s_xj + e * W + tx * RP, V, xb);
#pragma unroll
                for (int a = 0; a < R; ++a)
#pragma unroll
                    for (int b = 0; b < R; ++b) acc[a][b] = fma(xa[a], xb[b], acc[a][b]);
            }
        }
        __syncthreads();
    }
    if (active) {
        CT *o = part + (int64_t)it.slot * p * p;
#pragma unroll
        for (int a = 0; a < R; ++a) {
            const int alpha = ty * R + a;
            if (alpha < p)
#pragma unroll
                for (int b = 0; b < R; ++b) {
                    const int beta = tx * R + b;
                    if (beta < p) o[(int64_t)alpha * p + beta] = acc[a][b];
                }
        }
    }
}

// out(k, beta(beta+1)/2 + alpha) = sum over slice k's chunks c, in order, of
// M_c(alpha, beta) + M_c(beta, alpha), alpha <= beta (zero for an empty slice).
// One workgroup per slice walks the 32 x 32 tile pairs (I <= J): tiles
// M_c(I, J) and M_c(J, I) are read row by row (coalesced) into LDS and the
// transpose is taken there.
template <typename CT>
__global__ __launch_bounds__(256) void sym_gram_reduce(const Fixup *__restrict__ fix,
                                                       const CT *__restrict__ part, int p,
                                                       CT *__restrict__ out, int64_t ldo) {
    __shared__ CT tA[32][33], tB[32][33];
    const Fixup f = fix[blockIdx.x];
    const int64_t pp = (int64_t)p * p;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const int nt = (p + 31) / 32;
    for (int I = 0; I < nt; ++I)
        for (int J = I; J < nt; ++J) {
            CT acc[4] = {CT(0), CT(0), CT(0), CT(0)};
            for (int c = 0; c < f.nslots; ++c) {
                const CT *m = part + (int64_t)(f.first_slot + c) * pp;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int r = ty + 8 * k;
                    const int ra = I * 32 + r, ca = J * 32 + tx;
                    const int rb = J * 32 + r, cb = I * 32 + tx;
                    tA[r][tx] = (ra < p && ca < p) ? m[(int64_t)ra * p + ca] : CT(0);
                    tB[r][tx] = (rb < p && cb < p) ? m[(int64_t)rb * p + cb] : CT(0);
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int r = ty + 8 * k;
                    acc[k] += tA[r][tx];
                    acc[k] += tB[tx][r];
                }
                __syncthreads();
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int alpha = I * 32 + ty + 8 * k, beta = J * 32 + tx;
                if (alpha <= beta && beta < p)
                    out[(int64_t)f.seg * ldo + beta * (beta + 1) / 2 + alpha] = acc[k];
            }
        }
}

// ---------------------------------------------------------------- wide sym, matrix cores
// The same per-chunk matrix M = sum v' X(i,:)^T X(j,:) on the FP32 matrix
// cores (V_MFMA_F32_16X16X4_F32, 157 TFLOP/s on MI355X against 79 for
// unpacked FP32 FMA).  k1 is padded to T tiles of 16; wave w of the
// workgroup owns tile rows w*ROWS .. w*ROWS+ROWS-1 and every tile column.
// Entries are staged kMfmaChunk at a time (rows X(i,:) and X(j,:) in LDS,
// row stride Wl staggered over the banks); one K-step takes 4 entries: lane
// l feeds A(r, k) = v'(k) xi(k, 16 I + r) and B(k, c) = xj(k, 16 J + c) with
// r = c = l % 16, k = l / 16, and holds D(4 (l / 16) + i, l % 16) of each
// 16 x 16 output tile.
// Software pipeline over the chunks of an item: while the matrix cores work
// on chunk c from LDS, the row gathers of chunk c + 1 (into registers) and
// the index loads of chunk c + 3 are in flight; chunk c + 1's and c + 2's
// index pairs wait in two small LDS buffers.
constexpr int kMfmaChunk = 32;
typedef float f32x4v __attribute__((ext_vector_type(4)));

// DIRECT: every item is a whole slice; instead of a partial slot the
// workgroup writes the slice's output row, the upper triangle of M + M^T,
// through LDS (the staging buffers are free once the chunks are done; the
// launch gives at least p^2 floats of LDS).
template <typename VT, int T, int ROWS, bool DIRECT>
__global__ __launch_bounds__(512) void ttmc_sym_gram_mfma(const Item *__restrict__ items,
                                                          const int2 *__restrict__ c12,
                                                          const VT *__restrict__ val,
                                                          const float *__restrict__ Xp, int Wl,
                                                          int p, float *__restrict__ part,
                                                          float *__restrict__ out, int64_t ldo) {
    constexpr int W = 16 * T;  // packed row width of X
    constexpr int U = W / 4;   // 16-byte units per row
    constexpr int NW = (T + ROWS - 1) / ROWS;
    constexpr int NTH = 64 * NW;                // threads of the workgroup
    constexpr int NG = kMfmaChunk * 2 * U;      // 16-byte row gathers per chunk
    constexpr int NQ = (NG + NTH - 1) / NTH;    // per thread
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float *s_xi = reinterpret_cast<float *>(lds_raw);  // [kMfmaChunk][Wl]
    float *s_xj = s_xi + kMfmaChunk * Wl;
    float *s_v = s_xj + kMfmaChunk * Wl;                      // [2][kMfmaChunk]
    i32x2 *s_ij = reinterpret_cast<i32x2 *>(s_v + 2 * kMfmaChunk);  // [2][kMfmaChunk]
    const i32x2 *__restrict__ cp = reinterpret_cast<const i32x2 *>(c12);

    const Item it = items[blockIdx.x];
    const int64_t beg = it.beg, end = it.end;
    const int nchunk = (int)((end - beg + kMfmaChunk - 1) / kMfmaChunk);
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int kq = lane >> 4, rc = lane & 15;
    f32x4v acc[ROWS][T];
#pragma unroll
    for (int a = 0; a < ROWS; ++a)
#pragma unroll
        for (int J = 0; J < T; ++J) acc[a][J] = f32x4v{0.f, 0.f, 0.f, 0.f};

    // index pair and value of entry tid of a chunk (threads tid < kMfmaChunk);
    // positions past the item read its last entry (in bounds) with v' = 0
    i32x2 nidx = i32x2{0, 0};
    float nv = 0.f;
    bool nin = false;
    auto fetch_idx = [&](int ch) {
        if (tid < kMfmaChunk) {
            const int64_t e = beg + (int64_t)ch * kMfmaChunk + tid;
            nin = e < end;
            const int64_t ec = nin ? e : end - 1;
            nidx = cp[ec];
            nv = static_cast<float>(val[ec]);
        }
    };
    auto commit_idx = [&](int buf) {
        if (tid < kMfmaChunk) {
            float v = nin ? nv : 0.f;
            if (nidx.x == nidx.y) v *= 0.5f;
            s_ij[buf * kMfmaChunk + tid] = nidx;
            s_v[buf * kMfmaChunk + tid] = v;
        }
    };
    // row gathers of the chunk whose indices are in buffer `buf`: gather x
    // is unit u of row w (0: X(i,:), 1: X(j,:)) of entry e
    f32x4v g[NQ];
    int lo[NQ];  // LDS destination (floats from s_xi) of gather q
    auto fetch_rows = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int x = min(tid + q * NTH, NG - 1);
            const int e = x / (2 * U), rem = x - e * (2 * U);
            const int w = rem >= U ? 1 : 0, u = rem - w * U;
            const i32x2 c = s_ij[buf * kMfmaChunk + e];
            g[q] = reinterpret_cast<const f32x4v *>(Xp + (int64_t)(w ? c.y : c.x) * W)[u];
            lo[q] = w * kMfmaChunk * Wl + e * Wl + 4 * u;
        }
    };
    auto commit_rows = [&]() {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (NG % NTH == 0 || tid + q * NTH < NG)
                *reinterpret_cast<f32x4v *>(s_xi + lo[q]) = g[q];
    };

    // prologue: indices of chunks 0 and 1 in LDS, rows of chunk 0 in LDS,
    // indices of chunk 2 in registers
    fetch_idx(0);
    commit_idx(0);
    fetch_idx(1);
    commit_idx(1);
    __syncthreads();
    fetch_rows(0);
    fetch_idx(2);
    commit_rows();
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        const bool more = ch + 1 < nchunk;
        if (more) fetch_rows((ch + 1) & 1);
        const int cnt = (int)min<int64_t>(kMfmaChunk, end - beg - (int64_t)ch * kMfmaChunk);
        const int nk = (cnt + 3) >> 2;
        const float *sv = s_v + (ch & 1) * kMfmaChunk;
        for (int kk = 0; kk < nk; ++kk) {
            const int e = kk * 4 + kq;
            const float ve = sv[e];  // v' of the entry (0 past the item)
            float a[ROWS], b[T];
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int I = wave * ROWS + r;
                a[r] = I < T ? s_xi[e * Wl + I * 16 + rc] * ve : 0.f;
            }
#pragma unroll
            for (int J = 0; J < T; ++J) b[J] = s_xj[e * Wl + J * 16 + rc];
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
#pragma unroll
                for (int J = 0; J < T; ++J)
                    acc[r][J] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r], b[J], acc[r][J], 0, 0, 0);
        }
        __syncthreads();  // chunk ch's rows and indices, chunk ch + 1's indices are consumed
        if (more) commit_rows();
        commit_idx(ch & 1);  // chunk ch + 2
        fetch_idx(ch + 3);
        __syncthreads();
    }
    if constexpr (DIRECT) {
        // the loop ended on a barrier: the staging LDS is free for M
        float *Ms = reinterpret_cast<float *>(lds_raw);
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int I = wave * ROWS + r;
            if (I >= T) break;
#pragma unroll
            for (int J = 0; J < T; ++J)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = I * 16 + 4 * kq + i, col = J * 16 + rc;
                    if (row < p && col < p) Ms[row * p + col] = acc[r][J][i];
                }
        }
        __syncthreads();
        // column beta (beta + 1) / 2 + alpha, alpha <= beta: M(alpha, beta) +
        // M(beta, alpha), the sum the chunk reduction forms for one chunk
        float *orow = out + (int64_t)it.seg * ldo;
        for (int beta = wave; beta < p; beta += NW) {
            const int c0 = beta * (beta + 1) / 2;
            for (int alpha = lane; alpha <= beta; alpha += 64)
                orow[c0 + alpha] = Ms[alpha * p + beta] + Ms[beta * p + alpha];
        }
        return;
    }
    float *o = part + (int64_t)it.slot * p * p;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int I = wave * ROWS + r;
        if (I >= T) break;
#pragma unroll
        for (int J = 0; J < T; ++J)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = I * 16 + 4 * kq + i, col = J * 16 + rc;
                if (row < p && col < p) o[(int64_t)row * p + col] = acc[r][J][i];
            }
    }
}

// The same product for widths beyond 12 tiles (k1 > 192): the T x T tiles
// of M are cut into TR x TC blocks, one workgroup per (slice chunk, block);
// block (R, C) stages only the rows X(i, R-block) and X(j, C-block) of each
// chunk and writes its part of the chunk's partial M (full p x p per slot,
// summed and symmetrised by sym_gram_reduce as above).  Xp rows hold T16
// tiles (16 T16 floats); tiles past T16 of the last blocks are skipped.
// Wide products come with few, long chunks (the partials are p^2 each): a
// chunk of a 1e6-row tensor holds ~4e5 entries, and one FP32 accumulator
// chain that long loses ~1e-5 relative accuracy.  The matrix-core
// accumulators are therefore added into a second set every kBlkFlush
// chunks (blocked summation), which keeps the error near 1e-6.
constexpr int kBlkFlush = 8;
template <typename VT, int TR, int TC, int ROWS>
__global__ __launch_bounds__(64 * ((TR + ROWS - 1) / ROWS)) void ttmc_sym_gram_mfma_blk(
    const Item *__restrict__ items, const int2 *__restrict__ c12, const VT *__restrict__ val,
    const float *__restrict__ Xp, int T16, int Wli, int Wlj, int p, float *__restrict__ part) {
    constexpr int UI = 4 * TR, UJ = 4 * TC;     // 16-byte units of the staged rows
    constexpr int NW = (TR + ROWS - 1) / ROWS;
    constexpr int NTH = 64 * NW;
    constexpr int NG = kMfmaChunk * (UI + UJ);  // row gathers per chunk
    constexpr int NQ = (NG + NTH - 1) / NTH;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float *s_xi = reinterpret_cast<float *>(lds_raw);  // [kMfmaChunk][Wli]
    float *s_xj = s_xi + kMfmaChunk * Wli;             // [kMfmaChunk][Wlj]
    float *s_v = s_xj + kMfmaChunk * Wlj;              // [2][kMfmaChunk]
    i32x2 *s_ij = reinterpret_cast<i32x2 *>(s_v + 2 * kMfmaChunk);
    const i32x2 *__restrict__ cp = reinterpret_cast<const i32x2 *>(c12);
    const int W = 16 * T16;
    const int nbc = (T16 + TC - 1) / TC;
    const int R0 = (int)(blockIdx.y / nbc) * TR, C0 = (int)(blockIdx.y % nbc) * TC;

    const Item it = items[blockIdx.x];
    const int64_t beg = it.beg, end = it.end;
    const int nchunk = (int)((end - beg + kMfmaChunk - 1) / kMfmaChunk);
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int kq = lane >> 4, rc = lane & 15;
    f32x4v acc[ROWS][TC], tot[ROWS][TC];
#pragma unroll
    for (int a = 0; a < ROWS; ++a)
#pragma unroll
        for (int J = 0; J < TC; ++J) {
            acc[a][J] = f32x4v{0.f, 0.f, 0.f, 0.f};
            tot[a][J] = f32x4v{0.f, 0.f, 0.f, 0.f};
        }

    i32x2 nidx = i32x2{0, 0};
    float nv = 0.f;
    bool nin = false;
    auto fetch_idx = [&](int ch) {
        if (tid < kMfmaChunk) {
            const int64_t e = beg + (int64_t)ch * kMfmaChunk + tid;
            nin = e < end;
            const int64_t ec = nin ? e : end - 1;
            nidx = cp[ec];
            nv = static_cast<float>(val[ec]);
        }
    };
    auto commit_idx = [&](int buf) {
        if (tid < kMfmaChunk) {
            float v = nin ? nv : 0.f;
            if (nidx.x == nidx.y) v *= 0.5f;
            s_ij[buf * kMfmaChunk + tid] = nidx;
            s_v[buf * kMfmaChunk + tid] = v;
        }
    };
    auto flush = [&]() {
#pragma unroll
        for (int a = 0; a < ROWS; ++a)
#pragma unroll
            for (int J = 0; J < TC; ++J) {
                tot[a][J] += acc[a][J];
                acc[a][J] = f32x4v{0.f, 0.f, 0.f, 0.f};
            }
    };
    // gather x: unit u of the staged part of row X(i,:) (u < UI, tiles
    // R0..) or of X(j,:) (u >= UI, tiles C0..) of entry e; units past the
    // packed row (the last blocks' missing tiles) re-read unit 0
    f32x4v g[NQ];
    int lo[NQ];
    auto fetch_rows = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int x = min(tid + q * NTH, NG - 1);
            const int e = x / (UI + UJ), rem = x - e * (UI + UJ);
            const bool wj = rem >= UI;
            const int u = wj ? rem - UI : rem;
            const int col4 = (wj ? C0 : R0) * 4 + u;     // unit within the packed row
            const i32x2 c = s_ij[buf * kMfmaChunk + e];
            const int uc = col4 < 4 * T16 ? col4 : 0;
            g[q] = reinterpret_cast<const f32x4v *>(Xp + (int64_t)(wj ? c.y : c.x) * W)[uc];
            lo[q] = wj ? kMfmaChunk * Wli + e * Wlj + 4 * u : e * Wli + 4 * u;
        }
    };
    auto commit_rows = [&]() {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (NG % NTH == 0 || tid + q * NTH < NG)
                *reinterpret_cast<f32x4v *>(s_xi + lo[q]) = g[q];
    };

    fetch_idx(0);
    commit_idx(0);
    fetch_idx(1);
    commit_idx(1);
    __syncthreads();
    fetch_rows(0);
    fetch_idx(2);
    commit_rows();
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        const bool more = ch + 1 < nchunk;
        if (more) fetch_rows((ch + 1) & 1);
        const int cnt = (int)min<int64_t>(kMfmaChunk, end - beg - (int64_t)ch * kMfmaChunk);
        const int nk = (cnt + 3) >> 2;
        const float *sv = s_v + (ch & 1) * kMfmaChunk;
        for (int kk = 0; kk < nk; ++kk) {
            const int e = kk * 4 + kq;
            const float ve = sv[e];
            float a[ROWS], b[TC];
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int I = wave * ROWS + r;
                a[r] = I < TR ? s_xi[e * Wli + I * 16 + rc] * ve : 0.f;
            }
#pragma unroll
            for (int J = 0; J < TC; ++J) b[J] = s_xj[e * Wlj + J * 16 + rc];
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
#pragma unroll
                for (int J = 0; J < TC; ++J)
                    acc[r][J] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r], b[J], acc[r][J], 0, 0, 0);
        }
        if (ch % kBlkFlush == kBlkFlush - 1) flush();
        __syncthreads();
        if (more) commit_rows();
        commit_idx(ch & 1);
        fetch_idx(ch + 3);
        __syncthreads();
    }
    flush();
    float *o = part + (int64_t)it.slot * p * p;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int I = wave * ROWS + r;
        if (I >= TR) break;
#pragma unroll
        for (int J = 0; J < TC; ++J)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = (R0 + I) * 16 + 4 * kq + i, col = (C0 + J) * 16 + rc;
                if (row < p && col < p) o[(int64_t)row * p + col] = tot[r][J][i];
            }
    }
}

// ---------------------------------------------------------------- dispatch
template <typename VT, typename CT, int PA, int PB, int MODE>
void launch_wave(dim3 grid, size_t lds, hipStream_t s, const Item *items,
                 const int64_t *segptr, const int2 *c12, const int32_t *ck, const void *val,
                 const void *F1, const void *F2, const Geo &geo, void *out,
                 int64_t ldo, void *partial) {
    hipLaunchKernelGGL((ttmc_wave<VT, CT, PA, PB, MODE>), grid, dim3(64), lds, s, items,
                       segptr, c12, ck, static_cast<const VT *>(val),
                       static_cast<const CT *>(F1), static_cast<const CT *>(F2), geo,
                       static_cast<CT *>(out), ldo, static_cast<CT *>(partial));
}

using Launcher = void (*)(dim3, size_t, hipStream_t, const Item *, const int64_t *,
                          const int2 *, const int32_t *, const void *, const void *,
                          const void *, const Geo &, void *, int64_t, void *);

template <typename VT, typename CT, int MODE>
struct Table {
    Launcher f[kMaxP][kMaxP];
    Table() {
        fill<1>();
    }
    template <int PA>
    void fill() {
        fillb<PA, 1>();
        if constexpr (PA < kMaxP) fill<PA + 1>();
    }
    template <int PA, int PB>
    void fillb() {
        if constexpr (MODE == MODE_M3 && PA != 1) {
            f[PA - 1][PB - 1] = nullptr;
        } else {
            f[PA - 1][PB - 1] = &launch_wave<VT, CT, PA, PB, MODE>;
        }
        if constexpr (PB < kMaxP) fillb<PA, PB + 1>();
    }
};

template <typename VT, typename CT>
Launcher pick(int mode, int PA, int PB) {
    static Table<VT, CT, MODE_TWO> t0;
    static Table<VT, CT, MODE_ONE> t1;
    static Table<VT, CT, MODE_M3> t2;
    if (mode == MODE_TWO) return t0.f[PA - 1][PB - 1];
    if (mode == MODE_ONE) return t1.f[PA - 1][PB - 1];
    return t2.f[PA - 1][PB - 1];
}

// Pick the per-lane block size for width p: minimise padded width plus a
// per-lane-group penalty.
void choose_block(int p, int &P, int &ng) {
    double best = 1e30;
    for (int c = 1; c <= kMaxP; ++c) {
        int g = (p + c - 1) / c;
        double cost = g * c + 0.5 * g;
        if (cost < best - 1e-9) {
            best = cost;
            P = c;
            ng = g;
        }
    }
}

template <typename VT, typename CT>
void launch_sym_wide(const Segmented &o, const VT *val, const CT *X, int64_t ldx, int p,
                     CT *out, int64_t ldo, int64_t n, hipStream_t s) {
    const int ntile = (p + kTile - 1) / kTile;
    const int64_t blocks = n * (int64_t)(ntile * (ntile + 1) / 2);
    if (blocks == 0) return;
    hipLaunchKernelGGL((ttmc_sym_wide<VT, CT>), dim3((unsigned)blocks), dim3(256), 0, s,
                       o.segptr.as<int64_t>(), o.c1.as<int2>(), val, X,
                       ldx, p, ntile, out, ldo);
}

template <typename VT, typename CT, int R>
void launch_gram(dim3 grid, dim3 block, size_t lds, hipStream_t s, const Item *items,
                 const int2 *c12, const VT *val, const CT *Xp, int T, int RP, int p, CT *part) {
    hipLaunchKernelGGL((ttmc_sym_gram<VT, CT, R>), grid, block, lds, s, items, c12, val, Xp, T,
                       RP, p, part);
}

template <typename VT, typename CT>
bool launch_gram_r(int R, dim3 grid, dim3 block, size_t lds, hipStream_t s, const Item *items,
                   const int2 *c12, const VT *val, const CT *Xp, int T, int RP, int p, CT *part) {
    switch (R) {
    case 4: launch_gram<VT, CT, 4>(grid, block, lds, s, items, c12, val, Xp, T, RP, p, part); return true;
    case 5: launch_gram<VT, CT, 5>(grid, block, lds, s, items, c12, val, Xp, T, RP, p, part); return true;
    case 6: launch_gram<VT, CT, 6>(grid, block, lds, s, items, c12, val, Xp, T, RP, p, part); return true;
    case 7: launch_gram<VT, CT, 7>(grid, block, lds, s, items, c12, val, Xp, T, RP, p, part); return true;
    case 8: launch_gram<VT, CT, 8>(grid, block, lds, s, items, c12, val, Xp, T, RP, p, part); return true;
    default: break;
    }
    if constexpr (sizeof(CT) == 4) {
        switch (R) {
        case 9: launch_gram<VT, CT, 9>(grid, block, lds, s, items, c12, val, Xp, T, RP, p, part); return true;
        case 10: launch_gram<VT, CT, 10>(grid, block, lds, s, items, c12, val, Xp, T, RP, p, part); return true;
        case 11: launch_gram<VT, CT, 11>(grid, block, lds, s, items, c12, val, Xp, T, RP, p, part); return true;
        case 12: launch_gram<VT, CT, 12>(grid, block, lds, s, items, c12, val, Xp, T, RP, p, part); return true;
        default: break;
        }
    }
    return false;
}

template <int T, bool DIRECT>
void launch_mfma_t(dim3 grid, size_t lds, hipStream_t s, const Item *items, const int2 *c12,
                   const float *val, const float *Xp, int Wl, int p, float *part, float *out,
                   int64_t ldo) {
    constexpr int ROWS = T <= 8 ? 1 : 2;
    constexpr int NW = (T + ROWS - 1) / ROWS;
    hipLaunchKernelGGL((ttmc_sym_gram_mfma<float, T, ROWS, DIRECT>), grid, dim3(64 * NW), lds, s,
                       items, c12, val, Xp, Wl, p, part, out, ldo);
}

// FP32 Gram product on the matrix cores for 2 <= T = ceil(p / 16) <= 12;
// direct (one item per slice, output rows written by the kernel) for
// T <= kDirectMaxT.
constexpr int kDirectMaxT = 6;
constexpr int64_t kDirectMinSlices = 1024;   // items: 4 per CU at least
constexpr int64_t kDirectMaxLen = 16384;     // entries of the longest slice
bool launch_gram_mfma(int T, bool direct, dim3 grid, size_t lds, hipStream_t s,
                      const Item *items, const int2 *c12, const float *val, const float *Xp,
                      int Wl, int p, float *part, float *out, int64_t ldo) {
#define BKS_MFMA_CASE(TT)                                                                      \
    case TT:                                                                                   \
        if constexpr (TT <= kDirectMaxT) {                                                     \
            if (direct) {                                                                      \
                launch_mfma_t<TT, true>(grid, lds, s, items, c12, val, Xp, Wl, p, part, out,   \
                                        ldo);                                                  \
                return true;                                                                   \
            }                                                                                  \
        }                                                                                      \
        if (direct) return false;                                                              \
        launch_mfma_t<TT, false>(grid, lds, s, items, c12, val, Xp, Wl, p, part, out, ldo);    \
        return true;
    switch (T) {
        BKS_MFMA_CASE(2)
        BKS_MFMA_CASE(3)
        BKS_MFMA_CASE(4)
        BKS_MFMA_CASE(5)
        BKS_MFMA_CASE(6)
        BKS_MFMA_CASE(7)
        BKS_MFMA_CASE(8)
        BKS_MFMA_CASE(9)
        BKS_MFMA_CASE(10)
        BKS_MFMA_CASE(11)
        BKS_MFMA_CASE(12)
    default: return false;
    }
#undef BKS_MFMA_CASE
}

// Output rows of the slices with no entries (no item writes them in the
// direct form): zero.
__global__ void zero_empty_rows(const Fixup *__restrict__ fix, int q, float *__restrict__ out,
                                int64_t ldo) {
    const Fixup f = fix[blockIdx.x];
    if (f.nslots != 0) return;
    for (int c = threadIdx.x; c < q; c += blockDim.x) out[(int64_t)f.seg * ldo + c] = 0.f;
}

// Register tile R and thread grid T x T for width p: the fewest lane-FMAs
// per entry (whole waves x R^2) with T <= 16; R <= 12 (FP32) or 8 (FP64).
// false if p is too wide for one workgroup.
bool choose_gram(int p, bool dbl, int &R, int &T) {
    const int rmax = dbl ? 8 : 12;
    double best = 1e300;
    R = 0;
    for (int r = 4; r <= rmax; ++r) {
        const int t = (p + r - 1) / r;
        if (t > 16) continue;
        const int waves = (t * t + 63) / 64;
        const double cost = (double)waves * 64 * (r * r + 2 * r);
        if (cost < best) {
            best = cost;
            R = r;
            T = t;
        }
    }
    return R > 0;
}

}  // namespace

constexpr int kWideThreshold = 24;
constexpr int kWideThresholdPublic = kWideThreshold;

// Device workspace of one product call: regions 0 and 1 hold block-packed
// factor copies, 2 the partial rows of split segments, 3 intermediate
// products; plus the call's schedule.
struct TtmcWs {
    virtual ~TtmcWs() = default;
    virtual void *get(int which, size_t bytes) = 0;
    virtual SchedView sched(Tensor &t, int order, int E, hipStream_t s) = 0;
    virtual bool allow_wide() const = 0;
};

// The ctx's grow-only buffers and the tensor's cached device schedules.
struct CtxWs final : TtmcWs {
    Ctx &c;
    explicit CtxWs(Ctx &c_) : c(c_) {}
    void *get(int which, size_t bytes) override {
        DevBuf *b[4] = {&c.ws_fac1, &c.ws_fac2, &c.ws_partial, &c.ws_tmp};
        b[which]->ensure(bytes);
        return b[which]->ptr;
    }
    SchedView sched(Tensor &t, int order, int E, hipStream_t) override {
        const Schedule &sc = t.schedule(order, E);
        SchedView v;
        v.nitems = sc.nitems;
        v.nfix = sc.nfix;
        v.nslots = sc.nslots;
        v.items = sc.items.as<Item>();
        v.fix = sc.fix.as<Fixup>();
        for (const auto &L : sc.levels) v.levels.emplace_back(L->nfix, L->fix.as<Fixup>());
        return v;
    }
    bool allow_wide() const override { return true; }
};

// ---------------------------------------------------------------- scratch
// Fixed device scratch of the allocation-free product entry point: every
// workspace of a call is carved out of it in order.  Each device that loads
// the library holds its own copy for the life of the process.  Host code
// never names the array as an address: the per-device address comes from
// hipGetSymbolAddress at context creation (scratch_init).
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::vector<void *> g_scratch_ptr;  // by device id

static void *scratch_ptr(int device) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (device < 0 || device >= (int)g_scratch_ptr.size() || !g_scratch_ptr[device])
        fail(BKS_EDEVICE, "scratch not initialised on this device");
    return g_scratch_ptr[device];
}

struct ScratchWs final : TtmcWs {
    unsigned char *base;
    size_t off = 0;
    explicit ScratchWs(void *b) : base(static_cast<unsigned char *>(b)) {}
    void *take(size_t bytes) {
        const size_t at = (off + 255) & ~(size_t)255;
        if (at + bytes > kScratchBytes || at + bytes < at)
            fail(BKS_EINVAL, "the product needs " + std::to_string((at + bytes) >> 20) +
                                 " MiB of workspace, beyond the " +
                                 std::to_string(kScratchBytes >> 20) +
                                 " MiB scratch of the allocation-free entry point");
        off = at + bytes;
        return base + at;
    }
    void *get(int, size_t bytes) override { return take(bytes); }
    SchedView sched(Tensor &t, int order, int E, hipStream_t s) override {
        const HostSchedule *h;
        {
            std::lock_guard<std::mutex> g(t.sched_mu);
            h = &t.host_schedule(order, E);
        }
        SchedView v;
        v.nitems = (int64_t)h->items.size();
        v.nfix = (int64_t)h->fix.size();
        v.nslots = h->nslots;
        auto put = [&](const void *src, size_t bytes) -> void * {
            if (!bytes) return nullptr;
            void *d = take(bytes);
            // the host schedule is kept by the tensor, so the source outlives
            // the copy
            HIPCHECK(hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, s));
            return d;
        };
        v.items = static_cast<const Item *>(put(h->items.data(), h->items.size() * sizeof(Item)));
        v.fix = static_cast<const Fixup *>(put(h->fix.data(), h->fix.size() * sizeof(Fixup)));
        for (const auto &l : h->levels)
            v.levels.emplace_back((int64_t)l.size(),
                                  static_cast<const Fixup *>(put(l.data(), l.size() * sizeof(Fixup))));
        return v;
    }
    bool allow_wide() const override { return false; }
};

static void ttmc_launch(TtmcWs &ws, Tensor &t, int op, const void *B1, int64_t ld1, int p1,
                        const void *B2, int64_t ld2, int p2, bool sym_half, int prec, void *out,
                        int64_t ldo, hipStream_t s, hipEvent_t *mk = nullptr);

// What every segmented narrow product of one call shares.
struct NarrowArgs {
    TtmcWs &ws;
    Tensor &t;
    hipStream_t s;
    int prec;
    bool val64, dbl;
    size_t cts;
    hipEvent_t *mk;  // profiling: events around the call's main kernels, or NULL
    void mark(int w) {
        if (mk) HIPCHECK(hipEventRecord(mk[w], s));
    }
};
static void narrow(NarrowArgs &A, int mode, const Segmented &o, int fmt, const void *val,
                   const void *F1, int64_t l1, int64_t rows1, int px, const void *F2, int64_t l2,
                   int64_t rows2, int py, int outmode, int q, void *out, int64_t ldo, bool first,
                   bool last);

// Register-direct launchers, by precision, mode and widths (NULL where the
// kernel does not apply: more accumulators than a lane should hold).
using RegLauncher = void (*)(dim3, hipStream_t, const Item *, int64_t, const int64_t *,
                             const int2 *, const int32_t *, const void *, const void *, int,
                             const void *, int, void *, int64_t, void *, int);

template <typename CT, int MODE, int P1, int P2, bool SYM>
constexpr int reg_unroll() {
    constexpr int V = Vec<CT>::V;
    constexpr int r1 = (P1 + V - 1) / V * V * (int)sizeof(CT) / 4;
    constexpr int r2 = (P2 + V - 1) / V * V * (int)sizeof(CT) / 4;
    constexpr int per = 3 + (MODE == MODE_M3 ? r2
                                             : (MODE == MODE_ONE ? r1 + r2 : (SYM ? 2 * r1 : 2 * r1 + 2 * r2)));
    constexpr int u = 80 / per;
    return u < 1 ? 1 : (u > 8 ? 8 : u);
}

template <typename VT, typename CT, int MODE, int P1, int P2, bool SYM>
void launch_reg(dim3 grid, hipStream_t s, const Item *items, int64_t nitems, const int64_t *segptr,
                const int2 *c12, const int32_t *ck, const void *val, const void *F1, int W1,
                const void *F2, int W2, void *out, int64_t ldo, void *partial, int q) {
    constexpr int U = reg_unroll<CT, MODE, P1, P2, SYM>();
    hipLaunchKernelGGL((ttmc_reg<VT, CT, MODE, P1, P2, SYM, U>), grid, dim3(256), 0, s, items,
                       nitems, segptr, c12, ck, static_cast<const VT *>(val),
                       static_cast<const CT *>(F1), W1, static_cast<const CT *>(F2), W2,
                       static_cast<CT *>(out), ldo, static_cast<CT *>(partial), q);
}

constexpr int kRegDefaultMask = 8;
constexpr int kRegMaxP = 5;   // rectangular blocks up to 5 x 5
constexpr int kRegMaxSym = 6; // symmetric halves up to 6 (21 accumulators)
constexpr int kRegMaxM3 = 8;  // mode-3 rows up to 8

template <typename VT, typename CT>
struct RegTable {
    RegLauncher two[kRegMaxP][kRegMaxP], one[kRegMaxP][kRegMaxP], sym[kRegMaxSym], m3[kRegMaxM3];
    RegTable() {
        rect<1, 1>();
        syms<1>();
        m3s<1>();
    }
    template <int A, int B>
    void rect() {
        two[A - 1][B - 1] = &launch_reg<VT, CT, MODE_TWO, A, B, false>;
        one[A - 1][B - 1] = &launch_reg<VT, CT, MODE_ONE, A, B, false>;
        if constexpr (B < kRegMaxP) rect<A, B + 1>();
        else if constexpr (A < kRegMaxP) rect<A + 1, 1>();
    }
    template <int A>
    void syms() {
        sym[A - 1] = &launch_reg<VT, CT, MODE_TWO, A, A, true>;
        if constexpr (A < kRegMaxSym) syms<A + 1>();
    }
    template <int B>
    void m3s() {
        m3[B - 1] = &launch_reg<VT, CT, MODE_M3, 1, B, false>;
        if constexpr (B < kRegMaxM3) m3s<B + 1>();
    }
    RegLauncher get(int mode, bool sy, int px, int py) const {
        if (mode == MODE_M3) return py <= kRegMaxM3 ? m3[py - 1] : nullptr;
        if (mode == MODE_TWO && sy) return px <= kRegMaxSym ? sym[px - 1] : nullptr;
        if (px > kRegMaxP || py > kRegMaxP) return nullptr;
        return mode == MODE_TWO ? two[px - 1][py - 1] : one[px - 1][py - 1];
    }
};

// Which products take the register-direct kernel (the LDS-staged one
// otherwise): bit 0 FREE3 symmetric half, bit 1 FREE3 X != Y, bit 2 MODE3
// (also step 1 of FREE1), bit 3 step 2 of FREE1.  BKS_NARROW_REG overrides
// the default (read once; results differ only by rounding order).
int reg_mask() {
    static const int mask = [] {
        const char *e = std::getenv("BKS_NARROW_REG");
        return e ? std::atoi(e) : kRegDefaultMask;
    }();
    return mask;
}

RegLauncher reg_pick(int prec, bool val64, int mode, bool sym, int px, int py) {
    const int bit = mode == MODE_TWO ? (sym ? 1 : 2) : (mode == MODE_M3 ? 4 : 8);
    if (!(reg_mask() & bit)) return nullptr;
    static const RegTable<float, float> f;
    static const RegTable<double, double> d;
    static const RegTable<float, double> fd;
    if (prec == BKS_F32) return f.get(mode, sym, px, py);
    return val64 ? d.get(mode, sym, px, py) : fd.get(mode, sym, px, py);
}

// Algorithmic traffic and flops of one product: the stored tensor read once
// (two 4-byte indices and the value per stored entry; the mode-3 product
// reads one index), each factor read once, the output written once; 2 flops
// per fused multiply-add.
static void ttmc_cost(const Tensor &t, int op, int p1, int p2, bool sym, bool same, int prec,
                      std::string &name, double &bytes, double &flops) {
    const double eb = prec == BKS_F32 ? 4.0 : 8.0;
    const double vb = (prec == BKS_F64 && t.has64) ? 8.0 : 4.0;
    const double nnz = (double)t.nnz, m = (double)t.m, n = (double)t.n, P = (double)t.npairs;
    const char *suf = prec == BKS_F32 ? "_f32" : (prec == BKS_F64 ? "_f64" : "_f32in");
    if (op == BKS_FREE3) {
        const double px = p1, py = sym || same ? p1 : p2;
        const double q = sym ? px * (px + 1) / 2 : px * py;
        bytes = nnz * (8.0 + vb) + m * (px + (sym || same ? 0.0 : py)) * eb + n * q * eb;
        flops = sym ? 2.0 * nnz * px * px : 4.0 * nnz * px * py;
        name = std::string(sym ? (p1 > kWideThresholdPublic ? "free3_sym_wide" : "free3_sym") : "free3") + suf;
    } else if (op == BKS_FREE1) {
        bytes = nnz * (8.0 + vb) + m * p1 * eb + n * p2 * eb + m * (double)p1 * p2 * eb;
        flops = 4.0 * nnz * p1 * p2;
        name = std::string("free1") + suf;
    } else {
        bytes = nnz * (4.0 + vb) + P * 8.0 + n * p2 * eb + P * p2 * eb;
        flops = 2.0 * nnz * p2;
        name = std::string("mode3") + suf;
    }
}

void ttmc(Ctx &c, Tensor &t, int op, const void *B1, int64_t ld1, int p1, const void *B2,
          int64_t ld2, int p2, bool sym_half, int prec, void *out, int64_t ldo, hipStream_t s) {
    CtxWs ws(c);
    if (!c.prof) {
        ttmc_launch(ws, t, op, B1, ld1, p1, B2, ld2, p2, sym_half, prec, out, ldo, s);
        return;
    }
    // two classes per product: `name` times its main kernel alone (what a
    // kernel trace reports for it), `name_call` the whole call (factor
    // packing, split-segment fixup or chunk reduction included)
    hipEvent_t a, b, mk[2];
    HIPCHECK(hipEventCreate(&a));
    HIPCHECK(hipEventCreate(&b));
    HIPCHECK(hipEventCreate(&mk[0]));
    HIPCHECK(hipEventCreate(&mk[1]));
    HIPCHECK(hipEventRecord(a, s));
    ttmc_launch(ws, t, op, B1, ld1, p1, B2, ld2, p2, sym_half, prec, out, ldo, s, mk);
    HIPCHECK(hipEventRecord(b, s));
    std::string name;
    double bytes, flops;
    ttmc_cost(t, op, p1, p2, sym_half, B2 == nullptr || B2 == B1, prec, name, bytes, flops);
    c.prof_record(name, mk[0], mk[1], bytes, flops);
    c.prof_record(name + "_call", a, b, bytes, flops);
}

void gttmc(Ctx &c, Tensor &t, int mode, const void *B1, int64_t ld1, int p1, const void *B2,
           int64_t ld2, int p2, int prec, void *out, int64_t ldo, hipStream_t s) {
    if (!t.general) fail(BKS_EINVAL, "not a general tensor (use bks_ttmc)");
    if (mode < 0 || mode > 2) fail(BKS_EINVAL, "mode must be 0, 1 or 2");
    if (prec != BKS_F32 && prec != BKS_F64 && prec != BKS_F32IN_F64ACC)
        fail(BKS_EINVAL, "unknown precision");
    if (!B1 || !B2 || p1 < 1 || p2 < 1 || ld1 < p1 || ld2 < p2) fail(BKS_EINVAL, "bad factors");
    if (!out || ldo < (int64_t)p1 * p2) fail(BKS_EINVAL, "bad output");
    const int64_t dims[3] = {t.l, t.m, t.n};
    const int64_t rows1 = dims[mode == 0 ? 1 : 0], rows2 = dims[mode == 2 ? 1 : 2];
    const bool dbl = prec != BKS_F32;
    const bool val64 = prec == BKS_F64 && t.has64;
    const Segmented &o = t.g[mode];
    const void *val = val64 ? o.v64.ptr : o.v32.ptr;
    CtxWs ws(c);
    hipEvent_t a = nullptr, b = nullptr, mk[2] = {nullptr, nullptr};
    if (c.prof) {
        for (hipEvent_t *e : {&a, &b, &mk[0], &mk[1]}) HIPCHECK(hipEventCreate(e));
        HIPCHECK(hipEventRecord(a, s));
    }
    NarrowArgs na{ws, t, s, prec, val64, dbl, dbl ? (size_t)8 : (size_t)4, c.prof ? mk : nullptr};
    narrow(na, MODE_ONE, o, 4 + mode, val, B1, ld1, rows1, p1, B2, ld2, rows2, p2, OUT_RECT,
           p1 * p2, out, ldo, true, true);
    if (c.prof) {
        HIPCHECK(hipEventRecord(b, s));
        // algorithmic traffic: the entry stream once (two indices, value),
        // both factors and the output once
        const double vb = val64 ? 8.0 : 4.0, eb = dbl ? 8.0 : 4.0;
        const double bytes = t.nnz * (8.0 + vb) + (rows1 * p1 + rows2 * p2) * eb +
                             (double)dims[mode] * p1 * p2 * eb;
        const double flops = 2.0 * t.nnz * p1 * p2;
        const std::string name = "gmode" + std::to_string(mode + 1) + (dbl ? "_f64" : "_f32");
        c.prof_record(name, mk[0], mk[1], bytes, flops);
        c.prof_record(name + "_call", a, b, bytes, flops);
    }
}

void ttmc_noalloc(Ctx &c, Tensor &t, int op, const void *B1, int64_t ld1, int p1,
                  const void *B2, int64_t ld2, int p2, bool sym_half, int prec, void *out,
                  int64_t ldo, hipStream_t s) {
    ScratchWs ws(scratch_ptr(c.device));
    ttmc_launch(ws, t, op, B1, ld1, p1, B2, ld2, p2, sym_half, prec, out, ldo, s);
}

void scratch_init(int device) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (device >= (int)g_scratch_ptr.size()) g_scratch_ptr.resize(device + 1, nullptr);
    if (g_scratch_ptr[device]) return;
    void *p = nullptr;
    // the caller made `device` current; each device has its own copy
    HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(BKS_EDEVICE, "no device address for the scratch array");
    g_scratch_ptr[device] = p;
}

size_t scratch_bytes() { return kScratchBytes; }

void Ctx::prof_record(const std::string &name, hipEvent_t a, hipEvent_t b, double bytes,
                      double flops) {
    std::lock_guard<std::mutex> g(prof_mu);
    ProfClass &pc = prof_stats[name];
    pc.calls += 1;
    pc.bytes += bytes;
    pc.flops += flops;
    pc.pending.emplace_back(a, b);
}

void Ctx::prof_flush() {
    std::lock_guard<std::mutex> g(prof_mu);
    for (auto &kv : prof_stats) {
        for (auto &ev : kv.second.pending) {
            HIPCHECK(hipEventSynchronize(ev.second));
            float ms = 0.f;
            HIPCHECK(hipEventElapsedTime(&ms, ev.first, ev.second));
            kv.second.ms += ms;
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
        kv.second.pending.clear();
    }
}

static void ttmc_launch(TtmcWs &ws, Tensor &t, int op, const void *B1, int64_t ld1, int p1,
                        const void *B2, int64_t ld2, int p2, bool sym_half, int prec, void *out,
                        int64_t ldo, hipStream_t s, hipEvent_t *mk) {
    // mk (profiling): events recorded right around the product's main kernel
    auto mark = [&](int w) {
        if (mk) HIPCHECK(hipEventRecord(mk[w], s));
    };
    if (prec != BKS_F32 && prec != BKS_F64 && prec != BKS_F32IN_F64ACC)
        fail(BKS_EINVAL, "unknown precision");
    const bool dbl = prec != BKS_F32;
    const bool val64 = (prec == BKS_F64) && t.has64;
    const size_t cts = dbl ? 8 : 4;
    int mode, outmode = OUT_RECT, order;
    int px, py;
    const void *F1 = B1, *F2 = B2;
    int64_t l1 = ld1, l2 = ld2;
    int q;
    if (op == BKS_FREE3) {
        if (p1 < 1 || !B1 || ld1 < p1) fail(BKS_EINVAL, "FREE3: bad X");
        order = 0;
        mode = MODE_TWO;
        px = p1;
        if (sym_half) {
            if (B2 && B2 != B1) fail(BKS_EINVAL, "sym_half needs Y = X");
            F2 = B1;
            l2 = ld1;
            py = p1;
            outmode = OUT_SYM;
            q = p1 * (p1 + 1) / 2;
        } else {
            if (!B2) {
                F2 = B1;
                l2 = ld1;
                py = p1;
            } else {
                if (p2 < 1 || ld2 < p2) fail(BKS_EINVAL, "FREE3: bad Y");
                py = p2;
            }
            q = px * py;
        }
        if (ldo < q) fail(BKS_EINVAL, "ldo too small");
    } else if (op == BKS_FREE1) {
        if (p1 < 1 || p2 < 1 || !B1 || !B2 || ld1 < p1 || ld2 < p2)
            fail(BKS_EINVAL, "FREE1: bad factors");
        order = 1;
        mode = MODE_ONE;
        px = p1;
        py = p2;
        q = px * py;
        if (ldo < q) fail(BKS_EINVAL, "ldo too small");
    } else if (op == BKS_MODE3) {
        if (p2 < 1 || !B2 || ld2 < p2) fail(BKS_EINVAL, "MODE3: bad Z");
        order = 2;
        mode = MODE_M3;
        px = 1;
        py = p2;
        F1 = nullptr;
        l1 = 0;
        q = py;
        if (ldo < q) fail(BKS_EINVAL, "ldo too small");
    } else {
        fail(BKS_EINVAL, "unknown op");
    }
    if (!out) fail(BKS_EINVAL, "null output");
    if (t.general) fail(BKS_EINVAL, "a general tensor: use bks_gttmc");
    const Segmented &o = order == 0 ? t.o3 : t.op;
    if (op != BKS_FREE1 && o.nseg == 0) {
        mark(0);
        mark(1);
        return;
    }
    const void *val = val64 ? o.v64.ptr : o.v32.ptr;

    if (op == BKS_FREE3 && outmode == OUT_SYM && px > kWideThreshold) {
        if (!ws.allow_wide())
            fail(BKS_EINVAL, "symmetric halves wider than " + std::to_string(kWideThreshold) +
                                 " columns need bks_ttmc (the allocation-free entry point "
                                 "runs the narrow products only)");
        int R, T;
        // FP32: the matrix-core kernel (tiles of 16) for widths up to 192
        const int T16 = (px + 15) / 16;
        // beyond 12 tiles: the same matrix-core product in 8 x 8-tile blocks
        const bool blocked = prec == BKS_F32 && T16 > 12;
        const bool mfma = prec == BKS_F32 && T16 >= 2;
        if (mfma) {
            R = 16;
            T = T16;
        }
        if (mfma || choose_gram(px, dbl, R, T)) {
            const int V = dbl ? 2 : 4;
            const int RP = mfma ? 16 : pad_to(R, V), W = T * RP;
            // chunk width: about kGramItems chunks in all (enough waves to hide
            // the staging latency), 256..2048 entries, and at most ~512 MB
            // of partial matrices
            const double per_item = (double)px * px * cts;
            const int64_t max_items = std::max<int64_t>(o.nseg + 1, (int64_t)(536870912.0 / per_item));
            int64_t cw64 = std::min<int64_t>(2048, std::max<int64_t>(256, t.nnz / kGramItems));
            cw64 = std::max<int64_t>(cw64, t.nnz / std::max<int64_t>(1, max_items - o.nseg) + 1);
            // direct form (one workgroup per slice writes its output row, no
            // partials): narrow enough for M in LDS, slices many enough to
            // fill the chip and short enough for one FP32 accumulator chain
            bool direct = false;
            if (mfma && !blocked && T16 <= kDirectMaxT && o.nseg >= kDirectMinSlices) {
                int64_t maxlen = 0;
                for (int64_t k = 0; k < o.nseg; ++k)
                    maxlen = std::max<int64_t>(maxlen, o.h_segptr[k + 1] - o.h_segptr[k]);
                direct = maxlen <= kDirectMaxLen;
            }
            const int CW = direct ? (1 << 30) : (int)std::min<int64_t>(cw64, 1 << 30);
            const SchedView sc = ws.sched(t, kWideOrder, CW, s);
            void *fac = ws.get(0, (size_t)std::max<int64_t>(t.m, 1) * W * cts);
            void *part = sc.nitems > 0 && !direct ? ws.get(2, (size_t)sc.nitems * px * px * cts)
                                                  : nullptr;
            {
                const int64_t total = t.m * W;
                const unsigned grid = (unsigned)std::max<int64_t>(
                    1, std::min<int64_t>((total + 255) / 256, 4096));
                if (dbl)
                    hipLaunchKernelGGL(pack_blocks<double>, dim3(grid), dim3(256), 0, s,
                                       static_cast<const double *>(F1), l1, t.m, px, R, RP, W,
                                       static_cast<double *>(fac));
                else
                    hipLaunchKernelGGL(pack_blocks<float>, dim3(grid), dim3(256), 0, s,
                                       static_cast<const float *>(F1), l1, t.m, px, R, RP, W,
                                       static_cast<float *>(fac));
                HIPCHECK(hipGetLastError());
            }
            if (blocked) {
                constexpr int TB = 8;
                const int nb = (T16 + TB - 1) / TB;
                const int Wb = TB * 16 + ((16 - (TB * 16) % 64) + 64) % 64;
                const size_t lds_b = (size_t)(2 * kMfmaChunk * Wb + 2 * kMfmaChunk) * 4 +
                                     (size_t)2 * kMfmaChunk * 8;
                mark(0);
                if (sc.nitems > 0) {
                    hipLaunchKernelGGL((ttmc_sym_gram_mfma_blk<float, TB, TB, 1>),
                                       dim3((unsigned)sc.nitems, (unsigned)(nb * nb)),
                                       dim3(64 * TB), lds_b, s, sc.items, o.c1.as<int2>(),
                                       o.v32.as<float>(), static_cast<const float *>(fac), T16,
                                       Wb, Wb, px, static_cast<float *>(part));
                    HIPCHECK(hipGetLastError());
                }
                mark(1);
                if (sc.nfix > 0) {
                    hipLaunchKernelGGL(sym_gram_reduce<float>, dim3((unsigned)sc.nfix), dim3(256), 0,
                                       s, sc.fix, static_cast<const float *>(part), px,
                                       static_cast<float *>(out), ldo);
                    HIPCHECK(hipGetLastError());
                }
                return;
            }
            if (mfma) {
                // row stride with (Wl * 4) % 256 == 64: the four 16-float rows a
                // K-step reads fall in different banks
                const int Wl = W + ((16 - W % 64) + 64) % 64;
                size_t lds_m = (size_t)(2 * kMfmaChunk * Wl + 2 * kMfmaChunk) * 4 +
                               (size_t)2 * kMfmaChunk * 8;
                if (direct) lds_m = std::max<size_t>(lds_m, (size_t)px * px * 4);
                mark(0);
                if (sc.nitems > 0) {
                    if (!launch_gram_mfma(T, direct, dim3((unsigned)sc.nitems), lds_m, s, sc.items,
                                          o.c1.as<int2>(), o.v32.as<float>(),
                                          static_cast<const float *>(fac), Wl, px,
                                          static_cast<float *>(part), static_cast<float *>(out),
                                          ldo))
                        fail(BKS_EINVAL, "no matrix-core kernel for this width");
                    HIPCHECK(hipGetLastError());
                }
                mark(1);
                if (direct) {
                    if (sc.nfix > 0) {
                        hipLaunchKernelGGL(zero_empty_rows, dim3((unsigned)sc.nfix), dim3(256), 0, s,
                                           sc.fix, px * (px + 1) / 2, static_cast<float *>(out),
                                           ldo);
                        HIPCHECK(hipGetLastError());
                    }
                    return;
                }
                if (sc.nfix > 0) {
                    hipLaunchKernelGGL(sym_gram_reduce<float>, dim3((unsigned)sc.nfix), dim3(256), 0,
                                       s, sc.fix, static_cast<const float *>(part), px,
                                       static_cast<float *>(out), ldo);
                    HIPCHECK(hipGetLastError());
                }
                return;
            }
            const dim3 block((unsigned)((T * T + 63) / 64 * 64));
            const size_t lds = (size_t)(2 * kGramChunk * W + pad_to(kGramChunk, V)) * cts +
                               (size_t)kGramChunk * 8;
            bool ok = true;
            mark(0);
            if (sc.nitems > 0) {
                const dim3 grid((unsigned)sc.nitems);
                if (prec == BKS_F32)
                    ok = launch_gram_r<float, float>(R, grid, block, lds, s, sc.items,
                                                     o.c1.as<int2>(), o.v32.as<float>(),
                                                     static_cast<const float *>(fac), T, RP, px,
                                                     static_cast<float *>(part));
                else if (val64)
                    ok = launch_gram_r<double, double>(R, grid, block, lds, s, sc.items,
                                                       o.c1.as<int2>(), o.v64.as<double>(),
                                                       static_cast<const double *>(fac), T, RP, px,
                                                       static_cast<double *>(part));
                else
                    ok = launch_gram_r<float, double>(R, grid, block, lds, s, sc.items,
                                                      o.c1.as<int2>(), o.v32.as<float>(),
                                                      static_cast<const double *>(fac), T, RP, px,
                                                      static_cast<double *>(part));
                HIPCHECK(hipGetLastError());
            }
            mark(1);
            if (!ok) fail(BKS_EINVAL, "no wide kernel for this width");
            if (sc.nfix > 0) {
                if (dbl)
                    hipLaunchKernelGGL(sym_gram_reduce<double>, dim3((unsigned)sc.nfix), dim3(256),
                                       0, s, sc.fix, static_cast<const double *>(part), px,
                                       static_cast<double *>(out), ldo);
                else
                    hipLaunchKernelGGL(sym_gram_reduce<float>, dim3((unsigned)sc.nfix), dim3(256),
                                       0, s, sc.fix, static_cast<const float *>(part), px,
                                       static_cast<float *>(out), ldo);
                HIPCHECK(hipGetLastError());
            }
            return;
        }
        mark(0);
        if (prec == BKS_F32)
            launch_sym_wide<float, float>(o, o.v32.as<float>(), static_cast<const float *>(F1),
                                          l1, px, static_cast<float *>(out), ldo, o.nseg, s);
        else if (val64)
            launch_sym_wide<double, double>(o, o.v64.as<double>(),
                                            static_cast<const double *>(F1), l1, px,
                                            static_cast<double *>(out), ldo, o.nseg, s);
        else
            launch_sym_wide<float, double>(o, o.v32.as<float>(),
                                           static_cast<const double *>(F1), l1, px,
                                           static_cast<double *>(out), ldo, o.nseg, s);
        mark(1);
        HIPCHECK(hipGetLastError());
        return;
    }

    // Narrow products: the register-direct kernel where one lane holds the
    // whole output block, else the LDS-staged kernel.  FREE1 runs in two
    // steps over the stored pairs, so that every stored entry is read once:
    // t = A.(Z)_3 on the pair pattern, then T1(r, :) = sum over the pairs
    // (r, c) and (c, r) of Y(c, :) (x) t(pair, :).
    NarrowArgs na{ws, t, s, prec, val64, dbl, cts, mk};
    if (op == BKS_FREE3) {
        narrow(na, MODE_TWO, t.o3, 0, val, F1, l1, t.m, px, F2, l2, t.m, py, outmode,
               q, out, ldo, true, true);
        return;
    }
    if (op == BKS_MODE3) {
        narrow(na, MODE_M3, t.op, 2, val, nullptr, 0, 0, 1, F2, l2, t.n, py, OUT_RECT, q, out,
               ldo, true, true);
        return;
    }
    // FREE1, step 1: t = A.(Z)_3 into the intermediate region, with rows
    // padded to whole 16-byte vectors (the second step gathers them)
    const int V = dbl ? 2 : 4;
    const int Wt = pad_to(py, V);
    void *tmid = ws.get(3, (size_t)std::max<int64_t>(t.npairs, 1) * Wt * cts);
    if (t.npairs > 0)
        narrow(na, MODE_M3, t.op, 2, val, nullptr, 0, 0, 1, F2, l2, t.n, py, OUT_RECT, py, tmid,
               Wt, true, false);
    // step 2: pair rows, no values; t plays the part of the mode-3 factor
    narrow(na, MODE_ONE, t.pr, 1, nullptr, F1, l1, t.m, px, tmid, Wt, t.npairs, py, OUT_RECT, q,
           out, ldo, t.npairs == 0, true);
}

// One segmented narrow product (see ttmc_launch).  mode MODE_TWO: entries
// (i, j, v) of `o`, factors F1 (and F2) with rows1 rows; MODE_M3: entries
// (k, v), factor F2; MODE_ONE: entries (col, k) and values `val` (NULL: all
// one), factors F1 (rows1) and F2 (rows2).  first / last: whether the
// profiling marks around the main kernels open / close here.
static void narrow(NarrowArgs &A, int mode, const Segmented &o, int fmt, const void *val,
                   const void *F1, int64_t l1, int64_t rows1, int px, const void *F2, int64_t l2,
                   int64_t rows2, int py, int outmode, int q, void *out, int64_t ldo, bool first,
                   bool last) {
    TtmcWs &ws = A.ws;
    Tensor &t = A.t;
    hipStream_t s = A.s;
    const bool dbl = A.dbl;
    const size_t cts = A.cts;
    const int prec = A.prec;
    const int V = dbl ? 2 : 4;
    auto pack = [&](int which, const void *F, int64_t ld, int64_t rows, int p, int P, int PAD,
                    int W) -> const void * {
        void *dst = ws.get(which, (size_t)std::max<int64_t>(rows, 1) * W * cts);
        const int64_t total = rows * W;
        const unsigned grid = (unsigned)std::max<int64_t>(
            1, std::min<int64_t>((total + 255) / 256, 4096));
        if (total > 0) {
            if (dbl)
                hipLaunchKernelGGL(pack_blocks<double>, dim3(grid), dim3(256), 0, s,
                                   static_cast<const double *>(F), ld, rows, p, P, PAD, W,
                                   static_cast<double *>(dst));
            else
                hipLaunchKernelGGL(pack_blocks<float>, dim3(grid), dim3(256), 0, s,
                                   static_cast<const float *>(F), ld, rows, p, P, PAD, W,
                                   static_cast<float *>(dst));
            HIPCHECK(hipGetLastError());
        }
        return dst;
    };
    auto fixups = [&](const SchedView &sc, void *partial) {
        for (const auto &L : sc.levels) {
            if (dbl)
                hipLaunchKernelGGL(ttmc_fixup<double>, dim3((unsigned)L.first), dim3(256), 0, s,
                                   L.second, static_cast<const double *>(partial), q,
                                   static_cast<double *>(partial), (int64_t)q);
            else
                hipLaunchKernelGGL(ttmc_fixup<float>, dim3((unsigned)L.first), dim3(256), 0, s,
                                   L.second, static_cast<const float *>(partial), q,
                                   static_cast<float *>(partial), (int64_t)q);
            HIPCHECK(hipGetLastError());
        }
        if (sc.nfix > 0) {
            if (dbl)
                hipLaunchKernelGGL(ttmc_fixup<double>, dim3((unsigned)sc.nfix), dim3(256), 0, s,
                                   sc.fix, static_cast<const double *>(partial), q,
                                   static_cast<double *>(out), ldo);
            else
                hipLaunchKernelGGL(ttmc_fixup<float>, dim3((unsigned)sc.nfix), dim3(256), 0, s,
                                   sc.fix, static_cast<const float *>(partial), q,
                                   static_cast<float *>(out), ldo);
            HIPCHECK(hipGetLastError());
        }
    };
    const bool same = mode == MODE_TWO && F2 == F1 && l2 == l1 && py == px;
    const bool sym = outmode == OUT_SYM;

    // register-direct kernel
    RegLauncher rfn = reg_pick(prec, A.val64, mode, sym, px, py);
    if (rfn) {
        const int PAD1 = pad_to(px, V), PAD2 = pad_to(py, V);
        const void *P1 = nullptr, *P2 = nullptr;
        int W1 = 0, W2 = 0;
        if (mode != MODE_M3) {
            P1 = pack(0, F1, l1, rows1, px, px, PAD1, PAD1);
            W1 = PAD1;
        }
        if (mode == MODE_M3 || mode == MODE_ONE || !sym) {
            if (mode == MODE_ONE && fmt == 1) {
                // the intermediate t of FREE1 arrives padded: gathered in place
                P2 = F2;
                W2 = (int)l2;
            } else if (same) {
                P2 = P1;
                W2 = W1;
            } else {
                P2 = pack(1, F2, l2, rows2, py, py, PAD2, PAD2);
                W2 = PAD2;
            }
        }
        const SchedView sc = ws.sched(t, kGroupOrder + fmt, 0, s);
        void *partial = sc.nslots > 0 ? ws.get(2, (size_t)sc.nslots * q * cts) : nullptr;
        if (first) A.mark(0);
        if (sc.nitems > 0)
            rfn(dim3((unsigned)((sc.nitems + 3) / 4)), s, sc.items, sc.nitems,
                o.segptr.as<int64_t>(), mode == MODE_M3 ? nullptr : o.c1.as<int2>(),
                mode == MODE_M3 ? o.c2.as<int32_t>() : nullptr, val, P1, W1, P2, W2, out, ldo,
                partial, q);
        HIPCHECK(hipGetLastError());
        fixups(sc, partial);
        if (last) A.mark(1);
        return;
    }

    // LDS-staged kernel (several lanes per entry)
    int PA, ga, PB, gb;
    int G;
    if (mode == MODE_M3) {
        PA = 1;
        ga = 1;
        choose_block(py, PB, gb);
        G = gb;
        if (G > 64) fail(BKS_EINVAL, "MODE3 width too large");
    } else if (sym) {
        choose_block(px, PA, ga);
        PB = PA;
        gb = ga;
        G = ga * (ga + 1) / 2;
        if (G > 64) fail(BKS_EINVAL, "width too large");
    } else {
        choose_block(px, PA, ga);
        choose_block(py, PB, gb);
        G = ga * gb;
        if (G > 64) fail(BKS_EINVAL, "widths too large for the narrow kernel");
    }
    const int E = 64 / G;
    Geo geo;
    std::memset(&geo, 0, sizeof(geo));
    geo.px = px;
    geo.py = py;
    geo.G = G;
    geo.ga = ga;
    geo.outmode = outmode;
    geo.q = q;
    geo.same = same ? 1 : 0;
    geo.PAD1 = pad_to(PA, V);
    geo.PAD2 = pad_to(PB, V);
    geo.W1 = mode == MODE_M3 ? 0 : ga * geo.PAD1;
    geo.W2 = gb * geo.PAD2;
    const int nA = mode == MODE_TWO ? 2 : (mode == MODE_ONE ? 1 : 0);
    const int nB = mode == MODE_TWO ? (geo.same ? 0 : 2) : 1;
    // entries per batch: fill the staging budget, a multiple of E when possible
    const size_t bpe = 8 + 2 * cts + (size_t)(nA * geo.W1 + nB * geo.W2) * cts;
    int NB = (int)std::min<size_t>(64 * kIdxRegs, std::max<size_t>(1, kStageBytes / bpe));
    if (NB >= E) NB = NB / E * E;
    geo.NB = NB;
    geo.offv = pad_to((int)((size_t)NB * 8 / cts), V);
    geo.offw = geo.offv + pad_to(NB, V);
    geo.PS = pad_to(NB, 8) + 4;  // staggers the planes' banks (see stage_rows)
    geo.offa = geo.offw + pad_to(NB, V);
    geo.offb = geo.offa + geo.PS * nA * geo.W1;
    const size_t lds_elems = (size_t)geo.offb + (size_t)geo.PS * nB * geo.W2;
    const size_t lds = std::max(lds_elems, (size_t)64 * PA * PB) * cts;
    if (lds > 65536) fail(BKS_EINVAL, "widths too large for the narrow kernel");

    // block-pack the factors
    const void *P1 = nullptr, *P2 = nullptr;
    if (mode == MODE_TWO) {
        P1 = pack(0, F1, l1, rows1, px, PA, geo.PAD1, geo.W1);
        P2 = geo.same ? P1 : pack(1, F2, l2, rows2, py, PB, geo.PAD2, geo.W2);
    } else if (mode == MODE_ONE) {
        P1 = pack(0, F1, l1, rows1, px, PA, geo.PAD1, geo.W1);
        P2 = pack(1, F2, l2, rows2, py, PB, geo.PAD2, geo.W2);
    } else {
        P2 = pack(1, F2, l2, rows2, py, PB, geo.PAD2, geo.W2);
    }

    const SchedView sc = ws.sched(t, fmt, E, s);
    void *partial = sc.nslots > 0 ? ws.get(2, (size_t)sc.nslots * q * cts) : nullptr;
    Launcher fn;
    if (prec == BKS_F32)
        fn = pick<float, float>(mode, PA, PB);
    else if (A.val64)
        fn = pick<double, double>(mode, PA, PB);
    else
        fn = pick<float, double>(mode, PA, PB);
    if (!fn) fail(BKS_EINVAL, "no kernel for this width");
    if (first) A.mark(0);
    if (sc.nitems > 0)
        fn(dim3((unsigned)sc.nitems), lds, s, sc.items, o.segptr.as<int64_t>(),
           mode == MODE_M3 ? nullptr : o.c1.as<int2>(),
           mode == MODE_M3 ? o.c2.as<int32_t>() : nullptr, val, P1, P2, geo, out, ldo,
           partial);
    HIPCHECK(hipGetLastError());
    fixups(sc, partial);
    if (last) A.mark(1);
}

}  // namespace bks
