// Tensor-times-block products over a stored (1,2)-symmetric tensor
// (Section 2.2 mode products; Algorithm 3 step (i); Section 3.3.1).
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
#include <cstring>

#include "bks_internal.h"

namespace bks {

namespace {

constexpr int kMaxP = 5;

enum { MODE_TWO = 0, MODE_ONE = 1, MODE_M3 = 2 };
enum { OUT_RECT = 0, OUT_SYM = 1 };

struct BlockMap {
    int8_t a[64];
    int8_t b[64];
};

template <typename CT, typename VT>
__device__ __forceinline__ CT cv(VT v) {
    return static_cast<CT>(v);
}

template <typename VT, typename CT, int PA, int PB, int MODE>
__device__ __forceinline__ void accumulate(int64_t e, const int32_t *__restrict__ c1,
                                           const int32_t *__restrict__ c2,
                                           const VT *__restrict__ val,
                                           const CT *__restrict__ F1, int64_t ld1,
                                           const CT *__restrict__ F2, int64_t ld2, int a0,
                                           int b0, int px, int py, CT (&acc)[PA][PB]) {
    const int i2 = c2[e];
    const CT v = cv<CT>(val[e]);
    CT yb[PB];
#pragma unroll
    for (int b = 0; b < PB; ++b)
        yb[b] = (b0 + b < py) ? F2[(int64_t)i2 * ld2 + b0 + b] : CT(0);
    if constexpr (MODE == MODE_M3) {
#pragma unroll
        for (int b = 0; b < PB; ++b) acc[0][b] += v * yb[b];
    } else {
        const int i1 = c1[e];
        CT xa[PA];
#pragma unroll
        for (int a = 0; a < PA; ++a)
            xa[a] = (a0 + a < px) ? v * F1[(int64_t)i1 * ld1 + a0 + a] : CT(0);
#pragma unroll
        for (int a = 0; a < PA; ++a)
#pragma unroll
            for (int b = 0; b < PB; ++b) acc[a][b] = fma(xa[a], yb[b], acc[a][b]);
        if constexpr (MODE == MODE_TWO) {
            // mirrored entry (j, i, k); absent on the diagonal i == j
            const CT w = (i1 != i2) ? v : CT(0);
            CT xa2[PA], yb2[PB];
#pragma unroll
            for (int a = 0; a < PA; ++a)
                xa2[a] = (a0 + a < px) ? w * F1[(int64_t)i2 * ld1 + a0 + a] : CT(0);
#pragma unroll
            for (int b = 0; b < PB; ++b)
                yb2[b] = (b0 + b < py) ? F2[(int64_t)i1 * ld2 + b0 + b] : CT(0);
#pragma unroll
            for (int a = 0; a < PA; ++a)
#pragma unroll
                for (int b = 0; b < PB; ++b) acc[a][b] = fma(xa2[a], yb2[b], acc[a][b]);
        }
    }
}

__device__ __forceinline__ int out_col(int alpha, int beta, int px, int outmode) {
    if (outmode == OUT_SYM) return beta * (beta + 1) / 2 + alpha;
    return alpha + px * beta;
}

template <typename VT, typename CT, int PA, int PB, int MODE>
__global__ __launch_bounds__(64) void ttmc_wave(
    const Item *__restrict__ items, const int64_t *__restrict__ segptr,
    const int32_t *__restrict__ c1, const int32_t *__restrict__ c2,
    const VT *__restrict__ val, const CT *__restrict__ F1, int64_t ld1,
    const CT *__restrict__ F2, int64_t ld2, int px, int py, int G, BlockMap bm,
    CT *__restrict__ out, int64_t ldo, CT *__restrict__ partial, int q, int outmode) {
    __shared__ CT red[64 * PA * PB];
    const Item it = items[blockIdx.x];
    const int lane = threadIdx.x;
    const int E = 64 / G;
    const int el = lane / G;
    const int g = lane - el * G;
    const bool active = el < E;
    const int a0 = active ? bm.a[g] * PA : 0;
    const int b0 = active ? bm.b[g] * PB : 0;
    CT acc[PA][PB];
#pragma unroll
    for (int a = 0; a < PA; ++a)
#pragma unroll
        for (int b = 0; b < PB; ++b) acc[a][b] = CT(0);

    if (it.seg_end < 0) {
        // heavy: one chunk of one segment
        if (active)
            for (int64_t e = it.beg + el; e < it.end; e += E)
                accumulate<VT, CT, PA, PB, MODE>(e, c1, c2, val, F1, ld1, F2, ld2, a0, b0, px,
                                                 py, acc);
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
            const int alpha = bm.a[gg] * PA + a, beta = bm.b[gg] * PB + b;
            if (alpha >= px || beta >= py) continue;
            if (outmode == OUT_SYM && alpha > beta) continue;
            CT s = CT(0);
            for (int x = 0; x < E; ++x) s += red[(x * G + gg) * PA * PB + ab];
            const int col = out_col(alpha, beta, px, outmode);
            if (it.slot < 0)
                out[(int64_t)it.seg * ldo + col] = s;
            else
                partial[(int64_t)it.slot * q + col] = s;
        }
    } else {
        // light: whole short segments, one lane group each
        const int64_t seg = (int64_t)it.seg + el;
        if (active && seg < it.seg_end) {
            const int64_t e1 = segptr[seg + 1];
            for (int64_t e = segptr[seg]; e < e1; ++e)
                accumulate<VT, CT, PA, PB, MODE>(e, c1, c2, val, F1, ld1, F2, ld2, a0, b0, px,
                                                 py, acc);
#pragma unroll
            for (int a = 0; a < PA; ++a)
#pragma unroll
                for (int b = 0; b < PB; ++b) {
                    const int alpha = a0 + a, beta = b0 + b;
                    if (alpha < px && beta < py && (outmode == OUT_RECT || alpha <= beta))
                        out[seg * ldo + out_col(alpha, beta, px, outmode)] = acc[a][b];
                }
        }
    }
}

// Sum the partial rows of one split segment: 256 threads as (slot lane,
// column); each lane sums a strided subset of the slots, then a fixed-order
// tree over the lanes in LDS (deterministic).
template <typename CT>
__global__ __launch_bounds__(256) void ttmc_fixup(const Fixup *__restrict__ fix,
                                                  const CT *__restrict__ partial, int q,
                                                  CT *__restrict__ out, int64_t ldo) {
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
    const int64_t *__restrict__ segptr, const int32_t *__restrict__ ci,
    const int32_t *__restrict__ cj, const VT *__restrict__ val, const CT *__restrict__ X,
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
                const int i = ci[ee], j = cj[ee];
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

// ---------------------------------------------------------------- dispatch
using WaveFn = void (*)(const Item *, const int64_t *, const int32_t *, const int32_t *,
                        const void *, const void *, int64_t, const void *, int64_t, int, int,
                        int, BlockMap, void *, int64_t, void *, int, int);

template <typename VT, typename CT, int PA, int PB, int MODE>
void launch_wave(dim3 grid, hipStream_t s, const Item *items, const int64_t *segptr,
                 const int32_t *c1, const int32_t *c2, const void *val, const void *F1,
                 int64_t ld1, const void *F2, int64_t ld2, int px, int py, int G,
                 const BlockMap &bm, void *out, int64_t ldo, void *partial, int q,
                 int outmode) {
    hipLaunchKernelGGL((ttmc_wave<VT, CT, PA, PB, MODE>), grid, dim3(64), 0, s, items, segptr,
                       c1, c2, static_cast<const VT *>(val), static_cast<const CT *>(F1), ld1,
                       static_cast<const CT *>(F2), ld2, px, py, G, bm,
                       static_cast<CT *>(out), ldo, static_cast<CT *>(partial), q, outmode);
}

using Launcher = void (*)(dim3, hipStream_t, const Item *, const int64_t *, const int32_t *,
                          const int32_t *, const void *, const void *, int64_t, const void *,
                          int64_t, int, int, int, const BlockMap &, void *, int64_t, void *,
                          int, int);

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
                       o.segptr.as<int64_t>(), o.c1.as<int32_t>(), o.c2.as<int32_t>(), val, X,
                       ldx, p, ntile, out, ldo);
}

}  // namespace

constexpr int kWideThreshold = 24;
constexpr int kWideThresholdPublic = kWideThreshold;

static void ttmc_launch(Ctx &c, Tensor &t, int op, const void *B1, int64_t ld1, int p1,
                        const void *B2, int64_t ld2, int p2, bool sym_half, int prec, void *out,
                        int64_t ldo, hipStream_t s);

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
    if (!c.prof) {
        ttmc_launch(c, t, op, B1, ld1, p1, B2, ld2, p2, sym_half, prec, out, ldo, s);
        return;
    }
    hipEvent_t a, b;
    HIPCHECK(hipEventCreate(&a));
    HIPCHECK(hipEventCreate(&b));
    HIPCHECK(hipEventRecord(a, s));
    ttmc_launch(c, t, op, B1, ld1, p1, B2, ld2, p2, sym_half, prec, out, ldo, s);
    HIPCHECK(hipEventRecord(b, s));
    std::string name;
    double bytes, flops;
    ttmc_cost(t, op, p1, p2, sym_half, B2 == nullptr || B2 == B1, prec, name, bytes, flops);
    c.prof_record(name, a, b, bytes, flops);
}

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

static void ttmc_launch(Ctx &c, Tensor &t, int op, const void *B1, int64_t ld1, int p1,
                        const void *B2, int64_t ld2, int p2, bool sym_half, int prec, void *out,
                        int64_t ldo, hipStream_t s) {
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
    const Segmented &o = order == 0 ? t.o3 : (order == 1 ? t.o1 : t.op);
    if (o.nseg == 0) return;
    const void *val = val64 ? o.v64.ptr : o.v32.ptr;

    if (op == BKS_FREE3 && outmode == OUT_SYM && px > kWideThreshold) {
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
        HIPCHECK(hipGetLastError());
        return;
    }

    int PA, ga, PB, gb;
    BlockMap bm;
    std::memset(&bm, 0, sizeof(bm));
    int G;
    if (mode == MODE_M3) {
        PA = 1;
        ga = 1;
        choose_block(py, PB, gb);
        G = gb;
        if (G > 64) fail(BKS_EINVAL, "MODE3 width too large");
        for (int x = 0; x < G; ++x) {
            bm.a[x] = 0;
            bm.b[x] = (int8_t)x;
        }
    } else if (outmode == OUT_SYM) {
        choose_block(px, PA, ga);
        PB = PA;
        gb = ga;
        G = ga * (ga + 1) / 2;
        if (G > 64) fail(BKS_EINVAL, "width too large");
        int x = 0;
        for (int bb = 0; bb < ga; ++bb)
            for (int aa = 0; aa <= bb; ++aa) {
                bm.a[x] = (int8_t)aa;
                bm.b[x] = (int8_t)bb;
                ++x;
            }
    } else {
        choose_block(px, PA, ga);
        choose_block(py, PB, gb);
        G = ga * gb;
        if (G > 64) fail(BKS_EINVAL, "widths too large for the narrow kernel");
        for (int x = 0; x < G; ++x) {
            bm.a[x] = (int8_t)(x % ga);
            bm.b[x] = (int8_t)(x / ga);
        }
    }
    const int E = 64 / G;
    const Schedule &sc = t.schedule(order, E);
    void *partial = nullptr;
    if (sc.nslots > 0) {
        c.ws_partial.ensure((size_t)sc.nslots * q * cts);
        partial = c.ws_partial.ptr;
    }
    Launcher fn;
    if (prec == BKS_F32)
        fn = pick<float, float>(mode, PA, PB);
    else if (val64)
        fn = pick<double, double>(mode, PA, PB);
    else
        fn = pick<float, double>(mode, PA, PB);
    if (!fn) fail(BKS_EINVAL, "no kernel for this width");
    if (sc.nitems > 0)
        fn(dim3((unsigned)sc.nitems), s, sc.items.as<Item>(), o.segptr.as<int64_t>(),
           o.c1.as<int32_t>(), o.c2.as<int32_t>(), val, F1, l1, F2, l2, px, py, G, bm, out, ldo,
           partial, q, outmode);
    HIPCHECK(hipGetLastError());
    if (sc.nfix > 0) {
        if (dbl)
            hipLaunchKernelGGL(ttmc_fixup<double>, dim3((unsigned)sc.nfix), dim3(256), 0, s,
                               sc.fix.as<Fixup>(), static_cast<const double *>(partial), q,
                               static_cast<double *>(out), ldo);
        else
            hipLaunchKernelGGL(ttmc_fixup<float>, dim3((unsigned)sc.nfix), dim3(256), 0, s,
                               sc.fix.as<Fixup>(), static_cast<const float *>(partial), q,
                               static_cast<float *>(out), ldo);
        HIPCHECK(hipGetLastError());
    }
}

}  // namespace bks
