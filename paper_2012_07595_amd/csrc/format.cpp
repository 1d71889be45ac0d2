// Host-side build of the device formats of a (1,2)-symmetric tensor.
//
// A (1,2)-symmetric tensor (Definition in section "Notation") is stored once per
// (i <= j, k) position.  The paper reorganises its sparse tensor before every
// product (section "Block-Krylov methods", discussion of block-Krylov methods; the Discussion of experiments); here
// the reorganisation is paid once at upload, into sorted segmented streams
// that each hold every stored entry once:
//   o3: slice-major (k, i, j) -- A.(X, Y)_{1,2} reduces within a slice
//   op: the stored pair pattern (i <= j) with its k-fibres -- A.(Z)_3, and
//       the first half of A.(Y, Z)_{2,3}
//   pr: an index over the pairs, not the entries: for each row r the pairs
//       (r, c) and (c, r) it belongs to, as (c, pair id) -- the second half
//       of A.(Y, Z)_{2,3} reduces within a row without atomics
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

#include "bks_internal.h"
#include "scale.h"

namespace bks {

namespace {

struct KV {
    uint64_t key;
    uint64_t idx;
};

unsigned nthreads() {
    unsigned h = std::thread::hardware_concurrency();
    if (h == 0) h = 4;
    return std::min(h, 16u);
}

template <class F>
void parallel_for(int64_t n, F f) {
    unsigned T = nthreads();
    if (n < 65536 || T == 1) {
        f(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + T - 1) / T;
    for (unsigned t = 0; t < T; ++t) {
        int64_t b = t * chunk, e = std::min<int64_t>(n, b + chunk);
        if (b >= e) break;
        th.emplace_back(f, b, e, (int)t);
    }
    for (auto &x : th) x.join();
}

// LSD radix sort of (key, idx) by key, 11-bit digits, multithreaded
// histogram/scatter per pass.  Stable.
void radix_sort(std::vector<KV> &a, int key_bits) {
    const int D = 11, B = 1 << D;
    std::vector<KV> tmp(a.size());
    unsigned T = nthreads();
    int64_t n = (int64_t)a.size();
    if (n < 65536) T = 1;
    int64_t chunk = (n + T - 1) / T;
    std::vector<int64_t> hist((size_t)T * B);
    for (int shift = 0; shift < key_bits; shift += D) {
        std::fill(hist.begin(), hist.end(), 0);
        auto count = [&](unsigned t) {
            int64_t b = t * chunk, e = std::min<int64_t>(n, b + chunk);
            int64_t *h = &hist[(size_t)t * B];
            for (int64_t x = b; x < e; ++x) h[(a[x].key >> shift) & (B - 1)]++;
        };
        {
            std::vector<std::thread> th;
            for (unsigned t = 1; t < T; ++t) th.emplace_back(count, t);
            count(0);
            for (auto &x : th) x.join();
        }
        // exclusive prefix over (digit, thread)
        int64_t run = 0;
        for (int d = 0; d < B; ++d)
            for (unsigned t = 0; t < T; ++t) {
                int64_t c = hist[(size_t)t * B + d];
                hist[(size_t)t * B + d] = run;
                run += c;
            }
        auto scatter = [&](unsigned t) {
            int64_t b = t * chunk, e = std::min<int64_t>(n, b + chunk);
            int64_t *h = &hist[(size_t)t * B];
            for (int64_t x = b; x < e; ++x) tmp[h[(a[x].key >> shift) & (B - 1)]++] = a[x];
        };
        {
            std::vector<std::thread> th;
            for (unsigned t = 1; t < T; ++t) th.emplace_back(scatter, t);
            scatter(0);
            for (auto &x : th) x.join();
        }
        a.swap(tmp);
    }
}

int bits_for(uint64_t maxv) {
    int b = 1;
    while (b < 64 && (maxv >> b) != 0) ++b;
    return b;
}

// A blocking copy from pageable memory may return before its DMA has landed,
// and the kernels run on non-blocking streams that do not wait for the null
// stream: wait for the null stream before the data is used.
void h2d_blocking(void *d, const void *h, size_t bytes) {
    HIPCHECK(hipMemcpy(d, h, bytes, hipMemcpyHostToDevice));
    HIPCHECK(hipStreamSynchronize(nullptr));
}

void upload(DevBuf &d, const void *h, size_t bytes) {
    if (bytes == 0) return;
    d.alloc(bytes);
    h2d_blocking(d.ptr, h, bytes);
}

}  // namespace

void build_formats(Tensor &t, const int32_t *I, const int32_t *J, const int32_t *K,
                   const void *val, int val_dtype, unsigned flags) {
    const int64_t m = t.m, n = t.n, nnz = t.nnz;
    // sort keys pack (k, lo, hi, orientation) into 64 bits: 2 n m^2 must fit
    if ((long double)n * (long double)m * (long double)m * 2.0L >= 18446744073709551616.0L)
        fail(BKS_EINVAL, "index space too large: 2 n m^2 must be below 2^64");
    const bool f64 = (val_dtype == BKS_F64);
    const float *v32in = static_cast<const float *>(val);
    const double *v64in = static_cast<const double *>(val);
    auto value = [&](int64_t e) -> double { return f64 ? v64in[e] : (double)v32in[e]; };

    // 1. validate, canonicalise, key = ((k*m + lo)*m + hi) << 1 | orientation
    std::vector<KV> a((size_t)nnz);
    std::atomic<int> bad{0};
    parallel_for(nnz, [&](int64_t b, int64_t e, int) {
        for (int64_t x = b; x < e; ++x) {
            int64_t i = I[x], j = J[x], k = K[x];
            if (i < 0 || j < 0 || k < 0 || i >= m || j >= m || k >= n) {
                bad.store(1);
                continue;
            }
            if (!std::isfinite(value(x))) {
                int z = 0;
                bad.compare_exchange_strong(z, 2);
                continue;
            }
            int64_t lo = std::min(i, j), hi = std::max(i, j);
            uint64_t orient = (flags & BKS_FULL_SYMMETRIC) && (i > j) ? 1u : 0u;
            a[(size_t)x].key = ((((uint64_t)k * m + lo) * m + hi) << 1) | orient;
            a[(size_t)x].idx = (uint64_t)x;
        }
    });
    if (bad.load() == 1) fail(BKS_EINDEX, "coordinate out of range");
    if (bad.load() == 2) fail(BKS_EVALUE, "non-finite value");
    int kb = bits_for((((uint64_t)n * m) * m) << 1);
    radix_sort(a, kb);

    // 2. merge repeated canonical positions
    std::vector<int64_t> si, sj, sk;
    std::vector<double> sv;
    si.reserve(nnz); sj.reserve(nnz); sk.reserve(nnz); sv.reserve(nnz);
    int64_t x = 0;
    while (x < nnz) {
        uint64_t canon = a[x].key >> 1;
        double s0 = 0.0, s1 = 0.0;
        int c0 = 0, c1 = 0;
        int64_t y = x;
        while (y < nnz && (a[y].key >> 1) == canon) {
            if (a[y].key & 1) { s1 += value((int64_t)a[y].idx); c1++; }
            else { s0 += value((int64_t)a[y].idx); c0++; }
            ++y;
        }
        int64_t hi = (int64_t)(canon % (uint64_t)m);
        uint64_t rest = canon / (uint64_t)m;
        int64_t lo = (int64_t)(rest % (uint64_t)m);
        int64_t k = (int64_t)(rest / (uint64_t)m);
        double v;
        if (flags & BKS_FULL_SYMMETRIC) {
            if (lo != hi) {
                if (c0 > 1 || c1 > 1) {
                    if (!(flags & BKS_SUM_DUPLICATES)) fail(BKS_EDUP, "repeated position");
                }
                if (c0 == 0 || c1 == 0 || std::fabs(s0 - s1) > 1e-12 * std::max(std::fabs(s0), std::fabs(s1)))
                    fail(BKS_EASYM, "(i,j,k) and (j,i,k) values differ or one is missing");
            } else if (c0 > 1 && !(flags & BKS_SUM_DUPLICATES)) {
                fail(BKS_EDUP, "repeated position");
            }
            v = s0;
        } else {
            if (c0 > 1 && !(flags & BKS_SUM_DUPLICATES)) fail(BKS_EDUP, "repeated position");
            v = s0;
        }
        si.push_back(lo); sj.push_back(hi); sk.push_back(k); sv.push_back(v);
        x = y;
    }
    a.clear();
    a.shrink_to_fit();
    const int64_t S = (int64_t)sv.size();
    t.nnz = S;
    // optional slice scaling (Examples 3 and 4 of the Experiments section):
    // the merged entries are sorted by (k, lo, hi), so slices are contiguous
    if (flags & (BKS_SCALE_FROBENIUS | BKS_SCALE_LAMBDA_MAX)) {
        if ((flags & BKS_SCALE_FROBENIUS) && (flags & BKS_SCALE_LAMBDA_MAX))
            fail(BKS_EINVAL, "choose one slice scaling");
        std::vector<int64_t> kp(n + 1, 0);
        for (int64_t e = 0; e < S; ++e) kp[sk[e] + 1]++;
        for (int64_t q = 0; q < n; ++q) kp[q + 1] += kp[q];
        const bool frob = flags & BKS_SCALE_FROBENIUS;
        std::atomic<int64_t> next{0};
        auto work = [&]() {
            for (int64_t k; (k = next.fetch_add(1)) < n;) {
                const int64_t b = kp[k], c = kp[k + 1] - kp[k];
                if (c == 0) continue;
                const double f = frob ? sym_frobenius(c, &si[b], &sj[b], &sv[b])
                                      : sym_spectral_radius(c, &si[b], &sj[b], &sv[b]);
                // a zero slice stays zero
                if (f > 0.0)
                    for (int64_t e = b; e < b + c; ++e) sv[e] /= f;
            }
        };
        std::vector<std::thread> th;
        for (unsigned x = 1; x < nthreads(); ++x) th.emplace_back(work);
        work();
        for (auto &x : th) x.join();
    }
    double f2 = 0.0;
    for (int64_t e = 0; e < S; ++e) f2 += (si[e] == sj[e] ? 1.0 : 2.0) * sv[e] * sv[e];
    t.frob2 = f2;
    t.has64 = f64;

    // 3. o3: already sorted by (k, i, j)
    {
        std::vector<int64_t> ptr(n + 1, 0);
        for (int64_t e = 0; e < S; ++e) ptr[sk[e] + 1]++;
        for (int64_t q = 0; q < n; ++q) ptr[q + 1] += ptr[q];
        std::vector<int32_t> c12(2 * S);
        std::vector<float> v32(S);
        for (int64_t e = 0; e < S; ++e) {
            c12[2 * e] = (int32_t)si[e];
            c12[2 * e + 1] = (int32_t)sj[e];
            v32[e] = (float)sv[e];
        }
        Segmented &o = t.o3;
        o.nseg = n;
        o.nent = S;
        upload(o.segptr, ptr.data(), ptr.size() * 8);
        upload(o.c1, c12.data(), S * 8);
        upload(o.v32, v32.data(), S * 4);
        if (f64) upload(o.v64, sv.data(), S * 8);
        o.h_segptr = std::move(ptr);
    }

    // 4. op: stored entries sorted by (i, j, k), segmented by pair; pr: for
    // every row r the pairs it belongs to, (col, pair id) sorted by col --
    // pairs (c, r) with c < r first, then (r, c) with c >= r
    {
        std::vector<KV> b((size_t)S);
        for (int64_t e = 0; e < S; ++e) {
            b[e].key = ((uint64_t)si[e] * m + sj[e]) * n + sk[e];
            b[e].idx = (uint64_t)e;
        }
        radix_sort(b, bits_for(((uint64_t)m * m) * n));
        std::vector<int64_t> pptr;
        pptr.reserve(S / 2 + 2);
        std::vector<int32_t> pk(S);
        std::vector<float> pv32(S);
        std::vector<double> pv64(f64 ? S : 0);
        t.pair_i.clear();
        t.pair_j.clear();
        uint64_t last = ~(uint64_t)0;
        for (int64_t q = 0; q < S; ++q) {
            const uint64_t key = b[q].key;
            const uint64_t pid = key / (uint64_t)n;
            if (pid != last) {
                pptr.push_back(q);
                t.pair_i.push_back((int32_t)(pid / (uint64_t)m));
                t.pair_j.push_back((int32_t)(pid % (uint64_t)m));
                last = pid;
            }
            pk[q] = (int32_t)(key % (uint64_t)n);
            const double v = sv[b[q].idx];
            pv32[q] = (float)v;
            if (f64) pv64[q] = v;
        }
        pptr.push_back(S);
        b.clear();
        b.shrink_to_fit();
        const int64_t P = (int64_t)t.pair_i.size();
        Segmented &p = t.op;
        p.nseg = P;
        p.nent = S;
        t.npairs = P;
        upload(p.segptr, pptr.data(), pptr.size() * 8);
        upload(p.c2, pk.data(), pk.size() * 4);
        upload(p.v32, pv32.data(), pv32.size() * 4);
        if (f64) upload(p.v64, pv64.data(), pv64.size() * 8);
        p.h_segptr = std::move(pptr);

        std::vector<int64_t> mc(m, 0), dc(m, 0);
        for (int64_t q = 0; q < P; ++q) {
            dc[t.pair_i[q]]++;
            if (t.pair_i[q] != t.pair_j[q]) mc[t.pair_j[q]]++;
        }
        std::vector<int64_t> rptr(m + 1, 0);
        for (int64_t r = 0; r < m; ++r) rptr[r + 1] = rptr[r] + mc[r] + dc[r];
        const int64_t R = rptr[m];
        std::vector<int64_t> cm(m), cd(m);
        for (int64_t r = 0; r < m; ++r) {
            cm[r] = rptr[r];
            cd[r] = rptr[r] + mc[r];
        }
        std::vector<int32_t> cp(2 * R);
        for (int64_t q = 0; q < P; ++q) {
            const int32_t i = t.pair_i[q], j = t.pair_j[q];
            int64_t w = cd[i]++;
            cp[2 * w] = j;
            cp[2 * w + 1] = (int32_t)q;
            if (i != j) {
                w = cm[j]++;
                cp[2 * w] = i;
                cp[2 * w + 1] = (int32_t)q;
            }
        }
        Segmented &o = t.pr;
        o.nseg = m;
        o.nent = R;
        upload(o.segptr, rptr.data(), rptr.size() * 8);
        upload(o.c1, cp.data(), R * 8);
        o.h_segptr = std::move(rptr);
    }
    auto bytes = [](const Segmented &o) {
        return o.segptr.bytes + o.c1.bytes + o.c2.bytes + o.v32.bytes + o.v64.bytes;
    };
    t.dev_bytes = bytes(t.o3) + bytes(t.pr) + bytes(t.op);
}

void build_formats_general(Tensor &t, const int32_t *I, const int32_t *J, const int32_t *K,
                           const void *val, int val_dtype, unsigned flags) {
    const int64_t l = t.l, m = t.m, n = t.n, nnz = t.nnz;
    if ((long double)l * (long double)m * (long double)n >= 18446744073709551616.0L)
        fail(BKS_EINVAL, "index space too large: l m n must be below 2^64");
    const bool f64 = (val_dtype == BKS_F64);
    const float *v32in = static_cast<const float *>(val);
    const double *v64in = static_cast<const double *>(val);
    auto value = [&](int64_t e) -> double { return f64 ? v64in[e] : (double)v32in[e]; };
    // validate, then sort by (i, j, k) and merge repeats
    std::vector<KV> a((size_t)nnz);
    for (int64_t x = 0; x < nnz; ++x) {
        const int64_t i = I[x], j = J[x], k = K[x];
        if (i < 0 || j < 0 || k < 0 || i >= l || j >= m || k >= n)
            fail(BKS_EINDEX, "coordinate out of range");
        if (!std::isfinite(value(x))) fail(BKS_EVALUE, "non-finite value");
        a[x].key = ((uint64_t)i * m + j) * n + k;
        a[x].idx = (uint64_t)x;
    }
    radix_sort(a, bits_for(((uint64_t)l * m) * n));
    std::vector<int64_t> gi, gj, gk;
    std::vector<double> gv;
    for (int64_t x = 0; x < nnz;) {
        int64_t y = x;
        double sum = 0.0;
        while (y < nnz && a[y].key == a[x].key) sum += value((int64_t)a[y++].idx);
        if (y - x > 1 && !(flags & BKS_SUM_DUPLICATES)) fail(BKS_EDUP, "repeated position");
        const uint64_t key = a[x].key;
        gk.push_back((int64_t)(key % (uint64_t)n));
        gj.push_back((int64_t)((key / (uint64_t)n) % (uint64_t)m));
        gi.push_back((int64_t)(key / ((uint64_t)n * m)));
        gv.push_back(sum);
        x = y;
    }
    a.clear();
    a.shrink_to_fit();
    const int64_t S = (int64_t)gv.size();
    t.nnz = S;
    t.has64 = f64;
    double f2 = 0.0;
    for (double v : gv) f2 += v * v;
    t.frob2 = f2;
    // mode a: segments by index a, entries (the other two, in mode order)
    const std::vector<int64_t> *idx[3] = {&gi, &gj, &gk};
    const int64_t dims[3] = {l, m, n};
    for (int md = 0; md < 3; ++md) {
        const std::vector<int64_t> &sg = *idx[md];
        const std::vector<int64_t> &c1 = *idx[md == 0 ? 1 : 0];
        const std::vector<int64_t> &c2 = *idx[md == 2 ? 1 : 2];
        std::vector<int64_t> ptr(dims[md] + 1, 0);
        for (int64_t e = 0; e < S; ++e) ptr[sg[e] + 1]++;
        for (int64_t q = 0; q < dims[md]; ++q) ptr[q + 1] += ptr[q];
        // stable counting sort by the segment index keeps (c1, c2) ascending
        // within a segment for mode 0; modes 1 and 2 follow the (i, j, k)
        // order of the merged entries
        std::vector<int64_t> at(ptr.begin(), ptr.end() - 1);
        std::vector<int32_t> cc(2 * S);
        std::vector<float> v32(S);
        std::vector<double> v64(f64 ? S : 0);
        for (int64_t e = 0; e < S; ++e) {
            const int64_t w = at[sg[e]]++;
            cc[2 * w] = (int32_t)c1[e];
            cc[2 * w + 1] = (int32_t)c2[e];
            v32[w] = (float)gv[e];
            if (f64) v64[w] = gv[e];
        }
        Segmented &o = t.g[md];
        o.nseg = dims[md];
        o.nent = S;
        upload(o.segptr, ptr.data(), ptr.size() * 8);
        upload(o.c1, cc.data(), (size_t)S * 8);
        upload(o.v32, v32.data(), (size_t)S * 4);
        if (f64) upload(o.v64, v64.data(), (size_t)S * 8);
        o.h_segptr = std::move(ptr);
    }
    auto bytes = [](const Segmented &o) {
        return o.segptr.bytes + o.c1.bytes + o.c2.bytes + o.v32.bytes + o.v64.bytes;
    };
    t.general = true;
    t.dev_bytes = bytes(t.g[0]) + bytes(t.g[1]) + bytes(t.g[2]);
}

void Tensor::release_device() {
    std::lock_guard<std::mutex> lk(sched_mu);
    for (Segmented *o : {&o3, &pr, &op, &g[0], &g[1], &g[2]}) {
        o->segptr.release();
        o->c1.release();
        o->c2.release();
        o->v32.release();
        o->v64.release();
        o->nseg = 0;
        o->nent = 0;
    }
    sched.clear();
    hsched.clear();
    dev_bytes = 0;
}

const HostSchedule &Tensor::host_schedule(int order, int E) {
    // caller holds sched_mu
    auto key = std::make_pair(order, E);
    auto it = hsched.find(key);
    if (it != hsched.end()) return *it->second;
    auto h = std::make_unique<HostSchedule>();
    if (order == kWideOrder) {
        build_wide_schedule(o3.h_segptr, E, h->items, h->fix, h->nslots);
    } else {
        const int fmt = order >= kGroupOrder ? order - kGroupOrder : order;
        const Segmented &o = seg_of(fmt);
        if (order >= kGroupOrder)
            build_group_schedule(o.h_segptr, h->items, h->fix, h->nslots);
        else
            build_schedule(o.h_segptr, E, h->items, h->fix, h->nslots);
        // tree levels for segments with many partial slots (see Schedule); the
        // wide schedule's chunks are summed by their own reduce kernel
        build_fix_tree(h->fix, h->nslots, h->levels);
    }
    auto &ref = *h;
    hsched[key] = std::move(h);
    return ref;
}

const Schedule &Tensor::schedule(int order, int E) {
    std::lock_guard<std::mutex> lk(sched_mu);
    auto key = std::make_pair(order, E);
    auto it = sched.find(key);
    if (it != sched.end()) return *it->second;
    const HostSchedule &h = host_schedule(order, E);
    auto sc = std::make_unique<Schedule>();
    sc->nslots = h.nslots;
    for (auto &l : h.levels) {
        auto L = std::make_unique<Schedule::Level>();
        L->nfix = (int64_t)l.size();
        L->fix.alloc(l.size() * sizeof(Fixup));
        h2d_blocking(L->fix.ptr, l.data(), l.size() * sizeof(Fixup));
        sc->levels.push_back(std::move(L));
    }
    sc->nitems = (int64_t)h.items.size();
    sc->nfix = (int64_t)h.fix.size();
    if (!h.items.empty()) {
        sc->items.alloc(h.items.size() * sizeof(Item));
        h2d_blocking(sc->items.ptr, h.items.data(), h.items.size() * sizeof(Item));
    }
    if (!h.fix.empty()) {
        sc->fix.alloc(h.fix.size() * sizeof(Fixup));
        h2d_blocking(sc->fix.ptr, h.fix.data(), h.fix.size() * sizeof(Fixup));
    }
    auto &ref = *sc;
    sched[key] = std::move(sc);
    return ref;
}

}  // namespace bks
