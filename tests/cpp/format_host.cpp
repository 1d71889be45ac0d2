// Host check of the tensor upload (bks_tensor_upload's formats) without a GPU.
//
// The upload canonicalises each coordinate (i, j, k) of a (1,2)-symmetric
// tensor to (min(i,j), max(i,j), k), merges repeated positions, validates,
// and lays the stored entries out three ways: slice-major (segments k,
// entries (i, j) with i <= j), row-major over both orientations (segments
// row, entries (col, k)) and over the stored pair pattern (segments (i, j),
// entries k).  The few HIP runtime calls it makes are provided below over
// host memory, so the "device" arrays can be read back directly and every
// access is visible to AddressSanitizer.  The expected layout is built here
// from an ordered map of the canonical positions, independently of the
// library's radix sorts.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <set>
#include <tuple>
#include <vector>

#include "bks_internal.h"

// ---------------------------------------------------------------- host stand-ins
namespace bks {
void fail(int code, const std::string &msg) { throw Error{code, msg}; }
void check_hip(hipError_t e, const char *what) {
    if (e != hipSuccess) fail(BKS_EDEVICE, what);
}
DevBuf::~DevBuf() { release(); }
void DevBuf::alloc(size_t b) {
    release();
    if (b == 0) return;
    ptr = std::malloc(b);
    if (!ptr) fail(BKS_ENOMEM, "malloc");
    bytes = b;
}
void DevBuf::release() {
    std::free(ptr);
    ptr = nullptr;
    bytes = 0;
}
}  // namespace bks

extern "C" hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind) {
    std::memcpy(dst, src, n);
    return hipSuccess;
}
extern "C" hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }

// ---------------------------------------------------------------- checks
static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);          \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

struct Coo {
    int64_t m, n;
    std::vector<int32_t> i, j, k;
    std::vector<double> v;
};

// canonical position (k, lo, hi) -> summed value
using Canon = std::map<std::tuple<int64_t, int64_t, int64_t>, double>;

static Canon canon_of(const Coo &c) {
    Canon M;
    for (size_t e = 0; e < c.v.size(); ++e) {
        int64_t lo = std::min(c.i[e], c.j[e]), hi = std::max(c.i[e], c.j[e]);
        M[{c.k[e], lo, hi}] += c.v[e];
    }
    return M;
}

static int upload(bks::Tensor &t, const Coo &c, bool f64, unsigned flags) {
    t.m = c.m;
    t.n = c.n;
    t.nnz = (int64_t)c.v.size();
    std::vector<float> v32(c.v.begin(), c.v.end());
    try {
        bks::build_formats(t, c.i.data(), c.j.data(), c.k.data(),
                           f64 ? (const void *)c.v.data() : (const void *)v32.data(),
                           f64 ? BKS_F64 : BKS_F32, flags);
    } catch (const bks::Error &e) {
        return e.code;
    }
    return 0;
}

template <class T> static const T *dev(const bks::DevBuf &b) { return b.as<T>(); }

// Compare the three layouts of t with the canonical map M (values as the
// upload's value type gives them).
static void check_layouts(const bks::Tensor &t, const Canon &M, int64_t m, int64_t n, bool f64) {
    const int64_t S = (int64_t)M.size();
    CHECK(t.nnz == S);
    double f2 = 0.0;
    for (auto &kv : M) f2 += (std::get<1>(kv.first) == std::get<2>(kv.first) ? 1.0 : 2.0) *
                             kv.second * kv.second;
    CHECK(std::fabs(t.frob2 - f2) <= 1e-12 * std::max(1.0, f2));

    // slice-major: segments k in order, entries (lo, hi) ascending
    CHECK(t.o3.nseg == n && t.o3.nent == S);
    {
        const int64_t *ptr = dev<int64_t>(t.o3.segptr);
        CHECK(S == 0 || ptr[0] == 0);
        int64_t e = 0;
        for (auto &kv : M) {
            auto [k, lo, hi] = kv.first;
            CHECK(ptr[k] <= e && e < ptr[k + 1]);
            CHECK(dev<int32_t>(t.o3.c1)[2 * e] == lo && dev<int32_t>(t.o3.c1)[2 * e + 1] == hi);
            CHECK(dev<float>(t.o3.v32)[e] == (float)kv.second);
            if (f64) CHECK(dev<double>(t.o3.v64)[e] == kv.second);
            ++e;
        }
        if (S) CHECK(ptr[n] == S);
        CHECK(t.o3.h_segptr.size() == (size_t)n + 1);
    }

    // stored pair pattern: pairs (lo, hi) ascending, each with its k ascending
    std::map<std::pair<int64_t, int64_t>, std::vector<std::pair<int64_t, double>>> P;
    for (auto &kv : M) {
        auto [k, lo, hi] = kv.first;
        P[{lo, hi}].push_back({k, kv.second});
    }
    CHECK(t.npairs == (int64_t)P.size() && t.op.nseg == (int64_t)P.size());
    CHECK(t.op.nent == S);
    {
        const int64_t *ptr = dev<int64_t>(t.op.segptr);
        int64_t q = 0, e = 0;
        for (auto &pv : P) {
            CHECK(t.pair_i[q] == pv.first.first && t.pair_j[q] == pv.first.second);
            CHECK(ptr[q] == e && ptr[q + 1] == e + (int64_t)pv.second.size());
            auto ks = pv.second;
            std::sort(ks.begin(), ks.end());
            for (auto &kv : ks) {
                CHECK(dev<int32_t>(t.op.c2)[e] == kv.first);
                CHECK(dev<float>(t.op.v32)[e] == (float)kv.second);
                if (f64) CHECK(dev<double>(t.op.v64)[e] == kv.second);
                ++e;
            }
            ++q;
        }
    }

    // pair rows: row r lists every stored pair touching it as (col, pair id),
    // sorted by col (pairs (c, r) with c < r, then (r, c) with c >= r); an
    // index over the pairs, no values
    std::map<std::pair<int64_t, int64_t>, int64_t> pid;  // (row, col) -> pair id
    {
        int64_t q = 0;
        for (auto &pv : P) {
            pid[{pv.first.first, pv.first.second}] = q;
            if (pv.first.first != pv.first.second) pid[{pv.first.second, pv.first.first}] = q;
            ++q;
        }
    }
    CHECK(t.pr.nseg == m && t.pr.nent == (int64_t)pid.size());
    CHECK(t.pr.v32.ptr == nullptr && t.pr.v64.ptr == nullptr);
    {
        const int64_t *ptr = dev<int64_t>(t.pr.segptr);
        CHECK(ptr[0] == 0);
        int64_t e = 0;
        for (auto &kv : pid) {
            const int64_t row = kv.first.first, col = kv.first.second;
            CHECK(ptr[row] <= e && e < ptr[row + 1]);
            CHECK(dev<int32_t>(t.pr.c1)[2 * e] == col && dev<int32_t>(t.pr.c1)[2 * e + 1] == kv.second);
            ++e;
        }
        CHECK(ptr[m] == (int64_t)pid.size());
        CHECK(t.pr.h_segptr.size() == (size_t)m + 1);
    }
}

static Coo random_coo(int64_t m, int64_t n, int64_t nnz, unsigned seed, bool ints) {
    std::mt19937_64 g(seed);
    Coo c{m, n, {}, {}, {}, {}};
    std::uniform_int_distribution<int64_t> di(0, m - 1), dk(0, n - 1), dv(-4, 4);
    std::normal_distribution<double> nv;
    for (int64_t e = 0; e < nnz; ++e) {
        c.i.push_back((int32_t)di(g));
        c.j.push_back((int32_t)di(g));
        c.k.push_back((int32_t)dk(g));
        // small integers keep the merged sums exact in any order
        c.v.push_back(ints ? (double)dv(g) : nv(g));
    }
    return c;
}

int main() {
    // random tensors with repeated positions, both value types; small index
    // spaces force many repeats, the large one runs the threaded sort
    const int64_t shapes[][3] = {{1, 1, 5}, {7, 3, 200}, {50, 9, 3000}, {300, 40, 20000},
                                 {5000, 700, 300000}};
    for (auto &sh : shapes)
        for (int f64 = 0; f64 < 2; ++f64) {
            Coo c = random_coo(sh[0], sh[1], sh[2], 11 + (unsigned)sh[2] + f64, true);
            bks::Tensor t;
            int rc = upload(t, c, f64, BKS_SUM_DUPLICATES);
            CHECK(rc == 0);
            if (rc == 0) check_layouts(t, canon_of(c), c.m, c.n, f64);
            // without the flag a repeated position is an error (every shape
            // above repeats one, by the pigeonhole principle or by chance)
            bks::Tensor t2;
            if (canon_of(c).size() < c.v.size()) CHECK(upload(t2, c, f64, 0) == BKS_EDUP);
        }
    std::printf("ok formats_random\n");

    // distinct positions need no flag; the values are kept exactly
    {
        Coo c{20, 4, {}, {}, {}, {}};
        for (int k = 0; k < 4; ++k)
            for (int i = 0; i < 20; ++i)
                for (int j = i; j < 20; j += 3) {
                    c.i.push_back((k + i) % 2 ? i : j);  // both orientations of input
                    c.j.push_back((k + i) % 2 ? j : i);
                    c.k.push_back(k);
                    c.v.push_back(0.1 * (1 + i + 20 * j + 400 * k));
                }
        bks::Tensor t;
        CHECK(upload(t, c, true, 0) == 0);
        check_layouts(t, canon_of(c), c.m, c.n, true);
    }
    std::printf("ok formats_distinct\n");

    // full-symmetric input: both orientations given, one copy kept
    {
        Coo c{6, 2, {0, 1, 2, 2, 3, 5}, {1, 0, 2, 4, 3, 4}, {0, 0, 1, 1, 1, 1},
              {1.5, 1.5, 2.0, 3.0, 4.0, 3.0}};
        bks::Tensor t;
        // (2,4,1) and (5,4,1) have no mirror
        CHECK(upload(t, c, true, BKS_FULL_SYMMETRIC) == BKS_EASYM);
        c.i = {0, 1, 2, 2, 4, 3, 5, 4};
        c.j = {1, 0, 2, 4, 2, 3, 4, 5};
        c.k = {0, 0, 1, 1, 1, 1, 1, 1};
        c.v = {1.5, 1.5, 2.0, 3.0, 3.0, 4.0, -1.0, -1.0};
        bks::Tensor t2;
        CHECK(upload(t2, c, true, BKS_FULL_SYMMETRIC) == 0);
        Canon M = {{{0, 0, 1}, 1.5}, {{1, 2, 2}, 2.0}, {{1, 2, 4}, 3.0}, {{1, 3, 3}, 4.0},
                   {{1, 4, 5}, -1.0}};
        check_layouts(t2, M, 6, 2, true);
        c.v[4] = 3.5;  // mirror disagrees
        bks::Tensor t3;
        CHECK(upload(t3, c, true, BKS_FULL_SYMMETRIC) == BKS_EASYM);
    }
    std::printf("ok formats_full_symmetric\n");

    // validation: out-of-range indices, non-finite values, empty input,
    // index spaces beyond the 64-bit sort keys
    {
        Coo c{4, 2, {0, 4}, {1, 1}, {0, 0}, {1.0, 1.0}};
        bks::Tensor t;
        CHECK(upload(t, c, true, 0) == BKS_EINDEX);
        c.i = {0, 1};
        c.k = {0, 2};
        bks::Tensor t2;
        CHECK(upload(t2, c, true, 0) == BKS_EINDEX);
        c.k = {0, 1};
        c.i[1] = -1;
        bks::Tensor t3;
        CHECK(upload(t3, c, true, 0) == BKS_EINDEX);
        c.i[1] = 2;
        c.v[0] = NAN;
        bks::Tensor t4;
        CHECK(upload(t4, c, true, 0) == BKS_EVALUE);
        c.v[0] = INFINITY;
        bks::Tensor t5;
        CHECK(upload(t5, c, false, 0) == BKS_EVALUE);
        Coo e{9, 3, {}, {}, {}, {}};
        bks::Tensor t6;
        CHECK(upload(t6, e, false, 0) == 0);
        check_layouts(t6, Canon{}, 9, 3, false);
        // m = n = 2^21 gives 2 n m^2 = 2^64 exactly: refused; n one smaller
        // fits, with entries at the far corners of the index space
        const int64_t M21 = (int64_t)1 << 21;
        Coo big{M21, M21, {0}, {1}, {0}, {1.0}};
        bks::Tensor t7;
        CHECK(upload(t7, big, true, 0) == BKS_EINVAL);
        Coo fits{M21, M21 - 1, {0, (int32_t)M21 - 1, 5}, {(int32_t)M21 - 1, (int32_t)M21 - 1, 3},
                 {(int32_t)M21 - 2, (int32_t)M21 - 2, 0}, {1.0, 2.0, 3.0}};
        bks::Tensor t8;
        CHECK(upload(t8, fits, true, 0) == 0);
        check_layouts(t8, canon_of(fits), fits.m, fits.n, true);
    }
    std::printf("ok formats_validation\n");

    // slice scaling at upload: every nonempty slice of the Frobenius-scaled
    // tensor has norm 1 (||A||^2 = nonempty slices); the lambda_max scaling
    // of a slice that is 2.5 times the complete graph K_6 divides by 12.5;
    // both flags at once are refused
    {
        Coo c = random_coo(60, 7, 900, 5, false);
        bks::Tensor t;
        CHECK(upload(t, c, true, BKS_SUM_DUPLICATES | BKS_SCALE_FROBENIUS) == 0);
        const int64_t *ptr = dev<int64_t>(t.o3.segptr);
        const int32_t *c12 = dev<int32_t>(t.o3.c1);
        const double *v = dev<double>(t.o3.v64);
        int nonempty = 0;
        for (int64_t k = 0; k < c.n; ++k) {
            double s = 0.0;
            for (int64_t e = ptr[k]; e < ptr[k + 1]; ++e)
                s += (c12[2 * e] == c12[2 * e + 1] ? 1.0 : 2.0) * v[e] * v[e];
            if (ptr[k + 1] > ptr[k]) {
                ++nonempty;
                CHECK(std::fabs(s - 1.0) <= 1e-13);
            }
        }
        CHECK(std::fabs(t.frob2 - nonempty) <= 1e-12 * nonempty);
        Coo g{10, 2, {}, {}, {}, {}};
        for (int a = 0; a < 6; ++a)
            for (int b = a + 1; b < 6; ++b) {
                g.i.push_back(a + 2);
                g.j.push_back(b + 2);
                g.k.push_back(1);
                g.v.push_back(2.5);
            }
        bks::Tensor t2;
        CHECK(upload(t2, g, true, BKS_SCALE_LAMBDA_MAX) == 0);
        const double *v2 = dev<double>(t2.o3.v64);
        for (int64_t e = 0; e < t2.o3.nent; ++e) CHECK(std::fabs(v2[e] - 0.2) <= 1e-15);
        bks::Tensor t3;
        CHECK(upload(t3, g, true, BKS_SCALE_LAMBDA_MAX | BKS_SCALE_FROBENIUS) == BKS_EINVAL);
    }
    std::printf("ok formats_scaling\n");

    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    return 0;
}
