// Internal declarations of libbks (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bks.h"
#include "inner.h"
#include "schedule.h"

namespace bks {

// ---------------------------------------------------------------- errors
struct Error {
    int code;
    std::string msg;
};
[[noreturn]] void fail(int code, const std::string &msg);
void check_hip(hipError_t e, const char *what);
#define HIPCHECK(x) ::bks::check_hip((x), #x)

// ---------------------------------------------------------------- device memory
// Device bytes held by the library's buffers, counted per accounting scope:
// a thread that sets DevAccount::current (a served session) has every buffer
// it allocates counted there until the buffer is released.
struct DevAccount {
    std::atomic<size_t> live{0}, peak{0};
    void add(size_t b);
    void sub(size_t b) { live.fetch_sub(b); }
    static thread_local std::shared_ptr<DevAccount> current;
};

// A device buffer owned by the library.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    std::shared_ptr<DevAccount> acct;  // scope that counted this allocation
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf();
    void alloc(size_t b);
    void ensure(size_t b);  // grow-only
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Page-locked, coherent host staging memory owned by the library (freed
// with its owner; the owner synchronises its stream first).
struct PinnedBuf {
    char *ptr = nullptr;
    size_t bytes = 0;
    PinnedBuf() = default;
    PinnedBuf(const PinnedBuf &) = delete;
    PinnedBuf &operator=(const PinnedBuf &) = delete;
    ~PinnedBuf();
    void ensure(size_t b);  // grow-only; contents are not kept
};

// ---------------------------------------------------------------- formats
// A segmented entry stream: segments (slices, rows or pairs) own contiguous
// runs of entries; entry e carries two indices c1[e], c2[e] and a value.
struct Segmented {
    int64_t nseg = 0;
    int64_t nent = 0;
    DevBuf segptr;   // int64 [nseg + 1]
    DevBuf c1;       // int32 pairs (c1, c2) interleaved [2 nent] (slice- and row-major)
    DevBuf c2;       // int32 [nent] (pair pattern: k only)
    DevBuf v32;      // float [nent]
    DevBuf v64;      // double [nent] (only for FP64-valued tensors)
    std::vector<int64_t> h_segptr;  // host copy for schedule building
};

// Host copy of a schedule (built once per tensor, order and E; kept so
// that a schedule can be placed in caller-provided device memory).
struct HostSchedule {
    int64_t nslots = 0;
    std::vector<Item> items;
    std::vector<Fixup> fix;
    std::vector<std::vector<Fixup>> levels;  // tree levels, run in order before fix
};

// Device pointers of a schedule as one product call uses it.
struct SchedView {
    int64_t nitems = 0, nfix = 0, nslots = 0;
    const Item *items = nullptr;
    const Fixup *fix = nullptr;
    std::vector<std::pair<int64_t, const Fixup *>> levels;
};

struct Schedule {
    int64_t nitems = 0;
    int64_t nfix = 0;
    int64_t nslots = 0;  // partial slots incl. the tree levels' slots
    DevBuf items;  // Item[nitems]
    DevBuf fix;    // Fixup[nfix]: final sums into the output rows
    // Segments with more than kFixFan partial slots are first reduced in a
    // fixed tree: each level's Fixup sums up to kFixFan slots into the slot
    // named by its `seg` field; levels run in order before `fix`.
    struct Level {
        int64_t nfix = 0;
        DevBuf fix;
    };
    std::vector<std::unique_ptr<Level>> levels;
};

struct Tensor;

// Device Cholesky solver for large inner Newton systems (devsolve.cpp).
struct DevSolver {
    void *handle = nullptr;  // rocblas_handle
    void *get_handle(hipStream_t s);  // created on first use, bound to s
    DevBuf dH, dA, db;
    PinnedBuf pin;           // staging of the right-hand side and the result
    DevSolver() = default;
    DevSolver(const DevSolver &) = delete;
    DevSolver &operator=(const DevSolver &) = delete;
    ~DevSolver();
    // Solve (H + mu I) x = b (H N x N symmetric, row-major host) in place of
    // b; false if it is not positive definite (b is then unchanged).  H is
    // uploaded only when new_matrix (it stays on the device between calls).
    bool solve(hipStream_t s, int N, const double *H, double mu, bool new_matrix, double *b);
    // The same with H already in dH (formed on the device).
    bool solve_resident(hipStream_t s, int N, double mu, double *b);
};
// dst = src + mu I for N x N matrices on the device (cholesky.hip).
void shift_copy_dev(hipStream_t s, double *dst, const double *src, int N, double mu);
// x <- (L L^T)^{-1} x on the device for a lower Cholesky factor L (N x N,
// column-major, leading dimension N), one right-hand side (trisolve.hip):
// chol_solve_small in one workgroup (x staged in LDS; it returns at once
// when the device int *info is non-zero; orders up to kSolveWgLimit fit;
// used up to kSolveWgMax), the multi-launch chol_solve_dev beyond
// kPotrsMax; in between rocBLAS's trsv (rocSOLVER's potrs after potrf) is
// the faster.
constexpr int kSolveWgLimit = 8192;
constexpr int kSolveWgMax = 1024;
constexpr int kPotrsMax = 8192;
// forward = false: only the backward solve L^T x = x (after a factorisation
// that substituted forward already)
void chol_solve_small(hipStream_t s, const double *L, int N, double *x, const int *info,
                      bool forward = true);
void chol_solve_dev(hipStream_t s, const double *L, int N, double *x, bool forward = true);
// A = L L^T in place on the device (lower triangle, column-major, leading
// dimension N); *info (device) gets 0, or the 1-based index of the first
// non-positive pivot (cholesky.hip).  With b (device, N) the forward
// substitution runs along and b becomes L^{-1} b.  work (device,
// kCholWork doubles, required) holds a diagonal block between two steps.
// Given a rocBLAS handle bound to s, large orders take panels of 256
// columns with a dsyrk update of the rest after each.  Used up to order
// kSmallCholMax, rocSOLVER's potrf beyond.
constexpr int kSmallCholMax = 32768;
constexpr int kCholWork = 32 * 32 + 32;
void chol_factor_dev(hipStream_t s, double *A, int N, int *info, double *b, double *work,
                     void *blas = nullptr);

// Device products of the inner solve for large cores (devsolve.cpp):
// rocBLAS FP64 on the ctx stream, sharing the DevSolver's handle.
struct DevInner : InnerDevice {
    DevSolver *ds = nullptr;
    hipStream_t s = nullptr;
    int k1 = 0, k3 = 0;
    DevBuf dC, dA, dOut, dT, dY, dOnes, dNw;
    int rot_r = -1, rot_r3 = -1;    // rank of the rotation held in dY
    int newton_n = 0;               // order of the Newton matrix held in ds->dH
    PinnedBuf pin;                  // staging of the small transfers
    double *stage(size_t count);    // pinned host space for `count` doubles
    // out_host(0:len) = sum of the nparts device vectors parts(:, q) (ld len)
    void sum_parts(const double *parts, int len, int nparts, double *out_host);
    void set_core(const double *C, int k1, int k3) override;
    void gram1(double *G1) override;
    void gram3(double *G3) override;
    void mode3p(const double *Sv, int ldS, int l0, int nl, const double *P, int r,
                double *out) override;
    void hooi3(const double *P, int r, double *M3) override;
    void rotate(const double *Qp, const double *Qs, int r, int r3, double *Y, double *Y2,
                bool partial) override;
    bool forms_newton() const override { return true; }
    bool newton_matrix(int r, int r3, double *diag) override;  // newton.hip
    bool newton_solve(double mu, double *b) override;
};

// Event-timed launches of one kernel class (profiling).
struct ProfClass {
    int64_t calls = 0;
    double ms = 0.0, bytes = 0.0, flops = 0.0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

struct Ctx {
    int device = 0;
    size_t budget = 0;
    size_t used = 0;
    std::string last_error;
    hipStream_t stream = nullptr;   // ctx-owned stream for solver work
    DevBuf ws_partial;              // TTMc partial rows
    DevBuf ws_pack1, ws_pack2;      // dense-kernel partials
    DevBuf ws_fac1, ws_fac2;        // block-packed factor copies for TTMc
    DevBuf ws_tmp;                  // intermediate products of two-step TTMc
    PinnedBuf pin;                  // staging of the solver's small copies
    std::mutex mu;
    std::mutex tensors_mu;
    std::vector<Tensor *> tensors;  // live tensors uploaded through this ctx
    // optional bracket around host-side dense solves (serving: bounded pool)
    std::function<void()> host_acquire, host_release;
    // set by a server while a request runs: the solve stops at its next outer
    // iteration once this reads true
    const std::atomic<bool> *cancel = nullptr;
    DevSolver devsolve;
    DevInner devinner;
    bool prof = false;
    std::mutex prof_mu;
    std::map<std::string, ProfClass> prof_stats;
    // Record a launch of class `name` bracketed by (a, b) on its stream.
    void prof_record(const std::string &name, hipEvent_t a, hipEvent_t b, double bytes,
                     double flops);
    void prof_flush();
    // free the grow-only device workspaces (a served slot between requests)
    void release_workspaces();
};

struct Tensor {
    Ctx *ctx = nullptr;
    int64_t m = 0, n = 0, nnz = 0, npairs = 0;
    bool has64 = false;
    double frob2 = 0.0;
    size_t dev_bytes = 0;
    Segmented o3;    // slices k: entries (i, j) with i <= j          (FREE3)
    Segmented op;    // pairs (i <= j): entries (-, k)                (MODE3, FREE1)
    Segmented pr;    // rows r: (col, pair id) of the pairs touching r (FREE1, no values)
    // a general (non-symmetric) l x m x n tensor instead: segments by the
    // index of mode a + 1, entries (the other two indices in mode order, value)
    bool general = false;
    int64_t l = 0;
    Segmented g[3];
    // the segmented stream of schedule format `fmt` (0 o3, 1 pr, 2 op, 4..6 g)
    const Segmented &seg_of(int fmt) const {
        return fmt == 0 ? o3 : fmt == 1 ? pr : fmt == 2 ? op : g[fmt - 4];
    }
    std::vector<int32_t> pair_i, pair_j;
    std::mutex sched_mu;
    std::map<std::pair<int, int>, std::unique_ptr<Schedule>> sched;  // (order, E or CW) -> schedule
    std::map<std::pair<int, int>, std::unique_ptr<HostSchedule>> hsched;
    const Schedule &schedule(int order, int E);
    const HostSchedule &host_schedule(int order, int E);
    void release_device();  // free every device buffer (ctx teardown)
};

// Build formats from host COO (validated, canonicalised).  Throws Error.
void build_formats(Tensor &t, const int32_t *i, const int32_t *j, const int32_t *k,
                   const void *val, int val_dtype, unsigned flags);
// The same for a general tensor (t.l, t.m, t.n set; repeats summed with
// BKS_SUM_DUPLICATES, else BKS_EDUP).
void build_formats_general(Tensor &t, const int32_t *i, const int32_t *j, const int32_t *k,
                           const void *val, int val_dtype, unsigned flags);
// Product of a general tensor with one free mode `mode` (0, 1, 2): B1, B2
// are the factors of the other two modes in mode order; out(row, a + p1 b).
void gttmc(Ctx &c, Tensor &t, int mode, const void *B1, int64_t ld1, int p1, const void *B2,
           int64_t ld2, int p2, int prec, void *out, int64_t ldo, hipStream_t s);

// ---------------------------------------------------------------- TTMc
// Launch a TTMc on device buffers; dtype of B/out follows prec.
void ttmc(Ctx &c, Tensor &t, int op, const void *B1, int64_t ld1, int p1, const void *B2,
          int64_t ld2, int p2, bool sym_half, int prec, void *out, int64_t ldo,
          hipStream_t s);
// The same product with every device workspace (packed factors, partial
// rows, intermediate products, the schedule) carved out of the library's
// fixed per-device scratch array: no device memory is allocated.  Narrow
// products only (symmetric halves up to 24 columns); BKS_EINVAL beyond the
// scratch size.
void ttmc_noalloc(Ctx &c, Tensor &t, int op, const void *B1, int64_t ld1, int p1,
                  const void *B2, int64_t ld2, int p2, bool sym_half, int prec, void *out,
                  int64_t ldo, hipStream_t s);
// Look up (once per device, with that device current) the device address of
// the scratch array used by ttmc_noalloc; called at context creation.
void scratch_init(int device);
size_t scratch_bytes();

// ---------------------------------------------------------------- dense kernels (dense.hip)
// out(k x q, ldo) = A^T B with A (rows x k, lda), B (rows x q, ldb); FP64 out.
void gemm_tn_f64(const double *A, int64_t lda, const double *B, int64_t ldb, int64_t rows,
                 int k, int q, double *out, int64_t ldo, Ctx &c, hipStream_t s);
void gemm_tn_f32f64(const double *A, int64_t lda, const float *B, int64_t ldb, int64_t rows,
                    int k, int q, double *out, int64_t ldo, Ctx &c, hipStream_t s);
// C(rows x q, ldc) = beta*C + alpha * A(rows x k, lda) H(k x q, ldh)
void gemm_nn_f64(const double *A, int64_t lda, const double *H, int64_t ldh, int64_t rows,
                 int k, int q, double alpha, double beta, double *C, int64_t ldc, hipStream_t s);
// G (q x q, double-double hi/lo, upper triangle) = B^T B, B rows x q (ldb)
void gram_dd(const double *B, int64_t ldb, int64_t rows, int q, double *Ghi, double *Glo,
             Ctx &c, hipStream_t s);
// column squared norms (FP64)
void colnorm2(const double *B, int64_t ldb, int64_t rows, int q, double *out, Ctx &c,
              hipStream_t s);
void convert_f64_f32(const double *src, int64_t lds, float *dst, int64_t ldd, int64_t rows,
                     int cols, hipStream_t s);
void convert_f32_f64(const float *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                     int cols, hipStream_t s);
void copy2d_f64(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                int cols, hipStream_t s);

}  // namespace bks
