// C ABI entry points of libbks: context, tensor upload, tensor-times-block
// products.  Solver and server entry points live in solver.cpp / server.cpp.
#include <algorithm>
#include <cstring>
#include <new>

#include "bks_internal.h"

namespace bks {

void fail(int code, const std::string &msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) fail(BKS_ENOMEM, std::string("out of device memory: ") + what);
    fail(BKS_EDEVICE, std::string(hipGetErrorString(e)) + " in " + what);
}

thread_local std::shared_ptr<DevAccount> DevAccount::current;

void DevAccount::add(size_t b) {
    const size_t now = live.fetch_add(b) + b;
    size_t p = peak.load();
    while (now > p && !peak.compare_exchange_weak(p, now)) {
    }
}

DevBuf::~DevBuf() { release(); }

void DevBuf::alloc(size_t b) {
    release();
    if (b == 0) return;
    if (const char *f = std::getenv("BKS_FAIL_NEXT_ALLOC")) {
        if (f[0] == '1') {
            unsetenv("BKS_FAIL_NEXT_ALLOC");
            fail(BKS_ENOMEM, "injected allocation failure");
        }
    }
    hipError_t e = hipMalloc(&ptr, b);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        fail(BKS_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed");
    }
    bytes = b;
    acct = DevAccount::current;
    if (acct) acct->add(b);
}

void DevBuf::ensure(size_t b) {
    if (b <= bytes) return;
    alloc(b + b / 4);
}

void DevBuf::release() {
    if (ptr) (void)hipFree(ptr);
    if (ptr && acct) acct->sub(bytes);
    ptr = nullptr;
    bytes = 0;
    acct.reset();
}

PinnedBuf::~PinnedBuf() {
    if (ptr) (void)hipHostFree(ptr);
}

void PinnedBuf::ensure(size_t b) {
    if (b <= bytes) return;
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
    void *q = nullptr;
    // coherent (fine-grained): the same staging bytes are written by the host
    // and read by the copy engines or blit kernels over and over, so no
    // device cache may keep an old copy of them
    hipError_t e = hipHostMalloc(&q, b, hipHostMallocCoherent);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(BKS_ENOMEM, "hipHostMalloc of " + std::to_string(b) + " bytes failed");
    }
    ptr = static_cast<char *>(q);
    bytes = b;
}

void Ctx::release_workspaces() {
    for (DevBuf *b : {&ws_partial, &ws_pack1, &ws_pack2, &ws_fac1, &ws_fac2, &devsolve.dH,
                      &devsolve.dA, &devsolve.db, &devinner.dC, &devinner.dA,
                      &devinner.dOut, &devinner.dT, &devinner.dY, &devinner.dOnes})
        b->release();
}

}  // namespace bks

using namespace bks;

struct bks_ctx_s : public Ctx {};
struct bks_tensor_s : public Tensor {};

namespace {

template <class F>
int guard(Ctx *c, F f) {
    try {
        f();
        return BKS_OK;
    } catch (const Error &e) {
        if (c) c->last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        if (c) c->last_error = "host allocation failed";
        return BKS_ENOMEM;
    } catch (const std::exception &e) {
        if (c) c->last_error = e.what();
        return BKS_EDEVICE;
    }
}

}  // namespace

extern "C" {

const char *bks_version(void) { return "libbks 0.1 (gfx950)"; }

int bks_ctx_create(int device, size_t mem_budget_bytes, bks_ctx *out) {
    if (!out) return BKS_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return BKS_EDEVICE;
    }
    if (device < 0 || device >= ndev) return BKS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return BKS_EDEVICE;
    auto *c = new (std::nothrow) bks_ctx_s();
    if (!c) return BKS_ENOMEM;
    c->device = device;
    c->budget = mem_budget_bytes;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return BKS_EDEVICE;
    }
    // the allocation-free product's scratch address on this device (once
    // per device, with the device current)
    try {
        scratch_init(device);
    } catch (const Error &) {
        (void)hipStreamDestroy(c->stream);
        delete c;
        return BKS_EDEVICE;
    }
    *out = c;
    return BKS_OK;
}

void bks_ctx_destroy(bks_ctx ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    {
        // tensors still alive become empty handles (bks_tensor_free stays valid)
        std::lock_guard<std::mutex> g(ctx->tensors_mu);
        for (Tensor *t : ctx->tensors) {
            t->release_device();
            t->ctx = nullptr;
        }
        ctx->tensors.clear();
    }
    ctx->prof_flush();
    (void)hipStreamDestroy(ctx->stream);
    (void)hipGetLastError();
    delete ctx;
}

const char *bks_last_error(bks_ctx ctx) {
    if (!ctx) return "null context";
    return ctx->last_error.c_str();
}

int bks_tensor_upload(bks_ctx ctx, int64_t m, int64_t n, int64_t nnz, const int32_t *i,
                      const int32_t *j, const int32_t *k, const void *val, int val_dtype,
                      unsigned flags, bks_tensor *out) {
    if (!ctx || !out) return BKS_EINVAL;
    *out = nullptr;
    return guard(ctx, [&] {
        if (m < 1 || n < 1 || nnz < 0) fail(BKS_EINVAL, "m, n must be >= 1 and nnz >= 0");
        if (m > (int64_t)INT32_MAX || n > (int64_t)INT32_MAX) fail(BKS_EINVAL, "m or n too large");
        if (val_dtype != BKS_F32 && val_dtype != BKS_F64) fail(BKS_EINVAL, "val_dtype");
        if (nnz > 0 && (!i || !j || !k || !val)) fail(BKS_EINVAL, "null coordinate array");
        HIPCHECK(hipSetDevice(ctx->device));
        std::vector<int32_t> hi, hj, hk;
        std::vector<char> hv;
        const int32_t *I = i, *J = j, *K = k;
        const void *V = val;
        const size_t vb = val_dtype == BKS_F64 ? 8 : 4;
        if (flags & BKS_DEVICE_PTRS) {
            hi.resize(nnz); hj.resize(nnz); hk.resize(nnz); hv.resize(nnz * vb);
            if (nnz) {
                HIPCHECK(hipMemcpy(hi.data(), i, nnz * 4, hipMemcpyDeviceToHost));
                HIPCHECK(hipMemcpy(hj.data(), j, nnz * 4, hipMemcpyDeviceToHost));
                HIPCHECK(hipMemcpy(hk.data(), k, nnz * 4, hipMemcpyDeviceToHost));
                HIPCHECK(hipMemcpy(hv.data(), val, nnz * vb, hipMemcpyDeviceToHost));
            }
            I = hi.data(); J = hj.data(); K = hk.data(); V = hv.data();
        }
        auto t = std::make_unique<bks_tensor_s>();
        t->ctx = ctx;
        t->m = m;
        t->n = n;
        t->nnz = nnz;
        build_formats(*t, I, J, K, V, val_dtype, flags);
        if (ctx->budget && ctx->used + t->dev_bytes > ctx->budget)
            fail(BKS_ENOMEM, "tensor exceeds the context memory budget");
        ctx->used += t->dev_bytes;
        {
            std::lock_guard<std::mutex> g(ctx->tensors_mu);
            ctx->tensors.push_back(t.get());
        }
        *out = t.release();
    });
}

int bks_tensor_info(bks_tensor t, int64_t *m, int64_t *n, int64_t *nnz_stored, int64_t *npairs,
                    double *frob_norm, size_t *dev_bytes) {
    if (!t) return BKS_EINVAL;
    // a general tensor reports its mode-1 size as m and its mode-2 size as npairs
    if (m) *m = t->general ? t->l : t->m;
    if (n) *n = t->n;
    if (nnz_stored) *nnz_stored = t->nnz;
    if (npairs) *npairs = t->general ? t->m : t->npairs;
    if (frob_norm) *frob_norm = std::sqrt(t->frob2);
    if (dev_bytes) *dev_bytes = t->dev_bytes;
    return BKS_OK;
}

int bks_tensor_pairs(bks_tensor t, int32_t *pi, int32_t *pj) {
    if (!t || !pi || !pj) return BKS_EINVAL;
    std::memcpy(pi, t->pair_i.data(), t->pair_i.size() * 4);
    std::memcpy(pj, t->pair_j.data(), t->pair_j.size() * 4);
    return BKS_OK;
}

void bks_tensor_free(bks_tensor t) {
    if (!t) return;
    if (Ctx *c = t->ctx) {
        (void)hipSetDevice(c->device);
        if (c->used >= t->dev_bytes) c->used -= t->dev_bytes;
        std::lock_guard<std::mutex> g(c->tensors_mu);
        auto &v = c->tensors;
        v.erase(std::remove(v.begin(), v.end(), static_cast<Tensor *>(t)), v.end());
    }
    delete t;
    (void)hipGetLastError();
}

int bks_ctx_profile(bks_ctx ctx, int enable) {
    if (!ctx) return BKS_EINVAL;
    return guard(ctx, [&] {
        ctx->prof_flush();
        std::lock_guard<std::mutex> g(ctx->prof_mu);
        ctx->prof_stats.clear();
        ctx->prof = enable != 0;
    });
}

int bks_ctx_profile_read(bks_ctx ctx, int idx, char *name, int name_len, int64_t *calls,
                         double *ms, double *bytes, double *flops) {
    if (!ctx || idx < 0) return BKS_EINVAL;
    int rc = guard(ctx, [&] { ctx->prof_flush(); });
    if (rc) return rc;
    std::lock_guard<std::mutex> g(ctx->prof_mu);
    int i = 0;
    for (auto &kv : ctx->prof_stats) {
        if (i++ != idx) continue;
        if (name && name_len > 0) {
            std::strncpy(name, kv.first.c_str(), name_len - 1);
            name[name_len - 1] = 0;
        }
        if (calls) *calls = kv.second.calls;
        if (ms) *ms = kv.second.ms;
        if (bytes) *bytes = kv.second.bytes;
        if (flops) *flops = kv.second.flops;
        return BKS_OK;
    }
    return BKS_ENOTFOUND;
}

int bks_ttmc(bks_ctx ctx, bks_tensor t, int op, const void *B1, int64_t ld1, int p1,
             const void *B2, int64_t ld2, int p2, int sym_half, int prec, void *out, int64_t ldo,
             void *stream) {
    if (!ctx || !t) return BKS_EINVAL;
    return guard(ctx, [&] {
        HIPCHECK(hipSetDevice(ctx->device));
        ttmc(*ctx, *t, op, B1, ld1, p1, B2, ld2, p2, sym_half != 0, prec, out, ldo,
             static_cast<hipStream_t>(stream));
    });
}

int bks_gtensor_upload(bks_ctx ctx, int64_t l, int64_t m, int64_t n, int64_t nnz,
                       const int32_t *i, const int32_t *j, const int32_t *k, const void *val,
                       int val_dtype, unsigned flags, bks_tensor *out) {
    if (!ctx || !out) return BKS_EINVAL;
    *out = nullptr;
    if (l < 1 || m < 1 || n < 1 || nnz < 0 || l > (int64_t)INT32_MAX || m > (int64_t)INT32_MAX ||
        n > (int64_t)INT32_MAX || (val_dtype != BKS_F32 && val_dtype != BKS_F64))
        return guard(ctx, [] { fail(BKS_EINVAL, "bad sizes or value type"); });
    if (nnz > 0 && (!i || !j || !k || !val)) return BKS_EINVAL;
    if (flags & ~(unsigned)(BKS_DEVICE_PTRS | BKS_SUM_DUPLICATES))
        return guard(ctx, [] { fail(BKS_EINVAL, "flags: only BKS_DEVICE_PTRS and BKS_SUM_DUPLICATES"); });
    auto t = std::make_unique<bks_tensor_s>();
    t->ctx = ctx;
    t->l = l;
    t->m = m;
    t->n = n;
    t->nnz = nnz;
    const int rc = guard(ctx, [&] {
        HIPCHECK(hipSetDevice(ctx->device));
        const size_t vb = val_dtype == BKS_F64 ? 8 : 4;
        std::vector<int32_t> hi, hj, hk;
        std::vector<char> hv;
        const int32_t *pi = i, *pj = j, *pk = k;
        const void *pv = val;
        if (flags & BKS_DEVICE_PTRS) {
            hi.resize(nnz);
            hj.resize(nnz);
            hk.resize(nnz);
            hv.resize((size_t)nnz * vb);
            if (nnz) {
                HIPCHECK(hipMemcpy(hi.data(), i, nnz * 4, hipMemcpyDeviceToHost));
                HIPCHECK(hipMemcpy(hj.data(), j, nnz * 4, hipMemcpyDeviceToHost));
                HIPCHECK(hipMemcpy(hk.data(), k, nnz * 4, hipMemcpyDeviceToHost));
                HIPCHECK(hipMemcpy(hv.data(), val, nnz * vb, hipMemcpyDeviceToHost));
            }
            pi = hi.data();
            pj = hj.data();
            pk = hk.data();
            pv = hv.data();
        }
        build_formats_general(*t, pi, pj, pk, pv, val_dtype, flags & ~(unsigned)BKS_DEVICE_PTRS);
        if (ctx->budget && ctx->used + t->dev_bytes > ctx->budget)
            fail(BKS_ENOMEM, "tensor exceeds the context memory budget");
        ctx->used += t->dev_bytes;
    });
    if (rc != BKS_OK) {
        t->release_device();
        return rc;
    }
    {
        std::lock_guard<std::mutex> g(ctx->tensors_mu);
        ctx->tensors.push_back(t.get());
    }
    *out = t.release();
    return BKS_OK;
}

int bks_gttmc(bks_ctx ctx, bks_tensor t, int mode, const void *B1, int64_t ld1, int p1,
              const void *B2, int64_t ld2, int p2, int prec, void *out, int64_t ldo,
              void *stream) {
    if (!ctx || !t) return BKS_EINVAL;
    return guard(ctx, [&] {
        HIPCHECK(hipSetDevice(ctx->device));
        gttmc(*ctx, *t, mode, B1, ld1, p1, B2, ld2, p2, prec, out, ldo,
              static_cast<hipStream_t>(stream));
    });
}

int bks_ttmc_noalloc(bks_ctx ctx, bks_tensor t, int op, const void *B1, int64_t ld1, int p1,
                     const void *B2, int64_t ld2, int p2, int sym_half, int prec, void *out,
                     int64_t ldo, void *stream) {
    if (!ctx || !t) return BKS_EINVAL;
    return guard(ctx, [&] {
        HIPCHECK(hipSetDevice(ctx->device));
        ttmc_noalloc(*ctx, *t, op, B1, ld1, p1, B2, ld2, p2, sym_half != 0, prec, out, ldo,
                     static_cast<hipStream_t>(stream));
    });
}

}  // extern "C"
