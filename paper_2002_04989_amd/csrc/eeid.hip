// libeeid host runtime: the C ABI declared in include/eeid.h.
//
// Validation, workspace, the (matrix, minor) problem table and kernel
// launches.  All arithmetic of the method runs in the kernels of
// eeid_tridiag.hpp (eigenvalues of A and of its minors) and eeid_identity.hpp
// (Eq. (2) of the paper); the host only schedules.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "eeid.h"
#include "eeid_identity.hpp"
#include "eeid_tridiag.hpp"
#include "eeid_tridiag_c.hpp"

namespace {


struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct eeid_handle_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int cu_count = 0;
    std::string err;
    Buf work, items, desc, dpair, flags1;
    int *counter = nullptr;
    std::vector<int64_t> items_key, desc_key;
    int64_t n_items = 0;
    int variant = 0;  // kernel configuration (dispatch_variant)
};

namespace {

eeid_status_t fail(eeid_handle_t h, eeid_status_t s, const std::string &msg) {
    if (h) h->err = msg;
    return s;
}

#define HIP_TRY(h, call)                                                                      \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail((h), EEID_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Grow `b` to at least `bytes`; the stream is drained first so no queued
// kernel still reads the old allocation.
eeid_status_t ensure(eeid_handle_t h, Buf &b, size_t bytes) {
    if (b.bytes >= bytes) return EEID_OK;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (b.p) HIP_TRY(h, hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(h, EEID_ERR_ALLOC, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    b.bytes = bytes;
    return EEID_OK;
}

eeid_status_t check_batch(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t count,
                          const int64_t *n, const int64_t *a_offset, const void *A) {
    if (!h) return EEID_ERR_INVALID_ARG;
    if (t != EEID_R64 && t != EEID_C128) return fail(h, EEID_ERR_INVALID_ARG, "unknown dtype");
    if (p != EEID_PREC_FP64 && p != EEID_PREC_FP32_TRAILING)
        return fail(h, EEID_ERR_INVALID_ARG, "unknown precision");
    if (count < 1) return fail(h, EEID_ERR_INVALID_ARG, "count must be >= 1");
    if (!n || !a_offset || !A) return fail(h, EEID_ERR_INVALID_ARG, "null pointer argument");
    const int64_t nmax = (t == EEID_R64) ? EEID_MAX_N_R64 : EEID_MAX_N_C128;
    for (int64_t b = 0; b < count; ++b) {
        if (n[b] < 1) return fail(h, EEID_ERR_INVALID_ARG, "n[" + std::to_string(b) + "] must be >= 1");
        if (a_offset[b] < 0) return fail(h, EEID_ERR_INVALID_ARG, "negative a_offset");
        if (n[b] > nmax)
            return fail(h, EEID_ERR_UNSUPPORTED, "n[" + std::to_string(b) + "] exceeds the supported maximum");
    }
    return EEID_OK;
}

// Per-matrix descriptors (offsets of every output); cached on the batch shape.
eeid_status_t upload_desc(eeid_handle_t h, int64_t count, const int64_t *n, const int64_t *a_offset) {
    std::vector<int64_t> key;
    key.reserve(2 * count + 1);
    key.push_back(count);
    for (int64_t b = 0; b < count; ++b) { key.push_back(n[b]); key.push_back(a_offset ? a_offset[b] : 0); }
    if (key == h->desc_key) return EEID_OK;
    std::vector<eeid::BatchDesc> d(count);
    int64_t lam = 0, mu = 0, v2 = 0;
    for (int64_t b = 0; b < count; ++b) {
        d[b].a_off = a_offset ? a_offset[b] : 0;
        d[b].lam_off = lam;
        d[b].mu_off = mu;
        d[b].v2_off = v2;
        d[b].n = (int32_t)n[b];
        d[b].pad = 0;
        lam += n[b];
        mu += n[b] * (n[b] - 1);
        v2 += n[b] * n[b];
    }
    eeid_status_t s = ensure(h, h->desc, sizeof(eeid::BatchDesc) * count);
    if (s != EEID_OK) return s;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpy(h->desc.p, d.data(), sizeof(eeid::BatchDesc) * count, hipMemcpyHostToDevice));
    h->desc_key.swap(key);
    return EEID_OK;
}

// Launch one compiled configuration of the persistent eigenvalue kernel over
// the problem table: one workgroup per slot, as many slots as fit the device
// (occupancy x CUs, capped by the problem count and by free memory).
eeid_status_t launch_persistent(eeid_handle_t h, const void *kern, int nt, int64_t slot, size_t lds,
                                const std::vector<eeid::Item> &items, const std::vector<int64_t> &key,
                                int LDmax, const int32_t *flags) {
    using namespace eeid;
    if (items.empty()) return EEID_OK;
    if (key != h->items_key) {
        eeid_status_t s = ensure(h, h->items, sizeof(Item) * items.size());
        if (s != EEID_OK) return s;
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        HIP_TRY(h, hipMemcpy(h->items.p, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice));
        h->items_key = key;
        h->n_items = (int64_t)items.size();
    }
    HIP_TRY(h, hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    HIP_TRY(h, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nt, lds));
    if (per_cu < 1) return fail(h, EEID_ERR_UNSUPPORTED, "eigenvalue kernel cannot be resident");
    int64_t slots = (int64_t)per_cu * h->cu_count;
    slots = std::min<int64_t>(slots, (int64_t)items.size());
    size_t free_b = 0, total_b = 0;
    HIP_TRY(h, hipMemGetInfo(&free_b, &total_b));
    const size_t budget = (size_t)((double)(free_b + h->work.bytes) * 0.85);
    slots = std::min<int64_t>(slots, (int64_t)(budget / (size_t)slot));
    if (slots < 1) return fail(h, EEID_ERR_ALLOC, "not enough device memory for one problem slot");
    eeid_status_t s = ensure(h, h->work, (size_t)(slots * slot));
    if (s != EEID_OK) return s;
    TriArgs a;
    a.items = reinterpret_cast<const Item *>(h->items.p);
    a.n_items = h->n_items;
    a.counter = h->counter;
    a.flags = flags;
    a.work = reinterpret_cast<char *>(h->work.p);
    a.slot_bytes = slot;
    a.LDmax = LDmax;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, h->stream, h->counter);
    void *argv[] = {&a};
    HIP_TRY(h, hipLaunchKernel(kern, dim3((unsigned)slots), dim3((unsigned)nt), argv, lds, h->stream));
    return EEID_OK;
}

template <class S, int NB, int NT, int CW, bool STAGE, int WPE>
eeid_status_t launch_tridiag(eeid_handle_t h, const std::vector<eeid::Item> &items,
                             const std::vector<int64_t> &key, int max_m, const int32_t *flags) {
    using namespace eeid;
    const int LDmax = ((max_m + TILE - 1) / TILE) * TILE;
    return launch_persistent(h, (const void *)tridiag_bisect_kernel<S, NB, NT, CW, STAGE, WPE>, NT,
                             slot_bytes_for<S, NB>(LDmax), (size_t)lds_bytes_for<NB, NT, STAGE>(LDmax), items, key,
                             LDmax, flags);
}

template <class R, int NB, int NT, int CW>
eeid_status_t launch_tridiag_c(eeid_handle_t h, const std::vector<eeid::Item> &items,
                               const std::vector<int64_t> &key, int max_m, const int32_t *flags) {
    using namespace eeid;
    const int LDmax = ((max_m + TILE - 1) / TILE) * TILE;
    return launch_persistent(h, (const void *)tridiag_bisect_kernel_c<R, NB, NT, CW>, NT, slot_bytes_c<R, NB>(LDmax),
                             (size_t)lds_bytes_c<NB, NT>(LDmax), items, key, LDmax, flags);
}

// Kernel configurations: (panel width NB, threads NT, SYMV unit width CW,
// LDS staging of the trailing update, waves per SIMD).
eeid_status_t dispatch_variant(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p,
                               const std::vector<eeid::Item> &items, const std::vector<int64_t> &key, int nmax,
                               const int32_t *flags) {
    const bool d = (p == EEID_PREC_FP64);
    if (t == EEID_C128)  // complex: panel 16, 16-column SYMV units, no LDS staging
        return d ? launch_tridiag_c<double, 16, 512, 16>(h, items, key, nmax, flags)
                 : launch_tridiag_c<float, 16, 512, 16>(h, items, key, nmax, flags);
    switch (h->variant) {
        case 1:
            return d ? launch_tridiag<double, 32, 256, 32, true, 2>(h, items, key, nmax, flags)
                     : launch_tridiag<float, 32, 256, 32, true, 2>(h, items, key, nmax, flags);
        default:
            return d ? launch_tridiag<double, 32, 512, 32, true, 2>(h, items, key, nmax, flags)
                     : launch_tridiag<float, 32, 512, 32, true, 2>(h, items, key, nmax, flags);
    }
}

// kind 0: eigenvalues of the matrices only; kind 1: matrices and all minors;
// kind 2: one matrix and a subset of minors.
eeid_status_t run_eigs(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t count, const int64_t *n,
                       const int64_t *a_offset, const void *A, double *lambda, double *mu,
                       int32_t *flags, int kind, int64_t nsel, const int64_t *js) {
    using eeid::Item;
    HIP_TRY(h, hipSetDevice(h->device));
    eeid_status_t s = upload_desc(h, count, n, a_offset);
    if (s != EEID_OK) return s;
    const eeid::BatchDesc *desc = reinterpret_cast<const eeid::BatchDesc *>(h->desc.p);
    std::vector<int64_t> key;
    key.push_back(kind);
    key.push_back((int64_t)t);
    key.push_back((int64_t)p);
    key.push_back((int64_t)(intptr_t)A);
    key.push_back((int64_t)(intptr_t)lambda);
    key.push_back((int64_t)(intptr_t)mu);
    key.push_back(count);
    for (int64_t b = 0; b < count; ++b) { key.push_back(n[b]); key.push_back(a_offset[b]); }
    for (int64_t q = 0; q < nsel; ++q) key.push_back(js[q]);

    std::vector<Item> items;
    int64_t nmax = 0, lam = 0, muo = 0;
    const double *Ad = reinterpret_cast<const double *>(A);
    const int64_t esz = (t == EEID_C128) ? 2 : 1;  // doubles per element
    for (int64_t b = 0; b < count; ++b) {
        const int nb = (int)n[b];
        const double *src = Ad + esz * a_offset[b];
        nmax = std::max<int64_t>(nmax, nb);
        if (lambda) items.push_back(Item{src, lambda + lam, nb, -1, nb, (int32_t)b});
        if (kind == 1 && nb >= 2)
            for (int j = 0; j < nb; ++j)
                items.push_back(Item{src, mu + muo + (int64_t)j * (nb - 1), nb, j, nb - 1, (int32_t)b});
        if (kind == 2 && nb >= 2)
            for (int64_t q = 0; q < nsel; ++q)
                items.push_back(Item{src, mu + q * (nb - 1), nb, (int)js[q], nb - 1, (int32_t)b});
        lam += nb;
        muo += (int64_t)nb * (nb - 1);
    }
    // largest problems first so that the tail of the queue is short
    std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.m > y.m; });

    const int64_t nn_blocks = (nmax * nmax + 4095) / 4096;
    hipLaunchKernelGGL(eeid::prep_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, h->stream,
                       flags, count, (int *)nullptr);
    hipLaunchKernelGGL(eeid::nonfinite_kernel, dim3((unsigned)nn_blocks, (unsigned)count), dim3(256), 0,
                       h->stream, desc, Ad, t == EEID_C128 ? 1 : 0, flags);
    HIP_TRY(h, hipGetLastError());
    return dispatch_variant(h, t, p, items, key, (int)nmax, flags);
}

}  // namespace

extern "C" {

eeid_status_t eeid_create(eeid_handle_t *out, int hip_device) {
    if (!out) return EEID_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return EEID_ERR_NO_DEVICE;
    }
    if (hip_device < 0 || hip_device >= ndev) return EEID_ERR_NO_DEVICE;
    eeid_handle_t h = new (std::nothrow) eeid_handle_s();
    if (!h) return EEID_ERR_ALLOC;
    h->device = hip_device;
    if (const char *e = getenv("EEID_VARIANT")) h->variant = atoi(e);
    if (hipSetDevice(hip_device) != hipSuccess ||
        hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess ||
        hipMalloc(&h->counter, sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        return EEID_ERR_HIP;
    }
    *out = h;
    return EEID_OK;
}

eeid_status_t eeid_destroy(eeid_handle_t h) {
    if (!h) return EEID_ERR_INVALID_ARG;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    Buf *bufs[] = {&h->work, &h->items, &h->desc, &h->dpair, &h->flags1};
    for (Buf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (h->counter) (void)hipFree(h->counter);
    delete h;
    return EEID_OK;
}

eeid_status_t eeid_set_stream(eeid_handle_t h, void *stream) {
    if (!h) return EEID_ERR_INVALID_ARG;
    h->stream = reinterpret_cast<hipStream_t>(stream);
    return EEID_OK;
}

const char *eeid_status_string(eeid_status_t s) {
    switch (s) {
        case EEID_OK: return "EEID_OK: success";
        case EEID_ERR_INVALID_ARG: return "EEID_ERR_INVALID_ARG: invalid argument";
        case EEID_ERR_NO_DEVICE: return "EEID_ERR_NO_DEVICE: no usable HIP device";
        case EEID_ERR_ALLOC: return "EEID_ERR_ALLOC: device allocation failed";
        case EEID_ERR_HIP: return "EEID_ERR_HIP: HIP runtime error";
        case EEID_ERR_UNSUPPORTED: return "EEID_ERR_UNSUPPORTED: request not supported by this build";
    }
    return "unknown eeid status";
}

const char *eeid_last_error(eeid_handle_t h) { return h ? h->err.c_str() : ""; }

eeid_status_t eeid_eigvalsh_batched(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t count,
                                    const int64_t *n, const int64_t *a_offset, const void *A,
                                    double *lambda, int32_t *flags) {
    eeid_status_t s = check_batch(h, t, p, count, n, a_offset, A);
    if (s != EEID_OK) return s;
    if (!lambda || !flags) return fail(h, EEID_ERR_INVALID_ARG, "null output pointer");
    return run_eigs(h, t, p, count, n, a_offset, A, lambda, nullptr, flags, 0, 0, nullptr);
}

eeid_status_t eeid_minor_eigvals(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t count,
                                 const int64_t *n, const int64_t *a_offset, const void *A,
                                 double *lambda, double *mu, int32_t *flags) {
    eeid_status_t s = check_batch(h, t, p, count, n, a_offset, A);
    if (s != EEID_OK) return s;
    if (!lambda || !flags) return fail(h, EEID_ERR_INVALID_ARG, "null output pointer");
    bool need_mu = false;
    for (int64_t b = 0; b < count; ++b) need_mu = need_mu || n[b] >= 2;
    if (need_mu && !mu) return fail(h, EEID_ERR_INVALID_ARG, "mu is null");
    return run_eigs(h, t, p, count, n, a_offset, A, lambda, mu, flags, 1, 0, nullptr);
}

eeid_status_t eeid_minor_eigvals_subset(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t n,
                                        const void *A, int64_t nsel, const int64_t *js, double *lambda,
                                        double *mu_sel, int32_t *flag) {
    const int64_t zero = 0;
    eeid_status_t s = check_batch(h, t, p, 1, &n, &zero, A);
    if (s != EEID_OK) return s;
    if (nsel < 1 || !js) return fail(h, EEID_ERR_INVALID_ARG, "nsel must be >= 1 and js non-null");
    if (!flag) return fail(h, EEID_ERR_INVALID_ARG, "null flag pointer");
    if (n >= 2 && !mu_sel) return fail(h, EEID_ERR_INVALID_ARG, "mu_sel is null");
    for (int64_t q = 0; q < nsel; ++q)
        if (js[q] < 0 || js[q] >= n) return fail(h, EEID_ERR_INVALID_ARG, "js entry out of range");
    return run_eigs(h, t, p, 1, &n, &zero, A, lambda, mu_sel, flag, 2, nsel, js);
}

eeid_status_t eeid_components(eeid_handle_t h, int64_t count, const int64_t *n, const double *lambda,
                              const double *mu, double *V2, int32_t *flags) {
    if (!h) return EEID_ERR_INVALID_ARG;
    if (count < 1) return fail(h, EEID_ERR_INVALID_ARG, "count must be >= 1");
    if (!n || !lambda || !V2 || !flags) return fail(h, EEID_ERR_INVALID_ARG, "null pointer argument");
    int64_t nmax = 0, ntot = 0;
    bool need_mu = false;
    for (int64_t b = 0; b < count; ++b) {
        if (n[b] < 1) return fail(h, EEID_ERR_INVALID_ARG, "n[" + std::to_string(b) + "] must be >= 1");
        if (n[b] > EEID_MAX_N_R64) return fail(h, EEID_ERR_UNSUPPORTED, "n exceeds the supported maximum");
        nmax = std::max(nmax, n[b]);
        ntot += n[b];
        need_mu = need_mu || n[b] >= 2;
    }
    if (need_mu && !mu) return fail(h, EEID_ERR_INVALID_ARG, "mu is null");
    HIP_TRY(h, hipSetDevice(h->device));
    // descriptors: a_offset is irrelevant here; keep any cached one for the same n list
    std::vector<int64_t> zeros(count, 0);
    const int64_t *aoff = zeros.data();
    if (h->desc_key.size() == (size_t)(2 * count + 1) && h->desc_key[0] == count) {
        bool same = true;
        for (int64_t b = 0; b < count && same; ++b) same = h->desc_key[1 + 2 * b] == n[b];
        if (same)
            for (int64_t b = 0; b < count; ++b) zeros[b] = h->desc_key[2 + 2 * b];
    }
    eeid_status_t s = upload_desc(h, count, n, aoff);
    if (s != EEID_OK) return s;
    s = ensure(h, h->dpair, sizeof(double) * 2 * (size_t)ntot);
    if (s != EEID_OK) return s;
    const eeid::BatchDesc *desc = reinterpret_cast<const eeid::BatchDesc *>(h->desc.p);
    double *dpair = reinterpret_cast<double *>(h->dpair.p);
    const unsigned ib = (unsigned)((nmax + 255) / 256);
    hipLaunchKernelGGL(eeid::denominators_kernel, dim3(ib, (unsigned)count), dim3(256), 0, h->stream, desc,
                       lambda, dpair, flags);
    const unsigned jb = (unsigned)((nmax + eeid::ID_JT - 1) / eeid::ID_JT);
    hipLaunchKernelGGL(eeid::identity_kernel, dim3(ib, jb, (unsigned)count), dim3(256), 0, h->stream, desc,
                       lambda, mu, dpair, V2);
    HIP_TRY(h, hipGetLastError());
    return EEID_OK;
}

eeid_status_t eeid_all_components(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t count,
                                  const int64_t *n, const int64_t *a_offset, const void *A, double *lambda,
                                  double *mu, double *V2, int32_t *flags) {
    eeid_status_t s = eeid_minor_eigvals(h, t, p, count, n, a_offset, A, lambda, mu, flags);
    if (s != EEID_OK) return s;
    return eeid_components(h, count, n, lambda, mu, V2, flags);
}

}  // extern "C"
