// libeeid host runtime: the C ABI declared in include/eeid.h.
//
// Validation, workspace, the (matrix, minor) problem table, kernel selection
// (autotuned), optional hipGraph capture and kernel launches.  All arithmetic
// of the method runs in the kernels of eeid_tridiag.hpp / eeid_tridiag_c.hpp
// (eigenvalues of A and of its minors) and eeid_identity.hpp (Eq. (2) of the
// paper); the host only schedules.
//
// Every entry point is split into a prepare step (argument checks, uploads of
// descriptor tables, workspace growth -- host-synchronous, never captured)
// and an enqueue step (kernel launches only), so that the enqueue steps can
// be recorded into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "eeid.h"
#include "eeid_band.hpp"
#include "eeid_identity.hpp"
#include "eeid_latency.hpp"
#include "eeid_tridiag.hpp"
#include "eeid_tridiag_c.hpp"

namespace {

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

typedef std::function<hipError_t(hipStream_t)> Enqueue;

// Compiled configurations of the real eigenvalue kernel (the complex kernel
// has one): one-stage reduction with panel width NB and threads per
// workgroup, or the two-stage (dense -> band -> tridiagonal) reduction.
constexpr int N_REAL_VARIANTS = 5;
const char *const VARIANT_NAME[N_REAL_VARIANTS] = {"nb32_nt512", "nb32_nt256x2", "nb16_nt512", "band32_nt512",
                                                   "band32_nt256x2"};

// Device scratch of eeid_components_noalloc: the batch descriptors, then the
// (mantissa, exponent) pairs of the denominators.  Every GPU the library runs
// on holds its own copy until the process ends; host code never uses this
// name as an address (it is a host-side stand-in), only the per-device
// address that hipGetSymbolAddress returns.
constexpr size_t NOALLOC_DESC_BYTES = 4096;
constexpr int64_t NOALLOC_MAX_EIGENVALUES = 16384;   // sum of n_b per call
constexpr size_t NOALLOC_SCRATCH_BYTES = NOALLOC_DESC_BYTES + 2 * sizeof(double) * NOALLOC_MAX_EIGENVALUES;
static_assert(eeid::NLIST_MAX * sizeof(eeid::BatchDesc) <= NOALLOC_DESC_BYTES, "descriptor region");
static_assert(NOALLOC_MAX_EIGENVALUES == EEID_NOALLOC_MAX_EIGENVALUES, "header and library agree");
static_assert(eeid::NLIST_MAX == EEID_NOALLOC_MAX_MATRICES, "header and library agree");
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

}  // namespace

struct eeid_handle_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int cu_count = 0;
    std::string err;
    Buf work, items, desc, desc_sub, dpair, dpair_sub, lam_ready, sbuf, lat_work, lat_items, lat_bar;
    Buf comp;   // eeid_component: lambda, mu and the column of its matrix
    int *counter = nullptr;
    char *scratch_ptr = nullptr;   // this device's copy of `scratch` (hipGetSymbolAddress at create)
    std::vector<int64_t> items_key, desc_key, desc_sub_key;
    int64_t n_items = 0;
    int variant = -1;           // >= 0: real-kernel configuration when the tune table has no entry
    int forced_variant = -1;    // >= 0: use this configuration (autotuning, EEID_VARIANT)
    int64_t max_slots = 0;      // > 0: cap on resident problems (EEID_MAX_SLOTS)
    unsigned spin_limit = 1u << 26;   // polls before a bounded inter-wave wait gives up (EEID_SPIN_LIMIT)
    int identity_form = EEID_IDENTITY_PRODUCTS;
    uint64_t generation = 0;    // bumped whenever a buffer the kernels read is reallocated or rewritten
    // graph mode
    bool graph_mode = false;
    hipStream_t gstream = nullptr;
    struct Graph { std::vector<int64_t> key; hipGraphExec_t exec; };
    std::vector<Graph> graphs;   // recorded launches, least recently used first (at most GRAPH_CACHE)
    // tune table: {dtype, prec, n_max, problems, variant}
    std::vector<std::array<int64_t, 5>> tune;
    std::string tune_path;
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

// Drain every stream the handle launches on.
eeid_status_t drain(eeid_handle_t h) {
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (h->gstream) HIP_TRY(h, hipStreamSynchronize(h->gstream));
    return EEID_OK;
}

// Grow `b` to at least `bytes`; queued work is drained first so no kernel
// still reads the old allocation, and captured graphs are invalidated.
eeid_status_t ensure(eeid_handle_t h, Buf &b, size_t bytes) {
    if (b.bytes >= bytes) return EEID_OK;
    eeid_status_t s = drain(h);
    if (s != EEID_OK) return s;
    if (b.p) HIP_TRY(h, hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
    ++h->generation;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(h, EEID_ERR_ALLOC, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    b.bytes = bytes;
    return EEID_OK;
}

// Upload a host table to `b` when `key` differs from the cached one.
template <class T>
eeid_status_t upload_table(eeid_handle_t h, Buf &b, std::vector<int64_t> &cached, std::vector<int64_t> &key,
                           const std::vector<T> &rows) {
    if (key == cached) return EEID_OK;
    eeid_status_t s = ensure(h, b, sizeof(T) * std::max<size_t>(rows.size(), 1));
    if (s != EEID_OK) return s;
    s = drain(h);
    if (s != EEID_OK) return s;
    if (!rows.empty())
        HIP_TRY(h, hipMemcpy(b.p, rows.data(), sizeof(T) * rows.size(), hipMemcpyHostToDevice));
    cached.swap(key);
    ++h->generation;
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

// Per-matrix descriptors (offsets of every output).  ncol < 0: all n columns.
eeid_status_t upload_desc(eeid_handle_t h, Buf &buf, std::vector<int64_t> &cached, int64_t count,
                          const int64_t *n, const int64_t *a_offset, int64_t ncol) {
    std::vector<int64_t> key;
    key.reserve(2 * count + 2);
    key.push_back(count);
    key.push_back(ncol);
    for (int64_t b = 0; b < count; ++b) { key.push_back(n[b]); key.push_back(a_offset ? a_offset[b] : 0); }
    std::vector<eeid::BatchDesc> d(count);
    int64_t lam = 0, mu = 0, v2 = 0;
    for (int64_t b = 0; b < count; ++b) {
        const int64_t nc = (ncol < 0) ? n[b] : ncol;
        d[b].a_off = a_offset ? a_offset[b] : 0;
        d[b].lam_off = lam;
        d[b].mu_off = mu;
        d[b].v2_off = v2;
        d[b].n = (int32_t)n[b];
        d[b].ncol = (int32_t)nc;
        lam += n[b];
        mu += nc * (n[b] - 1);
        v2 += n[b] * nc;
    }
    return upload_table(h, buf, cached, key, d);
}

struct KernelChoice {
    const void *kern;
    int nt;
    int64_t slot;
    size_t lds;
};

template <class S, int NB, int NT>
KernelChoice real_kernel(int LDmax) {
    using namespace eeid;
    return {(const void *)tridiag_bisect_kernel<S, NB, NT, 32, true, 2>, NT, slot_bytes_for<S, NB>(LDmax),
            (size_t)lds_bytes_for<NB, NT, true>(LDmax)};
}

template <class S, int NT>
KernelChoice band_kernel(int LDmax) {
    using namespace eeid;
    return {(const void *)band_bisect_kernel<S, NT>, NT, slot_bytes_band<S>(LDmax), (size_t)lds_bytes_band<NT>(LDmax)};
}

template <class R, int NB, int NT>
KernelChoice complex_kernel(int LDmax) {
    using namespace eeid;
    return {(const void *)tridiag_bisect_kernel_c<R, NB, NT, 16>, NT, slot_bytes_c<R, NB>(LDmax),
            (size_t)lds_bytes_c<NB, NT>(LDmax)};
}

KernelChoice choose_kernel(eeid_dtype_t t, eeid_prec_t p, int variant, int LDmax) {
    const bool d = (p == EEID_PREC_FP64);
    if (t == EEID_C128) return d ? complex_kernel<double, 16, 512>(LDmax) : complex_kernel<float, 16, 512>(LDmax);
    switch (variant) {
        case 1: return d ? real_kernel<double, 32, 256>(LDmax) : real_kernel<float, 32, 256>(LDmax);
        case 2: return d ? real_kernel<double, 16, 512>(LDmax) : real_kernel<float, 16, 512>(LDmax);
        case 3: return d ? band_kernel<double, 512>(LDmax) : band_kernel<float, 512>(LDmax);
        case 4: return d ? band_kernel<double, 256>(LDmax) : band_kernel<float, 256>(LDmax);
        default: return d ? real_kernel<double, 32, 512>(LDmax) : real_kernel<float, 32, 512>(LDmax);
    }
}

int pick_variant(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t nmax, int64_t problems) {
    if (h->forced_variant >= 0) return h->forced_variant;
    for (const auto &e : h->tune)
        if (e[0] == t && e[1] == p && e[2] == nmax && e[3] == problems) return (int)e[4];
    if (h->variant >= 0) return h->variant;
    // untuned default (measured on the n = 64 ... 2048 workloads): the two-stage
    // reduction, one problem per CU from n = 1024 on, two per CU below
    return (nmax >= 1024) ? 3 : 4;
}

// kind 0: eigenvalues of the matrices only; kind 1: matrices and all minors;
// kind 2: one matrix and a subset of minors; kind 3: one matrix, the minors
// at js[0] of its n - 1 rotated forms (partners k != js[0] ascending).
eeid_status_t prepare_eigs(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t count, const int64_t *n,
                           const int64_t *a_offset, const void *A, double *lambda, double *mu, int32_t *flags,
                           int kind, int64_t nsel, const int64_t *js, Enqueue *out, int *variant_used = nullptr) {
    using eeid::Item;
    HIP_TRY(h, hipSetDevice(h->device));
    eeid_status_t s = upload_desc(h, h->desc, h->desc_key, count, n, a_offset, -1);
    if (s != EEID_OK) return s;

    std::vector<Item> items;
    int64_t nmax = 0, lam = 0, muo = 0;
    const double *Ad = reinterpret_cast<const double *>(A);
    const int64_t esz = (t == EEID_C128) ? 2 : 1;  // doubles per element
    for (int64_t b = 0; b < count; ++b) {
        const int nb = (int)n[b];
        const double *src = Ad + esz * a_offset[b];
        nmax = std::max<int64_t>(nmax, nb);
        if (lambda) items.push_back(Item{src, lambda + lam, nb, -1, nb, (int32_t)b, -1, 0});
        if (kind == 1 && nb >= 2)
            for (int j = 0; j < nb; ++j)
                items.push_back(Item{src, mu + muo + (int64_t)j * (nb - 1), nb, j, nb - 1, (int32_t)b, -1, 0});
        if (kind == 2 && nb >= 2)
            for (int64_t q = 0; q < nsel; ++q)
                items.push_back(Item{src, mu + q * (nb - 1), nb, (int)js[q], nb - 1, (int32_t)b, -1, 0});
        // kind 3: minors at js[0] of the rotated matrices R^H A R, one per partner k != js[0]
        // (complex input: the real rotations, then the imaginary ones)
        if (kind == 3 && nb >= 2)
            for (int rot = 0, q = 0; rot < (t == EEID_C128 ? 2 : 1); ++rot)
                for (int k = 0; k < nb; ++k)
                    if (k != (int)js[0])
                        items.push_back(
                            Item{src, mu + (int64_t)(q++) * (nb - 1), nb, (int)js[0], nb - 1, (int32_t)b, k, rot});
        lam += nb;
        muo += (int64_t)nb * (nb - 1);
    }
    // largest problems first so that the tail of the queue is short
    std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.m > y.m; });
    std::vector<int64_t> ikey;
    ikey.reserve(5 * items.size() + 1);
    ikey.push_back((int64_t)items.size());
    for (const Item &it : items) {
        ikey.push_back((int64_t)(intptr_t)it.src);
        ikey.push_back((int64_t)(intptr_t)it.out);
        ikey.push_back(((int64_t)it.n << 32) | (uint32_t)it.j);
        ikey.push_back(((int64_t)it.m << 32) | (uint32_t)it.b);
        ikey.push_back(((int64_t)it.k << 32) | (uint32_t)it.rot);
    }
    s = upload_table(h, h->items, h->items_key, ikey, items);
    if (s != EEID_OK) return s;
    h->n_items = (int64_t)items.size();

    const int LDmax = (int)(((nmax + eeid::TILE - 1) / eeid::TILE) * eeid::TILE);
    const int variant = pick_variant(h, t, p, nmax, (int64_t)items.size());
    if (variant_used) *variant_used = variant;
    const KernelChoice kc = choose_kernel(t, p, variant, LDmax);
    HIP_TRY(h, hipFuncSetAttribute(kc.kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kc.lds));
    int per_cu = 0;
    HIP_TRY(h, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kc.kern, kc.nt, kc.lds));
    if (per_cu < 1) return fail(h, EEID_ERR_UNSUPPORTED, "eigenvalue kernel cannot be resident");
    int64_t slots = (int64_t)per_cu * h->cu_count;
    if (h->max_slots > 0) slots = std::min<int64_t>(slots, h->max_slots);
    slots = std::min<int64_t>(slots, std::max<int64_t>((int64_t)items.size(), 1));
    size_t free_b = 0, total_b = 0;
    HIP_TRY(h, hipMemGetInfo(&free_b, &total_b));
    const size_t budget = (size_t)((double)(free_b + h->work.bytes) * 0.85);
    slots = std::min<int64_t>(slots, (int64_t)(budget / (size_t)kc.slot));
    if (slots < 1) return fail(h, EEID_ERR_ALLOC, "not enough device memory for one problem slot");
    s = ensure(h, h->work, (size_t)(slots * kc.slot));
    if (s != EEID_OK) return s;

    s = ensure(h, h->lam_ready, sizeof(unsigned long long) * (size_t)count);
    if (s != EEID_OK) return s;
    unsigned long long *lam_ready = reinterpret_cast<unsigned long long *>(h->lam_ready.p);

    eeid::TriArgs a;
    a.lam_ready = lam_ready;
    a.items = reinterpret_cast<const Item *>(h->items.p);
    a.n_items = h->n_items;
    a.counter = h->counter;
    a.flags = flags;
    a.work = reinterpret_cast<char *>(h->work.p);
    a.slot_bytes = kc.slot;
    a.LDmax = LDmax;
    a.spin_limit = h->spin_limit;
    const eeid::BatchDesc *desc = reinterpret_cast<const eeid::BatchDesc *>(h->desc.p);
    const unsigned nn_blocks = (unsigned)((nmax * nmax + 4095) / 4096);
    const int cplx = (t == EEID_C128) ? 1 : 0;
    int *counter = h->counter;
    const bool any_items = !items.empty();
    *out = [=](hipStream_t st) -> hipError_t {
        hipLaunchKernelGGL(eeid::prep_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, flags, count,
                           (int *)nullptr, lam_ready);
        hipLaunchKernelGGL(eeid::nonfinite_kernel, dim3(nn_blocks, (unsigned)count), dim3(256), 0, st, desc, Ad,
                           cplx, flags);
        if (!any_items) return hipGetLastError();
        hipLaunchKernelGGL(eeid::reset_counter_kernel, dim3(1), dim3(64), 0, st, counter);
        eeid::TriArgs args = a;
        void *argv[] = {&args};
        hipError_t e = hipLaunchKernel(kc.kern, dim3((unsigned)slots), dim3((unsigned)kc.nt), argv, kc.lds, st);
        if (e != hipSuccess) return e;
        return hipGetLastError();
    };
    return EEID_OK;
}

// Eq. (2) for the columns described by the descriptors in desc_buf.
eeid_status_t prepare_identity(eeid_handle_t h, Buf &desc_buf, Buf &dpair_buf, int64_t count, int64_t nmax,
                               int64_t ncol_max, int64_t ntot, const double *lambda, const double *mu, double *V2,
                               int32_t *flags, Enqueue *out) {
    eeid_status_t s = ensure(h, dpair_buf, sizeof(double) * 2 * (size_t)std::max<int64_t>(ntot, 1));
    if (s != EEID_OK) return s;
    const eeid::BatchDesc *desc = reinterpret_cast<const eeid::BatchDesc *>(desc_buf.p);
    double *dpair = reinterpret_cast<double *>(dpair_buf.p);
    const unsigned ib = (unsigned)((nmax + 255) / 256);
    const unsigned jb = (unsigned)((ncol_max + eeid::ID_JT - 1) / eeid::ID_JT);
    const bool paired = (h->identity_form == EEID_IDENTITY_PAIRED);
    *out = [=](hipStream_t st) -> hipError_t {
        if (paired) {
            hipLaunchKernelGGL(eeid::identity_paired_kernel, dim3(ib, jb, (unsigned)count), dim3(256), 0, st, desc,
                               lambda, mu, V2, flags);
        } else {
            hipLaunchKernelGGL(eeid::denominators_kernel, dim3(ib, (unsigned)count), dim3(256), 0, st, desc, lambda,
                               dpair, flags);
            hipLaunchKernelGGL(eeid::identity_kernel, dim3(ib, jb, (unsigned)count), dim3(256), 0, st, desc, lambda,
                               mu, dpair, V2);
        }
        return hipGetLastError();
    };
    return EEID_OK;
}

eeid_status_t prepare_components(eeid_handle_t h, int64_t count, const int64_t *n, const double *lambda,
                                 const double *mu, double *V2, int32_t *flags, Enqueue *out) {
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
    // a_offset does not matter here: keep the cached descriptors when the orders match
    std::vector<int64_t> aoff(count, 0);
    if (h->desc_key.size() == (size_t)(2 * count + 2) && h->desc_key[0] == count && h->desc_key[1] == -1) {
        bool same = true;
        for (int64_t b = 0; b < count && same; ++b) same = h->desc_key[2 + 2 * b] == n[b];
        if (same)
            for (int64_t b = 0; b < count; ++b) aoff[b] = h->desc_key[3 + 2 * b];
    }
    eeid_status_t s = upload_desc(h, h->desc, h->desc_key, count, n, aoff.data(), -1);
    if (s != EEID_OK) return s;
    return prepare_identity(h, h->desc, h->dpair, count, nmax, nmax, ntot, lambda, mu, V2, flags, out);
}

eeid_status_t run_now(eeid_handle_t h, const Enqueue &e) {
    HIP_TRY(h, e(h->stream));
    return EEID_OK;
}

// Record (once per key, on the handle's private stream) and replay the
// enqueue steps as one hipGraph on the handle's stream.
// Up to GRAPH_CACHE recorded launches are kept per handle (a key names the
// entry point, its pointers and sizes, the kernel configuration and the
// generation of the handle's buffers), the least recently used replaced.
constexpr size_t GRAPH_CACHE = 8;
eeid_status_t run_graph(eeid_handle_t h, const std::vector<int64_t> &key, const std::vector<Enqueue> &steps) {
    if (!h->gstream) {
        HIP_TRY(h, hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
    }
    size_t at = h->graphs.size();
    for (size_t i = 0; i < h->graphs.size(); ++i)
        if (h->graphs[i].key == key) at = i;
    if (at < h->graphs.size()) {
        eeid_handle_s::Graph g = std::move(h->graphs[at]);
        h->graphs.erase(h->graphs.begin() + (std::ptrdiff_t)at);
        h->graphs.push_back(std::move(g));
    } else {
        if (h->graphs.size() >= GRAPH_CACHE) {
            HIP_TRY(h, hipStreamSynchronize(h->stream));   // its last replay has ended
            HIP_TRY(h, hipGraphExecDestroy(h->graphs.front().exec));
            h->graphs.erase(h->graphs.begin());
        }
        hipGraph_t g = nullptr;
        HIP_TRY(h, hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
        hipError_t err = hipSuccess;
        for (const Enqueue &e : steps)
            if (err == hipSuccess) err = e(h->gstream);
        hipError_t err2 = hipStreamEndCapture(h->gstream, &g);
        if (err != hipSuccess || err2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(h, EEID_ERR_HIP, std::string("graph capture failed: ") +
                                             hipGetErrorString(err != hipSuccess ? err : err2));
        }
        hipGraphExec_t exec = nullptr;
        hipError_t err3 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (err3 != hipSuccess)
            return fail(h, EEID_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(err3));
        h->graphs.push_back({key, exec});
    }
    // replayed on the handle's stream itself (ordered with the caller's work,
    // no cross-stream events); the private stream only records
    HIP_TRY(h, hipGraphLaunch(h->graphs.back().exec, h->stream));
    return EEID_OK;
}

void load_tune_table(eeid_handle_t h) {
    const char *path = getenv("EEID_TUNE_TABLE");
    if (!path || !*path) return;
    h->tune_path = path;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[256];
    while (fgets(line, sizeof line, f)) {
        long long a[5];
        if (line[0] == '#') continue;
        if (sscanf(line, "%lld %lld %lld %lld %lld", &a[0], &a[1], &a[2], &a[3], &a[4]) == 5 && a[4] >= 0 &&
            a[4] < N_REAL_VARIANTS) {
            bool replaced = false;  // later lines win
            for (auto &e : h->tune)
                if (e[0] == a[0] && e[1] == a[1] && e[2] == a[2] && e[3] == a[3]) { e[4] = a[4]; replaced = true; }
            if (!replaced) h->tune.push_back({a[0], a[1], a[2], a[3], a[4]});
        }
    }
    fclose(f);
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
    if (const char *e = getenv("EEID_VARIANT")) {
        const int v = atoi(e);
        if (v >= 0 && v < N_REAL_VARIANTS) h->forced_variant = v;
    }
    if (const char *e = getenv("EEID_MAX_SLOTS")) h->max_slots = atoll(e);
    if (const char *e = getenv("EEID_SPIN_LIMIT")) h->spin_limit = (unsigned)strtoul(e, nullptr, 10);
    load_tune_table(h);
    if (hipSetDevice(hip_device) != hipSuccess ||
        hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess ||
        hipMalloc(&h->counter, sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        return EEID_ERR_HIP;
    }
    // with this device current: the address of its copy of the scratch array
    if (hipGetSymbolAddress((void **)&h->scratch_ptr, HIP_SYMBOL(scratch)) != hipSuccess || !h->scratch_ptr) {
        (void)hipGetLastError();
        (void)hipFree(h->counter);
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
    if (h->gstream) (void)hipStreamSynchronize(h->gstream);
    for (const auto &g : h->graphs) (void)hipGraphExecDestroy(g.exec);
    if (h->gstream) (void)hipStreamDestroy(h->gstream);
    Buf *bufs[] = {&h->work,     &h->items,     &h->desc,    &h->desc_sub, &h->dpair, &h->dpair_sub,
                   &h->lam_ready, &h->sbuf, &h->lat_work, &h->lat_items, &h->lat_bar, &h->comp};
    for (Buf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (h->counter) (void)hipFree(h->counter);
    delete h;
    return EEID_OK;
}

eeid_status_t eeid_set_stream(eeid_handle_t h, void *stream) {
    if (!h) return EEID_ERR_INVALID_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (st != h->stream) {
        // work queued on the previous stream ends before the handle's buffers
        // (and recorded graphs) are used from the new one
        HIP_TRY(h, hipSetDevice(h->device));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    h->stream = st;
    return EEID_OK;
}

eeid_status_t eeid_set_graph_mode(eeid_handle_t h, int enable) {
    if (!h) return EEID_ERR_INVALID_ARG;
    h->graph_mode = (enable != 0);
    return EEID_OK;
}

eeid_status_t eeid_set_identity_form(eeid_handle_t h, int form) {
    if (!h) return EEID_ERR_INVALID_ARG;
    if (form != EEID_IDENTITY_PRODUCTS && form != EEID_IDENTITY_PAIRED)
        return fail(h, EEID_ERR_INVALID_ARG, "unknown identity form");
    h->identity_form = form;
    return EEID_OK;
}

eeid_status_t eeid_phase_ticks(unsigned long long *ticks, int reset) {
#ifdef EEID_PHASE_TIMERS
    if (reset) {
        const unsigned long long zero[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        return hipMemcpyToSymbol(HIP_SYMBOL(eeid::phase_ticks), zero, sizeof zero) == hipSuccess ? EEID_OK
                                                                                              : EEID_ERR_HIP;
    }
    if (!ticks) return EEID_ERR_INVALID_ARG;
    return hipMemcpyFromSymbol(ticks, HIP_SYMBOL(eeid::phase_ticks), 8 * sizeof(unsigned long long)) == hipSuccess
               ? EEID_OK
               : EEID_ERR_HIP;
#else
    (void)ticks;
    (void)reset;
    return EEID_ERR_UNSUPPORTED;
#endif
}

int eeid_variant_count(void) { return N_REAL_VARIANTS; }

eeid_status_t eeid_set_variant(eeid_handle_t h, int variant) {
    if (!h) return EEID_ERR_INVALID_ARG;
    if (variant < -1 || variant >= N_REAL_VARIANTS)
        return fail(h, EEID_ERR_INVALID_ARG, "variant out of range");
    h->forced_variant = variant;
    return EEID_OK;
}

const char *eeid_status_string(eeid_status_t s) {
    switch (s) {
        case EEID_OK: return "EEID_OK: success";
        case EEID_ERR_INVALID_ARG: return "EEID_ERR_INVALID_ARG: invalid argument";
        case EEID_ERR_NO_DEVICE: return "EEID_ERR_NO_DEVICE: no usable HIP device";
        case EEID_ERR_ALLOC: return "EEID_ERR_ALLOC: device allocation failed";
        case EEID_ERR_HIP: return "EEID_ERR_HIP: HIP runtime error";
        case EEID_ERR_UNSUPPORTED: return "EEID_ERR_UNSUPPORTED: request not supported by this library";
    }
    return "unknown eeid status";
}

const char *eeid_last_error(eeid_handle_t h) { return h ? h->err.c_str() : ""; }

eeid_status_t eeid_eigvalsh_batched(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t count,
                                    const int64_t *n, const int64_t *a_offset, const void *A, double *lambda,
                                    int32_t *flags) {
    eeid_status_t s = check_batch(h, t, p, count, n, a_offset, A);
    if (s != EEID_OK) return s;
    if (!lambda || !flags) return fail(h, EEID_ERR_INVALID_ARG, "null output pointer");
    Enqueue e;
    s = prepare_eigs(h, t, p, count, n, a_offset, A, lambda, nullptr, flags, 0, 0, nullptr, &e);
    return s != EEID_OK ? s : run_now(h, e);
}

eeid_status_t eeid_minor_eigvals(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t count,
                                 const int64_t *n, const int64_t *a_offset, const void *A, double *lambda,
                                 double *mu, int32_t *flags) {
    eeid_status_t s = check_batch(h, t, p, count, n, a_offset, A);
    if (s != EEID_OK) return s;
    if (!lambda || !flags) return fail(h, EEID_ERR_INVALID_ARG, "null output pointer");
    bool need_mu = false;
    for (int64_t b = 0; b < count; ++b) need_mu = need_mu || n[b] >= 2;
    if (need_mu && !mu) return fail(h, EEID_ERR_INVALID_ARG, "mu is null");
    Enqueue e;
    int variant = 0;
    s = prepare_eigs(h, t, p, count, n, a_offset, A, lambda, mu, flags, 1, 0, nullptr, &e, &variant);
    if (s != EEID_OK) return s;
    if (!h->graph_mode) return run_now(h, e);
    std::vector<int64_t> key = {1, (int64_t)t, (int64_t)p, count, (int64_t)(intptr_t)A, (int64_t)(intptr_t)lambda,
                                (int64_t)(intptr_t)mu, (int64_t)(intptr_t)flags, (int64_t)h->generation,
                                (int64_t)variant};
    for (int64_t b = 0; b < count; ++b) { key.push_back(n[b]); key.push_back(a_offset[b]); }
    return run_graph(h, key, {e});
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
    Enqueue e;
    s = prepare_eigs(h, t, p, 1, &n, &zero, A, lambda, mu_sel, flag, 2, nsel, js, &e);
    return s != EEID_OK ? s : run_now(h, e);
}

eeid_status_t eeid_minor_eigvals_latency(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t n,
                                         const void *A, int64_t nsel, const int64_t *js, double *lambda,
                                         double *mu_sel, int32_t *flag) {
    const int64_t zero = 0;
    eeid_status_t s = check_batch(h, t, p, 1, &n, &zero, A);
    if (s != EEID_OK) return s;
    if (t != EEID_R64 || p != EEID_PREC_FP64)
        return fail(h, EEID_ERR_UNSUPPORTED, "latency path: real symmetric input in the FP64 form only");
    if (nsel < 0 || (nsel > 0 && !js)) return fail(h, EEID_ERR_INVALID_ARG, "nsel must be >= 0 and js non-null");
    if (!flag) return fail(h, EEID_ERR_INVALID_ARG, "null flag pointer");
    if (nsel > 0 && n >= 2 && !mu_sel) return fail(h, EEID_ERR_INVALID_ARG, "mu_sel is null");
    for (int64_t q = 0; q < nsel; ++q)
        if (js[q] < 0 || js[q] >= n) return fail(h, EEID_ERR_INVALID_ARG, "js entry out of range");
    std::vector<eeid::Item> items;
    const double *src = reinterpret_cast<const double *>(A);
    if (lambda) items.push_back(eeid::Item{src, lambda, (int32_t)n, -1, (int32_t)n, 0, -1, 0});
    if (n >= 2)
        for (int64_t q = 0; q < nsel; ++q)
            items.push_back(eeid::Item{src, mu_sel + q * (n - 1), (int32_t)n, (int32_t)js[q], (int32_t)(n - 1), 0, -1, 0});
    if ((int64_t)items.size() > eeid::LAT_MAX_PROBLEMS)
        return fail(h, EEID_ERR_UNSUPPORTED, "latency path: at most " + std::to_string(eeid::LAT_MAX_PROBLEMS) +
                                                 " problems per call");
    HIP_TRY(h, hipSetDevice(h->device));
    s = upload_desc(h, h->desc_sub, h->desc_sub_key, 1, &n, &zero, 1);
    if (s != EEID_OK) return s;
    const eeid::BatchDesc *desc = reinterpret_cast<const eeid::BatchDesc *>(h->desc_sub.p);
    const int P = (int)items.size();
    int coop = 0;
    HIP_TRY(h, hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, h->device));
    if (!coop) return fail(h, EEID_ERR_UNSUPPORTED, "device does not support cooperative launches");
    const int LD = (int)((n + 7) / 8 * 8);
    const size_t lds = (size_t)eeid::lat_lds_bytes(LD);
    const void *kern = (const void *)eeid::latency_eig_kernel;
    HIP_TRY(h, hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    HIP_TRY(h, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, eeid::LAT_NT, lds));
    if (per_cu < 1) return fail(h, EEID_ERR_UNSUPPORTED, "latency kernel cannot be resident");
    // one workgroup per CU, split evenly over the problems, but at least 16
    // rows per workgroup: below that a grid barrier's arrivals cost more than
    // the rows' work (n = 502: 7.7 ms with 64 workgroups per problem, 10.3 ms
    // with 128; from n = 2002 on, every CU pays)
    const int G = std::max(1, std::min(h->cu_count / std::max(P, 1), (int)((n + 15) / 16)));
    const int64_t pb = eeid::lat_prob_bytes(LD, G);
    if (P > 0) {
        s = ensure(h, h->lat_work, (size_t)(pb * P));
        if (s != EEID_OK) return s;
        s = ensure(h, h->lat_bar, sizeof(unsigned) * eeid::LAT_MAX_PROBLEMS);
        if (s != EEID_OK) return s;
        s = ensure(h, h->lat_items, sizeof(eeid::Item) * eeid::LAT_MAX_PROBLEMS);
        if (s != EEID_OK) return s;
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        HIP_TRY(h, hipMemcpy(h->lat_items.p, items.data(), sizeof(eeid::Item) * P, hipMemcpyHostToDevice));
    }
    hipStream_t st = h->stream;
    unsigned *bar = reinterpret_cast<unsigned *>(h->lat_bar.p);
    hipLaunchKernelGGL(eeid::prep_kernel, dim3(1), dim3(256), 0, st, flag, (int64_t)1, (int *)nullptr,
                       (unsigned long long *)nullptr);
    hipLaunchKernelGGL(eeid::nonfinite_kernel, dim3((unsigned)((n * n + 4095) / 4096), 1u), dim3(256), 0, st, desc,
                       src, 0, flag);
    if (P == 0) {
        HIP_TRY(h, hipGetLastError());
        return EEID_OK;
    }
    hipLaunchKernelGGL(eeid::reset_barriers_kernel, dim3(1), dim3(64), 0, st, bar, P);
    eeid::LatArgs a;
    a.items = reinterpret_cast<const eeid::Item *>(h->lat_items.p);
    a.P = P;
    a.G = G;
    a.work = reinterpret_cast<char *>(h->lat_work.p);
    a.prob_bytes = pb;
    a.LD = LD;
    a.bar = bar;
    a.flags = flag;
    a.spin_limit = h->spin_limit >> 6;   // a grid barrier's poll is a device-scope load (~64 times an LDS poll)
    void *argv[] = {&a};
    HIP_TRY(h, hipLaunchCooperativeKernel(kern, dim3((unsigned)(P * G)), dim3(eeid::LAT_NT), argv, (unsigned)lds, st));
    HIP_TRY(h, hipGetLastError());
    return EEID_OK;
}

eeid_status_t eeid_components(eeid_handle_t h, int64_t count, const int64_t *n, const double *lambda,
                              const double *mu, double *V2, int32_t *flags) {
    if (!h) return EEID_ERR_INVALID_ARG;
    Enqueue e;
    eeid_status_t s = prepare_components(h, count, n, lambda, mu, V2, flags, &e);
    if (s != EEID_OK) return s;
    if (!h->graph_mode) return run_now(h, e);
    std::vector<int64_t> key = {2, count, (int64_t)(intptr_t)lambda, (int64_t)(intptr_t)mu, (int64_t)(intptr_t)V2,
                                (int64_t)(intptr_t)flags, (int64_t)h->generation, (int64_t)h->identity_form};
    for (int64_t b = 0; b < count; ++b) key.push_back(n[b]);
    return run_graph(h, key, {e});
}

eeid_status_t eeid_components_noalloc(eeid_handle_t h, int64_t count, const int64_t *n, const double *lambda,
                                      const double *mu, double *V2, int32_t *flags) {
    if (!h) return EEID_ERR_INVALID_ARG;
    if (count < 1) return fail(h, EEID_ERR_INVALID_ARG, "count must be >= 1");
    if (!n || !lambda || !V2 || !flags) return fail(h, EEID_ERR_INVALID_ARG, "null pointer argument");
    if (count > eeid::NLIST_MAX)
        return fail(h, EEID_ERR_UNSUPPORTED, "eeid_components_noalloc: count " + std::to_string(count) +
                                                 " exceeds EEID_NOALLOC_MAX_MATRICES (" +
                                                 std::to_string(eeid::NLIST_MAX) + ")");
    eeid::NList nl;
    nl.count = (int32_t)count;
    int64_t nmax = 0, ntot = 0;
    bool need_mu = false;
    for (int64_t b = 0; b < count; ++b) {
        if (n[b] < 1) return fail(h, EEID_ERR_INVALID_ARG, "n[" + std::to_string(b) + "] must be >= 1");
        if (n[b] > EEID_MAX_N_R64) return fail(h, EEID_ERR_UNSUPPORTED, "n exceeds the supported maximum");
        nl.n[b] = (int32_t)n[b];
        nmax = std::max(nmax, n[b]);
        ntot += n[b];
        need_mu = need_mu || n[b] >= 2;
    }
    if (ntot > NOALLOC_MAX_EIGENVALUES)
        return fail(h, EEID_ERR_UNSUPPORTED, "eeid_components_noalloc: sum of n is " + std::to_string(ntot) +
                                                 ", above EEID_NOALLOC_MAX_EIGENVALUES (" +
                                                 std::to_string(NOALLOC_MAX_EIGENVALUES) + ")");
    if (need_mu && !mu) return fail(h, EEID_ERR_INVALID_ARG, "mu is null");
    HIP_TRY(h, hipSetDevice(h->device));
    eeid::BatchDesc *desc = reinterpret_cast<eeid::BatchDesc *>(h->scratch_ptr);
    double *dpair = reinterpret_cast<double *>(h->scratch_ptr + NOALLOC_DESC_BYTES);
    const unsigned ib = (unsigned)((nmax + 255) / 256);
    const unsigned jb = (unsigned)((nmax + eeid::ID_JT - 1) / eeid::ID_JT);
    hipStream_t st = h->stream;
    // every scratch byte the later kernels read is written first (descriptors,
    // then every denominator pair), so nothing needs clearing
    hipLaunchKernelGGL(eeid::write_desc_kernel, dim3(1), dim3(64), 0, st, nl, desc);
    if (h->identity_form == EEID_IDENTITY_PAIRED) {
        hipLaunchKernelGGL(eeid::identity_paired_kernel, dim3(ib, jb, (unsigned)count), dim3(256), 0, st, desc,
                           lambda, mu, V2, flags);
    } else {
        hipLaunchKernelGGL(eeid::denominators_kernel, dim3(ib, (unsigned)count), dim3(256), 0, st, desc, lambda,
                           dpair, flags);
        hipLaunchKernelGGL(eeid::identity_kernel, dim3(ib, jb, (unsigned)count), dim3(256), 0, st, desc, lambda, mu,
                           dpair, V2);
    }
    HIP_TRY(h, hipGetLastError());
    return EEID_OK;
}

eeid_status_t eeid_components_subset(eeid_handle_t h, int64_t n, const double *lambda, int64_t nsel,
                                     const double *mu_sel, double *V2_sel, int32_t *flag) {
    if (!h) return EEID_ERR_INVALID_ARG;
    if (n < 1 || n > EEID_MAX_N_R64) return fail(h, EEID_ERR_INVALID_ARG, "n out of range");
    if (nsel < 1) return fail(h, EEID_ERR_INVALID_ARG, "nsel must be >= 1");
    if (!lambda || !V2_sel || !flag || (n >= 2 && !mu_sel))
        return fail(h, EEID_ERR_INVALID_ARG, "null pointer argument");
    HIP_TRY(h, hipSetDevice(h->device));
    const int64_t zero = 0;
    eeid_status_t s = upload_desc(h, h->desc_sub, h->desc_sub_key, 1, &n, &zero, nsel);
    if (s != EEID_OK) return s;
    Enqueue e;
    s = prepare_identity(h, h->desc_sub, h->dpair_sub, 1, n, nsel, n, lambda, mu_sel, V2_sel, flag, &e);
    return s != EEID_OK ? s : run_now(h, e);
}

eeid_status_t eeid_eigenvector_sq(eeid_handle_t h, int64_t n, const double *lambda, const double *mu, int64_t i,
                                  double *row, int32_t *flag) {
    if (!h) return EEID_ERR_INVALID_ARG;
    if (n < 1 || n > EEID_MAX_N_R64) return fail(h, EEID_ERR_INVALID_ARG, "n out of range");
    if (i < 0 || i >= n) return fail(h, EEID_ERR_INVALID_ARG, "eigenvalue index i out of range");
    if (!lambda || !row || !flag || (n >= 2 && !mu)) return fail(h, EEID_ERR_INVALID_ARG, "null pointer argument");
    HIP_TRY(h, hipSetDevice(h->device));
    const dim3 grid((unsigned)((n + 255) / 256));
    if (h->identity_form == EEID_IDENTITY_PAIRED)
        hipLaunchKernelGGL(eeid::eigenvector_row_kernel<true>, grid, dim3(256), 0, h->stream, (int)n, (int)i, lambda,
                           mu, row, flag);
    else
        hipLaunchKernelGGL(eeid::eigenvector_row_kernel<false>, grid, dim3(256), 0, h->stream, (int)n, (int)i, lambda,
                           mu, row, flag);
    HIP_TRY(h, hipGetLastError());
    return EEID_OK;
}

eeid_status_t eeid_component(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t n, const void *A, int64_t i,
                             int64_t j, double *out, int32_t *flag) {
    if (!h) return EEID_ERR_INVALID_ARG;
    if (n < 1) return fail(h, EEID_ERR_INVALID_ARG, "n must be >= 1");
    if (i < 0 || i >= n || j < 0 || j >= n) return fail(h, EEID_ERR_INVALID_ARG, "index i or j out of range");
    if (!A || !out || !flag) return fail(h, EEID_ERR_INVALID_ARG, "null pointer argument");
    HIP_TRY(h, hipSetDevice(h->device));
    // lambda [n], mu [n - 1] (at least one slot), the column [n]
    eeid_status_t s = ensure(h, h->comp, sizeof(double) * (size_t)(3 * n));
    if (s != EEID_OK) return s;
    double *lam = reinterpret_cast<double *>(h->comp.p), *mu = lam + n, *col = mu + n;
    s = eeid_minor_eigvals_latency(h, t, p, n, A, 1, &j, lam, mu, flag);
    if (s != EEID_OK) return s;
    s = eeid_components_subset(h, n, lam, 1, mu, col, flag);
    if (s != EEID_OK) return s;
    HIP_TRY(h, hipMemcpyAsync(out, col + i, sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    return EEID_OK;
}

eeid_status_t eeid_rotated_minor_eigvals(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t n,
                                         const void *A, int64_t r, double *mu_rot, int32_t *flag) {
    const int64_t zero = 0;
    eeid_status_t s = check_batch(h, t, p, 1, &n, &zero, A);
    if (s != EEID_OK) return s;
    if (r < 0 || r >= n) return fail(h, EEID_ERR_INVALID_ARG, "reference index r out of range");
    if (!flag) return fail(h, EEID_ERR_INVALID_ARG, "null flag pointer");
    if (n >= 2 && !mu_rot) return fail(h, EEID_ERR_INVALID_ARG, "mu_rot is null");
    Enqueue e;
    s = prepare_eigs(h, t, p, 1, &n, &zero, A, nullptr, mu_rot, flag, 3, 1, &r, &e);
    return s != EEID_OK ? s : run_now(h, e);
}

eeid_status_t eeid_signed_eigenvectors(eeid_handle_t h, eeid_dtype_t t, int64_t n, int64_t r, const double *lambda,
                                       const double *W, const double *mu_rot, double *V, int32_t *flag) {
    if (!h) return EEID_ERR_INVALID_ARG;
    if (t != EEID_R64 && t != EEID_C128) return fail(h, EEID_ERR_INVALID_ARG, "unknown dtype");
    if (n < 1 || n > (t == EEID_R64 ? EEID_MAX_N_R64 : EEID_MAX_N_C128))
        return fail(h, EEID_ERR_INVALID_ARG, "n out of range");
    const int64_t fam = (t == EEID_C128) ? 2 : 1;   // rotated families: real, and imaginary for complex input
    if (r < 0 || r >= n) return fail(h, EEID_ERR_INVALID_ARG, "reference index r out of range");
    if (!lambda || !W || !V || !flag || (n >= 2 && !mu_rot))
        return fail(h, EEID_ERR_INVALID_ARG, "null pointer argument");
    HIP_TRY(h, hipSetDevice(h->device));
    double *S = nullptr;
    Enqueue e;
    if (n >= 2) {
        const int64_t zero = 0;
        eeid_status_t s = upload_desc(h, h->desc_sub, h->desc_sub_key, 1, &n, &zero, fam * (n - 1));
        if (s != EEID_OK) return s;
        s = ensure(h, h->sbuf, sizeof(double) * (size_t)(n * fam * (n - 1)));
        if (s != EEID_OK) return s;
        S = reinterpret_cast<double *>(h->sbuf.p);
        s = prepare_identity(h, h->desc_sub, h->dpair_sub, 1, n, fam * (n - 1), n, lambda, mu_rot, S, flag, &e);
        if (s != EEID_OK) return s;
        s = run_now(h, e);
        if (s != EEID_OK) return s;
    }
    if (fam == 2)
        hipLaunchKernelGGL(eeid::signed_vectors_kernel<true>, dim3((unsigned)((n + 255) / 256), (unsigned)n),
                           dim3(256), 0, h->stream, (int)n, (int)r, W, S, V, flag);
    else
        hipLaunchKernelGGL(eeid::signed_vectors_kernel<false>, dim3((unsigned)((n + 255) / 256), (unsigned)n),
                           dim3(256), 0, h->stream, (int)n, (int)r, W, S, V, flag);
    HIP_TRY(h, hipGetLastError());
    return EEID_OK;
}

eeid_status_t eeid_all_components(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t count,
                                  const int64_t *n, const int64_t *a_offset, const void *A, double *lambda,
                                  double *mu, double *V2, int32_t *flags) {
    eeid_status_t s = check_batch(h, t, p, count, n, a_offset, A);
    if (s != EEID_OK) return s;
    if (!lambda || !flags || !V2) return fail(h, EEID_ERR_INVALID_ARG, "null output pointer");
    bool need_mu = false;
    for (int64_t b = 0; b < count; ++b) need_mu = need_mu || n[b] >= 2;
    if (need_mu && !mu) return fail(h, EEID_ERR_INVALID_ARG, "mu is null");
    Enqueue e1, e2;
    int variant = 0;
    s = prepare_eigs(h, t, p, count, n, a_offset, A, lambda, mu, flags, 1, 0, nullptr, &e1, &variant);
    if (s != EEID_OK) return s;
    s = prepare_components(h, count, n, lambda, mu, V2, flags, &e2);
    if (s != EEID_OK) return s;
    if (!h->graph_mode) {
        s = run_now(h, e1);
        return s != EEID_OK ? s : run_now(h, e2);
    }
    std::vector<int64_t> key = {3, (int64_t)t, (int64_t)p, count, (int64_t)(intptr_t)A, (int64_t)(intptr_t)lambda,
                                (int64_t)(intptr_t)mu, (int64_t)(intptr_t)V2, (int64_t)(intptr_t)flags,
                                (int64_t)h->generation, (int64_t)variant, (int64_t)h->identity_form};
    for (int64_t b = 0; b < count; ++b) { key.push_back(n[b]); key.push_back(a_offset[b]); }
    return run_graph(h, key, {e1, e2});
}

eeid_status_t eeid_autotune(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t count, const int64_t *n,
                            const int64_t *a_offset, const void *A, double *lambda, double *mu, int32_t *flags,
                            int *best_variant, double *best_ms) {
    eeid_status_t s = check_batch(h, t, p, count, n, a_offset, A);
    if (s != EEID_OK) return s;
    if (!lambda || !flags) return fail(h, EEID_ERR_INVALID_ARG, "null output pointer");
    bool need_mu = false;
    for (int64_t b = 0; b < count; ++b) need_mu = need_mu || n[b] >= 2;
    if (need_mu && !mu) return fail(h, EEID_ERR_INVALID_ARG, "mu is null");
    HIP_TRY(h, hipSetDevice(h->device));
    int64_t nmax = 0, problems = 0;
    for (int64_t b = 0; b < count; ++b) {
        nmax = std::max(nmax, n[b]);
        problems += 1 + (n[b] >= 2 ? n[b] : 0);
    }
    const int nvar = (t == EEID_C128) ? 1 : N_REAL_VARIANTS;
    hipEvent_t e0, e1;
    HIP_TRY(h, hipEventCreate(&e0));
    HIP_TRY(h, hipEventCreate(&e1));
    const int saved = h->forced_variant;
    int best = -1;
    float best_t = 0.f;
    for (int v = 0; v < nvar; ++v) {
        h->forced_variant = v;
        Enqueue e;
        s = prepare_eigs(h, t, p, count, n, a_offset, A, lambda, mu, flags, 1, 0, nullptr, &e);
        if (s != EEID_OK) break;
        if (hipEventRecord(e0, h->stream) != hipSuccess || e(h->stream) != hipSuccess ||
            hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            s = fail(h, EEID_ERR_HIP, "autotune launch failed");
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (best < 0 || ms < best_t) { best = v; best_t = ms; }
    }
    h->forced_variant = saved;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != EEID_OK) return s;
    const std::array<int64_t, 5> entry = {(int64_t)t, (int64_t)p, nmax, problems, (int64_t)best};
    bool replaced = false;
    for (auto &e : h->tune)
        if (e[0] == entry[0] && e[1] == entry[1] && e[2] == entry[2] && e[3] == entry[3]) { e = entry; replaced = true; }
    if (!replaced) h->tune.push_back(entry);
    if (!h->tune_path.empty()) {
        if (FILE *f = fopen(h->tune_path.c_str(), "a")) {
            fprintf(f, "%lld %lld %lld %lld %d  # %s %.3f ms\n", (long long)t, (long long)p, (long long)nmax,
                    (long long)problems, best, t == EEID_C128 ? "complex" : VARIANT_NAME[best], best_t);
            fclose(f);
        }
    }
    if (best_variant) *best_variant = best;
    if (best_ms) *best_ms = best_t;
    return EEID_OK;
}

}  // extern "C"
