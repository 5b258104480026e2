// The eigenvector-eigenvalue identity (Section 2, Eq. (2) of the paper) for
// every (i, j) of a batch, from the ascending spectra of A and of its minors:
//
//   |v_ij|^2 = prod_k |lambda_i - mu_jk| / prod_{k != i} |lambda_i - lambda_k|
//
// in FP64.  Raw products over- and underflow for n of a few hundred (the paper
// batches them for that reason, Section 3); here each product is carried as a
// mantissa and a separate integer exponent.  Every factor is split by frexp
// into a mantissa in [1/2, 1) and its exponent before it is multiplied in, so
// a factor may be as small as the smallest subnormal or as large as the
// largest double without any intermediate leaving the normal range; the
// running mantissa (at least 2^-8 after eight factors) is renormalised after
// every eighth factor.  The eigenvalues are used unscaled unless the largest
// |lambda| reaches 2^1021, where a difference could overflow: then all of
// them are scaled by the same power of two (exact; numerator and denominator
// have n - 1 factors each, so the scale cancels).  The rounding error is that
// of the n - 1 multiplications (relative, at most about n eps).  An exactly
// zero numerator factor gives 0; an exactly repeated lambda_i leaves the ratio
// undefined, so row i is NaN and the matrix is flagged degenerate.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eeid {

struct BatchDesc {
    int64_t a_off;    // element offset of the matrix in A
    int64_t lam_off;  // offset of its n eigenvalues in lambda
    int64_t mu_off;   // offset of its ncol (n - 1) minor eigenvalues in mu
    int64_t v2_off;   // offset of its n * ncol components in V2 (row i: ncol values)
    int32_t n;
    int32_t ncol;     // minors (columns) given: n for all of them, fewer for a subset
};

__global__ __launch_bounds__(256) void prep_kernel(int32_t *flags, int64_t count, int *counter,
                                                   unsigned long long *lam_ready) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) {
        flags[i] = 0;
        if (lam_ready) lam_ready[i] = 0;
    }
    if (i == 0 && counter) *counter = 0;
}

__global__ __launch_bounds__(64) void reset_counter_kernel(int *counter) {
    if (threadIdx.x == 0) *counter = 0;
}

// flags[b] |= 1 when the lower triangle of matrix b holds a NaN or an Inf.
__global__ __launch_bounds__(256) void nonfinite_kernel(const BatchDesc *desc, const double *A,
                                                         int cplx, int32_t *flags) {
    const int b = blockIdx.y;
    const int64_t n = desc[b].n;
    const int64_t nn = n * n;
    const int64_t base = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
    bool bad = false;
    if (base < nn) {
        const double *a = A + desc[b].a_off * (cplx ? 2 : 1);
        for (int t = 0; t < 16; ++t) {
            const int64_t e = base + t;
            if (e >= nn) break;
            const int64_t r = e / n, c = e % n;
            if (c > r) continue;
            if (cplx) {
                const double re = a[2 * e], im = a[2 * e + 1];
                if (!isfinite(re) || (c != r && !isfinite(im))) bad = true;
            } else if (!isfinite(a[e])) {
                bad = true;
            }
        }
    }
    if (__any(bad) && (threadIdx.x & 63) == __ffsll((unsigned long long)__ballot(bad)) - 1)
        atomicOr(&flags[b], 1);
}

// Power of two by which the eigenvalues of an ascending spectrum are divided
// before differences are taken: 0 unless the largest |lambda| is at least
// 2^1021, so that every difference stays finite.
__device__ __forceinline__ int spectrum_exponent(const double *lam, int n) {
    const double big = fmax(fabs(lam[0]), fabs(lam[n - 1]));
    const int e = (big > 0.0) ? ilogb(big) : 0;
    return (e >= 1021) ? e - 1020 : 0;
}

// Running product of factors as (mantissa, exponent): each factor's own
// mantissa and exponent are taken apart first, so no intermediate leaves the
// normal range; the mantissa is renormalised by the caller every RENORM
// factors.  A zero factor leaves the mantissa 0 for good.
constexpr int RENORM = 8;
__device__ __forceinline__ void mul_factor(double &pm, int &pe, double f) {
    int e;
    pm *= frexp(f, &e);
    pe += e;
}
__device__ __forceinline__ void renormalise(double &pm, int &pe) {
    int e;
    pm = frexp(pm, &e);
    pe += e;
}

// Denominator of Eq. (2) for each i: prod_{k != i} |lambda_i - lambda_k| 2^-(n-1)E
// as (mantissa, exponent) in Dpair[2 i], Dpair[2 i + 1].
__global__ __launch_bounds__(256) void denominators_kernel(const BatchDesc *desc, const double *lambda,
                                                            double *Dpair, int32_t *flags) {
    const int b = blockIdx.y;
    const int n = desc[b].n;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double *lam = lambda + desc[b].lam_off;
    const int E = spectrum_exponent(lam, n);
    const double li = ldexp(lam[i], -E);
    double q = 1.0;
    int qe = 0, cnt = 0;
    bool zero = false;
    for (int k = 0; k < n; ++k) {
        if (k == i) continue;
        const double d = li - ldexp(lam[k], -E);
        if (d == 0.0) zero = true;
        mul_factor(q, qe, fabs(d));
        if (++cnt == RENORM) { renormalise(q, qe); cnt = 0; }
    }
    renormalise(q, qe);
    double *out = Dpair + 2 * (desc[b].lam_off + i);
    if (zero) {
        out[0] = __builtin_nan("");
        out[1] = 0.0;
        atomicOr(&flags[b], 2);
    } else {
        out[0] = q;
        out[1] = (double)qe;
    }
}

// Descriptors of up to NLIST_MAX matrices written on the device from their
// orders (passed by value), for callers that cannot upload a table.
constexpr int NLIST_MAX = 64;
struct NList {
    int32_t count;
    int32_t n[NLIST_MAX];
};
__global__ __launch_bounds__(64) void write_desc_kernel(NList nl, BatchDesc *desc) {
    if (threadIdx.x != 0) return;
    int64_t lam = 0, mu = 0, v2 = 0;
    for (int b = 0; b < nl.count; ++b) {
        const int64_t n = nl.n[b];
        desc[b].a_off = 0;
        desc[b].lam_off = lam;
        desc[b].mu_off = mu;
        desc[b].v2_off = v2;
        desc[b].n = (int32_t)n;
        desc[b].ncol = (int32_t)n;
        lam += n;
        mu += n * (n - 1);
        v2 += n * n;
    }
}

constexpr int ID_JT = 8;    // minors (columns j) per thread
constexpr int ID_KC = 256;  // minor eigenvalues staged per LDS chunk

// V2[v2_off + i*ncol + j] for i in a 256-block (blockIdx.x) and j in an ID_JT-block (blockIdx.y):
// column j is the minor whose spectrum is row j of mu (all minors: ncol = n).
__global__ __launch_bounds__(256) void identity_kernel(const BatchDesc *desc, const double *lambda,
                                                        const double *mu, const double *Dpair, double *V2) {
    __shared__ double sm[ID_JT][ID_KC];
    const int b = blockIdx.z;
    const int n = desc[b].n;
    const int ncol = desc[b].ncol;
    const int j0 = blockIdx.y * ID_JT;
    if (j0 >= ncol || (int)blockIdx.x * 256 >= n) return;
    const int m = n - 1;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const bool live = i < n;
    const double *lam = lambda + desc[b].lam_off;
    const int E = spectrum_exponent(lam, n);
    const double li = live ? ldexp(lam[i], -E) : 0.0;
    const double *mub = mu + desc[b].mu_off;
    double pm[ID_JT];
    int pe[ID_JT];
#pragma unroll
    for (int t = 0; t < ID_JT; ++t) { pm[t] = 1.0; pe[t] = 0; }
    for (int kc = 0; kc < m; kc += ID_KC) {
        const int kn = min(ID_KC, m - kc);
        __syncthreads();
        // staged scaled by 2^-E
        for (int q = threadIdx.x; q < ID_JT * ID_KC; q += 256) {
            const int jj = q / ID_KC, kk = q % ID_KC;
            const int j = j0 + jj;
            sm[jj][kk] = (j < ncol && kk < kn) ? ldexp(mub[(int64_t)j * m + kc + kk], -E) : 0.0;
        }
        __syncthreads();
        int kk = 0;
        for (; kk + RENORM <= kn; kk += RENORM) {
#pragma unroll
            for (int t = 0; t < ID_JT; ++t) {
#pragma unroll
                for (int u = 0; u < RENORM; ++u) mul_factor(pm[t], pe[t], fabs(li - sm[t][kk + u]));
                renormalise(pm[t], pe[t]);
            }
        }
        for (; kk < kn; ++kk) {
#pragma unroll
            for (int t = 0; t < ID_JT; ++t) mul_factor(pm[t], pe[t], fabs(li - sm[t][kk]));
        }
#pragma unroll
        for (int t = 0; t < ID_JT; ++t) renormalise(pm[t], pe[t]);
    }
    if (!live) return;
    const double *dp = Dpair + 2 * (desc[b].lam_off + i);
    const double qm = dp[0];
    const int qe = (int)dp[1];
    double *out = V2 + desc[b].v2_off + (int64_t)i * ncol;
#pragma unroll
    for (int t = 0; t < ID_JT; ++t) {
        const int j = j0 + t;
        if (j >= ncol) break;
        // a zero numerator factor left pm = 0 (frexp keeps 0); a NaN denominator stays NaN
        out[j] = ldexp(pm[t] / qm, pe[t] - qe);
    }
}

// Signed (or phased) eigenvectors from Eq. (2) in the original basis and in
// rotated bases of the (r, k) planes (Section 2: the identity applied in other
// bases gives the directions).  W_ik = |v_ik|^2 (row-major, n x n); S holds,
// per row i, the identity at r of the rotated matrices: column q (the q-th
// partner k != r, ascending) = (W_ir + W_ik)/2 + Re(conj(v_ir) v_ik), and for
// complex input column n - 1 + q = (W_ir + W_ik)/2 + Im(conj(v_ir) v_ik).
// With the convention v_ir real >= 0:
//   V[i, r] = sqrt(W_ir),  V[i, k] = conj(v_ir) v_ik / sqrt(W_ir),
// real (CPLX false) or interleaved (re, im) (CPLX true).  A row with W_ir = 0
// has no reference: it is NaN and flag bit 8 is set.
template <bool CPLX>
__global__ __launch_bounds__(256) void signed_vectors_kernel(int n, int r, const double *W, const double *S,
                                                              double *V, int32_t *flag) {
    const int i = blockIdx.y;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const int fam = CPLX ? 2 : 1;
    const double wr = W[(int64_t)i * n + r];
    const double sr = sqrt(wr);
    double re, im = 0.0;
    if (!(wr > 0.0)) {
        re = im = __builtin_nan("");
        if (k == 0) atomicOr(flag, 8);
    } else if (k == r) {
        re = sr;
    } else {
        const int q = k - (k > r ? 1 : 0);
        const double half = 0.5 * (wr + W[(int64_t)i * n + k]);
        const double *Si = S + (int64_t)i * fam * (n - 1);
        re = (Si[q] - half) / sr;
        if (CPLX) im = (Si[n - 1 + q] - half) / sr;
    }
    if (CPLX) {
        V[2 * ((int64_t)i * n + k)] = re;
        V[2 * ((int64_t)i * n + k) + 1] = im;
    } else {
        V[(int64_t)i * n + k] = re;
    }
}

// Eq. (2) in the paired form of Algorithm 2 (Section 3): with lambda_i taken
// out, the remaining eigenvalues lambda'_k (k = 1..n-1, ascending) are paired
// with the ascending minor eigenvalues mu_jk, and
//
//   |v_ij|^2 = prod_k |lambda_i - mu_jk| / |lambda_i - lambda'_k|.
//
// By Cauchy interlacing (lambda_k <= mu_jk <= lambda_{k+1}) every paired
// factor lies in [0, 1], so the running product only decreases: it needs no
// exponent of its own and cannot underflow unless the result itself does.
// Each factor is one correctly rounded division; the product runs over k in
// ascending order.  Same launch geometry and LDS staging as identity_kernel;
// an exactly zero denominator factor (repeated lambda_i) makes row i NaN and
// sets the degenerate flag, an exactly zero numerator factor gives 0.
__global__ __launch_bounds__(256) void identity_paired_kernel(const BatchDesc *desc, const double *lambda,
                                                               const double *mu, double *V2, int32_t *flags) {
    __shared__ double sm[ID_JT][ID_KC];
    __shared__ double sl[ID_KC + 1];
    const int b = blockIdx.z;
    const int n = desc[b].n;
    const int ncol = desc[b].ncol;
    const int j0 = blockIdx.y * ID_JT;
    if (j0 >= ncol || (int)blockIdx.x * 256 >= n) return;
    const int m = n - 1;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const bool live = i < n;
    const double *lam = lambda + desc[b].lam_off;
    const int E = spectrum_exponent(lam, n);
    const double li = live ? ldexp(lam[i], -E) : 0.0;
    const double *mub = mu + desc[b].mu_off;
    double r[ID_JT];
#pragma unroll
    for (int t = 0; t < ID_JT; ++t) r[t] = 1.0;
    bool zero_den = false;
    for (int kc = 0; kc < m; kc += ID_KC) {
        const int kn = min(ID_KC, m - kc);
        __syncthreads();
        for (int q = threadIdx.x; q < ID_JT * ID_KC; q += 256) {
            const int jj = q / ID_KC, kk = q % ID_KC;
            const int j = j0 + jj;
            sm[jj][kk] = (j < ncol && kk < kn) ? ldexp(mub[(int64_t)j * m + kc + kk], -E) : 0.0;
        }
        // lambda_{kc} .. lambda_{kc + kn}: lambda'_k is lambda_k below i, lambda_{k+1} from i on
        for (int q = threadIdx.x; q <= kn; q += 256) sl[q] = ldexp(lam[kc + q], -E);
        __syncthreads();
        for (int kk = 0; kk < kn; ++kk) {
            const double den = fabs(li - sl[kk + ((kc + kk >= i) ? 1 : 0)]);
            zero_den = zero_den || den == 0.0;
#pragma unroll
            for (int t = 0; t < ID_JT; ++t) r[t] *= fabs(li - sm[t][kk]) / den;
        }
    }
    if (!live) return;
    if (zero_den) atomicOr(&flags[b], 2);
    double *out = V2 + desc[b].v2_off + (int64_t)i * ncol;
#pragma unroll
    for (int t = 0; t < ID_JT; ++t) {
        const int j = j0 + t;
        if (j >= ncol) break;
        out[j] = zero_den ? __builtin_nan("") : r[t];
    }
}

// Row i of Eq. (2) only (one eigenvector's squared components, all j), from
// lambda and the spectra of all n minors: one thread per column j, each
// reading its minor's spectrum directly.  The arithmetic is that of
// denominators_kernel + identity_kernel (PAIRED false: same factors, same
// grouping into chunks of ID_KC with renormalisation every RENORM factors) or
// of identity_paired_kernel (PAIRED true), so the row is bit for bit the
// corresponding row of the full W.
template <bool PAIRED>
__global__ __launch_bounds__(256) void eigenvector_row_kernel(int n, int i, const double *lam, const double *mu,
                                                               double *row, int32_t *flag) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const int m = n - 1;
    const int E = spectrum_exponent(lam, n);
    const double li = ldexp(lam[i], -E);
    const double *muj = mu + (int64_t)j * m;
    double w;
    if constexpr (PAIRED) {
        double r = 1.0;
        bool zero_den = false;
        for (int k = 0; k < m; ++k) {
            const double den = fabs(li - ldexp(lam[k + (k >= i ? 1 : 0)], -E));
            zero_den = zero_den || den == 0.0;
            r *= fabs(li - ldexp(muj[k], -E)) / den;
        }
        w = zero_den ? __builtin_nan("") : r;
        if (zero_den && j == 0) atomicOr(flag, 2);
    } else {
        double q = 1.0;
        int qe = 0, cnt = 0;
        bool zero = false;
        for (int k = 0; k < n; ++k) {
            if (k == i) continue;
            const double d = li - ldexp(lam[k], -E);
            if (d == 0.0) zero = true;
            mul_factor(q, qe, fabs(d));
            if (++cnt == RENORM) { renormalise(q, qe); cnt = 0; }
        }
        renormalise(q, qe);
        double pm = 1.0;
        int pe = 0;
        for (int kc = 0; kc < m; kc += ID_KC) {
            const int kn = min(ID_KC, m - kc);
            int kk = 0;
            for (; kk + RENORM <= kn; kk += RENORM) {
                for (int u = 0; u < RENORM; ++u) mul_factor(pm, pe, fabs(li - ldexp(muj[kc + kk + u], -E)));
                renormalise(pm, pe);
            }
            for (; kk < kn; ++kk) mul_factor(pm, pe, fabs(li - ldexp(muj[kc + kk], -E)));
            renormalise(pm, pe);
        }
        w = zero ? __builtin_nan("") : ldexp(pm / q, pe - qe);
        if (zero && j == 0) atomicOr(flag, 2);
    }
    row[j] = w;
}

}  // namespace eeid
