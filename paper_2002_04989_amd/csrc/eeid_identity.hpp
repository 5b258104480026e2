// The eigenvector-eigenvalue identity (Section 2, Eq. (2) of the paper) for
// every (i, j) of a batch, from the ascending spectra of A and of its minors:
//
//   |v_ij|^2 = prod_k |lambda_i - mu_jk| / prod_{k != i} |lambda_i - lambda_k|
//
// in FP64.  Raw products over- and underflow for n of a few hundred (the paper
// batches them for that reason, Section 3); here each product is carried as a
// mantissa in [1/2, 1) and a separate integer exponent, renormalised after
// every second factor.  The eigenvalues of a matrix are first scaled by 2^-E,
// E the exponent of its largest |lambda| (exact, and the same for numerator
// and denominator, which have n - 1 factors each), so every factor is below 4
// and two of them can neither overflow nor leave the normal range.  The
// rounding error is that of the n - 1 multiplications (relative, at most
// about n eps).  An exactly zero numerator factor gives 0; an exactly repeated
// lambda_i leaves the ratio undefined, so row i is NaN and the matrix is
// flagged degenerate.
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

// Dpair[2 (lam_off + i) + {0, 1}] = (hi, lo) of sum_{k != i} log|lambda_i - lambda_k|.
// Exponent of the largest |lambda| of an ascending spectrum (0 for an all-zero one).
__device__ __forceinline__ int spectrum_exponent(const double *lam, int n) {
    const double big = fmax(fabs(lam[0]), fabs(lam[n - 1]));
    return (big > 0.0) ? ilogb(big) : 0;
}

// Denominator of Eq. (2) for each i: prod_{k != i} |lambda_i - lambda_k| 2^-E as
// (mantissa, exponent) in Dpair[2 i], Dpair[2 i + 1].
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
    int qe = 0;
    bool zero = false;
    for (int k = 0; k < n; ++k) {
        if (k == i) continue;
        const double d = li - ldexp(lam[k], -E);
        if (d == 0.0) zero = true;
        int e;
        q = frexp(q * fabs(d), &e);
        qe += e;
    }
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
        for (; kk + 1 < kn; kk += 2) {
#pragma unroll
            for (int t = 0; t < ID_JT; ++t) {
                const double f = fabs(li - sm[t][kk]) * fabs(li - sm[t][kk + 1]);
                int e;
                pm[t] = frexp(pm[t] * f, &e);
                pe[t] += e;
            }
        }
        if (kk < kn) {
#pragma unroll
            for (int t = 0; t < ID_JT; ++t) {
                int e;
                pm[t] = frexp(pm[t] * fabs(li - sm[t][kk]), &e);
                pe[t] += e;
            }
        }
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

}  // namespace eeid
