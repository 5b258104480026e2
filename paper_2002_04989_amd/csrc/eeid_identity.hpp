// The eigenvector-eigenvalue identity (Section 2, Eq. (2) of the paper) for
// every (i, j) of a batch, from the ascending spectra of A and of its minors:
//
//   |v_ij|^2 = exp( sum_k log|lambda_i - mu_jk| - sum_{k != i} log|lambda_i - lambda_k| )
//
// in FP64.  Raw products over- and underflow for n of a few hundred (the paper
// batches them for that reason, Section 3); the logarithms cannot.  Both sums
// are Neumaier-compensated, and the denominator is kept as an unevaluated
// (hi, lo) pair so that the difference of two sums of order n log||A|| keeps
// its low-order bits.  An exactly zero numerator factor gives 0; an exactly
// repeated lambda_i leaves the ratio undefined, so row i is NaN and the matrix
// is flagged degenerate.
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

__device__ __forceinline__ void neumaier_add(double &s, double &c, double x) {
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
}

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
__global__ __launch_bounds__(256) void denominators_kernel(const BatchDesc *desc, const double *lambda,
                                                            double *Dpair, int32_t *flags) {
    const int b = blockIdx.y;
    const int n = desc[b].n;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double *lam = lambda + desc[b].lam_off;
    const double li = lam[i];
    double s = 0.0, c = 0.0;
    bool zero = false;
    for (int k = 0; k < n; ++k) {
        if (k == i) continue;
        const double d = li - lam[k];
        if (d == 0.0) zero = true;
        else neumaier_add(s, c, log(fabs(d)));
    }
    double *out = Dpair + 2 * (desc[b].lam_off + i);
    if (zero) {
        out[0] = __builtin_nan("");
        out[1] = 0.0;
        atomicOr(&flags[b], 2);
    } else {
        out[0] = s;
        out[1] = c;
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
    const double li = live ? lambda[desc[b].lam_off + i] : 0.0;
    const double *mub = mu + desc[b].mu_off;
    double s[ID_JT], c[ID_JT];
    bool zero[ID_JT];
#pragma unroll
    for (int t = 0; t < ID_JT; ++t) { s[t] = 0.0; c[t] = 0.0; zero[t] = false; }
    for (int kc = 0; kc < m; kc += ID_KC) {
        const int kn = min(ID_KC, m - kc);
        __syncthreads();
        for (int q = threadIdx.x; q < ID_JT * ID_KC; q += 256) {
            const int jj = q / ID_KC, kk = q % ID_KC;
            const int j = j0 + jj;
            sm[jj][kk] = (j < ncol && kk < kn) ? mub[(int64_t)j * m + kc + kk] : 0.0;
        }
        __syncthreads();
        for (int kk = 0; kk < kn; ++kk) {
#pragma unroll
            for (int t = 0; t < ID_JT; ++t) {
                const double d = li - sm[t][kk];
                if (d == 0.0) zero[t] = true;
                else neumaier_add(s[t], c[t], log(fabs(d)));
            }
        }
    }
    if (!live) return;
    const double *dp = Dpair + 2 * (desc[b].lam_off + i);
    const double dhi = dp[0], dlo = dp[1];
    double *out = V2 + desc[b].v2_off + (int64_t)i * ncol;
#pragma unroll
    for (int t = 0; t < ID_JT; ++t) {
        const int j = j0 + t;
        if (j >= ncol) break;
        double w;
        if (isnan(dhi)) w = __builtin_nan("");
        else if (zero[t]) w = 0.0;
        else w = exp((s[t] - dhi) + (c[t] - dlo));
        out[j] = w;
    }
}

}  // namespace eeid
