/*
 * libeeid -- squared eigenvector components of Hermitian matrices through the
 * eigenvector-eigenvalue identity, on one AMD Instinct MI355X (gfx950).
 *
 * The identity (arXiv 2002.04989, Section 2, Eq. (2)): for an n x n Hermitian
 * A with ascending eigenvalues lambda_1..lambda_n and M_j the principal minor
 * of A with row j and column j removed,
 *
 *     |v_ij|^2 = prod_{k=1}^{n-1} (lambda_i(A) - lambda_k(M_j))
 *                / prod_{k != i} (lambda_i(A) - lambda_k(A)).
 *
 * Algorithm 2 of Section 3 computes the spectrum of A once and the spectrum of
 * each minor once, then evaluates the ratio.  This library does the same on
 * the GPU: eeid_minor_eigvals computes lambda(A) and all lambda(M_j) of a batch
 * of matrices in one persistent launch (Householder tridiagonalisation +
 * Sturm bisection), and eeid_components evaluates the ratio for every (i, j)
 * as products of |differences| in FP64 with a separate exponent (no over- or
 * underflow at any n).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - C99-compatible.  Pointers named A, lambda, mu, V2 and flags are DEVICE
 *    pointers (memory of the handle's device).  Pointers named n, a_offset and
 *    js are HOST pointers and are only read during the call.
 *  - Matrices are row-major with leading dimension n_b.  Only the lower
 *    triangle (row >= column) is read; the imaginary parts of a complex
 *    diagonal are ignored (Hermitian by convention, Section 2).
 *    EEID_R64 elements are double; EEID_C128 elements are interleaved
 *    (re, im) doubles and a_offset counts complex elements.
 *  - Eigenvalues are ascending.  Outputs of a batch are densely packed in
 *    batch order (prefix sums of n_b):
 *      lambda: sum n_b doubles,            matrix b at offset sum_{c<b} n_c;
 *      mu:     sum n_b (n_b - 1) doubles,  row j of matrix b = spectrum of M_j;
 *      V2:     sum n_b^2 doubles,          V2_b[i * n_b + j] = |v_ij|^2, row i
 *              belongs to the i-th smallest eigenvalue of A_b;
 *      flags:  count int32 per batch (0 = clean; bits EEID_FLAG_*).
 *  - Every call is asynchronous on the handle's stream; results are valid once
 *    that stream has synchronised.  The caller owns A and all outputs; the
 *    library never frees or retains them after the call returns.  The library
 *    owns its workspace (grown lazily, freed by eeid_destroy).
 *  - Argument errors are detected before anything is enqueued and return a
 *    status; no C++ exception or abort crosses this interface.
 *  - One handle is used by one host thread at a time.
 */
#ifndef EEID_H
#define EEID_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eeid_handle_s *eeid_handle_t;

typedef enum {
    EEID_OK = 0,
    EEID_ERR_INVALID_ARG = 1,  /* null pointer, n_b < 1, count < 1, bad enum, ... */
    EEID_ERR_NO_DEVICE = 2,    /* no usable GPU, or the device index is out of range */
    EEID_ERR_ALLOC = 3,        /* device workspace could not be allocated */
    EEID_ERR_HIP = 4,          /* a HIP runtime call failed; see eeid_last_error */
    EEID_ERR_UNSUPPORTED = 5   /* valid request this library does not serve (e.g. n_b too large) */
} eeid_status_t;

typedef enum { EEID_R64 = 0, EEID_C128 = 1 } eeid_dtype_t;

/* Precision of the tridiagonalisation's trailing matrix.
 *  EEID_PREC_FP64:          everything in FP64 (the plain form).
 *  EEID_PREC_FP32_TRAILING: the trailing matrix is stored in FP32 (FP32
 *      complex for C128) and its rank-2k update runs on FP32 matrix cores
 *      with FP32 accumulation; Householder vectors, norms, the tridiagonal,
 *      the bisection and the identity stay FP64.  Eigenvalue error is of order
 *      sqrt(n) * 2^-24 * ||A||_2. */
typedef enum { EEID_PREC_FP64 = 0, EEID_PREC_FP32_TRAILING = 1 } eeid_prec_t;

enum {
    EEID_FLAG_NONFINITE_INPUT = 1, /* a NaN/Inf in the lower triangle: all outputs of b are NaN */
    EEID_FLAG_DEGENERATE = 2,      /* lambda_i(A) repeated exactly: row i of V2 is NaN (Eq. (2) is 0/0) */
    EEID_FLAG_WAIT_TIMEOUT = 4,    /* a bounded wait between the waves of a workgroup gave up (a library
                                      fault, never expected): the outputs of b are invalid.  The polls
                                      allowed (default 2^26) can be set by the environment variable
                                      EEID_SPIN_LIMIT, read by eeid_create */
    EEID_FLAG_NO_REFERENCE = 8     /* eeid_signed_eigenvectors: some eigenvector has a zero component at
                                      the reference index; its row of V is NaN */
};

/* Largest matrix order the library accepts (LDS holds two FP64/complex
 * vectors of the padded order during tridiagonalisation). */
#define EEID_MAX_N_R64 8192
#define EEID_MAX_N_C128 4160

/* Create a handle on HIP device `hip_device`.  Returns EEID_ERR_NO_DEVICE when
 * no GPU is present or the index is invalid.  The handle starts on the null
 * stream; workspace is allocated on first use. */
eeid_status_t eeid_create(eeid_handle_t *h, int hip_device);

/* Synchronise the handle's stream, free its workspace and the handle. */
eeid_status_t eeid_destroy(eeid_handle_t h);

/* Make subsequent calls enqueue on `stream` (a hipStream_t of the handle's
 * device, passed as void*; NULL = null stream).  When the stream changes,
 * the work already queued on the previous one is waited for first (the
 * handle's workspace is shared by all its calls). */
eeid_status_t eeid_set_stream(eeid_handle_t h, void *stream);

/* Static description of a status code (never NULL). */
const char *eeid_status_string(eeid_status_t s);

/* Detail of the last non-OK status returned on `h` ("" if none). */
const char *eeid_last_error(eeid_handle_t h);

/* Ascending eigenvalues of every matrix of a batch (the EigenValues(A) step
 * of Algorithms 1 and 2, Section 3).
 *   count     number of matrices (>= 1)
 *   n         host [count], n_b >= 1
 *   a_offset  host [count], element offset of matrix b inside A (>= 0)
 *   A         device, element type per `t`
 *   lambda    device [sum n_b] output
 *   flags     device [count] output (cleared, then EEID_FLAG_* bits) */
eeid_status_t eeid_eigvalsh_batched(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p,
                                    int64_t count, const int64_t *n, const int64_t *a_offset,
                                    const void *A, double *lambda, int32_t *flags);

/* lambda(A_b) and the spectra of all n_b principal minors M_j of every matrix
 * of the batch (Section 2: M_j removes row j and column j), in one
 * persistent launch over all (matrix, minor) problems, largest first.
 *   mu        device [sum n_b (n_b - 1)] output, row j of b = ascending spec(M_j)
 * Other arguments as for eeid_eigvalsh_batched. */
eeid_status_t eeid_minor_eigvals(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p,
                                 int64_t count, const int64_t *n, const int64_t *a_offset,
                                 const void *A, double *lambda, double *mu, int32_t *flags);

/* lambda(A) and the spectra of a chosen subset of minors of ONE matrix of
 * order n (the single-component and single-column queries of Section 4 and
 * Table 1 need only some minors).
 *   nsel      number of selected minors (>= 1)
 *   js        host [nsel], each 0 <= js[s] < n (repeats allowed)
 *   lambda    device [n] output, or NULL to skip lambda(A)
 *   mu_sel    device [nsel * (n - 1)] output, row s = ascending spec(M_{js[s]})
 *   flag      device [1] output */
eeid_status_t eeid_minor_eigvals_subset(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p,
                                        int64_t n, const void *A, int64_t nsel, const int64_t *js,
                                        double *lambda, double *mu_sel, int32_t *flag);

/* lambda(A) and the spectra of a few minors of ONE real symmetric matrix with
 * low latency (the single-component and single-column queries of Section 4,
 * Table 1, Fig. 1(a)): each eigenvalue problem is spread over many
 * workgroups (one per CU, the CUs split evenly over the problems, at most
 * one per 16 rows) instead of one, in one cooperative launch: unblocked
 * Householder tridiagonalisation
 * with the matrix rows dealt cyclically to the workgroups (two grid-wide
 * barriers per column, each bounded: a wait that gives up sets
 * EEID_FLAG_WAIT_TIMEOUT), then each workgroup bisects its slice of the
 * eigenvalues.  Arguments as for eeid_minor_eigvals_subset (nsel may be 0);
 * at most 16 problems per call (lambda counts as one); EEID_R64 and
 * EEID_PREC_FP64 only, else EEID_ERR_UNSUPPORTED.  The same request gives the
 * same bits on every call (the workgroups per problem depend on the order and
 * the number of problems, so other requests agree to rounding, as does the
 * batched path). */
eeid_status_t eeid_minor_eigvals_latency(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p,
                                         int64_t n, const void *A, int64_t nsel, const int64_t *js,
                                         double *lambda, double *mu_sel, int32_t *flag);

/* The identity, Eq. (2): V2_b[i * n_b + j] = prod_k |lambda_i - mu_jk|
 * / prod_{k != i} |lambda_i - lambda_k| for every matrix, evaluated in FP64
 * with each product carried as a mantissa and a separate integer exponent,
 * every factor split into its own mantissa and exponent first (relative
 * rounding at most about n_b eps, for any finite spectra: factors may range
 * from the smallest subnormal to the largest double).  An exactly zero
 * numerator factor gives 0; an exactly repeated lambda_i gives a NaN row and
 * sets EEID_FLAG_DEGENERATE in flags[b] (other bits are kept, so pass the
 * flags of eeid_minor_eigvals).
 *   lambda, mu  device, laid out as eeid_minor_eigvals writes them
 *   V2          device [sum n_b^2] output */
eeid_status_t eeid_components(eeid_handle_t h, int64_t count, const int64_t *n,
                              const double *lambda, const double *mu, double *V2,
                              int32_t *flags);

/* eeid_components for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with the library's scratch (the batch
 * descriptors and the denominator pairs) in a fixed device array of
 * EEID_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends, instead of
 * workspace it allocates.  The call allocates and frees nothing and copies
 * nothing from the host; it only launches kernels on the handle's stream.
 * Limits: count <= EEID_NOALLOC_MAX_MATRICES and sum n_b <=
 * EEID_NOALLOC_MAX_EIGENVALUES, else EEID_ERR_UNSUPPORTED (nothing enqueued).
 * Every call on one GPU shares that GPU's scratch: calls that overlap on one
 * GPU (other streams, other handles or threads) race and must be ordered by
 * the caller.  Arguments as for eeid_components. */
#define EEID_NOALLOC_MAX_MATRICES 64
#define EEID_NOALLOC_MAX_EIGENVALUES 16384
#define EEID_NOALLOC_SCRATCH_BYTES (4096 + 16 * EEID_NOALLOC_MAX_EIGENVALUES)
eeid_status_t eeid_components_noalloc(eeid_handle_t h, int64_t count, const int64_t *n,
                                      const double *lambda, const double *mu, double *V2,
                                      int32_t *flags);

/* Columns of Eq. (2) for a subset of minors of ONE matrix of order n: the
 * squared components j_s of every eigenvector, from lambda(A) and the spectra
 * of the chosen minors (as eeid_minor_eigvals_subset writes them).  With one
 * minor this is the single-component query of Table 1 for every i at once.
 *   lambda  device [n];  mu_sel device [nsel * (n - 1)]
 *   V2_sel  device [n * nsel] output, V2_sel[i * nsel + s] = |v_i(j_s)|^2
 *   flag    device [1], EEID_FLAG_DEGENERATE is OR-ed in */
eeid_status_t eeid_components_subset(eeid_handle_t h, int64_t n, const double *lambda, int64_t nsel,
                                     const double *mu_sel, double *V2_sel, int32_t *flag);

/* One component |v_ij|^2 of ONE real symmetric matrix: the paper's scalar
 * query EigenComponent(matrix, i, j) (Section 3, Algorithms 1 and 2; Section
 * 4, Table 1).  lambda(A) and the spectrum of the minor M_j on the latency
 * path (as eeid_minor_eigvals_latency), then Eq. (2) for the pair (i, j) in
 * the handle's identity form; bit for bit entry i of the column that
 * eeid_components_subset gives for j.
 *   A    device, n x n row-major, lower triangle read;  0 <= i, j < n
 *   out  device double [1] output;  flag device int32 [1] output (flags as
 *        for eeid_minor_eigvals)
 * EEID_R64 and EEID_PREC_FP64 only, else EEID_ERR_UNSUPPORTED; the spectra
 * live in workspace the handle owns. */
eeid_status_t eeid_component(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t n, const void *A, int64_t i,
                             int64_t j, double *out, int32_t *flag);

/* One eigenvector's squared components (the complete-eigenvector query of
 * Section 4, Fig. 1(b)): row i of Eq. (2), row[j] = |v_ij|^2 for every j, from
 * lambda(A) and the spectra of all n minors (as eeid_minor_eigvals writes
 * them for this matrix), in the handle's identity form; bit for bit row i of
 * eeid_components' V2.
 *   lambda device [n];  mu device [n * (n - 1)];  0 <= i < n
 *   row    device [n] output;  flag device [1], EEID_FLAG_DEGENERATE is OR-ed in */
eeid_status_t eeid_eigenvector_sq(eeid_handle_t h, int64_t n, const double *lambda, const double *mu, int64_t i,
                                  double *row, int32_t *flag);

/* Signs and phases of the eigenvector components (Section 2: the identity
 * applied in other bases gives the directions).  For a reference index r and
 * every partner k != r, B = R^H A R with R a rotation by pi/4 in the (r, k)
 * plane has A's eigenvalues; with the new basis e'_r = (e_r + e_k)/sqrt2,
 * e'_k = (e_k - e_r)/sqrt2, Eq. (2) on the minor of B at r gives
 * (W_ir + W_ik)/2 + Re(conj(v_ir) v_ik); with e'_r = (e_r + i e_k)/sqrt2,
 * e'_k = (e_k + i e_r)/sqrt2 (complex input only) it gives
 * (W_ir + W_ik)/2 + Im(conj(v_ir) v_ik).
 *
 * eeid_rotated_minor_eigvals: the ascending spectra of those minors (order
 * n - 1 each) in one persistent launch.
 *   r       0 <= r < n
 *   mu_rot  device output: EEID_R64 [(n - 1) * (n - 1)], row q = the q-th
 *           partner k != r in ascending order; EEID_C128 [2 (n - 1) * (n - 1)],
 *           rows 0..n-2 the real rotations, rows n-1..2n-3 the imaginary ones
 *   flag    device [1] output */
eeid_status_t eeid_rotated_minor_eigvals(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p, int64_t n,
                                         const void *A, int64_t r, double *mu_rot, int32_t *flag);

/* eeid_signed_eigenvectors: the unit eigenvectors with their signs (phases
 * for complex input), from lambda(A) and W (as eeid_all_components writes
 * them for this matrix) and mu_rot: with the convention v_ir real >= 0,
 *   V[i, r] = sqrt(W_ir),  V[i, k] = conj(v_ir) v_ik / sqrt(W_ir),
 * conj(v_ir) v_ik taken from the rotated identities above.  Row i is the
 * eigenvector of the i-th smallest eigenvalue; V is double [n * n] for
 * EEID_R64 and interleaved (re, im) double [2 * n * n] for EEID_C128.  Its
 * absolute error is about the error of W divided by sqrt(W_ir), so choose r
 * where the eigenvectors of interest are not small.  A row with W_ir = 0 has
 * no reference: it is NaN and bit 8 is OR-ed into *flag.
 *   lambda device [n], W device [n * n], mu_rot device as written above
 *   flag   device [1] (bits OR-ed in) */
eeid_status_t eeid_signed_eigenvectors(eeid_handle_t h, eeid_dtype_t t, int64_t n, int64_t r, const double *lambda,
                                       const double *W, const double *mu_rot, double *V, int32_t *flag);

/* eeid_minor_eigvals followed by eeid_components: every |v_ij|^2 of every
 * matrix of the batch from device-resident A to device-resident V2.  In graph
 * mode (eeid_set_graph_mode) the launches are recorded once per argument set
 * into a hipGraph and replayed on the handle's stream. */
eeid_status_t eeid_all_components(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p,
                                  int64_t count, const int64_t *n, const int64_t *a_offset,
                                  const void *A, double *lambda, double *mu, double *V2,
                                  int32_t *flags);

/* How the identity entry points (eeid_components, _noalloc, _subset and
 * eeid_all_components) evaluate the ratio of Eq. (2); a property of the handle.
 *  EEID_IDENTITY_PRODUCTS (default): numerator and denominator as two
 *      products, each a mantissa with a separate integer exponent.
 *  EEID_IDENTITY_PAIRED: Algorithm 2's pairing (Section 3): lambda_i taken
 *      out, the other eigenvalues lambda'_k are paired in ascending order with
 *      the minor's mu_k and W = prod_k |lambda_i - mu_k| / |lambda_i - lambda'_k|;
 *      by Cauchy interlacing every factor is in [0, 1], so the running product
 *      needs no exponent (it cannot underflow unless W does).  One correctly
 *      rounded division per factor.
 * Both give W within a few n eps (relative) of the exact ratio of the given
 * spectra; flags and NaN/zero conventions are the same.  Returns
 * EEID_ERR_INVALID_ARG for any other value. */
typedef enum { EEID_IDENTITY_PRODUCTS = 0, EEID_IDENTITY_PAIRED = 1 } eeid_identity_form_t;
eeid_status_t eeid_set_identity_form(eeid_handle_t h, int form);

/* Enable (1) or disable (0) graph mode for eeid_minor_eigvals,
 * eeid_components and eeid_all_components: each call's launches are recorded
 * into a hipGraph the first time an argument set (entry point, pointers,
 * orders, kernel configuration) is seen (recording on a private stream) and
 * replayed afterwards on the handle's stream.  Up to eight
 * recorded argument sets are kept per handle (least recently used replaced);
 * reallocation of the handle's buffers invalidates them.  Results are the
 * same as in eager mode. */
eeid_status_t eeid_set_graph_mode(eeid_handle_t h, int enable);

/* Phase timers of the two-stage kernel, in builds compiled with
 * -DEEID_PHASE_TIMERS (libeeid_phase.so; other builds return
 * EEID_ERR_UNSUPPORTED).  ticks: host [8], the sums over all workgroups of the
 * 100 MHz wall-clock ticks spent in 0 gather, 1 panel QR, 2 symmetric
 * product, 3 W, 4 rank-2k update, 5 band to tridiagonal, 6 bisection,
 * 7 queue and the rest, accumulated since the last reset (reset = 1 clears
 * them and ignores ticks).  Synchronous; an instrument for profiling only. */
eeid_status_t eeid_phase_ticks(unsigned long long *ticks, int reset);

/* Number of compiled configurations of the real eigenvalue kernel (the
 * complex kernel has one).  Configurations 0..2 use the one-stage Householder
 * reduction, 3..4 the two-stage (dense -> band -> tridiagonal) reduction. */
int eeid_variant_count(void);

/* Use configuration `variant` (0 .. eeid_variant_count() - 1) of the real
 * eigenvalue kernel for every real batch on this handle, or restore the
 * automatic choice (tune table, else a size rule) with variant = -1.
 * Returns EEID_ERR_INVALID_ARG for any other value. */
eeid_status_t eeid_set_variant(eeid_handle_t h, int variant);

/* Time every compiled configuration of the eigenvalue kernel on this batch
 * (one eeid_minor_eigvals each, outputs written to lambda/mu/flags) and use
 * the fastest for batches of the same dtype, precision, largest order and
 * problem count from now on.  If the environment variable EEID_TUNE_TABLE
 * names a file, the choice is appended to it ("dtype prec n_max problems
 * variant  # name ms") and eeid_create loads it.  Synchronises the stream.
 *   best_variant, best_ms  host outputs (may be NULL) */
eeid_status_t eeid_autotune(eeid_handle_t h, eeid_dtype_t t, eeid_prec_t p,
                            int64_t count, const int64_t *n, const int64_t *a_offset,
                            const void *A, double *lambda, double *mu, int32_t *flags,
                            int *best_variant, double *best_ms);

#ifdef __cplusplus
}
#endif

#endif /* EEID_H */
