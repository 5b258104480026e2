/*
 * Plain cyclic Jacobi eigensolver for the CPU oracle (test infrastructure
 * only: nothing in the product path links or calls this file).
 *
 * The paper treats the eigenvalues of A and of every principal minor as a
 * black-box step (EigenValues in Algorithms 1 and 2 of Section 3) over the
 * Hermitian domain stated in Section 2.  The oracle realises that step with
 * the textbook Jacobi method: repeatedly annihilate an off-diagonal pair
 * (p, q) with a plane rotation J, A <- J^H A J, until every off-diagonal
 * entry is negligible against its diagonal pair.  Jacobi is chosen because it
 * shares nothing with the Householder + bisection route of the GPU library.
 *
 * Working precision (the paper fixes none): by default the x87 extended
 * format (long double, 64-bit significand).  Eq. (2) divides by eigenvalue
 * gaps, so an eigenvalue error delta moves |v_ij|^2 by about
 * |v_ij|^2 * delta / gap per near factor; on spectra with 1e-6 gaps the
 * rounding that thousands of double-precision rotations accumulate (about
 * 1e-12 absolute at n = 2048) would already move |v_ij|^2 by more than 1e-9.
 * Extended precision keeps that accumulation some 2000 times smaller.
 * Compiled with -DJACOBI_DOUBLE the same code works in double precision
 * (about six times faster; used where the extended run would take hours and
 * the spectrum has no tiny gaps).  Inputs and outputs are double either way.
 *
 * Ordering: the round-robin ("tournament") ordering of Brent and Luk.  Each
 * round holds n/2 disjoint pairs; their rotations commute, so all of a round's
 * angles are taken from the matrix at the start of the round and the round is
 * applied as A <- J^H (A J) with J the product of its rotations.  Every pair
 * meets once per sweep, exactly as in the row-cyclic ordering.
 *
 * Rotation for the 2x2 Hermitian block [[a, b], [conj(b), d]], b = |b| e^{i phi}:
 *   theta = (d - a) / (2 |b|),  t = sign(theta) / (|theta| + sqrt(1 + theta^2)),
 *   c = 1 / sqrt(1 + t^2),  s = t c,
 *   J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]]        (real case: phi = 0).
 * Then (J^H B J)_{12} = c s (a - d) + |b| (c^2 - s^2) = 0.
 *
 * Skip rule (the paper is silent): a pair is left alone when
 *   |a_pq| <= max(eps * sqrt(|a_pp a_qq|), eps^2 * ||A||_F),
 * eps the machine epsilon of the working precision; the iteration stops after a
 * sweep in which every pair was skipped and fails (returns -1) after
 * max_sweeps sweeps.
 *
 * Timing aid (used only to time a bounded sample of a large problem): with
 * max_rounds > 0 the iteration stops after that many rounds and returns -2
 * (the outputs are then not eigenvalues).  If stats != NULL, stats[0]
 * receives the number of rotations applied and stats[1] the number of rounds.
 *
 * Storage: row-major n x n.  Complex matrices are interleaved (re, im)
 * doubles.  Only the lower triangle of the input is read; the upper triangle
 * is rebuilt from it and the imaginary parts of the diagonal are dropped.
 * The input array is left unchanged.  Eigenvalues are returned ascending
 * (rounded to double); if v != NULL its column i (row-major, v[r*n + i]) is a
 * unit eigenvector of w[i].
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef JACOBI_DOUBLE
typedef double wreal;
#define WEPS DBL_EPSILON
#define wsqrt sqrt
#define wfabs fabs
#define whypot hypot
#else
typedef long double wreal;
#define WEPS LDBL_EPSILON
#define wsqrt sqrtl
#define wfabs fabsl
#define whypot hypotl
#endif

static void tournament_init(int64_t *arr, int64_t N) {
    for (int64_t i = 0; i < N; ++i) arr[i] = i;
}

/* rotate players 1..N-1 by one position (player 0 stays fixed) */
static void tournament_step(int64_t *arr, int64_t N) {
    if (N <= 2) return;
    int64_t last = arr[N - 1];
    for (int64_t i = N - 1; i > 1; --i) arr[i] = arr[i - 1];
    arr[1] = last;
}

static void rotation(wreal app, wreal aqq, wreal beta, wreal *c, wreal *s) {
    wreal theta = (aqq - app) / (2 * beta);
    wreal t;
    if (wfabs(theta) > 1e150) {
        t = (wreal)0.5 / theta;
    } else {
        t = (theta >= 0 ? (wreal)1 : (wreal)-1) / (wfabs(theta) + wsqrt(1 + theta * theta));
    }
    *c = 1 / wsqrt(1 + t * t);
    *s = t * (*c);
}

/* ascending sort of w with matching permutation of the columns of v (n x n, row-major) */
static void sort_pairs(int64_t n, wreal *w, wreal *v, int complex_v) {
    /* selection sort: O(n^2) comparisons, O(n) column swaps; negligible next to Jacobi */
    int64_t stride = complex_v ? 2 : 1;
    for (int64_t i = 0; i < n - 1; ++i) {
        int64_t k = i;
        for (int64_t j = i + 1; j < n; ++j)
            if (w[j] < w[k]) k = j;
        if (k != i) {
            wreal t = w[i]; w[i] = w[k]; w[k] = t;
            if (v) {
                for (int64_t r = 0; r < n; ++r)
                    for (int64_t z = 0; z < stride; ++z) {
                        wreal *x = &v[(r * n + i) * stride + z];
                        wreal *y = &v[(r * n + k) * stride + z];
                        wreal u = *x; *x = *y; *y = u;
                    }
            }
        }
    }
}

int oracle_jacobi_r64(int64_t n, const double *a_in, double *w_out, double *v_out, int max_sweeps,
                      int64_t max_rounds, int64_t *stats) {
    if (stats) { stats[0] = 0; stats[1] = 0; }
    if (n <= 0) return 0;
    wreal *a = malloc(sizeof(wreal) * (size_t)(n * n));
    wreal *w = malloc(sizeof(wreal) * (size_t)n);
    wreal *v = v_out ? malloc(sizeof(wreal) * (size_t)(n * n)) : NULL;
    /* the symmetric matrix whose lower triangle is that of the input */
    for (int64_t r = 0; r < n; ++r)
        for (int64_t c = 0; c <= r; ++c) a[r * n + c] = a[c * n + r] = (wreal)a_in[r * n + c];
    if (v) {
        for (int64_t i = 0; i < n * n; ++i) v[i] = 0;
        for (int64_t i = 0; i < n; ++i) v[i * n + i] = 1;
    }
    wreal fro = 0;
    for (int64_t i = 0; i < n * n; ++i) fro += a[i] * a[i];
    fro = wsqrt(fro);
    const wreal floor_abs = WEPS * WEPS * fro;

    const int64_t N = n + (n & 1);
    const int64_t npairs = N / 2;
    int64_t *arr = malloc(sizeof(int64_t) * (size_t)N);
    int64_t *P = malloc(sizeof(int64_t) * (size_t)npairs);
    int64_t *Q = malloc(sizeof(int64_t) * (size_t)npairs);
    wreal *C = malloc(sizeof(wreal) * (size_t)npairs);
    wreal *S = malloc(sizeof(wreal) * (size_t)npairs);
    int sweeps = -1, capped = 0;
    int64_t rounds_done = 0, total_rot = 0;

    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        int64_t rotated = 0;
        tournament_init(arr, N);
        for (int64_t round = 0; round < N - 1; ++round) {
            if (max_rounds > 0 && rounds_done == max_rounds) { capped = 1; break; }
            ++rounds_done;
            int64_t act = 0;
            for (int64_t i = 0; i < npairs; ++i) {
                int64_t p = arr[i], q = arr[N - 1 - i];
                if (p >= n || q >= n) continue;
                if (p > q) { int64_t t = p; p = q; q = t; }
                wreal apq = a[p * n + q], app = a[p * n + p], aqq = a[q * n + q];
                wreal thr = WEPS * wsqrt(wfabs(app * aqq));
                if (thr < floor_abs) thr = floor_abs;
                if (wfabs(apq) <= thr) continue;
                wreal c, s;
                rotation(app, aqq, apq, &c, &s);
                P[act] = p; Q[act] = q; C[act] = c; S[act] = s;
                ++act;
            }
            if (act) {
                rotated += act;
                /* A <- A J (columns p, q of every row) */
                for (int64_t r = 0; r < n; ++r) {
                    wreal *row = a + r * n;
                    for (int64_t k = 0; k < act; ++k) {
                        wreal x = row[P[k]], y = row[Q[k]];
                        row[P[k]] = C[k] * x - S[k] * y;
                        row[Q[k]] = S[k] * x + C[k] * y;
                    }
                }
                /* A <- J^T A (rows p, q) */
                for (int64_t k = 0; k < act; ++k) {
                    wreal *rp = a + P[k] * n, *rq = a + Q[k] * n;
                    const wreal c = C[k], s = S[k];
                    for (int64_t j = 0; j < n; ++j) {
                        wreal x = rp[j], y = rq[j];
                        rp[j] = c * x - s * y;
                        rq[j] = s * x + c * y;
                    }
                }
                for (int64_t k = 0; k < act; ++k) {
                    a[P[k] * n + Q[k]] = 0;
                    a[Q[k] * n + P[k]] = 0;
                }
                if (v) {
                    for (int64_t r = 0; r < n; ++r) {
                        wreal *row = v + r * n;
                        for (int64_t k = 0; k < act; ++k) {
                            wreal x = row[P[k]], y = row[Q[k]];
                            row[P[k]] = C[k] * x - S[k] * y;
                            row[Q[k]] = S[k] * x + C[k] * y;
                        }
                    }
                }
            }
            tournament_step(arr, N);
        }
        total_rot += rotated;
        if (capped) break;
        if (rotated == 0) { sweeps = sweep + 1; break; }
    }
    for (int64_t i = 0; i < n; ++i) w[i] = a[i * n + i];
    sort_pairs(n, w, v, 0);
    for (int64_t i = 0; i < n; ++i) w_out[i] = (double)w[i];
    if (v)
        for (int64_t i = 0; i < n * n; ++i) v_out[i] = (double)v[i];
    if (stats) { stats[0] = total_rot; stats[1] = rounds_done; }
    free(a); free(w); free(v);
    free(arr); free(P); free(Q); free(C); free(S);
    return capped ? -2 : sweeps;
}

int oracle_jacobi_c128(int64_t n, const double *a_in, double *w_out, double *v_out, int max_sweeps,
                      int64_t max_rounds, int64_t *stats) {
    if (stats) { stats[0] = 0; stats[1] = 0; }
    if (n <= 0) return 0;
    wreal *a = malloc(sizeof(wreal) * 2 * (size_t)(n * n));
    wreal *w = malloc(sizeof(wreal) * (size_t)n);
    wreal *v = v_out ? malloc(sizeof(wreal) * 2 * (size_t)(n * n)) : NULL;
    /* a[(r*n+c)*2 + {0,1}] = (re, im): the Hermitian matrix whose lower triangle
       is that of the input, with a real diagonal */
    for (int64_t r = 0; r < n; ++r) {
        a[(r * n + r) * 2] = (wreal)a_in[(r * n + r) * 2];
        a[(r * n + r) * 2 + 1] = 0;
        for (int64_t c = 0; c < r; ++c) {
            const wreal re = (wreal)a_in[(r * n + c) * 2], im = (wreal)a_in[(r * n + c) * 2 + 1];
            a[(r * n + c) * 2] = re; a[(r * n + c) * 2 + 1] = im;
            a[(c * n + r) * 2] = re; a[(c * n + r) * 2 + 1] = -im;
        }
    }
    if (v) {
        for (int64_t i = 0; i < 2 * n * n; ++i) v[i] = 0;
        for (int64_t i = 0; i < n; ++i) v[(i * n + i) * 2] = 1;
    }
    wreal fro = 0;
    for (int64_t i = 0; i < 2 * n * n; ++i) fro += a[i] * a[i];
    fro = wsqrt(fro);
    const wreal floor_abs = WEPS * WEPS * fro;

    const int64_t N = n + (n & 1);
    const int64_t npairs = N / 2;
    int64_t *arr = malloc(sizeof(int64_t) * (size_t)N);
    int64_t *P = malloc(sizeof(int64_t) * (size_t)npairs);
    int64_t *Q = malloc(sizeof(int64_t) * (size_t)npairs);
    wreal *C = malloc(sizeof(wreal) * (size_t)npairs);
    wreal *S = malloc(sizeof(wreal) * (size_t)npairs);
    wreal *ER = malloc(sizeof(wreal) * (size_t)npairs);  /* cos(phi) */
    wreal *EI = malloc(sizeof(wreal) * (size_t)npairs);  /* sin(phi) */
    int sweeps = -1, capped = 0;
    int64_t rounds_done = 0, total_rot = 0;

    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        int64_t rotated = 0;
        tournament_init(arr, N);
        for (int64_t round = 0; round < N - 1; ++round) {
            if (max_rounds > 0 && rounds_done == max_rounds) { capped = 1; break; }
            ++rounds_done;
            int64_t act = 0;
            for (int64_t i = 0; i < npairs; ++i) {
                int64_t p = arr[i], q = arr[N - 1 - i];
                if (p >= n || q >= n) continue;
                if (p > q) { int64_t t = p; p = q; q = t; }
                wreal br = a[(p * n + q) * 2], bi = a[(p * n + q) * 2 + 1];
                wreal beta = whypot(br, bi);
                wreal app = a[(p * n + p) * 2], aqq = a[(q * n + q) * 2];
                wreal thr = WEPS * wsqrt(wfabs(app * aqq));
                if (thr < floor_abs) thr = floor_abs;
                if (beta <= thr) continue;
                wreal c, s;
                rotation(app, aqq, beta, &c, &s);
                P[act] = p; Q[act] = q; C[act] = c; S[act] = s;
                ER[act] = br / beta; EI[act] = bi / beta;
                ++act;
            }
            if (act) {
                rotated += act;
                /* A <- A J: x' = c x - s e^{-i phi} y,  y' = s x + c e^{-i phi} y */
                for (int64_t r = 0; r < n; ++r) {
                    wreal *row = a + 2 * r * n;
                    for (int64_t k = 0; k < act; ++k) {
                        wreal *x = row + 2 * P[k], *y = row + 2 * Q[k];
                        wreal xr = x[0], xi = x[1];
                        wreal yr = y[0] * ER[k] + y[1] * EI[k];   /* e^{-i phi} y */
                        wreal yi = y[1] * ER[k] - y[0] * EI[k];
                        x[0] = C[k] * xr - S[k] * yr; x[1] = C[k] * xi - S[k] * yi;
                        y[0] = S[k] * xr + C[k] * yr; y[1] = S[k] * xi + C[k] * yi;
                    }
                }
                /* A <- J^H A: row_p' = c row_p - s e^{i phi} row_q,  row_q' = s row_p + c e^{i phi} row_q */
                for (int64_t k = 0; k < act; ++k) {
                    wreal *rp = a + 2 * P[k] * n, *rq = a + 2 * Q[k] * n;
                    const wreal c = C[k], s = S[k], er = ER[k], ei = EI[k];
                    for (int64_t j = 0; j < n; ++j) {
                        wreal xr = rp[2 * j], xi = rp[2 * j + 1];
                        wreal yr = rq[2 * j] * er - rq[2 * j + 1] * ei;  /* e^{i phi} y */
                        wreal yi = rq[2 * j + 1] * er + rq[2 * j] * ei;
                        rp[2 * j] = c * xr - s * yr; rp[2 * j + 1] = c * xi - s * yi;
                        rq[2 * j] = s * xr + c * yr; rq[2 * j + 1] = s * xi + c * yi;
                    }
                }
                for (int64_t k = 0; k < act; ++k) {
                    int64_t p = P[k], q = Q[k];
                    a[(p * n + q) * 2] = 0; a[(p * n + q) * 2 + 1] = 0;
                    a[(q * n + p) * 2] = 0; a[(q * n + p) * 2 + 1] = 0;
                    a[(p * n + p) * 2 + 1] = 0; a[(q * n + q) * 2 + 1] = 0;
                }
                if (v) {
                    for (int64_t r = 0; r < n; ++r) {
                        wreal *row = v + 2 * r * n;
                        for (int64_t k = 0; k < act; ++k) {
                            wreal *x = row + 2 * P[k], *y = row + 2 * Q[k];
                            wreal xr = x[0], xi = x[1];
                            wreal yr = y[0] * ER[k] + y[1] * EI[k];
                            wreal yi = y[1] * ER[k] - y[0] * EI[k];
                            x[0] = C[k] * xr - S[k] * yr; x[1] = C[k] * xi - S[k] * yi;
                            y[0] = S[k] * xr + C[k] * yr; y[1] = S[k] * xi + C[k] * yi;
                        }
                    }
                }
            }
            tournament_step(arr, N);
        }
        total_rot += rotated;
        if (capped) break;
        if (rotated == 0) { sweeps = sweep + 1; break; }
    }
    for (int64_t i = 0; i < n; ++i) w[i] = a[(i * n + i) * 2];
    sort_pairs(n, w, v, 1);
    for (int64_t i = 0; i < n; ++i) w_out[i] = (double)w[i];
    if (v)
        for (int64_t i = 0; i < 2 * n * n; ++i) v_out[i] = (double)v[i];
    if (stats) { stats[0] = total_rot; stats[1] = rounds_done; }
    free(a); free(w); free(v);
    free(arr); free(P); free(Q); free(C); free(S); free(ER); free(EI);
    return capped ? -2 : sweeps;
}
