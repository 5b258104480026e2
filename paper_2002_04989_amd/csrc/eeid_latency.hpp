// Eigenvalues of a FEW problems with many workgroups each: the latency path
// for the single-component and single-column queries (Section 4, Table 1 and
// Fig. 1(a): lambda(A) and the spectrum of one minor M_j, Section 2).
//
// The batched kernels run one problem per workgroup, so one query at n = 2000
// uses two of 256 CUs.  Here the G workgroups of a problem share it:
//
//   * the matrix (A, or the minor with row and column j removed) is stored in
//     full, both triangles, row-major; row i belongs to workgroup i mod G
//     (cyclic, so every workgroup keeps an equal share of the shrinking
//     trailing matrix);
//   * unblocked Householder tridiagonalisation (the textbook two-sided
//     reduction, one reflector per column k):
//       sigma^2 = sum_{i > k+1} A(i, k)^2 (partial sums per workgroup),
//       beta = -sign(alpha) sqrt(alpha^2 + sigma^2), tau = (beta - alpha) / beta,
//       u = e_{k+1} + A(k+2.., k) / (alpha - beta),
//       y = A22 u (each workgroup its own rows),
//       w = tau y - (tau^2 / 2) (u^T y) u,   A22 <- A22 - u w^T - w u^T;
//     every workgroup reads the column as row k (the stored matrix stays
//     exactly symmetric: the update term u_i w_j + w_i u_j is formed as two
//     rounded products added, which commutes), forms u itself, and all of w
//     from the global y, so each column needs two grid barriers: after the
//     sigma^2 partials and after y and the u^T y partials;
//   * then each workgroup bisects its slice of the eigenvalues of the
//     tridiagonal (d = diagonal, e = beta), with the certified bisection of
//     eeid_tridiag.hpp.
//
// Communication between workgroups.  The L2 caches of the XCDs are not
// coherent with each other, and an agent-scope release/acquire fence writes
// back and invalidates a whole L2, which per column would cost more than the
// column's work.  So only the data other workgroups read is written and read
// coherently, with agent-scope atomic stores and loads (written through to,
// and read from, the device-coherent level): the partial sums, y, the
// diagonal and e, and the next pivot row (row k + 1, which every workgroup
// reads as column k + 1).  A workgroup's own rows stay in its caches.  At a
// grid barrier every thread first waits for its own stores to complete, then
// one thread per workgroup adds to a monotone counter (device-scope atomic)
// and polls it; the rows a workgroup reads after the barrier were stored
// coherently and completed before their writers arrived.  A wait gives up
// after spin_limit polls (FLAG_WAIT_TIMEOUT on the problem's matrix; the
// kernel still ends); the host launches cooperatively, so all workgroups are
// resident.  All sums run in a fixed order: reruns give the same bits.
#pragma once
#include "eeid_tridiag.hpp"

namespace eeid {

constexpr int LAT_NT = 256;
constexpr int LAT_NWAVE = LAT_NT / 64;
constexpr int LAT_MAX_PROBLEMS = 16;

struct LatArgs {
    const Item *items;   // P problems
    int P;
    int G;               // workgroups per problem
    char *work;          // per problem: prob_bytes
    int64_t prob_bytes;
    int LD;              // row stride of the stored matrices (doubles)
    unsigned *bar;       // P barrier counters, zero at launch
    int32_t *flags;      // flags[item.b]
    unsigned spin_limit;
};

// Per-problem workspace (doubles): A [m * LD], y [LD], d [LD], e [LD], s2 [2 G]
// (two buffers: column k's partials are read while column k + 1's may already
// be written), dot [G].
__host__ __device__ inline int64_t lat_prob_bytes(int LD, int G) {
    return ((int64_t)LD * LD + 3 * (int64_t)LD + 3 * (int64_t)G) * 8;
}

// LDS (doubles): u and w (2 LD; the bisection's (d, e^2) pairs reuse them),
// then per-wave partial sums.
__host__ __device__ inline int64_t lat_lds_bytes(int LD) { return (2 * (int64_t)LD + 8 * LAT_NWAVE + 16) * 8; }

__device__ __forceinline__ double ld_coh(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct LatGrid {
    unsigned *bar;
    unsigned gen;
    int G;
    bool bail;           // a wait gave up: do not wait again (uniform)
    unsigned spin_limit;
    int32_t *flag;
    unsigned *s_bail;    // LDS word: thread 0's verdict for the workgroup

    // full: also release and acquire every cached global write at agent scope
    // (used once, before the bisection reads the whole tridiagonal)
    __device__ void sync(bool full = false) {
        if (full) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);   // this thread's stores have completed
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned target = (gen + 1) * (unsigned)G;
            unsigned b = bail ? 1u : 0u;
            if (!b) {
                unsigned polls = 0;
                while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                    if (++polls > spin_limit) {
                        b = 1u;
                        atomicOr(flag, FLAG_WAIT_TIMEOUT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            *s_bail = b;
        }
        __syncthreads();
        bail = *s_bail != 0u;
        ++gen;
        if (full) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
};

// Sum of the G per-workgroup partials v[0..G) (global), in a fixed order: one
// load per thread, a fixed reduction tree per wave, the waves in order.  The
// same value in every thread and every workgroup.  part: LDS, >= 2 NWAVE doubles.
__device__ __forceinline__ double grid_sum(const double *v, int G, double *part, int tid, int lane, int wave) {
    double acc = 0.0;
    for (int q = tid; q < G; q += LAT_NT) acc += ld_coh(v + q);
    acc = wave_sum(acc);
    if (lane == 0) part[LAT_NWAVE + wave] = acc;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < LAT_NWAVE; ++w) s += part[LAT_NWAVE + w];
    __syncthreads();
    return s;
}

__global__ __launch_bounds__(LAT_NT) void latency_eig_kernel(LatArgs a) {
    extern __shared__ double lds[];
    __shared__ unsigned s_bail;
    const int p = blockIdx.x / a.G, g = blockIdx.x % a.G;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const Item it = a.items[p];
    const int m = it.m, LD = a.LD, G = a.G;
    if (a.flags[it.b] & 1) {   // non-finite input (uniform over the problem's workgroups)
        for (int i = g * LAT_NT + tid; i < m; i += G * LAT_NT) it.out[i] = __builtin_nan("");
        return;
    }
    double *A = reinterpret_cast<double *>(a.work + (int64_t)p * a.prob_bytes);
    double *y = A + (int64_t)m * LD;
    double *d = y + LD;
    double *e = d + LD;
    double *s2 = e + LD;
    double *dot = s2 + 2 * G;
    double *u = lds, *w = lds + LD;
    double *wpart = lds + 2 * LD;           // per-wave partials (2 NWAVE)
    LatGrid grid{a.bar + p, 0u, G, false, a.spin_limit, &a.flags[it.b], &s_bail};

    // rows of this workgroup: g, g + G, ...; the l-th of them goes to wave l % NWAVE
    auto own_first = [&](int from) { return from + (((g - from) % G) + G) % G; };

    // ---- gather (minor formation by index remap, both triangles) and sigma^2 of column 0
    {
        double part = 0.0;
        for (int i = g; i < m; i += G) {
            const int rs = i + ((it.j >= 0 && i >= it.j) ? 1 : 0);
            for (int c = tid; c < m; c += LAT_NT) {
                const int cs = c + ((it.j >= 0 && c >= it.j) ? 1 : 0);
                const double v = lower_at(it.src, it.n, rs, cs);
                if (i == 0) st_coh(A + c, v);   // row 0: the first pivot row, read by every workgroup
                else A[(int64_t)i * LD + c] = v;
            }
            if (i >= 2 && tid == 0) {
                const int cs0 = (it.j == 0) ? 1 : 0;
                const double x = lower_at(it.src, it.n, rs, cs0);
                part = fma(x, x, part);
            }
        }
        if (tid == 0) st_coh(s2 + g, part);
    }
    grid.sync();

    for (int k = 0; k + 1 < m; ++k) {
        const int t0 = k + 1;   // first row/column of the trailing matrix
        // ---- reflector (every workgroup, same arithmetic in the same order)
        const double sg = grid_sum(s2 + (k & 1) * G, G, wpart, tid, lane, wave);
        const double alpha = ld_coh(A + (int64_t)k * LD + t0);   // A(k + 1, k) = A(k, k + 1)
        double tau = 0.0, scal = 0.0, beta = alpha;
        if (sg != 0.0) {
            const double nrm = sqrt(fma(alpha, alpha, sg));
            beta = (alpha >= 0.0) ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        if (g == 0 && tid == 0) {
            st_coh(e + k, beta);
            st_coh(d + k, ld_coh(A + (int64_t)k * LD + k));   // d_k, final since column k - 1
        }
        const int tn = k + 2;   // column of the next reflector
        if (tau == 0.0) {
            // nothing to eliminate: the trailing matrix is unchanged; sigma^2 of column k + 1
            double part = 0.0;
            if (tid == 0)
                for (int i = own_first(tn + 1); i < m; i += G) {
                    const double x = A[(int64_t)i * LD + t0];
                    part = fma(x, x, part);
                }
            // row k + 1 is the next pivot row: republish it coherently (it was last
            // written as one of its owner's rows)
            if ((t0 % G) == g)
                for (int j = t0 + tid; j < m; j += LAT_NT) st_coh(A + (int64_t)t0 * LD + j, A[(int64_t)t0 * LD + j]);
            __syncthreads();
            if (tid == 0) st_coh(s2 + ((k + 1) & 1) * G + g, part);
            grid.sync();
            continue;
        }
        // u from row k (= column k), in LDS
        for (int j = t0 + tid; j < m; j += LAT_NT) u[j] = (j == t0) ? 1.0 : ld_coh(A + (int64_t)k * LD + j) * scal;
        __syncthreads();
        // ---- y = A22 u on this workgroup's rows; partial u^T y per wave, rows in order
        {
            double acc_dot = 0.0;
            int l = 0;
            for (int i = own_first(t0); i < m; i += G, ++l) {
                if ((l % LAT_NWAVE) != wave) continue;
                const double *Ai = A + (int64_t)i * LD;
                double s[4] = {0.0, 0.0, 0.0, 0.0};
                int j = t0 + lane;
                for (; j + 192 < m; j += 256) {
                    s[0] = fma(Ai[j], u[j], s[0]);
                    s[1] = fma(Ai[j + 64], u[j + 64], s[1]);
                    s[2] = fma(Ai[j + 128], u[j + 128], s[2]);
                    s[3] = fma(Ai[j + 192], u[j + 192], s[3]);
                }
                for (int q = 0; j < m; j += 64, ++q) s[q] = fma(Ai[j], u[j], s[q]);
                const double yi = wave_sum((s[0] + s[1]) + (s[2] + s[3]));
                if (lane == 0) {
                    st_coh(y + i, yi);
                    acc_dot = fma(u[i], yi, acc_dot);
                }
            }
            if (lane == 0) wpart[wave] = acc_dot;
            __syncthreads();
            if (tid == 0) {
                double sum = 0.0;
                for (int q = 0; q < LAT_NWAVE; ++q) sum += wpart[q];
                st_coh(dot + g, sum);
            }
        }
        grid.sync();
        // ---- w = tau y - (tau^2 / 2) (u^T y) u, all of it, in LDS
        {
            const double kap = 0.5 * tau * tau * grid_sum(dot, G, wpart, tid, lane, wave);
            for (int j = t0 + tid; j < m; j += LAT_NT) w[j] = fma(-kap, u[j], tau * ld_coh(y + j));
        }
        __syncthreads();
        // ---- A22 -= u w^T + w u^T on this workgroup's rows; sigma^2 of column k + 1
        {
            double part = 0.0;
            int l = 0;
            for (int i = own_first(t0); i < m; i += G, ++l) {
                if ((l % LAT_NWAVE) != wave) continue;
                double *Ai = A + (int64_t)i * LD;
                const double ui = u[i], wi = w[i];
                const bool pivot = (i == t0);   // next pivot row: every workgroup reads it
                for (int j = t0 + lane; j < m; j += 64) {
                    // two rounded products added: the same value for (i, j) and (j, i)
                    const double upd = __dadd_rn(__dmul_rn(ui, w[j]), __dmul_rn(wi, u[j]));
                    const double v = Ai[j] - upd;
                    if (pivot) st_coh(Ai + j, v);
                    else Ai[j] = v;
                    if (j == t0 && i >= tn + 1) part = fma(v, v, part);
                }
            }
            // only lane 0 (j = t0) holds squares: its rows' column-(k+1) entries, in row order
            const double wsum = wave_sum(part);
            if (lane == 0) wpart[wave] = wsum;
            __syncthreads();
            if (tid == 0) {
                double sum = 0.0;
                for (int q = 0; q < LAT_NWAVE; ++q) sum += wpart[q];
                st_coh(s2 + ((k + 1) & 1) * G + g, sum);
            }
        }
        grid.sync();
    }

    // ---- the tridiagonal (d collected by workgroup 0 column by column, e = the
    // betas); then this workgroup's slice of the eigenvalues
    if (g == 0 && tid == 0) st_coh(d + m - 1, ld_coh(A + (int64_t)(m - 1) * LD + (m - 1)));
    grid.sync(true);
    const int per = (m + G - 1) / G;
    const int i0 = min(m, g * per), i1 = min(m, i0 + per);
    if (i0 < i1) bisect_tridiagonal<LAT_NT, 1>(d, e, m, it.out, lds, wpart, tid, lane, wave, nullptr, i0, i1);
}

__global__ __launch_bounds__(64) void reset_barriers_kernel(unsigned *bar, int P) {
    if ((int)threadIdx.x < P) bar[threadIdx.x] = 0u;
}

}  // namespace eeid
