// Batched eigenvalues of Hermitian matrices and of their principal minors on
// gfx950: one workgroup per (matrix, minor) problem, persistent over a queue.
//
// Per problem (the EigenValues step of Algorithms 1 and 2, Section 3 of the
// paper, applied to A and to each minor M_j of Section 2):
//   1. gather the minor (row j and column j removed) into a tile-packed lower
//      triangle in the workgroup's HBM slot;
//   2. blocked Householder tridiagonalisation Q^T M Q = T (textbook sytrd
//      form, lower storage): per column an update of the column with the
//      panel so far, a Householder reflector, and a symmetric matrix-vector
//      product that streams the stale trailing triangle from HBM once; per
//      panel of NB columns a rank-2NB update of the trailing triangle on MFMA;
//   3. all eigenvalues of T by Sturm-count bisection, FP64, one lane per
//      eigenvalue.
//
// Storage of the trailing matrix (type S = double or float): the lower
// triangle in 64x64 tiles (diagonal tiles hold both triangles).  Tile (I, J),
// I >= J, is at index J*T - J*(J-1)/2 + (I-J) (tile columns contiguous).  In a
// tile, element (r, c) sits at (c / VW) * 64 * VW + r * VW + c % VW with
// VW = 16 / sizeof(S): one 16-byte load gives a lane VW consecutive columns of
// its row, and 64 lanes cover 1 KiB of contiguous memory.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#ifndef EEID_NT_LOADS
#define EEID_NT_LOADS 1
#endif

namespace eeid {

constexpr int TILE = 64;
constexpr int TILE_ELEMS = TILE * TILE;
constexpr int SEG = 8;      // tiles per SYMV work unit (down a tile column)

struct Item {
    const double *src;  // matrix (row-major, lda = n)
    double *out;        // m ascending eigenvalues go here
    int32_t n;          // order of the source matrix
    int32_t j;          // deleted row/column, -1 for the matrix itself
    int32_t m;          // order of the problem (n or n - 1)
    int32_t b;          // batch index (flags)
    int32_t k;          // >= 0: the minor is taken of R^H A R, R a pi/4 rotation in the (j, k) plane
    int32_t rot;        // the rotation: 0 real (e_j + e_k)/sqrt2, 1 imaginary (e_j + i e_k)/sqrt2 (complex input)
};

// Element (p, q) of the symmetric matrix whose lower triangle is A (row-major, order n).
__device__ __forceinline__ double lower_at(const double *A, int n, int p, int q) {
    return (p >= q) ? A[(int64_t)p * n + q] : A[(int64_t)q * n + p];
}

// Element (p, q), p, q != r, of B = R^T A R with R the rotation by pi/4 in the
// (r, k) plane: new basis vectors e'_r = (e_r + e_k)/sqrt2, e'_k = (e_k - e_r)/sqrt2,
// the others unchanged.  B has A's eigenvalues, and component r of its
// eigenvector i is (v_ir + v_ik)/sqrt2, so Eq. (2) applied to B at r gives
// (v_ir + v_ik)^2 / 2 (the identity in another basis, Section 2).  Of the
// minor without row and column r only row and column k differ from A's.
__device__ __forceinline__ double rotated_at(const double *A, int n, int r, int k, int p, int q) {
    constexpr double h = 0.70710678118654752440;   // 1/sqrt2
    if (p == k && q == k) return 0.5 * (lower_at(A, n, k, k) - 2.0 * lower_at(A, n, r, k) + lower_at(A, n, r, r));
    if (p == k) return h * (lower_at(A, n, k, q) - lower_at(A, n, r, q));
    if (q == k) return h * (lower_at(A, n, p, k) - lower_at(A, n, p, r));
    return lower_at(A, n, p, q);
}

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

template <class S> struct Vec;
template <> struct Vec<double> { static constexpr int W = 2; typedef dvec2 type; };
template <> struct Vec<float> { static constexpr int W = 4; typedef fvec4 type; };

// The stale trailing matrix is streamed exactly once per column: its loads
// are non-temporal so they do not displace the panel (V, W) in the caches.
template <class VT>
__device__ __forceinline__ VT stream_load(const VT *p) {
#if EEID_NT_LOADS
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

__device__ __forceinline__ int64_t tile_index(int I, int J, int T) {
    return (int64_t)J * T - (int64_t)J * (J - 1) / 2 + (I - J);
}

template <class S>
__device__ __forceinline__ int tile_off(int r, int c) {
    constexpr int W = Vec<S>::W;
    return (c / W) * (TILE * W) + r * W + (c % W);
}

// ---- cross-lane moves without the LDS crossbar
// Within rows of 16 lanes a DPP move (quad permutations, row mirrors, and the
// one-lane wave shift); across rows the lane-swap instructions of gfx950:
// permlane32 swaps the upper half of its first operand with the lower half of
// its second, permlane16 the odd rows of the first with the even rows of the
// second.  A double moves as two dwords.
enum : int {
    DPP_XOR1 = 0xB1,         // quad_perm [1,0,3,2]: lane l ^ 1
    DPP_XOR2 = 0x4E,         // quad_perm [2,3,0,1]: lane l ^ 2
    DPP_MIRROR = 0x140,      // lane l ^ 15 within a row of 16
    DPP_HALF_MIRROR = 0x141, // lane l ^ 7 within 8
    DPP_WAVE_SHL1 = 0x130,   // lane l + 1 (lane 63 keeps its own value)
};

__device__ __forceinline__ unsigned lo32(double x) { return (unsigned)__builtin_bit_cast(unsigned long long, x); }
__device__ __forceinline__ unsigned hi32(double x) { return (unsigned)(__builtin_bit_cast(unsigned long long, x) >> 32); }
__device__ __forceinline__ double mk64(unsigned lo, unsigned hi) {
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
    const unsigned lo = __builtin_amdgcn_update_dpp(lo32(x), lo32(x), CTRL, 0xf, 0xf, false);
    const unsigned hi = __builtin_amdgcn_update_dpp(hi32(x), hi32(x), CTRL, 0xf, 0xf, false);
    return mk64(lo, hi);
}

// Swap of a's upper 32 lanes with b's lower 32 lanes (OFF = 32) or of a's odd
// rows with b's even rows (OFF = 16).  Afterwards, in every lane, a + b is the
// lane's own a (lower half / even row) or own b (upper half / odd row) plus
// the partner lane's (l ^ OFF) copy of the same operand.
template <int OFF>
__device__ __forceinline__ void lane_swap(double &a, double &b) {
    static_assert(OFF == 16 || OFF == 32, "OFF");
    if constexpr (OFF == 32) {
        const auto l = __builtin_amdgcn_permlane32_swap(lo32(a), lo32(b), false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi32(a), hi32(b), false, false);
        a = mk64(l[0], h[0]); b = mk64(l[1], h[1]);
    } else {
        const auto l = __builtin_amdgcn_permlane16_swap(lo32(a), lo32(b), false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi32(a), hi32(b), false, false);
        a = mk64(l[0], h[0]); b = mk64(l[1], h[1]);
    }
}

// x + x of lane l ^ 32, in every lane.
__device__ __forceinline__ double xsum32(double x) { double a = x, b = x; lane_swap<32>(a, b); return a + b; }
// x of lane l ^ 32.
__device__ __forceinline__ double xswap32(double x, int lane) {
    double a = x, b = x; lane_swap<32>(a, b); return (lane < 32) ? b : a;
}
// x of lane l % 32 (the lower half's copy) and of lane l % 32 + 32 (the upper half's).
__device__ __forceinline__ double from_lower(double x) { double a = x, b = x; lane_swap<32>(a, b); return a; }
__device__ __forceinline__ double from_upper(double x) { double a = x, b = x; lane_swap<32>(a, b); return b; }

// x of lane 0, in every lane.
__device__ __forceinline__ double bcast0(double x) {
    return mk64(__builtin_amdgcn_readlane(lo32(x), 0), __builtin_amdgcn_readlane(hi32(x), 0));
}

// x combined with the copy of a partner lane that differs in bit OFF and in no
// higher bit of the lane index (l ^ OFF for OFF = 32, 16, 2, 1; l ^ 15 for
// OFF = 8, l ^ 7 for OFF = 4).  Applying it for OFF = 32, 16, ..., 1 combines
// all 64 lanes: the partners' offsets 32, 16, 15, 7, 2, 1 span every index.
template <int OFF>
__device__ __forceinline__ double partner(double x) {
    if constexpr (OFF == 8) return dpp_mov<DPP_MIRROR>(x);
    else if constexpr (OFF == 4) return dpp_mov<DPP_HALF_MIRROR>(x);
    else if constexpr (OFF == 2) return dpp_mov<DPP_XOR2>(x);
    else {
        static_assert(OFF == 1, "partner: OFF in {8, 4, 2, 1}");
        return dpp_mov<DPP_XOR1>(x);
    }
}
template <int OFF>
__device__ __forceinline__ double psum(double x) {
    if constexpr (OFF == 32 || OFF == 16) {
        double a = x, b = x;
        lane_swap<OFF>(a, b);
        return a + b;
    } else {
        return x + partner<OFF>(x);
    }
}

// One halving step: lanes with bit OFF set keep the upper half of v[0..CNT),
// the others the lower half, each adding the partner lane's copy of that half
// (the partner differs in bit OFF and no higher bit, so it holds the same
// entries of v).
template <int CNT, int OFF, int N>
__device__ __forceinline__ void halve_step(double (&v)[N], int lane) {
    if constexpr (OFF == 32 || OFF == 16) {
#pragma unroll
        for (int t = 0; t < CNT / 2; ++t) {
            double a = v[t], b = v[CNT / 2 + t];
            lane_swap<OFF>(a, b);
            v[t] = a + b;
        }
    } else {
        const bool hi = (lane & OFF) != 0;
#pragma unroll
        for (int t = 0; t < CNT / 2; ++t) {
            const double keep = hi ? v[CNT / 2 + t] : v[t];
            const double send = hi ? v[t] : v[CNT / 2 + t];
            v[t] = keep + partner<OFF>(send);
        }
    }
}

// Sum v[0..N) over the 64 lanes of a wave by recursive halving.  Returns the
// total of column (lane >> (6 - log2 N)); every lane ends with one column.
template <int N>
__device__ __forceinline__ double wave_transpose_sum(double (&v)[N], int lane) {
    static_assert(N == 8 || N == 16 || N == 32, "N");
    if constexpr (N == 32) halve_step<32, 32>(v, lane);
    if constexpr (N >= 16) halve_step<16, (N == 32 ? 16 : 32)>(v, lane);
    halve_step<8, (N == 32 ? 8 : N == 16 ? 16 : 32)>(v, lane);
    halve_step<4, (N == 32 ? 4 : N == 16 ? 8 : 16)>(v, lane);
    halve_step<2, (N == 32 ? 2 : N == 16 ? 4 : 8)>(v, lane);
    double s = v[0];
    if constexpr (N <= 8) s = psum<4>(s);
    if constexpr (N <= 16) s = psum<2>(s);
    s = psum<1>(s);
    return s;
}

__device__ __forceinline__ double wave_sum(double x) {
    x = psum<32>(x); x = psum<16>(x); x = psum<8>(x); x = psum<4>(x); x = psum<2>(x); x = psum<1>(x);
    return x;
}
template <int OFF>
__device__ __forceinline__ double pmin(double x) {
    if constexpr (OFF == 32 || OFF == 16) { double a = x, b = x; lane_swap<OFF>(a, b); return fmin(a, b); }
    else return fmin(x, partner<OFF>(x));
}
template <int OFF>
__device__ __forceinline__ double pmax(double x) {
    if constexpr (OFF == 32 || OFF == 16) { double a = x, b = x; lane_swap<OFF>(a, b); return fmax(a, b); }
    else return fmax(x, partner<OFF>(x));
}
__device__ __forceinline__ double wave_min(double x) {
    x = pmin<32>(x); x = pmin<16>(x); x = pmin<8>(x); x = pmin<4>(x); x = pmin<2>(x); x = pmin<1>(x);
    return x;
}
__device__ __forceinline__ double wave_max(double x) {
    x = pmax<32>(x); x = pmax<16>(x); x = pmax<8>(x); x = pmax<4>(x); x = pmax<2>(x); x = pmax<1>(x);
    return x;
}

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// Shared scalars of one problem (lives in LDS).
template <int NB>
struct Panel {
    double tau, alpha2, beta, scal, atb;
    double a[NB], b[NB];     // a = W^T u, b = V^T u of the latest column
    double vk[NB], wk[NB];   // row k of V and W for the next column
    double tmp[2 * NB + 8];
};

// All eigenvalues of the symmetric tridiagonal (d, e) ascending, by Sturm
// counts: count(x) = #{i : q_i < 0}, q_0 = d_0 - x, q_i = d_i - x - e_{i-1}^2 / q_{i-1},
// tiny pivots replaced by -pivmin.  Bisection from a widened Gershgorin
// interval stops at ulp level (relative 2 eps, absolute eps ||T||), at most
// 80 halvings.  One lane per eigenvalue, up to ILP eigenvalues per lane in
// lockstep (fewer when the block holds fewer eigenvalues); de (LDS, >= 2m
// doubles) receives (d_i, e_{i-1}^2) pairs, red (LDS) the workgroup reductions.
//
// Two forms of the count.  With every operation correctly rounded (IEEE
// division) the computed count is monotone in x, which makes bisection
// provably converge to eigenvalue k; with e^2 / q taken as e^2 times the
// hardware reciprocal refined by one Newton step (a few ulp off, and about
// twice as fast) it can decrease within a few ulp of an eigenvalue.  The
// halvings use the fast form down to the stopping width; then a bracket of
// four stopping widths on either side of the result is certified by two
// correctly rounded counts (count(lo) <= k < count(hi); where that fails, a
// 64 times wider one or the Gershgorin interval), and correctly rounded
// halvings bring it back to the stopping width.  Every returned eigenvalue
// therefore comes from a bracket certified by the monotone count.
//
// i_begin, i_end: only eigenvalues i_begin .. i_end - 1 are computed (the
// workgroup's share when several share one tridiagonal); default all.  Small
// tridiagonals (all eigenvalues, m <= NT / 2) use multisect_small instead.
//
// brk (optional): the m + 1 ascending eigenvalues of a matrix of which T is
// similar to a principal minor.  By Cauchy interlacing eigenvalue k of the
// minor lies in [brk[k], brk[k + 1]], widened by the rounding pad (checked
// with two counts).  The bracket does not change the result: the halvings
// always follow the path of bisection from the Gershgorin interval, and the
// bracket only lets the halvings whose midpoints fall outside it (by more
// than the fast count's few-ulp error zone) be taken without a count -- the
// count there could only have said what the bracket says.  So a minor's
// eigenvalues have the same bits whether or not its matrix's eigenvalues
// were ready when it started.
// Sturm counts at S points x[t] on the (d_i, e_{i-1}^2) pairs in LDS (de, 2m
// doubles): cnt[t] = #{i : q_i < 0}.  EXACT: e^2 / q by correctly rounded
// division; else e^2 times the hardware reciprocal refined by one Newton
// step.  With few points per lane, four (or two) steps at a time with their
// LDS loads issued first (the loop is otherwise bound by the LDS latency of
// every step); the arithmetic of each point is the same sequence either way.
typedef const __attribute__((address_space(3))) double lds_cdouble;
template <int S, bool EXACT>
__device__ __forceinline__ void sturm_counts(const double *de, int m, const double (&x)[S], int (&cnt)[S],
                                             double pivmin) {
    lds_cdouble *dl = (lds_cdouble *)de;
    double q[S];
#pragma unroll
    for (int t = 0; t < S; ++t) { q[t] = 1.0; cnt[t] = 0; }
    auto step = [&](double d, double e2) {
#pragma unroll
        for (int t = 0; t < S; ++t) {
            double v;
            if constexpr (EXACT) {
                v = (d - x[t]) - e2 / q[t];
            } else {
                double r = __builtin_amdgcn_rcp(q[t]);
                r = fma(fma(-q[t], r, 1.0), r, r);
                v = (d - x[t]) - e2 * r;
            }
            v = (fabs(v) < pivmin) ? -pivmin : v;   // |q| >= pivmin keeps e2 / q finite
            cnt[t] += (v < 0.0) ? 1 : 0;
            q[t] = v;
        }
    };
    constexpr int U = (S <= 2) ? 4 : ((S <= 4) ? 2 : 1);   // eight points hide the latency by themselves
    int i = 0;
    if constexpr (U > 1) {
        for (; i + U <= m; i += U) {
            double d[U], e2[U];
#pragma unroll
            for (int u = 0; u < U; ++u) { d[u] = dl[2 * (i + u)]; e2[u] = dl[2 * (i + u) + 1]; }
#pragma unroll
            for (int u = 0; u < U; ++u) step(d[u], e2[u]);
        }
    }
    for (; i < m; ++i) step(dl[2 * i], dl[2 * i + 1]);
}

template <int NT, int S>
__device__ void bisect_block(int base, int ie, int m, const double *de, double *out, int tid, double gl,
                             double gu, double pad, double pivmin, double atol, const double *brk) {
    constexpr double eps = 2.220446049250313e-16;
    double lo[S], hi[S];
    int idx[S];
    bool done[S];
#pragma unroll
    for (int t = 0; t < S; ++t) {
        idx[t] = base + t * NT + tid;
        lo[t] = gl; hi[t] = gu;
        done[t] = idx[t] >= ie;
    }
    // Sturm counts at S points; EXACT: correctly rounded division
    auto counts = [&](const double (&x)[S], int (&cnt)[S], auto exact) {
        sturm_counts<S, decltype(exact)::value>(de, m, x, cnt, pivmin);
    };
    const std::integral_constant<bool, false> fast{};
    const std::integral_constant<bool, true> exact{};
    auto stop = [&](int t) {
        const double w = hi[t] - lo[t];
        const double mid = 0.5 * (lo[t] + hi[t]);
        return w <= fmax(2.0 * eps * fmax(fabs(lo[t]), fabs(hi[t])), atol) || mid <= lo[t] || mid >= hi[t];
    };
    auto halve = [&](auto form) {
        for (int it = 0; it < 80; ++it) {
            bool all = true;
#pragma unroll
            for (int t = 0; t < S; ++t) all = all && done[t];
            if (all) break;
            double x[S];
            int cnt[S];
#pragma unroll
            for (int t = 0; t < S; ++t) x[t] = 0.5 * (lo[t] + hi[t]);
            counts(x, cnt, form);
#pragma unroll
            for (int t = 0; t < S; ++t) {
                if (done[t]) continue;
                if (cnt[t] > idx[t]) hi[t] = x[t]; else lo[t] = x[t];
                if (stop(t)) done[t] = true;
            }
        }
    };
    if (brk) {
        // the bracket, widened by the rounding pad and the fast count's error zone
        double bl[S], bh[S];
        int cl[S], ch[S];
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const int k = done[t] ? 0 : idx[t];
            bl[t] = fmax(gl, brk[k] - pad);
            bh[t] = fmin(gu, brk[k + 1] + pad);
        }
        counts(bl, cl, fast);
        counts(bh, ch, fast);
        const double zone = 64.0 * eps * fmax(fabs(gl), fabs(gu)) + atol;
#pragma unroll
        for (int t = 0; t < S; ++t) {
            if (done[t] || !(bl[t] < bh[t] && cl[t] <= idx[t] && ch[t] > idx[t])) continue;
            // take the Gershgorin path's halvings whose midpoints lie outside the bracket
            for (int it = 0; it < 80 && !stop(t); ++it) {
                const double x = 0.5 * (lo[t] + hi[t]);
                if (x < bl[t] - zone) lo[t] = x;
                else if (x > bh[t] + zone) hi[t] = x;
                else break;
            }
            if (stop(t)) done[t] = true;
        }
    }
    halve(fast);
    // Certify with the monotone count: a bracket of four stopping widths on
    // either side of the fast result (its endpoints then lie outside the
    // few ulp where the fast count can err), widened 64 times or reset to
    // the Gershgorin interval where that fails; then correctly rounded
    // halvings (three, typically) back to the stopping width.
    {
        int cl[S], ch[S];
        double mid[S], sw[S];
#pragma unroll
        for (int t = 0; t < S; ++t) {
            mid[t] = 0.5 * (lo[t] + hi[t]);
            sw[t] = fmax(2.0 * eps * fmax(fabs(lo[t]), fabs(hi[t])), atol);
            lo[t] = fmax(gl, mid[t] - 4.0 * sw[t]);
            hi[t] = fmin(gu, mid[t] + 4.0 * sw[t]);
        }
        counts(lo, cl, exact);
        counts(hi, ch, exact);
        bool bad = false;
#pragma unroll
        for (int t = 0; t < S; ++t) {
            done[t] = idx[t] >= ie;
            bad = bad || (!done[t] && !(cl[t] <= idx[t] && ch[t] > idx[t]));
        }
        if (__any(bad)) {
            bool ok[S];
#pragma unroll
            for (int t = 0; t < S; ++t) ok[t] = done[t] || (cl[t] <= idx[t] && ch[t] > idx[t]);
            double wl[S], wh[S];
#pragma unroll
            for (int t = 0; t < S; ++t) {
                wl[t] = fmax(gl, mid[t] - 256.0 * sw[t]);
                wh[t] = fmin(gu, mid[t] + 256.0 * sw[t]);
            }
            counts(wl, cl, exact);
            counts(wh, ch, exact);
#pragma unroll
            for (int t = 0; t < S; ++t) {
                if (ok[t]) continue;
                const bool wok = cl[t] <= idx[t] && ch[t] > idx[t];
                lo[t] = wok ? wl[t] : gl;
                hi[t] = wok ? wh[t] : gu;
            }
        }
        halve(exact);
    }
#pragma unroll
    for (int t = 0; t < S; ++t)
        if (idx[t] < ie) out[idx[t]] = 0.5 * (lo[t] + hi[t]);
}

// Small tridiagonals (m <= NT / 2): multisection.  Eigenvalue k gets a group
// of L adjacent lanes (L = 2, 4, 8 or 16, as many as fit), which count at L
// points dividing [lo, hi] into L + 1 equal parts; the first point whose count
// exceeds k and the one before it bound the new interval, so each round gains
// log2(L + 1) bits instead of one (the bisection of one eigenvalue per lane
// leaves most lanes idle for small m).  Same counts, certification and
// bracket use as bisect_block: the rounds follow the path from the Gershgorin
// interval, and a round whose points all lie outside the interlacing bracket
// (beyond the fast count's error zone) is decided without counts.
template <int NT>
__device__ void multisect_small(int m, const double *de, double *out, int tid, int lane, double gl, double gu,
                                double pad, double pivmin, double atol, const double *brk) {
    constexpr double eps = 2.220446049250313e-16;
    const int L = (NT / m >= 16) ? 16 : ((NT / m >= 8) ? 8 : ((NT / m >= 4) ? 4 : 2));
    const int k = tid / L, p = tid % L;
    const bool live = k < m;
    const int kk = live ? k : m - 1;   // idle lanes shadow the last eigenvalue; their results are not stored
    const int gbase = lane & ~(L - 1);
    const unsigned long long gmask = (1ull << L) - 1;
    double lo = gl, hi = gu;
    auto count1 = [&](double x, auto exact) {
        const double xs[1] = {x};
        int cnt[1];
        sturm_counts<1, decltype(exact)::value>(de, m, xs, cnt, pivmin);
        return cnt[0];
    };
    const std::integral_constant<bool, false> fast{};
    const std::integral_constant<bool, true> exact{};
    auto point = [&](int qq) { return lo + (hi - lo) * ((double)(qq + 1) / (double)(L + 1)); };
    auto finished = [&]() {
        const double mid = 0.5 * (lo + hi);
        return (hi - lo) <= fmax(2.0 * eps * fmax(fabs(lo), fabs(hi)), atol) || mid <= lo || mid >= hi;
    };
    double bl = -1e308, bh = 1e308;
    bool fwd = false;
    if (brk) {
        bl = fmax(gl, brk[kk] - pad);
        bh = fmin(gu, brk[kk + 1] + pad);
        const int cl = count1(bl, fast), ch = count1(bh, fast);
        fwd = bl < bh && cl <= kk && ch > kk;   // the same in every lane of the group
    }
    const double zone = 64.0 * eps * fmax(fabs(gl), fabs(gu)) + atol;
    auto rounds = [&](auto form, bool use_fwd) {
        for (int it = 0; it < 80; ++it) {
            const bool fin = finished();
            if (__all(fin)) break;
            const double x = point(p);
            const bool inside = x >= bl - zone && x <= bh + zone;
            const bool known = use_fwd && !((__ballot(inside) >> gbase) & gmask);   // no point of the group inside
            int c = 0;
            if (__any(!known)) c = count1(x, form);
            const bool above = known ? (x > bh + zone) : (c > kk);
            const unsigned long long bits = (__ballot(above) >> gbase) & gmask;
            const int first = bits ? __ffsll((long long)bits) - 1 : L;
            const double nlo = (first == 0) ? lo : point(first - 1);
            const double nhi = (first == L) ? hi : point(first);
            if (!fin) { lo = nlo; hi = nhi; }
        }
    };
    rounds(fast, fwd);
    // certify: a bracket of four stopping widths on either side (every lane of
    // the group counts both ends), else 64 times wider, else Gershgorin; then
    // rounds with correctly rounded counts back to the stopping width
    const double mid = 0.5 * (lo + hi);
    const double sw = fmax(2.0 * eps * fmax(fabs(lo), fabs(hi)), atol);
    double clo = fmax(gl, mid - 4.0 * sw), chi = fmin(gu, mid + 4.0 * sw);
    bool ok = count1(clo, exact) <= kk && count1(chi, exact) > kk;
    if (__any(!ok)) {
        const double wl = fmax(gl, mid - 256.0 * sw), wh = fmin(gu, mid + 256.0 * sw);
        const bool wok = count1(wl, exact) <= kk && count1(wh, exact) > kk;
        if (!ok) {
            clo = wok ? wl : gl;
            chi = wok ? wh : gu;
        }
    }
    lo = clo;
    hi = chi;
    rounds(exact, false);
    if (live && p == 0) out[k] = 0.5 * (lo + hi);
}

template <int NT, int ILP>
__device__ void bisect_tridiagonal(const double *dg, const double *eg, int m, double *out, double *de,
                                   double *red, int tid, int lane, int wave, const double *brk = nullptr,
                                   int i_begin = 0, int i_end = -1) {
    const int ie = (i_end < 0) ? m : i_end;   // eigenvalues i_begin .. ie - 1 (all by default)
    constexpr int NWAVE = NT / 64;
    double gl = 1e308, gu = -1e308, emax2 = 0.0;
    for (int i = tid; i < m; i += NT) {
        const double d = dg[i];
        const double el = (i > 0) ? fabs(eg[i - 1]) : 0.0;
        const double er = (i < m - 1) ? fabs(eg[i]) : 0.0;
        de[2 * i] = d;
        de[2 * i + 1] = el * el;
        gl = fmin(gl, d - el - er);
        gu = fmax(gu, d + el + er);
        emax2 = fmax(emax2, el * el);
    }
    gl = wave_min(gl); gu = wave_max(gu); emax2 = wave_max(emax2);
    if (lane == 0) {
        red[wave * 4 + 0] = gl; red[wave * 4 + 1] = gu; red[wave * 4 + 2] = emax2;
    }
    __syncthreads();
    gl = 1e308; gu = -1e308; emax2 = 0.0;
    for (int w = 0; w < NWAVE; ++w) {
        gl = fmin(gl, red[w * 4]); gu = fmax(gu, red[w * 4 + 1]); emax2 = fmax(emax2, red[w * 4 + 2]);
    }
    const double eps = 2.220446049250313e-16;
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
    const double tnorm = fmax(fabs(gl), fabs(gu));
    const double pad = 2.0 * eps * tnorm * (double)m + 4.0 * pivmin;
    gl -= pad; gu += pad;
    const double atol = eps * tnorm;
    if (i_begin == 0 && ie == m && 2 * m <= NT) {
        multisect_small<NT>(m, de, out, tid, lane, gl, gu, pad, pivmin, atol, brk);
        return;
    }
    for (int base = i_begin; base < ie; base += NT * ILP) {
        // eigenvalues per lane in this block (uniform): no chains for empty slots
        const int slots = min(ILP, (ie - base + NT - 1) / NT);
        if (slots <= 1) bisect_block<NT, 1>(base, ie, m, de, out, tid, gl, gu, pad, pivmin, atol, brk);
        else if (slots <= 2) bisect_block<NT, (ILP < 2 ? ILP : 2)>(base, ie, m, de, out, tid, gl, gu, pad, pivmin, atol, brk);
        else if (slots <= 4) bisect_block<NT, (ILP < 4 ? ILP : 4)>(base, ie, m, de, out, tid, gl, gu, pad, pivmin, atol, brk);
        else bisect_block<NT, ILP>(base, ie, m, de, out, tid, gl, gu, pad, pivmin, atol, brk);
    }
}

// S: storage type of the trailing matrix; NB: panel width; NT: threads per
// workgroup; CW: columns per SYMV work unit (32 or 16); STAGE: stage the
// trailing update's J-side panel rows in LDS; BILP: eigenvalues bisected
// together per lane.
template <class S, int NB, int NT, int CW, bool STAGE, int BILP>
struct Tri {
    static constexpr int NWAVE = NT / 64;

    // slot pointers
    S *tiles;
    double *V, *Wm, *dg, *eg;
    // LDS
    double *y, *u, *red, *stage;  // stage: 2 * NB * 64 doubles for the trailing update
    Panel<NB> *P;
    // problem
    int m, T, LD;
    int tid, lane, wave;

    __device__ S *tile_ptr(int I, int J) const { return tiles + tile_index(I, J, T) * TILE_ELEMS; }

    __device__ double Mget(int r, int c) const {  // stored (stale) entry, r >= c region
        const S *tp = tile_ptr(r / TILE, c / TILE);
        return (double)tp[tile_off<S>(r % TILE, c % TILE)];
    }

    // -------------------------------------------------------------- gather
    __device__ void gather(const Item &it) {
        const int n = it.n, j = it.j;
        const double *A = it.src;
        constexpr int W = Vec<S>::W;
        for (int J = 0; J < T; ++J)
            for (int I = J; I < T; ++I) {
                S *tp = tile_ptr(I, J);
                for (int q = tid; q < TILE_ELEMS; q += NT) {
                    const int cp = q / (TILE * W), rem = q % (TILE * W);
                    const int r = rem / W, c = cp * W + rem % W;
                    const int row = I * TILE + r, col = J * TILE + c;
                    double v = 0.0;
                    if (row < m && col < m) {
                        const int rs = row + ((j >= 0 && row >= j) ? 1 : 0);
                        const int cs = col + ((j >= 0 && col >= j) ? 1 : 0);
                        v = (it.k >= 0) ? rotated_at(A, n, j, it.k, rs, cs) : lower_at(A, n, rs, cs);
                    }
                    tp[q] = (S)v;
                }
            }
    }

    // ---------------------------------------------------- column update (pass A)
    // rows r >= k: finalise W(r, i-1) from the previous column's y, a, b, and
    // form the updated column x_r = M(r,k) - V(r,:) W(k,:)^T - W(r,:) V(k,:)^T.
    // Partial sums of |x|^2 and of W^T x, V^T x over rows >= k+2 go to red[].
    __device__ void column_pass(int k, int i) {
        const double tau_p = P->tau, a2_p = P->alpha2;
        double accp = 0.0, accq = 0.0, sig = 0.0;
        for (int r0 = k; r0 < m; r0 += NT) {
            // keep the panel scalars in LDS (re-read per row) instead of 4*NB hoisted registers
            asm volatile("" ::: "memory");
            const int r = r0 + tid;
            const bool live = r < m;
            double vr[NB], wr[NB];
#pragma unroll
            for (int l = 0; l < NB; ++l) { vr[l] = 0.0; wr[l] = 0.0; }
            if (live) {
                // columns l >= i of the panel are still zero; whole chunks past i are skipped
#pragma unroll
                for (int c = 0; c < NB / 8; ++c) {
                    if (c * 8 < i) {
#pragma unroll
                        for (int l = c * 8; l < c * 8 + 8; ++l) {
                            vr[l] = V[(int64_t)l * LD + r];
                            wr[l] = Wm[(int64_t)l * LD + r];
                        }
                    }
                }
            }
            double x = 0.0;
            if (live) {
                if (i > 0) {
                    double sf = 0.0;
#pragma unroll
                    for (int l = 0; l < NB; ++l) sf = fma(vr[l], P->a[l], fma(wr[l], P->b[l], sf));
                    double vlast = 0.0;
#pragma unroll
                    for (int l = 0; l < NB; ++l) vlast = (l == i - 1) ? vr[l] : vlast;
                    const double wnew = (tau_p != 0.0) ? fma(tau_p, y[r] - sf, a2_p * vlast) : 0.0;
                    if (r > k) Wm[(int64_t)(i - 1) * LD + r] = wnew;  // row k: written by the previous tail
#pragma unroll
                    for (int l = 0; l < NB; ++l) wr[l] = (l == i - 1) ? wnew : wr[l];
                }
                double sx = 0.0;
#pragma unroll
                for (int l = 0; l < NB; ++l) sx = fma(vr[l], P->wk[l], fma(wr[l], P->vk[l], sx));
                x = Mget(r, k) - sx;
                u[r] = x;
                if (r == k) dg[k] = x;
            }
            const double xd = (live && r >= k + 2) ? x : 0.0;
            sig = fma(xd, xd, sig);
            if (i > 0) {
#pragma unroll
                for (int l = 0; l < NB; ++l) wr[l] *= xd;
                accp += wave_transpose_sum<NB>(wr, lane);
#pragma unroll
                for (int l = 0; l < NB; ++l) vr[l] *= xd;
                accq += wave_transpose_sum<NB>(vr, lane);
            }
        }
        sig = wave_sum(sig);
        constexpr int SH = (NB == 32) ? 1 : (NB == 16) ? 2 : 3;
        if ((lane & ((1 << SH) - 1)) == 0) {
            const int c = lane >> SH;
            red[wave * (2 * NB + 8) + c] = accp;
            red[wave * (2 * NB + 8) + NB + c] = accq;
        }
        if (lane == 0) red[wave * (2 * NB + 8) + 2 * NB] = sig;
    }

    // Finalise W(r, i) for rows r >= r_lo with the current column's y, a, b.
    __device__ void finalize_pass(int r_lo, int i) {
        const double tau = P->tau, a2 = P->alpha2;
        for (int r = r_lo + tid; r < m; r += NT) {
            double sf = 0.0;
            for (int l = 0; l < i; ++l)
                sf = fma(V[(int64_t)l * LD + r], P->a[l], fma(Wm[(int64_t)l * LD + r], P->b[l], sf));
            const double vl = V[(int64_t)i * LD + r];
            Wm[(int64_t)i * LD + r] = (tau != 0.0) ? fma(tau, y[r] - sf, a2 * vl) : 0.0;
        }
    }

    // ------------------------------------------------------------------- SYMV
    // y(r) += sum_c M(r, c) u(c) over the stale trailing triangle, each stored
    // element read once and used twice (row product and column product).  A
    // unit is CW columns of tile column J over tile rows [Ib, Ie); lane = row.
    typedef typename Vec<S>::type VT;
    static constexpr int VW = Vec<S>::W;
    static constexpr int NV = CW / VW;  // 16-byte vectors per lane per tile

    // Tiles loaded together per step: an FP32 tile row is half as many bytes,
    // so two tiles keep as many bytes in flight per wave as one FP64 tile.
    static constexpr int UT = (sizeof(S) == 4) ? 2 : 1;

    __device__ void symv_unit(int J, int h, int Ib, int Ie, int k) {
        const int c0 = J * TILE + h * CW;
        // Columns left of the trailing matrix are loaded too (one base address,
        // immediate offsets, all loads in flight together): they meet u = 0 in
        // the row product, and their column sums land in entries of y that are
        // never read.
        double pc[CW];
#pragma unroll
        for (int c = 0; c < CW; ++c) pc[c] = 0.0;
        for (int I = Ib; I < Ie; I += UT) {
            VT buf[UT][NV];
            // Only the first tile of a step can hold rows <= k (tile J0); they
            // are not loaded.  A missing last tile of a step re-reads the
            // step's first tile and is not used.
            // The unconditional loads go first: loads under the lane condition
            // make the compiler wait for every outstanding load before any
            // later load that reuses a register.
#pragma unroll
            for (int t = 1; t < UT; ++t) {
                const S *tp = tile_ptr(min(I + t, Ie - 1), J) + h * (CW * TILE);
#pragma unroll
                for (int q = 0; q < NV; ++q) buf[t][q] = stream_load(reinterpret_cast<const VT *>(tp + q * (TILE * VW) + lane * VW));
            }
            const bool live0 = I * TILE + lane > k;
            if (live0) {
                const S *tp = tile_ptr(I, J) + h * (CW * TILE);
#pragma unroll
                for (int q = 0; q < NV; ++q) buf[0][q] = stream_load(reinterpret_cast<const VT *>(tp + q * (TILE * VW) + lane * VW));
            } else {
#pragma unroll
                for (int q = 0; q < NV; ++q) buf[0][q] = VT{};
            }
#pragma unroll
            for (int t = 0; t < UT; ++t) {
                if (t > 0 && I + t >= Ie) break;
                int uo = c0;
                asm volatile("" : "+v"(uo));  // u(c0 .. c0+CW) is re-read from LDS, not held in registers
                const double2 *uj2 = reinterpret_cast<const double2 *>(u + uo);
                const int row = (I + t) * TILE + lane;
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < NV; ++q)
#pragma unroll
                    for (int z = 0; z < VW; z += 2) {
                        const double2 w = uj2[(q * VW + z) / 2];
                        s = fma((double)buf[t][q][z], w.x, s);
                        s = fma((double)buf[t][q][z + 1], w.y, s);
                    }
                if (I + t != J) {
                    const double ui = u[row];
#pragma unroll
                    for (int q = 0; q < NV; ++q)
#pragma unroll
                        for (int z = 0; z < VW; ++z) pc[q * VW + z] = fma((double)buf[t][q][z], ui, pc[q * VW + z]);
                }
                if (t > 0 || live0) atomicAdd(&y[row], s);
            }
        }
        if (Ie > Ib + (Ib == J ? 1 : 0)) {  // some off-diagonal tile contributed column sums
            constexpr int SH = (CW == 32) ? 1 : 2;
            const double tot = wave_transpose_sum<CW>(pc, lane);
            if ((lane & ((1 << SH) - 1)) == 0) atomicAdd(&y[c0 + (lane >> SH)], tot);
        }
    }

    // Work units (tile column J, half h, run of up to SEG tiles down the column)
    // are dealt to the waves longest first in snake order (0..7, 7..0, ...),
    // which keeps the waves within a few percent of each other.
    __device__ void symv(int k) {
        const int J0 = (k + 1) / TILE;
        int cnt = 0;
        auto take = [&](int J, int h, int Ib, int Ie) {
            const int r = cnt / NWAVE, c = cnt % NWAVE;
            const int w = (r & 1) ? (NWAVE - 1 - c) : c;
            ++cnt;
            if (w == wave) symv_unit(J, h, Ib, Ie, k);
        };
        // full-length runs
        for (int J = J0; J < T; ++J)
            for (int h = 0; h < TILE / CW; ++h) {
                if (J * TILE + h * CW + CW - 1 < k + 1) continue;
                for (int s0 = J; s0 + SEG <= T; s0 += SEG) take(J, h, s0, s0 + SEG);
            }
        // the shorter tail runs, longest first
        for (int L = SEG - 1; L >= 1; --L)
            for (int J = T - L; J >= J0; J -= SEG)
                for (int h = 0; h < TILE / CW; ++h) {
                    if (J * TILE + h * CW + CW - 1 < k + 1) continue;
                    take(J, h, T - L, T);
                }
    }

    // ------------------------------------------------------------------ SYR2K
    // C(I, J) -= V_I W_J^T + W_I V_J^T for the trailing tiles J >= J1 (MFMA).
    // C(I, J) -= V_I W_J^T + W_I V_J^T on MFMA.  The J-side panel rows (V_J,
    // W_J) come from LDS (staged once per tile column for all waves, column k
    // of the panel at vs[k*64 + row]); the I-side rows are loaded from the slot
    // once per tile.  Two passes of two 16-row blocks keep 8 accumulators live.
    // SLD = TILE: vs/ws are the LDS copies (column k at vs[k*64 + row]);
    // SLD = 0: vs/ws point at row J*64 of the slot's V/W (column k at k*LD).
    template <int SLD>
    __device__ void syr2k_tile(int I, int J, const double *vs, const double *ws) {
        S *tp = tile_ptr(I, J);
        const int lr = lane & 15, lk = lane >> 4;
        const double *vI = V + I * TILE + lr, *wI = Wm + I * TILE + lr;
#pragma unroll 1
        for (int ip = 0; ip < 4; ip += 2) {
            if constexpr (sizeof(S) == 8) {
                dbl4 acc[4][2];  // [jb][ib - ip]
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib) acc[jb][ib] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
                for (int kk = 0; kk < NB; kk += 4) {
                    const int64_t col = (int64_t)(kk + lk) * LD;
                    const int64_t sc = (int64_t)(kk + lk) * (SLD ? SLD : LD) + lr;
                    double aw[4], av[4], bv[2], bw[2];
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        bv[q] = vI[col + (ip + q) * 16];
                        bw[q] = wI[col + (ip + q) * 16];
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) { aw[q] = ws[sc + q * 16]; av[q] = vs[sc + q * 16]; }
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                        for (int ib = 0; ib < 2; ++ib)
                            acc[jb][ib] = __builtin_amdgcn_mfma_f64_16x16x4f64(aw[jb], bv[ib], acc[jb][ib], 0, 0, 0);
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                        for (int ib = 0; ib < 2; ++ib)
                            acc[jb][ib] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[jb], bw[ib], acc[jb][ib], 0, 0, 0);
                }
                // The f64 16x16x4 result holds element (lk + 4g, lr) of the block in
                // lane (lr + 16 lk), register g: acc[jb][ib][g] = dC(ib*16 + lr, jb*16 + lk + 4g).
#pragma unroll
                for (int ib = 0; ib < 2; ++ib) {
                    const int row = (ip + ib) * 16 + lr;
                    double c[4][4];
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                        for (int g = 0; g < 4; ++g)
                            c[jb][g] = __builtin_nontemporal_load(&tp[tile_off<S>(row, jb * 16 + lk + 4 * g)]);
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                        for (int g = 0; g < 4; ++g)
                            __builtin_nontemporal_store(c[jb][g] - acc[jb][ib][g], &tp[tile_off<S>(row, jb * 16 + lk + 4 * g)]);
                }
            } else {
                flt4 acc[4][2];
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib) acc[jb][ib] = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
                for (int kk = 0; kk < NB; kk += 4) {
                    const int64_t col = (int64_t)(kk + lk) * LD;
                    const int64_t sc = (int64_t)(kk + lk) * (SLD ? SLD : LD) + lr;
                    float aw[4], av[4], bv[2], bw[2];
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        bv[q] = (float)vI[col + (ip + q) * 16];
                        bw[q] = (float)wI[col + (ip + q) * 16];
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) { aw[q] = (float)ws[sc + q * 16]; av[q] = (float)vs[sc + q * 16]; }
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                        for (int ib = 0; ib < 2; ++ib)
                            acc[jb][ib] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw[jb], bv[ib], acc[jb][ib], 0, 0, 0);
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                        for (int ib = 0; ib < 2; ++ib)
                            acc[jb][ib] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[jb], bw[ib], acc[jb][ib], 0, 0, 0);
                }
                // The f32 16x16x4 result holds element (4 lk + g, lr) of the block in
                // lane (lr + 16 lk), register g: acc[jb][ib][g] = dC(ib*16 + lr, jb*16 + 4 lk + g).
#pragma unroll
                for (int ib = 0; ib < 2; ++ib) {
                    const int row = (ip + ib) * 16 + lr;
                    fvec4 c[4];
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb)
                        c[jb] = __builtin_nontemporal_load(reinterpret_cast<const fvec4 *>(tp + tile_off<S>(row, jb * 16 + 4 * lk)));
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb)
                        __builtin_nontemporal_store(c[jb] - acc[jb][ib],
                                                    reinterpret_cast<fvec4 *>(tp + tile_off<S>(row, jb * 16 + 4 * lk)));
                }
            }
        }
    }

    // Trailing update of the tiles J >= J1.  With STAGE, one tile column at a
    // time with its J-side panel rows in LDS; otherwise every wave takes whole
    // tiles and reads both sides from the slot (ld = LD).
    __device__ void syr2k(int J1) {
        if constexpr (STAGE) {
            double *vs = stage, *ws = stage + NB * TILE;
            for (int J = J1; J < T; ++J) {
                for (int q = tid; q < NB * TILE; q += NT) {
                    const int kc = q / TILE, r = q % TILE;
                    vs[q] = V[(int64_t)kc * LD + J * TILE + r];
                    ws[q] = Wm[(int64_t)kc * LD + J * TILE + r];
                }
                __syncthreads();
                for (int I = J + wave; I < T; I += NWAVE) syr2k_tile<TILE>(I, J, vs, ws);
                __syncthreads();
            }
        } else {
            int cnt = 0;
            for (int J = J1; J < T; ++J)
                for (int I = J; I < T; ++I)
                    if ((cnt++ % NWAVE) == wave) syr2k_tile<0>(I, J, V + J * TILE, Wm + J * TILE);
        }
    }

    // --------------------------------------------------------- tridiagonalise
    __device__ void tridiagonalize() {
        for (int r = tid; r < LD; r += NT) u[r] = 0.0;
        if (tid < NB) { P->vk[tid] = 0.0; P->wk[tid] = 0.0; P->a[tid] = 0.0; P->b[tid] = 0.0; }
        if (tid == 0) { P->tau = 0.0; P->alpha2 = 0.0; }
        __syncthreads();
        for (int k0 = 0; k0 < m; k0 += NB) {
            const int nbe = min(NB, m - k0);
            {   // clear the panel's V and W from the first tile row the update can touch
                const int rz = (k0 / TILE) * TILE, len = LD - rz;
                for (int q = tid; q < NB * len; q += NT) {
                    const int l = q / len, r = rz + q % len;
                    V[(int64_t)l * LD + r] = 0.0;
                    Wm[(int64_t)l * LD + r] = 0.0;
                }
            }
            __syncthreads();
            for (int i = 0; i < nbe; ++i) {
                const int k = k0 + i;
                column_pass(k, i);
                __syncthreads();
                if (k == m - 1) break;  // last diagonal entry: no reflector
                // -------- reflector (wave 0)
                if (wave == 0) {
                    // lane l < 2NB: p_l (l < NB) or q_{l-NB}; sigma^2 read by every lane
                    double s = 0.0, sig = 0.0;
                    for (int w = 0; w < NWAVE; ++w) {
                        if (lane < 2 * NB) s += red[w * (2 * NB + 8) + lane];
                        sig += red[w * (2 * NB + 8) + 2 * NB];
                    }
                    const double pl = __shfl(s, lane & (NB - 1));
                    const double ql = __shfl(s, NB + (lane & (NB - 1)));
                    const double alpha = u[k + 1];
                    double beta, tau, scal;
                    if (sig == 0.0) {
                        beta = alpha; tau = 0.0; scal = 0.0;
                    } else {
                        const double nrm = sqrt(fma(alpha, alpha, sig));
                        beta = (alpha >= 0.0) ? -nrm : nrm;
                        tau = (beta - alpha) / beta;
                        scal = 1.0 / (alpha - beta);
                    }
                    double al = 0.0, bl = 0.0;
                    if (lane < i) {
                        al = Wm[(int64_t)lane * LD + k + 1] + scal * pl;
                        bl = V[(int64_t)lane * LD + k + 1] + scal * ql;
                    }
                    const double atb = wave_sum(al * bl);
                    if (lane < NB) { P->a[lane] = al; P->b[lane] = bl; }
                    if (lane == 0) {
                        P->tau = tau; P->beta = beta; P->scal = scal; P->atb = atb;
                        eg[k] = beta;
                    }
                }
                __syncthreads();
                const double tau = P->tau, scal = P->scal;
                // -------- u = [0..0, 1, x(k+2:) * scal], V(:, i) = u, y = 0
                for (int r = k + tid; r < LD; r += NT) {
                    double v = 0.0;
                    if (r == k + 1) v = 1.0;
                    else if (r > k + 1 && r < m) v = u[r] * scal;
                    u[r] = v;
                    if (r > k) V[(int64_t)i * LD + r] = v;
                }
                for (int r = ((k + 1) / TILE) * TILE + tid; r < LD; r += NT) y[r] = 0.0;
                __syncthreads();
                if (tau != 0.0) symv(k);
                __syncthreads();
                // -------- alpha2 = -tau^2 (y^T u - 2 a^T b) / 2
                {
                    double s = 0.0;
                    for (int r = k + 1 + tid; r < m; r += NT) s = fma(y[r], u[r], s);
                    s = wave_sum(s);
                    if (lane == 0) red[wave * (2 * NB + 8) + 2 * NB + 1] = s;
                }
                __syncthreads();
                if (wave == 0) {
                    double s = 0.0;
                    for (int w = 0; w < NWAVE; ++w) s += red[w * (2 * NB + 8) + 2 * NB + 1];
                    const double a2 = -0.5 * tau * tau * (s - 2.0 * P->atb);
                    // W(k+1, i) and row k+1 of V, W for the next column
                    const int kn = k + 1;
                    double vn = 0.0, wn = 0.0;
                    if (lane < i) {
                        vn = V[(int64_t)lane * LD + kn];
                        wn = Wm[(int64_t)lane * LD + kn];
                    }
                    const double sf = wave_sum(lane < i ? fma(vn, P->a[lane], wn * P->b[lane]) : 0.0);
                    const double wkn = (tau != 0.0) ? fma(tau, y[kn] - sf, a2) : 0.0;
                    if (lane < NB) {
                        P->vk[lane] = (lane < i) ? vn : (lane == i ? 1.0 : 0.0);
                        P->wk[lane] = (lane < i) ? wn : (lane == i ? wkn : 0.0);
                    }
                    if (lane == 0) {
                        P->alpha2 = a2;
                        Wm[(int64_t)i * LD + kn] = wkn;
                    }
                }
                __syncthreads();
            }
            // -------- finish the panel: last W column, then the trailing update
            const int klast = k0 + nbe - 1;
            if (klast < m - 1) {
                finalize_pass(klast + 2, nbe - 1);
                __syncthreads();
                const int J1 = (k0 + nbe) / TILE;
                syr2k(J1);
                __syncthreads();
                if (tid < NB) { P->vk[tid] = 0.0; P->wk[tid] = 0.0; }
                __syncthreads();
            }
        }
    }

    // ------------------------------------------------------------- bisection
    __device__ void bisect(double *out, const double *brk) {
        bisect_tridiagonal<NT, BILP>(dg, eg, m, out, y, red, tid, lane, wave, brk);
    }
};

// Phase timers (built with -DEEID_PHASE_TIMERS only): thread 0 of every
// workgroup measures each phase of each problem with the constant 100 MHz
// wall clock and adds the ticks into phase_ticks[] once per problem.  Phases:
// 0 gather, 1 panel QR, 2 symmetric product, 3 W, 4 rank-2k update (with the
// panel's bookkeeping), 5 band to tridiagonal, 6 bisection (with the wait for
// the interlacing brackets), 7 queue and the rest.  The sums over workgroups
// divided by the resident workgroups give each phase's share of the launch.
#ifdef EEID_PHASE_TIMERS
__device__ unsigned long long phase_ticks[8];
struct PhaseClock {
    unsigned long long t = 0, acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    __device__ void start() { if (threadIdx.x == 0) t = wall_clock64(); }
    __device__ void mark(int q) {
        if (threadIdx.x == 0) {
            const unsigned long long now = wall_clock64();
            acc[q] += now - t;
            t = now;
        }
    }
    __device__ void flush() {
        if (threadIdx.x == 0)
            for (int q = 0; q < 8; ++q) atomicAdd(&phase_ticks[q], acc[q]);
    }
};
#define EEID_PHASE_MARK(clk, q) (clk).mark(q)
#else
struct PhaseClock {
    __device__ void start() {}
    __device__ void mark(int) {}
    __device__ void flush() {}
};
#define EEID_PHASE_MARK(clk, q) ((void)0)
#endif

struct TriArgs {
    const Item *items;
    int64_t n_items;
    int *counter;
    int32_t *flags;
    char *work;
    int64_t slot_bytes;
    int LDmax;
    // per batch: address of the matrix's own eigenvalues once they are final,
    // else 0 (cleared before every launch)
    unsigned long long *lam_ready;
    // polls after which a wave waiting for another wave of its workgroup gives
    // up (bounded waits: the problem is then flagged, and the kernel still ends)
    unsigned spin_limit;
};

// flags bit of a problem whose bounded inter-wave wait gave up (its outputs are invalid)
constexpr int32_t FLAG_WAIT_TIMEOUT = 4;

// Bracket source for the bisection of item `it`: the eigenvalues of its
// matrix if it is a plain minor and they are final already (published by the
// workgroup that computed them), else nullptr.  The bracket only saves
// halvings; the result is the same either way (bisect_block), so whether the
// eigenvalues were ready in time does not change any bit.  Uniform over the
// workgroup; s_flag is LDS scratch.
__device__ inline const double *interlacing_bracket(const TriArgs &a, const Item &it, unsigned long long *s_flag) {
    if (it.j < 0 || it.k >= 0) return nullptr;
    if (threadIdx.x == 0)
        *s_flag = __hip_atomic_load(&a.lam_ready[it.b], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const unsigned long long p = *s_flag;
    __syncthreads();
    if (p == 0) return nullptr;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return reinterpret_cast<const double *>(p);
}

// After the eigenvalues of a matrix (it.j < 0) are stored: publish them.
__device__ inline void publish_eigenvalues(const TriArgs &a, const Item &it) {
    if (it.j >= 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(&a.lam_ready[it.b], (unsigned long long)it.out, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <class S, int NB>
__host__ __device__ inline int64_t slot_bytes_for(int LDmax) {
    const int64_t T = LDmax / TILE;
    const int64_t tiles = T * (T + 1) / 2 * TILE_ELEMS * (int64_t)sizeof(S);
    const int64_t panel = 2 * (int64_t)NB * LDmax * 8;
    const int64_t de = 2 * (int64_t)LDmax * 8;
    return ((tiles + 255) / 256) * 256 + panel + de;
}

template <int NB, int NT, bool STAGE>
__host__ __device__ inline int64_t lds_bytes_for(int LDmax) {
    return (2 * (int64_t)LDmax + (NT / 64) * (2 * NB + 8) + (STAGE ? 2 * NB * TILE : 0)) * 8 +
           (int64_t)sizeof(Panel<NB>) + 64;
}

// WPE waves per SIMD: the register budget is 512 / WPE per lane, and the
// HBM bytes a CU keeps in flight grow with WPE (the SYMV is latency-bound per
// wave).  NT = 512 with WPE = 2 is one problem per CU; NT = 256 runs
// 4 * WPE / 4 problems per CU, overlapping the latency-bound phases of one
// problem with the HBM stream of the others.
template <class S, int NB, int NT, int CW, bool STAGE, int WPE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void tridiag_bisect_kernel(TriArgs args) {
    extern __shared__ double lds[];
    __shared__ int s_item;
    __shared__ unsigned long long s_flag;
    Tri<S, NB, NT, CW, STAGE, (WPE >= 3 ? 2 : 4)> t;
    t.tid = threadIdx.x;
    t.lane = threadIdx.x & 63;
    t.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: keep in an SGPR
    const int LDmax = args.LDmax;
    t.y = lds;
    t.u = lds + LDmax;
    t.red = lds + 2 * LDmax;
    t.stage = t.red + (NT / 64) * (2 * NB + 8);
    t.P = reinterpret_cast<Panel<NB> *>(t.stage + (STAGE ? 2 * NB * TILE : 0));
    char *slot = args.work + (int64_t)blockIdx.x * args.slot_bytes;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(args.counter, 1);
        __syncthreads();
        const int64_t it_idx = __builtin_amdgcn_readfirstlane(s_item);  // uniform: scalar loads of the item
        __syncthreads();
        if (it_idx >= args.n_items) break;
        const Item it = args.items[it_idx];
        if (args.flags[it.b] & 1) {  // non-finite input: NaN out
            for (int i = threadIdx.x; i < it.m; i += NT) it.out[i] = __builtin_nan("");
            continue;
        }
        t.m = it.m;
        t.T = (it.m + TILE - 1) / TILE;
        t.LD = t.T * TILE;
        t.tiles = reinterpret_cast<S *>(slot);
        const int64_t T = t.T;
        const int64_t tile_bytes = ((T * (T + 1) / 2 * TILE_ELEMS * (int64_t)sizeof(S) + 255) / 256) * 256;
        t.V = reinterpret_cast<double *>(slot + tile_bytes);
        t.Wm = t.V + (int64_t)NB * t.LD;
        t.dg = t.Wm + (int64_t)NB * t.LD;
        t.eg = t.dg + t.LD;
        t.gather(it);
        __syncthreads();
        t.tridiagonalize();
        __syncthreads();
        t.bisect(it.out, interlacing_bracket(args, it, &s_flag));
        publish_eigenvalues(args, it);
        __syncthreads();
    }
}

}  // namespace eeid
