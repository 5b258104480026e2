// Two-stage tridiagonalisation of real symmetric problems on gfx950, for the
// EigenValues step of Algorithms 1 and 2 (Section 3 of the paper), applied to
// A and to each principal minor M_j (Section 2).  One workgroup per problem,
// persistent over the same queue as the one-stage kernel of eeid_tridiag.hpp.
//
//   stage 1, dense -> band of half-bandwidth BW: per panel of BW columns a
//     Householder QR of the panel below the band (left-looking, compact WY
//     form I - V T V^T), then the two-sided update of the trailing matrix
//     A22 <- Q^T A22 Q = A22 - V W^T - W V^T with Y = A22 V (two MFMA passes
//     over the stored lower triangle), X = Y T, W = X - 1/2 V (T^T V^T X);
//     with an FP64 trailing matrix the panels go in pairs that share one
//     update (see reduce_to_band);
//   stage 2, band -> tridiagonal by Householder bulge chasing: sweep s removes
//     column s below the subdiagonal; each step of a sweep applies the
//     previous reflector from the right to the BW x BW block below it,
//     annihilates the first column of the bulge this creates and applies the
//     new reflector to the rest of that block and two-sidedly to the next
//     diagonal block;
//   then all eigenvalues of the tridiagonal by the Sturm bisection of the
//   one-stage kernel.
//
// The one-stage reduction streams the whole trailing triangle from HBM once
// per column; here it is read twice per panel of BW columns for the SYMM and
// read and written once per pair of panels (once per panel with an FP32
// trailing matrix) for the update, so HBM traffic drops by about BW / 3.
// Both stages are orthogonal similarities, so the eigenvalues are those of
// the problem up to backward-stable rounding.
//
// Trailing-matrix storage (S = double or float): the lower triangle in 64x64
// tiles as in eeid_tridiag.hpp, but inside a tile 8x4 micro-tiles (8 rows,
// 4 columns, column-major inside), micro-tile (mr, mc) at (mc * 8 + mr) * 32:
// element (r, c) at ((c / 4) * 8 + r / 8) * 32 + (c % 4) * 8 + r % 8.  The
// operands of one matrix-core step are then whole micro-tiles in every pass:
// 32 rows x 4 columns (row pass: 1 KiB contiguous), 8 rows x 16 columns
// (column pass: four 256-byte runs), 16 rows x 4 columns (update: 512 bytes).
// Band storage: column c holds A(c + d, c), d in [0, 2 BW), at bnd[c * BLD + d]
// (the chase leaves fill up to d = 2 BW - 1 during a step), for LD + BW
// columns; entries outside the matrix stay zero.  The trailing
// matrix is streamed with non-temporal accesses so that it does not evict the
// band, V and W of the problems in the chase from L2.
#pragma once
#include "eeid_tridiag.hpp"

namespace eeid {

constexpr int BW = 32;        // half-bandwidth of the intermediate band = panel width
constexpr int BLD = 2 * BW;   // band storage per column

__device__ __forceinline__ int mtile_off(int r, int c) {
    return (((c >> 2) << 3) + (r >> 3)) * 32 + ((c & 3) << 3) + (r & 7);
}

template <class S, int NT>
struct Band {
    static constexpr int NWAVE = NT / 64;
    static constexpr int RED = 2 * BW + 8;

    S *tiles;
    double *V, *Wm, *bnd, *dg, *eg;    // slot; V, Wm: the current panel's columns of V0, W0
    double *V0, *W0;                   // slot: V and W of a pair of panels (2 BW columns each; FP32: BW)
    double *Tm, *Mm, *Nm;              // LDS: T, V^T X, T^T V^T X (BW x BW each); SYR2K staging from Tm on
    double *red, *vec;                 // LDS: per-wave partial sums, small vectors
    double *de;                        // LDS: bisection (aliases the stage-1 and chase region)
    int m, T, LD;
    int tid, lane, wave;
    PhaseClock clk;

    __device__ S *tile_ptr(int I, int J) const { return tiles + tile_index(I, J, T) * TILE_ELEMS; }
    __device__ double Mget(int r, int c) const {
        return (double)tile_ptr(r >> 6, c >> 6)[mtile_off(r & 63, c & 63)];
    }

    // -------------------------------------------------------------- gather
    __device__ void gather(const Item &it) {
        const int n = it.n, j = it.j;
        const double *A = it.src;
        for (int J = 0; J < T; ++J)
            for (int I = J; I < T; ++I) {
                S *tp = tile_ptr(I, J);
                for (int q = tid; q < TILE_ELEMS; q += NT) {
                    const int mt = q >> 5, in = q & 31;   // micro-tile, element inside it
                    const int r = ((mt & 7) << 3) + (in & 7), c = ((mt >> 3) << 2) + (in >> 3);
                    const int row = I * TILE + r, col = J * TILE + c;
                    double v = 0.0;
                    if (row < m && col < m) {
                        const int rs = row + ((j >= 0 && row >= j) ? 1 : 0);
                        const int cs = col + ((j >= 0 && col >= j) ? 1 : 0);
                        v = (it.k >= 0) ? rotated_at(A, n, j, it.k, rs, cs) : lower_at(A, n, rs, cs);
                    }
                    __builtin_nontemporal_store((S)v, tp + q);
                }
            }
        for (int q = tid; q < (LD + BW) * BLD; q += NT) bnd[q] = 0.0;
    }

    // ------------------------------------------------------------ panel QR
    // Block reduction of per-row products: lanes of every wave end with one
    // column sum each (wave_transpose_sum); the column sums of all waves go to
    // red[w * RED + off + c].
    __device__ void to_red(double acc, int off) {
        if ((lane & 1) == 0) red[wave * RED + off + (lane >> 1)] = acc;
    }

    // Left-looking Householder QR of P = A(r0:m, k0:k0+BW), r0 = k0 + BW, in
    // compact WY form I - V T V^T.  Column c is brought up to date with the
    // reflectors 0..c-1 of the panel, x_c = P(:,c) - V T^T V^T P(:,c), and
    // reflector c annihilates x_c below row r0 + c: v_c = e_{r0+c} + s_c x_c(below)
    // with s_c = 1 / (alpha - beta).  One pass over the rows per column forms
    // x_c and, looking ahead, every sum the next column needs:
    //   V^T P(:,c+1) for columns 0..c-1 of V, and x_c(below) . P(:,c+1) (gives
    //   v_c . P(:,c+1) once s_c is known);
    //   V^T x_c(below) (gives V^T v_c, hence column c of T).
    // One block barrier per column; every wave then forms reflector c, column c
    // of T and t = T^T V^T P(:,c+1) itself.  R goes to the band, v_c to V(:, c)
    // (written by the owner of each row at the start of the next pass), T to
    // LDS.
    // sum over the wave of vr[l] * x for l < N, transposed: lane l ends with
    // column l >> (6 - log2 N)
    template <int N>
    __device__ __forceinline__ double part_sum(const double (&vr)[BW], double x) const {
        double w[N];
#pragma unroll
        for (int l = 0; l < N; ++l) w[l] = vr[l] * x;
        return wave_transpose_sum<N>(w, lane);
    }

    __device__ void panel_qr(int k0) {
        const int r0 = k0 + BW;
        double *zt = Nm + wave * 2 * BW;   // this wave's z = V^T P(:, c+1) and t = T^T z
        double scal_p = 0.0;               // s_{c-1} (uniform)
        if (lane < 2 * BW) zt[lane] = 0.0;
        __builtin_amdgcn_wave_barrier();
#pragma unroll 1
        for (int c = 0; c < BW; ++c) {
            const bool more = c + 1 < BW;
            // partial sums and scalars alternate between two LDS buffers by column
            // parity, so one barrier per column suffices: a wave writes the other
            // buffer while slower waves still read this one
            double *rd = (c & 1) ? Mm : red;
            double *sc = vec + 64 + (c & 1) * 40;  // [0] alpha_c, [1] P(r0+c, c+1), [2..) V(r0+c, 0..c-1)
            double accq = 0.0, accg = 0.0, sig = 0.0, dx = 0.0;
            for (int r0i = r0; r0i < m; r0i += NT) {
                asm volatile("" ::: "memory");
                const int r = r0i + tid;
                const bool live = r < m;
                const int rl = live ? r : r0;
                // v_{c-1} at this row (x_{c-1} was kept in Wm(:, c-1))
                double vprev = 0.0;
                if (c > 0 && live && r >= r0 + c - 1) {
                    vprev = (r == r0 + c - 1) ? 1.0 : Wm[(int64_t)(c - 1) * LD + r] * scal_p;
                    V[(int64_t)(c - 1) * LD + r] = vprev;
                }
                const double p0 = Mget(rl, k0 + c);
                const double p1 = Mget(rl, k0 + min(c + 1, BW - 1));
                // only columns < c of V are nonzero: load them in chunks of 8 (the
                // chunk count is uniform, so the loads stay unmasked and batched)
                double vr[BW];
#pragma unroll
                for (int ch = 0; ch < BW / 8; ++ch) {
                    if (ch * 8 < c) {
#pragma unroll
                        for (int l = ch * 8; l < ch * 8 + 8; ++l) vr[l] = V[(int64_t)l * LD + rl];
                    } else {
#pragma unroll
                        for (int l = ch * 8; l < ch * 8 + 8; ++l) vr[l] = 0.0;
                    }
                }
                __builtin_amdgcn_sched_barrier(0);   // (v_{c-1} was stored above by this thread)
                double s4[4] = {p0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int l = 0; l < BW; ++l) s4[l & 3] = fma(-vr[l], zt[BW + l], s4[l & 3]);  // t[l >= c] = 0
                const double xc = live ? (s4[0] + s4[1]) + (s4[2] + s4[3]) : 0.0;
                const double xn = (live && more) ? p1 : 0.0;
                const int rr = r - r0;
                const bool below = live && rr > c;
                if (live) {
                    if (rr < c) bnd[(int64_t)(k0 + c) * BLD + (r - k0 - c)] = xc;      // R(rr, c)
                    else if (rr == c) {
                        sc[0] = xc;
                        sc[1] = xn;
#pragma unroll
                        for (int l = 0; l < BW; ++l) sc[2 + l] = vr[l];
                    } else {
                        Wm[(int64_t)c * LD + r] = xc;
                    }
                }
                const double xb = below ? xc : 0.0;
                sig = fma(xb, xb, sig);
                dx = fma(xb, xn, dx);
                // V^T P(:, c+1) and V^T x_c(below): only columns l < c are nonzero, so
                // the transpose-sum runs over 8, 16 or 32 of them (uniform choice)
                if (c <= 8) {
                    accq += part_sum<8>(vr, xn); accg += part_sum<8>(vr, xb);
                } else if (c <= 16) {
                    accq += part_sum<16>(vr, xn); accg += part_sum<16>(vr, xb);
                } else {
                    accq += part_sum<32>(vr, xn); accg += part_sum<32>(vr, xb);
                }
            }
            sig = wave_sum(sig);
            dx = wave_sum(dx);
            {   // lane l holds column l >> (6 - log2 N) of the sums (columns >= N are not read)
                const int sh = (c <= 8) ? 3 : ((c <= 16) ? 2 : 1);
                if ((lane & ((1 << sh) - 1)) == 0) { rd[wave * RED + (lane >> sh)] = accq; rd[wave * RED + BW + (lane >> sh)] = accg; }
            }
            if (lane == 0) { rd[wave * RED + 2 * BW] = sig; rd[wave * RED + 2 * BW + 1] = dx; }
            __syncthreads();
            // ---- every wave: reflector c, column c of T, t for column c + 1
            double sg = 0.0, dxt = 0.0;
            for (int w = 0; w < NWAVE; ++w) { sg += rd[w * RED + 2 * BW]; dxt += rd[w * RED + 2 * BW + 1]; }
            double tau = 0.0, scal = 0.0;
            if (r0 + c < m) {
                const double alpha = sc[0];
                double beta = alpha;
                if (sg != 0.0) {
                    const double nrm = sqrt(fma(alpha, alpha, sg));
                    beta = (alpha >= 0.0) ? -nrm : nrm;
                    tau = (beta - alpha) / beta;
                    scal = 1.0 / (alpha - beta);
                }
                if (tid == 0) bnd[(int64_t)(k0 + c) * BLD + BW] = beta;   // R(c, c) = A(r0 + c, k0 + c)
            }
            {
                double q = 0.0, g = 0.0;
                if (lane < BW)
                    for (int w = 0; w < NWAVE; ++w) { q += rd[w * RED + lane]; g += rd[w * RED + BW + lane]; }
                // V^T v_c (l < c) and z = V(:,0:c+1)^T P(:,c+1)
                const bool has = r0 + c < m;
                const double gl = (lane < c && has) ? sc[2 + lane] + scal * g : 0.0;
                const double zl = (lane < c) ? q : ((lane == c && has) ? sc[1] + scal * dxt : 0.0);
                if (lane < BW) zt[lane] = gl;
                __builtin_amdgcn_wave_barrier();
                // column c of T: T(l, c) = -tau T(l, l..c-1) (V^T v_c)(l..c-1), T(c, c) = tau
                double tcol = 0.0;
                if (lane < c) {
                    double s = 0.0;
                    for (int l = lane; l < c; ++l) s = fma(Tm[lane * BW + l], zt[l], s);
                    tcol = -tau * s;
                } else if (lane == c) {
                    tcol = tau;
                }
                if (wave == 0 && lane <= c) Tm[lane * BW + c] = tcol;
                // t = T(0:c+1, 0:c+1)^T z: columns < c of T from LDS, column c from tcol
                __builtin_amdgcn_wave_barrier();
                if (lane < BW) zt[lane] = zl;
                __builtin_amdgcn_wave_barrier();
                double t = 0.0;
                if (lane < c)
                    for (int l = 0; l <= lane; ++l) t = fma(Tm[l * BW + lane], zt[l], t);
                const double tc = wave_sum((lane <= c) ? tcol * zl : 0.0);
                __builtin_amdgcn_wave_barrier();
                if (lane < BW) zt[BW + lane] = (lane < c) ? t : ((lane == c) ? tc : 0.0);
                __builtin_amdgcn_wave_barrier();
            }
            scal_p = scal;
        }
        // v_{BW-1}
        for (int r = r0 + BW - 1 + tid; r < m; r += NT)
            V[(int64_t)(BW - 1) * LD + r] = (r == r0 + BW - 1) ? 1.0 : Wm[(int64_t)(BW - 1) * LD + r] * scal_p;
        __syncthreads();
    }

    // ---------------------------------------------------------------- SYMM
    // Y = A22 V over tile rows/columns >= J1 in two passes of f64 16x16x4
    // matrix-core products (an FP32 trailing matrix is widened on load, so Y
    // accumulates in FP64 in both forms; only the update is FP32 arithmetic):
    // column pass Y_J = sum_{I > J} A_IJ^T V_I (one wave per tile column),
    // row pass Y_I += sum_{J1 <= J <= I} A_IJ V_J (one wave per tile row,
    // diagonal tiles are stored whole).  Y goes to Wm (column l at l * LD).
    // The operands of 8 K-steps are loaded while those of the previous 8 feed
    // the matrix cores.
    //
    // f64 16x16x4: operand a of lane l is A(l % 16, l / 16), operand b is
    // B(l / 16, l % 16); result register g of lane l is D(l / 16 + 4 g, l % 16).
    typedef double dpair __attribute__((ext_vector_type(2)));
    typedef S spair __attribute__((ext_vector_type(2)));

    // Column pass, tile (I, J): Y_J += A_IJ^T V_I.  K runs down the tile rows in
    // pairs: lane l loads rows kq + 2 (l / 16) and + 1 of column cb*16 + l % 16
    // (one 16- or 8-byte load) and the matching two rows of V_I, and feeds two
    // MFMAs.  acc[cb][jb] holds Y_J(cb*16 + i, jb*16 + j).
    struct ColOps { spair a[4]; dpair b[2]; };
    __device__ __forceinline__ void col_load(ColOps &o, const S *tp, const double *vI, int kq) const {
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
            o.a[cb] = __builtin_nontemporal_load(reinterpret_cast<const spair *>(tp + mtile_off(kq + 2 * lk, cb * 16 + lr)));
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
            o.b[jb] = *reinterpret_cast<const dpair *>(vI + (int64_t)(jb * 16 + lr) * LD + kq + 2 * lk);
    }
    __device__ __forceinline__ void col_mfma(const ColOps &o, dbl4 (&acc)[4][2]) const {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) {
                acc[cb][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)o.a[cb].x, o.b[jb].x, acc[cb][jb], 0, 0, 0);
                acc[cb][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)o.a[cb].y, o.b[jb].y, acc[cb][jb], 0, 0, 0);
            }
    }
    __device__ void symm_col_tile(const S *tp, const double *vI, dbl4 (&acc)[4][2]) const {
        ColOps o0, o1;
        col_load(o0, tp, vI, 0);
#pragma unroll 1
        for (int kq = 0; kq < TILE; kq += 16) {
            col_load(o1, tp, vI, kq + 8);
            __builtin_amdgcn_sched_barrier(0);
            col_mfma(o0, acc);
            if (kq + 16 < TILE) col_load(o0, tp, vI, kq + 16);
            __builtin_amdgcn_sched_barrier(0);
            col_mfma(o1, acc);
        }
    }

    // Row pass, tile (I, J): Y_I += A_IJ V_J.  Lane l loads rows h*32 + 2 (l % 16)
    // and + 1 of column kq + l / 16 (consecutive in a sub-block); the even rows
    // feed one MFMA and the odd rows another.  acc[2h + p][jb] holds
    // Y_I(h*32 + 2 i + p, jb*16 + j).
    struct RowOps { spair a[2][2]; double b[2][2]; };   // [kk][h], [kk][jb]
    __device__ __forceinline__ void row_load(RowOps &o, const S *tp, const double *vJ, int kq) const {
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
                o.a[kk][h] = __builtin_nontemporal_load(reinterpret_cast<const spair *>(tp + mtile_off(h * 32 + 2 * lr, kq + 4 * kk + lk)));
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) o.b[kk][jb] = vJ[(int64_t)(jb * 16 + lr) * LD + kq + 4 * kk + lk];
        }
    }
    __device__ __forceinline__ void row_mfma(const RowOps &o, dbl4 (&acc)[4][2]) const {
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int jb = 0; jb < 2; ++jb) {
                    acc[2 * h][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)o.a[kk][h].x, o.b[kk][jb], acc[2 * h][jb], 0, 0, 0);
                    acc[2 * h + 1][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)o.a[kk][h].y, o.b[kk][jb], acc[2 * h + 1][jb], 0, 0, 0);
                }
    }
    __device__ void symm_row_tile(const S *tp, const double *vJ, dbl4 (&acc)[4][2]) const {
        RowOps o0, o1;
        row_load(o0, tp, vJ, 0);
#pragma unroll 1
        for (int kq = 0; kq < TILE; kq += 16) {
            row_load(o1, tp, vJ, kq + 8);
            __builtin_amdgcn_sched_barrier(0);
            row_mfma(o0, acc);
            if (kq + 16 < TILE) row_load(o0, tp, vJ, kq + 16);
            __builtin_amdgcn_sched_barrier(0);
            row_mfma(o1, acc);
        }
    }

    // FP32 trailing matrix: four consecutive rows of a micro-tile column come in
    // one 16-byte load.  Column pass: lane l loads rows kq + 4 (l / 16) .. + 3 of
    // column cb*16 + l % 16 and the same rows of V_I; the j-th MFMA of the four
    // takes row kq + 4 (l / 16) + j as its K index.  acc as in the FP64 pass.
    struct ColOps4 { flt4 a[4]; dpair b[2][2]; };   // a[cb]; b[jb][rows +0,+1 | +2,+3]
    __device__ __forceinline__ void col_load4(ColOps4 &o, const S *tp, const double *vI, int kq) const {
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
            o.a[cb] = __builtin_nontemporal_load(reinterpret_cast<const flt4 *>(tp + mtile_off(kq + 4 * lk, cb * 16 + lr)));
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int hf = 0; hf < 2; ++hf)
                o.b[jb][hf] = *reinterpret_cast<const dpair *>(vI + (int64_t)(jb * 16 + lr) * LD + kq + 4 * lk + 2 * hf);
    }
    __device__ __forceinline__ void col_mfma4(const ColOps4 &o, dbl4 (&acc)[4][2]) const {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[cb][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)o.a[cb][j], o.b[jb][j >> 1][j & 1],
                                                                      acc[cb][jb], 0, 0, 0);
    }
    __device__ void symm_col_tile4(const S *tp, const double *vI, dbl4 (&acc)[4][2]) const {
        ColOps4 o0, o1;
        col_load4(o0, tp, vI, 0);
#pragma unroll 1
        for (int kq = 0; kq < TILE; kq += 32) {
            col_load4(o1, tp, vI, kq + 16);
            __builtin_amdgcn_sched_barrier(0);
            col_mfma4(o0, acc);
            if (kq + 32 < TILE) col_load4(o0, tp, vI, kq + 32);
            __builtin_amdgcn_sched_barrier(0);
            col_mfma4(o1, acc);
        }
    }
    // Row pass: lane l loads rows 4 (l % 16) .. + 3 of column kq + l / 16;
    // acc[x][jb] holds Y_I(4 i + x, jb*16 + j).
    struct RowOps4 { flt4 a[2]; double b[2][2]; };   // a[kk]; b[kk][jb]
    __device__ __forceinline__ void row_load4(RowOps4 &o, const S *tp, const double *vJ, int kq) const {
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            o.a[kk] = __builtin_nontemporal_load(reinterpret_cast<const flt4 *>(tp + mtile_off(4 * lr, kq + 4 * kk + lk)));
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) o.b[kk][jb] = vJ[(int64_t)(jb * 16 + lr) * LD + kq + 4 * kk + lk];
        }
    }
    __device__ __forceinline__ void row_mfma4(const RowOps4 &o, dbl4 (&acc)[4][2]) const {
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int jb = 0; jb < 2; ++jb)
                    acc[x][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)o.a[kk][x], o.b[kk][jb], acc[x][jb], 0, 0, 0);
    }
    __device__ void symm_row_tile4(const S *tp, const double *vJ, dbl4 (&acc)[4][2]) const {
        RowOps4 o0, o1;
        row_load4(o0, tp, vJ, 0);
#pragma unroll 1
        for (int kq = 0; kq < TILE; kq += 16) {
            row_load4(o1, tp, vJ, kq + 8);
            __builtin_amdgcn_sched_barrier(0);
            row_mfma4(o0, acc);
            if (kq + 16 < TILE) row_load4(o0, tp, vJ, kq + 16);
            __builtin_amdgcn_sched_barrier(0);
            row_mfma4(o1, acc);
        }
    }

    // Y block of tile row/column K (64 x BW) from the accumulators: result
    // register g of lane l is D(l / 16 + 4 g, l % 16) of block acc[x][jb], which
    // is Y row `rowof(x, l / 16 + 4 g)` of the block, column jb*16 + l % 16.
    template <class RowOf>
    __device__ void store_y(int K, const dbl4 (&acc)[4][2], bool add, RowOf rowof) {
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    double *p = Wm + (int64_t)(jb * 16 + lr) * LD + K * TILE + rowof(x, lk + 4 * g);
                    const double v = acc[x][jb][g];
                    *p = add ? *p + v : v;
                }
    }

    __device__ void symm(int J1) {
        const int NJ = T - J1;
        // column pass: tile column J1 + q has T - 1 - (J1 + q) tiles below the diagonal;
        // columns dealt longest first in snake order
        for (int q = 0; q < NJ; ++q) {
            const int rnd = q / NWAVE, cc = q % NWAVE;
            if (((rnd & 1) ? (NWAVE - 1 - cc) : cc) != wave) continue;
            const int J = J1 + q;
            dbl4 acc[4][2];
#pragma unroll
            for (int a = 0; a < 4; ++a) { acc[a][0] = dbl4{0, 0, 0, 0}; acc[a][1] = dbl4{0, 0, 0, 0}; }
            for (int I = J + 1; I < T; ++I) {
                if constexpr (sizeof(S) == 4) symm_col_tile4(tile_ptr(I, J), V + I * TILE, acc);
                else symm_col_tile(tile_ptr(I, J), V + I * TILE, acc);
            }
            store_y(J, acc, false, [](int x, int i) { return x * 16 + i; });
        }
        __syncthreads();
        // row pass: tile row T - 1 - q has T - J1 - q tiles
        for (int q = 0; q < NJ; ++q) {
            const int rnd = q / NWAVE, cc = q % NWAVE;
            if (((rnd & 1) ? (NWAVE - 1 - cc) : cc) != wave) continue;
            const int I = T - 1 - q;
            dbl4 acc[4][2];
#pragma unroll
            for (int a = 0; a < 4; ++a) { acc[a][0] = dbl4{0, 0, 0, 0}; acc[a][1] = dbl4{0, 0, 0, 0}; }
            if constexpr (sizeof(S) == 4) {
                for (int J = J1; J <= I; ++J) symm_row_tile4(tile_ptr(I, J), V + J * TILE, acc);
                store_y(I, acc, true, [](int x, int i) { return 4 * i + x; });
            } else {
                for (int J = J1; J <= I; ++J) symm_row_tile(tile_ptr(I, J), V + J * TILE, acc);
                store_y(I, acc, true, [](int x, int i) { return (x >> 1) * 32 + 2 * i + (x & 1); });
            }
        }
    }

    // ------------------------------------------------------------ W from Y
    // X = Y T (rows >= r0), M = V^T X (matrix cores), N = T^T M,
    // W = X - 1/2 V N; rows [J1*64, r0) of W are zero.  M is summed over the
// waves in a fixed order (no atomics), so a rerun gives the same bits.
    // Rows [r0, LD) of Z = X2 - s * Y2 Q (in place in Wm when X2 = Wm), in
    // 16-row blocks on matrix cores: Z^T = X2^T - s * Q^T Y2^T, with Q (BW x BW)
    // in LDS (Q(k, n) at q[k * BW + n]).  For a block of rows rb..rb+15,
    // operand a of lane l is Q^T(m, k) = Q(k, m), operand b is Y2(rb + l % 16, k),
    // and result register g of lane l is Z^T(mb * 16 + l / 16 + 4 g, l % 16).
    template <bool SUB>
    __device__ void rows_times_small(int r0, const double *Y2, const double *q, double s) {
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const int lr = ln & 15, lk = ln >> 4;
        for (int rb = r0 + 16 * wave; rb < LD; rb += 16 * NWAVE) {
            double bv[BW / 4];
#pragma unroll
            for (int kk = 0; kk < BW / 4; ++kk) bv[kk] = Y2[(int64_t)(4 * kk + lk) * LD + rb + lr];
            dbl4 acc[2];
            acc[0] = dbl4{0, 0, 0, 0};
            acc[1] = dbl4{0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < BW / 4; ++kk)
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
                    acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(q[(4 * kk + lk) * BW + mb * 16 + lr], bv[kk], acc[mb], 0, 0, 0);
            double xo[2][4];
            if (SUB) {
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                    for (int g = 0; g < 4; ++g) xo[mb][g] = Wm[(int64_t)(mb * 16 + lk + 4 * g) * LD + rb + lr];
            }
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    Wm[(int64_t)(mb * 16 + lk + 4 * g) * LD + rb + lr] = SUB ? fma(-s, acc[mb][g], xo[mb][g]) : acc[mb][g];
        }
    }

    // dst = P^T Q (BW x BW, dst(i, j) at [i * BW + j]) over rows [r0, LD) of
    // P and Q (column l at l * LD): rows in chunks of 4 per MFMA, chunks dealt
    // to waves, per-wave partial sums added in wave order afterwards (a fixed
    // order: reruns give the same bits).  dst must not overlap Nm + BW^2 on.
    __device__ void cross_sum(const double *P, const double *Q, int r0, double *dst) {
        double *part = Nm + BW * BW;
        {
            const int lr = lane & 15, lk = lane >> 4;
            dbl4 acc[2][2];
#pragma unroll
            for (int a = 0; a < 2; ++a) { acc[a][0] = dbl4{0, 0, 0, 0}; acc[a][1] = dbl4{0, 0, 0, 0}; }
            for (int rk = r0 + 4 * wave; rk < LD; rk += 4 * NWAVE) {
                double av[2], bx[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    av[q] = P[(int64_t)(q * 16 + lr) * LD + rk + lk];
                    bx[q] = Q[(int64_t)(q * 16 + lr) * LD + rk + lk];
                }
#pragma unroll
                for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                    for (int jb = 0; jb < 2; ++jb)
                        acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ib], bx[jb], acc[ib][jb], 0, 0, 0);
            }
#pragma unroll
            for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                    for (int g = 0; g < 4; ++g)
                        part[wave * BW * BW + (ib * 16 + lk + 4 * g) * BW + jb * 16 + lr] = acc[ib][jb][g];
        }
        __syncthreads();
        for (int q = tid; q < BW * BW; q += NT) {
            double sum = part[q];
            for (int w = 1; w < NWAVE; ++w) sum += part[w * BW * BW + q];
            dst[q] = sum;
        }
        __syncthreads();
    }

    __device__ void make_w(int J1, int r0) {
        // X = Y T (T upper triangular, its lower part zero in LDS); each block's Y
        // is read before its X is written, by the same wave
        rows_times_small<false>(r0, Wm, Tm, 0.0);
        __syncthreads();
        cross_sum(V, Wm, r0, Mm);   // M = V^T X
        for (int q = tid; q < BW * BW; q += NT) {
            const int i = q / BW, j = q % BW;
            double s = 0.0;
            for (int l = 0; l <= i; ++l) s = fma(Tm[l * BW + i], Mm[l * BW + j], s);
            Nm[q] = s;
        }
        __syncthreads();
        for (int q = tid; q < BW * (r0 - J1 * TILE); q += NT) {
            const int l = q / (r0 - J1 * TILE), r = J1 * TILE + q % (r0 - J1 * TILE);
            Wm[(int64_t)l * LD + r] = 0.0;
        }
        // W = X - 1/2 V N
        rows_times_small<true>(r0, V, Nm, 0.5);
    }

    // ---------------------------------------------------------------- SYR2K
    // C(I, J) -= V_I W_J^T + W_I V_J^T for tiles J in [J1, J2), I >= J, with
    // the first KW columns of V and W (KW = BW: one panel; 2 BW: a pair of
    // panels, V = [V_p V_p+1], W = [W_p W_p+1]), a group of tile columns at a
    // time (FP64: two for one panel, one for a pair; FP32: four, two): their
    // J-side rows are staged in LDS (tile column J + j at stg + j * 2 KW TILE,
    // V then W, column k at [k * TILE + row]), and the I-side rows of each row
    // block are loaded once for the NJ tiles of the row in the group.
    // 16-row blocks (FP64 trailing matrix)
    template <int NJ, int KW>
    __device__ void syr2k_rows16(int I, int J, const double *stg, const double *vb, const double *wb, int ib0,
                                 int ibstep) {
        typedef typename std::conditional<sizeof(S) == 8, double, float>::type OpT;
        typedef typename std::conditional<sizeof(S) == 8, dbl4, flt4>::type AccT;
#pragma unroll 1
        for (int ib = ib0; ib < 4; ib += ibstep) {
            // lane-dependent offsets are recomputed here (not hoisted out of the
            // panel loop and kept live through the other phases)
            int ln = lane;
            asm volatile("" : "+v"(ln));
            const int lr = ln & 15, lk = ln >> 4;
            const double *vI = vb + I * TILE + lr, *wI = wb + I * TILE + lr;
            // I-side operands of rows ib * 16 + lr, all K
            OpT bv[KW / 4], bw[KW / 4];
#pragma unroll
            for (int kk = 0; kk < KW / 4; ++kk) {
                const int64_t col = (int64_t)(4 * kk + lk) * LD + ib * 16;
                bv[kk] = (OpT)vI[col];
                bw[kk] = (OpT)wI[col];
            }
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                S *tp = tile_ptr(I, J + j);
                const double *vs = stg + j * 2 * KW * TILE, *ws = vs + KW * TILE;
                AccT acc[4];
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) acc[jb] = AccT{0, 0, 0, 0};
#pragma unroll
                for (int kk = 0; kk < KW / 4; ++kk) {
                    const int sc = (4 * kk + lk) * TILE + lr;
                    OpT aw[4], av[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) { aw[q] = (OpT)ws[sc + q * 16]; av[q] = (OpT)vs[sc + q * 16]; }
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb) {
                        if constexpr (sizeof(S) == 8) {
                            acc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aw[jb], bv[kk], acc[jb], 0, 0, 0);
                            acc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[jb], bw[kk], acc[jb], 0, 0, 0);
                        } else {
                            acc[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw[jb], bv[kk], acc[jb], 0, 0, 0);
                            acc[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[jb], bw[kk], acc[jb], 0, 0, 0);
                        }
                    }
                }
                // f64: acc[jb][g] = dC(row ib*16 + lr, col jb*16 + lk + 4g) (64 lanes x one
                // register cover 512 contiguous bytes of the tile); f32: col jb*16 + 4 lk + g.
                // All loads of the 16-row block are issued before its stores.
                S c[4][4];
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const int cc = (sizeof(S) == 8) ? jb * 16 + lk + 4 * g : jb * 16 + 4 * lk + g;
                        c[jb][g] = __builtin_nontemporal_load(tp + mtile_off(ib * 16 + lr, cc));
                    }
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const int cc = (sizeof(S) == 8) ? jb * 16 + lk + 4 * g : jb * 16 + 4 * lk + g;
                        __builtin_nontemporal_store(c[jb][g] - acc[jb][g], tp + mtile_off(ib * 16 + lr, cc));
                    }
            }
        }
    }

    // 32-row blocks (FP32 trailing matrix: its operands take half the registers);
    // stg holds FP32 copies of the J-side rows of up to four tile columns
    template <int NJ, int KW>
    __device__ void syr2k_rows32(int I, int J, const float *stg, const double *vb, const double *wb, int ip0,
                                 int ipstep) {
        typedef typename std::conditional<sizeof(S) == 8, double, float>::type OpT;
        typedef typename std::conditional<sizeof(S) == 8, dbl4, flt4>::type AccT;
#pragma unroll 1
        for (int ip = ip0; ip < 4; ip += ipstep) {
            // lane-dependent offsets are recomputed here (not hoisted out of the
            // panel loop and kept live through the other phases)
            int ln = lane;
            asm volatile("" : "+v"(ln));
            const int lr = ln & 15, lk = ln >> 4;
            const double *vI = vb + I * TILE + lr, *wI = wb + I * TILE + lr;
            // I-side operands of rows (ip + q) * 16 + lr, all K
            OpT bv[KW / 4][2], bw[KW / 4][2];
#pragma unroll
            for (int kk = 0; kk < KW / 4; ++kk) {
                const int64_t col = (int64_t)(4 * kk + lk) * LD + ip * 16;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    bv[kk][q] = (OpT)vI[col + q * 16];
                    bw[kk][q] = (OpT)wI[col + q * 16];
                }
            }
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                S *tp = tile_ptr(I, J + j);
                const float *vs = stg + j * 2 * KW * TILE, *ws = vs + KW * TILE;
                AccT acc[4][2];
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) { acc[jb][0] = AccT{0, 0, 0, 0}; acc[jb][1] = AccT{0, 0, 0, 0}; }
#pragma unroll
                for (int kk = 0; kk < KW / 4; ++kk) {
                    const int sc = (4 * kk + lk) * TILE + lr;
                    OpT aw[4], av[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) { aw[q] = (OpT)ws[sc + q * 16]; av[q] = (OpT)vs[sc + q * 16]; }
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                        for (int ib = 0; ib < 2; ++ib) {
                            if constexpr (sizeof(S) == 8) {
                                acc[jb][ib] = __builtin_amdgcn_mfma_f64_16x16x4f64(aw[jb], bv[kk][ib], acc[jb][ib], 0, 0, 0);
                                acc[jb][ib] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[jb], bw[kk][ib], acc[jb][ib], 0, 0, 0);
                            } else {
                                acc[jb][ib] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw[jb], bv[kk][ib], acc[jb][ib], 0, 0, 0);
                                acc[jb][ib] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[jb], bw[kk][ib], acc[jb][ib], 0, 0, 0);
                            }
                        }
                }
                // f64: acc[jb][ib][g] = dC(row (ip+ib)*16 + lr, col jb*16 + lk + 4g) (64 lanes x
                // one register cover 512 contiguous bytes of the tile); f32: col jb*16 + 4 lk + g.
                // All loads of a 16-row block are issued before its stores.
#pragma unroll
                for (int ib = 0; ib < 2; ++ib) {
                    S c[4][4];
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            const int cc = (sizeof(S) == 8) ? jb * 16 + lk + 4 * g : jb * 16 + 4 * lk + g;
                            c[jb][g] = __builtin_nontemporal_load(tp + mtile_off((ip + ib) * 16 + lr, cc));
                        }
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            const int cc = (sizeof(S) == 8) ? jb * 16 + lk + 4 * g : jb * 16 + 4 * lk + g;
                            __builtin_nontemporal_store(c[jb][g] - acc[jb][ib][g], tp + mtile_off((ip + ib) * 16 + lr, cc));
                        }
                }
            }
        }
    }

    // Row blocks dealt to the waves: the 16-row (FP64) or 32-row (FP32) blocks
    // of every tile row are spread over the waves, so each wave gets the same
    // number of blocks in every group of tile columns (no wave waits for
    // another's extra tile row at the barrier).
    static constexpr int RB = (sizeof(S) == 8) ? 16 : 32;     // rows per block
    static constexpr int BPR = TILE / RB;                     // blocks per tile row
    static constexpr int RSTEP = (NWAVE >= BPR) ? NWAVE / BPR : 1;   // tile rows in flight
    static constexpr int B0STEP = (NWAVE >= BPR) ? BPR : 1;
    __device__ int block0() const { return (NWAVE >= BPR) ? wave % BPR : 0; }

    template <int KW>
    __device__ void syr2k(int J1, int J2, const double *vb, const double *wb) {
        if constexpr (sizeof(S) == 8) {
            constexpr int G = 2 * BW / KW;   // tile columns per group (the staging holds 4 BW TILE doubles)
            double *stg = Tm;   // T, M and N are not needed again in this panel
            for (int J = J1; J < J2; J += G) {
                const int nj = min(G, J2 - J);
                for (int q = tid; q < nj * KW * TILE; q += NT) {
                    const int j = q / (KW * TILE), qq = q % (KW * TILE);
                    const int kc = qq / TILE, r = qq % TILE;
                    stg[j * 2 * KW * TILE + qq] = vb[(int64_t)kc * LD + (J + j) * TILE + r];
                    stg[j * 2 * KW * TILE + KW * TILE + qq] = wb[(int64_t)kc * LD + (J + j) * TILE + r];
                }
                __syncthreads();
                // row J holds one tile of the group (the other is above the diagonal)
                for (int I = J + wave / BPR; I < T; I += RSTEP) {
                    if constexpr (G == 1) {
                        syr2k_rows16<1, KW>(I, J, stg, vb, wb, block0(), B0STEP);
                    } else {
                        if (I == J || nj == 1) syr2k_rows16<1, KW>(I, J, stg, vb, wb, block0(), B0STEP);
                        else syr2k_rows16<2, KW>(I, J, stg, vb, wb, block0(), B0STEP);
                    }
                }
                __syncthreads();
            }
        } else {
            // FP32 operands (the update's arithmetic is FP32)
            constexpr int G = 4 * BW / KW;
            float *stg = reinterpret_cast<float *>(Tm);
            for (int J = J1; J < J2; J += G) {
                const int nj = min(G, J2 - J);
                for (int q = tid; q < nj * KW * TILE; q += NT) {
                    const int j = q / (KW * TILE), qq = q % (KW * TILE);
                    const int kc = qq / TILE, r = qq % TILE;
                    stg[j * 2 * KW * TILE + qq] = (float)vb[(int64_t)kc * LD + (J + j) * TILE + r];
                    stg[j * 2 * KW * TILE + KW * TILE + qq] = (float)wb[(int64_t)kc * LD + (J + j) * TILE + r];
                }
                __syncthreads();
                // row J + k holds k + 1 tiles of the group (the rest are above the diagonal)
                for (int I = J + wave / BPR; I < T; I += RSTEP) {
                    const int ntl = min(nj, I - J + 1);
                    if (ntl == 1) syr2k_rows32<1, KW>(I, J, stg, vb, wb, 2 * block0(), 2 * B0STEP);
                    else if constexpr (G >= 2) {
                        if (ntl == 2) syr2k_rows32<2, KW>(I, J, stg, vb, wb, 2 * block0(), 2 * B0STEP);
                        else if constexpr (G >= 4) {
                            if (ntl == 3) syr2k_rows32<3, KW>(I, J, stg, vb, wb, 2 * block0(), 2 * B0STEP);
                            else syr2k_rows32<4, KW>(I, J, stg, vb, wb, 2 * block0(), 2 * B0STEP);
                        }
                    }
                }
                __syncthreads();
            }
        }
    }

    // --------------------------------------------------------------- stage 1
    // Diagonal block A(k0:k0+kb, k0:k0+kb) is final: lower triangle to the
    // band.  Then V and W of the panel (the current V, Wm) are cleared from the
    // first tile row its update can touch, and T.
    __device__ void begin_panel(int k0) {
        const int kb = min(BW, m - k0);
        for (int q = tid; q < BW * BW; q += NT) {
            const int i = q % BW, j = q / BW;
            if (j <= i && i < kb) bnd[(int64_t)(k0 + j) * BLD + (i - j)] = Mget(k0 + i, k0 + j);
        }
        if (k0 + BW >= m) return;
        const int rz = (k0 / TILE) * TILE, len = LD - rz;
        for (int q = tid; q < BW * len; q += NT) {
            const int l = q / len, r = rz + q % len;
            V[(int64_t)l * LD + r] = 0.0;
            Wm[(int64_t)l * LD + r] = 0.0;
        }
        for (int q = tid; q < BW * BW; q += NT) Tm[q] = 0.0;
    }

    // Panels go in pairs (p at k0 = 64 q, p + 1 at k0 + BW) with one update of
    // the trailing matrix for both: after panel p only tile column q (which
    // holds panel p + 1) is updated; panel p + 1 is factored from it, and its
    // Y = A' V_p+1 with A' = A - V_p W_p^T - W_p V_p^T is formed from the
    // trailing matrix A not yet updated by panel p:
    //   Y = A V_p+1 - V_p (W_p^T V_p+1) - W_p (V_p^T V_p+1);
    // then A <- A - V W^T - W V^T with V = [V_p V_p+1], W = [W_p W_p+1] (rank
    // 4 BW) over tile columns >= q + 1.  One read-modify-write of the trailing
    // triangle per pair instead of one per panel.  A last panel without a
    // partner is updated alone.  (FP64 trailing matrix only: with an FP32
    // one the update is cheaper than the extra corrections and staging.)
    static constexpr int PANELS = (sizeof(S) == 8) ? 2 : 1;   // panels whose V and W the slot holds
    __device__ void reduce_to_band() {
        int k0 = 0;
        while (k0 < m) {
            V = V0;
            Wm = W0;
            begin_panel(k0);
            const int r0 = k0 + BW;
            if (r0 >= m) break;
            __syncthreads();
            EEID_PHASE_MARK(clk, 4);
            panel_qr(k0);
            EEID_PHASE_MARK(clk, 1);
            const int J1 = r0 / TILE;
            symm(J1);
            __syncthreads();
            EEID_PHASE_MARK(clk, 2);
            make_w(J1, r0);
            __syncthreads();
            EEID_PHASE_MARK(clk, 3);
            const bool pair = PANELS == 2 && (k0 % TILE == 0) && (r0 + BW < m);
            syr2k<BW>(J1, pair ? J1 + 1 : T, V0, W0);
            __syncthreads();
            EEID_PHASE_MARK(clk, 4);
            if (!pair) {
                k0 += BW;
                continue;
            }
            // ---- panel p + 1: columns r0 .. r0 + BW - 1, trailing rows from r1
            const int r1 = r0 + BW, J2 = r1 / TILE;
            V = V0 + (int64_t)BW * LD;
            Wm = W0 + (int64_t)BW * LD;
            begin_panel(r0);
            __syncthreads();
            EEID_PHASE_MARK(clk, 4);
            panel_qr(r0);
            EEID_PHASE_MARK(clk, 1);
            symm(J2);
            __syncthreads();
            EEID_PHASE_MARK(clk, 2);
            cross_sum(W0, V, r1, Mm);   // W_p^T V_p+1
            cross_sum(V0, V, r1, Nm);   // V_p^T V_p+1
            rows_times_small<true>(r1, V0, Mm, 1.0);
            rows_times_small<true>(r1, W0, Nm, 1.0);
            __syncthreads();
            make_w(J2, r1);
            __syncthreads();
            EEID_PHASE_MARK(clk, 3);
            if constexpr (PANELS == 2) syr2k<2 * BW>(J2, T, V0, W0);
            __syncthreads();
            EEID_PHASE_MARK(clk, 4);
            k0 = r1;
        }
    }

    // --------------------------------------------------------------- stage 2
    // Bulge chasing.  Sweep s removes column s below the subdiagonal; its step t
    // acts on rows lo .. lo + 31, lo = s + 1 + 32 t: the previous reflector is
    // applied from the right to the block B = A(lo.., lo-32..) below the
    // previous diagonal block, the first column of B is annihilated by a new
    // reflector that is applied to the rest of B and two-sidedly to the diagonal
    // block D = A(lo.., lo..).  (Step 0 annihilates column s itself.)
    //
    // Sweeps run in chains of CHAIN = 3 (s, s + 1, s + 2), one chain per wave,
    // chain c on wave c mod NWAVE.  Step t of sweep s + 1 acts on the blocks of
    // step t of sweep s shifted down and right by one, plus the first row of
    // step t + 1 of sweep s; the rest of its last row is zero (annihilated by
    // earlier sweeps).  So the wave runs sweep s + k one step behind sweep
    // s + k - 1 and builds its blocks from those of sweep s + k - 1: sweep s
    // loads its blocks, sweep s + 2 stores its results, and the band makes one
    // trip through memory per chain.  The blocks of sweep s of the previous
    // step stay in registers; those of sweep s + 1 wait in LDS for sweep s + 2.
    // A sweep whose blocks pass on stores only what leaves them: the final
    // column (first step) or the annihilated first column of B.  Sweep s of a
    // chain waits for the last sweep of the previous chain to have finished
    // its steps t and t + 1 (progress counters in LDS, sweep * 4096 + steps
    // done, 4095 when complete, ordered by workgroup-scope release and acquire).
    //
    // Lane l holds row i = l % 32 of a 32 x 32 block and its columns
    // 16 h .. 16 h + 15, h = l / 32.
    __device__ double colsum32(double (&p)[16]) {
        // sum of p[q] over the 32 lanes of this half; returns the sum of column
        // 8 b4 + 4 b3 + 2 b2 + b1 (b_k = bit k of the lane) of this half
        halve_step<16, 16>(p, lane);
        halve_step<8, 8>(p, lane);
        halve_step<4, 4>(p, lane);
        halve_step<2, 2>(p, lane);
        return psum<1>(p[0]);
    }

    // LDS vectors of one wave: the previous reflector vp of a sweep, and the
    // per-step temporaries vc, wv, cs (shared by the sweeps of a chain).
    struct ChaseVecs { double *vp, *vc, *wv, *cs; };

    // One step on blocks held in registers.  first: step 0 (x = column s given,
    // no B block).  Otherwise the previous reflector (vp, taup) is applied to B
    // from the right and x is B's first column.  On return: bk = B with column 0
    // = beta e0 (not first), dk = D updated, vc = new reflector, vp = vc, taup =
    // tau; beta returned.  L rows of the step exist (L < 2: only the right
    // application is done).
    __device__ double chase_compute(bool first, double x, double (&bk)[16], double (&dk)[16], int L, double &taup,
                                    const ChaseVecs &cv, int i, int hh, int csel) {
        if (!first) {
            double u = 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) u = fma(bk[q], cv.vp[hh * 16 + q], u);
            u = xsum32(u);
#pragma unroll
            for (int q = 0; q < 16; ++q) bk[q] = fma(-taup * u, cv.vp[hh * 16 + q], bk[q]);
            x = from_lower(bk[0]);  // column 0 of the block: lane i of half 0
        }
        double tau = 0.0, beta, v;
        if (L >= 2) {
            const double alpha = bcast0(x);
            const double sg = wave_sum((hh == 0 && i >= 1 && i < L) ? x * x : 0.0);
            double scal = 0.0;
            beta = alpha;
            if (sg != 0.0) {
                const double nrm = sqrt(fma(alpha, alpha, sg));
                beta = (alpha >= 0.0) ? -nrm : nrm;
                tau = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
            v = (i == 0) ? 1.0 : ((i < L) ? x * scal : 0.0);
        } else {
            beta = bcast0(x);
            v = (i == 0) ? 1.0 : 0.0;
        }
        if (hh == 0) cv.vc[i] = v;
        __builtin_amdgcn_wave_barrier();
        if (!first) {
            // left application to the columns 1.. of B; column 0 becomes beta e0
            double p[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) p[q] = v * bk[q];
            const double sum = colsum32(p);
            if ((lane & 1) == 0) cv.cs[hh * 16 + csel] = sum;
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int c = hh * 16 + q;
                bk[q] = (c == 0) ? ((i == 0) ? beta : 0.0) : fma(-tau * v, cv.cs[c], bk[q]);
            }
        }
        if (L >= 2) {
            // two-sided update of the diagonal block
            double pr = 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) pr = fma(dk[q], cv.vc[hh * 16 + q], pr);
            pr = xsum32(pr);
            const double w0 = tau * pr;
            const double kap = 0.5 * tau * wave_sum((hh == 0) ? v * w0 : 0.0);
            const double w = fma(-kap, v, w0);
            if (hh == 0) cv.wv[i] = w;
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int c = hh * 16 + q;
                dk[q] -= fma(v, cv.wv[c], w * cv.vc[c]);
            }
            if (hh == 0) cv.vp[i] = v;   // applied from the right in the next step
            __builtin_amdgcn_wave_barrier();
        }
        taup = tau;
        return beta;
    }

    // Stores of a step of sweep `sw` at rows lo..: column sw (first step) or B,
    // and the lower triangle of D.
    __device__ void chase_store(bool first, int sw, int lo, int L, double beta, const double (&bk)[16],
                                const double (&dk)[16], int i, int hh) {
        if (first) {
            if (hh == 0 && i < L) bnd[(unsigned)(sw * BLD + 1 + i)] = (i == 0) ? beta : 0.0;
        } else {
            double *pb = bnd + (unsigned)((lo - BW) * BLD + BW + i + (BLD - 1) * hh * 16);
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if (i < L) pb[(BLD - 1) * q] = bk[q];
        }
        {   // (also for L = 1: in a chain the diagonal entry may come from another sweep)
            double *pd = bnd + (unsigned)(lo * BLD + i + (BLD - 1) * hh * 16);
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if (i < L && hh * 16 + q <= i) pd[(BLD - 1) * q] = dk[q];   // A(lo + i, lo + c), c <= i
        }
    }

    // Blocks (fb, fd) of step t of sweep s + 1 from the blocks (pb, pd) of step
    // t of sweep s and row0 = the first row of step t + 1 of sweep s (B part,
    // then D(0, 0) at row0[BW]).
    __device__ void shift_blocks(const double (&pb)[16], const double (&pd)[16], const double *row0,
                                 double (&fb)[16], double (&fd)[16], int i, int hh) {
        // shift left by one column.  Column 15 of the lower half takes column 16
        // from the upper half; column 31 takes D(i, 0) of the previous step (block
        // B) or row0[i] (block D; D is symmetric).
        const double sb = xswap32(pb[0], lane);   // lower half: B(i, 16)
        const double sd = xswap32(pd[0], lane);   // lower half: D(i, 16); upper half: D(i, 0)
#pragma unroll
        for (int q = 0; q < 15; ++q) { fb[q] = pb[q + 1]; fd[q] = pd[q + 1]; }
        fb[15] = hh ? sd : sb;
        fd[15] = hh ? row0[i] : sd;
        // shift up by one row; row 31 of B is zero but for its last column,
        // row 31 of D is row0
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const double nb = dpp_mov<DPP_WAVE_SHL1>(fb[q]);   // lane + 1 (rows 31 replaced)
            const double nd = dpp_mov<DPP_WAVE_SHL1>(fd[q]);
            const int c = hh * 16 + q;
            fb[q] = (i < 31) ? nb : ((c == 31) ? row0[0] : 0.0);
            fd[q] = (i < 31) ? nd : row0[c + 1];
        }
    }

    // Stores of a sweep whose blocks pass on to the next sweep of the chain:
    // column sw and A(lo, lo) at its first step, else the annihilated first
    // column of B below its first row.
    __device__ void chase_store_passing(bool first, int sw, int lo, int L, double beta, double d00, int i, int hh) {
        if (first) {
            if (hh == 0 && i < L) bnd[(unsigned)(sw * BLD + 1 + i)] = (i == 0) ? beta : 0.0;
            if (lane == 0) bnd[(unsigned)(lo * BLD)] = d00;
        } else {
            if (hh == 0 && i >= 1 && i < L) bnd[(unsigned)((lo - BW) * BLD + BW + i)] = 0.0;
        }
    }

    // Row 0 of blocks (b, d) to LDS (B part, then D(0, 0) at row0[BW]).
    __device__ void put_row0(double *row0, const double (&b)[16], const double (&d)[16], int i, int hh) {
        if (i == 0) {
#pragma unroll
            for (int q = 0; q < 16; ++q) row0[hh * 16 + q] = b[q];
        }
        if (lane == 0) row0[BW] = d[0];
        __builtin_amdgcn_wave_barrier();
    }

    static constexpr int CHAIN = 3;
    // LDS doubles per wave: 3 vp + vc, wv, cs; two first rows; the saved blocks
    static constexpr int CHASE_PER_WAVE = 6 * BW + 2 * 40 + 2 * 16 * 64;

    // spin_limit bounds every wait for the previous chain: a wave that polls
    // that often without progress gives up waiting for the rest of the problem,
    // sets FLAG_WAIT_TIMEOUT in *flag and runs on, so the kernel always ends.
    __device__ void band_to_tridiagonal(double *scratch, unsigned spin_limit, int32_t *flag) {
        int *prog = reinterpret_cast<int *>(scratch + NWAVE * CHASE_PER_WAVE);
        if (tid < NWAVE) prog[tid] = (CHAIN * (tid - NWAVE) + CHAIN - 1) * 4096 + 4095;
        __syncthreads();
        double *ws = scratch + wave * CHASE_PER_WAVE;
        double *vc = ws + 3 * BW, *wv = ws + 4 * BW, *cs = ws + 5 * BW;
        const ChaseVecs cv0{ws, vc, wv, cs}, cv1{ws + BW, vc, wv, cs}, cv2{ws + 2 * BW, vc, wv, cs};
        double *row0a = ws + 6 * BW;        // first row of the current step of sweep s
        double *row0b = row0a + 40;         // ... of sweep s + 1
        double *saved = row0b + 40;         // blocks of sweep s + 1 of the previous step: [q * 64 + lane], D at + 1024
        const int pw = (wave + NWAVE - 1) % NWAVE;
        bool bail = false;       // wave-uniform: a wait gave up, do not wait again
        for (int s = CHAIN * wave; s + 2 < m; s += CHAIN * NWAVE) {
            const bool has1 = s + 3 < m, has2 = s + 4 < m;
            const int last0 = (m - 2 - s) / BW;
            const int last1 = has1 ? (m - 3 - s) / BW : -1;
            const int last2 = has2 ? (m - 4 - s) / BW : -1;
            const int tmax = max(last0, max(has1 ? last1 + 1 : 0, has2 ? last2 + 2 : 0));
            const int sl = s + (has2 ? 2 : (has1 ? 1 : 0));   // last sweep of the chain
            double tau0 = 0.0, tau1 = 0.0, tau2 = 0.0;
            double pb[16], pd[16];   // sweep s, previous step
#pragma unroll
            for (int q = 0; q < 16; ++q) { pb[q] = 0.0; pd[q] = 0.0; }
            int tf = -1;             // steps of the last sweep stored and not yet published
            for (int t = 0; t <= tmax; ++t) {
                // lane-dependent indices are recomputed every step (not hoisted and
                // kept live across the sweep loops)
                int ln = lane;
                asm volatile("" : "+v"(ln));
                const int i = ln & 31, hh = ln >> 5;
                const int csel = (((ln >> 4) & 1) << 3) | (((ln >> 3) & 1) << 2) | (((ln >> 2) & 1) << 1) | ((ln >> 1) & 1);
                // ---- step t of sweep s
                double cb[16], cd[16];
                double x = 0.0;
                const bool run0 = t <= last0;
                const int lo = s + 1 + t * BW;
                if (run0) {
                    if (s > 0 && !bail) {
                        const int need = (s - 1) * 4096 + min(t + 2, 4095);
                        unsigned polls = 0;
                        while (__atomic_load_n(&prog[pw], __ATOMIC_RELAXED) < need) {
                            if (++polls > spin_limit) { bail = true; break; }
                            __builtin_amdgcn_s_sleep(1);
                        }
                        if (bail && lane == 0) atomicOr(flag, FLAG_WAIT_TIMEOUT);
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                    }
                    // all loads of the step at once; entries outside the matrix are
                    // band storage that is never written (zero)
                    if (t == 0) {
                        x = bnd[(unsigned)(s * BLD + 1 + i)];                  // A(lo + i, s)
                    } else {
                        const double *pbp = bnd + (unsigned)((lo - BW) * BLD + BW + i + (BLD - 1) * hh * 16);
#pragma unroll
                        for (int q = 0; q < 16; ++q) cb[q] = pbp[(BLD - 1) * q];
                    }
                    const unsigned b1 = (unsigned)(lo * BLD + i), b2 = (unsigned)(lo * BLD + (BLD - 1) * i);
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int c = hh * 16 + q;
                        cd[q] = bnd[(c <= i) ? b1 + (unsigned)((BLD - 1) * c) : b2 + (unsigned)c];
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 16; ++q) { cb[q] = 0.0; cd[q] = 0.0; }
                }
                // publish the steps of the last sweep stored so far (they complete with these loads)
                if (tf >= 0) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    if (lane == 0) __atomic_store_n(&prog[wave], sl * 4096 + tf + 1, __ATOMIC_RELAXED);
                    tf = -1;
                }
                if (run0) {
                    const int L = min(BW, m - lo);
                    const double beta = chase_compute(t == 0, x, cb, cd, L, tau0, cv0, i, hh, csel);
                    if (!has1) {
                        chase_store(t == 0, s, lo, L, beta, cb, cd, i, hh);
                        tf = t;
                    } else {
                        chase_store_passing(t == 0, s, lo, L, beta, cd[0], i, hh);
                    }
                }
                // ---- step t - 1 of sweep s + 1, from steps t - 1 (pb, pd) and t (cb, cd) of sweep s
                double fb[16], fd[16];
                const int t1 = t - 1;
                const bool run1 = has1 && t1 >= 0 && t1 <= last1;
                if (run1) {
                    const int lo1 = s + 2 + t1 * BW;
                    const int L1 = min(BW, m - lo1);
                    put_row0(row0a, cb, cd, i, hh);
                    shift_blocks(pb, pd, row0a, fb, fd, i, hh);
                    const bool first1 = (t1 == 0);
                    const double x1 = from_upper(first1 ? fb[15] : 0.0);   // first step: column s + 1 is column 31
                    const double beta1 = chase_compute(first1, x1, fb, fd, L1, tau1, cv1, i, hh, csel);
                    if (!has2) {
                        chase_store(first1, s + 1, lo1, L1, beta1, fb, fd, i, hh);
                        tf = t1;
                    } else {
                        chase_store_passing(first1, s + 1, lo1, L1, beta1, fd[0], i, hh);
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 16; ++q) { fb[q] = 0.0; fd[q] = 0.0; }
                }
                // ---- step t - 2 of sweep s + 2, from steps t - 2 (saved) and t - 1 (fb, fd) of sweep s + 1
                if (has2) {
                    const int t2 = t - 2;
                    const bool run2 = t2 >= 0 && t2 <= last2;
                    if (run2) put_row0(row0b, fb, fd, i, hh);
                    // the saved blocks of step t - 2 of sweep s + 1 are read and this
                    // step's blocks take their place, entry by entry (few live registers)
                    double gb[16], gd[16];
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        gb[q] = saved[q * 64 + lane];
                        gd[q] = saved[1024 + q * 64 + lane];
                        if (run1) { saved[q * 64 + lane] = fb[q]; saved[1024 + q * 64 + lane] = fd[q]; }
                    }
                    if (run2) {
                        const int lo2 = s + 3 + t2 * BW;
                        const int L2 = min(BW, m - lo2);
                        double hb[16], hd[16];
                        shift_blocks(gb, gd, row0b, hb, hd, i, hh);
                        const bool first2 = (t2 == 0);
                        const double x2 = from_upper(first2 ? hb[15] : 0.0);
                        const double beta2 = chase_compute(first2, x2, hb, hd, L2, tau2, cv2, i, hh, csel);
                        chase_store(first2, s + 2, lo2, L2, beta2, hb, hd, i, hh);
                        tf = t2;
                    }
                }
#pragma unroll
                for (int q = 0; q < 16; ++q) { pb[q] = cb[q]; pd[q] = cd[q]; }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) __atomic_store_n(&prog[wave], sl * 4096 + 4095, __ATOMIC_RELAXED);
        }
        __syncthreads();
        for (int r = tid; r < m; r += NT) {
            dg[r] = bnd[(int64_t)r * BLD];
            if (r + 1 < m) eg[r] = bnd[(int64_t)r * BLD + 1];
        }
        __syncthreads();
    }

    __device__ void bisect(double *out, const double *brk) {
        bisect_tridiagonal<NT, 8>(dg, eg, m, out, de, red, tid, lane, wave, brk);
    }

    // ------------------------------------------------- small orders, in LDS
    // m <= SMALL_MAX: the problem lives in LDS as a packed lower triangle
    // (column c at c (2m - c + 1) / 2, rows c..m-1) and is reduced by unblocked
    // Householder steps -- per column the norm, the reflector (beta real),
    // y = A u, w = tau y - (tau^2 / 2)(u^T y) u and A -= u w^T + w u^T on the
    // trailing triangle, with every reduction over the waves in a fixed order
    // -- then bisected like the large problems.  No HBM traffic but the
    // gather; the two-stage path's panels, tiles and chase are latency there.
    static constexpr int SMALL_MAX = 128;
    __device__ __forceinline__ int pk(int r, int c) const { return c * (2 * m - c + 1) / 2 + (r - c); }

    __device__ void small_tridiagonal(const Item &it, double *L) {
        double *u = L + SMALL_MAX * (SMALL_MAX + 1) / 2;
        double *yw = u + SMALL_MAX;
        double *ds = yw + SMALL_MAX, *es = ds + SMALL_MAX;
        const int n = it.n, j = it.j;
        // all threads over the m x m index space, eight loads in flight per thread
        // before their stores (the loads are independent; issued one by one they
        // would serialise on the memory latency)
        for (int q0 = 0; q0 < m * m; q0 += 8 * NT) {
            double v[8];
#pragma unroll
            for (int z = 0; z < 8; ++z) {
                const int q = q0 + z * NT + tid, r = q / m, c = q - r * m;
                v[z] = 0.0;
                if (q < m * m && c <= r) {
                    const int rs = r + ((j >= 0 && r >= j) ? 1 : 0);
                    const int cs = c + ((j >= 0 && c >= j) ? 1 : 0);
                    v[z] = (it.k >= 0) ? rotated_at(it.src, n, j, it.k, rs, cs) : lower_at(it.src, n, rs, cs);
                }
            }
#pragma unroll
            for (int z = 0; z < 8; ++z) {
                const int q = q0 + z * NT + tid, r = q / m, c = q - r * m;
                if (q < m * m && c <= r) L[pk(r, c)] = v[z];
            }
        }
        __syncthreads();
        for (int k = 0; k + 2 < m; ++k) {
            const int t0 = k + 1;
            // sigma^2 = sum_{i > k+1} L(i, k)^2: one wave, fixed tree
            if (wave == 0) {
                double sg = 0.0;
                for (int i = k + 2 + lane; i < m; i += 64) { const double x = L[pk(i, k)]; sg = fma(x, x, sg); }
                sg = wave_sum(sg);
                if (lane == 0) red[0] = sg;
            }
            __syncthreads();
            const double sg = red[0];
            const double alpha = L[pk(t0, k)];
            double tau = 0.0, scal = 0.0, beta = alpha;
            if (sg != 0.0) {
                const double nrm = sqrt(fma(alpha, alpha, sg));
                beta = (alpha >= 0.0) ? -nrm : nrm;
                tau = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
            if (tid == 0) { ds[k] = L[pk(k, k)]; es[k] = beta; }
            if (tau == 0.0) { __syncthreads(); continue; }
            for (int i = t0 + tid; i < m; i += NT) u[i] = (i == t0) ? 1.0 : L[pk(i, k)] * scal;
            __syncthreads();
            // y = A22 u with tpr threads per row (adjacent lanes, each a residue class of
            // columns, summed across the group): row i's entries (i, t0..i) step
            // through the packed columns, its entries (i+1.., i) are contiguous in
            // column i; and the per-wave parts of u^T y
            const int tpr = (m <= NT / 4) ? 4 : ((m <= NT / 2) ? 2 : 1);
            double part = 0.0;
            for (int i0 = t0; i0 < m; i0 += NT / tpr) {
                const int i = i0 + tid / tpr, sub = tid % tpr;
                double y0 = 0.0, y1 = 0.0;
                if (i < m) {
                    for (int c = t0 + sub; c <= i; c += tpr) y0 = fma(L[pk(i, c)], u[c], y0);
                    const int qd = pk(i, i) - i;
                    for (int c = i + 1 + sub; c < m; c += tpr) y1 = fma(L[qd + c], u[c], y1);
                }
                double y = y0 + y1;
                if (tpr >= 2) y = psum<1>(y);
                if (tpr >= 4) y = psum<2>(y);
                if (i < m && sub == 0) {
                    yw[i] = y;
                    part = fma(u[i], y, part);
                }
            }
            part = wave_sum(part);
            if (lane == 0) red[8 + wave] = part;
            __syncthreads();
            double uy = 0.0;
            for (int w = 0; w < NWAVE; ++w) uy += red[8 + w];
            const double kap = 0.5 * tau * tau * uy;
            for (int i = t0 + tid; i < m; i += NT) yw[i] = fma(-kap, u[i], tau * yw[i]);   // y -> w
            __syncthreads();
            // A22 -= u w^T + w u^T on the packed trailing triangle, tpr threads per row
            for (int r0 = t0; r0 < m; r0 += NT / tpr) {
                const int r = r0 + tid / tpr, sub = tid % tpr;
                if (r >= m) continue;
                const double ur = u[r], wr = yw[r];
                for (int c = t0 + sub; c <= r; c += tpr) L[pk(r, c)] -= fma(ur, yw[c], wr * u[c]);
            }
            __syncthreads();
        }
        if (tid == 0) {
            if (m >= 2) {
                ds[m - 2] = L[pk(m - 2, m - 2)];
                es[m - 2] = L[pk(m - 1, m - 2)];
            }
            ds[m - 1] = L[pk(m - 1, m - 1)];
        }
        __syncthreads();
        dg = ds;
        eg = es;
    }
};

template <class S>
__host__ __device__ inline int64_t slot_bytes_band(int LDmax) {
    const int64_t T = LDmax / TILE;
    const int64_t tiles = T * (T + 1) / 2 * TILE_ELEMS * (int64_t)sizeof(S);
    const int64_t panel = 2 * (int64_t)Band<S, 256>::PANELS * BW * LDmax * 8;   // V and W (one panel or a pair)
    const int64_t band = (int64_t)(LDmax + BW) * BLD * 8;
    const int64_t de = 2 * (int64_t)LDmax * 8;
    return ((tiles + 255) / 256) * 256 + panel + band + de;
}

// Doubles of the LDS region shared in turn by stage 1 (T, M, N, SYR2K
// staging), the bulge chase (per-wave vectors, first rows and saved blocks,
// then the progress counters) and the bisection (d, e^2).
template <int NT>
__host__ __device__ inline int64_t lds_big_band(int LDmax) {
    constexpr int64_t nw = NT / 64;
    // T, M, N (3 BW^2) and the per-wave partial sums of M; then the SYR2K staging of two tile columns
    const int64_t stage1 = (4 * BW * TILE > (3 + nw) * BW * BW) ? 4 * BW * TILE : (3 + nw) * BW * BW;
    const int64_t chase = nw * (6 * BW + 2 * 40 + 2 * 16 * 64) + (nw + 1) / 2;
    const int64_t bis = 2 * (int64_t)LDmax;
    return (stage1 > chase ? (stage1 > bis ? stage1 : bis) : (chase > bis ? chase : bis));
}

// The small-order path keeps a packed triangle of order 128 and five vectors in
// the same region (the chase's share alone is larger for every configuration).
static_assert((4 * (6 * BW + 2 * 40 + 2 * 16 * 64)) >= 128 * 129 / 2 + 4 * 128 + 2 * 128,
              "LDS region too small for the small-order path");

template <int NT>
__host__ __device__ inline int64_t lds_bytes_band(int LDmax) {
    return (lds_big_band<NT>(LDmax) + (NT / 64) * (2 * BW + 8) + 160) * 8 + 64;
}

template <class S, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
void band_bisect_kernel(TriArgs args) {
    extern __shared__ double lds[];
    __shared__ int s_item;
    __shared__ unsigned long long s_flag;
    Band<S, NT> t;
    t.tid = threadIdx.x;
    t.lane = threadIdx.x & 63;
    t.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int LDmax = args.LDmax;
    const int64_t big = lds_big_band<NT>(LDmax);
    t.Tm = lds;
    t.Mm = lds + BW * BW;
    t.Nm = lds + 2 * BW * BW;
    t.de = lds;
    t.red = lds + big;
    t.vec = t.red + (NT / 64) * (2 * BW + 8);
    char *slot = args.work + (int64_t)blockIdx.x * args.slot_bytes;
    t.clk.start();
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(args.counter, 1);
        __syncthreads();
        const int64_t it_idx = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (it_idx >= args.n_items) break;
        const Item it = args.items[it_idx];
        if (args.flags[it.b] & 1) {
            for (int i = threadIdx.x; i < it.m; i += NT) it.out[i] = __builtin_nan("");
            continue;
        }
        EEID_PHASE_MARK(t.clk, 7);
        t.m = it.m;
        t.T = (it.m + TILE - 1) / TILE;
        t.LD = t.T * TILE;
        t.tiles = reinterpret_cast<S *>(slot);
        const int64_t T = t.T;
        const int64_t tile_bytes = ((T * (T + 1) / 2 * TILE_ELEMS * (int64_t)sizeof(S) + 255) / 256) * 256;
        t.V0 = reinterpret_cast<double *>(slot + tile_bytes);
        t.W0 = t.V0 + (int64_t)Band<S, NT>::PANELS * BW * t.LD;
        t.V = t.V0;
        t.Wm = t.W0;
        t.bnd = t.W0 + (int64_t)Band<S, NT>::PANELS * BW * t.LD;
        t.dg = t.bnd + (int64_t)BLD * (t.LD + BW);
        t.eg = t.dg + t.LD;
        if (it.m <= Band<S, NT>::SMALL_MAX) {
            // small order: reduced in LDS (the slot's d and e are not used)
            t.small_tridiagonal(it, lds);
            EEID_PHASE_MARK(t.clk, 5);
            t.de = t.dg + 2 * Band<S, NT>::SMALL_MAX;   // the (d, e^2) pairs after d and e, in LDS
            t.bisect(it.out, interlacing_bracket(args, it, &s_flag));
            t.de = lds;
            publish_eigenvalues(args, it);
            __syncthreads();
            EEID_PHASE_MARK(t.clk, 6);
            continue;
        }
        t.gather(it);
        __syncthreads();
        EEID_PHASE_MARK(t.clk, 0);
        t.reduce_to_band();
        __syncthreads();
        EEID_PHASE_MARK(t.clk, 4);
        t.band_to_tridiagonal(t.Tm, args.spin_limit, &args.flags[it.b]);
        EEID_PHASE_MARK(t.clk, 5);
        t.bisect(it.out, interlacing_bracket(args, it, &s_flag));
        publish_eigenvalues(args, it);
        __syncthreads();
        EEID_PHASE_MARK(t.clk, 6);
    }
    EEID_PHASE_MARK(t.clk, 7);
    t.clk.flush();
}

}  // namespace eeid
