// Complex Hermitian counterpart of eeid_tridiag.hpp: eigenvalues of Hermitian
// matrices and of all their principal minors, one workgroup per problem.
//
// The Householder reduction of a Hermitian matrix (Section 2 of the paper
// states the identity for Hermitian A; real symmetric is the special case)
// yields a REAL symmetric tridiagonal when every reflector H = I - tau u u^H
// is chosen so that H^H x = beta e_1 with beta real: tau = (beta - alpha) /
// beta, u = [1; x(2:) / (alpha - beta)], beta = -sign(Re alpha) ||x||.  The
// Sturm bisection of eeid_tridiag.hpp then applies unchanged.
//
// Per column (lower storage, panel of NB columns, V and W hold the panel):
//   x      = M(:,k) - V W(k,:)^H - W V(k,:)^H             (column update)
//   y      = M_stale u, corrected by - V (W^H u) - W (V^H u)
//   W(:,i) = tau y + alpha2 u,  alpha2 = -|tau|^2 Re(y^H u) / 2
// and per panel M -= V W^H + W V^H on the trailing tiles (each complex
// product as four real MFMAs).
//
// Storage: complex elements of type R (double: C128, float: C64 = the FP32
// trailing-update form) in 64x64 tiles as for the real kernel; within a tile
// complex (r, c) sits at (c / CV) * 64 * CV + r * CV + c % CV, CV = complex
// elements per 16 bytes.  Accumulation (V, W, u, y) is complex double.
#pragma once
#include "eeid_tridiag.hpp"

namespace eeid {

struct cd {
    double re, im;
};

__device__ __forceinline__ cd cz() { return cd{0.0, 0.0}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cmul(cd a, cd b) { return cd{fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)}; }
__device__ __forceinline__ cd cconj(cd a) { return cd{a.re, -a.im}; }
__device__ __forceinline__ cd cscale(double s, cd a) { return cd{s * a.re, s * a.im}; }
// s + a * b
__device__ __forceinline__ cd cfma(cd a, cd b, cd s) {
    return cd{fma(a.re, b.re, fma(-a.im, b.im, s.re)), fma(a.re, b.im, fma(a.im, b.re, s.im))};
}
// s + conj(a) * b
__device__ __forceinline__ cd cfmac(cd a, cd b, cd s) {
    return cd{fma(a.re, b.re, fma(a.im, b.im, s.re)), fma(a.re, b.im, fma(-a.im, b.re, s.im))};
}
__device__ __forceinline__ cd cselect(bool c, cd a, cd b) { return cd{c ? a.re : b.re, c ? a.im : b.im}; }
__device__ __forceinline__ cd cshfl(cd a, int src) { return cd{__shfl(a.re, src), __shfl(a.im, src)}; }

// Element (p, q) of the Hermitian matrix whose lower triangle is A
// (interleaved (re, im), row-major, order n); the diagonal's imaginary part is ignored.
__device__ __forceinline__ cd herm_at(const double *A, int n, int p, int q) {
    if (p > q) return cd{A[2 * ((int64_t)p * n + q)], A[2 * ((int64_t)p * n + q) + 1]};
    if (p < q) return cd{A[2 * ((int64_t)q * n + p)], -A[2 * ((int64_t)q * n + p) + 1]};
    return cd{A[2 * ((int64_t)p * n + p)], 0.0};
}

// Element (p, q), p, q != r, of B = R^H A R with R a rotation by pi/4 in the
// (r, k) plane.  rot 0: new basis e'_r = (e_r + e_k)/sqrt2, e'_k = (e_k - e_r)/sqrt2,
// so component r of eigenvector i of B is (v_ir + v_ik)/sqrt2 and Eq. (2) at r
// gives (W_ir + W_ik)/2 + Re(conj(v_ir) v_ik); rot 1: e'_r = (e_r + i e_k)/sqrt2,
// e'_k = (e_k + i e_r)/sqrt2, component r is (v_ir - i v_ik)/sqrt2 and Eq. (2)
// gives (W_ir + W_ik)/2 + Im(conj(v_ir) v_ik).  Only row and column k of the
// minor at r differ from A's.
__device__ __forceinline__ cd herm_rotated_at(const double *A, int n, int r, int k, int rot, int p, int q) {
    constexpr double h = 0.70710678118654752440;   // 1/sqrt2
    if (p == k && q == k) {
        const cd akr = herm_at(A, n, k, r);
        const double dd = herm_at(A, n, k, k).re + herm_at(A, n, r, r).re;
        return cd{rot ? 0.5 * dd - akr.im : 0.5 * dd - akr.re, 0.0};
    }
    if (p == k) {   // e'_k^H A e_q
        const cd a = herm_at(A, n, k, q), b = herm_at(A, n, r, q);
        return rot ? cd{h * (a.re + b.im), h * (a.im - b.re)} : cd{h * (a.re - b.re), h * (a.im - b.im)};
    }
    if (q == k) {   // e_p^H A e'_k = conj(e'_k^H A e_p)
        const cd a = herm_at(A, n, p, k), b = herm_at(A, n, p, r);
        return rot ? cd{h * (a.re - b.im), h * (a.im + b.re)} : cd{h * (a.re - b.re), h * (a.im - b.im)};
    }
    return herm_at(A, n, p, q);
}

template <class R> struct CVec;
template <> struct CVec<double> { static constexpr int CV = 1; typedef double2 type; };
template <> struct CVec<float> { static constexpr int CV = 2; typedef float4 type; };

template <class R>
__device__ __forceinline__ int ctile_off(int r, int c) {
    constexpr int CV = CVec<R>::CV;
    return (c / CV) * (TILE * CV) + r * CV + (c % CV);
}

template <int NB>
struct PanelC {
    double tau_re, tau_im, alpha2, atb;
    cd a[NB], b[NB];    // a = W^H u, b = V^H u of the latest column
    cd vk[NB], wk[NB];  // row k of V and W for the next column
};

template <class R, int NB, int NT, int CW>
struct TriC {
    static constexpr int NWAVE = NT / 64;
    static constexpr int RED = 4 * NB + 8;  // doubles per wave in red[]
    typedef typename CVec<R>::type VT;
    static constexpr int CV = CVec<R>::CV;
    static constexpr int NV = CW / CV;      // 16-byte vectors per lane per tile in the SYMV

    R *tiles;
    cd *V, *Wm;
    double *dg, *eg;
    cd *y, *u;
    double *red;
    PanelC<NB> *P;
    int m, T, LD;
    int tid, lane, wave;

    __device__ R *tile_ptr(int I, int J) const { return tiles + tile_index(I, J, T) * (2 * TILE_ELEMS); }

    __device__ cd Mget(int r, int c) const {
        const R *p = tile_ptr(r / TILE, c / TILE) + 2 * ctile_off<R>(r % TILE, c % TILE);
        return cd{(double)p[0], (double)p[1]};
    }

    // -------------------------------------------------------------- gather
    __device__ void gather(const Item &it) {
        const int n = it.n, j = it.j;
        const double *A = it.src;  // interleaved (re, im), row-major
        for (int J = 0; J < T; ++J)
            for (int I = J; I < T; ++I) {
                R *tp = tile_ptr(I, J);
                for (int q = tid; q < TILE_ELEMS; q += NT) {
                    const int cp = q / (TILE * CV), rem = q % (TILE * CV);
                    const int r = rem / CV, c = cp * CV + rem % CV;
                    const int row = I * TILE + r, col = J * TILE + c;
                    double vr = 0.0, vi = 0.0;
                    if (row < m && col < m) {
                        const int rs = row + ((j >= 0 && row >= j) ? 1 : 0);
                        const int cs = col + ((j >= 0 && col >= j) ? 1 : 0);
                        const cd v = (it.k >= 0) ? herm_rotated_at(A, n, j, it.k, it.rot, rs, cs) : herm_at(A, n, rs, cs);
                        vr = v.re;
                        vi = v.im;
                    }
                    tp[2 * q] = (R)vr;
                    tp[2 * q + 1] = (R)vi;
                }
            }
    }

    // ---------------------------------------------------- column update (pass A)
    __device__ void column_pass(int k, int i) {
        const cd tau_p = cd{P->tau_re, P->tau_im};
        const double a2_p = P->alpha2;
        double accp = 0.0, accq = 0.0, sig = 0.0;
        for (int r0 = k; r0 < m; r0 += NT) {
            asm volatile("" ::: "memory");  // panel scalars are re-read from LDS per row
            const int r = r0 + tid;
            const bool live = r < m;
            cd vr[NB], wr[NB];
#pragma unroll
            for (int l = 0; l < NB; ++l) { vr[l] = cz(); wr[l] = cz(); }
            if (live) {
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
            cd x = cz();
            if (live) {
                if (i > 0) {
                    cd sf = cz();
#pragma unroll
                    for (int l = 0; l < NB; ++l) sf = cfma(vr[l], P->a[l], cfma(wr[l], P->b[l], sf));
                    cd vlast = cz();
#pragma unroll
                    for (int l = 0; l < NB; ++l) vlast = cselect(l == i - 1, vr[l], vlast);
                    cd wnew = cz();
                    if (tau_p.re != 0.0 || tau_p.im != 0.0)
                        wnew = cadd(cmul(tau_p, csub(y[r], sf)), cscale(a2_p, vlast));
                    if (r > k) Wm[(int64_t)(i - 1) * LD + r] = wnew;  // row k: written by the previous tail
#pragma unroll
                    for (int l = 0; l < NB; ++l) wr[l] = cselect(l == i - 1, wnew, wr[l]);
                }
                cd sx = cz();
#pragma unroll
                for (int l = 0; l < NB; ++l) sx = cfma(vr[l], cconj(P->wk[l]), cfma(wr[l], cconj(P->vk[l]), sx));
                x = csub(Mget(r, k), sx);
                u[r] = x;
                if (r == k) dg[k] = x.re;
            }
            const cd xd = (live && r >= k + 2) ? x : cz();
            sig = fma(xd.re, xd.re, fma(xd.im, xd.im, sig));
            if (i > 0) {
                double bp[2 * NB];
#pragma unroll
                for (int l = 0; l < NB; ++l) {  // conj(W(r,l)) x, conj(V(r,l)) x
                    const cd t = cfmac(wr[l], xd, cz());
                    bp[2 * l] = t.re; bp[2 * l + 1] = t.im;
                }
                accp += wave_transpose_sum<2 * NB>(bp, lane);
#pragma unroll
                for (int l = 0; l < NB; ++l) {
                    const cd t = cfmac(vr[l], xd, cz());
                    bp[2 * l] = t.re; bp[2 * l + 1] = t.im;
                }
                accq += wave_transpose_sum<2 * NB>(bp, lane);
            }
        }
        sig = wave_sum(sig);
        static_assert(2 * NB == 32, "complex column pass assumes NB = 16");
        if ((lane & 1) == 0) {
            red[wave * RED + (lane >> 1)] = accp;           // p flattened (re, im)
            red[wave * RED + 2 * NB + (lane >> 1)] = accq;  // q flattened
        }
        if (lane == 0) red[wave * RED + 4 * NB] = sig;
    }

    __device__ void finalize_pass(int r_lo, int i) {
        const cd tau = cd{P->tau_re, P->tau_im};
        const double a2 = P->alpha2;
        const bool zero = (tau.re == 0.0 && tau.im == 0.0);
        for (int r = r_lo + tid; r < m; r += NT) {
            cd sf = cz();
            for (int l = 0; l < i; ++l)
                sf = cfma(V[(int64_t)l * LD + r], P->a[l], cfma(Wm[(int64_t)l * LD + r], P->b[l], sf));
            const cd vl = V[(int64_t)i * LD + r];
            Wm[(int64_t)i * LD + r] = zero ? cz() : cadd(cmul(tau, csub(y[r], sf)), cscale(a2, vl));
        }
    }

    // ------------------------------------------------------------------- SYMV
    // Hermitian: y_I += M_IJ u_J (row product) and y_J += M_IJ^H u_I (column
    // product) for off-diagonal tiles; diagonal tiles hold both triangles.
    __device__ void symv_unit(int J, int h, int Ib, int Ie, int k) {
        const int c0 = J * TILE + h * CW;
        double pc[2 * CW];
#pragma unroll
        for (int c = 0; c < 2 * CW; ++c) pc[c] = 0.0;
        for (int I = Ib; I < Ie; ++I) {
            int uo = c0;
            asm volatile("" : "+v"(uo));  // u(c0 .. c0+CW) is re-read from LDS, not held in registers
            const R *tp = tile_ptr(I, J) + 2 * (h * CW * TILE);
            const int row = I * TILE + lane;
            const bool live = row > k;
            VT buf[NV];
            if (live) {
#pragma unroll
                for (int q = 0; q < NV; ++q) buf[q] = *reinterpret_cast<const VT *>(tp + 2 * (q * TILE * CV + lane * CV));
            } else {
#pragma unroll
                for (int q = 0; q < NV; ++q) buf[q] = VT{};
            }
            cd s = cz();
            const bool off = (I != J);
            const cd ui = u[row];
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const int q = c / CV, z = 2 * (c % CV);
                const cd a = cd{(double)buf[q][z], (double)buf[q][z + 1]};
                s = cfma(a, u[uo + c], s);
                if (off) {
                    const cd t = cfmac(a, ui, cd{pc[2 * c], pc[2 * c + 1]});
                    pc[2 * c] = t.re; pc[2 * c + 1] = t.im;
                }
            }
            if (live) {
                atomicAdd(&y[row].re, s.re);
                atomicAdd(&y[row].im, s.im);
            }
        }
        if (Ie > Ib + (Ib == J ? 1 : 0)) {
            const double tot = wave_transpose_sum<2 * CW>(pc, lane);  // flattened index lane >> 1
            if ((lane & 1) == 0) {
                const int f = lane >> 1;
                double *yc = reinterpret_cast<double *>(&y[c0 + (f >> 1)]);
                atomicAdd(yc + (f & 1), tot);
            }
        }
    }

    __device__ void symv(int k) {
        const int J0 = (k + 1) / TILE;
        int cnt = 0;
        auto take = [&](int J, int h, int Ib, int Ie) {
            const int r = cnt / NWAVE, c = cnt % NWAVE;
            const int w = (r & 1) ? (NWAVE - 1 - c) : c;
            ++cnt;
            if (w == wave) symv_unit(J, h, Ib, Ie, k);
        };
        for (int J = J0; J < T; ++J)
            for (int h = 0; h < TILE / CW; ++h) {
                if (J * TILE + h * CW + CW - 1 < k + 1) continue;
                for (int s0 = J; s0 + SEG <= T; s0 += SEG) take(J, h, s0, s0 + SEG);
            }
        for (int L = SEG - 1; L >= 1; --L)
            for (int J = T - L; J >= J0; J -= SEG)
                for (int h = 0; h < TILE / CW; ++h) {
                    if (J * TILE + h * CW + CW - 1 < k + 1) continue;
                    take(J, h, T - L, T);
                }
    }

    // ------------------------------------------------------------------ SYR2K
    // C(I, J) -= V_I W_J^H + W_I V_J^H.  With X_I one of (V_I, W_I) and Y_J the
    // other: Re dC = Xr Yr^T + Xi Yi^T, Im dC = Xi Yr^T - Xr Yi^T, each a real
    // 16x16x4 MFMA on the transposed block (A operand = J side, B = I side).
    __device__ void syr2k_tile(int I, int J) {
        R *tp = tile_ptr(I, J);
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll 1
        for (int ib = 0; ib < 4; ++ib) {
            if constexpr (sizeof(R) == 8) {
                dbl4 are[4], aim[4];
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) { are[jb] = dbl4{0, 0, 0, 0}; aim[jb] = dbl4{0, 0, 0, 0}; }
#pragma unroll 2
                for (int kk = 0; kk < NB; kk += 4) {
                    const int64_t col = (int64_t)(kk + lk) * LD;
                    const cd vi = V[col + I * TILE + ib * 16 + lr], wi = Wm[col + I * TILE + ib * 16 + lr];
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb) {
                        const cd vj = V[col + J * TILE + jb * 16 + lr], wj = Wm[col + J * TILE + jb * 16 + lr];
                        // X = V, Y = W
                        are[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(wj.re, vi.re, are[jb], 0, 0, 0);
                        are[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(wj.im, vi.im, are[jb], 0, 0, 0);
                        aim[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(wj.re, vi.im, aim[jb], 0, 0, 0);
                        aim[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-wj.im, vi.re, aim[jb], 0, 0, 0);
                        // X = W, Y = V
                        are[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(vj.re, wi.re, are[jb], 0, 0, 0);
                        are[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(vj.im, wi.im, are[jb], 0, 0, 0);
                        aim[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(vj.re, wi.im, aim[jb], 0, 0, 0);
                        aim[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-vj.im, wi.re, aim[jb], 0, 0, 0);
                    }
                }
                // f64 layout: register g of lane (lr + 16 lk) = dC(ib*16 + lr, jb*16 + lk + 4g)
                const int row = ib * 16 + lr;
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        double2 *p = reinterpret_cast<double2 *>(tp + 2 * ctile_off<R>(row, jb * 16 + lk + 4 * g));
                        double2 c = *p;
                        c.x -= are[jb][g];
                        c.y -= aim[jb][g];
                        *p = c;
                    }
            } else {
                flt4 are[4], aim[4];
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) { are[jb] = flt4{0, 0, 0, 0}; aim[jb] = flt4{0, 0, 0, 0}; }
#pragma unroll 2
                for (int kk = 0; kk < NB; kk += 4) {
                    const int64_t col = (int64_t)(kk + lk) * LD;
                    const cd vi = V[col + I * TILE + ib * 16 + lr], wi = Wm[col + I * TILE + ib * 16 + lr];
                    const float vir = (float)vi.re, vii = (float)vi.im, wir = (float)wi.re, wii = (float)wi.im;
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb) {
                        const cd vj = V[col + J * TILE + jb * 16 + lr], wj = Wm[col + J * TILE + jb * 16 + lr];
                        const float vjr = (float)vj.re, vji = (float)vj.im, wjr = (float)wj.re, wji = (float)wj.im;
                        are[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wjr, vir, are[jb], 0, 0, 0);
                        are[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wji, vii, are[jb], 0, 0, 0);
                        aim[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wjr, vii, aim[jb], 0, 0, 0);
                        aim[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(-wji, vir, aim[jb], 0, 0, 0);
                        are[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(vjr, wir, are[jb], 0, 0, 0);
                        are[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(vji, wii, are[jb], 0, 0, 0);
                        aim[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(vjr, wii, aim[jb], 0, 0, 0);
                        aim[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(-vji, wir, aim[jb], 0, 0, 0);
                    }
                }
                // f32 layout: register g of lane (lr + 16 lk) = dC(ib*16 + lr, jb*16 + 4 lk + g)
                const int row = ib * 16 + lr;
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                    for (int g2 = 0; g2 < 4; g2 += 2) {  // two complex floats per 16 bytes
                        float4 *p = reinterpret_cast<float4 *>(tp + 2 * ctile_off<R>(row, jb * 16 + 4 * lk + g2));
                        float4 c = *p;
                        c.x -= are[jb][g2]; c.y -= aim[jb][g2];
                        c.z -= are[jb][g2 + 1]; c.w -= aim[jb][g2 + 1];
                        *p = c;
                    }
            }
        }
    }

    __device__ void syr2k(int J1) {
        int cnt = 0;
        for (int J = J1; J < T; ++J)
            for (int I = J; I < T; ++I)
                if ((cnt++ % NWAVE) == wave) syr2k_tile(I, J);
    }

    // --------------------------------------------------------- tridiagonalise
    __device__ void tridiagonalize() {
        for (int r = tid; r < LD; r += NT) u[r] = cz();
        if (tid < NB) { P->vk[tid] = cz(); P->wk[tid] = cz(); P->a[tid] = cz(); P->b[tid] = cz(); }
        if (tid == 0) { P->tau_re = 0.0; P->tau_im = 0.0; P->alpha2 = 0.0; }
        __syncthreads();
        for (int k0 = 0; k0 < m; k0 += NB) {
            const int nbe = min(NB, m - k0);
            {
                const int rz = (k0 / TILE) * TILE, len = LD - rz;
                for (int q = tid; q < NB * len; q += NT) {
                    const int l = q / len, r = rz + q % len;
                    V[(int64_t)l * LD + r] = cz();
                    Wm[(int64_t)l * LD + r] = cz();
                }
            }
            __syncthreads();
            for (int i = 0; i < nbe; ++i) {
                const int k = k0 + i;
                column_pass(k, i);
                __syncthreads();
                if (k == m - 1) break;
                // -------- reflector (wave 0)
                if (wave == 0) {
                    double s = 0.0, sig = 0.0;
                    for (int w = 0; w < NWAVE; ++w) {
                        s += red[w * RED + lane];  // lanes 0..2NB-1: p, 2NB..4NB-1: q (flattened)
                        sig += red[w * RED + 4 * NB];
                    }
                    const int c = lane & (NB - 1);
                    const cd p = cd{__shfl(s, 2 * c), __shfl(s, 2 * c + 1)};
                    const cd q = cd{__shfl(s, 2 * NB + 2 * c), __shfl(s, 2 * NB + 2 * c + 1)};
                    const cd alpha = u[k + 1];
                    double beta, tre, tim;
                    cd scal;
                    if (sig == 0.0 && alpha.im == 0.0) {
                        beta = alpha.re; tre = 0.0; tim = 0.0; scal = cz();
                    } else {
                        const double nrm = sqrt(fma(alpha.re, alpha.re, fma(alpha.im, alpha.im, sig)));
                        beta = (alpha.re >= 0.0) ? -nrm : nrm;
                        tre = (beta - alpha.re) / beta;
                        tim = -alpha.im / beta;
                        const cd dd = cd{alpha.re - beta, alpha.im};
                        const double den = dd.re * dd.re + dd.im * dd.im;
                        scal = cd{dd.re / den, -dd.im / den};
                    }
                    cd al = cz(), bl = cz();
                    if (lane < i) {
                        al = cadd(cconj(Wm[(int64_t)lane * LD + k + 1]), cmul(scal, p));
                        bl = cadd(cconj(V[(int64_t)lane * LD + k + 1]), cmul(scal, q));
                    }
                    const double atb = wave_sum(al.re * bl.re + al.im * bl.im);  // Re(a^H b)
                    if (lane < NB) { P->a[lane] = al; P->b[lane] = bl; }
                    if (lane == 0) {
                        P->tau_re = tre; P->tau_im = tim; P->atb = atb;
                        red[NWAVE * RED] = scal.re;
                        red[NWAVE * RED + 1] = scal.im;
                        eg[k] = beta;
                    }
                }
                __syncthreads();
                const bool tau_nz = (P->tau_re != 0.0 || P->tau_im != 0.0);
                const cd scal = cd{red[NWAVE * RED], red[NWAVE * RED + 1]};
                for (int r = k + tid; r < LD; r += NT) {
                    cd v = cz();
                    if (r == k + 1) v = cd{1.0, 0.0};
                    else if (r > k + 1 && r < m) v = cmul(u[r], scal);
                    u[r] = v;
                    if (r > k) V[(int64_t)i * LD + r] = v;
                }
                for (int r = ((k + 1) / TILE) * TILE + tid; r < LD; r += NT) y[r] = cz();
                __syncthreads();
                if (tau_nz) symv(k);
                __syncthreads();
                {
                    double s = 0.0;
                    for (int r = k + 1 + tid; r < m; r += NT) s = fma(y[r].re, u[r].re, fma(y[r].im, u[r].im, s));
                    s = wave_sum(s);
                    if (lane == 0) red[wave * RED + 4 * NB + 1] = s;
                }
                __syncthreads();
                if (wave == 0) {
                    double s = 0.0;
                    for (int w = 0; w < NWAVE; ++w) s += red[w * RED + 4 * NB + 1];
                    const cd tau = cd{P->tau_re, P->tau_im};
                    const double t2 = tau.re * tau.re + tau.im * tau.im;
                    const double a2 = -0.5 * t2 * (s - 2.0 * P->atb);
                    const int kn = k + 1;
                    cd vn = cz(), wn = cz();
                    if (lane < i) {
                        vn = V[(int64_t)lane * LD + kn];
                        wn = Wm[(int64_t)lane * LD + kn];
                    }
                    const cd term = (lane < i) ? cfma(vn, P->a[lane & (NB - 1)], cmul(wn, P->b[lane & (NB - 1)])) : cz();
                    const cd sf = cd{wave_sum(term.re), wave_sum(term.im)};
                    const cd wkn = tau_nz ? cadd(cmul(tau, csub(y[kn], sf)), cd{a2, 0.0}) : cz();
                    if (lane < NB) {
                        P->vk[lane] = (lane < i) ? vn : (lane == i ? cd{1.0, 0.0} : cz());
                        P->wk[lane] = (lane < i) ? wn : (lane == i ? wkn : cz());
                    }
                    if (lane == 0) {
                        P->alpha2 = a2;
                        Wm[(int64_t)i * LD + kn] = wkn;
                    }
                }
                __syncthreads();
            }
            const int klast = k0 + nbe - 1;
            if (klast < m - 1) {
                finalize_pass(klast + 2, nbe - 1);
                __syncthreads();
                syr2k((k0 + nbe) / TILE);
                __syncthreads();
                if (tid < NB) { P->vk[tid] = cz(); P->wk[tid] = cz(); }
                __syncthreads();
            }
        }
    }

    __device__ void bisect(double *out, const double *brk) {
        bisect_tridiagonal<NT, 4>(dg, eg, m, out, reinterpret_cast<double *>(y), red, tid, lane, wave, brk);
    }
};

template <class R, int NB>
__host__ __device__ inline int64_t slot_bytes_c(int LDmax) {
    const int64_t T = LDmax / TILE;
    const int64_t tiles = T * (T + 1) / 2 * TILE_ELEMS * 2 * (int64_t)sizeof(R);
    const int64_t panel = 2 * (int64_t)NB * LDmax * 16;
    const int64_t de = 2 * (int64_t)LDmax * 8;
    return ((tiles + 255) / 256) * 256 + panel + de;
}

template <int NB, int NT>
__host__ __device__ inline int64_t lds_bytes_c(int LDmax) {
    return 2 * (int64_t)LDmax * 16 + ((NT / 64) * (4 * NB + 8) + 8) * 8 + (int64_t)sizeof(PanelC<NB>) + 64;
}

template <class R, int NB, int NT, int CW>
__global__ __launch_bounds__(NT, 2) void tridiag_bisect_kernel_c(TriArgs args) {
    extern __shared__ double lds[];
    __shared__ int s_item;
    __shared__ unsigned long long s_flag;
    TriC<R, NB, NT, CW> t;
    t.tid = threadIdx.x;
    t.lane = threadIdx.x & 63;
    t.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int LDmax = args.LDmax;
    t.y = reinterpret_cast<cd *>(lds);
    t.u = t.y + LDmax;
    t.red = reinterpret_cast<double *>(t.u + LDmax);
    t.P = reinterpret_cast<PanelC<NB> *>(t.red + (NT / 64) * (4 * NB + 8) + 8);
    char *slot = args.work + (int64_t)blockIdx.x * args.slot_bytes;
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
        t.m = it.m;
        t.T = (it.m + TILE - 1) / TILE;
        t.LD = t.T * TILE;
        t.tiles = reinterpret_cast<R *>(slot);
        const int64_t T = t.T;
        const int64_t tile_bytes = ((T * (T + 1) / 2 * TILE_ELEMS * 2 * (int64_t)sizeof(R) + 255) / 256) * 256;
        t.V = reinterpret_cast<cd *>(slot + tile_bytes);
        t.Wm = t.V + (int64_t)NB * t.LD;
        t.dg = reinterpret_cast<double *>(t.Wm + (int64_t)NB * t.LD);
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
