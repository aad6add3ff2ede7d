// Kernels of the non-Hermitian path (guide: section "FEAST v3.0", dual
// subspaces Q, Q-hat for right and left eigenvectors, and Table
// "tab_common" for E, X, res).  Everything here is FP64 complex, column-major.
//
// The reduced pencil (Aq, Bq) = (Qh^H A Q, Qh^H B Q) is small (M0 x M0).  It
// is solved as the standard problem C = Bq^{-1} Aq: Householder reduction to
// Hessenberg form, the complex implicit single-shift QR algorithm to the
// Schur form T = Z^H C Z, eigenvectors of T by back substitution, W = Z Y.
// The left eigenvectors follow from the right ones: Wh^H = W^{-1} Bq^{-1}
// satisfies Wh^H Aq = Lambda Wh^H Bq.  One workgroup does each of these
// dense steps; the products between them are matrix-core products.
#pragma once

#include "common.hpp"

namespace fx {

__device__ inline double2 zmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 zscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ inline double zabs1(double2 a) { return fabs(a.x) + fabs(a.y); }
__device__ inline double zabs(double2 a) { return hypot(a.x, a.y); }
__device__ inline double2 zdiv(double2 a, double2 b)
{
    // Smith's algorithm
    if (fabs(b.x) >= fabs(b.y)) {
        const double r = b.y / b.x, d = b.x + b.y * r;
        return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
    }
    const double r = b.x / b.y, d = b.y + b.x * r;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__device__ inline double2 zsqrt(double2 a)
{
    const double m = zabs(a);
    if (m == 0.0) return make_double2(0.0, 0.0);
    double re = sqrt(0.5 * (m + fabs(a.x)));
    double im = 0.5 * a.y / re;
    if (a.x < 0.0) {
        const double t = fabs(im);
        im = copysign(re, a.y);
        re = t;
    }
    return make_double2(re, im);
}

// Quadrature of the full contour, right and left subspaces, in node order:
//   Q[:, c]  = rho_c X[:, c]        + sum_j coef[j][c]       Y_j[:, c]
//   Qh[:, c] = conj(rho_c) Xh[:, c] + sum_j conj(coef[j][c]) Yh_j[:, c]
// Plain form: coef[j][c] = w_j and no X term (rho = NULL); Y_j = (z_j B -
// A)^{-1} B X, Yh_j = (z_j B - A)^{-H} B^H Xh.  Correction form (mixed
// precision): Y_j, Yh_j solve against the Ritz residuals, coef[j][c] =
// w_j / (z_j - lambda_c) and rho_c = sum_j coef[j][c].  Y, Yh in the solve
// precision T (n x ncols, leading dimension ldy, stride sY); sums in FP64.
template <typename T>
__global__ __launch_bounds__(256) void accumulate_general_kernel(int n, int ncols, int ne, const cplx<T> *__restrict__ Y,
                                                                 const cplx<T> *__restrict__ Yh, long ldy, long sY,
                                                                 const double2 *__restrict__ coef,
                                                                 const double2 *__restrict__ rho,
                                                                 const double2 *__restrict__ X,
                                                                 const double2 *__restrict__ Xh, long ldx,
                                                                 double2 *__restrict__ Q, double2 *__restrict__ Qh,
                                                                 long ldq)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * ncols) return;
    const int i = (int)(idx % n), c = (int)(idx / n);
    double2 q = make_double2(0.0, 0.0), qh = make_double2(0.0, 0.0);
    for (int j = 0; j < ne; ++j) {
        const double2 w = coef[(long)j * ncols + c];
        const cplx<T> y = Y[j * sY + i + (long)c * ldy], yh = Yh[j * sY + i + (long)c * ldy];
        q = zadd(q, zmul(w, make_double2(y.x, y.y)));
        qh = zadd(qh, zmul(zconj(w), make_double2(yh.x, yh.y)));
    }
    if (rho) {
        const double2 r = rho[c];
        q = zadd(q, zmul(r, X[i + (long)c * ldx]));
        qh = zadd(qh, zmul(zconj(r), Xh[i + (long)c * ldx]));
    }
    Q[i + (long)c * ldq] = q;
    Qh[i + (long)c * ldq] = qh;
}

// R[:, c] = AX[:, c] - mu_c BX[:, c], mu_c = lam[c] or conj(lam[c]) (the
// right or left Ritz residual block of the correction form), FP64.
__global__ __launch_bounds__(256) void ritz_residual_general_kernel(int n, int ncols, const double2 *__restrict__ AX,
                                                                   const double2 *__restrict__ BX, long ld,
                                                                   const double2 *__restrict__ lam, int conj_lam,
                                                                   double2 *__restrict__ R)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * ncols) return;
    const int i = (int)(idx % n), c = (int)(idx / n);
    const double2 l = conj_lam ? zconj(lam[c]) : lam[c];
    R[i + (long)c * ld] = zsub(AX[i + (long)c * ld], zmul(l, BX[i + (long)c * ld]));
}

constexpr int NH_NT = 256;   // threads of the single-workgroup dense kernels
constexpr int NH_MAXM = 1024;

// Inverse of an m x m matrix by Gauss-Jordan elimination with partial
// pivoting (largest |re| + |im|, ties to the lowest row).  Mx is destroyed
// (left as is when LDSM > 0).  status = 0, or k + 1 when column k has no
// nonzero pivot.  NT threads; with LDSM > 0 (m <= LDSM) both matrices are
// worked on in LDS (leading dimension LDSM + 1) and Inv is written at the end.
template <int NT, int LDSM>
__global__ __launch_bounds__(NT) void gj_inverse_kernel(int m, double2 *__restrict__ Mg, double2 *__restrict__ Ig,
                                                        int *__restrict__ status)
{
    constexpr int HLD = LDSM > 0 ? LDSM + 1 : 1;
    __shared__ double2 Ms[LDSM > 0 ? HLD * LDSM : 1];
    __shared__ double2 Is[LDSM > 0 ? HLD * LDSM : 1];
    __shared__ double2 fcol[LDSM > 0 ? LDSM : NH_MAXM];
    __shared__ double s_v[NT / 64];
    __shared__ int s_i[NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const long ld = LDSM > 0 ? HLD : m;
    double2 *Mx = Mg, *Inv = Ig;
    if constexpr (LDSM > 0) {
        Mx = Ms;
        Inv = Is;
    }
    for (long e = tid; e < (long)m * m; e += NT) {
        const int i = (int)(e % m), j = (int)(e / m);
        Inv[i + j * ld] = make_double2(i == j ? 1.0 : 0.0, 0.0);
        if constexpr (LDSM > 0) Mx[i + j * ld] = Mg[e];
    }
    int fail = 0;
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        double best = -1.0;
        int bi = m;
        for (int i = k + tid; i < m; i += NT) {
            const double v = zabs1(Mx[i + (long)k * ld]);
            if (v > best) {
                best = v;
                bi = i;
            }
        }
        // argmax: within each wave by shuffles, then across the waves
        for (int off = 32; off > 0; off >>= 1) {
            const double v2 = __shfl_xor(best, off, 64);
            const int i2 = __shfl_xor(bi, off, 64);
            if (v2 > best || (v2 == best && i2 < bi)) {
                best = v2;
                bi = i2;
            }
        }
        if (lane == 0) {
            s_v[wid] = best;
            s_i[wid] = bi;
        }
        __syncthreads();
        double pv = s_v[0];
        int p = s_i[0];
        for (int w = 1; w < NT / 64; ++w)
            if (s_v[w] > pv || (s_v[w] == pv && s_i[w] < p)) {
                pv = s_v[w];
                p = s_i[w];
            }
        __syncthreads();
        if (!(pv > 0.0)) {
            fail = k + 1;
            break;
        }
        if (p != k) {
            for (int j = tid; j < m; j += NT) {
                const double2 a = Mx[k + (long)j * ld], b = Mx[p + (long)j * ld];
                Mx[k + (long)j * ld] = b;
                Mx[p + (long)j * ld] = a;
                const double2 c = Inv[k + (long)j * ld], d = Inv[p + (long)j * ld];
                Inv[k + (long)j * ld] = d;
                Inv[p + (long)j * ld] = c;
            }
        }
        __syncthreads();
        const double2 pinv = zdiv(make_double2(1.0, 0.0), Mx[k + (long)k * ld]);
        __syncthreads();
        for (int j = tid; j < m; j += NT) {
            if (j >= k) Mx[k + (long)j * ld] = zmul(Mx[k + (long)j * ld], pinv);
            Inv[k + (long)j * ld] = zmul(Inv[k + (long)j * ld], pinv);
        }
        __syncthreads();
        for (int i = tid; i < m; i += NT) fcol[i] = (i == k) ? make_double2(0.0, 0.0) : Mx[i + (long)k * ld];
        __syncthreads();
        for (long e = tid; e < (long)m * m; e += NT) {
            const int i = (int)(e % m), j = (int)(e / m);
            const double2 f = fcol[i];
            if (i == k || (f.x == 0.0 && f.y == 0.0)) continue;
            if (j >= k) Mx[i + j * ld] = zsub(Mx[i + j * ld], zmul(f, Mx[k + (long)j * ld]));
            Inv[i + j * ld] = zsub(Inv[i + j * ld], zmul(f, Inv[k + (long)j * ld]));
        }
        __syncthreads();
    }
    if constexpr (LDSM > 0) {
        for (long e = tid; e < (long)m * m; e += NT) Ig[e] = Inv[(e % m) + (e / m) * ld];
    }
    if (tid == 0) status[0] = fail;
}

// Eigenvalues and eigenvectors of a general complex m x m matrix (m <=
// NH_MAXM) held in H (destroyed).  Z (m x m) gets the unitary Schur vectors
// (C = Z T Z^H, T the Schur form), Y (m x m) the eigenvectors of T (upper
// triangular, Y[k][k] = 1), lam the eigenvalues T[k][k].  The caller forms
// W = Z Y.  status[0] = 0, or -1 when the QR iteration did not converge
// within 30 m sweeps; status[1] = sweeps.
// NT threads.  With LDSM > 0 (m <= LDSM) the working copy of H lives in LDS
// (leading dimension LDSM + 1): each Givens rotation then costs a few LDS
// accesses instead of dependent round trips to memory, which is what bounds
// this kernel; so does Z, written out at the end.
template <int NT, int LDSM>
__global__ __launch_bounds__(NT) void eig_general_kernel(int m, double2 *__restrict__ H, double2 *__restrict__ Z,
                                                         double2 *__restrict__ Y, double2 *__restrict__ lam,
                                                         int *__restrict__ status)
{
    constexpr int HLD = LDSM > 0 ? LDSM + 1 : 1;
    __shared__ double2 Hs[LDSM > 0 ? HLD * LDSM : 1];
    __shared__ double2 Zs[LDSM > 0 ? HLD * LDSM : 1];
    __shared__ double2 sv[LDSM > 0 ? LDSM : NH_MAXM];
    __shared__ double s_red[NT / 64];
    const int tid = threadIdx.x;
    const double ulp = 2.220446049250313e-16, smlnum = 2.2250738585072014e-308 * ((double)m / ulp);
    const long ldh = LDSM > 0 ? HLD : m;   // leading dimension of the working H and Z
    double2 *Hw = H, *Zw = Z;
    if constexpr (LDSM > 0) {
        for (long e = tid; e < (long)m * m; e += NT) Hs[(e % m) + (e / m) * HLD] = H[e];
        Hw = Hs;
        Zw = Zs;
    }
    auto at = [&](int i, int j) -> double2 & { return Hw[i + (long)j * ldh]; };
    auto block_sum = [&](double v) {
        v = wave_sum(v);
        if ((tid & 63) == 0) s_red[tid >> 6] = v;
        __syncthreads();
        double t = 0.0;
        for (int q = 0; q < NT / 64; ++q) t += s_red[q];
        __syncthreads();
        return t;
    };
    for (long e = tid; e < (long)m * m; e += NT) {
        const int i = (int)(e % m), j = (int)(e / m);
        Zw[i + j * ldh] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();

    // ---- Householder reduction to upper Hessenberg form, H <- P H P, Z <- Z P
    for (int k = 0; k + 2 < m; ++k) {
        const int L = m - k - 1;   // rows k+1 .. m-1 of column k
        double part = 0.0;
        for (int t = 1 + tid; t < L; t += NT) {
            const double2 x = at(k + 1 + t, k);
            part += x.x * x.x + x.y * x.y;
        }
        const double sig = block_sum(part);
        if (sig == 0.0) continue;   // column already reduced (uniform decision)
        const double2 x0 = at(k + 1, k);
        const double a0 = zabs(x0), xnorm = sqrt(a0 * a0 + sig);
        const double2 ph = a0 > 0.0 ? zscale(1.0 / a0, x0) : make_double2(1.0, 0.0);
        const double2 alpha = zscale(-xnorm, ph);
        const double beta = 1.0 / (xnorm * (xnorm + a0));   // 2 / ||v||^2
        for (int t = tid; t < L; t += NT) sv[t] = t == 0 ? zsub(x0, alpha) : at(k + 1 + t, k);
        __syncthreads();
        // left: columns k+1 .. m-1
        for (int j = k + 1 + tid; j < m; j += NT) {
            double2 d = make_double2(0.0, 0.0);
            for (int t = 0; t < L; ++t) d = zadd(d, zmul(zconj(sv[t]), at(k + 1 + t, j)));
            d = zscale(beta, d);
            for (int t = 0; t < L; ++t) at(k + 1 + t, j) = zsub(at(k + 1 + t, j), zmul(sv[t], d));
        }
        for (int t = tid; t < L; t += NT) at(k + 1 + t, k) = t == 0 ? alpha : make_double2(0.0, 0.0);
        __syncthreads();
        // right: rows 0 .. m-1 of H, and of Z
        for (int i = tid; i < 2 * m; i += NT) {
            double2 *Mx = i < m ? Hw : Zw;
            const long ld = ldh;
            const int r = i < m ? i : i - m;
            double2 d = make_double2(0.0, 0.0);
            for (int t = 0; t < L; ++t) d = zadd(d, zmul(Mx[r + (long)(k + 1 + t) * ld], sv[t]));
            d = zscale(beta, d);
            for (int t = 0; t < L; ++t)
                Mx[r + (long)(k + 1 + t) * ld] = zsub(Mx[r + (long)(k + 1 + t) * ld], zmul(d, zconj(sv[t])));
        }
        __syncthreads();
    }

    // a norm for the deflation test of zero diagonals
    double part = 0.0;
    for (long e = tid; e < (long)m * m; e += NT) part = fmax(part, zabs1(at((int)(e % m), (int)(e / m))));
    s_red[0] = 0.0;
    __syncthreads();
    {
        // max over the block through the wave maxima
        double v = part;
        for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
        __shared__ double s_max[NT / 64];
        if ((tid & 63) == 0) s_max[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int q = 0; q < NT / 64; ++q) t = fmax(t, s_max[q]);
            s_red[0] = t;
        }
        __syncthreads();
    }
    const double hnorm = s_red[0];
    __syncthreads();

    // ---- complex implicit single-shift QR on the Hessenberg matrix; the
    //      rotations are applied to whole rows and columns so that H ends as
    //      the full Schur form and Z accumulates them
    int hi = m - 1, its = 0, total = 0, fail = 0;
    while (hi >= 1) {
        // l: the last negligible subdiagonal entry at or below hi (0: none)
        int l = hi;
        if constexpr (NT == 64 && LDSM > 0 && LDSM <= 64) {
            // one wave: lane t tests position t, a ballot picks the largest
            bool small = false;
            if (tid >= 1 && tid <= hi) {
                double tst = zabs1(at(tid - 1, tid - 1)) + zabs1(at(tid, tid));
                if (tst == 0.0) tst = hnorm;
                small = zabs1(at(tid, tid - 1)) <= fmax(ulp * tst, smlnum);
            }
            const unsigned long long bal = __ballot(small);
            l = bal ? 63 - __clzll(bal) : 0;
        } else {
            for (; l >= 1; --l) {
                double tst = zabs1(at(l - 1, l - 1)) + zabs1(at(l, l));
                if (tst == 0.0) tst = hnorm;
                if (zabs1(at(l, l - 1)) <= fmax(ulp * tst, smlnum)) break;
            }
        }
        __syncthreads();
        if (l >= 1 && tid == 0) at(l, l - 1) = make_double2(0.0, 0.0);
        __syncthreads();
        if (l == hi) {
            --hi;
            its = 0;
            continue;
        }
        if (total >= 30 * m) {
            fail = 1;
            break;
        }
        double2 mu;
        if (its == 10) {
            mu = zadd(at(l, l), make_double2(0.75 * fabs(at(l + 1, l).x), 0.0));
        } else if (its == 20) {
            mu = zadd(at(hi, hi), make_double2(0.75 * fabs(at(hi, hi - 1).x), 0.0));
        } else {
            // eigenvalue of the trailing 2 x 2 block closer to its last diagonal
            const double2 a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
            const double2 half = zscale(0.5, zsub(a, d));
            const double2 disc = zsqrt(zadd(zmul(half, half), zmul(b, c)));
            const double2 mid = zscale(0.5, zadd(a, d));
            const double2 m1 = zadd(mid, disc), m2 = zsub(mid, disc);
            mu = zabs1(zsub(m1, d)) <= zabs1(zsub(m2, d)) ? m1 : m2;
        }
        for (int k = l; k < hi; ++k) {
            double2 x, y;
            if (k == l) {
                x = zsub(at(l, l), mu);
                y = at(l + 1, l);
            } else {
                x = at(k, k - 1);
                y = at(k + 1, k - 1);
            }
            // rotation G = [[c, s], [-conj(s), c]] with G [x; y] = [r; 0]
            double c;
            double2 sg;
            // moduli by plain square roots: the entries are of the order of
            // the matrix norm, far from overflow
            const double ax2 = x.x * x.x + x.y * x.y, ay2 = y.x * y.x + y.y * y.y;
            if (ay2 == 0.0) {
                c = 1.0;
                sg = make_double2(0.0, 0.0);
            } else if (ax2 == 0.0) {
                c = 0.0;
                sg = zscale(1.0 / sqrt(ay2), zconj(y));
            } else {
                const double ax = sqrt(ax2), inv = 1.0 / (ax * sqrt(ax2 + ay2));
                c = ax2 * inv;
                sg = zscale(inv, zmul(x, zconj(y)));
            }
            __syncthreads();   // every thread has read x and y
            const int j0 = k == l ? l : k - 1;
            for (int j = j0 + tid; j < m; j += NT) {
                const double2 h1 = at(k, j), h2 = at(k + 1, j);
                at(k, j) = zadd(zscale(c, h1), zmul(sg, h2));
                at(k + 1, j) = zsub(zscale(c, h2), zmul(zconj(sg), h1));
            }
            __syncthreads();
            const int iend = min(k + 2, hi);
            for (int i = tid; i < (iend + 1) + m; i += NT) {
                double2 *Mx = i <= iend ? Hw : Zw;
                const long ld = ldh;
                const int r = i <= iend ? i : i - (iend + 1);
                const double2 h1 = Mx[r + (long)k * ld], h2 = Mx[r + (long)(k + 1) * ld];
                Mx[r + (long)k * ld] = zadd(zscale(c, h1), zmul(h2, zconj(sg)));
                Mx[r + (long)(k + 1) * ld] = zsub(zscale(c, h2), zmul(h1, sg));
            }
            __syncthreads();
            if (k > l && tid == 0) at(k + 1, k - 1) = make_double2(0.0, 0.0);
            __syncthreads();
        }
        ++its;
        ++total;
    }
    __syncthreads();

    // ---- eigenvalues, and eigenvectors of the triangular T by back
    //      substitution (one column per thread): (T - t_kk) y = 0, y_k = 1
    for (int k = tid; k < m; k += NT) {
        const double2 tk = at(k, k);
        lam[k] = tk;
        const double smin = fmax(ulp * zabs1(tk), smlnum);
        for (int i = k + 1; i < m; ++i) Y[i + (long)k * m] = make_double2(0.0, 0.0);
        Y[k + (long)k * m] = make_double2(1.0, 0.0);
        for (int i = k - 1; i >= 0; --i) {
            double2 sum = make_double2(0.0, 0.0);
            for (int j = i + 1; j <= k; ++j) sum = zadd(sum, zmul(at(i, j), Y[j + (long)k * m]));
            double2 d = zsub(at(i, i), tk);
            if (zabs1(d) < smin) d = make_double2(smin, 0.0);
            Y[i + (long)k * m] = zdiv(make_double2(-sum.x, -sum.y), d);
        }
    }
    if constexpr (LDSM > 0) {
        for (long e = tid; e < (long)m * m; e += NT) Z[e] = Zw[(e % m) + (e / m) * ldh];
    }
    if (tid == 0) {
        status[0] = fail ? -1 : 0;
        status[1] = total;
    }
}

// Out (m x m) = In^H.
__global__ __launch_bounds__(256) void conj_transpose_kernel(int m, const double2 *__restrict__ In,
                                                             double2 *__restrict__ Out)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)m * m) return;
    const int i = (int)(e % m), j = (int)(e / m);
    Out[j + (long)i * m] = zconj(In[e]);
}

// Scale every column of X (n x ncols) to unit 2-norm.  One block per column.
__global__ __launch_bounds__(256) void normalize_cols_kernel(int n, double2 *__restrict__ X, long ldx)
{
    const int c = blockIdx.x, tid = threadIdx.x;
    double s = 0.0;
    for (int i = tid; i < n; i += 256) {
        const double2 v = X[i + (long)c * ldx];
        s += v.x * v.x + v.y * v.y;
    }
    __shared__ double sr[4];
    s = wave_sum(s);
    if ((tid & 63) == 0) sr[tid >> 6] = s;
    __syncthreads();
    const double nrm = sqrt(sr[0] + sr[1] + sr[2] + sr[3]);
    if (nrm == 0.0) return;
    const double inv = 1.0 / nrm;
    for (int i = tid; i < n; i += 256) X[i + (long)c * ldx] = zscale(inv, X[i + (long)c * ldx]);
}

// res[c] = ||AX[:, c] - mu_c BX[:, c]||_1 / (alpha ||BX[:, c]||_1), mu_c =
// lam[c] (right residual) or conj(lam[c]) (left residual, with AX = A^H Xh
// and BX = B^H Xh), Table "tab_common".  One block per column.
__global__ __launch_bounds__(256) void resid_general_kernel(int n, const double2 *__restrict__ AX,
                                                            const double2 *__restrict__ BX, long ld,
                                                            const double2 *__restrict__ lam, int conj_lam,
                                                            double alpha, double *__restrict__ res)
{
    const int c = blockIdx.x, tid = threadIdx.x;
    const double2 l = conj_lam ? zconj(lam[c]) : lam[c];
    double num = 0.0, den = 0.0;
    for (int i = tid; i < n; i += 256) {
        const double2 a = AX[i + (long)c * ld], b = BX[i + (long)c * ld];
        num += zabs(zsub(a, zmul(l, b)));
        den += zabs(b);
    }
    __shared__ double sn[4], sd[4];
    num = wave_sum(num);
    den = wave_sum(den);
    if ((tid & 63) == 0) {
        sn[tid >> 6] = num;
        sd[tid >> 6] = den;
    }
    __syncthreads();
    if (tid == 0) res[c] = (sn[0] + sn[1] + sn[2] + sn[3]) / (alpha * (sd[0] + sd[1] + sd[2] + sd[3]));
}

}  // namespace fx
