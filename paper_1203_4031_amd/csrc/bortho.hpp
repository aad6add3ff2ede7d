// B-orthonormalisation of the Rayleigh-Ritz basis without an eigensolve.
//
// Given Bq = Q^H B Q (m x m, Hermitian positive semi-definite), build T with
// T^H Bq T = I on a subset of the columns of Q:
//   1. d = diag(Bq)^{-1/2},  Bt = D Bq D  (unit diagonal)
//   2. Bt = L L^H by left-looking Cholesky in column order; a column whose
//      Schur-complement pivot is <= tol is numerically dependent on the
//      columns before it and is dropped (its column of L is zero)
//   3. T = D * (L_KK)^{-H} on the kept index set K (zero rows elsewhere),
//      obtained from a blocked backward sweep with inverted 64 x 64
//      diagonal blocks and matrix-core updates.
// A pivot below -neg_tol means B is not positive definite (info -3).
#pragma once

#include "common.hpp"
#include "gemm.hpp"
#include "jacobi.hpp"

namespace fx {

constexpr int CHOL_MAXM = 1024;   // one row per thread
// Columns per left-looking block.  A block costs one global round trip per
// 32 (real) or 8 (complex) earlier columns, so wider blocks mean fewer round
// trips; 16 columns fit the registers of a 512-thread launch
// (m <= 512), not of a 1024-thread one.
template <bool CPLX, int NT> constexpr int chol_cb() { return NT <= 512 ? 16 : 8; }
constexpr int TRI_NB = 64;

// d_i = 1 / sqrt(Re Bq_ii); status[0] = -3 if some diagonal is not positive
template <bool CPLX>
__global__ __launch_bounds__(256) void diag_rsqrt_kernel(int m, const typename jelem<CPLX>::type *Bq, long ld,
                                                         double *d, int *status)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const double v = jre(Bq[i + (long)i * ld]);
    if (!(v > 0.0)) {
        status[0] = -3;
        d[i] = 0.0;
    } else {
        d[i] = 1.0 / sqrt(v);
    }
}

// out[a, b] = d_i d_j in[i, j] with i = ord[a], j = ord[b]  (symmetric
// permutation: the Cholesky then visits the columns in the order ord)
template <bool CPLX>
__global__ __launch_bounds__(256) void sym_scale_kernel(int m, const typename jelem<CPLX>::type *in, long ldi,
                                                        const double *d, const int *ord,
                                                        typename jelem<CPLX>::type *out, long ldo)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)m * m) return;
    const int a = (int)(e % m), b = (int)(e / m);
    const int i = ord[a], j = ord[b];
    const double s = d[i] * d[j];
    typename jelem<CPLX>::type v = in[i + (long)j * ldi];
    if constexpr (CPLX) v = make_double2(v.x * s, v.y * s);
    else v = v * s;
    out[a + (long)b * ldo] = v;
}

template <bool CPLX>
__global__ __launch_bounds__(256) void set_identity_kernel(int r, typename jelem<CPLX>::type *X, long ld)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)r * r) return;
    const int a = (int)(e % r), b = (int)(e / r);
    X[a + (long)b * ld] = jreal<typename jelem<CPLX>::type>(a == b ? 1.0 : 0.0);
}

// Left-looking Cholesky with column dropping, one workgroup, thread i owns
// row i.  L (m x m, lower, column-major) receives the factor; keep[j] = 1
// for kept columns.  status[0] = -3 on a negative pivot, status[1] = rank.
template <bool CPLX, int NT>
__global__ __launch_bounds__(NT) void chol_drop_kernel(int m, const typename jelem<CPLX>::type *Bt, long ldb,
                                                              typename jelem<CPLX>::type *L, long ldl, int *keep,
                                                              double tol, double neg_tol, int *status)
{
    using E = typename jelem<CPLX>::type;
    constexpr int CHOL_CB = chol_cb<CPLX, NT>();
    __shared__ E Lrow[CHOL_CB][NT];   // rows k0.. of L, previous columns
    __shared__ E pv[CHOL_CB];
    __shared__ int s_bad, s_rank;
    const int i = threadIdx.x;
    if (i == 0) {
        s_bad = 0;
        s_rank = 0;
    }
    __syncthreads();
    // rows of L are fetched this many columns at a time, all loads issued
    // before the multiply-adds, so the left-looking sum is not bound by one
    // memory round trip per column
    constexpr int CH = CPLX ? 8 : 32;
    for (int k0 = 0; k0 < m; k0 += CHOL_CB) {
        const int cb = min(CHOL_CB, m - k0);
        for (int e = i; e < CHOL_CB * k0; e += NT) {
            const int c = e % CHOL_CB, j = e / CHOL_CB;
            Lrow[c][j] = (c < cb) ? L[(k0 + c) + (long)j * ldl] : jzero<E>();   // zero rows past the end
        }
        __syncthreads();
        E w[CHOL_CB];
        const bool mine = i >= k0 && i < m;
#pragma unroll
        for (int c = 0; c < CHOL_CB; ++c)
            w[c] = (mine && c < cb) ? Bt[i + (long)(k0 + c) * ldb] : jzero<E>();
        if (mine) {
            int j = 0;
            for (; j + CH <= k0; j += CH) {
                E lv[CH];
#pragma unroll
                for (int u = 0; u < CH; ++u) lv[u] = L[i + (long)(j + u) * ldl];
#pragma unroll
                for (int u = 0; u < CH; ++u)
#pragma unroll
                    for (int c = 0; c < CHOL_CB; ++c) w[c] = jsub(w[c], jmul(lv[u], jconj(Lrow[c][j + u])));
            }
            for (; j < k0; ++j) {
                const E lij = L[i + (long)j * ldl];
#pragma unroll
                for (int c = 0; c < CHOL_CB; ++c) w[c] = jsub(w[c], jmul(lij, jconj(Lrow[c][j])));
            }
        }
#pragma unroll
        for (int c = 0; c < CHOL_CB; ++c) {
            if (c < cb) {
                const int kk = k0 + c;
                if (i >= kk && i < k0 + cb) pv[i - k0] = w[c];   // column c of the diagonal block rows
                __syncthreads();
                const double dpiv = jre(pv[c]);
                const bool kept = dpiv > tol;
                if (i == 0) {
                    if (dpiv < -neg_tol) s_bad = 1;
                    if (kept) s_rank += 1;
                    keep[kk] = kept ? 1 : 0;
                }
                const double lkk = kept ? sqrt(dpiv) : 0.0;
                const double rl = kept ? 1.0 / lkk : 0.0;
                if (mine) {
                    if (i == kk) {
                        w[c] = jreal<E>(lkk);
                    } else if (i > kk) {
                        const E l = jmul(jreal<E>(rl), w[c]);
                        w[c] = l;
#pragma unroll
                        for (int c2 = 0; c2 < CHOL_CB; ++c2)
                            if (c2 > c && c2 < cb)
                                w[c2] = jadd(w[c2], jmul(jreal<E>(-rl), jmul(l, jconj(pv[c2]))));
                    }
                }
                __syncthreads();
            }
        }
        // column block k0..k0+cb of L: rows above the diagonal are zero
#pragma unroll
        for (int c = 0; c < CHOL_CB; ++c) {
            if (c < cb && i < m) L[i + (long)(k0 + c) * ldl] = (i >= k0 + c) ? w[c] : jzero<E>();
        }
        __syncthreads();
    }
    if (i == 0) {
        status[0] = s_bad ? -3 : 0;
        status[1] = s_rank;
    }
}

// Kept columns only: Lk (r x r) = L[K, K] (K in the Cholesky's order)
template <bool CPLX>
__global__ __launch_bounds__(256) void gather_kk_kernel(int r, const int *idx, const typename jelem<CPLX>::type *L,
                                                        long ldl, typename jelem<CPLX>::type *Lk, long ldk)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)r * r) return;
    const int a = (int)(e % r), b = (int)(e / r);
    Lk[a + (long)b * ldk] = (a >= b) ? L[idx[a] + (long)idx[b] * ldl] : jzero<typename jelem<CPLX>::type>();
}

// Inverses of the TRI_NB diagonal blocks of a lower-triangular (non-unit)
// matrix; thread c forms column c of the block inverse by forward
// substitution in LDS.  Blocks past r are padded with the identity.
template <bool CPLX>
__global__ __launch_bounds__(TRI_NB) void lower_block_inv_kernel(int r, const typename jelem<CPLX>::type *Lk,
                                                                 long ldk, typename jelem<CPLX>::type *Dinv)
{
    using E = typename jelem<CPLX>::type;
    const int b = blockIdx.x, kb = b * TRI_NB, w = min(TRI_NB, r - kb);
    __shared__ E Ls[TRI_NB][TRI_NB + 1];
    __shared__ E Xs[TRI_NB][TRI_NB + 1];
    const int c = threadIdx.x;
    for (int e = c; e < TRI_NB * TRI_NB; e += TRI_NB) {
        const int i = e % TRI_NB, l = e / TRI_NB;
        Ls[i][l] = (i < w && l < w) ? Lk[(kb + i) + (long)(kb + l) * ldk] : jreal<E>(i == l ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int i = 0; i < TRI_NB; ++i) {
        E s = jreal<E>(i == c ? 1.0 : 0.0);
        for (int l = c; l < i; ++l) s = jadd(s, jmul(jreal<E>(-1.0), jmul(Ls[i][l], Xs[l][c])));
        // divide by the (real, positive) diagonal of the Cholesky factor
        Xs[i][c] = (i < c) ? jzero<E>() : jmul(jreal<E>(1.0 / jre(Ls[i][i])), s);
    }
    E *out = Dinv + (long)b * TRI_NB * TRI_NB;
    for (int i = 0; i < TRI_NB; ++i) out[i + c * TRI_NB] = Xs[i][c];
}

// Tm[i, c] = d_i T[row_of[i], c] for kept original indices i, zero for the
// dropped ones; Tm is m x r.
template <bool CPLX>
__global__ __launch_bounds__(256) void scatter_scale_rows_kernel(int m, int r, const double *d,
                                                                 const typename jelem<CPLX>::type *T, long ldt,
                                                                 typename jelem<CPLX>::type *Tm, long ldm,
                                                                 const int *row_of)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)m * r) return;
    const int i = (int)(e % m), c = (int)(e / m);
    const int a = row_of[i];   // -1 for dropped indices
    typename jelem<CPLX>::type v = jzero<typename jelem<CPLX>::type>();
    if (a >= 0) {
        v = T[a + (long)c * ldt];
        if constexpr (CPLX) v = make_double2(v.x * d[i], v.y * d[i]);
        else v = v * d[i];
    }
    Tm[i + (long)c * ldm] = v;
}

// T = Lk^{-H} (r x r, upper): backward sweep on the identity with the
// inverted diagonal blocks, every step a matrix-core product.  X is scratch
// of the same size.  The result ends in T.
template <bool CPLX>
void lower_inv_h(hipStream_t s, int r, const typename jelem<CPLX>::type *Lk, long ldk,
                 const typename jelem<CPLX>::type *Dinv, typename jelem<CPLX>::type *T,
                 typename jelem<CPLX>::type *X, long ld)
{
    using E = typename jelem<CPLX>::type;
    const int nblk = ceil_div(r, TRI_NB);
    // X = I
    // solve L^H T = X for block rows b = nblk-1 .. 0:
    //   T_b = Dinv_b^H X_b;  X_{0:kb} -= (L_{b, 0:kb})^H T_b
    for (int b = nblk - 1; b >= 0; --b) {
        const int kb = b * TRI_NB, w = std::min(TRI_NB, r - kb);
        gemm<double, CPLX, true>(s, w, r, w, 1.0, Dinv + (long)b * TRI_NB * TRI_NB, TRI_NB, 0, X + kb, ld, 0, 0.0,
                                 T + kb, ld, 0, 1);
        if (kb > 0)
            gemm<double, CPLX, true>(s, kb, r, w, -1.0, Lk + kb, ldk, 0, T + kb, ld, 0, 1.0, X, ld, 0, 1);
    }
    (void)sizeof(E);
}

}  // namespace fx
