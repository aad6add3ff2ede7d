// B-orthonormalisation of the Rayleigh-Ritz basis without an eigensolve.
//
// Given Bq = Q^H B Q (m x m, Hermitian positive semi-definite), build T with
// T^H Bq T = I on a subset of the columns of Q:
//   1. d = diag(Bq)^{-1/2},  Bt = D Bq D  (unit diagonal)
//   2. Bt = L L^H by right-looking blocked Cholesky in column order; a
//      column whose Schur-complement pivot is <= tol is numerically
//      dependent on the columns before it and is dropped (its column of L
//      is zero)
//   3. T = D * (L_KK)^{-H} on the kept index set K (zero rows elsewhere),
//      obtained from a blocked backward sweep with inverted 64 x 64
//      diagonal blocks and matrix-core updates.
// A pivot below -neg_tol means B is not positive definite (info -3).
#pragma once

#include "common.hpp"
#include "gemm.hpp"
#include "jacobi.hpp"

namespace fx {

constexpr int CHOL_MAXM = 1024;   // larger subspaces take the eigendecomposition of Bq
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

// One panel [k0, k0 + nb) of the right-looking blocked Cholesky with column
// dropping, in place on S (lower triangle: the Schur complement left by the
// earlier panels' trailing updates).  Every workgroup factors the nb x nb
// diagonal block itself -- the same operations in the same order, so the
// same bits -- together with its own CHP_NT - CHP_NB rows below it, so no
// workgroup waits for another.  One thread per row.  At column c the pivot
// and the diagonal rows' column-c entries go through LDS (double-buffered:
// one barrier per column); a pivot <= tol drops the column (its L column is
// zero), one below -neg_tol flags an indefinite B.  Writes L's panel columns
// into S (zero above the diagonal), their conjugate transpose below the
// diagonal block into P (CHP_NB x m) for the trailing update, and, from
// workgroup 0, keep flags and status (status[0] = -3 on a negative pivot,
// status[1] += kept columns; status starts at zero).
constexpr int CHP_NB = 32;
constexpr int CHP_NT = 256;
template <bool CPLX>
__global__ __launch_bounds__(CHP_NT) void chol_panel_kernel(int m, int k0, typename jelem<CPLX>::type *S, long lds,
                                                            typename jelem<CPLX>::type *P, int *keep, double tol,
                                                            double neg_tol, int *status)
{
    using E = typename jelem<CPLX>::type;
    constexpr int NB = CHP_NB, BELOW = CHP_NT - CHP_NB;
    __shared__ E col[2][NB];
    __shared__ double piv[2];
    const int tid = threadIdx.x;
    const int nb = min(NB, m - k0);
    const bool diag = tid < NB;
    const int row = diag ? k0 + tid : k0 + nb + blockIdx.x * BELOW + (tid - NB);
    const bool live = diag ? tid < nb : row < m;
    E w[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) w[c] = (live && c < nb) ? S[row + (long)(k0 + c) * lds] : jzero<E>();
    int rank = 0, bad = 0;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        if (c < nb) {   // uniform
            const int b = c & 1;
            if (tid == c) piv[b] = jre(w[c]);
            if (diag && tid > c && tid < nb) col[b][tid] = w[c];
            __syncthreads();
            const double p = piv[b];
            const bool kept = p > tol;
            const double lcc = kept ? sqrt(p) : 0.0;
            const double rl = kept ? 1.0 / lcc : 0.0;
            if (tid == c) {
                w[c] = jreal<E>(lcc);
            } else if (!diag || tid > c) {
                // l_ic = w_ic / l_cc; w_ij -= l_ic conj(l_jc) = (w_ic / l_cc^2) conj(w_jc)
                const E lr = jscale(w[c], rl * rl);
                w[c] = jscale(w[c], rl);
#pragma unroll
                for (int j = c + 1; j < NB; ++j)
                    if (j < nb) w[j] = jsub(w[j], jmul(lr, jconj(col[b][j])));
            }
            if (tid == 0) {
                bad |= (p < -neg_tol) ? 1 : 0;
                rank += kept ? 1 : 0;
                if (blockIdx.x == 0) keep[k0 + c] = kept ? 1 : 0;
            }
        }
    }
    if (diag) {
        if (blockIdx.x == 0 && live)
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < nb) S[row + (long)(k0 + c) * lds] = (c <= tid) ? w[c] : jzero<E>();
    } else if (live) {
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (c < nb) {
                S[row + (long)(k0 + c) * lds] = w[c];
                P[c + (long)row * NB] = jconj(w[c]);
            }
        }
    }
    if (blockIdx.x == 0 && tid == 0) {
        if (bad) status[0] = -3;
        status[1] += rank;
    }
}

// Cholesky with column dropping of the m x m matrix S, in place (lower
// triangle), by panels of CHP_NB columns: panel kernel, then the trailing
// update S22 -= P^H P on the matrix cores.  P is CHP_NB x m scratch.
template <bool CPLX>
void chol_drop_blocked(hipStream_t s, int m, typename jelem<CPLX>::type *S, long lds, typename jelem<CPLX>::type *P,
                       int *keep, double tol, double neg_tol, int *status)
{
    for (int k0 = 0; k0 < m; k0 += CHP_NB) {
        const int nb = std::min(CHP_NB, m - k0), below = m - k0 - nb;
        const int g = std::max(1, ceil_div(below, CHP_NT - CHP_NB));
        hipLaunchKernelGGL((chol_panel_kernel<CPLX>), dim3(g), dim3(CHP_NT), 0, s, m, k0, S, lds, P, keep, tol,
                           neg_tol, status);
        FX_LAUNCH_CHECK();
        if (below > 0) {
            const long o = k0 + nb;
            gemm<double, CPLX, true>(s, below, below, nb, -1.0, P + o * CHP_NB, CHP_NB, 0, P + o * CHP_NB, CHP_NB, 0,
                                     1.0, S + o + o * lds, lds, 0, 1);
        }
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
// matrix, one workgroup per block, by recursive doubling: the four 16 x 16
// diagonal blocks by forward substitution (a thread per column), then pairs
// of inverted blocks merged as
//   [[A, 0], [C, D]]^{-1} = [[A^{-1}, 0], [-D^{-1} C A^{-1}, D^{-1}]]
// at width 16 and then 32, each merge two small products in LDS.  Blocks past
// r are padded with the identity.
constexpr int TRI_NT = 256;
template <bool CPLX>
__global__ __launch_bounds__(TRI_NT) void lower_block_inv_kernel(int r, const typename jelem<CPLX>::type *Lk,
                                                                 long ldk, typename jelem<CPLX>::type *Dinv)
{
    using E = typename jelem<CPLX>::type;
    static_assert(TRI_NB == 64, "four 16-wide diagonal blocks, merged twice");
    const int b = blockIdx.x, kb = b * TRI_NB, w = min(TRI_NB, r - kb);
    __shared__ E Ls[TRI_NB][TRI_NB + 1];
    __shared__ E Xs[TRI_NB][TRI_NB + 1];
    __shared__ E Ts[TRI_NB * TRI_NB / 4];
    const int t = threadIdx.x;
    for (int e = t; e < TRI_NB * TRI_NB; e += TRI_NT) {
        const int i = e % TRI_NB, l = e / TRI_NB;
        Ls[i][l] = (i < w && l < w) ? Lk[(kb + i) + (long)(kb + l) * ldk] : jreal<E>(i == l ? 1.0 : 0.0);
        Xs[i][l] = jzero<E>();
    }
    __syncthreads();
    if (t < 64) {
        const int o = (t >> 4) * 16, c = t & 15;
        E x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            E sacc = jreal<E>(i == c ? 1.0 : 0.0);
#pragma unroll
            for (int l = 0; l < i; ++l) sacc = jsub(sacc, jmul(Ls[o + i][o + l], x[l]));
            // divide by the (real, positive) diagonal of the Cholesky factor
            x[i] = (i < c) ? jzero<E>() : jscale(sacc, 1.0 / jre(Ls[o + i][o + i]));
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) Xs[o + i][o + c] = x[i];
    }
    __syncthreads();
    for (int h = 16; h < TRI_NB; h *= 2) {
        const int npair = TRI_NB / (2 * h);
        // T = C A^{-1} (A^{-1} lower triangular: k >= j)
        for (int e = t; e < npair * h * h; e += TRI_NT) {
            const int pq = e / (h * h), i = e % h, j = (e / h) % h, o = pq * 2 * h;
            E sacc = jzero<E>();
            for (int k = j; k < h; ++k) sacc = jadd(sacc, jmul(Ls[o + h + i][o + k], Xs[o + k][o + j]));
            Ts[e] = sacc;
        }
        __syncthreads();
        // X21 = -D^{-1} T (D^{-1} lower triangular: k <= i)
        for (int e = t; e < npair * h * h; e += TRI_NT) {
            const int pq = e / (h * h), i = e % h, j = (e / h) % h, o = pq * 2 * h;
            E sacc = jzero<E>();
            for (int k = 0; k <= i; ++k) sacc = jsub(sacc, jmul(Xs[o + h + i][o + h + k], Ts[pq * h * h + k + j * h]));
            Xs[o + h + i][o + j] = sacc;
        }
        __syncthreads();
    }
    E *out = Dinv + (long)b * TRI_NB * TRI_NB;
    for (int e = t; e < TRI_NB * TRI_NB; e += TRI_NT) out[e] = Xs[e % TRI_NB][e / TRI_NB];
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
