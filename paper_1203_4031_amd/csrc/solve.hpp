// Multi-right-hand-side solves with the stored LU factors (the solve steps
// of the FEAST contour: ijob 11, and ijob 21 -- the adjoint -- for complex
// Hermitian pencils, reusing the same factors):
//   A_z Y = R   :  Y = U^{-1} L^{-1} P R
//   A_z^H Y = R :  Y = P^T L^{-H} U^{-H} R
// Blocked by solve_nb rows (128 in FP64, 64 in complex64), with the
// diagonal blocks of L and U inverted once per factorisation (128-row
// blocks from inverted 64 x 64 halves), so every step is a matrix-core
// product of that depth.  All contour nodes are
// solved in one launch per step (blockIdx.y / blockIdx.z = node).
#pragma once

#include "common.hpp"
#include "gemm.hpp"

namespace fx {

constexpr int TRI_INV_NB = 64;   // diagonal blocks inverted directly
// Solve block: 128 rows (two inverted halves composed) in FP64; 64 in
// complex64, where the explicit inverse of a 128-row triangle loses enough
// accuracy (its condition number times the unit roundoff) to cost the mixed
// path an extra FEAST loop.
template <typename T> constexpr int solve_nb() { return sizeof(T) == 8 ? 128 : 64; }

// Y_b[i, c] = R[perm_b[i], c] in the solve precision.  R is FP64 real or
// complex, shared by all nodes.
template <typename T, bool CPLX_IN>
__global__ __launch_bounds__(256) void gather_rows_kernel(int n, int ncols,
                                                          const int *__restrict__ perm_all, long sPiv,
                                                          const double *__restrict__ R, long ldr,
                                                          cplx<T> *__restrict__ Y, long ldy, long sY)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * ncols) return;
    const int i = (int)(idx % n), c = (int)(idx / n);
    const int src = perm_all[blockIdx.y * sPiv + i];
    cplx<T> v;
    if constexpr (CPLX_IN) {
        const double2 r = reinterpret_cast<const double2 *>(R)[src + c * ldr];
        v.x = (T)r.x;
        v.y = (T)r.y;
    } else {
        v.x = (T)R[src + c * ldr];
        v.y = T(0);
    }
    Y[blockIdx.y * sY + i + (long)c * ldy] = v;
}

// Y_b[:, c] = R[:, c] in the solve precision (adjoint solves permute last).
template <typename T, bool CPLX_IN>
__global__ __launch_bounds__(256) void copy_rhs_kernel(int n, int ncols, const double *__restrict__ R,
                                                       long ldr, cplx<T> *__restrict__ Y, long ldy,
                                                       long sY)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * ncols) return;
    const int i = (int)(idx % n), c = (int)(idx / n);
    cplx<T> v;
    if constexpr (CPLX_IN) {
        const double2 r = reinterpret_cast<const double2 *>(R)[i + c * ldr];
        v.x = (T)r.x;
        v.y = (T)r.y;
    } else {
        v.x = (T)R[i + c * ldr];
        v.y = T(0);
    }
    Y[blockIdx.y * sY + i + (long)c * ldy] = v;
}

// out_b[perm_b[i], c] = Y_b[i, c]  (applies P^T)
template <typename T>
__global__ __launch_bounds__(256) void scatter_rows_kernel(int n, int ncols,
                                                           const int *__restrict__ perm_all, long sPiv,
                                                           const cplx<T> *__restrict__ Y, long ldy,
                                                           long sY, cplx<T> *__restrict__ out,
                                                           long ldo, long sO)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * ncols) return;
    const int i = (int)(idx % n), c = (int)(idx / n);
    const int dst = perm_all[blockIdx.y * sPiv + i];
    out[blockIdx.y * sO + dst + (long)c * ldo] = Y[blockIdx.y * sY + i + (long)c * ldy];
}

// Inverses of the NBS x NBS diagonal blocks of L (unit lower) and U (upper)
// of every factor, computed once per factorisation: the triangular solves
// then consist of matrix products only.  One workgroup per (block, node);
// thread c solves for column c of the identity in LDS.
template <typename T, int NBS>
__global__ __launch_bounds__(NBS) void tri_inv_kernel(int n, const cplx<T> *__restrict__ Fall, long ldf,
                                                      long sF, cplx<T> *__restrict__ Linv_all,
                                                      cplx<T> *__restrict__ Uinv_all, long sInv)
{
    using V = cplx<T>;
    const int blk = blockIdx.x, kb = blk * NBS, w = min(NBS, n - kb);
    const V *a = Fall + blockIdx.y * sF;
    V *Li = Linv_all + blockIdx.y * sInv + (long)blk * NBS * NBS;
    V *Ui = Uinv_all + blockIdx.y * sInv + (long)blk * NBS * NBS;
    __shared__ V Tsh[NBS][NBS + 1];   // the diagonal block (L below, U on and above the diagonal)
    __shared__ V Xs[NBS][NBS + 1];    // column c of the inverse is owned by thread c
    const int c = threadIdx.x;
    for (int e = c; e < NBS * NBS; e += NBS) {
        const int i = e % NBS, l = e / NBS;
        Tsh[i][l] = (i < w && l < w) ? a[(kb + i) + (long)(kb + l) * ldf] : cmake<V>(i == l ? 1 : 0, 0);
    }
    __syncthreads();
    // Column c of each inverse, column-oriented substitution (once x_l is
    // final it updates every later row), so the dependency chain is NBS
    // steps long.
    // L^{-1}: forward substitution on e_c, unit diagonal
    for (int i = 0; i < NBS; ++i) Xs[i][c] = cmake<V>(i == c ? 1 : 0, 0);
    for (int l = c; l < NBS - 1; ++l) {
        const V xl = Xs[l][c];
        for (int i = l + 1; i < NBS; ++i) Xs[i][c] = csub(Xs[i][c], cmul(Tsh[i][l], xl));
    }
    for (int i = 0; i < NBS; ++i) Li[i + c * NBS] = Xs[i][c];
    // U^{-1}: backward substitution on e_c
    for (int i = 0; i < NBS; ++i) Xs[i][c] = cmake<V>(i == c ? 1 : 0, 0);
    for (int l = c; l >= 0; --l) {
        const V xl = cmul(Xs[l][c], cinv(Tsh[l][l]));
        Xs[l][c] = xl;
        for (int i = 0; i < l; ++i) Xs[i][c] = csub(Xs[i][c], cmul(Tsh[i][l], xl));
    }
    for (int i = 0; i < NBS; ++i) Ui[i + c * NBS] = Xs[i][c];
}

template <typename T>
void tri_inv_batched(hipStream_t s, int n, const cplx<T> *F, long ldf, long sF, cplx<T> *Linv, cplx<T> *Uinv,
                     long sInv, int batch)
{
    dim3 grid(ceil_div(n, TRI_INV_NB), batch);
    hipLaunchKernelGGL((tri_inv_kernel<T, TRI_INV_NB>), grid, dim3(TRI_INV_NB), 0, s, n, F, ldf, sF, Linv, Uinv,
                       sInv);
    FX_LAUNCH_CHECK();
}

inline long tri_inv_stride(int n) { return (long)ceil_div(n, TRI_INV_NB) * TRI_INV_NB * TRI_INV_NB; }
template <typename T> inline long solve_inv_stride(int n)
{
    return (long)ceil_div(n, solve_nb<T>()) * solve_nb<T>() * solve_nb<T>();
}

// 128 x 128 inverse blocks from the 64 x 64 ones: the diagonal halves are
// copied here (identity past the matrix end), the off-diagonal half is zero
// and, where both halves exist, filled by solve_inverses with
//   [[A, 0], [C, D]]^{-1} = [[A^{-1}, 0], [-D^{-1} C A^{-1}, D^{-1}]]   (L)
//   [[A, B], [0, D]]^{-1} = [[A^{-1}, -A^{-1} B D^{-1}], [0, D^{-1}]]   (U)
template <typename T>
__global__ __launch_bounds__(256) void inv128_assemble_kernel(int n, const cplx<T> *__restrict__ L64,
                                                              const cplx<T> *__restrict__ U64, long s64,
                                                              cplx<T> *__restrict__ L128, cplx<T> *__restrict__ U128,
                                                              long s128)
{
    using V = cplx<T>;
    constexpr int H = TRI_INV_NB, W = 2 * TRI_INV_NB;
    const int b = blockIdx.x, nb64 = (n + H - 1) / H;
    const V *l = L64 + blockIdx.y * s64, *u = U64 + blockIdx.y * s64;
    V *lo = L128 + blockIdx.y * s128 + (long)b * W * W, *uo = U128 + blockIdx.y * s128 + (long)b * W * W;
    for (int e = threadIdx.x; e < W * W; e += 256) {
        const int i = e % W, j = e / W, hi = i / H, hj = j / H;
        V lv = cmake<V>(0, 0), uv = cmake<V>(0, 0);
        if (hi == hj) {
            const int blk = 2 * b + hi;
            if (blk < nb64) {
                const long o = (long)blk * H * H + (i % H) + (long)(j % H) * H;
                lv = l[o];
                uv = u[o];
            } else if (i == j) {
                lv = uv = cmake<V>(1, 0);
            }
        }
        lo[e] = lv;
        uo[e] = uv;
    }
}

// Inverted diagonal blocks for the solves (L128, U128, stride s128, blocks
// of solve_nb rows).  For 128-row blocks: 64 x 64 inverses first (L64,
// U64, stride s64), then the composition; tmp: ceil(n / 128) * 64 * 64
// elements per matrix (stride stmp).  For 64-row blocks only L128/U128 are
// used.
template <typename T>
void solve_inverses(hipStream_t s, int n, const cplx<T> *F, long ldf, long sF, cplx<T> *L64, cplx<T> *U64, long s64,
                    cplx<T> *L128, cplx<T> *U128, long s128, cplx<T> *tmp, long stmp, int batch)
{
    constexpr int H = TRI_INV_NB, W = solve_nb<T>();
    constexpr long HH = (long)H * H, WW = (long)W * W;
    if constexpr (W == H) {   // the 64-row inverses are the solve blocks
        tri_inv_batched<T>(s, n, F, ldf, sF, L128, U128, s128, batch);
        return;
    } else {
    tri_inv_batched<T>(s, n, F, ldf, sF, L64, U64, s64, batch);
    const int nb128 = ceil_div(n, W);
    hipLaunchKernelGGL((inv128_assemble_kernel<T>), dim3(nb128, batch), dim3(256), 0, s, n, L64, U64, s64, L128, U128,
                       s128);
    FX_LAUNCH_CHECK();
    const int nfull = n / W;
    const long sFb = W + (long)W * ldf;   // one 128-block down the diagonal
    const T one = T(1), mone = T(-1), zero = T(0);
    if (nfull > 0) {
        // L: tmp = C A^{-1}, lower-left = -D^{-1} tmp
        gemm2<T, true, false>(s, H, H, H, one, F + H, ldf, sF, sFb, L64, H, s64, 2 * HH, zero, tmp, H, stmp, HH,
                              batch, nfull);
        gemm2<T, true, false>(s, H, H, H, mone, L64 + HH, H, s64, 2 * HH, tmp, H, stmp, HH, zero, L128 + H, W, s128,
                              WW, batch, nfull);
        // U: tmp = A^{-1} B, upper-right = -tmp D^{-1}
        gemm2<T, true, false>(s, H, H, H, one, U64, H, s64, 2 * HH, F + (long)H * ldf, ldf, sF, sFb, zero, tmp, H,
                              stmp, HH, batch, nfull);
        gemm2<T, true, false>(s, H, H, H, mone, tmp, H, stmp, HH, U64 + HH, H, s64, 2 * HH, zero, U128 + (long)H * W,
                              W, s128, WW, batch, nfull);
    }
    const int w = n - nfull * W;
    if (w > H) {   // a last, partial 128-block whose second half has w2 rows
        const int b = nfull, kb = b * W, w2 = w - H;
        const long o64a = (long)(2 * b) * HH, o64b = (long)(2 * b + 1) * HH, o128 = (long)b * WW;
        gemm<T, true, false>(s, w2, H, H, one, F + (kb + H) + (long)kb * ldf, ldf, sF, L64 + o64a, H, s64, zero, tmp,
                             H, stmp, batch);
        gemm<T, true, false>(s, w2, H, w2, mone, L64 + o64b, H, s64, tmp, H, stmp, zero, L128 + o128 + H, W, s128,
                             batch);
        gemm<T, true, false>(s, H, w2, H, one, U64 + o64a, H, s64, F + kb + (long)(kb + H) * ldf, ldf, sF, zero, tmp,
                             H, stmp, batch);
        gemm<T, true, false>(s, H, w2, w2, mone, tmp, H, stmp, U64 + o64b, H, s64, zero, U128 + o128 + (long)H * W, W,
                             s128, batch);
    }
    }
}

// W for the solves with A_z (not its adjoint): below each diagonal block b
// (NB = solve_nb rows), W = L_{.,b} Linv_b; above it, W = U_{.,b} Uinv_b.
// With it a triangular sweep is one product per block on the unscaled
// running right-hand side, and the diagonal inverses are applied once at
// the end (getrs_batched).  W has the factors' layout (ld ldf, stride sF);
// its diagonal blocks are not used.
template <typename T>
void build_w(hipStream_t s, int n, const cplx<T> *F, long ldf, long sF, const cplx<T> *Linv, const cplx<T> *Uinv,
             long sInv, cplx<T> *W, int batch)
{
    constexpr int NB = solve_nb<T>();
    constexpr long NN = (long)NB * NB;
    const int nfull = n / NB, w = n - nfull * NB;
    const long sdiag = NB + (long)NB * ldf;
    if (nfull > 0) {
        // L part of block b: rows (b + 1) NB .. n-1, i.e. n - NB - b NB rows
        gemm2<T, true, false>(s, n - NB, NB, NB, T(1), F + NB, ldf, sF, sdiag, Linv, NB, sInv, NN, T(0), W + NB, ldf,
                              sF, sdiag, batch, nfull, -NB);
        // U part of block b: rows 0 .. b NB - 1
        gemm2<T, true, false>(s, 0, NB, NB, T(1), F, ldf, sF, (long)NB * ldf, Uinv, NB, sInv, NN, T(0), W, ldf, sF,
                              (long)NB * ldf, batch, nfull, NB);
    }
    if (w > 0 && nfull > 0) {   // U part of a last, partial block
        const int kb = nfull * NB;
        gemm<T, true, false>(s, kb, w, w, T(1), F + (long)kb * ldf, ldf, sF, Uinv + nfull * NN, NB, sInv, T(0),
                             W + (long)kb * ldf, ldf, sF, batch);
    }
}

// Out = blockdiag(Dinv) In, both n x ncols (ld ldy, stride sY), one launch
// for the full blocks and one for a partial last block.
template <typename T>
static void apply_block_diag(hipStream_t s, int n, int ncols, const cplx<T> *Dinv, long sInv, const cplx<T> *In,
                             cplx<T> *Out, long ldy, long sY, int batch)
{
    constexpr int NB = solve_nb<T>();
    constexpr long NN = (long)NB * NB;
    const int nfull = n / NB, w = n - nfull * NB;
    if (nfull > 0)
        gemm2<T, true, false>(s, NB, ncols, NB, T(1), Dinv, NB, sInv, NN, In, ldy, sY, NB, T(0), Out, ldy, sY, NB,
                              batch, nfull);
    if (w > 0)
        gemm<T, true, false>(s, w, ncols, w, T(1), Dinv + nfull * NN, NB, sInv, In + nfull * NB, ldy, sY, T(0),
                             Out + nfull * NB, ldy, sY, batch);
}

// Multi-RHS solve with the stored factors using only matrix products:
//   adjoint = false:  Y <- U^{-1} L^{-1} Y   (Y already row-permuted)
//   adjoint = true:   Y <- L^{-H} U^{-H} Y   (row permutation applied by the caller)
// The sweeps alternate between Y and X, so the result ends in Y with no
// copies.  Dinv_b are the inverted diagonal blocks (NB = solve_nb rows).
// Solves with A_z use W (build_w): the diagonal inverses go last, and the
// blocks are taken in groups of GB as below (each block updates the later
// blocks of its group, the rows past the group get one product of the
// group's depth, 256), so the right-hand side is swept once per group
// rather than once per block.  Adjoint solves:
// block b of the forward sweep is X_b = Dinv_b^H Y_b, then the rows below
// get -= T^H X_b; blocks are taken in groups of GB (four 64-row blocks in
// complex64, two 128-row blocks in FP64): inside a group the later blocks
// are updated block by block, the rows past the group get one product of
// the group's depth (256).  Measured at N = 4096, 300 columns, 8 nodes, per
// solve of 4 loops: 19.0 ms with groups of one, 17.1 with depth 128, 16.7
// with depth 256.
template <typename T>
void getrs_batched(hipStream_t s, bool adjoint, int n, int ncols, const cplx<T> *F, const cplx<T> *W, long ldf,
                   long sF, const cplx<T> *Linv, const cplx<T> *Uinv, long sInv, cplx<T> *Y, cplx<T> *X, long ldy,
                   long sY, int batch)
{
    constexpr int NB = solve_nb<T>();
    constexpr int GB = 256 / NB;   // blocks per group
    const int nblk = ceil_div(n, NB), ngrp = ceil_div(nblk, GB);
    auto inv_blk = [&](const cplx<T> *base, int b) { return base + (long)b * NB * NB; };
    auto grp = [&](int g, int &gs, int &ge, int &b0, int &b1) {   // rows [gs, ge), blocks [b0, b1)
        b0 = g * GB;
        b1 = std::min(nblk, b0 + GB);
        gs = b0 * NB;
        ge = std::min(n, b1 * NB);
    };
    int gs, ge, b0, b1;
    if (!adjoint) {
        // L, forward, on Y in place with W, then X = blockdiag(Linv) Y.
        // Within a group each block updates the group's later blocks; the
        // rows past the group get one product of the group's depth.
        for (int g = 0; g < ngrp; ++g) {
            grp(g, gs, ge, b0, b1);
            for (int b = b0; b < b1; ++b) {
                const int kb = b * NB, w = std::min(NB, n - kb);
                if (kb + w < ge)
                    gemm<T, true, false>(s, ge - kb - w, ncols, w, T(-1), W + (kb + w) + (long)kb * ldf, ldf, sF,
                                         Y + kb, ldy, sY, T(1), Y + kb + w, ldy, sY, batch);
            }
            if (ge < n)
                gemm<T, true, false>(s, n - ge, ncols, ge - gs, T(-1), W + ge + (long)gs * ldf, ldf, sF, Y + gs, ldy,
                                     sY, T(1), Y + ge, ldy, sY, batch);
        }
        apply_block_diag<T>(s, n, ncols, Linv, sInv, Y, X, ldy, sY, batch);
        // U, backward, on X in place with W, then Y = blockdiag(Uinv) X
        for (int g = ngrp - 1; g >= 0; --g) {
            grp(g, gs, ge, b0, b1);
            for (int b = b1 - 1; b >= b0; --b) {
                const int kb = b * NB, w = std::min(NB, n - kb);
                if (kb > gs)
                    gemm<T, true, false>(s, kb - gs, ncols, w, T(-1), W + gs + (long)kb * ldf, ldf, sF, X + kb, ldy,
                                         sY, T(1), X + gs, ldy, sY, batch);
            }
            if (gs > 0)
                gemm<T, true, false>(s, gs, ncols, ge - gs, T(-1), W + (long)gs * ldf, ldf, sF, X + gs, ldy, sY,
                                     T(1), X, ldy, sY, batch);
        }
        apply_block_diag<T>(s, n, ncols, Uinv, sInv, X, Y, ldy, sY, batch);
    } else {
        for (int g = 0; g < ngrp; ++g) {       // U^H, forward: Y -> X
            grp(g, gs, ge, b0, b1);
            for (int b = b0; b < b1; ++b) {
                const int kb = b * NB, w = std::min(NB, n - kb);
                gemm<T, true, true>(s, w, ncols, w, T(1), inv_blk(Uinv, b), NB, sInv, Y + kb, ldy, sY, T(0),
                                    X + kb, ldy, sY, batch);
                if (kb + w < ge)
                    gemm<T, true, true>(s, ge - kb - w, ncols, w, T(-1), F + kb + (long)(kb + w) * ldf, ldf, sF,
                                        X + kb, ldy, sY, T(1), Y + kb + w, ldy, sY, batch);
            }
            if (ge < n)
                gemm<T, true, true>(s, n - ge, ncols, ge - gs, T(-1), F + gs + (long)ge * ldf, ldf, sF, X + gs, ldy,
                                    sY, T(1), Y + ge, ldy, sY, batch);
        }
        for (int g = ngrp - 1; g >= 0; --g) {  // L^H, backward: X -> Y
            grp(g, gs, ge, b0, b1);
            for (int b = b1 - 1; b >= b0; --b) {
                const int kb = b * NB, w = std::min(NB, n - kb);
                gemm<T, true, true>(s, w, ncols, w, T(1), inv_blk(Linv, b), NB, sInv, X + kb, ldy, sY, T(0),
                                    Y + kb, ldy, sY, batch);
                if (kb > gs)
                    gemm<T, true, true>(s, kb - gs, ncols, w, T(-1), F + kb + (long)gs * ldf, ldf, sF, Y + kb, ldy,
                                        sY, T(1), X + gs, ldy, sY, batch);
            }
            if (gs > 0)
                gemm<T, true, true>(s, gs, ncols, ge - gs, T(-1), F + gs, ldf, sF, Y + gs, ldy, sY, T(1), X, ldy, sY,
                                    batch);
        }
    }
}

}  // namespace fx
