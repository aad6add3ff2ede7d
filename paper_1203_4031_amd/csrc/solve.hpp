// Multi-right-hand-side solves with the stored LU factors (the solve steps
// of the FEAST contour: ijob 11, and ijob 21 -- the adjoint -- for complex
// Hermitian pencils, reusing the same factors):
//   A_z Y = R   :  Y = U^{-1} L^{-1} P R
//   A_z^H Y = R :  Y = P^T L^{-H} U^{-H} R
// Blocked by NBS rows: a diagonal-block triangular solve (one thread per
// right-hand side, the block's triangle in LDS), then a matrix-core update
// of the remaining rows.  All contour nodes are solved in one launch per
// step (blockIdx.y / blockIdx.z = node).
#pragma once

#include "common.hpp"
#include "gemm.hpp"

namespace fx {

constexpr int SOLVE_NB = 64;

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

enum tri_mode { TRI_L = 0, TRI_U = 1, TRI_UH = 2, TRI_LH = 3 };

// Solve the w x w diagonal block at rows kb..kb+w-1 for every right-hand
// side.  MODE selects op(T): L (unit lower, forward), U (upper, backward),
// U^H (lower, forward), L^H (unit upper, backward).
template <typename T, int MODE, int NBS>
__global__ __launch_bounds__(64) void trsm_diag_kernel(int ncols, const cplx<T> *__restrict__ Fall,
                                                       long ldf, long sF, int kb, int w,
                                                       cplx<T> *__restrict__ Yall, long ldy, long sY)
{
    using V = cplx<T>;
    const V *a = Fall + blockIdx.y * sF;
    V *Y = Yall + blockIdx.y * sY;
    __shared__ V Tsh[NBS][NBS + 1];   // op(T)[i][l]
    const int tid = threadIdx.x;
    for (int e = tid; e < w * w; e += 64) {
        const int i = e % w, l = e / w;
        V v;
        if (MODE == TRI_L || MODE == TRI_U) v = a[(kb + i) + (long)(kb + l) * ldf];
        else v = cconj(a[(kb + l) + (long)(kb + i) * ldf]);
        Tsh[i][l] = v;
    }
    __syncthreads();
    const int c = blockIdx.x * 64 + tid;
    if (c >= ncols) return;
    V *y = Y + kb + (long)c * ldy;
    V x[NBS];
#pragma unroll
    for (int i = 0; i < NBS; ++i) x[i] = (i < w) ? y[i] : cmake<V>(0, 0);
    if constexpr (MODE == TRI_L || MODE == TRI_UH) {
#pragma unroll
        for (int i = 0; i < NBS; ++i) {
            if (i < w) {
                V s = x[i];
#pragma unroll
                for (int l = 0; l < i; ++l) s = csub(s, cmul(Tsh[i][l], x[l]));
                if constexpr (MODE == TRI_UH) s = cmul(s, cinv(Tsh[i][i]));
                x[i] = s;
            }
        }
    } else {
#pragma unroll
        for (int i = NBS - 1; i >= 0; --i) {
            if (i < w) {
                V s = x[i];
#pragma unroll
                for (int l = i + 1; l < NBS; ++l)
                    if (l < w) s = csub(s, cmul(Tsh[i][l], x[l]));
                if constexpr (MODE == TRI_U) s = cmul(s, cinv(Tsh[i][i]));
                x[i] = s;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NBS; ++i)
        if (i < w) y[i] = x[i];
}

template <typename T, int MODE>
static void trsm_diag(hipStream_t s, int ncols, const cplx<T> *F, long ldf, long sF, int kb, int w,
                      cplx<T> *Y, long ldy, long sY, int batch)
{
    dim3 grid(ceil_div(ncols, 64), batch);
    hipLaunchKernelGGL((trsm_diag_kernel<T, MODE, SOLVE_NB>), grid, dim3(64), 0, s, ncols, F, ldf, sF,
                       kb, w, Y, ldy, sY);
    FX_LAUNCH_CHECK();
}

// In place: Y_b <- A_b^{-1} Y_b (adjoint = false, Y already row-permuted) or
// Y_b <- U^{-H} then L^{-H} (adjoint = true, permutation applied afterwards
// by the caller).
template <typename T>
void getrs_batched(hipStream_t s, bool adjoint, int n, int ncols, const cplx<T> *F, long ldf, long sF,
                   cplx<T> *Y, long ldy, long sY, int batch)
{
    constexpr int NB = SOLVE_NB;
    const int nblk = ceil_div(n, NB);
    if (!adjoint) {
        for (int b = 0; b < nblk; ++b) {       // L, forward
            const int kb = b * NB, w = std::min(NB, n - kb);
            trsm_diag<T, TRI_L>(s, ncols, F, ldf, sF, kb, w, Y, ldy, sY, batch);
            if (kb + w < n)
                gemm<T, true, false>(s, n - kb - w, ncols, w, T(-1), F + (kb + w) + (long)kb * ldf, ldf,
                                     sF, Y + kb, ldy, sY, T(1), Y + kb + w, ldy, sY, batch);
        }
        for (int b = nblk - 1; b >= 0; --b) {  // U, backward
            const int kb = b * NB, w = std::min(NB, n - kb);
            trsm_diag<T, TRI_U>(s, ncols, F, ldf, sF, kb, w, Y, ldy, sY, batch);
            if (kb > 0)
                gemm<T, true, false>(s, kb, ncols, w, T(-1), F + (long)kb * ldf, ldf, sF, Y + kb, ldy,
                                     sY, T(1), Y, ldy, sY, batch);
        }
    } else {
        for (int b = 0; b < nblk; ++b) {       // U^H, forward
            const int kb = b * NB, w = std::min(NB, n - kb);
            trsm_diag<T, TRI_UH>(s, ncols, F, ldf, sF, kb, w, Y, ldy, sY, batch);
            if (kb + w < n)
                gemm<T, true, true>(s, n - kb - w, ncols, w, T(-1), F + kb + (long)(kb + w) * ldf, ldf,
                                    sF, Y + kb, ldy, sY, T(1), Y + kb + w, ldy, sY, batch);
        }
        for (int b = nblk - 1; b >= 0; --b) {  // L^H, backward
            const int kb = b * NB, w = std::min(NB, n - kb);
            trsm_diag<T, TRI_LH>(s, ncols, F, ldf, sF, kb, w, Y, ldy, sY, batch);
            if (kb > 0)
                gemm<T, true, true>(s, kb, ncols, w, T(-1), F + kb, ldf, sF, Y + kb, ldy, sY, T(1), Y,
                                    ldy, sY, batch);
        }
    }
}

}  // namespace fx
