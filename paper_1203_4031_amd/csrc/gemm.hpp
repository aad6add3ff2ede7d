// Batched dense matrix product on the gfx950 matrix cores:
//   C = alpha * op(A) * B + beta * C,  op(A) = A or A^H (A^T for real data),
// column-major operands, one batch entry per blockIdx.z.
//
// Complex products are four real 16x16x4 MFMAs on the real and imaginary
// parts of interleaved {re, im} elements.  The MFMA computes the transposed
// tile (B^T A^T) so that the 16 lanes sharing an accumulator register hold
// 16 consecutive rows of one column of C: stores to column-major C are then
// contiguous.  Tiles are staged through LDS, k-major with one element of
// padding per row.
#pragma once

#include "common.hpp"

namespace fx {

template <typename T, bool CPLX> struct elem { using type = T; };
template <typename T> struct elem<T, true> { using type = cplx<T>; };

template <typename E> __device__ inline E zero_elem();
template <> __device__ inline float zero_elem<float>() { return 0.f; }
template <> __device__ inline double zero_elem<double>() { return 0.0; }
template <> __device__ inline float2 zero_elem<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ inline double2 zero_elem<double2>() { return make_double2(0.0, 0.0); }

template <typename E> __device__ inline E conj_elem(E v) { return v; }
template <> __device__ inline float2 conj_elem<float2>(float2 v) { return make_float2(v.x, -v.y); }
template <> __device__ inline double2 conj_elem<double2>(double2 v) { return make_double2(v.x, -v.y); }

template <typename T, bool CPLX, bool OPA_H, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64) void gemm_kernel(
    int m, int n, int k, T alpha, const typename elem<T, CPLX>::type *__restrict__ A, long lda,
    long sA, const typename elem<T, CPLX>::type *__restrict__ B, long ldb, long sB, T beta,
    typename elem<T, CPLX>::type *__restrict__ C, long ldc, long sC)
{
    using E = typename elem<T, CPLX>::type;
    using MF = mfma16<T>;
    using acc_t = typename MF::acc;
    constexpr int WAVES_M = BM / WM, WAVES_N = BN / WN;
    constexpr int NT = WAVES_M * WAVES_N * 64;
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr int PAD = 1;
    static_assert(BK % 4 == 0, "BK must be a multiple of 4");

    __shared__ E As[BK][BM + PAD];
    __shared__ E Bs[BK][BN + PAD];

    const int tiles_m = (m + BM - 1) / BM;
    const int tile = blockIdx.x;
    const int tm = tile % tiles_m, tn = tile / tiles_m;
    const int m0 = tm * BM, n0 = tn * BN;
    const long bz = blockIdx.z;
    A += bz * sA;
    B += bz * sB;
    C += bz * sC;

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid % WAVES_M, wn = wid / WAVES_M;

    acc_t acc_re[FN][FM];
    acc_t acc_im[CPLX ? FN : 1][CPLX ? FM : 1];
#pragma unroll
    for (int a = 0; a < FN; ++a)
#pragma unroll
        for (int b = 0; b < FM; ++b) {
            acc_re[a][b] = acc_t{0, 0, 0, 0};
            if constexpr (CPLX) acc_im[a][b] = acc_t{0, 0, 0, 0};
        }

    for (int k0 = 0; k0 < k; k0 += BK) {
        // ---- stage A tile (BM x BK of op(A)) and B tile (BK x BN)
        if constexpr (!OPA_H) {
#pragma unroll 4
            for (int e = tid; e < BM * BK; e += NT) {
                const int i = e % BM, kk = e / BM;
                const int gi = m0 + i, gk = k0 + kk;
                As[kk][i] = (gi < m && gk < k) ? A[gi + (long)gk * lda] : zero_elem<E>();
            }
        } else {
#pragma unroll 4
            for (int e = tid; e < BM * BK; e += NT) {
                const int kk = e % BK, i = e / BK;
                const int gi = m0 + i, gk = k0 + kk;
                As[kk][i] = (gi < m && gk < k) ? conj_elem(A[gk + (long)gi * lda]) : zero_elem<E>();
            }
        }
#pragma unroll 4
        for (int e = tid; e < BN * BK; e += NT) {
            const int kk = e % BK, j = e / BK;
            const int gj = n0 + j, gk = k0 + kk;
            Bs[kk][j] = (gj < n && gk < k) ? B[gk + (long)gj * ldb] : zero_elem<E>();
        }
        __syncthreads();

#pragma unroll
        for (int k4 = 0; k4 < BK / 4; ++k4) {
            const int kr = k4 * 4 + (lane >> 4);
            E af[FM], bf[FN];
#pragma unroll
            for (int b = 0; b < FM; ++b) af[b] = As[kr][wm * WM + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < FN; ++a) bf[a] = Bs[kr][wn * WN + a * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < FN; ++a)
#pragma unroll
                for (int b = 0; b < FM; ++b) {
                    if constexpr (CPLX) {
                        acc_re[a][b] = MF::step(bf[a].x, af[b].x, acc_re[a][b]);
                        acc_re[a][b] = MF::step(-bf[a].y, af[b].y, acc_re[a][b]);
                        acc_im[a][b] = MF::step(bf[a].y, af[b].x, acc_im[a][b]);
                        acc_im[a][b] = MF::step(bf[a].x, af[b].y, acc_im[a][b]);
                    } else {
                        acc_re[a][b] = MF::step(bf[a], af[b], acc_re[a][b]);
                    }
                }
        }
        __syncthreads();
    }

    // ---- epilogue: acc'[row j][col i] of the transposed tile
#pragma unroll
    for (int a = 0; a < FN; ++a)
#pragma unroll
        for (int b = 0; b < FM; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gj = n0 + wn * WN + a * 16 + MF::acc_row(lane, r);
                const int gi = m0 + wm * WM + b * 16 + (lane & 15);
                if (gi < m && gj < n) {
                    E *p = C + gi + (long)gj * ldc;
                    if constexpr (CPLX) {
                        T vr = alpha * acc_re[a][b][r], vi = alpha * acc_im[a][b][r];
                        if (beta != T(0)) {
                            E c = *p;
                            vr += beta * c.x;
                            vi += beta * c.y;
                        }
                        E o;
                        o.x = vr;
                        o.y = vi;
                        *p = o;
                    } else {
                        T v = alpha * acc_re[a][b][r];
                        if (beta != T(0)) v += beta * *p;
                        *p = v;
                    }
                }
            }
}

// Tile shapes per element type.
template <typename T, bool CPLX> struct gemm_cfg;
template <> struct gemm_cfg<float, true> {
    static constexpr int BM = 128, BN = 128, BK = 16, WM = 64, WN = 64;
};
template <> struct gemm_cfg<double, true> {
    static constexpr int BM = 64, BN = 64, BK = 16, WM = 32, WN = 32;
};
template <> struct gemm_cfg<double, false> {
    static constexpr int BM = 64, BN = 64, BK = 16, WM = 32, WN = 32;
};
template <> struct gemm_cfg<float, false> {
    static constexpr int BM = 128, BN = 128, BK = 16, WM = 64, WN = 64;
};

template <typename T, bool CPLX, bool OPA_H>
void gemm(hipStream_t s, int m, int n, int k, T alpha, const typename elem<T, CPLX>::type *A,
          long lda, long sA, const typename elem<T, CPLX>::type *B, long ldb, long sB, T beta,
          typename elem<T, CPLX>::type *C, long ldc, long sC, int batch)
{
    if (m <= 0 || n <= 0 || batch <= 0) return;
    using cfg = gemm_cfg<T, CPLX>;
    constexpr int NT = (cfg::BM / cfg::WM) * (cfg::BN / cfg::WN) * 64;
    if (k <= 0) {
        // C = beta C: reuse the kernel with k = 0 (the k loop does not run)
    }
    dim3 grid(ceil_div(m, cfg::BM) * ceil_div(n, cfg::BN), 1, batch);
    hipLaunchKernelGGL((gemm_kernel<T, CPLX, OPA_H, cfg::BM, cfg::BN, cfg::BK, cfg::WM, cfg::WN>),
                       grid, dim3(NT), 0, s, m, n, k, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc,
                       sC);
    FX_LAUNCH_CHECK();
}

}  // namespace fx
