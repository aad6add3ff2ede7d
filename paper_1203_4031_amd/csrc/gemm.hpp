// Batched dense matrix product on the gfx950 matrix cores:
//   C = alpha * op(A) * B + beta * C,  op(A) = A or A^H (A^T for real data),
// column-major operands, one batch entry per (blockIdx.z, blockIdx.y) with
// strides (sA, sB, sC) and (sA2, sB2, sC2).
//
// Complex products are four real 16x16x4 MFMAs on the real and imaginary
// parts of interleaved {re, im} elements.  The MFMA computes the transposed
// tile (B^T A^T) so that the 16 lanes sharing an accumulator register hold
// 16 consecutive rows of one column of C: stores to column-major C are then
// contiguous.  Tiles are staged through LDS, k-major with one element of
// padding per row.
#pragma once

#include <type_traits>

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

// C = alpha op(A) B + beta C for one tile of BM x BN per workgroup.
// DB: the LDS tiles are double-buffered (one barrier per BK step instead of
// two).  G3: complex products in the three-multiplication form -- with
// T1 = sum Br Ar, T2 = sum Bi Ai, T3 = sum (Br + Bi)(Ar + Ai),
// re = T1 - T2 and im = T3 - T1 - T2 -- three real matrix-core products
// per complex step instead of four.  Its rounding error is bounded by a
// small multiple of eps |A| |B| like the four-product form, but it is not
// the same per component (the imaginary part carries the error of T1 and T2).
template <typename T, bool CPLX, bool OPA_H, int BM, int BN, int BK, int WM, int WN, int MINB, bool DB, bool G3_>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64, MINB) void gemm_kernel(
    int m_in, int n, int k, T alpha, const typename elem<T, CPLX>::type *__restrict__ A, long lda,
    long sA, const typename elem<T, CPLX>::type *__restrict__ B, long ldb, long sB, T beta,
    typename elem<T, CPLX>::type *__restrict__ C, long ldc, long sC, long sA2, long sB2, long sC2, int dm)
{
    using E = typename elem<T, CPLX>::type;
    using MF = mfma16<T>;
    using acc_t = typename MF::acc;
    constexpr int WAVES_M = BM / WM, WAVES_N = BN / WN;
    constexpr int NT = WAVES_M * WAVES_N * 64;
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr int PAD = 1;
    constexpr int LA = BM * BK / NT, LB = BN * BK / NT;   // staged elements per thread
    static_assert(BK % 4 == 0, "BK must be a multiple of 4");
    static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "tile not divisible");

    constexpr bool G3 = CPLX && G3_;
    __shared__ E As_[DB ? 2 : 1][BK][BM + PAD];
    __shared__ E Bs_[DB ? 2 : 1][BK][BN + PAD];

    // rows of this batch entry: m_in + y * dm (the grid covers the largest)
    const int tiles_m = (m_in + (dm > 0 ? (int)(gridDim.y - 1) * dm : 0) + BM - 1) / BM;
    const int m = m_in + (int)blockIdx.y * dm;
    const int tile = blockIdx.x;
    const int tm = tile % tiles_m, tn = tile / tiles_m;
    const int m0 = tm * BM, n0 = tn * BN;
    if (m0 >= m) return;   // whole workgroup, before any barrier
    const long bz = blockIdx.z, by = blockIdx.y;
    A += bz * sA + by * sA2;
    B += bz * sB + by * sB2;
    C += bz * sC + by * sC2;

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid % WAVES_M, wn = wid / WAVES_M;

    // accumulators start from beta * C / alpha so that the epilogue is a
    // plain store of alpha * acc; the loads are issued before the k loop
    acc_t acc_re[FN][FM];
    acc_t acc_im[CPLX ? FN : 1][CPLX ? FM : 1];
    acc_t acc_t2[G3 ? FN : 1][G3 ? FM : 1];
    const T cscale = (beta != T(0)) ? beta / alpha : T(0);
#pragma unroll
    for (int a = 0; a < FN; ++a)
#pragma unroll
        for (int b = 0; b < FM; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gj = n0 + wn * WN + a * 16 + MF::acc_row(lane, r);
                const int gi = m0 + wm * WM + b * 16 + (lane & 15);
                E c = zero_elem<E>();
                if (cscale != T(0) && gi < m && gj < n) c = C[gi + (long)gj * ldc];
                if constexpr (G3) {
                    acc_re[a][b][r] = cscale * c.x;
                    acc_im[a][b][r] = cscale * (c.x + c.y);
                    acc_t2[a][b][r] = T(0);
                } else if constexpr (CPLX) {
                    acc_re[a][b][r] = cscale * c.x;
                    acc_im[a][b][r] = cscale * c.y;
                } else {
                    acc_re[a][b][r] = cscale * c;
                }
            }

    E ra[LA], rb[LB];
    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int u = 0; u < LA; ++u) {
            const int e = tid + u * NT;
            int i, kk;
            if constexpr (!OPA_H) {
                i = e % BM;
                kk = e / BM;
            } else {
                kk = e % BK;
                i = e / BK;
            }
            const int gi = m0 + i, gk = k0 + kk;
            if (gi < m && gk < k) ra[u] = OPA_H ? conj_elem(A[gk + (long)gi * lda]) : A[gi + (long)gk * lda];
            else ra[u] = zero_elem<E>();
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int e = tid + u * NT;
            const int kk = e % BK, j = e / BK;
            const int gj = n0 + j, gk = k0 + kk;
            rb[u] = (gj < n && gk < k) ? B[gk + (long)gj * ldb] : zero_elem<E>();
        }
    };
    auto store_tiles = [&](int buf) {
#pragma unroll
        for (int u = 0; u < LA; ++u) {
            const int e = tid + u * NT;
            if constexpr (!OPA_H) As_[buf][e / BM][e % BM] = ra[u];
            else As_[buf][e % BK][e / BK] = ra[u];
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int e = tid + u * NT;
            Bs_[buf][e % BK][e / BK] = rb[u];
        }
    };
    auto compute = [&](int buf) {
#pragma unroll
        for (int k4 = 0; k4 < BK / 4; ++k4) {
            const int kr = k4 * 4 + (lane >> 4);
            E af[FM], bf[FN];
#pragma unroll
            for (int b = 0; b < FM; ++b) af[b] = As_[buf][kr][wm * WM + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < FN; ++a) bf[a] = Bs_[buf][kr][wn * WN + a * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < FN; ++a)
#pragma unroll
                for (int b = 0; b < FM; ++b) {
                    if constexpr (G3) {
                        acc_re[a][b] = MF::step(bf[a].x, af[b].x, acc_re[a][b]);
                        acc_t2[a][b] = MF::step(bf[a].y, af[b].y, acc_t2[a][b]);
                        acc_im[a][b] = MF::step(bf[a].x + bf[a].y, af[b].x + af[b].y, acc_im[a][b]);
                    } else if constexpr (CPLX) {
                        acc_re[a][b] = MF::step(bf[a].x, af[b].x, acc_re[a][b]);
                        acc_re[a][b] = MF::step(-bf[a].y, af[b].y, acc_re[a][b]);
                        acc_im[a][b] = MF::step(bf[a].y, af[b].x, acc_im[a][b]);
                        acc_im[a][b] = MF::step(bf[a].x, af[b].y, acc_im[a][b]);
                    } else {
                        acc_re[a][b] = MF::step(bf[a], af[b], acc_re[a][b]);
                    }
                }
        }
    };

    if constexpr (DB) {
        if (k > 0) {
            load_tiles(0);
            store_tiles(0);
        }
        __syncthreads();
        int buf = 0;
        for (int k0 = 0; k0 < k; k0 += BK) {
            const bool more = k0 + BK < k;
            if (more) load_tiles(k0 + BK);
            compute(buf);
            if (more) store_tiles(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    } else {
        if (k > 0) load_tiles(0);
        for (int k0 = 0; k0 < k; k0 += BK) {
            store_tiles(0);
            __syncthreads();
            if (k0 + BK < k) load_tiles(k0 + BK);
            compute(0);
            __syncthreads();
        }
    }

    // ---- epilogue: acc'[row j][col i] of the transposed tile; 16 lanes
    //      write 16 consecutive rows of one column of C
#pragma unroll
    for (int a = 0; a < FN; ++a)
#pragma unroll
        for (int b = 0; b < FM; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gj = n0 + wn * WN + a * 16 + MF::acc_row(lane, r);
                const int gi = m0 + wm * WM + b * 16 + (lane & 15);
                if (gi < m && gj < n) {
                    E o;
                    if constexpr (G3) {
                        o.x = alpha * (acc_re[a][b][r] - acc_t2[a][b][r]);
                        o.y = alpha * (acc_im[a][b][r] - acc_re[a][b][r] - acc_t2[a][b][r]);
                    } else if constexpr (CPLX) {
                        o.x = alpha * acc_re[a][b][r];
                        o.y = alpha * acc_im[a][b][r];
                    } else {
                        o = alpha * acc_re[a][b][r];
                    }
                    C[gi + (long)gj * ldc] = o;
                }
            }
}

// Tile shapes per element type.  MINB workgroups per CU bound the register
// use so that one workgroup's loads overlap another's matrix-core work.
// Complex64, measured at N = 4096 over 8 matrices (depth-64 LU update /
// 300-column solve update, zero data): 64x64 at four per CU 94 / 81 TF/s,
// 128x64 at three 89 / 81, 128x128 at two 91 / 54, 256x64 at one 79 / 62.
// On random data the 64x64 four-product kernel gives 74-90 TF/s on the
// depth-64 updates and 64-77 on the solve updates; double-buffered with the
// three-product form, 96-109 and 81-90 (flops counted as 8 per complex
// multiply-add).  A depth sweep at N = 8192 over 16 matrices (random data,
// depth-64 LU update / 600-column depth-256 solve update): BK 8 against 16
// gives complex64 104 / 135 against 100 / 131 TF/s, and complex128, with
// three workgroups per CU instead of two, 62 / 75 against 58 / 66; BK 32 and
// 128x128 tiles are slower in both.
template <typename T, bool CPLX> struct gemm_cfg;
template <> struct gemm_cfg<float, true> {
    static constexpr int BM = 64, BN = 64, BK = 8, WM = 32, WN = 32, MINB = 4;
    static constexpr bool DB = true, G3 = true;
};
template <> struct gemm_cfg<double, true> {
    static constexpr int BM = 64, BN = 64, BK = 8, WM = 32, WN = 32, MINB = 3;
    static constexpr bool DB = true, G3 = true;
};
template <> struct gemm_cfg<double, false> {
    static constexpr int BM = 64, BN = 64, BK = 16, WM = 32, WN = 32, MINB = 2;
    static constexpr bool DB = false, G3 = false;
};
template <> struct gemm_cfg<float, false> {
    static constexpr int BM = 128, BN = 64, BK = 16, WM = 64, WN = 32, MINB = 3;
    static constexpr bool DB = false, G3 = false;
};
// Products with at most 32 columns (the LU's panel-column updates): a
// 64x64 tile would leave half of each matrix-core product empty.  Complex64
// at N = 4096 over 8 matrices, 32 columns, depth 32 / 64: 28 / 38 TF/s with
// 64x64 tiles, 36 / 52 with 64x32.
template <typename T, bool CPLX> struct gemm_cfg_narrow;
template <> struct gemm_cfg_narrow<float, true> {
    static constexpr int BM = 64, BN = 32, BK = 16, WM = 32, WN = 16, MINB = 4;
    static constexpr bool DB = true, G3 = true;
};

// Tile variants of the complex products, chosen per precision and depth
// class from a table that the autotuner (feast_autotune) fills; variant 0 is
// the default.  Every variant accumulates each output over k in the same
// order, four terms per matrix-core step, so the choice changes time, not
// results.
template <typename T, int V> struct gemm_var;
template <> struct gemm_var<float, 0> : gemm_cfg<float, true> {};
template <> struct gemm_var<float, 1> {   // eight waves, 128x64
    static constexpr int BM = 128, BN = 64, BK = 8, WM = 32, WN = 32, MINB = 2;
    static constexpr bool DB = true, G3 = true;
};
template <> struct gemm_var<float, 2> {   // deeper staging
    static constexpr int BM = 64, BN = 64, BK = 16, WM = 32, WN = 32, MINB = 4;
    static constexpr bool DB = true, G3 = true;
};
template <> struct gemm_var<double, 0> : gemm_cfg<double, true> {};
template <> struct gemm_var<double, 1> {  // waves of 64x16
    static constexpr int BM = 64, BN = 64, BK = 8, WM = 64, WN = 16, MINB = 3;
    static constexpr bool DB = true, G3 = true;
};
template <> struct gemm_var<double, 2> {  // deeper staging, two per CU
    static constexpr int BM = 64, BN = 64, BK = 16, WM = 32, WN = 32, MINB = 2;
    static constexpr bool DB = true, G3 = true;
};
constexpr int GEMM_VARIANTS = 3;
constexpr int GEMM_CLASSES = 2;   // 0: depth <= 64 (LU and Cholesky updates), 1: deeper (solves, Rayleigh-Ritz)
inline int gemm_depth_class(int k) { return k <= 64 ? 0 : 1; }
int gemm_tile_choice(bool f64, int cls);   // defined by the driver (the autotuner's table)

template <typename T, bool CPLX, bool OPA_H, typename cfg>
void gemm_launch_cfg(hipStream_t s, int m, int mmax, int n, int k, T alpha, const typename elem<T, CPLX>::type *A,
                     long lda, long sA, long sA2, const typename elem<T, CPLX>::type *B, long ldb, long sB, long sB2,
                     T beta, typename elem<T, CPLX>::type *C, long ldc, long sC, long sC2, int batch, int batch2,
                     int dm)
{
    constexpr int NT = (cfg::BM / cfg::WM) * (cfg::BN / cfg::WN) * 64;
    dim3 grid(ceil_div(mmax, cfg::BM) * ceil_div(n, cfg::BN), batch2, batch);
    hipLaunchKernelGGL((gemm_kernel<T, CPLX, OPA_H, cfg::BM, cfg::BN, cfg::BK, cfg::WM, cfg::WN, cfg::MINB, cfg::DB,
                                    cfg::G3>),
                       grid, dim3(NT), 0, s, m, n, k, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, sA2, sB2, sC2,
                       dm);
}

// One complex product C = alpha A B + beta C (batch of `batch`) with tile
// variant v, no timing hook (the autotuner's launches).
template <typename T>
void gemm_variant(hipStream_t s, int v, int m, int n, int k, T alpha, const cplx<T> *A, long lda, long sA,
                  const cplx<T> *B, long ldb, long sB, T beta, cplx<T> *C, long ldc, long sC, int batch)
{
    if (m <= 0 || n <= 0 || batch <= 0) return;
    if (v == 1)
        gemm_launch_cfg<T, true, false, gemm_var<T, 1>>(s, m, m, n, k, alpha, A, lda, sA, 0, B, ldb, sB, 0, beta, C,
                                                        ldc, sC, 0, batch, 1, 0);
    else if (v == 2)
        gemm_launch_cfg<T, true, false, gemm_var<T, 2>>(s, m, m, n, k, alpha, A, lda, sA, 0, B, ldb, sB, 0, beta, C,
                                                        ldc, sC, 0, batch, 1, 0);
    else
        gemm_launch_cfg<T, true, false, gemm_var<T, 0>>(s, m, m, n, k, alpha, A, lda, sA, 0, B, ldb, sB, 0, beta, C,
                                                        ldc, sC, 0, batch, 1, 0);
    FX_LAUNCH_CHECK();
}

// Optional per-launch timing of the complex products (defined by the driver;
// f64 tells the element precision, the driver records one of the two).
void gemm_timing_begin(hipStream_t s, hipEvent_t *e, bool f64);
void gemm_timing_end(hipStream_t s, hipEvent_t e0, double flops, bool f64);

// Two-level batch: entry (z, y), z < batch, y < batch2, at offsets
// z * s? + y * s?2, with m + y * dm rows (dm may be negative; entries with
// no rows do nothing).
template <typename T, bool CPLX, bool OPA_H>
void gemm2(hipStream_t s, int m, int n, int k, T alpha, const typename elem<T, CPLX>::type *A, long lda, long sA,
           long sA2, const typename elem<T, CPLX>::type *B, long ldb, long sB, long sB2, T beta,
           typename elem<T, CPLX>::type *C, long ldc, long sC, long sC2, int batch, int batch2, int dm = 0)
{
    const int mmax = std::max(m, m + (batch2 - 1) * dm);
    if (mmax <= 0 || n <= 0 || batch <= 0 || batch2 <= 0) return;
    if (alpha == T(0)) throw hip_error{hipErrorInvalidValue};   // the kernel scales C by beta / alpha
    constexpr bool timed = CPLX;
    constexpr bool f64 = std::is_same<T, double>::value;
    hipEvent_t e0 = nullptr;
    if (timed) gemm_timing_begin(s, &e0, f64);
    // k <= 0: C = beta C (the k loop does not run)
    auto launch = [&](auto cfg_tag) {
        using cfg = decltype(cfg_tag);
        gemm_launch_cfg<T, CPLX, OPA_H, cfg>(s, m, mmax, n, k, alpha, A, lda, sA, sA2, B, ldb, sB, sB2, beta, C, ldc,
                                             sC, sC2, batch, batch2, dm);
    };
    if constexpr (CPLX) {
        bool done = false;
        if constexpr (!f64 && !OPA_H) {
            if (n <= 32) {
                launch(gemm_cfg_narrow<T, CPLX>{});
                done = true;
            }
        }
        if (!done) {
            const int v = gemm_tile_choice(f64, gemm_depth_class(k));
            if (v == 1) launch(gemm_var<T, 1>{});
            else if (v == 2) launch(gemm_var<T, 2>{});
            else launch(gemm_var<T, 0>{});
        }
    } else {
        launch(gemm_cfg<T, CPLX>{});
    }
    FX_LAUNCH_CHECK();
    double rows = 0;   // summed over the y entries
    for (int y = 0; y < batch2; ++y) rows += std::max(0, m + y * dm);
    if (timed) gemm_timing_end(s, e0, 8.0 * rows * (double)n * (k > 0 ? k : 0) * batch, f64);
}

template <typename T, bool CPLX, bool OPA_H>
void gemm(hipStream_t s, int m, int n, int k, T alpha, const typename elem<T, CPLX>::type *A,
          long lda, long sA, const typename elem<T, CPLX>::type *B, long ldb, long sB, T beta,
          typename elem<T, CPLX>::type *C, long ldc, long sC, int batch)
{
    gemm2<T, CPLX, OPA_H>(s, m, n, k, alpha, A, lda, sA, 0, B, ldb, sB, 0, beta, C, ldc, sC, 0, batch, 1);
}

}  // namespace fx
