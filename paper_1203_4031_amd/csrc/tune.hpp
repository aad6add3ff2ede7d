// Tile autotuner of the complex product kernel: times every tile variant
// (gemm_var in gemm.hpp) on the device at the shapes of a solve and installs
// the fastest per precision and depth class in the table that gemm2 reads.
// Included once, by feastx.hip, after its error types (alloc_error).
#pragma once

#include <algorithm>
#include <atomic>
#include <vector>

#include "common.hpp"
#include "feastx.h"
#include "gemm.hpp"

namespace fx {
static_assert(GEMM_VARIANTS == FEAST_TILE_VARIANTS, "tile variants of the product kernel and the ABI agree");
// [precision: 0 complex64, 1 complex128][depth class] -> variant
static std::atomic<int> g_tiles[2][GEMM_CLASSES];
int gemm_tile_choice(bool f64, int cls) { return g_tiles[f64 ? 1 : 0][cls].load(std::memory_order_relaxed); }

struct TileTimes {
    double tf[2][GEMM_CLASSES][GEMM_VARIANTS] = {};
};

// deterministic values in [-0.5, 0.5) (tuning data; any finite values time the same)
template <typename T>
__global__ __launch_bounds__(256) void tune_fill_kernel(T *p, long cnt)
{
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < cnt; i += (long)gridDim.x * 256) {
        unsigned h = (unsigned)(i * 2654435761u) ^ (unsigned)(i >> 32);
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        p[i] = (T)((double)(h >> 8) * (1.0 / 16777216.0) - 0.5);
    }
}

// Rates of the variants of one precision per depth class; the buffers hold
// F (batch matrices nt x nt) and Y (batch blocks nt x mt).  Class 0 is timed
// on a depth-64 product of nt - 64 rows and columns (the LU's panel updates
// and the Cholesky updates); class 1 on a depth-128 product of nt - 128 rows
// and columns (the LU's block updates) together with a depth-256 product of
// nt - 256 rows and mt columns (the solve updates), at the rate of the two
// together.
template <typename T>
static void time_variants(hipStream_t s, int nt, int mt, int batch, cplx<T> *F, cplx<T> *Y, hipEvent_t e0,
                          hipEvent_t e1, double tf[GEMM_CLASSES][GEMM_VARIANTS])
{
    struct Shape {
        int m, ncol, d;
        const cplx<T> *A, *B;
        cplx<T> *C;
        long sB, sC;
    };
    const long sF = (long)nt * nt, sY = (long)nt * mt;
    auto square = [&](int d) { return Shape{nt - d, nt - d, d, F + d, F + (long)d * nt, F + d + (long)d * nt, sF, sF}; };
    for (int c = 0; c < GEMM_CLASSES; ++c) {
        std::vector<Shape> sh;
        if (c == 0 && nt > 64) sh.push_back(square(64));
        if (c == 1 && nt > 128) sh.push_back(square(128));
        if (c == 1 && nt > 256) sh.push_back(Shape{nt - 256, mt, 256, F + 256, Y, Y + 256, sY, sY});
        if (sh.empty()) continue;
        double flops = 0;
        for (const Shape &q : sh) flops += 8.0 * q.m * (double)q.ncol * q.d * batch;
        auto run = [&](int v) {
            for (const Shape &q : sh)
                gemm_variant<T>(s, v, q.m, q.ncol, q.d, T(-1), q.A, nt, sF, q.B, nt, q.sB, T(1), q.C, nt, q.sC,
                                batch);
        };
        // one untimed launch of each variant, then rounds that visit the
        // variants in turn; each keeps its best round, so clock ramps and
        // other transients do not favour whichever variant runs later
        for (int v = 0; v < GEMM_VARIANTS; ++v) run(v);
        constexpr int rounds = 3, reps = 3;
        for (int r = 0; r < rounds; ++r)
            for (int v = 0; v < GEMM_VARIANTS; ++v) {
                FX_CHECK(hipEventRecord(e0, s));
                for (int q = 0; q < reps; ++q) run(v);
                FX_CHECK(hipEventRecord(e1, s));
                FX_CHECK(hipEventSynchronize(e1));
                float ms = 0;
                FX_CHECK(hipEventElapsedTime(&ms, e0, e1));
                const double rate = ms > 0 ? flops * reps / (ms * 1e-3) / 1e12 : 0.0;
                tf[c][v] = std::max(tf[c][v], rate);
            }
    }
}

static TileTimes autotune(int n, int m0, int ne)
{
    const int nt = std::min(n, 4096), mt = std::min(std::max(m0, 32), nt), batch = std::min(ne, 8);
    const size_t bytes_f = sizeof(double2) * (size_t)nt * nt * batch;
    const size_t bytes_y = sizeof(double2) * (size_t)nt * mt * batch;
    void *F = nullptr, *Y = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TileTimes tt;
    auto cleanup = [&]() {
        if (s) (void)hipStreamSynchronize(s);
        if (F) (void)hipFree(F);
        if (Y) (void)hipFree(Y);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
    };
    try {
        if (hipMalloc(&F, bytes_f) != hipSuccess || hipMalloc(&Y, bytes_y) != hipSuccess) {
            (void)hipGetLastError();
            throw alloc_error{};
        }
        FX_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        FX_CHECK(hipEventCreate(&e0));
        FX_CHECK(hipEventCreate(&e1));
        // complex128 timing first (the buffers' full size), then complex64 on the same bytes
        hipLaunchKernelGGL((tune_fill_kernel<double>), dim3(2048), dim3(256), 0, s, static_cast<double *>(F),
                           (long)(bytes_f / 8));
        hipLaunchKernelGGL((tune_fill_kernel<double>), dim3(2048), dim3(256), 0, s, static_cast<double *>(Y),
                           (long)(bytes_y / 8));
        FX_LAUNCH_CHECK();
        time_variants<double>(s, nt, mt, batch, static_cast<double2 *>(F), static_cast<double2 *>(Y), e0, e1, tt.tf[1]);
        hipLaunchKernelGGL((tune_fill_kernel<float>), dim3(2048), dim3(256), 0, s, static_cast<float *>(F),
                           (long)(bytes_f / 8));
        hipLaunchKernelGGL((tune_fill_kernel<float>), dim3(2048), dim3(256), 0, s, static_cast<float *>(Y),
                           (long)(bytes_y / 8));
        FX_LAUNCH_CHECK();
        time_variants<float>(s, nt, mt, batch, static_cast<float2 *>(F), static_cast<float2 *>(Y), e0, e1, tt.tf[0]);
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
    // the fastest variant per precision and class; another one replaces the
    // default only when at least 5 % faster (timing noise keeps the default)
    for (int p = 0; p < 2; ++p)
        for (int c = 0; c < GEMM_CLASSES; ++c) {
            int best = 0;
            for (int v = 1; v < GEMM_VARIANTS; ++v)
                if (tt.tf[p][c][v] > 1.05 * tt.tf[p][c][0] && tt.tf[p][c][v] > tt.tf[p][c][best]) best = v;
            g_tiles[p][c].store(best);
        }
    return tt;
}
}  // namespace fx

