// Shared device helpers for the FEAST library: complex arithmetic on
// interleaved {re, im} pairs, matrix-core (MFMA) wrappers for gfx950, and
// error plumbing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fx {

// ---------------------------------------------------------------- errors
struct hip_error {
    hipError_t code;
};

#define FX_CHECK(expr)                                     \
    do {                                                   \
        hipError_t fx_e_ = (expr);                         \
        if (fx_e_ != hipSuccess) throw ::fx::hip_error{fx_e_}; \
    } while (0)

#define FX_LAUNCH_CHECK() FX_CHECK(hipGetLastError())

// ------------------------------------------------------- complex helpers
template <typename T> struct c2;
template <> struct c2<float> { using type = float2; };
template <> struct c2<double> { using type = double2; };
template <typename T> using cplx = typename c2<T>::type;

template <typename V> __host__ __device__ inline V cmake(decltype(V{}.x) r, decltype(V{}.x) i)
{
    V v;
    v.x = r;
    v.y = i;
    return v;
}
template <typename V> __host__ __device__ inline V cadd(V a, V b) { return cmake<V>(a.x + b.x, a.y + b.y); }
template <typename V> __host__ __device__ inline V csub(V a, V b) { return cmake<V>(a.x - b.x, a.y - b.y); }
template <typename V> __host__ __device__ inline V cmul(V a, V b)
{
    return cmake<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename V> __host__ __device__ inline V cmulc(V a, V b)
{
    return cmake<V>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename V> __host__ __device__ inline V cconj(V a) { return cmake<V>(a.x, -a.y); }
// 1 / a, scaled to avoid overflow of |a|^2
template <typename V> __host__ __device__ inline V cinv(V a)
{
    auto s = fabs(a.x) > fabs(a.y) ? fabs(a.x) : fabs(a.y);
    if (s == 0) return cmake<V>(a.x / s, a.y);   // inf/nan propagate
    auto ar = a.x / s, ai = a.y / s;
    auto d = (ar * ar + ai * ai) * s;
    return cmake<V>(ar / d, -ai / d);
}
template <typename V> __host__ __device__ inline auto cabs1(V a) { return fabs(a.x) + fabs(a.y); }

// ---------------------------------------------------- matrix-core wrappers
// 16x16x4 MFMA for fp32 and fp64.  Operand layout (both types): lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16] of the 16x4 / 4x16 blocks.
// Accumulator layout differs per type; acc_row(l, r) gives the row of the
// 16x16 result held in register r of lane l, the column is always l % 16.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct mfma16;
template <> struct mfma16<float> {
    using acc = f32x4;
    __device__ static inline acc step(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static inline int acc_row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct mfma16<double> {
    using acc = f64x4;
    __device__ static inline acc step(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static inline int acc_row(int lane, int r) { return 4 * r + (lane >> 4); }
};

// ------------------------------------------------------------ reductions
template <typename T> __device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace fx
