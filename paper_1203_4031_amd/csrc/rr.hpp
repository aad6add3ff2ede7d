// Element-wise and reduction kernels around the contour solves and the
// Rayleigh-Ritz step: quadrature accumulation, residual norms, Hermitian
// symmetrisation, column scaling and gathering, and the seeded random start.
#pragma once

#include "common.hpp"
#include "jacobi.hpp"

namespace fx {

// Quadrature accumulation (the guide's Q = sum_j w_j Q_j), fixed node order.
//   real pencils:      Q = rho .* X + sum_j Re(coef_jc Y_j)
//   Hermitian pencils: Q = rho .* X + sum_j (coef_jc Y_j + conj(coef_jc) Yh_j) / 2
// coef_jc = w_j for the plain form, w_j / (z_j - lambda_c) for the residual
// correction form (then rho_c = sum_j Re coef_jc and X is the Ritz basis);
// rho == nullptr means no X term.  Y_j, Yh_j are in the solve precision; Q is
// FP64.
template <typename T, bool CPLX>
__global__ __launch_bounds__(256) void accumulate_kernel(int n, int ncols, int ne,
                                                         const cplx<T> *__restrict__ Y, long ldy,
                                                         long sY, const cplx<T> *__restrict__ Yh,
                                                         const double2 *__restrict__ coef,
                                                         const double *__restrict__ rho,
                                                         const typename jelem<CPLX>::type *__restrict__ X,
                                                         long ldx, typename jelem<CPLX>::type *__restrict__ Q,
                                                         long ldq, int add)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * ncols) return;
    const int i = (int)(idx % n), c = (int)(idx / n);
    double qr = 0.0, qi = 0.0;
    for (int j = 0; j < ne; ++j) {
        const double2 w = coef[(long)j * ncols + c];
        const cplx<T> y = Y[j * sY + i + (long)c * ldy];
        const double yr = y.x, yi = y.y;
        if constexpr (!CPLX) {
            qr += w.x * yr - w.y * yi;
        } else {
            const cplx<T> yh = Yh[j * sY + i + (long)c * ldy];
            const double hr = yh.x, hi = yh.y;
            // (w y + conj(w) yh) / 2
            qr += 0.5 * ((w.x * yr - w.y * yi) + (w.x * hr + w.y * hi));
            qi += 0.5 * ((w.x * yi + w.y * yr) + (w.x * hi - w.y * hr));
        }
    }
    if (rho) {
        const double2 x = jload<CPLX>(X, i + (long)c * ldx);
        qr += rho[c] * x.x;
        qi += rho[c] * x.y;
    }
    if (add) {   // a second node group: Q += its sum
        const double2 q0 = jload<CPLX>(Q, i + (long)c * ldq);
        qr = q0.x + qr;
        qi = q0.y + qi;
    }
    jstore<CPLX>(Q, i + (long)c * ldq, make_double2(qr, qi));
}

// Per-block sums of |a_ij|^2 over an n x n matrix (SUMSQ_BLOCKS blocks,
// summed on the host in block order).
constexpr int SUMSQ_BLOCKS = 256;
template <bool CPLX>
__global__ __launch_bounds__(256) void sumsq_kernel(int n, const double *__restrict__ A, long lda,
                                                    double *__restrict__ part)
{
    __shared__ double red[4];
    double acc = 0.0;
    const long nn = (long)n * n;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < nn; e += (long)gridDim.x * 256) {
        const long i = e % n, j = e / n;
        if constexpr (CPLX) {
            const double2 a = reinterpret_cast<const double2 *>(A)[i + j * lda];
            acc += a.x * a.x + a.y * a.y;
        } else {
            const double a = A[i + j * lda];
            acc += a * a;
        }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// R = AX - BX diag(lambda)   (residual of the current Ritz pairs, FP64)
template <bool CPLX>
__global__ __launch_bounds__(256) void ritz_residual_kernel(int n, int ncols,
                                                            const typename jelem<CPLX>::type *__restrict__ AX,
                                                            const typename jelem<CPLX>::type *__restrict__ BX,
                                                            long ld, const double *__restrict__ lam,
                                                            typename jelem<CPLX>::type *__restrict__ R)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * ncols) return;
    const int i = (int)(idx % n), c = (int)(idx / n);
    const double2 a = jload<CPLX>(AX, i + (long)c * ld), b = jload<CPLX>(BX, i + (long)c * ld);
    const double l = lam[c];
    jstore<CPLX>(R, i + (long)c * ld, make_double2(a.x - l * b.x, a.y - l * b.y));
}

// res_c = ||AX_c - lambda_c BX_c||_1 / (alpha ||BX_c||_1), complex modulus
// (the guide's residual definition, argument res of Table "tab_common").
// One block per column, fixed reduction order.
template <bool CPLX>
__global__ __launch_bounds__(256) void resid_norm_kernel(int n, const typename jelem<CPLX>::type *__restrict__ AX,
                                                         const typename jelem<CPLX>::type *__restrict__ BX,
                                                         long ld, const double *__restrict__ lam, double alpha,
                                                         double *__restrict__ res)
{
    const int c = blockIdx.x, tid = threadIdx.x;
    const double l = lam[c];
    double num = 0.0, den = 0.0;
    for (int i = tid; i < n; i += 256) {
        const double2 a = jload<CPLX>(AX, i + (long)c * ld), b = jload<CPLX>(BX, i + (long)c * ld);
        const double rr = a.x - l * b.x, ri = a.y - l * b.y;
        num += sqrt(rr * rr + ri * ri);
        den += sqrt(b.x * b.x + b.y * b.y);
    }
    __shared__ double sn[4], sd[4];
    num = wave_sum(num);
    den = wave_sum(den);
    if ((tid & 63) == 0) {
        sn[tid >> 6] = num;
        sd[tid >> 6] = den;
    }
    __syncthreads();
    if (tid == 0) {
        const double N = sn[0] + sn[1] + sn[2] + sn[3], D = sd[0] + sd[1] + sd[2] + sd[3];
        res[c] = N / (alpha * D);
    }
}

// M = (M + M^H) / 2, m x m
template <bool CPLX>
__global__ __launch_bounds__(256) void hermitian_part_kernel(int m, typename jelem<CPLX>::type *M, long ld)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)m * m) return;
    const int i = (int)(idx % m), j = (int)(idx / m);
    if (i > j) return;
    const double2 a = jload<CPLX>(M, i + (long)j * ld), b = jload<CPLX>(M, j + (long)i * ld);
    const double2 s = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    jstore<CPLX>(M, i + (long)j * ld, s);
    jstore<CPLX>(M, j + (long)i * ld, make_double2(s.x, -s.y));
}

// T[:, c] = W[:, first + c] / sqrt(beta[first + c])
template <bool CPLX>
__global__ __launch_bounds__(256) void scale_cols_kernel(int m, int ncols, int first,
                                                         const typename jelem<CPLX>::type *__restrict__ W,
                                                         long ldw, const double *__restrict__ beta,
                                                         typename jelem<CPLX>::type *__restrict__ T, long ldt)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)m * ncols) return;
    const int i = (int)(idx % m), c = (int)(idx / m);
    const double sc = 1.0 / sqrt(beta[first + c]);
    const double2 v = jload<CPLX>(W, i + (long)(first + c) * ldw);
    jstore<CPLX>(T, i + (long)c * ldt, make_double2(v.x * sc, v.y * sc));
}

// out[:, c] = in[:, idx[c]]
template <bool CPLX>
__global__ __launch_bounds__(256) void gather_cols_kernel(int n, int ncols, const int *__restrict__ sel,
                                                          const typename jelem<CPLX>::type *__restrict__ in,
                                                          long ldi, typename jelem<CPLX>::type *__restrict__ out,
                                                          long ldo)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * ncols) return;
    const int i = (int)(idx % n), c = (int)(idx / n);
    out[i + (long)c * ldo] = in[i + (long)sel[c] * ldi];
}

// Seeded start subspace: real uniform(-1, 1), one splitmix64 draw per entry
// (counter = column-major index).  With signs != 0 each entry is the sign of
// that draw, -1 below the middle of [-1, 1) and +1 from it on (probe
// vectors of the count estimate).
template <bool CPLX>
__global__ __launch_bounds__(256) void random_start_kernel(int n, int ncols, unsigned long long seed, int signs,
                                                           typename jelem<CPLX>::type *__restrict__ X, long ldx)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * ncols) return;
    const int i = (int)(idx % n), c = (int)(idx / n);
    unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(idx + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    const double v = 2.0 * u - 1.0;
    jstore<CPLX>(X, i + (long)c * ldx, make_double2(signs ? (v < 0.0 ? -1.0 : 1.0) : v, 0.0));
}

// Stochastic count estimate (section "Stochastic estimate"): one contour pass
// maps probe x_c to q_c = rho(B^{-1} A) x_c, and the trace of rho(B^{-1} A)
// is sum_i rho(lambda_i), about the number of eigenvalues in the interval.
// Probe c gives the sample e_c = n Re(x_c^H q_c) / (x_c^H x_c), the
// Hutchinson estimator for +-1 probes.  One block per column.
template <bool CPLX>
__global__ __launch_bounds__(256) void count_sample_kernel(int n, const typename jelem<CPLX>::type *__restrict__ X,
                                                           long ldx, const typename jelem<CPLX>::type *__restrict__ Q,
                                                           long ldq, double *__restrict__ samp)
{
    const int c = blockIdx.x, tid = threadIdx.x;
    double num = 0.0, den = 0.0;
    for (int i = tid; i < n; i += 256) {
        const double2 x = jload<CPLX>(X, i + (long)c * ldx), q = jload<CPLX>(Q, i + (long)c * ldq);
        num += x.x * q.x + x.y * q.y;
        den += x.x * x.x + x.y * x.y;
    }
    __shared__ double sn[4], sd[4];
    num = wave_sum(num);
    den = wave_sum(den);
    if ((tid & 63) == 0) {
        sn[tid >> 6] = num;
        sd[tid >> 6] = den;
    }
    __syncthreads();
    if (tid == 0) {
        const double N = sn[0] + sn[1] + sn[2] + sn[3], D = sd[0] + sd[1] + sd[2] + sd[3];
        samp[c] = D > 0.0 ? (double)n * N / D : 0.0;
    }
}

// Running averages res[c] = (e_0 + ... + e_c) / (c + 1) of the samples, and
// the estimate: the nearest integer to res[m - 1], at least 0.  One block of
// 1024 threads scans the samples in chunks of 1024 (Hillis-Steele in LDS),
// carrying each chunk's total into the next.
__global__ __launch_bounds__(1024) void count_mean_kernel(int m, const double *__restrict__ samp,
                                                          double *__restrict__ res, int *__restrict__ est)
{
    __shared__ double sh[2][1024];
    const int tid = threadIdx.x;
    double carry = 0.0;
    for (int base = 0; base < m; base += 1024) {
        const int i = base + tid;
        int cur = 0;
        sh[0][tid] = i < m ? samp[i] : 0.0;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const double v = sh[cur][tid] + (tid >= d ? sh[cur][tid - d] : 0.0);
            sh[cur ^ 1][tid] = v;
            cur ^= 1;
            __syncthreads();
        }
        const double incl = carry + sh[cur][tid];
        if (i < m) res[i] = incl / (double)(i + 1);
        carry += sh[cur][1023];
        __syncthreads();
    }
    if (tid == 0) {
        const double e = floor(res[m - 1] + 0.5);
        *est = e > 0.0 ? (int)e : 0;
    }
}

// Copy an n x ncols FP64 block between leading dimensions.
template <bool CPLX>
__global__ __launch_bounds__(256) void copy_block_kernel(int n, int ncols,
                                                         const typename jelem<CPLX>::type *__restrict__ in,
                                                         long ldi, typename jelem<CPLX>::type *__restrict__ out,
                                                         long ldo)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * ncols) return;
    const int i = (int)(idx % n), c = (int)(idx / n);
    out[i + (long)c * ldo] = in[i + (long)c * ldi];
}

}  // namespace fx
