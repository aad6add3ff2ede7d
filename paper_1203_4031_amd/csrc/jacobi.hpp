// Reduced dense Hermitian eigenproblem of the Rayleigh-Ritz step, solved on
// the GPU in FP64 by parallel two-sided Jacobi.
//
// Ordering: round-robin ("circle") tournament over p = m rounded up to even
// indices; each of the p-1 rounds of a sweep rotates p/2 disjoint pairs.
// Rotations of one round commute, so every 2x2 block (row pair P, column
// pair Q) is updated independently: C'_PQ = J_P^H C_PQ J_Q.  The matrix is
// double-buffered (read C_cur, write C_next) so that each round needs one
// grid barrier.  The off-diagonal norm is summed from per-block partials in
// a fixed order, so every block takes the same stopping decision and the
// result does not depend on scheduling.
//
// Rotation for a pair (a < b), c_ab = |c_ab| e^{i phi}:
//   tau = (c_bb - c_aa) / (2 |c_ab|), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1/sqrt(1 + t^2), s = t c,  J = [[c, s e^{i phi}], [-s e^{-i phi}, c]].
#pragma once

#include "common.hpp"

namespace fx {

template <bool CPLX> struct jelem { using type = double; };
template <> struct jelem<true> { using type = double2; };

__device__ inline double2 jc_make(double r, double i) { return make_double2(r, i); }

template <bool CPLX> __device__ inline double2 jload(const typename jelem<CPLX>::type *p, long i)
{
    if constexpr (CPLX) return p[i];
    else return make_double2(p[i], 0.0);
}
template <bool CPLX> __device__ inline void jstore(typename jelem<CPLX>::type *p, long i, double2 v)
{
    if constexpr (CPLX) p[i] = v;
    else p[i] = v.x;
}

__device__ inline void rr_pair(int s, int i, int p, int &a, int &b)
{
    // circle method: index p-1 is fixed, the others rotate
    if (i == 0) {
        a = p - 1;
        b = s;
    } else {
        a = (s + i) % (p - 1);
        b = (s - i + (p - 1)) % (p - 1);
    }
    if (a > b) {
        const int t = a;
        a = b;
        b = t;
    }
}

// ------------------------------------------------------------------------
// Two-level (block) parallel Jacobi.  The index set is split into blocks of
// BJ_BS; each round of a sweep pairs the blocks (circle method) and, for
// every block pair P = (I, J), one workgroup runs inner Jacobi sweeps on the
// 2*BJ_BS principal submatrix in LDS and accumulates its rotations into a
// unitary R_P.  After a grid barrier every 2BS x 2BS tile of the matrix is
// replaced by R_P^H C_PQ R_Q and the eigenvector columns by V_Q R_Q.  Each
// outer sweep applies every scalar rotation pair at least once, so the
// convergence is that of cyclic Jacobi, with two grid barriers per round
// instead of one per scalar round.
constexpr int BJ_BS = 16;
constexpr int BJ_W = 2 * BJ_BS;
constexpr int BJ_NT = 256;

__device__ inline double jmul(double a, double b) { return a * b; }
__device__ inline double2 jmul(double2 a, double2 b) { return cmul(a, b); }
__device__ inline double jconj(double a) { return a; }
__device__ inline double2 jconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double jadd(double a, double b) { return a + b; }
__device__ inline double2 jadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double jabs2(double a) { return a * a; }
__device__ inline double jabs2(double2 a) { return a.x * a.x + a.y * a.y; }
template <typename E> __device__ inline E jzero();
template <> __device__ inline double jzero<double>() { return 0.0; }
template <> __device__ inline double2 jzero<double2>() { return make_double2(0.0, 0.0); }
template <typename E> __device__ inline E jreal(double v);
template <> __device__ inline double jreal<double>(double v) { return v; }
template <> __device__ inline double2 jreal<double2>(double v) { return make_double2(v, 0.0); }
__device__ inline double jre(double a) { return a; }
__device__ inline double jre(double2 a) { return a.x; }
// s e^{+i phi} (sign = +1) or s e^{-i phi} (sign = -1) as an element
template <typename E> __device__ inline E jphase(double s, double2 ph, double sign);
template <> __device__ inline double jphase<double>(double s, double2 ph, double) { return s * ph.x; }
template <> __device__ inline double2 jphase<double2>(double s, double2 ph, double sign)
{
    return make_double2(s * ph.x, sign * s * ph.y);
}

template <bool CPLX>
__global__ __launch_bounds__(BJ_NT) void bjacobi_kernel(int n, typename jelem<CPLX>::type *C, long ldc,
                                                        typename jelem<CPLX>::type *V, long ldv,
                                                        typename jelem<CPLX>::type *Rbuf, double *partial,
                                                        unsigned *bar, int max_sweeps, double tol,
                                                        int inner_sweeps, int *status, double *hist)
{
    using E = typename jelem<CPLX>::type;
    __shared__ E L0[BJ_W][BJ_W + 1];
    __shared__ E L1[BJ_W][BJ_W + 1];
    __shared__ double s_c[BJ_BS], s_s[BJ_BS];
    __shared__ double2 s_ph[BJ_BS];
    __shared__ int s_ia[BJ_BS], s_ib[BJ_BS];
    __shared__ int s_iP[BJ_W], s_iQ[BJ_W];
    __shared__ double s_red[BJ_NT / 64];

    grid_sync gs;
    gs.init(bar, bar + 1, gridDim.x);
    const int G = gridDim.x, tid = threadIdx.x, bid = blockIdx.x;
    const long gtid = (long)bid * BJ_NT + tid, gthreads = (long)G * BJ_NT;
    const int nb = (n + BJ_BS - 1) / BJ_BS;
    const int nbp = nb + (nb & 1), npairs = nbp / 2, rounds = nbp - 1;
    const int nrc = (n + BJ_W - 1) / BJ_W;   // row chunks of V
    E *Rall = Rbuf;

    auto block_reduce = [&](double v) {
        v = wave_sum(v);
        if ((tid & 63) == 0) s_red[tid >> 6] = v;
        __syncthreads();
        double t = 0.0;
        for (int q = 0; q < BJ_NT / 64; ++q) t += s_red[q];
        __syncthreads();
        return t;
    };
    // indices of the 2 * BS rows of block pair P in round s (-1 = padding)
    auto pair_idx = [&](int s, int P, int *dst) {
        int I, J;
        rr_pair(s, P, nbp, I, J);
        for (int t = tid; t < BJ_W; t += BJ_NT) {
            const int g = (t < BJ_BS) ? I * BJ_BS + t : J * BJ_BS + (t - BJ_BS);
            dst[t] = g < n ? g : -1;
        }
    };

    double acc = 0.0;
    for (long e = gtid; e < (long)n * n; e += gthreads) {
        const int i = (int)(e % n), j = (int)(e / n);
        V[i + j * ldv] = jreal<E>(i == j ? 1.0 : 0.0);
        acc += jabs2(C[i + j * ldc]);
    }
    double bs = block_reduce(acc);
    if (tid == 0) partial[G + bid] = bs;
    gs.sync();
    double fro2 = 0.0;
    for (int q = 0; q < G; ++q) fro2 += partial[G + q];
    const double fro = sqrt(fro2);

    int sweep = 0, conv = 0;
    double off_prev = 1e300;
    for (sweep = 0; sweep < max_sweeps && !conv; ++sweep) {
        double offacc = 0.0;
        for (int s = 0; s < rounds; ++s) {
            const bool last = (s == rounds - 1);
            // ---------------- phase 1: inner Jacobi on each block pair
            for (int P = bid; P < npairs; P += G) {
                pair_idx(s, P, s_iP);
                __syncthreads();
                for (int e = tid; e < BJ_W * BJ_W; e += BJ_NT) {
                    const int a = e % BJ_W, b = e / BJ_W;
                    const int ia = s_iP[a], ib = s_iP[b];
                    L0[a][b] = (ia >= 0 && ib >= 0) ? C[ia + (long)ib * ldc] : jzero<E>();
                    L1[a][b] = jreal<E>(a == b ? 1.0 : 0.0);
                }
                __syncthreads();
                for (int isw = 0; isw < inner_sweeps; ++isw)
                    for (int r = 0; r < BJ_W - 1; ++r) {
                        if (tid < BJ_BS) {
                            int a, b;
                            rr_pair(r, tid, BJ_W, a, b);
                            double c = 1.0, sn = 0.0;
                            double2 ph = make_double2(1.0, 0.0);
                            if (s_iP[a] >= 0 && s_iP[b] >= 0) {
                                const E sab = L0[a][b];
                                const double babs = sqrt(jabs2(sab));
                                if (babs > 1e-300) {
                                    const double tau = (jre(L0[b][b]) - jre(L0[a][a])) / (2.0 * babs);
                                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                                    c = 1.0 / sqrt(1.0 + t * t);
                                    sn = t * c;
                                    if constexpr (CPLX) ph = make_double2(sab.x / babs, sab.y / babs);
                                    else ph = make_double2(sab / babs, 0.0);
                                }
                            }
                            s_c[tid] = c;
                            s_s[tid] = sn;
                            s_ph[tid] = ph;
                            s_ia[tid] = a;
                            s_ib[tid] = b;
                        }
                        __syncthreads();
                        for (int e = tid; e < BJ_BS * BJ_BS; e += BJ_NT) {
                            const int p = e % BJ_BS, q = e / BJ_BS;
                            const int ra = s_ia[p], rb = s_ib[p], ca = s_ia[q], cb = s_ib[q];
                            const E x00 = L0[ra][ca], x01 = L0[ra][cb], x10 = L0[rb][ca], x11 = L0[rb][cb];
                            const double cq = s_c[q], cp = s_c[p];
                            const E sqe = jphase<E>(s_s[q], s_ph[q], 1.0), sqc = jphase<E>(s_s[q], s_ph[q], -1.0);
                            const E spe = jphase<E>(s_s[p], s_ph[p], 1.0), spc = jphase<E>(s_s[p], s_ph[p], -1.0);
                            // M = X J_q,  J = [[c, s e^{i phi}], [-s e^{-i phi}, c]]
                            const E m00 = jadd(jmul(jreal<E>(cq), x00), jmul(jreal<E>(-1.0), jmul(sqc, x01)));
                            const E m01 = jadd(jmul(sqe, x00), jmul(jreal<E>(cq), x01));
                            const E m10 = jadd(jmul(jreal<E>(cq), x10), jmul(jreal<E>(-1.0), jmul(sqc, x11)));
                            const E m11 = jadd(jmul(sqe, x10), jmul(jreal<E>(cq), x11));
                            // C' = J_p^H M
                            E y00 = jadd(jmul(jreal<E>(cp), m00), jmul(jreal<E>(-1.0), jmul(spe, m10)));
                            E y01 = jadd(jmul(jreal<E>(cp), m01), jmul(jreal<E>(-1.0), jmul(spe, m11)));
                            E y10 = jadd(jmul(spc, m00), jmul(jreal<E>(cp), m10));
                            E y11 = jadd(jmul(spc, m01), jmul(jreal<E>(cp), m11));
                            if (p == q) {
                                y01 = jzero<E>();
                                y10 = jzero<E>();
                                y00 = jreal<E>(jre(y00));
                                y11 = jreal<E>(jre(y11));
                            }
                            L0[ra][ca] = y00;
                            L0[ra][cb] = y01;
                            L0[rb][ca] = y10;
                            L0[rb][cb] = y11;
                        }
                        for (int e = tid; e < BJ_W * BJ_BS; e += BJ_NT) {
                            const int x = e % BJ_W, q = e / BJ_W;
                            const int ca = s_ia[q], cb = s_ib[q];
                            const E va = L1[x][ca], vb = L1[x][cb];
                            const double cq = s_c[q];
                            const E sqe = jphase<E>(s_s[q], s_ph[q], 1.0), sqc = jphase<E>(s_s[q], s_ph[q], -1.0);
                            L1[x][ca] = jadd(jmul(jreal<E>(cq), va), jmul(jreal<E>(-1.0), jmul(sqc, vb)));
                            L1[x][cb] = jadd(jmul(sqe, va), jmul(jreal<E>(cq), vb));
                        }
                        __syncthreads();
                    }
                E *R = Rall + (long)P * BJ_W * BJ_W;
                for (int e = tid; e < BJ_W * BJ_W; e += BJ_NT) {
                    const int a = e % BJ_W, b = e / BJ_W;
                    R[a + b * BJ_W] = L1[a][b];
                }
                __syncthreads();
            }
            gs.sync();
            // ---------------- phase 2: C_PQ <- R_P^H C_PQ R_Q,  V_Q <- V_Q R_Q
            const int nc_items = npairs * npairs, nitems = nc_items + nrc * npairs;
            for (int it = bid; it < nitems; it += G) {
                const bool is_c = it < nc_items;
                const int Q = is_c ? it / npairs : (it - nc_items) / nrc;
                const int P = is_c ? it % npairs : 0;
                const int rc = is_c ? 0 : (it - nc_items) % nrc;
                pair_idx(s, Q, s_iQ);
                if (is_c) pair_idx(s, P, s_iP);
                else
                    for (int t = tid; t < BJ_W; t += BJ_NT) s_iP[t] = (rc * BJ_W + t < n) ? rc * BJ_W + t : -1;
                __syncthreads();
                const E *RQ = Rall + (long)Q * BJ_W * BJ_W;
                const E *src = is_c ? C : V;
                const long lds = is_c ? ldc : ldv;
                for (int e = tid; e < BJ_W * BJ_W; e += BJ_NT) {
                    const int a = e % BJ_W, b = e / BJ_W;
                    const int ia = s_iP[a], ib = s_iQ[b];
                    L0[a][b] = (ia >= 0 && ib >= 0) ? src[ia + (long)ib * lds] : jzero<E>();
                    L1[a][b] = RQ[a + b * BJ_W];
                }
                __syncthreads();
                // T = X R_Q, 16 entries per thread
                E tv[BJ_W * BJ_W / BJ_NT];
#pragma unroll
                for (int u = 0; u < BJ_W * BJ_W / BJ_NT; ++u) {
                    const int e = tid + u * BJ_NT;
                    const int a = e % BJ_W, b = e / BJ_W;
                    E sum = jzero<E>();
                    for (int k = 0; k < BJ_W; ++k) sum = jadd(sum, jmul(L0[a][k], L1[k][b]));
                    tv[u] = sum;
                }
                __syncthreads();
                if (is_c) {
                    const E *RP = Rall + (long)P * BJ_W * BJ_W;
#pragma unroll
                    for (int u = 0; u < BJ_W * BJ_W / BJ_NT; ++u) {
                        const int e = tid + u * BJ_NT;
                        L0[e % BJ_W][e / BJ_W] = tv[u];
                    }
                    for (int e = tid; e < BJ_W * BJ_W; e += BJ_NT) {
                        const int a = e % BJ_W, b = e / BJ_W;
                        L1[a][b] = RP[a + b * BJ_W];
                    }
                    __syncthreads();
#pragma unroll
                    for (int u = 0; u < BJ_W * BJ_W / BJ_NT; ++u) {
                        const int e = tid + u * BJ_NT;
                        const int a = e % BJ_W, b = e / BJ_W;
                        E sum = jzero<E>();
                        for (int k = 0; k < BJ_W; ++k) sum = jadd(sum, jmul(jconj(L1[k][a]), L0[k][b]));
                        const int ia = s_iP[a], ib = s_iQ[b];
                        if (ia >= 0 && ib >= 0) {
                            if (ia == ib) sum = jreal<E>(jre(sum));
                            C[ia + (long)ib * ldc] = sum;
                            if (last && ia != ib) offacc += jabs2(sum);
                        }
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < BJ_W * BJ_W / BJ_NT; ++u) {
                        const int e = tid + u * BJ_NT;
                        const int a = e % BJ_W, b = e / BJ_W;
                        const int ia = s_iP[a], ib = s_iQ[b];
                        if (ia >= 0 && ib >= 0) V[ia + (long)ib * ldv] = tv[u];
                    }
                }
                __syncthreads();
            }
            if (last) {
                const double b2 = block_reduce(offacc);
                if (tid == 0) partial[bid] = b2;
            }
            gs.sync();
        }
        double off2 = 0.0;
        for (int q = 0; q < G; ++q) off2 += partial[q];
        const double off = sqrt(off2);
        if (gtid == 0 && sweep < 64) hist[sweep] = fro > 0.0 ? off / fro : 0.0;
        // Stop once the off-diagonal norm is below tol * ||C||_F (a Ritz vector
        // error of size off mixes only pairs whose eigenvalues differ by about
        // off / error, so its residual contribution is ~off), or once rounding
        // noise stops the decrease.
        if (off <= tol * fro || fro == 0.0) conv = 1;
        else if (off <= 1e-11 * fro && off >= 0.5 * off_prev) conv = 1;
        off_prev = off;
    }
    if (gtid == 0) {
        status[0] = conv ? 0 : -1;
        status[1] = sweep;
    }
}

// Eigenvalues from the diagonal of the converged matrix, sorted ascending
// (stable by index); eigenvector columns follow.  One block.
template <bool CPLX>
__global__ __launch_bounds__(1024) void jacobi_sort_kernel(int m, const typename jelem<CPLX>::type *C,
                                                           long ldc, const typename jelem<CPLX>::type *V,
                                                           long ldv, double *w, typename jelem<CPLX>::type *Vout,
                                                           long ldo, int *rank)
{
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double di = jload<CPLX>(C, i + (long)i * ldc).x;
        int r = 0;
        for (int j = 0; j < m; ++j) {
            const double dj = jload<CPLX>(C, j + (long)j * ldc).x;
            r += (dj < di) || (dj == di && j < i);
        }
        rank[i] = r;
        w[r] = di;
    }
    __syncthreads();
    for (long e = threadIdx.x; e < (long)m * m; e += blockDim.x) {
        const int x = (int)(e % m), c = (int)(e / m);
        Vout[x + (long)rank[c] * ldo] = V[x + (long)c * ldv];
    }
}

}  // namespace fx
