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

constexpr int JAC_NT = 256;
constexpr int JAC_MAXPAIRS = 2048;   // m <= 4096

template <bool CPLX>
__global__ __launch_bounds__(JAC_NT) void jacobi_kernel(int m, typename jelem<CPLX>::type *C0,
                                                         typename jelem<CPLX>::type *C1, long ldc,
                                                         typename jelem<CPLX>::type *V, long ldv,
                                                         double *partial, unsigned *bar, int max_sweeps,
                                                         double tol, int *status)
{
    using E = typename jelem<CPLX>::type;
    __shared__ double s_c[JAC_MAXPAIRS], s_s[JAC_MAXPAIRS];
    __shared__ double2 s_ph[JAC_MAXPAIRS];
    __shared__ short s_a[JAC_MAXPAIRS], s_b[JAC_MAXPAIRS];
    __shared__ double s_red[JAC_NT / 64];

    grid_sync gs;
    gs.init(bar, bar + 1, gridDim.x);
    const int G = gridDim.x, tid = threadIdx.x;
    const long gtid = (long)blockIdx.x * JAC_NT + tid, gthreads = (long)G * JAC_NT;
    const int p = m + (m & 1), npairs = p / 2, rounds = p - 1;

    // V = I; Frobenius norm
    double acc = 0.0;
    for (long e = gtid; e < (long)m * m; e += gthreads) {
        const int i = (int)(e % m), j = (int)(e / m);
        jstore<CPLX>(V, i + j * ldv, jc_make(i == j ? 1.0 : 0.0, 0.0));
        const double2 v = jload<CPLX>(C0, i + j * ldc);
        acc += v.x * v.x + v.y * v.y;
    }
    auto block_reduce = [&](double v) {
        v = wave_sum(v);
        if ((tid & 63) == 0) s_red[tid >> 6] = v;
        __syncthreads();
        double t = 0.0;
        for (int q = 0; q < JAC_NT / 64; ++q) t += s_red[q];
        __syncthreads();
        return t;
    };
    double bs = block_reduce(acc);
    if (tid == 0) partial[blockIdx.x] = bs;
    gs.sync();
    double fro2 = 0.0;
    for (int q = 0; q < G; ++q) fro2 += partial[q];
    gs.sync();

    E *cur = C0, *nxt = C1;
    int sweep = 0, conv = 0;
    double off_prev = 1e300;
    for (sweep = 0; sweep < max_sweeps; ++sweep) {
        double offacc = 0.0;
        for (int s = 0; s < rounds; ++s) {
            for (int i = tid; i < npairs; i += JAC_NT) {
                int a, b;
                rr_pair(s, i, p, a, b);
                double c = 1.0, sn = 0.0;
                double2 ph = jc_make(1.0, 0.0);
                if (b < m) {
                    const double2 cab = jload<CPLX>(cur, a + (long)b * ldc);
                    const double babs = sqrt(cab.x * cab.x + cab.y * cab.y);
                    if (babs > 1e-300) {
                        const double caa = jload<CPLX>(cur, a + (long)a * ldc).x;
                        const double cbb = jload<CPLX>(cur, b + (long)b * ldc).x;
                        const double tau = (cbb - caa) / (2.0 * babs);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        sn = t * c;
                        ph = jc_make(cab.x / babs, cab.y / babs);
                    }
                }
                s_c[i] = c;
                s_s[i] = sn;
                s_ph[i] = ph;
                s_a[i] = (short)a;
                s_b[i] = (short)b;
            }
            __syncthreads();
            const bool last = (s == rounds - 1);
            // 2x2 block updates
            for (long e = gtid; e < (long)npairs * npairs; e += gthreads) {
                const int P = (int)(e % npairs), Q = (int)(e / npairs);
                const int ra = s_a[P], rb = s_b[P], ca = s_a[Q], cb = s_b[Q];
                const bool rbv = rb < m, cbv = cb < m;
                double2 x00 = jload<CPLX>(cur, ra + (long)ca * ldc);
                double2 x01 = cbv ? jload<CPLX>(cur, ra + (long)cb * ldc) : jc_make(0, 0);
                double2 x10 = rbv ? jload<CPLX>(cur, rb + (long)ca * ldc) : jc_make(0, 0);
                double2 x11 = (rbv && cbv) ? jload<CPLX>(cur, rb + (long)cb * ldc) : jc_make(0, 0);
                // M = X J_Q
                const double cq = s_c[Q], sq = s_s[Q];
                const double2 pq = s_ph[Q];
                const double2 sqe = jc_make(sq * pq.x, sq * pq.y);    // s e^{i phi}
                const double2 sqc = jc_make(sq * pq.x, -sq * pq.y);   // s e^{-i phi}
                double2 m00 = csub(cmake<double2>(cq * x00.x, cq * x00.y), cmul(sqc, x01));
                double2 m01 = cadd(cmul(sqe, x00), cmake<double2>(cq * x01.x, cq * x01.y));
                double2 m10 = csub(cmake<double2>(cq * x10.x, cq * x10.y), cmul(sqc, x11));
                double2 m11 = cadd(cmul(sqe, x10), cmake<double2>(cq * x11.x, cq * x11.y));
                // C' = J_P^H M
                const double cp = s_c[P], sp = s_s[P];
                const double2 pp = s_ph[P];
                const double2 spe = jc_make(sp * pp.x, sp * pp.y);
                const double2 spc = jc_make(sp * pp.x, -sp * pp.y);
                double2 y00 = csub(cmake<double2>(cp * m00.x, cp * m00.y), cmul(spe, m10));
                double2 y01 = csub(cmake<double2>(cp * m01.x, cp * m01.y), cmul(spe, m11));
                double2 y10 = cadd(cmul(spc, m00), cmake<double2>(cp * m10.x, cp * m10.y));
                double2 y11 = cadd(cmul(spc, m01), cmake<double2>(cp * m11.x, cp * m11.y));
                if (P == Q) {
                    y01 = jc_make(0, 0);
                    y10 = jc_make(0, 0);
                    y00.y = 0.0;
                    y11.y = 0.0;
                }
                jstore<CPLX>(nxt, ra + (long)ca * ldc, y00);
                if (cbv) jstore<CPLX>(nxt, ra + (long)cb * ldc, y01);
                if (rbv) jstore<CPLX>(nxt, rb + (long)ca * ldc, y10);
                if (rbv && cbv) jstore<CPLX>(nxt, rb + (long)cb * ldc, y11);
                if (last) {
                    if (ra != ca) offacc += y00.x * y00.x + y00.y * y00.y;
                    if (cbv && ra != cb) offacc += y01.x * y01.x + y01.y * y01.y;
                    if (rbv && rb != ca) offacc += y10.x * y10.x + y10.y * y10.y;
                    if (rbv && cbv && rb != cb) offacc += y11.x * y11.x + y11.y * y11.y;
                }
            }
            // V <- V J
            for (long e = gtid; e < (long)m * npairs; e += gthreads) {
                const int x = (int)(e % m), Q = (int)(e / m);
                const int ca = s_a[Q], cb = s_b[Q];
                if (cb >= m) continue;
                const double cq = s_c[Q], sq = s_s[Q];
                const double2 pq = s_ph[Q];
                const double2 va = jload<CPLX>(V, x + (long)ca * ldv), vb = jload<CPLX>(V, x + (long)cb * ldv);
                const double2 na = csub(cmake<double2>(cq * va.x, cq * va.y), cmul(jc_make(sq * pq.x, -sq * pq.y), vb));
                const double2 nb = cadd(cmul(jc_make(sq * pq.x, sq * pq.y), va), cmake<double2>(cq * vb.x, cq * vb.y));
                jstore<CPLX>(V, x + (long)ca * ldv, na);
                jstore<CPLX>(V, x + (long)cb * ldv, nb);
            }
            if (last) {
                const double b2 = block_reduce(offacc);
                if (tid == 0) partial[blockIdx.x] = b2;
            }
            gs.sync();
            E *t = cur;
            cur = nxt;
            nxt = t;
        }
        double off2 = 0.0;
        for (int q = 0; q < G; ++q) off2 += partial[q];
        const double off = sqrt(off2), fro = sqrt(fro2);
        // stop at the requested level, or once rounding noise stops the decrease
        if (off <= tol * fro || fro == 0.0) {
            conv = 1;
            ++sweep;
            break;
        }
        if (off <= 1e-13 * fro && off >= 0.5 * off_prev) {
            conv = 1;
            ++sweep;
            break;
        }
        off_prev = off;
        gs.sync();   // partial[] is rewritten in the next sweep
    }
    // leave the final matrix in C0
    if (cur != C0)
        for (long e = gtid; e < (long)m * m; e += gthreads) {
            const int i = (int)(e % m), j = (int)(e / m);
            C0[i + j * ldc] = cur[i + j * ldc];
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
