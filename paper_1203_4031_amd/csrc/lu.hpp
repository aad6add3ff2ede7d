// Shifted complex LU with partial pivoting, batched over contour nodes
// (the factorisation step of the FEAST contour, ijob 10 of the guide's RCI
// figure).  Blocked right-looking:
//   for each panel of NB columns:
//     lu_panel       factor the tall panel with partial pivoting (one
//                    workgroup per matrix, IB-column sub-blocks in registers)
//     lu_swap_trsm   apply the panel's row interchanges to the other
//                    columns and solve U12 = L11^{-1} A12
//     gemm           trailing update A22 -= L21 U12 on the matrix cores
// The shifted matrix z_j B - A is formed by shift_build from the FP64 inputs
// straight into the factor storage.
#pragma once

#include <algorithm>
#include <atomic>
#include <vector>

#include "common.hpp"
#include "gemm.hpp"

namespace fx {

// F_j = z_j B - A  (B == nullptr: B = I), converted to the factor precision.
template <typename T, bool CPLX_IN>
__global__ __launch_bounds__(256) void shift_build_kernel(int n, const double *__restrict__ A,
                                                          long lda, const double *__restrict__ B,
                                                          long ldb, const double2 *__restrict__ z,
                                                          int ne, cplx<T> *__restrict__ F,
                                                          long ldf, long sF)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long nn = (long)n * n;
    if (idx >= nn) return;
    const int i = (int)(idx % n), c = (int)(idx / n);
    double ar, ai = 0.0, br, bi = 0.0;
    if constexpr (CPLX_IN) {
        const double2 a = reinterpret_cast<const double2 *>(A)[i + c * lda];
        ar = a.x;
        ai = a.y;
        if (B) {
            const double2 b = reinterpret_cast<const double2 *>(B)[i + c * ldb];
            br = b.x;
            bi = b.y;
        } else {
            br = (i == c) ? 1.0 : 0.0;
        }
    } else {
        ar = A[i + c * lda];
        br = B ? B[i + c * ldb] : ((i == c) ? 1.0 : 0.0);
    }
    for (int j = 0; j < ne; ++j) {
        const double2 zj = z[j];
        cplx<T> v;
        v.x = (T)(zj.x * br - zj.y * bi - ar);
        v.y = (T)(zj.x * bi + zj.y * br - ai);
        F[j * sF + i + (long)c * ldf] = v;
    }
}

// Compose the row interchanges (r0 + i <-> piv[i]), i = 0..cnt-1 (cnt <= 32),
// applied in order, into moves "row dst[q] receives the old row src[q]".
// Run by one whole wave: lane q tracks one touched row position (at most
// 2 cnt <= 64 of them) and the row it currently holds; each interchange is a
// ballot lookup and two shuffles.  piv is in LDS.  Returns the number of
// moves (the same in every lane); dst/src (LDS) are written by the wave.
__device__ inline int compose_moves_wave(const int *piv, int r0, int cnt, int *dst, int *src)
{
    const int lane = threadIdx.x & 63;
    int pos = lane < cnt ? r0 + lane : -1;
    int val = pos;
    int n = cnt;
    for (int i = 0; i < cnt; ++i) {
        const int p = piv[i];
        const unsigned long long m = __ballot(pos == p);
        int ip;
        if (m) {
            ip = __ffsll((unsigned long long)m) - 1;
        } else {
            ip = n;
            if (lane == n) pos = val = p;
            ++n;
        }
        const int vi = __shfl(val, i, 64), vip = __shfl(val, ip, 64);
        if (lane == i) val = vip;
        if (lane == ip) val = vi;
    }
    const bool mv = lane < n && val != pos;
    const unsigned long long mm = __ballot(mv);
    if (mv) {
        const int slot = __popcll(mm & ((1ull << lane) - 1ull));
        dst[slot] = pos;
        src[slot] = val;
    }
    return __popcll(mm);
}

// Bit moves for the DPP lane permutations (32-bit lanes).
__device__ inline int as_bits(float v) { return __float_as_int(v); }
__device__ inline float from_bits(int b, float) { return __int_as_float(b); }
template <int CTRL> __device__ inline float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ inline double dpp_mov(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL> __device__ inline int dpp_mov(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
__device__ inline float lane_read(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
__device__ inline double lane_read(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// (v, i) <- the better of (v, i) and (ov, oi): larger v, ties to the lower i
template <typename T> __device__ inline void amax_take(T &v, int &i, T ov, int oi)
{
    const bool take = (ov > v) | ((ov == v) & (oi < i));   // branch-free
    v = take ? ov : v;
    i = take ? oi : i;
}
// Argmax over the 64 lanes of a wave with DPP row permutations (quad xor 1
// and 2, half-row and row mirror) and one read of each 16-lane row; the
// result is uniform over the wave.  All lanes must be active.
template <typename T> __device__ inline void wave_argmax(T &v, int &i)
{
    amax_take(v, i, dpp_mov<0xB1>(v), dpp_mov<0xB1>(i));    // quad_perm [1,0,3,2]
    amax_take(v, i, dpp_mov<0x4E>(v), dpp_mov<0x4E>(i));    // quad_perm [2,3,0,1]
    amax_take(v, i, dpp_mov<0x141>(v), dpp_mov<0x141>(i));  // row_half_mirror
    amax_take(v, i, dpp_mov<0x140>(v), dpp_mov<0x140>(i));  // row_mirror
    T bv = lane_read(v, 0);
    int bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
    for (int r = 1; r < 4; ++r) amax_take(bv, bi, lane_read(v, 16 * r), __builtin_amdgcn_readlane(i, 16 * r));
    v = bv;
    i = bi;
}
// 1 / p for a pivot: hardware reciprocal in FP32 (the factors are an
// FP32 preconditioner), correctly rounded division in FP64.
__device__ inline float2 pivot_inv(float2 p)
{
    const float rn = __builtin_amdgcn_rcpf(p.x * p.x + p.y * p.y);
    return make_float2(p.x * rn, -p.y * rn);
}
__device__ inline double2 pivot_inv(double2 p) { return cinv(p); }

// Panel factorisation.  One workgroup of NT threads per matrix.  The panel
// is processed in sub-blocks of IB columns: each sub-block is first brought
// up to date from the panel's earlier sub-blocks (left-looking), then held
// in registers -- R rows per thread, rows c0 + tid + NT*r -- while its IB
// columns are factored one by one (pivot search, swap, scale, rank-1
// update).  After each sub-block its interchanges are composed into row
// moves and applied to the rest of the panel in one pass; at the end the
// whole panel's interchanges are composed into moves for the other columns
// and applied to the row permutation perm (row i of P A is row perm[i] of A).
// The sequential parts (move composition, the small triangular solve for
// the sub-block's U rows) run on whole waves so that no step waits on one
// thread's chain of memory round trips.
template <typename T, int NT, int R, int IB, int NB>
__global__ __launch_bounds__(NT) void lu_panel_kernel(int n, cplx<T> *__restrict__ Fall, long ldf,
                                                      long sF, int k, int *__restrict__ ipiv_all,
                                                      int *__restrict__ perm_all, long sPiv,
                                                      int *__restrict__ swapmap_all,
                                                      int *__restrict__ info_all)
{
    using V = cplx<T>;
    static_assert(NB <= 32, "move composition tracks at most 64 rows");
    V *a = Fall + blockIdx.x * sF;
    int *ipiv = ipiv_all + blockIdx.x * sPiv;
    int *perm = perm_all + blockIdx.x * sPiv;
    int *swapmap = swapmap_all + blockIdx.x * (1 + 4 * NB);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr int NW = NT / 64;
    const int nbw = min(NB, n - k);

    __shared__ V Lsh[NB][NB + 1];      // L11 of the panel so far (unit lower)
    __shared__ V Ush[NB][IB];          // U rows k..c0-1 of the current sub-block
    __shared__ V cand_row[2][NW][IB];  // each wave's best row (pivot candidate)
    __shared__ V grow[2][IB];          // row g before the exchange
    __shared__ T cand_v[2][NW];
    __shared__ int cand_i[2][NW];
    __shared__ int s_ipiv[NB];
    __shared__ int s_mvd[2 * NB], s_mvs[2 * NB];
    __shared__ V s_stage[2 * IB][NB];
    __shared__ int s_nmv;

    if (k == 0)
        for (int i = tid; i < n; i += NT) perm[i] = i;

    for (int jb = 0; jb < nbw; jb += IB) {
        const int c0 = k + jb;
        const int w = min(IB, nbw - jb);

        // (a) U rows k..c0-1 of this sub-block: L11 (jb x jb, unit lower)
        //     solve, one wave per column (waves take columns in turn), lane i
        //     holding row k + i
        if (jb > 0) {
            for (int e = tid; e < jb * jb; e += NT) {
                const int i = e % jb, l = e / jb;
                Lsh[i][l] = a[(k + i) + (long)(k + l) * ldf];
            }
            __syncthreads();
            for (int c = wid; c < IB; c += NW) {
                V x = (c < w && lane < jb) ? a[(k + lane) + (long)(c0 + c) * ldf] : cmake<V>(0, 0);
                for (int l = 0; l + 1 < jb; ++l) {
                    V xl;
                    xl.x = lane_read(x.x, l);
                    xl.y = lane_read(x.y, l);
                    if (lane > l && lane < jb) x = csub(x, cmul(Lsh[lane][l], xl));
                }
                if (lane < jb) {
                    Ush[lane][c] = x;
                    if (c < w) a[(k + lane) + (long)(c0 + c) * ldf] = x;
                }
            }
            __syncthreads();
        }

        // (b) load rows c0..n-1 of the sub-block and subtract L[c0:, k:c0] * U[k:c0, sub];
        //     the L columns are fetched CW at a time so the loads overlap
        V val[R][IB];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int row = c0 + tid + NT * r;
#pragma unroll
            for (int c = 0; c < IB; ++c)
                val[r][c] = (row < n && c < w) ? a[row + (long)(c0 + c) * ldf] : cmake<V>(0, 0);
        }
        constexpr int CW = (16 / R) < 1 ? 1 : ((16 / R) > IB ? IB : (16 / R));   // columns per fetch
        for (int l0 = 0; l0 < jb; l0 += CW) {
            V lv[R][CW];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int row = c0 + tid + NT * r;
#pragma unroll
                for (int q = 0; q < CW; ++q)
                    lv[r][q] = (row < n) ? a[row + (long)(k + l0 + q) * ldf] : cmake<V>(0, 0);
            }
#pragma unroll
            for (int q = 0; q < CW; ++q) {
                V u[IB];
#pragma unroll
                for (int c = 0; c < IB; ++c) u[c] = Ush[l0 + q][c];
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int c = 0; c < IB; ++c) val[r][c] = csub(val[r][c], cmul(lv[r][q], u[c]));
            }
        }

        // (c) factor the sub-block column by column, one barrier per column:
        //     every wave publishes its best pivot candidate together with
        //     that row's IB values, and the owner of row g publishes row g;
        //     after the barrier every thread picks the winner the same way.
        //     The buffers alternate between two copies: a thread writing
        //     copy b for column jj + 1 has passed the barrier of column jj,
        //     by which time every read of copy b (column jj - 1) is done.
#pragma unroll
        for (int jj = 0; jj < IB; ++jj) {
            if (jj < w) {
                const int g = c0 + jj, b = jj & 1;
                // pivot search: largest |re|+|im|, ties to the lowest row
                T best = T(-1);
                int bi = 0x7fffffff;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int row = c0 + tid + NT * r;
                    if (row >= g && row < n) {
                        const T v = cabs1(val[r][jj]);
                        if (v > best) {
                            best = v;
                            bi = row;
                        }
                    }
                }
                wave_argmax(best, bi);
                if (lane == 0) {
                    cand_v[b][wid] = best;
                    cand_i[b][wid] = bi;
                }
                if (bi < n && tid == (bi - c0) % NT) {
                    const int rr = (bi - c0) / NT;
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (r == rr)
#pragma unroll
                            for (int c = 0; c < IB; ++c) cand_row[b][wid][c] = val[r][c];
                }
                const int own_g = (g - c0) % NT, rg = (g - c0) / NT;
                if (tid == own_g) {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (r == rg)
#pragma unroll
                            for (int c = 0; c < IB; ++c) grow[b][c] = val[r][c];
                }
                __syncthreads();
                // all candidates are loaded before any comparison
                T cv[NW];
                int ci[NW];
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    cv[q] = cand_v[b][q];
                    ci[q] = cand_i[b][q];
                }
                T bv = cv[0];
                int p = ci[0], ww = 0;
#pragma unroll
                for (int q = 1; q < NW; ++q) {
                    const bool take = (cv[q] > bv) | ((cv[q] == bv) & (ci[q] < p));
                    bv = take ? cv[q] : bv;
                    p = take ? ci[q] : p;
                    ww = take ? q : ww;
                }
                V pr[IB];
                if (!(bv > T(0)) || p >= n) {
                    // zero or non-finite column: keep the diagonal, flag the error
                    p = g;
#pragma unroll
                    for (int c = 0; c < IB; ++c) pr[c] = grow[b][c];
                    if (tid == 0 && info_all[blockIdx.x] == 0) info_all[blockIdx.x] = g + 1;
                } else {
#pragma unroll
                    for (int c = 0; c < IB; ++c) pr[c] = cand_row[b][ww][c];
                }
                if (tid == 0) s_ipiv[jb + jj] = p;
                // exchange rows g and p
                const int own_p = (p - c0) % NT, rp = (p - c0) / NT;
                if (tid == own_p) {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (r == rp)
#pragma unroll
                            for (int c = 0; c < IB; ++c) val[r][c] = grow[b][c];
                }
                if (tid == own_g) {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (r == rg)
#pragma unroll
                            for (int c = 0; c < IB; ++c) val[r][c] = pr[c];
                }
                // scale the column below the diagonal and update the sub-block
                const V inv = (cabs1(pr[jj]) > T(0)) ? pivot_inv(pr[jj]) : cmake<V>(0, 0);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int row = c0 + tid + NT * r;
                    if (row > g && row < n) {
                        const V l = cmul(val[r][jj], inv);
                        val[r][jj] = l;
#pragma unroll
                        for (int c = jj + 1; c < IB; ++c) val[r][c] = csub(val[r][c], cmul(l, pr[c]));
                    }
                }
            }
        }

        // (d) write the sub-block back
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int row = c0 + tid + NT * r;
            if (row < n)
#pragma unroll
                for (int c = 0; c < IB; ++c)
                    if (c < w) a[row + (long)(c0 + c) * ldf] = val[r][c];
        }
        // (e) the sub-block's interchanges, composed into row moves, applied
        //     to the other columns of the panel (all loads before any store)
        __syncthreads();
        if (wid == 0) {
            const int nm = compose_moves_wave(s_ipiv + jb, c0, w, s_mvd, s_mvs);
            if (lane == 0) s_nmv = nm;
        }
        __syncthreads();
        {
            const int nmv = s_nmv, nother = nbw - w;
            for (int e = tid; e < nmv * nother; e += NT) {
                const int q = e % nmv, t = e / nmv;
                const int col = (t < jb) ? (k + t) : (c0 + w + (t - jb));
                s_stage[q][t] = a[s_mvs[q] + (long)col * ldf];
            }
            __syncthreads();
            for (int e = tid; e < nmv * nother; e += NT) {
                const int q = e % nmv, t = e / nmv;
                const int col = (t < jb) ? (k + t) : (c0 + w + (t - jb));
                a[s_mvd[q] + (long)col * ldf] = s_stage[q][t];
            }
        }
        __syncthreads();
    }

    // the panel's interchanges: pivot indices, composed moves for the
    // columns outside the panel, and the same moves applied to perm (set to
    // the identity above when k == 0; the loop's last barrier orders it)
    if (tid < nbw) ipiv[k + tid] = s_ipiv[tid];
    if (wid == 0) {
        const int nm = compose_moves_wave(s_ipiv, k, nbw, s_mvd, s_mvs);
        int d = 0, v = 0;
        if (lane < nm) {
            d = s_mvd[lane];
            const int sr = s_mvs[lane];
            swapmap[1 + lane] = d;
            swapmap[1 + 2 * NB + lane] = sr;
            v = perm[sr];
        }
        // the wave's loads of perm all return before its store is issued
        if (lane < nm) perm[d] = v;
        if (lane == 0) swapmap[0] = nm;
    }
}

// Row interchanges of one panel (columns k..k+nbw-1) applied to a set of
// columns outside it -- the concatenation of [c0, c1) and [c2, c3) -- (mode
// bit 0), and U12 = L11^{-1} A12 for those of them right of the panel (mode
// bit 1).  Each block owns 64 columns of that set.  The kernel is latency
// bound, so it is laid out for few dependent steps:
//   1. the move list, L11 and the top nbw rows of the solve columns are
//      fetched at once;
//   2. the moved rows are staged through LDS (all reads before any write;
//      a column's moves sit on consecutive lanes, so the panel's top rows,
//      contiguous in a column, share cache lines);
//   3. moved rows are stored, except the top rows of solve columns, which
//      the solve takes from the stage and writes itself;
//   4. the solve: column c's rows g, g + 4, ... are held by lane g of a
//      quad, so the pivot row of step l is a DPP broadcast within the quad
//      and the substitution needs no barrier.
template <int CTRL> __device__ inline float2 dpp_v(float2 v)
{
    return make_float2(dpp_mov<CTRL>(v.x), dpp_mov<CTRL>(v.y));
}
template <int CTRL> __device__ inline double2 dpp_v(double2 v)
{
    return make_double2(dpp_mov<CTRL>(v.x), dpp_mov<CTRL>(v.y));
}
// v of lane g of each quad, for every lane of the quad (quad_perm [g,g,g,g]);
// g is a constant once the caller's loop is unrolled
template <typename V> __device__ inline V quad_bcast(V v, int g)
{
    switch (g) {
    case 0: return dpp_v<0x00>(v);
    case 1: return dpp_v<0x55>(v);
    case 2: return dpp_v<0xAA>(v);
    default: return dpp_v<0xFF>(v);
    }
}

template <typename T, int NB, bool CORR_MODE>
__global__ __launch_bounds__(256) void lu_swap_trsm_kernel(int n, cplx<T> *__restrict__ Fall, long ldf,
                                                           long sF, int k, int nbw, int c0, int c1, int c2,
                                                           int c3, int kc0, int kc1, int mode,
                                                           const int *__restrict__ swapmap_all)
{
    using V = cplx<T>;
    constexpr int CB = 64;
    static_assert(NB % 4 == 0 && NB <= 32, "rows of the solve in 4 groups; at most 2 NB moves");
    V *a = Fall + blockIdx.y * sF;
    const int *swapmap = swapmap_all + blockIdx.y * (1 + 4 * NB);
    const int tid = threadIdx.x;
    __shared__ V stage[2 * NB][CB + 1];
    __shared__ V Lsh[NB][NB + 1];
    __shared__ int dst[2 * NB], src[2 * NB];
    __shared__ int top_q[NB];   // top row k + i is written by move top_q[i] (-1: none)
    __shared__ int s_nm;
    __shared__ V Lc[(CORR_MODE ? NB : 1)][NB + 1];

    const int w1 = c1 - c0, ncols = w1 + (c3 - c2);
    auto col_of = [&](int oc) { return oc < w1 ? c0 + oc : c2 + (oc - w1); };
    const int colbase = blockIdx.x * CB;
    bool right = false;   // block holds a column right of the panel (and U12 is asked for)
    if (mode & 2)
        for (int c = 0; c < CB; ++c)
            if (colbase + c < ncols && col_of(colbase + c) >= k + nbw) right = true;

    // solve layout: column c = 16 wave + lane / 4, rows g + 4 j (g = lane mod 4)
    const int sc = (tid >> 6) * 16 + ((tid & 63) >> 2), g = tid & 3;
    const int soc = colbase + sc;
    const bool colok = right && soc < ncols && col_of(soc) >= k + nbw;
    V *pc = a + (long)(colok ? col_of(soc) : 0) * ldf + k;

    // 1. move list, L11, the solve columns' top rows
    if (mode & 1) {
        for (int e = tid; e < 1 + 4 * NB; e += 256) {
            const int v = swapmap[e];
            if (e == 0) s_nm = v;
            else if (e <= 2 * NB) dst[e - 1] = v;
            else src[e - 1 - 2 * NB] = v;
        }
    } else if (tid == 0) {
        s_nm = 0;
    }
    if (tid < NB) top_q[tid] = -1;
    // L11 strictly below the diagonal; zeros elsewhere (and past nbw), so
    // that the substitution below needs no per-row guard
    if (right)
        for (int e = tid; e < NB * NB; e += 256) {
            const int i = e % NB, l = e / NB;
            Lsh[i][l] = (i > l && i < nbw) ? a[(k + i) + (long)(k + l) * ldf] : cmake<V>(0, 0);
        }
    V xr[NB / 4];
#pragma unroll
    for (int j = 0; j < NB / 4; ++j) {
        const int i = g + 4 * j;
        xr[j] = (colok && i < nbw) ? pc[i] : cmake<V>(0, 0);
    }
    // correction rows of the solve column (rows kc0..kc1, final before this
    // launch), NB at a time; the first NB are fetched here
    const int kw = (mode & 4) ? kc1 - kc0 : 0;
    V u0[CORR_MODE ? NB : 1];
    const V *pu = a + (long)(colok ? col_of(soc) : 0) * ldf + kc0;
    if constexpr (CORR_MODE) {
#pragma unroll
        for (int q = 0; q < NB; ++q) u0[q] = (colok && q < kw) ? pu[q] : cmake<V>(0, 0);
    }
    __syncthreads();
    const int nm = s_nm;

    // 2. stage the moved rows
    if (right && tid < nm) {
        const int d = dst[tid] - k;
        if (d >= 0 && d < nbw) top_q[d] = tid;
    }
    for (int e = tid; e < nm * CB; e += 256) {
        const int q = e % nm, c = e / nm;
        const int oc = colbase + c;
        if (oc < ncols) stage[q][c] = a[src[q] + (long)col_of(oc) * ldf];
    }
    __syncthreads();

    // 3. store the moves (the solve writes the top rows of its columns)
    for (int e = tid; e < nm * CB; e += 256) {
        const int q = e % nm, c = e / nm;
        const int oc = colbase + c;
        if (oc < ncols) {
            const int col = col_of(oc), d = dst[q];
            const bool solved = (mode & 2) && col >= k + nbw && d >= k && d < k + nbw;
            if (!solved) a[d + (long)col * ldf] = stage[q][c];
        }
    }

    // 4. U12 = L11^{-1} A12, column-oriented forward substitution, after
    //    the correction of the top rows by earlier panels when asked (mode
    //    bit 2): rows k.. -= F[k.., kc0:kc1] F[kc0:kc1, col], up to three
    //    panels deep, NB correction rows at a time.  Those L rows are read
    //    back after this launch's moves are stored, so they may be columns
    //    of this launch, handled by this block.
    if (right) {
#pragma unroll
        for (int j = 0; j < NB / 4; ++j) {
            const int i = g + 4 * j;
            if (colok && i < nbw) {
                const int q = top_q[i];
                if (q >= 0) xr[j] = stage[q][sc];
            }
        }
        if constexpr (CORR_MODE) {
            for (int q0 = 0; q0 < kw; q0 += NB) {   // uniform
                if (q0 > 0) {
#pragma unroll
                    for (int q = 0; q < NB; ++q) u0[q] = (colok && q0 + q < kw) ? pu[q0 + q] : cmake<V>(0, 0);
                }
                __syncthreads();   // the previous chunk's reads of Lc are done
                for (int e = tid; e < NB * NB; e += 256) {
                    const int i = e % NB, q = e / NB;
                    Lc[i][q] = (i < nbw && q0 + q < kw) ? a[(k + i) + (long)(kc0 + q0 + q) * ldf] : cmake<V>(0, 0);
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < NB; ++q)
#pragma unroll
                    for (int j = 0; j < NB / 4; ++j) xr[j] = csub(xr[j], cmul(Lc[g + 4 * j][q], u0[q]));
            }
        }
#pragma unroll
        for (int l = 0; l < NB - 1; ++l) {
            if (l + 1 >= nbw) break;   // uniform
            const V xl = quad_bcast(xr[l >> 2], l & 3);
#pragma unroll
            for (int j = 0; j < NB / 4; ++j) xr[j] = csub(xr[j], cmul(Lsh[g + 4 * j][l], xl));
        }
        if (colok)
#pragma unroll
            for (int j = 0; j < NB / 4; ++j) {
                const int i = g + 4 * j;
                if (i < nbw) pc[i] = xr[j];
            }
    }
}

// After the last panel: flag a non-finite or zero diagonal of U (the first
// such index + 1, unless the panels already flagged a pivot).
template <typename T>
__global__ __launch_bounds__(256) void lu_finish_kernel(int n, const cplx<T> *__restrict__ Fall,
                                                        long ldf, long sF, int *__restrict__ info_all)
{
    const cplx<T> *a = Fall + blockIdx.x * sF;
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0x7fffffff;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const cplx<T> d = a[i + (long)i * ldf];
        if (!(cabs1(d) > T(0)) || !isfinite(d.x) || !isfinite(d.y)) atomicMin(&bad, i + 1);
    }
    __syncthreads();
    if (threadIdx.x == 0 && bad != 0x7fffffff && info_all[blockIdx.x] == 0) info_all[blockIdx.x] = bad;
}

constexpr int LU_NB = 32;

// Register budget: R rows x IB columns of complex values per thread.  Rows
// per thread grow with n; the sub-block is as wide as the registers allow
// without spilling (R * IB <= 64 complex values), since every sub-block costs
// global round trips (L11, the left-looking reloads, the in-panel moves).
// Measured per 32-column panel, batch 8: c64 4096 rows 224 -> 194 us going
// from IB 4 to 8; c128 4096 rows 370 -> 296 us (IB 2 -> 4), 2048 rows
// 192 -> 168 us and 1024 rows 133 -> 118 us (IB 4 -> 8).  Wider sub-blocks
// (16, 32) spill and run several times slower.
template <typename T> struct panel_cfg;
template <> struct panel_cfg<float> {
    static constexpr int NT = 512;
    static constexpr int ib(int R) { return R <= 8 ? 8 : 4; }
};
template <> struct panel_cfg<double> {
    static constexpr int NT = 512;
    static constexpr int ib(int R) { return R == 1 ? 4 : (R <= 4 ? 8 : (R <= 8 ? 4 : 2)); }
};

template <typename T, int R>
static void launch_panel(hipStream_t s, int n, cplx<T> *F, long ldf, long sF, int k, int *ipiv, int *perm,
                         long sPiv, int *swapmap, int *info, int batch)
{
    using P = panel_cfg<T>;
    constexpr int IB = P::ib(R);
    hipLaunchKernelGGL((lu_panel_kernel<T, P::NT, R, IB, LU_NB>), dim3(batch), dim3(P::NT), 0, s, n,
                       F, ldf, sF, k, ipiv, perm, sPiv, swapmap, info);
    FX_LAUNCH_CHECK();
}

// Largest n the register-resident panel supports (16 rows per thread).
template <typename T> constexpr int lu_max_n() { return 16 * panel_cfg<T>::NT; }

// The panel kernel instance for the rows left at column k.
template <typename T>
static void launch_panel_rows(hipStream_t s, int n, cplx<T> *F, long ldf, long sF, int k, int *ipiv, int *perm,
                              long sPiv, int *swapmap, int *info, int batch)
{
    using P = panel_cfg<T>;
    const int R = ceil_div(n - k, P::NT);
    if (R <= 1) launch_panel<T, 1>(s, n, F, ldf, sF, k, ipiv, perm, sPiv, swapmap, info, batch);
    else if (R <= 2) launch_panel<T, 2>(s, n, F, ldf, sF, k, ipiv, perm, sPiv, swapmap, info, batch);
    else if (R <= 4) launch_panel<T, 4>(s, n, F, ldf, sF, k, ipiv, perm, sPiv, swapmap, info, batch);
    else if (R <= 8) launch_panel<T, 8>(s, n, F, ldf, sF, k, ipiv, perm, sPiv, swapmap, info, batch);
    else launch_panel<T, 16>(s, n, F, ldf, sF, k, ipiv, perm, sPiv, swapmap, info, batch);
}

constexpr int LU_SWAP = 1, LU_TRSM = 2, LU_CORR = 4;
constexpr int LU_QB = 4;                     // panels per block of the blocked schedule
constexpr int LU_CORR_MAX = (LU_QB - 1) * LU_NB;
constexpr int LU_LISTS = 2 * LU_QB;          // move lists live at once (two blocks)
constexpr int LU_LIST_INTS = 1 + 4 * LU_NB;  // one move list of one matrix

// mode LU_CORR (with LU_TRSM): before the U-row solve, the top rows of the
// solved columns get -= F[k:k+nbw, kc0:kc1] F[kc0:kc1, col].  When those L
// columns are among this launch's columns, one block must hold them all.
template <typename T>
static void swap_trsm(hipStream_t s, int n, cplx<T> *F, long ldf, long sF, int k, int nbw, int c0, int c1, int c2,
                      int c3, int mode, const int *swapmap, int batch, int kc0 = 0, int kc1 = 0)
{
    const int ncols = (c1 - c0) + (c3 - c2);
    if (ncols <= 0) return;
    dim3 grid(ceil_div(ncols, 64), batch);
    if (mode & LU_CORR) {
        const bool inside = (kc0 < c1 && kc1 > c0) || (kc0 < c3 && kc1 > c2);
        if (!(mode & LU_TRSM) || kc1 - kc0 > LU_CORR_MAX || kc1 < kc0 || kc1 > k || (inside && ncols > 64))
            throw hip_error{hipErrorInvalidValue};
        hipLaunchKernelGGL((lu_swap_trsm_kernel<T, LU_NB, true>), grid, dim3(256), 0, s, n, F, ldf, sF, k, nbw, c0,
                           c1, c2, c3, kc0, kc1, mode, swapmap);
    } else {
        hipLaunchKernelGGL((lu_swap_trsm_kernel<T, LU_NB, false>), grid, dim3(256), 0, s, n, F, ldf, sF, k, nbw, c0,
                           c1, c2, c3, 0, 0, mode, swapmap);
    }
    FX_LAUNCH_CHECK();
}

// F[r0:r1, c0:c1] -= F[r0:r1, kc0:kc1] F[kc0:kc1, c0:c1]
template <typename T>
static void lu_gemm(hipStream_t s, cplx<T> *F, long ldf, long sF, int r0, int r1, int c0, int c1, int kc0, int kc1,
                    int batch)
{
    if (r1 <= r0 || c1 <= c0 || kc1 <= kc0) return;
    gemm<T, true, false>(s, r1 - r0, c1 - c0, kc1 - kc0, T(-1), F + r0 + (long)kc0 * ldf, ldf, sF,
                         F + kc0 + (long)c0 * ldf, ldf, sF, T(1), F + r0 + (long)c0 * ldf, ldf, sF, batch);
}

// One step of the factorisation's launch schedule (host logic, no device
// state): the executor below turns it into a launch, the host-side tests
// replay it.  kind: LU_OP_PANEL factors columns k..k+nbw-1 (rows k..n-1)
// and writes move list `list`; LU_OP_SWAP is swap_trsm() with that list;
// LU_OP_GEMM is F[c0:c1, c2:c3] -= F[c0:c1, kc0:kc1] F[kc0:kc1, c2:c3] (c0,
// c1 the row range); LU_OP_RECORD / LU_OP_WAIT order the two streams
// (`side` records, the other stream waits).  side: 1 for the panel stream.
enum { LU_OP_PANEL = 0, LU_OP_SWAP = 1, LU_OP_GEMM = 2, LU_OP_RECORD = 3, LU_OP_WAIT = 4 };
struct LuOp {
    int kind, side, k, nbw, c0, c1, c2, c3, kc0, kc1, mode, list;
};
constexpr int LU_OP_INTS = 12;

// The blocked right-looking schedule.  Panels are NB = 32 columns wide and
// grouped in blocks of QB = 4 (128 columns).  Each block updates most of the
// trailing matrix with one product of depth 128, where a panel-by-panel
// update would take four of depth 32.  For block B (columns b..e; f = e + NB
// ends the next block's first panel):
//   * N_j, after panel j of B: panel j's interchanges on B's columns left of
//     it; on the columns right of it up to f, the interchanges, its U rows
//     (swap_trsm) and the depth-32 update of the rows below.  This keeps B's
//     next panel and the next block's first panel current (right-looking).
//   * The previous block P (pb..b) finishes on the columns N_j of P did not
//     reach, in three parts: beside B's panel 0, P's interchanges, U rows
//     (corrected by P's earlier panels, mode LU_CORR) and depth-128 update
//     on columns b + NB .. f (needed by B's N_0); after N_0, the same
//     interchanges and U rows on the columns left of P and past f; then
//     the depth-128 product past f in QB - 1 column chunks, one beside each
//     of B's later panels.
// Only the panels run on the panel stream; every other step is on the main
// stream, so that the wide products keep the whole device.  A row
// permutation commutes with a row-wise update as long as the update's L rows
// get it too.  That is why a block's interchanges can reach the far columns
// after later panels are factored: the far columns and the L columns of
// earlier blocks get each block's interchanges in block order.  Move lists:
// four per block, the two most recent blocks' live at once.  Without a panel
// stream (side = false) the same steps run in the same order on one stream,
// and the records and waits are left out.
inline std::vector<LuOp> lu_schedule_blocks(int n, bool side)
{
    constexpr int NB = LU_NB, BW = LU_QB * LU_NB;
    std::vector<LuOp> ops;
    auto add = [&](LuOp o) { ops.push_back(o); };
    auto record = [&](int sd) {
        if (side) add({LU_OP_RECORD, sd, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0});
    };
    auto wait = [&](int sd) {
        if (side) add({LU_OP_WAIT, sd, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0});
    };
    auto list_of = [](int B, int j) { return (B & 1) * LU_QB + j; };
    auto panel = [&](int B, int j, int k) {   // on the panel stream, after the main stream's work so far
        record(0);
        wait(1);
        add({LU_OP_PANEL, side ? 1 : 0, k, std::min(NB, n - k), 0, 0, 0, 0, 0, 0, 0, list_of(B, j)});
        record(1);
    };
    auto swap = [&](int B, int j, int k, int nbw, int c0, int c1, int c2, int c3, int mode, int kc0) {
        c1 = std::max(c0, c1);
        c3 = std::max(c2, c3);
        if (c1 - c0 + c3 - c2 <= 0) return;
        if (!(mode & LU_TRSM) || kc0 >= k) mode &= ~LU_CORR;
        add({LU_OP_SWAP, 0, k, nbw, c0, c1, c2, c3, (mode & LU_CORR) ? kc0 : 0, (mode & LU_CORR) ? k : 0, mode,
             list_of(B, j)});
    };
    auto gemm = [&](int r0, int r1, int c0, int c1, int kc0, int kc1) {
        if (r1 <= r0 || c1 <= c0 || kc1 <= kc0) return;
        add({LU_OP_GEMM, 0, 0, 0, r0, r1, c0, c1, kc0, kc1, 0, 0});
    };
    const int nblk = ceil_div(n, BW);
    for (int B = 0; B < nblk; ++B) {
        const int b = B * BW, e = std::min(n, b + BW), f = std::min(n, e + NB);
        const int np = ceil_div(e - b, NB);
        panel(B, 0, b);
        // the previous block P (pb..b, four full panels): its interchanges,
        // U rows and depth-128 update of this block's columns past its first
        // panel and of the next block's first panel (b + NB .. f), beside
        // panel 0 of this block
        const int pb = b - BW;
        std::vector<int> chunk;   // column chunks of P's depth-128 product on its far columns f..n
        if (B > 0) {
            for (int j = 0; j < LU_QB; ++j)
                swap(B - 1, j, pb + j * NB, NB, b + NB, f, 0, 0, LU_SWAP | LU_TRSM | LU_CORR, pb);
            gemm(b, n, b + NB, f, pb, b);
            const int nch = std::max(1, np - 1);
            for (int c = 0; c <= nch; ++c) chunk.push_back(f + (int)((long)(n - f) * c / nch / 64 * 64));
            chunk.back() = n;
        }
        // P's interchanges, U rows and update on the columns left of it and
        // past f, after this block's N_0 so that they do not hold it up
        auto far_of_previous = [&]() {
            for (int j = 0; j < LU_QB; ++j)
                swap(B - 1, j, pb + j * NB, NB, 0, pb, f, n, LU_SWAP | LU_TRSM | LU_CORR, pb);
        };
        for (int j = 0; j < np; ++j) {
            const int kj = b + j * NB, wj = std::min(NB, e - kj);
            wait(0);   // panel j
            swap(B, j, kj, wj, b, kj, kj + wj, f, LU_SWAP | LU_TRSM, 0);
            gemm(kj + wj, n, kj + wj, f, kj, kj + wj);
            if (j + 1 < np) {
                panel(B, j + 1, kj + wj);
                if (B > 0) {
                    if (j == 0) far_of_previous();
                    gemm(b, n, chunk[j], chunk[j + 1], pb, b);
                }
            }
        }
        if (B > 0 && np == 1) {
            far_of_previous();
            gemm(b, n, chunk[0], chunk[1], pb, b);
        }
    }
    // the last block's interchanges on the columns left of it
    if (nblk > 0) {
        const int B = nblk - 1, b = B * BW, np = ceil_div(n - b, NB);
        for (int j = 0; j < np; ++j) {
            const int kj = b + j * NB;
            swap(B, j, kj, std::min(NB, n - kj), 0, b, 0, 0, LU_SWAP, 0);
        }
    }
    return ops;
}

// The paired schedule: panels in pairs (k0, k1 = k0 + 32), whose far
// trailing update is one product of depth 64.  Its chain is one interchange
// step and one narrow product per panel, against the blocked schedule's
// extra steps per block (the next columns' corrections by the previous
// block), so it is the faster one where the panel chain, not the trailing
// products, sets the time.  Per pair:
//   1. panel k1's columns get panel k0's interchanges, U rows and update;
//      panel k1 is factored on the panel stream while
//   2. the far columns get the previous pair's deferred update, then panel
//      k0's interchanges and U rows in one launch (the left columns, which
//      hold the deferred update's L rows, get the interchanges in the same
//      launch, after the update has read them);
//   3. panel k2 = k1 + 32's columns get panel k1's interchanges (applied to
//      panel k0's L too, so that its rows match), the depth-32 correction of
//      rows k1..k2 by panel k0, panel k1's U rows and the depth-64 update of
//      rows k2.. by both panels; panel k2 is factored on the panel stream
//      while
//   4. the far columns get the same as in 3, except that the depth-64
//      update of the far half of them is deferred to step 2 of the next
//      pair, so that both panels of a pair overlap a trailing product.
// Move lists alternate between two buffers.
inline std::vector<LuOp> lu_schedule_pairs(int n, bool side)
{
    constexpr int NB = LU_NB;
    std::vector<LuOp> ops;
    auto add = [&](LuOp o) { ops.push_back(o); };
    auto lst = [](int k) { return (k / NB) & 1; };
    auto swap = [&](int k, int nbw, int c0, int c1, int c2, int c3, int mode, int kc0 = 0, int kc1 = 0) {
        if ((c1 - c0) + (c3 - c2) <= 0) return;
        add({LU_OP_SWAP, 0, k, nbw, c0, c1, c2, c3, kc0, kc1, mode, lst(k)});
    };
    auto gemm = [&](int r0, int r1, int c0, int c1, int kc0, int kc1) {
        if (r1 <= r0 || c1 <= c0 || kc1 <= kc0) return;
        add({LU_OP_GEMM, 0, 0, 0, r0, r1, c0, c1, kc0, kc1, 0, 0});
    };
    auto panel_side = [&](int k) {
        if (side) {
            add({LU_OP_RECORD, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0});
            add({LU_OP_WAIT, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0});
        }
        add({LU_OP_PANEL, side ? 1 : 0, k, std::min(NB, n - k), 0, 0, 0, 0, 0, 0, 0, lst(k)});
        if (side) add({LU_OP_RECORD, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0});
    };
    auto join = [&]() {
        if (side) add({LU_OP_WAIT, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0});
    };
    int pc0 = n, pr0 = n, pk0 = 0, pk1 = 0;   // the deferred update: F[pr0:, pc0:] -= F[pr0:, pk0:pk1] F[pk0:pk1, pc0:]
    add({LU_OP_PANEL, 0, 0, std::min(NB, n), 0, 0, 0, 0, 0, 0, 0, 0});
    for (int k0 = 0; k0 < n; k0 += 2 * NB) {
        const int w0 = std::min(NB, n - k0), k1 = k0 + w0;
        if (k1 >= n) {   // a last panel on its own (no far columns, nothing deferred)
            swap(k0, w0, 0, k0, 0, 0, LU_SWAP);
            break;
        }
        const int w1 = std::min(NB, n - k1), k2 = k1 + w1;
        swap(k0, w0, k1, k2, 0, 0, LU_SWAP | LU_TRSM);   // 1.
        gemm(k1, n, k1, k2, k0, k1);
        panel_side(k1);
        gemm(pr0, n, pc0, n, pk0, pk1);   // 2.
        pc0 = n;
        swap(k0, w0, 0, k0, k2, n, LU_SWAP | LU_TRSM);
        join();
        if (k2 >= n) {   // panel k1 was the last
            swap(k1, w1, 0, k1, 0, 0, LU_SWAP);
            break;
        }
        const int w2 = std::min(NB, n - k2), k3 = k2 + w2;
        swap(k1, w1, k0, k1, k2, k3, LU_SWAP | LU_CORR | LU_TRSM, k0, k1);   // 3.
        gemm(k2, n, k2, k3, k0, k2);
        panel_side(k2);
        swap(k1, w1, 0, k0, k3, n, LU_SWAP | LU_CORR | LU_TRSM, k0, k1);   // 4.
        const int mid = std::min(n, k3 + NB + ((n - k3 - NB) / 2 + 63) / 64 * 64);
        gemm(k2, n, k3, mid, k0, k2);
        pc0 = mid;
        pr0 = k2;
        pk0 = k0;
        pk1 = k2;
        join();
    }
    return ops;
}

// Which schedule: the blocked one from this order up, where the trailing
// products outweigh the panel chain (measured: at n = 4096 and 8 matrices
// the paired schedule factors faster, at n = 8192 and 16 the blocked one).
constexpr int LU_BLOCKS_MIN_N = 6144;
enum { LU_FORM_AUTO = -1, LU_FORM_PAIRS = 0, LU_FORM_BLOCKS = 1 };
// process-wide choice (LU_FORM_AUTO: by order); both give an LU with
// partial pivoting, equal up to rounding
static std::atomic<int> g_lu_form{LU_FORM_AUTO};
inline std::vector<LuOp> lu_schedule(int n, bool side, int form = LU_FORM_AUTO)
{
    if (form == LU_FORM_AUTO) form = g_lu_form.load(std::memory_order_relaxed);
    if (form == LU_FORM_AUTO) form = n >= LU_BLOCKS_MIN_N ? LU_FORM_BLOCKS : LU_FORM_PAIRS;
    return form == LU_FORM_BLOCKS ? lu_schedule_blocks(n, side) : lu_schedule_pairs(n, side);
}

// Factor `batch` matrices of order n (stride sF, leading dimension ldf) in
// place by the schedule lu_schedule picks.  ipiv/perm: n ints per matrix
// (stride sPiv).  swapmap: LU_LISTS * LU_LIST_INTS ints per matrix of
// scratch.  info: one int per matrix, 0 on success, else 1 + the first
// zero/non-finite pivot index.  s2: the panel stream (nullptr: everything
// on s); ev_a orders s2 after s, ev_b s after s2.
template <typename T>
void getrf_batched(hipStream_t s, hipStream_t s2, hipEvent_t ev_a, hipEvent_t ev_b, int n, cplx<T> *F, long ldf,
                   long sF, int *ipiv, int *perm, long sPiv, int *swapmap, int *info, int batch)
{
    const long smap = (long)batch * LU_LIST_INTS;
    for (const LuOp &o : lu_schedule(n, s2 != nullptr)) {
        hipStream_t st = (o.side && s2) ? s2 : s;
        int *sm = swapmap + o.list * smap;
        switch (o.kind) {
        case LU_OP_PANEL:
            launch_panel_rows<T>(st, n, F, ldf, sF, o.k, ipiv, perm, sPiv, sm, info, batch);
            break;
        case LU_OP_SWAP:
            swap_trsm<T>(st, n, F, ldf, sF, o.k, o.nbw, o.c0, o.c1, o.c2, o.c3, o.mode, sm, batch, o.kc0, o.kc1);
            break;
        case LU_OP_GEMM:
            lu_gemm<T>(st, F, ldf, sF, o.c0, o.c1, o.c2, o.c3, o.kc0, o.kc1, batch);
            break;
        case LU_OP_RECORD:
            FX_CHECK(hipEventRecord(o.side ? ev_b : ev_a, st));
            break;
        case LU_OP_WAIT:
            FX_CHECK(hipStreamWaitEvent(st, o.side ? ev_a : ev_b, 0));
            break;
        }
    }
    hipLaunchKernelGGL((lu_finish_kernel<T>), dim3(batch), dim3(256), 0, s, n, F, ldf, sF, info);
    FX_LAUNCH_CHECK();
}

template <typename T>
void shift_build(hipStream_t s, bool cplx_in, int n, const double *A, long lda, const double *B,
                 long ldb, const double2 *z, int ne, cplx<T> *F, long ldf, long sF)
{
    const long nn = (long)n * n;
    dim3 grid((unsigned)((nn + 255) / 256));
    if (cplx_in)
        hipLaunchKernelGGL((shift_build_kernel<T, true>), grid, dim3(256), 0, s, n, A, lda, B, ldb, z,
                           ne, F, ldf, sF);
    else
        hipLaunchKernelGGL((shift_build_kernel<T, false>), grid, dim3(256), 0, s, n, A, lda, B, ldb, z,
                           ne, F, ldf, sF);
    FX_LAUNCH_CHECK();
}

}  // namespace fx
