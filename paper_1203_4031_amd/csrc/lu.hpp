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
    // correction rows of the solve column (rows kc0..kc1, final before this launch)
    const int kw = (mode & 4) ? kc1 - kc0 : 0;
    V u0[CORR_MODE ? NB : 1];
    if constexpr (CORR_MODE) {
        const V *pu = a + (long)(colok ? col_of(soc) : 0) * ldf + kc0;
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
    //    the correction of the top rows by an earlier panel when asked
    //    (mode bit 2): rows k.. -= F[k.., kc0:kc1] F[kc0:kc1, col].  Those
    //    L rows are read back after this launch's moves are stored, so
    //    they may be columns of this launch, handled by this block.
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
            if (kw > 0) {
                __syncthreads();
                for (int e = tid; e < NB * NB; e += 256) {
                    const int i = e % NB, q = e / NB;
                    Lc[i][q] = (i < nbw && q < kw) ? a[(k + i) + (long)(kc0 + q) * ldf] : cmake<V>(0, 0);
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
        if (!(mode & LU_TRSM) || kc1 - kc0 > LU_NB || kc1 < kc0 || kc1 > k || (inside && ncols > 64))
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

// Factor `batch` matrices of order n (stride sF, leading dimension ldf) in
// place.  ipiv/perm: n ints per matrix (stride sPiv).  swapmap: 2 (1 + 4 NB)
// ints per matrix of scratch.  info: one int per matrix, 0 on success, else
// 1 + the first zero/non-finite pivot index.
//
// Panels are NB = 32 columns wide and taken in pairs (k0, k1 = k0 + 32).
// The far trailing update of a pair is one product of depth 64 instead of
// two of depth 32, which halves the trailing-matrix traffic.  Per pair:
//   1. panel k1's columns get panel k0's interchanges, U rows and update;
//      panel k1 is factored on s2 (the look-ahead stream) while
//   2. the far columns get the previous pair's deferred update (below),
//      then panel k0's interchanges and U rows in one launch (the left
//      columns, which hold the deferred update's L rows, get the
//      interchanges in the same launch, after the update has read them);
//   3. panel k2 = k1 + 32's columns get panel k1's interchanges (applied
//      to panel k0's L too, so that its rows match), the depth-32
//      correction of rows k1..k2 by panel k0, panel k1's U rows and the
//      depth-64 update of rows k2.. by both panels; panel k2 is factored
//      on s2 while
//   4. the far columns get the same as in 3, except that the depth-64
//      update of the far half of them is deferred to step 2 of the next
//      pair, so that both panels of a pair overlap a trailing product.
// A row permutation commutes with a row-wise update, so applying a later
// panel's interchanges before an earlier panel's update gives the same
// matrix, as long as the update's L rows get them too.  The columns left
// of a panel get its interchanges off the critical chain.  ev_a and ev_b
// order the two streams; s2 == nullptr runs everything on s in the same
// order.  The move lists alternate between two buffers.
template <typename T>
void getrf_batched(hipStream_t s, hipStream_t s2, hipEvent_t ev_a, hipEvent_t ev_b, int n, cplx<T> *F, long ldf,
                   long sF, int *ipiv, int *perm, long sPiv, int *swapmap, int *info, int batch)
{
    constexpr int NB = LU_NB;
    const long smap = (long)batch * (1 + 4 * NB);   // one move list per matrix
    auto sm = [&](int k) { return swapmap + ((k / NB) & 1) * smap; };
    hipStream_t sp = s2 ? s2 : s;
    auto panel_side = [&](int k) {
        if (s2) {
            FX_CHECK(hipEventRecord(ev_a, s));
            FX_CHECK(hipStreamWaitEvent(s2, ev_a, 0));
        }
        launch_panel_rows<T>(sp, n, F, ldf, sF, k, ipiv, perm, sPiv, sm(k), info, batch);
        if (s2) FX_CHECK(hipEventRecord(ev_b, s2));
    };
    auto join = [&]() {
        if (s2) FX_CHECK(hipStreamWaitEvent(s, ev_b, 0));
    };
    // the deferred depth-64 update: F[pr0:, pc0:] -= F[pr0:, pk0:pk1] F[pk0:pk1, pc0:]
    int pc0 = n, pr0 = n, pk0 = 0, pk1 = 0;
    launch_panel_rows<T>(s, n, F, ldf, sF, 0, ipiv, perm, sPiv, sm(0), info, batch);
    for (int k0 = 0; k0 < n; k0 += 2 * NB) {
        const int w0 = std::min(NB, n - k0), k1 = k0 + w0;
        if (k1 >= n) {   // a last panel on its own (no far columns, nothing deferred)
            swap_trsm<T>(s, n, F, ldf, sF, k0, w0, 0, k0, 0, 0, LU_SWAP, sm(k0), batch);
            break;
        }
        const int w1 = std::min(NB, n - k1), k2 = k1 + w1;
        // 1. panel k1's columns
        swap_trsm<T>(s, n, F, ldf, sF, k0, w0, k1, k2, 0, 0, LU_SWAP | LU_TRSM, sm(k0), batch);
        lu_gemm<T>(s, F, ldf, sF, k1, n, k1, k2, k0, k1, batch);
        panel_side(k1);
        // 2. far and left columns: the deferred update first, on rows and L
        //    columns that panel k0's interchanges have not reached yet (the
        //    two stay consistent), then panel k0's interchanges on the left
        //    and far columns and its U rows on the far ones, in one launch
        lu_gemm<T>(s, F, ldf, sF, pr0, n, pc0, n, pk0, pk1, batch);
        pc0 = n;
        swap_trsm<T>(s, n, F, ldf, sF, k0, w0, 0, k0, k2, n, LU_SWAP | LU_TRSM, sm(k0), batch);
        join();
        if (k2 >= n) {   // panel k1 was the last
            swap_trsm<T>(s, n, F, ldf, sF, k1, w1, 0, k1, 0, 0, LU_SWAP, sm(k1), batch);
            break;
        }
        const int w2 = std::min(NB, n - k2), k3 = k2 + w2;
        // 3. panel k2's columns: panel k1's interchanges (on panel k0's L
        //    columns too), the depth-32 correction of rows k1..k2 by panel
        //    k0 and panel k1's U rows in one launch, then the depth-64
        //    update of rows k2.. by both panels
        swap_trsm<T>(s, n, F, ldf, sF, k1, w1, k0, k1, k2, k3, LU_SWAP | LU_CORR | LU_TRSM, sm(k1), batch, k0, k1);
        lu_gemm<T>(s, F, ldf, sF, k2, n, k2, k3, k0, k2, batch);
        panel_side(k2);
        // 4. far and left columns; the far columns past `mid` wait for the
        //    next pair's step 2 (panel k3 = k2 + 32's columns are before mid)
        swap_trsm<T>(s, n, F, ldf, sF, k1, w1, 0, k0, k3, n, LU_SWAP | LU_CORR | LU_TRSM, sm(k1), batch, k0, k1);
        const int mid = std::min(n, k3 + NB + ((n - k3 - NB) / 2 + 63) / 64 * 64);
        lu_gemm<T>(s, F, ldf, sF, k2, n, k3, mid, k0, k2, batch);
        pc0 = mid;
        pr0 = k2;
        pk0 = k0;
        pk1 = k2;
        join();
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
