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
    static_assert(IB <= NT / 64, "one wave per sub-block column in the U-row solve");
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
    __shared__ V prow[2][IB], grow[2][IB];
    __shared__ T redv[2][NW];
    __shared__ int redi[2][NW];
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
        //     solve, one wave per column, lane i holding row k + i
        if (jb > 0) {
            for (int e = tid; e < jb * jb; e += NT) {
                const int i = e % jb, l = e / jb;
                Lsh[i][l] = a[(k + i) + (long)(k + l) * ldf];
            }
            __syncthreads();
            if (wid < IB) {
                const int c = wid;
                V x = (c < w && lane < jb) ? a[(k + lane) + (long)(c0 + c) * ldf] : cmake<V>(0, 0);
                for (int l = 0; l + 1 < jb; ++l) {
                    V xl;
                    xl.x = __shfl(x.x, l, 64);
                    xl.y = __shfl(x.y, l, 64);
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

        // (c) factor the sub-block column by column.  The reduction and row
        //     buffers alternate between two copies, so one column needs two
        //     barriers: a thread that writes copy b for column jj + 1 has
        //     passed the second barrier of column jj, by which time every
        //     read of copy b (column jj - 1) is done.
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
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    const T ov = __shfl_xor(best, off, 64);
                    const int oi = __shfl_xor(bi, off, 64);
                    if (ov > best || (ov == best && oi < bi)) {
                        best = ov;
                        bi = oi;
                    }
                }
                if (lane == 0) {
                    redv[b][wid] = best;
                    redi[b][wid] = bi;
                }
                __syncthreads();
                // every thread reduces the NW wave results the same way
                T bv = redv[b][0];
                int p = redi[b][0];
#pragma unroll
                for (int q = 1; q < NW; ++q) {
                    const T ov = redv[b][q];
                    const int oi = redi[b][q];
                    if (ov > bv || (ov == bv && oi < p)) {
                        bv = ov;
                        p = oi;
                    }
                }
                if (!(bv > T(0)) || p >= n) {
                    // zero or non-finite column: keep the diagonal, flag the error
                    p = g;
                    if (tid == 0 && info_all[blockIdx.x] == 0) info_all[blockIdx.x] = g + 1;
                }
                if (tid == 0) s_ipiv[jb + jj] = p;
                // exchange rows g and p of the sub-block through LDS
                const int own_p = (p - c0) % NT, rp = (p - c0) / NT;
                const int own_g = (g - c0) % NT, rg = (g - c0) / NT;
                if (tid == own_p) {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (r == rp)
#pragma unroll
                            for (int c = 0; c < IB; ++c) prow[b][c] = val[r][c];
                }
                if (tid == own_g) {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (r == rg)
#pragma unroll
                            for (int c = 0; c < IB; ++c) grow[b][c] = val[r][c];
                }
                __syncthreads();
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
                            for (int c = 0; c < IB; ++c) val[r][c] = prow[b][c];
                }
                // scale the column below the diagonal and update the sub-block
                V pr[IB];
#pragma unroll
                for (int c = 0; c < IB; ++c) pr[c] = prow[b][c];
                const V inv = (cabs1(pr[jj]) > T(0)) ? cinv(pr[jj]) : cmake<V>(0, 0);
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

// Row interchanges of one panel applied to every column outside it, then
// U12 = L11^{-1} A12 for the columns right of the panel.  Each block owns
// 64 columns; moved values are staged through LDS so that all reads happen
// before any write.
template <typename T, int NB>
__global__ __launch_bounds__(256) void lu_swap_trsm_kernel(int n, cplx<T> *__restrict__ Fall, long ldf,
                                                           long sF, int k, int nbw,
                                                           const int *__restrict__ swapmap_all)
{
    using V = cplx<T>;
    constexpr int CB = 64;
    V *a = Fall + blockIdx.y * sF;
    const int *swapmap = swapmap_all + blockIdx.y * (1 + 4 * NB);
    const int tid = threadIdx.x;
    __shared__ V stage[2 * NB][CB];
    __shared__ V Lsh[NB][NB + 1];
    __shared__ int dst[2 * NB], src[2 * NB];

    const int nm = swapmap[0];
    for (int e = tid; e < nm; e += 256) {
        dst[e] = swapmap[1 + e];
        src[e] = swapmap[1 + 2 * NB + e];
    }
    const int colbase = blockIdx.x * CB;     // index among the n - nbw outer columns
    const bool right = colbase + CB > k;     // block holds columns right of the panel
    if (right)
        for (int e = tid; e < nbw * nbw; e += 256) {
            const int i = e % nbw, l = e / nbw;
            Lsh[i][l] = a[(k + i) + (long)(k + l) * ldf];
        }
    __syncthreads();
    for (int e = tid; e < nm * CB; e += 256) {
        const int c = e % CB, q = e / CB;
        const int oc = colbase + c;
        if (oc < n - nbw) {
            const int col = oc < k ? oc : oc + nbw;
            stage[q][c] = a[src[q] + (long)col * ldf];
        }
    }
    __syncthreads();
    for (int e = tid; e < nm * CB; e += 256) {
        const int c = e % CB, q = e / CB;
        const int oc = colbase + c;
        if (oc < n - nbw) {
            const int col = oc < k ? oc : oc + nbw;
            a[dst[q] + (long)col * ldf] = stage[q][c];
        }
    }
    __syncthreads();
    if (right && tid < CB) {
        const int oc = colbase + tid;
        if (oc >= k && oc < n - nbw) {
            const int col = oc + nbw;
            V *pc = a + (long)col * ldf + k;
            V x[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) x[i] = (i < nbw) ? pc[i] : cmake<V>(0, 0);
#pragma unroll
            for (int i = 1; i < NB; ++i)
#pragma unroll
                for (int l = 0; l < i; ++l)
                    if (i < nbw) x[i] = csub(x[i], cmul(Lsh[i][l], x[l]));
#pragma unroll
            for (int i = 0; i < NB; ++i)
                if (i < nbw) pc[i] = x[i];
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



template <typename T> struct panel_cfg;
// Register budget: R rows x IB columns of complex values per thread.  Rows
// per thread grow with n; the sub-block narrows so that R * IB stays <= 64
// (c64) / 32 (c128) complex values.
template <typename T> struct panel_cfg;
template <> struct panel_cfg<float> {
    static constexpr int NT = 512;
    static constexpr int ib(int R) { return R <= 4 ? 8 : 4; }
};
template <> struct panel_cfg<double> {
    static constexpr int NT = 512;
    static constexpr int ib(int R) { return R <= 4 ? 4 : 2; }
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

// Factor `batch` matrices of order n (stride sF, leading dimension ldf) in
// place.  ipiv/perm: n ints per matrix (stride sPiv).  swapmap: (1 + 4 NB)
// ints per matrix of scratch.  info: one int per matrix, 0 on success, else
// 1 + the first zero/non-finite pivot index.
//
// Look-ahead of depth one: after the interchanges and U12 of panel k, the
// columns of panel k+1 are updated first and that panel is factored on the
// side stream s2 while the rest of the trailing update runs on s.  ev_a and
// ev_b order the two streams; s2 == nullptr disables the look-ahead.
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

template <typename T>
static void lu_update(hipStream_t s, int n, cplx<T> *F, long ldf, long sF, int k, int nbw, int c0, int c1,
                      int batch)
{
    // A[k+nbw:, c0:c1] -= L21 U12[:, c0:c1]
    const int m2 = n - k - nbw, nc = c1 - c0;
    if (m2 <= 0 || nc <= 0) return;
    cplx<T> *L21 = F + (k + nbw) + (long)k * ldf;
    cplx<T> *U12 = F + k + (long)c0 * ldf;
    cplx<T> *A22 = F + (k + nbw) + (long)c0 * ldf;
    gemm<T, true, false>(s, m2, nc, nbw, T(-1), L21, ldf, sF, U12, ldf, sF, T(1), A22, ldf, sF, batch);
}

template <typename T>
void getrf_batched(hipStream_t s, hipStream_t s2, hipEvent_t ev_a, hipEvent_t ev_b, int n, cplx<T> *F, long ldf,
                   long sF, int *ipiv, int *perm, long sPiv, int *swapmap, int *info, int batch)
{
    launch_panel_rows<T>(s, n, F, ldf, sF, 0, ipiv, perm, sPiv, swapmap, info, batch);
    for (int k = 0; k < n; k += LU_NB) {
        const int nbw = std::min(LU_NB, n - k);
        const int outer = n - nbw;
        if (outer > 0) {
            dim3 grid(ceil_div(outer, 64), batch);
            hipLaunchKernelGGL((lu_swap_trsm_kernel<T, LU_NB>), grid, dim3(256), 0, s, n, F, ldf, sF,
                               k, nbw, swapmap);
            FX_LAUNCH_CHECK();
        }
        const int kn = k + nbw;            // next panel start
        if (kn >= n) break;
        const int nbw2 = std::min(LU_NB, n - kn);
        if (s2) {
            lu_update<T>(s, n, F, ldf, sF, k, nbw, kn, kn + nbw2, batch);
            FX_CHECK(hipEventRecord(ev_a, s));
            FX_CHECK(hipStreamWaitEvent(s2, ev_a, 0));
            launch_panel_rows<T>(s2, n, F, ldf, sF, kn, ipiv, perm, sPiv, swapmap, info, batch);
            FX_CHECK(hipEventRecord(ev_b, s2));
            lu_update<T>(s, n, F, ldf, sF, k, nbw, kn + nbw2, n, batch);
            FX_CHECK(hipStreamWaitEvent(s, ev_b, 0));
        } else {
            lu_update<T>(s, n, F, ldf, sF, k, nbw, kn, n, batch);
            launch_panel_rows<T>(s, n, F, ldf, sF, kn, ipiv, perm, sPiv, swapmap, info, batch);
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
