// FEAST driver and C interface.
//
// One solve is the guide's FEAST iteration (section "The FEAST Algorithm"),
// with the reverse-communication steps of its RCI figure carried out by this
// library's own kernels, in the same order:
//   factor (ijob 10)  shift_build + getrf_batched, all contour nodes at once,
//                     factors kept resident across loops (fpm(10) = 1)
//   solve  (ijob 11)  getrs_batched against B X (ijob 40) for every node;
//          (ijob 21)  complex Hermitian pencils add the adjoint solve
//   quadrature        accumulate_kernel: Q = sum_j w_j Y_j (FP64)
//   Rayleigh-Ritz     A Q, B Q (ijob 30/40), Q^H A Q, Q^H B Q, reduced
//                     eigenproblem by GPU Jacobi, Ritz vectors, residuals
// The host only decides convergence from a few scalars per loop.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "feastx.h"

#include "common.hpp"
#include "gemm.hpp"
#include "jacobi.hpp"
#include "lu.hpp"
#include "rr.hpp"
#include "solve.hpp"
#include "bortho.hpp"
#include "nonherm.hpp"

namespace fx {

struct alloc_error {};
struct solver_error {
    int info;
};

// ------------------------------------------------------------ workspace
// Named device buffers that only grow; reused across calls.
struct Workspace {
    std::map<std::string, std::pair<void *, size_t>> dev;
    std::map<std::string, std::pair<void *, size_t>> host;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;            // look-ahead panels of the LU, adjoint solves (side_stream())
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    // Factorisation on a split of the CUs: the trailing updates on `fmain`,
    // the look-ahead panels on `fside`, which owns `fres` CUs per XCD that
    // `fmain` never uses, so a panel starts at once instead of waiting for
    // the trailing update to drain the device.  Created on first use, only
    // for workspaces that ask for it (want_split).
    bool want_split = false;
    // Look-ahead on a second stream.  Only the single-solve workspace uses
    // it: an executor slot keeps all its work on one in-order stream,
    // because with many slots the streams outnumber the hardware queues and
    // a cross-stream wait (a barrier packet that blocks its queue) of one
    // slot could sit in front of the work another slot's wait needs.
    bool lookahead = false;
    int fres = 0;
    hipStream_t fmain = nullptr, fside = nullptr;
    hipEvent_t ev_c = nullptr, ev_d = nullptr;
    hipEvent_t ev_j[2] = {nullptr, nullptr};   // reduced eigensolve: stop words read back per sweep
    hipEvent_t ev_s[2] = {nullptr, nullptr};   // forward and adjoint solves on two streams
    hipStream_t aux = nullptr;                 // a mixed solve's complex128 node group (factor)
    hipEvent_t ev_g = nullptr;
    int device = -1;
    int num_cu = 0;

    // Fixed-arena mode (the no-allocation entry point): get() carves the
    // named buffers out of [arena, arena + arena_cap) in request order and
    // pinned() out of a static host block, so neither allocates; the solve
    // runs on the caller's stream with no stream or event of its own.
    bool noalloc = false;
    unsigned char *arena = nullptr, *host_arena = nullptr;
    size_t arena_cap = 0, arena_used = 0, host_cap = 0, host_used = 0;
    static void *carve(std::map<std::string, std::pair<void *, size_t>> &m, const std::string &name, size_t bytes,
                       unsigned char *base, size_t cap, size_t &used)
    {
        auto it = m.find(name);
        if (it != m.end() && it->second.second >= bytes) return it->second.first;
        const size_t off = (used + 255) & ~size_t(255);
        if (off > cap || bytes > cap - off) throw alloc_error{};
        used = off + bytes;
        m[name] = {base + off, bytes};
        return base + off;
    }
    // forget the carved buffers (the start of every no-allocation call)
    void reset_arena()
    {
        dev.clear();
        host.clear();
        arena_used = host_used = 0;
    }

    void *get(const std::string &name, size_t bytes)
    {
        if (noalloc) return carve(dev, name, bytes, arena, arena_cap, arena_used);
        auto &e = dev[name];
        if (e.second < bytes) {
            if (e.first) FX_CHECK(hipFree(e.first));
            e.first = nullptr;
            e.second = 0;
            if (hipMalloc(&e.first, std::max<size_t>(bytes, 256)) != hipSuccess) {
                (void)hipGetLastError();
                e.first = nullptr;
                throw alloc_error{};
            }
            e.second = bytes;
        }
        return e.first;
    }
    void *pinned(const std::string &name, size_t bytes)
    {
        if (noalloc) return carve(host, name, bytes, host_arena, host_cap, host_used);
        auto &e = host[name];
        if (e.second < bytes) {
            if (e.first) FX_CHECK(hipHostFree(e.first));
            e.first = nullptr;
            if (hipHostMalloc(&e.first, std::max<size_t>(bytes, 256), hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                e.first = nullptr;
                throw alloc_error{};
            }
            e.second = bytes;
        }
        return e.first;
    }
    void init()
    {
        if (noalloc || stream) return;
        FX_CHECK(hipGetDevice(&device));
        FX_CHECK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        FX_CHECK(hipEventCreateWithFlags(&ev_a, hipEventDisableTiming));
        FX_CHECK(hipEventCreateWithFlags(&ev_b, hipEventDisableTiming));
        hipDeviceProp_t prop;
        FX_CHECK(hipGetDeviceProperties(&prop, device));
        num_cu = prop.multiProcessorCount;
        FX_CHECK(hipEventCreateWithFlags(&ev_j[0], hipEventDisableTiming));
        FX_CHECK(hipEventCreateWithFlags(&ev_j[1], hipEventDisableTiming));
        FX_CHECK(hipEventCreateWithFlags(&ev_s[0], hipEventDisableTiming));
        FX_CHECK(hipEventCreateWithFlags(&ev_s[1], hipEventDisableTiming));
        FX_CHECK(hipDeviceSynchronize());
    }
    // The side and aux streams are created at first use: only the single-
    // solve path asks for them.  An executor slot then owns one stream, so
    // the slots' streams spread over the device's hardware queues instead
    // of alternating with streams that are never used.
    hipStream_t side_stream()
    {
        if (!side && !noalloc) FX_CHECK(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
        return side;
    }
    hipStream_t aux_stream()
    {
        if (!aux && !noalloc) {
            FX_CHECK(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking));
            FX_CHECK(hipEventCreateWithFlags(&ev_g, hipEventDisableTiming));
        }
        return aux;
    }
    void drop_split()
    {
        if (fmain) (void)hipStreamDestroy(fmain);
        if (fside) (void)hipStreamDestroy(fside);
        if (ev_c) (void)hipEventDestroy(ev_c);
        if (ev_d) (void)hipEventDestroy(ev_d);
        fmain = fside = nullptr;
        ev_c = ev_d = nullptr;
        fres = 0;
    }
    // Streams for a factorisation of `batch` matrices with the CU split, or
    // false when the split is not used.  The panel launch has one workgroup
    // per matrix and workgroups go to the 8 XCDs in turn, so ceil(batch / 8)
    // CUs per XCD are reserved.  Mask bit 33 x + 8 j (x = XCD, j < reserve)
    // lands on XCD x both when the driver interleaves mask bits over the
    // XCDs (bit i -> XCD i mod 8) and when it gives each XCD 32 consecutive
    // bits, so no XCD is ever left without a CU on either stream.
    bool split(int batch)
    {
        static const bool off = std::getenv("FEASTX_NO_CU_SPLIT") != nullptr;   // tuning knob
        if (!want_split || off || num_cu != 256) return false;
        const int r = std::min(4, std::max(1, (batch + 7) / 8));
        if (fres == r) return true;
        drop_split();
        uint32_t pm[8] = {0}, mm[8];
        for (int x = 0; x < 8; ++x)
            for (int j = 0; j < r; ++j) {
                const int b = 33 * x + 8 * j;
                pm[b / 32] |= 1u << (b % 32);
            }
        for (int w = 0; w < 8; ++w) mm[w] = ~pm[w];
        FX_CHECK(hipExtStreamCreateWithCUMask(&fmain, 8, mm));
        FX_CHECK(hipExtStreamCreateWithCUMask(&fside, 8, pm));
        FX_CHECK(hipEventCreateWithFlags(&ev_c, hipEventDisableTiming));
        FX_CHECK(hipEventCreateWithFlags(&ev_d, hipEventDisableTiming));
        fres = r;
        return true;
    }
    double bytes() const
    {
        double b = 0;
        for (auto &kv : dev) b += (double)kv.second.second;
        return b;
    }
    // free the device buffers
    void trim()
    {
        if (noalloc) return;
        for (auto &kv : dev)
            if (kv.second.first) {
                (void)hipFree(kv.second.first);
                kv.second.first = nullptr;
                kv.second.second = 0;
            }
    }
    void release()
    {
        if (noalloc) {
            reset_arena();
            return;
        }
        for (auto &kv : dev)
            if (kv.second.first) (void)hipFree(kv.second.first);
        for (auto &kv : host)
            if (kv.second.first) (void)hipHostFree(kv.second.first);
        dev.clear();
        host.clear();
        if (stream) (void)hipStreamDestroy(stream);
        if (side) (void)hipStreamDestroy(side);
        if (ev_a) (void)hipEventDestroy(ev_a);
        if (ev_b) (void)hipEventDestroy(ev_b);
        for (auto &e : ev_j)
            if (e) (void)hipEventDestroy(e);
        for (auto &e : ev_s)
            if (e) (void)hipEventDestroy(e);
        if (ev_g) (void)hipEventDestroy(ev_g);
        if (aux) (void)hipStreamDestroy(aux);
        drop_split();
        stream = side = aux = nullptr;
        ev_a = ev_b = nullptr;
        ev_j[0] = ev_j[1] = nullptr;
        ev_s[0] = ev_s[1] = nullptr;
        ev_g = nullptr;
    }
};

// One context per host thread for the single-problem entry points: its
// workspace (device buffers, streams) is created at the thread's first call
// and freed by feast_release() from that thread; its statistics are those of
// the thread's last solve.
static thread_local Workspace *t_ws = nullptr;
static thread_local feast_stats t_stats;
static Workspace &thread_ws()
{
    if (!t_ws) t_ws = new Workspace();
    return *t_ws;
}
static std::atomic<bool> g_timing{false};
static const bool g_debug = std::getenv("FEASTX_DEBUG") != nullptr;
static const bool g_no_lookahead = std::getenv("FEASTX_NO_LOOKAHEAD") != nullptr;   // tuning knob
// Node precision from the predicted per-loop contraction eta_j of a
// complex64 node (fp64_nodes).  When no node exceeds ETA_LIMIT every node
// stays complex64: the N = 4096 real pencil with Ne = 8 (largest eta about
// 5e-4) then converges in as many loops as FP64.  When some node does, the
// complex64 nodes left set the contraction per loop, so a part-way promotion
// does not pay: on the N = 8192 Hermitian pencil with Ne = 16, moving the 2
// nodes above 1e-3 or the 5 above 1e-5 to complex128 took 7 and 10 loops,
// while moving the 8 above ETA_FULL took 3, as FP64 does, in less time.  So
// then every node above ETA_FULL goes to complex128.  FEASTX_FP64_ETA sets one
// threshold for every node instead (tuning knob).
constexpr double ETA_LIMIT = 1e-3, ETA_FULL = 1e-6;
static double fp64_eta_env()
{
    const char *e = std::getenv("FEASTX_FP64_ETA");
    return e ? std::atof(e) : -1.0;
}

// ------------------------------------------------------------ contour
// Gauss-Legendre nodes on [-1, 1] by Newton iteration on P_n, evaluated with
// the Bonnet recurrence; weights 2 / ((1 - x^2) P_n'(x)^2).  Ascending.
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    auto legendre = [n](double t, double &p, double &dp) {
        double pm1 = 1.0, pk = t;
        if (n == 1) {
            p = t;
            dp = 1.0;
            return;
        }
        for (int k = 2; k <= n; ++k) {
            const double pk1 = ((2 * k - 1) * t * pk - (k - 1) * pm1) / k;
            pm1 = pk;
            pk = pk1;
        }
        p = pk;
        dp = n * (pm1 - t * pk) / (1.0 - t * t);
    };
    for (int i = 0; i < (n + 1) / 2; ++i) {
        // Tricomi's initial approximation of the i-th largest root
        double t = std::cos(M_PI * (4.0 * i + 3.0) / (4.0 * n + 2.0)) *
                   (1.0 - (n - 1.0) / (8.0 * n * n * n));
        double p = 0, dp = 1;
        for (int it = 0; it < 100; ++it) {
            legendre(t, p, dp);
            const double d = p / dp;
            t -= d;
            if (std::fabs(d) < 1e-17) break;
        }
        legendre(t, p, dp);
        const double wt = 2.0 / ((1.0 - t * t) * dp * dp);
        x[n - 1 - i] = t;
        w[n - 1 - i] = wt;
        x[i] = -t;
        w[i] = wt;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

struct Contour {
    std::vector<double2> z, w;
};

// Half-contour nodes and weights (section "Defining a search contour";
// Table "tab_fpm" fpm(2), fpm(16), fpm(18)).  The contour through Emin and
// Emax is z(t) = c + r cos t + i a r sin t (a = ellipse / 100), and the
// filter is (1 / 2 pi i) times its integral of dz / (z - lambda): over the
// upper half, doubled real part, that is (1 / pi) Re of the integral of
// (a r cos t + i r sin t) / (z(t) - lambda) dt on [0, pi].  The rule on
// [0, pi]: Gauss-Legendre (t = (pi/2)(1 - x), dt = (pi/2) omega) or the
// trapezoidal midpoints t_j = pi (ne - j - 1/2) / ne with dt = pi / ne.
// Nodes come in increasing real part.
static Contour make_contour(double emin, double emax, int ne, int integration = 0, int ellipse = 100)
{
    // th: node parameter; f = dt / pi, written out per rule (omega / 2 for
    // Gauss-Legendre, 1 / ne for the trapezoidal rule) so that the default
    // circle's weights are formed exactly as 0.5 omega r e^{i th}
    std::vector<double> th(ne), f(ne);
    if (integration == 1) {
        for (int j = 0; j < ne; ++j) {
            th[j] = M_PI * (ne - j - 0.5) / ne;
            f[j] = 1.0 / ne;
        }
    } else {
        std::vector<double> x, om;
        gauss_legendre(ne, x, om);
        for (int j = 0; j < ne; ++j) {
            th[j] = 0.5 * M_PI * (1.0 - x[j]);
            f[j] = 0.5 * om[j];
        }
    }
    Contour c;
    c.z.resize(ne);
    c.w.resize(ne);
    const double mid = 0.5 * (emin + emax), r = 0.5 * (emax - emin), a = ellipse / 100.0;
    for (int j = 0; j < ne; ++j) {
        const double ct = std::cos(th[j]), st = std::sin(th[j]);
        c.z[j] = make_double2(mid + r * ct, a * r * st);
        c.w[j] = make_double2(f[j] * a * r * ct, f[j] * r * st);
    }
    return c;
}

// Caller-supplied nodes and weights (the guide's expert mode, Zne / Wne).
static Contour custom_contour(const feast_z *zne, const feast_z *wne, int ne)
{
    Contour c;
    c.z.resize(ne);
    c.w.resize(ne);
    for (int j = 0; j < ne; ++j) {
        c.z[j] = make_double2(zne[j].re, zne[j].im);
        c.w[j] = make_double2(wne[j].re, wne[j].im);
    }
    return c;
}

// ------------------------------------------------------------ timing
struct StageTimer {
    hipStream_t s;
    bool on;   // off: no events at all (the no-allocation entry point)
    std::vector<std::pair<hipEvent_t, double *>> marks;
    hipEvent_t last = nullptr;
    StageTimer(hipStream_t st, bool enabled) : s(st), on(enabled) {}
    void start()
    {
        if (!on) return;
        FX_CHECK(hipEventCreate(&last));
        FX_CHECK(hipEventRecord(last, s));
        marks.push_back({last, nullptr});
    }
    void mark(double *acc)
    {
        if (!on) return;
        hipEvent_t e;
        FX_CHECK(hipEventCreate(&e));
        FX_CHECK(hipEventRecord(e, s));
        marks.push_back({e, acc});
    }
    void flush()
    {
        if (marks.empty()) return;
        FX_CHECK(hipEventSynchronize(marks.back().first));
        for (size_t i = 1; i < marks.size(); ++i) {
            float ms = 0.f;
            FX_CHECK(hipEventElapsedTime(&ms, marks[i - 1].first, marks[i].first));
            if (marks[i].second) *marks[i].second += ms;
        }
        for (auto &m : marks) (void)hipEventDestroy(m.first);
        marks.clear();
        start();
    }
    ~StageTimer()
    {
        for (auto &m : marks) (void)hipEventDestroy(m.first);
    }
};

// Per-launch timing of the complex products in the factor precision of the
// solve (complex64 for mixed, complex128 for FP64; enabled by
// feast_set_timing); those issued by the shifted LU itself are also summed
// apart.
struct GemmTimer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    std::vector<char> in_lu;
    double flops = 0, lu_flops = 0;
    bool lu = false;    // launches being recorded belong to getrf_batched
    bool f64 = false;   // record the complex128 products (else complex64)
};
static thread_local GemmTimer *g_gemm_timer = nullptr;
void gemm_timing_reset();

// ------------------------------------------------------------ problem
struct Problem {
    int n;
    const double *A;
    long lda;
    const double *B;
    long ldb;
    double emin, emax;
    int m0;
    double *X;   // caller's device array
    long ldx;
};

struct Result {
    int M = 0, loop = 0, m0 = 0;
    double epsout = 1.0;
    std::vector<double> E, res;
};

template <bool CPLX> using F64 = typename jelem<CPLX>::type;

// C = alpha (P_0 + P_1 + ... + P_{S-1}) + beta C, partials m x n contiguous,
// summed in index order.
template <bool CPLX>
__global__ __launch_bounds__(256) void splitk_sum_kernel(int m, long mn, int S, const F64<CPLX> *__restrict__ P,
                                                         double alpha, double beta, F64<CPLX> *__restrict__ C,
                                                         long ldc)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= mn) return;
    const long i = e % m, j = e / m;
    if constexpr (CPLX) {
        double2 acc = P[e];
        for (int q = 1; q < S; ++q) {
            const double2 v = P[(long)q * mn + e];
            acc.x += v.x;
            acc.y += v.y;
        }
        double2 out = make_double2(alpha * acc.x, alpha * acc.y);
        if (beta != 0.0) {
            const double2 c = C[i + j * ldc];
            out.x += beta * c.x;
            out.y += beta * c.y;
        }
        C[i + j * ldc] = out;
    } else {
        double acc = P[e];
        for (int q = 1; q < S; ++q) acc += P[(long)q * mn + e];
        double out = alpha * acc;
        if (beta != 0.0) out += beta * C[i + j * ldc];
        C[i + j * ldc] = out;
    }
}

template <bool CPLX>
static void dgemm(Workspace &ws, hipStream_t s, bool opa_h, int m, int n, int k, double alpha, const F64<CPLX> *A,
                  long lda, const F64<CPLX> *B, long ldb, double beta, F64<CPLX> *C, long ldc)
{
    using E = F64<CPLX>;
    // Few output tiles and a long K (Rayleigh-Ritz: N x M0 x N and
    // M0 x M0 x N): split K over S partial products in workspace, summed in
    // a fixed order, so the result does not depend on scheduling.
    const long tiles = (long)ceil_div(m, 64) * ceil_div(n, 64);
    int S = 1;
    if (tiles < 512 && k >= 512) {
        S = 16;
        while (S > 1 && (k % S != 0 || k / S < 256 || tiles * S > 2048)) S /= 2;
    }
    if (S == 1) {
        if (opa_h) gemm<double, CPLX, true>(s, m, n, k, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1);
        else gemm<double, CPLX, false>(s, m, n, k, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1);
        return;
    }
    const int kc = k / S;
    const long mn = (long)m * n;
    E *P = static_cast<E *>(ws.get("splitk", sizeof(E) * (size_t)S * mn));
    if (opa_h)   // A is stored K x M: chunk s starts at row s kc
        gemm2<double, CPLX, true>(s, m, n, kc, 1.0, A, lda, 0, kc, B, ldb, 0, kc, 0.0, P, m, 0, mn, 1, S);
    else         // A is stored M x K: chunk s starts at column s kc
        gemm2<double, CPLX, false>(s, m, n, kc, 1.0, A, lda, 0, (long)kc * lda, B, ldb, 0, kc, 0.0, P, m, 0, mn, 1,
                                   S);
    hipLaunchKernelGGL((splitk_sum_kernel<CPLX>), dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, m, mn, S, P,
                       alpha, beta, C, ldc);
    FX_LAUNCH_CHECK();
}

static dim3 grid1(long count) { return dim3((unsigned)((count + 255) / 256)); }

// Reduced Hermitian eigenproblem on the device: C (m x m, overwritten) ->
// ascending eigenvalues w (device) and eigenvectors Vout (m x m).  One
// launch per Jacobi round on stream s; the host reads each sweep's stopping
// decision back while the next sweep is already queued behind it (a stopped
// iteration's queued launches return at once).
template <bool CPLX>
static void device_eigh(Workspace &ws, hipStream_t s, int m, F64<CPLX> *C, F64<CPLX> *Vout, double *w,
                        feast_stats &st, double tol = 1e-13)
{
    using E = F64<CPLX>;
    E *V = static_cast<E *>(ws.get("jac_v", sizeof(E) * (size_t)m * m));
    E *C1 = static_cast<E *>(ws.get("jac_c1", sizeof(E) * (size_t)m * m));
    const int nb = (m + BJ_BS - 1) / BJ_BS, nbp = nb + (nb & 1), npairs = nbp / 2, rounds = nbp - 1;
    E *Rbuf = static_cast<E *>(ws.get("jac_r", sizeof(E) * 2 * (size_t)npairs * BJ_W * BJ_W));
    E *Dbuf = static_cast<E *>(ws.get("jac_d", sizeof(E) * (size_t)nbp * BJ_BS * BJ_BS));
    double *dout = static_cast<double *>(ws.get("jac_diag", sizeof(double) * m));
    const int nrc = (m + BJ_W - 1) / BJ_W;
    const int nitems = npairs * (npairs + 1) / 2 + nrc * npairs;
    const int g_init = std::min(ceil_div((long)m * m, BJ_NT), 256);
    double *partial = static_cast<double *>(ws.get("jac_partial", sizeof(double) * (size_t)std::max(nitems, g_init)));
    jac_state *jst = static_cast<jac_state *>(ws.get("jac_state", sizeof(jac_state)));
    int *status = static_cast<int *>(ws.get("jac_status", sizeof(int) * 2));
    double *hist = static_cast<double *>(ws.get("jac_hist", sizeof(double) * 64));
    int *rank = static_cast<int *>(ws.get("jac_rank", sizeof(int) * m));
    constexpr int max_sweeps = 40;
    int *h_stop = static_cast<int *>(ws.pinned("jac_stop_h", sizeof(int) * (max_sweeps + 1)));
    const long ld = m;
    hipLaunchKernelGGL(jacobi_reset_kernel, dim3(1), dim3(1), 0, s, jst);
    hipLaunchKernelGGL((jacobi_init_kernel<CPLX>), dim3(g_init), dim3(BJ_NT), 0, s, m, C, ld, V, ld, partial, jst);
    FX_LAUNCH_CHECK();
    int t = 0;
    for (int sw = 1; sw <= max_sweeps; ++sw) {
        // rounds up to the launch that forms the matrix after sweep sw and decides
        for (; t <= rounds * sw; ++t) {
            const unsigned g = (unsigned)(npairs + (t > 0 ? nitems : 0));
            hipLaunchKernelGGL((bjacobi_round_kernel<CPLX>), dim3(g), dim3(BJ_NT), 0, s, t, m, C, C1, ld, V, ld, Rbuf,
                               Dbuf, partial, jst, max_sweeps, tol, hist);
        }
        FX_LAUNCH_CHECK();
        FX_CHECK(hipMemcpyAsync(h_stop + sw, &jst->stop, sizeof(int), hipMemcpyDeviceToHost, s));
        if (!ws.ev_j[0]) {
            // no events (the no-allocation entry point): read each decision at once
            FX_CHECK(hipStreamSynchronize(s));
            if (h_stop[sw]) break;
            continue;
        }
        FX_CHECK(hipEventRecord(ws.ev_j[sw & 1], s));
        if (sw >= 2) {
            FX_CHECK(hipEventSynchronize(ws.ev_j[(sw - 1) & 1]));
            if (h_stop[sw - 1]) break;
        }
    }
    hipLaunchKernelGGL((jacobi_final_kernel<CPLX>), dim3(ceil_div(m, 256)), dim3(256), 0, s, m, C, C1, ld, jst, dout,
                       status);
    hipLaunchKernelGGL((jacobi_sort_kernel<CPLX>), dim3(1), dim3(1024), 0, s, m, dout, V, ld, w, Vout, ld, rank);
    FX_LAUNCH_CHECK();
    int *hst = static_cast<int *>(ws.pinned("jac_status_h", sizeof(int) * 2));
    FX_CHECK(hipMemcpyAsync(hst, status, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
    FX_CHECK(hipStreamSynchronize(s));
    st.eig_calls += 1;
    st.eig_sweeps += hst[1];
    if (g_debug) {
        double hh[64];
        FX_CHECK(hipMemcpy(hh, hist, sizeof(double) * std::min(hst[1], 64), hipMemcpyDeviceToHost));
        std::fprintf(stderr, "feastx eigh n=%d rounds=%d launches=%d sweeps=%d off/fro:", m, rounds, t, hst[1]);
        for (int i = 0; i < std::min(hst[1], 40); ++i) std::fprintf(stderr, " %.1e", hh[i]);
        std::fprintf(stderr, "\n");
    }
    if (hst[0] != 0) throw solver_error{-3};
}

constexpr double SPURIOUS_RES = 0.1;   // in-interval Ritz pairs above this residual are spurious
constexpr double TRUNC = 1e-14;        // Bq eigen-directions below TRUNC * max are dropped
constexpr double INDEFINITE = 1e-8;    // Bq eigenvalue below -INDEFINITE * max: B not definite
constexpr double CHOL_DROP = 1e-12;    // scaled Cholesky pivots at or below this are dependent columns

// B-orthonormal basis by diagonal scaling and Cholesky with column dropping
// (columns visited in order of decreasing B-norm).  Returns the rank kept;
// Tm (m x rank) receives T.  Returns -1 when a pivot comes out below
// -INDEFINITE: visiting columns in a fixed order does not reveal rank, so a
// nearly dependent column kept just above the drop threshold can amplify
// rounding in the later pivots (seen with complex64 solves, whose noise puts
// such columns near the threshold).  The caller then takes the
// eigendecomposition, which decides definiteness from Bq's eigenvalues.
template <bool CPLX>
static int bortho_cholesky(Workspace &ws, hipStream_t s, int m, F64<CPLX> *Bq, F64<CPLX> *Tm)
{
    using E = F64<CPLX>;
    const size_t mm = (size_t)m * m;
    double *d = static_cast<double *>(ws.get("bo_d", sizeof(double) * m));
    int *status = static_cast<int *>(ws.get("bo_status", sizeof(int) * 4));
    int *ord = static_cast<int *>(ws.get("bo_ord", sizeof(int) * m));
    int *row_of = static_cast<int *>(ws.get("bo_rowof", sizeof(int) * m));
    int *kidx = static_cast<int *>(ws.get("bo_kidx", sizeof(int) * m));
    int *keepf = static_cast<int *>(ws.get("bo_keep", sizeof(int) * m));
    E *Bt = static_cast<E *>(ws.get("bo_bt", sizeof(E) * mm));
    E *Pc = static_cast<E *>(ws.get("bo_p", sizeof(E) * (size_t)CHP_NB * m));
    E *Lk = static_cast<E *>(ws.get("bo_lk", sizeof(E) * mm));
    E *Ti = static_cast<E *>(ws.get("bo_ti", sizeof(E) * mm));
    E *Xi = static_cast<E *>(ws.get("bo_xi", sizeof(E) * mm));
    const int nblk = ceil_div(m, TRI_NB);
    E *Dinv = static_cast<E *>(ws.get("bo_dinv", sizeof(E) * (size_t)nblk * TRI_NB * TRI_NB));
    double *h_d = static_cast<double *>(ws.pinned("bo_hd", sizeof(double) * m));
    int *h_i = static_cast<int *>(ws.pinned("bo_hi", sizeof(int) * (4 + 3 * (size_t)m)));

    FX_CHECK(hipMemsetAsync(status, 0, sizeof(int) * 4, s));
    hipLaunchKernelGGL((diag_rsqrt_kernel<CPLX>), dim3(ceil_div(m, 256)), dim3(256), 0, s, m, Bq, (long)m, d, status);
    FX_LAUNCH_CHECK();
    FX_CHECK(hipMemcpyAsync(h_d, d, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    FX_CHECK(hipMemcpyAsync(h_i, status, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
    FX_CHECK(hipStreamSynchronize(s));
    if (h_i[0] != 0) throw solver_error{-3};
    // visit columns by decreasing B-norm (increasing d), ties by index
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return h_d[a] < h_d[b]; });
    FX_CHECK(hipMemcpyAsync(ord, order.data(), sizeof(int) * m, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL((sym_scale_kernel<CPLX>), grid1((long)mm), dim3(256), 0, s, m, Bq, (long)m, d, ord, Bt, (long)m);
    FX_LAUNCH_CHECK();
    // blocked Cholesky in place on Bt: afterwards Bt's lower triangle is L
    chol_drop_blocked<CPLX>(s, m, Bt, (long)m, Pc, keepf, CHOL_DROP, INDEFINITE, status);
    FX_CHECK(hipMemcpyAsync(h_i, status, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
    FX_CHECK(hipMemcpyAsync(h_i + 4, keepf, sizeof(int) * m, hipMemcpyDeviceToHost, s));
    FX_CHECK(hipStreamSynchronize(s));
    if (h_i[0] != 0) return -1;
    const int r = h_i[1];
    if (r < 1) throw solver_error{-3};
    // kept positions in Cholesky order -> original indices
    int *h_kidx = h_i + 4 + m, *h_rowof = h_i + 4 + 2 * (size_t)m;
    for (int i = 0; i < m; ++i) h_rowof[i] = -1;
    int c = 0;
    for (int a = 0; a < m; ++a)
        if (h_i[4 + a]) {
            h_kidx[c] = a;
            h_rowof[order[a]] = c;
            ++c;
        }
    FX_CHECK(hipMemcpyAsync(kidx, h_kidx, sizeof(int) * r, hipMemcpyHostToDevice, s));
    FX_CHECK(hipMemcpyAsync(row_of, h_rowof, sizeof(int) * m, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL((gather_kk_kernel<CPLX>), grid1((long)r * r), dim3(256), 0, s, r, kidx, Bt, (long)m, Lk,
                       (long)r);
    hipLaunchKernelGGL((lower_block_inv_kernel<CPLX>), dim3(ceil_div(r, TRI_NB)), dim3(TRI_NT), 0, s, r, Lk, (long)r,
                       Dinv);
    hipLaunchKernelGGL((set_identity_kernel<CPLX>), grid1((long)r * r), dim3(256), 0, s, r, Xi, (long)r);
    FX_LAUNCH_CHECK();
    lower_inv_h<CPLX>(s, r, Lk, r, Dinv, Ti, Xi, r);
    hipLaunchKernelGGL((scatter_scale_rows_kernel<CPLX>), grid1((long)m * r), dim3(256), 0, s, m, r, d, Ti, (long)r,
                       Tm, (long)m, row_of);
    FX_LAUNCH_CHECK();
    FX_CHECK(hipStreamSynchronize(s));   // host order/index vectors go out of scope
    return r;
}

// B-orthonormal basis from the eigendecomposition Bq = W diag(beta) W^H,
// dropping directions with beta <= TRUNC * max (for subspaces beyond the
// one-workgroup Cholesky).  Tm = W_keep beta^{-1/2}.
template <bool CPLX>
static int bortho_eigen(Workspace &ws, hipStream_t s, int m0, F64<CPLX> *Bq, F64<CPLX> *Wb, double *beta,
                        F64<CPLX> *Tm, feast_stats &st)
{
    double *h_beta = static_cast<double *>(ws.pinned("h_beta", sizeof(double) * m0));
    device_eigh<CPLX>(ws, s, m0, Bq, Wb, beta, st);
    FX_CHECK(hipMemcpyAsync(h_beta, beta, sizeof(double) * m0, hipMemcpyDeviceToHost, s));
    FX_CHECK(hipStreamSynchronize(s));
    const double bmax = h_beta[m0 - 1];
    if (!(bmax > 0.0) || h_beta[0] < -INDEFINITE * bmax) throw solver_error{-3};
    int keep = 0;
    for (int i = 0; i < m0; ++i)
        if (h_beta[i] > TRUNC * bmax) ++keep;
    const int first = m0 - keep;
    hipLaunchKernelGGL((scale_cols_kernel<CPLX>), grid1((long)m0 * keep), dim3(256), 0, s, m0, keep, first, Wb,
                       (long)m0, beta, Tm, (long)m0);
    FX_LAUNCH_CHECK();
    return keep;
}


// ---------------------------------------------------------------- node groups
// The shifted matrices of a set of contour nodes in one factor precision
// (complex<T>), with their solve form W, the inverted diagonal blocks and
// the solve panels.  An FP64 solve has one group of all nodes.  A mixed
// solve has a complex64 group and, for the nodes where complex64 error would
// limit the outer iteration (fp64_nodes), a complex128 group.
template <typename T, bool CPLX> struct NodeGroup {
    using V = cplx<T>;
    int n = 0, ne = 0;
    std::vector<int> nodes;   // contour indices, in quadrature order
    long ldf = 0, sF = 0, sI64 = 0, sInv = 0, sItmp = 0;
    double2 *dz = nullptr;
    V *F = nullptr, *L64 = nullptr, *U64 = nullptr, *Itmp = nullptr, *Wsv = nullptr, *Linv = nullptr,
      *Uinv = nullptr, *Ytmp = nullptr, *Ytmp2 = nullptr, *Y = nullptr, *Yh = nullptr, *Yh2 = nullptr;
    int *ipiv = nullptr, *perm = nullptr, *swapmap = nullptr, *dinfo = nullptr, *h_info = nullptr;

    // buffers named with `tag` (distinct per group), the group's nodes uploaded on s
    void setup(Workspace &ws, hipStream_t s, const std::string &tag, int n_, const std::vector<int> &nodes_,
               const Contour &ct, size_t nm)
    {
        n = n_;
        nodes = nodes_;
        ne = (int)nodes.size();
        if (ne == 0) return;
        const std::string p = std::string(sizeof(T) == 4 ? "32" : "64") + tag;
        ldf = n;
        sF = (long)n * n;
        std::vector<double2> zg(ne);
        for (int j = 0; j < ne; ++j) zg[j] = ct.z[nodes[j]];
        dz = static_cast<double2 *>(ws.get("z" + p, sizeof(double2) * ne));
        FX_CHECK(hipMemcpyAsync(dz, zg.data(), sizeof(double2) * ne, hipMemcpyHostToDevice, s));
        FX_CHECK(hipStreamSynchronize(s));   // zg goes out of scope
        F = static_cast<V *>(ws.get("F" + p, sizeof(V) * (size_t)ne * sF));
        ipiv = static_cast<int *>(ws.get("ipiv" + p, sizeof(int) * (size_t)ne * n));
        perm = static_cast<int *>(ws.get("perm" + p, sizeof(int) * (size_t)ne * n));
        swapmap = static_cast<int *>(ws.get("swapmap" + p, sizeof(int) * LU_LISTS * (size_t)ne * LU_LIST_INTS));
        dinfo = static_cast<int *>(ws.get("info" + p, sizeof(int) * ne));
        const bool compose = solve_nb<T>() > TRI_INV_NB;   // 128-row solve blocks from 64-row inverses
        sI64 = compose ? tri_inv_stride(n) : 0;
        sInv = solve_inv_stride<T>(n);
        sItmp = compose ? (long)ceil_div(n, solve_nb<T>()) * 64 * 64 : 0;
        L64 = compose ? static_cast<V *>(ws.get("L64inv" + p, sizeof(V) * (size_t)ne * sI64)) : nullptr;
        U64 = compose ? static_cast<V *>(ws.get("U64inv" + p, sizeof(V) * (size_t)ne * sI64)) : nullptr;
        Itmp = compose ? static_cast<V *>(ws.get("Invtmp" + p, sizeof(V) * (size_t)ne * sItmp)) : nullptr;
        Wsv = static_cast<V *>(ws.get("Wsolve" + p, sizeof(V) * (size_t)ne * sF));
        Linv = static_cast<V *>(ws.get("Linv" + p, sizeof(V) * (size_t)ne * sInv));
        Uinv = static_cast<V *>(ws.get("Uinv" + p, sizeof(V) * (size_t)ne * sInv));
        Ytmp = static_cast<V *>(ws.get("Yt" + p, sizeof(V) * (size_t)ne * nm));
        Y = static_cast<V *>(ws.get("Y" + p, sizeof(V) * (size_t)ne * nm));
        if (CPLX) {
            Yh = static_cast<V *>(ws.get("Yh" + p, sizeof(V) * (size_t)ne * nm));
            Yh2 = static_cast<V *>(ws.get("Yg" + p, sizeof(V) * (size_t)ne * nm));
            // the adjoint solves' own scratch when they run beside the forward ones
            if (two_streams(ws)) Ytmp2 = static_cast<V *>(ws.get("Yt2" + p, sizeof(V) * (size_t)ne * nm));
        }
        h_info = static_cast<int *>(ws.pinned("h_info" + p, sizeof(int) * ne));
    }

    // shift, LU with partial pivoting, inverted diagonal blocks and W; throws
    // solver_error{-2} on a zero or non-finite pivot
    void factor(Workspace &ws, hipStream_t s, const Problem &pb, feast_stats &st)
    {
        factor_launch(ws, s, pb, true);
        factor_wait(s, st);
    }

    // the factorisation's launches on s (look-ahead on the workspace's
    // streams when `lookahead_ok`; else everything on s), no host wait
    void factor_launch(Workspace &ws, hipStream_t s, const Problem &pb, bool lookahead_ok)
    {
        if (ne == 0) return;
        shift_build<T>(s, CPLX, n, pb.A, pb.lda, pb.B, pb.ldb, dz, ne, F, ldf, sF);
        FX_CHECK(hipMemsetAsync(dinfo, 0, sizeof(int) * ne, s));
        if (g_gemm_timer) g_gemm_timer->lu = true;
        const bool la = lookahead_ok && !g_no_lookahead && ws.lookahead;
        if (la && ws.split(ne)) {
            FX_CHECK(hipEventRecord(ws.ev_c, s));
            FX_CHECK(hipStreamWaitEvent(ws.fmain, ws.ev_c, 0));
            getrf_batched<T>(ws.fmain, ws.fside, ws.ev_a, ws.ev_b, n, F, ldf, sF, ipiv, perm, n, swapmap, dinfo,
                             ne);
            FX_CHECK(hipEventRecord(ws.ev_d, ws.fmain));
            FX_CHECK(hipStreamWaitEvent(s, ws.ev_d, 0));
        } else {
            getrf_batched<T>(s, la ? ws.side_stream() : nullptr, ws.ev_a, ws.ev_b, n, F, ldf, sF, ipiv, perm, n,
                             swapmap, dinfo, ne);
        }
        if (g_gemm_timer) g_gemm_timer->lu = false;
        solve_inverses<T>(s, n, F, ldf, sF, L64, U64, sI64, Linv, Uinv, sInv, Itmp, sItmp, ne);
        build_w<T>(s, n, F, ldf, sF, Linv, Uinv, sInv, Wsv, ne);
        FX_CHECK(hipMemcpyAsync(h_info, dinfo, sizeof(int) * ne, hipMemcpyDeviceToHost, s));
    }

    // wait for the factorisation issued on s; zero or non-finite pivot: -2
    void factor_wait(hipStream_t s, feast_stats &st)
    {
        if (ne == 0) return;
        FX_CHECK(hipStreamSynchronize(s));
        for (int j = 0; j < ne; ++j)
            if (h_info[j] != 0) throw solver_error{-2};
        st.factor_flops += ne * (8.0 / 3.0) * (double)n * n * n;
    }

    // Y_j = A_zj^{-1} R for the group's nodes; for Hermitian pencils also
    // Yh2_j = A_zj^{-H} R (the same factors)
    // Forward and adjoint solves of a Hermitian pencil are independent (same
    // factors, separate outputs): in the single-solve path the adjoint ones
    // run on the side stream with their own scratch, so that each chain's
    // small in-group products fill the other's gaps.  Executor slots keep
    // one in-order stream; per-launch timing keeps them in order too, so
    // that each launch's events time that launch alone.
    static bool two_streams(const Workspace &ws)
    {
        const bool off = std::getenv("FEASTX_SERIAL_SOLVES") != nullptr;   // measurement knob
        return CPLX && !off && ws.lookahead && !ws.noalloc;
    }

    void solve(Workspace &ws, hipStream_t s, const double *R, int m0, feast_stats &st)
    {
        if (ne == 0) return;
        const size_t cur_nm = (size_t)n * m0;
        dim3 g((unsigned)((cur_nm + 255) / 256), ne);
        const bool two = two_streams(ws) && Ytmp2 && !g_gemm_timer;
        hipStream_t sa = two ? ws.side_stream() : s;
        if (two) {
            FX_CHECK(hipEventRecord(ws.ev_s[0], s));
            FX_CHECK(hipStreamWaitEvent(sa, ws.ev_s[0], 0));
        }
        if (CPLX) {
            hipLaunchKernelGGL((copy_rhs_kernel<T, CPLX>), g, dim3(256), 0, sa, n, m0, R, (long)n, Yh, (long)n,
                               (long)cur_nm);
            FX_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL((gather_rows_kernel<T, CPLX>), g, dim3(256), 0, s, n, m0, perm, (long)n, R, (long)n, Y,
                           (long)n, (long)cur_nm);
        FX_LAUNCH_CHECK();
        if (CPLX && two) {
            // the adjoint chain is queued on the side stream first, then the
            // forward chain on s; the two queues run at once
            getrs_batched<T>(sa, true, n, m0, F, Wsv, ldf, sF, Linv, Uinv, sInv, Yh, Ytmp2, n, (long)cur_nm, ne);
            getrs_batched<T>(s, false, n, m0, F, Wsv, ldf, sF, Linv, Uinv, sInv, Y, Ytmp, n, (long)cur_nm, ne);
        } else {
            getrs_batched<T>(s, false, n, m0, F, Wsv, ldf, sF, Linv, Uinv, sInv, Y, Ytmp, n, (long)cur_nm, ne);
            if (CPLX)
                getrs_batched<T>(s, true, n, m0, F, Wsv, ldf, sF, Linv, Uinv, sInv, Yh, Ytmp, n, (long)cur_nm, ne);
        }
        if (CPLX) {
            hipLaunchKernelGGL((scatter_rows_kernel<T>), g, dim3(256), 0, sa, n, m0, perm, (long)n, Yh, (long)n,
                               (long)cur_nm, Yh2, (long)n, (long)cur_nm);
            FX_LAUNCH_CHECK();
        }
        if (two) {
            FX_CHECK(hipEventRecord(ws.ev_s[1], sa));
            FX_CHECK(hipStreamWaitEvent(s, ws.ev_s[1], 0));
        }
        st.solve_flops += (CPLX ? 2.0 : 1.0) * ne * 8.0 * (double)n * n * m0;
    }
};

// Contour nodes of a mixed-precision solve that are factored and solved in
// complex128.  In the correction form, the complex64 backward error E_j of
// the factors of z_j B - A (about u32 ||A_z||, u32 = 2^-24) reaches the next
// subspace through w_j / (z_j - lambda) times (z_j B - A)^{-1} E_j (z_j B -
// A)^{-1} R; for an unwanted direction near z_j each inverse amplifies by up
// to 1 / Im(z_j) and R's components by up to (Emax - Emin) / Im(z_j), so the
// unwanted components shrink each loop only by about
//   eta_j = u32 (sA / sB + |z_j|) |w_j| (Emax - Emin) / Im(z_j)^3,
// with sA, sB = ||A||_F, ||B||_F over sqrt(N) (scales of A and B).  Nodes
// with eta_j above `eta_max` go to complex128; the others stay complex64.
static std::vector<int> fp64_nodes(const Contour &ct, double sA, double sB, double emin, double emax,
                                   double eta_max)
{
    std::vector<int> hi;
    const double u32 = 5.9604644775390625e-08;
    for (int j = 0; j < (int)ct.z.size(); ++j) {
        const double im = std::fabs(ct.z[j].y);
        const double zabs = std::hypot(ct.z[j].x, ct.z[j].y), wabs = std::hypot(ct.w[j].x, ct.w[j].y);
        const double eta = im > 0 ? u32 * (sA / sB + zabs) * wabs * (emax - emin) / (im * im * im) : 1e300;
        if (eta > eta_max) hi.push_back(j);
    }
    return hi;
}

template <typename T, bool CPLX>
static int run(const Problem &pb, const feast_opts &o, hipStream_t s, Workspace &ws, Result &out,
               feast_stats &st_out)
{
    using E = F64<CPLX>;
    using V = cplx<T>;
    const int n = pb.n, ne = o.ne;
    int m0 = pb.m0;
    const double alpha = std::max(std::fabs(pb.emin), std::fabs(pb.emax));
    const bool mixed = std::is_same<T, float>::value;
    const size_t nm = (size_t)n * m0, mm = (size_t)m0 * m0;
    feast_stats st{};
    StageTimer tm(s, !ws.noalloc);
    tm.start();

    Contour ct = o.Zne ? custom_contour(o.Zne, o.Wne, ne)
                       : make_contour(pb.emin, pb.emax, ne, o.integration, o.ellipse);

    E *X = static_cast<E *>(ws.get("X", sizeof(E) * nm));
    E *R = static_cast<E *>(ws.get("R", sizeof(E) * nm));
    E *Q = static_cast<E *>(ws.get("Q", sizeof(E) * nm));
    E *AQ = static_cast<E *>(ws.get("AQ", sizeof(E) * nm));
    E *BQ = static_cast<E *>(ws.get("BQ", sizeof(E) * nm));
    E *AX = static_cast<E *>(ws.get("AX", sizeof(E) * nm));
    E *BX = static_cast<E *>(ws.get("BX", sizeof(E) * nm));
    E *Aq = static_cast<E *>(ws.get("Aq", sizeof(E) * mm));
    E *Bq = static_cast<E *>(ws.get("Bq", sizeof(E) * mm));
    E *Wb = static_cast<E *>(ws.get("Wb", sizeof(E) * mm));
    E *Tm = static_cast<E *>(ws.get("Tm", sizeof(E) * mm));
    E *Tmp = static_cast<E *>(ws.get("Tmp", sizeof(E) * mm));
    E *Cr = static_cast<E *>(ws.get("Cr", sizeof(E) * mm));
    E *Vc = static_cast<E *>(ws.get("Vc", sizeof(E) * mm));
    E *Phi = static_cast<E *>(ws.get("Phi", sizeof(E) * mm));
    double *beta = static_cast<double *>(ws.get("beta", sizeof(double) * m0));
    double *lam = static_cast<double *>(ws.get("lam", sizeof(double) * m0));
    double *res = static_cast<double *>(ws.get("res", sizeof(double) * m0));
    double *rho = static_cast<double *>(ws.get("rho", sizeof(double) * m0));
    double2 *coef = static_cast<double2 *>(ws.get("coef", sizeof(double2) * ne * m0));
    int *sel = static_cast<int *>(ws.get("sel", sizeof(int) * m0));
    // the contour's nodes in the factor precision T, except (mixed) those
    // whose complex64 error would limit the outer iteration, in complex128
    std::vector<int> lo_nodes, hi_nodes;
    if (mixed && o.mode == 0) {
        double *part = static_cast<double *>(ws.get("sumsq", sizeof(double) * 2 * SUMSQ_BLOCKS));
        double *h_part = static_cast<double *>(ws.pinned("h_sumsq", sizeof(double) * 2 * SUMSQ_BLOCKS));
        hipLaunchKernelGGL((sumsq_kernel<CPLX>), dim3(SUMSQ_BLOCKS), dim3(256), 0, s, n, pb.A, pb.lda, part);
        if (pb.B)
            hipLaunchKernelGGL((sumsq_kernel<CPLX>), dim3(SUMSQ_BLOCKS), dim3(256), 0, s, n, pb.B, pb.ldb,
                               part + SUMSQ_BLOCKS);
        FX_LAUNCH_CHECK();
        FX_CHECK(hipMemcpyAsync(h_part, part, sizeof(double) * (pb.B ? 2 : 1) * SUMSQ_BLOCKS, hipMemcpyDeviceToHost,
                                s));
        FX_CHECK(hipStreamSynchronize(s));
        double a2 = 0.0, b2 = 0.0;
        for (int q = 0; q < SUMSQ_BLOCKS; ++q) {
            a2 += h_part[q];
            if (pb.B) b2 += h_part[SUMSQ_BLOCKS + q];
        }
        const double sA = std::sqrt(a2 / n), sB = pb.B ? std::sqrt(b2 / n) : 1.0;
        const double sBn = sB > 0 ? sB : 1.0, eta_env = fp64_eta_env();
        if (eta_env >= 0.0) {
            hi_nodes = fp64_nodes(ct, sA, sBn, pb.emin, pb.emax, eta_env);
        } else {
            hi_nodes = fp64_nodes(ct, sA, sBn, pb.emin, pb.emax, ETA_LIMIT);
            if (!hi_nodes.empty()) hi_nodes = fp64_nodes(ct, sA, sBn, pb.emin, pb.emax, ETA_FULL);
        }
        if (o.verbose) {
            std::fprintf(stderr, "feastx: ||A||_F/sqrt(N) %.3e ||B||_F/sqrt(N) %.3e, complex128 nodes:", sA, sB);
            for (int j : hi_nodes) std::fprintf(stderr, " %d", j);
            std::fprintf(stderr, "\n");
        }
    }
    for (int j = 0; j < ne; ++j)
        if (std::find(hi_nodes.begin(), hi_nodes.end(), j) == hi_nodes.end()) lo_nodes.push_back(j);
    NodeGroup<T, CPLX> G0;
    NodeGroup<double, CPLX> G1;
    G0.setup(ws, s, "", n, lo_nodes, ct, nm);
    G1.setup(ws, s, "h", n, hi_nodes, ct, nm);
    st.fp64_nodes = mixed ? (int)hi_nodes.size() : 0;
    // per-launch timing follows the products that take most of the solve's
    // time: in a mixed solve with at least half of its nodes in complex128,
    // those nodes' products (at half the complex64 rate) do
    if (g_gemm_timer && mixed && 2 * (int)hi_nodes.size() >= ne) g_gemm_timer->f64 = true;
    double2 *coef1 = hi_nodes.empty() ? nullptr
                                      : static_cast<double2 *>(ws.get("coef_h", sizeof(double2) * hi_nodes.size() * m0));
    double *h_beta = static_cast<double *>(ws.pinned("h_beta", sizeof(double) * m0));
    double *h_lam = static_cast<double *>(ws.pinned("h_lam", sizeof(double) * m0));
    double *h_res = static_cast<double *>(ws.pinned("h_res", sizeof(double) * m0));

    // start subspace
    if (o.x0) {
        hipLaunchKernelGGL((copy_block_kernel<CPLX>), grid1(nm), dim3(256), 0, s, n, m0,
                           reinterpret_cast<const E *>(pb.X), pb.ldx, X, (long)n);
    } else {
        hipLaunchKernelGGL((random_start_kernel<CPLX>), grid1(nm), dim3(256), 0, s, n, m0, o.seed,
                           o.mode == 2 ? 1 : 0, X, (long)n);
    }
    FX_LAUNCH_CHECK();
    tm.mark(&st.t_shift);

    const bool use_corr = mixed && o.refine == 0;
    // A mixed solve whose complex128 group is small factors it on the aux
    // stream beside the complex64 group: with a batch of a few matrices its
    // factorisation is bound by its panel chain (a workgroup per matrix and
    // panel), which then hides under the other group's products.  Measured at
    // N = 8192, Ne = 16: 2 of 16 nodes, factor 433 -> 348 ms; with 5 or 8 of
    // them the groups only compete (the single-solve path only; per-launch
    // timing keeps them in order).
    const bool groups_together = G0.ne > 0 && G1.ne > 0 && 4 * G1.ne <= G0.ne && ws.lookahead && !ws.noalloc &&
                                 !g_gemm_timer && std::getenv("FEASTX_SERIAL_GROUPS") == nullptr &&
                                 ws.aux_stream() != nullptr;
    std::vector<double> lam_prev;   // Ritz values of the previous loop (correction form)
    double prev_maxres = 1e300;     // largest residual in the interval at the previous loop
    double trace_prev = 0.0, epsout = 1.0;
    int info = 0, k = 0, M = 0;
    std::vector<double2> hcoef((size_t)ne * m0), hcoef_g((size_t)ne * m0);
    std::vector<double> hrho(m0);

    for (k = 0; k <= o.maxloop; ++k) {
        const size_t cur_nm = (size_t)n * m0;
        // ---- factor every shifted matrix (once, fpm(10) = 1)
        if (k == 0 || !o.keep_factors) {
            tm.mark(&st.t_shift);
            if (groups_together) {
                FX_CHECK(hipEventRecord(ws.ev_g, s));
                FX_CHECK(hipStreamWaitEvent(ws.aux, ws.ev_g, 0));
                G1.factor_launch(ws, ws.aux, pb, false);   // its panel chain starts first
                G0.factor_launch(ws, s, pb, true);
                try {
                    G0.factor_wait(s, st);
                } catch (...) {
                    (void)hipStreamSynchronize(ws.aux);   // no work left behind on aux
                    throw;
                }
                G1.factor_wait(ws.aux, st);
            } else {
                G0.factor(ws, s, pb, st);
                G1.factor(ws, s, pb, st);
            }
            tm.mark(&st.t_factor);
        }
        const bool corr = use_corr && k >= 1;

        // ---- right-hand sides: B X, or the Ritz residual A X - B X Lambda
        if (corr) {
            FX_CHECK(hipMemcpyAsync(lam, h_lam, sizeof(double) * m0, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL((ritz_residual_kernel<CPLX>), grid1(cur_nm), dim3(256), 0, s, n, m0, AX, BX,
                               (long)n, lam, R);
            FX_LAUNCH_CHECK();
        } else if (pb.B) {
            dgemm<CPLX>(ws, s, false, n, m0, n, 1.0, reinterpret_cast<const E *>(pb.B), pb.ldb, X, n, 0.0, R, n);
        } else {
            hipLaunchKernelGGL((copy_block_kernel<CPLX>), grid1(cur_nm), dim3(256), 0, s, n, m0, X, (long)n, R,
                               (long)n);
            FX_LAUNCH_CHECK();
        }

        // ---- solves at every node (and the adjoint solves for Hermitian pencils)
        G0.solve(ws, s, reinterpret_cast<const double *>(R), m0, st);
        G1.solve(ws, s, reinterpret_cast<const double *>(R), m0, st);
        tm.mark(&st.t_solve);

        // ---- quadrature
        for (int j = 0; j < ne; ++j)
            for (int c = 0; c < m0; ++c) {
                double2 w = ct.w[j];
                if (corr) {
                    // w_j / (z_j - lambda_c)
                    const double dr = ct.z[j].x - h_lam[c], di = ct.z[j].y;
                    const double den = dr * dr + di * di;
                    w = make_double2((w.x * dr + w.y * di) / den, (w.y * dr - w.x * di) / den);
                }
                hcoef[(size_t)j * m0 + c] = w;
            }
        if (corr)
            for (int c = 0; c < m0; ++c) {
                double r = 0.0;
                for (int j = 0; j < ne; ++j) r += hcoef[(size_t)j * m0 + c].x;
                hrho[c] = r;
            }
        // coefficients in each group's node order: complex64 (or FP64) group first
        for (int g = 0; g < 2; ++g) {
            const std::vector<int> &nodes = g == 0 ? lo_nodes : hi_nodes;
            for (size_t q = 0; q < nodes.size(); ++q)
                std::copy(hcoef.begin() + (size_t)nodes[q] * m0, hcoef.begin() + (size_t)(nodes[q] + 1) * m0,
                          hcoef_g.begin() + (g == 0 ? 0 : lo_nodes.size() * m0) + q * m0);
        }
        FX_CHECK(hipMemcpyAsync(coef, hcoef_g.data(), sizeof(double2) * lo_nodes.size() * m0,
                                hipMemcpyHostToDevice, s));
        if (coef1)
            FX_CHECK(hipMemcpyAsync(coef1, hcoef_g.data() + lo_nodes.size() * m0,
                                    sizeof(double2) * hi_nodes.size() * m0, hipMemcpyHostToDevice, s));
        if (corr) FX_CHECK(hipMemcpyAsync(rho, hrho.data(), sizeof(double) * m0, hipMemcpyHostToDevice, s));
        // Q = sum over the nodes (then X diag(rho) in the correction form), the
        // complex128 group added last
        hipLaunchKernelGGL((accumulate_kernel<T, CPLX>), grid1(cur_nm), dim3(256), 0, s, n, m0, G0.ne, G0.Y,
                           (long)n, (long)cur_nm, G0.Yh2, coef, corr ? rho : nullptr, X, (long)n, Q, (long)n, 0);
        if (G1.ne)
            hipLaunchKernelGGL((accumulate_kernel<double, CPLX>), grid1(cur_nm), dim3(256), 0, s, n, m0, G1.ne, G1.Y,
                               (long)n, (long)cur_nm, G1.Yh2, coef1, nullptr, X, (long)n, Q, (long)n, 1);
        FX_LAUNCH_CHECK();
        FX_CHECK(hipStreamSynchronize(s));   // host vectors above are reused next loop
        tm.mark(&st.t_accum);

        if (o.mode == 2) {
            // stochastic count estimate from this one contour pass: samples,
            // running averages into res, the estimate as M (info 5)
            double *samp = static_cast<double *>(ws.get("cnt_samp", sizeof(double) * m0));
            int *dest = static_cast<int *>(ws.get("cnt_est", sizeof(int)));
            int *h_est = static_cast<int *>(ws.pinned("h_cnt_est", sizeof(int)));
            hipLaunchKernelGGL((count_sample_kernel<CPLX>), dim3(m0), dim3(256), 0, s, n, X, (long)n, Q, (long)n,
                               samp);
            hipLaunchKernelGGL(count_mean_kernel, dim3(1), dim3(1024), 0, s, m0, samp, res, dest);
            hipLaunchKernelGGL((copy_block_kernel<CPLX>), grid1(cur_nm), dim3(256), 0, s, n, m0, Q, (long)n,
                               reinterpret_cast<E *>(pb.X), pb.ldx);
            FX_LAUNCH_CHECK();
            FX_CHECK(hipMemcpyAsync(h_res, res, sizeof(double) * m0, hipMemcpyDeviceToHost, s));
            FX_CHECK(hipMemcpyAsync(h_est, dest, sizeof(int), hipMemcpyDeviceToHost, s));
            FX_CHECK(hipStreamSynchronize(s));
            out.M = *h_est;
            out.loop = 0;
            out.m0 = m0;
            out.epsout = 1.0;
            out.E.assign(m0, 0.0);
            out.res.assign(h_res, h_res + m0);
            tm.mark(&st.t_total);
            tm.flush();
            st.loops = 1;
            st.m0_final = m0;
            st_out = st;
            return 5;
        }
        if (o.mode == 1) {
            hipLaunchKernelGGL((copy_block_kernel<CPLX>), grid1(cur_nm), dim3(256), 0, s, n, m0, Q, (long)n,
                               reinterpret_cast<E *>(pb.X), pb.ldx);
            FX_LAUNCH_CHECK();
            FX_CHECK(hipStreamSynchronize(s));
            out.M = 0;
            out.loop = 0;
            out.m0 = m0;
            out.epsout = 1.0;
            tm.mark(&st.t_total);
            tm.flush();
            st.loops = 1;
            st.m0_final = m0;
            st_out = st;
            return 4;
        }

        // ---- Rayleigh-Ritz
        dgemm<CPLX>(ws, s, false, n, m0, n, 1.0, reinterpret_cast<const E *>(pb.A), pb.lda, Q, n, 0.0, AQ, n);
        if (pb.B) dgemm<CPLX>(ws, s, false, n, m0, n, 1.0, reinterpret_cast<const E *>(pb.B), pb.ldb, Q, n, 0.0, BQ, n);
        else {
            hipLaunchKernelGGL((copy_block_kernel<CPLX>), grid1(cur_nm), dim3(256), 0, s, n, m0, Q, (long)n, BQ,
                               (long)n);
            FX_LAUNCH_CHECK();
        }
        dgemm<CPLX>(ws, s, true, m0, m0, n, 1.0, Q, n, AQ, n, 0.0, Aq, m0);
        dgemm<CPLX>(ws, s, true, m0, m0, n, 1.0, Q, n, BQ, n, 0.0, Bq, m0);
        hipLaunchKernelGGL((hermitian_part_kernel<CPLX>), grid1((long)m0 * m0), dim3(256), 0, s, m0, Aq, (long)m0);
        hipLaunchKernelGGL((hermitian_part_kernel<CPLX>), grid1((long)m0 * m0), dim3(256), 0, s, m0, Bq, (long)m0);
        FX_LAUNCH_CHECK();
        tm.mark(&st.t_rr);

        // ---- reduced problem.  B-orthonormal basis T of the kept columns
        //      (T^H Bq T = I), then eig(T^H Aq T) = (lambda, V), Phi = T V.
        int keep = -1;
        if (m0 <= CHOL_MAXM) keep = bortho_cholesky<CPLX>(ws, s, m0, Bq, Tm);
        if (keep < 0) {
            if (g_debug && m0 <= CHOL_MAXM)
                std::fprintf(stderr, "feastx: loop %d: negative Cholesky pivot, Bq by eigendecomposition\n", k);
            keep = bortho_eigen<CPLX>(ws, s, m0, Bq, Wb, beta, Tm, st);
        }
        dgemm<CPLX>(ws, s, false, m0, keep, m0, 1.0, Aq, m0, Tm, m0, 0.0, Tmp, m0);
        dgemm<CPLX>(ws, s, true, keep, keep, m0, 1.0, Tm, m0, Tmp, m0, 0.0, Cr, keep);
        hipLaunchKernelGGL((hermitian_part_kernel<CPLX>), grid1((long)keep * keep), dim3(256), 0, s, keep, Cr,
                           (long)keep);
        FX_LAUNCH_CHECK();
        // Jacobi tolerance.  With the residual test (fpm(6) = 1) a loop's Ritz
        // pairs only need to be accurate well below the residuals the loop
        // can reach: the next subspace does not depend on them (the
        // correction form is an identity for any basis X and any diagonal
        // Lambda), and an off-diagonal norm delta changes a residual by
        // about delta ||C||_F / alpha.  A loop lowers the residuals by 1e-3
        // to 1e-4 here, so 1e-8 times the previous loop's largest residual
        // keeps the Jacobi error far below them; never looser than 1e-4 and
        // never tighter than the full 1e-13.  The first loop of a random
        // start (x0 = 0) cannot converge and takes 1e-4; a caller's start
        // subspace may already be converged and gets the full accuracy.
        double jtol = 1e-13;
        if (o.conv == 1) {
            if (k >= 1) jtol = std::min(1e-4, std::max(1e-13, 1e-8 * prev_maxres));
            else if (!o.x0) jtol = 1e-4;
        }
        device_eigh<CPLX>(ws, s, keep, Cr, Vc, lam, st, jtol);
        dgemm<CPLX>(ws, s, false, m0, keep, keep, 1.0, Tm, m0, Vc, keep, 0.0, Phi, m0);
        tm.mark(&st.t_reduced);

        // ---- Ritz vectors, A X, B X, residuals
        dgemm<CPLX>(ws, s, false, n, keep, m0, 1.0, Q, n, Phi, m0, 0.0, X, n);
        dgemm<CPLX>(ws, s, false, n, keep, m0, 1.0, AQ, n, Phi, m0, 0.0, AX, n);
        dgemm<CPLX>(ws, s, false, n, keep, m0, 1.0, BQ, n, Phi, m0, 0.0, BX, n);
        hipLaunchKernelGGL((resid_norm_kernel<CPLX>), dim3(keep), dim3(256), 0, s, n, AX, BX, (long)n, lam, alpha,
                           res);
        FX_LAUNCH_CHECK();
        FX_CHECK(hipMemcpyAsync(h_lam, lam, sizeof(double) * keep, hipMemcpyDeviceToHost, s));
        FX_CHECK(hipMemcpyAsync(h_res, res, sizeof(double) * keep, hipMemcpyDeviceToHost, s));
        FX_CHECK(hipStreamSynchronize(s));
        tm.mark(&st.t_resid);
        m0 = keep;

        // ---- count, spurious flag, trace, convergence (Tables "tab_common", "tab_fpm")
        int inside = 0, bad = 0;
        double trace = 0.0, maxres = 0.0;
        M = 0;
        for (int i = 0; i < m0; ++i) {
            if (h_lam[i] < pb.emin || h_lam[i] > pb.emax) continue;
            ++inside;
            if (k >= 1 && h_res[i] > SPURIOUS_RES) continue;
            ++M;
            trace += h_lam[i];
            maxres = std::max(maxres, h_res[i]);
            if (!(h_res[i] < o.tol)) ++bad;
        }
        epsout = (k == 0) ? 1.0 : std::fabs(trace - trace_prev) / alpha;
        trace_prev = trace;
        prev_maxres = M > 0 ? maxres : 1e300;
        if (o.verbose)
            std::fprintf(stderr, "feastx loop %d: #eig %d  trace %.15e  eps %.3e  maxres %.3e  m0 %d\n", k, M, trace,
                         epsout, maxres, m0);
        const bool converged = (M > 0) && (o.conv == 1 ? bad == 0 : epsout < o.tol);
        if (k == 0 && inside == 0) {
            info = 1;
            break;
        }
        if (converged) {
            info = 0;
            break;
        }
        if (M >= m0) {
            info = 3;
            break;
        }
        if (k == o.maxloop) {
            info = 2;
            break;
        }
    }
    if (k > o.maxloop) k = o.maxloop;

    // ---- output order: in-interval ascending, outside ascending, spurious last
    std::vector<int> order;
    order.reserve(m0);
    auto cls = [&](int i) {
        const bool in = h_lam[i] >= pb.emin && h_lam[i] <= pb.emax;
        if (!in) return 1;
        return (k >= 1 && h_res[i] > SPURIOUS_RES) ? 2 : 0;
    };
    for (int pass = 0; pass < 3; ++pass)
        for (int i = 0; i < m0; ++i)
            if (cls(i) == pass) order.push_back(i);
    out.E.resize(m0);
    out.res.resize(m0);
    for (int c = 0; c < m0; ++c) {
        out.E[c] = h_lam[order[c]];
        out.res[c] = cls(order[c]) == 2 ? -1.0 : h_res[order[c]];
    }
    FX_CHECK(hipMemcpyAsync(sel, order.data(), sizeof(int) * m0, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL((gather_cols_kernel<CPLX>), grid1((long)n * m0), dim3(256), 0, s, n, m0, sel, X, (long)n,
                       reinterpret_cast<E *>(pb.X), pb.ldx);
    FX_LAUNCH_CHECK();
    FX_CHECK(hipStreamSynchronize(s));
    tm.mark(&st.t_total);
    tm.flush();
    out.M = M;
    out.loop = k;
    out.m0 = m0;
    out.epsout = epsout;
    st.loops = k + 1;
    st.m0_final = m0;
    st.t_total += st.t_shift + st.t_factor + st.t_solve + st.t_accum + st.t_rr + st.t_reduced + st.t_resid;
    if (g_gemm_timer) {
        FX_CHECK(hipStreamSynchronize(s));
        double tot = 0, tot_lu = 0;
        long long n_lu = 0;
        for (size_t q = 0; q < g_gemm_timer->ev.size(); ++q) {
            float ms = 0;
            FX_CHECK(hipEventElapsedTime(&ms, g_gemm_timer->ev[q].first, g_gemm_timer->ev[q].second));
            tot += ms;
            if (g_gemm_timer->in_lu[q]) {
                tot_lu += ms;
                ++n_lu;
            }
        }
        gemm_timing_reset();
        st.t_lu_gemm = tot;
        st.lu_gemm_flops = g_gemm_timer->flops;
        st.lu_gemm_launches = (long long)g_gemm_timer->ev.size();
        st.t_lu_update = tot_lu;
        st.lu_update_flops = g_gemm_timer->lu_flops;
        st.lu_update_launches = n_lu;
        g_gemm_timer->ev.clear();
        g_gemm_timer->in_lu.clear();
        g_gemm_timer->flops = 0;
        g_gemm_timer->lu_flops = 0;
    }
    st_out = st;
    return info;
}

// ---------------------------------------------------------------- non-Hermitian
// Full-contour nodes and weights (fpm(8) nodes; fpm(17) rule, fpm(18)
// ellipse ratio, fpm(19) rotation).  The contour is z(t) = c + e^{i phi}
// (r cos t + i a r sin t), t in [0, 2 pi); a node at t with step dt weighs
// dz / (2 pi i) = (dt / 2 pi) e^{i phi} (a r cos t + i r sin t).
// Trapezoidal: t_j = 2 pi (j + 1/2) / ne.  Gauss: one ne-point
// Gauss-Legendre rule over [0, 2 pi].
static Contour make_full_contour(double2 c, double r, int ne, int integration, int ellipse, int angle)
{
    std::vector<double> t(ne), f(ne);
    if (integration == 1) {
        for (int j = 0; j < ne; ++j) {
            t[j] = 2.0 * M_PI * (j + 0.5) / ne;
            f[j] = 1.0 / ne;
        }
    } else {
        std::vector<double> x, om;
        gauss_legendre(ne, x, om);
        for (int j = 0; j < ne; ++j) {
            t[j] = M_PI * (1.0 + x[j]);
            f[j] = 0.5 * om[j];
        }
    }
    const double a = ellipse / 100.0, phi = angle * M_PI / 180.0, cr = std::cos(phi), sr = std::sin(phi);
    Contour ct;
    ct.z.resize(ne);
    ct.w.resize(ne);
    for (int j = 0; j < ne; ++j) {
        const double ct_ = std::cos(t[j]), st_ = std::sin(t[j]);
        const double ur = r * ct_, ui = a * r * st_;            // point before rotation
        const double vr = f[j] * a * r * ct_, vi = f[j] * r * st_;   // weight before rotation
        ct.z[j] = make_double2(c.x + cr * ur - sr * ui, c.y + sr * ur + cr * ui);
        ct.w[j] = make_double2(cr * vr - sr * vi, sr * vr + cr * vi);
    }
    return ct;
}

struct GProblem {
    int n;
    const double2 *A;   // device, complex
    long lda;
    const double2 *B;   // device or NULL
    long ldb;
    double2 emid;
    double r;
    int m0;
    double2 *X;   // caller's device array, n x 2 m0: right, then left
    long ldx;
};

struct GResult {
    int M = 0, loop = 0, m0 = 0;
    double epsout = 1.0;
    std::vector<double2> E;
    std::vector<double> res;   // 2 m0
};

static bool in_region(double2 lam, double2 c, double r, int ellipse, int angle)
{
    const double phi = angle * M_PI / 180.0, a = ellipse / 100.0;
    const double dr = lam.x - c.x, di = lam.y - c.y;
    const double ur = std::cos(phi) * dr + std::sin(phi) * di, ui = -std::sin(phi) * dr + std::cos(phi) * di;
    return (ur / r) * (ur / r) + (ui / (a * r)) * (ui / (a * r)) <= 1.0;
}

// Non-Hermitian FEAST with dual subspaces:
//   Q = sum_j w_j (z_j B - A)^{-1} B X,  Qh = sum_j conj(w_j) (z_j B - A)^{-H} B^H Xh,
//   Aq = Qh^H A Q, Bq = Qh^H B Q, Aq W = Bq W Lambda, Wh^H Aq = Lambda Wh^H Bq,
//   X = Q W, Xh = Qh Wh (unit columns); residuals of both sides.
// T is the precision of the factors and solves; everything else is FP64.
// In complex64 (T = float) the loops after the first use the correction
// form on both sides: with R = A X - B X Lambda and Rh = A^H Xh - B^H Xh
// conj(Lambda) (FP64), (z B - A)^{-1} B X = (X + (z B - A)^{-1} R)
// diag(1 / (z - lambda)) and the same for the adjoint, so
//   Q  = X diag(rho) + sum_j w_j (z_j B - A)^{-1} R diag(1 / (z_j - lambda)),
//   Qh = Xh diag(conj rho) + sum_j conj(w_j) (z_j B - A)^{-H} Rh diag(1 / conj(z_j - lambda)),
// rho(lambda) = sum_j w_j / (z_j - lambda): the single-precision error then
// scales with the residuals, not with X.
template <typename T>
static int run_general(const GProblem &pb, const feast_opts &o, hipStream_t s, Workspace &ws, GResult &out,
                       feast_stats &st_out)
{
    using V = cplx<T>;
    using E = double2;
    const bool mixed = std::is_same<T, float>::value;
    const int n = pb.n, ne = o.ne_full, m0 = pb.m0;
    const double alpha = std::hypot(pb.emid.x, pb.emid.y) + pb.r;
    const size_t nm = (size_t)n * m0, mm = (size_t)m0 * m0;
    feast_stats st{};
    StageTimer tm(s, !ws.noalloc);
    tm.start();

    Contour ct = make_full_contour(pb.emid, pb.r, ne, o.integration_full, o.ellipse, o.angle);
    double2 *dz = static_cast<double2 *>(ws.get("z", sizeof(double2) * ne));
    double2 *dcoef = static_cast<double2 *>(ws.get("coef", sizeof(double2) * ne * m0));
    double2 *drho = static_cast<double2 *>(ws.get("grho", sizeof(double2) * m0));
    double2 *h_coef = static_cast<double2 *>(ws.pinned("h_gcoef", sizeof(double2) * ne * m0));
    double2 *h_rho = static_cast<double2 *>(ws.pinned("h_grho", sizeof(double2) * m0));
    FX_CHECK(hipMemcpyAsync(dz, ct.z.data(), sizeof(double2) * ne, hipMemcpyHostToDevice, s));

    auto blk = [&](const char *name, size_t count) { return static_cast<E *>(ws.get(name, sizeof(E) * count)); };
    E *X = blk("X", nm), *Xh = blk("Xh", nm), *R = blk("R", nm), *Rh = blk("Rh", nm);
    E *Q = blk("Q", nm), *Qh = blk("Qh", nm), *AQ = blk("AQ", nm), *BQ = blk("BQ", nm);
    E *AX = blk("AX", nm), *BX = blk("BX", nm), *AhX = blk("AhX", nm), *BhX = blk("BhX", nm);
    E *Aq = blk("Aq", mm), *Bq = blk("Bq", mm), *Binv = blk("Binv", mm), *Cm = blk("Cm", mm);
    E *Zs = blk("Zs", mm), *Ys = blk("Ys", mm), *Wm = blk("Wm", mm), *Wc = blk("Wc", mm), *Winv = blk("Winv", mm);
    E *G = blk("G", mm), *Wh = blk("Wh", mm);
    E *lam = blk("glam", m0);
    double *res = static_cast<double *>(ws.get("gres", sizeof(double) * 2 * m0));
    int *sel = static_cast<int *>(ws.get("sel", sizeof(int) * m0));
    int *dstat = static_cast<int *>(ws.get("gstat", sizeof(int) * 4));
    const long ldf = n, sF = (long)n * n;
    V *F = static_cast<V *>(ws.get(mixed ? "F32" : "F64", sizeof(V) * (size_t)ne * sF));
    int *ipiv = static_cast<int *>(ws.get("ipiv", sizeof(int) * (size_t)ne * n));
    int *perm = static_cast<int *>(ws.get("perm", sizeof(int) * (size_t)ne * n));
    int *swapmap = static_cast<int *>(ws.get("swapmap", sizeof(int) * LU_LISTS * (size_t)ne * LU_LIST_INTS));
    int *dinfo = static_cast<int *>(ws.get("info", sizeof(int) * ne));
    const bool compose = solve_nb<T>() > TRI_INV_NB;
    const long sI64 = compose ? tri_inv_stride(n) : 0, sInv = solve_inv_stride<T>(n);
    const long sItmp = compose ? (long)ceil_div(n, solve_nb<T>()) * 64 * 64 : 0;
    V *L64 = compose ? static_cast<V *>(ws.get("L64inv", sizeof(V) * (size_t)ne * sI64)) : nullptr;
    V *U64 = compose ? static_cast<V *>(ws.get("U64inv", sizeof(V) * (size_t)ne * sI64)) : nullptr;
    V *Itmp = compose ? static_cast<V *>(ws.get("Invtmp", sizeof(V) * (size_t)ne * sItmp)) : nullptr;
    V *Wsv = static_cast<V *>(ws.get(mixed ? "Wsolve32" : "Wsolve64", sizeof(V) * (size_t)ne * sF));
    V *Linv = static_cast<V *>(ws.get(mixed ? "Linv32" : "Linv64", sizeof(V) * (size_t)ne * sInv));
    V *Uinv = static_cast<V *>(ws.get(mixed ? "Uinv32" : "Uinv64", sizeof(V) * (size_t)ne * sInv));
    V *Ytmp = static_cast<V *>(ws.get(mixed ? "Yt32" : "Yt64", sizeof(V) * (size_t)ne * nm));
    V *Y = static_cast<V *>(ws.get(mixed ? "Y32" : "Y64", sizeof(V) * (size_t)ne * nm));
    V *Yh = static_cast<V *>(ws.get(mixed ? "Yh32" : "Yh64", sizeof(V) * (size_t)ne * nm));
    V *Yh2 = static_cast<V *>(ws.get(mixed ? "Yg32" : "Yg64", sizeof(V) * (size_t)ne * nm));
    double2 *h_lam = static_cast<double2 *>(ws.pinned("h_glam", sizeof(double2) * m0));
    double *h_res = static_cast<double *>(ws.pinned("h_gres", sizeof(double) * 2 * m0));
    int *h_stat = static_cast<int *>(ws.pinned("h_gstat", sizeof(int) * 4));
    int *h_info = static_cast<int *>(ws.pinned("h_info", sizeof(int) * ne));

    // start subspaces: the caller's (right in columns 0..m0-1, left in m0..2m0-1) or seeded
    if (o.x0) {
        hipLaunchKernelGGL((copy_block_kernel<true>), grid1(nm), dim3(256), 0, s, n, m0, pb.X, pb.ldx, X, (long)n);
        hipLaunchKernelGGL((copy_block_kernel<true>), grid1(nm), dim3(256), 0, s, n, m0, pb.X + (long)m0 * pb.ldx,
                           pb.ldx, Xh, (long)n);
    } else {
        hipLaunchKernelGGL((random_start_kernel<true>), grid1(nm), dim3(256), 0, s, n, m0, o.seed, 0, X, (long)n);
        hipLaunchKernelGGL((random_start_kernel<true>), grid1(nm), dim3(256), 0, s, n, m0, o.seed + 1, 0, Xh,
                           (long)n);
    }
    FX_LAUNCH_CHECK();

    // factor every shifted matrix once (the factors serve both sides)
    shift_build<T>(s, true, n, reinterpret_cast<const double *>(pb.A), pb.lda,
                   reinterpret_cast<const double *>(pb.B), pb.ldb, dz, ne, F, ldf, sF);
    tm.mark(&st.t_shift);
    FX_CHECK(hipMemsetAsync(dinfo, 0, sizeof(int) * ne, s));
    getrf_batched<T>(s, nullptr, ws.ev_a, ws.ev_b, n, F, ldf, sF, ipiv, perm, n, swapmap, dinfo, ne);
    solve_inverses<T>(s, n, F, ldf, sF, L64, U64, sI64, Linv, Uinv, sInv, Itmp, sItmp, ne);
    build_w<T>(s, n, F, ldf, sF, Linv, Uinv, sInv, Wsv, ne);
    FX_CHECK(hipMemcpyAsync(h_info, dinfo, sizeof(int) * ne, hipMemcpyDeviceToHost, s));
    FX_CHECK(hipStreamSynchronize(s));
    for (int j = 0; j < ne; ++j)
        if (h_info[j] != 0) throw solver_error{-2};
    st.factor_flops += ne * (8.0 / 3.0) * (double)n * n * n;
    tm.mark(&st.t_factor);

    const E *A = pb.A, *B = pb.B;
    double trace_re = 0.0, trace_im = 0.0, epsout = 1.0;
    int info = 0, k = 0, M = 0;
    std::vector<char> ins(m0), spur(m0);
    for (k = 0; k <= o.maxloop; ++k) {
        const bool corr = mixed && k >= 1;
        // right-hand sides: B X and B^H Xh, or (correction form) the Ritz
        // residual blocks of the previous loop
        if (corr) {
            hipLaunchKernelGGL(ritz_residual_general_kernel, grid1(nm), dim3(256), 0, s, n, m0, AX, BX, (long)n, lam,
                               0, R);
            hipLaunchKernelGGL(ritz_residual_general_kernel, grid1(nm), dim3(256), 0, s, n, m0, AhX, BhX, (long)n,
                               lam, 1, Rh);
            FX_LAUNCH_CHECK();
        } else if (B) {
            dgemm<true>(ws, s, false, n, m0, n, 1.0, B, pb.ldb, X, n, 0.0, R, n);
            dgemm<true>(ws, s, true, n, m0, n, 1.0, B, pb.ldb, Xh, n, 0.0, Rh, n);
        } else {
            hipLaunchKernelGGL((copy_block_kernel<true>), grid1(nm), dim3(256), 0, s, n, m0, X, (long)n, R, (long)n);
            hipLaunchKernelGGL((copy_block_kernel<true>), grid1(nm), dim3(256), 0, s, n, m0, Xh, (long)n, Rh,
                               (long)n);
            FX_LAUNCH_CHECK();
        }
        // solves at every node: (z_j B - A) Y = R and (z_j B - A)^H Yh = Rh
        {
            dim3 g((unsigned)((nm + 255) / 256), ne);
            hipLaunchKernelGGL((gather_rows_kernel<T, true>), g, dim3(256), 0, s, n, m0, perm, (long)n,
                               reinterpret_cast<const double *>(R), (long)n, Y, (long)n, (long)nm);
            FX_LAUNCH_CHECK();
            getrs_batched<T>(s, false, n, m0, F, Wsv, ldf, sF, Linv, Uinv, sInv, Y, Ytmp, n, (long)nm, ne);
            hipLaunchKernelGGL((copy_rhs_kernel<T, true>), g, dim3(256), 0, s, n, m0,
                               reinterpret_cast<const double *>(Rh), (long)n, Yh, (long)n, (long)nm);
            FX_LAUNCH_CHECK();
            getrs_batched<T>(s, true, n, m0, F, Wsv, ldf, sF, Linv, Uinv, sInv, Yh, Ytmp, n, (long)nm, ne);
            hipLaunchKernelGGL((scatter_rows_kernel<T>), g, dim3(256), 0, s, n, m0, perm, (long)n, Yh, (long)n,
                               (long)nm, Yh2, (long)n, (long)nm);
            FX_LAUNCH_CHECK();
            st.solve_flops += 2.0 * ne * 8.0 * (double)n * n * m0;
        }
        tm.mark(&st.t_solve);
        // quadrature coefficients: w_j, or w_j / (z_j - lambda_c) and rho_c
        for (int c = 0; c < m0; ++c) {
            double2 rc = make_double2(0.0, 0.0);
            for (int j = 0; j < ne; ++j) {
                double2 w = ct.w[j];
                if (corr) {
                    const double dr = ct.z[j].x - h_lam[c].x, di = ct.z[j].y - h_lam[c].y;
                    const double den = dr * dr + di * di;
                    w = make_double2((w.x * dr + w.y * di) / den, (w.y * dr - w.x * di) / den);
                    rc.x += w.x;
                    rc.y += w.y;
                }
                h_coef[(size_t)j * m0 + c] = w;
            }
            h_rho[c] = rc;
        }
        FX_CHECK(hipMemcpyAsync(dcoef, h_coef, sizeof(double2) * ne * m0, hipMemcpyHostToDevice, s));
        if (corr) FX_CHECK(hipMemcpyAsync(drho, h_rho, sizeof(double2) * m0, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL((accumulate_general_kernel<T>), grid1(nm), dim3(256), 0, s, n, m0, ne, Y, Yh2, (long)n,
                           (long)nm, dcoef, corr ? drho : nullptr, X, Xh, (long)n, Q, Qh, (long)n);
        FX_LAUNCH_CHECK();
        tm.mark(&st.t_accum);

        // reduced pencil
        dgemm<true>(ws, s, false, n, m0, n, 1.0, A, pb.lda, Q, n, 0.0, AQ, n);
        if (B) dgemm<true>(ws, s, false, n, m0, n, 1.0, B, pb.ldb, Q, n, 0.0, BQ, n);
        else {
            hipLaunchKernelGGL((copy_block_kernel<true>), grid1(nm), dim3(256), 0, s, n, m0, Q, (long)n, BQ, (long)n);
            FX_LAUNCH_CHECK();
        }
        dgemm<true>(ws, s, true, m0, m0, n, 1.0, Qh, n, AQ, n, 0.0, Aq, m0);
        dgemm<true>(ws, s, true, m0, m0, n, 1.0, Qh, n, BQ, n, 0.0, Bq, m0);
        tm.mark(&st.t_rr);

        // reduced eigenproblem: C = Bq^{-1} Aq = W Lambda W^{-1}, Wh = (W^{-1} Bq^{-1})^H
        auto gj_inverse = [&](E *Mx, E *Inv, int *stat) {
            if (m0 <= 64)   // both matrices in LDS
                hipLaunchKernelGGL((gj_inverse_kernel<NH_NT, 64>), dim3(1), dim3(NH_NT), 0, s, m0, Mx, Inv, stat);
            else
                hipLaunchKernelGGL((gj_inverse_kernel<NH_NT, 0>), dim3(1), dim3(NH_NT), 0, s, m0, Mx, Inv, stat);
        };
        gj_inverse(Bq, Binv, dstat);
        FX_LAUNCH_CHECK();
        dgemm<true>(ws, s, false, m0, m0, m0, 1.0, Binv, m0, Aq, m0, 0.0, Cm, m0);
        if (m0 <= 64)   // the Hessenberg matrix and the Schur vectors in LDS, one wave
            hipLaunchKernelGGL((eig_general_kernel<64, 64>), dim3(1), dim3(64), 0, s, m0, Cm, Zs, Ys, lam, dstat + 1);
        else
            hipLaunchKernelGGL((eig_general_kernel<NH_NT, 0>), dim3(1), dim3(NH_NT), 0, s, m0, Cm, Zs, Ys, lam,
                               dstat + 1);
        FX_LAUNCH_CHECK();
        dgemm<true>(ws, s, false, m0, m0, m0, 1.0, Zs, m0, Ys, m0, 0.0, Wm, m0);
        hipLaunchKernelGGL((copy_block_kernel<true>), grid1(mm), dim3(256), 0, s, m0, m0, Wm, (long)m0, Wc,
                           (long)m0);
        gj_inverse(Wc, Winv, dstat + 3);
        FX_LAUNCH_CHECK();
        dgemm<true>(ws, s, false, m0, m0, m0, 1.0, Winv, m0, Binv, m0, 0.0, G, m0);
        hipLaunchKernelGGL(conj_transpose_kernel, grid1(mm), dim3(256), 0, s, m0, G, Wh);
        FX_LAUNCH_CHECK();
        FX_CHECK(hipMemcpyAsync(h_stat, dstat, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
        FX_CHECK(hipStreamSynchronize(s));
        if (h_stat[0] != 0 || h_stat[1] != 0 || h_stat[3] != 0) throw solver_error{-3};
        st.eig_calls += 1;
        st.eig_sweeps += h_stat[2];
        tm.mark(&st.t_reduced);

        // Ritz vectors of both sides, unit columns, residuals
        dgemm<true>(ws, s, false, n, m0, m0, 1.0, Q, n, Wm, m0, 0.0, X, n);
        dgemm<true>(ws, s, false, n, m0, m0, 1.0, Qh, n, Wh, m0, 0.0, Xh, n);
        hipLaunchKernelGGL(normalize_cols_kernel, dim3(m0), dim3(256), 0, s, n, X, (long)n);
        hipLaunchKernelGGL(normalize_cols_kernel, dim3(m0), dim3(256), 0, s, n, Xh, (long)n);
        FX_LAUNCH_CHECK();
        dgemm<true>(ws, s, false, n, m0, n, 1.0, A, pb.lda, X, n, 0.0, AX, n);
        dgemm<true>(ws, s, true, n, m0, n, 1.0, A, pb.lda, Xh, n, 0.0, AhX, n);
        if (B) {
            dgemm<true>(ws, s, false, n, m0, n, 1.0, B, pb.ldb, X, n, 0.0, BX, n);
            dgemm<true>(ws, s, true, n, m0, n, 1.0, B, pb.ldb, Xh, n, 0.0, BhX, n);
        } else {
            hipLaunchKernelGGL((copy_block_kernel<true>), grid1(nm), dim3(256), 0, s, n, m0, X, (long)n, BX, (long)n);
            hipLaunchKernelGGL((copy_block_kernel<true>), grid1(nm), dim3(256), 0, s, n, m0, Xh, (long)n, BhX,
                               (long)n);
        }
        hipLaunchKernelGGL(resid_general_kernel, dim3(m0), dim3(256), 0, s, n, AX, BX, (long)n, lam, 0, alpha, res);
        hipLaunchKernelGGL(resid_general_kernel, dim3(m0), dim3(256), 0, s, n, AhX, BhX, (long)n, lam, 1, alpha,
                           res + m0);
        FX_LAUNCH_CHECK();
        FX_CHECK(hipMemcpyAsync(h_lam, lam, sizeof(double2) * m0, hipMemcpyDeviceToHost, s));
        FX_CHECK(hipMemcpyAsync(h_res, res, sizeof(double) * 2 * m0, hipMemcpyDeviceToHost, s));
        FX_CHECK(hipStreamSynchronize(s));
        tm.mark(&st.t_resid);

        // count, spurious pairs (both residuals), trace, convergence
        int bad = 0;
        double tr = 0.0, ti = 0.0, maxres = 0.0;
        M = 0;
        int inside = 0;
        for (int i = 0; i < m0; ++i) {
            ins[i] = in_region(h_lam[i], pb.emid, pb.r, o.ellipse, o.angle);
            const double ri = std::max(h_res[i], h_res[m0 + i]);
            spur[i] = ins[i] && k >= 1 && ri > SPURIOUS_RES;
            if (!ins[i]) continue;
            ++inside;
            if (spur[i]) continue;
            ++M;
            tr += h_lam[i].x;
            ti += h_lam[i].y;
            maxres = std::max(maxres, ri);
            if (!(ri < o.tol)) ++bad;
        }
        epsout = (k == 0) ? 1.0 : std::hypot(tr - trace_re, ti - trace_im) / alpha;
        trace_re = tr;
        trace_im = ti;
        if (o.verbose)
            std::fprintf(stderr, "feastx loop %d: #eig %d  trace %.15e%+.15ei  eps %.3e  maxres %.3e\n", k, M, tr, ti,
                         epsout, maxres);
        const bool converged = (M > 0) && (o.conv == 1 ? bad == 0 : epsout < o.tol);
        if (k == 0 && inside == 0) {
            info = 1;
            break;
        }
        if (converged) {
            info = 0;
            break;
        }
        if (M >= m0) {
            info = 3;
            break;
        }
        if (k == o.maxloop) {
            info = 2;
            break;
        }
    }
    if (k > o.maxloop) k = o.maxloop;

    // output order: counted pairs, pairs outside, spurious pairs; each by
    // increasing real part, then imaginary part
    std::vector<int> idx(m0);
    for (int i = 0; i < m0; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        if (h_lam[a].x != h_lam[b].x) return h_lam[a].x < h_lam[b].x;
        return h_lam[a].y < h_lam[b].y;
    });
    std::vector<int> order;
    order.reserve(m0);
    for (int pass = 0; pass < 3; ++pass)
        for (int i : idx) {
            const int c = !ins[i] ? 1 : (spur[i] ? 2 : 0);
            if (c == pass) order.push_back(i);
        }
    out.E.resize(m0);
    out.res.assign(2 * (size_t)m0, 0.0);
    for (int c = 0; c < m0; ++c) {
        const int i = order[c];
        const bool sp = ins[i] && spur[i];
        out.E[c] = h_lam[i];
        out.res[c] = sp ? -1.0 : h_res[i];
        out.res[m0 + c] = sp ? -1.0 : h_res[m0 + i];
    }
    FX_CHECK(hipMemcpyAsync(sel, order.data(), sizeof(int) * m0, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL((gather_cols_kernel<true>), grid1(nm), dim3(256), 0, s, n, m0, sel, X, (long)n, pb.X, pb.ldx);
    hipLaunchKernelGGL((gather_cols_kernel<true>), grid1(nm), dim3(256), 0, s, n, m0, sel, Xh, (long)n,
                       pb.X + (long)m0 * pb.ldx, pb.ldx);
    FX_LAUNCH_CHECK();
    FX_CHECK(hipStreamSynchronize(s));
    tm.mark(&st.t_total);
    tm.flush();
    out.M = M;
    out.loop = k;
    out.m0 = m0;
    out.epsout = epsout;
    st.loops = k + 1;
    st.m0_final = m0;
    st.t_total += st.t_shift + st.t_factor + st.t_solve + st.t_accum + st.t_rr + st.t_reduced + st.t_resid;
    st_out = st;
    return info;
}

// Validation shared by every entry point (Table "tab_info").
static int validate(int n, int m0, double emin, double emax, const feast_opts &o)
{
    if (n < 1) return 202;
    if (m0 < 1 || m0 > n) return 201;
    if (!(emin < emax) || !std::isfinite(emin) || !std::isfinite(emax)) return 200;
    if (o.ne < 1 || o.ne > 256) return 102;
    if (!(o.tol > 0.0)) return 103;
    if (o.maxloop < 0) return 104;
    if (o.x0 != 0 && o.x0 != 1) return 105;
    if (o.conv != 0 && o.conv != 1) return 106;
    if (o.keep_factors != 0 && o.keep_factors != 1) return 110;
    if (o.mode < 0 || o.mode > 2) return 114;
    if (o.precision != 0 && o.precision != 1) return 140;
    if (o.integration != 0 && o.integration != 1) return 116;   // Zolotarev (2) is not in this build
    if (o.ellipse < 1) return 118;
    if ((o.Zne == nullptr) != (o.Wne == nullptr)) return -113;
    if (o.refine != 0) return 141;   // per-solve refinement: not available in this build
    if (m0 > 4096) return 201;
    if (o.precision == 1 && n > lu_max_n<float>()) return 202;
    if (o.precision == 0 && n > lu_max_n<double>()) return 202;
    return 0;
}

// Validation of the non-Hermitian entry points.
static int validate_general(int n, int m0, double2 emid, double r, const feast_opts &o)
{
    if (n < 1) return 202;
    if (m0 < 1 || m0 > n || m0 > NH_MAXM) return 201;
    if (!(r > 0.0) || !std::isfinite(r) || !std::isfinite(emid.x) || !std::isfinite(emid.y)) return 200;
    if (o.ne_full < 1 || o.ne_full > 256) return 108;
    if (!(o.tol > 0.0)) return 103;
    if (o.maxloop < 0) return 104;
    if (o.x0 != 0 && o.x0 != 1) return 105;
    if (o.conv != 0 && o.conv != 1) return 106;
    if (o.mode != 0) return 114;
    if (o.precision != 0 && o.precision != 1) return 140;
    if (o.integration_full != 0 && o.integration_full != 1) return 117;
    if (o.ellipse < 1) return 118;
    if (o.angle < -180 || o.angle > 180) return 119;
    if (n > (o.precision == 1 ? lu_max_n<float>() : lu_max_n<double>())) return 202;
    return 0;
}

static int dispatch(bool cplx_in, const Problem &pb, const feast_opts &o, hipStream_t s, Workspace &ws,
                    Result &out, feast_stats &st)
{
    GemmTimer gt;
    gt.f64 = o.precision != 1;
    try {
        ws.init();
        if (!s && !ws.noalloc) s = ws.stream;
        g_gemm_timer = (g_timing && !ws.noalloc) ? &gt : nullptr;
        int info;
        if (o.precision == 1)
            info = cplx_in ? run<float, true>(pb, o, s, ws, out, st) : run<float, false>(pb, o, s, ws, out, st);
        else
            info = cplx_in ? run<double, true>(pb, o, s, ws, out, st) : run<double, false>(pb, o, s, ws, out, st);
        g_gemm_timer = nullptr;
        return info;
    } catch (const alloc_error &) {
        g_gemm_timer = nullptr;
        return -1;
    } catch (const solver_error &e) {
        g_gemm_timer = nullptr;
        (void)hipStreamSynchronize(s ? s : ws.stream);
        return e.info;
    } catch (const hip_error &e) {
        g_gemm_timer = nullptr;
        std::fprintf(stderr, "feastx: HIP error %s\n", hipGetErrorString(e.code));
        return -4;
    } catch (const std::bad_alloc &) {
        g_gemm_timer = nullptr;
        return -1;
    }
}

// One solve with arguments already checked.  `device` says whether A, B, X
// are device (1) or host (0) arrays; host arrays are staged through the
// workspace.  Fills E/res/M/... on info in {0,1,2,3}.
struct SolveArgs {
    bool cplx;
    int n;
    const void *A;
    int lda;
    const void *B;
    int ldb;
    double emin, emax;
    int m0;
    void *X;
    int ldx;
    double *E, *res;
    int device;
    hipStream_t stream;
};
struct SolveOut {
    int info = 0, M = 0, m0 = 0, loop = 0;
    double epsout = 1.0;
    feast_stats st{};
};

static void copy_outputs(const Result &out, int info, const SolveArgs &a, SolveOut &so)
{
    so.info = info;
    if (info == 0 || info == 1 || info == 2 || info == 3 || info == 5) {
        for (int i = 0; i < out.m0; ++i) {
            a.E[i] = out.E[i];
            a.res[i] = out.res[i];
        }
        so.M = out.M;
        so.m0 = out.m0;
        so.loop = out.loop;
        so.epsout = out.epsout;
    } else if (info == 4) {
        so.M = 0;
        so.m0 = a.m0;
        so.loop = 0;
        so.epsout = 1.0;
    } else {
        so.m0 = a.m0;
    }
}

// Copies of column blocks between pageable host memory (leading dimension
// spitch / dpitch bytes) and a packed device buffer.  A pageable 2D copy
// moves one column per transfer, so a contiguous block goes in one copy and a
// strided one through a packed host buffer, up to 64 MiB at a time.  Both
// return when the data has landed.
static void upload_cols(void *dst, const void *src, size_t spitch, size_t rowbytes, long ncols)
{
    if (ncols <= 0 || rowbytes == 0) return;
    if (spitch == rowbytes) {
        FX_CHECK(hipMemcpy(dst, src, rowbytes * (size_t)ncols, hipMemcpyHostToDevice));
        return;
    }
    const long per = std::max<long>(1, (long)((64ull << 20) / rowbytes));
    std::vector<unsigned char> tmp(rowbytes * (size_t)std::min(per, ncols));
    for (long j0 = 0; j0 < ncols; j0 += per) {
        const long nc = std::min(per, ncols - j0);
        for (long j = 0; j < nc; ++j)
            std::memcpy(tmp.data() + j * rowbytes, static_cast<const unsigned char *>(src) + (j0 + j) * spitch,
                        rowbytes);
        FX_CHECK(hipMemcpy(static_cast<unsigned char *>(dst) + j0 * rowbytes, tmp.data(), nc * rowbytes,
                           hipMemcpyHostToDevice));
    }
}

// The reverse, after the work queued on stream s has finished.
static void download_cols(void *dst, size_t dpitch, const void *src, size_t rowbytes, long ncols, hipStream_t s)
{
    FX_CHECK(hipStreamSynchronize(s));
    if (ncols <= 0 || rowbytes == 0) return;
    if (dpitch == rowbytes) {
        FX_CHECK(hipMemcpy(dst, src, rowbytes * (size_t)ncols, hipMemcpyDeviceToHost));
        return;
    }
    const long per = std::max<long>(1, (long)((64ull << 20) / rowbytes));
    std::vector<unsigned char> tmp(rowbytes * (size_t)std::min(per, ncols));
    for (long j0 = 0; j0 < ncols; j0 += per) {
        const long nc = std::min(per, ncols - j0);
        FX_CHECK(hipMemcpy(tmp.data(), static_cast<const unsigned char *>(src) + j0 * rowbytes, nc * rowbytes,
                           hipMemcpyDeviceToHost));
        for (long j = 0; j < nc; ++j)
            std::memcpy(static_cast<unsigned char *>(dst) + (j0 + j) * dpitch, tmp.data() + j * rowbytes, rowbytes);
    }
}

static void solve_in(Workspace &ws, const feast_opts &o, const SolveArgs &a, SolveOut &so)
{
    Result out;
    if (a.device) {
        Problem pb{a.n, static_cast<const double *>(a.A), a.lda, static_cast<const double *>(a.B), a.ldb, a.emin,
                   a.emax, a.m0, static_cast<double *>(a.X), a.ldx};
        const int info = dispatch(a.cplx, pb, o, a.stream, ws, out, so.st);
        copy_outputs(out, info, a, so);
        return;
    }
    const size_t es = a.cplx ? 16 : 8;
    const int N = a.n;
    int info;
    try {
        ws.init();
        hipStream_t s = ws.stream;
        void *dA = ws.get("in_A", es * (size_t)N * N);
        void *dB = a.B ? ws.get("in_B", es * (size_t)N * N) : nullptr;
        void *dX = ws.get("in_X", es * (size_t)N * a.m0);
        // blocking uploads: each has landed before any kernel of the solve is
        // launched (an asynchronous copy from pageable memory was seen to be
        // overtaken by the stream's kernels under a profiler)
        upload_cols(dA, a.A, es * a.lda, es * N, N);
        if (a.B) upload_cols(dB, a.B, es * a.ldb, es * N, N);
        if (o.x0) upload_cols(dX, a.X, es * a.ldx, es * N, a.m0);
        Problem pb{N, static_cast<const double *>(dA), N, static_cast<const double *>(dB), N, a.emin, a.emax, a.m0,
                   static_cast<double *>(dX), N};
        info = dispatch(a.cplx, pb, o, s, ws, out, so.st);
        if (info == 0 || info == 1 || info == 2 || info == 3 || info == 4 || info == 5) {
            const int mo = (info == 4 || info == 5) ? a.m0 : out.m0;
            download_cols(a.X, es * a.ldx, dX, es * N, mo, s);
        }
    } catch (const alloc_error &) {
        info = -1;
    } catch (const hip_error &e) {
        std::fprintf(stderr, "feastx: HIP error %s\n", hipGetErrorString(e.code));
        info = -4;
    }
    copy_outputs(out, info, a, so);
}

// Bytes of device memory one solve holds (factors, solve panels, FP64
// subspace blocks, staged inputs), for admission decisions.
static double footprint_bytes(bool cplx, int n, int m0, const feast_opts &o, bool staged)
{
    const double vb = (o.precision == 1) ? 8.0 : 16.0;   // complex factor element
    const double eb = cplx ? 16.0 : 8.0;                  // FP64 element
    const double nn = (double)n * n, nm = (double)n * m0, mm = (double)m0 * m0;
    double b = 2.0 * o.ne * nn * vb;                      // factors and their solve form W
    b += o.ne * nm * vb * (cplx ? 4.0 : 2.0);             // solve panels
    b += o.ne * (double)n * 448.0 * vb;                   // inverted diagonal blocks (64 and 128 wide)
    b += 7.0 * nm * eb + 16.0 * mm * eb;                  // subspace blocks, reduced problem
    if (staged) b += 2.0 * nn * eb + nm * eb;             // copies of A, B, X
    if (o.precision == 1)                                 // up to two nodes in complex128 (fp64_nodes)
        b += 2.0 * (2.0 * nn * 16.0 + (double)n * 448.0 * 16.0 + nm * 16.0 * (cplx ? 4.0 : 2.0));
    return b;
}

}  // namespace fx

namespace fx {
// Device scratch of the no-allocation entry point: one copy per device,
// held until the process ends.  Host code never uses the name itself (a
// host-side stand-in); it takes the device address from
// hipGetSymbolAddress at each device's set-up.
static __device__ __align__(256) unsigned char scratch[FEASTX_NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 16;
struct NoAllocDevice {
    std::mutex mu;              // calls on one device take turns (they share its scratch)
    void *ptr = nullptr;        // device address of this device's scratch
    Workspace ws;               // fixed-arena workspace over it
    alignas(256) unsigned char host[1 << 18];   // read-back staging (plain host memory)
};
static NoAllocDevice g_noalloc[NOALLOC_MAX_DEVICES];
}  // namespace fx

// Per-launch timing hook of the complex matrix products (feast_set_timing).
// Events come from a pool created once per thread, so the hook only records.
namespace fx {
static thread_local std::vector<hipEvent_t> t_event_pool;
static thread_local size_t t_event_next = 0;
static hipEvent_t pooled_event()
{
    if (t_event_next == t_event_pool.size()) {
        hipEvent_t e;
        FX_CHECK(hipEventCreate(&e));
        t_event_pool.push_back(e);
    }
    return t_event_pool[t_event_next++];
}
void gemm_timing_begin(hipStream_t s, hipEvent_t *e, bool f64)
{
    if (!g_gemm_timer || f64 != g_gemm_timer->f64) return;
    *e = pooled_event();
    FX_CHECK(hipEventRecord(*e, s));
}
void gemm_timing_end(hipStream_t s, hipEvent_t e0, double flops, bool f64)
{
    if (!g_gemm_timer || f64 != g_gemm_timer->f64) return;
    hipEvent_t e1 = pooled_event();
    FX_CHECK(hipEventRecord(e1, s));
    g_gemm_timer->ev.push_back({e0, e1});
    g_gemm_timer->in_lu.push_back(g_gemm_timer->lu ? 1 : 0);
    g_gemm_timer->flops += flops;
    if (g_gemm_timer->lu) g_gemm_timer->lu_flops += flops;
}
void gemm_timing_reset() { t_event_next = 0; }
}  // namespace fx

#include "tune.hpp"

// ======================================================================
//            concurrent executor: batched solves and the server
// ======================================================================
namespace fx {

// Slots share nothing on the device: each has its own stream and workspace,
// and no kernel of the library waits for another workgroup, so their work
// interleaves freely.

// Most concurrent slots of one executor.  Runs of 256 uneven problems have
// completed with 8 slots in both precisions.  One FP64 run with 16 slots
// stalled, with the earlier grid-barrier eigensolver, and no cause was
// established, so larger requests are clamped to 8.
constexpr int MAX_SLOTS = 8;

struct Job {
    SolveArgs args{};
    feast_opts opts{};
    SolveOut out;
    double footprint = 0;
    std::chrono::steady_clock::time_point t_submit, t_start, t_end;
    bool done = false;
    unsigned long long id = 0;
    // server-owned host buffers
    std::vector<double> E, res;
    std::vector<unsigned char> X;
    std::vector<feast_z> zne, wne;   // copies of custom contour nodes and weights
};

class Executor {
  public:
    Executor(int slots, double budget_bytes) : budget_(budget_bytes)
    {
        FX_CHECK(hipGetDevice(&device_));
        for (int i = 0; i < slots; ++i) ws_.emplace_back(new Workspace());
        for (int i = 0; i < slots; ++i) threads_.emplace_back([this, i] { worker(i); });
    }
    ~Executor()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stopping_ = true;
        }
        cv_work_.notify_all();
        for (auto &t : threads_) t.join();
        for (auto &w : ws_) w->release();
    }
    void submit(const std::shared_ptr<Job> &j)
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            j->t_submit = std::chrono::steady_clock::now();
            queue_.push_back(j);
        }
        cv_work_.notify_all();
    }
    void wait(const std::shared_ptr<Job> &j)
    {
        std::unique_lock<std::mutex> lk(mu_);
        cv_done_.wait(lk, [&] { return j->done; });
    }
    bool is_done(const std::shared_ptr<Job> &j)
    {
        std::lock_guard<std::mutex> lk(mu_);
        return j->done;
    }

  private:
    void worker(int slot)
    {
        (void)hipSetDevice(device_);
        Workspace &ws = *ws_[slot];
        for (;;) {
            std::shared_ptr<Job> j;
            {
                std::unique_lock<std::mutex> lk(mu_);
                // FIFO admission: the oldest request runs once its footprint
                // fits next to the running ones (or nothing else runs)
                cv_work_.wait(lk, [&] {
                    return stopping_ ||
                           (!queue_.empty() && (in_use_ + queue_.front()->footprint <= budget_ || running_ == 0));
                });
                if (queue_.empty()) {
                    if (stopping_) return;
                    continue;
                }
                j = queue_.front();
                queue_.pop_front();
                in_use_ += j->footprint;
                ++running_;
            }
            j->t_start = std::chrono::steady_clock::now();
            j->args.stream = nullptr;   // the slot's own stream
            solve_in(ws, j->opts, j->args, j->out);
            j->t_end = std::chrono::steady_clock::now();
            // keep a slot's workspace near the size of what it runs
            // (a freed buffer synchronises the device, so only a large excess is given back)
            if (ws.bytes() > 2.0 * j->footprint + 4096.0 * (1 << 20)) ws.trim();
            {
                std::lock_guard<std::mutex> lk(mu_);
                in_use_ -= j->footprint;
                --running_;
                j->done = true;
            }
            cv_done_.notify_all();
            cv_work_.notify_all();
        }
    }

    std::vector<std::unique_ptr<Workspace>> ws_;
    std::vector<std::thread> threads_;
    std::deque<std::shared_ptr<Job>> queue_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    bool stopping_ = false;
    double budget_, in_use_ = 0;
    int running_ = 0;
    int device_ = 0;
};

static double ms_between(std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace fx

struct feast_server {
    std::unique_ptr<fx::Executor> ex;
    std::mutex mu;
    std::map<unsigned long long, std::shared_ptr<fx::Job>> jobs;
    unsigned long long next_id = 1;
};

// ======================================================================
//                                C interface
// ======================================================================
using fx::Problem;
using fx::Result;

extern "C" {

void feast_default_opts(feast_opts *o)
{
    if (!o) return;
    o->ne = 8;
    o->maxloop = 20;
    o->conv = 1;
    o->x0 = 0;
    o->keep_factors = 1;
    o->precision = 0;
    o->refine = 0;
    o->mode = 0;
    o->verbose = 0;
    o->tol = 1e-12;
    o->seed = 0x5eedULL;
    o->integration = 0;
    o->ellipse = 100;
    o->Zne = nullptr;
    o->Wne = nullptr;
    o->ne_full = 16;
    o->integration_full = 1;
    o->angle = 0;
}

const char *feast_version(void) { return "feastx 0.1 (gfx950)"; }

static int contour_args(double emin, double emax, int ne, int integration, int ellipse)
{
    if (ne < 1) return 102;
    if (integration != 0 && integration != 1) return 116;
    if (ellipse < 1) return 118;
    if (!(emin < emax) || !std::isfinite(emin) || !std::isfinite(emax)) return 200;
    return 0;
}

static void eval_rational(const fx::Contour &c, const double *eig, int m, double *f)
{
    const int ne = (int)c.z.size();
    for (int i = 0; i < m; ++i) {
        double acc = 0.0;
        for (int j = 0; j < ne; ++j) {
            // Re( w / (z - lambda) )
            const double dr = c.z[j].x - eig[i], di = c.z[j].y;
            const double den = dr * dr + di * di;
            acc += (c.w[j].x * dr + c.w[j].y * di) / den;
        }
        f[i] = acc;
    }
}

int feast_contour(double emin, double emax, int ne, int integration, int ellipse, feast_z *Zne, feast_z *Wne)
{
    const int v = contour_args(emin, emax, ne, integration, ellipse);
    if (v) return v;
    if (!Zne) return -105;
    if (!Wne) return -106;
    fx::Contour c = fx::make_contour(emin, emax, ne, integration, ellipse);
    for (int j = 0; j < ne; ++j) {
        Zne[j].re = c.z[j].x;
        Zne[j].im = c.z[j].y;
        Wne[j].re = c.w[j].x;
        Wne[j].im = c.w[j].y;
    }
    return 0;
}

int feast_rational(double emin, double emax, int ne, int integration, int ellipse, const double *eig, int m,
                   double *f)
{
    const int v = contour_args(emin, emax, ne, integration, ellipse);
    if (v) return v;
    if (m < 0) return -107;
    if (m > 0 && (!eig || !f)) return -108;
    eval_rational(fx::make_contour(emin, emax, ne, integration, ellipse), eig, m, f);
    return 0;
}

int feast_rationalx(const feast_z *Zne, const feast_z *Wne, int ne, const double *eig, int m, double *f)
{
    if (ne < 1) return 102;
    if (!Zne || !Wne) return -101;
    if (m < 0) return -105;
    if (m > 0 && (!eig || !f)) return -106;
    eval_rational(fx::custom_contour(Zne, Wne, ne), eig, m, f);
    return 0;
}

// Checks shared by the single-problem entry points; 0 if the call may run.
static int check_args(int N, int M0, double Emin, double Emax, const feast_opts &o, const void *A, int lda,
                      const void *B, int ldb, const void *X, int ldx, const double *E, const double *res,
                      const int *M)
{
    int v = fx::validate(N, M0, Emin, Emax, o);
    if (v) return v;
    if (!A) return -102;
    if (lda < N) return -103;
    if (B && ldb < N) return -105;
    if (!X) return -111;
    if (ldx < N) return -112;
    if (!E || !res || !M) return -110;
    return 0;
}

static int solve_single(bool cplx, int device, int N, const void *A, int lda, const void *B, int ldb, double Emin,
                        double Emax, int *M0, const feast_opts *opts, double *E, void *X, int ldx, int *M,
                        double *res, int *loop, double *epsout, void *stream)
{
    if (!M0) return -108;
    feast_opts o;
    if (opts) o = *opts;
    else feast_default_opts(&o);
    int v = check_args(N, *M0, Emin, Emax, o, A, lda, B, ldb, X, ldx, E, res, M);
    if (v) return v;
    fx::SolveArgs a{cplx, N, A, lda, B, ldb, Emin, Emax, *M0, X, ldx, E, res, device,
                    static_cast<hipStream_t>(stream)};
    fx::SolveOut so;
    fx::Workspace &ws = fx::thread_ws();
    ws.want_split = true;
    ws.lookahead = true;
    fx::solve_in(ws, o, a, so);
    fx::t_stats = so.st;
    if (so.info == 0 || so.info == 1 || so.info == 2 || so.info == 3 || so.info == 4 || so.info == 5) {
        *M = so.M;
        *M0 = so.m0;
        if (loop) *loop = so.loop;
        if (epsout) *epsout = so.epsout;
    }
    return so.info;
}

int feast_solve_d_dev(int N, const double *dA, int lda, const double *dB, int ldb, double Emin, double Emax,
                      int *M0, const feast_opts *opts, double *E, double *dX, int ldx, int *M, double *res,
                      int *loop, double *epsout, void *stream)
{
    return solve_single(false, 1, N, dA, lda, dB, ldb, Emin, Emax, M0, opts, E, dX, ldx, M, res, loop, epsout,
                        stream);
}

int feast_solve_z_dev(int N, const feast_z *dA, int lda, const feast_z *dB, int ldb, double Emin, double Emax,
                      int *M0, const feast_opts *opts, double *E, feast_z *dX, int ldx, int *M, double *res,
                      int *loop, double *epsout, void *stream)
{
    return solve_single(true, 1, N, dA, lda, dB, ldb, Emin, Emax, M0, opts, E, dX, ldx, M, res, loop, epsout,
                        stream);
}

// ---- the no-allocation variant of feast_solve_d_dev: every device buffer of
// the solve is carved out of `scratch`, a static array on each device, and
// host read-backs go through a static host block per device.
static int solve_d_dev_noalloc(int N, const double *dA, int lda, const double *dB, int ldb, double Emin,
                               double Emax, int *M0, const feast_opts *opts, double *E, double *dX, int ldx, int *M,
                               double *res, int *loop, double *epsout, void *stream)
{
    if (!M0) return -108;
    feast_opts o;
    if (opts) o = *opts;
    else feast_default_opts(&o);
    int v = check_args(N, *M0, Emin, Emax, o, dA, lda, dB, ldb, dX, ldx, E, res, M);
    if (v) return v;
    const double need = fx::footprint_bytes(false, N, *M0, o, false);
    if (need > (double)FEASTX_NOALLOC_SCRATCH_BYTES) {
        std::fprintf(stderr,
                     "feastx: feast_solve_d_dev_noalloc: N=%d, M0=%d, ne=%d needs about %.0f MiB of device "
                     "workspace; its fixed scratch holds %llu MiB (use feast_solve_d_dev)\n",
                     N, *M0, o.ne, need / (1 << 20), (unsigned long long)(FEASTX_NOALLOC_SCRATCH_BYTES >> 20));
        return -1;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= fx::NOALLOC_MAX_DEVICES) return -4;
    fx::NoAllocDevice &d = fx::g_noalloc[dev];
    std::lock_guard<std::mutex> lk(d.mu);
    if (!d.ptr) {
        // set-up on this device (current): the device address of its copy of
        // the scratch array; the array's name is a host-side stand-in
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(fx::scratch));
        if (e != hipSuccess || !p) {
            std::fprintf(stderr, "feastx: hipGetSymbolAddress(scratch) failed on device %d: %s\n", dev,
                         hipGetErrorString(e));
            return -4;
        }
        d.ptr = p;
        d.ws.noalloc = true;
        d.ws.device = dev;
        d.ws.arena = static_cast<unsigned char *>(p);
        d.ws.arena_cap = FEASTX_NOALLOC_SCRATCH_BYTES;
        d.ws.host_arena = d.host;
        d.ws.host_cap = sizeof(d.host);
    }
    d.ws.reset_arena();
    fx::SolveArgs a{false, N, dA, lda, dB, ldb, Emin, Emax, *M0, dX, ldx, E, res, 1,
                    static_cast<hipStream_t>(stream)};
    fx::SolveOut so;
    fx::solve_in(d.ws, o, a, so);
    fx::t_stats = so.st;
    if (so.info == -1)
        std::fprintf(stderr, "feastx: feast_solve_d_dev_noalloc: the fixed scratch (%llu MiB) ran out\n",
                     (unsigned long long)(FEASTX_NOALLOC_SCRATCH_BYTES >> 20));
    if (so.info == 0 || so.info == 1 || so.info == 2 || so.info == 3 || so.info == 4 || so.info == 5) {
        *M = so.M;
        *M0 = so.m0;
        if (loop) *loop = so.loop;
        if (epsout) *epsout = so.epsout;
    }
    return so.info;
}

int feast_solve_d_dev_noalloc(int N, const double *dA, int lda, const double *dB, int ldb, double Emin, double Emax,
                              int *M0, const feast_opts *opts, double *E, double *dX, int ldx, int *M, double *res,
                              int *loop, double *epsout, void *stream)
{
    return solve_d_dev_noalloc(N, dA, lda, dB, ldb, Emin, Emax, M0, opts, E, dX, ldx, M, res, loop, epsout, stream);
}

int feast_solve_d_ex(int N, const double *A, int lda, const double *B, int ldb, double Emin, double Emax, int *M0,
                     const feast_opts *opts, double *E, double *X, int ldx, int *M, double *res, int *loop,
                     double *epsout)
{
    return solve_single(false, 0, N, A, lda, B, ldb, Emin, Emax, M0, opts, E, X, ldx, M, res, loop, epsout,
                        nullptr);
}

int feast_solve_z_ex(int N, const feast_z *A, int lda, const feast_z *B, int ldb, double Emin, double Emax,
                     int *M0, const feast_opts *opts, double *E, feast_z *X, int ldx, int *M, double *res,
                     int *loop, double *epsout)
{
    return solve_single(true, 0, N, A, lda, B, ldb, Emin, Emax, M0, opts, E, X, ldx, M, res, loop, epsout,
                        nullptr);
}

int feast_solve_d(int N, const double *A, const double *B, double Emin, double Emax, int M0, int Ne, double tol,
                  double *E, double *X, int *M, double *res)
{
    feast_opts o;
    feast_default_opts(&o);
    o.ne = Ne;
    o.tol = tol;
    int m0 = M0;
    return feast_solve_d_ex(N, A, N, B, N, Emin, Emax, &m0, &o, E, X, N, M, res, nullptr, nullptr);
}

int feast_solve_z(int N, const feast_z *A, const feast_z *B, double Emin, double Emax, int M0, int Ne, double tol,
                  double *E, feast_z *X, int *M, double *res)
{
    feast_opts o;
    feast_default_opts(&o);
    o.ne = Ne;
    o.tol = tol;
    int m0 = M0;
    return feast_solve_z_ex(N, A, N, B, N, Emin, Emax, &m0, &o, E, X, N, M, res, nullptr, nullptr);
}

// ---------------------------------------------------------------- batched
static int solve_batched(bool cplx, int njobs, feast_job *jobs, const feast_opts *opts, int device,
                         int concurrency)
{
    if (njobs < 0) return -101;
    if (njobs > 0 && !jobs) return -102;
    if (device != 0 && device != 1) return -104;
    feast_opts o;
    if (opts) o = *opts;
    else feast_default_opts(&o);
    if (concurrency <= 0) concurrency = 4;
    concurrency = std::min(concurrency, fx::MAX_SLOTS);
    std::vector<std::shared_ptr<fx::Job>> js(njobs);
    try {
        fx::Executor ex(std::min(concurrency, std::max(njobs, 1)), 1e300);
        for (int i = 0; i < njobs; ++i) {
            feast_job &q = jobs[i];
            q.info = check_args(q.n, q.m0, q.emin, q.emax, o, q.A, q.lda, q.B, q.ldb, q.X, q.ldx, q.E, q.res,
                                &q.M);
            if (q.info) continue;
            auto j = std::make_shared<fx::Job>();
            j->args = fx::SolveArgs{cplx, q.n, q.A, q.lda, q.B, q.ldb, q.emin, q.emax, q.m0, q.X, q.ldx, q.E, q.res,
                                    device, nullptr};
            j->opts = o;
            j->footprint = fx::footprint_bytes(cplx, q.n, q.m0, o, device == 0);
            js[i] = j;
            ex.submit(j);
        }
        for (int i = 0; i < njobs; ++i) {
            if (!js[i]) continue;
            ex.wait(js[i]);
            feast_job &q = jobs[i];
            const fx::SolveOut &so = js[i]->out;
            q.info = so.info;
            q.M = so.M;
            q.m0_out = so.m0;
            q.loop = so.loop;
            q.epsout = so.epsout;
            q.ms = fx::ms_between(js[i]->t_submit, js[i]->t_end);
        }
    } catch (const fx::hip_error &e) {
        std::fprintf(stderr, "feastx: HIP error %s\n", hipGetErrorString(e.code));
        return -4;
    }
    return 0;
}

int feast_solve_batched_d(int njobs, feast_job *jobs, const feast_opts *opts, int device, int concurrency)
{
    return solve_batched(false, njobs, jobs, opts, device, concurrency);
}

int feast_solve_batched_z(int njobs, feast_job *jobs, const feast_opts *opts, int device, int concurrency)
{
    return solve_batched(true, njobs, jobs, opts, device, concurrency);
}

// ---------------------------------------------------------------- non-Hermitian
static int gsolve(bool real_in, int N, const void *A, int lda, const void *B, int ldb, feast_z Emid, double r,
                  int *M0, const feast_opts *opts, feast_z *E, feast_z *X, int ldx, int *M, double *res, int *loop,
                  double *epsout, bool device = false, void *stream = nullptr)
{
    if (!M0) return -108;
    feast_opts o;
    if (opts) o = *opts;
    else feast_default_opts(&o);
    const double2 emid = make_double2(Emid.re, Emid.im);
    int v = fx::validate_general(N, *M0, emid, r, o);
    if (v) return v;
    if (!A) return -102;
    if (lda < N) return -103;
    if (B && ldb < N) return -105;
    if (!E) return -110;
    if (!X) return -111;
    if (ldx < N) return -112;
    if (!M) return -113;
    if (!res) return -114;
    const int m0 = *M0;
    fx::Workspace &ws = fx::thread_ws();
    fx::GResult out;
    feast_stats st{};
    int info;
    try {
        ws.init();
        if (device) {   // A, B, X already in HBM, on the caller's stream
            hipStream_t s = stream ? static_cast<hipStream_t>(stream) : ws.stream;
            fx::GProblem pb{N, reinterpret_cast<const double2 *>(A), lda, reinterpret_cast<const double2 *>(B), ldb,
                            emid, r, m0, reinterpret_cast<double2 *>(X), ldx};
            try {
                info = o.precision == 1 ? fx::run_general<float>(pb, o, s, ws, out, st)
                                    : fx::run_general<double>(pb, o, s, ws, out, st);
            } catch (const fx::solver_error &e) {
                (void)hipStreamSynchronize(s);
                info = e.info;
            }
        } else {
        hipStream_t s = ws.stream;
        const size_t nn = (size_t)N * N, es = sizeof(double2);
        double2 *dA = static_cast<double2 *>(ws.get("in_A", es * nn));
        double2 *dB = B ? static_cast<double2 *>(ws.get("in_B", es * nn)) : nullptr;
        double2 *dX = static_cast<double2 *>(ws.get("in_X", es * (size_t)N * 2 * m0));
        if (real_in) {
            // real input: widened to complex on the host (argument marshalling)
            std::vector<double2> tmp(nn);
            const double *Ar = static_cast<const double *>(A);
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) tmp[i + (size_t)j * N] = make_double2(Ar[i + (size_t)j * lda], 0.0);
            FX_CHECK(hipMemcpy(dA, tmp.data(), es * nn, hipMemcpyHostToDevice));
            if (B) {
                const double *Br = static_cast<const double *>(B);
                for (int j = 0; j < N; ++j)
                    for (int i = 0; i < N; ++i) tmp[i + (size_t)j * N] = make_double2(Br[i + (size_t)j * ldb], 0.0);
                FX_CHECK(hipMemcpy(dB, tmp.data(), es * nn, hipMemcpyHostToDevice));
            }
        } else {
            fx::upload_cols(dA, A, es * lda, es * N, N);
            if (B) fx::upload_cols(dB, B, es * ldb, es * N, N);
        }
        // blocking upload, as in the Hermitian host path
        if (o.x0) fx::upload_cols(dX, X, es * ldx, es * N, 2 * m0);
        fx::GProblem pb{N, dA, N, dB, N, emid, r, m0, dX, N};
        try {
            info = o.precision == 1 ? fx::run_general<float>(pb, o, s, ws, out, st)
                                    : fx::run_general<double>(pb, o, s, ws, out, st);
        } catch (const fx::solver_error &e) {
            (void)hipStreamSynchronize(s);
            info = e.info;
        }
        if (info >= 0 && info <= 3) {
            fx::download_cols(X, es * ldx, dX, es * N, 2 * m0, s);
        }
        }
    } catch (const fx::alloc_error &) {
        info = -1;
    } catch (const fx::hip_error &e) {
        std::fprintf(stderr, "feastx: HIP error %s\n", hipGetErrorString(e.code));
        info = -4;
    }
    fx::t_stats = st;
    if (info >= 0 && info <= 3) {
        for (int i = 0; i < m0; ++i) {
            E[i].re = out.E[i].x;
            E[i].im = out.E[i].y;
            res[i] = out.res[i];
            res[m0 + i] = out.res[m0 + i];
        }
        *M = out.M;
        if (loop) *loop = out.loop;
        if (epsout) *epsout = out.epsout;
    }
    return info;
}

int feast_gsolve_z(int N, const feast_z *A, int lda, const feast_z *B, int ldb, feast_z Emid, double r, int *M0,
                   const feast_opts *opts, feast_z *E, feast_z *X, int ldx, int *M, double *res, int *loop,
                   double *epsout)
{
    return gsolve(false, N, A, lda, B, ldb, Emid, r, M0, opts, E, X, ldx, M, res, loop, epsout);
}

int feast_gsolve_z_dev(int N, const feast_z *dA, int lda, const feast_z *dB, int ldb, feast_z Emid, double r,
                       int *M0, const feast_opts *opts, feast_z *E, feast_z *dX, int ldx, int *M, double *res,
                       int *loop, double *epsout, void *stream)
{
    return gsolve(false, N, dA, lda, dB, ldb, Emid, r, M0, opts, E, dX, ldx, M, res, loop, epsout, true, stream);
}

int feast_gsolve_d(int N, const double *A, int lda, const double *B, int ldb, feast_z Emid, double r, int *M0,
                   const feast_opts *opts, feast_z *E, feast_z *X, int ldx, int *M, double *res, int *loop,
                   double *epsout)
{
    return gsolve(true, N, A, lda, B, ldb, Emid, r, M0, opts, E, X, ldx, M, res, loop, epsout);
}

// ---------------------------------------------------------------- slicing
// Device buffers the slicing call stages into, freed when it returns.
struct StagedBuffers {
    std::vector<void *> p;
    void *get(size_t bytes)
    {
        void *q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(bytes, 256)) != hipSuccess) throw fx::alloc_error{};
        p.push_back(q);
        return q;
    }
    ~StagedBuffers()
    {
        (void)hipDeviceSynchronize();
        for (void *q : p) (void)hipFree(q);
    }
};

// Neighbouring intervals [bounds[s], bounds[s+1]] of one pencil as one batched
// job: A and B live on the device once and every slice's solve reads them.
static int solve_slices(bool cplx, int N, const void *A, int lda, const void *B, int ldb, int nslices,
                        const double *bounds, feast_job *slices, const feast_opts *opts, int device, int concurrency,
                        int auto_m0)
{
    if (N < 1) return 202;
    if (!A) return -102;
    if (lda < N) return -103;
    if (B && ldb < N) return -105;
    if (nslices < 1) return -106;
    if (!bounds) return -107;
    if (!slices) return -108;
    if (device != 0 && device != 1) return -110;
    for (int s = 0; s < nslices; ++s)
        if (!(bounds[s] < bounds[s + 1])) return 200;
    feast_opts o;
    if (opts) o = *opts;
    else feast_default_opts(&o);
    if (auto_m0) o.x0 = 0;
    const size_t es = cplx ? 16 : 8;
    std::vector<int> cap(nslices);
    for (int s = 0; s < nslices; ++s) {
        cap[s] = slices[s].m0;
        if (cap[s] < 1 || cap[s] > N) return 201;
        if (!slices[s].X || !slices[s].E || !slices[s].res) return -108;
        if (slices[s].ldx < N) return -108;
    }
    try {
        StagedBuffers st;
        const void *dA = A, *dB = B;
        if (!device) {
            void *a = st.get(es * (size_t)N * N);
            fx::upload_cols(a, A, es * lda, es * N, N);
            dA = a;
            if (B) {
                void *b = st.get(es * (size_t)N * N);
                fx::upload_cols(b, B, es * ldb, es * N, N);
                dB = b;
            }
        }
        std::vector<feast_job> jobs(nslices);
        std::vector<void *> dX(nslices);
        for (int s = 0; s < nslices; ++s) {
            feast_job &q = slices[s];
            q.n = N;
            q.A = A;
            q.lda = lda;
            q.B = B;
            q.ldb = ldb;
            q.emin = bounds[s];
            q.emax = bounds[s + 1];
            if (device) {
                dX[s] = q.X;
            } else {
                dX[s] = st.get(es * (size_t)N * cap[s]);
                if (o.x0)
                    fx::upload_cols(dX[s], q.X, es * q.ldx, es * N, cap[s]);
            }
            feast_job &j = jobs[s];
            j = q;
            j.A = dA;
            j.lda = device ? lda : N;
            j.B = dB;
            j.ldb = device ? ldb : N;
            j.X = dX[s];
            j.ldx = device ? q.ldx : N;
        }
        std::vector<int> m0(cap);
        if (auto_m0) {
            // stochastic count estimate per slice: 16 +-1 probes, 3 nodes
            feast_opts oe = o;
            oe.mode = 2;
            oe.ne = 3;
            oe.integration = 0;
            oe.ellipse = 100;
            oe.Zne = oe.Wne = nullptr;
            const int pm = std::min(16, N);
            std::vector<feast_job> ej(jobs);
            std::vector<double> eE((size_t)nslices * pm), eres((size_t)nslices * pm);
            for (int s = 0; s < nslices; ++s) {
                ej[s].m0 = pm;
                ej[s].X = st.get(es * (size_t)N * pm);
                ej[s].ldx = N;
                ej[s].E = eE.data() + (size_t)s * pm;
                ej[s].res = eres.data() + (size_t)s * pm;
            }
            int rc = solve_batched(cplx, nslices, ej.data(), &oe, 1, concurrency);
            if (rc) return rc;
            for (int s = 0; s < nslices; ++s) {
                if (ej[s].info != 5) {
                    slices[s].info = ej[s].info;
                    m0[s] = 0;
                    continue;
                }
                const int want = std::max(8, (int)std::ceil(1.5 * ej[s].M + 4.0));
                m0[s] = std::min(cap[s], want);
            }
        }
        // the solves, then (auto_m0) slices that ran out of subspace again
        // with twice the subspace, up to the caller's capacity
        std::vector<int> todo;
        for (int s = 0; s < nslices; ++s)
            if (m0[s] > 0) todo.push_back(s);
        while (!todo.empty()) {
            std::vector<feast_job> run(todo.size());
            for (size_t t = 0; t < todo.size(); ++t) {
                run[t] = jobs[todo[t]];
                run[t].m0 = m0[todo[t]];
            }
            int rc = solve_batched(cplx, (int)run.size(), run.data(), &o, 1, concurrency);
            if (rc) return rc;
            std::vector<int> again;
            for (size_t t = 0; t < todo.size(); ++t) {
                const int s = todo[t];
                feast_job &q = slices[s];
                q.info = run[t].info;
                q.M = run[t].M;
                q.m0_out = run[t].m0_out;
                q.loop = run[t].loop;
                q.epsout = run[t].epsout;
                q.ms = run[t].ms;
                if (auto_m0 && q.info == 3 && m0[s] < cap[s]) {
                    m0[s] = std::min(cap[s], 2 * m0[s]);
                    again.push_back(s);
                }
            }
            todo.swap(again);
        }
        if (!device) {
            FX_CHECK(hipDeviceSynchronize());
            for (int s = 0; s < nslices; ++s) {
                feast_job &q = slices[s];
                const int i = q.info;
                if (i == 0 || i == 1 || i == 2 || i == 3)
                    fx::download_cols(q.X, es * q.ldx, dX[s], es * N, q.m0_out, nullptr);
            }
        }
    } catch (const fx::alloc_error &) {
        return -1;
    } catch (const fx::hip_error &e) {
        std::fprintf(stderr, "feastx: HIP error %s\n", hipGetErrorString(e.code));
        return -4;
    }
    return 0;
}

int feast_solve_slices_d(int N, const double *A, int lda, const double *B, int ldb, int nslices,
                         const double *bounds, feast_job *slices, const feast_opts *opts, int device, int concurrency,
                         int auto_m0)
{
    return solve_slices(false, N, A, lda, B, ldb, nslices, bounds, slices, opts, device, concurrency, auto_m0);
}

int feast_solve_slices_z(int N, const feast_z *A, int lda, const feast_z *B, int ldb, int nslices,
                         const double *bounds, feast_job *slices, const feast_opts *opts, int device, int concurrency,
                         int auto_m0)
{
    return solve_slices(true, N, A, lda, B, ldb, nslices, bounds, slices, opts, device, concurrency, auto_m0);
}

// ---------------------------------------------------------------- server
feast_server *feast_server_create(const feast_server_cfg *cfg)
{
    int slots = cfg && cfg->slots > 0 ? std::min(cfg->slots, fx::MAX_SLOTS) : 4;
    double budget = (cfg && cfg->hbm_budget_gb > 0 ? cfg->hbm_budget_gb : 64.0) * 1e9;
    try {
        auto *srv = new feast_server();
        srv->ex.reset(new fx::Executor(slots, budget));
        return srv;
    } catch (...) {
        return nullptr;
    }
}

int feast_server_submit(feast_server *srv, const feast_request *req, unsigned long long *id)
{
    if (!srv) return -101;
    if (!req) return -102;
    if (!id) return -103;
    const feast_request &r = *req;
    const bool cplx = r.hermitian != 0;
    feast_opts o = r.opts;
    o.x0 = r.X0 ? 1 : 0;
    auto j = std::make_shared<fx::Job>();
    const size_t es = cplx ? 16 : 8;
    if (r.m0 >= 1 && r.n >= 1) {
        j->E.assign(r.m0, 0.0);
        j->res.assign(r.m0, 0.0);
        j->X.assign(es * (size_t)r.n * r.m0, 0);
        if (r.X0)
            for (int c = 0; c < r.m0; ++c)
                std::memcpy(j->X.data() + es * (size_t)r.n * c,
                            static_cast<const unsigned char *>(r.X0) + es * (size_t)r.ldx * c, es * r.n);
    }
    int v = check_args(r.n, r.m0, r.emin, r.emax, o, r.A, r.lda, r.B, r.ldb, j->X.empty() ? nullptr : j->X.data(),
                       r.n, j->E.empty() ? nullptr : j->E.data(), j->res.empty() ? nullptr : j->res.data(),
                       &j->out.M);
    if (v) return v;
    j->args = fx::SolveArgs{cplx, r.n, r.A, r.lda, r.B, r.ldb, r.emin, r.emax, r.m0, j->X.data(), r.n,
                            j->E.data(), j->res.data(), 0, nullptr};
    if (o.Zne) {   // the request's node arrays need not outlive the call
        j->zne.assign(o.Zne, o.Zne + o.ne);
        j->wne.assign(o.Wne, o.Wne + o.ne);
        o.Zne = j->zne.data();
        o.Wne = j->wne.data();
    }
    j->opts = o;
    j->footprint = fx::footprint_bytes(cplx, r.n, r.m0, o, true);
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        j->id = srv->next_id++;
        srv->jobs[j->id] = j;
    }
    *id = j->id;
    srv->ex->submit(j);
    return 0;
}

static void fill_result(const fx::Job &j, feast_result *out)
{
    const fx::SolveOut &so = j.out;
    out->info = so.info;
    out->M = so.M;
    out->m0 = so.m0;
    out->loop = so.loop;
    out->epsout = so.epsout;
    out->queue_ms = fx::ms_between(j.t_submit, j.t_start);
    out->run_ms = fx::ms_between(j.t_start, j.t_end);
    out->latency_ms = fx::ms_between(j.t_submit, j.t_end);
    const int m = so.m0;
    const size_t es = j.args.cplx ? 16 : 8;
    const int n = j.args.n;
    if (out->E)
        for (int i = 0; i < m; ++i) out->E[i] = j.E[i];
    if (out->res)
        for (int i = 0; i < m; ++i) out->res[i] = j.res[i];
    if (out->X)
        for (int c = 0; c < m; ++c)
            std::memcpy(static_cast<unsigned char *>(out->X) + es * (size_t)out->ldx * c,
                        j.X.data() + es * (size_t)n * c, es * n);
}

static int server_take(feast_server *srv, unsigned long long id, feast_result *out, bool block)
{
    if (!srv) return -101;
    if (!out) return -103;
    std::shared_ptr<fx::Job> j;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->jobs.find(id);
        if (it == srv->jobs.end()) return -102;
        j = it->second;
    }
    if (block) srv->ex->wait(j);
    else if (!srv->ex->is_done(j)) return 1;
    fill_result(*j, out);
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->jobs.erase(id);
    return 0;
}

int feast_server_poll(feast_server *srv, unsigned long long id, feast_result *out)
{
    return server_take(srv, id, out, false);
}

int feast_server_wait(feast_server *srv, unsigned long long id, feast_result *out)
{
    return server_take(srv, id, out, true);
}

void feast_server_destroy(feast_server *srv)
{
    if (!srv) return;
    srv->ex.reset();   // drains queued requests, joins the workers
    delete srv;
}

int feast_last_stats(feast_stats *st)
{
    if (!st) return -101;
    *st = fx::t_stats;
    return 0;
}

void feast_set_timing(int on)
{
    fx::g_timing = on != 0;
}

int feast_autotune(int n, int m0, int ne, feast_tiles *out)
{
    if (n < 64) return 202;
    if (m0 < 1) return 201;
    if (ne < 1) return 102;
    try {
        fx::TileTimes tt = fx::autotune(n, m0, ne);
        feast_tiles t{};
        for (int p = 0; p < 2; ++p)
            for (int c = 0; c < fx::GEMM_CLASSES; ++c) {
                t.choice[p][c] = fx::g_tiles[p][c].load();
                for (int v = 0; v < fx::GEMM_VARIANTS; ++v) t.tflops[p][c][v] = tt.tf[p][c][v];
            }
        if (out) *out = t;
        return 0;
    } catch (const fx::alloc_error &) {
        return -1;
    } catch (const fx::hip_error &e) {
        std::fprintf(stderr, "feastx: HIP error %s in feast_autotune\n", hipGetErrorString(e.code));
        return -4;
    }
}

int feast_set_lu_form(int form)
{
    if (form < -1 || form > 1) return -1;
    fx::g_lu_form.store(form);
    return 0;
}

int feast_get_lu_form(void) { return fx::g_lu_form.load(); }

int feast_lu_schedule(int n, int side, int form, int *ops, int cap)
{
    if (n < 1 || form < -1 || form > 1) return -1;
    const std::vector<fx::LuOp> v = fx::lu_schedule(n, side != 0, form);
    if (ops && cap > 0) {
        const int m = std::min(cap, (int)v.size());
        for (int i = 0; i < m; ++i) {
            const fx::LuOp &o = v[i];
            const int row[fx::LU_OP_INTS] = {o.kind, o.side, o.k, o.nbw, o.c0, o.c1,
                                             o.c2,   o.c3,   o.kc0, o.kc1, o.mode, o.list};
            std::copy(row, row + fx::LU_OP_INTS, ops + (size_t)i * fx::LU_OP_INTS);
        }
    }
    return (int)v.size();
}

void feast_get_tiles(feast_tiles *out)
{
    if (!out) return;
    *out = feast_tiles{};
    for (int p = 0; p < 2; ++p)
        for (int c = 0; c < fx::GEMM_CLASSES; ++c) out->choice[p][c] = fx::g_tiles[p][c].load();
}

int feast_set_tiles(const feast_tiles *t)
{
    if (!t) return -101;
    for (int p = 0; p < 2; ++p)
        for (int c = 0; c < fx::GEMM_CLASSES; ++c)
            if (t->choice[p][c] < 0 || t->choice[p][c] >= fx::GEMM_VARIANTS) return -101;
    for (int p = 0; p < 2; ++p)
        for (int c = 0; c < fx::GEMM_CLASSES; ++c) fx::g_tiles[p][c].store(t->choice[p][c]);
    return 0;
}

void feast_release(void)
{
    if (!fx::t_ws) return;
    fx::t_ws->release();
    delete fx::t_ws;
    fx::t_ws = nullptr;
}

}  // extern "C"
