// C ABI of the mfdkc library and the host driver of the band solve.
// The host only orders kernels and reads back a few scalars per iteration
// (Ritz values, residual norms); every step of the method runs on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>
#include <atomic>
#include <initializer_list>
#include <mutex>
#include <thread>

#include "../../include/mfdkc.h"
#include "common.h"
#include "internal.h"
#include "mlp.h"
#include "solver.h"

using namespace mfd;

static thread_local std::string g_last_error;

// Largest block (nbands + guard) of a band solve: the basis of 3 blocks must
// fit the Rayleigh-Ritz step, the Gram and the update kernels.
constexpr int MAX_BLOCK = 22;

static int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

#define HIPCHK(call)                                                                                      \
    do {                                                                                                  \
        hipError_t _e = (call);                                                                           \
        if (_e != hipSuccess)                                                                             \
            return fail(_e == hipErrorOutOfMemory ? MFD_ENOMEM : MFD_EDEVICE,                             \
                        std::string(#call) + ": " + hipGetErrorString(_e));                               \
    } while (0)

// Optional per-kernel timing with HIP events on the solve's stream.
// Categories: 0 stencil, 1 FFT preconditioner, 2 Gram, 3 Rayleigh-Ritz,
// 4 block update, 5 other.
struct Prof {
    static constexpr int NCAT = 6;
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec { int cat; hipEvent_t a, b; double bytes; };
    std::vector<Rec> pending;
    double ms[NCAT] = {0}, bytes[NCAT] = {0};
    long long count[NCAT] = {0};
    hipEvent_t get() {
        if (used == pool.size()) {
            hipEvent_t e;
            hipEventCreate(&e);
            pool.push_back(e);
        }
        return pool[used++];
    }
    hipEvent_t begin(hipStream_t s) {
        if (!on) return nullptr;
        hipEvent_t e = get();
        hipEventRecord(e, s);
        return e;
    }
    void end(hipEvent_t a, int cat, double by, hipStream_t s) {
        if (!on || !a) return;
        hipEvent_t b = get();
        hipEventRecord(b, s);
        pending.push_back({cat, a, b, by});
    }
    // call after a stream synchronisation
    void drain() {
        for (auto& r : pending) {
            float t = 0.f;
            hipEventElapsedTime(&t, r.a, r.b);
            ms[r.cat] += t;
            bytes[r.cat] += r.bytes;
            count[r.cat] += 1;
        }
        pending.clear();
        used = 0;
    }
    void clear() {
        for (int i = 0; i < NCAT; ++i) { ms[i] = 0; bytes[i] = 0; count[i] = 0; }
    }
    void reset() {
        drain();
        clear();
    }
    void add(const Prof& o) {
        for (int i = 0; i < NCAT; ++i) { ms[i] += o.ms[i]; bytes[i] += o.bytes[i]; count[i] += o.count[i]; }
    }
    ~Prof() {
        for (auto e : pool) hipEventDestroy(e);
    }
};

// Band-solve workspace: one per concurrently solved k-path segment or
// crystal, each with its own stream (default priority) and timing.
struct Ws {
    int mb = 0;
    bool mixed = false;
    size_t n = 0;
    float2* V32 = nullptr;     // mixed precision: FP32 W, P, AW, AP (same column positions as V)
    float2* U32 = nullptr;
    float2* stage32 = nullptr; // FP64 workspaces on grids without an FP64 FFT plan: W staged in FP32 (n x mb)
    hipStream_t stream = nullptr;
    double2* V = nullptr;      // n x 6mb: [X | W | P | AX | AW | AP]
    double2* U = nullptr;      // the next V
    double2* gpart = nullptr;
    double2* G = nullptr;
    double2* C = nullptr;
    double* npart = nullptr;
    double* norms = nullptr;
    double* theta = nullptr;
    int* info = nullptr;
    double* cpart = nullptr;
    double* cout = nullptr;
    double* host = nullptr;    // pinned: theta | norms | info | column sums
    int nparts_upd = 0, nparts_gram = 0, nparts_col = 0;
    int cap_upd = 0, cap_gram = 0; // workgroups the npart / gpart buffers hold partials for
    size_t gpart_elems = 0;        // complex elements of gpart
    int stencil_wgs = 2048, fft_xc = 0, upd_rows = 0;   // upd_rows 0: one wave per 16-row strip
    WarmStart* warm = nullptr; // learned warm start (warm_start = 2), allocated on first use
    void* wtmp = nullptr;      // two-pass operator: scratch of this workspace's stream
    MGWork* mg = nullptr;      // multigrid preconditioner work space (precond 1), on first use
    int precond = 0;           // 0 FFT solve, 1 multigrid solve
    bool hardlock = false;     // opts.hard_lock
    double* theta_a = nullptr; // hard locking: Ritz values of the bands still iterating (on first use)
    double2* lpart = nullptr;  // hard locking: per-workgroup partials of X_L^H Y
    double2* lcoef = nullptr;  // hard locking: X_L^H Y
    MGOpts mgo;
    // graph chunks (opts.graph): two LOBPCG iterations captured once per basis
    // shape and replayed; the key is the shape the graph was captured for
    bool graph = false;
    hipGraphExec_t gexec = nullptr;
    std::vector<int> gkey_act;
    double gkey[6] = {0, 0, 0, 0, 0, 0};   // k, gamma, shift
    int gkey_flags = -1;                    // mixed + 2 accurate
    int syncs = 0;             // host synchronisations of the current k-point
    Prof prof;
};

struct mfd_ctx {
    int N = 0;
    double L = 1.0, h = 1.0;
    int order = 2;
    int device = 0;
    void* wtmp = nullptr;      // two-pass operator: scratch for the ABI calls
    int wtmp_bands = 0;
    int lattice = 0;           // general lattice: B[i][j] = N (A^-1)_ji (Section 4.2)
    double B[3][3] = {};
    // launch shapes chosen by the autotuner for one block shape (mb, precision)
    int tune_mb = 0, tune_mixed = -1;   // tune_mb: 0 untuned, -1 pinned by mfd_set_tuning
    int tune[5] = {0, 0, 0, 0, 0};   // Gram workgroups, update workgroups, stencil workgroups, FFT x run,
                                     // update rows per block
    double gamma_override = 0.0;
    double* mu64 = nullptr;
    float* mu32 = nullptr;
    void* tw64 = nullptr;
    void* tw32 = nullptr;
    size_t n = 0;
    std::vector<Ws*> ws;
    MGWork* mg = nullptr;      // multigrid work space of mfd_precond_solve_mg
    bool prof_on = false;
    Prof prof_done;            // timing of finished solves (summed over workspaces)
};

namespace {

__global__ void mu_kernel(const double* __restrict__ eps, int N, double* __restrict__ mu64, float* __restrict__ mu32) {
    const size_t NN = (size_t)N * N, N3 = NN * N;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N3; i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % N), y = (int)((i / N) % N), z = (int)(i / NN);
        const int xm = x ? x - 1 : N - 1, ym = y ? y - 1 : N - 1, zm = z ? z - 1 : N - 1;
        auto E = [&](int a, int b, int c) { return eps[(size_t)c * NN + (size_t)b * N + a]; };
        // Section 4.4: harmonic average of eps^-1 over the four cells sharing the edge
        const double m1 = 4.0 / (E(x, y, z) + E(x, ym, z) + E(x, y, zm) + E(x, ym, zm));
        const double m2 = 4.0 / (E(x, y, z) + E(xm, y, z) + E(x, y, zm) + E(xm, y, zm));
        const double m3 = 4.0 / (E(x, y, z) + E(xm, y, z) + E(x, ym, z) + E(xm, ym, z));
        mu64[i] = m1; mu64[N3 + i] = m2; mu64[2 * N3 + i] = m3;
        mu32[i] = (float)m1; mu32[N3 + i] = (float)m2; mu32[2 * N3 + i] = (float)m3;
    }
}

// M_0 given on the edges: the FP32 copy
__global__ void mu_copy_kernel(const double* __restrict__ mu, size_t count, float* __restrict__ mu32) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        mu32[i] = (float)mu[i];
}

__global__ void twiddle_kernel(int N, double2* tw64, float2* tw32) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    double s, c;
    sincospi(-2.0 * (double)j / (double)N, &s, &c);
    tw64[j] = make_double2(c, s);
    tw32[j] = make_float2((float)c, (float)s);
}

OpParams params(const mfd_ctx* ctx, const double k[3]) {
    OpParams p;
    p.N = ctx->N;
    p.L = ctx->L;
    p.h = ctx->h;
    for (int i = 0; i < 3; ++i) p.k[i] = k[i];
    const double kn = std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    // Near Gamma (|k| < pi / (2L)) the shift of Remark 5.1 is used and |k| in
    // the penalty rule is clamped at pi / (2L): the unclamped |k|^-2 term makes
    // FP64 rounding of gamma B'B x exceed a 1e-8 relative residual there.
    const double kball = M_PI / (2.0 * ctx->L);
    if (ctx->gamma_override > 0.0) {
        p.gamma = ctx->gamma_override;
    } else {
        const double a = ctx->N / (2.0 * M_PI);
        const double b = std::pow(2.0 * M_PI / (ctx->L * std::max(kn, kball)), 2);
        p.gamma = 2.0 * std::max(a, b);
    }
    p.shift = (kn < kball) ? std::pow(M_PI / ctx->L, 2) : 0.0;
    p.order = ctx->order;
    p.wtmp = ctx->wtmp;
    p.wtmp_bands = ctx->wtmp_bands;
    p.lattice = ctx->lattice;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) p.B[i][j] = ctx->B[i][j];
    return p;
}

// Bands of scratch for the two-pass higher-order operator: 4 FP64 complex
// fields per band, at most 8 bands (or 256 MB) per pass.
int wide_bands(int N) {
    const size_t per = 4 * (size_t)N * N * N * sizeof(double2);
    return (int)std::max<size_t>(1, std::min<size_t>(8, (256u << 20) / per));
}

bool finite3(const double* k) { return std::isfinite(k[0]) && std::isfinite(k[1]) && std::isfinite(k[2]); }

void ws_free(Ws* w) {
    if (!w) return;
    hipFree(w->V); hipFree(w->U); hipFree(w->gpart); hipFree(w->G); hipFree(w->C);
    hipFree(w->V32); hipFree(w->U32); hipFree(w->stage32);
    hipFree(w->npart); hipFree(w->norms); hipFree(w->theta); hipFree(w->info);
    hipFree(w->cpart); hipFree(w->cout); hipFree(w->wtmp);
    hipFree(w->theta_a); hipFree(w->lpart); hipFree(w->lcoef);
    mg_destroy(w->mg);
    if (w->gexec) hipGraphExecDestroy(w->gexec);
    if (w->host) hipHostFree(w->host);
    if (w->warm) {
        w->warm->release();
        delete w->warm;
    }
    if (w->stream) hipStreamDestroy(w->stream);
    delete w;
}

int ws_alloc(const mfd_ctx* c, int mb, bool mixed, Ws** out) {
    Ws* w = new Ws();
    *out = nullptr;
    const size_t n = c->n;
    w->mb = mb;
    w->mixed = mixed;
    w->n = n;
    w->nparts_upd = (int)std::min<size_t>(1024, (n + 255) / 256);
    w->nparts_gram = gram_mfma_parts(n);
    // buffers sized for the largest launch shapes the autotuner tries
    // (update: down to 16 rows per block, at most 2048 workgroups; Gram: at most 1024)
    const int max_upd = (int)std::max<size_t>(w->nparts_upd, std::min<size_t>(2048, (n + 15) / 16));
    const int max_gram = (int)std::max<size_t>(w->nparts_gram, std::min<size_t>(1024, (n + 31) / 32));
    w->cap_upd = std::max(max_upd, 1024);
    w->cap_gram = max_gram;
    w->nparts_col = (int)std::min<size_t>(256, (n + 255) / 256);
    const size_t K = 3 * (size_t)mb;
    hipError_t e;
    auto chk = [&](hipError_t r) { e = r; return r == hipSuccess; };
    if (!(chk(hipStreamCreate(&w->stream)) && chk(hipMalloc(&w->V, n * 6 * mb * sizeof(double2))) &&
          chk(hipMalloc(&w->U, n * 6 * mb * sizeof(double2))) &&
          chk(hipMalloc(&w->gpart, (w->gpart_elems = std::max((size_t)max_gram * K * 2 * K,
                                                              gram_mfma_part_elems((int)K, max_gram))) *
                                       sizeof(double2))) &&
          chk(hipMalloc(&w->G, K * 2 * K * sizeof(double2))) && chk(hipMalloc(&w->C, K * mb * sizeof(double2))) &&
          chk(hipMalloc(&w->npart, (size_t)w->cap_upd * 2 * mb * sizeof(double))) &&
          chk(hipMalloc(&w->norms, 2 * mb * sizeof(double))) && chk(hipMalloc(&w->theta, (mb + 1) * sizeof(double))) &&
          chk(hipMalloc(&w->info, 16 * sizeof(int))) &&
          chk(hipMalloc(&w->cpart, (size_t)std::max(w->nparts_col, 1024) * 2 * mb * sizeof(double))) &&
          chk(hipMalloc(&w->cout, 2 * mb * sizeof(double))) &&
          chk(hipHostMalloc(&w->host, (12 * mb + 64) * sizeof(double), hipHostMallocDefault)) &&
          (!mixed || (chk(hipMalloc(&w->V32, n * 6 * mb * sizeof(float2))) &&
                      chk(hipMalloc(&w->U32, n * 6 * mb * sizeof(float2))))) &&
          (mixed || fft_plane_fits(c->N, 8) || chk(hipMalloc(&w->stage32, n * mb * sizeof(float2)))) &&
          (c->order == 2 || chk(hipMalloc(&w->wtmp, (size_t)c->wtmp_bands * 4 * (n / 3) * sizeof(double2)))))) {
        ws_free(w);
        return fail(e == hipErrorOutOfMemory ? MFD_ENOMEM : MFD_EDEVICE, hipGetErrorString(e));
    }
    w->prof.on = c->prof_on;
    *out = w;
    return MFD_OK;
}

// Make ctx hold `count` workspaces for block size mb and the given precision.
int ensure_ws(mfd_ctx* c, int mb, bool mixed, int count) {
    for (Ws* w : c->ws)
        if (w->mb != mb || w->mixed != mixed) {
            for (Ws* x : c->ws) ws_free(x);
            c->ws.clear();
            break;
        }
    while ((int)c->ws.size() < count) {
        Ws* w = nullptr;
        int st = ws_alloc(c, mb, mixed, &w);
        if (st) return st;
        c->ws.push_back(w);
    }
    return MFD_OK;
}

// Column j of the solver block V (n x 6mb, c128).
inline double2* col(double2* V, size_t n, int j) { return V + (size_t)j * n; }

struct KResult {
    int iters = 0;
    bool converged = false;
    bool fp64_fallback = false;
    bool proposal_used = false;
    int rejected = 0;   // Rayleigh-Ritz steps rejected
    std::vector<double> theta, res;
};

// W <- T W in place for the listed FP64 fields (field fl(t) at W + n fl(t)).
// Grids whose FP64 plane FFT does not fit in LDS (N = 100, 120, 128, 150) stage the
// fields through FP32 in `stage` (same field positions): T only approximates
// the operator's inverse, so its rounding slows LOBPCG at most slightly and
// does not limit the accuracy the residual test certifies.
hipError_t precond_fp64(const mfd_ctx* c, const OpParams& p, int na, double2* W, float2* stage, size_t n,
                        const FieldList& fl, hipStream_t s) {
    if (fft_plane_fits(c->N, 8)) return launch_precond<double>(p, na, W, W, c->tw64, s, fl);
    if (!stage) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    for (int t = 0; t < na && e == hipSuccess; ++t) e = launch_convert(W + n * fl(t), stage + n * fl(t), n, true, s);
    if (e == hipSuccess) e = launch_precond<float>(p, na, stage, stage, c->tw32, s, fl);
    for (int t = 0; t < na && e == hipSuccess; ++t) e = launch_convert(stage + n * fl(t), W + n * fl(t), n, false, s);
    return e;
}

// LOBPCG at one k-point from the start block in V[:, :mb] (FP64).  Stops when
// the lowest `nreq` columns have converged (or after max_iter iterations).
// tr((S^H S)^-1 S^H A S) for the m columns at offset r of the basis, from the
// Gram matrix G (K x 2K row-major, [S^H S | S^H A S]): the sum of the Ritz
// values of that block (+inf when its Gram matrix is not positive definite).
double ritz_trace(const double2* G, int K, int r, int m) {
    std::vector<double> Lr(m * m, 0.0), Li(m * m, 0.0);
    auto gs = [&](int i, int j) { return G[(size_t)(r + i) * 2 * K + r + j]; };
    for (int j = 0; j < m; ++j) {
        double d = gs(j, j).x;
        for (int k = 0; k < j; ++k) d -= Lr[j * m + k] * Lr[j * m + k] + Li[j * m + k] * Li[j * m + k];
        if (!(d > 0.0)) return HUGE_VAL;
        const double ljj = std::sqrt(d);
        Lr[j * m + j] = ljj;
        for (int i = j + 1; i < m; ++i) {
            double sr = gs(i, j).x, si = gs(i, j).y;
            for (int k = 0; k < j; ++k) {   // L[i][k] conj(L[j][k])
                sr -= Lr[i * m + k] * Lr[j * m + k] + Li[i * m + k] * Li[j * m + k];
                si -= Li[i * m + k] * Lr[j * m + k] - Lr[i * m + k] * Li[j * m + k];
            }
            Lr[i * m + j] = sr / ljj;
            Li[i * m + j] = si / ljj;
        }
    }
    // tr(S^-1 A) = sum_q e_q^T L^-H L^-1 A e_q: forward solves L y = A e_q, then y_q of L^H z = y
    double tr = 0.0;
    std::vector<double> yr(m), yi(m);
    for (int q = 0; q < m; ++q) {
        for (int i = 0; i < m; ++i) {
            const double2 a = G[(size_t)(r + i) * 2 * K + K + r + q];
            double sr = a.x, si = a.y;
            for (int k = 0; k < i; ++k) {
                sr -= Lr[i * m + k] * yr[k] - Li[i * m + k] * yi[k];
                si -= Lr[i * m + k] * yi[k] + Li[i * m + k] * yr[k];
            }
            yr[i] = sr / Lr[i * m + i];
            yi[i] = si / Lr[i * m + i];
        }
        for (int i = m - 1; i >= q; --i) {   // back substitution with L^H, keep component q
            double sr = yr[i], si = yi[i];
            for (int k = i + 1; k < m; ++k) {   // conj(L[k][i]) z_k
                sr -= Lr[k * m + i] * yr[k] + Li[k * m + i] * yi[k];
                si -= Lr[k * m + i] * yi[k] - Li[k * m + i] * yr[k];
            }
            yr[i] = sr / Lr[i * m + i];
            yi[i] = si / Lr[i * m + i];
        }
        tr += yr[q];
    }
    return tr;
}

// A host synchronisation with the workspace's stream, counted per k-point.
hipError_t wsync(Ws& w) {
    ++w.syncs;
    return hipStreamSynchronize(w.stream);
}

// The Rayleigh-Ritz basis [X, W(act), P(pact)] as a column map of V.
BasisMap make_basis(int mb, const std::vector<int>& act, const std::vector<int>& pact, bool mixed) {
    BasisMap bm;
    const int na = (int)act.size(), np = (int)pact.size();
    bm.mb = mb;
    bm.na = na;
    bm.K = mb + na + np;
    const int K = bm.K;
    auto vcol = [&](int l) {   // basis column l < K -> column of V
        if (l < mb) return l;
        if (l < mb + na) return mb + act[l - mb];
        return 2 * mb + pact[l - mb - na];
    };
    int q = 0;
    auto put = [&](int l) {
        bm.lc[q] = (short)l;
        bm.pc[q] = (short)(l < K ? vcol(l) : 3 * mb + vcol(l - K));
        ++q;
    };
    if (mixed) {   // FP64 columns (X, AX) first, so that a wave's loads are of one precision
        for (int l = 0; l < mb; ++l) put(l);
        for (int l = 0; l < mb; ++l) put(K + l);
        for (int l = mb; l < K; ++l) put(l);
        for (int l = mb; l < K; ++l) put(K + l);
    } else {
        for (int l = 0; l < 2 * K; ++l) put(l);
    }
    for (int j = 0; j < 32; ++j) bm.tpos[j] = -1;
    for (int t = 0; t < na; ++t) {
        bm.tpos[act[t]] = (signed char)t;
        bm.act[t] = (unsigned char)act[t];
    }
    return bm;
}

// Basis [X_A W_A P_A] of the bands act still iterating under hard locking:
// basis column t < na is X of band act[t]; the W and P columns follow.
BasisMap make_basis_hl(int mb, const std::vector<int>& act, const std::vector<int>& pact, bool mixed) {
    BasisMap bm;
    const int na = (int)act.size(), np = (int)pact.size();
    bm.mb = mb;
    bm.na = na;
    bm.K = na + na + np;
    const int K = bm.K;
    auto vcol = [&](int l) {   // basis column l < K -> column of V
        if (l < na) return act[l];
        if (l < 2 * na) return mb + act[l - na];
        return 2 * mb + pact[l - 2 * na];
    };
    int q = 0;
    auto put = [&](int l) {
        bm.lc[q] = (short)l;
        bm.pc[q] = (short)(l < K ? vcol(l) : 3 * mb + vcol(l - K));
        ++q;
    };
    if (mixed) {   // FP64 columns (X, AX) first
        for (int l = 0; l < na; ++l) put(l);
        for (int l = 0; l < na; ++l) put(K + l);
        for (int l = na; l < K; ++l) put(l);
        for (int l = na; l < K; ++l) put(K + l);
    } else {
        for (int l = 0; l < 2 * K; ++l) put(l);
    }
    for (int j = 0; j < 32; ++j) bm.tpos[j] = -1;
    for (int t = 0; t < na; ++t) {
        bm.tpos[act[t]] = (signed char)t;
        bm.act[t] = (unsigned char)act[t];
    }
    return bm;
}

// Gram workgroups for a basis of K columns: the tuned count (set for the full
// basis, whose instance fits one workgroup per CU), doubled for bases of at
// most 32 columns (four times for at most 16), whose instances leave LDS and
// registers for two (four) per CU
// (at the tuned count half the chip's slots stay empty: 252 -> 193 us at
// K = 32, N = 64), when the partial-tile buffer holds them.
int gram_nparts(const Ws& w, int K) {
    const int T = (K + 15) / 16;
    if (T <= 2) {
        // one-tile bases (hard locking's small ones) fit four per CU
        const int np = (T == 1 ? 4 : 2) * w.nparts_gram;
        if ((size_t)(np + 1) * T * (T + 1) * 256 <= w.gpart_elems) return np;
    }
    return w.nparts_gram;
}

// With union_start the W columns hold a proposed start block.  The proposal
// replaces nothing: when the sum of its Ritz values is below that of X the
// first Rayleigh-Ritz step runs on span[X, W], otherwise on span[X] alone.
int lobpcg_k(mfd_ctx* c, Ws& w, const OpParams& p, int nreq, double tol, int max_iter, int stall_window,
             bool union_start, KResult& out) {
    const size_t n = w.n;
    const int mb = w.mb;
    const int K = 3 * mb;
    bool mixed = w.mixed;
    hipStream_t s = w.stream;
    double2* V = w.V;
    double2* U = w.U;
    float2* V32 = w.V32;
    float2* U32 = w.U32;
    out.fp64_fallback = false;
    out.rejected = 0;
    out.proposal_used = false;
    // AX = op(X) (FP64); with a proposal, AW = op(W).  The basis holds the W
    // and P columns of unconverged bands only, so nothing needs clearing: a W
    // column is formed before it is used, and a P column is used only when the
    // previous update wrote it.
    HIPCHK(launch_stencil<double>(p, mb, col(V, n, 0), col(V, n, 3 * mb), c->mu64, s));
    if (union_start) {
        if (mixed) HIPCHK(launch_stencil_f64_s32(p, mb, V32 + n * mb, V32 + n * 4 * mb, c->mu64, s));
        else HIPCHK(launch_stencil<double>(p, mb, col(V, n, mb), col(V, n, 4 * mb), c->mu64, s));
    }
    std::vector<int> act, pact;
    bool have_p = false;
    // Hard locking (w.hardlock): `locked` bands keep X and AX (equal in V and
    // U, so the update, which skips them, leaves them in place); pvalid: the
    // bands whose P the last update wrote.
    const unsigned all_bands = mb >= 32 ? ~0u : (1u << mb) - 1u;
    bool hard = false;
    unsigned locked = 0, pvalid = 0;
    if (union_start)
        for (int j = 0; j < mb; ++j) act.push_back(j);
    RRArgs ra;
    ra.G = w.G; ra.theta = w.theta; ra.C = w.C; ra.info = w.info; ra.floor = w.theta + mb;
    ra.mb = mb;
    // the Gram of FP32-stored directions is exact for the stored values, but
    // their images AW, AP carry FP32 rounding: drop nearly dependent ones sooner
    ra.drop_w = mixed ? 1e-6 : 1e-10;
    ra.drop_p = mixed ? 1e-5 : 1e-8;
    double* hth = w.host;
    double* hnorm = w.host + mb;
    double* hfloor = w.host + 7 * mb + 16;   // the Rayleigh-Ritz step's accuracy estimate
    *hfloor = 0.0;
    bool accurate_rr = false;
    static const bool trace = std::getenv("MFD_TRACE") != nullptr;
    const double N3 = (double)c->N * c->N * c->N;
    int it = 0, last_refresh = 0, refreshes = 0, best_it = 0, rejected = 0;
    bool rejected_last = false;
    double best = HUGE_VAL, rprev = HUGE_VAL;
    std::vector<double> th_prev(mb, 0.0);
    auto residuals = [&](double* rmax_out) {
        bool conv = true;
        double rmax = 0.0;
        for (int j = 0; j < nreq; ++j) {
            const double r = std::sqrt(hnorm[j]) / (std::fabs(hth[j]) * std::sqrt(hnorm[mb + j]));
            if (!(r <= tol)) conv = false;
            rmax = std::max(rmax, r);
        }
        *rmax_out = rmax;
        return conv;
    };
    // One iteration's kernels on stream s from buffers (Vi, Vi32) into (Ui,
    // Ui32), for the basis of the active bands `act` with their P columns,
    // as the eager loop below issues them (no timing events: used under
    // graph capture).
    auto issue = [&](double2* Vi, double2* Ui, float2* Vi32, float2* Ui32, const std::vector<int>& act_,
                     bool acc) -> hipError_t {
        const BasisMap bm = make_basis(mb, act_, act_, mixed);
        const int na = (int)act_.size();
        FieldList fl;
        fl.on = 1;
        for (int t = 0; t < na; ++t) fl.idx[t] = (unsigned char)act_[t];
        hipError_t e;
        if (w.precond == 1)
            e = mixed ? launch_precond_mg<float2>(w.mg, p, w.mgo, na, Vi32 + n * mb, Vi32 + n * mb, s, fl)
                      : launch_precond_mg<double2>(w.mg, p, w.mgo, na, col(Vi, n, mb), col(Vi, n, mb), s, fl);
        else if (mixed)
            e = launch_precond<float>(p, na, Vi32 + n * mb, Vi32 + n * mb, c->tw32, s, fl);
        else
            e = precond_fp64(c, p, na, col(Vi, n, mb), w.mixed ? Vi32 + n * mb : w.stage32, n, fl, s);
        if (e != hipSuccess) return e;
        e = mixed ? launch_stencil_f64_s32(p, na, Vi32 + n * mb, Vi32 + n * 4 * mb, c->mu64, s, fl)
                  : launch_stencil<double>(p, na, col(Vi, n, mb), col(Vi, n, 4 * mb), c->mu64, s, fl);
        if (e != hipSuccess) return e;
        if ((e = launch_gram_mfma(Vi, mixed ? Vi32 : nullptr, n, n, bm, gram_nparts(w, bm.K), w.gpart, w.G, s)) !=
            hipSuccess)
            return e;
        RRArgs r2 = ra;
        r2.K = bm.K;
        r2.nw = bm.na;
        if ((e = acc ? launch_rr_jacobi(r2, s) : launch_rr(r2, s)) != hipSuccess) return e;
        return launch_update_mfma(Vi, mixed ? Vi32 : nullptr, Ui, mixed ? Ui32 : nullptr, n, n, bm, w.C, w.theta,
                                  w.nparts_upd, w.npart, w.norms, s, w.upd_rows);
    };
    // A chunk of `cn` (even) iterations: a graph of two iterations (V -> U,
    // U -> V) captured for the current basis shape, Bloch vector and
    // precision, replayed cn / 2 times.  Returns 1 when the graph cannot be
    // captured (graph chunks are then off for this workspace).
    auto run_chunk = [&](int cn) -> int {
        const int flags = (mixed ? 1 : 0) + (accurate_rr ? 2 : 0);
        const double key[6] = {p.k[0], p.k[1], p.k[2], p.gamma, p.shift, (double)(size_t)V};
        bool same = w.gexec && flags == w.gkey_flags && act == w.gkey_act;
        for (int q = 0; q < 6 && same; ++q) same = key[q] == w.gkey[q];
        if (!same) {
            if (w.gexec) {
                hipGraphExecDestroy(w.gexec);
                w.gexec = nullptr;
            }
            if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return 1;
            hipError_t e = issue(V, U, V32, U32, act, accurate_rr);
            if (e == hipSuccess) e = issue(U, V, U32, V32, act, accurate_rr);
            hipGraph_t g = nullptr;
            const hipError_t ee = hipStreamEndCapture(s, &g);
            if (e != hipSuccess || ee != hipSuccess || !g) {
                if (g) hipGraphDestroy(g);
                (void)hipGetLastError();
                return 1;
            }
            e = hipGraphInstantiate(&w.gexec, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (e != hipSuccess) {
                w.gexec = nullptr;
                return 1;
            }
            w.gkey_act = act;
            w.gkey_flags = flags;
            for (int q = 0; q < 6; ++q) w.gkey[q] = key[q];
        }
        for (int r = 0; r < cn / 2; ++r)
            if (hipGraphLaunch(w.gexec, s) != hipSuccess) return -1;
        return 0;
    };
    double rate = 0.85, r_chunk0 = HUGE_VAL;   // residual reduction per iteration, for the chunk length
    int chunk_prev = 0;
    // lock the bands in `nw`: X, AX copied into U; the P, AP of the bands
    // still iterating made orthogonal to the new locked vectors
    auto lock_bands = [&](unsigned nw) -> int {
        if (!nw) return MFD_OK;
        if (!w.theta_a) {
            const size_t npl = 2048;
            if (hipMalloc(&w.theta_a, 64 * sizeof(double)) != hipSuccess ||
                hipMalloc(&w.lpart, (npl + npl / 64 + 1) * LK_MAXL * LK_MAXT * sizeof(double2)) != hipSuccess ||
                hipMalloc(&w.lcoef, LK_MAXL * LK_MAXT * sizeof(double2)) != hipSuccess) {
                (void)hipGetLastError();
                return fail(MFD_ENOMEM, "hard locking: allocation failed");
            }
        }
        LockCols lc;
        for (int j = 0; j < mb; ++j)
            if ((nw >> j) & 1u) {
                HIPCHK(hipMemcpyAsync(col(U, n, j), col(V, n, j), n * sizeof(double2), hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemcpyAsync(col(U, n, 3 * mb + j), col(V, n, 3 * mb + j), n * sizeof(double2),
                                      hipMemcpyDeviceToDevice, s));
                lc.xc[lc.nl] = (short)j;
                lc.axc[lc.nl] = (short)(3 * mb + j);
                ++lc.nl;
            }
        if (have_p) {
            for (int j : act)
                if ((pvalid >> j) & 1u) {
                    lc.yc[lc.nt] = (short)(2 * mb + j);
                    lc.zc[lc.nt] = (short)(5 * mb + j);
                    ++lc.nt;
                }
            if (lc.nt) {
                lc.y32 = mixed ? 1 : 0;
                lc.zpair = 1;
                hipEvent_t ep = w.prof.begin(s);
                HIPCHK(launch_lock_coef(lc, V, mixed ? V32 : nullptr, n, n, 2048, w.lpart, w.lcoef, s));
                HIPCHK(launch_lock_apply(lc, w.lcoef, V, mixed ? V32 : nullptr, n, n, 1024, s));
                w.prof.end(ep, 5, 0.0, s);
            }
        }
        locked |= nw;
        return MFD_OK;
    };
    auto resync_locked = [&]() -> int {   // V's AX was recomputed: U's copies of the locked ones follow
        for (int j = 0; j < mb; ++j)
            if ((locked >> j) & 1u)
                HIPCHK(hipMemcpyAsync(col(U, n, 3 * mb + j), col(V, n, 3 * mb + j), n * sizeof(double2),
                                      hipMemcpyDeviceToDevice, s));
        return MFD_OK;
    };
    auto leave_hard = [&]() {
        hard = false;
        locked = 0;
        have_p = false;   // P of bands that were locked is missing: restart
    };
    for (;; ++it) {
        const int rb = mixed ? 8 : 16;   // bytes per complex of the W/AW blocks
        // Hard locking: from the point where at most LK_NA bands iterate, the
        // others are locked; bands that iterate again leave the locked set,
        // and more than LK_NA iterating bands end hard locking
        if (w.hardlock && it > 0 && have_p && !union_start) {
            unsigned am = 0;
            for (int j : act) am |= 1u << j;
            if (!hard) {
                if (!act.empty() && (int)act.size() <= LK_NA) {
                    const int st = lock_bands(all_bands & ~am);
                    if (st) return st;
                    hard = true;
                }
            } else if (act.empty() || (int)act.size() > LK_NA) {
                leave_hard();
            } else {
                locked &= ~am;
                const int st = lock_bands(all_bands & ~am & ~locked);
                if (st) return st;
            }
        }
        // Graph chunks: from the third iteration on, several iterations run
        // from one captured graph with no host step between them; the active
        // set is the one of the chunk's start (bands that converge inside a
        // chunk keep iterating until its end).  The chunk's length follows
        // the residual's rate of decrease, so that it ends near convergence.
        bool chunked = false;
        if (w.graph && !hard && it >= 2 && have_p && !act.empty() && !union_start) {
            if (chunk_prev > 0 && r_chunk0 < HUGE_VAL && rprev > 0.0)
                rate = std::min(0.98, std::max(0.3, std::pow(rprev / r_chunk0, 1.0 / chunk_prev)));
            const double left = (rprev > tol) ? std::log(tol / rprev) / std::log(rate) : 1.0;
            int cn = 2 * std::min(4, std::max(1, (int)std::floor(left / 2.0)));
            cn = std::min(cn, std::max(2, (max_iter - it) / 2 * 2));
            if (cn >= 2 && it + cn - 1 <= max_iter) {
                const int st = run_chunk(cn);
                if (st < 0) return fail(MFD_EDEVICE, "graph launch failed");
                if (st == 0) {
                    chunked = true;
                    it += cn - 1;
                    r_chunk0 = rprev;
                    chunk_prev = cn;
                } else {
                    w.graph = false;
                }
            }
        }
        bool hard_step = false;
        if (!chunked && hard) {
            // the iteration on the bands still iterating (all W and P
            // orthogonal to the locked X)
            const int na = (int)act.size();
            pact.clear();
            for (int j : act)
                if ((pvalid >> j) & 1u) pact.push_back(j);
            const int np = (int)pact.size();
            FieldList fl;
            fl.on = 1;
            for (int t = 0; t < na; ++t) fl.idx[t] = (unsigned char)act[t];
            hipEvent_t e0 = w.prof.begin(s);
            if (w.precond == 1) {
                if (mixed) HIPCHK(launch_precond_mg<float2>(w.mg, p, w.mgo, na, V32 + n * mb, V32 + n * mb, s, fl));
                else HIPCHK(launch_precond_mg<double2>(w.mg, p, w.mgo, na, col(V, n, mb), col(V, n, mb), s, fl));
            } else if (mixed) {
                HIPCHK(launch_precond<float>(p, na, V32 + n * mb, V32 + n * mb, c->tw32, s, fl));
            } else {
                HIPCHK(precond_fp64(c, p, na, col(V, n, mb), w.mixed ? V32 + n * mb : w.stage32, n, fl, s));
            }
            w.prof.end(e0, 1, N3 * 3 * rb * 2.0 * na, s);
            if (locked) {   // W -= X_L (X_L^H W)
                LockCols lc;
                for (int j = 0; j < mb; ++j)
                    if ((locked >> j) & 1u) {
                        lc.xc[lc.nl] = (short)j;
                        lc.axc[lc.nl] = (short)(3 * mb + j);
                        ++lc.nl;
                    }
                for (int t = 0; t < na; ++t) lc.yc[lc.nt++] = (short)(mb + act[t]);
                lc.y32 = mixed ? 1 : 0;
                hipEvent_t ep = w.prof.begin(s);
                HIPCHK(launch_lock_coef(lc, V, mixed ? V32 : nullptr, n, n, 2048, w.lpart, w.lcoef, s));
                HIPCHK(launch_lock_apply(lc, w.lcoef, V, mixed ? V32 : nullptr, n, n, 1024, s));
                w.prof.end(ep, 5, 0.0, s);
            }
            e0 = w.prof.begin(s);
            if (mixed) HIPCHK(launch_stencil_f64_s32(p, na, V32 + n * mb, V32 + n * 4 * mb, c->mu64, s, fl));
            else HIPCHK(launch_stencil<double>(p, na, col(V, n, mb), col(V, n, 4 * mb), c->mu64, s, fl));
            w.prof.end(e0, 0, N3 * (6.0 * rb * na + 24.0), s);
            const BasisMap bm = make_basis_hl(mb, act, pact, mixed);
            hipEvent_t e1 = w.prof.begin(s);
            HIPCHK(launch_gram_mfma(V, mixed ? V32 : nullptr, n, n, bm, gram_nparts(w, bm.K), w.gpart, w.G, s));
            w.prof.end(e1, 2, 8.0 * (double)n * bm.K * (bm.K + 1), s);
            RRArgs r2 = ra;
            r2.K = bm.K;
            r2.nw = na;
            r2.mb = na;
            r2.theta = w.theta_a;
            e1 = w.prof.begin(s);
            HIPCHK(accurate_rr ? launch_rr_jacobi(r2, s) : launch_rr(r2, s));
            w.prof.end(e1, 3, 0.0, s);
            LockBasis lb;
            lb.na = na;
            lb.K = bm.K;
            lb.mb = mb;
            for (int k = 0; k < bm.K; ++k) {
                const int vc = k < na ? act[k] : (k < 2 * na ? mb + act[k - na] : 2 * mb + pact[k - 2 * na]);
                lb.sc[k] = (short)vc;
                lb.ic[k] = (short)(3 * mb + vc);
                if (mixed && k >= na) lb.f32 |= 1ull << k;
            }
            for (int t = 0; t < na; ++t) lb.act[t] = (unsigned char)act[t];
            e1 = w.prof.begin(s);
            HIPCHK(launch_lock_update(lb, V, mixed ? V32 : nullptr, U, mixed ? U32 : nullptr, n, n, w.C, w.theta_a,
                                      1024, w.npart, w.norms, s));
            w.prof.end(e1, 4, (double)n * (2 * na * 16.0 + 2 * (na + np) * rb + 2 * na * 16.0 + 3 * na * rb), s);
            std::swap(V, U);
            if (mixed) std::swap(V32, U32);
            have_p = true;
            pvalid = 0;
            for (int j : act) pvalid |= 1u << j;
            hard_step = true;
        } else if (!chunked) {
        // P columns: every update writes P' of every band, so each active band
        // has one from the second iteration on (zero after the first, which the
        // Rayleigh-Ritz step leaves out)
        pact.clear();
        if (have_p) pact = act;
        BasisMap bm = make_basis(mb, act, pact, mixed);
        const int na = (int)act.size(), np = (int)pact.size();
        if (it > 0 && na > 0) {
            // W = T R (in place), AW = op(W), for the active bands' columns
            FieldList fl;
            fl.on = 1;
            for (int t = 0; t < na; ++t) fl.idx[t] = (unsigned char)act[t];
            hipEvent_t e0 = w.prof.begin(s);
            if (w.precond == 1) {
                if (mixed) HIPCHK(launch_precond_mg<float2>(w.mg, p, w.mgo, na, V32 + n * mb, V32 + n * mb, s, fl));
                else HIPCHK(launch_precond_mg<double2>(w.mg, p, w.mgo, na, col(V, n, mb), col(V, n, mb), s, fl));
            } else if (mixed) {
                HIPCHK(launch_precond<float>(p, na, V32 + n * mb, V32 + n * mb, c->tw32, s, fl));
            } else {
                HIPCHK(precond_fp64(c, p, na, col(V, n, mb), w.mixed ? V32 + n * mb : w.stage32, n, fl, s));
            }
            w.prof.end(e0, 1, N3 * 3 * rb * 2.0 * na, s);
            e0 = w.prof.begin(s);
            if (mixed) HIPCHK(launch_stencil_f64_s32(p, na, V32 + n * mb, V32 + n * 4 * mb, c->mu64, s, fl));
            else HIPCHK(launch_stencil<double>(p, na, col(V, n, mb), col(V, n, 4 * mb), c->mu64, s, fl));
            w.prof.end(e0, 0, N3 * (6.0 * rb * na + 24.0), s);
        }
        hipEvent_t e1 = w.prof.begin(s);
        HIPCHK(launch_gram_mfma(V, mixed ? V32 : nullptr, n, n, bm, gram_nparts(w, bm.K), w.gpart, w.G, s, 1));
        w.prof.end(e1, 2, 8.0 * (double)n * bm.K * (bm.K + 1), s);   // flops, not bytes
        e1 = w.prof.begin(s);
        HIPCHK(launch_gram_mfma(V, mixed ? V32 : nullptr, n, n, bm, gram_nparts(w, bm.K), w.gpart, w.G, s, 2));
        w.prof.end(e1, 5, 0.0, s);
        if (it == 0 && union_start) {
            const int Kb = bm.K;
            std::vector<double2> hG((size_t)Kb * 2 * Kb);
            HIPCHK(hipMemcpyAsync(hG.data(), w.G, hG.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
            HIPCHK(wsync(w));
            const double tx = ritz_trace(hG.data(), Kb, 0, mb), tw = ritz_trace(hG.data(), Kb, mb, mb);
            out.proposal_used = tw < tx;
            if (trace) std::fprintf(stderr, "[%p] proposal: Ritz sum %.6e vs previous-k %.6e -> %s\n", (void*)&w,
                                    tw, tx, out.proposal_used ? "used" : "dropped");
            if (!out.proposal_used) {   // X alone
                act.clear();
                bm = make_basis(mb, act, pact, mixed);
                HIPCHK(launch_gram_mfma(V, mixed ? V32 : nullptr, n, n, bm, gram_nparts(w, bm.K), w.gpart, w.G, s));
            }
        }
        ra.K = bm.K;
        ra.nw = bm.na;
        e1 = w.prof.begin(s);
        // The Householder route (launch_rr) has Ritz values accurate to about
        // Kv eps |H| in absolute terms; within a factor 100 of that floor the
        // iteration takes the Jacobi route, whose errors are relative.
        HIPCHK(accurate_rr ? launch_rr_jacobi(ra, s) : launch_rr(ra, s));
        w.prof.end(e1, 3, 0.0, s);
        e1 = w.prof.begin(s);
        HIPCHK(launch_update_mfma(V, mixed ? V32 : nullptr, U, mixed ? U32 : nullptr, n, n, bm, w.C, w.theta,
                                  w.nparts_upd, w.npart, w.norms, s, w.upd_rows, false));
        // reads X, AX (FP64) and the W, P, AW, AP of the basis; writes X', AX'
        // (FP64) and R', P', AP' of every band
        w.prof.end(e1, 4, (double)n * (2 * mb * 16.0 + 2 * (bm.na + np) * rb + 2 * mb * 16.0 + 3 * mb * rb), s);
        e1 = w.prof.begin(s);
        HIPCHK(launch_reduce(w.npart, w.nparts_upd, 2 * mb, w.norms, s));
        w.prof.end(e1, 5, 0.0, s);
        std::swap(V, U);
        if (mixed) std::swap(V32, U32);
        have_p = true;   // the update wrote P', AP' of every band
        pvalid = all_bands;
        }   // eager iteration
        int* hinfo = (int*)(w.host + 3 * mb);
        if (hard_step) {
            // the iterating bands' Ritz values and norms, scattered to their
            // bands; the locked ones keep theirs.  The device theta of every
            // band follows (refreshes and residuals read it).
            double* tha = w.host + 8 * mb + 32;
            double* nra = tha + mb;
            const int na = (int)act.size();
            HIPCHK(hipMemcpyAsync(tha, w.theta_a, na * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(hfloor, w.theta + mb, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(nra, w.norms, 2 * na * sizeof(double), hipMemcpyDeviceToHost, s));
            if (trace) HIPCHK(hipMemcpyAsync(hinfo, w.info, 10 * sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(wsync(w));
            for (int t = 0; t < na; ++t) {
                hth[act[t]] = tha[t];
                hnorm[act[t]] = nra[t];
                hnorm[mb + act[t]] = nra[na + t];
            }
            HIPCHK(hipMemcpyAsync(w.theta, hth, mb * sizeof(double), hipMemcpyHostToDevice, s));
        } else {
        HIPCHK(hipMemcpyAsync(hth, w.theta, mb * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hfloor, w.theta + mb, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hnorm, w.norms, 2 * mb * sizeof(double), hipMemcpyDeviceToHost, s));
        if (trace) HIPCHK(hipMemcpyAsync(hinfo, w.info, 10 * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(wsync(w));
        }
        w.prof.drain();
        double rmax = 0.0;
        bool conv = residuals(&rmax);
        auto active_set = [&]() {
            act.clear();
            for (int j = 0; j < mb; ++j)
                if (!(std::sqrt(hnorm[j]) / (std::fabs(hth[j]) * std::sqrt(hnorm[mb + j])) <= tol)) act.push_back(j);
        };
        active_set();
        if (trace) {
            int nact = 0;
            for (int j = 0; j < mb; ++j)
                nact += std::sqrt(hnorm[j]) / (std::fabs(hth[j]) * std::sqrt(hnorm[mb + j])) > tol;
            std::fprintf(stderr, "[%p] it %4d rmax %.3e active %2d kept %2d dropP %d sweeps %d th0 %.8f thn %.8f "
                         "rr-ticks %d %d %d %d %d Kk %d\n", (void*)&w, it, rmax, nact, hinfo[0], hinfo[1], hinfo[3], hth[0],
                         hth[nreq - 1], hinfo[4], hinfo[5], hinfo[6], hinfo[7], hinfo[8], hinfo[9]);
        }
        // Rayleigh-Ritz breakdown: a nearly dependent W or P column that the
        // Cholesky pivots let through amplifies the rounding of its Gram
        // entries (FP32-stored AW, AP; drift of the tracked AX, AP), and the
        // step returns garbage.  A suspect step (a negative Ritz value, which
        // the positive semidefinite operator cannot have, or a worst residual
        // up more than 20 times, from the third iteration on) is checked with
        // a fresh A X': a sound step's Ritz values are the Rayleigh quotients
        // of its vectors (a residual can also jump when the subspace finds an
        // eigenvalue the block had missed), a broken one's are not.  A broken
        // step is rejected: the previous X, AX are still in the other buffer;
        // AX is recomputed, R = A X - theta X with the previous theta, and the
        // conjugate directions restart.  Mixed precision (unless its FP64
        // fallback is off) continues in FP64, where the Gram entries of the
        // search directions carry no FP32 rounding.  Two steps in a row are
        // never rejected, so the iteration cannot loop.
        bool suspect = !(rmax == rmax) || (it >= 3 && rmax > 20.0 * rprev && rmax > 1e-4);
        for (int j = 0; j < mb; ++j) suspect |= !(hth[j] >= 0.0);
        bool reject = false;
        if (suspect && it > 0) {
            double* rq = w.host + 5 * mb;
            HIPCHK(launch_stencil<double>(p, mb, col(V, n, 0), col(V, n, 3 * mb), c->mu64, s));
            HIPCHK(launch_colstats(col(V, n, 0), col(V, n, 3 * mb), n, n, mb, nullptr, w.nparts_col, w.cpart, w.cout,
                                   s));
            HIPCHK(hipMemcpyAsync(rq, w.cout, 2 * mb * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(wsync(w));
            double dev = 0.0, scale = 0.0;
            for (int j = 0; j < mb; ++j) {
                const double t = rq[2 * j + 1] / rq[2 * j];
                dev = std::max(dev, std::fabs(t - hth[j]));
                scale = std::max(scale, std::fabs(t));
            }
            reject = !(dev <= 1e-6 * scale) && !rejected_last;
            if (trace) std::fprintf(stderr, "[%p] it %d: suspect step, Ritz values vs fresh Rayleigh quotients %.3e "
                                    "(scale %.3e)%s\n", (void*)&w, it, dev, scale, reject ? ": rejected" : "");
            if (!reject) {   // the fresh A X' stands in for the tracked one
                if (hard) {
                    const int st = resync_locked();
                    if (st) return st;
                }
                HIPCHK(launch_residual(col(V, n, 0), col(V, n, 3 * mb),
                                       mixed ? (void*)(V32 + n * mb) : col(V, n, mb), mixed, n, n, mb, w.theta,
                                       w.nparts_col, w.npart, w.norms, s));
                HIPCHK(hipMemcpyAsync(hnorm, w.norms, 2 * mb * sizeof(double), hipMemcpyDeviceToHost, s));
                HIPCHK(wsync(w));
                conv = residuals(&rmax);
                active_set();
                last_refresh = it;
            }
        }
        rejected_last = reject;
        if (reject) {
            if (hard) leave_hard();
            std::swap(V, U);
            if (mixed) std::swap(V32, U32);
            if (mixed && stall_window > 0) {
                mixed = false;
                out.fp64_fallback = true;
                ra.drop_w = 1e-10;
                ra.drop_p = 1e-8;
                best_it = it;
            }
            std::memcpy(hth, th_prev.data(), mb * sizeof(double));
            HIPCHK(hipMemcpyAsync(w.theta, hth, mb * sizeof(double), hipMemcpyHostToDevice, s));
            HIPCHK(launch_stencil<double>(p, mb, col(V, n, 0), col(V, n, 3 * mb), c->mu64, s));
            HIPCHK(launch_residual(col(V, n, 0), col(V, n, 3 * mb), mixed ? (void*)(V32 + n * mb) : col(V, n, mb),
                                   mixed, n, n, mb, w.theta, w.nparts_col, w.npart, w.norms, s));
            HIPCHK(hipMemcpyAsync(hnorm, w.norms, 2 * mb * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(wsync(w));
            have_p = false;
            conv = residuals(&rmax);
            active_set();
            last_refresh = it;
            ++rejected;
            if (trace) std::fprintf(stderr, "[%p] it %d: Rayleigh-Ritz step rejected (%s), P restarted: rmax %.3e\n",
                                    (void*)&w, it, mixed ? "mixed" : "FP64", rmax);
        }
        // The tracked AX = [AX AW AP] C drifts from A X (in mixed precision by
        // the FP32 rounding of AW and AP, every 15 iterations recomputed with
        // the FP64 operator).  Convergence is confirmed with a fresh A X in
        // every mode, the FP64 fallback included; if the fresh residuals miss
        // the target, the iteration goes on from the refreshed state.
        if (it > 0 && it != last_refresh && (conv || (mixed && it - last_refresh >= 15))) {
            HIPCHK(launch_stencil<double>(p, mb, col(V, n, 0), col(V, n, 3 * mb), c->mu64, s));
            if (hard) {
                const int st = resync_locked();
                if (st) return st;
            }
            HIPCHK(launch_residual(col(V, n, 0), col(V, n, 3 * mb), mixed ? (void*)(V32 + n * mb) : col(V, n, mb),
                                   mixed, n, n, mb, w.theta, w.nparts_col, w.npart, w.norms, s));
            HIPCHK(hipMemcpyAsync(hnorm, w.norms, 2 * mb * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(wsync(w));
            conv = residuals(&rmax);
            active_set();
            last_refresh = it;
            ++refreshes;
            if (trace) std::fprintf(stderr, "[%p] refresh %d: rmax %.3e\n", (void*)&w, refreshes, rmax);
        }
        if (conv || it >= max_iter) {
            out.converged = conv;
            break;
        }
        if (rmax < 0.5 * best) {
            best = rmax;
            best_it = it;
        }
        // A clustered spectrum (a compensation mode among the bands near
        // Gamma) can stall the FP32-stored directions: when the residual has
        // not halved in stall_window iterations, finish this k-point in FP64
        // from the current X with fresh A X, R = A X - theta X and no P.
        if (mixed && stall_window > 0 && it - best_it >= stall_window) {
            if (hard) leave_hard();
            mixed = false;
            out.fp64_fallback = true;
            have_p = false;   // no P in FP64 storage yet
            HIPCHK(launch_stencil<double>(p, mb, col(V, n, 0), col(V, n, 3 * mb), c->mu64, s));
            HIPCHK(launch_residual(col(V, n, 0), col(V, n, 3 * mb), col(V, n, mb), false, n, n, mb, w.theta,
                                   w.nparts_col, w.npart, w.norms, s));
            HIPCHK(hipMemcpyAsync(hnorm, w.norms, 2 * mb * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(wsync(w));
            active_set();
            ra.drop_w = 1e-10;
            ra.drop_p = 1e-8;
            best_it = it;
            if (trace) std::fprintf(stderr, "[%p] it %d: mixed precision stalled at %.3e, continuing in FP64\n",
                                    (void*)&w, it, rmax);
        } else if (!mixed && stall_window > 0 && it - best_it >= std::max(stall_window, 40)) {
            if (hard) leave_hard();
            // FP64 stall (a nearly dependent search direction kept in the
            // basis can hold the Rayleigh-Ritz step at a floor): restart the
            // conjugate directions once from the current X, with fresh A X and
            // R = A X - theta X; judged over at least 40 iterations, however
            // short the window that sends mixed precision to FP64
            have_p = false;
            HIPCHK(launch_stencil<double>(p, mb, col(V, n, 0), col(V, n, 3 * mb), c->mu64, s));
            HIPCHK(launch_residual(col(V, n, 0), col(V, n, 3 * mb), col(V, n, mb), false, n, n, mb, w.theta,
                                   w.nparts_col, w.npart, w.norms, s));
            HIPCHK(hipMemcpyAsync(hnorm, w.norms, 2 * mb * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(wsync(w));
            active_set();
            best = rmax;
            best_it = it;
            if (trace) std::fprintf(stderr, "[%p] it %d: stalled at %.3e, P restarted\n", (void*)&w, it, rmax);
        }
        {
            double tmin = HUGE_VAL;
            for (int j = 0; j < nreq; ++j) tmin = std::min(tmin, std::fabs(hth[j]));
            accurate_rr = rmax < 100.0 * *hfloor / tmin;
        }
        rprev = rmax;
        std::memcpy(th_prev.data(), hth, mb * sizeof(double));
    }
    out.rejected = rejected;
    w.V32 = V32;
    w.U32 = U32;
    w.V = V;
    w.U = U;
    out.iters = it;
    // final check with a fresh FP64 operator application: AX slot <- op(X)
    HIPCHK(launch_stencil<double>(p, mb, col(V, n, 0), col(V, n, 3 * mb), c->mu64, s));
    HIPCHK(launch_colstats(col(V, n, 0), col(V, n, 3 * mb), n, n, mb, nullptr, w.nparts_col, w.cpart, w.cout, s));
    HIPCHK(hipMemcpyAsync(w.host, w.cout, 2 * mb * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(wsync(w));
    out.theta.assign(mb, 0.0);
    std::vector<double> xx(mb);
    for (int j = 0; j < mb; ++j) {
        out.theta[j] = w.host[2 * j + 1] / w.host[2 * j];
        xx[j] = w.host[2 * j];
    }
    std::memcpy(w.host + 4 * mb, out.theta.data(), mb * sizeof(double));
    HIPCHK(hipMemcpyAsync(w.theta, w.host + 4 * mb, mb * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(launch_colstats(col(V, n, 0), col(V, n, 3 * mb), n, n, mb, w.theta, w.nparts_col, w.cpart, w.cout, s));
    HIPCHK(hipMemcpyAsync(w.host, w.cout, 2 * mb * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(wsync(w));
    out.res.assign(mb, 0.0);
    for (int j = 0; j < mb; ++j) out.res[j] = std::sqrt(w.host[2 * j]) / (std::fabs(out.theta[j]) * std::sqrt(xx[j]));
    return MFD_OK;
}

// lambda_re of Alg 4.1 for nb c128 fields on the workspace's stream.
int lambda_re_ws(mfd_ctx* c, Ws& w, const OpParams& p, int nb, const void* X, double* out) {
    const int nparts = 128;
    HIPCHK(launch_lambda_re(p, nb, X, c->mu64, w.cpart, nparts, w.cout, w.stream));
    HIPCHK(hipMemcpyAsync(w.host, w.cout, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, w.stream));
    HIPCHK(wsync(w));
    for (int b = 0; b < nb; ++b) out[b] = w.host[2 * b] / w.host[2 * b + 1];
    return MFD_OK;
}

struct KOut {
    double* evals;       // nbands
    double2* evecs;      // nbands x n or null
    mfd_kstats* stats;   // or null
};

// One k-point: LOBPCG on mb = nbands + guard columns starting from V[:, :mb],
// then Alg 4.1 (discard flagged bands, or double gamma and solve again).
int solve_k(mfd_ctx* c, Ws& w, const double* k, int nbands, double tol, const mfd_opts& o, uint64_t seed_k,
            const KOut& ko, bool proposal, bool* proposal_used, double* lam_all, int* converged) {
    const size_t n = w.n;
    const int mb = w.mb;
    hipStream_t s = w.stream;
    auto t0 = std::chrono::steady_clock::now();
    w.syncs = 0;
    OpParams p = params(c, k);
    p.wtmp = w.wtmp;
    p.stencil_wgs = w.stencil_wgs;
    p.fft_xc = w.fft_xc;
    const double scale = std::pow(2.0 * M_PI / c->L, 2);
    KResult kr;
    int doublings = 0, total_iters = 0, nspur = 0, discarded = 0, fp64_fallback = 0, rejected = 0;
    int nreq = nbands;
    std::vector<double> lam(mb), lre(mb);
    std::vector<int> sel;
    for (;;) {
        int st = lobpcg_k(c, w, p, nreq, tol, o.max_iter, o.stall_window, proposal, kr);
        if (proposal && proposal_used) *proposal_used = kr.proposal_used;
        proposal = false;
        if (st) return st;
        total_iters += kr.iters;
        fp64_fallback |= kr.fp64_fallback;
        rejected += kr.rejected;
        for (int j = 0; j < mb; ++j) lam[j] = kr.theta[j] - p.shift;
        // Alg 4.1: recompute lambda_re = |M_0^(1/2) A'x|^2 / |x|^2; a band with
        // lambda - lambda_re visibly > 0 is a compensation (spurious) mode
        st = lambda_re_ws(c, w, p, mb, w.V, lre.data());
        if (st) return st;
        std::vector<int> phys, spur;
        for (int j = 0; j < mb; ++j) {
            const bool sp = lam[j] - lre[j] > 1e-4 * std::fabs(lam[j]) + 1e-10 * scale;
            (sp ? spur : phys).push_back(j);
        }
        if ((int)phys.size() >= nbands) {
            const int need = phys[nbands - 1] + 1;
            if (need > nreq && kr.converged) {
                nreq = need;   // flagged bands are discarded: converge one band further
                continue;
            }
            sel.assign(phys.begin(), phys.begin() + nbands);
            discarded = need - nbands;
            nspur = 0;
            break;
        }
        nspur = (int)spur.size();
        if (doublings >= o.max_gamma_doublings) {
            for (int j = 0; j < nbands; ++j) sel.push_back(j);
            break;
        }
        // too few physical bands: enlarge gamma and solve again (Alg 4.1)
        p.gamma *= 2.0;
        ++doublings;
        nreq = nbands;
        for (size_t q = 0; q < spur.size(); ++q)
            HIPCHK(launch_fill_random(col(w.V, n, spur[q]), n, seed_k + 7919ull * doublings + spur[q], s));
    }
    if (lam_all)
        for (int j = 0; j < mb; ++j) lam_all[j] = lam[j];
    std::vector<int> idx(sel);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return lam[a] < lam[b]; });
    double maxres = 0.0;
    for (int j = 0; j < nbands; ++j) {
        ko.evals[j] = lam[idx[j]];
        maxres = std::max(maxres, kr.res[idx[j]]);
    }
    if (ko.evecs) {
        for (int j = 0; j < nbands; ++j)
            HIPCHK(hipMemcpyAsync(ko.evecs + (size_t)j * n, col(w.V, n, idx[j]), n * sizeof(double2),
                                  hipMemcpyDeviceToDevice, s));
        HIPCHK(wsync(w));
    }
    auto t1 = std::chrono::steady_clock::now();
    if (ko.stats) {
        mfd_kstats& ks = *ko.stats;
        ks.iters = total_iters;
        ks.gamma_doublings = doublings;
        ks.gamma = p.gamma;
        ks.max_rel_resid = maxres;
        ks.spurious = nspur;
        ks.discarded = discarded;
        ks.used_fallback = 0;
        ks.fp64_fallback = fp64_fallback;
        ks.rejected_steps = rejected;
        ks.host_syncs = w.syncs;
        ks.ms = (float)std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    *converged = (maxres <= tol) ? (nspur ? 2 : 1) : 0;
    return MFD_OK;
}

// A caller's start block must span mb dimensions: a column whose squared
// distance to the span of the columns before it is below 1e-10 of its squared
// norm (a pivot of the Cholesky factor of X^H X) is replaced by seeded random
// values.  Checked twice (a replacement is itself checked once more).
int fix_dependent_start(Ws& w, uint64_t seed) {
    const size_t n = w.n;
    const int mb = w.mb;
    hipStream_t s = w.stream;
    std::vector<double2> G((size_t)mb * mb);
    for (int pass = 0; pass < 2; ++pass) {
        HIPCHK(launch_gram(w.V, n, n, mb, mb, gram_parts(n), w.gpart, w.G, s));
        HIPCHK(hipMemcpyAsync(G.data(), w.G, G.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::vector<double> Lr((size_t)mb * mb, 0.0), Li((size_t)mb * mb, 0.0);
        std::vector<int> dep;
        for (int j = 0; j < mb; ++j) {
            const double gjj = G[(size_t)j * mb + j].x;
            double d = gjj;
            for (int k = 0; k < j; ++k) d -= Lr[j * mb + k] * Lr[j * mb + k] + Li[j * mb + k] * Li[j * mb + k];
            if (!(d > 1e-10 * gjj) || !(gjj > 0.0)) {   // dependent (or zero, or not finite): row j of L stays 0
                dep.push_back(j);
                continue;
            }
            const double ljj = std::sqrt(d);
            Lr[j * mb + j] = ljj;
            for (int i = j + 1; i < mb; ++i) {
                double sr = G[(size_t)i * mb + j].x, si = G[(size_t)i * mb + j].y;
                for (int k = 0; k < j; ++k) {
                    sr -= Lr[i * mb + k] * Lr[j * mb + k] + Li[i * mb + k] * Li[j * mb + k];
                    si -= Li[i * mb + k] * Lr[j * mb + k] - Lr[i * mb + k] * Li[j * mb + k];
                }
                Lr[i * mb + j] = sr / ljj;
                Li[i * mb + j] = si / ljj;
            }
        }
        if (dep.empty()) return MFD_OK;
        for (int j : dep) HIPCHK(launch_fill_random(col(w.V, n, j), n, seed + 7ull * (uint64_t)(pass + 1) + j, s));
    }
    return MFD_OK;
}

// A run of consecutive k-points on one workspace: random start at the first
// (or the caller's block), warm start from the previous k-point afterwards.
struct Segment {
    mfd_ctx* ctx;
    Ws* ws;
    const double* kpts;    // nk x 3
    int k0, k1;            // [k0, k1)
    int nbands;
    double tol;
    mfd_opts opts;
    double* evals;         // nk x nbands
    double2* evecs;        // nk x nbands x n or null
    mfd_kstats* stats;     // nk or null
    int status = MFD_OK;
    int worst = 1;         // 1 all converged, 0 some not, 2 spurious remain
    std::string err;
    // opts.balance: the segments of one call share a lock over their [k0, k1)
    // and the k-point each is solving (cur; -1 when done)
    struct Balance* bal = nullptr;
    int cur = -1;
};

struct Balance {
    std::mutex mu;
    std::vector<Segment*> segs;
};

// Under the lock: a segment with nothing left takes the second half of the
// k-points beyond the one the busiest other segment is solving (at least 2
// of them; that segment keeps the larger half, which it reaches warm).
// Returns the new first k-point, or -1 when no segment has 2 left.
static int steal(Segment* sg) {
    Segment* v = nullptr;
    int best = 1;
    for (Segment* o : sg->bal->segs) {
        if (o == sg || o->cur < 0) continue;
        const int rem = o->k1 - (o->cur + 1);
        if (rem > best) {
            best = rem;
            v = o;
        }
    }
    if (!v) return -1;
    const int mid = v->cur + 1 + (best + 1) / 2;
    sg->k0 = mid;
    sg->k1 = v->k1;
    v->k1 = mid;
    return mid;
}

int planewave_start(const mfd_ctx* c, Ws& w, const double* k, int mb, uint64_t seed);

void run_segment(Segment* sg) {
    mfd_ctx* c = sg->ctx;
    Ws& w = *sg->ws;
    const size_t n = w.n;
    const int mb = w.mb;
    const mfd_opts& o = sg->opts;
    w.precond = o.precond;
    w.graph = o.graph != 0;
    w.hardlock = o.hard_lock != 0;
    w.mgo.cycles = o.mg_cycles;
    w.mgo.n1 = w.mgo.n2 = o.mg_smooth;
    w.mgo.sweeps = o.mg_sweeps;
    if (o.precond == 1 && !w.mg) w.mg = mg_create();
    const bool learned = o.warm_start == 2;
    if (learned) {
        if (!w.warm) {
            w.warm = new WarmStart();
            const int st = w.warm->init(n, mb, c->L, o.seed + 1);
            if (st) {
                w.warm->release();
                delete w.warm;
                w.warm = nullptr;
                sg->status = fail(st, "learned warm start: allocation failed");
                sg->err = g_last_error;
                return;
            }
        }
        if (w.warm->reset(w.stream)) {
            sg->status = fail(MFD_EDEVICE, "learned warm start: reset failed");
            sg->err = g_last_error;
            return;
        }
    }
    std::vector<double> lam_all(mb);
    for (int ik = sg->k0;; ++ik) {
        if (sg->bal) {
            std::lock_guard<std::mutex> lk(sg->bal->mu);
            if (ik >= sg->k1) ik = steal(sg);
            sg->cur = ik;
            if (ik < 0) break;
        } else if (ik >= sg->k1) {
            break;
        }
        const uint64_t seed_k = o.seed * 1000003ull + 104729ull * (uint64_t)ik;
        int st = MFD_OK;
        bool proposal = false;
        if (learned && ik > sg->k0) {
            void* W = w.mixed ? (void*)(w.V32 + n * mb) : (void*)col(w.V, n, mb);
            st = w.warm->propose(sg->kpts + 3 * ik, W, w.mixed, &proposal, w.stream);
            if (st) st = fail(st, "learned warm start: proposal failed");
        }
        if (ik == sg->k0 && ik == 0 && o.x0) {
            hipError_t e = hipMemcpyAsync(w.V, o.x0, n * sg->nbands * sizeof(double2), hipMemcpyDeviceToDevice,
                                          w.stream);
            if (e == hipSuccess && mb > sg->nbands)
                e = launch_fill_random(col(w.V, n, sg->nbands), n * (mb - sg->nbands), seed_k + 17, w.stream);
            if (e != hipSuccess) st = fail(MFD_EDEVICE, hipGetErrorString(e));
            else st = fix_dependent_start(w, seed_k + 101);
        } else if (!st && ik == sg->k0 && o.cold_start == 1) {
            st = planewave_start(c, w, sg->kpts + 3 * ik, mb, seed_k);
        } else if (!st && (ik == sg->k0 || !o.warm_start)) {
            hipError_t e = launch_fill_random(w.V, n * mb, seed_k, w.stream);
            if (e != hipSuccess) st = fail(MFD_EDEVICE, hipGetErrorString(e));
        }
        int conv = 1;
        if (!st) {
            KOut ko{sg->evals + (size_t)ik * sg->nbands,
                    sg->evecs ? sg->evecs + (size_t)ik * sg->nbands * n : nullptr,
                    sg->stats ? sg->stats + ik : nullptr};
            bool used = false;
            st = solve_k(c, w, sg->kpts + 3 * ik, sg->nbands, sg->tol, o, seed_k, ko, proposal, &used,
                         lam_all.data(), &conv);
            if (!st && ko.stats) {
                ko.stats->used_fallback = (learned && ik > sg->k0 && !used) ? 1 : 0;
                ko.stats->segment_start = (ik == sg->k0 || !o.warm_start) ? 1 : 0;
            }
            if (!st && learned) {
                st = w.warm->after_solve(w.V, lam_all.data(), sg->kpts + 3 * ik, o.learn_steps, o.learn_rate,
                                         w.stream);
                if (st) st = fail(st, "learned warm start: training step failed");
            }
        }
        if (st) {
            sg->status = st;
            sg->err = g_last_error;
            if (sg->bal) {
                std::lock_guard<std::mutex> lk(sg->bal->mu);
                sg->cur = -1;
            }
            return;
        }
        if (conv == 0) sg->worst = 0;
        else if (conv == 2 && sg->worst == 1) sg->worst = 2;
    }
}

// Autotuner: launch shapes of the Gram, update, stencil and FFT kernels for
// this grid and block shape, each the fastest of a few candidates timed with
// HIP events on the workspace's stream (full basis, random data).  Run once
// per context and block shape, before concurrent work starts.
int autotune(mfd_ctx* c, Ws& w, const double* k) {
    const size_t n = w.n;
    const int mb = w.mb;
    hipStream_t s = w.stream;
    OpParams p = params(c, k);
    p.wtmp = w.wtmp;
    HIPCHK(launch_fill_random(w.V, n * 6 * mb, 12345, s));
    if (w.mixed) {
        HIPCHK(launch_convert(w.V, w.V32, n * 6 * mb, true, s));
    }
    std::vector<int> all(mb);
    for (int j = 0; j < mb; ++j) all[j] = j;
    const BasisMap bm = make_basis(mb, all, all, w.mixed);
    HIPCHK(hipMemsetAsync(w.theta, 0, mb * sizeof(double), s));
    HIPCHK(hipMemsetAsync(w.C, 0, (size_t)3 * mb * mb * sizeof(double2), s));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto timeit = [&](auto&& launch) -> double {
        if (launch() != hipSuccess) return HUGE_VAL;   // also the warm-up
        float best = 1e30f;
        for (int r = 0; r < 3; ++r) {
            if (hipEventRecord(e0, s) != hipSuccess || launch() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess)
                return HUGE_VAL;
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            best = std::min(best, ms);
        }
        return best;
    };
    float2* V32 = w.mixed ? w.V32 : nullptr;
    float2* U32 = w.mixed ? w.U32 : nullptr;
    int best_gram = w.nparts_gram, best_upd = w.nparts_upd, best_wgs = 2048, best_xc = 0, best_rows = 0;
    double tb = HUGE_VAL;
    for (int np : {128, 256, 512, 1024}) {
        if (((size_t)np * 32 > n + 31 && np != w.nparts_gram) || np > w.cap_gram) continue;
        const double t = timeit([&] { return launch_gram_mfma(w.V, V32, n, n, bm, np, w.gpart, w.G, s); });
        if (t < tb) { tb = t; best_gram = np; }
    }
    tb = HUGE_VAL;
    for (int rows : {0, 32, 16})   // 0: one wave per 16-row strip, 4 per workgroup
        for (int np : {256, 512, 1024, 2048}) {
            const size_t rows_wg = rows ? (size_t)rows : 64;
            if (((size_t)np * rows_wg > n + rows_wg - 1 && np != w.nparts_upd) || np > w.cap_upd) continue;
            const double t = timeit([&] {
                return launch_update_mfma(w.V, V32, w.U, U32, n, n, bm, w.C, w.theta, np, w.npart, w.norms, s,
                                          rows);
            });
            if (t < tb) { tb = t; best_upd = np; best_rows = rows; }
        }
    tb = HUGE_VAL;
    for (int wg : {512, 1024, 2048, 4096}) {
        OpParams q = p;
        q.stencil_wgs = wg;
        const double t = timeit([&] {
            return w.mixed ? launch_stencil_f64_s32(q, mb, w.V32 + n * mb, w.V32 + n * 4 * mb, c->mu64, s)
                           : launch_stencil<double>(q, mb, col(w.V, n, mb), col(w.V, n, 4 * mb), c->mu64, s);
        });
        if (t < tb) { tb = t; best_wgs = wg; }
    }
    tb = HUGE_VAL;
    best_xc = 0;   // the built-in choice when no candidate applies
    for (int xc : {4, 8, 16, -1}) {   // -1: the register-resident passes (FP32, cubic order 2, N = 16, 32, 64)
        if (xc > 0 && c->N % xc) continue;
        if (xc < 0 && !(w.mixed && reg_precond_ok(p))) continue;
        OpParams q = p;
        q.fft_xc = xc;
        const double t = timeit([&] {
            if (w.mixed) return launch_precond<float>(q, mb, w.V32 + n * mb, w.V32 + n * mb, c->tw32, s);
            FieldList fl;
            fl.on = 1;
            for (int t = 0; t < mb; ++t) fl.idx[t] = (unsigned char)t;
            return precond_fp64(c, q, mb, col(w.V, n, mb), w.stage32, n, fl, s);
        });
        if (t < tb) { tb = t; best_xc = xc; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->tune_mb = mb;
    c->tune_mixed = w.mixed ? 1 : 0;
    c->tune[0] = best_gram;
    c->tune[1] = best_upd;
    c->tune[2] = best_wgs;
    c->tune[3] = best_xc;
    c->tune[4] = best_rows;
    return MFD_OK;
}

void apply_tune(const mfd_ctx* c, Ws& w) {
    if (c->tune_mb == 0) return;
    if (c->tune_mb > 0 && (c->tune_mb != w.mb || c->tune_mixed != (w.mixed ? 1 : 0))) return;
    // workgroup counts beyond what the partial buffers hold keep the built-in ones
    if (c->tune[0] <= w.cap_gram) w.nparts_gram = c->tune[0];
    if (c->tune[1] <= w.cap_upd) w.nparts_upd = c->tune[1];
    w.stencil_wgs = c->tune[2];
    w.fft_xc = c->tune[3];
    w.upd_rows = c->tune[4];
}

// Run segments on their workspaces, one host thread each; collect timing.
int run_segments(std::vector<Segment>& segs) {
    std::vector<std::thread> th;
    for (size_t i = 1; i < segs.size(); ++i) th.emplace_back(run_segment, &segs[i]);
    if (!segs.empty()) run_segment(&segs[0]);
    for (auto& t : th) t.join();
    for (auto& sg : segs) {
        sg.ws->prof.drain();
        sg.ctx->prof_done.add(sg.ws->prof);
        sg.ws->prof.clear();
    }
    for (auto& sg : segs)
        if (sg.status) return fail(sg.status, sg.err);
    int ret = MFD_OK;
    for (auto& sg : segs) {
        if (sg.worst == 2 && ret == MFD_OK) ret = fail(MFD_ESPURIOUS, "Alg 4.1 still flags a band");
        if (sg.worst == 0 && ret == MFD_OK) ret = fail(MFD_ENOTCONV, "max_iter reached");
    }
    return ret;
}

// Cold start from the lowest transverse plane waves at k.  With a uniform
// medium the operator's eigenvectors are plane waves exp(i (k + G) . x)
// (Section 4.4, Prop 3.2): the curl-curl part acts on the two polarisations
// perpendicular to k + G, the compensation term on the third.  Columns take,
// in order of |k + G|, those two polarisations of each reciprocal vector G
// (all three where k + G = 0), plus 0.1 of a seeded random block; G = 2 pi m / L
// on a cubic grid and 2 pi A^-T m on a lattice, m the grid frequency.
int planewave_start(const mfd_ctx* c, Ws& w, const double* k, int mb, uint64_t seed) {
    struct Cand {
        double len;
        int m[3];
        double q[3];
    };
    std::vector<Cand> cand;
    const int P = 3;
    for (int a = -P; a <= P; ++a)
        for (int b = -P; b <= P; ++b)
            for (int d = -P; d <= P; ++d) {
                Cand x;
                x.m[0] = a; x.m[1] = b; x.m[2] = d;
                double l2 = 0.0;
                for (int i = 0; i < 3; ++i) {
                    const double G = c->lattice ? 2.0 * M_PI / c->N * (c->B[i][0] * a + c->B[i][1] * b + c->B[i][2] * d)
                                                : 2.0 * M_PI * x.m[i] / c->L;
                    x.q[i] = k[i] + G;
                    l2 += x.q[i] * x.q[i];
                }
                x.len = std::sqrt(l2);
                cand.push_back(x);
            }
    std::stable_sort(cand.begin(), cand.end(), [](const Cand& u, const Cand& v) { return u.len < v.len; });
    PlaneWaves pw;
    pw.mb = mb;
    const double tiny = 1e-9 * 2.0 * M_PI / c->L;
    int j = 0;
    for (const Cand& x : cand) {
        if (j >= mb) break;
        double e[3][3];
        int npol = 2;
        if (x.len < tiny) {
            npol = 3;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) e[a][b] = a == b ? 1.0 : 0.0;
        } else {
            const double u[3] = {x.q[0] / x.len, x.q[1] / x.len, x.q[2] / x.len};
            // e1 = u x (the axis least aligned with u), normalised; e2 = u x e1
            int ax = 0;
            for (int i = 1; i < 3; ++i)
                if (std::fabs(u[i]) < std::fabs(u[ax])) ax = i;
            double t[3] = {0.0, 0.0, 0.0};
            t[ax] = 1.0;
            double e1[3] = {u[1] * t[2] - u[2] * t[1], u[2] * t[0] - u[0] * t[2], u[0] * t[1] - u[1] * t[0]};
            const double n1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
            for (int i = 0; i < 3; ++i) e[0][i] = e1[i] / n1;
            e[1][0] = u[1] * e[0][2] - u[2] * e[0][1];
            e[1][1] = u[2] * e[0][0] - u[0] * e[0][2];
            e[1][2] = u[0] * e[0][1] - u[1] * e[0][0];
        }
        for (int p = 0; p < npol && j < mb; ++p, ++j) {
            for (int i = 0; i < 3; ++i) {
                pw.m[j][i] = x.m[i];
                pw.pol[j][i] = mk<double2>(e[p][i], 0.0);
            }
        }
    }
    const size_t n = c->n;
    hipError_t e = launch_fill_random(w.V, n * mb, seed, w.stream);
    if (e == hipSuccess) e = launch_planewave_start(w.V, c->N, pw, 0.1, w.stream);
    return e == hipSuccess ? MFD_OK : fail(MFD_EDEVICE, hipGetErrorString(e));
}

int check_opts(const mfd_ctx* ctx, int nbands, double tol, const mfd_opts& o) {
    if (nbands <= 0) return fail(MFD_EINVAL, "nbands must be > 0");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(MFD_EINVAL, "tol must be finite and > 0");
    if (o.guard < 0 || o.max_iter < 1 || o.max_gamma_doublings < 0 || o.streams < 1 || o.streams > 16 ||
        o.stall_window < 0 || o.warm_start < 0 || o.warm_start > 2 || o.learn_steps < 0 || o.graph < 0 || o.graph > 1 ||
        o.cold_start < 0 || o.cold_start > 1 || o.balance < 0 || o.balance > 1 || o.hard_lock < 0 ||
        o.hard_lock > 1 ||
        (o.balance && o.warm_start == 2) || !(o.learn_rate >= 0.0f))
        return fail(MFD_EINVAL, "bad options");
    const int mb = nbands + o.guard;
    if (mb > MAX_BLOCK) return fail(MFD_EUNSUPPORTED, "nbands + guard exceeds mfd_max_block()");
    if ((size_t)mb > ctx->n) return fail(MFD_EINVAL, "nbands exceeds the problem size");
    if (o.precision != 0 && o.precision != 1) return fail(MFD_EINVAL, "precision must be 0 or 1");
    if (o.precond != 0 && o.precond != 1) return fail(MFD_EINVAL, "precond must be 0 or 1");
    if (o.precond == 1) {
        if (o.mg_cycles < 1 || o.mg_smooth < 0 || o.mg_sweeps < 0) return fail(MFD_EINVAL, "bad multigrid options");
        if (ctx->order != 2 || ctx->lattice || !mg_supported(ctx->N))
            return fail(MFD_EUNSUPPORTED, "multigrid needs a cubic order-2 context and a grid mfd_mg_supported accepts");
    }
    return MFD_OK;
}

}  // namespace

// Accessors for the other translation units of the library (noalloc.hip).
namespace mfd {
OpParams ctx_params(const mfd_ctx* ctx, const double k[3]) { return params(ctx, k); }
int ctx_device(const mfd_ctx* ctx) { return ctx->device; }
const void* ctx_mu64(const mfd_ctx* ctx) { return ctx->mu64; }
int set_error(int status, const char* msg) { return fail(status, msg); }
}  // namespace mfd

extern "C" {

void mfd_default_opts(mfd_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->max_iter = 400;
    o->precision = 0;
    o->warm_start = 1;
    o->seed = 0;
    o->max_gamma_doublings = 4;
    o->guard = 2;
    o->streams = 4;
    o->x0 = nullptr;
    o->stall_window = 40;
    o->learn_steps = 30;
    o->learn_rate = 1e-3f;
    o->autotune = 1;
    o->precond = 0;
    o->mg_cycles = 2;
    o->mg_smooth = 2;
    o->mg_sweeps = 2;
    o->graph = 0;
    o->cold_start = 0;
    o->balance = 0;
    o->hard_lock = 0;
}

int mfd_tuning(const mfd_ctx* ctx, int* out) {
    if (!ctx || !out) return fail(MFD_EINVAL, "NULL argument");
    for (int i = 0; i < 5; ++i) out[i] = ctx->tune[i];
    return ctx->tune_mb != 0 ? 1 : 0;
}

int mfd_set_tuning(mfd_ctx* ctx, const int* in) {
    if (!ctx) return fail(MFD_EINVAL, "ctx is NULL");
    if (!in) {
        ctx->tune_mb = 0;
        ctx->tune_mixed = -1;
        for (int i = 0; i < 5; ++i) ctx->tune[i] = 0;
        return MFD_OK;
    }
    auto one_of = [](int v, std::initializer_list<int> set) {
        for (int x : set)
            if (v == x) return true;
        return false;
    };
    if (!one_of(in[0], {128, 256, 512, 1024})) return fail(MFD_EINVAL, "Gram workgroups not a candidate");
    if (!one_of(in[1], {256, 512, 1024, 2048})) return fail(MFD_EINVAL, "update workgroups not a candidate");
    if (!one_of(in[2], {512, 1024, 2048, 4096})) return fail(MFD_EINVAL, "stencil workgroups not a candidate");
    if (!one_of(in[3], {0, 4, 8, 16, -1}) || (in[3] > 0 && ctx->N % in[3]))
        return fail(MFD_EINVAL, "FFT x run must be 0, -1, or 4, 8 or 16 dividing N");
    if (in[3] < 0) {
        const double k0[3] = {0.0, 0.0, 0.0};
        const OpParams q = ctx_params(ctx, k0);
        if (!reg_precond_ok(q)) return fail(MFD_EINVAL, "register-resident FFT passes need a cubic order-2 grid of 16, 32 or 64");
    }
    if (!one_of(in[4], {0, 16, 32})) return fail(MFD_EINVAL, "update form must be 0, 16 or 32");
    for (int i = 0; i < 5; ++i) ctx->tune[i] = in[i];
    ctx->tune_mb = -1;
    ctx->tune_mixed = -1;
    return MFD_OK;
}

int mfd_max_block(void) { return MAX_BLOCK; }

int mfd_supported_n(int N) {
    return (N >= 4 && N <= 150 && fft_supported(N, 4)) ? 1 : 0;
}

}  // extern "C"

namespace {

// A context from cell permittivities (mu_kernel forms M_0) or, when
// `edges`, from M_0 itself on the 3 N^3 edges.  `lat` (nullable): row-major
// 3 x 3 matrix whose columns are the lattice vectors; L is then |det|^(1/3).
int build_ctx(int N, double L, int order, const double* src, bool edges, void* stream, mfd_ctx** out,
              const double* lat = nullptr) {
    if (!out) return fail(MFD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!src) return fail(MFD_EINVAL, edges ? "mu_edges is NULL" : "eps_cells is NULL");
    if (N < 4 || N > 150) return fail(MFD_EINVAL, "N must be in [4, 150]");
    if (!(L > 0.0) || !std::isfinite(L)) return fail(MFD_EINVAL, "L must be finite and > 0");
    if (order != 2 && order != 4 && order != 6 && order != 8)
        return fail(MFD_EUNSUPPORTED, "stencil order must be 2, 4, 6 or 8");
    if (!mfd_supported_n(N)) return fail(MFD_EUNSUPPORTED, "no FFT plan for this N");
    double Bl[3][3] = {};
    if (lat) {
        double scale = 0.0;
        for (int i = 0; i < 9; ++i) {
            if (!std::isfinite(lat[i])) return fail(MFD_EINVAL, "lattice vectors must be finite");
            scale = std::max(scale, std::fabs(lat[i]));
        }
        auto a = [&](int r, int c) { return lat[3 * r + c]; };
        const double det = a(0, 0) * (a(1, 1) * a(2, 2) - a(1, 2) * a(2, 1)) -
                           a(0, 1) * (a(1, 0) * a(2, 2) - a(1, 2) * a(2, 0)) +
                           a(0, 2) * (a(1, 0) * a(2, 1) - a(1, 1) * a(2, 0));
        if (!(std::fabs(det) > 1e-12 * scale * scale * scale))
            return fail(MFD_EINVAL, "lattice vectors are linearly dependent");
        // inverse by cofactors: inv[r][c] = cof[c][r] / det
        double inv[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                const int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
                inv[r][c] = (a(r1, c1) * a(r2, c2) - a(r1, c2) * a(r2, c1)) / det;
            }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Bl[i][j] = N * inv[j][i];
        L = std::cbrt(std::fabs(det));
    }
    const size_t N3 = (size_t)N * N * N;
    const size_t count = edges ? 3 * N3 : N3;
    for (size_t i = 0; i < count; ++i)
        if (!std::isfinite(src[i]) || !(src[i] > 0.0))
            return fail(MFD_EINVAL, edges ? "mu must be finite and > 0" : "eps must be finite and > 0");
    hipStream_t s = (hipStream_t)stream;
    mfd_ctx* c = new mfd_ctx();
    c->N = N;
    c->L = L;
    c->h = L / N;
    c->order = order;
    c->n = 3 * N3;
    c->lattice = lat ? 1 : 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c->B[i][j] = Bl[i][j];
    hipGetDevice(&c->device);
    double* eps_d = nullptr;
    auto cleanup = [&](int st) {
        hipFree(eps_d);
        mfd_destroy(c);
        return st;
    };
    hipError_t e;
    const bool wide = order > 2;   // order 2 (cubic or lattice) needs no operator scratch
    if (wide) c->wtmp_bands = wide_bands(N);
    if ((wide && (e = hipMalloc(&c->wtmp, (size_t)c->wtmp_bands * 4 * N3 * sizeof(double2))) != hipSuccess) ||
        (e = hipMalloc(&c->mu64, 3 * N3 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&c->mu32, 3 * N3 * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&c->tw64, N * sizeof(double2))) != hipSuccess ||
        (e = hipMalloc(&c->tw32, N * sizeof(float2))) != hipSuccess ||
        (!edges && (e = hipMalloc(&eps_d, N3 * sizeof(double))) != hipSuccess))
        return cleanup(fail(MFD_ENOMEM, hipGetErrorString(e)));
    if (edges) {
        if ((e = hipMemcpyAsync(c->mu64, src, 3 * N3 * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess)
            return cleanup(fail(MFD_EDEVICE, hipGetErrorString(e)));
        hipLaunchKernelGGL(mu_copy_kernel, dim3(1024), dim3(256), 0, s, c->mu64, 3 * N3, c->mu32);
    } else {
        if ((e = hipMemcpyAsync(eps_d, src, N3 * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess)
            return cleanup(fail(MFD_EDEVICE, hipGetErrorString(e)));
        hipLaunchKernelGGL(mu_kernel, dim3(1024), dim3(256), 0, s, eps_d, N, c->mu64, c->mu32);
    }
    hipLaunchKernelGGL(twiddle_kernel, dim3((N + 127) / 128), dim3(128), 0, s, N, (double2*)c->tw64, (float2*)c->tw32);
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
        return cleanup(fail(MFD_EDEVICE, hipGetErrorString(e)));
    hipFree(eps_d);
    *out = c;
    return MFD_OK;
}

}  // namespace

extern "C" {

int mfd_build(int N, double L, int order, const double* eps_cells, void* stream, mfd_ctx** out) {
    return build_ctx(N, L, order, eps_cells, false, stream, out);
}

int mfd_build_mu(int N, double L, int order, const double* mu_edges, void* stream, mfd_ctx** out) {
    return build_ctx(N, L, order, mu_edges, true, stream, out);
}

int mfd_build_lattice(int N, const double* lattice, int order, const double* eps_cells, void* stream,
                      mfd_ctx** out) {
    if (!lattice) {
        if (out) *out = nullptr;
        return fail(MFD_EINVAL, "lattice is NULL");
    }
    return build_ctx(N, 1.0, order, eps_cells, false, stream, out, lattice);
}

int mfd_build_lattice_mu(int N, const double* lattice, int order, const double* mu_edges, void* stream,
                         mfd_ctx** out) {
    if (!lattice) {
        if (out) *out = nullptr;
        return fail(MFD_EINVAL, "lattice is NULL");
    }
    return build_ctx(N, 1.0, order, mu_edges, true, stream, out, lattice);
}

int mfd_gap_ratio(int nk, int nbands, const double* kpts, const double* evals, double* ratio, int* below) {
    if (!evals || !ratio || !below) return fail(MFD_EINVAL, "NULL argument");
    if (nk < 1 || nbands < 2) return fail(MFD_EINVAL, "need nk >= 1 and nbands >= 2");
    for (long long i = 0; i < (long long)nk * nbands; ++i)
        if (!std::isfinite(evals[i])) return fail(MFD_EINVAL, "evals must be finite");
    if (kpts)
        for (long long i = 0; i < 3LL * nk; ++i)
            if (!std::isfinite(kpts[i])) return fail(MFD_EINVAL, "kpts must be finite");
    // At k = 0 the returned bands 1-3 are the three constant fields; only two
    // of them continue bands as k -> 0, the third (along the direction of
    // approach) is static, so band b >= 3 of a k = 0 row is column b.
    auto col = [&](int i, int j) {
        const bool gamma = kpts && kpts[3 * i] == 0.0 && kpts[3 * i + 1] == 0.0 && kpts[3 * i + 2] == 0.0;
        return (gamma && j >= 2) ? j + 1 : j;
    };
    // omega = sqrt(lambda) in the units of lambda (the ratio is scale free);
    // the zero bands at Gamma can come out as roundoff below zero
    auto omega = [&](int i, int c) { return std::sqrt(std::max(evals[(size_t)i * nbands + c], 0.0)); };
    double best = -HUGE_VAL;
    int band = 0;
    for (int j = 0; j + 1 < nbands; ++j) {
        double low = -HUGE_VAL, up = HUGE_VAL;
        for (int i = 0; i < nk; ++i) {
            const int c0 = col(i, j), c1 = col(i, j + 1);
            if (c0 < nbands) low = std::max(low, omega(i, c0));
            if (c1 < nbands) up = std::min(up, omega(i, c1));
        }
        if (low == -HUGE_VAL || up == HUGE_VAL) continue;   // only k = 0 rows, which lack band j + 1
        const double r = (up - low) / (0.5 * (up + low));
        if (r > best) {
            best = r;
            band = j + 1;
        }
    }
    if (band == 0) return fail(MFD_EINVAL, "no band pair gives a ratio");
    *ratio = best;
    *below = band;
    return MFD_OK;
}

int mfd_set_gamma(mfd_ctx* ctx, double gamma) {
    if (!ctx) return fail(MFD_EINVAL, "ctx is NULL");
    if (!std::isfinite(gamma)) return fail(MFD_EINVAL, "gamma must be finite");
    ctx->gamma_override = gamma > 0.0 ? gamma : 0.0;
    return MFD_OK;
}

int mfd_gamma_shift(const mfd_ctx* ctx, const double k[3], double* gamma, double* shift) {
    if (!ctx || !k) return fail(MFD_EINVAL, "NULL argument");
    if (!finite3(k)) return fail(MFD_EINVAL, "k must be finite");
    OpParams p = params(ctx, k);
    if (gamma) *gamma = p.gamma;
    if (shift) *shift = p.shift;
    return MFD_OK;
}

// The direct operator and preconditioner calls take the launch shapes the
// autotuner chose (or mfd_set_tuning pinned) for this context, so that they
// run the kernel instances the band solve runs.
static void tuned_shapes(const mfd_ctx* ctx, OpParams& p) {
    if (ctx->tune_mb == 0) return;
    p.stencil_wgs = ctx->tune[2];
    p.fft_xc = ctx->tune[3];
}

static int check_block(mfd_ctx* ctx, const double* k, int nb, int dtype, const void* X, const void* Y,
                       bool allow_c64_f64 = false) {
    if (!ctx || !k || !X || !Y) return fail(MFD_EINVAL, "NULL argument");
    if (nb < 0) return fail(MFD_EINVAL, "nb < 0");
    if (dtype != MFD_C64 && dtype != MFD_C128 && !(allow_c64_f64 && dtype == MFD_C64_F64))
        return fail(MFD_EINVAL, allow_c64_f64 ? "dtype must be MFD_C64, MFD_C128 or MFD_C64_F64"
                                              : "dtype must be MFD_C64 or MFD_C128");
    if (!finite3(k)) return fail(MFD_EINVAL, "k must be finite");
    return MFD_OK;
}

int mfd_op_apply(mfd_ctx* ctx, const double k[3], int nb, int dtype, const void* X, void* Y, void* stream) {
    int st = check_block(ctx, k, nb, dtype, X, Y, true);
    if (st) return st;
    const size_t bytes = ctx->n * nb * (dtype == MFD_C128 ? 16 : 8);
    const char* x = (const char*)X;
    const char* y = (const char*)Y;
    if (nb > 0 && x < y + bytes && y < x + bytes) return fail(MFD_EINVAL, "X and Y overlap");
    if (nb == 0) return MFD_OK;
    OpParams p = params(ctx, k);
    tuned_shapes(ctx, p);
    hipStream_t s = (hipStream_t)stream;
    if (dtype == MFD_C128) HIPCHK(launch_stencil<double>(p, nb, X, Y, ctx->mu64, s));
    else if (dtype == MFD_C64_F64) HIPCHK(launch_stencil_f64_s32(p, nb, X, Y, ctx->mu64, s));
    else HIPCHK(launch_stencil<float>(p, nb, X, Y, ctx->mu32, s));
    return MFD_OK;
}

int mfd_precond_solve(mfd_ctx* ctx, const double k[3], int nb, int dtype, const void* R, void* T, void* stream) {
    int st = check_block(ctx, k, nb, dtype, R, T);
    if (st) return st;
    if (nb == 0) return MFD_OK;
    const size_t bytes = ctx->n * nb * (dtype == MFD_C64 ? 8 : 16);
    const char* r = (const char*)R;
    const char* t = (const char*)T;
    if (r != t && r < t + bytes && t < r + bytes) return fail(MFD_EINVAL, "R and T overlap partially");
    if (!fft_supported(ctx->N, dtype == MFD_C64 ? 4 : 8))
        return fail(MFD_EUNSUPPORTED, "no FFT plan for this N and precision");
    OpParams p = params(ctx, k);
    tuned_shapes(ctx, p);
    hipStream_t s = (hipStream_t)stream;
    if (dtype == MFD_C128) HIPCHK(launch_precond<double>(p, nb, R, T, ctx->tw64, s));
    else HIPCHK(launch_precond<float>(p, nb, R, T, ctx->tw32, s));
    return MFD_OK;
}

int mfd_mg_supported(int N) { return mg_supported(N) ? 1 : 0; }

int mfd_precond_solve_mg(mfd_ctx* ctx, const double k[3], int nb, int dtype, int cycles, int smooth, int sweeps,
                         const void* R, void* T, void* stream) {
    int st = check_block(ctx, k, nb, dtype, R, T);
    if (st) return st;
    if (cycles < 1 || smooth < 0 || sweeps < 0) return fail(MFD_EINVAL, "bad multigrid options");
    if (ctx->order != 2 || ctx->lattice || !mg_supported(ctx->N))
        return fail(MFD_EUNSUPPORTED, "multigrid needs a cubic order-2 context and a grid mfd_mg_supported accepts");
    if (nb == 0) return MFD_OK;
    const size_t bytes = ctx->n * nb * (dtype == MFD_C64 ? 8 : 16);
    const char* r = (const char*)R;
    const char* t = (const char*)T;
    if (r != t && r < t + bytes && t < r + bytes) return fail(MFD_EINVAL, "R and T overlap partially");
    if (!ctx->mg) ctx->mg = mg_create();
    MGOpts o;
    o.cycles = cycles;
    o.n1 = o.n2 = smooth;
    o.sweeps = sweeps;
    OpParams p = params(ctx, k);
    hipStream_t s = (hipStream_t)stream;
    if (dtype == MFD_C128) HIPCHK(launch_precond_mg<double2>(ctx->mg, p, o, nb, R, T, s));
    else HIPCHK(launch_precond_mg<float2>(ctx->mg, p, o, nb, R, T, s));
    return MFD_OK;
}

int mfd_lambda_re(mfd_ctx* ctx, const double k[3], int nb, const void* X, double* out, void* stream) {
    if (!ctx || !k || !X || !out) return fail(MFD_EINVAL, "NULL argument");
    if (nb <= 0) return fail(MFD_EINVAL, "nb must be > 0");
    if (!finite3(k)) return fail(MFD_EINVAL, "k must be finite");
    OpParams p = params(ctx, k);
    hipStream_t s = (hipStream_t)stream;
    const int nparts = 128;
    double *part = nullptr, *res = nullptr;
    HIPCHK(hipMalloc(&part, (size_t)nparts * 2 * nb * sizeof(double)));
    hipError_t e = hipMalloc(&res, 2 * nb * sizeof(double));
    if (e != hipSuccess) { hipFree(part); return fail(MFD_ENOMEM, hipGetErrorString(e)); }
    std::vector<double> h(2 * nb);
    e = launch_lambda_re(p, nb, X, ctx->mu64, part, nparts, res, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), res, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(part);
    hipFree(res);
    if (e != hipSuccess) return fail(MFD_EDEVICE, hipGetErrorString(e));
    for (int b = 0; b < nb; ++b) out[b] = h[2 * b] / h[2 * b + 1];
    return MFD_OK;
}

int mfd_bands(mfd_ctx* ctx, int nk, const double* kpts, int nbands, double tol, const mfd_opts* opts,
              double* evals, void* evecs, mfd_kstats* stats, void* stream) {
    if (!ctx || !kpts || !evals) return fail(MFD_EINVAL, "NULL argument");
    if (nk <= 0) return fail(MFD_EINVAL, "nk must be > 0");
    mfd_opts o;
    mfd_default_opts(&o);
    if (opts) o = *opts;
    int st = check_opts(ctx, nbands, tol, o);
    if (st) return st;
    for (int i = 0; i < 3 * nk; ++i)
        if (!std::isfinite(kpts[i])) return fail(MFD_EINVAL, "k must be finite");
    const int mb = nbands + o.guard;
    const int nseg = std::min(o.streams, nk);
    if ((st = ensure_ws(ctx, mb, o.precision == 1, nseg))) return st;
    // the workspaces' streams start after the caller's stream work
    hipEvent_t ready;
    HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ready, (hipStream_t)stream));
    for (int i = 0; i < nseg; ++i) HIPCHK(hipStreamWaitEvent(ctx->ws[i]->stream, ready, 0));
    hipEventDestroy(ready);
    if (o.autotune && ctx->tune_mb >= 0 && (ctx->tune_mb != mb || ctx->tune_mixed != (o.precision == 1 ? 1 : 0)))
        if ((st = autotune(ctx, *ctx->ws[0], kpts))) return st;
    for (int i = 0; i < nseg; ++i) apply_tune(ctx, *ctx->ws[i]);
    std::vector<Segment> segs(nseg);
    for (int i = 0; i < nseg; ++i) {
        Segment& sg = segs[i];
        sg.ctx = ctx;
        sg.ws = ctx->ws[i];
        sg.kpts = kpts;
        sg.k0 = (int)((long long)nk * i / nseg);
        sg.k1 = (int)((long long)nk * (i + 1) / nseg);
        sg.nbands = nbands;
        sg.tol = tol;
        sg.opts = o;
        sg.evals = evals;
        sg.evecs = (double2*)evecs;
        sg.stats = stats;
    }
    Balance bal;
    if (o.balance) {
        for (auto& sg : segs) {
            sg.bal = &bal;
            bal.segs.push_back(&sg);
        }
    }
    return run_segments(segs);
}

int mfd_bands_batch(int ncrys, mfd_ctx* const* ctxs, const int* nk, const double* const* kpts, int nbands,
                    double tol, const mfd_opts* opts, double* const* evals, mfd_kstats* const* stats, void* stream) {
    if (ncrys <= 0 || !ctxs || !nk || !kpts || !evals) return fail(MFD_EINVAL, "NULL or empty argument");
    mfd_opts o;
    mfd_default_opts(&o);
    if (opts) o = *opts;
    if (o.x0) return fail(MFD_EINVAL, "x0 is not used by the batch call");
    const int mb = nbands + o.guard;
    for (int c = 0; c < ncrys; ++c) {
        if (!ctxs[c] || !kpts[c] || !evals[c] || nk[c] <= 0) return fail(MFD_EINVAL, "bad crystal entry");
        int st = check_opts(ctxs[c], nbands, tol, o);
        if (st) return st;
        for (int i = 0; i < 3 * nk[c]; ++i)
            if (!std::isfinite(kpts[c][i])) return fail(MFD_EINVAL, "k must be finite");
        for (int d = 0; d < c; ++d)
            if (ctxs[d] == ctxs[c]) return fail(MFD_EINVAL, "a context appears twice in the batch");
    }
    // crystals are taken in the caller's order by `streams` workers.  Largest
    // grid first measured slower (32 crystals of N = 24..64 interleaved:
    // 27 -> 16 k-points/s): the small solves are bound by their per-iteration
    // host round trip, and run side by side with large ones their latency
    // hides behind the large ones' kernels
    hipEvent_t ready;
    HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ready, (hipStream_t)stream));
    std::vector<Segment> segs(ncrys);
    for (int c = 0; c < ncrys; ++c) {
        int st = ensure_ws(ctxs[c], mb, o.precision == 1, 1);
        if (st) { hipEventDestroy(ready); return st; }
        HIPCHK(hipStreamWaitEvent(ctxs[c]->ws[0]->stream, ready, 0));
        if (o.autotune && ctxs[c]->tune_mb >= 0 &&
            (ctxs[c]->tune_mb != mb || ctxs[c]->tune_mixed != (o.precision == 1 ? 1 : 0)))
            if ((st = autotune(ctxs[c], *ctxs[c]->ws[0], kpts[c]))) { hipEventDestroy(ready); return st; }
        apply_tune(ctxs[c], *ctxs[c]->ws[0]);
        Segment& sg = segs[c];
        sg.ctx = ctxs[c];
        sg.ws = ctxs[c]->ws[0];
        sg.kpts = kpts[c];
        sg.k0 = 0;
        sg.k1 = nk[c];
        sg.nbands = nbands;
        sg.tol = tol;
        sg.opts = o;
        sg.evals = evals[c];
        sg.evecs = nullptr;
        sg.stats = stats ? stats[c] : nullptr;
    }
    hipEventDestroy(ready);
    const int nw = std::min(o.streams, ncrys);
    std::atomic<int> next(0);
    auto worker = [&]() {
        for (int c; (c = next.fetch_add(1)) < ncrys;) run_segment(&segs[c]);
    };
    std::vector<std::thread> th;
    for (int i = 1; i < nw; ++i) th.emplace_back(worker);
    worker();
    for (auto& t : th) t.join();
    for (auto& sg : segs) {
        sg.ws->prof.drain();
        sg.ctx->prof_done.add(sg.ws->prof);
        sg.ws->prof.clear();
    }
    for (auto& sg : segs)
        if (sg.status) return fail(sg.status, sg.err);
    int ret = MFD_OK;
    for (auto& sg : segs) {
        if (sg.worst == 2 && ret == MFD_OK) ret = fail(MFD_ESPURIOUS, "Alg 4.1 still flags a band");
        if (sg.worst == 0 && ret == MFD_OK) ret = fail(MFD_ENOTCONV, "max_iter reached");
    }
    return ret;
}

int mfd_profile(mfd_ctx* ctx, int enable) {
    if (!ctx) return fail(MFD_EINVAL, "ctx is NULL");
    ctx->prof_on = enable != 0;
    ctx->prof_done.clear();
    for (Ws* w : ctx->ws) {
        w->prof.drain();
        w->prof.clear();
        w->prof.on = ctx->prof_on;
    }
    return MFD_OK;
}

int mfd_profile_read(mfd_ctx* ctx, double* ms, long long* count, double* bytes) {
    if (!ctx || !ms || !count || !bytes) return fail(MFD_EINVAL, "NULL argument");
    for (int i = 0; i < Prof::NCAT; ++i) {
        ms[i] = ctx->prof_done.ms[i];
        count[i] = ctx->prof_done.count[i];
        bytes[i] = ctx->prof_done.bytes[i];
    }
    return MFD_OK;
}

void mfd_destroy(mfd_ctx* ctx) {
    if (!ctx) return;
    for (Ws* w : ctx->ws) ws_free(w);
    ctx->ws.clear();
    hipFree(ctx->mu64);
    hipFree(ctx->mu32);
    hipFree(ctx->tw64);
    hipFree(ctx->tw32);
    hipFree(ctx->wtmp);
    mg_destroy(ctx->mg);
    delete ctx;
}

const char* mfd_strerror(int status) {
    switch (status) {
        case MFD_OK: return "ok";
        case MFD_EINVAL: return "invalid argument";
        case MFD_ENOMEM: return "out of device memory";
        case MFD_EDEVICE: return "device error";
        case MFD_ENOTCONV: return "not converged";
        case MFD_ESPURIOUS: return "spurious eigenvalue persists";
        case MFD_EUNSUPPORTED: return "unsupported size or order";
        default: return "unknown status";
    }
}

const char* mfd_last_error(void) { return g_last_error.c_str(); }

struct mfd_mlp {
    mfd::Mlp net;
};

int mfd_mlp_create(int nin, int nhidden, int nlayers, int nout, int max_batch, int bf16_weights,
                   unsigned long long seed, mfd_mlp** out) {
    if (!out) return fail(MFD_EINVAL, "out is NULL");
    *out = nullptr;
    if (nin < 1 || nout < 1 || nlayers < 0 || (nlayers > 0 && nhidden < 1) || max_batch < 1)
        return fail(MFD_EINVAL, "bad network sizes");
    mfd_mlp* m = new mfd_mlp();
    const int st = m->net.init(nin, nlayers > 0 ? nhidden : 0, nlayers, nout, max_batch, bf16_weights != 0, seed);
    if (st) {
        m->net.release();
        delete m;
        return fail(st, "network allocation failed");
    }
    *out = m;
    return MFD_OK;
}

long long mfd_mlp_num_params(const mfd_mlp* m) { return m ? (long long)m->net.nparam : 0; }

int mfd_mlp_set_params(mfd_mlp* m, const float* params) {
    if (!m || !params) return fail(MFD_EINVAL, "NULL argument");
    const int st = m->net.set_params(params, nullptr);
    return st ? fail(st, "set_params failed") : MFD_OK;
}

int mfd_mlp_get_params(mfd_mlp* m, float* params) {
    if (!m || !params) return fail(MFD_EINVAL, "NULL argument");
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(params, m->net.p, m->net.nparam * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(MFD_EDEVICE, "copy failed");
    return MFD_OK;
}

int mfd_mlp_forward(mfd_mlp* m, int batch, const float* X, float* Y, void* stream) {
    if (!m || !X || !Y) return fail(MFD_EINVAL, "NULL argument");
    if (batch < 1 || batch > m->net.bmax) return fail(MFD_EINVAL, "batch out of range");
    if (m->net.forward(batch, X, Y, (hipStream_t)stream) != hipSuccess) return fail(MFD_EDEVICE, "launch failed");
    return MFD_OK;
}

int mfd_mlp_loss_grad(mfd_mlp* m, int batch, const float* X, const float* T, double* loss, float* grad,
                      void* stream) {
    if (!m || !X || !T || !loss) return fail(MFD_EINVAL, "NULL argument");
    if (batch < 1 || batch > m->net.bmax) return fail(MFD_EINVAL, "batch out of range");
    hipStream_t s = (hipStream_t)stream;
    if (m->net.loss_grad(batch, X, T, s) != hipSuccess) return fail(MFD_EDEVICE, "launch failed");
    if (grad && hipMemcpyAsync(grad, m->net.g, m->net.nparam * sizeof(float), hipMemcpyDeviceToDevice, s) !=
                    hipSuccess)
        return fail(MFD_EDEVICE, "copy failed");
    if (hipMemcpyAsync(loss, m->net.dloss, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(MFD_EDEVICE, "copy failed");
    return MFD_OK;
}

int mfd_mlp_adam_step(mfd_mlp* m, float lr, void* stream) {
    if (!m) return fail(MFD_EINVAL, "NULL argument");
    if (!(lr >= 0.0f)) return fail(MFD_EINVAL, "learning rate must be >= 0");
    if (m->net.adam(lr, (hipStream_t)stream) != hipSuccess) return fail(MFD_EDEVICE, "launch failed");
    return MFD_OK;
}

void mfd_mlp_destroy(mfd_mlp* m) {
    if (!m) return;
    m->net.release();
    delete m;
}

int mfd_warm_target(long long n, int mb, const void* Xa, const void* Xb, const void* Xc, void* C, void* Rinv,
                    void* stream) {
    if (!Xa || !Xb || !Xc || !C) return fail(MFD_EINVAL, "NULL argument");
    if (n < 1 || mb < 1 || mb > 22 || 2 * mb > n) return fail(MFD_EINVAL, "bad sizes");
    const int st = mfd::warm_target_blocks((size_t)n, mb, (const double2*)Xa, (const double2*)Xb,
                                           (const double2*)Xc, (double2*)C, (double2*)Rinv, (hipStream_t)stream);
    if (st == MFD_ENOTCONV) return fail(st, "history blocks are numerically dependent");
    return st ? fail(st, "warm target failed") : MFD_OK;
}

int mfd_warm_features(double L, int mb, const double* k_prev, const double* k_next, const double* lam_j,
                      const double* lam_jm1, const void* C, float* row, void* stream) {
    if (!k_prev || !k_next || !lam_j || !lam_jm1 || !C || !row) return fail(MFD_EINVAL, "NULL argument");
    if (!(L > 0.0) || mb < 1 || mb > 22) return fail(MFD_EINVAL, "bad sizes");
    std::vector<float> stage(6 + 2 * mb);
    hipStream_t s = (hipStream_t)stream;
    if (mfd::warm_feature_row(L, mb, k_prev, k_next, lam_j, lam_jm1, (const double2*)C, row, stage.data(), s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(MFD_EDEVICE, "feature row failed");
    return MFD_OK;
}

}  // extern "C"
