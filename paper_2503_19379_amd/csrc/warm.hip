// Learned warm start of the band solve along a k-path.
//
// After each converged k-point the three latest blocks X_{j-1}, X_j, X_{j+1}
// (n x mb each) give one training pair for the network:
//   Y_j = [X_j X_{j-1}] R^-1     (R^H R = Gram of [X_j X_{j-1}], Cholesky),
//   C*  = Y_j^H X_{j+1} Q,       Q = the unitary polar factor of X_{j+1}^H X_j
// (Q is the closest unitary aligning X_{j+1} with X_j; it removes the phases
// and in-cluster rotations an eigensolver leaves arbitrary).  The network sees
// k_{j+1}, k_{j+1} - k_j, the Ritz values at k_j and k_{j-1} and the previous
// target C*_j, and learns the change C*_{j+1} - C*_j.  At the next k-point the
// proposal is X0 = Y_{j+1} (C*_{j+1} + network output), built from the basis
// of [X_{j+1} X_j]; it enters the first LOBPCG step beside the previous-k
// block, so the first Rayleigh-Ritz step picks the best of both.
//
// All inner products come from one Gram of the three history slots; the small
// dense algebra (Cholesky, triangular inverse, Hermitian Jacobi for the polar
// factor) runs in one workgroup.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "common.h"
#include "mlp.h"
#include "solver.h"

namespace mfd {

using C128 = double2;
constexpr int WS_NT = 256;
constexpr int WS_MB = 22;        // mb <= 22
constexpr int WS_K2 = 2 * WS_MB;

// Upper Cholesky factor in place (A = R^H R, lower part zeroed).  Returns false
// when a pivot falls below tol times the largest diagonal entry.
__device__ bool chol_upper(C128* A, int n, int ld, double tol, double* piv_s, int* ok_s) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        double dmax = 0.0;
        for (int j = 0; j < n; ++j) dmax = fmax(dmax, A[j * ld + j].x);
        piv_s[1] = dmax;
        *ok_s = 1;
    }
    __syncthreads();
    const double dmax = piv_s[1];
    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            const double p = A[j * ld + j].x;
            if (!(p > tol * dmax)) *ok_s = 0;
            piv_s[0] = (p > 0.0) ? sqrt(p) : 1.0;
        }
        __syncthreads();
        const double d = piv_s[0];
        for (int l = j + 1 + tid; l < n; l += WS_NT) A[j * ld + l] = cscale(A[j * ld + l], 1.0 / d);
        if (tid == 0) A[j * ld + j] = mk<C128>(d, 0.0);
        __syncthreads();
        const int m = n - j - 1;
        for (int e = tid; e < m * m; e += WS_NT) {
            const int i = j + 1 + e / m, l = j + 1 + e % m;
            if (l >= i) A[i * ld + l] = csub(A[i * ld + l], cmulc(A[j * ld + i], A[j * ld + l]));
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += WS_NT)
        if (e / n > e % n) A[(e / n) * ld + e % n] = mk<C128>(0.0, 0.0);
    __syncthreads();
    return *ok_s != 0;
}

// Ri = R^-1 for upper triangular R (one column per thread).
__device__ void tri_inv_upper(const C128* R, C128* Ri, int n, int ld) {
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += WS_NT) Ri[(e / n) * ld + e % n] = mk<C128>(0.0, 0.0);
    __syncthreads();
    for (int j = tid; j < n; j += WS_NT) {
        Ri[j * ld + j] = mk<C128>(1.0 / R[j * ld + j].x, 0.0);
        for (int i = j - 1; i >= 0; --i) {
            C128 s = mk<C128>(0.0, 0.0);
            for (int k = i + 1; k <= j; ++k) s = cfma(s, R[i * ld + k], Ri[k * ld + j]);
            Ri[i * ld + j] = cscale(s, -1.0 / R[i * ld + i].x);
        }
    }
    __syncthreads();
}

// Eigen-decomposition of the Hermitian n x n matrix H (in place, becomes
// diagonal) by cyclic two-sided Jacobi; V <- the eigenvectors (columns).
__device__ void jacobi_herm(C128* H, C128* V, int n, int ld, double* sh) {
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += WS_NT) V[(e / n) * ld + e % n] = mk<C128>((e / n) == (e % n) ? 1.0 : 0.0, 0.0);
    __syncthreads();
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) {
            double off = 0.0, dia = 0.0;
            for (int i = 0; i < n; ++i)
                for (int l = 0; l < n; ++l) {
                    const double a = cabs2(H[i * ld + l]);
                    if (i == l) dia += a; else off += a;
                }
            sh[0] = (off <= 1e-30 * dia) ? 1.0 : 0.0;
        }
        __syncthreads();
        if (sh[0] != 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                __syncthreads();   // every thread has read the previous pair's flag
                if (tid == 0) {
                    const C128 c = H[p * ld + q];
                    const double r = sqrt(cabs2(c));
                    const double a = H[p * ld + p].x, b = H[q * ld + q].x;
                    if (r <= 1e-300 || r <= 1e-18 * sqrt(fabs(a * b))) {
                        sh[1] = 0.0;   // skip
                    } else {
                        const double tau = (b - a) / (2.0 * r);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        const double cs = 1.0 / sqrt(1.0 + t * t);
                        sh[1] = 1.0;
                        sh[2] = cs;
                        sh[3] = t * cs;
                        sh[4] = c.x / r;    // e^{i phi}
                        sh[5] = c.y / r;
                        sh[6] = a - t * r;
                        sh[7] = b + t * r;
                    }
                }
                __syncthreads();
                if (sh[1] == 0.0) continue;   // uniform: every thread reads the same flag
                const double cs = sh[2], sn = sh[3];
                const C128 e = mk<C128>(sh[4], sh[5]), ec = mk<C128>(sh[4], -sh[5]);
                // columns: H J and V J, J = [[cs, sn], [-sn e^-i, cs e^-i]]
                for (int i = tid; i < n; i += WS_NT) {
                    const C128 hp = H[i * ld + p], hq = cmul(H[i * ld + q], ec);
                    H[i * ld + p] = csub(cscale(hp, cs), cscale(hq, sn));
                    H[i * ld + q] = cadd(cscale(hp, sn), cscale(hq, cs));
                    const C128 vp = V[i * ld + p], vq = cmul(V[i * ld + q], ec);
                    V[i * ld + p] = csub(cscale(vp, cs), cscale(vq, sn));
                    V[i * ld + q] = cadd(cscale(vp, sn), cscale(vq, cs));
                }
                __syncthreads();
                // rows: J^H H, J^H = [[cs, -sn e^i], [sn, cs e^i]]
                for (int l = tid; l < n; l += WS_NT) {
                    const C128 hp = H[p * ld + l], hq = cmul(e, H[q * ld + l]);
                    H[p * ld + l] = csub(cscale(hp, cs), cscale(hq, sn));
                    H[q * ld + l] = cadd(cscale(hp, sn), cscale(hq, cs));
                }
                __syncthreads();
                if (tid == 0) {
                    H[p * ld + q] = mk<C128>(0.0, 0.0);
                    H[q * ld + p] = mk<C128>(0.0, 0.0);
                    H[p * ld + p] = mk<C128>(sh[6], 0.0);
                    H[q * ld + q] = mk<C128>(sh[7], 0.0);
                }
                __syncthreads();
            }
    }
    __syncthreads();
}

struct TargetArgs {
    const C128* G;     // 3mb x 3mb, slots in physical order
    int mb, a, b, c;   // slot of X_{j-1}, X_j, X_{j+1}
    C128* Cout;        // 2mb x mb
    C128* Qout;        // mb x mb: the polar factor aligning X_{j+1} with X_j
    C128* Rinv;        // 2mb x 2mb: R^-1 of [X_c Q, X_b]
    int* status;       // 0 ok; 1: [X_b X_a] dependent; 2: [X_c X_b] dependent
};

__global__ __launch_bounds__(WS_NT) void warm_target_kernel(TargetArgs t) {
    extern __shared__ unsigned char smem_raw[];
    C128* Z = reinterpret_cast<C128*>(smem_raw);     // K2 x K2
    C128* Ri = Z + WS_K2 * WS_K2;                      // K2 x K2
    C128* E = Ri + WS_K2 * WS_K2;                      // K2 x mb
    C128* A = E + WS_K2 * WS_MB;                       // mb x mb
    C128* Hm = A + WS_MB * WS_MB;
    C128* V = Hm + WS_MB * WS_MB;
    C128* Q = V + WS_MB * WS_MB;
    __shared__ double sh[8];
    __shared__ double piv_s[2];
    __shared__ int ok_s;
    const int tid = threadIdx.x;
    const int mb = t.mb, K2 = 2 * mb, Q3 = 3 * mb;
    const int ld = WS_K2, lm = WS_MB;
    auto ph = [&](int slotA, int slotB, int i) { return i < mb ? slotA * mb + i : slotB * mb + i - mb; };
    auto g = [&](int i, int j) { return t.G[i * Q3 + j]; };

    // 1. polar factor Q of A = X_c^H X_b: Hm = A^H A = V diag(s) V^H, Q = A V diag(s^-1/2) V^H
    for (int e = tid; e < mb * mb; e += WS_NT) {
        const int p = e / mb, q = e % mb;
        A[p * lm + q] = g(t.c * mb + p, t.b * mb + q);
    }
    __syncthreads();
    for (int e = tid; e < mb * mb; e += WS_NT) {
        const int p = e / mb, q = e % mb;
        C128 s = mk<C128>(0.0, 0.0);
        for (int k = 0; k < mb; ++k) s = cfmac(s, A[k * lm + p], A[k * lm + q]);
        Hm[p * lm + q] = s;
    }
    __syncthreads();
    jacobi_herm(Hm, V, mb, lm, sh);
    if (tid == 0) {
        double smax = 0.0;
        for (int q = 0; q < mb; ++q) smax = fmax(smax, Hm[q * lm + q].x);
        sh[0] = smax;
    }
    __syncthreads();
    const double smax = sh[0];
    for (int e = tid; e < mb * mb; e += WS_NT) {   // E <- A V diag(s^-1/2)
        const int p = e / mb, q = e % mb;
        C128 s = mk<C128>(0.0, 0.0);
        for (int k = 0; k < mb; ++k) s = cfma(s, A[p * lm + k], V[k * lm + q]);
        const double sv = Hm[q * lm + q].x;
        E[p * lm + q] = cscale(s, sv > 1e-24 * smax ? 1.0 / sqrt(sv) : 0.0);
    }
    __syncthreads();
    for (int e = tid; e < mb * mb; e += WS_NT) {
        const int p = e / mb, q = e % mb;
        C128 s = mk<C128>(0.0, 0.0);
        for (int k = 0; k < mb; ++k) s = cfma(s, E[p * lm + k], cconj(V[q * lm + k]));
        Q[p * lm + q] = s;
        t.Qout[p * mb + q] = s;
    }
    __syncthreads();

    // 2. target C* = Ri^H [X_b X_a]^H X_c Q with Ri = R^-1, R^H R = Gram of [X_b X_a]
    for (int e = tid; e < K2 * K2; e += WS_NT) {
        const int i = e / K2, l = e % K2;
        Z[i * ld + l] = g(ph(t.b, t.a, i), ph(t.b, t.a, l));
    }
    for (int e = tid; e < K2 * mb; e += WS_NT) {   // E = [X_b X_a]^H X_c Q
        const int i = e / mb, q = e % mb;
        C128 s = mk<C128>(0.0, 0.0);
        for (int k = 0; k < mb; ++k) s = cfma(s, g(ph(t.b, t.a, i), t.c * mb + k), Q[k * lm + q]);
        E[i * lm + q] = s;
    }
    __syncthreads();
    int status = 0;
    if (!chol_upper(Z, K2, ld, 1e-10, piv_s, &ok_s)) status = 1;
    if (status == 0) {
        tri_inv_upper(Z, Ri, K2, ld);
        for (int e = tid; e < K2 * mb; e += WS_NT) {
            const int i = e / mb, q = e % mb;
            C128 s = mk<C128>(0.0, 0.0);
            for (int k = 0; k <= i; ++k) s = cfmac(s, Ri[k * ld + i], E[k * lm + q]);
            t.Cout[i * mb + q] = s;
        }
        __syncthreads();
    }

    // 3. basis of [X_c Q, X_b] for the next proposal: its Gram from G and Q
    for (int e = tid; e < K2 * K2; e += WS_NT) {
        const int i = e / K2, l = e % K2;
        C128 v;
        if (i >= mb && l >= mb) {
            v = g(t.b * mb + i - mb, t.b * mb + l - mb);
        } else if (i < mb && l >= mb) {   // (Q^H X_c^H X_b)[i][l]
            v = mk<C128>(0.0, 0.0);
            for (int k = 0; k < mb; ++k) v = cfmac(v, Q[k * lm + i], g(t.c * mb + k, t.b * mb + l - mb));
        } else if (i >= mb && l < mb) {   // (X_b^H X_c Q)[i][l]
            v = mk<C128>(0.0, 0.0);
            for (int k = 0; k < mb; ++k) v = cfma(v, g(t.b * mb + i - mb, t.c * mb + k), Q[k * lm + l]);
        } else {                          // (Q^H X_c^H X_c Q)[i][l]
            v = mk<C128>(0.0, 0.0);
            for (int k = 0; k < mb; ++k) {
                C128 u = mk<C128>(0.0, 0.0);
                for (int r = 0; r < mb; ++r) u = cfma(u, g(t.c * mb + k, t.c * mb + r), Q[r * lm + l]);
                v = cfmac(v, Q[k * lm + i], u);
            }
        }
        Z[i * ld + l] = v;
    }
    __syncthreads();
    const bool ok2 = chol_upper(Z, K2, ld, 1e-10, piv_s, &ok_s);
    if (ok2) {
        tri_inv_upper(Z, Ri, K2, ld);
        for (int e = tid; e < K2 * K2; e += WS_NT) t.Rinv[e] = Ri[(e / K2) * ld + e % K2];
    }
    if (tid == 0) *t.status = status ? status : (ok2 ? 0 : 2);
}

// X <- X Q in place (n x mb c128 column-major; one row per thread).
__global__ __launch_bounds__(256) void warm_rotate_kernel(C128* __restrict__ X, size_t n, int mb,
                                                          const C128* __restrict__ Qg) {
    __shared__ C128 Qs[WS_MB * WS_MB];
    for (int e = threadIdx.x; e < mb * mb; e += blockDim.x) Qs[e] = Qg[e];
    __syncthreads();
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    C128 x[WS_MB], y[WS_MB];
#pragma unroll
    for (int k = 0; k < WS_MB; ++k) x[k] = (k < mb) ? X[(size_t)k * n + r] : mk<C128>(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < WS_MB; ++q) {
        y[q] = mk<C128>(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < WS_MB; ++k)
            if (k < mb && q < mb) y[q] = cfma(y[q], x[k], Qs[k * mb + q]);
    }
#pragma unroll
    for (int q = 0; q < WS_MB; ++q)
        if (q < mb) X[(size_t)q * n + r] = y[q];
}

// D = Rinv (Cb + pred): the proposal coefficients over [X_c X_b].
__global__ void warm_coef_kernel(const C128* __restrict__ Rinv, const C128* __restrict__ Cb,
                                 const float* __restrict__ pred, int mb, C128* __restrict__ D) {
    const int K2 = 2 * mb;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K2 * mb) return;
    const int i = e / mb, q = e % mb;
    C128 s = mk<C128>(0.0, 0.0);
    for (int k = i; k < K2; ++k) {
        const C128 ch = cadd(Cb[k * mb + q], mk<C128>(pred[2 * (k * mb + q)], pred[2 * (k * mb + q) + 1]));
        s = cfma(s, Rinv[i * K2 + k], ch);
    }
    D[e] = s;
}

// W[:, q] = sum_l B_l D[l][q], B = [H slot c | H slot b] (c128 in; c128 or c64 out).
template <class S>
__global__ __launch_bounds__(256) void warm_combine_kernel(const C128* __restrict__ Hc, const C128* __restrict__ Hb,
                                                           size_t n, int mb, const C128* __restrict__ Dg,
                                                           cplx<S>* __restrict__ W) {
    __shared__ C128 Ds[WS_K2 * WS_MB];
    for (int e = threadIdx.x; e < 2 * mb * mb; e += blockDim.x) Ds[e] = Dg[e];
    __syncthreads();
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    C128 acc[WS_MB];
#pragma unroll
    for (int q = 0; q < WS_MB; ++q) acc[q] = mk<C128>(0.0, 0.0);
    for (int l = 0; l < 2 * mb; ++l) {
        const C128 x = (l < mb) ? Hc[(size_t)l * n + r] : Hb[(size_t)(l - mb) * n + r];
#pragma unroll
        for (int q = 0; q < WS_MB; ++q)
            if (q < mb) acc[q] = cfma(acc[q], x, Ds[l * mb + q]);
    }
#pragma unroll
    for (int q = 0; q < WS_MB; ++q)
        if (q < mb) W[(size_t)q * n + r] = mk<cplx<S>>(acc[q].x, acc[q].y);
}

// sum of (y - t)^2 over count entries (one workgroup, fixed order).
__global__ __launch_bounds__(1024) void mse_row_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                       int count, double* __restrict__ out) {
    __shared__ double red[1024];
    double acc = 0.0;
    for (int e = threadIdx.x; e < count; e += 1024) {
        const double d = (double)y[e] - (double)t[e];
        acc += d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// FP32 reals of a (or of a - b) for count complex entries.
__global__ void warm_reals_kernel(const C128* __restrict__ a, const C128* __restrict__ b, int count,
                                  float* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    C128 v = a[e];
    if (b) v = csub(v, b[e]);
    out[2 * e] = (float)v.x;
    out[2 * e + 1] = (float)v.y;
}

// ---------------------------------------------------------------------------

hipError_t launch_warm_target(const double2* G, int mb, int a, int b, int c, double2* Cout, double2* Qout,
                              double2* Rinv, int* status, hipStream_t s) {
    if (mb < 1 || mb > WS_MB) return hipErrorInvalidValue;
    TargetArgs ta{G, mb, a, b, c, Cout, Qout, Rinv, status};
    const size_t lds = (2 * WS_K2 * WS_K2 + WS_K2 * WS_MB + 4 * WS_MB * WS_MB) * sizeof(C128);
    hipError_t e = hipFuncSetAttribute((const void*)warm_target_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(warm_target_kernel, dim3(1), dim3(WS_NT), lds, s, ta);
    return hipGetLastError();
}

int warm_target_blocks(size_t n, int mb, const double2* Xa, const double2* Xb, const double2* Xc, double2* C,
                       double2* Rinv, hipStream_t s) {
    if (mb < 1 || mb > WS_MB) return MFD_EINVAL;
    const int K3 = 3 * mb;
    const int np = gram_parts(n);
    C128 *H = nullptr, *G = nullptr, *part = nullptr, *Ri = nullptr, *Qd = nullptr;
    int* st = nullptr;
    int status = MFD_EDEVICE;
    if (hipMalloc(&H, n * K3 * sizeof(C128)) == hipSuccess && hipMalloc(&G, (size_t)K3 * K3 * sizeof(C128)) == hipSuccess &&
        hipMalloc(&part, (size_t)np * K3 * K3 * sizeof(C128)) == hipSuccess &&
        hipMalloc(&Ri, 4 * (size_t)mb * mb * sizeof(C128)) == hipSuccess && hipMalloc(&st, sizeof(int)) == hipSuccess &&
        hipMalloc(&Qd, (size_t)mb * mb * sizeof(C128)) == hipSuccess) {
        const size_t bytes = n * mb * sizeof(C128);
        int hst = -1;
        if (hipMemcpyAsync(H, Xa, bytes, hipMemcpyDeviceToDevice, s) == hipSuccess &&
            hipMemcpyAsync(H + n * mb, Xb, bytes, hipMemcpyDeviceToDevice, s) == hipSuccess &&
            hipMemcpyAsync(H + 2 * n * mb, Xc, bytes, hipMemcpyDeviceToDevice, s) == hipSuccess &&
            launch_gram(H, n, n, K3, K3, np, part, G, s) == hipSuccess &&
            launch_warm_target(G, mb, 0, 1, 2, C, Qd, Ri, st, s) == hipSuccess &&
            hipMemcpyAsync(&hst, st, sizeof(int), hipMemcpyDeviceToHost, s) == hipSuccess &&
            hipStreamSynchronize(s) == hipSuccess) {
            status = hst == 0 ? MFD_OK : MFD_ENOTCONV;
            if (hst == 0 && Rinv &&
                (hipMemcpy(Rinv, Ri, 4 * (size_t)mb * mb * sizeof(C128), hipMemcpyDeviceToDevice) != hipSuccess))
                status = MFD_EDEVICE;
        }
    } else {
        status = MFD_ENOMEM;
    }
    hipFree(H); hipFree(G); hipFree(part); hipFree(Ri); hipFree(st); hipFree(Qd);
    return status;
}

int WarmStart::init(size_t n_, int mb_, double L_, uint64_t seed_) {
    n = n_;
    mb = mb_;
    L = L_;
    seed = seed_;
    nin = 6 + 2 * mb + 4 * mb * mb;
    nout = 4 * mb * mb;
    nparts = gram_parts(n);
    const size_t K3 = 3 * (size_t)mb;
    hipError_t e;
    auto ok = [&](hipError_t r) { e = r; return r == hipSuccess; };
    if (!(ok(hipMalloc(&H, n * K3 * sizeof(C128))) && ok(hipMalloc(&G, K3 * K3 * sizeof(C128))) &&
          ok(hipMalloc(&gpart, (size_t)nparts * K3 * K3 * sizeof(C128))) &&
          ok(hipMalloc(&Cb, 2 * mb * mb * sizeof(C128))) && ok(hipMalloc(&Cc, 2 * mb * mb * sizeof(C128))) &&
          ok(hipMalloc(&Rinv, 4 * mb * mb * sizeof(C128))) && ok(hipMalloc(&D, 2 * mb * mb * sizeof(C128))) &&
          ok(hipMalloc(&Qc, mb * mb * sizeof(C128))) &&
          ok(hipMalloc(&F, (size_t)pmax * nin * sizeof(float))) &&
          ok(hipMalloc(&T, (size_t)pmax * nout * sizeof(float))) && ok(hipMalloc(&feat, nin * sizeof(float))) &&
          ok(hipMalloc(&pred, nout * sizeof(float))) && ok(hipMalloc(&dstatus, sizeof(int))) &&
          ok(hipHostMalloc(&hstage, (6 + 2 * mb) * sizeof(float), hipHostMallocDefault)) &&
          ok(hipHostMalloc(&hstatus, sizeof(int), hipHostMallocDefault)) &&
          ok(hipMalloc(&zeros, nout * sizeof(float))) && ok(hipMalloc(&dsq, sizeof(double))) &&
          ok(hipHostMalloc(&hsq, sizeof(double), hipHostMallocDefault)) &&
          ok(hipMemset(zeros, 0, nout * sizeof(float)))))
        return e == hipErrorOutOfMemory ? MFD_ENOMEM : MFD_EDEVICE;
    return net.init(nin, 256, 3, nout, pmax, true, seed);
}

void WarmStart::release() {
    hipFree(H); hipFree(G); hipFree(gpart); hipFree(Cb); hipFree(Cc); hipFree(Rinv); hipFree(D); hipFree(Qc);
    hipFree(F); hipFree(T); hipFree(feat); hipFree(pred); hipFree(dstatus);
    if (hstage) hipHostFree(hstage);
    if (hstatus) hipHostFree(hstatus);
    if (hsq) hipHostFree(hsq);
    hipFree(zeros); hipFree(dsq);
    net.release();
}

int WarmStart::reset(hipStream_t s) {
    nsolved = 0;
    npairs = 0;
    pnext = 0;
    have_cb = false;
    rinv_ok = false;
    nscore = 0;
    last_used_net = false;
    slot[0] = 0; slot[1] = 1; slot[2] = 2;
    return net.randomize(seed, s);
}

// The network's input row (device FP32, 6 + 2 mb + 4 mb^2): k_next L / pi,
// (k_next - k_prev) L / pi, the Ritz values at k_j and k_{j-1} over
// (2 pi / L)^2, then C_j (2mb x mb c128, row-major) as (re, im) pairs.  The
// head is staged in `stage` (pinned host, 6 + 2 mb floats), which the copy
// reads until the stream reaches it.
hipError_t warm_feature_row(double L, int mb, const double* k_prev, const double* k_next, const double* lam_j,
                            const double* lam_jm1, const double2* Cj, float* row, float* stage, hipStream_t s) {
    const double sc = L / M_PI, ls = std::pow(2.0 * M_PI / L, 2);
    for (int i = 0; i < 3; ++i) {
        stage[i] = (float)(k_next[i] * sc);
        stage[3 + i] = (float)((k_next[i] - k_prev[i]) * sc);
    }
    for (int q = 0; q < mb; ++q) {
        stage[6 + q] = (float)(lam_j[q] / ls);
        stage[6 + mb + q] = (float)(lam_jm1[q] / ls);
    }
    hipError_t e = hipMemcpyAsync(row, stage, (6 + 2 * mb) * sizeof(float), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    const int cnt = 2 * mb * mb;
    hipLaunchKernelGGL(warm_reals_kernel, dim3((cnt + 255) / 256), dim3(256), 0, s, (const C128*)Cj,
                       (const C128*)nullptr, cnt, row + 6 + 2 * mb);
    return hipGetLastError();
}

static hipError_t feature_row(WarmStart& w, const double* k_prev, const double* k_next, const double* lam_j,
                              const double* lam_jm1, const C128* Cj, float* row, hipStream_t s) {
    hipError_t e = warm_feature_row(w.L, w.mb, k_prev, k_next, lam_j, lam_jm1, (const double2*)Cj, row, w.hstage, s);
    if (e != hipSuccess) return e;
    // the staging buffer is reused by the next row: wait for the copy
    return hipStreamSynchronize(s);
}

// mean squared error of a network output row (or of zeros) against a target row
static int pair_error(WarmStart& w, const float* y, const float* t, double* out, hipStream_t s) {
    hipLaunchKernelGGL(mse_row_kernel, dim3(1), dim3(1024), 0, s, y ? y : w.zeros, t, w.nout, w.dsq);
    if (hipGetLastError() != hipSuccess) return MFD_EDEVICE;
    if (hipMemcpyAsync(w.hsq, w.dsq, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return MFD_EDEVICE;
    *out = *w.hsq;
    return MFD_OK;
}

int WarmStart::after_solve(const double2* X, const double* theta, const double* k, int steps, float lr,
                           hipStream_t s) {
    const int snew = nsolved < 3 ? nsolved : slot[0];
    hipError_t e = hipMemcpyAsync(H + (size_t)snew * mb * n, X, n * mb * sizeof(C128), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return MFD_EDEVICE;
    for (int q = 0; q < mb; ++q) lam[snew][q] = theta[q];
    for (int i = 0; i < 3; ++i) kk[snew][i] = k[i];
    slot[0] = slot[1];
    slot[1] = slot[2];
    slot[2] = snew;
    if (++nsolved < 3) return MFD_OK;
    const int a = slot[0], b = slot[1], c = slot[2];
    if ((e = launch_gram(H, n, n, 3 * mb, 3 * mb, nparts, gpart, G, s)) != hipSuccess) return MFD_EDEVICE;
    if (launch_warm_target(G, mb, a, b, c, Cc, Qc, Rinv, dstatus, s) != hipSuccess) return MFD_EDEVICE;
    // keep the history in one smooth gauge: store X_{j+1} aligned with X_j
    hipLaunchKernelGGL(warm_rotate_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       H + (size_t)c * mb * n, n, mb, (const C128*)Qc);
    if (hipGetLastError() != hipSuccess) return MFD_EDEVICE;
    if (hipMemcpyAsync(hstatus, dstatus, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return MFD_EDEVICE;
    const int status = *hstatus;
    static const bool trace = std::getenv("MFD_TRACE") != nullptr;
    if (trace) std::fprintf(stderr, "[warm %p] solved %d status %d pairs %d\n", (void*)this, nsolved, status, npairs);
    rinv_ok = (status == 0);
    if (status == 1) {   // X_{j-1} and X_j (nearly) dependent: no target from this triple
        have_cb = false;
        return MFD_OK;
    }
    if (have_cb) {
        // pair: features at (k_b -> k_c) with C*_b, target C*_c - C*_b
        float* frow = F + (size_t)pnext * nin;
        float* trow = T + (size_t)pnext * nout;
        if (feature_row(*this, kk[b], kk[c], lam[b], lam[a], Cb, frow, s) != hipSuccess) return MFD_EDEVICE;
        const int cnt = 2 * mb * mb;
        hipLaunchKernelGGL(warm_reals_kernel, dim3((cnt + 255) / 256), dim3(256), 0, s, Cc, Cb, cnt, trow);
        if (hipGetLastError() != hipSuccess) return MFD_EDEVICE;
        // held-out check before training on the new pair: the network's error
        // against the error of proposing no change (the plain extrapolation)
        if (npairs >= 4) {
            if (net.forward(1, frow, pred, s) != hipSuccess) return MFD_EDEVICE;
            double e_net = 0.0, e_base = 0.0;
            if (pair_error(*this, pred, trow, &e_net, s) || pair_error(*this, nullptr, trow, &e_base, s))
                return MFD_EDEVICE;
            const double r = e_base > 0.0 ? e_net / e_base : 1.0;
            score[nscore % 4] = r;
            ++nscore;
            if (std::getenv("MFD_TRACE"))
                std::fprintf(stderr, "[warm %p] held-out error: network %.3e, no change %.3e\n", (void*)this, e_net,
                             e_base);
        }
        pnext = (pnext + 1) % pmax;
        npairs = std::min(npairs + 1, pmax);
        for (int it = 0; it < steps; ++it) {
            if (net.loss_grad(npairs, F, T, s) != hipSuccess || net.adam(lr, s) != hipSuccess) return MFD_EDEVICE;
        }
    }
    std::swap(Cb, Cc);
    have_cb = true;
    return MFD_OK;
}

bool WarmStart::net_trusted() const {
    if (nscore < 2) return false;
    const int k = std::min(nscore, 4);
    double m = 0.0;
    for (int i = 0; i < k; ++i) m += score[i];
    return m / k < 0.8;
}

int WarmStart::propose(const double* k_next, void* W, bool w32, bool* made, hipStream_t s) {
    *made = false;
    if (!rinv_ok || !have_cb || npairs < 4 || nsolved < 3) return MFD_OK;
    const int b = slot[1], c = slot[2];
    if (net_trusted()) {
        if (feature_row(*this, kk[c], k_next, lam[c], lam[b], Cb, feat, s) != hipSuccess) return MFD_EDEVICE;
        if (net.forward(1, feat, pred, s) != hipSuccess) return MFD_EDEVICE;
    } else if (hipMemsetAsync(pred, 0, nout * sizeof(float), s) != hipSuccess) {
        return MFD_EDEVICE;
    }
    last_used_net = net_trusted();
    const int cnt = 2 * mb * mb;
    hipLaunchKernelGGL(warm_coef_kernel, dim3((cnt + 255) / 256), dim3(256), 0, s, Rinv, Cb, pred, mb, D);
    if (hipGetLastError() != hipSuccess) return MFD_EDEVICE;
    const C128* Hc = H + (size_t)c * mb * n;
    const C128* Hb = H + (size_t)b * mb * n;
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (w32)
        hipLaunchKernelGGL(warm_combine_kernel<float>, dim3(nb), dim3(256), 0, s, Hc, Hb, n, mb, D, (float2*)W);
    else
        hipLaunchKernelGGL(warm_combine_kernel<double>, dim3(nb), dim3(256), 0, s, Hc, Hb, n, mb, D, (double2*)W);
    if (hipGetLastError() != hipSuccess) return MFD_EDEVICE;
    *made = true;
    return MFD_OK;
}

}  // namespace mfd
