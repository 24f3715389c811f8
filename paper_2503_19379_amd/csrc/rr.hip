// Rayleigh-Ritz step of the block eigensolver, on the device, one workgroup.
//
// Section 5.1 takes the eigenpairs from LOBPCG, which minimises the Rayleigh
// quotient over span[X, W, P] at every step.  Given the Gram matrices
// Gs = S^H S and Ga = S^H A S of the basis S = [X, W, P] (3 mb columns) this
// kernel returns coefficients C with S C = the mb lowest Ritz vectors:
//   1. keep X, the columns of W and P belonging to unconverged bands
//      (residual above tol, "soft locking"), scale every kept column to unit
//      norm (d = diag(Gs)^-1/2);
//   2. Cholesky factor D Gs D = R^H R column by column; a column whose pivot
//      (squared distance to the span of the previous columns) falls below a
//      threshold is dropped, and if a P column does, all of P is dropped for
//      this step (the conjugate direction is restarted);
//   3. H = Z^H (D Ga D) Z with Z = R^-1, so that H is the operator in an
//      orthonormal basis of the kept span;
//   4. cyclic Jacobi on the Hermitian H (round-robin pairs, all disjoint
//      rotations of a round applied at once), accumulating Z <- Z J;
//   5. C = D Z[:, lowest mb eigenvalues].
// Dropped columns are isolated in H with a huge diagonal entry, so the shapes
// stay fixed and they are never selected.
#include "common.h"
#include "solver.h"

namespace mfd {

using C128 = double2;
constexpr int RR_NT = 512;
constexpr int RR_KMAX = 64;
constexpr double RR_BIG = 1e300;

struct Rot {
    double c, s;
    C128 em;   // e^{-i phi}
    int p, q;
    int skip;
};

__global__ __launch_bounds__(RR_NT) void rr_kernel(RRArgs a) {
    extern __shared__ unsigned char smem_raw[];
    const int mb = a.mb;
    const int K = 3 * mb;
    const int KE = K + (K & 1);
    C128* A = reinterpret_cast<C128*>(smem_raw);   // K x K: Gs -> R -> Z
    C128* B = A + K * K;                           // K x K: Ga -> T -> H
    __shared__ double dsc[RR_KMAX];
    __shared__ int kept[RR_KMAX];
    __shared__ int dropped[RR_KMAX];
    __shared__ double piv_s;
    __shared__ int dropP;
    __shared__ Rot rot[RR_KMAX / 2];
    __shared__ double redv[2][RR_NT / 64];
    __shared__ int perm[RR_KMAX];
    __shared__ int sweeps_s;
    __shared__ int active_s;
    const int tid = threadIdx.x;
    const int Q = 6 * mb;

    // 1. active columns and scaling
    if (tid < K) {
        const int j = tid;
        int keep = 1;
        if (j >= mb) {
            if (a.first) keep = 0;
            else {
                const int b = (j < 2 * mb) ? j - mb : j - 2 * mb;
                const double th = fabs(a.theta[b]);
                const double res = sqrt(a.norms[b]) / (th * sqrt(a.norms[mb + b]));
                keep = (res > a.tol) ? 1 : 0;
            }
        }
        const double g = a.G[j * Q + j].x;
        if (!(g > 0.0)) keep = 0;
        kept[j] = keep;
        dropped[j] = 0;
        dsc[j] = keep ? 1.0 / sqrt(g) : 0.0;
    }
    if (tid == 0) {
        dropP = 0;
        int act = 0;
        if (!a.first)
            for (int b = 0; b < mb; ++b) {
                const double res = sqrt(a.norms[b]) / (fabs(a.theta[b]) * sqrt(a.norms[mb + b]));
                act += (res > a.tol);
            }
        active_s = act;
    }
    __syncthreads();
    for (int e = tid; e < K * K; e += RR_NT) {
        const int i = e / K, j = e % K;
        const double s = dsc[i] * dsc[j];
        const C128 gs = a.G[i * Q + j];
        const C128 g1 = a.G[i * Q + K + j], g2 = a.G[j * Q + K + i];
        A[e] = mk<C128>(gs.x * s, gs.y * s);
        B[e] = mk<C128>(0.5 * (g1.x + g2.x) * s, 0.5 * (g1.y - g2.y) * s);
    }
    __syncthreads();

    // 2. Cholesky with column dropping (upper factor R in A)
    for (int j = 0; j < K; ++j) {
        if (tid == 0) {
            double rjj = 0.0;
            if (kept[j]) {
                const double piv = A[j * K + j].x;
                const bool isP = j >= 2 * mb;
                const double thr = isP ? a.drop_p : a.drop_w;
                if (!(piv > thr) || (isP && dropP)) {
                    dropped[j] = 1;
                    if (isP) dropP = 1;
                } else {
                    rjj = sqrt(piv);
                }
            }
            piv_s = rjj;
        }
        __syncthreads();
        const double rjj = piv_s;
        if (rjj > 0.0) {
            const double inv = 1.0 / rjj;
            for (int l = j + 1 + tid; l < K; l += RR_NT) A[j * K + l] = cscale(A[j * K + l], inv);
            if (tid == 0) A[j * K + j] = mk<C128>(rjj, 0.0);
            __syncthreads();
            // trailing update of the upper triangle: A[i][l] -= conj(R[j][i]) R[j][l], j < i <= l
            const int m = K - j - 1;
            for (int e = tid; e < m * m; e += RR_NT) {
                const int i = j + 1 + e / m, l = j + 1 + e % m;
                if (l >= i) {
                    const C128 ri = A[j * K + i], rl = A[j * K + l];
                    C128 v = A[i * K + l];
                    v.x -= ri.x * rl.x + ri.y * rl.y;
                    v.y -= ri.x * rl.y - ri.y * rl.x;
                    A[i * K + l] = v;
                }
            }
        }
        __syncthreads();
    }
    // a restarted P drops every P column; isolate all dropped / unkept columns
    if (tid < K) {
        const int j = tid;
        if (dropP && j >= 2 * mb && kept[j]) dropped[j] = 1;
        if (!kept[j]) dropped[j] = 1;
    }
    __syncthreads();
    for (int e = tid; e < K * K; e += RR_NT) {
        const int i = e / K, l = e % K;
        if (l < i) A[e] = mk<C128>(0.0, 0.0);            // lower part unused: keep it zero
        else if (dropped[i] || dropped[l]) A[e] = mk<C128>(i == l ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();

    // 3a. Z = R^-1 in place, column by column (upper triangular)
    for (int j = 0; j < K; ++j) {
        const double inv = 1.0 / A[j * K + j].x;
        C128 zij = mk<C128>(0.0, 0.0);
        const int i = tid;
        if (i < j) {
            C128 s = mk<C128>(0.0, 0.0);
            for (int l = i; l < j; ++l) s = cfma(s, A[i * K + l], A[l * K + j]);
            zij = mk<C128>(-s.x * inv, -s.y * inv);
        }
        __syncthreads();
        if (i < j) A[i * K + j] = zij;
        if (i == j) A[j * K + j] = mk<C128>(inv, 0.0);
        __syncthreads();
    }
    // 3b. T = Ga Z, then H = Z^H T (register-staged in place in B)
    constexpr int PER = (RR_KMAX * RR_KMAX + RR_NT - 1) / RR_NT;
    {
        C128 t[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            t[q] = mk<C128>(0.0, 0.0);
            if (e < K * K) {
                const int i = e / K, j = e % K;
                C128 s = mk<C128>(0.0, 0.0);
                for (int l = 0; l <= j; ++l) s = cfma(s, B[i * K + l], A[l * K + j]);
                t[q] = s;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < K * K) B[e] = t[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < K * K) {
                const int i = e / K, j = e % K;
                C128 s = mk<C128>(0.0, 0.0);
                for (int l = 0; l <= i; ++l) s = cfmac(s, A[l * K + i], B[l * K + j]);
                t[q] = s;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < K * K) B[e] = t[q];
        }
        __syncthreads();
        // Hermitian part; isolate dropped columns
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < K * K) {
                const int i = e / K, j = e % K;
                if (dropped[i] || dropped[j]) t[q] = mk<C128>(i == j ? RR_BIG : 0.0, 0.0);
                else if (i == j) t[q] = mk<C128>(B[e].x, 0.0);
                else {
                    const C128 u = B[e], v = B[j * K + i];
                    t[q] = mk<C128>(0.5 * (u.x + v.x), 0.5 * (u.y - v.y));
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * RR_NT;
            if (e < K * K) B[e] = t[q];
        }
        __syncthreads();
    }

    // 4. cyclic Jacobi, round-robin ordering
    const int npairs = KE / 2;
    int sweep = 0;
    for (; sweep < 30; ++sweep) {
        // convergence test: off-diagonal mass vs diagonal mass (kept columns)
        double off = 0.0, dn = 0.0;
        for (int e = tid; e < K * K; e += RR_NT) {
            const int i = e / K, j = e % K;
            if (dropped[i] || dropped[j]) continue;
            const C128 v = B[e];
            if (i == j) dn += v.x * v.x;
            else off += cabs2(v);
        }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_down(off, o);
            dn += __shfl_down(dn, o);
        }
        if ((tid & 63) == 0) { redv[0][tid >> 6] = off; redv[1][tid >> 6] = dn; }
        __syncthreads();
        off = 0.0; dn = 0.0;
        for (int w = 0; w < RR_NT / 64; ++w) { off += redv[0][w]; dn += redv[1][w]; }
        __syncthreads();
        if (off <= 1e-30 * dn) break;
        for (int r = 0; r < KE - 1; ++r) {
            if (tid < npairs) {
                const int i = tid;
                int p, q;
                if (i == 0) { p = KE - 1; q = r; }
                else { p = (r + i) % (KE - 1); q = (r - i + (KE - 1)) % (KE - 1); }
                if (p > q) { const int t = p; p = q; q = t; }
                Rot ro;
                ro.p = p; ro.q = q; ro.skip = 1; ro.c = 1.0; ro.s = 0.0; ro.em = mk<C128>(1.0, 0.0);
                if (q < K && !dropped[p] && !dropped[q]) {
                    const C128 b = B[p * K + q];
                    const double beta = sqrt(cabs2(b));
                    const double ap = B[p * K + p].x, dq = B[q * K + q].x;
                    if (beta > 1e-300 && beta > 1e-18 * sqrt(fabs(ap * dq))) {
                        const double tau = (dq - ap) / (2.0 * beta);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        ro.c = 1.0 / sqrt(1.0 + t * t);
                        ro.s = t * ro.c;
                        ro.em = mk<C128>(b.x / beta, -b.y / beta);
                        ro.skip = 0;
                    }
                }
                rot[i] = ro;
            }
            __syncthreads();
            // rows: J^H H
            for (int e = tid; e < npairs * K; e += RR_NT) {
                const Rot ro = rot[e / K];
                if (ro.skip) continue;
                const int col = e % K;
                const C128 hp = B[ro.p * K + col], hq = B[ro.q * K + col];
                const C128 ep = mk<C128>(ro.em.x, -ro.em.y);   // e^{i phi}
                const C128 t = cmul(ep, hq);
                B[ro.p * K + col] = mk<C128>(ro.c * hp.x - ro.s * t.x, ro.c * hp.y - ro.s * t.y);
                B[ro.q * K + col] = mk<C128>(ro.s * hp.x + ro.c * t.x, ro.s * hp.y + ro.c * t.y);
            }
            __syncthreads();
            // columns: H J and Z J
            for (int e = tid; e < 2 * npairs * K; e += RR_NT) {
                const int pe = e % (npairs * K);
                const Rot ro = rot[pe / K];
                if (ro.skip) continue;
                const int row = pe % K;
                C128* M = (e < npairs * K) ? B : A;
                const C128 hp = M[row * K + ro.p], hq = M[row * K + ro.q];
                const C128 t = cmul(ro.em, hq);
                C128 np = mk<C128>(ro.c * hp.x - ro.s * t.x, ro.c * hp.y - ro.s * t.y);
                C128 nq = mk<C128>(ro.s * hp.x + ro.c * t.x, ro.s * hp.y + ro.c * t.y);
                if (M == B) {
                    if (row == ro.p) nq = mk<C128>(0.0, 0.0);
                    if (row == ro.q) np = mk<C128>(0.0, 0.0);
                }
                M[row * K + ro.p] = np;
                M[row * K + ro.q] = nq;
            }
            __syncthreads();
        }
    }
    // 5. order the eigenvalues, emit coefficients of the lowest mb
    if (tid < K) {
        const double ti = B[tid * K + tid].x;
        int rank = 0;
        for (int j = 0; j < K; ++j) {
            const double tj = B[j * K + j].x;
            rank += (tj < ti) || (tj == ti && j < tid);
        }
        perm[rank] = tid;
    }
    __syncthreads();
    for (int e = tid; e < K * mb; e += RR_NT) {
        const int j = e / mb, r = e % mb;
        const int c = perm[r];
        const C128 z = A[j * K + c];
        a.C[e] = mk<C128>(dsc[j] * z.x, dsc[j] * z.y);
    }
    if (tid < mb) a.theta[tid] = B[perm[tid] * K + perm[tid]].x;
    if (tid == 0) {
        int nk = 0;
        for (int j = 0; j < K; ++j) nk += !dropped[j];
        a.info[0] = nk;
        a.info[1] = dropP;
        a.info[2] = active_s;
        a.info[3] = sweep;
    }
}

hipError_t launch_rr(const RRArgs& a, hipStream_t s) {
    const int K = 3 * a.mb;
    if (K > RR_KMAX) return hipErrorInvalidValue;
    const size_t lds = (size_t)2 * K * K * sizeof(C128);
    hipError_t e = hipFuncSetAttribute((const void*)rr_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rr_kernel, dim3(1), dim3(RR_NT), lds, s, a);
    return hipGetLastError();
}

}  // namespace mfd
